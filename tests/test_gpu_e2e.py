"""End-to-end parity of whole HOTRG runs on the GPU (through the C ABI) against the
FP64 oracle: exact tori while nothing is truncated, then the oracle fixtures of the
physics configurations (gauge-invariant quantities only: lnZ/V after every step,
normalised Gram spectra, judgement values)."""

import json
import math
import os

import numpy as np
import pytest

from oracle import exact as E
from oracle import hotrg as H
from tests import parity as PT

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


def run_gpu(kind, d, beta, chi, steps, precision="fp64", q=None, axes=None, chunk=0):
    r = P.HOTRG(kind, d, beta, chi, q=q, precision=precision, max_steps=max(steps, 1), chunk=chunk)
    out = []
    for p in range(steps):
        r.step(None if axes is None else axes[p])
        out.append(r.log_z())
    return r, out


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# Exact tori (untruncated steps) -- brute force, independent of the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind,d,q,beta,chi,steps", [
    ("ising", 2, 2, 0.44, 16, 4),
    ("ising", 3, 2, 0.2216544, 16, 3),
    ("potts", 3, 3, 0.55, 9, 1),
    ("potts", 2, 3, 0.9, 9, 1),
    # 4D: one step is exact (legs of dimension 4); FP64 runs 4D up to chi = 7
    ("ising", 4, 2, 0.15, 7, 1),
])
def test_untruncated_steps_equal_brute_force(kind, d, q, beta, chi, steps):
    r, lnz = run_gpu(kind, d, beta, chi, steps, q=q)
    for p in range(1, steps + 1):
        L = H.lattice_shape(d, p)
        z, _ = E.torus_log_z(kind, beta, L, q=q)
        assert lnz[p - 1] == pytest.approx(z / np.prod(L), abs=1e-13), (p, L)


def test_initial_lnz_closed_form():
    for d in (2, 3, 4):
        r = P.HOTRG("ising", d, 0.3, 4)
        assert r.log_z() == pytest.approx(math.log(2) + d * 0.3, abs=1e-15)


# ---------------------------------------------------------------------------
# Physics configurations against the oracle fixtures
# ---------------------------------------------------------------------------

def _rel(a, b):
    return abs(a - b) / abs(b)


# The trace t_p and the Gu-Wen ratio X after every step against the oracle fixture.
# FP64: 1e-10 (the bound of lnZ/V) at every step up to the first cut whose effective gap
# (lambda_{kept-1} - lambda_kept) / lambda_0 is below 1e-5; after it the kept subspace, and with
# it t_p and X, moves by (rounding of A) / gap in any two FP64 implementations (in config 2 at
# T = 4.0 the gaps fall to 1e-7 and t_p parts by up to 5e-4 while lnZ/V, where t_p enters with
# weight 1/2^p, stays within 1e-11).  Reduced forms: t_p and X carry the form's rounding
# amplified by the flow (near T_c a perturbation of T grows by about 2^(y_t / 3) = 1.44 per step,
# y_t the thermal exponent of the 3D Ising class), up to 1e-4 (FP32, split FP16) and 0.1 (split
# BF16) at late steps; there only a gross-error bound is asserted and the values are printed.
TRACE_TIGHT = {"fp64": 1e-10}
TRACE_GROSS = {"fp64": 1e-2, "fp32": 0.5, "split_fp16": 0.5, "split_bf16": 0.5}
FP64_GAP_THRESHOLD = 1e-5


def compare_run(r, run_fix, lnz_gpu, precision, dirs):
    """Per-step errors of lnZ/V, t_p and X against one oracle run, and the steps where the
    kept column counts differ.  FP64 must keep the oracle's column counts, except at a cut
    decided by rounding (tests/parity.py).  Returns (max lnZ/V error, final lnZ/V error)."""
    steps = len(run_fix["steps"])
    e_lnz, e_tr, e_x, kdiff, krounding = [], [], [], [], []
    for p in range(1, steps + 1):
        rec, info = run_fix["steps"][p - 1], r.info(p)
        e_lnz.append(_rel(lnz_gpu[p - 1], rec["lnz_per_site"]))
        e_tr.append(_rel(info.trace, rec["trace"]))
        e_x.append(_rel(info.gu_wen, rec["gu_wen"]))
        assert info.lnz_per_site == lnz_gpu[p - 1]
        for j in dirs:
            dd = rec["dirs"][str(j)]
            if info.kept[j - 1] != dd["kept"]:
                (krounding if PT.rounding_decided_cut(dd, info.kept[j - 1]) else kdiff).append(p)
    fmt = lambda v: " ".join(f"{e:.1e}" for e in v)   # noqa: E731
    ncond = PT.conditioned_steps(run_fix, FP64_GAP_THRESHOLD)
    print(f"  lnZ/V per step: {fmt(e_lnz)}\n  trace per step: {fmt(e_tr)}\n  Gu-Wen X per step: {fmt(e_x)}"
          f"\n  kept differs at steps: {kdiff} (at rounding-decided cuts: {krounding}); "
          f"steps before an effective gap < {FP64_GAP_THRESHOLD:.0e}: {ncond}")
    if precision == "fp64":
        assert kdiff == [], f"FP64 kept counts differ from the oracle at steps {kdiff}"
        assert max(e_tr[:ncond]) < TRACE_TIGHT["fp64"] and max(e_x[:ncond]) < TRACE_TIGHT["fp64"]
    assert max(e_tr) < TRACE_GROSS[precision] and max(e_x) < TRACE_GROSS[precision]
    return max(e_lnz), e_lnz[-1]


def test_config1_fp64_2d_ising_chi8():
    fx = load("config1.json")
    for run in fx["runs"]:
        r, lnz = run_gpu("ising", 2, run["beta"], fx["chi"], fx["steps"])
        print(f"config1 beta={run['beta']:.6f}")
        emax, elast = compare_run(r, run, lnz, "fp64", dirs=(1,))
        print(f"  max|df|/|f|={emax:.2e} final={elast:.2e}")
        assert emax < 1e-10


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("fp32", 1e-6), ("split_fp16", 1e-6),
                                             ("split_bf16", 1e-4)])
def test_config2_3d_ising_chi8(precision, bound):
    fx = load("config2.json")
    worst = 0.0
    for run in fx["runs"]:
        r, lnz = run_gpu("ising", 3, run["beta"], fx["chi"], fx["steps"], precision=precision)
        print(f"config2 {precision} beta={run['beta']:.6f}")
        emax, elast = compare_run(r, run, lnz, precision, dirs=(1, 2))
        print(f"  max rel err={emax:.2e} final={elast:.2e}")
        worst = max(worst, emax)
    assert worst < bound


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("split_fp16", 1e-6), ("fp32", 1e-6),
                                             ("split_bf16", 1e-4)])
def test_config3_3d_ising_chi16(precision, bound):
    """3D Ising, chi = 16, T = 4.5115, 25 steps (the benchmark workload) against the oracle
    fixture after every step: lnZ/V, trace and Gu-Wen ratio, and in FP64 the kept column
    counts; steps 1-3 are untruncated, step 3 is the 2x2x2 torus."""
    fx = load("config3.json")
    run = fx["runs"][0]
    r, lnz = run_gpu("ising", 3, run["beta"], fx["chi"], fx["steps"], precision=precision)
    print(f"config3 {precision} beta={run['beta']:.7f}")
    emax, elast = compare_run(r, run, lnz, precision, dirs=(1, 2))
    print(f"  max rel err={emax:.2e} final={elast:.2e}")
    assert emax < bound


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("split_fp16", 1e-6), ("fp32", 1e-6)])
def test_config6_4d_ising_chi4(precision, bound):
    """4D Ising (the paper's own model), chi = 4, T = 6.0, 6.68, 7.5, 12 steps: three Next
    directions per step, against the oracle fixture after every step (lnZ/V, trace, Gu-Wen
    ratio, and in FP64 the kept column counts)."""
    fx = load("config6.json")
    worst = 0.0
    for run in fx["runs"]:
        r, lnz = run_gpu("ising", 4, run["beta"], fx["chi"], fx["steps"], precision=precision)
        print(f"config6 {precision} beta={run['beta']:.6f}")
        emax, elast = compare_run(r, run, lnz, precision, dirs=(1, 2, 3))
        print(f"  max rel err={emax:.2e} final={elast:.2e}")
        worst = max(worst, emax)
    assert worst < bound


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("split_fp16", 1e-6)])
def test_config7_4d_ising_chi5(precision, bound):
    """4D Ising, chi = 5 (H = 625, no dimension a multiple of a tile), T = 6.68, 8 steps."""
    fx = load("config7.json")
    run = fx["runs"][0]
    r, lnz = run_gpu("ising", 4, run["beta"], fx["chi"], fx["steps"], precision=precision)
    print(f"config7 {precision} beta={run['beta']:.6f}")
    emax, elast = compare_run(r, run, lnz, precision, dirs=(1, 2, 3))
    print(f"  max rel err={emax:.2e} final={elast:.2e}")
    assert emax < bound


def test_config2_spectra_and_judgement_values():
    fx = load("config2.json")
    run = fx["runs"][1]
    r, _ = run_gpu("ising", 3, run["beta"], fx["chi"], 12)
    for p in range(1, 13):
        rec = run["steps"][p - 1]
        info = r.info(p)
        for j in (1, 2):
            dref = rec["dirs"][str(j)]
            assert info.chi_new[j - 1] == dref["chi_new"]
            if not info.truncated[j - 1]:
                continue
            for side, key in ((0, "spec"), (1, "spec_p")):
                spec = r.spectrum(p, j, side, cap=dref["chi_new"])
                ref = dref[key][: len(spec)]
                np.testing.assert_allclose(spec, ref, rtol=0, atol=1e-9)
            # judgement values relative to the leading eigenvalue are gauge invariant
            assert info.eps[j - 1] == pytest.approx(dref["eps"], rel=1e-5, abs=1e-13)


def test_fp64_run_is_bitwise_deterministic():
    _, a = run_gpu("ising", 3, 1 / 4.5115, 8, 10)
    _, b = run_gpu("ising", 3, 1 / 4.5115, 8, 10)
    assert a == b


def test_axis_relabelling_invariance():
    # isotropic model: the order x, z, y is the mirror image of x, y, z
    beta = 1 / 4.5115
    _, a = run_gpu("ising", 3, beta, 8, 9, axes=[0, 1, 2] * 3)
    _, b = run_gpu("ising", 3, beta, 8, 9, axes=[0, 2, 1] * 3)
    np.testing.assert_allclose(b, a, rtol=1e-12)


def test_chunking_does_not_change_results():
    beta = 1 / 4.5115
    _, a = run_gpu("ising", 3, beta, 8, 8, chunk=0)
    _, b = run_gpu("ising", 3, beta, 8, 8, chunk=5)
    np.testing.assert_allclose(b, a, rtol=1e-13)


@pytest.mark.parametrize("precision", ["split_fp16", "fp32"])
@pytest.mark.parametrize("chi", [8, 12])
def test_chunking_reduced_forms(precision, chi):
    """Pair chunks of 5 cut the n1' blocks (k2 = 8 or 12) of the MFMA prime chain: every entry
    of B and of the product is computed by the same arithmetic as without chunking."""
    beta = 1 / 4.5115
    _, a = run_gpu("ising", 3, beta, chi, 7, precision=precision, chunk=0)
    _, b = run_gpu("ising", 3, beta, chi, 7, precision=precision, chunk=5)
    print(f"{precision} chi={chi}: max rel diff {np.max(np.abs(np.array(b) - np.array(a)) / np.abs(np.array(a))):.2e}")
    np.testing.assert_allclose(b, a, rtol=1e-13)


def test_state_errors():
    r = P.HOTRG("ising", 2, 0.4, 4, max_steps=2)
    r.step()
    r.step()
    with pytest.raises(P.HotrgError) as e:
        r.step()
    assert e.value.code == P.HOTRG_E_STATE
    with pytest.raises(P.HotrgError) as e:
        P.hotrg_step(r.handle, 5)
    assert e.value.code == P.HOTRG_E_ARG
    with pytest.raises(P.HotrgError) as e:
        P.hotrg_grad(r.handle)
    assert e.value.code == P.HOTRG_E_STATE


# ---------------------------------------------------------------------------
# Ising model in a field h != 0 (Section 2, eqs. 1-2: g = beta h s, V_s = e^{beta h s})
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d,beta,h,steps", [(2, 0.5, 0.3, 4), (3, 0.25, -0.2, 3), (2, 0.42, 0.05, 4)])
def test_field_untruncated_steps_equal_brute_force(d, beta, h, steps):
    """Untruncated steps (chi = 16) with a field: the exact periodic tori 2x1, 2x2, 4x2, 4x4 (2D)
    and 2x1x1, 2x2x1, 2x2x2 (3D), including the derivative (minus the energy per site)."""
    r = P.HOTRG("ising", d, beta, 16, h=h, max_steps=steps, record_grad=True)
    for p in range(1, steps + 1):
        r.step()
        L = H.lattice_shape(d, p)
        z, dz = E.torus_log_z("ising", beta, L, h=h)
        assert r.log_z() == pytest.approx(z / np.prod(L), abs=1e-13), (p, L)
        assert r.grad() == pytest.approx(dz / np.prod(L), abs=1e-12), (p, L)
    r.close()


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("split_fp16", 1e-6)])
@pytest.mark.parametrize("d,beta,h,chi,steps", [(2, 0.44, 0.05, 12, 16), (3, 0.23, 0.02, 6, 12)])
def test_field_truncated_run_matches_oracle(d, beta, h, chi, steps, precision, bound):
    """Truncated runs in a field against the oracle run (computed here; the field breaks the
    s -> -s symmetry, so U and U' and the even/odd structure of the spectra differ from h = 0):
    lnZ/V, trace and Gu-Wen ratio after every step, kept counts in FP64."""
    _, recs = H.run(H.Model("ising", d, h=h), beta, chi, steps)
    r = P.HOTRG("ising", d, beta, chi, h=h, precision=precision, max_steps=steps)
    e_lnz, e_x = [], []
    for p in range(1, steps + 1):
        r.step()
        info = r.info(p)
        e_lnz.append(_rel(r.log_z(), recs[p - 1].lnz_per_site))
        e_x.append(_rel(info.gu_wen, recs[p - 1].gu_wen))
        if precision == "fp64":
            assert [info.kept[j] for j in range(d - 1)] == [recs[p - 1].truncations[j + 1].kept for j in range(d - 1)]
    r.close()
    print(f"field h={h} d={d} chi={chi} {precision}: lnZ/V per step " + " ".join(f"{e:.1e}" for e in e_lnz)
          + "; X per step " + " ".join(f"{e:.1e}" for e in e_x))
    assert max(e_lnz) < bound
    if precision == "fp64":
        assert max(e_x) < 1e-9
