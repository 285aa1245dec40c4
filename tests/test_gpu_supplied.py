"""Runs started from a supplied local tensor (hotrg_init_tensor) against the oracle run on the
same tensor, and the numeric-failure paths: a non-positive or non-finite trace, and an
eigensolver failure, reported as a sticky HOTRG_E_NUMERIC while every kernel exits normally."""

import math

import numpy as np
import pytest

from oracle import hotrg as H
from tests import layout as LY
from tests import parity as PT
from tests import seeded_inputs as SI

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


CASES = [((3, 4, 2), 6, 7), ((5, 7), 8, 10), ((4, 4, 4), 8, 6)]


@pytest.mark.parametrize("precision,bound", [("fp64", 1e-10), ("split_fp16", 1e-6)])
@pytest.mark.parametrize("dims,chi,steps", CASES)
def test_supplied_tensor_matches_oracle(dims, chi, steps, precision, bound):
    """A random positive tensor (no symmetry, generic spectra) coarse-grained by the GPU and by
    the oracle (oracle.hotrg.run with T0): lnZ/V, trace and the kept counts after every step."""
    d = len(dims)
    Ts = SI.random_positive_tensor(tuple(dims) * 2, seed=21 + d)
    lnz0, recs = H.run(H.Model("ising", d), 0.0, chi, steps, T0=LY.to_paper(Ts))
    r = P.HOTRG.from_tensor(gu.dev(Ts), chi, precision=precision, max_steps=steps)
    assert r.log_z() == pytest.approx(lnz0, rel=1e-14)
    e_lnz, e_tr = [], []
    for p in range(1, steps + 1):
        r.step()
        info = r.info(p)
        e_lnz.append(abs(r.log_z() - recs[p - 1].lnz_per_site) / abs(recs[p - 1].lnz_per_site))
        e_tr.append(abs(info.trace - recs[p - 1].trace) / abs(recs[p - 1].trace))
        if precision == "fp64":
            assert [info.kept[j] for j in range(d - 1)] == [recs[p - 1].truncations[j + 1].kept for j in range(d - 1)]
    r.close()
    print(f"supplied tensor dims={dims} chi={chi} {precision}: lnZ/V per step "
          + " ".join(f"{e:.1e}" for e in e_lnz) + "; trace per step " + " ".join(f"{e:.1e}" for e in e_tr))
    assert max(e_lnz) < bound
    assert max(e_tr) < (1e-10 if precision == "fp64" else 1e-4)


def _expect_numeric(fn):
    with pytest.raises(P.HotrgError) as e:
        fn()
    assert e.value.code == P.HOTRG_E_NUMERIC, e.value


def test_non_positive_trace_is_a_sticky_numeric_error():
    Ts = SI.random_positive_tensor((3, 3, 3) * 2, seed=5)
    H_ = 27
    M = Ts.reshape(H_, H_)
    M[np.arange(H_), np.arange(H_)] = -1.0               # Tr T0 = -27
    r = P.HOTRG.from_tensor(gu.dev(M.reshape(Ts.shape)), 4, max_steps=4)
    _expect_numeric(r.log_z)
    with pytest.raises(P.HotrgError) as e:               # the handle stays failed
        r.step()
    assert e.value.code == P.HOTRG_E_STATE
    _expect_numeric(r.log_z)
    r.close()


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_non_finite_entry_is_a_numeric_error(precision):
    """A NaN off the diagonal: Tr T0 is finite, the Gram matrices and the eigensolver input are
    not; the first step reports HOTRG_E_NUMERIC (eigensolver failure, then a non-finite trace)."""
    Ts = SI.random_positive_tensor((4, 4, 4) * 2, seed=6)
    M = Ts.reshape(64, 64)
    M[3, 17] = np.nan
    r = P.HOTRG.from_tensor(gu.dev(M.reshape(Ts.shape)), 8, precision=precision, max_steps=4)
    assert math.isfinite(r.log_z())
    r.step()
    _expect_numeric(r.log_z)
    r.close()


def test_eigensolver_reports_non_finite_input():
    n = 64
    A = np.eye(n)[None].copy()
    A[0, 5, 9] = A[0, 9, 5] = np.inf
    _expect_numeric(lambda: gu.eigh(A))
    # the same solver on a valid matrix afterwards: no failure, correct eigenvalues
    B = np.diag(np.arange(n, dtype=np.float64))[None].copy()
    w, _ = gu.eigh(B)
    np.testing.assert_allclose(w[0], np.arange(n)[::-1], atol=1e-12)


def test_gpu_is_healthy_after_the_failures():
    r = P.HOTRG("ising", 3, 1 / 4.5115, 8, max_steps=6)
    r.run(6)
    lnz = r.log_z()
    r.close()
    _, recs = H.run(H.Model("ising", 3), 1 / 4.5115, 8, 6)
    assert abs(lnz - recs[-1].lnz_per_site) < 1e-10 * abs(recs[-1].lnz_per_site)


# ---------------------------------------------------------------------------
# Choice criteria (Section 4.2.6) and normalisation factors (Section 3.1.3)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("norm,choice", [("trace", "U"), ("trace", "Uprime"), ("maxabs", "epsilon"),
                                         ("maxabs", "Uprime")])
def test_choice_and_norm_options_match_oracle(norm, choice):
    """A tensor without reflection symmetry (U and U' differ): the GPU run with a fixed choice or
    the max-element normalisation against the oracle run with the same options, lnZ/V and kept
    counts after every step; a fixed choice shows in every truncated direction's record."""
    dims, chi, steps = (3, 4, 2), 6, 7
    Ts = SI.random_positive_tensor(tuple(dims) * 2, seed=24)
    _, recs = H.run(H.Model("ising", 3), 0.0, chi, steps, T0=LY.to_paper(Ts), norm=norm, choice=choice)
    r = P.HOTRG.from_tensor(gu.dev(Ts), chi, max_steps=steps, norm=norm, choice=choice)
    errs = []
    for p in range(1, steps + 1):
        r.step()
        info = r.info(p)
        errs.append(abs(r.log_z() - recs[p - 1].lnz_per_site) / abs(recs[p - 1].lnz_per_site))
        for j in (1, 2):
            t = recs[p - 1].truncations[j]
            assert info.kept[j - 1] == t.kept
            if info.truncated[j - 1]:
                assert info.chose_prime[j - 1] == int(t.chose_prime)
                if choice != "epsilon":
                    assert info.chose_prime[j - 1] == (choice == "Uprime")
    r.close()
    print(f"norm={norm} choice={choice}: lnZ/V per step " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) < 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("split_fp16", 1e-6)])
def test_normalisation_does_not_change_lnz(precision, tol):
    """3D Ising chi = 8, 10 steps: f = 1/max|T| against f = 1/Tr T (lnZ/V is independent of the
    normalisation factor)."""
    out = {}
    for norm in ("trace", "maxabs"):
        r = P.HOTRG("ising", 3, 1 / 4.5115, 8, precision=precision, max_steps=10, norm=norm)
        r.run(10)
        out[norm] = [r.info(p).lnz_per_site for p in range(1, 11)]
        r.close()
    np.testing.assert_allclose(out["maxabs"], out["trace"], rtol=tol)
