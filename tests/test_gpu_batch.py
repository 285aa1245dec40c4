"""Batched runs (hotrg_batch_*): every instance of a batch equals the same run made alone,
step by step, including the steps replayed from the recorded HIP graphs; and the sweep
of independent 3D and 2D instances against the oracle on sampled instances."""

import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P
from tests import seeded_inputs as SI  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


MIXED = [("ising", 3, 1 / 4.0, 6, None), ("ising", 3, 1 / 4.5115, 6, None), ("potts", 3, 0.55, 9, 3),
         ("ising", 2, 0.44, 8, None), ("ising", 2, 0.30, 12, None), ("ising", 2, 0.5, 16, None)]


def single_run(kind, d, beta, chi, q, steps, precision):
    r = P.HOTRG(kind, d, beta, chi, q=q, precision=precision, max_steps=steps)
    out = []
    for _ in range(steps):
        r.step()
        out.append(r.log_z())
    r.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_batch_equals_single_runs_step_by_step(precision):
    steps = 12
    inst = [P.make_instance(k, d, b, c, q=q) for k, d, b, c, q in MIXED]
    bt = P.HOTRGBatch(inst, precision=precision, max_steps=steps)
    got = []
    for _ in range(steps):
        bt.step()
        got.append(bt.log_z())          # eager synchronisation between graph replays
    graphs, eager = bt.graph_stats()
    bt.close()
    print(f"batch {precision}: {graphs} steps as graph launches, {eager} enqueued kernel by kernel")
    assert graphs >= steps - 6 and graphs + eager == steps
    for i, (k, d, b, c, q) in enumerate(MIXED):
        ref = single_run(k, d, b, c, q, steps, precision)
        for p in range(steps):
            assert got[p][i] == ref[p], (i, p + 1, got[p][i], ref[p])


def test_batch_records_match_single_run():
    steps = 8
    inst = [P.make_instance(k, d, b, c, q=q) for k, d, b, c, q in MIXED[:3]]
    bt = P.HOTRGBatch(inst, precision="fp64", max_steps=steps)
    bt.run(steps)
    r = P.HOTRG("potts", 3, 0.55, 9, q=3, max_steps=steps)
    r.run(steps)
    for p in range(1, steps + 1):
        a, b = bt.info(2, p), r.info(p)
        assert a.p == b.p == p and a.axis == b.axis == (p - 1) % 3
        assert list(a.kept) == list(b.kept) and list(a.chose_prime) == list(b.chose_prime)
        assert a.trace == b.trace
    r.close()
    bt.close()


def config4_instances():
    c3, c2 = SI.CONFIG4_3D, SI.CONFIG4_2D
    inst = [P.make_instance("ising", 3, 1.0 / T, c3["chi"]) for T in c3["temps"]]
    inst += [P.make_instance("ising", 2, float(b), c2["chis"][i % len(c2["chis"])]) for i, b in enumerate(c2["betas"])]
    return inst


@pytest.mark.parametrize("precision,bound", [("split_fp16", 1e-5), ("fp64", 1e-10)])
def test_config4_sweep_against_oracle(precision, bound):
    """64 x 3D Ising chi = 12 (T = linspace(4, 5, 64)) and 48 x 2D Ising (beta = linspace(0.3,
    0.6, 48), chi round-robin 16, 24, 32), 20 steps, as one batch; sampled instances against
    the oracle after every step.  Split FP16: 1e-5 over the sweep.  In the ordered phase
    (T = 4.0 in 3D, beta near 0.6 in 2D) even/odd pairs of Gram eigenvalues come within the
    form's noise floor of each other at some cuts; the split form then drops the pair where
    FP64 keeps it (or the reverse), which moves lnZ/V by a few 1e-6 at that step (printed:
    the steps where the kept counts differ)."""
    path = os.path.join(GOLDEN, "config4.json")
    if not os.path.exists(path):
        pytest.skip("config4 fixture not generated")
    fx = json.load(open(path))
    inst = config4_instances()
    steps = SI.CONFIG4_3D["steps"]
    bt = P.HOTRGBatch(inst, precision=precision, max_steps=steps)
    lnz = []
    for p in range(steps):
        bt.step()
        lnz.append(bt.log_z())
        if (p + 1) % 5 == 0:
            print(f"  [config4 {precision}: {p + 1} steps]", flush=True)
    graphs, eager = bt.graph_stats()
    worst = 0.0
    for run in fx["runs"]:
        idx = run["index"] if run["d"] == 3 else 64 + run["index"]
        ref = [s["lnz_per_site"] for s in run["steps"]]
        per = [abs(lnz[p][idx] - ref[p]) / abs(ref[p]) for p in range(steps)]
        kept = [[bt.info(idx, p + 1).kept[j] for j in range(run["d"] - 1)] for p in range(steps)]
        kref = [[s["dirs"][str(j)]["kept"] for j in range(1, run["d"])] for s in run["steps"]]
        print(f"config4 {precision} d={run['d']} chi={run['chi']} beta={run['beta']:.6f}: max rel err {max(per):.2e}"
              f"\n  per step: " + " ".join(f"{e:.1e}" for e in per)
              + f"\n  kept differs at steps: {[p + 1 for p in range(steps) if kept[p] != kref[p]]}")
        worst = max(worst, max(per))
    bt.close()
    print(f"config4 {precision}: {graphs} graph launches, {eager} eager steps; worst {worst:.2e}")
    assert all(np.isfinite(v) for row in lnz for v in row)
    assert worst < bound


@pytest.mark.parametrize("precision", ["fp64", "split_fp16"])
def test_autotuned_batch_matches_untuned(precision):
    """The autotuner picks a GEMM tile and chunk size per (d, chi) class; FP64 results do not
    depend on that choice (bitwise), split FP16 ones only through the MFMA summation order."""
    steps = 10
    inst = [P.make_instance(k, d, b, c, q=q) for k, d, b, c, q in MIXED]
    plain = P.HOTRGBatch(inst, precision=precision, max_steps=steps)
    plain.run(steps)
    ref = plain.log_z()
    plain.close()
    tuned = P.HOTRGBatch(inst, precision=precision, max_steps=steps, tune=True)
    print(f"{precision} tuning:", tuned.tuned)
    classes = {(i.model.d, i.chi) for i in inst}
    assert {(t["d"], t["chi"]) for t in tuned.tuned} == classes
    assert all(t["chunk_pairs"] >= 1 and t["contract_ms"] > 0 for t in tuned.tuned)
    tuned.run(steps)
    got = tuned.log_z()
    tuned.close()
    for g, r in zip(got, ref):
        if precision == "fp64":
            assert g == r
        else:
            assert abs(g - r) <= 1e-6 * abs(r)
