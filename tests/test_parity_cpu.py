"""The comparison used by the GPU parity tests can fail (CPU only): a zeroed, rescaled or
locally wrong new tensor is rejected at the bounds the GPU tests use, and the oracle's
sampled contraction (only=) equals its full contraction on the sampled slices."""

import numpy as np
import pytest

from oracle import hotrg as H
from tests import layout as LY
from tests import parity as PT
from tests import seeded_inputs as SI

# the loosest per-slice bound any GPU parity test applies to a contraction (BF16 form)
LOOSEST_BOUND = 3e-2


def _case(dims, kdims, seed):
    d = len(dims)
    Ts = SI.random_tensor(tuple(dims) * 2, seed=seed)
    Us = [SI.random_isometry(dims[j + 1] ** 2, kdims[j], seed=seed + 1 + j) for j in range(d - 1)]
    ref = LY.to_storage(H.rename(H.new_tensor(LY.to_paper(Ts), {j + 1: Us[j] for j in range(d - 1)})))
    return ref


@pytest.mark.parametrize("dims,kdims", [((3, 5, 4), (7, 6)), ((5, 7), (9,))])
def test_zeroed_rescaled_or_perturbed_output_fails(dims, kdims):
    ref = _case(dims, kdims, seed=3)
    d = len(dims)
    picks = PT.spread_picks(kdims, 4)
    assert PT.worst_slice_error(ref, ref, picks)[0] == 0.0
    assert PT.worst_slice_error(np.zeros_like(ref), ref, picks)[0] == pytest.approx(1.0)
    assert PT.worst_slice_error(1.1 * ref, ref, picks)[0] > LOOSEST_BOUND
    bad = ref.copy()
    sl = (0,) * d + picks[-1] + (0,)
    bad[sl] += 0.05 * np.max(np.abs(ref))            # one element of one slice
    worst, errs = PT.worst_slice_error(bad, ref, picks)
    assert worst > LOOSEST_BOUND and sum(e > 0 for e in errs) == 1
    nan = ref.copy()
    nan[sl] = np.nan
    assert PT.worst_slice_error(nan, ref, picks)[0] == float("inf")


def test_spread_picks_cover_the_grid():
    p = PT.spread_picks((16, 16), 16)
    assert len(p) == 16 and len(set(p)) == 16
    assert p[0] == (0, 0) and p[-1] == (15, 15)
    assert all(0 <= a < 16 and 0 <= b < 16 for a, b in p)
    assert len({a for a, _ in p}) >= 8              # spread over n'_1, not one row
    assert PT.spread_picks((5,), 99) == [(i,) for i in range(5)]
    assert PT.spread_picks((7, 6), 42)[-1] == (6, 5)


@pytest.mark.parametrize("dims,kdims,picks", [
    ((3, 5, 4), (7, 6), [(0, 0), (6, 5), (2, 3)]),
    ((4, 3, 3), (9, 2), [(8, 1), (0, 1)]),
    ((5, 7), (9,), [(0,), (4,), (8,)]),
])
def test_oracle_sampled_contraction_equals_full(dims, kdims, picks):
    """new_tensor(..., only=picks) computes exactly the picked (n'_1, .., n'_{d-1}) slices of the
    full contraction (same arithmetic, bitwise) and leaves every other slice zero."""
    d = len(dims)
    Tp = LY.to_paper(SI.random_tensor(tuple(dims) * 2, seed=11))
    Us = {j + 1: SI.random_isometry(dims[j + 1] ** 2, kdims[j], seed=12 + j) for j in range(d - 1)}
    full = H.new_tensor(Tp, Us)
    part = H.new_tensor(Tp, Us, only=picks)
    # paper order T^new[n_{d-1}..n_1, n'_{d-1}..n'_1, c, c']: slice (n'_1, .., n'_{d-1})
    mask = np.zeros(full.shape, dtype=bool)
    for pk in picks:
        idx = (slice(None),) * (d - 1) + tuple(reversed(pk)) + (slice(None), slice(None))
        mask[idx] = True
        np.testing.assert_array_equal(part[idx], full[idx])
    assert np.all(part[~mask] == 0.0)
    assert np.any(full[~mask] != 0.0)


def _dir(spec, kept, chi_new, gap=0.1):
    return dict(spec=spec, spec_p=spec, chose_prime=False, kept=kept, chi_new=chi_new, gap=gap)


def test_rounding_decided_cut_and_gaps():
    # an exact pair at positions 2, 3 straddling the nominal cut chi_new = 3: the oracle drops it
    # (kept 2); an implementation that keeps 3 parts from it over a pair 1e-17 apart
    dd = _dir([1.0, 0.3, 1e-6, 1e-6 - 1e-17, 1e-9], kept=2, chi_new=3)
    assert PT.rounding_decided_cut(dd, 3)
    assert not PT.rounding_decided_cut(_dir([1.0, 0.3, 2e-6, 1e-6, 1e-9], kept=3, chi_new=3), 2)
    assert PT.effective_gap(dd) == pytest.approx(0.3 - 1e-6)
    assert PT.effective_gap(_dir([1.0, 0.5], kept=2, chi_new=2, gap=None)) == 1.0
    run = {"steps": [{"dirs": {"1": _dir([1.0, 0.5, 0.1], 2, 2)}},
                     {"dirs": {"1": _dir([1.0, 0.5, 0.5 - 1e-7], 2, 2)}},
                     {"dirs": {"1": _dir([1.0, 0.5, 0.1], 2, 2)}}]}
    assert PT.conditioned_steps(run, 1e-5) == 2
    assert PT.conditioned_steps(run, 1e-8) == 3


def test_cut_beyond_the_recorded_spectrum():
    # the fixtures record the leading eigenvalues only: a cut at chi_new past them is judged by
    # the gap recorded at that cut, any other cut there is unknown (never rounding-decided)
    dd = _dir([1.0, 0.5, 0.2], kept=4, chi_new=4, gap=2.7e-13)
    assert PT.rounding_decided_cut(dd, 2)
    assert PT.effective_gap(dd) == 2.7e-13
    assert not PT.rounding_decided_cut(_dir([1.0, 0.5, 0.2], kept=4, chi_new=4, gap=1e-9), 2)
    assert PT.effective_gap(_dir([1.0, 0.5, 0.2], kept=4, chi_new=4, gap=1e-9)) == 1e-9
    dd = _dir([1.0, 0.5, 0.2], kept=3, chi_new=4, gap=1e-14)
    assert not PT.rounding_decided_cut(dd, 2)
    assert PT.effective_gap(dd) == 1.0
    run = {"steps": [{"dirs": {"1": _dir([1.0, 0.5, 0.1], 4, 4, gap=0.05)}},
                     {"dirs": {"1": _dir([1.0, 0.5, 0.1], 4, 4, gap=2e-12)}}]}
    assert PT.first_cut_below(run, PT.SUBSPACE_LEVEL["fp64"]) == 2
    assert PT.conditioned_steps(run, PT.SUBSPACE_LEVEL["fp64"]) == 2


def test_first_cut_below():
    run = {"steps": [{"dirs": {"1": _dir([1.0, 0.5, 0.1], 2, 2)}},
                     {"dirs": {"1": _dir([1.0, 2e-5, 2e-5 - 1e-14], 2, 2)}}]}
    assert PT.first_cut_below(run, PT.SUBSPACE_LEVEL["fp64"]) == 2
    assert PT.first_cut_below({"steps": run["steps"][:1]}, PT.SUBSPACE_LEVEL["fp64"]) == 2
