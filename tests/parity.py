"""Element-by-element comparison of a computed tensor with the oracle's (no torch, no GPU).

The new tensor of one (n'_1, .., n'_{d-1}) column slice is compared as

    err = max |got - ref| / max |ref|       over the elements of the slice,

so that a wrong element anywhere in the slice shows, and a result that is zero, or off by
a constant factor, fails for any bound below 1.  Bounds are stated per precision form in
the tests that use this module.
"""

import numpy as np


def slice_error(got, ref):
    """max |got - ref| / max |ref| (inf if ref is all zero while got is not)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.shape != ref.shape:
        raise ValueError(f"shape mismatch {got.shape} vs {ref.shape}")
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    diff = float(np.max(np.abs(got - ref))) if ref.size else 0.0
    if not np.all(np.isfinite(got)):
        return float("inf")
    if scale == 0.0:
        return 0.0 if diff == 0.0 else float("inf")
    return diff / scale


def storage_slices(T_next_storage, picks):
    """Column slices (n'_1, .., n'_{d-1}) of a renamed new tensor in storage order
    [n_1]..[n_{d-1}][c][n'_1]..[n'_{d-1}][c']: one array per pick."""
    d = T_next_storage.ndim // 2
    out = []
    for pk in picks:
        idx = (slice(None),) * d + tuple(pk) + (slice(None),)
        out.append(T_next_storage[idx])
    return out


def worst_slice_error(got_storage, ref_storage, picks):
    """The largest slice_error over the picked column slices, and the list of all of them."""
    errs = [slice_error(g, r) for g, r in zip(storage_slices(got_storage, picks), storage_slices(ref_storage, picks))]
    return max(errs), errs


def spread_picks(ks, count):
    """`count` (n'_1, .., n'_{d-1}) tuples spread over the grid of column slices with ks[j-1]
    values of n'_j (n'_{d-1} fastest), the first and the last slice included (deterministic)."""
    ks = list(ks)
    total = int(np.prod(ks))
    if count >= total:
        flat = list(range(total))
    else:
        step = (total - 1) / (count - 1)
        flat = sorted({int(round(i * step)) for i in range(count)})
    picks = []
    for f in flat:
        t = []
        for k in reversed(ks):
            t.append(f % k)
            f //= k
        picks.append(tuple(reversed(t)))
    return picks


# ---------------------------------------------------------------------------------------
# Truncation decisions recorded in the oracle fixtures (per step, per direction j: the
# normalised spectra lambda_l / lambda_0 of A and A', the adopted side and the kept count).
# ---------------------------------------------------------------------------------------

# Eigenvalue pairs closer than this (relative to lambda_0) are resolved by rounding in any FP64
# eigensolver (its absolute accuracy is about n u lambda_0 = 2e-13 lambda_0 at n = 1024, and
# the Gram matrices themselves carry the rounding of the steps before).
ROUNDING_LEVEL = 1e-11


def _adopted_spectrum(dd):
    return dd["spec_p"] if dd["chose_prime"] else dd["spec"]


def rounding_decided_cut(dd, kept_other):
    """True when a different kept count `kept_other` and the oracle's dd["kept"] part over a pair
    of eigenvalues whose difference is at rounding level: the multiplet rule (difference at
    most 1e-10 of the pair) is then decided by the last bits of either eigensolver.  The
    disputed pair is the one at max(kept, kept_other): one side stopped there, the other
    went past it."""
    g = _gap_at(dd, max(dd["kept"], kept_other))
    return g is not None and g <= ROUNDING_LEVEL


def _gap_at(dd, k):
    """(lambda_{k-1} - lambda_k) / lambda_0 of the adopted spectrum: from the recorded spectrum
    when it reaches index k, else the recorded gap at the nominal cut chi_new when k is that cut
    (the fixtures keep the leading part of the spectrum only, so a cut at chi = 32 lies beyond
    it); None when it is not known or nothing is cut there."""
    sp = _adopted_spectrum(dd)
    if k < 1:
        return None
    if k < len(sp):
        return sp[k - 1] - sp[k]
    if k == dd["chi_new"]:
        return dd.get("gap")
    return None


def effective_gap(dd):
    """(lambda_{kept-1} - lambda_kept) / lambda_0 at the cut actually made (1.0 when nothing
    was truncated, or when the gap at the cut is not recorded)."""
    if dd.get("gap") is None:
        return 1.0
    g = _gap_at(dd, dd["kept"])
    return 1.0 if g is None else g


def conditioned_steps(run, threshold):
    """Number of leading steps of an oracle run before the first step that follows a cut with
    effective gap below `threshold`: the kept subspace moves by (perturbation of A) / gap, so
    after such a cut two correct FP64 implementations part by more than rounding."""
    for i, st in enumerate(run["steps"]):
        if min(effective_gap(dd) for dd in st["dirs"].values()) < threshold:
            return i + 1
    return len(run["steps"])


# Effective gaps (relative to lambda_0) below which the kept vector of a near-degenerate pair
# moves, under the rounding of A, by enough to change lnZ/V at the bound of the form: the
# subspace rotates by about (perturbation of A) / gap.  FP64: cuts with gaps of 3e-11 to 5e-9
# lambda_0 part two FP64 implementations by 4e-10 to 6e-10 within a few steps (2D Ising chi =
# 16 at beta = 0.357, 0.415, 0.434), so 1e-7 leaves a margin.  Split FP16 (A perturbed at about
# 1e-7 relative): after cuts with gaps of 7e-6 the 3D chi = 12 run at T = 4.19 parts from the
# oracle by 1.1e-6 at step 13.
SUBSPACE_LEVEL = {"fp64": 1e-7, "split_fp16": 1e-5}


def first_cut_below(run, threshold):
    """First step (1-based) whose cut has an effective gap at or below `threshold` (relative to
    lambda_0); len(steps) + 1 if there is none."""
    for i, st in enumerate(run["steps"]):
        if min(effective_gap(dd) for dd in st["dirs"].values()) <= threshold:
            return i + 1
    return len(run["steps"]) + 1
