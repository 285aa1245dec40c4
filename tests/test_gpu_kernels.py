"""Kernel-level parity: the library's Gram, eigensolver and contraction kernels against
the FP64 oracle on the same seeded inputs (random dense T, isometries from QR).

Because the isometries are inputs here, no eigenvector gauge is involved and the new
tensors are compared element by element: for every compared (n'_1, .., n'_{d-1}) column
slice, max |got - ref| / max |ref| over the slice (tests/parity.py) must stay below the
form's bound.  Small shapes compare every slice; the full chi = 16 shape compares 16 slices
spread over the 256.
"""

import functools

import numpy as np
import scipy.linalg
import pytest

from oracle import hotrg as H
from tests import layout as LY
from tests import parity as PT
from tests import seeded_inputs as SI

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P

# Per-slice bound of max|got - ref| / max|ref| per precision form, for the seeded N(0, 1)
# tensors and QR isometries below.  Each bound is at most ten times the largest error
# measured on an MI355X over all the shapes of this file: a change that loses a term, a plane
# or a scale factor fails.  Measured maxima (MI355X, all shapes, 2D to 4D): FP64 3.3e-15, FP32
# 1.6e-6, split FP16 1.0e-6, split BF16 6.7e-6, FP16 5.2e-4, BF16 4.1e-3.
SLICE_BOUND = {P.HOTRG_FP64: 3e-14, P.HOTRG_FP32: 1.5e-5, P.HOTRG_SPLIT_FP16: 9e-6,
               P.HOTRG_SPLIT_BF16: 6e-5, P.HOTRG_FP16: 4e-3, P.HOTRG_BF16: 3e-2}
# Gram matrices (FP64 in every form): measured max 3.3e-15.
GRAM_BOUND = 3e-14
FORM_NAME = {P.HOTRG_FP64: "fp64", P.HOTRG_FP32: "fp32", P.HOTRG_SPLIT_FP16: "split_fp16",
             P.HOTRG_SPLIT_BF16: "split_bf16", P.HOTRG_FP16: "fp16", P.HOTRG_BF16: "bf16"}


def oracle_next_storage(T_paper, Us, only=None):
    d = T_paper.ndim // 2
    Tnew = H.new_tensor(T_paper, {j + 1: Us[j] for j in range(d - 1)}, only=only)
    return LY.to_storage(H.rename(Tnew))


CASES_3D = [
    # (chi_c, chi_1, chi_2), (k1, k2): several tiles, ragged M/N/K tails, degenerate k = 1
    ((8, 8, 8), (8, 8)),
    ((3, 5, 4), (7, 6)),
    ((2, 1, 3), (1, 2)),
    ((4, 4, 2), (16, 4)),
]
CASES_2D = [((8, 8), (16,)), ((5, 7), (9,)), ((32, 32), (32,))]
# 4D: b = chi1 chi2 chi3 a multiple of 8, of 4 only, and odd (the three store widths of the prime
# chain); every dim <= 8 (register width 8) and some dim above 8 (width 12), with chi3 a multiple
# of 4 (16-byte loads in the non-prime chain) and not
CASES_4D = [((2, 3, 2, 2), (4, 3, 2)), ((3, 2, 3, 2), (4, 4, 4)), ((4, 4, 4, 4), (7, 7, 7)),
            ((3, 3, 3, 3), (5, 6, 7)), ((2, 12, 2, 4), (12, 4, 12)), ((2, 9, 3, 10), (12, 9, 11))]


def _random_case(dims, kdims, seed):
    d = len(dims)
    # storage order dims: (c, n1, .., c', n1', ..)
    shape_storage = tuple(dims) * 2
    Ts = SI.random_tensor(shape_storage, seed=seed)
    Us = [SI.random_isometry(dims[j + 1] ** 2, kdims[j], seed=seed + 1 + j) for j in range(d - 1)]
    return Ts, Us


@functools.lru_cache(maxsize=None)
def _small_reference(dims, kdims, seed):
    Ts, Us = _random_case(dims, kdims, seed)
    return Ts, Us, oracle_next_storage(LY.to_paper(Ts), Us)


def _check_all_slices(form, dims, kdims, seed):
    Ts, Us, ref = _small_reference(dims, kdims, seed)
    got = gu.contract(Ts, Us, list(kdims), form)
    picks = PT.spread_picks(kdims, 10 ** 9)              # every slice
    worst, errs = PT.worst_slice_error(got, ref, picks)
    print(f"{FORM_NAME[form]} dims={dims} k={kdims}: {len(picks)} slices, max slice error {worst:.2e} "
          f"(bound {SLICE_BOUND[form]:.0e})")
    assert worst < SLICE_BOUND[form]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


@pytest.mark.parametrize("dims,kdims", CASES_3D + CASES_2D + CASES_4D)
def test_contract_fp64_matches_oracle(dims, kdims):
    _check_all_slices(P.HOTRG_FP64, dims, kdims, seed=0)


@pytest.mark.parametrize("form", [P.HOTRG_FP32, P.HOTRG_SPLIT_FP16, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16,
                                  P.HOTRG_BF16])
@pytest.mark.parametrize("dims,kdims", [((8, 8, 8), (8, 8)), ((3, 5, 4), (7, 6)), ((8, 8), (16,)),
                                       ((3, 12, 12), (12, 12)), ((2, 12, 12), (12, 12)),
                                       ((3, 3, 3, 3), (4, 4, 4)), ((2, 12, 2, 4), (12, 4, 12))])
def test_contract_forms_match_oracle(form, dims, kdims):
    # (3, 12, 12): chi = 12 with an odd number of c, the 256 x 256 GEMM and a separate non-prime
    # kernel; (2, 12, 12): the 288 x 288 GEMM with the non-prime chain in its epilogue
    _check_all_slices(form, dims, kdims, seed=3)


FULL_DIMS, FULL_K, FULL_SEED = (16, 16, 16), (16, 16), 8
FULL_PICKS = PT.spread_picks(FULL_K, 16)


@functools.lru_cache(maxsize=None)
def _full_reference():
    """chi = 16 in 3D (the bottleneck at full size, M = K = 4096): the oracle computes only the
    16 picked (n'_1, n'_2) slices of the new tensor."""
    Ts, Us = _random_case(FULL_DIMS, FULL_K, FULL_SEED)
    return Ts, Us, oracle_next_storage(LY.to_paper(Ts), Us, only=FULL_PICKS)


@pytest.mark.parametrize("form", [P.HOTRG_FP64, P.HOTRG_SPLIT_FP16, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16,
                                  P.HOTRG_FP32, P.HOTRG_BF16])
def test_contract_full_size_sampled(form):
    """chi = 16 in 3D through the production kernels of each form (for the reduced forms the
    non-prime chain runs in the GEMM epilogue at this size): 16 spread (n'_1, n'_2) slices of
    the new tensor against the oracle, element by element."""
    Ts, Us, ref = _full_reference()
    got = gu.contract(Ts, Us, list(FULL_K), form)
    worst, errs = PT.worst_slice_error(got, ref, FULL_PICKS)
    print(f"{FORM_NAME[form]} full size, 16 slices: max slice error {worst:.2e} (bound {SLICE_BOUND[form]:.0e}); "
          "per slice " + " ".join(f"{e:.1e}" for e in errs))
    assert worst < SLICE_BOUND[form]


FULL4D_DIMS, FULL4D_K, FULL4D_SEED = (8, 8, 8, 8), (8, 8, 8), 14
FULL4D_PICKS = PT.spread_picks(FULL4D_K, 8)


@functools.lru_cache(maxsize=None)
def _full4d_reference():
    Ts, Us = _random_case(FULL4D_DIMS, FULL4D_K, FULL4D_SEED)
    return Ts, Us, oracle_next_storage(LY.to_paper(Ts), Us, only=FULL4D_PICKS)


@pytest.mark.parametrize("form", [P.HOTRG_SPLIT_FP16, P.HOTRG_FP64, P.HOTRG_FP32, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16,
                                  P.HOTRG_BF16])
def test_contract_4d_full_size_sampled(form):
    """4D chi = 8 (M = K = 4096, the three-leg prime and non-prime chains, the 256 x 256 GEMM):
    8 spread (n'_1, n'_2, n'_3) slices of the new tensor against the oracle, element by element."""
    Ts, Us, ref = _full4d_reference()
    got = gu.contract(Ts, Us, list(FULL4D_K), form)
    worst, errs = PT.worst_slice_error(got, ref, FULL4D_PICKS)
    print(f"{FORM_NAME[form]} 4D chi=8 full size, 8 slices: max slice error {worst:.2e} "
          f"(bound {SLICE_BOUND[form]:.0e}); per slice " + " ".join(f"{e:.1e}" for e in errs))
    assert worst < SLICE_BOUND[form]


CHI10_4D_DIMS, CHI10_4D_K, CHI10_4D_SEED = (10, 10, 10, 10), (10, 10, 10), 21
CHI10_4D_PICKS = PT.spread_picks(CHI10_4D_K, 3)


@functools.lru_cache(maxsize=None)
def _chi10_4d_reference():
    Ts, Us = _random_case(CHI10_4D_DIMS, CHI10_4D_K, CHI10_4D_SEED)
    return Ts, Us, oracle_next_storage(LY.to_paper(Ts), Us, only=CHI10_4D_PICKS)


@pytest.mark.parametrize("form", [P.HOTRG_SPLIT_FP16, P.HOTRG_FP64, P.HOTRG_FP32])
def test_contract_4d_chi10_sampled(form):
    """4D chi = 10 (M = K = 10^4, ragged 256 x 256 tiles; the chain kernels at register width 12
    with chi3 not a multiple of 4): 3 spread (n'_1, n'_2, n'_3) slices against the oracle."""
    Ts, Us, ref = _chi10_4d_reference()
    got = gu.contract(Ts, Us, list(CHI10_4D_K), form)
    worst, errs = PT.worst_slice_error(got, ref, CHI10_4D_PICKS)
    print(f"{FORM_NAME[form]} 4D chi=10, 3 slices: max slice error {worst:.2e} (bound {SLICE_BOUND[form]:.0e}); "
          "per slice " + " ".join(f"{e:.1e}" for e in errs))
    assert worst < SLICE_BOUND[form]


FULL12_DIMS, FULL12_K, FULL12_SEED = (12, 12, 12), (12, 12), 12
FULL12_PICKS = PT.spread_picks(FULL12_K, 16)


@functools.lru_cache(maxsize=None)
def _full12_reference():
    Ts, Us = _random_case(FULL12_DIMS, FULL12_K, FULL12_SEED)
    return Ts, Us, oracle_next_storage(LY.to_paper(Ts), Us, only=FULL12_PICKS)


@pytest.mark.parametrize("form", [P.HOTRG_SPLIT_FP16, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16, P.HOTRG_FP32, P.HOTRG_BF16])
def test_contract_chi12_full_size_sampled(form):
    """chi = 12 in 3D (M = K = 1728, the sweep's 3D shape): the reduced forms run the 288 x 288
    GEMM with the non-prime chain in its epilogue; 16 spread (n'_1, n'_2) slices of the new
    tensor against the oracle, element by element."""
    Ts, Us, ref = _full12_reference()
    got = gu.contract(Ts, Us, list(FULL12_K), form)
    worst, errs = PT.worst_slice_error(got, ref, FULL12_PICKS)
    print(f"{FORM_NAME[form]} chi=12 full size, 16 slices: max slice error {worst:.2e} "
          f"(bound {SLICE_BOUND[form]:.0e}); per slice " + " ".join(f"{e:.1e}" for e in errs))
    assert worst < SLICE_BOUND[form]


@pytest.mark.parametrize("dims", [(4, 4, 4), (3, 5, 2), (8, 8, 8), (12, 12, 12), (8, 8), (16, 24), (32, 32),
                                  (3, 4, 3, 2), (8, 8, 8, 8)])
def test_gram_matches_oracle(dims):
    # (16, 24) and (32, 32): Gram matrices of size 576 and 1024, third step as a GEMM;
    # (12, 12, 12) and (32, 32): first two steps on the 256 x 128 FP64 tiles (ragged rows: 144 of 256)
    d = len(dims)
    Ts = SI.random_tensor(tuple(dims) * 2, seed=5)
    Tp = LY.to_paper(Ts)
    for j in range(1, d):
        for side in (0, 1):
            ax = H.axis_n(d, j) if side == 0 else H.axis_np(d, j)
            ref = H.gram_matrix(Tp, ax)
            got = gu.gram(Ts, j, side)
            err = PT.slice_error(got, ref)
            print(f"gram dims={dims} j={j} side={side} max|dA|/max|A|={err:.3e}")
            assert err < GRAM_BOUND


@pytest.mark.parametrize("n", [1, 2, 7, 64, 144, 256])
def test_eigh_matches_library(n):
    rng = np.random.default_rng(n)
    batch = 2
    # PSD with a fast-decaying spectrum like the Gram matrices, plus one exact degeneracy
    A = np.zeros((batch, n, n))
    for b in range(batch):
        Q = SI.random_isometry(n, n, seed=100 + n + b)
        lam = np.exp(-0.35 * np.arange(n)) * (1 + 0.1 * rng.random(n))
        if n > 3:
            lam[2] = lam[3]
        A[b] = (Q * lam) @ Q.T
        A[b] = 0.5 * (A[b] + A[b].T)
    w, V = gu.eigh(A.copy())
    for b in range(batch):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        assert np.all(np.diff(w[b]) <= 0)
        # backward-stable eigensolver: |dlambda| <= c n u ||A||_2 (c = 2)
        np.testing.assert_allclose(w[b], ref, rtol=0, atol=2 * n * 2.0 ** -52 * abs(ref[0]))
        # residual and orthogonality
        R = A[b] @ V[b] - V[b] * w[b][None, :]
        assert np.linalg.norm(R) < 1e-13 * abs(ref[0]) * n
        assert np.linalg.norm(V[b].T @ V[b] - np.eye(n)) < 1e-13 * n


@pytest.mark.parametrize("n,kvec", [(256, 16), (576, 24), (1024, 32), (200, 40), (256, 64)])
def test_eigh_leading_vectors_match_library(n, kvec):
    """The solver of a truncating step: only the leading kvec eigenvectors (n >= 128 and 7 kvec <= n:
    the kernels spread over many workgroups; (200, 40) and (256, 64): the one-workgroup solver).
    Leading eigenvalues, the sum of the unresolved ones, residuals and orthonormality of the
    vectors, and the kept subspace against LAPACK."""
    rng = np.random.default_rng(n + kvec)
    batch = 2
    A = np.zeros((batch, n, n))
    for b in range(batch):
        Q = SI.random_isometry(n, n, seed=300 + n + b)
        lam = np.exp(-0.35 * np.arange(n)) * (1 + 0.1 * rng.random(n))
        lam[2] = lam[3]                                  # an exact doublet
        lam[kvec + 3] = lam[kvec + 4]
        A[b] = (Q * lam) @ Q.T
        A[b] = 0.5 * (A[b] + A[b].T)
    w, tail, V = gu.eigh_lead(A.copy(), kvec)
    nev = n if n <= 256 else max(kvec + 1, 24)
    u = 2.0 ** -52
    for b in range(batch):
        ref, Vr = np.linalg.eigh(A[b])
        ref, Vr = ref[::-1], Vr[:, ::-1]
        np.testing.assert_allclose(w[b, :nev], ref[:nev], rtol=0, atol=2 * n * u * abs(ref[0]))
        assert np.all(w[b, nev:] == 0.0)
        assert abs(tail[b] - ref[nev:].sum()) <= 4 * n * u * (abs(ref[0]) + np.trace(A[b]))
        res = np.linalg.norm(A[b] @ V[b] - V[b] * w[b, :kvec][None, :])
        orth = np.linalg.norm(V[b].T @ V[b] - np.eye(kvec))
        gap = ref[kvec - 1] - ref[kvec]
        sub = np.linalg.norm(V[b] @ V[b].T - Vr[:, :kvec] @ Vr[:, :kvec].T)
        print(f"n={n} kvec={kvec}: residual {res:.1e}, orthogonality {orth:.1e}, subspace {sub:.1e} "
              f"(gap {gap:.1e}), tail {tail[b]:.6e} vs {ref[nev:].sum():.6e}")
        assert res < 1e-13 * abs(ref[0]) * n
        assert orth < 1e-13 * n
        assert sub < 100 * n * u * abs(ref[0]) / gap


@pytest.mark.parametrize("form", ["dense", "tridiagonal"])
@pytest.mark.parametrize("n,kvec", [(256, 16), (576, 24), (120, 16)])
def test_eigh_rank_deficient_gram(n, kvec, form):
    """Fewer non-negligible eigenvalues than kept vectors (the Gram matrices of an ordered phase):
    the kept vectors past the rank lie in the near-null space, where inverse iteration alone can
    miss (shifts far below the pivot floor, growth compounding over runs of tiny pivots) and
    leave rounding noise on the leading eigenvectors, or NaN; the solver must still return
    orthonormal eigenvectors within the residual bound that span the non-negligible part.
    "tridiagonal": the same matrices reduced by scipy's Householder, passed as they are (a column
    with nothing below the subdiagonal takes no reflection, so the eigenpair stage sees exactly
    these diagonals); without the repair of vectors above the residual bound the spread solver
    reported a numeric failure on (n, m, sectors, seed) = (256, 5, 1, 13), (256, 4, 2, 17) and
    (576, 4, 2, 17).  (256, 16) and (576, 24): the solver spread over many workgroups; (120, 16):
    the one-workgroup solver."""
    u = 2.0 ** -52
    cases = [(3, 1, 11), (4, 1, 12), (5, 1, 13), (4, 1, 14), (3, 2, 15), (5, 3, 16), (4, 2, 17), (3, 1, 18)]
    for start in range(0, len(cases), 4):
        part = cases[start:start + 4]
        A = np.stack([SI.rank_deficient_gram(n, m, s, seed) for m, s, seed in part])
        if form == "tridiagonal":
            for b in range(len(part)):
                H = scipy.linalg.hessenberg(A[b])
                d, e = np.diag(H), np.diag(H, -1)
                A[b] = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        print(f"n={n} kvec={kvec} {form} (m, sectors, seed) = {part}", flush=True)
        w, tail, V = gu.eigh_lead(A.copy(), kvec)
        nev = n if n <= 256 else max(kvec + 1, 24)
        for b, (m, s, seed) in enumerate(part):
            ref, Vr = np.linalg.eigh(A[b])
            ref, Vr = ref[::-1], Vr[:, ::-1]
            np.testing.assert_allclose(w[b, :nev], ref[:nev], rtol=0, atol=2 * n * u * abs(ref[0]))
            rank = int(np.sum(ref > 1e-12 * ref[0]))
            assert rank == s < kvec
            res = np.linalg.norm(A[b] @ V[b] - V[b] * w[b, :kvec][None, :])
            orth = np.linalg.norm(V[b].T @ V[b] - np.eye(kvec))
            lead = Vr[:, :rank]
            miss = np.linalg.norm(lead - V[b] @ (V[b].T @ lead))
            print(f"  m={m} sectors={s} seed={seed}: residual {res:.1e}, orthogonality {orth:.1e}, "
                  f"leading span missed {miss:.1e}")
            assert res < 1e-13 * abs(ref[0]) * n
            assert orth < 1e-13 * n
            assert miss < 100 * n * u


def _near_tridiagonal(n, eps, seed):
    rng = np.random.default_rng(seed)
    B = np.diag(2 + rng.random(n)) + np.diag(0.5 * rng.random(n - 1), 1)
    B = B + np.triu(B, 1).T
    N = rng.standard_normal((n, n)) * eps
    return B + (N + N.T) / 2


def _gram_with_null_index(chi, seed):
    # Gram matrix of a bond with one null index (a multiplet dropped at the previous cut):
    # rows and columns (a, b) with a or b = chi - 1 are exactly zero
    n = chi * chi
    Q = SI.random_isometry(n, n, seed=seed)
    lam = np.exp(-0.05 * np.arange(n))
    lam[1::7] = lam[0::7][: lam[1::7].size]          # exact doublets
    A = (Q * lam) @ Q.T
    null = [a * chi + b for a in range(chi) for b in range(chi) if a == chi - 1 or b == chi - 1]
    A[null, :] = 0.0
    A[:, null] = 0.0
    return 0.5 * (A + A.T)


@pytest.mark.parametrize("case", ["near_tridiagonal_1e-10", "near_tridiagonal_1e-11", "gram_null_index"])
def test_eigh_structured_matrices(case):
    """Matrices whose Householder columns have a dominant subdiagonal entry and a tail below
    sqrt(u) of it (the tail norm must not be taken by cancellation), and a Gram matrix with
    exactly zero rows and columns."""
    n = 256
    if case.startswith("near"):
        A = _near_tridiagonal(n, float(case.split("_")[-1]), seed=7)
    else:
        A = _gram_with_null_index(16, seed=11)
    w, V = gu.eigh(A[None].copy())
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    err = np.max(np.abs(w[0] - ref)) / abs(ref[0])
    print(f"{case}: max |dlambda| / |lambda_0| = {err:.2e}")
    assert err <= 2 * n * 2.0 ** -52
    R = A @ V[0] - V[0] * w[0][None, :]
    assert np.linalg.norm(R) < 1e-13 * abs(ref[0]) * n
    assert np.linalg.norm(V[0].T @ V[0] - np.eye(n)) < 1e-13 * n
