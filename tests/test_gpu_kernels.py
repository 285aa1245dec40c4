"""Kernel-level parity: the library's Gram, eigensolver and contraction kernels against
the FP64 oracle on the same seeded inputs (random dense T, isometries from QR).

Because the isometries are inputs here, no eigenvector gauge is involved and the new
tensors are compared element by element (normwise relative error).
"""

import numpy as np
import pytest

from oracle import hotrg as H
from tests import layout as LY
from tests import seeded_inputs as SI

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P

# Normwise relative tolerance of the new tensor per form ("Parity tolerances"):
# tol = C * u_form * sqrt(K) with K = H the bottleneck contraction length, C = 16.
U_FORM = {P.HOTRG_FP64: 2.0 ** -53, P.HOTRG_FP32: 2.0 ** -24, P.HOTRG_SPLIT_FP16: 2.0 ** -21,
          P.HOTRG_SPLIT_BF16: 2.0 ** -16, P.HOTRG_FP16: 2.0 ** -11, P.HOTRG_BF16: 2.0 ** -8}


def tol(form, Hdim):
    return 16.0 * U_FORM[form] * np.sqrt(Hdim)


def oracle_next_storage(T_paper, Us):
    d = T_paper.ndim // 2
    Tnew = H.new_tensor(T_paper, {j + 1: Us[j] for j in range(d - 1)})
    return LY.to_storage(H.rename(Tnew))


CASES_3D = [
    # (chi_c, chi_1, chi_2), (k1, k2): several tiles, ragged M/N/K tails, degenerate k = 1
    ((8, 8, 8), (8, 8)),
    ((3, 5, 4), (7, 6)),
    ((2, 1, 3), (1, 2)),
    ((4, 4, 2), (16, 4)),
]
CASES_2D = [((8, 8), (16,)), ((5, 7), (9,)), ((32, 32), (32,))]


def _random_case(dims, kdims, seed):
    d = len(dims)
    # storage order dims: (c, n1, .., c', n1', ..)
    shape_storage = tuple(dims) * 2
    Ts = SI.random_tensor(shape_storage, seed=seed)
    Us = [SI.random_isometry(dims[j + 1] ** 2, kdims[j], seed=seed + 1 + j) for j in range(d - 1)]
    return Ts, Us


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


@pytest.mark.parametrize("dims,kdims", CASES_3D + CASES_2D)
def test_contract_fp64_matches_oracle(dims, kdims):
    Ts, Us = _random_case(dims, kdims, seed=0)
    ref = oracle_next_storage(LY.to_paper(Ts), Us)
    got = gu.contract(Ts, Us, list(kdims), P.HOTRG_FP64)
    Hd = int(np.prod(dims))
    err = gu.relerr(got, ref)
    print(f"fp64 dims={dims} k={kdims} relerr={err:.3e}")
    assert err < tol(P.HOTRG_FP64, Hd)


@pytest.mark.parametrize("form", [P.HOTRG_FP32, P.HOTRG_SPLIT_FP16, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16,
                                  P.HOTRG_BF16])
@pytest.mark.parametrize("dims,kdims", [((8, 8, 8), (8, 8)), ((3, 5, 4), (7, 6)), ((8, 8), (16,)),
                                       ((3, 12, 12), (12, 12))])
def test_contract_forms_match_oracle(form, dims, kdims):
    Ts, Us = _random_case(dims, kdims, seed=3)
    ref = oracle_next_storage(LY.to_paper(Ts), Us)
    got = gu.contract(Ts, Us, list(kdims), form)
    Hd = int(np.prod(dims))
    err = gu.relerr(got, ref)
    print(f"form={form} dims={dims} k={kdims} relerr={err:.3e} tol={tol(form, Hd):.1e}")
    assert err < tol(form, Hd)


def test_contract_full_size_sampled():
    """chi = 16 in 3D (the bottleneck at full size, M = K = 4096): the oracle computes
    only a few (n'_1, n'_2) slices of the new tensor; compare those element by element."""
    dims, kdims = (16, 16, 16), (16, 16)
    Ts, Us = _random_case(dims, kdims, seed=7)
    Tp = LY.to_paper(Ts)
    got = gu.contract(Ts, Us, list(kdims), P.HOTRG_FP64)
    picks = [(0, 0), (15, 15), (3, 11)]
    Tnew = H.new_tensor(Tp, {1: Us[0], 2: Us[1]}, only=picks)
    ref = LY.to_storage(H.rename(Tnew))
    # T^next storage [n1][n2][c][n1'][n2'][c']: compare the picked (n1', n2') columns
    for (n1p, n2p) in picks:
        g = got[:, :, :, n1p, n2p, :]
        r = ref[:, :, :, n1p, n2p, :]
        err = gu.relerr(g, r)
        print(f"full-size slice ({n1p},{n2p}) relerr={err:.3e}")
        assert err < tol(P.HOTRG_FP64, 4096)


@pytest.mark.parametrize("form", [P.HOTRG_SPLIT_FP16, P.HOTRG_SPLIT_BF16, P.HOTRG_FP16, P.HOTRG_FP32])
def test_contract_forms_full_size_sampled(form):
    """chi = 16 in 3D through the production kernels of each form (for the 16-bit forms the
    non-prime chain runs in the GEMM epilogue at this size); sampled slices vs the oracle."""
    dims, kdims = (16, 16, 16), (16, 16)
    Ts, Us = _random_case(dims, kdims, seed=8)
    Tp = LY.to_paper(Ts)
    got = gu.contract(Ts, Us, list(kdims), form)
    picks = [(0, 0), (15, 15), (7, 2)]
    ref = LY.to_storage(H.rename(H.new_tensor(Tp, {1: Us[0], 2: Us[1]}, only=picks)))
    for (n1p, n2p) in picks:
        err = gu.relerr(got[:, :, :, n1p, n2p, :], ref[:, :, :, n1p, n2p, :])
        print(f"form={form} full-size slice ({n1p},{n2p}) relerr={err:.3e} tol={tol(form, 4096):.1e}")
        assert err < tol(form, 4096)


@pytest.mark.parametrize("dims", [(4, 4, 4), (3, 5, 2), (8, 8, 8), (12, 12, 12), (8, 8), (16, 24), (32, 32)])
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
            err = gu.relerr(got, ref)
            print(f"gram dims={dims} j={j} side={side} relerr={err:.3e}")
            assert err < 1e-13


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
