"""The allocation-free eigensolver entry point (hotrg_eigh_noalloc, static device scratch)
against the workspace entry point it varies (hotrg_debug_eigh): identical kernels, so identical
eigenvalues and eigenvectors, on two calls in a row (the second smaller, with the first call's
contents still in the static array), a rejected oversize request, and the failure status."""

import numpy as np
import pytest
import scipy.linalg

from tests import seeded_inputs as SI

pytestmark = pytest.mark.gpu

gu = pytest.importorskip("tests.gpu_util")
P = gu.P
torch = gu.torch


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    gu.require_gpu()


def _psd_batch(n, batch, seed):
    A = np.zeros((batch, n, n))
    for b in range(batch):
        Q = SI.random_isometry(n, n, seed=seed + b)
        lam = np.exp(-0.3 * np.arange(n))
        A[b] = (Q * lam) @ Q.T
        A[b] = 0.5 * (A[b] + A[b].T)
    return A


def _noalloc(A):
    batch, n, _ = A.shape
    Ad = gu.dev(A)
    w = torch.zeros(batch * n, dtype=torch.float64, device="cuda")
    V = torch.zeros(batch * n * n, dtype=torch.float64, device="cuda")
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    P.hotrg_eigh_noalloc(n, batch, Ad.data_ptr(), w.data_ptr(), V.data_ptr(), status.data_ptr(), gu.stream_ptr())
    torch.cuda.synchronize()
    return w.cpu().numpy().reshape(batch, n), V.cpu().numpy().reshape(batch, n, n), int(status.item())


@pytest.mark.parametrize("first,second", [((256, 4), (100, 3)), ((512, 4), (144, 2))])
def test_noalloc_equals_workspace_entry_point(first, second):
    for (n, batch), seed in ((first, 30), (second, 40)):
        A = _psd_batch(n, batch, seed)
        w_ref, V_ref = gu.eigh(A.copy())
        w, V, status = _noalloc(A.copy())
        print(f"n={n} batch={batch}: max |dw| {np.max(np.abs(w - w_ref)):.1e}, max |dV| {np.max(np.abs(V - V_ref)):.1e}")
        assert status == 0
        np.testing.assert_array_equal(w, w_ref)
        np.testing.assert_array_equal(V, V_ref)


def test_noalloc_rejects_sizes_beyond_the_static_scratch():
    assert P.hotrg_eigh_noalloc_max_bytes() == 16 << 20
    n, batch = 1024, 2                                   # 32 MiB of scratch
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    dummy = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(P.HotrgError) as e:
        P.hotrg_eigh_noalloc(n, batch, dummy.data_ptr(), dummy.data_ptr(), dummy.data_ptr(), status.data_ptr(),
                             gu.stream_ptr())
    assert e.value.code == P.HOTRG_E_ARG
    torch.cuda.synchronize()
    assert int(status.item()) == 7                       # nothing was enqueued


def test_noalloc_reports_failure_in_status():
    A = np.eye(64)[None].copy()
    A[0, 3, 4] = A[0, 4, 3] = np.nan
    _, _, status = _noalloc(A)
    assert status == 1
    A = _psd_batch(64, 1, 50)
    w, _, status = _noalloc(A.copy())
    assert status == 0
    np.testing.assert_allclose(w[0], np.sort(np.linalg.eigvalsh(A[0]))[::-1], atol=1e-14)


def _tridiagonal_form(A):
    H = scipy.linalg.hessenberg(A)
    d, e = np.diag(H), np.diag(H, -1)
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


def test_noalloc_rank_deficient_gram():
    """Every eigenvector of matrices of rank 1 and 2 at n = 256 (tridiagonal forms of ordered-phase
    Gram matrices, with near-null clusters of 254 and 255 vectors): status 0, the same bits as the
    workspace entry point, and the solver's own bounds: every residual within 1e-9 |T|, and so
    every overlap with the non-negligible eigenvectors within 1e-9 |T| / gap per residual.  The
    first matrix is one on which the full solver reported a numeric failure before vectors above
    the residual bound were rebuilt."""
    n, u = 256, 2.0 ** -52
    A = np.stack([_tridiagonal_form(SI.rank_deficient_gram(n, m, s, seed)) for m, s, seed in ((5, 1, 13), (4, 2, 17))])
    w_ref, V_ref = gu.eigh(A.copy())
    w, V, status = _noalloc(A.copy())
    assert status == 0
    np.testing.assert_array_equal(w, w_ref)
    np.testing.assert_array_equal(V, V_ref)
    for b, rank in enumerate((1, 2)):
        ref = np.sort(np.linalg.eigvalsh(A[b]))[::-1]
        np.testing.assert_allclose(w[b], ref, rtol=0, atol=2 * n * u * abs(ref[0]))
        tnorm = np.abs(np.diag(A[b])).max() + 2 * np.abs(np.diag(A[b], -1)).max()
        res = np.linalg.norm(A[b] @ V[b] - V[b] * w[b][None, :], axis=0)
        orth = np.abs(V[b].T @ V[b] - np.eye(n))
        gap = ref[rank - 1]
        print(f"matrix {b}: max residual {res.max():.1e} (bound {1e-9 * tnorm:.1e}), max overlap {orth.max():.1e} "
              f"(bound {2e-9 * tnorm / gap:.1e})")
        assert res.max() <= 1e-9 * tnorm
        assert orth.max() <= 2e-9 * tnorm / gap + 1e-12
