"""Shared helpers of the GPU tests: torch buffers and calls through the C ABI."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_03607_amd as P  # noqa: E402


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def workspace(nbytes):
    w = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device="cuda")
    base = w.data_ptr()
    return w, (base + 255) // 256 * 256


def stream_ptr():
    return torch.cuda.current_stream().cuda_stream


def contract(T_storage, Us, kdims, form):
    """hotrg_debug_contract: T (storage order) and isometries -> renamed T^next (storage order)."""
    d = T_storage.ndim // 2
    dims = list(T_storage.shape[:d])
    nbytes = P.hotrg_debug_workspace_bytes(d, dims, kdims, form)
    assert nbytes > 0
    ws, wptr = workspace(nbytes)
    Td = dev(T_storage)
    Ud = [dev(U) for U in Us]
    Hn = dims[0] * int(np.prod(kdims))
    out = torch.zeros(Hn * Hn, dtype=torch.float64, device="cuda")
    P.hotrg_debug_contract(d, dims, kdims, form, Td.data_ptr(), [u.data_ptr() for u in Ud], out.data_ptr(),
                           wptr, nbytes, stream_ptr())
    torch.cuda.synchronize()
    newdims = list(kdims) + [dims[0]]
    return out.cpu().numpy().reshape(newdims + newdims)


def gram(T_storage, direction, side):
    d = T_storage.ndim // 2
    dims = list(T_storage.shape[:d])
    nbytes = P.hotrg_debug_workspace_bytes(d, dims, None, P.HOTRG_FP64)
    ws, wptr = workspace(nbytes)
    Td = dev(T_storage)
    n = dims[direction] ** 2
    A = torch.zeros(n * n, dtype=torch.float64, device="cuda")
    P.hotrg_debug_gram(d, dims, direction, side, Td.data_ptr(), A.data_ptr(), wptr, nbytes, stream_ptr())
    torch.cuda.synchronize()
    return A.cpu().numpy().reshape(n, n)


def eigh(A_batch):
    batch, n, _ = A_batch.shape
    Ad = dev(A_batch)
    w = torch.zeros(batch * n, dtype=torch.float64, device="cuda")
    V = torch.zeros(batch * n * n, dtype=torch.float64, device="cuda")
    nbytes = P.hotrg_debug_eigh_workspace_bytes(n, batch)
    ws, wptr = workspace(nbytes)
    P.hotrg_debug_eigh(n, batch, Ad.data_ptr(), w.data_ptr(), V.data_ptr(), wptr, nbytes, stream_ptr())
    torch.cuda.synchronize()
    return w.cpu().numpy().reshape(batch, n), V.cpu().numpy().reshape(batch, n, n)


def eigh_lead(A_batch, kvec):
    """hotrg_debug_eigh_lead: resolved eigenvalues (descending, zeros after them), the sum of the
    others per matrix, and the leading kvec eigenvectors as columns."""
    batch, n, _ = A_batch.shape
    Ad = dev(A_batch)
    w = torch.zeros(batch * n, dtype=torch.float64, device="cuda")
    V = torch.zeros(batch * n * n, dtype=torch.float64, device="cuda")
    tail = torch.zeros(batch, dtype=torch.float64, device="cuda")
    nbytes = P.hotrg_debug_eigh_workspace_bytes(n, batch)
    ws, wptr = workspace(nbytes)
    P.hotrg_debug_eigh_lead(n, batch, kvec, Ad.data_ptr(), w.data_ptr(), V.data_ptr(), tail.data_ptr(), wptr, nbytes,
                            stream_ptr())
    torch.cuda.synchronize()
    return (w.cpu().numpy().reshape(batch, n), tail.cpu().numpy(),
            V.cpu().numpy().reshape(batch, n, n)[:, :, :kvec])


def relerr(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
