"""MI355X-native HOTRG coarse-graining (arXiv 2110.03607) -- Python binding.

Thin ctypes layer over libhotrg.so (C ABI in include/hotrg.h).  The functions below
carry the C names and only marshal arguments; every step of the method runs in the
library's HIP kernels.  PyTorch supplies device memory (the workspace) and the
stream.  There is no fallback: if the library is missing, importing works but the
first call raises.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhotrg.so")

# status codes
HOTRG_OK, HOTRG_E_ARG, HOTRG_E_STATE, HOTRG_E_NUMERIC, HOTRG_E_OOM, HOTRG_E_DEVICE, HOTRG_E_NOT_PSD = range(7)
# models
HOTRG_ISING, HOTRG_POTTS = 0, 1
# precision forms
HOTRG_FP64, HOTRG_FP32, HOTRG_BF16, HOTRG_FP16, HOTRG_SPLIT_BF16, HOTRG_SPLIT_FP16 = range(6)
# normalisation factor and choice between U and U'
HOTRG_NORM_TRACE, HOTRG_NORM_MAXABS = 0, 1
NORMS = {"trace": HOTRG_NORM_TRACE, "maxabs": HOTRG_NORM_MAXABS}
HOTRG_CHOOSE_EPSILON, HOTRG_CHOOSE_U, HOTRG_CHOOSE_UPRIME = 0, 1, 2
CHOICES = {"epsilon": HOTRG_CHOOSE_EPSILON, "U": HOTRG_CHOOSE_U, "Uprime": HOTRG_CHOOSE_UPRIME}
FORMS = {"fp64": HOTRG_FP64, "fp32": HOTRG_FP32, "bf16": HOTRG_BF16, "fp16": HOTRG_FP16,
         "split_bf16": HOTRG_SPLIT_BF16, "split_fp16": HOTRG_SPLIT_FP16}
HOTRG_MAX_DIRS = 4


class hotrg_model(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("d", ctypes.c_int), ("q", ctypes.c_int),
                ("J", ctypes.c_double), ("h", ctypes.c_double)]


class hotrg_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("max_steps", ctypes.c_int), ("chunk", ctypes.c_int),
                ("record_grad", ctypes.c_int), ("norm", ctypes.c_int), ("choice", ctypes.c_int)]


class hotrg_step_record(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("axis", ctypes.c_int),
                ("dims_before", ctypes.c_int * HOTRG_MAX_DIRS),
                ("trace", ctypes.c_double), ("lnz_per_site", ctypes.c_double), ("gu_wen", ctypes.c_double),
                ("chi_new", ctypes.c_int * HOTRG_MAX_DIRS),
                ("eps", ctypes.c_double * HOTRG_MAX_DIRS), ("eps_p", ctypes.c_double * HOTRG_MAX_DIRS),
                ("chose_prime", ctypes.c_int * HOTRG_MAX_DIRS), ("truncated", ctypes.c_int * HOTRG_MAX_DIRS),
                ("kept", ctypes.c_int * HOTRG_MAX_DIRS)]


HOTRG_T_COUNT = 7
TIMING_PHASES = ("decomp", "prime", "bottleneck", "nonprime", "trace", "contract", "step")


class hotrg_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * HOTRG_T_COUNT), ("count", ctypes.c_long * HOTRG_T_COUNT),
                ("flops_bottleneck", ctypes.c_double), ("flops_contract", ctypes.c_double)]


class hotrg_instance(ctypes.Structure):
    _fields_ = [("model", hotrg_model), ("beta", ctypes.c_double), ("chi", ctypes.c_int), ("pad", ctypes.c_int)]


class HotrgError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"hotrg error {code}: {message}")
        self.code = code


_lib = None

_SIGS = {
    "hotrg_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hotrg_model), ctypes.c_int, ctypes.POINTER(hotrg_opts)]),
    "hotrg_init": (ctypes.c_int, [ctypes.POINTER(hotrg_model), ctypes.c_double, ctypes.c_int,
                                  ctypes.POINTER(hotrg_opts), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]),
    "hotrg_tensor_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                                       ctypes.POINTER(hotrg_opts)]),
    "hotrg_init_tensor": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p, ctypes.c_int,
                                         ctypes.POINTER(hotrg_opts), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "hotrg_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hotrg_log_z": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    "hotrg_step_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(hotrg_step_record)]),
    "hotrg_spectrum": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "hotrg_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "hotrg_timings": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(hotrg_timing)]),
    "hotrg_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "hotrg_destroy": (None, [ctypes.c_void_p]),
    "hotrg_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "hotrg_debug_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                      ctypes.POINTER(ctypes.c_int), ctypes.c_int]),
    "hotrg_debug_contract": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                            ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "hotrg_debug_gram": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_void_p]),
    "hotrg_debug_eigh_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, ctypes.c_int]),
    "hotrg_batch_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(hotrg_instance), ctypes.c_int,
                                                      ctypes.POINTER(hotrg_opts)]),
    "hotrg_batch_init": (ctypes.c_int, [ctypes.POINTER(hotrg_instance), ctypes.c_int, ctypes.POINTER(hotrg_opts),
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "hotrg_batch_step": (ctypes.c_int, [ctypes.c_void_p]),
    "hotrg_batch_log_z": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int)]),
    "hotrg_batch_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "hotrg_batch_instance": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int]),
    "hotrg_batch_tune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "hotrg_batch_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]),
    "hotrg_batch_destroy": (None, [ctypes.c_void_p]),
    "hotrg_batch_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "hotrg_debug_eigh": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]),
    "hotrg_debug_eigh_lead": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_size_t, ctypes.c_void_p]),
    "hotrg_probe_mfma_rate": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "hotrg_eigh_noalloc_max_bytes": (ctypes.c_size_t, []),
    "hotrg_eigh_noalloc": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
}


def exported_symbols():
    """Names the C ABI exports (and this module binds)."""
    return list(_SIGS)


def lib():
    """Load libhotrg.so (raises if it has not been built).

    PyTorch is imported first when it is installed: PyTorch ships its own HIP runtime, and the
    library must bind to the same one as the tensors and streams it is handed.  Loaded before
    PyTorch, the library would pull in the system HIP runtime and the process would hold two,
    each rejecting the other's device pointers and streams."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2110_03607_amd.build.build()")
        try:
            import torch  # noqa: F401  (one HIP runtime per process, see above)
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    if rc != HOTRG_OK:
        msg = lib().hotrg_last_error(handle)
        raise HotrgError(rc, msg.decode() if msg else "")


def _ints(vals):
    arr = (ctypes.c_int * len(vals))(*vals)
    return arr


# ---- C ABI, same names --------------------------------------------------------

def hotrg_workspace_bytes(model: hotrg_model, chi: int, opts: hotrg_opts) -> int:
    return lib().hotrg_workspace_bytes(ctypes.byref(model), chi, ctypes.byref(opts))


def hotrg_init(model: hotrg_model, beta: float, chi: int, opts: hotrg_opts, workspace_ptr: int,
               workspace_bytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    rc = lib().hotrg_init(ctypes.byref(model), beta, chi, ctypes.byref(opts), ctypes.c_void_p(workspace_ptr),
                          workspace_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(h))
    _check(rc, None)
    return h


def hotrg_tensor_workspace_bytes(d: int, dims, chi: int, opts: hotrg_opts) -> int:
    return lib().hotrg_tensor_workspace_bytes(d, _ints(dims), chi, ctypes.byref(opts))


def hotrg_init_tensor(d: int, dims, T0_ptr: int, chi: int, opts: hotrg_opts, workspace_ptr: int,
                      workspace_bytes: int, stream_ptr: int):
    h = ctypes.c_void_p()
    rc = lib().hotrg_init_tensor(d, _ints(dims), ctypes.c_void_p(T0_ptr), chi, ctypes.byref(opts),
                                 ctypes.c_void_p(workspace_ptr), workspace_bytes, ctypes.c_void_p(stream_ptr),
                                 ctypes.byref(h))
    _check(rc, None)
    return h


def hotrg_step(h, axis: int) -> None:
    _check(lib().hotrg_step(h, axis), h)


def hotrg_log_z(h):
    v = ctypes.c_double()
    n = ctypes.c_int()
    _check(lib().hotrg_log_z(h, ctypes.byref(v), ctypes.byref(n)), h)
    return v.value, n.value


def hotrg_step_info(h, step: int) -> hotrg_step_record:
    r = hotrg_step_record()
    _check(lib().hotrg_step_info(h, step, ctypes.byref(r)), h)
    return r


def hotrg_spectrum(h, step: int, direction: int, side: int, cap: int = 64):
    buf = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(lib().hotrg_spectrum(h, step, direction, side, buf, cap, ctypes.byref(n)), h)
    return [buf[i] for i in range(n.value)]


def hotrg_profile(h, enable: bool) -> None:
    _check(lib().hotrg_profile(h, 1 if enable else 0), h)


def hotrg_timings(h) -> hotrg_timing:
    t = hotrg_timing()
    _check(lib().hotrg_timings(h, ctypes.byref(t)), h)
    return t


def hotrg_grad(h) -> float:
    v = ctypes.c_double()
    _check(lib().hotrg_grad(h, ctypes.byref(v)), h)
    return v.value


def hotrg_destroy(h) -> None:
    lib().hotrg_destroy(h)


def hotrg_last_error(h=None) -> str:
    m = lib().hotrg_last_error(h)
    return m.decode() if m else ""


def hotrg_debug_workspace_bytes(d: int, dims, kdims, precision: int) -> int:
    return lib().hotrg_debug_workspace_bytes(d, _ints(dims), _ints(kdims) if kdims is not None else None, precision)


def hotrg_debug_contract(d, dims, kdims, precision, T_ptr, U_ptrs, Tnext_ptr, ws_ptr, ws_bytes, stream_ptr):
    ups = (ctypes.c_void_p * len(U_ptrs))(*U_ptrs)
    rc = lib().hotrg_debug_contract(d, _ints(dims), _ints(kdims), precision, ctypes.c_void_p(T_ptr), ups,
                                    ctypes.c_void_p(Tnext_ptr), ctypes.c_void_p(ws_ptr), ws_bytes,
                                    ctypes.c_void_p(stream_ptr))
    _check(rc, None)


def hotrg_debug_gram(d, dims, direction, side, T_ptr, A_ptr, ws_ptr, ws_bytes, stream_ptr):
    rc = lib().hotrg_debug_gram(d, _ints(dims), direction, side, ctypes.c_void_p(T_ptr), ctypes.c_void_p(A_ptr),
                                ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream_ptr))
    _check(rc, None)


def hotrg_debug_eigh_workspace_bytes(n: int, batch: int) -> int:
    return lib().hotrg_debug_eigh_workspace_bytes(n, batch)


def hotrg_debug_eigh(n, batch, A_ptr, w_ptr, V_ptr, ws_ptr, ws_bytes, stream_ptr):
    rc = lib().hotrg_debug_eigh(n, batch, ctypes.c_void_p(A_ptr), ctypes.c_void_p(w_ptr), ctypes.c_void_p(V_ptr),
                                ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.c_void_p(stream_ptr))
    _check(rc, None)


def hotrg_debug_eigh_lead(n, batch, kvec, A_ptr, w_ptr, V_ptr, tail_ptr, ws_ptr, ws_bytes, stream_ptr):
    rc = lib().hotrg_debug_eigh_lead(n, batch, kvec, ctypes.c_void_p(A_ptr), ctypes.c_void_p(w_ptr),
                                     ctypes.c_void_p(V_ptr), ctypes.c_void_p(tail_ptr), ctypes.c_void_p(ws_ptr),
                                     ws_bytes, ctypes.c_void_p(stream_ptr))
    _check(rc, None)


def hotrg_probe_mfma_rate(precision: int, stream_ptr: int) -> float:
    v = ctypes.c_double()
    _check(lib().hotrg_probe_mfma_rate(precision, ctypes.byref(v), ctypes.c_void_p(stream_ptr)), None)
    return v.value


def hotrg_eigh_noalloc_max_bytes() -> int:
    return lib().hotrg_eigh_noalloc_max_bytes()


def hotrg_eigh_noalloc(n, batch, A_ptr, w_ptr, V_ptr, status_ptr, stream_ptr):
    rc = lib().hotrg_eigh_noalloc(n, batch, ctypes.c_void_p(A_ptr), ctypes.c_void_p(w_ptr), ctypes.c_void_p(V_ptr),
                                  ctypes.c_void_p(status_ptr), ctypes.c_void_p(stream_ptr))
    _check(rc, None)


def _check_batch(rc: int, b=None):
    if rc != HOTRG_OK:
        msg = lib().hotrg_batch_last_error(b)
        raise HotrgError(rc, msg.decode() if msg else "")


def _instances(inst):
    arr = (hotrg_instance * len(inst))(*inst)
    return arr


def hotrg_batch_workspace_bytes(inst, opts: hotrg_opts) -> int:
    return lib().hotrg_batch_workspace_bytes(_instances(inst), len(inst), ctypes.byref(opts))


def hotrg_batch_init(inst, opts: hotrg_opts, workspace_ptr: int, workspace_bytes: int, stream_ptr: int):
    b = ctypes.c_void_p()
    rc = lib().hotrg_batch_init(_instances(inst), len(inst), ctypes.byref(opts), ctypes.c_void_p(workspace_ptr),
                                workspace_bytes, ctypes.c_void_p(stream_ptr), ctypes.byref(b))
    _check_batch(rc, None)
    return b


def hotrg_batch_step(b) -> None:
    _check_batch(lib().hotrg_batch_step(b), b)


def hotrg_batch_log_z(b, n: int):
    out = (ctypes.c_double * n)()
    steps = ctypes.c_int()
    _check_batch(lib().hotrg_batch_log_z(b, out, ctypes.byref(steps)), b)
    return [out[i] for i in range(n)], steps.value


def hotrg_batch_info(b):
    g, e = ctypes.c_int(), ctypes.c_int()
    _check_batch(lib().hotrg_batch_info(b, ctypes.byref(g), ctypes.byref(e)), b)
    return g.value, e.value


def hotrg_batch_tune(b) -> int:
    n = ctypes.c_int()
    _check_batch(lib().hotrg_batch_tune(b, ctypes.byref(n)), b)
    return n.value


def hotrg_batch_tuning(b, cls: int) -> dict:
    d, chi, tile, chunk = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_double()
    _check_batch(lib().hotrg_batch_tuning(b, cls, ctypes.byref(d), ctypes.byref(chi), ctypes.byref(tile),
                                          ctypes.byref(chunk), ctypes.byref(ms)), b)
    return {"d": d.value, "chi": chi.value, "gemm_tile": tile.value, "chunk_pairs": chunk.value,
            "contract_ms": ms.value}


def hotrg_batch_instance(b, i: int):
    return ctypes.c_void_p(lib().hotrg_batch_instance(b, i))


def hotrg_batch_destroy(b) -> None:
    lib().hotrg_batch_destroy(b)


def hotrg_batch_last_error(b=None) -> str:
    m = lib().hotrg_batch_last_error(b)
    return m.decode() if m else ""


# ---- convenience wrapper (torch for memory and the stream) ----------------------

class HOTRG:
    """One HOTRG run on the current GPU: init, steps along the axis cycle, lnZ/V.

    >>> r = HOTRG("ising", d=3, beta=1/4.5115, chi=16, precision="fp64")
    >>> r.run(25); r.log_z()
    """

    def __init__(self, kind: str, d: int, beta: float, chi: int, q: int | None = None, J: float = 1.0,
                 h: float = 0.0, precision: str = "fp64", max_steps: int = 64, chunk: int = 0,
                 record_grad: bool = False, norm: str = "trace", choice: str = "epsilon"):
        import torch

        kind_id = {"ising": HOTRG_ISING, "potts": HOTRG_POTTS}[kind]
        q = 2 if kind == "ising" else (3 if q is None else q)
        self.model = hotrg_model(kind_id, d, q, J, h)
        self.opts = hotrg_opts(FORMS[precision], max_steps, chunk, 1 if record_grad else 0, NORMS[norm],
                               CHOICES[choice])
        self.d = d
        nbytes = hotrg_workspace_bytes(self.model, chi, self.opts)
        if nbytes == 0:
            raise HotrgError(HOTRG_E_ARG, "invalid model/chi/options")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        self.handle = hotrg_init(self.model, beta, chi, self.opts, aligned, nbytes, self.stream.cuda_stream)
        self.steps = 0

    @classmethod
    def from_tensor(cls, T0, chi: int, precision: str = "fp64", max_steps: int = 64, chunk: int = 0,
                    norm: str = "trace", choice: str = "epsilon"):
        """A run started from a local tensor T0 (a float64 torch tensor on the GPU, storage order
        T[c][n_1]..[c'][n'_1].., shape dims + dims) instead of a lattice model."""
        import torch

        self = cls.__new__(cls)
        d = T0.dim() // 2
        dims = list(T0.shape[:d])
        self.model = None
        self.opts = hotrg_opts(FORMS[precision], max_steps, chunk, 0, NORMS[norm], CHOICES[choice])
        self.d = d
        nbytes = hotrg_tensor_workspace_bytes(d, dims, chi, self.opts)
        if nbytes == 0:
            raise HotrgError(HOTRG_E_ARG, "invalid tensor dims, chi or options")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.current_stream()
        T0c = T0.contiguous().to(dtype=torch.float64)
        self.handle = None
        self.handle = hotrg_init_tensor(d, dims, T0c.data_ptr(), chi, self.opts, aligned, nbytes,
                                        self.stream.cuda_stream)
        self._t0 = T0c          # kept alive until the stream has read it
        self.steps = 0
        return self

    def step(self, axis: int | None = None) -> None:
        if axis is None:
            axis = self.steps % self.d
        hotrg_step(self.handle, axis)
        self.steps += 1

    def run(self, steps: int) -> None:
        for _ in range(steps):
            self.step()

    def log_z(self) -> float:
        return hotrg_log_z(self.handle)[0]

    def grad(self) -> float:
        """d(lnZ/V)/d(beta) after the steps so far (needs record_grad=True)."""
        return hotrg_grad(self.handle)

    def info(self, step: int) -> hotrg_step_record:
        return hotrg_step_info(self.handle, step)

    def spectrum(self, step: int, direction: int, side: int, cap: int = 64):
        return hotrg_spectrum(self.handle, step, direction, side, cap)

    def profile(self, enable: bool = True) -> None:
        hotrg_profile(self.handle, enable)

    def timings(self) -> dict:
        t = hotrg_timings(self.handle)
        out = {k: {"ms": t.ms[i], "count": t.count[i]} for i, k in enumerate(TIMING_PHASES)}
        out["flops_bottleneck"] = t.flops_bottleneck
        out["flops_contract"] = t.flops_contract
        return out

    def close(self) -> None:
        if self.handle is not None:
            hotrg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lnz_per_site(beta, kind: str = "ising", d: int = 3, chi: int = 16, steps: int = 20, q: int | None = None,
                 J: float = 1.0, precision: str = "fp64"):
    """lnZ/V after `steps` steps as a differentiable function of beta (a 0-d torch tensor).

    The forward pass runs HOTRG on the GPU with the derivative carried along
    (record_grad); backward multiplies the incoming gradient by d(lnZ/V)/d(beta).
    """
    import torch

    class _LnZ(torch.autograd.Function):
        @staticmethod
        def forward(ctx, b):
            r = HOTRG(kind, d, float(b), chi, q=q, J=J, precision=precision, max_steps=steps, record_grad=True)
            r.run(steps)
            val, der = r.log_z(), r.grad()
            r.close()
            ctx.der = der
            return torch.tensor(val, dtype=torch.float64)

        @staticmethod
        def backward(ctx, g):
            return g * ctx.der

    return _LnZ.apply(beta)


def make_instance(kind: str, d: int, beta: float, chi: int, q: int | None = None, J: float = 1.0,
                  h: float = 0.0) -> hotrg_instance:
    kind_id = {"ising": HOTRG_ISING, "potts": HOTRG_POTTS}[kind]
    q = 2 if kind == "ising" else (3 if q is None else q)
    return hotrg_instance(hotrg_model(kind_id, d, q, J, h), beta, chi, 0)


class HOTRGBatch:
    """Many independent HOTRG runs advanced together (a temperature sweep, mixed d and chi).

    Runs on a stream of its own (default priority) so that the saturated steps can be
    recorded into HIP graphs and replayed with one launch per step.

    >>> b = HOTRGBatch([make_instance("ising", 3, 1 / T, 12) for T in (4.0, 4.5, 5.0)], precision="split_fp16")
    >>> b.run(20); b.log_z()
    """

    def __init__(self, instances, precision: str = "fp64", max_steps: int = 64, chunk: int = 0,
                 graphs: bool = True, tune: bool = False, norm: str = "trace", choice: str = "epsilon"):
        import torch

        self.instances = list(instances)
        self.n = len(self.instances)
        self.opts = hotrg_opts(FORMS[precision], max_steps, chunk, 0, NORMS[norm], CHOICES[choice])
        nbytes = hotrg_batch_workspace_bytes(self.instances, self.opts)
        if nbytes == 0:
            raise HotrgError(HOTRG_E_ARG, "invalid instance or options")
        self.workspace_bytes = nbytes
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        aligned = (self.workspace.data_ptr() + 255) // 256 * 256
        if graphs:
            self.stream = torch.cuda.Stream()
            # the workspace was allocated on the current stream: make ours wait for that
            self.stream.wait_stream(torch.cuda.current_stream())
            stream_ptr = self.stream.cuda_stream
        else:
            # the NULL stream cannot be recorded: every step is enqueued kernel by kernel
            self.stream = torch.cuda.default_stream()
            stream_ptr = 0
        self.handle = hotrg_batch_init(self.instances, self.opts, aligned, nbytes, stream_ptr)
        self.steps = 0
        self.tuned = []
        if tune:
            n = hotrg_batch_tune(self.handle)
            self.tuned = [hotrg_batch_tuning(self.handle, c) for c in range(n)]

    def step(self) -> None:
        hotrg_batch_step(self.handle)
        self.steps += 1

    def run(self, steps: int) -> None:
        for _ in range(steps):
            self.step()

    def log_z(self):
        return hotrg_batch_log_z(self.handle, self.n)[0]

    def info(self, i: int, step: int) -> hotrg_step_record:
        return hotrg_step_info(hotrg_batch_instance(self.handle, i), step)

    def graph_stats(self):
        """(steps run as one graph launch, steps enqueued kernel by kernel)."""
        return hotrg_batch_info(self.handle)

    def synchronize(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if self.handle is not None:
            self.stream.synchronize()
            hotrg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
