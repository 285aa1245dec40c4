"""C-ABI checks that need no GPU: the library loads, exports every declared symbol,
and its host-side argument validation and workspace planning behave."""

import ctypes
import os
import re

import pytest

import paper_2110_03607_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hotrg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hotrg_\w+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    L = P.lib()
    for n in names:
        assert hasattr(L, n), n
    # the binding covers the same set
    assert sorted(P.exported_symbols()) == names


def test_struct_layouts_match_header():
    # hotrg_model: int, int, int, (pad), double, double
    assert ctypes.sizeof(P.hotrg_model) == 32
    assert ctypes.sizeof(P.hotrg_opts) == 24


def _model(kind=P.HOTRG_ISING, d=3, q=2, J=1.0, h=0.0):
    return P.hotrg_model(kind, d, q, J, h)


def test_workspace_bytes_validation():
    o = P.hotrg_opts(P.HOTRG_FP64, 32, 0, 0)
    assert P.hotrg_workspace_bytes(_model(), 16, o) > 0
    assert P.hotrg_workspace_bytes(_model(d=4), 16, o) == 0            # d not supported
    assert P.hotrg_workspace_bytes(_model(), 17, o) == 0               # chi above the 3D maximum
    assert P.hotrg_workspace_bytes(_model(d=2), 32, o) > 0
    assert P.hotrg_workspace_bytes(_model(q=3), 16, o) == 0            # Ising needs q = 2
    assert P.hotrg_workspace_bytes(_model(P.HOTRG_POTTS, 3, 3), 16, o) > 0
    assert P.hotrg_workspace_bytes(_model(P.HOTRG_POTTS, 3, 3), 2, o) == 0   # chi < q
    bad = P.hotrg_opts(9, 32, 0, 0)
    assert P.hotrg_workspace_bytes(_model(), 16, bad) == 0


def test_workspace_grows_with_chi_and_form():
    o64 = P.hotrg_opts(P.HOTRG_FP64, 32, 0, 0)
    o32 = P.hotrg_opts(P.HOTRG_FP32, 32, 0, 0)
    sizes = [P.hotrg_workspace_bytes(_model(), c, o64) for c in (4, 8, 12, 16)]
    assert sizes == sorted(sizes)
    assert P.hotrg_workspace_bytes(_model(), 16, o32) < P.hotrg_workspace_bytes(_model(), 16, o64)
    # chi = 16, FP64: two copies of the chi^6 tensor at least
    assert sizes[-1] > 2 * 16 ** 6 * 8


def test_init_argument_errors_without_device():
    o = P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0)
    h = ctypes.c_void_p()
    L = P.lib()
    # NULL out pointer
    assert L.hotrg_init(ctypes.byref(_model()), 0.2, 8, ctypes.byref(o), None, 0, None, None) == P.HOTRG_E_ARG
    # invalid beta
    rc = L.hotrg_init(ctypes.byref(_model()), float("nan"), 8, ctypes.byref(o), ctypes.c_void_p(256), 1 << 40,
                      None, ctypes.byref(h))
    assert rc == P.HOTRG_E_ARG and not h.value
    # antiferromagnet: W not PSD
    rc = L.hotrg_init(ctypes.byref(_model(J=-1.0)), 0.2, 8, ctypes.byref(o), ctypes.c_void_p(256), 1 << 40,
                      None, ctypes.byref(h))
    assert rc == P.HOTRG_E_NOT_PSD
    # workspace too small
    rc = L.hotrg_init(ctypes.byref(_model()), 0.2, 8, ctypes.byref(o), ctypes.c_void_p(256), 16, None,
                      ctypes.byref(h))
    assert rc == P.HOTRG_E_OOM
    assert "workspace" in P.hotrg_last_error(None)
    # NULL handle
    assert L.hotrg_step(None, 0) == P.HOTRG_E_ARG
    assert L.hotrg_log_z(None, None, None) == P.HOTRG_E_ARG
    L.hotrg_destroy(None)


def test_debug_workspace_bytes():
    assert P.hotrg_debug_workspace_bytes(3, [4, 4, 4], [8, 8], P.HOTRG_FP64) > 0
    assert P.hotrg_debug_workspace_bytes(3, [4, 4, 4], [17, 8], P.HOTRG_FP64) == 0   # k > chi^2
    assert P.hotrg_debug_workspace_bytes(2, [8, 8], [16], P.HOTRG_SPLIT_FP16) > 0
    assert P.hotrg_debug_eigh_workspace_bytes(256, 2) >= 2 * 256 * 256 * 8
    assert P.hotrg_debug_eigh_workspace_bytes(2000, 1) == 0


def test_derivative_mode_forms():
    o = P.hotrg_opts(P.HOTRG_FP64, 8, 0, 1)
    assert P.hotrg_workspace_bytes(_model(), 8, o) > P.hotrg_workspace_bytes(_model(), 8, P.hotrg_opts(0, 8, 0, 0))
    assert P.hotrg_workspace_bytes(_model(), 8, P.hotrg_opts(P.HOTRG_FP32, 8, 0, 1)) > 0
    assert P.hotrg_workspace_bytes(_model(), 8, P.hotrg_opts(P.HOTRG_SPLIT_FP16, 8, 0, 1)) == 0
    h = ctypes.c_void_p()
    rc = P.lib().hotrg_init(ctypes.byref(_model()), 0.0, 8, ctypes.byref(o), ctypes.c_void_p(256), 1 << 40, None,
                            ctypes.byref(h))
    assert rc == P.HOTRG_E_ARG     # the derivative needs beta > 0


def test_batch_workspace_and_argument_errors():
    o = P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0)
    inst = [P.make_instance("ising", 3, 0.22, 8), P.make_instance("ising", 2, 0.44, 16),
            P.make_instance("potts", 3, 0.55, 9)]
    nb = P.hotrg_batch_workspace_bytes(inst, o)
    single = [P.hotrg_workspace_bytes(i.model, i.chi, o) for i in inst]
    # private state per instance, one shared scratch area: less than separate handles
    assert max(single) < nb < sum(single)
    assert P.hotrg_batch_workspace_bytes(inst + [P.make_instance("ising", 3, 0.22, 17)], o) == 0
    assert P.hotrg_batch_workspace_bytes(inst, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 1)) == 0   # no derivative
    assert P.lib().hotrg_batch_workspace_bytes(None, 0, ctypes.byref(o)) == 0
    b = ctypes.c_void_p()
    arr = (P.hotrg_instance * 3)(*inst)
    rc = P.lib().hotrg_batch_init(arr, 3, ctypes.byref(o), ctypes.c_void_p(256), 16, None, ctypes.byref(b))
    assert rc == P.HOTRG_E_OOM and not b.value
    assert "workspace" in P.hotrg_batch_last_error(None)
    assert P.lib().hotrg_batch_step(None) == P.HOTRG_E_ARG
    assert not P.lib().hotrg_batch_instance(None, 0)
    P.lib().hotrg_batch_destroy(None)


def test_supplied_tensor_argument_validation():
    o = P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0)
    assert P.hotrg_tensor_workspace_bytes(3, [3, 4, 2], 6, o) > 0
    assert P.hotrg_tensor_workspace_bytes(2, [32, 32], 32, o) > 0
    assert P.hotrg_tensor_workspace_bytes(3, [17, 4, 2], 6, o) == 0       # above the 3D maximum
    assert P.hotrg_tensor_workspace_bytes(3, [0, 4, 2], 6, o) == 0
    assert P.hotrg_tensor_workspace_bytes(5, [2, 2, 2, 2, 2], 6, o) == 0
    assert P.hotrg_tensor_workspace_bytes(4, [2, 2, 2, 2], 13, o) == 0     # 4D: chi <= 12
    assert P.hotrg_tensor_workspace_bytes(4, [2, 2, 2, 2], 12, o) > 0
    assert P.hotrg_tensor_workspace_bytes(3, [3, 4, 2], 6, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 1)) == 0   # no beta
    # the plan covers the dims the run reaches from (3, 4, 2): it is at least that of a model run
    # whose dims pass through the same values
    assert P.hotrg_tensor_workspace_bytes(3, [16, 16, 16], 16, o) >= \
        P.hotrg_workspace_bytes(P.hotrg_model(P.HOTRG_ISING, 3, 2, 1.0, 0.0), 16, o)
    with pytest.raises(P.HotrgError) as e:
        P.hotrg_init_tensor(3, [3, 4, 2], 0, 6, o, 0, 0, 0)
    assert e.value.code == P.HOTRG_E_ARG


def test_truncated_eigensolver_argument_validation():
    # kvec outside 1 .. n and missing buffers are refused before anything touches a device
    L = P.lib()
    ws = ctypes.c_void_p(16)
    for n, batch, kvec in [(256, 1, 0), (256, 1, 257), (2000, 1, 8), (256, 5, 8)]:
        rc = L.hotrg_debug_eigh_lead(n, batch, kvec, ws, ws, ws, None, ws, 1 << 30, None)
        assert rc == P.HOTRG_E_ARG, (n, batch, kvec)
    assert L.hotrg_debug_eigh_lead(256, 1, 16, None, ws, ws, None, ws, 1 << 30, None) == P.HOTRG_E_ARG


def test_four_dimensional_limits():
    # 4D: chi <= 12 in every form (the register width of the 4D chain kernels); no derivative
    # mode and no batches for d = 4
    ising4 = P.hotrg_model(P.HOTRG_ISING, 4, 2, 1.0, 0.0)
    for prec, chi, ok in [(P.HOTRG_SPLIT_FP16, 8, True), (P.HOTRG_FP32, 12, True), (P.HOTRG_SPLIT_FP16, 13, False),
                          (P.HOTRG_FP64, 12, True), (P.HOTRG_FP64, 13, False)]:
        assert (P.hotrg_workspace_bytes(ising4, chi, P.hotrg_opts(prec, 8, 0, 0)) > 0) == ok, (prec, chi)
    assert P.hotrg_workspace_bytes(ising4, 4, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 1)) == 0
    inst = (P.hotrg_instance * 1)(P.hotrg_instance(ising4, 0.15, 4, 0))
    assert P.lib().hotrg_batch_workspace_bytes(inst, 1, ctypes.byref(P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0))) == 0
    assert P.hotrg_debug_workspace_bytes(4, [8, 8, 8, 8], [8, 8, 8], P.HOTRG_SPLIT_FP16) > 0
    assert P.hotrg_debug_workspace_bytes(4, [12, 12, 12, 12], [12, 12, 12], P.HOTRG_FP64) > 0
    assert P.hotrg_debug_workspace_bytes(4, [13, 2, 2, 2], [4, 4, 4], P.HOTRG_FP32) == 0


def test_eigh_workspace_holds_the_failure_flag():
    assert P.hotrg_debug_eigh_workspace_bytes(256, 4) >= 4 * 2 * 256 * 256 * 8 + 4


def test_norm_and_choice_options_are_validated():
    m = _model()
    assert P.hotrg_workspace_bytes(m, 8, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0, P.HOTRG_NORM_MAXABS,
                                                      P.HOTRG_CHOOSE_UPRIME)) > 0
    assert P.hotrg_workspace_bytes(m, 8, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0, 2, 0)) == 0       # no such norm
    assert P.hotrg_workspace_bytes(m, 8, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0, 0, 3)) == 0       # no such choice
    # the derivative is carried with the trace normalisation only
    assert P.hotrg_workspace_bytes(m, 8, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 1, P.HOTRG_NORM_MAXABS, 0)) == 0
    with pytest.raises(P.HotrgError) as e:
        P.hotrg_init(m, 0.3, 8, P.hotrg_opts(P.HOTRG_FP64, 8, 0, 0, 0, 7), 256, 1 << 30, 0)
    assert e.value.code == P.HOTRG_E_ARG


def test_one_hip_runtime_per_process():
    """Loading the library before PyTorch must not map a second HIP runtime next to PyTorch's
    (device pointers and streams of one are invalid in the other)."""
    import subprocess
    import sys
    code = ("import paper_2110_03607_amd as P; P.lib(); import torch; "
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'amdhip64' in l}))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
