"""Host-side behaviour of bench.py that needs no GPU: the one-GPU rule, the refusal to run
without a device, and the work model used for the reported TFLOP/s."""

import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_no_device_is_an_error(monkeypatch):
    import torch
    if torch.cuda.is_available():
        return
    r = run_bench("--steps", "1", "--warmup", "0", "--no-cpu")
    assert r.returncode == 1
    assert "needs a GPU" in r.stderr


def test_step_flop_model():
    # three-stage contraction of a saturated step: prime chain 2 chi^8 + 2 chi^9 (the two
    # isometries), bottleneck chi^11, non-prime chain the same as the prime chain (MACs x 2)
    chi = 16.0
    assert bench.batch_flops(3, 16) == 2.0 * (chi ** 11 + 2 * chi ** 9 + 2 * chi ** 8)
    assert abs(bench.batch_flops(3, 16) - 3.548e13) / 3.548e13 < 1e-3
    # 2D: bottleneck chi^7 and two chi^6 chains
    assert bench.batch_flops(2, 32) == 2.0 * (32.0 ** 7 + 2 * 32.0 ** 6)


def test_algorithmic_bytes_of_the_bottleneck_launch():
    # A (two FP16 planes of 4096^2), B chunk (two planes of 65536 x 4096), output chunk (4096 x 256 FP32)
    assert bench.GEMM_ALGO_BYTES["split_fp16"] == 2 * 4096 ** 2 * 2 + 2 * 65536 * 4096 * 2 + 4096 * 256 * 4
    assert bench.GEMM_TRAFFIC_BYTES["split_fp16"] > bench.GEMM_ALGO_BYTES["split_fp16"]


def test_host_info_reads_the_cpu_model():
    model, _ = bench.host_info()
    assert model is None or isinstance(model, str)
