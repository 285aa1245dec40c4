"""Benchmark: 3D Ising HOTRG, chi = 16, T = 4.5115 on one MI355X.

One "step" is one whole coarse-graining step at saturated bond dimensions (Gram
matrices, FP64 eigendecomposition, choice, prime chain, bottleneck contraction,
non-prime chain, trace and normalisation), everything on the GPU through the C ABI.

Prints one JSON line: contraction TFLOP/s (algorithmic flops of the new-tensor
contraction / its measured time) for the headline precision form, RG steps/s, the
roofline of the bottleneck GEMM (the dominant kernel), the free-energy error against
the stored FP64 oracle fixture, the same figures for the FP64 form, and the oracle
timed on a bounded sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--form split_fp16] [--no-cpu]

Measurement helpers (each prints its own lines and exits):
  --mfma-ceiling          issue rate of the MFMA instruction of each form (register-only loop)
  --counter-steps N       N steps of the headline workload, lnZ/V printed after each step (a short
                          run for rocprofv3 counter passes)
  --copy-calibration MiB  a plain device copy of MiB, three times (the reference that turns the
                          FETCH_SIZE / WRITE_SIZE counters into bytes)
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "3D HOTRG chi=16 contraction TFLOP/s + RG steps/s, MFMA vs FP64 at |df|<1e-6"
CHI, TEMP, STEPS_FIXTURE = 16, 4.5115, 25
UNSATURATED = 3            # steps 1-3 have bond dims below chi (untruncated)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16": 2516.6, "fp16": 2516.6,
               "split_bf16": 2516.6, "split_fp16": 2516.6}
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16": "bf16 (f32 acc)", "fp16": "f16 (f32 acc)",
         "split_bf16": "bf16x3 hi/lo split (f32 acc)", "split_fp16": "f16x3 hi/lo split (f32 acc)"}
PRODUCTS = {"split_bf16": 3, "split_fp16": 3}
CEILING_KEY = {"fp64": "fp64", "fp32": "fp32", "bf16": "bf16", "fp16": "fp16", "split_bf16": "bf16",
               "split_fp16": "fp16"}
# HBM bytes per launch of the bottleneck kernel of the split FP16 form at chi = 16 (16 pair
# groups per launch), from two rocprofv3 counter runs of `bench.py --counter-steps 5`
# (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors read off a 1 GiB copy);
# profiles/hotrg3d_chi16_split_fp16_gemm_counters.md (the direct-load kernel). Valid only while
# that kernel is unchanged.
GEMM_TRAFFIC_BYTES = {"split_fp16": 6.475e9}
# Algorithmic bytes of the same launch: A operand (2 planes x 4096^2 x 2 B), B chunk
# (2 planes x 65536 x 4096 x 2 B) and the new-tensor chunk written (4096 x 256 x 4 B).
GEMM_ALGO_BYTES = {"split_fp16": 2 * 4096 * 4096 * 2 + 2 * 65536 * 4096 * 2 + 4096 * 256 * 4}


def mfma_ceiling(P, torch):
    """TFLOP/s of the MFMA instruction each form contracts with, from a loop of independent
    register-only MFMAs over the whole GPU (hotrg_probe_mfma_rate)."""
    s = torch.cuda.current_stream().cuda_stream
    return {f: round(P.hotrg_probe_mfma_rate(P.FORMS[f], s), 1) for f in ("fp64", "fp32", "fp16", "bf16")}


def counter_steps(P, torch, form, steps):
    r = P.HOTRG("ising", 3, 1.0 / TEMP, CHI, precision=form, max_steps=steps)
    for p in range(steps):
        r.step()
        print(f"step {p + 1} lnZ/V {r.log_z():.15f}", flush=True)
    r.close()


def copy_calibration(torch, mib):
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB three times ({3 * mib * 1024} KiB read and written)", flush=True)


def fixture_lnz():
    path = os.path.join(ROOT, "tests", "golden", "config3.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        fx = json.load(f)
    return [s["lnz_per_site"] for s in fx["runs"][0]["steps"]]


def run_form(P, torch, form, steps, warmup, record_grad=False, finish=True):
    """Full run in one precision form; times exactly `steps` saturated steps."""
    beta = 1.0 / TEMP
    total = max(STEPS_FIXTURE, UNSATURATED + warmup + steps) if finish else UNSATURATED + warmup + steps
    r = P.HOTRG("ising", 3, beta, CHI, precision=form, max_steps=total, record_grad=record_grad)
    lnz = []
    for _ in range(UNSATURATED + warmup):
        r.step()
    lnz_hist = None
    torch.cuda.synchronize()
    r.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        r.step()
    r.log_z()                      # synchronises the library's stream
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tm = r.timings()
    r.profile(False)
    while r.steps < total:
        r.step()
    final = r.log_z()
    grad = r.grad() if record_grad else None
    # per-step lnZ/V from the step records
    lnz = [r.info(p).lnz_per_site for p in range(1, total + 1)]
    r.close()
    return dict(wall=wall, timings=tm, lnz=lnz, final=final, total_steps=total, grad=grad)


def batch_flops(d, chi):
    """Algorithmic flops of one saturated step of one instance (three-stage contraction)."""
    x = float(chi)
    return 2.0 * (x ** 11 + 2 * x ** 9 + 2 * x ** 8) if d == 3 else 2.0 * (x ** 7 + 2 * x ** 6)


def run_batch(P, torch, form, steps=20, graphs=True):
    """The temperature sweep as one batch: 64 x 3D Ising chi = 12 (T = linspace(4, 5, 64)) and
    48 x 2D Ising (beta = linspace(0.3, 0.6, 48), chi round-robin 16, 24, 32), 20 steps.
    Times the steps replayed from the recorded graphs (all instances saturated)."""
    import numpy as np
    inst = [P.make_instance("ising", 3, 1.0 / T, 12) for T in np.linspace(4.0, 5.0, 64)]
    chis = (16, 24, 32)
    inst += [P.make_instance("ising", 2, float(b), chis[i % 3]) for i, b in enumerate(np.linspace(0.3, 0.6, 48))]
    t_tune = time.perf_counter()
    b = P.HOTRGBatch(inst, precision=form, max_steps=steps, graphs=graphs, tune=True)
    tune_s = time.perf_counter() - t_tune
    t_start = time.perf_counter()
    first_timed = 9                      # 2D chi = 32 saturates at step 7; graphs recorded at steps 7, 8
    for p in range(1, steps + 1):
        if p == first_timed:
            b.synchronize()
            t0 = time.perf_counter()
        b.step()
    b.synchronize()
    t1 = time.perf_counter()
    lnz = b.log_z()
    graphs, eager = b.graph_stats()
    b_tuned = b.tuned
    # phase identification (Section 4.1.2, eq. ratio_X): the Gu-Wen ratio after the last step of
    # each 3D instance -> 2 in the ordered phase (two degenerate fixed-point sectors), 1 in the
    # disordered one; the crossing of X = 1.5 between neighbouring temperatures estimates T_c
    temps = [1.0 / i.beta for i in inst[:64]]
    xs = [b.info(i, steps).gu_wen for i in range(64)]
    cross = None
    for i in range(63):
        if (xs[i] - 1.5) * (xs[i + 1] - 1.5) <= 0 and xs[i] != xs[i + 1]:
            cross = temps[i] + (1.5 - xs[i]) * (temps[i + 1] - temps[i]) / (xs[i + 1] - xs[i])
            break
    b.close()
    timed = steps - first_timed + 1
    ms = (t1 - t0) * 1e3 / timed
    flops = sum(batch_flops(i.model.d, i.chi) for i in inst)
    return {"form": form, "instances": len(inst), "steps": steps, "timed_steps": timed,
            "ms_per_batched_step": round(ms, 3), "batched_steps_per_s": round(1e3 / ms, 4),
            "instance_steps_per_s": round(len(inst) * 1e3 / ms, 2),
            "contract_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
            "graph_launches": graphs, "eager_steps": eager, "wall_s_all_steps": round(t1 - t_start, 3),
            "autotuner": {"seconds": round(tune_s, 3), "classes": b_tuned},
            "lnz_per_site_first_last": [lnz[0], lnz[63], lnz[64], lnz[-1]],
            "gu_wen_scan_3d": {"T": [round(t, 5) for t in temps], "X_after_step_20": [round(x, 5) for x in xs],
                               "T_where_X_crosses_1.5": None if cross is None else round(cross, 4)}}


def eigh_2d_chi32(P, torch, beta=0.44, steps=8, timed=3):
    """The FP64 decomposition of a saturated 2D Ising chi = 32 step on its own: the two
    1024 x 1024 Gram matrices (built, tridiagonalised, 33 leading eigenpairs)."""
    r = P.HOTRG("ising", 2, beta, 32, precision="split_fp16", max_steps=steps)
    for _ in range(steps - timed):
        r.step()
    torch.cuda.synchronize()
    r.profile(True)
    for _ in range(timed):
        r.step()
    r.log_z()
    torch.cuda.synchronize()
    tm = r.timings()
    r.profile(False)
    r.close()
    return {"workload": f"2D Ising chi=32, beta={beta}, saturated steps {steps - timed + 1}-{steps}: Gram build and "
                        "FP64 eigendecomposition of the two 1024 x 1024 Gram matrices per step",
            "ms_per_step": round(tm["decomp"]["ms"] / timed, 3), "bound": "latency (serial Householder and "
            "Sturm recurrences)"}


def run_4d(P, torch, form, chi=8, temp=6.68, warmup=8, timed=4):
    """The paper's own workload at one GPU's size: 4D Ising HOTRG (three Next directions per step),
    chi = 8, T near the 4D critical point; `timed` saturated steps after `warmup`."""
    r = P.HOTRG("ising", 4, 1.0 / temp, chi, precision=form, max_steps=warmup + timed)
    for _ in range(warmup):
        r.step()
    r.log_z()
    torch.cuda.synchronize()
    r.profile(True)
    t0 = time.perf_counter()
    for _ in range(timed):
        r.step()
    lz = r.log_z()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / timed
    tm = r.timings()
    r.profile(False)
    r.close()
    b = tm["bottleneck"]
    return {"workload": f"4D Ising HOTRG, chi={chi}, T={temp}, J=1, h=0; steps {warmup + 1}-{warmup + timed}",
            "form": form, "ms_per_step": round(wall * 1e3, 2), "steps_per_s": round(1.0 / wall, 3),
            "contract_tflops": round(tm["flops_contract"] / (timed * wall) / 1e12, 1),
            "bottleneck_tflops": round(tm["flops_bottleneck"] / (b["ms"] * 1e-3) / 1e12, 1),
            "phase_ms_per_step": {k: round(tm[k]["ms"] / timed, 3) for k in ("decomp", "prime", "bottleneck",
                                                                              "nonprime", "trace")},
            "lnz_per_site": lz,
            "context": "the paper reports 510.76 s per step for 4D Ising chi=13 and 1247.65 s for chi=14 on "
                       "169 and 196 Xeon Phi nodes (chi=8..12 only plotted); not comparable hardware or size"}


def scan_4d(P, torch, form, chis, steps=6, first_timed=5, temp=6.68):
    """Time per coarse-graining step of 4D Ising HOTRG against chi (the paper's Section 5
    measurement: steps 1-4 excluded, the rest averaged), and the exponent p of a least-squares
    fit tau = alpha chi^p over the scanned chi."""
    import math
    rows = []
    for chi in chis:
        r = P.HOTRG("ising", 4, 1.0 / temp, chi, precision=form, max_steps=steps)
        per = []
        for p in range(1, steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.step()
            r.log_z()
            torch.cuda.synchronize()
            per.append(time.perf_counter() - t0)
            print(f"4D chi={chi} step {p}: {per[-1]:.3f} s", file=sys.stderr, flush=True)
        lz = r.log_z()
        r.close()
        timed = per[first_timed - 1:]
        rows.append({"chi": chi, "s_per_step": round(sum(timed) / len(timed), 4),
                     "s_per_step_all": [round(x, 4) for x in per], "lnz_per_site": lz})
    fit = None
    if len(rows) >= 2:
        xs = [math.log(x["chi"]) for x in rows]
        ys = [math.log(x["s_per_step"]) for x in rows]
        n = len(xs)
        mx, my = sum(xs) / n, sum(ys) / n
        slope = sum((x - mx) * (y - my) for x, y in zip(xs, ys)) / sum((x - mx) ** 2 for x in xs)
        alpha = math.exp(my - slope * mx)
        fit = {"exponent": round(slope, 2), "alpha_s": alpha,
               "projected_s_per_step": {str(c): round(alpha * c ** slope, 1) for c in (13, 14)}}
    return {"workload": f"4D Ising HOTRG, T={temp}, J=1, h=0; steps {first_timed}-{steps} averaged",
            "form": form, "rows": rows, "fit": fit,
            "context": "the paper fits tau = alpha chi^13 and reports 510.76 s (chi=13, 169 nodes) and "
                       "1247.65 s (chi=14, 196 nodes) per step on Xeon Phi; not comparable hardware"}


def host_info():
    """CPU model and BLAS library of the host that ran the oracle."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        info = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        if info:
            blas = f"{info[0].get('internal_api')} {info[0].get('version')}"
    except Exception:
        pass
    return model, blas


def cpu_baseline(sample_pairs=16):
    """The FP64 oracle on the host: a bounded sample of one saturated chi = 16 step --
    the new-tensor contraction restricted to `sample_pairs` of the 256 (n'_1, n'_2)
    slices, on a seeded random tensor (the cost does not depend on the values)."""
    import numpy as np
    from oracle import hotrg as H
    from tests import seeded_inputs as SI
    T = SI.random_tensor((CHI,) * 6, seed=0)
    U1 = SI.random_isometry(CHI * CHI, CHI, seed=1)
    U2 = SI.random_isometry(CHI * CHI, CHI, seed=2)
    picks = [(i // CHI, i % CHI) for i in range(0, CHI * CHI, (CHI * CHI) // sample_pairs)][:sample_pairs]
    t0 = time.perf_counter()
    H.new_tensor(T, {1: U1, 2: U2}, only=picks)
    dt = time.perf_counter() - t0
    frac = len(picks) / float(CHI * CHI)
    flops = 2.0 * (CHI ** 11 + 2 * CHI ** 9 + 2 * CHI ** 8) * frac
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        info = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        if info:
            threads = info[0].get("num_threads", threads)
    except Exception:
        pass
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(picks)}/256 (n'_1, n'_2) slices of one saturated chi=16 new-tensor contraction "
                      f"(FP64 NumPy, {dt:.1f} s); full-step estimate {dt / frac:.0f} s/step",
            "seconds_per_step_estimate": dt / frac}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="split_fp16")
    ap.add_argument("--reference-form", default="fp64")
    ap.add_argument("--reference-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the timing of the derivative mode")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched temperature sweep")
    ap.add_argument("--no-4d", action="store_true", help="skip the 4D HOTRG line")
    ap.add_argument("--only-4d", action="store_true", help="only the 4D HOTRG line (profiling)")
    ap.add_argument("--scan-4d", default="", help="only the 4D time per step at these chi (comma-separated)")
    ap.add_argument("--scan-steps", type=int, default=6, help="steps per chi of --scan-4d (steps 5.. timed)")
    ap.add_argument("--batch-only", action="store_true", help="only the batched temperature sweep (profiling)")
    ap.add_argument("--batch-no-graphs", action="store_true",
                    help="batched sweep enqueued kernel by kernel (for kernel tracing)")
    ap.add_argument("--no-reference", action="store_true",
                    help="skip the FP64 reference run (profiling runs of the headline form only)")
    ap.add_argument("--other-forms", default="fp32,split_bf16,fp16,bf16",
                    help="comma-separated forms also reported (2 timed steps each); empty for none")
    ap.add_argument("--mfma-ceiling", action="store_true", help="only the MFMA issue-rate probe")
    ap.add_argument("--counter-steps", type=int, default=0, help="only N steps with per-step output")
    ap.add_argument("--copy-calibration", type=int, default=0, help="only a device copy of MiB, three times")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "contraction over several GPUs is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2110_03607_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P.lib()
    if args.mfma_ceiling:
        print(json.dumps({"mfma_ceiling_tflops": mfma_ceiling(P, torch)}), flush=True)
        return
    if args.counter_steps:
        counter_steps(P, torch, args.form, args.counter_steps)
        return
    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return
    if args.batch_only:
        print(json.dumps({"batch_sweep": run_batch(P, torch, args.form, graphs=not args.batch_no_graphs)}), flush=True)
        return
    if args.scan_4d:
        chis = [int(x) for x in args.scan_4d.split(",")]
        print(json.dumps({"hotrg_4d_scan": scan_4d(P, torch, args.form, chis, args.scan_steps)}), flush=True)
        return
    if args.only_4d:
        print(json.dumps({"hotrg_4d": run_4d(P, torch, args.form)}), flush=True)
        return
    ref_lnz = fixture_lnz()

    ceiling = mfma_ceiling(P, torch)
    head = run_form(P, torch, args.form, args.steps, args.warmup)
    tm = head["timings"]
    ms_per_step = head["wall"] * 1e3 / args.steps
    contract_ms = tm["contract"]["ms"]
    contract_tflops = tm["flops_contract"] / (contract_ms * 1e-3) / 1e12
    bott_ms_avg = tm["bottleneck"]["ms"] / max(1, tm["bottleneck"]["count"])
    bott_flops_per_launch = tm["flops_bottleneck"] / max(1, tm["bottleneck"]["count"])
    bott_tflops = bott_flops_per_launch / (bott_ms_avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.form]
    err = None
    if ref_lnz is not None:
        n = min(len(ref_lnz), len(head["lnz"]))
        err = max(abs(head["lnz"][i] - ref_lnz[i]) / abs(ref_lnz[i]) for i in range(n))
        err_final = abs(head["lnz"][n - 1] - ref_lnz[n - 1]) / abs(ref_lnz[n - 1])

    ref_ms_per_step = ref_contract_tflops = ref_err = None
    if not args.no_reference:
        ref = run_form(P, torch, args.reference_form, args.reference_steps, 0)
        rtm = ref["timings"]
        ref_ms_per_step = ref["wall"] * 1e3 / args.reference_steps
        ref_contract_tflops = rtm["flops_contract"] / (rtm["contract"]["ms"] * 1e-3) / 1e12
        if ref_lnz is not None:
            n = min(len(ref_lnz), len(ref["lnz"]))
            ref_err = max(abs(ref["lnz"][i] - ref_lnz[i]) / abs(ref_lnz[i]) for i in range(n))

    forms = {}
    for form in [f for f in args.other_forms.split(",") if f]:
        res = run_form(P, torch, form, 2, 0)
        ftm = res["timings"]
        e = None
        if ref_lnz is not None:
            n = min(len(ref_lnz), len(res["lnz"]))
            e = max(abs(res["lnz"][i] - ref_lnz[i]) / abs(ref_lnz[i]) for i in range(n))
        forms[form] = {
            "ms_per_step": round(res["wall"] * 1e3 / 2, 3),
            "contract_tflops": round(ftm["flops_contract"] / (ftm["contract"]["ms"] * 1e-3) / 1e12, 3),
            "bottleneck_tflops": round(ftm["flops_bottleneck"] / (ftm["bottleneck"]["ms"] * 1e-3) / 1e12, 3),
            "free_energy_rel_err_vs_oracle": e,
        }

    deriv = {}
    if not args.no_grad:
        for form in ("fp32", "fp64"):
            res = run_form(P, torch, form, 1, 0, record_grad=True, finish=False)
            fwd_ms = forms[form]["ms_per_step"] if form in forms else (ref_ms_per_step if form == args.reference_form
                                                                         else None)
            deriv[form] = {"ms_per_step": round(res["wall"] * 1e3, 3), "forward_ms_per_step": fwd_ms,
                           "cost_vs_forward": round(res["wall"] * 1e3 / fwd_ms, 3) if fwd_ms else None,
                           "dlnz_dbeta_per_site_after_4_steps": res["grad"]}

    batch = None if args.no_batch else run_batch(P, torch, args.form)
    eig2d = None if args.no_batch else eigh_2d_chi32(P, torch)
    four_d = None if args.no_4d else run_4d(P, torch, args.form)

    out = {
        "metric": METRIC,
        "value": round(contract_tflops, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.form],
        "data": "synthetic",
        "config": {"workload": "3D Ising HOTRG, chi=16, T=4.5115, J=1, h=0; steps 1-3 unsaturated, "
                               f"timed steps {UNSATURATED + args.warmup + 1}-{UNSATURATED + args.warmup + args.steps}",
                   "form": args.form, "chi": CHI, "d": 3},
        "steps_per_s": round(1e3 / ms_per_step, 4),
        "contract_flops_per_step": tm["flops_contract"] / args.steps,
        "free_energy_rel_err_vs_oracle": err,
        "free_energy_rel_err_final": err_final if ref_lnz is not None else None,
        "phase_ms_per_step": {k: round(tm[k]["ms"] / args.steps, 3) for k in P.TIMING_PHASES},
        "roofline": {
            "bound": "mfma",
            "kernel": "k_gemm_big (bottleneck GEMM with the fused non-prime chain, eq. BottleneckPart)",
            "achieved": round(bott_tflops, 3),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(bott_tflops / peak, 4),
            "issued_frac": round(bott_tflops * PRODUCTS.get(args.form, 1) / peak, 4),
            "mfma_ceiling": ceiling[CEILING_KEY[args.form]],
            "issued_frac_of_ceiling": round(bott_tflops * PRODUCTS.get(args.form, 1) / ceiling[CEILING_KEY[args.form]], 4),
            "avg_launch_ms": round(bott_ms_avg, 4),
            "launches": tm["bottleneck"]["count"],
            "traffic": GEMM_TRAFFIC_BYTES.get(args.form),
            "traffic_algorithmic": GEMM_ALGO_BYTES.get(args.form),
        },
        "fp64_reference": None if args.no_reference else {
            "form": args.reference_form,
            "ms_per_step": round(ref_ms_per_step, 3),
            "steps_per_s": round(1e3 / ref_ms_per_step, 4),
            "contract_tflops": round(ref_contract_tflops, 3),
            "free_energy_rel_err_vs_oracle": ref_err,
            "speedup_of_headline_form": round(ref_ms_per_step / ms_per_step, 3),
        },
        "other_forms": forms,
        "derivative_mode": deriv,
        "batch_sweep": batch,
        "eigh_2d_chi32": eig2d,
        "hotrg_4d": four_d,
    }
    if not args.no_cpu:
        cb = cpu_baseline()
        out["cpu_baseline"] = {k: cb[k] for k in ("value", "unit", "cores", "kind", "sample")}
        out["cpu_baseline"]["value"] = round(cb["value"], 5)
        out["cpu_baseline"]["cpu_model"], out["cpu_baseline"]["blas"] = host_info()
        out["speedup_vs_oracle_steps"] = round(cb["seconds_per_step_estimate"] / (ms_per_step * 1e-3), 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
