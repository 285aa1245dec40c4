"""Write oracle fixtures for the physics configurations (calls only oracle/).

Usage:  python tests/golden/make_golden.py config1 config2 [config3 ...]
        python tests/golden/make_golden.py grad_config5 BETA [STEPS]

The script refuses to run while oracle/, this script or tests/seeded_inputs.py differ from
the committed tree, so that the commit stamped into every fixture is the code that wrote it.

Each fixture is JSON: the configuration, per-run lnZ/V after every step, the
trace t_p, the Gu-Wen ratio, the judgement values and the leading normalised
spectrum of every decomposed Gram matrix, plus provenance (oracle commit, host,
cores, wall time).  Stored values come from the FP64 oracle and nothing else.
"""

import json
import math
import os
import platform
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import hotrg as H  # noqa: E402
from oracle import tangent as TG  # noqa: E402
from tests import seeded_inputs as SI  # noqa: E402


def dump_json(doc, path):
    """Write `doc` to `path` through a temporary file and a rename, so that a reader never sees
    a partly written fixture while a long run is still adding to it."""
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(doc, f, indent=1)
    os.replace(tmp, path)



N_SPEC = 24


def _record(rec):
    out = dict(p=rec.p, lnz_per_site=rec.lnz_per_site, trace=rec.trace, gu_wen=rec.gu_wen,
               dims_before=list(rec.dims_before), dirs={})
    for j, t in rec.truncations.items():
        lam, lam_p = t.lam, t.lam_p
        out["dirs"][str(j)] = dict(
            chi_new=t.chi_new, kept=t.kept, eps=t.eps, eps_p=t.eps_p, chose_prime=bool(t.chose_prime),
            spec=[float(x / lam[0]) for x in lam[:N_SPEC]],
            spec_p=[float(x / lam_p[0]) for x in lam_p[:N_SPEC]],
            gap=float((lam[t.chi_new - 1] - lam[t.chi_new]) / lam[0]) if t.chi_new < lam.size else None,
        )
    return out


def run_config(name, cfg, betas):
    runs = []
    for beta in betas:
        t0 = time.time()
        step_times = []
        last = [time.time()]

        def on_step(rec):
            now = time.time()
            step_times.append(now - last[0])
            last[0] = now
            print(f"  {name} beta={beta:.6f} step {rec.p} lnz/V={rec.lnz_per_site:.15f} "
                  f"({step_times[-1]:.1f}s)", flush=True)

        model = H.Model(cfg["kind"], cfg["d"], cfg["q"])
        lnz0, recs = H.run(model, beta, cfg["chi"], cfg["steps"], on_step=on_step)
        runs.append(dict(beta=beta, lnz0=lnz0, steps=[_record(r) for r in recs],
                         step_seconds=step_times, wall_seconds=time.time() - t0))
    return runs


# Files whose committed state a fixture depends on.
SOURCES = ("oracle", "tests/golden/make_golden.py", "tests/seeded_inputs.py")


def committed_revision():
    """HEAD, after checking that the oracle and the input generators have no uncommitted
    changes (else the stamp would name code other than the code that ran)."""
    dirty = subprocess.check_output(["git", "-C", ROOT, "status", "--porcelain", "--", *SOURCES], text=True)
    if dirty.strip():
        raise SystemExit("make_golden.py: uncommitted changes in " + ", ".join(SOURCES) + ":\n" + dirty
                         + "commit them first; the fixture records the commit that wrote it")
    return subprocess.check_output(["git", "-C", ROOT, "rev-parse", "HEAD"], text=True).strip()


REVISION = None


def provenance():
    rev = REVISION
    cpu = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(oracle_commit=rev, host_cpu=cpu, cores=os.cpu_count(),
                numpy_blas_threads=os.environ.get("OMP_NUM_THREADS", "default"))


# d(lnZ/V)/dbeta cases: (kind, d, q, beta, chi, steps); 2D chi = 16 reaches n = 256 Gram
# matrices, 3D Potts chi = 9 has S3 doublets and multiplet cuts.  The 2D Potts run at
# beta = 1.0 (near its critical point) stops at step 14: from step 16 on, its cuts sit in
# clusters with relative gaps of 1e-6 to 1e-9, where the kept subspace moves by about
# (rounding of A) / gap, so two correct FP64 implementations part at the 1e-8 level.
GRAD_CASES = [
    ("ising", 2, 2, 0.44, 16, 20),
    ("potts", 2, 3, 1.0, 16, 14),
    ("potts", 3, 3, 0.55, 9, 8),
]


def run_grad():
    runs = []
    for kind, d, q, beta, chi, steps in GRAD_CASES:
        t0 = time.time()
        lnz0, dlnz0, recs = TG.run_with_tangent(H.Model(kind, d, q), beta, chi, steps)
        runs.append(dict(kind=kind, d=d, q=q, beta=beta, chi=chi, steps=steps, lnz0=lnz0, dlnz0=dlnz0,
                         lnz=[r[0] for r in recs], dlnz=[r[1] for r in recs], wall_seconds=time.time() - t0))
        print(f"  grad {kind} d={d} chi={chi} beta={beta}: dlnz/dbeta={recs[-1][1]:.15f} "
              f"({time.time() - t0:.1f}s)", flush=True)
    return runs


# Batched sweep: the instances of the sweep checked against the oracle -- every 4th 3D
# temperature and the last one (17 of 64), and all 48 2D instances.
CONFIG4_SAMPLE_3D = tuple(range(0, 64, 4)) + (63,)
CONFIG4_SAMPLE_2D = tuple(range(48))


def run_config4(write):
    """Runs the sampled instances one by one; write(runs) is called after each (partial file)."""
    c3, c2 = SI.CONFIG4_3D, SI.CONFIG4_2D
    runs = []
    for i in CONFIG4_SAMPLE_2D:
        chi = c2["chis"][i % len(c2["chis"])]
        cfg = dict(kind=c2["kind"], d=2, q=2, chi=chi, steps=c2["steps"])
        r = run_config(f"config4 2D[{i}]", cfg, [float(c2["betas"][i])])[0]
        r.update(index=i, d=2, chi=chi)
        runs.append(r)
        write(runs)
    for i in CONFIG4_SAMPLE_3D:
        cfg = dict(kind=c3["kind"], d=3, q=2, chi=c3["chi"], steps=c3["steps"])
        r = run_config(f"config4 3D[{i}]", cfg, [1.0 / c3["temps"][i]])[0]
        r.update(index=i, d=3, chi=c3["chi"])
        runs.append(r)
        write(runs)
    return runs


def grad_config5_path(beta):
    return os.path.join(HERE, f"grad_config5_beta{beta:.2f}.json")


def run_grad_config5(beta, steps):
    """The oracle's forward-mode derivative for 3D 3-state Potts, chi = 16 (the derivative
    configuration) at one beta; the file is rewritten after every step, so that a partial
    run leaves the steps it finished (`steps_done`)."""
    cfg = SI.CONFIG5
    t0 = time.time()
    doc = dict(config="grad_config5", kind=cfg["kind"], d=cfg["d"], q=cfg["q"], chi=cfg["chi"], beta=beta,
               steps_planned=steps, steps_done=0, lnz=[], dlnz=[], step_seconds=[], provenance=provenance(),
               source="oracle/tangent.py (FP64 NumPy), written by tests/golden/make_golden.py")
    last = [time.time()]

    def on_step(p, lnz, dlnz):
        now = time.time()
        doc["lnz"].append(lnz)
        doc["dlnz"].append(dlnz)
        doc["step_seconds"].append(now - last[0])
        doc["steps_done"] = p
        doc["wall_seconds"] = now - t0
        last[0] = now
        dump_json(doc, grad_config5_path(beta))
        print(f"  grad_config5 beta={beta:.2f} step {p} lnz/V={lnz:.15f} dlnz/dbeta={dlnz:.15f} "
              f"({doc['step_seconds'][-1]:.0f}s)", flush=True)

    lnz0, dlnz0, _ = TG.run_with_tangent(H.Model(cfg["kind"], cfg["d"], cfg["q"]), beta, cfg["chi"], steps,
                                          on_step=on_step)
    doc.update(lnz0=lnz0, dlnz0=dlnz0)
    dump_json(doc, grad_config5_path(beta))
    print("wrote", grad_config5_path(beta), flush=True)


def main(names):
    global REVISION
    REVISION = committed_revision()
    if names and names[0] == "grad_config5":
        beta = float(names[1])
        steps = int(names[2]) if len(names) > 2 else 6
        run_grad_config5(beta, steps)
        return
    if "config4" in names:
        path = os.path.join(HERE, "config4.json")

        def write(runs):
            doc = dict(config="config4", runs=runs, steps=SI.CONFIG4_3D["steps"], provenance=provenance(),
                       source="oracle/hotrg.py (FP64 NumPy), written by tests/golden/make_golden.py")
            dump_json(doc, path)

        run_config4(write)
        print("wrote", path, flush=True)
        names = [n for n in names if n != "config4"]
    if "grad" in names:
        doc = dict(config="grad", runs=run_grad(), provenance=provenance(),
                   source="oracle/tangent.py (FP64 NumPy), written by tests/golden/make_golden.py")
        path = os.path.join(HERE, "grad.json")
        dump_json(doc, path)
        print("wrote", path, flush=True)
        names = [n for n in names if n != "grad"]
    table = {
        "config1": (SI.CONFIG1, [1.0 / T for T in SI.CONFIG1["temps"]]),
        "config2": (SI.CONFIG2, [1.0 / T for T in SI.CONFIG2["temps"]]),
        "config3": (SI.CONFIG3, [1.0 / T for T in SI.CONFIG3["temps"]]),
        "config5": (SI.CONFIG5, list(SI.CONFIG5["betas"])),
        "config6": (SI.CONFIG6, [1.0 / T for T in SI.CONFIG6["temps"]]),
        "config7": (SI.CONFIG7, [1.0 / T for T in SI.CONFIG7["temps"]]),
    }
    for name in names:
        cfg, betas = table[name]
        runs = run_config(name, cfg, betas)
        doc = dict(config=name, kind=cfg["kind"], d=cfg["d"], q=cfg["q"], chi=cfg["chi"],
                   steps=cfg["steps"], runs=runs, provenance=provenance(),
                   source="oracle/hotrg.py (FP64 NumPy), written by tests/golden/make_golden.py")
        path = os.path.join(HERE, f"{name}.json")
        dump_json(doc, path)
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["config1", "config2"])
