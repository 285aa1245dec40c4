"""A short run of the headline workload for counter collection: 3D Ising, chi = 16, T = 4.5115,
split FP16, N coarse-graining steps (default 6: steps 4-6 saturated), printing lnZ/V after each
step so that a profiler-wrapped run shows progress.

    python3 -m paper_2110_03607_amd.step_probe [steps]
"""

import sys

import torch

import paper_2110_03607_amd as P


def main() -> None:
    steps = int(sys.argv[1]) if len(sys.argv) > 1 else 6
    P.lib()
    assert torch.cuda.is_available(), "step_probe needs a GPU"
    r = P.HOTRG("ising", 3, 1.0 / 4.5115, 16, precision="split_fp16", max_steps=steps)
    for p in range(steps):
        r.step()
        print("step", p + 1, "lnZ/V", r.log_z(), flush=True)
    r.close()


if __name__ == "__main__":
    main()
