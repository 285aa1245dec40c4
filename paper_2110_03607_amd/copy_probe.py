"""Plain device-to-device copy of a known size, the reference for reading HBM traffic
counters: run it under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE) next to the kernel
being measured; the counter value of this copy, divided by the bytes it moves, is the
factor that turns the counter into bytes.

Usage: python -m paper_2110_03607_amd.copy_probe [MiB]
"""

import sys


def main():
    import torch

    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB three times ({3 * mib * 1024} KiB read and written)", flush=True)


if __name__ == "__main__":
    main()
