"""Calibration run for hardware byte counters: copies a buffer of known size
a few times with a plain device copy, so that a counter profile of this
script gives the counter's reading per byte actually moved.

    rocprofv3 --pmc FETCH_SIZE -- python calib_copy.py
"""
import sys

import torch

MIB = 256
REPS = 5


def main():
    n = MIB * (1 << 20) // 4
    src = torch.rand(n, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(REPS):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {MIB} MiB x {REPS} (read {MIB} MiB and write {MIB} MiB per copy)", flush=True)


if __name__ == "__main__":
    sys.exit(main())
