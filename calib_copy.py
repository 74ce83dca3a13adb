"""Plain device-to-device copy of a known size, used to calibrate the HBM
byte counters (FETCH_SIZE / WRITE_SIZE) read by rocprofv3.

    python calib_copy.py [MiB] [repeats]

Each launch reads and writes MiB mebibytes once.
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 1024
    reps = int(sys.argv[2]) if len(sys.argv) > 2 else 5
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x {reps}")


if __name__ == "__main__":
    main()
