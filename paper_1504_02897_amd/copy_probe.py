"""HBM counter calibration: a plain device-to-device copy of a known size.

Used when reading rocprofv3 FETCH_SIZE / WRITE_SIZE counters: the counters of this copy
give the factor between counted and actual bytes on the device it runs on.

    python -m paper_1504_02897_amd.copy_probe [MiB]
"""
import sys

import torch


def main():
    mib = int(sys.argv[1]) if len(sys.argv) > 1 else 256
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"copied {mib} MiB x 3", flush=True)


if __name__ == "__main__":
    main()
