"""Plain device copy of a known size, used to calibrate rocprofv3's
FETCH_SIZE / WRITE_SIZE counters (bytes reported per byte actually moved).

    python3 -m paper_2606_30495_amd.calib [--mib 1024] [--reps 3]
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copy kernel: {a.reps} launches, {n * 4} bytes read and {n * 4} bytes written per launch",
          flush=True)


if __name__ == "__main__":
    main()
