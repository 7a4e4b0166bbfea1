"""Plain device-to-device copy of a known size, for scaling HBM traffic
counters: run under rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) and divide
the known bytes per copy by the counter's reading per dispatch.

Usage: python paper_1708_03621_amd/pmc_calibrate.py [--mib 256] [--reps 4]
"""
import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=256)
    ap.add_argument("--reps", type=int, default=4)
    args = ap.parse_args()
    import torch
    n = args.mib * 1024 * 1024 // 8
    x = torch.arange(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(args.reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8, "copies": args.reps}))


if __name__ == "__main__":
    main()
