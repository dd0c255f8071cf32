"""Reference traffic for HBM counters: one device-to-device copy of a known
size (torch's copy kernel), so that FETCH_SIZE / WRITE_SIZE readings of the
path kernels can be scaled by what the same counters report for exactly
`--mib` MiB read and written.

    python -m paper_2210_16998_amd.copyprobe --mib 1024
"""
import argparse

import torch


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    n = a.mib * (1 << 20) // 4
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    print(f"copied {a.mib} MiB in {ms:.3f} ms: {2 * a.mib / 1024 / (ms / 1e3):.0f} GiB/s "
          f"(read + write)", flush=True)


if __name__ == "__main__":
    main()
