"""Bandwidth probes: a plain device copy and an in-place read-modify-write of known size, timed with HIP events on
the stream they run on. They give the measured HBM ceiling the gate kernels are compared with, and the bytes a
hardware counter should report for a known amount of traffic (the calibration of FETCH_SIZE / WRITE_SIZE).

    python -m paper_2203_16044_amd.probe copy --gib 16 --reps 3
    python -m paper_2203_16044_amd.probe rmw --gib 64 --reps 3
"""
from __future__ import annotations

import argparse
import json

from . import binding as B


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["copy", "rmw"])
    ap.add_argument("--gib", type=float, default=16.0, help="bytes copied (copy) or buffer size (rmw), GiB")
    ap.add_argument("--reps", type=int, default=3)
    args = ap.parse_args()
    import torch
    nbytes = int(args.gib * (1 << 30)) // 256 * 256
    s = torch.cuda.current_stream()
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    buf.zero_()
    if args.kind == "copy":
        dst = torch.empty_like(buf)
        run = lambda: B.qs_probe_copy(dst.data_ptr(), buf.data_ptr(), nbytes, s.cuda_stream)  # noqa: E731
        moved = 2 * nbytes
    else:
        run = lambda: B.qs_probe_rmw(buf.data_ptr(), nbytes, s.cuda_stream)  # noqa: E731
        moved = 2 * nbytes
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run()
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    best = min(times)
    print(json.dumps({"probe": args.kind, "bytes_read": nbytes, "bytes_written": nbytes, "launches": args.reps + 1,
                      "best_ms": best * 1e3, "tbs": moved / best / 1e12}), flush=True)


if __name__ == "__main__":
    main()
