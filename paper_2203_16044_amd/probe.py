"""Bandwidth probes: a plain device copy and an in-place read-modify-write of known size, timed with HIP events on
the stream they run on. They give the measured HBM ceiling the gate kernels are compared with, and the bytes a
hardware counter should report for a known amount of traffic (the calibration of FETCH_SIZE / WRITE_SIZE). The
`gate` probe times one dense k-qubit gate (a fixed random unitary on qubits `--first` .. `--first` + k - 1) on an
n-qubit state, for per-kernel profiles (k = 5, 6 run on the matrix cores).

    python -m paper_2203_16044_amd.probe copy --gib 16 --reps 3
    python -m paper_2203_16044_amd.probe rmw --gib 64 --reps 3
    python -m paper_2203_16044_amd.probe gate --n 30 --k 6 --dtype c64 --reps 3
"""
from __future__ import annotations

import argparse
import json

from . import binding as B


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["copy", "rmw", "gate"])
    ap.add_argument("--gib", type=float, default=16.0, help="bytes copied (copy) or buffer size (rmw), GiB")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--n", type=int, default=30, help="gate: qubits of the state")
    ap.add_argument("--k", type=int, default=6, help="gate: target count")
    ap.add_argument("--first", type=int, default=0, help="gate: lowest target")
    ap.add_argument("--dtype", choices=["c128", "c64"], default="c128")
    args = ap.parse_args()
    import torch
    if args.kind == "gate":
        gate_probe(args, torch)
        return
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


def gate_probe(args, torch) -> None:
    import numpy as np

    from .state import State
    if not (1 <= args.k <= 6 and 0 <= args.first and args.first + args.k <= args.n):
        raise SystemExit("gate probe: need 1 <= k <= 6 and first + k <= n")
    rng = np.random.Generator(np.random.PCG64(args.k))
    z = rng.standard_normal((1 << args.k, 1 << args.k)) + 1j * rng.standard_normal((1 << args.k, 1 << args.k))
    q, r = np.linalg.qr(z)
    U = np.ascontiguousarray(q * (np.diag(r) / np.abs(np.diag(r))))
    targets = list(range(args.first, args.first + args.k))
    st = State(args.n, args.dtype)
    st.init_zero()
    s = st.stream
    run = lambda: B.qs_apply_gate(st.h, targets, U)  # noqa: E731
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
    amp = 16 if args.dtype == "c128" else 8
    nbytes = 2 * amp * (1 << args.n)
    flops = 8 * (1 << args.k) * (1 << args.n)
    print(json.dumps({"probe": "gate", "n": args.n, "k": args.k, "targets": targets, "dtype": args.dtype,
                      "launches": args.reps + 1, "best_ms": best * 1e3, "tbs": nbytes / best / 1e12,
                      "tflops": flops / best / 1e12}), flush=True)
    st.close()


if __name__ == "__main__":
    main()
