#!/usr/bin/env python
"""Throughput benchmark of the state-vector gate path on one MI355X.

Workload: the 32-qubit complex128 random circuit (40 layers; per layer a random qubit pairing with a Haar
SU(4) on every pair, then a random U3 on every qubit; 1,920 gates), a synthetic stand-in for the paper's
Quantum Volume / QSB suites (Sec. IV-E, IV-F). One step = reset to |0..0>, apply the whole circuit, FP64 norm
(the probability reduction) -- every step of the hot path -- with the state resident in HBM.

Reported: gates/s of the timed steps (whole job, one GPU); the dominant kernel's achieved HBM bandwidth against
the 8 TB/s peak, from HIP events recorded around every launch on the stream the kernels run on; the FP64 CPU
oracle timed on the host's cores over a bounded sample of the same circuit.

Modes: "plain" applies the circuit gate by gate (one HBM pass per gate); "tuned" runs the fused plan (see
paper_2203_16044_amd.plan) and also reports plain on a prefix of the circuit for the speedup.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_TBS = 8.0  # MI355X HBM3E, published


def _alg_bytes(op, n, amp):
    """Algorithmic bytes one op moves (read + write of every amplitude it changes)."""
    full = 2 * amp * (1 << n)
    if op.kind == "dense":
        return full
    if op.kind == "diag":
        return full  # the circuits here use diagonals with no unit entries
    if op.kind == "ctrl":
        return full >> len(op.controls)
    if op.kind == "fswap":
        return int(full * (1 - 2.0 ** -op.s))
    raise ValueError(op.kind)


def _kernel_class(op):
    if op.kind == "dense":
        return f"dense_k{len(op.targets)}"
    if op.kind == "ctrl":
        return f"ctrl_k{len(op.targets)}"
    return op.kind


def run_plain(st, ops, events, torch):
    """Apply ops one at a time; events[i] = (start, end) recorded around op i on the state's stream."""
    s = st.stream
    for i, op in enumerate(ops):
        events[i][0].record(s)
        st.apply_op(op)
        events[i][1].record(s)


def cpu_baseline(circ, budget_s, torch):
    """The FP64 oracle on the host's cores over the first ops of the same circuit (bounded by budget_s)."""
    import numpy as np
    import oracle

    n = circ.n
    need = 16 * (1 << n)
    try:
        import psutil
        avail = psutil.virtual_memory().available
    except Exception:
        avail = 0
    n_run = n
    while n_run > 20 and need * (1 << (n_run - n)) * 1.3 > avail:
        n_run -= 1
    ops = [o for o in circ.ops if max(o.qubits()) < n_run] if n_run < n else list(circ.ops)
    psi = oracle.zero_state(n_run)
    done, t0 = 0, time.perf_counter()
    for op in ops:
        oracle.apply_op(psi, op)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    rate = done / dt * (2.0 ** (n_run - n))
    sample = f"first {done} gates of the same circuit on a {n_run}-qubit state ({16 << n_run >> 30} GiB)"
    if n_run < n:
        sample += f", gates/s scaled by 2^({n_run}-{n}) to {n} qubits"
    del psi
    return {"value": rate, "unit": "gates/s", "cores": oracle.oracle_threads(), "kind": "oracle", "sample": sample,
            "seconds": round(dt, 2)}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--mode", choices=["plain", "tuned"], default="plain")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the gate path is single-GPU (multi-GPU sharding is a design note only). "
              "Run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import circuits as C
    import paper_2203_16044_amd as qs

    torch.cuda.set_device(0)
    circ = C.config2(n=args.n, seed=32, layers=args.layers)
    ops = circ.ops
    n = circ.n
    st = qs.State(n, "c128")
    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    events = [(mk(), mk()) for _ in ops]
    step_ev = (mk(), mk())

    def step(record):
        st.init_zero()
        if record:
            run_plain(st, ops, events, torch)
        else:
            for op in ops:
                st.apply_op(op)
        return qs.binding.qs_probs(st.h, None, False)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    step_times, per_class = [], {}
    t0 = time.perf_counter()
    for k in range(args.steps):
        step_ev[0].record(st.stream)
        step(True)
        step_ev[1].record(st.stream)
        step_ev[1].synchronize()
        step_times.append(step_ev[0].elapsed_time(step_ev[1]) / 1e3)
        for op, (e0, e1) in zip(ops, events):
            c = per_class.setdefault(_kernel_class(op), [0.0, 0, 0])
            c[0] += e0.elapsed_time(e1) / 1e3
            c[1] += 1
            c[2] += _alg_bytes(op, n, 16)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nrm = st.norm()
    st.close()

    t_step = sum(step_times) / len(step_times)
    gates = len(ops)
    dom = max(per_class, key=lambda c: per_class[c][0])
    tsum, cnt, bsum = per_class[dom]
    avg = tsum / cnt
    achieved = (bsum / cnt) / avg / 1e12
    alg_total = sum(_alg_bytes(o, n, 16) for o in ops)
    out = {
        "metric": "gates/s, 32-qubit complex128 random circuit (SU(4) pairings + U3, 40 layers)",
        "value": gates / t_step,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"random SU(4)+U3 circuit, n={n}, {args.layers} layers, {gates} gates, complex128 "
                               f"(seed 32)", "n": n, "gates": gates, "mode": args.mode, "parallelism": "none"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_TBS, "unit": "TB/s",
                     "frac": achieved / HBM_PEAK_TBS, "traffic": None, "kernel": dom,
                     "avg_launch_ms": avg * 1e3, "launches_per_step": cnt // args.steps,
                     "alg_bytes_per_launch": bsum // cnt},
        "hbm_tbs_whole_step": alg_total / t_step / 1e12,
        "paper_nominal_tbs": (1 << (n + 5)) * gates / t_step / 1e12,
        "per_kernel": {c: {"launches": v[1] // args.steps, "avg_ms": v[0] / v[1] * 1e3,
                           "tbs": v[2] / v[0] / 1e12} for c, v in sorted(per_class.items())},
        "norm_after": nrm,
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, args.cpu_seconds, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
