"""The paper's own benchmark circuits and metrics on one GPU.

Workloads (generated from the paper's descriptions; see circuits): the Hadamard benchmark, eleven H gates on
every qubit (Sec. IV-D); the QSB circuit, ten sets of an RZ.RX.RZ rotation layer and a CNOT layer (target i,
control i+1 mod n) plus a final rotation layer (Sec. IV-F); the Quantum Volume model circuit of depth 10
(Sec. IV-E); one RX gate on every target qubit in turn for the per-target gate time (Sec. IV-C); the swap
ablation of Sec. III-D (s single swaps against one fused-swap); and `mixed28`, the 28-qubit circuit of U3, CZ,
RZ, Toffoli and fused-swap operations, with per-kernel-class algorithmic bandwidth on the plain path.

Each circuit runs on the plain path (one HBM pass per gate, as the paper's simulator applies them) and through
the block plan. Timing follows the paper's protocol (Sec. IV-B): six runs, the mean of the last five, each run
starting from |0..0> (the reset is outside the timed region), timed with HIP events on the state's stream.

Metrics: effective memory bandwidth = 2^(n+5) x #gates / time (Sec. IV-F; the paper counts one full read and
write of the state per gate), its fraction of the 8 TB/s HBM peak, and the quantum B/F ratio
QBF = 2^(n+5) x #gates / (time x peak FP64 FLOP/s) (Sec. IV-B) with MI355X's 78.6 TFLOP/s.

    python -m paper_2203_16044_amd.paperbench --n 30 [--workloads hadamard qsb qv rx swap] [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

HBM_PEAK = 8.0e12
FP64_PEAK = 78.6e12
RUNS = 6


def _timed(st, enqueue, torch, runs=RUNS):
    """Mean seconds of the last runs-1 of `runs` executions of enqueue() on the state's stream, each after a reset
    to |0..0> that is not timed."""
    times = []
    s = st.stream
    for _ in range(runs):
        st.init_zero()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        enqueue()
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    return sum(times[1:]) / (len(times) - 1)


def metrics(n, gates, t):
    eff = (2.0 ** (n + 5)) * gates / t
    return {"seconds": t, "gates_per_s": gates / t, "effective_tbs": eff / 1e12, "frac_of_hbm_peak": eff / HBM_PEAK,
            "qbf": eff / FP64_PEAK}


def run_circuit(circ, torch, modes=("plain", "block")):
    import paper_2203_16044_amd as qs
    from paper_2203_16044_amd.plan import Circuit, Plan
    n = circ.n
    st = qs.State(n, "c128")
    out = {"workload": circ.name, "n": n, "gates": len(circ.ops)}
    c = Circuit.from_ops(n, circ.ops)
    if "plain" in modes:
        out["plain"] = metrics(n, len(circ.ops), _timed(st, lambda: c.run_plain(st), torch))
    if "block" in modes:
        p = Plan(c, "block", 12, 4, "c128")
        out["block"] = metrics(n, len(circ.ops), _timed(st, lambda: p.run(st), torch))
        out["block"]["passes"] = p.info()["passes"]
        p.close()
    out["norm_after"] = st.norm()
    c.close()
    st.close()
    return out


def run_rx_sweep(n, torch, seed=0):
    """Per-target RX gate time (Sec. IV-C): each gate timed alone, six runs, mean of the last five."""
    import circuits as C
    import paper_2203_16044_amd as qs
    circ = C.rx_sweep(n, seed)
    st = qs.State(n, "c128")
    st.init_zero()
    rows = []
    for op in circ.ops:
        s = st.stream
        times = []
        for _ in range(RUNS):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            st.apply_op(op)
            e1.record(s)
            e1.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        t = sum(times[1:]) / (RUNS - 1)
        rows.append({"target": int(op.targets[0]), "ms": t * 1e3, "effective_tbs": (2.0 ** (n + 5)) / t / 1e12})
    st.close()
    return {"workload": f"rx_sweep_n{n}", "n": n, "per_target": rows,
            "min_tbs": min(r["effective_tbs"] for r in rows), "max_tbs": max(r["effective_tbs"] for r in rows)}


def _op_bytes_class(op, n, S):
    """(kernel class, algorithmic bytes) of one op on the plain path: every amplitude the op changes is read and
    written once (a diagonal's unit entries and a controlled gate's inactive half are not touched; a fused-swap
    leaves its 2^(n-s) fixed points alone)."""
    full = 2 * S * (1 << n)
    if op.kind == "dense":
        return f"dense_k{len(op.targets)}", full
    if op.kind == "diag":
        d = np.asarray(op.mat).reshape(-1)
        frac = float(np.mean(d != 1.0))
        return f"diag_k{len(op.targets)}", int(full * frac)
    if op.kind == "ctrl":
        return f"ctrl_c{len(op.controls)}_k{len(op.targets)}", full >> len(op.controls)
    return f"fswap_s{op.s}", int(full * (1 - 2.0 ** -op.s))


def run_per_class(circ, torch):
    """The plain path op by op with HIP events around each op: per kernel class, launches, mean ms and algorithmic
    TB/s (and the fraction of the 8 TB/s peak)."""
    import paper_2203_16044_amd as qs
    n = circ.n
    st = qs.State(n, "c128")
    st.init_zero()
    s = st.stream
    per = {}
    for rep in range(2):  # the first sweep warms up
        for op in circ.ops:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(s)
            st.apply_op(op)
            e1.record(s)
            e1.synchronize()
            if rep == 1:
                cls, nbytes = _op_bytes_class(op, n, 16)
                c = per.setdefault(cls, [0, 0.0, 0])
                c[0] += 1
                c[1] += e0.elapsed_time(e1) / 1e3
                c[2] += nbytes
    st.close()
    rows = {cls: {"launches": v[0], "avg_ms": v[1] / v[0] * 1e3, "tbs": v[2] / v[1] / 1e12,
                  "frac_of_hbm_peak": v[2] / v[1] / HBM_PEAK} for cls, v in sorted(per.items())}
    tot_t = sum(v[1] for v in per.values())
    return {"workload": f"{circ.name}_per_class", "n": n, "gates": len(circ.ops), "seconds": tot_t,
            "gates_per_s": len(circ.ops) / tot_t, "per_class": rows}


def run_swap_ablation(n, torch, p=0, s_max=6):
    """Swap insertion against fused-swap in HBM (Sec. III-D, Fig. 2): for s = 1..s_max, s single swaps
    swap(p+j, q+j) against one fused_swap(p, q, s) with q = n - s_max. Both give the same permutation; the bytes
    differ: each single swap moves half of the state, the fused-swap a 1 - 2^-s share of it once."""
    import paper_2203_16044_amd as qs
    S = 16
    q = n - s_max
    a = qs.State(n, "c128")
    b = qs.State(n, "c128")
    rows = []
    for s in range(1, s_max + 1):
        idx = torch.arange(1 << n, dtype=torch.float64, device="cuda")
        for st in (a, b):
            st.buf.real.copy_(idx)
            st.buf.imag.copy_(-idx)
        del idx
        t_single = _timed_noreset(a, lambda: [a.fused_swap(p + j, q + j, 1) for j in range(s)], torch)
        t_fused = _timed_noreset(b, lambda: b.fused_swap(p, q, s), torch)
        torch.cuda.synchronize()
        same = bool(torch.equal(a.buf.view(torch.int64), b.buf.view(torch.int64)))  # RUNS applications each
        bytes_single = s * S * (1 << n)  # 2 x S x 2^n / 2 per swap
        bytes_fused = int(2 * S * (1 << n) * (1 - 2.0 ** -s))
        rows.append({"s": s, "p": p, "q": q, "single_ms": t_single * 1e3, "fused_ms": t_fused * 1e3,
                     "single_bytes": bytes_single, "fused_bytes": bytes_fused,
                     "byte_ratio": bytes_single / bytes_fused, "time_ratio": t_single / t_fused,
                     "single_tbs": bytes_single / t_single / 1e12, "fused_tbs": bytes_fused / t_fused / 1e12,
                     "bit_identical": same})
    a.close()
    b.close()
    return {"workload": f"swap_ablation_n{n}", "n": n, "rows": rows}


def _timed_noreset(st, enqueue, torch, runs=RUNS):
    times = []
    s = st.stream
    for _ in range(runs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        enqueue()
        e1.record(s)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    return sum(times[1:]) / (len(times) - 1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--n", type=int, default=30)
    ap.add_argument("--workloads", nargs="*", default=["hadamard", "qsb", "qv", "rx", "swap"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    import torch

    import circuits as C
    torch.cuda.set_device(0)
    res = {"n": args.n, "protocol": "6 runs, mean of the last 5, reset outside the timed region",
           "hbm_peak_tbs": HBM_PEAK / 1e12, "fp64_peak_tflops": FP64_PEAK / 1e12, "results": []}
    gen = {"hadamard": lambda: C.hadamard_x11(args.n), "qsb": lambda: C.qsb(args.n, args.seed),
           "qv": lambda: C.quantum_volume(args.n, args.seed), "mixed28": lambda: C.mixed_layers()}
    for w in args.workloads:
        t0 = time.perf_counter()
        if w == "rx":
            r = run_rx_sweep(args.n, torch, args.seed)
        elif w == "swap":
            r = run_swap_ablation(args.n, torch)
        elif w == "mixed28":
            r = run_circuit(gen[w](), torch)
            r["plain_per_class"] = run_per_class(gen[w](), torch)["per_class"]
        else:
            r = run_circuit(gen[w](), torch)
        r["wall_s"] = time.perf_counter() - t0
        res["results"].append(r)
        print(json.dumps(r), flush=True)
        torch.cuda.empty_cache()
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f, indent=1)
    return res


if __name__ == "__main__":
    sys.exit(0 if main() else 1)
