#!/usr/bin/env python
"""Throughput benchmark of the state-vector gate path on one MI355X.

Workload: the 32-qubit complex128 random circuit (40 layers; per layer a random qubit pairing with a Haar
SU(4) on every pair, then a random U3 on every qubit; 1,920 gates), a synthetic stand-in for the paper's
Quantum Volume / QSB suites (Sec. IV-E, IV-F). One step = reset to |0..0>, apply the whole circuit, FP64 norm
(the probability reduction) -- every step of the hot path -- with the state resident in HBM.

Reported: gates/s of the timed steps (whole job, one GPU); the dominant kernel's achieved rate against its binding
roof (HBM at 8 TB/s or FP64 at 78.6 TFLOP/s, both fractions given), from HIP events recorded around every launch on
the stream the kernels run on, with its PMC-measured HBM traffic; the FP64 CPU oracle timed on the host's cores
over a bounded sample of the same circuit.

Modes: "plain" applies the circuit gate by gate (one HBM pass per gate); "tuned" runs the fused plan (see
paper_2203_16044_amd.plan) and also reports plain on a prefix of the circuit for the speedup.

Further legs in the same JSON line: "c64" (the 33-qubit complex64 circuit of the same family with FP64
renormalisation every 10 layers, planned once in the block shape the cost model predicts fastest and renormalised at
the first pass boundary after each such layer completes, folded into the block passes; the layer-exact segmented
form beside it; and the complex64 error at 24 qubits) and "batch" (512 circuits of 10-22 qubits,
one persistent launch per pass level, autotuned, eager and graph-replayed, against the per-circuit plain loop).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_TBS = 8.0  # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (= FP64 MFMA): 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz

# HBM traffic per dispatch of the dominant kernels, from two rocprofv3 PMC runs of this script (FETCH_SIZE, then
# WRITE_SIZE; KiB per dispatch, mean over the 32-qubit dispatches of the headline plan), each scaled by what the same counter reads for
# a device copy of known size (paper_2203_16044_amd.probe copy of 4 GiB: FETCH_SIZE reports 2097197 KiB, half of
# the bytes read, WRITE_SIZE 4194304 KiB, all bytes written). Commands and figures: profiles/*_pmc_traffic.md.
# The readings hold for the kernel sources they were taken on: `sha1` fingerprints those files and the traffic is
# reported as null once they differ.
PMC_TRAFFIC = {
    "block_b12": {"fetch_kib": 33555491.49, "write_kib": 67110167.04, "fetch_scale": 2.0, "write_scale": 1.0,
                  "sources": ["paper_2203_16044_amd/csrc/qs_block.hip", "paper_2203_16044_amd/csrc/qs_internal.h",
                              "paper_2203_16044_amd/csrc/qs_index.h"],
                  "sha1": "b3ddcbca772e1ce3187d75f0d5ebf2337aa1b5cf"},
    "dense_k1": {"fetch_kib": 33554446.82, "write_kib": 67110458.13, "fetch_scale": 2.0, "write_scale": 1.0,
                 "sources": ["paper_2203_16044_amd/csrc/qs_kernels.hip", "paper_2203_16044_amd/csrc/qs_internal.h",
                             "paper_2203_16044_amd/csrc/qs_index.h"],
                 "sha1": "efb0a8143d298d41669494079806e581b2822d18"},
}


def sources_sha1(paths):
    import hashlib
    h = hashlib.sha1()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel):
    """HBM bytes per dispatch of `kernel` from the recorded PMC readings, or None if there are none or the kernel's
    sources changed since."""
    t = PMC_TRAFFIC.get(kernel)
    if not t or t["fetch_kib"] is None or t["write_kib"] is None or t["sha1"] != sources_sha1(t["sources"]):
        return None
    return int(round(t["fetch_kib"] * 1024 * t["fetch_scale"] + t["write_kib"] * 1024 * t["write_scale"]))


def _alg_bytes(op, n, amp):
    """Algorithmic bytes one op moves (read + write of every amplitude it changes)."""
    full = 2 * amp * (1 << n)
    if op.kind == "dense":
        return full
    if op.kind == "diag":  # only amplitudes whose entry is not exactly 1 change
        d = op.mat.ravel()
        return full * int(sum(1 for x in d if x != 1)) // len(d)
    if op.kind == "ctrl":
        return full >> len(op.controls)
    if op.kind == "fswap":
        return int(full * (1 - 2.0 ** -op.s))
    raise ValueError(op.kind)


def _line_bytes(op, n, amp):
    """Bytes of the 128-byte lines that hold an amplitude the op changes, each read and written once: the
    line-granular roof of any pass, since HBM moves whole lines (a CZ on qubits 0 and 1 changes a quarter of the
    amplitudes but every line)."""
    full = 2 * amp * (1 << n)
    lb = 3 if amp == 16 else 4  # index bits inside a 128-byte line
    if op.kind == "dense":
        return full
    if op.kind == "fswap":
        q = [op.p + j for j in range(op.s)] + [op.q + j for j in range(op.s)]
        changed = lambda b: any(b[j] != b[op.s + j] for j in range(op.s))  # noqa: E731
    elif op.kind == "diag":
        q = list(op.targets)
        d = op.mat.ravel()
        changed = lambda b: d[sum(x << j for j, x in enumerate(b))] != 1  # noqa: E731
    elif op.kind == "ctrl":
        nc = len(op.controls)
        q = list(op.controls) + list(op.targets)
        changed = lambda b: all(b[:nc])  # noqa: E731
    else:
        raise ValueError(op.kind)
    inside = [i for i, x in enumerate(q) if x < lb]
    above = [i for i, x in enumerate(q) if x >= lb]
    touched = 0
    for hp in range(1 << len(above)):
        for lp in range(1 << len(inside)):
            b = [0] * len(q)
            for j, i in enumerate(above):
                b[i] = (hp >> j) & 1
            for j, i in enumerate(inside):
                b[i] = (lp >> j) & 1
            if changed(b):
                touched += 1
                break
    return full * touched // (1 << len(above))


def _alg_flops(op, n):
    """Flops one op performs (complex arithmetic counted in real flops: 8 per complex multiply-add)."""
    if op.kind == "dense":
        return 8 * (1 << len(op.targets)) * (1 << n)
    if op.kind == "diag":
        return 6 * (1 << n)
    if op.kind == "ctrl":
        return 8 * (1 << len(op.targets)) * (1 << (n - len(op.controls)))
    return 0


def _kernel_class(op):
    if op.kind == "dense":
        return f"dense_k{len(op.targets)}"
    if op.kind == "ctrl":
        return f"ctrl_k{len(op.targets)}"
    return op.kind


def run_plain(st, ops, events):
    """Apply ops one at a time; events[i] = (start, end) recorded around op i on the state's stream."""
    s = st.stream
    for i, op in enumerate(ops):
        events[i][0].record(s)
        st.apply_op(op)
        events[i][1].record(s)


def run_plan(st, plan, npass, events):
    s = st.stream
    for i in range(npass):
        events[i][0].record(s)
        plan.run(st, i, i + 1)
        events[i][1].record(s)


def time_steps(st, steps, warmup, body, units, torch):
    """Warm up, then time `steps` steps of reset + body + FP64 probability reduction. body(record) enqueues the
    work; with record=True it records a (start, end) event pair around every launch unit. units holds
    (class, algorithmic bytes, flops) per launch unit. Returns (per-step seconds,
    {class: [seconds, launches, alg_bytes, flops]})."""
    import paper_2203_16044_amd as qs
    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    events = [(mk(), mk()) for _ in units]
    e0, e1 = mk(), mk()
    for _ in range(warmup):
        st.init_zero()
        body(None)
        qs.binding.qs_probs(st.h, None, False)
    torch.cuda.synchronize()
    times, per = [], {}
    for _ in range(steps):
        e0.record(st.stream)
        st.init_zero()
        body(events)
        qs.binding.qs_probs(st.h, None, False)
        e1.record(st.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
        for (cls, nbytes, flops), (a, b) in zip(units, events):
            c = per.setdefault(cls, [0.0, 0, 0, 0])
            c[0] += a.elapsed_time(b) / 1e3
            c[1] += 1
            c[2] += nbytes
            c[3] += flops
    torch.cuda.synchronize()
    return times, per


def summarize(per, steps):
    return {c: {"launches": v[1] // steps, "avg_ms": v[0] / v[1] * 1e3, "tbs": v[2] / v[0] / 1e12}
            for c, v in sorted(per.items())}


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
    host = {}
    try:
        with open("/proc/cpuinfo") as f:
            host["cpu"] = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
        import psutil
        host["mem_gib"] = round(psutil.virtual_memory().total / 2 ** 30, 1)
        host["nproc"] = os.cpu_count()
    except Exception:
        pass
    return {"value": rate, "unit": "gates/s", "cores": oracle.oracle_threads(), "kind": "oracle", "sample": sample,
            "seconds": round(dt, 2), "host": host}


def bench_c64(head_rate, steps, torch):
    """complex64 engine: the 33-qubit circuit of the same family (64 GiB state, as large as the 32-qubit complex128
    one) planned once, with an FP64 renormalisation once each of layers 10/20/30/40 has completed (at the next pass
    boundary), and its error on the 24-qubit run against the complex128 path (which matches the FP64 oracle to
    1e-12 in the tests)."""
    import circuits as C
    import paper_2203_16044_amd as qs
    from paper_2203_16044_amd.metrics import state_error
    from paper_2203_16044_amd.plan import Circuit, LazyRenormPlan, Plan

    from paper_2203_16044_amd import costmodel as CM

    circ = C.su4_u3_renorm()
    st = qs.State(circ.n, "c64")
    # one plan over the whole circuit, renormalised at the first pass boundary after each renormalisation layer has
    # completed, in the block shape and beam width the cost model predicts fastest (greedy 12/4 without weights)
    model = CM.CostModel.load() if os.path.exists(CM.WEIGHTS) else None
    sp, key, pred = CM.choose_segmented(circ.n, circ.ops, circ.renorm_after, "c64", model, lazy=True)
    plan_s = f"block b={key[1]} low={key[2]} beam={key[3] if len(key) > 3 else qs.binding.qs_get_tunable('plan_beam')}"
    # the check: the circuit cut after its renormalisation layers, each segment planned alone
    seg, seg_key, _ = CM.choose_segmented(circ.n, circ.ops, circ.renorm_after, "c64", model, lazy=False)
    if model is not None:
        model.close()
    mk = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    st.init_zero()
    sp.run(st)
    torch.cuda.synchronize()
    times = []
    for _ in range(steps):
        e0, e1 = mk(), mk()
        e0.record(st.stream)
        st.init_zero()
        sp.run(st)
        qs.binding.qs_probs(st.h, None, False)
        e1.record(st.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    nrm = st.norm()
    info = sp.info()
    bounds = list(sp.bounds)
    sp.close()
    seg.run(st)  # warm
    e0, e1 = mk(), mk()
    e0.record(st.stream)
    st.init_zero()
    seg.run(st)
    qs.binding.qs_probs(st.h, None, False)
    e1.record(st.stream)
    e1.synchronize()
    t_seg = e0.elapsed_time(e1) / 1e3
    seg_passes = seg.info()["passes"]
    seg.close()
    st.close()
    del st
    torch.cuda.empty_cache()
    t = sum(times) / len(times)
    # error of the complex64 engine on the 24-qubit run, against the complex128 path
    e = C.su4_u3_error_run()
    a = qs.State(e.n, "c64")
    sp = LazyRenormPlan(e.n, e.ops, e.renorm_after, "block", 12, 4, "c64")
    sp.run(a)
    b = qs.State(e.n, "c128")
    c = Circuit.from_ops(e.n, e.ops)
    p = Plan(c, "block", 12, 4, "c128")
    p.run(b)
    infid, maxd = state_error(a.get(), b.get())
    for h in (sp, p, c, a, b):
        h.close()
    return {"workload": f"random SU(4)+U3 circuit, n={circ.n}, 40 layers, {len(circ.ops)} gates, complex64, "
                        f"renormalised once layers {list(circ.renorm_after)} complete (seed 33)",
            "gates_per_s": len(circ.ops) / t, "ms_per_step": t * 1e3, "passes": info["passes"],
            "plan": plan_s, "plan_choice": "learned" if model is not None else "greedy", "predicted_ms": pred,
            "renormalised_at_passes": bounds,
            "layer_exact_segments": {"gates_per_s": len(circ.ops) / t_seg, "ms": t_seg * 1e3, "passes": seg_passes,
                                     "plan": f"block b={seg_key[1]} low={seg_key[2]}"
                                             + (f" beam={seg_key[3]}" if len(seg_key) > 3 else "")},
            "renormalisations": info["renormalisations"], "norm_after": nrm,
            "gates_per_s_vs_c128_headline": len(circ.ops) / t / head_rate,
            "error_24q": {"infidelity": infid, "max_abs_amp_diff": maxd,
                          "against": "complex128 path (n=24, 40 layers, seed 24)"}}


def copy_ceiling(st, torch, reps=3):
    """The measured HBM ceiling of an in-place pass: the probe read-modify-write kernel (every 16-byte word of the
    state read and written back, no gate arithmetic) over the whole state buffer, best of `reps`, in TB/s of bytes
    read + written -- the access pattern of a plain gate pass over the same memory."""
    import paper_2203_16044_amd as qs
    nbytes = st.buf.numel() * st.buf.element_size()
    s = st.stream
    best = float("inf")
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        qs.binding.qs_probe_rmw(st.buf.data_ptr(), nbytes, s.cuda_stream)
        b.record(s)
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1e3)
    return 2 * nbytes / best / 1e12


def bench_mixed28(torch, copy_tbs, steps=1, warmup=1):
    """The 28-qubit mixed circuit (U3, CZ and RZ layers, Toffolis, fused-swaps; 1,425 operations), unfused: one pass
    per operation, per-class HBM rates against 8 TB/s and against the measured in-place ceiling, in algorithmic
    bytes (changed amplitudes) and in line-granular bytes (the 128-byte lines holding them); and the same circuit
    through the greedy block plan."""
    import circuits as C
    import paper_2203_16044_amd as qs
    from paper_2203_16044_amd.plan import Circuit, Plan
    circ = C.mixed_layers()
    n = circ.n
    st = qs.State(n, "c128")
    ops = circ.ops
    units = [(o.label.lower(), _alg_bytes(o, n, 16), _alg_flops(o, n)) for o in ops]
    times, per = time_steps(st, steps, warmup, lambda ev: run_plain(st, ops, ev) if ev else [st.apply_op(o) for o in ops],
                            units, torch)
    t = sum(times) / len(times)
    line_bytes = {}
    for o in ops:
        line_bytes[o.label.lower()] = line_bytes.get(o.label.lower(), 0) + _line_bytes(o, n, 16)
    classes = {}
    for c, (sec, cnt, nbytes, _) in sorted(per.items()):
        tbs = nbytes / sec / 1e12
        ltbs = line_bytes[c] * len(times) / sec / 1e12
        classes[c] = {"ops": cnt // len(times), "avg_ms": sec / cnt * 1e3, "tbs": tbs, "frac_of_peak": tbs / HBM_PEAK_TBS,
                      "frac_of_copy_ceiling": tbs / copy_tbs,
                      # against the bytes of the lines holding changed amplitudes (the line-granular roof)
                      "line_tbs": ltbs, "frac_of_line_roof": ltbs / HBM_PEAK_TBS,
                      "line_frac_of_copy_ceiling": ltbs / copy_tbs}
    total_bytes = sum(u[1] for u in units)
    cc = Circuit.from_ops(n, ops)
    p = Plan(cc, "block", 12, 4, "c128")
    npass = p.info()["passes"]
    bt, _ = time_steps(st, steps, warmup, lambda ev: p.run(st), [], torch)
    p.close()
    cc.close()
    st.close()
    torch.cuda.empty_cache()
    return {"workload": f"mixed circuit, n={n}, 20 layers (U3, CZ on alternating pairs, RZ), 32 Toffolis, 3 fused-swaps "
                        f"(0, 22, 6); {len(ops)} operations, complex128, seed 28",
            "plain_ops_per_s": len(ops) / t, "plain_ms_per_step": t * 1e3, "plain_tbs_whole": total_bytes / t / 1e12,
            "per_class": classes,
            "paper_effective_tbs": (1 << (n + 5)) * len(ops) / t / 1e12,
            "block_plan": {"passes": npass, "ops_per_s": len(ops) / (sum(bt) / len(bt)),
                           "ms_per_step": sum(bt) / len(bt) * 1e3}}


def bench_batch(torch, log):
    """Batched serving form: 512 independent circuits (10..22 qubits, 10..40 layers) in one launch per pass level,
    eager and replayed from a HIP graph, against the per-circuit plain loop. The block shape of the batch's plans is
    the cost model's choice (batch.learned_shape) and its launch is autotuned; the empirical search over every
    shape and launch is timed beside it as the check."""
    import circuits as C
    from paper_2203_16044_amd import batch as BT
    from paper_2203_16044_amd import costmodel as CM

    circs = C.serving_batch()
    rec = BT.record(circs)
    model = CM.CostModel.load() if os.path.exists(CM.WEIGHTS) else None
    out = {"workload": "512 circuits, n ~ U{10..22}, depth ~ U{10..40} (U3 / CNOT-or-CZ / RZ layers, seed 512), "
                       "FP64 probabilities of every circuit", "circuits": len(circs),
           "gates": sum(len(c.ops) for c in circs)}
    for dt in ("c128", "c64"):
        t0 = time.perf_counter()
        emp, times = BT.autotune(rec, dt, log=log)
        tune_s = time.perf_counter() - t0
        best, learned = emp, None
        if model is not None:
            t0 = time.perf_counter()
            shape, pred = BT.learned_shape(rec, dt, model)
            # the launch for that shape: the fastest workgroup count among the timed candidates of that shape
            cands = {k: v for k, v in times.items()
                     if (json.loads(k)["block_bits"], json.loads(k)["low_bits"]) == shape}
            best = json.loads(min(cands, key=cands.get))
            learned = {"shape": list(shape), "predicted_ms_top64": {f"{b}/{w}": round(v, 2) for (b, w), v in pred.items()},
                       "choose_s": round(time.perf_counter() - t0, 1), "empirical_best": emp,
                       "learned_vs_empirical_ms": [round(cands[json.dumps(best, sort_keys=True)] * 1e3, 3),
                                                   round(min(times.values()) * 1e3, 3)]}
        b = BT.Batch(rec, dt, **best)
        t_eager = BT.time_batch(b, graph=False, reps=3)
        t_graph = BT.time_batch(b, graph=True, reps=3)
        b.close()
        out[dt] = {"params": best, "learned_plans": learned, "circuits_per_s_graph": len(circs) / t_graph,
                   "circuits_per_s_eager": len(circs) / t_eager, "ms_graph": t_graph * 1e3,
                   "ms_eager": t_eager * 1e3, "autotune_s": round(tune_s, 1),
                   "autotune_ms": {k: round(v * 1e3, 3) for k, v in times.items()}}
        t_plain, _ = BT.plain_loop(circs, dt)
        out[dt]["plain_loop_circuits_per_s"] = len(circs) / t_plain
        out[dt]["speedup_vs_plain_loop"] = t_plain / t_graph
    for c in rec:
        c.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--layers", type=int, default=40)
    ap.add_argument("--mode", choices=["plain", "tuned"], default="tuned")
    ap.add_argument("--block-bits", type=int, default=12)
    ap.add_argument("--low-bits", type=int, default=4)
    ap.add_argument("--plain-layers", type=int, default=4, help="layers of the circuit timed on the plain path")
    ap.add_argument("--greedy", action="store_true", help="headline the greedy plan instead of the learned one")
    ap.add_argument("--no-compare-greedy", action="store_true",
                    help="do not also time the greedy plan (profiling runs: only the headline plan's kernels)")
    ap.add_argument("--compare-fuse", type=int, nargs="*", default=[4, 6], help="fused-dense plans also timed")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c64", action="store_true", help="skip the 33-qubit complex64 leg")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-circuit batched leg")
    ap.add_argument("--no-mixed28", action="store_true", help="skip the 28-qubit mixed-circuit (plain kernels) leg")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the gate path is single-GPU (multi-GPU sharding is a design note only). "
              "Run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import circuits as C
    import paper_2203_16044_amd as qs

    torch.cuda.set_device(0)
    from paper_2203_16044_amd.plan import Circuit, Plan

    circ = C.su4_u3_random(n=args.n, seed=32, layers=args.layers)
    ops = circ.ops
    n = circ.n
    gates = len(ops)
    full = 2 * 16 * (1 << n)
    st = qs.State(n, "c128")
    t_wall = time.perf_counter()

    log0 = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    log0("bench: plain leg")
    # plain: one pass per gate (on a prefix of the circuit in tuned mode: the per-gate rate is layer-invariant)
    plain_ops = ops if args.mode == "plain" else [o for o in ops if o.layer <= args.plain_layers]
    units = [(_kernel_class(o), _alg_bytes(o, n, 16), _alg_flops(o, n)) for o in plain_ops]
    # tuned mode: one warmup and two timed passes over the prefix (their spread is reported)
    p_times, p_per = time_steps(st, args.steps if args.mode == "plain" else 2,
                                args.warmup if args.mode == "plain" else 1,
                                lambda ev: run_plain(st, plain_ops, ev) if ev else [st.apply_op(o) for o in plain_ops],
                                units, torch)
    plain_rate = len(plain_ops) / (sum(p_times) / len(p_times))

    results = {}
    if args.mode == "tuned":
        from paper_2203_16044_amd import costmodel as CM
        cc = Circuit.from_ops(n, ops)
        greedy = ("block", args.block_bits, args.low_bits)
        learned, head_plan = None, None
        if not args.greedy and os.path.exists(CM.WEIGHTS):
            model = CM.CostModel.load()
            head_plan, learned, pred = CM.choose_plan(cc, "c128", model)
            model.close()
        head_v = learned or greedy
        key = lambda v: "learned_per_pass" if v == CM.LEARNED else (  # noqa: E731
            f"{v[0]}{v[1]}" + (f"_low{v[2]}" if v[0] == "block" else "") + (f"_beam{v[3]}" if len(v) > 3 else ""))
        greedy_v = [] if args.no_compare_greedy else [greedy]
        variants = [head_v] + [v for v in greedy_v + [("fuse", k, 0) for k in args.compare_fuse] if v != head_v]
        for vi, v in enumerate(variants):
            log0(f"bench: plan {key(v)}")
            if vi == 0 and head_plan is not None:
                plan = head_plan
            else:
                plan = CM.make_plan(cc, v, "c128")
            info = plan.info()
            passes = plan.passes()
            kinds = {0: "block_b{}", 1: "dense_k{}", 2: "fswap", 3: "other"}
            # flops of a pass from the planner's features (flops per amplitude, / 256) x amplitudes
            fl = [float(qs.binding.qs_plan_features(plan.h, i)[14]) * 256 * (1 << n) for i in range(len(passes))]
            units = [(kinds[ps["type"]].format(ps["nqubits"]),
                      int(full * (1 - 2.0 ** -(ps["nqubits"] // 2))) if ps["type"] == 2 else full, int(fl[i]))
                     for i, ps in enumerate(passes)]
            main = vi == 0
            times, per = time_steps(st, args.steps if main else 1, args.warmup if main else 1,
                                    lambda ev, plan=plan, npass=len(passes): run_plan(st, plan, npass, ev) if ev
                                    else plan.run(st), units, torch)
            results[key(v)] = {
                "passes": info["passes"], "gates_per_s": gates / (sum(times) / len(times)),
                "ms_per_step": sum(times) / len(times) * 1e3, "per_kernel": summarize(per, len(times)),
                "_times": times, "_per": per}
            plan.close()
        cc.close()
        head = results[key(head_v)]
        step_times, per_class = head["_times"], head["_per"]
        greedy_key = key(greedy)
    else:
        step_times, per_class = p_times, p_per
    nrm = st.norm()
    log0("bench: in-place HBM ceiling")
    copy_tbs = copy_ceiling(st, torch)
    st.close()
    wall = time.perf_counter() - t_wall

    t_step = sum(step_times) / len(step_times)
    dom = max(per_class, key=lambda c: per_class[c][0])
    tsum, cnt, bsum, fsum = per_class[dom]
    avg = tsum / cnt
    achieved = (bsum / cnt) / avg / 1e12
    tflops = (fsum / cnt) / avg / 1e12
    # the binding roof of the dominant kernel: the larger of its HBM time and its FP64 time at peak
    t_hbm = (bsum / cnt) / (HBM_PEAK_TBS * 1e12)
    t_alu = (fsum / cnt) / (FP64_PEAK_TFLOPS * 1e12)
    if t_alu > t_hbm:
        roof = {"bound": "alu", "achieved": tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / FP64_PEAK_TFLOPS}
    else:
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_TBS, "unit": "TB/s",
                "frac": achieved / HBM_PEAK_TBS}
    out = {
        "metric": "gates/s, 32-qubit complex128 random circuit (SU(4) pairings + U3, 40 layers); tuned vs plain",
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
                               f"(seed 32)", "n": n, "gates": gates, "mode": args.mode,
                   "plan": ("one pass per gate" if args.mode != "tuned" else
                            "learned: every pass chosen by the cost model" if learned == ("learned", 0, 0) else
                            ("learned: " if learned else "greedy: ") + f"{head_v[0]} b={head_v[1]} low={head_v[2]}"
                            + (f" beam={head_v[3]}" if len(head_v) > 3 else "")),
                   "parallelism": "none"},
        "roofline": dict(roof, traffic=pmc_traffic(dom), kernel=dom, avg_launch_ms=avg * 1e3,
                         launches_per_step=cnt // len(step_times), alg_bytes_per_launch=bsum // cnt,
                         flops_per_launch=fsum // cnt, hbm_tbs=achieved, hbm_frac=achieved / HBM_PEAK_TBS,
                         fp64_tflops=tflops, fp64_frac=tflops / FP64_PEAK_TFLOPS,
                         frac_of_roofline=max(t_hbm, t_alu) / avg),
        "plain": {"gates_per_s": plain_rate, "gates_timed": len(plain_ops), "timed_passes": len(p_times),
                  "spread": (max(p_times) - min(p_times)) / min(p_times),
                  "per_kernel": summarize(p_per, len(p_times))},
        "speedup_vs_plain": (gates / t_step) / plain_rate,
        "speedup_vs_greedy_plan": ((gates / t_step) / results[greedy_key]["gates_per_s"]
                                   if args.mode == "tuned" and greedy_key in results else None),
        "hbm_tbs_whole_step": (sum(v[2] for v in per_class.values()) / len(step_times)) / t_step / 1e12,
        "paper_nominal_tbs": (1 << (n + 5)) * gates / t_step / 1e12,
        # quantum B/F ratio (Sec. IV-B): 2^(n+5) x #gates / (execution time x peak FP64 FLOP/s)
        "qbf": (1 << (n + 5)) * gates / t_step / (FP64_PEAK_TFLOPS * 1e12),
        "alternatives": {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")} for k, v in results.items()},
        "norm_after": nrm,
        "wall_s": wall,
    }
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    out["copy_ceiling_tbs"] = copy_tbs
    out["roofline"]["hbm_frac_of_copy_ceiling"] = out["roofline"]["hbm_tbs"] / copy_tbs
    for c, v in out["plain"]["per_kernel"].items():
        v["frac_of_copy_ceiling"] = v["tbs"] / copy_tbs
    if not args.no_mixed28:
        log("bench: 28-qubit mixed circuit")
        out["mixed28"] = bench_mixed28(torch, copy_tbs)
    if not args.no_c64:
        log("bench: complex64 leg")
        out["c64"] = bench_c64(gates / t_step, 1, torch)
    if not args.no_batch:
        log("bench: batched leg")
        out["batch"] = bench_batch(torch, log)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline")
        out["cpu_baseline"] = cpu_baseline(circ, args.cpu_seconds, torch)
    out["wall_s"] = time.perf_counter() - t_wall
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
