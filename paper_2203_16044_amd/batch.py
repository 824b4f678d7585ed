"""Batched serving form over libqs: hundreds of independent circuits in one persistent launch (qs_batch_*),
optionally replayed from a captured HIP graph, with launch parameters chosen by an autotuner.

The autotuner times every candidate (block bits, always-local low bits, persistent workgroups per CU) on the batch
itself and keeps the fastest; results are cached in a JSON file keyed by the batch's shape (dtype and the sorted
qubit counts and gate counts of its circuits).
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Dict, Iterable, List, Optional, Tuple

import numpy as np

from . import binding as B
from .plan import Circuit

CACHE = os.environ.get("QS_AUTOTUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), ".autotune_cache.json"))
DEFAULT = {"block_bits": 12, "low_bits": 4, "wg_per_cu": 2}
SPACE = [{"block_bits": b, "low_bits": w, "wg_per_cu": g} for b in (10, 11, 12) for w in (3, 4) for g in (2, 8, 32)]


def record(circuits) -> List[Circuit]:
    """Record gate-list circuits in the library once, so several batches (autotuner candidates) can share them."""
    return [c if isinstance(c, Circuit) else Circuit.from_ops(c.n, c.ops) for c in circuits]


class Batch:
    """`circuits` holds gate-list circuits or already recorded library circuits (the batch copies what it needs)."""

    def __init__(self, circuits, dtype: str = "c128", block_bits: int = 12, low_bits: int = 4, wg_per_cu: int = 2,
                 stream=None):
        import torch
        self.dtype = dtype
        self.qs_dtype = B.QS_C128 if dtype == "c128" else B.QS_C64
        self.ns = [c.n for c in circuits]
        # a stream of its own (default priority): graphs cannot be captured on the legacy null stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.params = {"block_bits": block_bits, "low_bits": low_bits, "wg_per_cu": wg_per_cu}
        self.h = B.qs_batch_create(self.qs_dtype, block_bits, low_bits, wg_per_cu, self.stream.cuda_stream)
        for circ in circuits:
            if isinstance(circ, Circuit):
                B.qs_batch_add(self.h, circ.h)
            else:
                c = Circuit.from_ops(circ.n, circ.ops)
                B.qs_batch_add(self.h, c.h)
                c.close()
        B.qs_batch_finalize(self.h)

    def set_launch(self, wg_per_cu: int) -> None:
        B.qs_batch_set_launch(self.h, wg_per_cu)
        self.params["wg_per_cu"] = int(wg_per_cu)

    def run(self, graph: bool = False) -> None:
        B.qs_batch_run(self.h, graph)

    def info(self) -> dict:
        return B.qs_batch_info(self.h)

    def probs(self, i: int) -> np.ndarray:
        return B.qs_batch_probs(self.h, i, self.ns[i])[1]

    def sync(self) -> None:
        self.stream.synchronize()

    def close(self) -> None:
        if getattr(self, "h", None):
            B.qs_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def time_batch(batch: Batch, graph: bool = False, reps: int = 3) -> float:
    import torch
    s = batch.stream
    batch.run(graph)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record(s)
        batch.run(graph)
        e1.record(s)
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return best


def signature(circuits, dtype: str) -> str:
    sizes = sorted((c.n, len(c.ops) if hasattr(c, "ops") else len(c)) for c in circuits)
    key = dtype + ":" + ",".join(f"{n}/{g}" for n, g in sizes)
    return hashlib.sha1(key.encode()).hexdigest()


SHAPES = sorted({(c["block_bits"], c["low_bits"]) for c in SPACE})


def learned_shape(circuits, dtype: str, model, shapes=None, top: int = 64) -> Tuple[Tuple[int, int], Dict]:
    """The (block bits, low bits) whose plans the cost model predicts fastest for this batch: the sum of the
    predicted plan times of its `top` largest circuits above 12 qubits (the HBM circuits, which hold almost all of a
    batch's work; smaller ones run whole in one workgroup's LDS under every candidate shape). Returns (shape,
    {shape: predicted ms})."""
    from .plan import Plan
    recorded = record(circuits)
    try:
        big = sorted((c for c in recorded if c.n > 12), key=lambda c: (c.n, len(c)), reverse=True)[:top]
        pred = {}
        for bb, lb in (shapes or SHAPES):
            tot = 0.0
            for c in big:
                p = Plan(c, "block", bb, lb, dtype)
                tot += model.predict_plan_ms(p)
                p.close()
            pred[(bb, lb)] = tot
    finally:
        for c, orig in zip(recorded, circuits):
            if c is not orig:  # recorded here: release it
                c.close()
    return min(pred, key=pred.get), pred


def autotune(circuits, dtype: str = "c128", cache: Optional[str] = CACHE, space: Optional[List[Dict]] = None,
             log=None, model=None) -> Tuple[Dict, Dict[str, float]]:
    """Time every candidate on the batch and return (best parameters, {candidate: seconds}). Cached by shape. With a
    cost model, the block shape is the model's choice (learned_shape) and only the launch (workgroups per CU) is
    timed."""
    if model is not None:
        shape, _ = learned_shape(circuits, dtype, model)
        space = [c for c in (space or SPACE) if (c["block_bits"], c["low_bits"]) == shape]
        cache = None
    sig = signature(circuits, dtype)
    data = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                data = json.load(f)
        except (OSError, ValueError):
            data = {}
    if sig in data:
        return data[sig]["best"], data[sig]["times"]
    times = {}
    recorded = record(circuits)
    # one planned batch per (block bits, low bits); the workgroup count only changes the launch
    groups: Dict[Tuple[int, int], List[int]] = {}
    for cand in (space or SPACE):
        groups.setdefault((cand["block_bits"], cand["low_bits"]), []).append(cand["wg_per_cu"])
    for (bb, lb), wgs in groups.items():
        b = Batch(recorded, dtype, bb, lb, wgs[0])
        for wg in wgs:
            b.set_launch(wg)
            t = time_batch(b, reps=2)
            cand = {"block_bits": bb, "low_bits": lb, "wg_per_cu": wg}
            times[json.dumps(cand, sort_keys=True)] = t
            if log:
                log(f"autotune {cand}: {t * 1e3:.2f} ms")
        b.close()
    best = json.loads(min(times, key=times.get))
    if cache:
        data[sig] = {"best": best, "times": times}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best, times


def plain_loop(circuits, dtype: str = "c128", keep: Iterable[int] = ()) -> Tuple[float, Dict[int, np.ndarray]]:
    """The per-circuit plain loop: for each circuit allocate a state, apply its gates one pass each (qs_circuit_run)
    and compute its FP64 probabilities. Returns (seconds on the stream, probabilities of the circuits in `keep`)."""
    import torch

    from .state import State
    keep = set(keep)
    s = torch.cuda.current_stream()
    handles = [Circuit.from_ops(c.n, c.ops) for c in circuits]  # recorded before the timed region
    states = {}
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    t0 = time.perf_counter()
    for i, (circ, c) in enumerate(zip(circuits, handles)):
        st = states.get(circ.n)
        if st is None:
            st = states[circ.n] = State(circ.n, dtype)
        st.init_zero()
        c.run_plain(st)
        P, _ = st.probs(want_norm=False)
        if i in keep:
            out[i] = P.cpu().numpy()
    e1.record(s)
    e1.synchronize()
    wall = time.perf_counter() - t0
    for st in states.values():
        st.close()
    for c in handles:
        c.close()
    return max(e0.elapsed_time(e1) / 1e3, wall), out
