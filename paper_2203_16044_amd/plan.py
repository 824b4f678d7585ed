"""Circuits and execution plans over libqs (marshalling only; planning happens in the library's C++ planner).

``Circuit.from_ops(n, ops)`` records a circuit in the library; ``Plan(circuit, mode, block_bits, low_bits, dtype)``
groups its operations into HBM passes (LDS block passes or fused dense blocks) and ``Plan.run(state)`` enqueues
them on the state's stream.
"""
from __future__ import annotations

from . import binding as B

MODES = {"block": B.QS_PLAN_BLOCK, "fuse": B.QS_PLAN_FUSE, "remap": B.QS_PLAN_REMAP}


class Circuit:
    def __init__(self, n: int):
        self.n = int(n)
        self.h = B.qs_circuit_create(self.n)

    @classmethod
    def from_ops(cls, n: int, ops) -> "Circuit":
        c = cls(n)
        for op in ops:
            c.add(op)
        return c

    def add(self, op) -> None:
        if op.kind == "dense":
            B.qs_circuit_add_gate(self.h, op.targets, op.mat)
        elif op.kind == "diag":
            B.qs_circuit_add_diag(self.h, op.targets, op.mat)
        elif op.kind == "ctrl":
            B.qs_circuit_add_controlled(self.h, op.controls, op.targets, op.mat)
        elif op.kind == "fswap":
            B.qs_circuit_add_fused_swap(self.h, op.p, op.q, op.s)
        else:
            raise ValueError(f"unknown op kind {op.kind!r}")

    def __len__(self) -> int:
        return B.qs_circuit_size(self.h)

    def run_plain(self, state) -> None:
        B.qs_circuit_run(state.h, self.h)

    def close(self) -> None:
        if getattr(self, "h", None):
            B.qs_circuit_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    def __init__(self, circuit: Circuit, mode: str = "block", block_bits: int = 12, low_bits: int = 4,
                 dtype: str = "c128"):
        self.n = circuit.n
        self.mode, self.block_bits, self.low_bits, self.dtype = mode, block_bits, low_bits, dtype
        self.h = B.qs_plan_create(circuit.h, MODES[mode], block_bits, low_bits,
                                  B.QS_C128 if dtype == "c128" else B.QS_C64)

    @classmethod
    def learned(cls, circuit: Circuit, model, shapes, per_shape: int = 4, dtype: str = "c128",
                gate_slack: int = 1 << 20, lookahead: int = 0) -> "Plan":
        """A plan whose every pass is chosen by the cost model `model` (a costmodel.CostModel) among candidate passes
        of the given (block_bits, low_bits) shapes (qs_plan_create_learned)."""
        self = cls.__new__(cls)
        self.n = circuit.n
        self.mode, self.block_bits, self.low_bits, self.dtype = "learned", 0, 0, dtype
        self.h = B.qs_plan_create_learned(circuit.h, B.QS_C128 if dtype == "c128" else B.QS_C64, model.h, model.mean,
                                          model.std, shapes, per_shape, gate_slack, lookahead)
        return self

    def info(self) -> dict:
        return B.qs_plan_info(self.h)

    def passes(self):
        return [B.qs_plan_pass_info(self.h, i) for i in range(self.info()["passes"])]

    def pass_gates(self):
        """Per pass, the indices of the circuit operations it carries, in the order it applies them."""
        return [B.qs_plan_pass_gates(self.h, i) for i in range(self.info()["passes"])]

    def run(self, state, begin: int = 0, end: int = None) -> None:
        if begin == 0 and end is None:
            B.qs_plan_run(state.h, self.h)
        else:
            B.qs_plan_run_range(state.h, self.h, begin, self.info()["passes"] if end is None else end)

    def close(self) -> None:
        if getattr(self, "h", None):
            B.qs_plan_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SegmentedPlan:
    """A circuit planned in segments that end at given layers, with the state renormalised (FP64 norm, FP64
    factor) after each of those layers -- the complex64 cadence. Segments are planned independently."""

    def __init__(self, n: int, ops, renorm_after, mode: str = "block", block_bits: int = 12, low_bits: int = 4,
                 dtype: str = "c64"):
        marks = sorted(set(renorm_after))
        self.n = n
        self.parts = []
        ops = list(ops)
        # split after the last op of each renormalisation layer (ops are in layer order)
        segs, start = [], 0
        for L in marks:
            idx = [i for i, o in enumerate(ops) if o.layer <= L]
            end = (max(idx) + 1) if idx else start
            if end > start:
                segs.append((ops[start:end], True))
                start = end
        if start < len(ops):
            segs.append((ops[start:], False))
        for seg, renorm in segs:
            c = Circuit.from_ops(n, seg)
            self.parts.append((c, Plan(c, mode, block_bits, low_bits, dtype), renorm))

    def info(self) -> dict:
        tot = {}
        for _, p, _ in self.parts:
            for k, v in p.info().items():
                tot[k] = tot.get(k, 0) + v
        tot["renormalisations"] = sum(1 for _, _, r in self.parts if r)
        return tot

    def run(self, state, folded: bool = True) -> None:
        """Run the segments in order, renormalising after each segment that ends at a renormalisation layer. With
        `folded` (default) each such renormalisation is folded into the passes around it (qs_plan_run_renorm: the
        norm taken as the segment's last pass stores the state, the scaling applied as the next segment's first pass
        loads it; a final one scales in a sweep of its own); otherwise qs_renormalize runs between segments."""
        if not folded:
            for _, p, renorm in self.parts:
                p.run(state)
                if renorm:
                    B.qs_renormalize(state.h, False)
            return
        pending = False
        for _, p, renorm in self.parts:
            flags = (B.QS_RUN_SCALE_FIRST if pending else 0) | (B.QS_RUN_NORM_LAST if renorm else 0)
            if flags:
                B.qs_plan_run_renorm(state.h, p.h, flags)
            else:
                p.run(state)
            pending = renorm
        if pending:
            B.qs_renormalize_pending(state.h, False)

    def plans(self) -> list:
        return [p for _, p, _ in self.parts]

    def close(self) -> None:
        for c, p, _ in self.parts:
            p.close()
            c.close()
        self.parts = []


def renorm_boundaries(plan, layers, marks) -> list:
    """For each renormalisation layer L (ascending), the smallest pass index i such that every operation of a layer
    <= L runs in passes 0..i: the renormalisation then follows pass i. Marks that no operation precedes are dropped
    and marks that land on the same pass merge. `layers` holds each operation's layer, in the circuit's order."""
    npass = plan.info()["passes"]
    where = [-1] * len(layers)
    for i in range(npass):
        for g in B.qs_plan_pass_gates(plan.h, i):
            where[g] = i
    if min(where, default=0) < 0:
        raise RuntimeError("plan does not place every operation of the circuit")
    out = []
    for L in sorted(set(marks)):
        idx = [where[g] for g in range(len(layers)) if layers[g] <= L]
        if idx and (not out or max(idx) > out[-1]):
            out.append(max(idx))
    return out


class LazyRenormPlan:
    """A circuit planned once, with the state renormalised (FP64 norm, FP64 factor) at pass boundaries: after each
    renormalisation layer L, at the first boundary by which every operation of the layers <= L has run (some of
    the next layers' operations may already have run there). A renormalisation multiplies the state by a scalar and
    so commutes with every gate; it differs from renormalising exactly after layer L only through the rounding
    drift of the norm it divides by. Each renormalisation is folded into the block passes on either side of its
    boundary (qs_plan_run_range_renorm), the last one scaled in a sweep of its own if it ends the plan."""

    def __init__(self, n: int, ops, renorm_after, mode: str = "block", block_bits: int = 12, low_bits: int = 4,
                 dtype: str = "c64"):
        ops = list(ops)
        self.n = n
        self.circuit = Circuit.from_ops(n, ops)
        self.plan = Plan(self.circuit, mode, block_bits, low_bits, dtype)
        self.bounds = renorm_boundaries(self.plan, [o.layer for o in ops], renorm_after)

    def info(self) -> dict:
        d = dict(self.plan.info())
        d["renormalisations"] = len(self.bounds)
        return d

    def plans(self) -> list:
        return [self.plan]

    def run(self, state) -> None:
        npass = self.plan.info()["passes"]
        start, pending = 0, False
        for b in self.bounds:
            flags = (B.QS_RUN_SCALE_FIRST if pending else 0) | B.QS_RUN_NORM_LAST
            B.qs_plan_run_range_renorm(state.h, self.plan.h, start, b + 1, flags)
            start, pending = b + 1, True
        if start < npass:
            B.qs_plan_run_range_renorm(state.h, self.plan.h, start, npass, B.QS_RUN_SCALE_FIRST if pending else 0)
        elif pending:
            B.qs_renormalize_pending(state.h, False)

    def close(self) -> None:
        if getattr(self, "plan", None) is not None:
            self.plan.close()
            self.circuit.close()
            self.plan = None
