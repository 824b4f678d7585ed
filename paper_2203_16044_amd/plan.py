"""Circuits and execution plans over libqs (marshalling only; planning happens in the library's C++ planner).

``Circuit.from_ops(n, ops)`` records a circuit in the library; ``Plan(circuit, mode, block_bits, low_bits, dtype)``
groups its operations into HBM passes (LDS block passes or fused dense blocks) and ``Plan.run(state)`` enqueues
them on the state's stream.
"""
from __future__ import annotations

from . import binding as B

MODES = {"block": B.QS_PLAN_BLOCK, "fuse": B.QS_PLAN_FUSE}


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

    def info(self) -> dict:
        return B.qs_plan_info(self.h)

    def passes(self):
        return [B.qs_plan_pass_info(self.h, i) for i in range(self.info()["passes"])]

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
