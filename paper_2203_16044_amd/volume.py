"""Exchange volume of a circuit on a state distributed over 2^g devices (Sec. III-B, III-D).

With n qubits and the top g of them global (held across devices), the paper counts, in bytes of complex128
amplitudes:
  * a gate that acts on a global qubit: the whole state crosses the network once, 2^(n+4);
  * a swap of a local and a global qubit: half of the amplitudes move, 2^(n+4) / 2;
  * a fused-swap of s local with s global qubits: all amplitudes except the 2^(n-s) fixed points move,
    2^(n+4) (1 - 2^-s);
  * anything acting on local qubits only: nothing.
This model is what a multi-device planner minimises when it chooses where to insert fused-swaps; on one device it
prices the same permutations in HBM bytes instead (see paperbench's swap ablation).
"""
from __future__ import annotations

from typing import Iterable


def exchange_bytes(n: int, n_global: int, ops: Iterable) -> int:
    """Bytes exchanged between devices by `ops` (circuits.Op) when qubits n - n_global .. n - 1 are global.
    A swap is a fused-swap with s = 1."""
    if not 0 <= n_global <= n:
        raise ValueError("n_global must lie in [0, n]")
    first_global = n - n_global
    full = 1 << (n + 4)
    total = 0
    for op in ops:
        qs = op.qubits()
        if not any(q >= first_global for q in qs):
            continue
        if op.kind == "fswap":
            # fixed points are the amplitudes whose swapped bit pairs agree: 2^(n-s) of them
            total += full - (full >> op.s)
        else:
            total += full
    return total
