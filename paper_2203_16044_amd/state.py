"""A torch-backed convenience wrapper over one libqs state handle.

torch allocates the amplitude buffer (complex128 / complex64 on the current device) and supplies the
stream; libqs does every step of the gate path. Nothing here computes on the state.
"""
from __future__ import annotations

from typing import Iterable

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


class State:
    def __init__(self, n: int, dtype: str = "c128", stream=None, buf=None):
        torch = _torch()
        if dtype not in ("c128", "c64"):
            raise ValueError("dtype must be 'c128' or 'c64'")
        self.n = int(n)
        self.dtype = dtype
        self.qs_dtype = B.QS_C128 if dtype == "c128" else B.QS_C64
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        if buf is None:
            buf = torch.empty(1 << self.n, dtype=tdt, device="cuda")
        elif buf.dtype != tdt or buf.numel() < (1 << self.n) or not buf.is_cuda or not buf.is_contiguous():
            raise ValueError("buf must be a contiguous CUDA tensor of 2^n amplitudes of the state's dtype")
        self.buf = buf
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = B.qs_alloc(self.n, self.qs_dtype, self.buf.data_ptr(), self.stream.cuda_stream)

    # -------------------------------------------------------------------------------------------- lifetime
    def close(self) -> None:
        if getattr(self, "h", None):
            B.qs_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------------------------------------- ops
    def apply_gate(self, targets, U):
        B.qs_apply_gate(self.h, targets, U)

    def apply_diag(self, targets, d):
        B.qs_apply_diag(self.h, targets, d)

    def apply_controlled(self, controls, targets, U):
        B.qs_apply_controlled(self.h, controls, targets, U)

    def fused_swap(self, p, q, s):
        B.qs_fused_swap(self.h, p, q, s)

    def apply_op(self, op) -> None:
        k = op.kind
        if k == "dense":
            B.qs_apply_gate(self.h, op.targets, op.mat)
        elif k == "diag":
            B.qs_apply_diag(self.h, op.targets, op.mat)
        elif k == "ctrl":
            B.qs_apply_controlled(self.h, op.controls, op.targets, op.mat)
        elif k == "fswap":
            B.qs_fused_swap(self.h, op.p, op.q, op.s)
        else:
            raise ValueError(f"unknown op kind {k!r}")

    def run(self, ops: Iterable, renorm_after=()) -> None:
        """Apply ops one at a time, unfused; renormalise after the listed 1-based layers (complex64)."""
        renorm = set(renorm_after)
        ops = list(ops)
        for i, op in enumerate(ops):
            self.apply_op(op)
            if renorm and op.layer in renorm and (i + 1 == len(ops) or ops[i + 1].layer != op.layer):
                B.qs_renormalize(self.h)

    # -------------------------------------------------------------------------------------------- I/O
    def measure(self, qubit: int, u: float):
        """Measure `qubit` with the uniform u in [0, 1): returns (outcome, P(1)); the state collapses."""
        return B.qs_measure(self.h, qubit, u)

    def reset(self, qubit: int, u: float) -> int:
        return B.qs_reset(self.h, qubit, u)

    def sample(self, u) -> np.ndarray:
        """One basis index per uniform in `u` (the state is unchanged)."""
        return B.qs_sample(self.h, u)

    def init_zero(self):
        B.qs_init_zero(self.h)

    def set(self, host: np.ndarray) -> None:
        want = np.complex128 if self.dtype == "c128" else np.complex64
        a = np.ascontiguousarray(np.asarray(host).astype(want, copy=False))
        if a.size != (1 << self.n):
            raise ValueError("host state has the wrong size")
        B.qs_copy_in(self.h, a)

    def get(self) -> np.ndarray:
        out = np.empty(1 << self.n, dtype=np.complex128 if self.dtype == "c128" else np.complex64)
        B.qs_copy_out(self.h, out)
        return out

    def probs(self, want_norm: bool = True):
        """Returns (probabilities as a CUDA float64 tensor, FP64 norm or None)."""
        torch = _torch()
        out = torch.empty(1 << self.n, dtype=torch.float64, device=self.buf.device)
        nrm = B.qs_probs(self.h, out.data_ptr(), want_norm)
        return out, nrm

    def norm(self) -> float:
        return B.qs_norm(self.h)

    def renormalize(self) -> float:
        return B.qs_renormalize(self.h, True)

    def sync(self):
        B.qs_sync(self.h)
