"""CPU oracle for state-vector gate application (mpiQulacs, Sec. II-A Eqs. 2-4, Sec. III-D Listing 1).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg, never by the product path. It shares no code with the GPU library; the only common
module is ``circuits`` (seeded input generators, no state arithmetic).

Two independent formulations live here:
  * ``qs_oracle.c`` (loaded via ctypes): plain FP64 loops, one op at a time, in list order (Sec. II-A: a
    circuit is an ordered sequence of gates). This is the oracle proper.
  * ``brute``: numpy tensor contractions / Kronecker products / axis transpositions for n <= ~12, used only to
    pin the loop oracle.
Pinned by ``tests/test_oracle_pins.py`` (closed forms, brute force, invariants, truth tables).
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, Optional

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QS_LIBQS_ORACLE")  # a sanitizer build (oracle/build.py --sanitize)
        if not path:
            path = _build.LIB
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
                _build.build()
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_init_zero.argtypes = [dp, ctypes.c_int]
        L.or_init_zero.restype = None
        L.or_apply_dense.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp]
        L.or_apply_controlled.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp]
        L.or_apply_diag.argtypes = [dp, ctypes.c_int, ip, ctypes.c_int, dp]
        L.or_swap.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_fused_swap.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.or_probs.argtypes = [dp, ctypes.c_int, dp, dp]
        L.or_scale.argtypes = [dp, ctypes.c_int, ctypes.c_double]
        for f in ("or_apply_dense", "or_apply_controlled", "or_apply_diag", "or_swap", "or_fused_swap",
                  "or_probs", "or_scale"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iarr(v) -> ctypes.Array:
    v = [int(x) for x in v]
    return (ctypes.c_int * max(1, len(v)))(*v)


def _check_state(psi: np.ndarray):
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous:
        raise TypeError("oracle state must be a C-contiguous complex128 array")
    n = int(psi.size).bit_length() - 1
    if (1 << n) != psi.size:
        raise ValueError("state size must be a power of two")
    return n


def _mat(m: np.ndarray, k: int, diag: bool = False) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    want = (1 << k,) if diag else (1 << k, 1 << k)
    if a.shape != want:
        raise ValueError(f"matrix shape {a.shape} does not match {k} target(s): expected {want}")
    return a


def zero_state(n: int) -> np.ndarray:
    psi = np.empty(1 << n, dtype=np.complex128)
    lib().or_init_zero(_dptr(psi.view(np.float64)), n)
    return psi


def apply_dense(psi: np.ndarray, targets, U) -> None:
    n = _check_state(psi)
    U = _mat(U, len(targets))
    rc = lib().or_apply_dense(_dptr(psi.view(np.float64)), n, _iarr(targets), len(targets), _dptr(U.view(np.float64)))
    if rc:
        raise ValueError(f"or_apply_dense rejected targets={targets}")


def apply_controlled(psi: np.ndarray, controls, targets, U) -> None:
    n = _check_state(psi)
    U = _mat(U, len(targets))
    rc = lib().or_apply_controlled(_dptr(psi.view(np.float64)), n, _iarr(controls), len(controls), _iarr(targets),
                                   len(targets), _dptr(U.view(np.float64)))
    if rc:
        raise ValueError(f"or_apply_controlled rejected controls={controls} targets={targets}")


def apply_diag(psi: np.ndarray, targets, d) -> None:
    n = _check_state(psi)
    d = _mat(d, len(targets), diag=True)
    rc = lib().or_apply_diag(_dptr(psi.view(np.float64)), n, _iarr(targets), len(targets), _dptr(d.view(np.float64)))
    if rc:
        raise ValueError(f"or_apply_diag rejected targets={targets}")


def swap(psi: np.ndarray, a: int, b: int) -> None:
    n = _check_state(psi)
    if lib().or_swap(_dptr(psi.view(np.float64)), n, a, b):
        raise ValueError("or_swap rejected")


def fused_swap(psi: np.ndarray, p: int, q: int, s: int) -> None:
    n = _check_state(psi)
    if lib().or_fused_swap(_dptr(psi.view(np.float64)), n, p, q, s):
        raise ValueError(f"or_fused_swap rejected p={p} q={q} s={s}")


def probs(psi: np.ndarray):
    """Returns (P, norm) with P_i = |psi_i|^2 and norm = Kahan sum of P."""
    n = _check_state(psi)
    out = np.empty(1 << n, dtype=np.float64)
    nrm = ctypes.c_double(0.0)
    lib().or_probs(_dptr(psi.view(np.float64)), n, _dptr(out), ctypes.byref(nrm))
    return out, nrm.value


def scale(psi: np.ndarray, f: float) -> None:
    n = _check_state(psi)
    lib().or_scale(_dptr(psi.view(np.float64)), n, float(f))


def apply_op(psi: np.ndarray, op) -> None:
    if op.kind == "dense":
        apply_dense(psi, op.targets, op.mat)
    elif op.kind == "diag":
        apply_diag(psi, op.targets, op.mat)
    elif op.kind == "ctrl":
        apply_controlled(psi, op.controls, op.targets, op.mat)
    elif op.kind == "fswap":
        fused_swap(psi, op.p, op.q, op.s)
    else:
        raise ValueError(f"unknown op kind {op.kind!r}")


def run(circuit, psi: Optional[np.ndarray] = None, ops: Optional[Iterable] = None) -> np.ndarray:
    """Apply the circuit's ops in list order to |0..0> (or to a copy of ``psi``), unfused."""
    st = zero_state(circuit.n) if psi is None else np.array(psi, dtype=np.complex128, copy=True)
    for op in (circuit.ops if ops is None else ops):
        apply_op(st, op)
    return st


def error_metrics(psi: np.ndarray, ref: np.ndarray):
    """Infidelity 1 - |<ref|psi>|^2 / (<psi|psi><ref|ref>) and max_i |psi_i - ref_i| (complex modulus), FP64."""
    a = np.asarray(psi, dtype=np.complex128)
    b = np.asarray(ref, dtype=np.complex128)
    ov = np.vdot(b, a)
    infid = 1.0 - (abs(ov) ** 2) / (np.vdot(a, a).real * np.vdot(b, b).real)
    return float(infid), float(np.max(np.abs(a - b)))


def oracle_threads() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v else (os.cpu_count() or 1)


__all__ = ["zero_state", "apply_dense", "apply_controlled", "apply_diag", "swap", "fused_swap", "probs", "scale",
           "apply_op", "run", "error_metrics", "oracle_threads"]
