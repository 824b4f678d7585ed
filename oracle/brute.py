"""Independent brute-force formulations used only to pin the loop oracle (test infrastructure).

The state is viewed as an n-dimensional tensor of shape (2,)*n in C order, so tensor axis m carries
qubit n-1-m (qubit q = bit q of the index, Sec. II-A Eq. 4). Gates become tensor contractions
(numpy.tensordot), Kronecker products (numpy.kron) or axis transpositions (numpy.transpose) -- none of
which shares structure with the oracle's index loops.
"""
from __future__ import annotations

import math

import numpy as np


def _axis(n: int, q: int) -> int:
    return n - 1 - q


def apply_dense(psi: np.ndarray, targets, U) -> np.ndarray:
    """psi' = U acting on ``targets`` (targets[j] <-> bit j of U's index) via tensordot."""
    n = int(psi.size).bit_length() - 1
    k = len(targets)
    T = np.asarray(psi, dtype=np.complex128).reshape((2,) * n)
    # U reshaped C-order: axis m of the output/input halves is matrix bit k-1-m, i.e. qubit targets[k-1-m]
    Ut = np.asarray(U, dtype=np.complex128).reshape((2,) * (2 * k))
    in_axes = [_axis(n, targets[k - 1 - m]) for m in range(k)]
    R = np.tensordot(Ut, T, axes=(list(range(k, 2 * k)), in_axes))
    # R axes: the k output bits first, then T's remaining axes in order; move the output bits back
    R = np.moveaxis(R, list(range(k)), in_axes)
    return np.ascontiguousarray(R).reshape(-1)


def apply_controlled(psi: np.ndarray, controls, targets, U) -> np.ndarray:
    """Controlled-U as a dense (c+k)-qubit block matrix diag(I, .., I, U) with the controls as the
    high bits of its index."""
    k, c = len(targets), len(controls)
    K = 1 << k
    full = np.eye(1 << (k + c), dtype=np.complex128)
    full[-K:, -K:] = np.asarray(U, dtype=np.complex128)
    return apply_dense(psi, list(targets) + list(controls), full)


def apply_diag(psi: np.ndarray, targets, d) -> np.ndarray:
    return apply_dense(psi, targets, np.diag(np.asarray(d, dtype=np.complex128)))


def kron_1q(n: int, q: int, U) -> np.ndarray:
    """The full 2^n x 2^n matrix I (x) .. (x) U (x) .. (x) I, U at Kronecker factor n-1-q from the left."""
    return np.kron(np.kron(np.eye(1 << (n - 1 - q)), np.asarray(U, dtype=np.complex128)), np.eye(1 << q))


def fused_swap(psi: np.ndarray, p: int, q: int, s: int) -> np.ndarray:
    """Fused-swap as one transposition of tensor axes: qubit p+j <-> qubit q+j for all j < s at once."""
    n = int(psi.size).bit_length() - 1
    T = np.asarray(psi).reshape((2,) * n)
    perm = list(range(n))
    for j in range(s):
        a, b = _axis(n, p + j), _axis(n, q + j)
        perm[a], perm[b] = perm[b], perm[a]
    return np.ascontiguousarray(np.transpose(T, perm)).reshape(-1)


def apply_op(psi: np.ndarray, op) -> np.ndarray:
    if op.kind == "dense":
        return apply_dense(psi, op.targets, op.mat)
    if op.kind == "diag":
        return apply_diag(psi, op.targets, op.mat)
    if op.kind == "ctrl":
        return apply_controlled(psi, op.controls, op.targets, op.mat)
    if op.kind == "fswap":
        return fused_swap(psi, op.p, op.q, op.s)
    raise ValueError(op.kind)


def run(circuit, psi=None) -> np.ndarray:
    st = np.zeros(1 << circuit.n, dtype=np.complex128) if psi is None else np.array(psi, dtype=np.complex128)
    if psi is None:
        st[0] = 1.0
    for op in circuit.ops:
        st = apply_op(st, op)
    return st


def norm_fsum(psi: np.ndarray) -> float:
    return math.fsum((np.abs(psi) ** 2).tolist())
