"""Oracle for measurement, reset and sampling (TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``).

A circuit may contain measurements and resets besides gates (Sec. II-A), and the probability of observing a
basis state is the squared modulus of its amplitude (Eq. 1, generalised to n qubits in Eq. 2). Written from those
definitions in FP64 with exactly rounded sums (math.fsum), independent of the GPU library:
  * masses(psi, q): (P0, P1), the total |a_i|^2 over the indices whose bit q is 0 / 1;
  * measure(psi, q, u): outcome 1 iff u (P0 + P1) < P1; the amplitudes of the observed outcome are multiplied by
    1/sqrt(P_outcome), the others set to 0 (the projection onto the observed outcome, renormalised);
  * reset(psi, q, u): measure, then flip the qubit to 0 if the outcome was 1;
  * sample_valid(psi, u, idx): whether index idx is the inverse-CDF sample of u (the smallest i whose cumulative
    mass exceeds u x total), allowing a rounding tolerance at the boundaries.
"""
from __future__ import annotations

import math

import numpy as np


def _p(psi: np.ndarray) -> np.ndarray:
    return psi.real.astype(np.float64) ** 2 + psi.imag.astype(np.float64) ** 2


def masses(psi: np.ndarray, q: int):
    p = _p(psi)
    bit = (np.arange(p.size, dtype=np.int64) >> q) & 1
    return math.fsum(p[bit == 0].tolist()), math.fsum(p[bit == 1].tolist())


def measure(psi: np.ndarray, q: int, u: float):
    """Returns (outcome, P1 / (P0 + P1), collapsed state as complex128)."""
    P0, P1 = masses(psi, q)
    tot = P0 + P1
    if not tot > 0.0:
        raise ValueError("state without mass")
    out = 1 if u * tot < P1 else 0
    keep = P1 if out else P0
    f = 1.0 / math.sqrt(keep)
    bit = (np.arange(psi.size, dtype=np.int64) >> q) & 1
    res = np.where(bit == out, psi.astype(np.complex128) * f, 0.0 + 0.0j)
    return out, P1 / tot, res


def reset(psi: np.ndarray, q: int, u: float):
    out, _, res = measure(psi, q, u)
    if out:
        idx = np.arange(res.size, dtype=np.int64)
        res = res[idx ^ (1 << q)]  # X on qubit q: a_i <- a_(i xor 2^q)
    return out, res


def _dist(psi: np.ndarray):
    p = _p(psi)
    return p, np.cumsum(p), math.fsum(p.tolist())


def samples_valid(psi: np.ndarray, us, idxs, rtol: float = 1e-12) -> np.ndarray:
    """For each (u, idx): idx is the smallest i with cum[i] > u * total, up to rtol * total at the boundaries, and
    has mass. The distribution is built once for all shots."""
    p, cum, total = _dist(psi)
    us = np.asarray(us, dtype=np.float64)
    idxs = np.asarray(idxs, dtype=np.int64)
    ok = (idxs >= 0) & (idxs < p.size)
    j = np.where(ok, idxs, 0)
    target = us * total
    tol = rtol * total
    excl = cum[j] - p[j]
    return ok & (p[j] > 0.0) & (excl <= target + tol) & (cum[j] > target - tol)


def sample_valid(psi: np.ndarray, u: float, idx: int, rtol: float = 1e-12) -> bool:
    return bool(samples_valid(psi, [u], [idx], rtol)[0])


def samples(psi: np.ndarray, us) -> np.ndarray:
    """The inverse-CDF indices of the uniforms `us` (FP64 cumulative sums)."""
    p, cum, _ = _dist(psi)
    i = np.searchsorted(cum, np.asarray(us, dtype=np.float64) * cum[-1], side="right")
    return np.minimum(i, p.size - 1).astype(np.int64)


def sample(psi: np.ndarray, u: float) -> int:
    return int(samples(psi, [u])[0])
