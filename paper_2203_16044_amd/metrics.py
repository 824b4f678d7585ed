"""Error of a computed state against a reference state (host-side measurement, not part of the gate path).

Used to state the complex64 engine's error next to its throughput: the infidelity
1 - |<ref|psi>|^2 / (<psi|psi> <ref|ref>), invariant under a global phase and under scaling of either state, and the
largest amplitude difference max_i |psi_i - ref_i| (complex modulus). Both are formed in FP64 from the real and
imaginary parts, accumulated with math.fsum-style exact partial sums so that a result of 0 is exactly 0.
"""
from __future__ import annotations

import math

import numpy as np


def _exact_sum(v: np.ndarray) -> float:
    return math.fsum(np.asarray(v, dtype=np.float64).ravel().tolist())


def state_error(psi, ref):
    """(infidelity, max |psi_i - ref_i|) in FP64; the infidelity is clamped at 0 against rounding below it."""
    a = np.asarray(psi).astype(np.complex128, copy=False).ravel()
    b = np.asarray(ref).astype(np.complex128, copy=False).ravel()
    if a.shape != b.shape:
        raise ValueError(f"state sizes differ: {a.shape} vs {b.shape}")
    ar, ai, br, bi = a.real, a.imag, b.real, b.imag
    # <ref|psi> = sum conj(b) a = sum (br ar + bi ai) + i (br ai - bi ar)
    ov_re = _exact_sum(br * ar) + _exact_sum(bi * ai)
    ov_im = _exact_sum(br * ai) - _exact_sum(bi * ar)
    na = _exact_sum(ar * ar) + _exact_sum(ai * ai)
    nb = _exact_sum(br * br) + _exact_sum(bi * bi)
    if not (na > 0.0 and nb > 0.0):
        raise ValueError("a state with zero norm has no fidelity")
    infid = 1.0 - (ov_re * ov_re + ov_im * ov_im) / (na * nb)
    maxd = float(np.max(np.hypot(ar - br, ai - bi))) if a.size else 0.0
    return max(0.0, infid), maxd
