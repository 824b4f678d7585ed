"""Pins of the state-error functions (infidelity, max |d amp|) to values the mathematics fixes.

Two independent implementations are pinned: ``oracle.error_metrics`` (numpy vdot; the tests' checker behind every
complex64 bound) and ``paper_2203_16044_amd.metrics.state_error`` (exact partial sums; used by the benchmark to state
the complex64 leg's error). Closed forms used:
  * identical states: infidelity 0, max |d| 0;
  * psi against e^{i phi} psi: infidelity 0 (a global phase is not observable), max |d| = |1 - e^{i phi}| max |psi_i|;
  * two different basis states: infidelity 1, max |d| = 1 (they differ by 1 in two places; the 2-norm of the
    difference, sqrt(2), is not what is reported);
  * cos(t)|0> + sin(t)|1> against |0>: infidelity 1 - cos^2 t = sin^2 t, max |d| = max(1 - cos t, |sin t|);
  * infidelity is invariant under scaling either state (the normalisation in its definition);
  * a planted unsquared overlap, a dropped normalisation, Re instead of the modulus of the overlap, or a max over
    real parts only fails at least one of the above.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2203_16044_amd import metrics

FUNCS = {"oracle": oracle.error_metrics, "product": metrics.state_error}


def _basis(n, x):
    v = np.zeros(1 << n, np.complex128)
    v[x] = 1.0
    return v


def _rand(n, seed):
    r = np.random.Generator(np.random.PCG64(seed))
    v = r.standard_normal(1 << n) + 1j * r.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def _violations(f):
    """Closed-form checks of an error function; returns the names of those it fails."""
    bad = []
    psi = _rand(6, 5)
    i0, d0 = f(psi, psi.copy())
    if abs(i0) > 1e-15 or d0 != 0.0:
        bad.append("identical")
    for phi in (0.3, 1.0, math.pi / 2, 2.5, math.pi):
        ph = complex(math.cos(phi), math.sin(phi))
        i1, d1 = f(ph * psi, psi)
        want = abs(1 - ph) * float(np.max(np.abs(psi)))
        if abs(i1) > 1e-14 or abs(d1 - want) > 1e-14:
            bad.append(f"phase {phi}")
        b = _basis(3, 5)
        i1, d1 = f(ph * b, b)
        if abs(i1) > 1e-15 or abs(d1 - abs(1 - ph)) > 1e-15:
            bad.append(f"basis phase {phi}")
    i2, d2 = f(_basis(4, 3), _basis(4, 9))
    if abs(i2 - 1.0) > 1e-15 or d2 != 1.0:
        bad.append("orthogonal")
    for t in (0.1, 0.7, 1.2, math.pi / 4, 3.0):
        a = np.array([math.cos(t), math.sin(t)], np.complex128)
        i3, d3 = f(a, _basis(1, 0))
        if abs(i3 - math.sin(t) ** 2) > 1e-15 or abs(d3 - max(1 - math.cos(t), abs(math.sin(t)))) > 1e-15:
            bad.append(f"rotation {t}")
    # complex overlap: (|0> + i|1>)/sqrt2 against |0>: infidelity 1/2
    a = np.array([1, 1j], np.complex128) / math.sqrt(2)
    i4, _ = f(a, _basis(1, 0))
    if abs(i4 - 0.5) > 1e-15:
        bad.append("complex overlap")
    # a state with an imaginary overlap against another: <ref|psi> = i/2 -> |.|^2 = 1/4
    ref = np.array([1, 0, 0, 0], np.complex128)
    ps = np.array([0.5j, math.sqrt(0.75), 0, 0], np.complex128)
    i5, d5 = f(ps, ref)
    if abs(i5 - 0.75) > 1e-15 or abs(d5 - max(abs(0.5j - 1), math.sqrt(0.75))) > 1e-15:
        bad.append("imaginary overlap")
    # scaling either state leaves the infidelity unchanged
    other = _rand(6, 6)
    base, _ = f(psi, other)
    for s1, s2 in ((3.0, 1.0), (1.0, 0.25), (2.0, 5.0)):
        i6, _ = f(s1 * psi, s2 * other)
        if abs(i6 - base) > 1e-14:
            bad.append(f"scale {s1},{s2}")
    return bad


@pytest.mark.parametrize("name", sorted(FUNCS))
def test_error_metrics_closed_forms(name):
    assert _violations(FUNCS[name]) == []


def test_error_functions_agree_on_random_states():
    for seed in range(4):
        a = _rand(10, 100 + seed)
        b = a + 1e-6 * _rand(10, 200 + seed)
        i1, d1 = oracle.error_metrics(a, b)
        i2, d2 = metrics.state_error(a, b)
        assert abs(i1 - i2) <= 1e-14 and abs(d1 - d2) <= 1e-18


def _unsquared(psi, ref):
    a, b = np.asarray(psi, np.complex128), np.asarray(ref, np.complex128)
    ov = np.vdot(b, a)
    return float(1 - abs(ov) / np.sqrt(np.vdot(a, a).real * np.vdot(b, b).real)), float(np.max(np.abs(a - b)))


def _unnormalised(psi, ref):
    a, b = np.asarray(psi, np.complex128), np.asarray(ref, np.complex128)
    return float(1 - abs(np.vdot(b, a)) ** 2), float(np.max(np.abs(a - b)))


def _real_part(psi, ref):
    a, b = np.asarray(psi, np.complex128), np.asarray(ref, np.complex128)
    ov = np.vdot(b, a)
    return float(1 - ov.real ** 2 / (np.vdot(a, a).real * np.vdot(b, b).real)), float(np.max(np.abs(a - b)))


def _max_real(psi, ref):
    a, b = np.asarray(psi, np.complex128), np.asarray(ref, np.complex128)
    i, _ = oracle.error_metrics(a, b)
    return i, float(np.max(np.abs((a - b).real)))


@pytest.mark.parametrize("planted", [_unsquared, _unnormalised, _real_part, _max_real])
def test_pins_catch_planted_mistakes(planted):
    assert _violations(planted) != []
