"""Pins of the measurement / reset / sampling oracle: closed forms on states whose statistics are known exactly."""
import math

import numpy as np
import pytest

import circuits as C
from oracle import measure as M


def _plus(n):
    return np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)


def _ghz(n):
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = psi[-1] = 1 / math.sqrt(2)
    return psi


def test_uniform_superposition_measure():
    n = 6
    out, p1, res = M.measure(_plus(n), 2, 0.3)
    assert p1 == 0.5 and out == 1
    idx = np.arange(1 << n)
    expect = np.where((idx >> 2) & 1, 2.0 ** (-(n - 1) / 2), 0.0)
    assert np.max(np.abs(res - expect)) <= 1e-15
    out, _, _ = M.measure(_plus(n), 2, 0.7)
    assert out == 0


def test_ghz_collapses_to_a_basis_state():
    n = 5
    out, p1, res = M.measure(_ghz(n), 0, 0.7)
    assert p1 == pytest.approx(0.5) and out == 0
    assert abs(res[0] - 1.0) <= 1e-15 and np.count_nonzero(res) == 1
    out, _, res = M.measure(_ghz(n), 3, 0.2)
    assert out == 1 and abs(res[-1] - 1.0) <= 1e-15


def test_basis_state_and_unnormalised_state():
    psi = C.basis_state(4, 5) * 3.0  # |0101>, mass 9
    assert M.measure(psi, 0, 0.999)[0] == 1 and M.measure(psi, 1, 0.0)[0] == 0
    out, p1, res = M.measure(psi, 2, 0.5)
    assert out == 1 and p1 == 1.0 and abs(np.sum(np.abs(res) ** 2) - 1.0) <= 1e-15


def test_reset_leaves_the_qubit_at_zero():
    rng = np.random.Generator(np.random.PCG64(3))
    psi = C.random_state(7, 11)
    for q in (0, 3, 6):
        out, res = M.reset(psi, q, float(rng.uniform()))
        P0, P1 = M.masses(res, q)
        assert P1 == 0.0 and abs(P0 - 1.0) <= 1e-14


def test_sampling_closed_forms():
    # uniform superposition on 3 qubits: u in [j/8, (j+1)/8) -> j
    psi = _plus(3)
    for j in range(8):
        for frac in (0.1, 0.5, 0.9):
            u = (j + frac) / 8
            assert M.sample(psi, u) == j and M.sample_valid(psi, u, j)
    # a basis state is always sampled
    psi = C.basis_state(6, 37)
    for u in (0.0, 0.25, 0.999999):
        assert M.sample(psi, u) == 37 and M.sample_valid(psi, u, 37)
        assert not M.sample_valid(psi, u, 36)


def test_planted_mistake_missing_renormalisation_is_caught():
    psi = _plus(4)
    _, _, res = M.measure(psi, 1, 0.2)
    wrong = np.where(res != 0, psi, 0)  # projection without the 1/sqrt(P) factor
    assert abs(np.sum(np.abs(res) ** 2) - 1.0) <= 1e-15
    assert abs(np.sum(np.abs(wrong) ** 2) - 1.0) > 0.4
