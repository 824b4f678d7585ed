"""Pins of the CPU oracle to things other than itself (closed forms, brute force, invariants, truth tables).

Every check here runs on the CPU. The brute-force side (``oracle.brute``) is built from numpy tensor
contractions, Kronecker products and axis transpositions, not from the oracle's index loops.
"""
import math

import numpy as np
import pytest

import circuits as C
import oracle
from oracle import brute

TOL = 1e-13


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _rand_u(rng, dim):
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


# ------------------------------------------------------------------------------------------------ brute force

@pytest.mark.parametrize("n", [1, 3, 6, 9])
def test_dense_matches_tensordot(n):
    rng = _rng(100 + n)
    for k in range(1, min(n, 5) + 1):
        for _ in range(3):
            t = [int(v) for v in rng.choice(n, size=k, replace=False)]
            U = _rand_u(rng, 1 << k)
            psi = C.random_state(n, int(rng.integers(1 << 30)))
            a = psi.copy()
            oracle.apply_dense(a, t, U)
            b = brute.apply_dense(psi, t, U)
            assert np.max(np.abs(a - b)) < TOL, (n, k, t)


@pytest.mark.parametrize("n", [2, 5, 8])
def test_one_qubit_matches_kronecker(n):
    """Eq. 4 at every target q equals I (x) .. (x) U (x) .. (x) I acting on the whole vector."""
    rng = _rng(200 + n)
    for q in range(n):
        U = _rand_u(rng, 2)
        psi = C.random_state(n, 7 * q + n)
        a = psi.copy()
        oracle.apply_dense(a, [q], U)
        ref = brute.kron_1q(n, q, U) @ psi
        assert np.max(np.abs(a - ref)) < TOL
        # the two brute formulations agree with each other too
        assert np.max(np.abs(brute.apply_dense(psi, [q], U) - ref)) < TOL


def test_brute_two_qubit_against_kronecker():
    """Adjacent targets (t0=q, t1=q+1): U acts as the Kronecker factor on bits (q+1, q) with bit j <-> t_j."""
    n, q = 6, 2
    rng = _rng(3)
    U = _rand_u(rng, 4)
    psi = C.random_state(n, 11)
    M = np.kron(np.kron(np.eye(1 << (n - 2 - q)), U), np.eye(1 << q))
    assert np.max(np.abs(brute.apply_dense(psi, [q, q + 1], U) - M @ psi)) < TOL
    a = psi.copy()
    oracle.apply_dense(a, [q, q + 1], U)
    assert np.max(np.abs(a - M @ psi)) < TOL


@pytest.mark.parametrize("n", [3, 7])
def test_controlled_matches_brute(n):
    rng = _rng(300 + n)
    for _ in range(6):
        k = int(rng.integers(1, min(3, n - 1) + 1))
        c = int(rng.integers(1, min(3, n - k) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + c, replace=False)]
        t, cc = qs[:k], qs[k:]
        U = _rand_u(rng, 1 << k)
        psi = C.random_state(n, int(rng.integers(1 << 30)))
        a = psi.copy()
        oracle.apply_controlled(a, cc, t, U)
        assert np.max(np.abs(a - brute.apply_controlled(psi, cc, t, U))) < TOL


def test_controlled_leaves_control_zero_subspace_bit_identical():
    n = 6
    rng = _rng(4)
    psi = C.random_state(n, 5)
    a = psi.copy()
    oracle.apply_controlled(a, [4, 1], [2], _rand_u(rng, 2))
    untouched = [i for i in range(1 << n) if not ((i >> 4) & 1 and (i >> 1) & 1)]
    assert a[untouched].tobytes() == psi[untouched].tobytes()


@pytest.mark.parametrize("n", [2, 8])
def test_diag_matches_brute(n):
    rng = _rng(400 + n)
    for k in range(1, min(n, 4) + 1):
        t = [int(v) for v in rng.choice(n, size=k, replace=False)]
        d = np.exp(1j * rng.uniform(0, 2 * math.pi, size=1 << k))
        psi = C.random_state(n, k)
        a = psi.copy()
        oracle.apply_diag(a, t, d)
        assert np.max(np.abs(a - brute.apply_diag(psi, t, d))) < TOL


@pytest.mark.parametrize("n", [4, 10])
def test_random_circuits_all_kinds_match_brute(n):
    for seed in range(3):
        circ = C.random_circuit(n, seed=1000 * n + seed, num_ops=30, kmax=3)
        a = oracle.run(circ, C.random_state(n, seed))
        b = brute.run(circ, C.random_state(n, seed))
        assert np.max(np.abs(a - b)) < 1e-12


def test_u3_cnot_small_matches_brute():
    circ = C.u3_cnot_layers(n=10, seed=16, layers=4)
    assert np.max(np.abs(oracle.run(circ) - brute.run(circ))) < 1e-12


# ------------------------------------------------------------------------------------------------ fused-swap

def _sigma(x, p, q, s):
    """The bit permutation of fused_swap(p, q, s): bit p+j <-> bit q+j."""
    y = x
    for j in range(s):
        bp, bq = (x >> (p + j)) & 1, (x >> (q + j)) & 1
        y &= ~((1 << (p + j)) | (1 << (q + j)))
        y |= (bq << (p + j)) | (bp << (q + j))
    return y


@pytest.mark.parametrize("n,p,q,s", [(4, 0, 2, 2), (8, 0, 4, 4), (8, 5, 1, 3), (9, 2, 6, 3), (7, 0, 1, 1),
                                     (10, 0, 7, 3), (6, 3, 0, 3), (5, 1, 3, 0)])
def test_fused_swap_against_axis_transpose_and_sigma(n, p, q, s):
    psi = C.random_state(n, n + 13 * s)
    a = psi.copy()
    oracle.fused_swap(a, p, q, s)
    # bit-exact against a single numpy axis transposition
    assert a.tobytes() == brute.fused_swap(psi, p, q, s).tobytes()
    # psi'[sigma(i)] = psi[i]
    sig = np.array([_sigma(i, p, q, s) for i in range(1 << n)])
    assert a[sig].tobytes() == psi.tobytes()
    # moved amplitudes: exactly 2^n (1 - 2^-s) (Sec. III-D communication volume)
    moved = int(np.count_nonzero(sig != np.arange(1 << n)))
    assert moved == (1 << n) - (1 << (n - s))
    # involution
    oracle.fused_swap(a, p, q, s)
    assert a.tobytes() == psi.tobytes()


def test_fused_swap_basis_states():
    n, p, q, s = 8, 1, 5, 3
    for x in [0, 1, 0b10110110, 0b01001010, 255, 37]:
        a = C.basis_state(n, x)
        oracle.fused_swap(a, p, q, s)
        assert np.flatnonzero(a).tolist() == [_sigma(x, p, q, s)]


@pytest.mark.parametrize("args", [(0, 1, 2), (2, 0, 3), (0, 6, 3), (-1, 3, 1), (0, 4, -1)])
def test_fused_swap_rejects_overlap_and_range(args):
    psi = C.random_state(8, 1)
    with pytest.raises(ValueError):
        oracle.fused_swap(psi, *args)


# ------------------------------------------------------------------------------------------------ closed forms

@pytest.mark.parametrize("n", [1, 5, 12])
def test_hadamard_all_qubits_uniform(n):
    circ = C.Circuit(n, [C.Op("dense", (q,), mat=C.h()) for q in range(n)])
    psi = oracle.run(circ)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-15


def test_hadamard_x11_benchmark_uniform():
    """Sec. IV-D: eleven H per qubit; H^2 = I so the result is H^{(x)n}|0..0>, uniform 2^(-n/2)."""
    n = 10
    psi = oracle.run(C.hadamard_x11(n))
    assert np.max(np.abs(psi - 2.0 ** (-n / 2))) < 1e-14


def test_product_state_closed_form():
    n = 9
    rng = _rng(9)
    us = [C.u3(*rng.uniform(0, 2 * math.pi, 3)) for _ in range(n)]
    circ = C.Circuit(n, [C.Op("dense", (q,), mat=us[q]) for q in range(n)])
    psi = oracle.run(circ)
    for i in range(1 << n):
        ref = np.prod([us[q][(i >> q) & 1, 0] for q in range(n)])
        assert abs(psi[i] - ref) < 1e-15


def test_ghz_two_amplitudes():
    n = 11
    psi = oracle.run(C.ghz(n))
    nz = np.flatnonzero(psi)
    assert nz.tolist() == [0, (1 << n) - 1]
    assert np.max(np.abs(psi[nz] - 1 / math.sqrt(2))) < 1e-15


def test_rz_layer_on_uniform_closed_form():
    n = 8
    rng = _rng(8)
    th = rng.uniform(0, 2 * math.pi, n)
    ops = [C.Op("dense", (q,), mat=C.h()) for q in range(n)] + [C.Op("diag", (q,), mat=C.rz(th[q])) for q in range(n)]
    psi = oracle.run(C.Circuit(n, ops))
    for i in range(1 << n):
        ph = sum((0.5 if (i >> q) & 1 else -0.5) * th[q] for q in range(n))
        assert abs(psi[i] - 2.0 ** (-n / 2) * np.exp(1j * ph)) < 1e-15


def test_echo_returns_to_zero_state():
    n = 10
    circ = C.random_circuit(n, seed=77, num_ops=40, kmax=4)
    inv = C.inverse_circuit(circ)
    psi = oracle.run(circ)
    back = oracle.run(inv, psi)
    assert abs(back[0] - 1.0) < 1e-12
    assert np.max(np.abs(back[1:])) < 1e-12


def test_norm_preserved_u3_cnot():
    psi = oracle.run(C.u3_cnot_layers())
    _, nrm = oracle.probs(psi)
    assert abs(nrm - 1.0) < 1e-12


# ------------------------------------------------------------------------------------------------ permutations

def _basis_map(n, op, x):
    a = C.basis_state(n, x)
    oracle.apply_op(a, op)
    nz = np.flatnonzero(a)
    assert len(nz) == 1 and a[nz[0]] == 1.0
    return int(nz[0])


def test_permutation_truth_tables():
    n = 5
    X = C.x_gate()
    swap2 = np.eye(4, dtype=np.complex128)[[0, 2, 1, 3]]
    for x in range(1 << n):
        assert _basis_map(n, C.Op("dense", (3,), mat=X), x) == x ^ (1 << 3)
        cnot = C.Op("ctrl", (4,), (1,), mat=X)
        assert _basis_map(n, cnot, x) == (x ^ (1 << 4) if (x >> 1) & 1 else x)
        tof = C.Op("ctrl", (0,), (2, 4), mat=X)
        assert _basis_map(n, tof, x) == (x ^ 1 if ((x >> 2) & 1 and (x >> 4) & 1) else x)
        b0, b3 = (x >> 0) & 1, (x >> 3) & 1
        assert _basis_map(n, C.Op("dense", (0, 3), mat=swap2), x) == (x & ~0b1001) | (b0 << 3) | b3


def test_permutation_moves_are_bit_exact_with_signed_zeros():
    n = 6
    rng = _rng(6)
    psi = C.random_state(n, 2)
    v = psi.view(np.float64)
    v[rng.choice(v.size, 20, replace=False)] = -0.0
    ref = psi.copy()
    a = psi.copy()
    oracle.apply_dense(a, [2], C.x_gate())
    perm = np.arange(1 << n) ^ (1 << 2)
    assert a.tobytes() == ref[perm].tobytes()
    # a monomial matrix with +-1, +-i entries is an exact move with sign/component exchange
    Y = np.array([[0, -1j], [1j, 0]])
    b = psi.copy()
    oracle.apply_dense(b, [4], Y)
    exp = np.empty_like(psi)
    for i in range(1 << n):
        j = i ^ (1 << 4)
        x = psi[j]
        exp[i] = complex(x.imag, -x.real) if not (i >> 4) & 1 else complex(-x.imag, x.real)
    assert b.view(np.uint64).tolist() == exp.view(np.uint64).tolist()


# ------------------------------------------------------------------------------------------------ probabilities

def test_probs_basis_one_hot_and_uniform():
    n = 7
    P, nrm = oracle.probs(C.basis_state(n, 93))
    assert P[93] == 1.0 and np.count_nonzero(P) == 1 and nrm == 1.0
    psi = oracle.run(C.Circuit(n, [C.Op("dense", (q,), mat=C.h()) for q in range(n)]))
    P, nrm = oracle.probs(psi)
    assert np.max(np.abs(P - 2.0 ** -n)) < 1e-17
    assert abs(nrm - 1.0) < 1e-14  # 1/sqrt(2) is rounded once per H


def test_probs_norm_is_compensated_sum():
    psi = C.random_state(12, 3) * 1.7
    P, nrm = oracle.probs(psi)
    assert np.array_equal(P, psi.real ** 2 + psi.imag ** 2)
    assert abs(nrm - math.fsum(P.tolist())) <= 2e-16 * nrm


def test_scale_closed_forms():
    """a_i <- f a_i (the renormalisation step): f = -1 negates every component exactly (signed zeros too), powers of
    two scale exactly, and f = 1/sqrt(norm) leaves the norm 1 (Sec. II-A: sum |a_i|^2 = 1)."""
    psi = C.random_state(9, 11) * 3.0
    psi[5] = complex(0.0, -0.0)
    a = psi.copy()
    oracle.scale(a, -1.0)
    assert np.array_equal(a.view(np.float64), -psi.view(np.float64))
    assert np.signbit(a.view(np.float64)[10]) and not np.signbit(a.view(np.float64)[11])
    for f in (0.5, 4.0, 2.0 ** -30):
        a = psi.copy()
        oracle.scale(a, f)
        assert np.array_equal(a.view(np.float64), psi.view(np.float64) * f)
    _, nrm = oracle.probs(psi)
    a = psi.copy()
    oracle.scale(a, 1.0 / math.sqrt(nrm))
    assert abs(oracle.probs(a)[1] - 1.0) < 1e-14
    b = C.random_state(6, 12)
    c = b.copy()
    oracle.scale(c, 0.3)
    assert np.max(np.abs(c - 0.3 * b)) <= 1e-16  # each component rounded once


# ------------------------------------------------------------------------------------------------ planted mistakes

def test_pins_catch_planted_mistakes():
    """Plausible oracle mistakes -- a transposed matrix, swapped target order, a conjugated entry, a dropped
    off-diagonal term -- each fail the brute-force pin (planted on the CPU, in the oracle's inputs)."""
    n = 6
    rng = _rng(12)
    U = _rand_u(rng, 4)
    t = [1, 4]
    psi = C.random_state(n, 12)
    ref = brute.apply_dense(psi, t, U)
    mistakes = {
        "transposed": (t, U.T),
        "swapped_targets": (t[::-1], U),
        "conjugated": (t, np.conj(U)),
        "dropped_term": (t, U * (1 - np.eye(4)[[0]].T @ np.eye(4)[[1]])),
    }
    for name, (tt, M) in mistakes.items():
        a = psi.copy()
        oracle.apply_dense(a, tt, M)
        assert np.max(np.abs(a - ref)) > 1e-3, name


# ------------------------------------------------------------------------------------------------ inputs

def test_haar_su4_is_special_unitary():
    rng = _rng(1)
    for _ in range(20):
        U = C.haar_su4(rng)
        assert np.max(np.abs(U.conj().T @ U - np.eye(4))) < 1e-14
        assert abs(np.linalg.det(U) - 1.0) < 1e-13


def test_config_shapes():
    c0 = C.u3_cnot_layers()
    assert c0.n == 16 and c0.count(["dense"]) == 160 and c0.count(["ctrl"]) == 75 and c0.count(["fswap"]) == 1
    c1 = C.mixed_layers()
    assert c1.count(["dense"]) == 560 and c1.count(["fswap"]) == 3 and c1.count(["ctrl"]) == 32
    assert sum(1 for o in c1.ops if o.label == "RZ") == 560 and sum(1 for o in c1.ops if o.label == "CZ") == 270
    c2 = C.su4_u3_random()
    assert c2.n == 32 and len(c2) == 1920
    c3 = C.su4_u3_renorm()
    assert c3.n == 33 and len(c3) == 40 * (16 + 33) and c3.renorm_after == (10, 20, 30, 40)
    b = C.serving_batch(count=16)
    assert all(10 <= c.n <= 22 for c in b)


def test_oracle_rejects_matrix_shape_mismatch():
    psi = C.random_state(4, 0)
    with pytest.raises(ValueError):
        oracle.apply_dense(psi, [0, 1], np.eye(2))
    with pytest.raises(ValueError):
        oracle.apply_controlled(psi, [2], [0, 1], np.eye(2))
    with pytest.raises(ValueError):
        oracle.apply_diag(psi, [0], np.ones(4))


def test_seeded_generators_are_deterministic():
    """The shared input generators give bit-identical circuits and states for the same seed (both sides of every
    comparison draw from them), and different ones for another seed."""
    a, b = C.su4_u3_random(n=10, seed=3, layers=4), C.su4_u3_random(n=10, seed=3, layers=4)
    assert [(o.kind, o.targets, o.mat.tobytes()) for o in a.ops] == [(o.kind, o.targets, o.mat.tobytes()) for o in b.ops]
    c = C.su4_u3_random(n=10, seed=4, layers=4)
    assert [o.mat.tobytes() for o in a.ops] != [o.mat.tobytes() for o in c.ops]
    assert C.random_state(9, 5).tobytes() == C.random_state(9, 5).tobytes()
    x, y = C.serving_batch(count=6, seed=9, nmin=10, nmax=12, dmin=2, dmax=3), C.serving_batch(count=6, seed=9, nmin=10, nmax=12, dmin=2, dmax=3)
    assert [len(u.ops) for u in x] == [len(v.ops) for v in y]
    assert all(p.mat.tobytes() == q.mat.tobytes() for u, v in zip(x, y) for p, q in zip(u.ops, v.ops))
