"""GPU parity of the plain gate path (through the C ABI) against the CPU oracle.

Bar: complex128 max |d amp| <= 1e-12; permutation and fused-swap paths bit-exact (signed zeros included);
complex64 within the error of FP32 arithmetic (max |d amp| stated per test) and bit-exact on moves.
Sizes span partial blocks (n < 9), several blocks with grid-stride tails, and the full 28/32-qubit shapes
(checked through closed forms and sampled amplitudes there).
"""
import math

import numpy as np
import pytest

import circuits as C
import oracle

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _rand_u(rng, dim):
    z = rng.standard_normal((dim, dim)) + 1j * rng.standard_normal((dim, dim))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _with_signed_zeros(psi, seed, count=32):
    rng = _rng(seed)
    v = psi.view(np.float64)
    v[rng.choice(v.size, min(count, v.size), replace=False)] = -0.0
    return psi


def _run_both(gpu, n, ops, psi0, dtype="c128"):
    st = gpu.State(n, dtype)
    st.set(psi0)
    for op in ops:
        st.apply_op(op)
    got = st.get()
    st.close()
    start = np.asarray(psi0.astype(np.complex64) if dtype == "c64" else psi0, dtype=np.complex128)
    ref = oracle.run(C.Circuit(n), start, ops=ops)
    return got, ref


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128))))


# ------------------------------------------------------------------------------------------------ dense

@pytest.mark.parametrize("n", [1, 3, 8, 11, 14])
def test_dense_one_qubit_every_target(gpu, n):
    rng = _rng(n)
    ops = [C.Op("dense", (q,), mat=_rand_u(rng, 2)) for q in range(n)]
    got, ref = _run_both(gpu, n, ops, C.random_state(n, n))
    assert _maxerr(got, ref) <= TOL128


@pytest.mark.parametrize("k", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("n", [7, 12])
def test_dense_k_qubit(gpu, k, n):
    rng = _rng(10 * n + k)
    ops = []
    for _ in range(4):
        t = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        ops.append(C.Op("dense", t, mat=_rand_u(rng, 1 << k)))
    got, ref = _run_both(gpu, n, ops, C.random_state(n, k))
    assert _maxerr(got, ref) <= TOL128


def test_dense_low_and_high_targets_full_coverage(gpu):
    """All ordered target pairs on 6 qubits (sorted / unsorted order, adjacent / distant)."""
    n = 6
    rng = _rng(66)
    ops = [C.Op("dense", (a, b), mat=_rand_u(rng, 4)) for a in range(n) for b in range(n) if a != b]
    got, ref = _run_both(gpu, n, ops, C.random_state(n, 6))
    assert _maxerr(got, ref) <= TOL128


# ------------------------------------------------------------------------------------------------ controlled

@pytest.mark.parametrize("n", [5, 13])
def test_controlled_dense(gpu, n):
    rng = _rng(300 + n)
    ops = []
    for _ in range(10):
        k = int(rng.integers(1, min(4, n - 1) + 1))
        c = int(rng.integers(1, min(3, n - k) + 1))
        qs = [int(v) for v in rng.choice(n, size=k + c, replace=False)]
        ops.append(C.Op("ctrl", tuple(qs[:k]), tuple(qs[k:]), mat=_rand_u(rng, 1 << k)))
    got, ref = _run_both(gpu, n, ops, C.random_state(n, 3))
    assert _maxerr(got, ref) <= TOL128


# ------------------------------------------------------------------------------------------------ diagonal

@pytest.mark.parametrize("n", [4, 12])
def test_diag_full_and_sparse(gpu, n):
    rng = _rng(500 + n)
    ops = []
    for k in range(1, 5):
        t = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        d = np.exp(1j * rng.uniform(0, 2 * math.pi, 1 << k))
        ops.append(C.Op("diag", t, mat=d))  # dense diagonal: full pass
        ds = np.ones(1 << k, dtype=np.complex128)
        ds[-1] = np.exp(1j * rng.uniform(0, 2 * math.pi))  # one non-unit entry: subspace pass
        ops.append(C.Op("diag", t, mat=ds))
        dm = d.copy()
        dm[::2] = 1.0
        dm[1] = -1.0
        ops.append(C.Op("diag", t, mat=dm))  # mixed classes
    ops.append(C.Op("diag", (0, 1), mat=C.CZ_DIAG))
    ops.append(C.Op("dense", (n - 1,), mat=np.diag(C.rz(0.7))))  # exactly diagonal dense -> diagonal path
    got, ref = _run_both(gpu, n, ops, C.random_state(n, 5))
    assert _maxerr(got, ref) <= TOL128


def test_diag_sign_flips_and_unit_entries_are_exact(gpu):
    n = 10
    psi = _with_signed_zeros(C.random_state(n, 9), 9)
    ops = [C.Op("diag", (2, 7), mat=C.CZ_DIAG), C.Op("diag", (5,), mat=np.array([1, -1], dtype=complex)),
           C.Op("diag", (1, 3, 8), mat=np.array([1, -1, 1, 1, -1, 1, 1, -1], dtype=complex))]
    got, ref = _run_both(gpu, n, ops, psi)
    assert got.tobytes() == ref.tobytes()


# ------------------------------------------------------------------------------------------------ permutations

def _monomial(rng, k):
    P = np.eye(1 << k, dtype=np.complex128)[rng.permutation(1 << k)]
    return P * rng.choice([1, -1, 1j, -1j], size=(1 << k))[None, :]


@pytest.mark.parametrize("n", [3, 9, 14])
def test_permutation_gates_bit_exact(gpu, n):
    rng = _rng(700 + n)
    X = C.x_gate()
    ops = [C.Op("dense", (n - 1,), mat=X), C.Op("dense", (0,), mat=X)]
    if n >= 2:
        ops.append(C.Op("ctrl", (0,), (n - 1,), mat=X))
        ops.append(C.Op("dense", (0, n - 1), mat=np.eye(4)[[0, 2, 1, 3]]))  # SWAP
    if n >= 3:
        ops.append(C.Op("ctrl", (1,), (0, n - 1), mat=X))  # Toffoli
    for k in range(1, min(6, n) + 1):
        t = tuple(int(v) for v in rng.choice(n, size=k, replace=False))
        ops.append(C.Op("dense", t, mat=_monomial(rng, k)))
        if n - k >= 1:
            rest = [q for q in range(n) if q not in t]
            ops.append(C.Op("ctrl", t, (int(rng.choice(rest)),), mat=_monomial(rng, k)))
    psi = _with_signed_zeros(C.random_state(n, n), n)
    got, ref = _run_both(gpu, n, ops, psi)
    assert got.tobytes() == ref.tobytes()


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n", [3, 6, 11, 15])
def test_whole_line_monomials_bit_exact(gpu, dtype, n):
    """Monomial diagonals and controlled moves with a target or control inside a 128-byte line (bits 0-2 for
    complex128, 0-3 for complex64): when every line holds a changed amplitude they run in lane order (cross-lane
    moves, 0-2 of their qubits outside the wave), otherwise as strided moves; both bit-exact, signed zeros kept.
    n = 3 and 6 are below the lane form's minimum state (every qubit involved, or fewer amplitudes than a wave)."""
    rng = _rng(1100 + n)
    X = C.x_gate()
    ph = np.array([1, -1, 1j, -1j], dtype=complex)
    ops = [C.Op("diag", (0, 1), mat=C.CZ_DIAG), C.Op("diag", (n - 1, 0), mat=C.CZ_DIAG),
           C.Op("diag", (2,), mat=np.array([1, 1j], dtype=complex)),
           C.Op("ctrl", (0,), (n - 1,), mat=X), C.Op("ctrl", (n - 1,), (1,), mat=X),  # targets, then controls
           C.Op("ctrl", (2,), (0, 1), mat=X), C.Op("ctrl", (0,), (1, n - 1), mat=X),  # Toffolis
           C.Op("dense", (1, n - 1), mat=np.eye(4)[[0, 1, 3, 2]])]  # CNOT as a 2-qubit gate: fixed points
    if n >= 9:  # two qubits outside the wave, every line changed
        ops.append(C.Op("diag", (0, n - 2, n - 1), mat=np.array([1, -1, 1j, 1, -1j, -1, 1, 1j], dtype=complex)))
        ops.append(C.Op("ctrl", (n - 1, n - 2), (0,), mat=_monomial(rng, 2)))
        ops.append(C.Op("ctrl", (n - 3,), (1, 2), mat=C.x_gate()))  # Toffoli, controls inside the line
    for k in range(1, min(6, n) + 1):
        t = [0] + [int(v) for v in rng.choice(np.arange(1, n), size=k - 1, replace=False)]
        rng.shuffle(t)
        d = rng.choice(ph, size=1 << k)
        d[0] = 1.0
        ops.append(C.Op("diag", tuple(t), mat=d))
        if k + 1 <= min(6, n):
            rest = [q for q in range(n) if q not in t]
            ops.append(C.Op("ctrl", tuple(t), (int(rng.choice(rest)),), mat=_monomial(rng, k)))
            low = [q for q in range(4) if q < n and q not in t]
            if low:
                ops.append(C.Op("ctrl", tuple(t), (low[-1],), mat=_monomial(rng, k)))
    psi = C.random_state(n, 1200 + n)
    if dtype == "c64":
        psi = psi.astype(np.complex64).astype(np.complex128)
    psi = _with_signed_zeros(psi, n)
    got, ref = _run_both(gpu, n, ops, psi, dtype=dtype)
    if dtype == "c64":
        assert got.tobytes() == ref.astype(np.complex64).tobytes()
    else:
        assert got.tobytes() == ref.tobytes()


# ------------------------------------------------------------------------------------------------ fused-swap

FSWAP_CASES = [
    (4, 0, 2, 2), (8, 0, 4, 4), (8, 5, 1, 3), (10, 0, 7, 3), (7, 0, 1, 1),  # small / generic
    (16, 0, 12, 4),  # the 16-qubit circuit's swap: runs of 1 amplitude
    (18, 1, 12, 5), (18, 2, 9, 6), (20, 0, 14, 6),  # LDS path, various run lengths
    (18, 4, 12, 6), (18, 6, 12, 6), (20, 5, 15, 5), (19, 4, 8, 3),  # run path (>= 128-byte runs)
    (18, 3, 12, 1), (19, 3, 10, 4), (12, 3, 7, 2),  # run path, runs of exactly one line (s <= 4)
    (18, 3, 11, 7), (20, 3, 13, 6),  # one-line runs with s > 4: LDS tiles
    (16, 12, 0, 4),  # reversed argument order
    # wide-row path (s <= 3, runs < 128 B): carried mid bits x = 9/7/5, capped by few mid bits, none at all
    (18, 0, 12, 1), (18, 0, 14, 2), (18, 0, 15, 3), (18, 1, 10, 2), (18, 2, 9, 3), (18, 2, 11, 2),
    (14, 0, 3, 1), (12, 0, 2, 2), (12, 1, 4, 3), (9, 0, 3, 3), (20, 0, 17, 3),
    (20, 0, 13, 6), (13, 0, 6, 6), (16, 0, 10, 5), (17, 1, 9, 5),  # wide rows with 32-64 KiB tiles
]


@pytest.mark.parametrize("n,p,q,s", [(18, 0, 12, 1), (18, 0, 14, 2), (18, 0, 15, 3), (18, 4, 9, 3), (12, 0, 2, 2),
                                     (18, 1, 12, 5), (18, 5, 12, 6), (20, 0, 13, 6), (16, 1, 8, 6),
                                     (18, 4, 12, 1), (16, 4, 9, 3)])  # runs of one 128-byte line
def test_fused_swap_complex64_bit_exact(gpu, n, p, q, s):
    psi = C.random_state(n, n + 3 * s).astype(np.complex64)
    st = gpu.State(n, "c64")
    st.set(psi)
    st.fused_swap(p, q, s)
    ref = psi.astype(np.complex128)
    oracle.fused_swap(ref, p, q, s)
    assert st.get().tobytes() == ref.astype(np.complex64).tobytes()
    st.close()


@pytest.mark.parametrize("n,p,q,s", FSWAP_CASES)
def test_fused_swap_bit_exact_and_involution(gpu, n, p, q, s):
    psi = _with_signed_zeros(C.random_state(n, n + p + q + s), s)
    st = gpu.State(n)
    st.set(psi)
    st.fused_swap(p, q, s)
    got = st.get()
    ref = psi.copy()
    oracle.fused_swap(ref, p, q, s)
    assert got.tobytes() == ref.tobytes()
    st.fused_swap(q, p, s)
    assert st.get().tobytes() == psi.tobytes()
    st.close()


def test_fused_swap_zero_and_rejections_leave_state_unchanged(gpu):
    n = 8
    psi = C.random_state(n, 1)
    st = gpu.State(n)
    st.set(psi)
    st.fused_swap(0, 4, 0)
    for args in [(0, 1, 2), (2, 0, 3), (0, 6, 3), (-1, 3, 1), (0, 4, -1), (5, 0, 4)]:
        with pytest.raises(gpu.QSError) as ei:
            st.fused_swap(*args)
        assert ei.value.code == gpu.binding.QS_EINVAL
    assert st.get().tobytes() == psi.tobytes()
    st.close()


# ------------------------------------------------------------------------------------------------ validation

def test_invalid_arguments_rejected_state_unchanged(gpu):
    n = 6
    psi = C.random_state(n, 2)
    st = gpu.State(n)
    st.set(psi)
    U2 = np.eye(2)
    bad = [
        lambda: st.apply_gate((6,), U2), lambda: st.apply_gate((-1,), U2), lambda: st.apply_gate((1, 1), np.eye(4)),
        lambda: st.apply_gate(tuple(range(7)), np.eye(128)), lambda: st.apply_diag((0, 0), np.ones(4)),
        lambda: st.apply_controlled((1,), (1,), U2), lambda: st.apply_controlled((), (1,), U2),
        lambda: st.apply_controlled((9,), (1,), U2),
    ]
    for f in bad:
        with pytest.raises(gpu.QSError) as ei:
            f()
        assert ei.value.code == gpu.binding.QS_EINVAL
        assert gpu.qs_last_error()
    assert st.get().tobytes() == psi.tobytes()
    st.close()


# ------------------------------------------------------------------------------------------------ probabilities

@pytest.mark.parametrize("n,dtype", [(1, "c128"), (10, "c128"), (17, "c128"), (12, "c64")])
def test_probs_and_norm(gpu, n, dtype):
    psi = C.random_state(n, 4) * 1.3
    st = gpu.State(n, dtype)
    st.set(psi)
    P, nrm = st.probs()
    Pc = P.cpu().numpy()
    start = psi.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi
    Pref, nref = oracle.probs(np.ascontiguousarray(start))
    assert np.max(np.abs(Pc - Pref) / np.maximum(Pref, 1e-300)) <= 4e-16
    assert abs(nrm - nref) <= 1e-13 * nref
    P2, nrm2 = st.probs()
    assert nrm2 == nrm and bool((P2 == P).all())  # fixed-order reduction: run-to-run identical
    st.close()


def test_probs_basis_and_uniform_closed_forms(gpu):
    n = 14
    st = gpu.State(n)
    P, nrm = st.probs()
    Pc = P.cpu().numpy()
    assert Pc[0] == 1.0 and np.count_nonzero(Pc) == 1 and nrm == 1.0
    for q in range(n):
        st.apply_gate((q,), C.h())
    P, nrm = st.probs()
    assert float((P - 2.0 ** -n).abs().max()) <= 4 * 2.0 ** -n * 2 ** -52 * n
    assert abs(nrm - 1.0) <= 1e-13
    st.close()


# ------------------------------------------------------------------------------------------------ circuits

def test_u3_cnot_all_amplitudes(gpu):
    circ = C.u3_cnot_layers()
    st = gpu.State(circ.n)
    st.run(circ.ops)
    got = st.get()
    st.close()
    ref = oracle.run(circ)
    assert _maxerr(got, ref) <= TOL128


@pytest.mark.parametrize("n", [5, 12])
def test_random_circuits_every_kind(gpu, n):
    for seed in range(3):
        circ = C.random_circuit(n, seed=90 + seed, num_ops=60, kmax=min(6, n - 1))
        got, ref = _run_both(gpu, n, circ.ops, C.random_state(n, seed))
        assert _maxerr(got, ref) <= TOL128


def test_mixed_family_at_20_qubits_all_amplitudes(gpu):
    circ = C.mixed_layers(n=20, seed=28)
    st = gpu.State(circ.n)
    st.run(circ.ops)
    got = st.get()
    st.close()
    assert _maxerr(got, oracle.run(circ)) <= TOL128


# ------------------------------------------------------------------------------------------------ complex64

def test_complex64_gates_within_fp32_error(gpu):
    n = 12
    circ = C.random_circuit(n, seed=5, num_ops=80, kmax=6, kinds=("dense", "diag", "ctrl"))
    got, ref = _run_both(gpu, n, circ.ops, C.random_state(n, 8), dtype="c64")
    infid, maxd = oracle.error_metrics(got, ref)
    assert maxd <= 2e-6 and infid <= 1e-9, (maxd, infid)


def test_complex64_moves_bit_exact(gpu):
    n = 12
    rng = _rng(12)
    ops = [C.Op("dense", (3,), mat=C.x_gate()), C.Op("ctrl", (5,), (0, 11), mat=C.x_gate()),
           C.Op("dense", (1, 2, 9), mat=_monomial(rng, 3)), C.Op("fswap", p=0, q=6, s=5),
           C.Op("fswap", p=2, q=8, s=3), C.Op("diag", (4, 6), mat=C.CZ_DIAG)]
    psi = _with_signed_zeros(C.random_state(n, 3).astype(np.complex64).astype(np.complex128), 3)
    got, ref = _run_both(gpu, n, ops, psi, dtype="c64")
    assert got.tobytes() == ref.astype(np.complex64).tobytes()


@pytest.mark.parametrize("n", [6, 7, 9, 12])
def test_complex64_one_qubit_every_target_and_diagonals(gpu, n):
    """complex64: every target of a 1-qubit gate (lane-exchange form below 4, shared-vector form at 0) and 1- and
    2-qubit diagonals (two amplitudes per 16-byte lane), against the FP64 oracle from the FP32-rounded input."""
    rng = _rng(900 + n)
    ops = [C.Op("dense", (q,), mat=_rand_u(rng, 2)) for q in range(n)]
    ops += [C.Op("diag", (q,), mat=C.rz(float(rng.uniform(0, 6.28)))) for q in range(n)]
    ops += [C.Op("diag", (0, n - 1), mat=C.CZ_DIAG), C.Op("diag", (1, 2), mat=np.exp(1j * rng.uniform(0, 6, 4)))]
    psi = C.random_state(n, 901).astype(np.complex64)
    st = gpu.State(n, "c64")
    st.set(psi)
    for op in ops:
        st.apply_op(op)
    ref = psi.astype(np.complex128)
    for op in ops:
        oracle.apply_op(ref, op)
    assert _maxerr(st.get(), ref) <= 1e-5
    st.close()
