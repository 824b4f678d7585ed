"""Measurement, reset and sampling on the GPU against the oracle (same uniforms on both sides)."""
import numpy as np
import pytest

import circuits as C
from oracle import measure as M
from paper_2203_16044_amd import binding as B

pytestmark = pytest.mark.gpu


def _uniforms(seed, k):
    return np.random.Generator(np.random.PCG64(seed)).uniform(size=k)


@pytest.mark.parametrize("dtype,tol,ptol", [("c128", 1e-12, 1e-12), ("c64", 2e-6, 1e-6)])
def test_measure_matches_oracle(gpu, dtype, tol, ptol):
    n = 14
    psi = C.random_state(n, 21)
    # the complex64 state holds the input rounded to FP32: the oracle starts from the same values
    ref = psi.astype(np.complex64).astype(np.complex128) if dtype == "c64" else psi.copy()
    st = gpu.State(n, dtype)
    st.set(psi)
    for q, u in zip((0, 5, 13, 2, 9), _uniforms(22, 5)):
        _, p1_ref, _ = M.measure(ref, q, 0.5)
        assert abs(u - p1_ref) > 1e-6  # the decision is not at a rounding boundary
        out, p1 = st.measure(q, float(u))
        out_ref, p1_ref, ref = M.measure(ref, q, float(u))
        assert out == out_ref and abs(p1 - p1_ref) <= ptol
        assert np.max(np.abs(st.get() - ref)) <= tol
    st.close()


def test_measuring_every_qubit_gives_a_basis_state(gpu):
    n = 12
    st = gpu.State(n, "c128")
    psi = C.random_state(n, 23)
    st.set(psi)
    ref = psi
    outs = []
    for q, u in enumerate(_uniforms(24, n)):
        o, _ = st.measure(q, float(u))
        o_ref, _, ref = M.measure(ref, q, float(u))
        assert o == o_ref
        outs.append(o)
    k = sum(o << q for q, o in enumerate(outs))
    got = st.get()
    assert abs(abs(got[k]) - 1.0) <= 1e-12 and np.count_nonzero(np.abs(got) > 0) == 1
    st.close()


def test_reset(gpu):
    n = 10
    st = gpu.State(n, "c128")
    psi = C.random_state(n, 25)
    st.set(psi)
    ref = psi
    for q, u in zip((0, 4, 9), _uniforms(26, 3)):
        o = st.reset(q, float(u))
        o_ref, ref = M.reset(ref, q, float(u))
        assert o == o_ref
        assert np.max(np.abs(st.get() - ref)) <= 1e-12
        assert M.masses(st.get(), q)[1] == 0.0
    st.close()


@pytest.mark.parametrize("n", [1, 5, 6, 12, 13, 17, 24])
def test_samples_are_the_inverse_cdf(gpu, n):
    """n = 1..6: a single chunk smaller than a wave's 64 x 64; 12: exactly one chunk; 24: 4096 chunks, two scan
    tiles."""
    psi = C.random_state(n, 30 + n)
    st = gpu.State(n, "c128")
    st.set(psi)
    u = _uniforms(40 + n, 2000)
    idx = st.sample(u)
    assert idx.dtype == np.int64 and idx.min() >= 0 and idx.max() < (1 << n)
    valid = M.samples_valid(psi, u, idx)
    ref = M.samples(psi, u)
    bad = np.nonzero(~valid)[0]
    assert bad.size == 0, [(float(u[k]), int(idx[k]), int(ref[k])) for k in bad[:5]]
    # away from boundaries the index is unique: the oracle's
    assert int(np.sum(idx == ref)) >= len(u) - 2
    # sampling leaves the state unchanged
    assert np.array_equal(st.get(), psi)
    st.close()


def test_sampling_statistics(gpu):
    n = 5
    psi = C.random_state(n, 50)
    st = gpu.State(n, "c64")
    st.set(psi)
    u = _uniforms(51, 200000)
    counts = np.bincount(st.sample(u), minlength=1 << n)
    p = np.abs(psi) ** 2
    expect = p / p.sum() * len(u)
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 90.0, chi2  # 31 degrees of freedom; p < 1e-6 above this
    st.close()


def test_full_size_basis_state_sampling_and_measure(gpu):
    """32 qubits: X on the bits of k prepares |k>; every sample is k, and measuring a qubit of H|0> gives 1/2."""
    n = 32
    k = 0x9AC35A17
    st = gpu.State(n, "c128")
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    for q in range(n):
        if (k >> q) & 1:
            st.apply_gate([q], X)
    assert set(st.sample(_uniforms(60, 64)).tolist()) == {k}
    Hm = np.array([[1, 1], [1, -1]], dtype=np.complex128) / np.sqrt(2)
    st.apply_gate([7], Hm)
    out, p1 = st.measure(7, 0.25)
    assert abs(p1 - 0.5) <= 1e-12 and out == 1
    assert abs(st.norm() - 1.0) <= 1e-12
    assert set(st.sample(_uniforms(61, 16)).tolist()) == {k | (1 << 7)}
    st.close()


def test_invalid_arguments(gpu):
    st = gpu.State(6, "c128")
    with pytest.raises(B.QSError):
        st.measure(6, 0.5)
    with pytest.raises(B.QSError):
        st.measure(0, 1.0)
    with pytest.raises(B.QSError):
        st.sample([0.2, -0.1])
    st.set(np.zeros(64, dtype=np.complex128))
    with pytest.raises(B.QSError):
        st.measure(0, 0.5)
    with pytest.raises(B.QSError):
        st.sample([0.5])
    assert st.sample([]).size == 0
    st.close()
