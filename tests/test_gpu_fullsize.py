"""Full-size checks (28 / 32 qubits) in the launch configurations the benchmark times.

The oracle cannot follow a 32-qubit circuit in seconds, so these check what holds at any size: closed forms
(H on every qubit gives 2^(-n/2) everywhere; a layer of 1-qubit gates on |0..0> gives a product state whose
amplitudes are products of matrix entries), sampled amplitudes against those closed forms, exact moves under
the fused-swap (psi'[sigma(i)] = psi[i]), the norm, and echo (C then its inverse returns |0..0>).
"""
import math

import numpy as np
import pytest
import torch

import circuits as C
from paper_2203_16044_amd.plan import Circuit, Plan

pytestmark = pytest.mark.gpu

N = 32


def _samples(n, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    idx = rng.integers(0, 1 << n, size=count, dtype=np.int64)
    return np.unique(np.concatenate([idx, [0, (1 << n) - 1, 1, 1 << (n - 1)]]))


CHUNK = 1 << 26


def _max_abs_dev(buf, value):
    """max_i |buf_i - value| over the whole state, in chunks (no full-size temporaries)."""
    m = 0.0
    for i in range(0, buf.numel(), CHUNK):
        m = max(m, float((buf[i:i + CHUNK] - value).abs().max()))
    return m


def _nonzero(buf):
    out = []
    for i in range(0, buf.numel(), CHUNK):
        nz = torch.nonzero(buf[i:i + CHUNK] != 0).flatten()
        out += (nz + i).cpu().tolist()
    return np.array(out, dtype=np.int64)


def _amps(st, idx):
    t = torch.as_tensor(idx, device=st.buf.device)
    return st.buf[t].cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module")
def big_state(gpu):
    torch.cuda.empty_cache()
    st = gpu.State(N, "c128")
    yield st
    st.close()
    del st
    torch.cuda.empty_cache()


def _product_reference(us, idx):
    ref = np.ones(len(idx), dtype=np.complex128)
    for q, u in enumerate(us):
        ref *= np.where((idx >> q) & 1, u[1, 0], u[0, 0])
    return ref


@pytest.mark.parametrize("how", ["plain", "block"])
def test_product_state_sampled_amplitudes(gpu, big_state, how):
    rng = np.random.Generator(np.random.PCG64(77))
    us = [C.u3(*rng.uniform(0, 2 * math.pi, 3)) for _ in range(N)]
    circ = C.Circuit(N, [C.Op("dense", (q,), mat=us[q]) for q in range(N)])
    st = big_state
    st.init_zero()
    if how == "plain":
        st.run(circ.ops)
    else:
        c = Circuit.from_ops(N, circ.ops)
        p = Plan(c, "block", 12, 4)
        p.run(st)
        p.close()
    idx = _samples(N, 4096, 1)
    assert np.max(np.abs(_amps(st, idx) - _product_reference(us, idx))) <= 1e-12
    assert abs(st.norm() - 1.0) <= 1e-12
    # fused-swap at full size: a pure move, psi'[sigma(i)] = psi[i] bit for bit
    before = _amps(st, idx)
    st.fused_swap(0, 26, 6)
    d = ((idx >> 0) ^ (idx >> 26)) & 63
    sig = idx ^ d ^ (d << 26)
    assert _amps(st, sig).tobytes() == before.tobytes()


def _product_pair_circuit(n, seed, layers):
    """The benchmark circuit's structure (per layer a random qubit pairing with a dense 2-qubit gate on every pair, then
    U3 on every qubit) with every 2-qubit gate a Kronecker product V (x) W of random U3s: the plans see the same dense
    4 x 4 matrices on the same qubit pairs, yet the state stays a product state, so every amplitude is known in closed
    form (the product over qubits of column 0 of that qubit's accumulated 2 x 2 factor) and is not invariant under
    any exchange of blocks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fac = [np.eye(2, dtype=np.complex128) for _ in range(n)]
    ops = []
    for L in range(1, layers + 1):
        perm = rng.permutation(n)
        for j in range(n // 2):
            a, b = int(perm[2 * j]), int(perm[2 * j + 1])
            W, V = (C.u3(*rng.uniform(0, 2 * math.pi, 3)) for _ in range(2))
            ops.append(C.Op("dense", (a, b), mat=np.kron(V, W), layer=L))  # matrix bit 0 <-> a (W), bit 1 <-> b (V)
            fac[a], fac[b] = W @ fac[a], V @ fac[b]
        for q in range(n):
            U = C.u3(*rng.uniform(0, 2 * math.pi, 3))
            ops.append(C.Op("dense", (q,), mat=U, layer=L))
            fac[q] = U @ fac[q]
    return C.Circuit(n, ops=ops, name="product_pairs"), fac


def _learned_shape():
    """What the benchmark runs: the learned cost model's choice for its 32-qubit circuit, a (mode, bits, low) shape or
    costmodel.LEARNED (every pass chosen by the model); greedy 12/4 without weights."""
    import os
    from paper_2203_16044_amd import costmodel as CM
    if not os.path.exists(CM.WEIGHTS):
        return ("block", 12, 4)
    circ = C.su4_u3_random(n=N, seed=32, layers=40)
    cc = Circuit.from_ops(N, circ.ops)
    model = CM.CostModel.load()
    lp, learned, _ = CM.choose_plan(cc, "c128", model)
    lp.close()
    model.close()
    cc.close()
    return learned or ("block", 12, 4)


def _plan_for(c, shape):
    """A plan of circuit c in the given shape; costmodel.LEARNED: the model chooses every pass of c."""
    from paper_2203_16044_amd import costmodel as CM
    if shape == CM.LEARNED:
        model = CM.CostModel.load()
        p = CM.learned_plan(c, "c128", model)
        model.close()
        return p
    return CM.make_plan(c, shape)


@pytest.mark.parametrize("shape", [("block", 12, 3), ("block", 12, 4), ("block", 13, 3), "learned"])
def test_benchmark_structured_product_circuit_sampled_amplitudes(gpu, big_state, shape):
    """40 layers of the benchmark's pairing structure at 32 qubits through the benchmark's plan shapes (the persistent
    block pipeline walks 32 blocks per workgroup per pass): 4,096 sampled amplitudes against the closed form."""
    shape = _learned_shape() if shape == "learned" else shape
    circ, fac = _product_pair_circuit(N, 3200, 40)
    st = big_state
    st.init_zero()
    c = Circuit.from_ops(N, circ.ops)
    p = _plan_for(c, shape)
    assert p.info()["passes"] >= 20
    p.run(st)
    p.close()
    c.close()
    idx = _samples(N, 4096, 5)
    ref = np.ones(len(idx), dtype=np.complex128)
    for q in range(N):
        ref *= np.where((idx >> q) & 1, fac[q][1, 0], fac[q][0, 0])
    assert np.max(np.abs(_amps(st, idx) - ref)) <= 1e-12
    assert abs(st.norm() - 1.0) <= 1e-12


def test_hadamard_x11_uniform_at_32_qubits(gpu, big_state):
    """Sec. IV-D's benchmark circuit (11 H per qubit) through the block plan: H^11 = H, so all 2^32 amplitudes
    equal 2^-16."""
    circ = C.hadamard_x11(N)
    st = big_state
    st.init_zero()
    c = Circuit.from_ops(N, circ.ops)
    p = Plan(c, "block", 12, 4)
    p.run(st)
    p.close()
    assert _max_abs_dev(st.buf, 2.0 ** -16) <= 1e-15
    assert abs(st.norm() - 1.0) <= 1e-12


def test_ghz_at_32_qubits(gpu, big_state):
    st = big_state
    st.init_zero()
    st.run(C.ghz(N).ops)
    nz = _nonzero(st.buf)
    assert nz.tolist() == [0, (1 << N) - 1]
    assert np.max(np.abs(_amps(st, nz) - 1 / math.sqrt(2))) <= 1e-15


@pytest.mark.parametrize("shape", [("block", 12, 4), "learned"])
def test_random_circuit_norm_and_echo_block_plan(gpu, big_state, shape):
    """The benchmark's 32-qubit random circuit (40 layers) through the greedy block plan and through the plan the
    benchmark runs preserves the norm, and running its inverse afterwards returns to |0..0>."""
    shape = _learned_shape() if shape == "learned" else shape
    circ = C.su4_u3_random(n=N, seed=32, layers=40)
    st = big_state
    st.init_zero()
    c = Circuit.from_ops(N, circ.ops)
    p = _plan_for(c, shape)
    p.run(st)
    assert abs(st.norm() - 1.0) <= 1e-12
    inv = C.inverse_circuit(circ)
    ci = Circuit.from_ops(N, inv.ops)
    pi = _plan_for(ci, shape)
    pi.run(st)
    a0 = _amps(st, np.array([0]))[0]
    assert abs(a0 - 1.0) <= 1e-12
    idx = _samples(N, 4096, 2)[1:]
    assert np.max(np.abs(_amps(st, idx))) <= 1e-12
    for x in (p, pi, c, ci):
        x.close()


def test_mixed_28_qubits_unfused_norm_and_echo(gpu):
    circ = C.mixed_layers()
    st = gpu.State(28, "c128")
    st.run(circ.ops)
    assert abs(st.norm() - 1.0) <= 1e-12
    st.run(C.inverse_circuit(circ).ops)
    assert abs(_amps(st, np.array([0]))[0] - 1.0) <= 1e-12
    st.close()
