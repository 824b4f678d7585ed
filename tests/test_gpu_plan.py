"""GPU parity of planned execution (LDS block passes, fused dense blocks) against the CPU oracle.

A plan reorders nothing that matters: every gate is applied after the earlier gates on its qubits, so the final
state equals the unfused oracle's up to rounding (complex128: max |d amp| <= 1e-12).
"""
import numpy as np
import pytest

import circuits as C
import oracle
from paper_2203_16044_amd.plan import Circuit, Plan

pytestmark = pytest.mark.gpu

TOL128 = 1e-12
PLANS = [("block", 8, 0), ("block", 8, 3), ("block", 10, 4), ("block", 11, 3), ("block", 12, 3), ("block", 12, 4),
         ("block", 13, 3),
         ("fuse", 2, 0), ("fuse", 3, 0), ("fuse", 4, 0), ("fuse", 5, 0), ("fuse", 6, 0)]


def _run_plan(gpu, circ, mode, bits, low, psi0=None, dtype="c128"):
    st = gpu.State(circ.n, dtype)
    if psi0 is not None:
        st.set(psi0)
    c = Circuit.from_ops(circ.n, circ.ops)
    p = Plan(c, mode, bits, low, dtype)
    p.run(st)
    got = st.get()
    info = p.info()
    p.close()
    c.close()
    st.close()
    return got, info


def _maxerr(a, b):
    return float(np.max(np.abs(np.asarray(a, np.complex128) - np.asarray(b, np.complex128))))


@pytest.mark.parametrize("mode,bits,low", PLANS)
@pytest.mark.parametrize("n", [9, 14])
def test_plan_random_circuits_every_kind(gpu, mode, bits, low, n):
    circ = C.random_circuit(n, seed=400 + n, num_ops=120, kmax=4)
    psi0 = C.random_state(n, n)
    got, _ = _run_plan(gpu, circ, mode, bits, low, psi0)
    assert _maxerr(got, oracle.run(circ, psi0)) <= TOL128


@pytest.mark.parametrize("mode,bits,low", [("block", 12, 4), ("block", 10, 3), ("fuse", 4, 0), ("fuse", 6, 0)])
def test_plan_u3_cnot_all_amplitudes(gpu, mode, bits, low):
    circ = C.u3_cnot_layers()
    got, _ = _run_plan(gpu, circ, mode, bits, low)
    assert _maxerr(got, oracle.run(circ)) <= TOL128


@pytest.mark.parametrize("mode,bits,low", [("block", 12, 3), ("block", 12, 4), ("block", 13, 3), ("fuse", 5, 0),
                                           ("fuse", 6, 0)])
def test_plan_su4_u3_family_18_qubits(gpu, mode, bits, low):
    circ = C.su4_u3_random(n=18, seed=32, layers=14)
    got, info = _run_plan(gpu, circ, mode, bits, low)
    assert info["passes"] < len(circ.ops) // 4
    assert _maxerr(got, oracle.run(circ)) <= TOL128


def test_plan_mixed_family_18_qubits(gpu):
    circ = C.mixed_layers(n=18, seed=28)
    got, info = _run_plan(gpu, circ, "block", 12, 4)
    assert info["other"] == 3  # the circuit's fused-swaps
    assert _maxerr(got, oracle.run(circ)) <= TOL128


def test_plan_small_state_fallback(gpu):
    circ = C.random_circuit(6, seed=8, num_ops=50, kmax=3)
    psi0 = C.random_state(6, 1)
    got, info = _run_plan(gpu, circ, "block", 12, 4, psi0)
    assert info["block"] == 0
    assert _maxerr(got, oracle.run(circ, psi0)) <= TOL128


def test_plan_complex64_error_against_fp64_oracle(gpu):
    circ = C.su4_u3_renorm(n=18, seed=33, layers=12)
    got, _ = _run_plan(gpu, circ, "block", 12, 4, dtype="c64")
    infid, maxd = oracle.error_metrics(got, oracle.run(circ))
    assert infid <= 1e-8 and maxd <= 1e-5, (infid, maxd)


def test_plan_rejects_mismatched_state(gpu):
    circ = C.u3_cnot_layers(n=12)
    c = Circuit.from_ops(12, circ.ops)
    p = Plan(c, "block", 10, 3, "c128")
    st = gpu.State(13)
    with pytest.raises(gpu.QSError):
        p.run(st)
    st.close()
    st = gpu.State(12, "c64")
    with pytest.raises(gpu.QSError):
        p.run(st)
    st.close()


@pytest.fixture
def stage_width_3():
    from paper_2203_16044_amd import binding as B
    B.qs_set_tunable("block_stage_width", 3)
    yield
    B.qs_set_tunable("block_stage_width", 4)


@pytest.mark.parametrize("bits,low", [(12, 4), (12, 3), (13, 3), (11, 3)])
@pytest.mark.parametrize("dtype,tol", [("c128", TOL128), ("c64", 2e-5)])
def test_plan_three_position_stages(gpu, stage_width_3, bits, low, dtype, tol):
    """3-position register stages (512-thread kernel for 12- and 13-qubit blocks; other sizes keep 4 positions)."""
    for circ in (C.random_circuit(15, seed=431, num_ops=150, kmax=3), C.su4_u3_random(n=17, seed=33, layers=8)):
        psi0 = C.random_state(circ.n, 7)
        got, _ = _run_plan(gpu, circ, "block", bits, low, psi0, dtype)
        assert _maxerr(got, oracle.run(circ, psi0)) <= tol, circ.name


@pytest.fixture
def block_async():
    from paper_2203_16044_amd import binding as B
    B.qs_set_tunable("block_async", 1)
    yield
    B.qs_set_tunable("block_async", 0)


@pytest.mark.parametrize("low", [4, 3])
@pytest.mark.parametrize("dtype,tol", [("c128", TOL128), ("c64", 2e-5)])
def test_plan_double_buffered_block_pass(gpu, block_async, low, dtype, tol):
    """12-qubit block passes with double-buffered LDS filled by direct-to-LDS loads (complex128; complex64 keeps the
    register-prefetch kernel under the same setting): same results as the oracle at 15 and 20 qubits. With the default
    grid (32 workgroups per CU, capped at the block count) every workgroup here runs exactly one block; the path of a
    workgroup that walks several blocks is checked with a 256-workgroup grid in test_gpu_fullpath.py."""
    for circ in (C.random_circuit(15, seed=441, num_ops=150, kmax=3), C.su4_u3_random(n=20, seed=34, layers=12)):
        psi0 = C.random_state(circ.n, 8)
        got, _ = _run_plan(gpu, circ, "block", 12, low, psi0, dtype)
        assert _maxerr(got, oracle.run(circ, psi0)) <= tol, circ.name


@pytest.mark.parametrize("dtype,tol", [("c128", TOL128), ("c64", 2e-5)])
@pytest.mark.parametrize("bits,low", [(10, 4), (11, 3), (12, 3), (12, 4), (13, 4)])
def test_plan_long_runs_of_ops_on_four_qubits(gpu, bits, low, dtype, tol):
    """40 two-qubit gates that cycle through the pairs of qubits 0-3 (no gate's qubits are a subset of its
    neighbour's, so none merge) all fall into stages over the same 4 local positions; a stage record holds at most
    8 ops, so the planner splits the run into several stages over those positions. In complex64 the first four of
    those stages run as fused 16 x 16 products on the matrix cores and the rest op by op, in the same pass."""
    rng = np.random.Generator(np.random.PCG64(71))
    pairs = [(0, 1), (1, 2), (2, 3), (0, 3), (0, 2), (1, 3)]
    ops = [C.Op("dense", pairs[i % len(pairs)], mat=C.haar_su4(rng)) for i in range(40)]
    ops += [C.Op("dense", (5, 9), mat=C.haar_su4(rng)), C.Op("dense", (0, 11), mat=C.haar_su4(rng))]
    circ = C.Circuit(14, ops=ops, name="four_qubit_run")
    psi0 = C.random_state(14, 77)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)  # the oracle starts from the rounded state
    got, info = _run_plan(gpu, circ, "block", bits, low, psi0, dtype)
    assert info["fused_ops"] >= 40
    assert _maxerr(got, oracle.run(circ, psi0)) <= tol


@pytest.mark.parametrize("ops_min", [0, 2, 3])
def test_plan_complex64_mfma_stages_match_op_by_op(gpu, ops_min):
    """The fused MFMA form of complex64 stages (tunable mfma_stage_ops; 0 turns it off) against the oracle on the
    random SU(4)+U3 family, whose 12-qubit passes have stages of 1-8 ops."""
    import paper_2203_16044_amd.binding as B
    circ = C.su4_u3_random(n=18, seed=318, layers=8)
    psi0 = C.random_state(18, 319).astype(np.complex64).astype(np.complex128)
    B.qs_set_tunable("mfma_stage_ops", ops_min)
    try:
        got, _ = _run_plan(gpu, circ, "block", 12, 4, psi0, "c64")
    finally:
        B.qs_set_tunable("mfma_stage_ops", 3)
    assert _maxerr(got, oracle.run(circ, psi0)) <= 2e-5


@pytest.mark.parametrize("dtype,tol", [("c128", TOL128), ("c64", 2e-5)])
def test_plan_runs_on_three_qubits_pad_the_stage(gpu, dtype, tol):
    """Gates cycling over the pairs of qubits 0-2 only: their stages hold 3 positions and are padded with an unused
    one (in complex64 the fused stage matrix acts as the identity on it)."""
    rng = np.random.Generator(np.random.PCG64(73))
    pairs = [(0, 1), (1, 2), (0, 2)]
    ops = [C.Op("dense", pairs[i % len(pairs)], mat=C.haar_su4(rng)) for i in range(24)]
    ops += [C.Op("dense", (4, 10), mat=C.haar_su4(rng))]
    circ = C.Circuit(13, ops=ops, name="three_qubit_run")
    psi0 = C.random_state(13, 78)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    got, _ = _run_plan(gpu, circ, "block", 12, 3, psi0, dtype)
    assert _maxerr(got, oracle.run(circ, psi0)) <= tol


@pytest.mark.parametrize("mode,bits,low", [("block", 12, 4), ("fuse", 4, 0)])
def test_plan_of_an_empty_circuit_leaves_the_state_unchanged(gpu, mode, bits, low):
    psi0 = C.random_state(14, 92)
    got, info = _run_plan(gpu, C.Circuit(14, name="empty"), mode, bits, low, psi0)
    assert info["passes"] == 0
    assert np.asarray(got, np.complex128).tobytes() == psi0.astype(np.complex128).tobytes()
