"""Element-by-element parity with the oracle on the code paths the full-size launches take.

At 32 qubits every persistent workgroup of the block pass walks many blocks (the prefetch of the next block, the
rotated loop, the waits that leave the previous block's stores in flight), and every workgroup of the k = 5, 6 MFMA
kernel walks many column tiles (double-buffered LDS, register prefetch). At the sizes the oracle finishes in seconds
the default grids give each workgroup one block or one tile, so these tests shrink the grids instead:
  * block_wg_per_cu = 1: 256 workgroups of 256 threads; 12-qubit blocks at n = 22 / 24 give 4 / 16 blocks each;
  * mfma_wg_per_cu = 1: 256 workgroups; k = 6 at n = 20 gives 1,024 tiles (4 each), k = 5 gives 2,048 (8 each);
and run the benchmark's own plan shape (12-qubit blocks, 3 always-local low bits, beam width 16) on the benchmark's
circuit family, in complex128 (<= 1e-12 against the oracle) and complex64 (error against the FP64 oracle stated and
bounded: infidelity <= 1e-8, max |d amp| <= 1e-6).
"""
import numpy as np
import pytest

import circuits as C
import oracle
from paper_2203_16044_amd import binding as B
from paper_2203_16044_amd.plan import Circuit, Plan

pytestmark = pytest.mark.gpu

TOL128 = 1e-12


@pytest.fixture
def tunables():
    """Set tunables for one test and restore the library defaults afterwards."""
    defaults = {"block_wg_per_cu": 32, "mfma_wg_per_cu": 2, "block_async": 0, "plan_beam": 16, "mfma_stage_ops": 3,
                "block_lanes": 0, "stage_pack": 1, "plan_beam_search": 0}
    touched = []

    def set_(name, value):
        touched.append(name)
        B.qs_set_tunable(name, value)

    yield set_
    for name in touched:
        B.qs_set_tunable(name, defaults[name])


def _plan_run(gpu, circ, bits, low, psi0, dtype):
    st = gpu.State(circ.n, dtype)
    st.set(psi0)
    c = Circuit.from_ops(circ.n, circ.ops)
    p = Plan(c, "block", bits, low, dtype) if bits >= 7 else Plan(c, "fuse", bits, 0, dtype)
    p.run(st)
    got = st.get()
    info = p.info()
    for h in (p, c, st):
        h.close()
    return got, info


def _check(got, ref, dtype):
    if dtype == "c128":
        err = float(np.max(np.abs(got - ref)))
        assert err <= TOL128, err
    else:
        infid, maxd = oracle.error_metrics(got, ref)
        assert infid <= 1e-8 and maxd <= 1e-6, (infid, maxd)


@pytest.mark.parametrize("n,layers", [(22, 10), (24, 5)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("low", [3, 4])
def test_block_pass_many_blocks_per_workgroup(gpu, tunables, n, layers, dtype, low):
    """The benchmark's block plan (12-qubit blocks, beam 16) with 256 persistent workgroups: every workgroup runs
    the prefetch / rotated-loop path over 4 (n = 22) or 16 (n = 24) blocks per pass."""
    tunables("block_wg_per_cu", 1)
    circ = C.su4_u3_random(n=n, seed=900 + n, layers=layers)
    psi0 = C.random_state(n, 901 + n)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    got, info = _plan_run(gpu, circ, 12, low, psi0, dtype)
    assert info["block"] >= 2 and (1 << (n - 12)) >= 4 * 256
    _check(np.asarray(got, np.complex128), oracle.run(circ, psi0), dtype)


@pytest.mark.parametrize("beam", [24, 64])
@pytest.mark.parametrize("low", [3, 4])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_plans_at_other_beam_widths(gpu, tunables, beam, low, dtype):
    """Block plans whose passes are formed at the other beam widths the learned planner prices (the benchmark runs
    12/3 at width 24), with 256 persistent workgroups so each walks 4 blocks per pass, element by element against
    the oracle."""
    from paper_2203_16044_amd import costmodel as CM
    tunables("block_wg_per_cu", 1)
    n = 22
    circ = C.su4_u3_random(n=n, seed=940 + low, layers=10)
    psi0 = C.random_state(n, 941 + low)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    st = gpu.State(n, dtype)
    st.set(psi0)
    c = Circuit.from_ops(n, circ.ops)
    p = CM.make_plan(c, ("block", 12, low, beam), dtype)
    assert B.qs_get_tunable("plan_beam") == 16  # restored after the plan was formed
    assert p.info()["block"] >= 2
    p.run(st)
    got = np.asarray(st.get(), np.complex128)
    for h in (p, c, st):
        h.close()
    _check(got, oracle.run(circ, psi0), dtype)


@pytest.mark.parametrize("low", [3, 4])
def test_thirteen_qubit_blocks_many_per_workgroup(gpu, tunables, low):
    """complex128 13-qubit blocks run one 16-amplitude register group per thread (512 threads, a CU per 128 KB
    block); with 256 persistent workgroups each walks 8 blocks per pass at n = 24."""
    tunables("block_wg_per_cu", 1)
    n = 24
    circ = C.su4_u3_random(n=n, seed=930 + low, layers=5)
    psi0 = C.random_state(n, 931 + low)
    got, info = _plan_run(gpu, circ, 13, low, psi0, "c128")
    assert info["block"] >= 2 and (1 << (n - 13)) >= 8 * 256
    _check(np.asarray(got, np.complex128), oracle.run(circ, psi0), "c128")


@pytest.mark.parametrize("n,layers,wg", [(14, 8, 32), (22, 6, 1), (24, 4, 32)])
def test_lane_pair_block_pass(gpu, tunables, n, layers, wg):
    """complex128 12-qubit block passes in lane-pair form (block_lanes 1: 512 threads, each 16-amplitude register
    group held by lanes l and l + 32, the lane bit exchanged with a register bit by v_permlane32_swap before an op on
    the lane's position) against the oracle, with 4 and 3 always-local low qubits; n = 22 with 128 workgroups walks
    8 blocks per workgroup."""
    tunables("block_lanes", 1)
    tunables("block_wg_per_cu", wg)
    circ = C.su4_u3_random(n=n, seed=970 + n, layers=layers)
    psi0 = C.random_state(n, 971 + n)
    ref = oracle.run(circ, psi0)
    for low in (4, 3):
        got, info = _plan_run(gpu, circ, 12, low, psi0, "c128")
        assert info["block"] >= 1
        _check(got, ref, "c128")


def test_lane_pair_form_with_three_position_ops(gpu, tunables):
    """With block_lanes 1, a plan whose passes mix 1-, 2- and 3-position ops: passes holding a 3-position op keep the
    one-lane kernel, the others run in lane-pair form, one after the other on the same state."""
    tunables("block_lanes", 1)
    n = 20
    circ = C.mixed_layers(n=n, seed=980, layers=6, toffolis=12, swap_s=4)
    extra = C.random_circuit(n, seed=981, num_ops=60, kmax=3, kinds=("dense", "diag", "ctrl"))
    circ = C.Circuit(n, list(circ.ops) + list(extra.ops), name="mixed+random3")
    psi0 = C.random_state(n, 982)
    got, info = _plan_run(gpu, circ, 12, 4, psi0, "c128")
    _check(got, oracle.run(circ, psi0), "c128")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,bits,low", [(16, 10, 0), (20, 12, 0), (22, 12, 3)])
def test_remap_plan(gpu, dtype, n, bits, low):
    """QS_PLAN_REMAP on the GPU: block passes over the lowest physical qubits, inserted fused-swaps, circuit
    fused-swaps absorbed as relabels, the identity map restored; against the oracle element by element."""
    circ = C.mixed_layers(n=n, seed=990 + n, layers=8, toffolis=8, swap_s=4)
    extra = C.su4_u3_random(n=n, seed=991 + n, layers=3)
    circ = C.Circuit(n, list(circ.ops) + list(extra.ops), name="mixed+su4")
    psi0 = C.random_state(n, 992 + n)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    st = gpu.State(n, dtype)
    st.set(psi0)
    c = Circuit.from_ops(n, circ.ops)
    p = Plan(c, "remap", bits, low, dtype)
    types = {x["type"] for x in p.passes()}
    assert 2 in types and 4 in types
    p.run(st)
    got = st.get()
    for h in (p, c, st):
        h.close()
    _check(np.asarray(got, np.complex128), oracle.run(circ, psi0), dtype)


def test_block_passes_with_three_position_ops(gpu):
    """A circuit with Toffolis, random 3-qubit gates and fused-swaps at 20 qubits: block passes whose stages hold
    3-position ops (8 x 8 matrices) beside 1- and 2-position ones, and fused-swap passes, in one plan."""
    n = 20
    circ = C.mixed_layers(n=n, seed=960, layers=6, toffolis=12, swap_s=4)
    extra = C.random_circuit(n, seed=961, num_ops=40, kmax=3, kinds=("dense", "diag", "ctrl"))
    circ = C.Circuit(n, list(circ.ops) + list(extra.ops), name="mixed+random3")
    psi0 = C.random_state(n, 962)
    got, info = _plan_run(gpu, circ, 12, 3, psi0, "c128")
    assert info["block"] >= 2
    _check(got, oracle.run(circ, psi0), "c128")


@pytest.mark.parametrize("n", [22, 24])
def test_double_buffered_block_pass_many_blocks_per_workgroup(gpu, tunables, n):
    """The direct-to-LDS double-buffered variant (complex128, 12-qubit blocks) with 256 workgroups: its explicit
    vmcnt waits for a block that follows a block (loads of the next block and stores of the previous in flight)."""
    tunables("block_wg_per_cu", 1)
    tunables("block_async", 1)
    circ = C.su4_u3_random(n=n, seed=910 + n, layers=4)
    psi0 = C.random_state(n, 911 + n)
    got, _ = _plan_run(gpu, circ, 12, 3, psi0, "c128")
    _check(got, oracle.run(circ, psi0), "c128")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("k", [5, 6])
@pytest.mark.parametrize("wg", [1, 2])
def test_mfma_dense_many_tiles_per_workgroup(gpu, tunables, dtype, k, wg):
    """k = 5, 6 dense gates at n = 20 with 256 / 512 MFMA workgroups (4-8 / 2-4 column tiles each), on targets that
    include the lowest and the highest qubits."""
    tunables("mfma_wg_per_cu", wg)
    n = 20
    rng = np.random.Generator(np.random.PCG64(930 + k))
    psi0 = C.random_state(n, 931 + k)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    target_sets = [list(range(k)), list(range(n - k, n)), [int(t) for t in rng.choice(n, size=k, replace=False)]]
    st = gpu.State(n, dtype)
    st.set(psi0)
    ref = psi0.copy()
    for t in target_sets:
        U = C._random_unitary(rng, 1 << k)
        st.apply_gate(t, U)
        oracle.apply_dense(ref, t, U)
    got = np.asarray(st.get(), np.complex128)
    st.close()
    if dtype == "c128":
        assert float(np.max(np.abs(got - ref))) <= TOL128
    else:
        infid, maxd = oracle.error_metrics(got, ref)
        assert infid <= 1e-10 and maxd <= 1e-6, (infid, maxd)


@pytest.mark.parametrize("k", [5, 6])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fused_dense_plan_many_tiles_per_workgroup(gpu, tunables, k, dtype):
    """The fused-dense plans the benchmark also times (k <= 5, 6 on MFMA) with 256 MFMA workgroups at n = 20."""
    tunables("mfma_wg_per_cu", 1)
    circ = C.su4_u3_random(n=20, seed=940 + k, layers=6)
    psi0 = C.random_state(20, 941 + k)
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    got, info = _plan_run(gpu, circ, k, 0, psi0, dtype)
    assert info["dense"] >= 1
    _check(np.asarray(got, np.complex128), oracle.run(circ, psi0), dtype)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_block_pass_renormalised_segments_many_blocks(gpu, tunables, dtype):
    """The complex64 leg's form (plans in segments with FP64 renormalisation between them) on many blocks per
    workgroup, against the oracle's renormalised run (oracle.scale by 1/sqrt(norm) after each segment)."""
    from paper_2203_16044_amd.plan import SegmentedPlan
    tunables("block_wg_per_cu", 1)
    circ = C.su4_u3_renorm(n=22, seed=950, layers=6)
    circ.renorm_after = (2, 4)
    psi0 = C.random_state(22, 951) * 1.25  # unnormalised start: the first renormalisation changes the state
    if dtype == "c64":
        psi0 = psi0.astype(np.complex64).astype(np.complex128)
    st = gpu.State(22, dtype)
    st.set(psi0)
    sp = SegmentedPlan(22, circ.ops, circ.renorm_after, "block", 12, 3, dtype)
    sp.run(st)
    got = np.asarray(st.get(), np.complex128)
    sp.close()
    st.close()
    ref = psi0.copy()
    for L in range(1, 7):
        for op in circ.ops:
            if op.layer == L:
                oracle.apply_op(ref, op)
        if L in circ.renorm_after:
            _, nrm = oracle.probs(ref)
            oracle.scale(ref, 1.0 / np.sqrt(nrm))
    _check(got, ref, dtype)
