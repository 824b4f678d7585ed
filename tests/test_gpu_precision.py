"""complex64 engine: FP32 state and FP32 MFMA / VALU arithmetic, FP64 reductions and renormalisation every 10
layers; its error against the FP64 oracle is measured (and bounded) on the 24-qubit run of the 33-qubit family."""

import numpy as np
import pytest

import circuits as C
import oracle
from paper_2203_16044_amd.plan import Circuit, Plan, SegmentedPlan

pytestmark = pytest.mark.gpu


def test_error_run_24_qubits_against_fp64_oracle(gpu):
    circ = C.su4_u3_error_run()
    assert circ.n == 24 and circ.renorm_after == (10, 20, 30, 40)
    ref = oracle.run(circ)
    st = gpu.State(24, "c64")
    sp = SegmentedPlan(24, circ.ops, circ.renorm_after, "block", 12, 4, "c64")
    sp.run(st)
    got = st.get()
    infid, maxd = oracle.error_metrics(got, ref)
    print(f"complex64, 24 qubits, 40 layers: infidelity {infid:.3e}, max |d amp| {maxd:.3e}")
    assert infid <= 1e-8 and maxd <= 1e-6, (infid, maxd)
    assert abs(st.norm() - 1.0) <= 1e-6
    sp.close()
    st.close()
    # the same circuit in complex128 through the same plan shape matches the oracle to 1e-12
    st = gpu.State(24, "c128")
    c = Circuit.from_ops(24, circ.ops)
    p = Plan(c, "block", 12, 4, "c128")
    p.run(st)
    assert float(np.max(np.abs(st.get() - ref))) <= 1e-12
    p.close()
    c.close()
    st.close()


def test_renormalisation_restores_the_norm(gpu):
    n = 20
    st = gpu.State(n, "c64")
    st.set(C.random_state(n, 3) * 1.37)
    before = st.renormalize()
    assert abs(before - 1.37 ** 2) <= 1e-5
    assert abs(st.norm() - 1.0) <= 1e-6


def test_33_qubit_complex64_run_keeps_the_norm(gpu):
    """The 33-qubit complex64 workload (64 GiB) for 10 layers through the block plan with its renormalisation:
    the FP64 norm stays 1 within FP32 rounding."""
    circ = C.su4_u3_renorm(layers=10)
    st = gpu.State(33, "c64")
    sp = SegmentedPlan(33, circ.ops, circ.renorm_after, "block", 12, 4, "c64")
    sp.run(st)
    assert abs(st.norm() - 1.0) <= 1e-6
    sp.close()
    st.close()
