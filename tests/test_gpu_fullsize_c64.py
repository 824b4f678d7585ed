"""Full-size complex64 checks (33 qubits, 64 GiB): 12-qubit block plans with 4 always-local low qubits, whose
heaviest stages run as fused products on the FP32 matrix cores, and the configuration the benchmark times (the
cost model's plan, renormalised at pass boundaries with the renormalisations folded into the block passes).

The oracle cannot follow a 33-qubit circuit, so this checks what holds at any size: the norm after the circuit
(FP64 reduction of FP32 amplitudes) and echo (the circuit, then its inverse, returns to |0..0>) with a complex64
tolerance.
"""
import numpy as np
import pytest
import torch

import circuits as C
from paper_2203_16044_amd.plan import Circuit, Plan

pytestmark = pytest.mark.gpu

N = 33


def test_complex64_33_qubit_circuit_norm_and_echo(gpu):
    circ = C.su4_u3_renorm(n=N, seed=33, layers=40)
    torch.cuda.empty_cache()
    st = gpu.State(N, "c64")
    plans = []
    try:
        st.init_zero()
        c = Circuit.from_ops(N, circ.ops)
        p = Plan(c, "block", 12, 4, dtype="c64")
        plans += [p, c]
        p.run(st)
        assert abs(st.norm() - 1.0) <= 1e-4
        inv = C.inverse_circuit(circ)
        ci = Circuit.from_ops(N, inv.ops)
        pi = Plan(ci, "block", 12, 4, dtype="c64")
        plans += [pi, ci]
        pi.run(st)
        rng = np.random.Generator(np.random.PCG64(34))
        idx = np.unique(np.concatenate([rng.integers(1, 1 << N, size=4096, dtype=np.int64), [(1 << N) - 1, 1]]))
        t = torch.as_tensor(np.concatenate([[0], idx]), device=st.buf.device)
        amps = st.buf[t].cpu().numpy().astype(np.complex128)
        assert abs(amps[0] - 1.0) <= 1e-4
        assert np.max(np.abs(amps[1:])) <= 1e-4
    finally:
        for x in plans:
            x.close()
        st.close()
        del st
        torch.cuda.empty_cache()


def test_complex64_33_qubit_lazy_renormalised_plan(gpu):
    """The complex64 leg as the benchmark times it: one plan chosen by the cost model (lazy renormalisation at pass
    boundaries, folded into the block passes), from |0..0> scaled by 1.3 so that every renormalisation has work to
    do. After the circuit the FP64 norm is 1; the inverse circuit (planned alike) then returns to |0..0> with
    amplitude 1 (the start renormalised), checked on sampled amplitudes."""
    import os

    from paper_2203_16044_amd import costmodel as CM
    circ = C.su4_u3_renorm(n=N, seed=33, layers=40)
    model = CM.CostModel.load() if os.path.exists(CM.WEIGHTS) else None
    lp, key, _ = CM.choose_segmented(N, circ.ops, circ.renorm_after, "c64", model, lazy=True)
    if model is not None:
        model.close()
    torch.cuda.empty_cache()
    st = gpu.State(N, "c64")
    plans = [lp]
    try:
        st.init_zero()
        st.buf[0] = 1.3  # torch's current stream, which the state runs on
        torch.cuda.synchronize()
        assert len(lp.bounds) == 4 and lp.bounds[-1] == lp.info()["passes"] - 1, lp.bounds
        lp.run(st)
        assert abs(st.norm() - 1.0) <= 1e-6, key
        inv = C.inverse_circuit(circ)
        ci = Circuit.from_ops(N, inv.ops)
        pi = CM.make_plan(ci, key, "c64")
        plans += [pi, ci]
        pi.run(st)
        rng = np.random.Generator(np.random.PCG64(35))
        idx = np.unique(np.concatenate([rng.integers(1, 1 << N, size=4096, dtype=np.int64), [(1 << N) - 1, 1]]))
        t = torch.as_tensor(np.concatenate([[0], idx]), device=st.buf.device)
        amps = st.buf[t].cpu().numpy().astype(np.complex128)
        assert abs(amps[0] - 1.0) <= 1e-4, (key, amps[0])
        assert np.max(np.abs(amps[1:])) <= 1e-4, key
    finally:
        for x in plans:
            x.close()
        st.close()
        del st
        torch.cuda.empty_cache()
