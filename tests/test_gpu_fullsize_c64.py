"""Full-size complex64 check (33 qubits, 64 GiB) in the configuration the benchmark times: 12-qubit block plans
with 4 always-local low qubits, whose heaviest stages run as fused products on the FP32 matrix cores.

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
