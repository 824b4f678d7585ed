"""The paper's own benchmark circuits (Hadamard x11, QSB, Quantum Volume, the RX sweep) and the swap ablation on
the GPU: plain and planned runs against the oracle or closed forms."""
import numpy as np
import pytest

import circuits as C
import oracle
from paper_2203_16044_amd import paperbench as PB
from paper_2203_16044_amd.plan import Circuit, Plan

pytestmark = pytest.mark.gpu


def _both(gpu, circ):
    out = []
    st = gpu.State(circ.n, "c128")
    c = Circuit.from_ops(circ.n, circ.ops)
    st.init_zero()
    c.run_plain(st)
    out.append(st.get())
    p = Plan(c, "block", 12, 4, "c128")
    st.init_zero()
    p.run(st)
    out.append(st.get())
    p.close()
    c.close()
    st.close()
    return out


@pytest.mark.parametrize("make", [lambda: C.qsb(14, seed=5), lambda: C.quantum_volume(14, seed=6),
                                  lambda: C.quantum_volume(15, seed=7), lambda: C.rx_sweep(13, seed=8)])
def test_paper_circuits_match_oracle(gpu, make):
    circ = make()
    ref = oracle.run(circ)
    for got in _both(gpu, circ):
        assert np.max(np.abs(got - ref)) <= 1e-12, circ.name


def test_hadamard_x11_closed_form(gpu):
    n = 18
    for got in _both(gpu, C.hadamard_x11(n)):
        # H^11 = H on every qubit: the uniform superposition
        assert np.max(np.abs(got - 2.0 ** (-n / 2))) <= 1e-12


def test_swap_ablation_is_bit_identical(gpu):
    import torch
    r = PB.run_swap_ablation(16, torch, p=0, s_max=5)
    assert [row["s"] for row in r["rows"]] == [1, 2, 3, 4, 5]
    assert all(row["bit_identical"] for row in r["rows"])
    # the fused-swap moves fewer bytes than the swaps it replaces, by the paper's ratio s / (2 (1 - 2^-s))
    for row in r["rows"]:
        assert row["byte_ratio"] == pytest.approx(row["s"] / (2 * (1 - 2.0 ** -row["s"])))


def test_paperbench_runs_every_workload(gpu):
    res = PB.main(["--n", "16"])
    names = [r["workload"] for r in res["results"]]
    assert names[0].startswith("hadamard") and names[-1].startswith("swap_ablation")
    for r in res["results"]:
        if "plain" in r:
            assert r["plain"]["effective_tbs"] > 0 and abs(r["norm_after"] - 1.0) <= 1e-12


def test_per_class_plain_run_on_a_small_mixed_circuit(gpu):
    import torch
    circ = C.mixed_layers(n=14, layers=3, toffolis=4, swap_s=2)
    r = PB.run_per_class(circ, torch)
    assert sum(v["launches"] for v in r["per_class"].values()) == len(circ.ops)
    assert {"dense_k1", "diag_k1", "diag_k2"} <= set(r["per_class"])
    assert all(v["tbs"] > 0 for v in r["per_class"].values())
