"""The exchange-volume model against the paper's worked example (Sec. III-D, Fig. 2), and the equivalence of the
three circuits of that example on the oracle."""
import json
import os

import numpy as np

import circuits as C
import oracle
from paper_2203_16044_amd.volume import exchange_bytes

GOLD = os.path.join(os.path.dirname(__file__), "golden", "fig2_exchange_bytes.json")


def _hr(q, theta):
    return [C.Op("dense", (q,), (), C.h(), label="H"), C.Op("dense", (q,), (), C.rx(theta), label="RX")]


def _fig2():
    th = [0.3, 1.1, 2.0, 2.9]
    original = sum((_hr(q, th[q]) for q in range(4)), [])
    sw = lambda a, b: C.Op("fswap", p=a, q=b, s=1)  # noqa: E731
    swapped = (_hr(0, th[0]) + _hr(1, th[1]) + [sw(0, 2), sw(1, 3)] + _hr(0, th[2]) + _hr(1, th[3])
               + [sw(0, 2), sw(1, 3)])
    fs = C.Op("fswap", p=0, q=2, s=2)
    fused = _hr(0, th[0]) + _hr(1, th[1]) + [fs] + _hr(0, th[2]) + _hr(1, th[3]) + [fs]
    return original, swapped, fused


def test_fig2_exchange_bytes():
    g = json.load(open(GOLD))
    original, swapped, fused = _fig2()
    assert exchange_bytes(g["n"], g["n_global"], original) == g["original_bytes"]
    assert exchange_bytes(g["n"], g["n_global"], swapped) == g["four_swaps_bytes"]
    assert exchange_bytes(g["n"], g["n_global"], fused) == g["two_fused_swaps_bytes"]


def test_fig2_circuits_are_equivalent():
    original, swapped, fused = _fig2()
    ref = oracle.run(C.Circuit(4, original))
    for ops in (swapped, fused):
        assert np.max(np.abs(oracle.run(C.Circuit(4, ops)) - ref)) <= 1e-14


def test_local_only_ops_cost_nothing_and_swaps_scale():
    n = 10
    ops = [C.Op("dense", (q,), (), C.h()) for q in range(6)] + [C.Op("fswap", p=0, q=2, s=2)]
    assert exchange_bytes(n, 4, ops) == 0
    one = exchange_bytes(n, 4, [C.Op("fswap", p=0, q=6, s=1)])
    assert one == (1 << (n + 4)) // 2
    assert exchange_bytes(n, 4, [C.Op("fswap", p=0, q=6, s=4)]) == (1 << (n + 4)) * 15 // 16


def test_paper_metrics_definitions():
    """Effective bandwidth (Sec. IV-F) and QBF (Sec. IV-B) as the paper defines them."""
    from paper_2203_16044_amd.paperbench import metrics
    m = metrics(30, 1290, 2.0)
    assert m["effective_tbs"] == 2.0 ** 35 * 1290 / 2.0 / 1e12
    assert m["qbf"] == 2.0 ** 35 * 1290 / (2.0 * 78.6e12)
    assert m["frac_of_hbm_peak"] == m["effective_tbs"] / 8.0


def test_plain_path_algorithmic_bytes_per_class():
    """Bytes an op moves on the plain path: a CZ changes a quarter of the amplitudes, a Toffoli a quarter, an RZ
    all of them, a fused-swap all but its 2^(n-s) fixed points."""
    from paper_2203_16044_amd.paperbench import _op_bytes_class
    n, S = 10, 16
    full = 2 * S * (1 << n)
    assert _op_bytes_class(C.Op("dense", (3,), mat=C.h()), n, S) == ("dense_k1", full)
    assert _op_bytes_class(C.Op("diag", (2, 5), mat=C.CZ_DIAG), n, S) == ("diag_k2", full // 4)
    assert _op_bytes_class(C.Op("diag", (4,), mat=C.rz(0.3)), n, S) == ("diag_k1", full)
    assert _op_bytes_class(C.Op("ctrl", (1,), (2, 3), mat=np.array([[0, 1], [1, 0]])), n, S) == ("ctrl_c2_k1", full // 4)
    assert _op_bytes_class(C.Op("fswap", p=0, q=6, s=4), n, S) == ("fswap_s4", full * 15 // 16)


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_bench_traffic_is_null_once_the_kernel_sources_change(tmp_path):
    import importlib.util
    import shutil
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    taken = {name: t for name, t in bench.PMC_TRAFFIC.items() if t["fetch_kib"] is not None}
    for name, t in bench.PMC_TRAFFIC.items():
        if name not in taken:  # no reading for the current kernel sources: reported as null
            assert bench.pmc_traffic(name) is None
    for name, t in taken.items():
        assert t["sha1"] == bench.sources_sha1(t["sources"]), name  # the readings match the committed sources
        assert bench.pmc_traffic(name) > 2 * 16 * (1 << 32)
    if not taken:
        return
    # a copy of the sources with one byte changed no longer matches
    fake = tmp_path / "k.hip"
    shutil.copy(os.path.join(root, bench.PMC_TRAFFIC["block_b12"]["sources"][0]), fake)
    with open(fake, "ab") as f:
        f.write(b" ")
    bench.ROOT = str(tmp_path)
    t = dict(bench.PMC_TRAFFIC["block_b12"], sources=["k.hip"])
    bench.PMC_TRAFFIC["block_b12"] = t
    assert bench.pmc_traffic("block_b12") is None


def _load_bench():
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_alg", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    return bench


def test_bench_algorithmic_bytes_and_flops_by_hand():
    """The roofline's algorithmic figures, counted by hand: every changed amplitude read and written once
    (16 B each in complex128), 8 real flops per complex multiply-add (2^k of them per amplitude of a k-qubit
    gate), 6 per amplitude for a diagonal; a controlled gate touches the 2^(n-c) amplitudes whose controls are 1;
    a fused-swap moves all but the 2^(n-s) fixed points (Sec. III-D)."""
    import circuits as C
    bench = _load_bench()
    n = 32
    full = 2 * 16 * 2 ** n
    assert bench._alg_bytes(C.Op("dense", (5,), mat=C.h()), n, 16) == full == 2 ** 37
    assert bench._alg_bytes(C.Op("dense", (5,), mat=C.h()), n, 8) == 2 ** 36
    assert bench._alg_bytes(C.Op("ctrl", (7,), controls=(3, 4), mat=C.x_gate()), n, 16) == full // 4
    assert bench._alg_bytes(C.Op("fswap", (), p=0, q=20, s=6), n, 16) == full - full // 64
    assert bench._alg_flops(C.Op("dense", (1, 9), mat=np.eye(4)), n) == 32 * 2 ** n
    assert bench._alg_flops(C.Op("dense", (1, 2, 9), mat=np.eye(8)), n) == 64 * 2 ** n
    assert bench._alg_flops(C.Op("diag", (3,), mat=np.ones(2)), n) == 6 * 2 ** n
    assert bench._alg_flops(C.Op("ctrl", (7,), controls=(3,), mat=C.x_gate()), n) == 16 * 2 ** (n - 1)
    assert bench._alg_flops(C.Op("fswap", (), p=0, q=20, s=6), n) == 0


def test_planner_flops_per_amplitude_match_the_gate_count():
    """The tuned roofline takes each block pass's flops from the planner (flops per amplitude x 2^n). On the
    benchmark circuit every fused op is a 2-qubit op (an SU(4) with its neighbouring U3s folded in), so the plan's
    flops per amplitude summed over passes equal 32 x the fused ops it reports."""
    import circuits as C
    from paper_2203_16044_amd import binding as B
    from paper_2203_16044_amd.plan import Circuit, Plan
    circ = C.su4_u3_random(n=32, seed=32, layers=40)
    c = Circuit.from_ops(circ.n, circ.ops)
    p = Plan(c, "block", 12, 3)
    try:
        tot = sum(B.qs_plan_features(p.h, i)[14] * 256 for i in range(p.info()["passes"]))
        assert abs(tot - 32 * p.info()["fused_ops"]) <= 1e-3 * tot
    finally:
        p.close()
        c.close()
