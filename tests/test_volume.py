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
