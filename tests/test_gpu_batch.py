"""Batched serving form: many circuits in one persistent launch (and its captured-graph replays) against the
oracle and the per-circuit plain path."""
import numpy as np
import pytest
import torch

import circuits as C
import oracle
from paper_2203_16044_amd import batch as BT

pytestmark = pytest.mark.gpu


def _oracle_probs(circ):
    P, _ = oracle.probs(oracle.run(circ))
    return P


@pytest.mark.parametrize("params", [{"block_bits": 12, "low_bits": 4, "wg_per_cu": 2},
                                    {"block_bits": 10, "low_bits": 3, "wg_per_cu": 1},
                                    {"block_bits": 11, "low_bits": 4, "wg_per_cu": 4}])
def test_batch_matches_oracle(gpu, params):
    circs = C.serving_batch(count=24, seed=77, nmin=10, nmax=16, dmin=4, dmax=12)
    b = BT.Batch(circs, "c128", **params)
    b.run()
    for i, circ in enumerate(circs):
        assert np.max(np.abs(b.probs(i) - _oracle_probs(circ))) <= 1e-12, (i, circ.n)
    b.close()


# The configurations the autotuner picks for the 512-circuit workload on the benchmark machine (complex128:
# 12-qubit blocks, 3 low bits, 32 workgroups per CU; complex64: 12 / 4 / 32), and the other 32-workgroup shapes.
TUNED = [("c128", {"block_bits": 12, "low_bits": 3, "wg_per_cu": 32}),
         ("c64", {"block_bits": 12, "low_bits": 4, "wg_per_cu": 32}),
         ("c128", {"block_bits": 11, "low_bits": 3, "wg_per_cu": 32}),
         ("c64", {"block_bits": 12, "low_bits": 3, "wg_per_cu": 32})]


@pytest.mark.parametrize("dtype,params", TUNED)
def test_batch_autotuned_configurations_match_oracle(gpu, dtype, params):
    """The autotuned launch shapes, eager and graph-replayed, on a batch that spans LDS-resident circuits and HBM
    circuits of up to 20 qubits (256 blocks per pass), against the oracle: complex128 to 1e-12, complex64 with every
    probability within 1e-5 and every distribution summing to 1 within 1e-5."""
    circs = C.serving_batch(count=32, seed=81, nmin=10, nmax=20, dmin=4, dmax=14)
    b = BT.Batch(circs, dtype, **params)
    tol = 1e-12 if dtype == "c128" else 1e-5
    for graph in (False, True):
        b.run(graph=graph)
        b.sync()
        for i, circ in enumerate(circs):
            P = b.probs(i)
            assert np.max(np.abs(P - _oracle_probs(circ))) <= tol, (graph, i, circ.n)
            assert abs(P.sum() - 1.0) <= tol
    b.close()


def test_batch_complex64_error(gpu):
    circs = C.serving_batch(count=12, seed=78, nmin=10, nmax=15, dmin=4, dmax=10)
    b = BT.Batch(circs, "c64")
    b.run()
    worst = 0.0
    for i, circ in enumerate(circs):
        P = b.probs(i)
        worst = max(worst, float(np.max(np.abs(P - _oracle_probs(circ)))))
        assert abs(P.sum() - 1.0) <= 1e-5
    assert worst <= 1e-5, worst
    b.close()


@pytest.mark.parametrize("dtype,tol", [("c128", 1e-12), ("c64", 1e-5)])
def test_batch_edge_circuits(gpu, dtype, tol):
    """Empty circuits inside and beyond the 12-qubit LDS block (the latter get one empty pass that generates |0..0>
    and writes its probabilities), the smallest batched size (8 qubits), circuits of exactly the block size and one
    qubit beyond it, GHZ across the block boundary (CNOT chain) and a single gate on the highest qubit."""
    rng = np.random.Generator(np.random.PCG64(91))
    x_top = C.Circuit(14, ops=[C.Op("dense", (13,), mat=C.x_gate())], name="x_top")
    circs = [C.Circuit(8, name="empty8"), C.Circuit(14, name="empty14"), C._batch_circuit(rng, 8, 5, 0),
             C._batch_circuit(rng, 12, 6, 1), C._batch_circuit(rng, 13, 6, 2), C.ghz(13), x_top,
             C._batch_circuit(rng, 16, 3, 3)]
    b = BT.Batch(circs, dtype, block_bits=12, low_bits=4, wg_per_cu=2)
    b.run()
    for i, circ in enumerate(circs):
        P = b.probs(i)
        assert P.shape == (1 << circ.n,)
        assert np.max(np.abs(P - _oracle_probs(circ))) <= tol, (i, circ.name)
    for i in (0, 1):
        assert b.probs(i)[0] == 1.0 and not np.any(b.probs(i)[1:])
    assert b.probs(6)[1 << 13] == 1.0
    b.close()


def test_graph_replays_match_eager(gpu):
    circs = C.serving_batch(count=40, seed=79, nmin=10, nmax=18, dmin=4, dmax=10)
    b = BT.Batch(circs, "c128")
    b.run(graph=False)
    ref = [b.probs(i).copy() for i in range(len(circs))]
    x = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(3):
        b.run(graph=True)
        x.mul_(1.0000001)  # unrelated eager work between replays
        b.sync()
        torch.cuda.synchronize()
        for i in range(len(circs)):
            assert b.probs(i).tobytes() == ref[i].tobytes(), (rep, i)
    # a new launch shape drops the captured graph; the next graph run captures the new one
    b.set_launch(1)
    b.run(graph=True)
    b.sync()
    for i in range(len(circs)):
        assert b.probs(i).tobytes() == ref[i].tobytes(), i
    b.close()


@pytest.mark.parametrize("dtype,params", [("c128", {"block_bits": 12, "low_bits": 3, "wg_per_cu": 32}),
                                          ("c64", {"block_bits": 12, "low_bits": 4, "wg_per_cu": 32})])
def test_full_512_circuit_batch_against_oracle(gpu, dtype, params):
    """The 512-circuit workload (10..22 qubits, 10..40 layers) at its autotuned launch shape, graph-replayed: every
    output is a distribution, and 15 sampled circuits (including the largest, 22 qubits) match the oracle's
    probabilities (complex128: 1e-12; complex64: 1e-5)."""
    circs = C.serving_batch()
    b = BT.Batch(circs, dtype, **params)
    b.run(graph=True)
    b.sync()
    tol = 1e-12 if dtype == "c128" else 1e-5
    sample = list(range(0, 512, 37)) + [int(np.argmax([c.n for c in circs]))]
    for i in sample:
        P = b.probs(i)
        assert abs(P.sum() - 1.0) <= tol
        assert np.max(np.abs(P - _oracle_probs(circs[i]))) <= tol, (i, circs[i].n)
    sums = [b.probs(i).sum() for i in range(0, 512, 5)]
    assert max(abs(s - 1.0) for s in sums) <= tol
    b.close()


def test_autotuner_picks_a_measured_candidate(gpu, tmp_path):
    circs = C.serving_batch(count=20, seed=80, nmin=10, nmax=16, dmin=4, dmax=8)
    space = [{"block_bits": 10, "low_bits": 3, "wg_per_cu": 1}, {"block_bits": 12, "low_bits": 4, "wg_per_cu": 2}]
    best, times = BT.autotune(circs, "c128", cache=str(tmp_path / "cache.json"), space=space)
    assert best in space and len(times) == 2
    best2, _ = BT.autotune(circs, "c128", cache=str(tmp_path / "cache.json"), space=space)
    assert best2 == best  # served from the cache


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_learned_batch_shape(gpu, dtype, tmp_path):
    """The cost model picks the batch's block shape from its plans' predicted times (one prediction per candidate
    shape, all finite and positive), the autotuner then times only that shape's launches, and the batch planned with
    the chosen parameters matches the oracle."""
    import json
    import os

    from paper_2203_16044_amd import costmodel as CM
    if not os.path.exists(CM.WEIGHTS):
        pytest.skip("no trained cost model in the package")
    model = CM.CostModel.load()
    circs = C.serving_batch(count=32, seed=91, nmin=10, nmax=16, dmin=4, dmax=12)
    shape, pred = BT.learned_shape(circs, dtype, model)
    assert shape in BT.SHAPES and set(pred) == set(BT.SHAPES)
    assert all(np.isfinite(v) and v > 0 for v in pred.values()) and pred[shape] == min(pred.values())
    best, times = BT.autotune(circs, dtype, cache=None, model=model)
    assert (best["block_bits"], best["low_bits"]) == shape
    assert {(k["block_bits"], k["low_bits"]) for k in map(json.loads, times)} == {shape}
    b = BT.Batch(circs, dtype, **best)
    b.run()
    for i, circ in enumerate(circs):
        ref = _oracle_probs(circ)
        err = np.max(np.abs(b.probs(i) - ref))
        assert err <= (1e-12 if dtype == "c128" else 1e-5), (i, circ.n, err)
    b.close()
