"""The cost-model MLP on the GPU (libqs's own forward/backward/Adam kernels) against the FP64 numpy twin, and
what the learned planner gains over the greedy planner."""
import os

import numpy as np
import pytest

import circuits as C
from oracle import mlp as omlp
from paper_2203_16044_amd import binding as B

pytestmark = pytest.mark.gpu

NIN, H = 12, 16


def _data(seed, Bn=100):
    rng = np.random.Generator(np.random.PCG64(seed))
    p = (rng.standard_normal(omlp.sizes(NIN, H)) * 0.3).astype(np.float32)
    X = rng.standard_normal((Bn, NIN)).astype(np.float32)
    T = rng.standard_normal(Bn).astype(np.float32)
    return p, X, T


def test_forward_matches_oracle(gpu):
    p, X, T = _data(1)
    m = B.qs_mlp_create(NIN, H)
    B.qs_mlp_set_params(m, p)
    y = B.qs_mlp_predict(m, X)
    ref, _ = omlp.forward(p.astype(np.float64), X.astype(np.float64), NIN, H)
    assert np.max(np.abs(y - ref)) <= 1e-4 * max(1.0, np.max(np.abs(ref)))
    B.qs_mlp_free(m)


@pytest.mark.parametrize("Bn", [1, 37, 256, 4096])
def test_gradients_match_oracle(gpu, Bn):
    p, X, T = _data(2, Bn)
    m = B.qs_mlp_create(NIN, H)
    B.qs_mlp_set_params(m, p)
    g, loss = B.qs_mlp_grad(m, X, T)
    gref, lref = omlp.grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64), NIN, H)
    assert abs(loss - lref) <= 1e-4 * max(1.0, lref)
    assert np.max(np.abs(g - gref)) <= 1e-4 * max(1.0, np.max(np.abs(gref)))
    B.qs_mlp_free(m)


def test_adam_steps_match_oracle_and_are_deterministic(gpu):
    p, X, T = _data(3, 64)
    runs = []
    for _ in range(2):
        m = B.qs_mlp_create(NIN, H)
        B.qs_mlp_set_params(m, p)
        for _ in range(5):
            B.qs_mlp_train_step(m, X, T, 1e-2)
        runs.append(B.qs_mlp_get_params(m))
        B.qs_mlp_free(m)
    assert runs[0].tobytes() == runs[1].tobytes()
    q = p.astype(np.float64)
    mm, vv = np.zeros_like(q), np.zeros_like(q)
    for t in range(1, 6):
        g, _ = omlp.grad(q, X.astype(np.float64), T.astype(np.float64), NIN, H)
        q, mm, vv = omlp.adam_step(q, g, mm, vv, t, 1e-2)
    assert np.max(np.abs(runs[0] - q)) <= 2e-4


def test_training_fits_a_smooth_function(gpu):
    rng = np.random.Generator(np.random.PCG64(4))
    X = rng.uniform(-1, 1, (2048, NIN)).astype(np.float32)
    y = (np.sin(X[:, 0] * 2) + X[:, 1] * X[:, 2]).astype(np.float32)
    m = B.qs_mlp_create(NIN, 32)
    B.qs_mlp_set_params(m, (rng.standard_normal(omlp.sizes(NIN, 32)) * 0.2).astype(np.float32))
    first = B.qs_mlp_grad(m, X, y)[1]
    for ep in range(60):
        perm = rng.permutation(len(y))
        for i in range(0, len(y), 256):
            idx = perm[i:i + 256]
            B.qs_mlp_train_step(m, X[idx], y[idx], 3e-3)
    last = B.qs_mlp_grad(m, X, y)[1]
    assert last < 0.15 * first, (first, last)
    B.qs_mlp_free(m)


def test_mlp_rejects_bad_batches(gpu):
    m = B.qs_mlp_create(NIN, H)
    with pytest.raises(B.QSError):
        B.qs_mlp_predict(m, np.zeros((5000, NIN), np.float32))
    with pytest.raises(B.QSError):
        B.qs_mlp_train_step(m, np.zeros((4, NIN), np.float32), np.zeros(4, np.float32), 0.0)
    B.qs_mlp_free(m)


def test_learned_planner_against_greedy(gpu):
    """On held-out circuits (other seeds and sizes than the training runs), the plan the trained model picks is
    measured against the greedy plan; the model must not lose (beyond timing noise) and its gain is reported."""
    from paper_2203_16044_amd import costmodel as CM
    from paper_2203_16044_amd.plan import Circuit
    if os.path.exists(CM.WEIGHTS):
        model = CM.CostModel.load()
    else:  # train a small model here from 16-22 qubit timings
        circs = [C.su4_u3_random(n=n, seed=5 + n, layers=2) for n in (16, 18, 20, 22)]
        X, y = CM.collect(circs, dtypes=("c128",), log=lambda m: None)
        model = CM.CostModel()
        model.fit(X, y, epochs=150)
    held = [(C.su4_u3_random(n=25, seed=901, layers=6), "c128"), (C.su4_u3_random(n=27, seed=902, layers=6), "c128"),
            (C.su4_u3_renorm(n=27, seed=903, layers=6), "c64")]
    report = []
    for circ, dt in held:
        st = gpu.State(circ.n, dt)
        c = Circuit.from_ops(circ.n, circ.ops)
        lp, cand, pred = CM.choose_plan(c, dt, model)
        gp, gcand, _ = CM.choose_plan(c, dt, None)
        t_l = min(CM.time_plan_passes(st, lp).sum() for _ in range(2))
        t_g = min(CM.time_plan_passes(st, gp).sum() for _ in range(2))
        report.append((circ.name, dt, cand, gcand, t_l, t_g))
        for x in (lp, gp, c):
            x.close()
        st.close()
    print("learned vs greedy:", report)
    tl = sum(r[4] for r in report)
    tg = sum(r[5] for r in report)
    assert tl <= 1.05 * tg, report
