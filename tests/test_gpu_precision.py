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


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_folded_renormalisation_matches_separate_sweeps(gpu, dtype):
    """Renormalisations folded into the block passes around them (complex64; complex128 falls back to sweeps)
    give the state that a qs_renormalize between the segments gives, from an unnormalised start."""
    n = 20
    circ = C.su4_u3_renorm(n=n, seed=960, layers=8)
    circ.renorm_after = (2, 5, 8)  # the last segment ends with one: scaled by qs_renormalize_pending
    psi0 = C.random_state(n, 961) * 1.3
    out = {}
    for folded in (True, False):
        st = gpu.State(n, dtype)
        st.set(psi0)
        sp = SegmentedPlan(n, circ.ops, circ.renorm_after, "block", 12, 4, dtype)
        sp.run(st, folded=folded)
        out[folded] = np.asarray(st.get(), np.complex128)
        assert abs(st.norm() - 1.0) <= (1e-6 if dtype == "c64" else 1e-12)
        sp.close()
        st.close()
    if dtype == "c64":
        infid, maxd = oracle.error_metrics(out[True], out[False])
        assert infid <= 1e-10 and maxd <= 1e-6, (infid, maxd)
    else:
        assert float(np.max(np.abs(out[True] - out[False]))) <= 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode,bits", [("block", 12), ("fuse", 4)])
def test_renorm_flags_on_one_plan(gpu, dtype, mode, bits):
    """qs_plan_run_renorm on a single plan with both flags (folded into the same block pass where the plan has one
    block pass; dense passes use the sweeps): the pending norm it leaves is the norm of the state the plan leaves,
    and the state equals plan-then-scale from the scaled start."""
    import paper_2203_16044_amd.binding as B
    n = 16
    circ = C.su4_u3_random(n=n, seed=970, layers=3)
    psi0 = C.random_state(n, 971) * 0.8
    c = Circuit.from_ops(n, circ.ops)
    p = Plan(c, mode, bits, 4 if mode == "block" else 0, dtype)
    st = gpu.State(n, dtype)
    st.set(psi0)
    ec = Circuit.from_ops(n, [])
    e = Plan(ec, "block", 12, 4, dtype)
    B.qs_plan_run_renorm(st.h, e.h, B.QS_RUN_NORM_LAST)  # empty plan: pending = |psi0|^2, taken by a sweep
    B.qs_plan_run_renorm(st.h, p.h, B.QS_RUN_SCALE_FIRST | B.QS_RUN_NORM_LAST)
    got_norm = B.qs_renormalize_pending(st.h, True)
    got = np.asarray(st.get(), np.complex128)
    ref = oracle.run(circ, psi0 / np.sqrt(np.vdot(psi0, psi0).real))
    tol = 1e-6 if dtype == "c64" else 1e-12
    assert abs(got_norm - 1.0) <= tol, got_norm  # the plan is unitary: the scaled start has norm 1
    assert float(np.max(np.abs(got - ref / np.sqrt(got_norm)))) <= (2e-6 if dtype == "c64" else 1e-12)
    with pytest.raises(B.QSError):
        B.qs_plan_run_renorm(st.h, p.h, 4)
    for h in (p, e, c, ec, st):
        h.close()


def test_renorm_flags_on_remapped_plans(gpu):
    """qs_plan_run_renorm on remapped plans (fused-swap and relabel passes around the block passes: the relabels
    launch nothing and are skipped when finding the first and last passes; fused-swaps take the sweeps): the state
    equals the one from qs_plan_run with qs_renormalize around it."""
    import paper_2203_16044_amd.binding as B
    n = 18
    circ = C.su4_u3_random(n=n, seed=980, layers=4)
    psi0 = C.random_state(n, 981) * 1.2
    c = Circuit.from_ops(n, circ.ops)
    p = Plan(c, "remap", 12, 0, "c64")
    assert p.info()["other"] >= 1  # fused-swaps (and relabels) besides block passes
    out = []
    for folded in (True, False):
        st = gpu.State(n, "c64")
        st.set(psi0)
        if folded:
            ec = Circuit.from_ops(n, [])
            e = Plan(ec, "block", 12, 4, "c64")
            B.qs_plan_run_renorm(st.h, e.h, B.QS_RUN_NORM_LAST)
            B.qs_plan_run_renorm(st.h, p.h, B.QS_RUN_SCALE_FIRST | B.QS_RUN_NORM_LAST)
            B.qs_renormalize_pending(st.h, False)
            e.close()
            ec.close()
        else:
            st.renormalize()
            p.run(st)
            st.renormalize()
        out.append(np.asarray(st.get(), np.complex128))
        st.close()
    infid, maxd = oracle.error_metrics(out[0], out[1])
    assert infid <= 1e-10 and maxd <= 1e-6, (infid, maxd)
    ref = oracle.run(circ, psi0 / np.sqrt(np.vdot(psi0, psi0).real))
    infid, maxd = oracle.error_metrics(out[0], ref)
    assert infid <= 1e-8 and maxd <= 1e-6, (infid, maxd)
    p.close()
    c.close()


def test_learned_segmented_plan_against_fp64_oracle(gpu):
    """The complex64 leg's planner: choose_segmented returns the candidate (block shape, beam width) whose segments
    the cost model predicts fastest in sum (every candidate re-priced here), without weights the greedy shape; the
    chosen plan, its renormalisations folded into its block passes, matches the FP64 oracle."""
    import os

    import paper_2203_16044_amd.binding as B
    from paper_2203_16044_amd import costmodel as CM
    if not os.path.exists(CM.WEIGHTS):
        pytest.skip("no trained cost model in the package")
    n = 20
    circ = C.su4_u3_renorm(n=n, seed=980, layers=12)
    circ.renorm_after = (4, 8, 12)
    g, gkey, gpred = CM.choose_segmented(n, circ.ops, circ.renorm_after, "c64", None)
    assert gkey == CM.greedy_for(n) and gpred is None
    g.close()
    model = CM.CostModel.load()
    sp, key, pred = CM.choose_segmented(n, circ.ops, circ.renorm_after, "c64", model)
    cur = B.qs_get_tunable("plan_beam")
    preds = {}
    for cand in [c for c in CM.candidates(n) if c[0] == "block"]:
        for k in [cand] + [cand + (w,) for w in CM.BEAMS if w != cur]:
            q = CM.make_segmented(n, circ.ops, circ.renorm_after, k, "c64")
            preds[k] = sum(model.predict_plan_ms(p) for p in q.plans())
            q.close()
    assert key in preds and preds[key] == pytest.approx(pred, rel=1e-6), (key, pred, preds)
    assert pred == pytest.approx(min(preds.values()), rel=1e-6), (key, pred, preds)
    assert B.qs_get_tunable("plan_beam") == cur
    st = gpu.State(n, "c64")
    sp.run(st)
    infid, maxd = oracle.error_metrics(st.get(), oracle.run(circ))
    assert infid <= 1e-8 and maxd <= 1e-6, (key, infid, maxd)
    assert abs(st.norm() - 1.0) <= 1e-6
    sp.close()
    st.close()
    model.close()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mode,bits,low", [("block", 12, 4), ("block", 10, 3), ("fuse", 4, 0)])
def test_lazy_renormalisation_against_fp64_oracle(gpu, dtype, mode, bits, low):
    """One plan renormalised at pass boundaries (LazyRenormPlan; folded into complex64 block passes, sweeps
    otherwise), from an unnormalised start: a unitary circuit keeps the norm, so the final state is the oracle's
    run of the normalised start; it also equals the layer-exact segmented form up to rounding."""
    import paper_2203_16044_amd.binding as B
    from paper_2203_16044_amd.plan import LazyRenormPlan
    n = 20
    circ = C.su4_u3_renorm(n=n, seed=995, layers=12)
    circ.renorm_after = (4, 8, 12)
    psi0 = C.random_state(n, 996) * 1.3
    ref = oracle.run(circ, psi0 / np.linalg.norm(psi0))
    out = {}
    for form in ("lazy", "segments"):
        cls = LazyRenormPlan if form == "lazy" else SegmentedPlan
        p = cls(n, circ.ops, circ.renorm_after, mode, bits, low, dtype)
        if form == "lazy":
            assert 1 <= len(p.bounds) <= 3 and p.info()["renormalisations"] == len(p.bounds)
        st = gpu.State(n, dtype)
        st.set(psi0)
        p.run(st)
        out[form] = np.asarray(st.get(), np.complex128)
        assert abs(st.norm() - 1.0) <= (1e-6 if dtype == "c64" else 1e-12), form
        if form == "lazy":
            np_ = p.info()["passes"]
            for a, b in ((1, 0), (0, np_ + 1), (-1, 0)):
                with pytest.raises(B.QSError):
                    B.qs_plan_run_range_renorm(st.h, p.plan.h, a, b, 0)
            with pytest.raises(B.QSError):
                B.qs_plan_run_range_renorm(st.h, p.plan.h, 0, 0, 4)
        p.close()
        st.close()
    if dtype == "c64":
        infid, maxd = oracle.error_metrics(out["lazy"], ref)
        assert infid <= 1e-8 and maxd <= 1e-6, (infid, maxd)
        infid, maxd = oracle.error_metrics(out["lazy"], out["segments"])
        assert infid <= 1e-10 and maxd <= 1e-6, (infid, maxd)
    else:
        assert float(np.max(np.abs(out["lazy"] - ref))) <= 1e-12
        assert float(np.max(np.abs(out["lazy"] - out["segments"]))) <= 1e-12
