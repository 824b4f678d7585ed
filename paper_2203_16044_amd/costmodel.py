"""Learned cost model for the planner: an MLP (trained and run by libqs's own GPU kernels) predicts the time of a
plan pass from its features; the planner scores candidate plans with it and keeps the cheapest. The greedy plan
(LDS blocks of 12 qubits incl. the 4 lowest) is the fallback and the reference the model is measured against.

Data: the simulator times every pass of candidate plans of 20-30-qubit circuits with HIP events on the state's
stream (the target is log(pass milliseconds)). Features come from ``qs_plan_features`` (QS_PLAN_NFEAT floats).
Usage (on a machine with the GPU):  python -m paper_2203_16044_amd.costmodel --out <weights.npz>
"""
from __future__ import annotations

import argparse
import math
import os
import time
from typing import List, Optional, Sequence, Tuple

import numpy as np

from . import binding as B

NIN = B.QS_PLAN_NFEAT
HIDDEN = 64
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel_weights.npz")
GREEDY = ("block", 12, 4)


def candidates(n: int) -> List[Tuple[str, int, int]]:
    out = [("block", b, w) for b in (10, 11, 12, 13) for w in (3, 4) if b <= n and n >= 8]
    out += [("fuse", k, 0) for k in (2, 3, 4, 5, 6) if k <= n]
    if n >= 13:  # the paper's swap-based remapping: blocks on the low 12 physical qubits, fused-swaps inserted
        out.append(("remap", 12, 0))
    return out


def greedy_for(n: int) -> Tuple[str, int, int]:
    return GREEDY if n >= 12 else ("block", max(8, n), min(4, n)) if n >= 8 else ("fuse", min(4, n), 0)


def plan_features(plan) -> np.ndarray:
    return np.stack([B.qs_plan_features(plan.h, i) for i in range(plan.info()["passes"])])


def kernel_passes(plan) -> np.ndarray:
    """Mask of the passes that run a kernel: relabels (type 4, a circuit fused-swap absorbed into a remapped plan's
    qubit map) move no data and cost nothing, so they are neither priced nor trained on."""
    return np.array([B.qs_plan_pass_info(plan.h, i)["type"] != 4 for i in range(plan.info()["passes"])], dtype=bool)


def time_plan_passes(state, plan, reps: int = 2) -> np.ndarray:
    """Per-pass milliseconds (the last of `reps` runs), recorded with events on the state's stream."""
    import torch
    npass = plan.info()["passes"]
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(npass)]
    s = state.stream
    for _ in range(reps):
        state.init_zero()
        for i in range(npass):
            ev[i][0].record(s)
            plan.run(state, i, i + 1)
            ev[i][1].record(s)
        torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in ev], dtype=np.float64)


def training_circuits(seed: int = 1000, nmax: int = 32):
    """The circuit families the model is trained on (20..nmax qubits). They are deep enough (8 SU(4)+U3 layers, 6 mixed
    layers, 150 random gates) that passes carry as many fused ops as passes in the middle of long circuits do: a pass's
    time depends on its ops, and a model trained on shallow circuits only under-predicts deep circuits' passes."""
    import circuits as C
    out = []
    for n in range(20, nmax + 1):
        out.append(C.su4_u3_random(n=n, seed=seed + n, layers=8))
        out.append(C.mixed_layers(n=n, seed=seed + 100 + n, layers=6, toffolis=8, swap_s=min(6, n // 4)))
        out.append(C.random_circuit(n, seed=seed + 200 + n, num_ops=150, kmax=3,
                                    kinds=("dense", "diag", "ctrl")))
    return out


def collect_learned(circs, model: "CostModel", dtypes=("c128", "c64"), log=print):
    """Time every pass of the plans the model itself chooses pass by pass (qs_plan_create_learned): the candidates a
    model prefers are where its errors cost most, so they are added to its training data."""
    import torch

    from .plan import Circuit
    from .state import State
    X, y = [], []
    for dt in dtypes:
        for circ in circs:
            n = circ.n
            if dt == "c64" and n > 31:
                continue
            st = State(n, dt)
            c = Circuit.from_ops(n, circ.ops)
            p = learned_plan(c, dt, model)
            if p is not None:
                ms = time_plan_passes(st, p)
                X.append(plan_features(p))
                y.append(np.log(np.maximum(ms, 1e-4)))
                p.close()
            c.close()
            st.close()
            del st
            torch.cuda.empty_cache()
        log(f"collected learned plans ({dt}): {sum(len(v) for v in y)} samples so far")
    return np.concatenate(X).astype(np.float32), np.concatenate(y).astype(np.float32)


def collect(circs, dtypes=("c128", "c64"), log=print, groups=None):
    """Time every pass of every candidate plan of every circuit: returns (features, log-ms targets). If `groups` is
    a list, one id per pass (circuit/dtype index, candidate index) is appended to it."""
    import torch

    from .plan import Circuit, Plan
    from .state import State
    X, y = [], []
    gid = 0
    for dt in dtypes:
        for circ in circs:
            n = circ.n
            if dt == "c64" and n > 31:
                continue  # complex64 runs stay within the same state sizes as complex128's
            st = State(n, dt)
            c = Circuit.from_ops(n, circ.ops)
            t0 = time.perf_counter()
            for ci, (mode, bits, low) in enumerate(candidates(n)):
                p = Plan(c, mode, bits, low, dt)
                keep = kernel_passes(p)
                ms = time_plan_passes(st, p)[keep]
                X.append(plan_features(p)[keep])
                y.append(np.log(np.maximum(ms, 1e-4)))
                if groups is not None:
                    groups.extend([(gid, ci)] * len(ms))
                p.close()
            gid += 1
            c.close()
            st.close()
            del st
            torch.cuda.empty_cache()
            log(f"collected {circ.name} {dt}: {sum(len(v) for v in y)} samples so far "
                f"({time.perf_counter() - t0:.1f} s)")
    return np.concatenate(X).astype(np.float32), np.concatenate(y).astype(np.float32)


class CostModel:
    """MLP over standardised pass features predicting log(ms); runs on libqs's kernels."""

    def __init__(self, params: Optional[np.ndarray] = None, mean=None, std=None, hidden: int = HIDDEN):
        self.hidden = hidden
        self.h = B.qs_mlp_create(NIN, hidden)
        self.mean = np.zeros(NIN, np.float32) if mean is None else np.asarray(mean, np.float32)
        self.std = np.ones(NIN, np.float32) if std is None else np.asarray(std, np.float32)
        if params is None:
            params = self.init_params(hidden)
        B.qs_mlp_set_params(self.h, params)

    @staticmethod
    def init_params(hidden: int, seed: int = 0) -> np.ndarray:
        rng = np.random.Generator(np.random.PCG64(seed))
        parts = [rng.standard_normal(hidden * NIN) * math.sqrt(2.0 / NIN), np.zeros(hidden),
                 rng.standard_normal(hidden * hidden) * math.sqrt(2.0 / hidden), np.zeros(hidden),
                 rng.standard_normal(hidden) * math.sqrt(1.0 / hidden), np.zeros(1)]
        return np.concatenate(parts).astype(np.float32)

    def _norm(self, X):
        return (np.asarray(X, np.float32) - self.mean) / self.std

    def fit(self, X, y, epochs: int = 300, batch: int = 256, lr: float = 2e-3, seed: int = 0, log=None):
        X = np.asarray(X, np.float32)
        self.mean = X.mean(axis=0)
        self.std = np.where(X.std(axis=0) > 1e-6, X.std(axis=0), 1.0).astype(np.float32)
        Xn = self._norm(X)
        y = np.asarray(y, np.float32)
        rng = np.random.Generator(np.random.PCG64(seed))
        hist = []
        for ep in range(epochs):
            perm = rng.permutation(len(y))
            tot = 0.0
            for i in range(0, len(y), batch):
                idx = perm[i:i + batch]
                tot += B.qs_mlp_train_step(self.h, Xn[idx], y[idx], lr) * len(idx)
            hist.append(tot / len(y))
            if log and (ep % 50 == 0 or ep == epochs - 1):
                log(f"epoch {ep}: train mse {hist[-1]:.4f}")
        return hist

    def fit_more(self, X, y, epochs: int = 100, batch: int = 256, lr: float = 3e-4, seed: int = 1):
        """Continue training with the current standardisation (a lower learning rate for the last epochs)."""
        Xn = self._norm(X)
        y = np.asarray(y, np.float32)
        rng = np.random.Generator(np.random.PCG64(seed))
        for _ in range(epochs):
            perm = rng.permutation(len(y))
            for i in range(0, len(y), batch):
                idx = perm[i:i + batch]
                B.qs_mlp_train_step(self.h, Xn[idx], y[idx], lr)

    def predict_log_ms(self, X) -> np.ndarray:
        X = self._norm(X)
        out = []
        for i in range(0, len(X), 4096):
            out.append(B.qs_mlp_predict(self.h, X[i:i + 4096]))
        return np.concatenate(out) if out else np.zeros(0, np.float32)

    def predict_plan_ms(self, plan) -> float:
        X = plan_features(plan)[kernel_passes(plan)]
        return float(np.exp(self.predict_log_ms(X).astype(np.float64)).sum()) if len(X) else 0.0

    def save(self, path: str) -> None:
        np.savez(path, params=B.qs_mlp_get_params(self.h), mean=self.mean, std=self.std, hidden=self.hidden,
                 nin=NIN)

    @classmethod
    def load(cls, path: str = WEIGHTS) -> "CostModel":
        d = np.load(path, allow_pickle=False)
        if int(d["nin"]) != NIN:
            raise ValueError("cost-model weights were trained for a different feature layout")
        return cls(d["params"], d["mean"], d["std"], int(d["hidden"]))

    def close(self):
        if getattr(self, "h", None):
            B.qs_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# switch away from the greedy plan only for a predicted saving above this fraction: 0, i.e. the predicted-fastest
# candidate (measured regret of that argmin on the training runs: 0.2 % mean; on the held-out circuits every switch
# it makes measured faster than greedy)
MARGIN = 0.0
# block shapes (block bits, always-local low bits) among which the learned planner chooses each pass
PASS_SHAPES = ((12, 3), (12, 4), (13, 3), (11, 3))
PER_SHAPE = 4  # candidate local sets per shape and pass
GATE_SLACK = 1 << 20  # a candidate pass must carry at least the largest candidate's gate count minus this
LOOKAHEAD = 1  # score a candidate pass together with the pass that would follow it
LEARNED = ("learned", 0, 0)


def learned_plan(circuit, dtype: str, model: CostModel, shapes=PASS_SHAPES, per_shape: int = PER_SHAPE,
                 gate_slack: int = GATE_SLACK, lookahead: int = LOOKAHEAD):
    """The plan whose every pass the model chooses (qs_plan_create_learned), or None for circuits too small for the
    shapes."""
    from .plan import Plan
    shapes = [s for s in shapes if s[0] <= circuit.n]
    if not shapes:
        return None
    return Plan.learned(circuit, model, shapes, per_shape, dtype, gate_slack, lookahead)


# pass-formation beam widths besides the planner's default that the whole-plan choice prices for every block-mode
# candidate (the pass count is not monotone in the width); a candidate key (mode, bits, low, width) names one
BEAMS = (24, 64)


def make_plan(circuit, cand, dtype: str = "c128"):
    """The plan a candidate key names: (mode, block bits, low bits) at the planner's beam width, or (mode, block
    bits, low bits, width) at that pass-formation beam width (the process-wide tunable, restored afterwards)."""
    from .plan import Plan
    if len(cand) == 3:
        return Plan(circuit, *cand, dtype)
    mode, bits, low, width = cand
    old = B.qs_get_tunable("plan_beam")
    B.qs_set_tunable("plan_beam", width)
    try:
        return Plan(circuit, mode, bits, low, dtype)
    finally:
        B.qs_set_tunable("plan_beam", old)


def choose_plan(circuit, dtype: str = "c128", model: Optional[CostModel] = None,
                cands: Optional[Sequence[Tuple[str, int, int]]] = None, margin: float = MARGIN,
                per_pass: bool = False, beams: Sequence[int] = BEAMS):
    """The candidate with the lowest predicted time, if it beats the greedy plan's prediction by more than `margin`
    (default MARGIN); otherwise (and without a model) the greedy plan. Candidates: whole plans of one shape each (`cands`, default
    candidates(n)), every block-mode shape also formed at the pass-formation beam widths `beams`, and, with
    per_pass, the plan whose passes the model chooses one by one (LEARNED). Per-pass
    choice is off by default: on held-out circuits it measured no faster than the best whole plan, and its
    predictions run low (the model is scored on the very passes it picked as cheapest). Returns
    (plan, its candidate key (mode, bits, low) or (mode, bits, low, beam width), predicted ms)."""
    from .plan import Plan
    n = circuit.n
    g = greedy_for(n)
    if model is None:
        return Plan(circuit, *g, dtype), g, None
    gp = Plan(circuit, *g, dtype)
    gt = model.predict_plan_ms(gp)
    best = (gp, g, gt)

    def offer(p, key):
        nonlocal best
        t = model.predict_plan_ms(p)
        if t < (1.0 - margin) * gt and t < best[2]:
            if best[0] is not gp:
                best[0].close()
            best = (p, key, t)
        else:
            p.close()

    for cand in (cands or candidates(n)):
        if cand != g:
            offer(Plan(circuit, *cand, dtype), cand)
        if cand[0] == "block" and beams:
            for width in beams:
                if width != B.qs_get_tunable("plan_beam"):
                    offer(make_plan(circuit, cand + (width,), dtype), cand + (width,))
    if per_pass:
        lp = learned_plan(circuit, dtype, model)
        if lp is not None:
            offer(lp, LEARNED)
    if best[0] is not gp:
        gp.close()
    return best



def make_segmented(n: int, ops, renorm_after, cand, dtype: str = "c64", lazy: bool = False):
    """The plan with renormalisations after given layers for a candidate key: (mode, block bits, low bits) at the
    planner's beam width, or with a fourth entry, that beam width (the process-wide tunable, restored afterwards).
    By default the circuit is cut after its renormalisation layers and each segment planned alone (SegmentedPlan);
    with `lazy` it is planned once and renormalised at pass boundaries (LazyRenormPlan)."""
    from .plan import LazyRenormPlan, SegmentedPlan
    cls = LazyRenormPlan if lazy else SegmentedPlan
    mode, bits, low = cand[:3]
    if len(cand) == 3:
        return cls(n, ops, renorm_after, mode, bits, low, dtype)
    old = B.qs_get_tunable("plan_beam")
    B.qs_set_tunable("plan_beam", cand[3])
    try:
        return cls(n, ops, renorm_after, mode, bits, low, dtype)
    finally:
        B.qs_set_tunable("plan_beam", old)


def choose_segmented(n: int, ops, renorm_after, dtype: str = "c64", model: Optional[CostModel] = None,
                     cands: Optional[Sequence[Tuple[str, int, int]]] = None, beams: Sequence[int] = BEAMS,
                     lazy: bool = False):
    """The renormalised plan (make_segmented; `lazy` selects the form) whose plans the model predicts fastest in
    sum: every block shape of candidates(n) (or `cands`) at the planner's beam width and at each of `beams`;
    without a model, the greedy shape. Block shapes only: the folded renormalisation rides on complex64 block
    passes, and fused-dense plans of these circuits run at half the block plans' rate. Returns (plan, its
    candidate key, predicted ms or None)."""
    g = greedy_for(n)
    if model is None:
        return make_segmented(n, ops, renorm_after, g, dtype, lazy), g, None
    cur = B.qs_get_tunable("plan_beam")
    best = None
    for cand in (cands or [c for c in candidates(n) if c[0] == "block"]):
        for key in [cand] + [cand + (w,) for w in beams if w != cur]:
            sp = make_segmented(n, ops, renorm_after, key, dtype, lazy)
            t = sum(model.predict_plan_ms(p) for p in sp.plans())
            if best is None or t < best[2]:
                if best is not None:
                    best[0].close()
                best = (sp, key, t)
            else:
                sp.close()
    return best

def main():
    ap = argparse.ArgumentParser(description="Collect pass timings on the GPU and train the cost model.")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--data", default=None, help="save / reuse the timing dataset (.npz)")
    ap.add_argument("--rounds", type=int, default=2, help="rounds of learned planning added to the data")
    args = ap.parse_args()
    fresh = not (args.data and os.path.exists(args.data))  # timings collected in this run (not reused from a file)
    if not fresh:
        d = np.load(args.data, allow_pickle=False)
        X, y = d["X"], d["y"]
    else:
        groups = []
        X, y = collect(training_circuits(), log=lambda m: print(m, flush=True), groups=groups)
        if args.data:
            np.savez(args.data, X=X, y=y, groups=np.array(groups, dtype=np.int32))
    print(f"dataset: {len(y)} passes", flush=True)
    rng = np.random.Generator(np.random.PCG64(7))
    perm = rng.permutation(len(y))
    cut = int(0.85 * len(y))
    tr, va = perm[:cut], perm[cut:]
    m = CostModel()
    m.fit(X[tr], y[tr], epochs=args.epochs, log=lambda s: print(s, flush=True))
    m.fit_more(X[tr], y[tr], epochs=args.epochs // 3, lr=3e-4)
    # rounds of learned planning: the passes the model prefers are timed and added, and the model is trained again
    if fresh:
        circs = training_circuits()
        for r in range(args.rounds):
            X2, y2 = collect_learned(circs, m, log=lambda s: print(s, flush=True))
            pv2 = m.predict_log_ms(X2)
            print(f"round {r}: model error on its own choices: median {np.median(np.abs(np.exp(pv2 - y2) - 1)):.3f},"
                  f" mean log bias {float(np.mean(pv2 - y2)):+.3f}", flush=True)
            X, y = np.concatenate([X, X2]), np.concatenate([y, y2])
            perm = rng.permutation(len(y))
            cut = int(0.85 * len(y))
            tr, va = perm[:cut], perm[cut:]
            m.close()
            m = CostModel()
            m.fit(X[tr], y[tr], epochs=args.epochs, log=lambda s: print(s, flush=True))
            m.fit_more(X[tr], y[tr], epochs=args.epochs // 3, lr=3e-4)
            groups = groups + [(-1 - r, 0)] * len(y2)
        if args.data:
            np.savez(args.data, X=X, y=y, groups=np.array(groups, dtype=np.int32))
    pv = m.predict_log_ms(X[va])
    mse = float(np.mean((pv - y[va]) ** 2))
    rel = float(np.median(np.abs(np.exp(pv - y[va]) - 1)))
    print(f"validation mse(log ms) {mse:.4f}, median relative error {rel:.3f}", flush=True)
    if "groups" in locals() or (args.data and os.path.exists(args.data)):
        g = np.asarray(groups if "groups" in locals() else np.load(args.data)["groups"])
        keep = g[:, 0] >= 0  # the whole-plan candidate groups (learned-plan rounds carry negative ids)
        g = g[keep]
        pall = np.exp(m.predict_log_ms(X[keep]).astype(np.float64))
        tall = np.exp(np.asarray(y[keep], np.float64))
        agree, regret = 0, []
        for gid in np.unique(g[:, 0]):
            sel = g[:, 0] == gid
            cands = np.unique(g[sel, 1])
            pt = np.array([pall[sel & (g[:, 1] == c)].sum() for c in cands])
            tt = np.array([tall[sel & (g[:, 1] == c)].sum() for c in cands])
            agree += int(np.argmin(pt) == np.argmin(tt))
            regret.append(tt[np.argmin(pt)] / tt.min() - 1)
        print(f"plan choice: model picks the fastest candidate in {agree}/{len(regret)} circuit runs, "
              f"mean regret {100 * np.mean(regret):.1f} %", flush=True)
    m.save(args.out)
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
