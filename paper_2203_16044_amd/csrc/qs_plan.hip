// Circuits and execution plans (host C++).
//
// A circuit is an ordered list of operations (Sec. II-A: gates applied in sequence). It can be run plainly --
// one kernel pass per operation, exactly the qs_apply_* calls in order -- or through a plan that groups
// operations into fewer HBM passes:
//   QS_PLAN_BLOCK  LDS block passes: each pass picks a set L of `block_bits` qubits (always containing the
//                  `low_bits` lowest ones) and applies, inside LDS, every pending gate whose qubits lie in L;
//   QS_PLAN_FUSE   dense fused blocks: each pass multiplies the pending gates on at most `block_bits` (<= 6) qubits
//                  into one matrix, run by the register kernel (k <= 4) or the MFMA kernel (k = 5, 6);
//   QS_PLAN_REMAP  the paper's local / global split (Sec. III-B) with fused-swap insertion (Sec. III-D): block passes
//                  only over the lowest `block_bits` physical qubits (contiguous blocks), a logical -> physical
//                  qubit map, fused-swaps that bring a pass's qubits into that range before it, circuit fused-swaps
//                  absorbed into the map, and the identity map restored at the end.
// Both respect the circuit's order: a gate joins a pass only when every earlier gate on its qubits has been
// placed. Fused-swaps and gates too large for a pass run as passes of their own. The plan's final state equals
// the circuit's (up to rounding): no qubit relabelling is left behind.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <vector>

#include "qs_internal.h"

using cd = std::complex<double>;

namespace {

constexpr int kMaxPlanGateQ = 6;  // gates on more qubits (large controlled gates) run through qs_apply_controlled

struct RawOp {
    int kind;  // 0 dense, 1 diag, 2 controlled, 3 fused-swap
    std::vector<int> t, c;
    std::vector<double> m;
    int p = 0, q = 0, s = 0;
};

// planner gate: matrix on an ordered qubit list (matrix bit j <-> q[j]); kind 1 = fused-swap, 2 = opaque raw op
struct PG {
    int kind = 0;
    std::vector<int> q;
    std::vector<cd> m;
    int raw = -1;              // index of the raw op
    std::vector<int> members;  // a fused op: the circuit gates it carries, in the order it applies them
};

std::vector<cd> embed(const PG &g, const std::vector<int> &Q)
{
    const int K = (int)Q.size(), D = 1 << K, k = (int)g.q.size(), d = 1 << k;
    int pos[kMaxPlanGateQ];
    uint32_t gmask = 0;
    for (int j = 0; j < k; ++j) {
        pos[j] = (int)(std::find(Q.begin(), Q.end(), g.q[j]) - Q.begin());
        gmask |= 1u << pos[j];
    }
    std::vector<cd> M((size_t)D * D, cd(0, 0));
    for (int a = 0; a < D; ++a) {
        int sa = 0;
        for (int j = 0; j < k; ++j)
            sa |= ((a >> pos[j]) & 1) << j;
        for (int b = 0; b < D; ++b) {
            if ((a ^ b) & ~gmask)
                continue;
            int sb = 0;
            for (int j = 0; j < k; ++j)
                sb |= ((b >> pos[j]) & 1) << j;
            M[(size_t)a * D + b] = g.m[(size_t)sa * d + sb];
        }
    }
    return M;
}

std::vector<cd> matmul(const std::vector<cd> &A, const std::vector<cd> &B, int D)
{
    std::vector<cd> C((size_t)D * D, cd(0, 0));
    for (int i = 0; i < D; ++i)
        for (int l = 0; l < D; ++l) {
            const cd a = A[(size_t)i * D + l];
            if (a == cd(0, 0))
                continue;
            for (int j = 0; j < D; ++j)
                C[(size_t)i * D + j] += a * B[(size_t)l * D + j];
        }
    return C;
}

bool subset(const std::vector<int> &a, const std::vector<int> &b)
{
    for (int x : a)
        if (std::find(b.begin(), b.end(), x) == b.end())
            return false;
    return true;
}

bool intersects(const std::vector<int> &a, const std::vector<int> &b)
{
    for (int x : a)
        if (std::find(b.begin(), b.end(), x) != b.end())
            return true;
    return false;
}

// re-express a gate on its qubits in ascending order (matrix bits follow)
PG sorted_gate(const PG &g)
{
    PG r = g;
    std::sort(r.q.begin(), r.q.end());
    r.m = embed(g, r.q);
    return r;
}

}  // namespace

struct qs_circuit {
    int n = 0;
    std::vector<RawOp> raw;
    std::vector<PG> gates;
};

struct PlanPass {
    int type = 0;  // 0 block, 1 dense, 2 fused-swap, 3 raw op, 4 relabel (a circuit fused-swap absorbed into the map)
    int b = 0;
    uint64_t lmask = 0;
    BlockMap bm{};
    int op_begin = 0, nops = 0;  // block: fused ops carried
    int stage_begin = 0, nstages = 0;  // block: range in stages
    int sw = 4;                        // block: register stage width (3 or 4)
    BlkMfma mf{};                      // block, complex64: fused stage matrices run on the matrix cores
    // dense
    int k = 0;
    TPos tp{};
    uint64_t tmask = 0;
    std::vector<double> Uh;  // sorted FP64 (kernel arguments for k <= 3)
    size_t mat_off = 0;      // offset in the matrix pool (real elements)
    int p = 0, q = 0, s = 0;
    int raw = -1;
    int ngates = 0;          // circuit gates carried by the pass
    std::vector<int> order;  // their raw-op indices, in the order the pass applies them
    int lstage_begin = -1;   // block: first of the pass's lane-pair stage records (-1: the pass has none)
};

struct qs_plan {
    int n = 0, dtype = QS_C128, mode = 0;
    std::vector<PlanPass> passes;
    std::vector<BlkStage> stages;
    std::vector<BlkStageL> lstages;  // lane-pair form of the stages of eligible passes
    std::vector<BlkStageOp> sops;
    std::vector<double> pool;  // matrices, FP64 (rounded to FP32 on upload for complex64)
    std::vector<RawOp> raw;    // copy: the plan stays valid after the circuit is freed
    BlkStage *dstages = nullptr;
    BlkStageL *dlstages = nullptr;
    void *dpool = nullptr;
    int dev = -1;
    int nfused_ops = 0;
};

namespace {

int add_raw(qs_circuit *c, RawOp &&r, PG &&g)
{
    g.raw = (int)c->raw.size();
    c->raw.push_back(std::move(r));
    c->gates.push_back(std::move(g));
    return QS_OK;
}

int check_list(int n, const int *q, int cnt, uint64_t *mask, const char *what)
{
    uint64_t m = 0;
    for (int j = 0; j < cnt; ++j) {
        if (q[j] < 0 || q[j] >= n)
            return qs_fail(QS_EINVAL, "%s[%d] = %d is outside [0, %d)", what, j, q[j], n);
        if (m & ((uint64_t)1 << q[j]))
            return qs_fail(QS_EINVAL, "%s repeats qubit %d", what, q[j]);
        m |= (uint64_t)1 << q[j];
    }
    *mask = m;
    return QS_OK;
}

// ---- pass formation ----------------------------------------------------------------------------------------
struct Former {
    const qs_circuit &c;
    int b, w, max_block_q, beam;
    std::vector<std::vector<int>> qlist;
    std::vector<size_t> head;

    Former(const qs_circuit &c_, int b_, int w_, int maxq, int beam_)
        : c(c_), b(b_), w(w_), max_block_q(maxq), beam(beam_)
    {
        qlist.assign(c.n, {});
        head.assign(c.n, 0);
        for (size_t g = 0; g < c.gates.size(); ++g)
            for (int q : c.gates[g].q)
                qlist[q].push_back((int)g);
    }
    bool ready(int g, const std::vector<size_t> &h) const
    {
        for (int q : c.gates[g].q)
            if (h[q] >= qlist[q].size() || qlist[q][h[q]] != g)
                return false;
        return true;
    }
    bool blockable(int g) const { return c.gates[g].kind == 0 && (int)c.gates[g].q.size() <= max_block_q; }
    // ready gates, ascending circuit index
    std::vector<int> front(const std::vector<size_t> &h) const
    {
        std::vector<int> f;
        for (int q = 0; q < c.n; ++q)
            if (h[q] < qlist[q].size()) {
                const int g = qlist[q][h[q]];
                if (ready(g, h) && std::find(f.begin(), f.end(), g) == f.end())
                    f.push_back(g);
            }
        std::sort(f.begin(), f.end());
        return f;
    }

    // A candidate pass: its local set L, the gates it takes (in a dependency-respecting order) and the DAG position
    // after them.
    struct Cand {
        std::vector<int> L;
        std::vector<size_t> h;
        std::vector<int> gates;
    };
    // take every ready blockable gate inside L, repeatedly (the result depends only on L and the start position)
    void closure(Cand &s) const
    {
        bool changed = true;
        while (changed) {
            changed = false;
            for (int g : front(s.h))
                if (blockable(g) && subset(c.gates[g].q, s.L)) {
                    for (int q : c.gates[g].q)
                        ++s.h[q];
                    s.gates.push_back(g);
                    changed = true;
                }
        }
    }
    // Grow L from the always-local low qubits. beam == 0: add the ready gate needing the fewest new qubits while
    // L has room. beam >= 1: a beam search over growth steps, keeping the `beam` candidates that take the most
    // gates (fewest qubits on ties); the pass is the candidate taking the most gates once none can grow.
    Cand form_pass() const
    {
        std::vector<Cand> leaves;
        return form_pass(leaves, 1);
    }
    // As above; `leaves` also receives up to `keep` of the final candidates (those that could not grow), most gates
    // first (fewest qubits on ties), distinct local sets: the alternatives a cost model may prefer.
    Cand form_pass(std::vector<Cand> &leaves, int keep) const
    {
        leaves.clear();
        auto offer = [&](const Cand &x) {
            if (x.gates.empty() || keep <= 0)
                return;
            for (const Cand &u : leaves)
                if (u.L == x.L && u.gates.size() == x.gates.size())
                    return;
            leaves.push_back(x);
            std::stable_sort(leaves.begin(), leaves.end(), [](const Cand &a, const Cand &b2) {
                return a.gates.size() != b2.gates.size() ? a.gates.size() > b2.gates.size() : a.L.size() < b2.L.size();
            });
            if ((int)leaves.size() > keep)
                leaves.pop_back();
        };
        Cand s0;
        for (int q = 0; q < w && q < c.n; ++q)
            s0.L.push_back(q);
        s0.h = head;
        closure(s0);
        if (beam == 0) {
            for (;;) {
                int best = -1, bestnew = 1 << 30;
                for (int g : front(s0.h)) {
                    if (!blockable(g))
                        continue;
                    int nw = 0;
                    for (int q : c.gates[g].q)
                        nw += std::find(s0.L.begin(), s0.L.end(), q) == s0.L.end();
                    if ((int)s0.L.size() + nw <= b && nw < bestnew) {
                        best = g;
                        bestnew = nw;
                    }
                }
                if (best < 0) {
                    offer(s0);
                    return s0;
                }
                for (int q : c.gates[best].q)
                    if (std::find(s0.L.begin(), s0.L.end(), q) == s0.L.end())
                        s0.L.push_back(q);
                closure(s0);
            }
        }
        std::vector<Cand> cur{s0};
        Cand best = s0;
        while (!cur.empty()) {
            std::vector<Cand> nxt;
            for (const Cand &st : cur) {
                bool grown = false;
                for (int g : front(st.h)) {
                    if (!blockable(g))
                        continue;
                    int nw = 0;
                    for (int q : c.gates[g].q)
                        nw += std::find(st.L.begin(), st.L.end(), q) == st.L.end();
                    if (nw == 0 || (int)st.L.size() + nw > b)
                        continue;
                    Cand t = st;
                    for (int q : c.gates[g].q)
                        if (std::find(t.L.begin(), t.L.end(), q) == t.L.end())
                            t.L.push_back(q);
                    std::sort(t.L.begin(), t.L.end());
                    closure(t);
                    nxt.push_back(std::move(t));
                    grown = true;
                }
                if (!grown) {
                    offer(st);
                    if (st.gates.size() > best.gates.size())
                        best = st;
                }
            }
            std::stable_sort(nxt.begin(), nxt.end(), [](const Cand &x, const Cand &y) {
                return x.gates.size() != y.gates.size() ? x.gates.size() > y.gates.size() : x.L.size() < y.L.size();
            });
            cur.clear();
            for (Cand &t : nxt) {
                bool dup = false;
                for (const Cand &u : cur)
                    if (u.L == t.L) {
                        dup = true;
                        break;
                    }
                if (!dup)
                    cur.push_back(std::move(t));
                if ((int)cur.size() >= beam)
                    break;
            }
        }
        return best;
    }

    void run(std::vector<std::pair<std::vector<int>, std::vector<int>>> &out_passes, std::vector<int> &singles_order)
    {
        // out_passes: (L sorted, gates) for blockable passes; singles are encoded as L empty + one gate
        size_t remaining = c.gates.size();
        while (remaining) {
            Cand p = form_pass();
            if (!p.gates.empty()) {
                std::sort(p.L.begin(), p.L.end());
                head = p.h;
                remaining -= p.gates.size();
                out_passes.emplace_back(p.L, p.gates);
                continue;
            }
            // nothing blockable is ready: emit the earliest ready non-blockable gate on its own
            std::vector<int> f = front(head);
            if (f.empty())
                break;  // cannot happen for a well-formed circuit
            const int g = f[0];
            for (int q : c.gates[g].q)
                ++head[q];
            --remaining;
            out_passes.emplace_back(std::vector<int>(), std::vector<int>{g});
            singles_order.push_back(g);
        }
    }
};

// Merge gates of one pass: later gates into an earlier op on a superset of their qubits (nothing in between
// touching them), then earlier small ops forward into a later superset op.
std::vector<PG> fuse_pass(const qs_circuit &c, const std::vector<int> &gates)
{
    std::vector<PG> out;
    for (int gi : gates) {
        const PG &g = c.gates[gi];
        bool merged = false;
        for (int h = (int)out.size() - 1; h >= 0; --h) {
            if (subset(g.q, out[h].q)) {
                out[h].m = matmul(embed(g, out[h].q), out[h].m, 1 << out[h].q.size());
                out[h].members.push_back(gi);
                merged = true;
                break;
            }
            if (intersects(g.q, out[h].q))
                break;
        }
        if (!merged) {
            out.push_back(g);
            out.back().members.assign(1, gi);
        }
    }
    for (size_t i = 0; i < out.size();) {
        bool moved = false;
        for (size_t j = i + 1; j < out.size(); ++j) {
            if (subset(out[i].q, out[j].q)) {
                out[j].m = matmul(out[j].m, embed(out[i], out[j].q), 1 << out[j].q.size());
                out[j].members.insert(out[j].members.begin(), out[i].members.begin(), out[i].members.end());
                out.erase(out.begin() + i);
                moved = true;
                break;
            }
            if (intersects(out[i].q, out[j].q))
                break;
        }
        if (!moved)
            ++i;
    }
    return out;
}

void push_matrix(std::vector<double> &pool, const std::vector<cd> &m)
{
    for (const cd &z : m) {
        pool.push_back(z.real());
        pool.push_back(z.imag());
    }
}

int make_dense_pass(qs_plan *P, const PG &g, PlanPass &pp)
{
    const PG sg = sorted_gate(g);
    pp.type = 1;
    pp.k = (int)sg.q.size();
    pp.tmask = 0;
    for (int j = 0; j < pp.k; ++j) {
        pp.tp.tpos[j] = sg.q[j];
        pp.tmask |= (uint64_t)1 << sg.q[j];
    }
    pp.Uh.clear();
    for (const cd &z : sg.m) {
        pp.Uh.push_back(z.real());
        pp.Uh.push_back(z.imag());
    }
    pp.mat_off = P->pool.size();
    push_matrix(P->pool, sg.m);
    return QS_OK;
}

int run_raw(qs_state *st, const RawOp &r)
{
    switch (r.kind) {
    case 0: return qs_apply_gate(st, r.t.data(), (int)r.t.size(), r.m.data());
    case 1: return qs_apply_diag(st, r.t.data(), (int)r.t.size(), r.m.data());
    case 2: return qs_apply_controlled(st, r.c.data(), (int)r.c.size(), r.t.data(), (int)r.t.size(), r.m.data());
    default: return qs_fused_swap(st, r.p, r.q, r.s);
    }
}

// Each buffer is recorded in the plan as soon as it exists, so upload() can release whatever a failed attempt left.
int upload_tables(qs_plan *P)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(P->stages.size(), 1) * sizeof(BlkStage));
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipMalloc(plan stages)");
    P->dstages = static_cast<BlkStage *>(p);
    if (!P->stages.empty())
        QS_HIP(hipMemcpy(P->dstages, P->stages.data(), P->stages.size() * sizeof(BlkStage), hipMemcpyHostToDevice));
    if (!P->lstages.empty()) {
        p = nullptr;
        e = hipMalloc(&p, P->lstages.size() * sizeof(BlkStageL));
        if (e != hipSuccess)
            return qs_hip_fail(e, "hipMalloc(plan lane-pair stages)");
        P->dlstages = static_cast<BlkStageL *>(p);
        QS_HIP(hipMemcpy(P->dlstages, P->lstages.data(), P->lstages.size() * sizeof(BlkStageL),
                         hipMemcpyHostToDevice));
    }
    // 64 zero elements past the end: slack for scalar loads that the kernels issue in whole 64-byte lines
    const size_t npool = P->pool.size() + 64;
    const size_t esz = P->dtype == QS_C128 ? sizeof(double) : sizeof(float);
    p = nullptr;
    e = hipMalloc(&p, npool * esz);
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipMalloc(plan matrices)");
    P->dpool = p;
    if (P->dtype == QS_C128) {
        std::vector<double> d(P->pool.begin(), P->pool.end());
        d.resize(npool, 0.0);
        QS_HIP(hipMemcpy(P->dpool, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(P->pool.begin(), P->pool.end());
        f.resize(npool, 0.0f);
        QS_HIP(hipMemcpy(P->dpool, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    }
    return QS_OK;
}

int upload(qs_plan *P)
{
    int dev = 0;
    QS_HIP(hipGetDevice(&dev));
    if (P->dstages || P->dpool) {
        if (dev == P->dev)
            return QS_OK;
        return qs_fail(QS_EINVAL, "qs_plan_run: plan was uploaded to device %d, current device is %d", P->dev, dev);
    }
    if (int rc = upload_tables(P)) {  // leave nothing half-uploaded: a later run starts over
        if (P->dstages)
            (void)hipFree(P->dstages);
        if (P->dlstages)
            (void)hipFree(P->dlstages);
        if (P->dpool)
            (void)hipFree(P->dpool);
        P->dstages = nullptr;
        P->dlstages = nullptr;
        P->dpool = nullptr;
        return rc;
    }
    P->dev = dev;
    return QS_OK;
}

}  // namespace

extern "C" {

QS_API int qs_circuit_create(qs_circuit **out, int n)
{
    qs_clear_error();
    if (!out)
        return qs_fail(QS_EINVAL, "qs_circuit_create: out is NULL");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS)
        return qs_fail(QS_EINVAL, "qs_circuit_create: n = %d outside [1, %d]", n, QS_MAX_QUBITS);
    qs_circuit *c = new (std::nothrow) qs_circuit();
    if (!c)
        return qs_fail(QS_ENOMEM, "qs_circuit_create: out of host memory");
    c->n = n;
    *out = c;
    return QS_OK;
}

QS_API int qs_circuit_free(qs_circuit *c)
{
    qs_clear_error();
    if (!c)
        return qs_fail(QS_EINVAL, "qs_circuit_free: NULL circuit");
    delete c;
    return QS_OK;
}

QS_API int qs_circuit_add_gate(qs_circuit *c, const int *targets, int k, const double *U)
{
    qs_clear_error();
    if (!c || !targets || !U)
        return qs_fail(QS_EINVAL, "qs_circuit_add_gate: NULL argument");
    if (k < 1 || k > QS_MAX_K || k > c->n)
        return qs_fail(QS_EINVAL, "qs_circuit_add_gate: k = %d outside [1, min(%d, n)]", k, QS_MAX_K);
    uint64_t m;
    if (int rc = check_list(c->n, targets, k, &m, "targets"))
        return rc;
    const int D = 1 << k;
    RawOp r;
    r.kind = 0;
    r.t.assign(targets, targets + k);
    r.m.assign(U, U + 2 * D * D);
    PG g;
    g.q = r.t;
    g.m.resize((size_t)D * D);
    for (int i = 0; i < D * D; ++i)
        g.m[i] = cd(U[2 * i], U[2 * i + 1]);
    return add_raw(c, std::move(r), std::move(g));
}

QS_API int qs_circuit_add_diag(qs_circuit *c, const int *targets, int k, const double *d)
{
    qs_clear_error();
    if (!c || !targets || !d)
        return qs_fail(QS_EINVAL, "qs_circuit_add_diag: NULL argument");
    if (k < 1 || k > QS_MAX_DIAG_K || k > c->n)
        return qs_fail(QS_EINVAL, "qs_circuit_add_diag: k = %d outside [1, min(%d, n)]", k, QS_MAX_DIAG_K);
    uint64_t m;
    if (int rc = check_list(c->n, targets, k, &m, "targets"))
        return rc;
    const int D = 1 << k;
    RawOp r;
    r.kind = 1;
    r.t.assign(targets, targets + k);
    r.m.assign(d, d + 2 * D);
    PG g;
    g.q = r.t;
    if (k <= kMaxPlanGateQ) {
        g.m.assign((size_t)D * D, cd(0, 0));
        for (int a = 0; a < D; ++a)
            g.m[(size_t)a * D + a] = cd(d[2 * a], d[2 * a + 1]);
    } else {
        g.kind = 2;
    }
    return add_raw(c, std::move(r), std::move(g));
}

QS_API int qs_circuit_add_controlled(qs_circuit *c, const int *controls, int nc, const int *targets, int k,
                                     const double *U)
{
    qs_clear_error();
    if (!c || !controls || !targets || !U)
        return qs_fail(QS_EINVAL, "qs_circuit_add_controlled: NULL argument");
    if (k < 1 || k > QS_MAX_K || nc < 1 || nc > QS_MAX_CONTROLS || nc + k > c->n)
        return qs_fail(QS_EINVAL, "qs_circuit_add_controlled: counts out of range (c = %d, k = %d, n = %d)", nc, k,
                       c->n);
    uint64_t tm, cm;
    if (int rc = check_list(c->n, targets, k, &tm, "targets"))
        return rc;
    if (int rc = check_list(c->n, controls, nc, &cm, "controls"))
        return rc;
    if (tm & cm)
        return qs_fail(QS_EINVAL, "qs_circuit_add_controlled: a control is also a target");
    const int D = 1 << k;
    RawOp r;
    r.kind = 2;
    r.t.assign(targets, targets + k);
    r.c.assign(controls, controls + nc);
    r.m.assign(U, U + 2 * D * D);
    PG g;
    g.q = r.t;
    g.q.insert(g.q.end(), controls, controls + nc);
    if (k + nc <= kMaxPlanGateQ) {
        const int DD = 1 << (k + nc);
        g.m.assign((size_t)DD * DD, cd(0, 0));
        const int cfull = ((1 << nc) - 1) << k;
        for (int a = 0; a < DD; ++a) {
            if ((a & cfull) != cfull) {
                g.m[(size_t)a * DD + a] = cd(1, 0);
                continue;
            }
            for (int b2 = 0; b2 < D; ++b2)
                g.m[(size_t)a * DD + (cfull | b2)] = cd(U[2 * ((a & (D - 1)) * D + b2)], U[2 * ((a & (D - 1)) * D + b2) + 1]);
        }
    } else {
        g.kind = 2;
    }
    return add_raw(c, std::move(r), std::move(g));
}

QS_API int qs_circuit_add_fused_swap(qs_circuit *c, int p, int q, int s)
{
    qs_clear_error();
    if (!c)
        return qs_fail(QS_EINVAL, "qs_circuit_add_fused_swap: NULL circuit");
    if (s < 0 || p < 0 || q < 0 || p + s > c->n || q + s > c->n || std::min(p, q) + s > std::max(p, q))
        return qs_fail(QS_EINVAL, "qs_circuit_add_fused_swap: invalid (p=%d q=%d s=%d) for n = %d", p, q, s, c->n);
    if (s == 0)
        return QS_OK;
    RawOp r;
    r.kind = 3;
    r.p = p;
    r.q = q;
    r.s = s;
    PG g;
    g.kind = 1;
    for (int j = 0; j < s; ++j) {
        g.q.push_back(p + j);
        g.q.push_back(q + j);
    }
    return add_raw(c, std::move(r), std::move(g));
}

QS_API int qs_circuit_size(const qs_circuit *c, int *nops)
{
    qs_clear_error();
    if (!c || !nops)
        return qs_fail(QS_EINVAL, "qs_circuit_size: NULL argument");
    *nops = (int)c->raw.size();
    return QS_OK;
}

QS_API int qs_circuit_run(qs_state *st, const qs_circuit *c)
{
    qs_clear_error();
    if (!st || !c)
        return qs_fail(QS_EINVAL, "qs_circuit_run: NULL argument");
    if (c->n != st->n)
        return qs_fail(QS_EINVAL, "qs_circuit_run: circuit has %d qubits, state has %d", c->n, st->n);
    for (const RawOp &r : c->raw)
        if (int rc = run_raw(st, r))
            return rc;
    return QS_OK;
}

}  // extern "C"

namespace {
int plan_create(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts, int stage_width,
                const qs_plan_model *model, bool beam_search = false);
}

extern "C" QS_API int qs_plan_create(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts)
{
    qs_clear_error();
    return plan_create(out, c, opts, qs_tunables().block_stage_width, nullptr, qs_tunables().plan_beam_search != 0);
}

extern "C" QS_API int qs_plan_create_learned(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts,
                                             const qs_plan_model *m)
{
    qs_clear_error();
    if (!out || !c || !opts || !m || !m->model || !m->mean || !m->std || !m->shape_bits || !m->shape_low)
        return qs_fail(QS_EINVAL, "qs_plan_create_learned: NULL argument");
    *out = nullptr;
    if (opts->mode != QS_PLAN_BLOCK)
        return qs_fail(QS_EINVAL, "qs_plan_create_learned: mode must be QS_PLAN_BLOCK");
    if (m->nshapes < 1 || m->nshapes > 16 || m->per_shape < 1 || m->per_shape > 8 || m->gate_slack < 0 ||
        m->lookahead < 0 || m->lookahead > 1)
        return qs_fail(QS_EINVAL,
                       "qs_plan_create_learned: nshapes = %d, per_shape = %d, gate_slack = %d or lookahead = %d invalid",
                       m->nshapes, m->per_shape, m->gate_slack, m->lookahead);
    for (int i = 0; i < m->nshapes; ++i)
        if (m->shape_bits[i] < 10 || m->shape_bits[i] > kMaxBlockBits || m->shape_bits[i] > c->n ||
            m->shape_low[i] < 0 || m->shape_low[i] > m->shape_bits[i])
            return qs_fail(QS_EINVAL, "qs_plan_create_learned: shape %d (%d bits, %d low) invalid for %d qubits", i,
                           m->shape_bits[i], m->shape_low[i], c->n);
    if (qs_mlp_nin(m->model) != QS_PLAN_NFEAT)
        return qs_fail(QS_EINVAL, "qs_plan_create_learned: the model takes %d inputs, not %d",
                       qs_mlp_nin(m->model), QS_PLAN_NFEAT);
    for (int j = 0; j < QS_PLAN_NFEAT; ++j)
        if (!(m->std[j] > 0.0f))
            return qs_fail(QS_EINVAL, "qs_plan_create_learned: std[%d] is not positive", j);
    qs_plan_opts o = *opts;
    o.block_bits = m->shape_bits[0];
    o.low_bits = m->shape_low[0];
    return plan_create(out, c, &o, 4, m);
}

namespace {
int append_pass(qs_plan *P, const qs_circuit *c, int mode, const std::vector<int> &L, const std::vector<int> &gs, int b,
                int stage_width);

// Lane-pair records (BlkStageL) of a pass's 4-position stages, for the 512-thread complex128 kernel of 12-qubit
// blocks, when every op acts on one or two positions. In each stage the lane starts on the position whose first
// use comes last; an op on the lane's position first exchanges it with the register position, among those the op
// leaves alone, whose next use comes last (fewest exchanges ahead). Register bits 0..2 hold the other positions in
// ascending order at the start; each op's matrix is appended to the pool in the bit order of its register bits.
void build_lane_stages(qs_plan *P, PlanPass &pp, const std::vector<std::vector<int>> &members,
                       const std::vector<PG> &sorted_ops)
{
    for (int t = 0; t < pp.nstages; ++t) {
        const BlkStage &st = P->stages[pp.stage_begin + t];
        if (st.nops < 1)
            return;
        for (int o = 0; o < st.nops; ++o)
            if (__builtin_popcount((st.masks >> (4 * o)) & 15u) > 2)
                return;
    }
    pp.lstage_begin = (int)P->lstages.size();
    for (int t = 0; t < pp.nstages; ++t) {
        const BlkStage &st = P->stages[pp.stage_begin + t];
        BlkStageL L{};
        for (int j = 0; j < pp.b - 4; ++j)
            L.order[j] = st.order[j];
        L.nops = st.nops;
        std::vector<uint32_t> pm(st.nops);
        for (int o = 0; o < st.nops; ++o)
            pm[o] = (st.masks >> (4 * o)) & 15u;
        auto next_use = [&](int j, int from) {
            for (int o = from; o < st.nops; ++o)
                if ((pm[o] >> j) & 1)
                    return o;
            return st.nops;
        };
        int lane = 0;
        for (int j = 1; j < 4; ++j)
            if (next_use(j, 0) > next_use(lane, 0))
                lane = j;
        int reg_of[4];
        for (int j = 0, r = 0; j < 4; ++j)
            reg_of[j] = j == lane ? -1 : r++;
        auto placement = [&](uint32_t *tab, uint32_t &lane_off) {
            for (int a = 0; a < 8; ++a) {
                uint32_t m = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != lane)
                        m |= (uint32_t)((a >> reg_of[j]) & 1) << j;
                tab[a] = st.soff[m];
            }
            lane_off = st.soff[1u << lane];
        };
        placement(L.rd, L.rd_lane);
        L.mat_base = (uint32_t)P->pool.size();
        for (int o = 0; o < st.nops; ++o) {
            if ((pm[o] >> lane) & 1) {
                int best = -1;
                for (int j = 0; j < 4; ++j)
                    if (j != lane && !((pm[o] >> j) & 1) && (best < 0 || next_use(j, o + 1) > next_use(best, o + 1)))
                        best = j;
                const int r = reg_of[best];
                reg_of[lane] = r;
                reg_of[best] = -1;
                lane = best;
                L.swaps |= (uint32_t)(r + 1) << (2 * o);
            }
            int regs[2], nr = 0;  // register bits of the op's positions, in ascending position order
            uint32_t rm = 0;
            for (int j = 0; j < 4; ++j)
                if ((pm[o] >> j) & 1) {
                    regs[nr++] = reg_of[j];
                    rm |= 1u << reg_of[j];
                }
            L.masks |= rm << (4 * o);
            const std::vector<cd> &U = sorted_ops[members[t][o]].m;
            if (nr == 2 && regs[0] > regs[1]) {  // matrix bits in register order: exchange index bits 0 and 1
                std::vector<cd> V(16);
                auto sw = [](int x) { return ((x & 1) << 1) | ((x >> 1) & 1); };
                for (int a = 0; a < 4; ++a)
                    for (int b2 = 0; b2 < 4; ++b2)
                        V[a * 4 + b2] = U[sw(a) * 4 + sw(b2)];
                push_matrix(P->pool, V);
            } else {
                push_matrix(P->pool, U);
            }
        }
        placement(L.wr, L.wr_lane);
        P->lstages.push_back(L);
    }
}

struct PassSpec {
    std::vector<int> L;      // local set (empty: a single non-blockable gate)
    std::vector<int> gates;  // circuit gates in application order
    int b;                   // block bits of the pass
};

// Pass formation driven by the cost model: at every step, candidate passes of every shape are built (as the plan
// would run them), scored by predicted time per circuit gate, and the cheapest is kept. Gates that no block can
// carry are emitted on their own, as the greedy formation does.
int learned_passes(const qs_circuit &c, int dtype, const qs_plan_model &M, int stage_width, std::vector<PassSpec> &out)
{
    const int beam = std::max(1, qs_tunables().plan_beam.load());
    std::vector<Former> F;
    for (int i = 0; i < M.nshapes; ++i)
        F.emplace_back(c, M.shape_bits[i], M.shape_low[i], kMaxBlockOpK, beam);
    std::vector<size_t> head(c.n, 0);
    size_t remaining = c.gates.size();
    qs_plan tmp;
    tmp.n = c.n;
    tmp.dtype = dtype;
    tmp.mode = QS_PLAN_BLOCK;
    std::vector<Former::Cand> leaves, cands;
    std::vector<int> cand_b;
    std::vector<float> X, Y;
    while (remaining) {
        cands.clear();
        cand_b.clear();
        for (int i = 0; i < M.nshapes; ++i) {
            F[i].head = head;
            F[i].form_pass(leaves, M.per_shape);
            for (Former::Cand &l : leaves) {
                cands.push_back(std::move(l));
                cand_b.push_back(M.shape_bits[i]);
            }
        }
        if (cands.empty()) {  // nothing blockable is ready: the earliest ready gate runs on its own
            std::vector<int> f = F[0].front(head);
            if (f.empty())
                break;  // cannot happen for a well-formed circuit
            const int g = f[0];
            for (int q : c.gates[g].q)
                ++head[q];
            --remaining;
            out.push_back({std::vector<int>(), std::vector<int>{g}, 0});
            continue;
        }
        // candidates that carry too few gates are dropped before the model is asked
        {
            size_t most = 0;
            for (const Former::Cand &x : cands)
                most = std::max(most, x.gates.size());
            size_t keep = 0;
            for (size_t k = 0; k < cands.size(); ++k)
                if (cands[k].gates.size() + (size_t)M.gate_slack >= most) {
                    if (keep != k) {
                        cands[keep] = std::move(cands[k]);
                        cand_b[keep] = cand_b[k];
                    }
                    ++keep;
                }
            cands.resize(keep);
            cand_b.resize(keep);
        }
        int pick = 0;
        if (cands.size() > 1) {
            const int nc = (int)cands.size();
            // rows 0..nc-1: the candidates; with lookahead, rows nc..2nc-1: the pass that would follow each
            std::vector<Former::Cand> follow(M.lookahead ? nc : 0);
            std::vector<int> follow_b(follow.size(), M.shape_bits[0]);
            for (int k = 0; k < (int)follow.size(); ++k) {
                F[0].head = cands[k].h;
                follow[k] = F[0].form_pass();
            }
            const int rows = nc + (int)follow.size();
            X.assign((size_t)rows * QS_PLAN_NFEAT, 0.0f);
            Y.assign(rows, 0.0f);
            for (int k = 0; k < rows; ++k) {
                const Former::Cand &cd = k < nc ? cands[k] : follow[k - nc];
                if (cd.gates.empty())
                    continue;  // nothing blockable follows: no time added
                std::vector<int> L = cd.L;
                std::sort(L.begin(), L.end());
                tmp.passes.clear();
                tmp.stages.clear();
                tmp.sops.clear();
                tmp.pool.clear();
                if (int rc = append_pass(&tmp, &c, QS_PLAN_BLOCK, L, cd.gates, k < nc ? cand_b[k] : follow_b[k - nc],
                                         stage_width))
                    return rc;
                float *x = &X[(size_t)k * QS_PLAN_NFEAT];
                if (int rc = qs_plan_features(&tmp, 0, x))
                    return rc;
                for (int j = 0; j < QS_PLAN_NFEAT; ++j)
                    x[j] = (x[j] - M.mean[j]) / M.std[j];
            }
            for (int k0 = 0; k0 < rows; k0 += 4096)
                if (int rc = qs_mlp_predict(M.model, &X[(size_t)k0 * QS_PLAN_NFEAT], std::min(4096, rows - k0), &Y[k0]))
                    return rc;
            double best = 0.0;
            for (int k = 0; k < nc; ++k) {
                double t = std::exp((double)Y[k]), g = (double)cands[k].gates.size();
                if (!follow.empty() && !follow[k].gates.empty()) {
                    t += std::exp((double)Y[nc + k]);
                    g += (double)follow[k].gates.size();
                }
                if (k == 0 || t / g < best) {
                    best = t / g;
                    pick = k;
                }
            }
        }
        Former::Cand &ch = cands[pick];
        std::sort(ch.L.begin(), ch.L.end());
        head = ch.h;
        remaining -= ch.gates.size();
        out.push_back({ch.L, ch.gates, cand_b[pick]});
    }
    return QS_OK;
}

// Append one pass to P: a single non-blockable gate (L empty), a fused dense block (FUSE mode) or an LDS block pass
// over the local set L (padded to b qubits) applying `gs` in the given order.
int append_pass(qs_plan *P, const qs_circuit *c, int mode, const std::vector<int> &L, const std::vector<int> &gs, int b,
                int stage_width)
{
    PlanPass pp;
    pp.ngates = (int)gs.size();
    if (L.empty()) {  // a single non-blockable gate
        const PG &g = c->gates[gs[0]];
        pp.order.assign(1, g.raw);
        if (g.kind == 1) {
            pp.type = 2;
            const RawOp &r = c->raw[g.raw];
            pp.p = std::min(r.p, r.q);
            pp.q = std::max(r.p, r.q);
            pp.s = r.s;
        } else if (g.kind == 2 || (int)g.q.size() > QS_MAX_K) {
            pp.type = 3;
            pp.raw = g.raw;
        } else {
            make_dense_pass(P, g, pp);
        }
        P->passes.push_back(std::move(pp));
        return QS_OK;
    }
    if (mode == QS_PLAN_FUSE) {
        PG blk;
        blk.q = L;
        const int D = 1 << L.size();
        blk.m.assign((size_t)D * D, cd(0, 0));
        for (int a = 0; a < D; ++a)
            blk.m[(size_t)a * D + a] = cd(1, 0);
        for (int gi : gs) {
            blk.m = matmul(embed(c->gates[gi], L), blk.m, D);
            pp.order.push_back(c->gates[gi].raw);
        }
        make_dense_pass(P, blk, pp);
        P->nfused_ops += 1;
        P->passes.push_back(std::move(pp));
        return QS_OK;
    }
    // LDS block pass
    pp.type = 0;
    pp.b = b;
    // pad L to b qubits with unused low qubits (any qubits work; low ones keep segments long)
    std::vector<int> LL = L;
    for (int q = 0; (int)LL.size() < b && q < c->n; ++q)
        if (std::find(LL.begin(), LL.end(), q) == LL.end())
            LL.push_back(q);
    std::sort(LL.begin(), LL.end());
    pp.lmask = 0;
    pp.bm.b = b;
    for (int t = 0; t < b; ++t) {
        pp.bm.lpos[t] = LL[t];
        pp.lmask |= (uint64_t)1 << LL[t];
    }
    std::vector<PG> fused = fuse_pass(*c, gs);
    pp.nops = (int)fused.size();
    // local positions of every fused op (ascending, as its sorted matrix expects)
    std::vector<PG> sorted_ops;
    std::vector<uint32_t> posmask;
    for (const PG &f : fused) {
        sorted_ops.push_back(sorted_gate(f));
        uint32_t pm = 0;
        for (int q : sorted_ops.back().q)
            pm |= 1u << (int)(std::find(LL.begin(), LL.end(), q) - LL.begin());
        posmask.push_back(pm);
    }
    // stages of at most W positions (W = 3 only where a 512-thread kernel exists). A stage is filled by repeatedly
    // taking a ready op (every earlier op sharing a position placed) that keeps it within W positions, fewest new
    // first. With stage_pack 1 each ready op seeds a candidate stage filled that way, and the candidate whose
    // remaining ops need the fewest stages under the plain rule wins (ties: more ops; then the earliest seed).
    const int W = (stage_width == 3 && (b == 12 || b == 13)) ? 3 : 4;
    pp.sw = W;
    const int nf = (int)fused.size();
    auto is_ready = [&](const std::vector<char> &pl, int i) {
        if (pl[i])
            return false;
        for (int j = 0; j < i; ++j)
            if (!pl[j] && (posmask[j] & posmask[i]))
                return false;
        return true;
    };
    auto fill = [&](std::vector<char> &pl, uint32_t &S, std::vector<int> &members) {
        while ((int)members.size() < kStageMaxOps) {
            int best = -1, bestnew = 99;
            for (int i = 0; i < nf; ++i) {
                if (!is_ready(pl, i))
                    continue;
                const int nw = __builtin_popcount(posmask[i] & ~S);
                if (__builtin_popcount(S | posmask[i]) <= W && nw < bestnew) {
                    best = i;
                    bestnew = nw;
                }
            }
            if (best < 0)
                break;
            pl[best] = 1;
            S |= posmask[best];
            members.push_back(best);
        }
    };
    auto greedy_stages = [&](std::vector<char> pl) {
        int cnt = 0;
        for (;;) {
            bool left = false;
            for (char c : pl)
                left |= !c;
            if (!left)
                return cnt;
            uint32_t S = 0;
            std::vector<int> m;
            fill(pl, S, m);
            ++cnt;
        }
    };
    const bool lookahead = qs_tunables().stage_pack != 0;
    std::vector<char> placed(nf, 0);
    int left = nf;
    pp.stage_begin = (int)P->stages.size();
    std::vector<std::vector<int>> stage_members;  // fused-op indices of each stage of this pass, in order
    while (left) {
        uint32_t S = 0;
        std::vector<int> members;
        if (!lookahead) {
            fill(placed, S, members);
        } else {
            int best_rest = 1 << 30;
            std::vector<char> best_pl;
            for (int i = 0; i < nf; ++i) {
                if (!is_ready(placed, i))
                    continue;
                std::vector<char> pl = placed;
                pl[i] = 1;
                uint32_t s2 = posmask[i];
                std::vector<int> m{i};
                fill(pl, s2, m);
                const int rest = greedy_stages(pl);
                if (rest < best_rest || (rest == best_rest && m.size() > members.size())) {
                    best_rest = rest;
                    best_pl = pl;
                    members = m;
                    S = s2;
                }
            }
            placed = best_pl;
        }
        left -= (int)members.size();
        for (int p = 0; __builtin_popcount(S) < W && p < b; ++p)
            S |= 1u << p;  // pad with unused positions
        BlkStage stg{};
        int j = 0;
        for (int p = 0; p < b; ++p)
            if ((S >> p) & 1)
                stg.pos[j++] = p;
        // group-counter bit order over the other positions: one position of each residue class mod 4 first
        {
            std::vector<int> rest;
            for (int p = 0; p < b; ++p)
                if (!((S >> p) & 1))
                    rest.push_back(p);
            std::vector<int> ord;
            for (int cls = 0; cls < 4; ++cls)
                for (size_t r = 0; r < rest.size(); ++r)
                    if (rest[r] % 4 == cls) {
                        ord.push_back(rest[r]);
                        rest.erase(rest.begin() + r);
                        break;
                    }
            ord.insert(ord.end(), rest.begin(), rest.end());
            for (int t = 0; t < b - W; ++t)
                stg.order[t] = ord[t];
        }
        for (int a = 0; a < (1 << W); ++a) {
            uint32_t o = 0;
            for (int jj = 0; jj < W; ++jj)
                o |= ((uint32_t)(a >> jj) & 1u) << stg.pos[jj];
            stg.soff[a] = blk_swz(o) * (uint32_t)amp_bytes(P->dtype);
        }
        stage_members.push_back(members);
        stg.op_begin = (int)P->sops.size();
        stg.nops = (int)members.size();
        stg.mat_base = (uint32_t)P->pool.size();
        for (size_t o = 0; o < members.size(); ++o) {
            const int i = members[o];
            BlkStageOp so{};
            for (int t = 0; t < W; ++t)
                if ((posmask[i] >> stg.pos[t]) & 1)
                    so.mask |= 1 << t;
            so.mat_off = (uint32_t)P->pool.size();
            push_matrix(P->pool, sorted_ops[i].m);
            P->sops.push_back(so);
            stg.masks |= (uint32_t)so.mask << (4 * o);
        }
        stg.mfma = -1;
        P->stages.push_back(stg);
    }
    pp.nstages = (int)P->stages.size() - pp.stage_begin;
    for (const std::vector<int> &members : stage_members)
        for (int i : members)
            for (int gi : fused[i].members)
                pp.order.push_back(c->gates[gi].raw);
    if (P->dtype == QS_C128 && W == 4 && b == 12 && qs_tunables().block_lanes)
        build_lane_stages(P, pp, stage_members, sorted_ops);
    // complex64: the pass's stages with the most arithmetic (at least that of mfma_stage_ops 2-qubit ops; up to
    // kMaxMfmaStages, the LDS they may take) become dense 16 x 16 products on the matrix cores. Op by op a
    // k-qubit op costs 2^(k+2) FMAs per amplitude; the dense product costs 64, but FP32 MFMA runs at twice the
    // FP32 FMA rate, so it pays from about three 2-qubit ops' worth on. The product of the stage's ops is formed
    // here in FP64 (op o first), with stage index bit j <-> pos[j] as in the per-op masks.
    const int mfma_ops = qs_tunables().mfma_stage_ops;
    if (P->dtype == QS_C64 && W == 4 && mfma_ops > 0) {
        auto weight = [&](int t) {  // FMAs per amplitude of stage t, op by op
            const BlkStage &st = P->stages[pp.stage_begin + t];
            int w = 0;
            for (int o = 0; o < st.nops; ++o)
                w += 4 << __builtin_popcount((st.masks >> (4 * o)) & 15u);
            return w;
        };
        std::vector<int> pick;
        for (int t = 0; t < pp.nstages; ++t)
            if (weight(t) >= 16 * mfma_ops)
                pick.push_back(t);
        std::stable_sort(pick.begin(), pick.end(), [&](int x, int y) { return weight(x) > weight(y); });
        if ((int)pick.size() > kMaxMfmaStages)
            pick.resize(kMaxMfmaStages);
        std::sort(pick.begin(), pick.end());
        for (int t : pick) {
            BlkStage &st = P->stages[pp.stage_begin + t];
            std::vector<cd> M(256, cd(0, 0));
            for (int r = 0; r < 16; ++r)
                M[r * 16 + r] = 1;
            for (int o = 0; o < st.nops; ++o) {
                const int mk = (int)((st.masks >> (4 * o)) & 15u);
                const std::vector<cd> &U = sorted_ops[stage_members[t][o]].m;
                const int D = 1 << __builtin_popcount(mk);
                auto sub = [mk](int x) {  // bits of x at the op's positions, packed (j-th set bit -> bit j)
                    int v = 0, jj = 0;
                    for (int q = 0; q < 4; ++q)
                        if ((mk >> q) & 1)
                            v |= ((x >> q) & 1) << jj++;
                    return v;
                };
                std::vector<cd> E(256, cd(0, 0));
                for (int r = 0; r < 16; ++r)
                    for (int c2 = 0; c2 < 16; ++c2)
                        if ((r & ~mk) == (c2 & ~mk))
                            E[r * 16 + c2] = U[sub(r) * D + sub(c2)];
                M = matmul(E, M, 16);
            }
            st.mfma = pp.mf.n;
            pp.mf.off[pp.mf.n++] = (uint32_t)P->pool.size();
            push_matrix(P->pool, M);
        }
    }
    P->nfused_ops += pp.nops;
    P->passes.push_back(std::move(pp));
    return QS_OK;
}

// QS_PLAN_REMAP: the block passes the former chose (logical qubit sets), run on the lowest b physical qubits. Before
// each pass, the pass's qubits that sit at physical positions >= b are exchanged with low positions whose qubits the
// pass does not use (those needed latest again), paired in ascending order and merged into fused_swap(p, q, s)
// wherever both sides run on contiguously; the gates then act on their physical qubits. A circuit fused-swap is a
// relabelling of the map (no data moves: a zero-cost pass keeps its place in the pass order). At the end, fused-swaps
// put every logical qubit back at its own position, so the plan's final state is the circuit's.
int plan_remap(qs_plan *P, const qs_circuit &c, int b, int stage_width, const std::vector<PassSpec> &passes)
{
    const int n = c.n;
    std::vector<int> phys(n), lg(n);  // logical -> physical, physical -> logical
    for (int q = 0; q < n; ++q)
        phys[q] = lg[q] = q;
    auto swap_pass = [&](int p, int q, int s) {
        PlanPass sp;
        sp.type = 2;
        sp.p = std::min(p, q);
        sp.q = std::max(p, q);
        sp.s = s;
        sp.ngates = 0;
        for (int j = 0; j < s; ++j) {
            std::swap(lg[p + j], lg[q + j]);
            phys[lg[p + j]] = p + j;
            phys[lg[q + j]] = q + j;
        }
        P->passes.push_back(std::move(sp));
    };
    // exchange the physical positions hs[i] (>= b) with vs[i] (< b), both ascending, as few fused-swaps as runs allow
    auto exchange = [&](const std::vector<int> &hs, const std::vector<int> &vs) {
        for (size_t i = 0; i < hs.size();) {
            size_t k = i + 1;
            while (k < hs.size() && hs[k] == hs[k - 1] + 1 && vs[k] == vs[k - 1] + 1)
                ++k;
            swap_pass(vs[i], hs[i], (int)(k - i));
            i = k;
        }
    };
    // whether pass ps uses logical qubit q, and the index of the next pass (from `from` on) that does
    auto uses = [&](const PassSpec &ps, int q) {
        if (!ps.L.empty())
            return std::find(ps.L.begin(), ps.L.end(), q) != ps.L.end();
        const PG &g = c.gates[ps.gates[0]];
        if (g.kind == 1) {
            const RawOp &r = c.raw[g.raw];
            return (q >= r.p && q < r.p + r.s) || (q >= r.q && q < r.q + r.s);
        }
        return std::find(g.q.begin(), g.q.end(), q) != g.q.end();
    };
    auto next_use = [&](size_t from, int q) {
        for (size_t k = from; k < passes.size(); ++k)
            if (uses(passes[k], q))
                return k;
        return passes.size();
    };
    qs_circuit pc;  // the gates on physical qubits, in the order the passes take them
    pc.n = n;
    auto physical = [&](const PG &g) {
        PG h = g;
        for (int &q : h.q)
            q = phys[q];
        return h;
    };
    for (size_t k = 0; k < passes.size(); ++k) {
        const PassSpec &ps = passes[k];
        if (ps.L.empty()) {
            const PG &g = c.gates[ps.gates[0]];
            if (g.kind == 1) {  // relabel: logical p + j and q + j trade physical positions
                const RawOp &r = c.raw[g.raw];
                for (int j = 0; j < r.s; ++j) {
                    const int a = r.p + j, d = r.q + j;
                    std::swap(phys[a], phys[d]);
                    lg[phys[a]] = a;
                    lg[phys[d]] = d;
                }
                PlanPass rp;
                rp.type = 4;
                rp.p = std::min(r.p, r.q);
                rp.q = std::max(r.p, r.q);
                rp.s = r.s;
                rp.ngates = 1;
                rp.order.assign(1, g.raw);
                P->passes.push_back(std::move(rp));
            } else if (g.kind == 2 || (int)g.q.size() > QS_MAX_K) {  // an opaque op on its physical qubits
                RawOp r = c.raw[g.raw];
                for (int &q : r.t)
                    q = phys[q];
                for (int &q : r.c)
                    q = phys[q];
                PlanPass op;
                op.type = 3;
                op.raw = (int)P->raw.size();
                P->raw.push_back(std::move(r));
                op.ngates = 1;
                op.order.assign(1, g.raw);
                P->passes.push_back(std::move(op));
            } else {
                PlanPass dp;
                dp.ngates = 1;
                dp.order.assign(1, g.raw);
                if (int rc = make_dense_pass(P, physical(g), dp))
                    return rc;
                P->passes.push_back(std::move(dp));
            }
            continue;
        }
        // bring the pass's qubits into the low b physical positions
        std::vector<int> hs, vs;
        for (int q : ps.L)
            if (phys[q] >= b)
                hs.push_back(phys[q]);
        if (!hs.empty()) {
            std::vector<std::pair<size_t, int>> free_low;  // (next use, position) of low positions the pass leaves
            for (int v = 0; v < b; ++v)
                if (std::find(ps.L.begin(), ps.L.end(), lg[v]) == ps.L.end())
                    free_low.push_back({next_use(k + 1, lg[v]), v});
            std::stable_sort(free_low.begin(), free_low.end(),
                             [](const std::pair<size_t, int> &x, const std::pair<size_t, int> &y) {
                                 return x.first > y.first;
                             });
            for (size_t i = 0; i < hs.size(); ++i)
                vs.push_back(free_low[i].second);
            std::sort(hs.begin(), hs.end());
            std::sort(vs.begin(), vs.end());
            exchange(hs, vs);
        }
        std::vector<int> L, gs;
        for (int q : ps.L)
            L.push_back(phys[q]);
        for (int gi : ps.gates) {
            gs.push_back((int)pc.gates.size());
            pc.gates.push_back(physical(c.gates[gi]));
        }
        if (int rc = append_pass(P, &pc, QS_PLAN_BLOCK, L, gs, b, stage_width))
            return rc;
    }
    // restore the identity map: the lowest misplaced position takes its qubit back, with the following positions as
    // long as their qubits lie just as far behind
    for (int i = 0; i < n; ++i) {
        if (lg[i] == i)
            continue;
        const int j = phys[i];  // > i: positions below i are already home
        int s = 1;
        while (i + s < n && j + s < n && lg[i + s] != i + s && phys[i + s] == j + s && j - i >= s + 1)
            ++s;
        swap_pass(i, j, s);  // positions i .. i + s - 1 now hold their own qubits
    }
    return QS_OK;
}

int plan_create(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts, int stage_width,
                const qs_plan_model *model, bool beam_search)
{
    if (model && c && c->n < 8)
        return qs_fail(QS_EINVAL, "qs_plan_create_learned: block passes need at least 8 qubits");
    if (!out || !c || !opts)
        return qs_fail(QS_EINVAL, "qs_plan_create: NULL argument");
    *out = nullptr;
    int mode = opts->mode, b = opts->block_bits, w = opts->low_bits;
    if (opts->dtype != QS_C128 && opts->dtype != QS_C64)
        return qs_fail(QS_EINVAL, "qs_plan_create: bad dtype %d", opts->dtype);
    if (mode == QS_PLAN_BLOCK || mode == QS_PLAN_REMAP) {
        if (c->n < 8) {  // a block needs at least 256 amplitudes: plan small states as fused dense blocks
            mode = QS_PLAN_FUSE;
            b = std::min(c->n, 4);
            w = 0;
        } else {
            if (b < 8 || b > kMaxBlockBits)
                return qs_fail(QS_EINVAL, "qs_plan_create: block_bits = %d outside [8, %d]", b, kMaxBlockBits);
            b = std::min(b, c->n);
            if (w < 0 || w > b)
                return qs_fail(QS_EINVAL, "qs_plan_create: low_bits = %d outside [0, block_bits]", w);
        }
    } else if (mode == QS_PLAN_FUSE) {
        if (b < 1 || b > QS_MAX_K)
            return qs_fail(QS_EINVAL, "qs_plan_create: block_bits = %d outside [1, %d] for fused blocks", b, QS_MAX_K);
        b = std::min(b, c->n);
        w = 0;
    } else {
        return qs_fail(QS_EINVAL, "qs_plan_create: unknown mode %d", mode);
    }
    qs_plan *P = new (std::nothrow) qs_plan();
    if (!P)
        return qs_fail(QS_ENOMEM, "qs_plan_create: out of host memory");
    P->n = c->n;
    P->dtype = opts->dtype;
    P->mode = mode;
    P->raw = c->raw;
    const int maxq = mode == QS_PLAN_FUSE ? b : kMaxBlockOpK;
    std::vector<PassSpec> passes;
    if (model) {
        if (int rc = learned_passes(*c, P->dtype, *model, stage_width, passes)) {
            delete P;
            return rc;
        }
    } else {
        // pass formation at the tunable beam width and, with beam_search, at 1.5x and 4x that width as well (the
        // pass count is not monotone in the width): the fewest passes win, ties going to the earlier width
        const int base = qs_tunables().plan_beam;
        std::vector<int> widths{base};
        if (beam_search && base > 0)
            for (int bw : {base * 3 / 2, std::min(64, base * 4)})
                if (std::find(widths.begin(), widths.end(), bw) == widths.end())
                    widths.push_back(bw);
        bool have = false;
        for (int bw : widths) {
            Former F(*c, b, w, maxq, bw);
            std::vector<std::pair<std::vector<int>, std::vector<int>>> fp;
            std::vector<int> singles;
            F.run(fp, singles);
            if (!have || fp.size() < passes.size()) {
                passes.clear();
                for (auto &pr : fp)
                    passes.push_back({pr.first, pr.second, b});
                have = true;
            }
        }
    }
    if (mode == QS_PLAN_REMAP) {
        if (int rc = plan_remap(P, *c, b, stage_width, passes)) {
            delete P;
            return rc;
        }
        *out = P;
        return QS_OK;
    }
    for (const PassSpec &ps : passes)
        if (int rc = append_pass(P, c, mode, ps.L, ps.gates, ps.b, stage_width)) {
            delete P;
            return rc;
        }
    *out = P;
    return QS_OK;
}

// Enqueue pass i of P on the state's stream (rn: a renormalisation folded into a complex64 block pass).
int run_pass(qs_state *st, qs_plan *P, int i, const BlkRenorm &rn)
{
    const size_t esz = P->dtype == QS_C128 ? sizeof(double) : sizeof(float);
    const PlanPass &pp = P->passes[i];
    switch (pp.type) {
    case 0: {
        const InsBits outer = qs_make_ins(pp.lmask, 0);
        QS_HIP(launch_block(st->dtype, pp.b, pp.sw, st->psi, (uint64_t)1 << (P->n - pp.b), outer, pp.bm,
                            P->dstages + pp.stage_begin, pp.nstages, P->dpool, pp.mf,
                            pp.lstage_begin >= 0 ? P->dlstages + pp.lstage_begin : nullptr, st->stream, rn));
        break;
    }
    case 1: {
        const InsBits ins = qs_make_ins(pp.tmask, 0);
        QS_HIP(launch_dense(st->dtype, pp.k, st->psi, (uint64_t)1 << (P->n - pp.k), ins, pp.tp, pp.Uh.data(),
                            (const char *)P->dpool + pp.mat_off * esz, st->stream));
        break;
    }
    case 2:
        QS_HIP(launch_fused_swap(st->dtype, st->psi, P->n, pp.p, pp.q, pp.s, st->stream));
        break;
    case 4:  // relabel: absorbed into the qubit map, no data moves
        break;
    default:
        if (int rc = run_raw(st, P->raw[pp.raw]))
            return rc;
    }
    return QS_OK;
}

int check_run(qs_state *st, qs_plan *P, const char *fn)
{
    if (!st || !P)
        return qs_fail(QS_EINVAL, "%s: NULL argument", fn);
    if (st->n != P->n || st->dtype != P->dtype)
        return qs_fail(QS_EINVAL, "%s: plan is for n = %d dtype %d, state is n = %d dtype %d", fn, P->n, P->dtype,
                       st->n, st->dtype);
    return QS_OK;
}

}  // namespace

extern "C" {

QS_API int qs_plan_run_range(qs_state *st, qs_plan *P, int begin, int end)
{
    qs_clear_error();
    if (int rc = check_run(st, P, "qs_plan_run"))
        return rc;
    const int np = (int)P->passes.size();
    if (begin < 0 || end > np || begin > end)
        return qs_fail(QS_EINVAL, "qs_plan_run: pass range [%d, %d) outside [0, %d]", begin, end, np);
    if (int rc = upload(P))
        return rc;
    for (int i = begin; i < end; ++i)
        if (int rc = run_pass(st, P, i, BlkRenorm{}))
            return rc;
    return QS_OK;
}

QS_API int qs_plan_run_range_renorm(qs_state *st, qs_plan *P, int begin, int end, int flags)
{
    qs_clear_error();
    if (int rc = check_run(st, P, "qs_plan_run_range_renorm"))
        return rc;
    if (flags & ~(QS_RUN_SCALE_FIRST | QS_RUN_NORM_LAST))
        return qs_fail(QS_EINVAL, "qs_plan_run_range_renorm: unknown flags 0x%x", flags);
    const int np = (int)P->passes.size();
    if (begin < 0 || end > np || begin > end)
        return qs_fail(QS_EINVAL, "qs_plan_run_range_renorm: pass range [%d, %d) outside [0, %d]", begin, end, np);
    if (int rc = upload(P))
        return rc;
    const uint64_t dim = (uint64_t)1 << st->n;
    double *pending = qs_pending_norm(st);
    // the range's passes that move data (relabels launch nothing); a renormalisation folds into a complex64 block
    // pass
    int first = -1, last = -1;
    for (int i = begin; i < end; ++i)
        if (P->passes[i].type != 4) {
            if (first < 0)
                first = i;
            last = i;
        }
    auto foldable = [&](int i) {
        return i >= 0 && st->dtype == QS_C64 && P->passes[i].type == 0 && P->passes[i].lstage_begin < 0;
    };
    const bool scale_in = (flags & QS_RUN_SCALE_FIRST) && foldable(first);
    if ((flags & QS_RUN_SCALE_FIRST) && !scale_in)
        QS_HIP(launch_scale_dev(st->dtype, st->psi, dim, pending, st->stream));
    double *parts = nullptr;
    uint64_t nparts = 0;
    if ((flags & QS_RUN_NORM_LAST) && foldable(last)) {
        const PlanPass &pp = P->passes[last];
        nparts = launch_block_grid(st->dtype, pp.b, pp.sw, (uint64_t)1 << (P->n - pp.b));
        if (nparts == 0)
            return qs_fail(QS_EUNSUPPORTED, "qs_plan_run_range_renorm: no block kernel for b = %d, w = %d", pp.b,
                           pp.sw);
        parts = qs_block_partials(st, (size_t)nparts);
        if (!parts)
            return QS_ENOMEM;
    }
    for (int i = begin; i < end; ++i) {
        BlkRenorm rn;
        if (scale_in && i == first)
            rn.scale_norm = pending;
        if (parts && i == last)
            rn.norm_part = parts;
        if (int rc = run_pass(st, P, i, rn))
            return rc;
    }
    if (flags & QS_RUN_NORM_LAST) {
        if (parts)
            QS_HIP(launch_sum_partials(parts, (int)nparts, pending, st->stream));
        else
            QS_HIP(launch_probs(st->dtype, st->psi, dim, nullptr, st->red, probs_blocks(dim), pending, st->stream));
    }
    return QS_OK;
}

QS_API int qs_plan_run_renorm(qs_state *st, qs_plan *P, int flags)
{
    if (!P) {
        qs_clear_error();
        return qs_fail(QS_EINVAL, "qs_plan_run_renorm: NULL plan");
    }
    return qs_plan_run_range_renorm(st, P, 0, (int)P->passes.size(), flags);
}

QS_API int qs_renormalize_pending(qs_state *st, double *norm)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_renormalize_pending: NULL handle");
    double *pending = qs_pending_norm(st);
    QS_HIP(launch_scale_dev(st->dtype, st->psi, (uint64_t)1 << st->n, pending, st->stream));
    if (norm) {
        QS_HIP(hipMemcpyAsync(norm, pending, sizeof(double), hipMemcpyDeviceToHost, st->stream));
        QS_HIP(hipStreamSynchronize(st->stream));
    }
    return QS_OK;
}

QS_API int qs_plan_run(qs_state *st, qs_plan *P)
{
    if (!P) {
        qs_clear_error();
        return qs_fail(QS_EINVAL, "qs_plan_run: NULL plan");
    }
    return qs_plan_run_range(st, P, 0, (int)P->passes.size());
}

QS_API int qs_plan_info(const qs_plan *P, int *npasses, int *nblock, int *ndense, int *nother, int *nfused_ops)
{
    qs_clear_error();
    if (!P)
        return qs_fail(QS_EINVAL, "qs_plan_info: NULL plan");
    int nb = 0, nd = 0, no = 0;
    for (const PlanPass &pp : P->passes)
        (pp.type == 0 ? nb : pp.type == 1 ? nd : no)++;
    if (npasses)
        *npasses = (int)P->passes.size();
    if (nblock)
        *nblock = nb;
    if (ndense)
        *ndense = nd;
    if (nother)
        *nother = no;
    if (nfused_ops)
        *nfused_ops = P->nfused_ops;
    return QS_OK;
}

QS_API int qs_plan_pass_info(const qs_plan *P, int i, int *type, int *nqubits, int64_t *qmask, int *nops, int *ngates)
{
    qs_clear_error();
    if (!P || i < 0 || i >= (int)P->passes.size())
        return qs_fail(QS_EINVAL, "qs_plan_pass_info: NULL plan or pass index out of range");
    const PlanPass &pp = P->passes[i];
    int nq = 0;
    int64_t m = 0;
    switch (pp.type) {
    case 0: nq = pp.b; m = (int64_t)pp.lmask; break;
    case 1: nq = pp.k; m = (int64_t)pp.tmask; break;
    case 2:
    case 4:
        nq = 2 * pp.s;
        for (int j = 0; j < pp.s; ++j)
            m |= ((int64_t)1 << (pp.p + j)) | ((int64_t)1 << (pp.q + j));
        break;
    default: {
        const RawOp &r = P->raw[pp.raw];
        for (int q : r.t)
            m |= (int64_t)1 << q;
        for (int q : r.c)
            m |= (int64_t)1 << q;
        nq = __builtin_popcountll((uint64_t)m);
    }
    }
    if (type)
        *type = pp.type;
    if (nqubits)
        *nqubits = nq;
    if (qmask)
        *qmask = m;
    if (nops)
        *nops = pp.type == 0 ? pp.nops : 1;
    if (ngates)
        *ngates = pp.ngates;
    return QS_OK;
}

QS_API int qs_plan_pass_gates(const qs_plan *P, int i, int *gates, int cap, int *count)
{
    qs_clear_error();
    if (!P || i < 0 || i >= (int)P->passes.size() || cap < 0 || (cap > 0 && !gates))
        return qs_fail(QS_EINVAL, "qs_plan_pass_gates: NULL plan or output, negative capacity or pass index out of "
                                  "range");
    const std::vector<int> &o = P->passes[i].order;
    for (int j = 0; j < cap && j < (int)o.size(); ++j)
        gates[j] = o[j];
    if (count)
        *count = (int)o.size();
    return QS_OK;
}

QS_API int qs_plan_features(const qs_plan *P, int i, float *f)
{
    qs_clear_error();
    if (!P || !f || i < 0 || i >= (int)P->passes.size())
        return qs_fail(QS_EINVAL, "qs_plan_features: NULL argument or pass index out of range");
    const PlanPass &pp = P->passes[i];
    int type = 0, nq = 0, nops = 0, ng = 0;
    int64_t m = 0;
    if (int rc = qs_plan_pass_info(P, i, &type, &nq, &m, &nops, &ng))
        return rc;
    for (int j = 0; j < QS_PLAN_NFEAT; ++j)
        f[j] = 0.0f;
    f[type < 4 ? type : 3] = 1.0f;
    f[4] = P->n / 40.0f;
    f[5] = P->dtype == QS_C64 ? 1.0f : 0.0f;
    f[6] = nq / 16.0f;
    f[7] = nops / 32.0f;
    f[8] = (pp.type == 0 ? pp.nstages : 0) / 16.0f;
    int contig = 0;
    while (contig < 64 && ((uint64_t)m >> contig) & 1)
        ++contig;
    f[9] = contig / 16.0f;
    int lo = 0, hi = 0;
    if (m) {
        lo = __builtin_ctzll((uint64_t)m);
        hi = 63 - __builtin_clzll((uint64_t)m);
    }
    f[10] = lo / 40.0f;
    f[11] = hi / 40.0f;
    f[12] = __builtin_popcountll((uint64_t)m & 15) / 4.0f;
    f[13] = (P->n + (P->dtype == QS_C64 ? 3 : 4)) / 40.0f;  // log2 of the state's bytes
    double flops = 0.0;                                     // per amplitude
    if (pp.type == 0) {
        for (int t = pp.stage_begin; t < pp.stage_begin + pp.nstages; ++t)
            for (int o = P->stages[t].op_begin; o < P->stages[t].op_begin + P->stages[t].nops; ++o)
                flops += 8.0 * (1 << __builtin_popcount(P->sops[o].mask));
    } else if (pp.type == 1) {
        flops = 8.0 * (1 << pp.k);
    }
    f[14] = (float)(flops / 256.0);
    f[15] = ng / 64.0f;
    if (pp.type == 0 && pp.b >= 10 && pp.b <= 13)
        f[16 + pp.b - 10] = 1.0f;  // block size one-hot
    if (pp.type == 1 && pp.k >= 3 && pp.k <= 6)
        f[20 + pp.k - 3] = 1.0f;  // dense target count one-hot
    f[24] = pp.type == 2 ? pp.s / 16.0f : 0.0f;
    f[25] = contig >= 4 ? 1.0f : 0.0f;
    for (int b = 0; b < 22; ++b)
        f[26 + b] = ((uint64_t)m >> b) & 1 ? 1.0f : 0.0f;
    return QS_OK;
}

QS_API int qs_plan_free(qs_plan *P)
{
    qs_clear_error();
    if (!P)
        return qs_fail(QS_EINVAL, "qs_plan_free: NULL plan");
    if (P->dstages)
        (void)hipFree(P->dstages);
    if (P->dlstages)
        (void)hipFree(P->dlstages);
    if (P->dpool)
        (void)hipFree(P->dpool);
    delete P;
    return QS_OK;
}

}  // extern "C"

// ============================================================================================================
// batches: many circuits, one persistent launch (optionally replayed from a captured HIP graph)
// ============================================================================================================
struct qs_batch {
    int dtype = QS_C128, b = 12, low = 4, wg_per_cu = 2;
    hipStream_t stream = nullptr;
    std::vector<BatchCirc> circs;
    std::vector<int> nops;  // fused ops per circuit (schedule cost)
    std::vector<BatchPass> passes;
    std::vector<BlkStage> stages;
    std::vector<double> pool;
    std::vector<BatchItem> items;      // all levels, level after level
    std::vector<int> level_begin;      // items of level k: [level_begin[k], level_begin[k + 1])
    std::vector<uint32_t> level_blocks;
    uint64_t state_amps = 0, prob_count = 0;
    bool finalized = false;
    void *psi = nullptr;
    double *probs = nullptr;
    BatchItem *ditems = nullptr;
    BatchPass *dpasses = nullptr;
    BlkStage *dstages = nullptr;
    void *dmats = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {
void batch_free_device(qs_batch *Bt);

void batch_release(qs_batch *Bt)
{
    if (!Bt)
        return;
    (void)hipStreamSynchronize(Bt->stream);
    if (Bt->exec)
        (void)hipGraphExecDestroy(Bt->exec);
    if (Bt->graph)
        (void)hipGraphDestroy(Bt->graph);
    batch_free_device(Bt);
    delete Bt;
}

// *dst is set only once the table is on the device; on failure nothing stays allocated.
template <class T> int upload_vec(T **dst, const std::vector<T> &v)
{
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(v.size(), 1) * sizeof(T));
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipMalloc(batch table)");
    if (!v.empty() && (e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(p);
        return qs_hip_fail(e, "hipMemcpy(batch table)");
    }
    *dst = static_cast<T *>(p);
    return QS_OK;
}

// State and probability slices, then the tables. Each buffer is recorded in the batch as soon as it exists, so
// batch_free_device releases whatever a failed attempt left.
int batch_upload(qs_batch *Bt)
{
    const size_t esz = Bt->dtype == QS_C128 ? 16 : 8;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<uint64_t>(Bt->state_amps, 1) * esz);
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipMalloc(batch states)");
    Bt->psi = p;
    p = nullptr;
    e = hipMalloc(&p, std::max<uint64_t>(Bt->prob_count, 1) * sizeof(double));
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipMalloc(batch probabilities)");
    Bt->probs = static_cast<double *>(p);
    if (int rc = upload_vec(&Bt->ditems, Bt->items))
        return rc;
    if (int rc = upload_vec(&Bt->dpasses, Bt->passes))
        return rc;
    if (int rc = upload_vec(&Bt->dstages, Bt->stages))
        return rc;
    if (Bt->dtype == QS_C128) {
        double *d = nullptr;
        if (int rc = upload_vec(&d, Bt->pool))
            return rc;
        Bt->dmats = d;
    } else {
        std::vector<float> f(Bt->pool.begin(), Bt->pool.end());
        float *d = nullptr;
        if (int rc = upload_vec(&d, f))
            return rc;
        Bt->dmats = d;
    }
    return QS_OK;
}

void batch_free_device(qs_batch *Bt)
{
    void *bufs[] = {Bt->psi, Bt->probs, Bt->ditems, Bt->dpasses, Bt->dstages, Bt->dmats};
    for (void *p : bufs)
        if (p)
            (void)hipFree(p);
    Bt->psi = nullptr;
    Bt->probs = nullptr;
    Bt->ditems = nullptr;
    Bt->dpasses = nullptr;
    Bt->dstages = nullptr;
    Bt->dmats = nullptr;
}
}  // namespace

extern "C" {

QS_API int qs_batch_create(qs_batch **out, int dtype, int block_bits, int low_bits, int wg_per_cu, void *hip_stream)
{
    qs_clear_error();
    if (!out)
        return qs_fail(QS_EINVAL, "qs_batch_create: out is NULL");
    *out = nullptr;
    if (dtype != QS_C128 && dtype != QS_C64)
        return qs_fail(QS_EINVAL, "qs_batch_create: bad dtype %d", dtype);
    if (block_bits < 10 || block_bits > 12)
        return qs_fail(QS_EINVAL, "qs_batch_create: block_bits = %d outside [10, 12]", block_bits);
    if (low_bits < 0 || low_bits > block_bits || wg_per_cu < 1 || wg_per_cu > 64)
        return qs_fail(QS_EINVAL, "qs_batch_create: low_bits or wg_per_cu out of range");
    qs_batch *Bt = new (std::nothrow) qs_batch();
    if (!Bt)
        return qs_fail(QS_ENOMEM, "qs_batch_create: out of host memory");
    Bt->dtype = dtype;
    Bt->b = block_bits;
    Bt->low = low_bits;
    Bt->wg_per_cu = wg_per_cu;
    Bt->stream = (hipStream_t)hip_stream;
    *out = Bt;
    return QS_OK;
}

QS_API int qs_batch_set_launch(qs_batch *Bt, int wg_per_cu)
{
    qs_clear_error();
    if (!Bt)
        return qs_fail(QS_EINVAL, "qs_batch_set_launch: NULL batch");
    if (wg_per_cu < 1 || wg_per_cu > 64)
        return qs_fail(QS_EINVAL, "qs_batch_set_launch: wg_per_cu = %d outside [1, 64]", wg_per_cu);
    if (wg_per_cu == Bt->wg_per_cu)
        return QS_OK;
    // a captured graph holds the old grid: drop it (after the stream has finished with it)
    if (Bt->exec || Bt->graph) {
        QS_HIP(hipStreamSynchronize(Bt->stream));
        if (Bt->exec)
            QS_HIP(hipGraphExecDestroy(Bt->exec));
        if (Bt->graph)
            QS_HIP(hipGraphDestroy(Bt->graph));
        Bt->exec = nullptr;
        Bt->graph = nullptr;
    }
    Bt->wg_per_cu = wg_per_cu;
    return QS_OK;
}

QS_API int qs_batch_add(qs_batch *Bt, const qs_circuit *c)
{
    qs_clear_error();
    if (!Bt || !c)
        return qs_fail(QS_EINVAL, "qs_batch_add: NULL argument");
    if (Bt->finalized)
        return qs_fail(QS_EINVAL, "qs_batch_add: the batch is finalized");
    if (c->n < 8 || c->n > 30)
        return qs_fail(QS_EINVAL, "qs_batch_add: circuits of %d qubits are outside [8, 30]", c->n);
    const int bb = std::min(c->n, Bt->b);
    qs_plan_opts o{QS_PLAN_BLOCK, bb, std::min(Bt->low, bb), Bt->dtype};
    qs_plan *P = nullptr;
    if (int rc = plan_create(&P, c, &o, 4, nullptr))  // the batch kernel runs 4-position stages
        return rc;
    for (const PlanPass &pp : P->passes)
        if (pp.type != 0) {
            const int type = pp.type;  // pp lives in P, which is released first
            qs_plan_free(P);
            return qs_fail(QS_EUNSUPPORTED, "qs_batch_add: batched circuits may hold gates on at most 3 qubits and "
                                            "no fused-swaps (pass of type %d)", type);
        }
    BatchCirc bc{};
    bc.n = c->n;
    bc.pass_begin = (int)Bt->passes.size();
    bc.npass = (int)P->passes.size();
    bc.prob_off = Bt->prob_count;
    Bt->prob_count += (uint64_t)1 << c->n;
    if (c->n > Bt->b) {
        bc.state_off = Bt->state_amps;
        Bt->state_amps += (uint64_t)1 << c->n;
    }
    const int s0 = (int)Bt->stages.size();
    const uint32_t m0 = (uint32_t)Bt->pool.size();
    for (const PlanPass &pp : P->passes) {
        BatchPass bp{};
        bp.outer = qs_make_ins(pp.lmask, 0);
        bp.bm = pp.bm;
        bp.stage_begin = s0 + pp.stage_begin;
        bp.nstages = pp.nstages;
        bp.mf = pp.mf;
        for (int i = 0; i < bp.mf.n; ++i)
            bp.mf.off[i] += m0;
        Bt->passes.push_back(bp);
    }
    if (P->passes.empty() && c->n > Bt->b) {
        // a circuit held in HBM needs one pass to initialise and measure its state: an empty one over the low qubits
        BatchPass bp{};
        bp.outer = qs_make_ins(((uint64_t)1 << Bt->b) - 1, 0);
        bp.bm.b = Bt->b;
        for (int t = 0; t < Bt->b; ++t)
            bp.bm.lpos[t] = t;
        bp.stage_begin = s0;
        bp.nstages = 0;
        Bt->passes.push_back(bp);
        bc.npass = 1;
    }
    for (BlkStage st : P->stages) {
        st.mat_base += m0;  // op_begin keeps indexing the circuit plan's host op table, which the batch drops
        Bt->stages.push_back(st);
    }
    Bt->pool.insert(Bt->pool.end(), P->pool.begin(), P->pool.end());
    int fused = 0;
    for (const PlanPass &pp : P->passes)
        fused += pp.nops;
    Bt->nops.push_back(fused);
    Bt->circs.push_back(bc);
    qs_plan_free(P);
    return QS_OK;
}

QS_API int qs_batch_finalize(qs_batch *Bt)
{
    qs_clear_error();
    if (!Bt)
        return qs_fail(QS_EINVAL, "qs_batch_finalize: NULL batch");
    if (Bt->finalized)
        return QS_OK;
    if (Bt->pool.size() >= ((size_t)1 << 32))
        return qs_fail(QS_EUNSUPPORTED, "qs_batch_finalize: matrix pool too large");
    // Level k holds pass k of every circuit kept in HBM; level 0 also holds the circuits that live in LDS, costliest
    // first, ahead of all blocks so that they start at once.
    std::vector<int> small, large;
    int nlev = 0;
    for (int i = 0; i < (int)Bt->circs.size(); ++i) {
        const BatchCirc &c = Bt->circs[i];
        if (c.n <= Bt->b) {
            small.push_back(i);
            nlev = std::max(nlev, 1);
        } else {
            large.push_back(i);
            nlev = std::max(nlev, c.npass);
        }
    }
    std::stable_sort(small.begin(), small.end(), [&](int a, int b) {
        return std::ldexp(1.0 + Bt->nops[a], Bt->circs[a].n) > std::ldexp(1.0 + Bt->nops[b], Bt->circs[b].n);
    });
    std::stable_sort(large.begin(), large.end(), [&](int a, int b) { return Bt->circs[a].n > Bt->circs[b].n; });
    Bt->items.clear();
    Bt->level_begin.clear();
    Bt->level_blocks.clear();
    for (int lev = 0; lev < nlev; ++lev) {
        Bt->level_begin.push_back((int)Bt->items.size());
        uint64_t blk = 0;
        if (lev == 0)
            for (int i : small) {
                const BatchCirc &c = Bt->circs[i];
                Bt->items.push_back(BatchItem{0, c.prob_off, (uint32_t)blk, c.pass_begin, c.npass, c.n, kBatchSmall});
                blk += 1;
            }
        for (int i : large) {
            const BatchCirc &c = Bt->circs[i];
            if (c.npass <= lev)
                continue;
            const int flags = (lev == 0 ? kBatchFirst : 0) | (lev == c.npass - 1 ? kBatchLast : 0);
            Bt->items.push_back(BatchItem{c.state_off, c.prob_off, (uint32_t)blk, c.pass_begin + lev, 1, c.n, flags});
            blk += (uint64_t)1 << (c.n - Bt->b);
        }
        if (blk >= ((uint64_t)1 << 31))
            return qs_fail(QS_EUNSUPPORTED, "qs_batch_finalize: %llu blocks in one level exceed 2^31",
                           (unsigned long long)blk);
        Bt->level_blocks.push_back((uint32_t)blk);
    }
    Bt->level_begin.push_back((int)Bt->items.size());
    if (int rc = batch_upload(Bt)) {  // leave nothing allocated: a later finalize starts over
        batch_free_device(Bt);
        return rc;
    }
    Bt->finalized = true;
    return QS_OK;
}

QS_API int qs_batch_run(qs_batch *Bt, int use_graph)
{
    qs_clear_error();
    if (!Bt)
        return qs_fail(QS_EINVAL, "qs_batch_run: NULL batch");
    if (!Bt->finalized)
        if (int rc = qs_batch_finalize(Bt))
            return rc;
    auto enqueue = [&]() {
        for (size_t lev = 0; lev + 1 < Bt->level_begin.size(); ++lev) {
            const int i0 = Bt->level_begin[lev], i1 = Bt->level_begin[lev + 1];
            hipError_t e = launch_batch_level(Bt->dtype, Bt->b, Bt->psi, Bt->probs, Bt->ditems + i0, i1 - i0,
                                              Bt->level_blocks[lev], Bt->dpasses, Bt->dstages, Bt->dmats,
                                              Bt->wg_per_cu, Bt->stream);
            if (e != hipSuccess)
                return e;
        }
        return hipSuccess;
    };
    if (!use_graph) {
        QS_HIP(enqueue());
        return QS_OK;
    }
    if (!Bt->exec) {
        // a graph left by an earlier failed instantiation is dropped before capturing again
        if (Bt->graph) {
            (void)hipGraphDestroy(Bt->graph);
            Bt->graph = nullptr;
        }
        QS_HIP(hipStreamBeginCapture(Bt->stream, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue();
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(Bt->stream, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return e != hipSuccess ? qs_hip_fail(e, "batch launch during capture")
                                   : qs_hip_fail(e2, "hipStreamEndCapture(batch)");
        }
        hipGraphExec_t x = nullptr;
        hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e3 != hipSuccess) {
            (void)hipGraphDestroy(g);
            return qs_hip_fail(e3, "hipGraphInstantiate(batch)");
        }
        Bt->graph = g;
        Bt->exec = x;
    }
    QS_HIP(hipGraphLaunch(Bt->exec, Bt->stream));
    return QS_OK;
}

QS_API int qs_batch_info(const qs_batch *Bt, int *ncirc, int64_t *state_bytes, int64_t *prob_count, int *npasses,
                         int *nlevels)
{
    qs_clear_error();
    if (!Bt)
        return qs_fail(QS_EINVAL, "qs_batch_info: NULL batch");
    if (ncirc)
        *ncirc = (int)Bt->circs.size();
    if (state_bytes)
        *state_bytes = (int64_t)(Bt->state_amps * (Bt->dtype == QS_C128 ? 16 : 8));
    if (prob_count)
        *prob_count = (int64_t)Bt->prob_count;
    if (npasses)
        *npasses = (int)Bt->passes.size();
    if (nlevels)
        *nlevels = Bt->finalized ? (int)Bt->level_blocks.size() : 0;
    return QS_OK;
}

QS_API int qs_batch_probs(qs_batch *Bt, int i, double **dev_ptr, double *host_out)
{
    qs_clear_error();
    if (!Bt || i < 0 || i >= (int)Bt->circs.size())
        return qs_fail(QS_EINVAL, "qs_batch_probs: NULL batch or circuit index out of range");
    if (!Bt->finalized)
        return qs_fail(QS_EINVAL, "qs_batch_probs: the batch has not run");
    const BatchCirc &c = Bt->circs[i];
    if (dev_ptr)
        *dev_ptr = Bt->probs + c.prob_off;
    if (host_out) {
        QS_HIP(hipStreamSynchronize(Bt->stream));
        QS_HIP(hipMemcpy(host_out, Bt->probs + c.prob_off, ((size_t)1 << c.n) * sizeof(double),
                         hipMemcpyDeviceToHost));
    }
    return QS_OK;
}

QS_API int qs_batch_free(qs_batch *Bt)
{
    qs_clear_error();
    if (!Bt)
        return qs_fail(QS_EINVAL, "qs_batch_free: NULL batch");
    batch_release(Bt);
    return QS_OK;
}

}  // extern "C"
