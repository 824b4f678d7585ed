// Host side of the libqs C ABI: validation, matrix classification and kernel dispatch.
//
// Every entry point validates all arguments before it enqueues anything, so a rejected call leaves the state
// unchanged. Work is enqueued on the state's stream; nothing synchronises unless the call says so.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "qs_internal.h"

namespace {
thread_local std::string g_err;
constexpr size_t kRingBytes = (size_t)8 << 20;
constexpr int kMaxPartials = 4096;
}  // namespace

int qs_fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int qs_hip_fail(hipError_t e, const char *what)
{
    (void)hipGetLastError();  // clear the sticky launch error so later calls report their own status
    return qs_fail(e == hipErrorOutOfMemory ? QS_ENOMEM : QS_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

void qs_clear_error() { g_err.clear(); }

extern "C" QS_API const char *qs_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------------------------------------------------
// staging ring: pinned host chunk -> async H2D copy on the state's stream. A host chunk is reused only after
// the copy that last read it has completed (event per chunk); device chunk reuse is ordered by the stream.
// ------------------------------------------------------------------------------------------------------------
void *qs_stage(qs_state *st, const void *host, size_t bytes)
{
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (need > st->ring_bytes) {
        qs_fail(QS_EINVAL, "staging request of %zu bytes exceeds the %zu-byte ring", bytes, st->ring_bytes);
        return nullptr;
    }
    if (st->ring_head + need > st->ring_bytes)
        st->ring_head = 0;
    const size_t csz = st->ring_bytes / kRingChunks;
    const int c0 = (int)(st->ring_head / csz), c1 = (int)((st->ring_head + need - 1) / csz);
    for (int c = c0; c <= c1; ++c) {
        if (st->ring_ev_live[c]) {
            hipError_t e = hipEventSynchronize(st->ring_ev[c]);
            if (e != hipSuccess) {
                qs_hip_fail(e, "hipEventSynchronize(staging ring)");
                return nullptr;
            }
            st->ring_ev_live[c] = false;
        }
    }
    std::memcpy(st->hring + st->ring_head, host, bytes);
    hipError_t e = hipMemcpyAsync(st->dring + st->ring_head, st->hring + st->ring_head, bytes, hipMemcpyHostToDevice,
                                  st->stream);
    if (e != hipSuccess) {
        qs_hip_fail(e, "hipMemcpyAsync(staging ring)");
        return nullptr;
    }
    for (int c = c0; c <= c1; ++c) {
        e = hipEventRecord(st->ring_ev[c], st->stream);
        if (e != hipSuccess) {
            qs_hip_fail(e, "hipEventRecord(staging ring)");
            return nullptr;
        }
        st->ring_ev_live[c] = true;
    }
    void *d = st->dring + st->ring_head;
    st->ring_head += need;
    return d;
}

// ---- device properties and kernel attributes, shared by the launchers ----
namespace {
constexpr int kMaxDev = 64;
std::atomic<int> g_cus[kMaxDev];  // 0: not queried yet
std::mutex g_lds_mu;
std::vector<std::tuple<int, const void *, size_t>> g_lds_set;  // (device, kernel, bytes allowed)
std::vector<std::pair<int, const void *>> g_nostatic;             // (device, kernel) checked to have no static LDS
}  // namespace

int qs_cu_count()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev)
        return 256;
    int c = g_cus[dev].load(std::memory_order_relaxed);
    if (c > 0)
        return c;
    if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
        c = 256;
    g_cus[dev].store(c, std::memory_order_relaxed);
    return c;
}

hipError_t qs_allow_lds(const void *fn, size_t bytes)
{
    if (bytes <= 65536)
        return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lock(g_lds_mu);
    for (auto &t : g_lds_set)
        if (std::get<0>(t) == dev && std::get<1>(t) == fn && std::get<2>(t) >= bytes)
            return hipSuccess;
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess)
        return e;
    g_lds_set.emplace_back(dev, fn, bytes);
    return hipSuccess;
}

hipError_t qs_check_no_static_lds(const void *fn)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    std::lock_guard<std::mutex> lock(g_lds_mu);
    for (auto &t : g_nostatic)
        if (t.first == dev && t.second == fn)
            return hipSuccess;
    hipFuncAttributes attr{};
    e = hipFuncGetAttributes(&attr, fn);
    if (e != hipSuccess)
        return e;
    if (attr.sharedSizeBytes != 0)
        return hipErrorInvalidDeviceFunction;
    g_nostatic.emplace_back(dev, fn);
    return hipSuccess;
}

double *qs_pending_norm(qs_state *st) { return st->red + kMaxPartials + 2; }

double *qs_block_partials(qs_state *st, size_t n)
{
    if (n <= st->blkred_cap)
        return st->blkred;
    if (st->blkred) {
        hipError_t e = hipStreamSynchronize(st->stream);  // the old buffer may still be read by queued work
        if (e != hipSuccess) {
            qs_hip_fail(e, "hipStreamSynchronize");
            return nullptr;
        }
        (void)hipFree(st->blkred);
        st->blkred = nullptr;
        st->blkred_cap = 0;
    }
    hipError_t e = hipMalloc((void **)&st->blkred, n * sizeof(double));
    if (e != hipSuccess) {
        st->blkred = nullptr;
        qs_hip_fail(e, "hipMalloc(block partial sums)");
        return nullptr;
    }
    st->blkred_cap = n;
    return st->blkred;
}

// ---- host helpers shared with the planner ----

// Sort the targets ascending; perm[j'] = the original matrix bit carried by sorted position j'.
void qs_sort_targets(const int *t, int k, TPos &tp, int *perm)
{
    int idx[QS_MAX_DIAG_K];
    for (int j = 0; j < k; ++j)
        idx[j] = j;
    std::sort(idx, idx + k, [&](int a, int b) { return t[a] < t[b]; });
    for (int j = 0; j < k; ++j) {
        perm[j] = idx[j];
        if (j < QS_MAX_K)
            tp.tpos[j] = t[idx[j]];
    }
}

static inline int map_index(int as, const int *perm, int k)
{
    int a = 0;
    for (int j = 0; j < k; ++j)
        a |= ((as >> j) & 1) << perm[j];
    return a;
}

// U (original bit order) -> U' in sorted bit order, interleaved FP64
void qs_permute_matrix(const double *U, int k, const int *perm, std::vector<double> &out)
{
    const int D = 1 << k;
    out.resize((size_t)2 * D * D);
    for (int a = 0; a < D; ++a) {
        const int oa = map_index(a, perm, k);
        for (int b = 0; b < D; ++b) {
            const int ob = map_index(b, perm, k);
            out[2 * (a * D + b)] = U[2 * (oa * D + ob)];
            out[2 * (a * D + b) + 1] = U[2 * (oa * D + ob) + 1];
        }
    }
}


namespace {

void release(qs_state *st)
{
    if (!st)
        return;
    if (st->stream || st->psi)
        (void)hipStreamSynchronize(st->stream);
    for (int c = 0; c < kRingChunks; ++c)
        if (st->ring_ev[c])
            (void)hipEventDestroy(st->ring_ev[c]);
    if (st->hring)
        (void)hipHostFree(st->hring);
    if (st->dring)
        (void)hipFree(st->dring);
    if (st->red)
        (void)hipFree(st->red);
    if (st->blkred)
        (void)hipFree(st->blkred);
    if (st->owns && st->psi)
        (void)hipFree(st->psi);
    delete st;
}

// qubit list checks: in range, distinct; returns the bit mask
int check_qubits(const qs_state *st, const int *q, int cnt, const char *what, uint64_t *mask)
{
    uint64_t m = 0;
    for (int j = 0; j < cnt; ++j) {
        if (q[j] < 0 || q[j] >= st->n)
            return qs_fail(QS_EINVAL, "%s[%d] = %d is outside [0, %d)", what, j, q[j], st->n);
        const uint64_t b = (uint64_t)1 << q[j];
        if (m & b)
            return qs_fail(QS_EINVAL, "%s repeats qubit %d", what, q[j]);
        m |= b;
    }
    *mask = m;
    return QS_OK;
}

// Monomial matrix with every nonzero in {1, -1, i, -i} (exact) -> move table. Returns false otherwise.
bool monomial_table(const std::vector<double> &Us, int k, PermTable &pt)
{
    const int D = 1 << k;
    std::memset(&pt, 0, sizeof pt);
    std::vector<int> colseen(D, 0);
    for (int a = 0; a < D; ++a) {
        int found = -1, ph = 0;
        for (int b = 0; b < D; ++b) {
            const double re = Us[2 * (a * D + b)], im = Us[2 * (a * D + b) + 1];
            if (re == 0.0 && im == 0.0)
                continue;
            if (found >= 0)
                return false;
            if (re == 1.0 && im == 0.0)
                ph = 0;
            else if (re == 0.0 && im == 1.0)
                ph = 1;
            else if (re == -1.0 && im == 0.0)
                ph = 2;
            else if (re == 0.0 && im == -1.0)
                ph = 3;
            else
                return false;
            found = b;
        }
        if (found < 0 || colseen[found])
            return false;
        colseen[found] = 1;
        pt.src[a] = (uint8_t)found;
        pt.phase[a] = (uint8_t)ph;
        if (found != a || ph != 0)
            pt.moving |= (uint64_t)1 << a;
    }
    return true;
}

bool is_diagonal(const double *U, int k)
{
    const int D = 1 << k;
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
            if (a != b && (U[2 * (a * D + b)] != 0.0 || U[2 * (a * D + b) + 1] != 0.0))
                return false;
    return true;
}

int diag_impl(qs_state *st, const int *targets, int k, const double *d);

// Lane-order form of a monomial op (qs_kernels.hip, k_perm_lanes) when it pays: the op's qubits Q = targets and
// controls (at most 6, at most 2 outside a wave's 64 16-byte lanes) and every 128-byte line of the state holds an
// amplitude it changes, so that a strided pass over the changed amplitudes would fetch and partly rewrite every line
// anyway. Then every amplitude is read and written once in lane order (unchanged ones bit-identical). pt maps target
// members (bit j <-> the j-th lowest target) and applies where every control bit is 1. Returns true if launched.
bool try_perm_lanes(qs_state *st, uint64_t tmask, uint64_t cmask, const PermTable &pt, int *rc)
{
    const uint64_t qmask = tmask | cmask;
    const int nq = __builtin_popcountll(qmask);
    const int LB = st->dtype == QS_C128 ? 6 : 7;          // in-wave index bits
    const int line = st->dtype == QS_C128 ? 3 : 4;        // index bits inside a 128-byte line
    if (nq > 6 || (qmask & (((uint64_t)1 << line) - 1)) == 0)
        return false;
    PermLanes pl{};
    int ut[6];  // member bit u -> target index, or -1 for a control
    int nh = 0;
    for (int p = 0, j = 0; p < 64; ++p) {
        if (!((qmask >> p) & 1))
            continue;
        pl.qpos[pl.nq] = p;
        ut[pl.nq] = ((tmask >> p) & 1) ? j++ : -1;
        nh += p >= LB;
        ++pl.nq;
    }
    if (nh > 2 || st->n < LB + nh)
        return false;
    uint64_t changed = 0;  // members a (over Q) whose amplitude changes
    for (int a = 0; a < (1 << nq); ++a) {
        bool on = true;
        int ta = 0;
        for (int u = 0; u < nq; ++u) {
            const int bit = (a >> u) & 1;
            if (ut[u] < 0)
                on = on && bit;
            else
                ta |= bit << ut[u];
        }
        int src = a, ph = 0;
        if (on) {
            const int s_ = pt.src[ta];
            ph = pt.phase[ta];
            src = 0;
            for (int u = 0; u < nq; ++u)
                src |= (ut[u] < 0 ? (a >> u) & 1 : (s_ >> ut[u]) & 1) << u;
        }
        pl.src[a] = (uint8_t)src;
        pl.phase[a] = (uint8_t)ph;
        if (src != a || ph != 0)
            changed |= (uint64_t)1 << a;
    }
    // every line holds a changed amplitude: each pattern of the Q bits above the line has one under some pattern of
    // the Q bits inside it
    int in_line = 0;
    for (int u = 0; u < nq; ++u)
        in_line |= (pl.qpos[u] < line) << u;
    for (int hi = 0; hi < (1 << nq); ++hi) {
        if (hi & in_line)
            continue;
        bool any = false;
        for (int lo = in_line;; lo = (lo - 1) & in_line) {
            any = any || ((changed >> (hi | lo)) & 1);
            if (lo == 0)
                break;
        }
        if (!any)
            return false;
    }
    hipError_t e = launch_perm_lanes(st->dtype, st->psi, st->n, pl, st->stream);
    *rc = e == hipSuccess ? QS_OK : qs_hip_fail(e, "launch_perm_lanes");
    return true;
}

// Dense / monomial gate on `targets`, restricted to indices whose `cmask` bits are all 1.
int matrix_impl(qs_state *st, const int *targets, int k, uint64_t tmask, uint64_t cmask, const double *U)
{
    const int n = st->n;
    TPos tp{};
    int perm[QS_MAX_DIAG_K];
    qs_sort_targets(targets, k, tp, perm);
    std::vector<double> Us;
    qs_permute_matrix(U, k, perm, Us);
    const InsBits ins = qs_make_ins(tmask | cmask, cmask);
    const int nins = __builtin_popcountll(tmask | cmask);
    const uint64_t ngroups = (uint64_t)1 << (n - nins);
    PermTable pt;
    if (monomial_table(Us, k, pt)) {
        if (!pt.moving)
            return QS_OK;  // identity
        int rc = QS_OK;
        if (try_perm_lanes(st, tmask, cmask, pt, &rc))
            return rc;
        QS_HIP(launch_perm(st->dtype, k, st->psi, ngroups, ins, tp, pt, st->stream));
        return QS_OK;
    }
    const void *Ud = nullptr;
    if (k >= 4) {  // matrices beyond the kernel-argument budget go through the staging ring
        if (st->dtype == QS_C128) {
            Ud = qs_stage(st, Us.data(), Us.size() * sizeof(double));
        } else {
            std::vector<float> f(Us.begin(), Us.end());
            Ud = qs_stage(st, f.data(), f.size() * sizeof(float));
        }
        if (!Ud)
            return QS_EDEVICE;
    }
    QS_HIP(launch_dense(st->dtype, k, st->psi, ngroups, ins, tp, Us.data(), Ud, st->stream));
    return QS_OK;
}

int diag_impl(qs_state *st, const int *targets, int k, const double *d)
{
    const int D = 1 << k;
    std::vector<uint8_t> cls(D);
    int m = 0;
    for (int a = 0; a < D; ++a) {
        const double re = d[2 * a], im = d[2 * a + 1];
        cls[a] = (re == 1.0 && im == 0.0) ? 0 : (re == -1.0 && im == 0.0) ? 1 : 2;
        m += cls[a] != 0;
    }
    if (m == 0)
        return QS_OK;
    uint64_t tmask = 0;
    for (int j = 0; j < k; ++j)
        tmask |= (uint64_t)1 << targets[j];
    // a diagonal of phases 1, -1, i, -i that changes part of every 128-byte line: the lane-order move form (exact,
    // every amplitude streamed once) instead of a strided pass that would fetch and partly rewrite every line
    if (m < D && k <= 6) {
        PermTable pt{};
        bool mono = true;
        for (int a = 0; a < D && mono; ++a) {
            const double re = d[2 * a], im = d[2 * a + 1];
            pt.src[a] = (uint8_t)a;
            if (re == 1.0 && im == 0.0)
                pt.phase[a] = 0;
            else if (re == 0.0 && im == 1.0)
                pt.phase[a] = 1;
            else if (re == -1.0 && im == 0.0)
                pt.phase[a] = 2;
            else if (re == 0.0 && im == -1.0)
                pt.phase[a] = 3;
            else
                mono = false;
        }
        if (mono) {
            // member bit j <-> the j-th lowest target; d is indexed in the caller's target order
            int order[QS_MAX_DIAG_K];
            for (int j = 0; j < k; ++j)
                order[j] = j;
            std::sort(order, order + k, [&](int x, int y) { return targets[x] < targets[y]; });
            PermTable ps{};
            for (int as = 0; as < D; ++as) {
                int a = 0;
                for (int j = 0; j < k; ++j)
                    a |= ((as >> j) & 1) << order[j];
                ps.src[as] = (uint8_t)as;
                ps.phase[as] = pt.phase[a];
            }
            int rc = QS_OK;
            if (try_perm_lanes(st, tmask, 0, ps, &rc))
                return rc;
            bool quarter = false;  // an entry i or -i: a component exchange, kept exact (signed zeros) as a move
            for (int a = 0; a < D; ++a) {
                quarter = quarter || (ps.phase[a] & 1);
                if (ps.phase[a])
                    ps.moving |= (uint64_t)1 << a;
            }
            if (quarter) {
                TPos tp{};
                int perm[QS_MAX_DIAG_K];
                qs_sort_targets(targets, k, tp, perm);
                QS_HIP(launch_perm(st->dtype, k, st->psi, (uint64_t)1 << (st->n - k), qs_make_ins(tmask, 0), tp, ps,
                                   st->stream));
                return QS_OK;
            }
        }
    }
    if (m <= D / 2 && m <= kMaxSparseDiag) {
        // visit only the subspaces of the non-unit patterns: 2^(n-k) amplitudes each
        DiagSparseEntry ent[kMaxSparseDiag];
        int e = 0;
        for (int a = 0; a < D; ++a) {
            if (!cls[a])
                continue;
            uint64_t orm = 0;
            for (int j = 0; j < k; ++j)
                if ((a >> j) & 1)
                    orm |= (uint64_t)1 << targets[j];
            ent[e].orm = orm;
            ent[e].re = d[2 * a];
            ent[e].im = d[2 * a + 1];
            ent[e].cls = cls[a];
            ++e;
        }
        const InsBits ins = qs_make_ins(tmask, 0);
        QS_HIP(launch_diag_sparse(st->dtype, st->psi, (uint64_t)1 << (st->n - k), ins, m, ent, st->stream));
        return QS_OK;
    }
    DiagArgs da{};
    da.k = k;
    for (int j = 0; j < k; ++j)
        da.t[j] = targets[j];
    const void *dd = nullptr, *cd = nullptr;
    if (k > 2) {
        if (st->dtype == QS_C128) {
            dd = qs_stage(st, d, (size_t)2 * D * sizeof(double));
        } else {
            std::vector<float> f(d, d + 2 * D);
            dd = qs_stage(st, f.data(), f.size() * sizeof(float));
        }
        if (!dd)
            return QS_EDEVICE;
        cd = qs_stage(st, cls.data(), cls.size());
        if (!cd)
            return QS_EDEVICE;
    }
    QS_HIP(launch_diag_full(st->dtype, st->psi, (uint64_t)1 << st->n, da, d, dd, cls.data(), cd, st->stream));
    return QS_OK;
}

}  // namespace

// ============================================================================================================
// C ABI
// ============================================================================================================
extern "C" {

QS_API int qs_alloc(qs_state **out, int n, int dtype, void *dev_buf, void *hip_stream)
{
    qs_clear_error();
    if (!out)
        return qs_fail(QS_EINVAL, "qs_alloc: out is NULL");
    *out = nullptr;
    if (n < 1 || n > QS_MAX_QUBITS)
        return qs_fail(QS_EINVAL, "qs_alloc: n = %d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dtype != QS_C128 && dtype != QS_C64)
        return qs_fail(QS_EINVAL, "qs_alloc: dtype = %d is neither QS_C128 nor QS_C64", dtype);
    if (dev_buf && ((uintptr_t)dev_buf & 255))
        return qs_fail(QS_EINVAL, "qs_alloc: dev_buf is not 256-byte aligned");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        return qs_fail(QS_EDEVICE, "qs_alloc: no HIP device is visible");
    }
    qs_state *st = new (std::nothrow) qs_state();
    if (!st)
        return qs_fail(QS_ENOMEM, "qs_alloc: out of host memory");
    st->n = n;
    st->dtype = dtype;
    st->stream = (hipStream_t)hip_stream;
    int rc = QS_OK;
    const size_t bytes = ((size_t)1 << n) * amp_bytes(dtype);
    hipError_t e = hipGetDevice(&st->device);
    if (e != hipSuccess) {
        rc = qs_hip_fail(e, "hipGetDevice");
        goto fail;
    }
    if (dev_buf) {
        st->psi = dev_buf;
    } else {
        e = hipMalloc(&st->psi, bytes);
        if (e != hipSuccess) {
            st->psi = nullptr;
            rc = qs_hip_fail(e, "hipMalloc(state)");
            goto fail;
        }
        st->owns = true;
    }
    st->ring_bytes = kRingBytes;
    e = hipHostMalloc((void **)&st->hring, kRingBytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        st->hring = nullptr;
        rc = qs_hip_fail(e, "hipHostMalloc(staging ring)");
        goto fail;
    }
    e = hipMalloc((void **)&st->dring, kRingBytes);
    if (e != hipSuccess) {
        st->dring = nullptr;
        rc = qs_hip_fail(e, "hipMalloc(staging ring)");
        goto fail;
    }
    for (int c = 0; c < kRingChunks; ++c) {
        e = hipEventCreateWithFlags(&st->ring_ev[c], hipEventDisableTiming);
        if (e != hipSuccess) {
            st->ring_ev[c] = nullptr;
            rc = qs_hip_fail(e, "hipEventCreate");
            goto fail;
        }
    }
    st->red_cap = kMaxPartials + 8;
    e = hipMalloc((void **)&st->red, st->red_cap * sizeof(double));
    if (e != hipSuccess) {
        st->red = nullptr;
        rc = qs_hip_fail(e, "hipMalloc(reduction scratch)");
        goto fail;
    }
    e = launch_init_zero(dtype, st->psi, (uint64_t)1 << n, st->stream);
    if (e != hipSuccess) {
        rc = qs_hip_fail(e, "init kernel launch");
        goto fail;
    }
    *out = st;
    return QS_OK;
fail:
    release(st);
    return rc;
}

QS_API int qs_free(qs_state *st)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_free: NULL handle");
    release(st);
    return QS_OK;
}

QS_API int qs_apply_gate(qs_state *st, const int *targets, int k, const double *U)
{
    qs_clear_error();
    if (!st || !targets || !U)
        return qs_fail(QS_EINVAL, "qs_apply_gate: NULL argument");
    if (k < 1 || k > QS_MAX_K || k > st->n)
        return qs_fail(QS_EINVAL, "qs_apply_gate: k = %d outside [1, min(%d, n = %d)]", k, QS_MAX_K, st->n);
    uint64_t tmask;
    if (int rc = check_qubits(st, targets, k, "targets", &tmask))
        return rc;
    if (is_diagonal(U, k)) {
        // exactly diagonal: entries on the diagonal, in the same bit order
        const int D = 1 << k;
        std::vector<double> d((size_t)2 * D);
        for (int a = 0; a < D; ++a) {
            d[2 * a] = U[2 * (a * D + a)];
            d[2 * a + 1] = U[2 * (a * D + a) + 1];
        }
        return diag_impl(st, targets, k, d.data());
    }
    return matrix_impl(st, targets, k, tmask, 0, U);
}

QS_API int qs_apply_diag(qs_state *st, const int *targets, int k, const double *d)
{
    qs_clear_error();
    if (!st || !targets || !d)
        return qs_fail(QS_EINVAL, "qs_apply_diag: NULL argument");
    if (k < 1 || k > QS_MAX_DIAG_K || k > st->n)
        return qs_fail(QS_EINVAL, "qs_apply_diag: k = %d outside [1, min(%d, n = %d)]", k, QS_MAX_DIAG_K, st->n);
    uint64_t tmask;
    if (int rc = check_qubits(st, targets, k, "targets", &tmask))
        return rc;
    return diag_impl(st, targets, k, d);
}

QS_API int qs_apply_controlled(qs_state *st, const int *controls, int c, const int *targets, int k, const double *U)
{
    qs_clear_error();
    if (!st || !controls || !targets || !U)
        return qs_fail(QS_EINVAL, "qs_apply_controlled: NULL argument");
    if (k < 1 || k > QS_MAX_K)
        return qs_fail(QS_EINVAL, "qs_apply_controlled: k = %d outside [1, %d]", k, QS_MAX_K);
    if (c < 1 || c > QS_MAX_CONTROLS)
        return qs_fail(QS_EINVAL, "qs_apply_controlled: c = %d outside [1, %d]", c, QS_MAX_CONTROLS);
    if (c + k > st->n)
        return qs_fail(QS_EINVAL, "qs_apply_controlled: c + k = %d exceeds n = %d", c + k, st->n);
    uint64_t tmask, cmask;
    if (int rc = check_qubits(st, targets, k, "targets", &tmask))
        return rc;
    if (int rc = check_qubits(st, controls, c, "controls", &cmask))
        return rc;
    if (tmask & cmask)
        return qs_fail(QS_EINVAL, "qs_apply_controlled: a control is also a target");
    return matrix_impl(st, targets, k, tmask, cmask, U);
}

QS_API int qs_fused_swap(qs_state *st, int p, int q, int s)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_fused_swap: NULL handle");
    if (s < 0 || p < 0 || q < 0)
        return qs_fail(QS_EINVAL, "qs_fused_swap: negative argument (p=%d q=%d s=%d)", p, q, s);
    if (s == 0)
        return QS_OK;
    if (p + s > st->n || q + s > st->n)
        return qs_fail(QS_EINVAL, "qs_fused_swap: range exceeds n = %d (p=%d q=%d s=%d)", st->n, p, q, s);
    const int lo = std::min(p, q), hi = std::max(p, q);
    if (lo + s > hi)
        return qs_fail(QS_EINVAL, "qs_fused_swap: ranges [%d,%d) and [%d,%d) overlap", p, p + s, q, q + s);
    QS_HIP(launch_fused_swap(st->dtype, st->psi, st->n, lo, hi, s, st->stream));
    return QS_OK;
}

QS_API int qs_probs(qs_state *st, double *out_dev, double *norm_out)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_probs: NULL handle");
    const uint64_t dim = (uint64_t)1 << st->n;
    const int nb = probs_blocks(dim);
    double *result = st->red + kMaxPartials;
    QS_HIP(launch_probs(st->dtype, st->psi, dim, out_dev, st->red, nb, result, st->stream));
    if (norm_out) {
        QS_HIP(hipMemcpyAsync(norm_out, result, sizeof(double), hipMemcpyDeviceToHost, st->stream));
        QS_HIP(hipStreamSynchronize(st->stream));
    }
    return QS_OK;
}

QS_API int qs_init_zero(qs_state *st)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_init_zero: NULL handle");
    QS_HIP(launch_init_zero(st->dtype, st->psi, (uint64_t)1 << st->n, st->stream));
    return QS_OK;
}

QS_API int qs_copy_in(qs_state *st, const void *host)
{
    qs_clear_error();
    if (!st || !host)
        return qs_fail(QS_EINVAL, "qs_copy_in: NULL argument");
    const size_t bytes = ((size_t)1 << st->n) * amp_bytes(st->dtype);
    QS_HIP(hipStreamSynchronize(st->stream));
    QS_HIP(hipMemcpy(st->psi, host, bytes, hipMemcpyHostToDevice));
    return QS_OK;
}

QS_API int qs_copy_out(qs_state *st, void *host)
{
    qs_clear_error();
    if (!st || !host)
        return qs_fail(QS_EINVAL, "qs_copy_out: NULL argument");
    const size_t bytes = ((size_t)1 << st->n) * amp_bytes(st->dtype);
    QS_HIP(hipStreamSynchronize(st->stream));
    QS_HIP(hipMemcpy(host, st->psi, bytes, hipMemcpyDeviceToHost));
    return QS_OK;
}

QS_API int qs_sync(qs_state *st)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_sync: NULL handle");
    QS_HIP(hipStreamSynchronize(st->stream));
    return QS_OK;
}

QS_API int qs_scale(qs_state *st, double f)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_scale: NULL handle");
    QS_HIP(launch_scale(st->dtype, st->psi, (uint64_t)1 << st->n, f, st->stream));
    return QS_OK;
}

QS_API int qs_norm(qs_state *st, double *norm_out)
{
    if (!norm_out) {
        qs_clear_error();
        return qs_fail(QS_EINVAL, "qs_norm: norm_out is NULL");
    }
    return qs_probs(st, nullptr, norm_out);
}

QS_API int qs_renormalize(qs_state *st, double *norm_before)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_renormalize: NULL handle");
    const uint64_t dim = (uint64_t)1 << st->n;
    const int nb = probs_blocks(dim);
    double *result = st->red + kMaxPartials;
    QS_HIP(launch_probs(st->dtype, st->psi, dim, nullptr, st->red, nb, result, st->stream));
    QS_HIP(launch_scale_dev(st->dtype, st->psi, dim, result, st->stream));
    if (norm_before) {
        QS_HIP(hipMemcpyAsync(norm_before, result, sizeof(double), hipMemcpyDeviceToHost, st->stream));
        QS_HIP(hipStreamSynchronize(st->stream));
    }
    return QS_OK;
}

QS_API int qs_get_info(qs_state *st, int *n, int *dtype, void **dev_ptr, void **hip_stream)
{
    qs_clear_error();
    if (!st)
        return qs_fail(QS_EINVAL, "qs_get_info: NULL handle");
    if (n)
        *n = st->n;
    if (dtype)
        *dtype = st->dtype;
    if (dev_ptr)
        *dev_ptr = st->psi;
    if (hip_stream)
        *hip_stream = (void *)st->stream;
    return QS_OK;
}

QS_API int qs_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    qs_clear_error();
    if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
        return qs_fail(QS_EINVAL, "qs_probe_copy: NULL or misaligned buffer or size");
    QS_HIP(launch_probe_copy(dst, src, bytes, (hipStream_t)hip_stream));
    return QS_OK;
}

QS_API int qs_probe_rmw(void *buf, size_t bytes, void *hip_stream)
{
    qs_clear_error();
    if (!buf || (bytes & 15) || ((uintptr_t)buf & 15))
        return qs_fail(QS_EINVAL, "qs_probe_rmw: NULL or misaligned buffer or size");
    QS_HIP(launch_probe_rmw(buf, bytes, (hipStream_t)hip_stream));
    return QS_OK;
}

QS_API int qs_get_tunable(const char *name, int64_t *value)
{
    qs_clear_error();
    if (!name || !value)
        return qs_fail(QS_EINVAL, "qs_get_tunable: NULL argument");
    const Tunables &t = qs_tunables();
    const std::pair<const char *, const std::atomic<int> *> all[] = {
        {"dense_gpt", &t.dense_gpt},          {"nontemporal", &t.nontemporal},
        {"mfma_wg_per_cu", &t.mfma_wg_per_cu}, {"block_wg_per_cu", &t.block_wg_per_cu},
        {"block_stage_width", &t.block_stage_width}, {"plan_beam", &t.plan_beam},
        {"plan_beam_search", &t.plan_beam_search}, {"block_async", &t.block_async},
        {"block_lanes", &t.block_lanes},      {"mfma_stage_ops", &t.mfma_stage_ops},
        {"stage_pack", &t.stage_pack}};
    for (const auto &kv : all)
        if (!std::strcmp(name, kv.first)) {
            *value = kv.second->load();
            return QS_OK;
        }
    return qs_fail(QS_EINVAL, "qs_get_tunable: unknown tunable '%s'", name);
}

QS_API int qs_set_tunable(const char *name, int64_t value)
{
    qs_clear_error();
    if (!name)
        return qs_fail(QS_EINVAL, "qs_set_tunable: NULL name");
    Tunables &t = qs_tunables();
    if (!std::strcmp(name, "dense_gpt")) {
        if (value != 1 && value != 2 && value != 4)
            return qs_fail(QS_EINVAL, "dense_gpt must be 1, 2 or 4");
        t.dense_gpt = (int)value;
    } else if (!std::strcmp(name, "nontemporal")) {
        t.nontemporal = value ? 1 : 0;
    } else if (!std::strcmp(name, "mfma_wg_per_cu")) {
        if (value < 1 || value > 16)
            return qs_fail(QS_EINVAL, "mfma_wg_per_cu must be in [1, 16]");
        t.mfma_wg_per_cu = (int)value;
    } else if (!std::strcmp(name, "block_wg_per_cu")) {
        if (value < 1 || value > 4096)
            return qs_fail(QS_EINVAL, "block_wg_per_cu must be in [1, 4096]");
        t.block_wg_per_cu = (int)value;
    } else if (!std::strcmp(name, "block_async")) {
        if (value != 0 && value != 1)
            return qs_fail(QS_EINVAL, "block_async must be 0 or 1");
        t.block_async = (int)value;
    } else if (!std::strcmp(name, "block_lanes")) {
        if (value != 0 && value != 1)
            return qs_fail(QS_EINVAL, "block_lanes must be 0 or 1");
        t.block_lanes = (int)value;
    } else if (!std::strcmp(name, "mfma_stage_ops")) {
        if (value < 0 || value > kStageMaxOps)
            return qs_fail(QS_EINVAL, "mfma_stage_ops must be in [0, %d]", kStageMaxOps);
        t.mfma_stage_ops = (int)value;
    } else if (!std::strcmp(name, "plan_beam")) {
        if (value < 0 || value > 64)
            return qs_fail(QS_EINVAL, "plan_beam must be in [0, 64]");
        t.plan_beam = (int)value;
    } else if (!std::strcmp(name, "plan_beam_search")) {
        if (value != 0 && value != 1)
            return qs_fail(QS_EINVAL, "plan_beam_search must be 0 or 1");
        t.plan_beam_search = (int)value;
    } else if (!std::strcmp(name, "stage_pack")) {
        if (value != 0 && value != 1)
            return qs_fail(QS_EINVAL, "stage_pack must be 0 or 1");
        t.stage_pack = (int)value;
    } else if (!std::strcmp(name, "block_stage_width")) {
        if (value != 3 && value != 4)
            return qs_fail(QS_EINVAL, "block_stage_width must be 3 or 4");
        t.block_stage_width = (int)value;
    } else {
        return qs_fail(QS_EINVAL, "qs_set_tunable: unknown tunable '%s'", name);
    }
    return QS_OK;
}

}  // extern "C"
