// Plain gate kernels of libqs for gfx950 (CDNA4, wave64).
//
// Every kernel is one in-place pass over the amplitudes it touches (HBM-bound): the gate rule of Sec. II-A,
// Eq. 4 applied to 2^k-member groups, the fused-swap permutation of Sec. III-D, and the FP64 probability /
// norm reduction. Group members are located by inserting zero bits at the (sorted) target and control
// positions of a group counter ("bit insert"); consecutive threads take consecutive counters, so every
// member stream is a coalesced 16-byte-per-lane stream whenever its bit positions are not the lowest ones.
#include "qs_internal.h"

#include <type_traits>

namespace {

template <class R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

__device__ __forceinline__ uint64_t ins0(uint64_t g, const InsBits &s) { return qs_ins0(g, s); }

template <int K> __device__ __forceinline__ uint64_t member_off(int a, const TPos &tp)
{
    return qs_member_off<K>(a, tp);
}

// Loads/stores with an optional non-temporal hint (the nontemporal builtins need native vector types).
template <class T> struct NativeVec;
template <> struct NativeVec<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NativeVec<float2> { typedef float type __attribute__((ext_vector_type(2))); };

template <class T> __device__ __forceinline__ T ld(const T *p, int nt)
{
    if (!nt)
        return *p;
    using N = typename NativeVec<T>::type;
    const N v = __builtin_nontemporal_load(reinterpret_cast<const N *>(p));
    T r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <class T> __device__ __forceinline__ void st(T *p, T v, int nt)
{
    if (!nt) {
        *p = v;
        return;
    }
    using N = typename NativeVec<T>::type;
    N w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<N *>(p));
}

// ---------------------------------------------------------------------------------------------------------
// dense k-qubit gate, k <= 4: the group's 2^k members live in registers; U comes from kernel arguments
// (k <= 3) or from device memory through uniform (scalar) loads (k = 4).
// ---------------------------------------------------------------------------------------------------------
template <class R, int K> struct MatByVal {
    R v[2 << (2 * K)];
    __device__ __forceinline__ R re(int i) const { return v[2 * i]; }
    __device__ __forceinline__ R im(int i) const { return v[2 * i + 1]; }
};
template <class R> struct MatByPtr {
    const R *__restrict__ p;
    __device__ __forceinline__ R re(int i) const { return p[2 * i]; }
    __device__ __forceinline__ R im(int i) const { return p[2 * i + 1]; }
};

// ---------------------------------------------------------------------------------------------------------
// 1-qubit gate whose target lies inside a wave's contiguous span (complex128: q < 6; complex64: q < 7). Every lane
// streams one 16-byte vector (one complex128 amplitude, or two adjacent complex64 ones) with full-width coalesced
// non-temporal loads and stores, and takes its pair partner from lane ^ 2^t by a cross-lane shuffle (complex64,
// q = 0: the partner is the other half of the lane's own vector). Each lane computes the outputs of its own
// amplitudes: a member with bit q = 0 gets U00 a + U01 b, with bit q = 1 gets U10 b + U11 a (b: the partner).
// The vector count is a multiple of 64 and so is the grid stride, so whole waves run the loop together.
// ---------------------------------------------------------------------------------------------------------
template <class R> struct LaneVec;
template <> struct LaneVec<double> { typedef double T __attribute__((ext_vector_type(2))); };
template <> struct LaneVec<float> { typedef float T __attribute__((ext_vector_type(4))); };

template <class R>
__device__ __forceinline__ void pair_out(R ar, R ai, R br, R bi, int bit, const MatByVal<R, 1> &m, R &outr, R &outi)
{
    // bit 0: U00 a + U01 b; bit 1: U11 a + U10 b
    const int ia = bit ? 3 : 0, ib = bit ? 2 : 1;
    const R ur = m.re(ia), ui = m.im(ia), vr = m.re(ib), vi = m.im(ib);
    outr = fma(ur, ar, fma(-ui, ai, fma(vr, br, -vi * bi)));
    outi = fma(ur, ai, fma(ui, ar, fma(vr, bi, vi * br)));
}

template <class R>
__global__ __launch_bounds__(256) void k_dense1_lane(typename LaneVec<R>::T *__restrict__ psi, uint64_t nvec, int q,
                                                     MatByVal<R, 1> m)
{
    using V = typename LaneVec<R>::T;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
        const V x = __builtin_nontemporal_load(psi + v);
        V y;
        if constexpr (sizeof(R) == 8) {
            const int d = 1 << q;
            const R pr = __shfl_xor(x.x, d, 64), pi = __shfl_xor(x.y, d, 64);
            const int bit = (int)((v >> q) & 1);
            R o0, o1;
            pair_out<R>(x.x, x.y, pr, pi, bit, m, o0, o1);
            y.x = o0;
            y.y = o1;
        } else {
            if (q == 0) {
                R o0, o1, o2, o3;
                pair_out<R>(x.x, x.y, x.z, x.w, 0, m, o0, o1);
                pair_out<R>(x.z, x.w, x.x, x.y, 1, m, o2, o3);
                y.x = o0;
                y.y = o1;
                y.z = o2;
                y.w = o3;
            } else {
                const int d = 1 << (q - 1);
                const R p0 = __shfl_xor(x.x, d, 64), p1 = __shfl_xor(x.y, d, 64);
                const R p2 = __shfl_xor(x.z, d, 64), p3 = __shfl_xor(x.w, d, 64);
                const int bit = (int)((v >> (q - 1)) & 1);
                R o0, o1, o2, o3;
                pair_out<R>(x.x, x.y, p0, p1, bit, m, o0, o1);
                pair_out<R>(x.z, x.w, p2, p3, bit, m, o2, o3);
                y.x = o0;
                y.y = o1;
                y.z = o2;
                y.w = o3;
            }
        }
        __builtin_nontemporal_store(y, psi + v);
    }
}


template <class R, int K, int G, class MS>
__global__ __launch_bounds__(256) void k_dense(typename CT<R>::T *__restrict__ psi, uint64_t ngroups, InsBits ins,
                                               TPos tp, MS ms, int nt)
{
    using C2 = typename CT<R>::T;
    constexpr int D = 1 << K;
    uint64_t off[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
        off[a] = member_off<K>(a, tp);
    const uint64_t bs = blockDim.x;
    const uint64_t stride = (uint64_t)gridDim.x * bs * G;
    for (uint64_t g0 = (uint64_t)blockIdx.x * bs * G + threadIdx.x; g0 < ngroups; g0 += stride) {
        C2 x[G][D];
        uint64_t base[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            uint64_t g = g0 + j * bs;
            base[j] = ins0(g < ngroups ? g : 0, ins);
            if (g < ngroups) {
#pragma unroll
                for (int a = 0; a < D; ++a)
                    x[j][a] = ld(psi + base[j] + off[a], nt);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (g0 + j * bs < ngroups) {
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    R yr = 0, yi = 0;
#pragma unroll
                    for (int b = 0; b < D; ++b) {
                        const R ur = ms.re(a * D + b), ui = ms.im(a * D + b);
                        yr = fma(ur, x[j][b].x, yr);
                        yr = fma(-ui, x[j][b].y, yr);
                        yi = fma(ur, x[j][b].y, yi);
                        yi = fma(ui, x[j][b].x, yi);
                    }
                    C2 y;
                    y.x = yr;
                    y.y = yi;
                    st(psi + base[j] + off[a], y, nt);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------------------------------------
// monomial ("permutation") gates: member a <- phase(a) * member src(a); pure moves, bit-exact.
// ---------------------------------------------------------------------------------------------------------
template <class C2> __device__ __forceinline__ C2 apply_phase(C2 x, int ph)
{
    C2 y;
    if (ph == 0) {
        y = x;
    } else if (ph == 1) {  // i * x
        y.x = -x.y;
        y.y = x.x;
    } else if (ph == 2) {  // -x
        y.x = -x.x;
        y.y = -x.y;
    } else {  // -i * x
        y.x = x.y;
        y.y = -x.x;
    }
    return y;
}

template <class R, int K, int G>
__global__ __launch_bounds__(256) void k_perm(typename CT<R>::T *__restrict__ psi, uint64_t ngroups, InsBits ins,
                                              TPos tp, PermTable pt, int nt)
{
    using C2 = typename CT<R>::T;
    constexpr int D = 1 << K;
    const uint64_t bs = blockDim.x;
    const uint64_t stride = (uint64_t)gridDim.x * bs * G;
    for (uint64_t g0 = (uint64_t)blockIdx.x * bs * G + threadIdx.x; g0 < ngroups; g0 += stride) {
        C2 v[G][D];
        uint64_t base[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            uint64_t g = g0 + j * bs;
            base[j] = ins0(g < ngroups ? g : 0, ins);
            if (g < ngroups) {
#pragma unroll
                for (int a = 0; a < D; ++a)
                    if ((pt.moving >> a) & 1)
                        v[j][a] = ld(psi + base[j] + member_off<K>(pt.src[a], tp), nt);
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (g0 + j * bs < ngroups) {
#pragma unroll
                for (int a = 0; a < D; ++a)
                    if ((pt.moving >> a) & 1)
                        st(psi + base[j] + member_off<K>(a, tp), apply_phase(v[j][a], pt.phase[a]), nt);
            }
        }
    }
}

// Lane-order form of a monomial op over Q for states where every 128-byte line holds amplitudes it changes (a CZ or
// controlled phase on qubits inside the line, a CNOT or Toffoli with a control there): a wave streams 64 consecutive
// 16-byte vectors (one complex128 amplitude or two complex64 ones per lane, LB = 6 or 7 in-wave index bits) for each
// of the 2^H combinations of the out-of-wave qubits of Q, so every access is a whole line in lane order, and each
// output takes its source from the lane, vector slot and member the move table names, by cross-lane reads. Which
// source feeds an output depends only on the lane, so it is worked out once per thread.
template <class R, int H>
__global__ __launch_bounds__(256) void k_perm_lanes(typename LaneVec<R>::T *__restrict__ psi, uint64_t nchunks,
                                                    InsBits ins_h, PermLanes pl)
{
    using V = typename LaneVec<R>::T;
    constexpr int P = sizeof(R) == 8 ? 1 : 2;  // amplitudes per 16-byte vector
    constexpr int LB = sizeof(R) == 8 ? 6 : 7;  // in-wave index bits
    constexpr int M = 1 << H;                   // members per lane
    const int lane = threadIdx.x & 63;
    uint64_t hoff[M];
    int sl[M][P], sp[M][P], sm[M][P], ph[M][P];
    {
        int hpos[2] = {0, 0}, nh = 0;
        for (int u = 0; u < pl.nq; ++u)
            if (pl.qpos[u] >= LB)
                hpos[nh++] = pl.qpos[u];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            hoff[m] = 0;
            for (int j = 0; j < H; ++j)
                hoff[m] |= (uint64_t)((m >> j) & 1) << hpos[j];
#pragma unroll
            for (int p = 0; p < P; ++p) {
                const int iw = lane * P + p;
                int a = 0;
                for (int u = 0, j = 0; u < pl.nq; ++u)
                    a |= (pl.qpos[u] < LB ? (iw >> pl.qpos[u]) & 1 : (m >> j++) & 1) << u;
                const int sa = pl.src[a];
                int siw = iw, smem = 0;
                for (int u = 0, j = 0; u < pl.nq; ++u) {
                    const int bit = (sa >> u) & 1;
                    if (pl.qpos[u] < LB)
                        siw = (siw & ~(1 << pl.qpos[u])) | (bit << pl.qpos[u]);
                    else
                        smem |= bit << j++;
                }
                sl[m][p] = siw / P;
                sp[m][p] = siw % P;
                sm[m][p] = smem;
                ph[m][p] = pl.phase[a];
            }
        }
    }
    const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    for (uint64_t c = wave; c < nchunks; c += nwaves) {
        const uint64_t base = qs_ins0(c << LB, ins_h) / P + lane;  // vector index of member 0
        V v[M];
#pragma unroll
        for (int m = 0; m < M; ++m)
            v[m] = __builtin_nontemporal_load(psi + base + hoff[m] / P);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            V y;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                // the source vector of every candidate member, read from the source lane; keep the named one
                R re = 0, im = 0;
#pragma unroll
                for (int cm = 0; cm < M; ++cm) {
                    R w[2 * P];
#pragma unroll
                    for (int e = 0; e < 2 * P; ++e)
                        w[e] = __shfl(v[cm][e], sl[m][p], 64);
                    if (cm == sm[m][p]) {
                        if constexpr (P == 1) {
                            re = w[0];
                            im = w[1];
                        } else {
                            re = sp[m][p] ? w[2] : w[0];
                            im = sp[m][p] ? w[3] : w[1];
                        }
                    }
                }
                typename CT<R>::T z;
                z.x = re;
                z.y = im;
                z = apply_phase(z, ph[m][p]);
                y[2 * p] = z.x;
                y[2 * p + 1] = z.y;
            }
            __builtin_nontemporal_store(y, psi + base + hoff[m] / P);
        }
    }
}

// ---------------------------------------------------------------------------------------------------------
// diagonal gates
// ---------------------------------------------------------------------------------------------------------
struct DiagSmall {  // k <= 2: entries and classes in kernel arguments (selected, never indexed)
    double re[4], im[4];
    int cls[4];  // 0: untouched (entry exactly 1), 1: negate (exactly -1), 2: multiply
};

template <class R, int K, int G>
__global__ __launch_bounds__(256) void k_diag_small(typename CT<R>::T *__restrict__ psi, uint64_t dim, DiagArgs da,
                                                    DiagSmall ds)
{
    using C2 = typename CT<R>::T;
    const uint64_t bs = blockDim.x;
    const uint64_t stride = (uint64_t)gridDim.x * bs * G;
    for (uint64_t i0 = (uint64_t)blockIdx.x * bs * G + threadIdx.x; i0 < dim; i0 += stride) {
        C2 x[G];
        int cl[G], pa[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t i = i0 + j * bs;
            int a = 0;
#pragma unroll
            for (int q = 0; q < K; ++q)
                a |= (int)((i >> da.t[q]) & 1) << q;
            pa[j] = a;
            cl[j] = i < dim ? ds.cls[a] : 0;
            if (cl[j])
                x[j] = ld(psi + i, 1);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (!cl[j])
                continue;
            const uint64_t i = i0 + j * bs;
            C2 y;
            if (cl[j] == 1) {
                y.x = -x[j].x;
                y.y = -x[j].y;
            } else {
                const R dr = (R)ds.re[pa[j]], di = (R)ds.im[pa[j]];
                y.x = fma(dr, x[j].x, -di * x[j].y);
                y.y = fma(dr, x[j].y, di * x[j].x);
            }
            st(psi + i, y, 1);
        }
    }
}

// complex64, k <= 2: each lane takes two adjacent amplitudes as one 16-byte vector (full-width lanes); a vector
// whose two entries are both 1 is neither read nor written, otherwise both are rewritten (an entry of 1 leaves
// its amplitude's bits unchanged).
template <int K>
__global__ __launch_bounds__(256) void k_diag_small_f2(float4 *__restrict__ psi, uint64_t nvec, DiagArgs da,
                                                       DiagSmall ds)
{
    typedef float F4 __attribute__((ext_vector_type(4)));
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nvec; v += stride) {
        int cl[2], pa[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t i = 2 * v + h;
            int a = 0;
#pragma unroll
            for (int q = 0; q < K; ++q)
                a |= (int)((i >> da.t[q]) & 1) << q;
            pa[h] = a;
            cl[h] = ds.cls[a];
        }
        if (!cl[0] && !cl[1])
            continue;
        F4 x = __builtin_nontemporal_load(reinterpret_cast<const F4 *>(psi + v));
        float re[2] = {x.x, x.z}, im[2] = {x.y, x.w};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (cl[h] == 1) {
                re[h] = -re[h];
                im[h] = -im[h];
            } else if (cl[h] == 2) {
                const float dr = (float)ds.re[pa[h]], di = (float)ds.im[pa[h]];
                const float r = fmaf(dr, re[h], -di * im[h]);
                im[h] = fmaf(dr, im[h], di * re[h]);
                re[h] = r;
            }
        }
        F4 y;
        y.x = re[0];
        y.y = im[0];
        y.z = re[1];
        y.w = im[1];
        __builtin_nontemporal_store(y, reinterpret_cast<F4 *>(psi + v));
    }
}

// k >= 3: the 2^k entries (in the compute precision) and classes come from device memory.
template <class R>
__global__ __launch_bounds__(256) void k_diag_table(typename CT<R>::T *__restrict__ psi, uint64_t dim, DiagArgs da,
                                                    const R *__restrict__ d, const uint8_t *__restrict__ cls)
{
    using C2 = typename CT<R>::T;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        int a = 0;
        for (int q = 0; q < da.k; ++q)
            a |= (int)((i >> da.t[q]) & 1) << q;
        const int c = cls[a];
        if (!c)
            continue;
        const C2 x = psi[i];
        C2 y;
        if (c == 1) {
            y.x = -x.x;
            y.y = -x.y;
        } else {
            const R dr = d[2 * a], di = d[2 * a + 1];
            y.x = fma(dr, x.x, -di * x.y);
            y.y = fma(dr, x.y, di * x.x);
        }
        psi[i] = y;
    }
}

struct SparseArgs {
    int m;
    DiagSparseEntry e[kMaxSparseDiag];
};

// Only the subspaces whose pattern has an entry != 1 are visited: blockIdx.y selects the pattern.
template <class R, int G>
__global__ __launch_bounds__(256) void k_diag_sparse(typename CT<R>::T *__restrict__ psi, uint64_t nsub,
                                                     InsBits ins, SparseArgs sa)
{
    using C2 = typename CT<R>::T;
    const DiagSparseEntry &e = sa.e[blockIdx.y];
    const uint64_t bs = blockDim.x;
    const uint64_t stride = (uint64_t)gridDim.x * bs * G;
    for (uint64_t g0 = (uint64_t)blockIdx.x * bs * G + threadIdx.x; g0 < nsub; g0 += stride) {
        C2 x[G];
        uint64_t idx[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const uint64_t g = g0 + j * bs;
            idx[j] = ins0(g < nsub ? g : 0, ins) | e.orm;
            if (g < nsub)
                x[j] = ld(psi + idx[j], 1);
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (g0 + j * bs >= nsub)
                continue;
            C2 y;
            if (e.cls == 1) {
                y.x = -x[j].x;
                y.y = -x[j].y;
            } else {
                const R dr = (R)e.re, di = (R)e.im;
                y.x = fma(dr, x[j].x, -di * x[j].y);
                y.y = fma(dr, x[j].y, di * x[j].x);
            }
            st(psi + idx[j], y, 1);
        }
    }
}

// ---------------------------------------------------------------------------------------------------------
// fused-swap (Sec. III-D, Listing 1): sigma exchanges bits [lo, lo+s) with [hi, hi+s), lo + s <= hi.
// Index layout: | top | A = bits [hi, hi+s) | mid | B = bits [lo, lo+s) | e = bits [0, lo) |.
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sigma_bits(uint64_t i, int lo, int hi, uint64_t smask)
{
    return fsw_sigma(i, lo, hi, smask);
}

// Generic form: one thread per index; the member of each moved pair with the smaller index does the swap.
template <class C2>
__global__ __launch_bounds__(256) void k_fswap_pairs(C2 *__restrict__ psi, uint64_t dim, int lo, int hi, uint64_t smask)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t j = sigma_bits(i, lo, hi, smask);
        if (j > i) {
            const C2 a = psi[i], b = psi[j];
            psi[i] = b;
            psi[j] = a;
        }
    }
}

// Run form (runs of at least 256 bytes, or one 128-byte line with s <= 4): thread -> (outer, pair a > b, element e);
// the runs (A=a, B=b) and (A=b, B=a) are exchanged with coalesced 16-byte lanes along e.
template <class C2>
__global__ __launch_bounds__(256) void k_fswap_runs(C2 *__restrict__ psi, uint64_t total, int lo, int hi, int s,
                                                    uint64_t npairs)
{
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t i1, i2;
        fsw_runs_pair(t, lo, hi, s, npairs, i1, i2);
        const C2 x1 = psi[i1], x2 = psi[i2];
        psi[i1] = x2;
        psi[i2] = x1;
    }
}

// LDS form (runs too short for the direct form): a workgroup exchanges the sub-tile pair (I, J) / (J, I) of one
// 2^s x 2^s tile (rows A, contiguous columns B of 2^lo-amplitude runs) through LDS; I == J transposes in
// place. Rows are read and written as contiguous (B, e) segments.
template <class C2, int TS>
__global__ __launch_bounds__(256) void k_fswap_lds(C2 *__restrict__ psi, uint64_t nwork, int lo, int hi, int s,
                                                   int ntile, uint64_t npairs_t)
{
    constexpr int T = 1 << TS;
    const int E = 1 << lo;
    const int row = T * E;         // amplitudes per sub-tile row
    const int rstride = row + 1;   // padded LDS row
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2 *X = reinterpret_cast<C2 *>(smem_raw);
    C2 *Y = X + (size_t)T * rstride;
    const int nel = T * row;
    (void)ntile;
    for (uint64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        uint64_t I, J, common;
        fsw_lds_item(w, lo, hi, s, npairs_t, I, J, common);
        // X: rows A in I-range, columns B in J-range.  Y: rows A in J-range, columns B in I-range.
        for (int u = threadIdx.x; u < nel; u += blockDim.x) {
            const int ra = u / row, rc = u % row;  // rc = cb * E + e
            X[ra * rstride + rc] = psi[fsw_lds_x(common, I, J, ra, rc, lo, hi, TS)];
            if (I != J)
                Y[ra * rstride + rc] = psi[fsw_lds_y(common, I, J, ra, rc, lo, hi, TS)];
        }
        lds_barrier();
        for (int u = threadIdx.x; u < nel; u += blockDim.x) {
            const int ra = u / row, rc = u % row;
            const int cb = rc / E, e = rc % E;
            // position (A = I*T + ra, B = J*T + cb) receives the old value at (A = J*T + cb, B = I*T + ra)
            if (I != J) {
                psi[fsw_lds_x(common, I, J, ra, rc, lo, hi, TS)] = Y[cb * rstride + ra * E + e];
                psi[fsw_lds_y(common, I, J, ra, rc, lo, hi, TS)] = X[cb * rstride + ra * E + e];
            } else if (ra != cb) {
                psi[fsw_lds_x(common, I, J, ra, rc, lo, hi, TS)] = X[cb * rstride + ra * E + e];
            }
        }
        lds_barrier();
    }
}

// Wide-row form for runs the direct form does not take, whose 2^s x 2^s tile fits 32 KiB. With x low "mid" bits carried along, the segment
// (mid_low, B, e) for fixed A is contiguous: 2^(x+s+lo) amplitudes (kilobytes). A workgroup loads the 2^s rows
// A = a of one work item with coalesced 16-byte lanes into LDS and writes every row b back with the element at
// (mid_low, B = a, e) taken from row a at (mid_low, B = b, e): 2^x independent 2^s x 2^s transposes at once.
// Fixed points (a == b) share cache lines with moved amplitudes at these sizes and are rewritten unchanged.
template <class C2>
__global__ __launch_bounds__(256) void k_fswap_wide(C2 *__restrict__ psi, uint64_t nwork, int lo, int hi, int s,
                                                    int x)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C2 *X = reinterpret_cast<C2 *>(smem_raw);
    const int R = 1 << (x + s + lo);  // amplitudes per row
    const int RP = R + 1;             // padded LDS row
    const int nel = (1 << s) * R;
    for (uint64_t w = blockIdx.x; w < nwork; w += gridDim.x) {
        const uint64_t base = fsw_wide_base(w, lo, hi, s, x);
        for (int u = threadIdx.x; u < nel; u += blockDim.x) {
            uint64_t g;
            int a, c;
            fsw_wide_load(base, u, lo, hi, s, x, g, a, c);
            X[a * RP + c] = psi[g];
        }
        lds_barrier();
        for (int u = threadIdx.x; u < nel; u += blockDim.x) {
            uint64_t g;
            int a, cs;
            fsw_wide_store(base, u, lo, hi, s, x, g, a, cs);
            psi[g] = X[a * RP + cs];
        }
        lds_barrier();
    }
}

// ---------------------------------------------------------------------------------------------------------
// probabilities, norm, scale, init
// ---------------------------------------------------------------------------------------------------------
__device__ __forceinline__ void kahan_add(double &s, double &c, double v)
{
    const double y = v - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
}

// out[i] = |a_i|^2 (FP64); partials[blockIdx.x] = compensated sum of this block's share, reduced in a fixed order.
template <class R>
__global__ __launch_bounds__(256) void k_probs(const typename CT<R>::T *__restrict__ psi, uint64_t dim,
                                               double *__restrict__ out, double *__restrict__ partials)
{
    __shared__ double red[256];
    double s = 0.0, c = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const auto x = psi[i];
        const double re = (double)x.x, im = (double)x.y;
        const double p = re * re + im * im;
        if (out)
            out[i] = p;
        kahan_add(s, c, p);
    }
    red[threadIdx.x] = s - c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        partials[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double *__restrict__ partials, int nb,
                                                      double *__restrict__ result)
{
    __shared__ double red[256];
    double s = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        kahan_add(s, c, partials[i]);
    red[threadIdx.x] = s - c;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        *result = red[0];
}

template <class R>
__global__ __launch_bounds__(256) void k_scale(typename CT<R>::T *__restrict__ psi, uint64_t dim, double f,
                                               const double *__restrict__ norm_dev)
{
    const double ff = norm_dev ? 1.0 / sqrt(*norm_dev) : f;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        auto x = psi[i];
        x.x = (R)((double)x.x * ff);
        x.y = (R)((double)x.y * ff);
        psi[i] = x;
    }
}

template <class R>
__global__ __launch_bounds__(256) void k_init_zero(typename CT<R>::T *__restrict__ psi, uint64_t dim)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        typename CT<R>::T v;
        v.x = i == 0 ? (R)1 : (R)0;
        v.y = 0;
        psi[i] = v;
    }
}

// ---------------------------------------------------------------------------------------------------------
// bandwidth probes
// ---------------------------------------------------------------------------------------------------------
template <int G>
__global__ __launch_bounds__(256) void k_probe_copy(double2 *__restrict__ dst, const double2 *__restrict__ src,
                                                    uint64_t nw)
{
    const uint64_t bs = blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * bs * G + threadIdx.x; i0 < nw; i0 += (uint64_t)gridDim.x * bs * G) {
        double2 v[G];
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (i0 + j * bs < nw)
                v[j] = src[i0 + j * bs];
#pragma unroll
        for (int j = 0; j < G; ++j)
            if (i0 + j * bs < nw)
                dst[i0 + j * bs] = v[j];
    }
}

// In-place pass: every 16-byte word is read, scaled by a runtime factor and written back (one word per thread,
// non-temporal), the access pattern of a gate pass with the arithmetic removed.
__global__ __launch_bounds__(256) void k_probe_rmw(double2 *__restrict__ buf, uint64_t nw, double f)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw; i += (uint64_t)gridDim.x * blockDim.x) {
        double2 v = ld(buf + i, 1);
        v.x *= f;
        v.y *= f;
        st(buf + i, v, 1);
    }
}

// Grid for a grid-stride loop over `work` items at `per_block` items per block. Streaming gate kernels run best
// with one item per thread and a grid that covers the work in a single sweep; the cap keeps the total thread
// count at or below 2^31 (the grid-stride loop covers anything larger).
unsigned grid_for(uint64_t work, uint64_t per_block)
{
    uint64_t b = (work + per_block - 1) / per_block;
    const uint64_t cap = (uint64_t)1 << 23;
    if (b > cap)
        b = cap;
    if (b == 0)
        b = 1;
    return (unsigned)b;
}

}  // namespace

Tunables &qs_tunables()
{
    static Tunables t;
    return t;
}

// =============================================================================================================
// launchers
// =============================================================================================================
hipError_t launch_init_zero(int dtype, void *psi, uint64_t dim, hipStream_t s)
{
    const unsigned g = grid_for(dim, 256 * 8);
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_init_zero<double>, dim3(g), dim3(256), 0, s, (double2 *)psi, dim);
    else
        hipLaunchKernelGGL(k_init_zero<float>, dim3(g), dim3(256), 0, s, (float2 *)psi, dim);
    return hipGetLastError();
}

namespace {
// Non-temporal accesses help streams of whole cache lines; when a target sits inside a 128-byte line the
// members of a group share lines across load instructions, so the loads go through the cache instead.
template <class R> int nt_for(const TPos &tp, int k)
{
    const int line_bits = sizeof(typename CT<R>::T) == 16 ? 3 : 4;
    for (int j = 0; j < k; ++j)
        if (tp.tpos[j] < line_bits)
            return 0;
    return qs_tunables().nontemporal;
}

template <class R, int K>
hipError_t dense_k(void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp, const double *Uh, const void *Ud,
                   hipStream_t s)
{
    using C2 = typename CT<R>::T;
    struct {
        int dense_gpt, nontemporal;
    } tu{qs_tunables().dense_gpt.load(), nt_for<R>(tp, K)};
    const int bs = 256;
    if constexpr (K <= 3) {
        MatByVal<R, K> m;
        for (int i = 0; i < (2 << (2 * K)); ++i)
            m.v[i] = (R)Uh[i];
        if constexpr (K == 1) {
            // a plain 1-qubit gate (no controls) whose partner lies inside the wave: the lane-exchange form
            // (measured faster than the group form on every such target: 6.3 vs 5.5-6.0 TB/s)
            const int lane_limit = sizeof(R) == 8 ? 6 : 7;
            const uint64_t dim = ngroups * 2;
            const uint64_t nvec = sizeof(R) == 8 ? dim : dim / 2;
            if (ins.np == 1 && ins.orm == 0 && tp.tpos[0] < lane_limit && nvec >= 64 && nvec % 64 == 0) {
                hipLaunchKernelGGL((k_dense1_lane<R>), dim3(grid_for(nvec, bs)), dim3(bs), 0, s,
                                   (typename LaneVec<R>::T *)psi, nvec, tp.tpos[0], m);
                return hipGetLastError();
            }
        }
        if (K <= 2 && tu.dense_gpt == 4) {
            hipLaunchKernelGGL((k_dense<R, K, 4, MatByVal<R, K>>), dim3(grid_for(ngroups, bs * 4)), dim3(bs), 0, s,
                               (C2 *)psi, ngroups, ins, tp, m, tu.nontemporal);
        } else if (K <= 2 && tu.dense_gpt == 2) {
            hipLaunchKernelGGL((k_dense<R, K, 2, MatByVal<R, K>>), dim3(grid_for(ngroups, bs * 2)), dim3(bs), 0, s,
                               (C2 *)psi, ngroups, ins, tp, m, tu.nontemporal);
        } else {
            hipLaunchKernelGGL((k_dense<R, K, 1, MatByVal<R, K>>), dim3(grid_for(ngroups, bs)), dim3(bs), 0, s,
                               (C2 *)psi, ngroups, ins, tp, m, tu.nontemporal);
        }
    } else if constexpr (K == 4) {
        MatByPtr<R> m{(const R *)Ud};
        hipLaunchKernelGGL((k_dense<R, 4, 1, MatByPtr<R>>), dim3(grid_for(ngroups, bs)), dim3(bs), 0, s, (C2 *)psi,
                           ngroups, ins, tp, m, tu.nontemporal);
    } else {
        return launch_dense_mfma(std::is_same<R, double>::value ? QS_C128 : QS_C64, K, psi, ngroups, ins, tp, Ud, s);
    }
    return hipGetLastError();
}

template <class R>
hipError_t dense_r(int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp, const double *Uh,
                   const void *Ud, hipStream_t s)
{
    switch (k) {
    case 1: return dense_k<R, 1>(psi, ngroups, ins, tp, Uh, Ud, s);
    case 2: return dense_k<R, 2>(psi, ngroups, ins, tp, Uh, Ud, s);
    case 3: return dense_k<R, 3>(psi, ngroups, ins, tp, Uh, Ud, s);
    case 4: return dense_k<R, 4>(psi, ngroups, ins, tp, Uh, Ud, s);
    case 5: return dense_k<R, 5>(psi, ngroups, ins, tp, Uh, Ud, s);
    case 6: return dense_k<R, 6>(psi, ngroups, ins, tp, Uh, Ud, s);
    default: return hipErrorInvalidValue;
    }
}

template <class R, int K>
hipError_t perm_k(void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp, const PermTable &pt, hipStream_t s)
{
    using C2 = typename CT<R>::T;
    constexpr int G = 1;
    hipLaunchKernelGGL((k_perm<R, K, G>), dim3(grid_for(ngroups, 256 * G)), dim3(256), 0, s, (C2 *)psi, ngroups, ins,
                       tp, pt, nt_for<R>(tp, K));
    return hipGetLastError();
}

template <class R>
hipError_t perm_r(int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp, const PermTable &pt,
                  hipStream_t s)
{
    switch (k) {
    case 1: return perm_k<R, 1>(psi, ngroups, ins, tp, pt, s);
    case 2: return perm_k<R, 2>(psi, ngroups, ins, tp, pt, s);
    case 3: return perm_k<R, 3>(psi, ngroups, ins, tp, pt, s);
    case 4: return perm_k<R, 4>(psi, ngroups, ins, tp, pt, s);
    case 5: return perm_k<R, 5>(psi, ngroups, ins, tp, pt, s);
    case 6: return perm_k<R, 6>(psi, ngroups, ins, tp, pt, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_dense(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                        const double *U_host_sorted, const void *U_dev, hipStream_t s)
{
    return dtype == QS_C128 ? dense_r<double>(k, psi, ngroups, ins, tp, U_host_sorted, U_dev, s)
                            : dense_r<float>(k, psi, ngroups, ins, tp, U_host_sorted, U_dev, s);
}

hipError_t launch_perm(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                       const PermTable &pt, hipStream_t s)
{
    return dtype == QS_C128 ? perm_r<double>(k, psi, ngroups, ins, tp, pt, s)
                            : perm_r<float>(k, psi, ngroups, ins, tp, pt, s);
}

hipError_t launch_perm_lanes(int dtype, void *psi, int n, const PermLanes &pl, hipStream_t s)
{
    const int LB = dtype == QS_C128 ? 6 : 7;
    int h = 0;
    uint64_t hmask = 0;
    for (int u = 0; u < pl.nq; ++u)
        if (pl.qpos[u] >= LB) {
            ++h;
            hmask |= (uint64_t)1 << pl.qpos[u];
        }
    if (pl.nq < 1 || pl.nq > 6 || h > 2 || n < LB + h)
        return hipErrorInvalidValue;
    const InsBits ins_h = qs_make_ins(hmask, 0);
    const uint64_t nchunks = (uint64_t)1 << (n - LB - h);
    const unsigned g = grid_for(nchunks * 64, 256);
    if (dtype == QS_C128) {
        using V = LaneVec<double>::T;
        if (h == 0)
            hipLaunchKernelGGL((k_perm_lanes<double, 0>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
        else if (h == 1)
            hipLaunchKernelGGL((k_perm_lanes<double, 1>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
        else
            hipLaunchKernelGGL((k_perm_lanes<double, 2>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
    } else {
        using V = LaneVec<float>::T;
        if (h == 0)
            hipLaunchKernelGGL((k_perm_lanes<float, 0>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
        else if (h == 1)
            hipLaunchKernelGGL((k_perm_lanes<float, 1>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
        else
            hipLaunchKernelGGL((k_perm_lanes<float, 2>), dim3(g), dim3(256), 0, s, (V *)psi, nchunks, ins_h, pl);
    }
    return hipGetLastError();
}

hipError_t launch_diag_full(int dtype, void *psi, uint64_t dim, const DiagArgs &da, const double *d_host,
                            const void *d_dev, const uint8_t *cls_host, const void *cls_dev, hipStream_t s)
{
    const int G = 1;
    if (da.k <= 2) {
        DiagSmall ds{};
        for (int a = 0; a < (1 << da.k); ++a) {
            ds.re[a] = d_host[2 * a];
            ds.im[a] = d_host[2 * a + 1];
            ds.cls[a] = cls_host[a];
        }
        const unsigned g = grid_for(dim, 256 * G);
        if (dtype == QS_C128) {
            if (da.k == 1)
                hipLaunchKernelGGL((k_diag_small<double, 1, G>), dim3(g), dim3(256), 0, s, (double2 *)psi, dim, da, ds);
            else
                hipLaunchKernelGGL((k_diag_small<double, 2, G>), dim3(g), dim3(256), 0, s, (double2 *)psi, dim, da, ds);
        } else {
            const uint64_t nvec = dim / 2;
            const unsigned gv = grid_for(nvec, 256);
            if (da.k == 1)
                hipLaunchKernelGGL((k_diag_small_f2<1>), dim3(gv), dim3(256), 0, s, (float4 *)psi, nvec, da, ds);
            else
                hipLaunchKernelGGL((k_diag_small_f2<2>), dim3(gv), dim3(256), 0, s, (float4 *)psi, nvec, da, ds);
        }
    } else {
        const unsigned g = grid_for(dim, 256);
        if (dtype == QS_C128)
            hipLaunchKernelGGL(k_diag_table<double>, dim3(g), dim3(256), 0, s, (double2 *)psi, dim, da,
                               (const double *)d_dev, (const uint8_t *)cls_dev);
        else
            hipLaunchKernelGGL(k_diag_table<float>, dim3(g), dim3(256), 0, s, (float2 *)psi, dim, da,
                               (const float *)d_dev, (const uint8_t *)cls_dev);
    }
    return hipGetLastError();
}

hipError_t launch_diag_sparse(int dtype, void *psi, uint64_t nsub, const InsBits &ins, int m,
                              const DiagSparseEntry *ent, hipStream_t s)
{
    if (m < 1 || m > kMaxSparseDiag)
        return hipErrorInvalidValue;
    SparseArgs sa{};
    sa.m = m;
    for (int i = 0; i < m; ++i)
        sa.e[i] = ent[i];
    const int G = 1;
    const dim3 grid(grid_for(nsub, 256 * G), m);
    if (dtype == QS_C128)
        hipLaunchKernelGGL((k_diag_sparse<double, G>), grid, dim3(256), 0, s, (double2 *)psi, nsub, ins, sa);
    else
        hipLaunchKernelGGL((k_diag_sparse<float, G>), grid, dim3(256), 0, s, (float2 *)psi, nsub, ins, sa);
    return hipGetLastError();
}

namespace {
template <class C2>
hipError_t fswap_t(void *psi_, int n, int lo, int hi, int s_, hipStream_t s)
{
    C2 *psi = (C2 *)psi_;
    const FswPlan f = fsw_plan(n, lo, hi, s_, (int)sizeof(C2));
    const unsigned g = (unsigned)(f.nwork < (1u << 20) ? f.nwork : (1u << 20));
    switch (f.form) {
    case FSW_RUNS:
        hipLaunchKernelGGL(k_fswap_runs<C2>, dim3(grid_for(f.nwork, 256)), dim3(256), 0, s, psi, f.nwork, lo, hi, s_,
                           f.npairs);
        break;
    case FSW_WIDE:
        hipLaunchKernelGGL(k_fswap_wide<C2>, dim3(g), dim3(256), f.shm, s, psi, f.nwork, lo, hi, s_, f.x);
        break;
    case FSW_LDS: {
        const int ntile = 1 << (s_ - f.ts);
        switch (f.ts) {
        case 2: hipLaunchKernelGGL((k_fswap_lds<C2, 2>), dim3(g), dim3(256), f.shm, s, psi, f.nwork, lo, hi, s_, ntile, f.npairs); break;
        case 3: hipLaunchKernelGGL((k_fswap_lds<C2, 3>), dim3(g), dim3(256), f.shm, s, psi, f.nwork, lo, hi, s_, ntile, f.npairs); break;
        case 4: hipLaunchKernelGGL((k_fswap_lds<C2, 4>), dim3(g), dim3(256), f.shm, s, psi, f.nwork, lo, hi, s_, ntile, f.npairs); break;
        default: hipLaunchKernelGGL((k_fswap_lds<C2, 5>), dim3(g), dim3(256), f.shm, s, psi, f.nwork, lo, hi, s_, ntile, f.npairs); break;
        }
        break;
    }
    default:
        hipLaunchKernelGGL(k_fswap_pairs<C2>, dim3(grid_for(f.nwork, 256)), dim3(256), 0, s, psi, f.nwork, lo, hi,
                           ((uint64_t)1 << s_) - 1);
        break;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_fused_swap(int dtype, void *psi, int n, int lo, int hi, int s_, hipStream_t s)
{
    return dtype == QS_C128 ? fswap_t<double2>(psi, n, lo, hi, s_, s) : fswap_t<float2>(psi, n, lo, hi, s_, s);
}

int probs_blocks(uint64_t dim)
{
    uint64_t b = (dim + 256 * 16 - 1) / (256 * 16);
    if (b > 4096)
        b = 4096;
    return (int)(b ? b : 1);
}

hipError_t launch_probs(int dtype, const void *psi, uint64_t dim, double *out, double *partials, int nblocks,
                        double *result, hipStream_t s)
{
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_probs<double>, dim3(nblocks), dim3(256), 0, s, (const double2 *)psi, dim, out, partials);
    else
        hipLaunchKernelGGL(k_probs<float>, dim3(nblocks), dim3(256), 0, s, (const float2 *)psi, dim, out, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, (const double *)partials, nblocks, result);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int nb, double *result, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_scale(int dtype, void *psi, uint64_t dim, double f, hipStream_t s)
{
    const unsigned g = grid_for(dim, 256 * 4);
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(256), 0, s, (double2 *)psi, dim, f, (const double *)nullptr);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(256), 0, s, (float2 *)psi, dim, f, (const double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_scale_dev(int dtype, void *psi, uint64_t dim, const double *norm_dev, hipStream_t s)
{
    const unsigned g = grid_for(dim, 256 * 4);
    if (dtype == QS_C128)
        hipLaunchKernelGGL(k_scale<double>, dim3(g), dim3(256), 0, s, (double2 *)psi, dim, 0.0, norm_dev);
    else
        hipLaunchKernelGGL(k_scale<float>, dim3(g), dim3(256), 0, s, (float2 *)psi, dim, 0.0, norm_dev);
    return hipGetLastError();
}

hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const uint64_t nw = bytes / 16;
    constexpr int G = 4;
    hipLaunchKernelGGL(k_probe_copy<G>, dim3(grid_for(nw, 256 * G)), dim3(256), 0, s, (double2 *)dst,
                       (const double2 *)src, nw);
    return hipGetLastError();
}

hipError_t launch_probe_rmw(void *buf, size_t bytes, hipStream_t s)
{
    const uint64_t nw = bytes / 16;
    hipLaunchKernelGGL(k_probe_rmw, dim3(grid_for(nw, 256)), dim3(256), 0, s, (double2 *)buf, nw, 1.0);
    return hipGetLastError();
}
