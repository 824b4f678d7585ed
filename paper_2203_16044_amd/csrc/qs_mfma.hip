// Dense k-qubit blocks (k = 5, 6) on the matrix cores (gfx950 MFMA).
//
// A k-qubit gate (Sec. II-A, Eq. 4 generalised) is the product Y = U X of the 2^k x 2^k matrix U with the
// 2^k x G matrix X whose columns are the amplitude groups (members = target-bit patterns). It is run as the
// real product Y' = A' X' with interleaved (re, im) rows:
//   A'[2a+0][2b+0] = Re U[a][b]   A'[2a+0][2b+1] = -Im U[a][b]
//   A'[2a+1][2b+0] = Im U[a][b]   A'[2a+1][2b+1] =  Re U[a][b]
// on 16x16x4 MFMA tiles (FP64 for complex128, FP32 with FP32 accumulation for complex64).
//
// Work split: a workgroup of 4 waves walks column tiles of 16 consecutive groups. Wave w owns the output rows
// [w*16*RT, (w+1)*16*RT) of Y' and keeps its slice of A' in registers for the whole launch. Each column tile
// (2^k members x 16 groups) is loaded with 16-byte lanes into an LDS buffer (double-buffered: the next tile's
// global loads are in flight while the current one is multiplied), the B operand is read from LDS, and the
// accumulators hold complete (re, im) pairs, stored back as 16-byte (complex128) / 8-byte (complex64) lanes.
#include "qs_internal.h"

namespace {

// Lane layouts of the 16x16x4 MFMAs (both types): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// The accumulator differs: lane l, register r holds D[4 (l / 16) + r][l % 16] for FP32 but
// D[l / 16 + 4 r][l % 16] for FP64 (measured on gfx950). Tile row i of A' is therefore assigned to the
// (member, component) pair that makes registers (0, 1) and (2, 3) of every lane two complete (re, im) pairs:
// members 2 (l / 16) and 2 (l / 16) + 1 of the tile.
template <class R> struct MF;
template <> struct MF<double> {
    using C2 = double2;
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // tile row i = l/16 + 4 r  ->  member 2 (i % 4) + (i / 8), component (i / 4) % 2
    static __device__ __forceinline__ int row_member(int i) { return 2 * (i & 3) + (i >> 3); }
    static __device__ __forceinline__ int row_comp(int i) { return (i >> 2) & 1; }
};
template <> struct MF<float> {
    using C2 = float2;
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // tile row i = 4 (l/16) + r  ->  member i / 2, component i % 2
    static __device__ __forceinline__ int row_member(int i) { return i >> 1; }
    static __device__ __forceinline__ int row_comp(int i) { return i & 1; }
};

__device__ __forceinline__ uint64_t ins0m(uint64_t g, const InsBits &s) { return qs_ins0(g, s); }

template <int K> __device__ __forceinline__ uint64_t moff(int a, const TPos &tp) { return qs_member_off<K>(a, tp); }

template <class R, int K>
__global__ __launch_bounds__(256) void k_dense_mfma(typename MF<R>::C2 *__restrict__ psi, uint64_t ngroups,
                                                    InsBits ins, TPos tp, const R *__restrict__ U)
{
    using C2 = typename MF<R>::C2;
    using acc_t = typename MF<R>::acc_t;
    constexpr int D = 1 << K;   // members per group
    constexpr int RT = D / 32;  // 16-row tiles of A' per wave (4 waves x RT x 16 = 2D rows)
    constexpr int KT = D / 4;   // member quads along the contraction; each quad feeds 2 MFMAs (re, im)
    constexpr int LPT = D / 16; // 16-byte loads per thread per column tile
    __shared__ C2 tile[2][D][16];

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int j = lane & 15, kq = lane >> 4;

    // this wave's slice of A': lane (i + 16 kk) holds A'[row i of the tile][contraction index kk of the step]
    R afr[RT][KT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int ao = (w * RT + rt) * 8 + MF<R>::row_member(j);  // output member of tile row j
        const int co = MF<R>::row_comp(j);
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            const int ai = 4 * t + kq;
            const R ur = U[2 * (ao * D + ai)], ui = U[2 * (ao * D + ai) + 1];
            afr[rt][t][0] = co == 0 ? ur : ui;   // multiplies Re x[ai]
            afr[rt][t][1] = co == 0 ? -ui : ur;  // multiplies Im x[ai]
        }
    }
    uint64_t loff[LPT];
#pragma unroll
    for (int it = 0; it < LPT; ++it)
        loff[it] = moff<K>((tid >> 4) + 16 * it, tp);
    uint64_t soff[RT][2];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int a0 = (w * RT + rt) * 8 + 2 * kq;  // D rows 4 kq .. 4 kq + 3 = members a0 (re, im), a0 + 1 (re, im)
        soff[rt][0] = moff<K>(a0, tp);
        soff[rt][1] = moff<K>(a0 + 1, tp);
    }

    const uint64_t ntiles = (ngroups + 15) / 16;
    const uint64_t G = gridDim.x;
    uint64_t T = blockIdx.x;
    if (T >= ntiles)
        return;
    int buf = 0;
    {
        const uint64_t g = T * 16 + (tid & 15);
        const bool ok = g < ngroups;
        const uint64_t base = ins0m(ok ? g : 0, ins);
#pragma unroll
        for (int it = 0; it < LPT; ++it) {
            C2 v;
            v.x = 0;
            v.y = 0;
            if (ok)
                v = psi[base + loff[it]];
            tile[0][(tid >> 4) + 16 * it][tid & 15] = v;
        }
    }
    lds_barrier();
    for (; T < ntiles; T += G) {
        const uint64_t Tn = T + G;
        // prefetch the next tile into registers
        C2 pre[LPT];
        const uint64_t gn = Tn * 16 + (tid & 15);
        const bool okn = Tn < ntiles && gn < ngroups;
        {
            const uint64_t bn = ins0m(okn ? gn : 0, ins);
#pragma unroll
            for (int it = 0; it < LPT; ++it) {
                pre[it].x = 0;
                pre[it].y = 0;
                if (okn)
                    pre[it] = psi[bn + loff[it]];
            }
        }
        // multiply the current tile: two partial accumulators per row tile keep two MFMA chains in flight
        acc_t acc[RT][2];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
            acc[rt][0] = acc[rt][1] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < KT; ++t) {
            const C2 bv = tile[buf][4 * t + kq][j];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                acc[rt][t & 1] = MF<R>::mma(afr[rt][t][0], bv.x, acc[rt][t & 1]);
                acc[rt][t & 1] = MF<R>::mma(afr[rt][t][1], bv.y, acc[rt][t & 1]);
            }
        }
        const uint64_t g = T * 16 + j;
        if (g < ngroups) {
            const uint64_t base = ins0m(g, ins);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                const acc_t s = acc[rt][0] + acc[rt][1];
                C2 y0, y1;
                y0.x = s[0];
                y0.y = s[1];
                y1.x = s[2];
                y1.y = s[3];
                psi[base + soff[rt][0]] = y0;
                psi[base + soff[rt][1]] = y1;
            }
        }
        if (Tn < ntiles) {
#pragma unroll
            for (int it = 0; it < LPT; ++it)
                tile[buf ^ 1][(tid >> 4) + 16 * it][tid & 15] = pre[it];
        }
        lds_barrier();
        buf ^= 1;
    }
}

template <class R, int K>
hipError_t mfma_k(void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp, const void *U, hipStream_t s)
{
    const uint64_t ntiles = (ngroups + 15) / 16;
    uint64_t grid = (uint64_t)qs_cu_count() * qs_tunables().mfma_wg_per_cu;
    if (grid > ntiles)
        grid = ntiles;
    hipLaunchKernelGGL((k_dense_mfma<R, K>), dim3((unsigned)grid), dim3(256), 0, s, (typename MF<R>::C2 *)psi,
                       ngroups, ins, tp, (const R *)U);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_dense_mfma(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                             const void *U_dev, hipStream_t s)
{
    if (dtype == QS_C128) {
        if (k == 5)
            return mfma_k<double, 5>(psi, ngroups, ins, tp, U_dev, s);
        if (k == 6)
            return mfma_k<double, 6>(psi, ngroups, ins, tp, U_dev, s);
    } else {
        if (k == 5)
            return mfma_k<float, 5>(psi, ngroups, ins, tp, U_dev, s);
        if (k == 6)
            return mfma_k<float, 6>(psi, ngroups, ins, tp, U_dev, s);
    }
    return hipErrorInvalidValue;
}
