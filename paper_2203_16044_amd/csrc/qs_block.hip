// LDS-staged multi-gate blocks ("local qubits" on one GPU).
//
// mpiQulacs splits the qubits of a distributed state into local ones (inside one process's memory, no
// communication) and global ones (Sec. III-B), and uses fused-swaps to bring global qubits into the local range
// before operating on them (Sec. III-D). On one GPU the same split appears between a workgroup's LDS and HBM: a
// workgroup gathers the 2^B amplitudes whose index bits over a chosen qubit set L (|L| = B) vary, the other bits
// fixed by the block number; every queued gate whose qubits lie in L is then applied in LDS, and the block is
// written back once. L is arbitrary, so the gather plays the role of the fused-swap remap without an extra pass;
// it always contains the lowest index bits so that every HBM segment is at least a full cache line.
//
// Inside the block the pass's ops are grouped into stages of at most 4 local qubits. In a stage every thread holds
// the 16 amplitudes of a group (the stage's 4 positions varying) in registers, applies all of the stage's ops there
// and writes the group back: one LDS round trip and one barrier per stage instead of per op. The stage records live
// in device memory: 4 ascending local positions, up to 8 ops as 4-bit masks of the stage positions they act on
// (k <= 3), and the pool offset of the first op's 2^k x 2^k matrix (compute precision; the others follow in order).
#include "qs_internal.h"

namespace {

template <class R> struct BT;
template <> struct BT<double> { using C2 = double2; };
template <> struct BT<float> { using C2 = float2; };

__device__ __forceinline__ uint64_t ins0b(uint64_t g, const InsBits &s) { return qs_ins0(g, s); }

// local index m -> global offset: bit t of m goes to global bit lpos[t]
__device__ __forceinline__ uint64_t spread(uint32_t m, const BlockMap &bm) { return qs_spread(m, bm); }

// LDS slot of local index m: its low 4 bits are XOR-ed with bits 4-7, 8-11 and 12, so local position p moves the
// 16-byte slot's bank group by the unit vector of class p mod 4. A stage's threads walk one position of each class
// with their lowest counter bits, so 16 consecutive lanes always touch 16 different bank groups.
__device__ __forceinline__ uint32_t swz(uint32_t m) { return blk_swz(m); }

// Apply a k-qubit op (k = popcount(MASK) <= 3) to the 2^W register amplitudes x[a], a = the W stage bits, writing
// the results to y (y must not alias x). Matrix bit j <-> the j-th set bit of MASK (ascending); U is 2^k x 2^k,
// interleaved, in the compute precision.
template <class R, int W, int MASK>
__device__ __forceinline__ void reg_op_to(const typename BT<R>::C2 *x, typename BT<R>::C2 *y, const R *__restrict__ U)
{
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;
    int bitpos[3] = {0, 0, 0};
    {
        int j = 0;
        for (int b = 0; b < W; ++b)
            if ((MASK >> b) & 1)
                bitpos[j++] = b;
    }
#pragma unroll
    for (int rest = 0; rest < (1 << W); ++rest) {
        if (rest & MASK)
            continue;  // enumerate the combinations of the other stage bits once
        int idx[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            int r = rest;
#pragma unroll
            for (int j = 0; j < K; ++j)
                r |= ((a >> j) & 1) << bitpos[j];
            idx[a] = r;
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            R yr = 0, yi = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const R ur = U[2 * (a * D + b)], ui = U[2 * (a * D + b) + 1];
                yr = fma(ur, x[idx[b]].x, yr);
                yr = fma(-ui, x[idx[b]].y, yr);
                yi = fma(ur, x[idx[b]].y, yi);
                yi = fma(ui, x[idx[b]].x, yi);
            }
            y[idx[a]].x = yr;
            y[idx[a]].y = yi;
        }
    }
}

// The same op in place.
template <class R, int W, int MASK>
__device__ __forceinline__ void reg_op(typename BT<R>::C2 *x, const R *__restrict__ U)
{
    typename BT<R>::C2 v[1 << W];
#pragma unroll
    for (int a = 0; a < (1 << W); ++a)
        v[a] = x[a];
    reg_op_to<R, W, MASK>(v, x, U);
}

template <class R, int W>
__device__ __forceinline__ void reg_op_dispatch(typename BT<R>::C2 *x, int mask, const R *__restrict__ U)
{
    if constexpr (W == 3) {
        switch (mask) {
        case 1: reg_op<R, 3, 1>(x, U); break;
        case 2: reg_op<R, 3, 2>(x, U); break;
        case 3: reg_op<R, 3, 3>(x, U); break;
        case 4: reg_op<R, 3, 4>(x, U); break;
        case 5: reg_op<R, 3, 5>(x, U); break;
        case 6: reg_op<R, 3, 6>(x, U); break;
        default: reg_op<R, 3, 7>(x, U); break;
        }
    } else {
        switch (mask) {
        case 1: reg_op<R, 4, 1>(x, U); break;
        case 2: reg_op<R, 4, 2>(x, U); break;
        case 3: reg_op<R, 4, 3>(x, U); break;
        case 4: reg_op<R, 4, 4>(x, U); break;
        case 5: reg_op<R, 4, 5>(x, U); break;
        case 6: reg_op<R, 4, 6>(x, U); break;
        case 7: reg_op<R, 4, 7>(x, U); break;
        case 8: reg_op<R, 4, 8>(x, U); break;
        case 9: reg_op<R, 4, 9>(x, U); break;
        case 10: reg_op<R, 4, 10>(x, U); break;
        case 11: reg_op<R, 4, 11>(x, U); break;
        case 12: reg_op<R, 4, 12>(x, U); break;
        case 13: reg_op<R, 4, 13>(x, U); break;
        default: reg_op<R, 4, 14>(x, U); break;
        }
    }
}

// Out-of-place dispatch over the masks of a 4-position stage (K2: ops on at most two positions only, whose matrix
// U may be a register array of 32 values: the largest such matrix, 4 x 4 complex, has 16 entries).
template <class R, bool K2>
__device__ __forceinline__ void reg_op_dispatch_to(const typename BT<R>::C2 *x, typename BT<R>::C2 *y, int mask,
                                                   const R *U)
{
    switch (mask) {
    case 1: reg_op_to<R, 4, 1>(x, y, U); break;
    case 2: reg_op_to<R, 4, 2>(x, y, U); break;
    case 3: reg_op_to<R, 4, 3>(x, y, U); break;
    case 4: reg_op_to<R, 4, 4>(x, y, U); break;
    case 5: reg_op_to<R, 4, 5>(x, y, U); break;
    case 6: reg_op_to<R, 4, 6>(x, y, U); break;
    case 8: reg_op_to<R, 4, 8>(x, y, U); break;
    case 9: reg_op_to<R, 4, 9>(x, y, U); break;
    case 10: reg_op_to<R, 4, 10>(x, y, U); break;
    default:
        if constexpr (K2) {
            reg_op_to<R, 4, 12>(x, y, U);
        } else {
            switch (mask) {
            case 7: reg_op_to<R, 4, 7>(x, y, U); break;
            case 11: reg_op_to<R, 4, 11>(x, y, U); break;
            case 12: reg_op_to<R, 4, 12>(x, y, U); break;
            case 13: reg_op_to<R, 4, 13>(x, y, U); break;
            default: reg_op_to<R, 4, 14>(x, y, U); break;
            }
        }
        break;
    }
}

// Byte offset in LDS of local index m. swz is linear over XOR and a group's base index m and a register offset
// off[a] have disjoint bits, so slot(m | off[a]) = slot(m) ^ slot(off[a]): the register offsets of a stage are
// computed once per stage (uniform) and every LDS access costs one XOR.
template <class C2>
__device__ __forceinline__ uint32_t slot_bytes(uint32_t m) { return swz(m) * (uint32_t)sizeof(C2); }
template <class C2>
__device__ __forceinline__ C2 &lds_at(C2 *s, uint32_t bytes)
{
    return *reinterpret_cast<C2 *>(reinterpret_cast<unsigned char *>(s) + bytes);
}

// LDS access by absolute byte address, for kernels whose only LDS is their dynamic buffer (which then starts at
// address 0; the launch checks that the kernel has no static LDS): no base address to add per access.
template <class R>
__device__ __forceinline__ typename BT<R>::C2 lds_get(uint32_t addr)
{
    using NV = typename NT2<R>::type;
    const NV v = *(const __attribute__((address_space(3))) NV *)(uintptr_t)addr;
    typename BT<R>::C2 c;
    c.x = v.x;
    c.y = v.y;
    return c;
}
template <class R>
__device__ __forceinline__ void lds_put(uint32_t addr, const typename BT<R>::C2 &c)
{
    using NV = typename NT2<R>::type;
    NV v;
    v.x = c.x;
    v.y = c.y;
    *(__attribute__((address_space(3))) NV *)(uintptr_t)addr = v;
}

// the stage's member offsets, formed by the planner for the plan's precision (slot_bytes of each member's offset)
template <class C2, int W>
__device__ __forceinline__ void stage_offsets(const BlkStage &stg, uint32_t *soff)
{
#pragma unroll
    for (int a = 0; a < (1 << W); ++a)
        soff[a] = stg.soff[a];
}

// One stage: every thread takes groups of 2^W amplitudes (the W stage positions varying), applies the stage's ops
// in registers and writes the group back. NT threads share the 2^(B-W) groups.
template <class R, int B, int W, int NT>
__device__ __forceinline__ void run_stage(typename BT<R>::C2 *s, const BlkStage &stg,
                                          const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    constexpr int NG = 1 << (B - W);
    uint32_t soff[1 << W];
    stage_offsets<C2, W>(stg, soff);
    for (int g = threadIdx.x; g < NG; g += NT) {
        uint32_t m = 0;
#pragma unroll
        for (int j = 0; j < B - W; ++j)
            m |= (((uint32_t)g >> j) & 1u) << stg.order[j];
        const uint32_t sm = slot_bytes<C2>(m);
        C2 x[1 << W];
#pragma unroll
        for (int a = 0; a < (1 << W); ++a)
            x[a] = lds_at(s, sm ^ soff[a]);
        uint32_t moff = stg.mat_base;
        for (int o = 0; o < stg.nops; ++o) {
            const int mask = (int)(stg.masks >> (4 * o)) & 15;
            reg_op_dispatch<R, W>(x, mask, mats + moff);
            moff += 2u << (2 * __builtin_popcount(mask));
        }
#pragma unroll
        for (int a = 0; a < (1 << W); ++a)
            lds_at(s, sm ^ soff[a]) = x[a];
    }
}

// Stage pipeline for workgroups with exactly one register group per thread (2^(B-W) == NT): the LDS addresses of a
// stage's 2^W members and its op fields are formed at the end of the previous stage, between its arithmetic and
// the barrier (the scalar load of the record and the address arithmetic then overlap the LDS writes and the wait
// for the other waves), so a stage starts with its reads right after the barrier. The group of thread t is t itself
// (its bits deposited at the positions `order` lists).
template <class R, int B, int W>
struct StagePipe {
    uint32_t addr[1 << W];  // LDS byte address of member a of this thread's group
    uint32_t masks, mat_base;
    int nops, mfma;
};

template <class R, int B, int W>
__device__ __forceinline__ void stage_fetch(StagePipe<R, B, W> &p, const BlkStage &stg, const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < B - W; ++j)
        m |= (((uint32_t)threadIdx.x >> j) & 1u) << stg.order[j];
    const uint32_t sm = slot_bytes<C2>(m);
#pragma unroll
    for (int a = 0; a < (1 << W); ++a)
        p.addr[a] = sm ^ stg.soff[a];
    p.masks = stg.masks;
    p.mat_base = stg.mat_base;
    p.nops = stg.nops;
    p.mfma = stg.mfma;
}

// Run stage `cur` (one group per thread) and form `nxt` from record `next` meanwhile. The ops alternate between two
// register arrays (x -> y -> x ...), so that no op's results have to be copied back over its inputs.
template <class R, int B, int W>
__device__ __forceinline__ void run_stage_piped(typename BT<R>::C2 *s, const StagePipe<R, B, W> &cur,
                                                StagePipe<R, B, W> &nxt, const BlkStage &next,
                                                const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    if constexpr (W != 4) {
        C2 x[1 << W];
#pragma unroll
        for (int a = 0; a < (1 << W); ++a)
            x[a] = lds_at(s, cur.addr[a]);
        uint32_t moff = cur.mat_base;
        for (int o = 0; o < cur.nops; ++o) {
            const int mask = (int)(cur.masks >> (4 * o)) & 15;
            reg_op_dispatch<R, W>(x, mask, mats + moff);
            moff += 2u << (2 * __builtin_popcount(mask));
        }
#pragma unroll
        for (int a = 0; a < (1 << W); ++a)
            lds_at(s, cur.addr[a]) = x[a];
        stage_fetch<R, B, W>(nxt, next, mats);
        return;
    }
    // The group is read into x when the stage has an odd number of ops (the first op then takes it to y) and into
    // y otherwise, so that pairs of ops (y -> x -> y) always leave it in y. (The empty asm statements keep the
    // compiler from hoisting the reads out of the two branches or merging the pair into one copying loop.)
    C2 x[16], y[16];
    uint32_t moff = cur.mat_base;
    int o = 0;
    if (cur.nops & 1) {
        asm volatile("; odd op count" ::: "memory");
#pragma unroll
        for (int a = 0; a < 16; ++a)
            x[a] = lds_get<R>(cur.addr[a]);
        const int mask = (int)(cur.masks & 15u);
        reg_op_dispatch_to<R, false>(x, y, mask, mats + moff);
        moff += 2u << (2 * __builtin_popcount(mask));
        o = 1;
    } else {
        asm volatile("; even op count" ::: "memory");
#pragma unroll
        for (int a = 0; a < 16; ++a)
            y[a] = lds_get<R>(cur.addr[a]);
    }
    for (; o < cur.nops; o += 2) {
        int mask = (int)(cur.masks >> (4 * o)) & 15;
        asm volatile("; y to x" ::: "memory");
        reg_op_dispatch_to<R, false>(y, x, mask, mats + moff);
        moff += 2u << (2 * __builtin_popcount(mask));
        mask = (int)(cur.masks >> (4 * (o + 1))) & 15;
        asm volatile("; x to y" ::: "memory");
        reg_op_dispatch_to<R, false>(x, y, mask, mats + moff);
        moff += 2u << (2 * __builtin_popcount(mask));
    }
#pragma unroll
    for (int a = 0; a < 16; ++a)
        lds_put<R>(cur.addr[a], y[a]);
    stage_fetch<R, B, W>(nxt, next, mats);
}

// A complex64 4-position stage as one dense product Y = M X on the matrix cores: M is the stage's fused 16 x 16
// complex matrix (its ops multiplied on the host; stage index bit j <-> pos[j]), X the 16 x 2^(B-4) matrix whose
// columns are the register groups. As in the dense MFMA kernel the product runs on real 16x16x4 FP32 tiles with
// interleaved (re, im) rows: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16], and register r of lane l
// holds D[4 (l / 16) + r][l % 16]; tile row i of A' is output member 8 rt + i / 2, component i % 2, so every lane's
// accumulators are two complete outputs. Each wave owns whole 16-group column tiles, so a tile is read and
// rewritten in place by one wave. slot_bytes is linear in XOR, so a member's LDS offset is the XOR of the offsets
// of its bits: no register array is indexed by a lane-dependent value.
template <int B, int NT>
__device__ __forceinline__ void run_stage_mfma(float2 *s, const BlkStage &stg, const float2 *Ml)
{
    typedef float acc_t __attribute__((ext_vector_type(4)));
    constexpr int NG = 1 << (B - 4);
    constexpr int NW = NT / 64;
    static_assert(NG % 16 == 0 && NT % 64 == 0, "MFMA stage shape");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 15, kq = lane >> 4;
    uint32_t soff[16];
    stage_offsets<float2, 4>(stg, soff);
    const uint32_t in_q = ((kq & 1) ? soff[1] : 0u) ^ ((kq & 2) ? soff[2] : 0u);   // members 4 t + kq
    const uint32_t out_q = ((kq & 1) ? soff[2] : 0u) ^ ((kq & 2) ? soff[4] : 0u);  // members 8 rt + 2 kq (+1)
    float afr[2][4][2];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const int ao = 8 * rt + (j >> 1), co = j & 1;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float2 u = Ml[ao * 16 + 4 * t + kq];
            afr[rt][t][0] = co == 0 ? u.x : u.y;   // multiplies Re x
            afr[rt][t][1] = co == 0 ? -u.y : u.x;  // multiplies Im x
        }
    }
    for (int ct = wv; ct < NG / 16; ct += NW) {
        const uint32_t g = (uint32_t)(ct * 16 + j);
        uint32_t m = 0;
#pragma unroll
        for (int b = 0; b < B - 4; ++b)
            m |= ((g >> b) & 1u) << stg.order[b];
        const uint32_t sm = slot_bytes<float2>(m);
        acc_t acc[2][2];
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
            acc[rt][0] = acc[rt][1] = acc_t{0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const float2 bv = lds_at(s, sm ^ soff[4 * t] ^ in_q);
#pragma unroll
            for (int rt = 0; rt < 2; ++rt) {
                acc[rt][t & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[rt][t][0], bv.x, acc[rt][t & 1], 0, 0, 0);
                acc[rt][t & 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[rt][t][1], bv.y, acc[rt][t & 1], 0, 0, 0);
            }
        }
#pragma unroll
        for (int rt = 0; rt < 2; ++rt) {
            const acc_t y = acc[rt][0] + acc[rt][1];
            const uint32_t o0 = sm ^ soff[8 * rt] ^ out_q;
            lds_at(s, o0) = make_float2(y[0], y[1]);
            lds_at(s, o0 ^ soff[1]) = make_float2(y[2], y[3]);
        }
    }
}

// A 4-position stage for a block of 2^nb amplitudes, nb <= B chosen at run time (whole small circuits in LDS).
template <class R>
__device__ __forceinline__ void run_stage_n(typename BT<R>::C2 *s, const BlkStage &stg,
                                            const R *__restrict__ mats, int nb)
{
    using C2 = typename BT<R>::C2;
    const int ng = (1 << nb) >> 4;
    uint32_t soff[16];
    stage_offsets<C2, 4>(stg, soff);
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        uint32_t m = 0;
        for (int j = 0; j < nb - 4; ++j)
            m |= (((uint32_t)g >> j) & 1u) << stg.order[j];
        const uint32_t sm = slot_bytes<C2>(m);
        C2 x[16];
#pragma unroll
        for (int a = 0; a < 16; ++a)
            x[a] = lds_at(s, sm ^ soff[a]);
        uint32_t moff = stg.mat_base;
        for (int o = 0; o < stg.nops; ++o) {
            const int mask = (int)(stg.masks >> (4 * o)) & 15;
            reg_op_dispatch<R, 4>(x, mask, mats + moff);
            moff += 2u << (2 * __builtin_popcount(mask));
        }
#pragma unroll
        for (int a = 0; a < 16; ++a)
            lds_at(s, sm ^ soff[a]) = x[a];
    }
}

// NT threads per workgroup: one register group per thread with 4-position stages (64 threads for 10-qubit blocks,
// 128 for 11, 256 for 12, 512 for complex128 13-qubit blocks, whose 128 KB hold a CU alone: 8 waves, 2 per SIMD);
// 512 with 3-position stages (8 register amplitudes per thread, so that two 64 KB complex128 blocks per CU run 16
// waves when the kernel stays within 128 VGPRs).
template <class R, int B, int W, int NT> struct BlockBounds {
    static constexpr int waves_per_eu = (NT == 512 && W == 3) || (sizeof(R) == 4 && NT >= 128 && B <= 12) ? 4 : 1;
};
// Complex64 blocks of 11-12 qubits (16-32 KB of LDS) are held to 128 VGPRs for 4 waves per SIMD: 2-4 % faster
// at 33 qubits than the 3 waves of the unconstrained ~130-VGPR build (the bound costs three 64-bit scratch reloads
// per block, outside the stage loop); 13-qubit complex64 blocks would spill far more and keep the compiler's choice.

// Threads of a block workgroup: one 2^W-amplitude group per thread (at least one wave; 4-position stages of
// complex64 13-qubit blocks take two groups per thread).
template <class R, int B, int W> struct BlockThreads {
    static constexpr int groups = 1 << (B - W);
    static constexpr int cap = sizeof(R) == 8 ? 512 : 256;
    static constexpr int value = W == 3 ? 512 : (groups < 64 ? 64 : (groups > cap ? cap : groups));
};

// RNF (complex64 only; a renormalisation folded into the passes on either side of it), a compile-time choice so
// that passes without it run the kernel without its registers: bit 1, the state is first scaled by
// 1 / sqrt(*scale_norm), in FP64, as each block is loaded; bit 2, norm_part[blockIdx.x] = FP64 sum of |amplitude|^2
// over every amplitude this workgroup stores (each workgroup's blocks in their fixed order, then a fixed reduction
// tree).
template <class R, int B, int W, int NT, int RNF = 0>
__global__ __launch_bounds__(NT, (BlockBounds<R, B, W, NT>::waves_per_eu)) void k_block(
    typename BT<R>::C2 *__restrict__ psi, uint64_t nblocks, InsBits outer, BlockMap bm,
    const BlkStage *__restrict__ stages, int nstages, const R *__restrict__ mats, BlkMfma mf,
    const double *__restrict__ scale_norm, double *__restrict__ norm_part)
{
    using C2 = typename BT<R>::C2;
    extern __shared__ __align__(16) unsigned char smem_blk[];
    C2 *s = reinterpret_cast<C2 *>(smem_blk);
    constexpr int N = 1 << B;
    constexpr bool MF = sizeof(R) == 4 && W == 4;  // complex64 stages may run fused on the matrix cores
    C2 *Ml = s + N;                                  // the pass's fused stage matrices (visible after the first barrier)
    if constexpr (MF) {
        for (int i = threadIdx.x; i < 256 * mf.n; i += NT) {
            const R *src = mats + mf.off[i >> 8] + 2 * (i & 255);
            Ml[i] = C2{src[0], src[1]};
        }
    }
    constexpr int PER = N / NT;  // amplitudes per thread for load / store
    constexpr int LNT = __builtin_ctz(NT);
    constexpr int PB = B - LNT;  // bits of the per-thread amplitude counter it
    static_assert(NT >= 16 && PB >= 1, "block kernel shape");
    // Local index m = tid + NT * it. Its HBM offset is spread(tid) (per thread) | spread(NT * it), the latter the OR of
    // hb[j] over the set bits j of it; its LDS slot is (swz(tid) ^ swz(NT * it) mod 16) + NT * it, since swz only
    // folds bits into the low 4. Both are recomputed at every use from a few registers (the empty asm statements keep
    // the compiler from hoisting 16-32 loop-invariant addresses into registers the stages need).
    const uint64_t own = spread(threadIdx.x, bm);
    uint64_t hb[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j)
        hb[j] = (uint64_t)1 << bm.lpos[LNT + j];
    const uint32_t sbase = slot_bytes<C2>(threadIdx.x);
    auto hi_of = [&](const uint64_t *h, int it) { return blk_hi<PB>(h, it); };
    auto slot_of = [&](uint32_t sb, int it) { return blk_phase_slot(sb, it, NT, (uint32_t)sizeof(C2)); };
    auto opaque_h = [&](uint64_t *h) {
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            h[j] = hb[j];
            asm volatile("" : "+s"(h[j]));
        }
    };
    auto opaque_s = [&]() {
        uint32_t sb = sbase;
        asm volatile("" : "+v"(sb));
        return sb;
    };
    // Software pipeline over this workgroup's blocks: the next block's global loads are issued into registers before
    // the current block's stages run, so HBM traffic overlaps the FP arithmetic. The loop is rotated so that wherever
    // the prefetched registers are consumed, exactly the prefetch loads and then the previous block's stores are in
    // flight: the wait needs only the loads (vmcnt(PER)) and the stores keep draining behind the next block's stages.
    using NV = typename NT2<R>::type;
    NV pre[PER];
    uint64_t blk = blockIdx.x;
    if (blk >= nblocks)
        return;
    static_assert(RNF >= 0 && RNF <= 3 && (RNF == 0 || sizeof(R) == 4), "folded renormalisation: complex64 only");
    constexpr bool SCL = (RNF & 1) != 0, NRM = (RNF & 2) != 0;
    double fsc = 1.0, nacc = 0.0;
    if constexpr (SCL)
        fsc = 1.0 / sqrt(*scale_norm);
    // one register group per thread: stage records are pipelined (complex128; the complex64 kernels, held to 128
    // VGPRs for 4 waves per SIMD, spill more with the addresses of the next stage live and measured slower)
    constexpr bool PIPED = (1 << (B - W)) == NT && sizeof(R) == 8;
    StagePipe<R, B, W> spc{}, spn{};  // the running stage and the next one
    if constexpr (PIPED) {
        if (nstages > 0)
            stage_fetch<R, B, W>(spc, stages[0], mats);
    }
    uint64_t base = ins0b(blk, outer) | own;
    {
        uint64_t h[PB];
        opaque_h(h);
        const C2 *pb = psi + base;
#pragma unroll
        for (int it = 0; it < PER; ++it)
            pre[it] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(pb + hi_of(h, it)));
        const uint32_t sb = opaque_s();
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            C2 v;
            v.x = pre[it].x;
            v.y = pre[it].y;
            if constexpr (SCL) {
                v.x = (R)((double)v.x * fsc);
                v.y = (R)((double)v.y * fsc);
            }
            lds_put<R>(slot_of(sb, it), v);
        }
    }
    lds_barrier();
    for (;;) {
        const uint64_t nxt = blk + gridDim.x;
        const bool more = nxt < nblocks;  // uniform
        const uint64_t nbase = ins0b(more ? nxt : blk, outer) | own;
        if (more) {
            uint64_t h[PB];
            opaque_h(h);
            const C2 *pb = psi + nbase;
#pragma unroll
            for (int it = 0; it < PER; ++it)
                pre[it] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(pb + hi_of(h, it)));
        }
        if constexpr (PIPED) {
            for (int t = 0; t < nstages; ++t) {
                // the record after the last stage is the first one again: the next block starts with it
                const BlkStage &next = stages[t + 1 < nstages ? t + 1 : 0];
                bool done = false;
                if constexpr (MF) {
                    if (spc.mfma >= 0) {
                        run_stage_mfma<B, NT>(s, stages[t], Ml + 256 * spc.mfma);
                        stage_fetch<R, B, W>(spn, next, mats);
                        done = true;
                    }
                }
                if (!done)
                    run_stage_piped<R, B, W>(s, spc, spn, next, mats);
                lds_barrier();
                spc = spn;
            }
        } else {
            for (int t = 0; t < nstages; ++t) {
                if constexpr (MF) {
                    const int slot = stages[t].mfma;
                    if (slot >= 0)
                        run_stage_mfma<B, NT>(s, stages[t], Ml + 256 * slot);
                    else
                        run_stage<R, B, W, NT>(s, stages[t], mats);
                } else {
                    run_stage<R, B, W, NT>(s, stages[t], mats);
                }
                lds_barrier();
            }
        }
        {
            uint64_t h[PB];
            opaque_h(h);
            C2 *pb = psi + base;
            const uint32_t sb = opaque_s();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const C2 v = lds_get<R>(slot_of(sb, it));
                if constexpr (NRM)
                    nacc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
                NV w;
                w.x = v.x;
                w.y = v.y;
                __builtin_nontemporal_store(w, reinterpret_cast<NV *>(pb + hi_of(h, it)));
            }
        }
        if (nxt >= nblocks)
            break;
        blk = nxt;
        base = nbase;
        lds_barrier();  // every thread has read its stored values out of LDS
        {
            const uint32_t sb = opaque_s();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                C2 v;
                v.x = pre[it].x;
                v.y = pre[it].y;
                if constexpr (SCL) {
                    v.x = (R)((double)v.x * fsc);
                    v.y = (R)((double)v.y * fsc);
                }
                lds_put<R>(slot_of(sb, it), v);
            }
        }
        lds_barrier();
    }
    if constexpr (NRM) {
        // the workgroup's sum: across each wave, then the waves' sums in wave order (LDS is free once every thread
        // has read its last block's values out of it)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
            nacc += __shfl_xor(nacc, off);
        lds_barrier();
        double *wsum = reinterpret_cast<double *>(smem_blk);
        if ((threadIdx.x & 63) == 0)
            wsum[threadIdx.x >> 6] = nacc;
        lds_barrier();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < NT / 64; ++w)
                t += wsum[w];
            norm_part[blockIdx.x] = t;
        }
    }
}

// ---------------------------------------------------------------------------------------------------------
// Lane-pair stages (complex128, 12-qubit blocks): a 4-position stage's 16-amplitude group is held by lanes l and
// l + 32 of a wave, 8 amplitudes each (register index a over three of the stage positions, the lane bit over the
// fourth), so that the 512-thread workgroups of two 64 KB blocks give a CU 16 waves (4 per SIMD) where the
// one-lane form gives 8, with the same stages and LDS round trips. An op on the lane's position is preceded by an
// exchange of the lane bit with a register bit it does not use (BlkStageL.swaps, chosen by the planner).
// ---------------------------------------------------------------------------------------------------------

// Exchange of the lane bit (thread bit 5) with register bit RB: for every a with bit RB clear, the upper
// half-wave's x[a] and the lower half-wave's x[a | 2^RB] trade places, which is what v_permlane32_swap does to
// its two operands (upper 32 lanes of the first with the lower 32 lanes of the second), one 32-bit word at a time.
__device__ __forceinline__ void swap_halves(double &u, double &v)
{
    const uint64_t bu = __builtin_bit_cast(uint64_t, u), bv = __builtin_bit_cast(uint64_t, v);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bu, (unsigned)bv, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bu >> 32), (unsigned)(bv >> 32), false, false);
    u = __builtin_bit_cast(double, (uint64_t)lo[0] | ((uint64_t)hi[0] << 32));
    v = __builtin_bit_cast(double, (uint64_t)lo[1] | ((uint64_t)hi[1] << 32));
}

template <int RB>
__device__ __forceinline__ void lane_swap_bit(double2 *x)
{
#pragma unroll
    for (int a = 0; a < 8; ++a) {
        if (a & (1 << RB))
            continue;
        swap_halves(x[a].x, x[a | 1 << RB].x);
        swap_halves(x[a].y, x[a | 1 << RB].y);
    }
}

// reg_op for the lane-pair stages, one group at a time: a scheduling barrier after each group's write-back keeps
// the compiler from interleaving the groups, so only one group's outputs are live beside the 8 amplitudes and the
// prefetched next block (the kernel has 128 registers for 4 waves per SIMD)
template <int MASK>
__device__ __forceinline__ void reg_op_seq(double2 *x, const double *__restrict__ U)
{
    constexpr int K = __builtin_popcount(MASK);
    constexpr int D = 1 << K;
    int bitpos[2] = {0, 0};
    {
        int j = 0;
        for (int b = 0; b < 3; ++b)
            if ((MASK >> b) & 1)
                bitpos[j++] = b;
    }
#pragma unroll
    for (int rest = 0; rest < 8; ++rest) {
        if (rest & MASK)
            continue;
        double2 v[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            int r = rest;
#pragma unroll
            for (int j = 0; j < K; ++j)
                r |= ((a >> j) & 1) << bitpos[j];
            v[a] = x[r];
        }
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double yr = 0, yi = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) {
                const double ur = U[2 * (a * D + b)], ui = U[2 * (a * D + b) + 1];
                yr = fma(ur, v[b].x, yr);
                yr = fma(-ui, v[b].y, yr);
                yi = fma(ur, v[b].y, yi);
                yi = fma(ui, v[b].x, yi);
            }
            int r = rest;
#pragma unroll
            for (int j = 0; j < K; ++j)
                r |= ((a >> j) & 1) << bitpos[j];
            x[r].x = yr;
            x[r].y = yi;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

__device__ __forceinline__ void run_stage_lanes(double2 *s, const BlkStageL &stg, const double *__restrict__ mats)
{
    const uint32_t t = threadIdx.x;
    const uint32_t g = (t & 31u) | ((t >> 6) << 5);  // group: lanes l and l + 32 share one
    const bool up = (t >> 5) & 1u;                   // the lane bit
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        m |= ((g >> j) & 1u) << stg.order[j];
    const uint32_t sm = slot_bytes<double2>(m);
    const uint32_t smr = sm ^ (up ? stg.rd_lane : 0u);
    double2 x[8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
        x[a] = lds_get<double>(smr ^ stg.rd[a]);
    uint32_t moff = stg.mat_base;
    for (int o = 0; o < stg.nops; ++o) {
        switch ((stg.swaps >> (2 * o)) & 3u) {
        case 1: lane_swap_bit<0>(x); break;
        case 2: lane_swap_bit<1>(x); break;
        case 3: lane_swap_bit<2>(x); break;
        default: break;
        }
        const int mask = (int)(stg.masks >> (4 * o)) & 7;  // one or two register bits (the planner's condition)
        switch (mask) {
        case 1: reg_op_seq<1>(x, mats + moff); break;
        case 2: reg_op_seq<2>(x, mats + moff); break;
        case 4: reg_op_seq<4>(x, mats + moff); break;
        case 3: reg_op_seq<3>(x, mats + moff); break;
        case 5: reg_op_seq<5>(x, mats + moff); break;
        default: reg_op_seq<6>(x, mats + moff); break;
        }
        moff += 2u << (2 * __builtin_popcount(mask));
    }
    const uint32_t smw = sm ^ (up ? stg.wr_lane : 0u);
#pragma unroll
    for (int a = 0; a < 8; ++a)
        lds_put<double>(smw ^ stg.wr[a], x[a]);
}

// The block loop of k_block (next block's loads issued into registers before the current block's stages, rotated
// so that the wait covers only those loads), 512 threads, 8 amplitudes per thread, lane-pair stages.
__global__ __launch_bounds__(512, 4) void k_block_lanes(double2 *__restrict__ psi, uint64_t nblocks, InsBits outer,
                                                        BlockMap bm, const BlkStageL *__restrict__ stages,
                                                        int nstages, const double *__restrict__ mats)
{
    using C2 = double2;
    extern __shared__ __align__(16) unsigned char smem_blk[];
    C2 *s = reinterpret_cast<C2 *>(smem_blk);
    constexpr int B = 12, NT = 512;
    constexpr int PER = (1 << B) / NT;
    constexpr int LNT = 9;
    constexpr int PB = B - LNT;
    const uint64_t own = spread(threadIdx.x, bm);  // this thread's offset inside a block (its bits at lpos[0..8])
    uint64_t hb[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j)
        hb[j] = (uint64_t)1 << bm.lpos[LNT + j];
    const uint32_t sbase = slot_bytes<C2>(threadIdx.x);
    auto opaque_h = [&](uint64_t *h) {
#pragma unroll
        for (int j = 0; j < PB; ++j) {
            h[j] = hb[j];
            asm volatile("" : "+s"(h[j]));
        }
    };
    auto opaque_s = [&]() {
        uint32_t sb = sbase;
        asm volatile("" : "+v"(sb));
        return sb;
    };
    using NV = typename NT2<double>::type;
    NV pre[PER];
    uint64_t blk = blockIdx.x;
    if (blk >= nblocks)
        return;
    uint64_t base = ins0b(blk, outer);  // the block's offset (uniform); `own` is OR-ed in at each access
    {
        uint64_t h[PB];
        opaque_h(h);
        const C2 *pb = psi + (base | own);
#pragma unroll
        for (int it = 0; it < PER; ++it)
            pre[it] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(pb + blk_hi<PB>(h, it)));
        const uint32_t sb = opaque_s();
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            C2 v;
            v.x = pre[it].x;
            v.y = pre[it].y;
            lds_put<double>(blk_phase_slot(sb, it, NT, (uint32_t)sizeof(C2)), v);
        }
    }
    lds_barrier();
    for (;;) {
        const uint64_t nxt = blk + gridDim.x;
        const bool more = nxt < nblocks;  // uniform
        const uint64_t nbase = ins0b(more ? nxt : blk, outer);
        if (more) {
            uint64_t h[PB];
            opaque_h(h);
            const C2 *pb = psi + (nbase | own);
#pragma unroll
            for (int it = 0; it < PER; ++it)
                pre[it] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(pb + blk_hi<PB>(h, it)));
        }
        for (int t = 0; t < nstages; ++t) {
            run_stage_lanes(s, stages[t], mats);
            lds_barrier();
        }
        {
            uint64_t h[PB];
            opaque_h(h);
            C2 *pb = psi + (base | own);
            const uint32_t sb = opaque_s();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const C2 v = lds_get<double>(blk_phase_slot(sb, it, NT, (uint32_t)sizeof(C2)));
                NV w;
                w.x = v.x;
                w.y = v.y;
                __builtin_nontemporal_store(w, reinterpret_cast<NV *>(pb + blk_hi<PB>(h, it)));
            }
        }
        if (nxt >= nblocks)
            break;
        blk = nxt;
        base = nbase;
        lds_barrier();  // every thread has read its stored values out of LDS
        {
            const uint32_t sb = opaque_s();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                C2 v;
                v.x = pre[it].x;
                v.y = pre[it].y;
                lds_put<double>(blk_phase_slot(sb, it, NT, (uint32_t)sizeof(C2)), v);
            }
        }
        lds_barrier();
    }
}

// Double-buffered block pass: the next block streams from HBM straight into the other LDS buffer (direct-to-LDS
// 16-byte loads, no registers involved) while the current block's stages run, so HBM traffic and arithmetic
// overlap inside one workgroup. Load instruction `it` of wave w fills slots [256 it + 64 w, +64), one 16-byte slot
// per lane in lane order; lane l fetches the element whose local index is swz(slot) (swz is an involution), so
// slot swz(m) holds local index m exactly as in k_block. Waits are explicit: before the stages a wave needs its
// loads of the current block, which precede at most the previous block's stores and the next block's loads.
// gfx9 s_waitcnt immediate waiting for vmcnt <= n only (expcnt and lgkmcnt left at their maxima)
template <int n> struct VmWait { static constexpr int imm = (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); };

// Workgroup barrier for the double-buffered pass: waits for this wave's LDS operations (lgkmcnt) only. A fence
// would also wait for the direct-to-LDS loads of the next block in flight, which count as LDS writes; the asm
// barrier with a memory clobber keeps the compiler from moving memory accesses across it, and the loads the
// stages read were waited for explicitly (vmcnt) before the first barrier of the block.
__device__ __forceinline__ void lds_sync_nofence()
{
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4) | (0 << 8));  // lgkmcnt(0); vmcnt, expcnt unconstrained
    asm volatile("s_barrier" ::: "memory");
}

template <class R, int B>
__global__ __launch_bounds__(256) void k_block_async(typename BT<R>::C2 *__restrict__ psi, uint64_t nblocks,
                                                     InsBits outer, BlockMap bm, const BlkStage *__restrict__ stages,
                                                     int nstages, const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    using NV = typename NT2<R>::type;
    constexpr int NT = 256;
    constexpr int N = 1 << B;
    constexpr int PER = N / NT;
    static_assert(PER == 16, "one 16-load fill per thread");
    extern __shared__ __align__(16) unsigned char smem_blk[];
    C2 *buf0 = reinterpret_cast<C2 *>(smem_blk);
    C2 *buf1 = buf0 + N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint64_t off[PER];  // load side: global offset (from the block base) of this lane's element for fill `it`
    uint64_t hi[PER];   // store side: as in k_block
#pragma unroll
    for (int it = 0; it < PER; ++it) {
        off[it] = spread(swz((uint32_t)(NT * it + 64 * wave + lane)), bm);
        hi[it] = spread((uint32_t)(NT * it), bm);
    }
    const uint64_t own = spread(threadIdx.x, bm);
    auto fill = [&](C2 *dst, uint64_t b) {
        const uint64_t base = ins0b(b, outer);
#pragma unroll
        for (int it = 0; it < PER; ++it)
            __builtin_amdgcn_global_load_lds((const void *)(psi + base + off[it]), (void *)(dst + NT * it + 64 * wave),
                                             16, 0, 0);
    };
    uint64_t blk = blockIdx.x;
    if (blk >= nblocks)
        return;
    fill(buf0, blk);
    bool first = true;
    int cur = 0;
    for (;;) {
        const uint64_t nxt = blk + gridDim.x;
        const bool more = nxt < nblocks;  // uniform
        C2 *sc = cur ? buf1 : buf0;
        C2 *sn = cur ? buf0 : buf1;
        if (more)
            fill(sn, nxt);  // sn was read out (previous block's stores) before the barrier that ended that block
        // this wave's loads of the current block are done once at most the loads and stores issued after them are
        // outstanding: first block: the next fill (PER); later: the previous stores (PER) and the next fill (PER)
        if (first || !more) {
            if (first && !more)
                __builtin_amdgcn_s_waitcnt(VmWait<0>::imm);
            else
                __builtin_amdgcn_s_waitcnt(VmWait<PER>::imm);
        } else {
            __builtin_amdgcn_s_waitcnt(VmWait<2 * PER>::imm);
        }
        lds_sync_nofence();  // every wave's part of the current block has landed in LDS
        for (int t = 0; t < nstages; ++t) {
            run_stage<R, B, 4, NT>(sc, stages[t], mats);
            lds_sync_nofence();
        }
        const uint64_t base = ins0b(blk, outer) | own;
#pragma unroll
        for (int it = 0; it < PER; ++it) {
            const C2 v = sc[swz(threadIdx.x + NT * it)];
            NV w;
            w.x = v.x;
            w.y = v.y;
            __builtin_nontemporal_store(w, reinterpret_cast<NV *>(psi + base + hi[it]));
        }
        if (!more)
            break;
        lds_sync_nofence();  // every thread has read its stored values out of sc before sc is refilled
        blk = nxt;
        cur ^= 1;
        first = false;
    }
}

// Batched circuits, level by level. A batch runs as a short sequence of persistent launches; launch k ("level k")
// executes pass k of every circuit that has more than k passes, all of those passes' blocks forming one flat index
// space that the whole grid walks, so a large circuit is spread over every CU instead of one workgroup. The items of
// a level are sorted by their first flat block; a workgroup finds the item of block g by binary search.
//   * a SMALL item (level 0 only, placed first) is a whole circuit of at most B qubits: one workgroup initialises,
//     evolves and measures it in LDS (FP64 probabilities written straight from LDS);
//   * any other item is one pass over a circuit of more than B qubits held in HBM: its FIRST pass generates the
//     basis state |0..0> in registers instead of reading it, its LAST pass writes |amp|^2 in FP64 instead of the
//     amplitudes. Passes of one circuit are ordered by the launch boundaries between levels.
// As in k_block, the next block's loads are issued before the current block's stages run (rotated loop).
__device__ __forceinline__ int find_item(const BatchItem *__restrict__ items, int nitems, uint32_t g)
{
    int lo = 0, hi = nitems - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].blk_begin <= g)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <class R, int B>
__device__ __forceinline__ void batch_small(typename BT<R>::C2 *s, const BatchItem &it, double *__restrict__ prob_base,
                                            const BatchPass *__restrict__ passes, const BlkStage *__restrict__ stages,
                                            const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    const uint32_t N = 1u << it.n;
    for (uint32_t m = threadIdx.x; m < N; m += blockDim.x) {
        C2 v;
        v.x = m == 0 ? (R)1 : (R)0;
        v.y = 0;
        s[swz(m)] = v;
    }
    lds_barrier();
    for (int p = 0; p < it.npass; ++p) {
        const BatchPass &bp = passes[it.pass + p];
        for (int t = 0; t < bp.nstages; ++t) {
            run_stage_n<R>(s, stages[bp.stage_begin + t], mats, it.n);
            lds_barrier();
        }
    }
    double *out = prob_base + it.prob_off;
    for (uint32_t m = threadIdx.x; m < N; m += blockDim.x) {
        const C2 v = s[swz(m)];
        const double re = (double)v.x, im = (double)v.y;
        out[m] = re * re + im * im;
    }
    lds_barrier();
}

// HBM offset of local index tid + 256 k of a batch block: spread(tid) | OR of h[j] over the set bits j of k, where
// h[j] = 1 << lpos[8 + j] (the block's map changes from block to block, so the four basis offsets are rebuilt per
// block and the sixteen offsets recomputed at every use, as in k_block).
template <int PB>
__device__ __forceinline__ void batch_basis(uint64_t *h, const BlockMap &bm)
{
#pragma unroll
    for (int j = 0; j < PB; ++j) {
        h[j] = (uint64_t)1 << bm.lpos[8 + j];
        asm volatile("" : "+s"(h[j]));
    }
}
template <int PB>
__device__ __forceinline__ uint64_t batch_hi(const uint64_t *h, int k)
{
    return blk_hi<PB>(h, k);
}
// LDS slot (bytes) of local index tid + 256 k from sb = slot_bytes(tid): swz only folds bits into the low 4
template <class C2>
__device__ __forceinline__ uint32_t batch_slot(uint32_t sb, int k)
{
    return blk_phase_slot(sb, k, 256, (uint32_t)sizeof(C2));
}
__device__ __forceinline__ uint32_t opaque_u32(uint32_t v)
{
    asm volatile("" : "+v"(v));
    return v;
}

// Loads of one block into registers. The loads are issued even for a FIRST pass (whose values are then replaced by
// the basis state) so that the wait before their use is the same on every path and can leave stores in flight.
template <class R, int B>
__device__ __forceinline__ void batch_fetch(typename NT2<R>::type *pre, const typename BT<R>::C2 *__restrict__ psi,
                                            uint64_t base, const BlockMap &bm)
{
    using NV = typename NT2<R>::type;
    constexpr int PER = (1 << B) / 256;
    constexpr int PB = B - 8;
    uint64_t h[PB];
    batch_basis<PB>(h, bm);
    const typename BT<R>::C2 *pb = psi + base;
#pragma unroll
    for (int it = 0; it < PER; ++it)
        pre[it] = __builtin_nontemporal_load(reinterpret_cast<const NV *>(pb + batch_hi<PB>(h, it)));
}

template <class R, int B>
__device__ __forceinline__ void batch_to_lds(typename BT<R>::C2 *s, const typename NT2<R>::type *pre, uint64_t base,
                                             const BlockMap &bm, bool first, uint32_t sbase)
{
    using C2 = typename BT<R>::C2;
    constexpr int PER = (1 << B) / 256;
    constexpr int PB = B - 8;
    uint64_t h[PB];
    batch_basis<PB>(h, bm);
    const uint32_t sb = opaque_u32(sbase);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        C2 v;
        if (first) {
            v.x = (base | batch_hi<PB>(h, k)) == 0 ? (R)1 : (R)0;
            v.y = 0;
        } else {
            v.x = pre[k].x;
            v.y = pre[k].y;
        }
        lds_at(s, batch_slot<C2>(sb, k)) = v;
    }
}

template <class R, int B>
__global__ __launch_bounds__(256, (sizeof(R) == 4 ? 4 : 1)) void k_batch_level(typename BT<R>::C2 *__restrict__ psi_base,
                                                     double *__restrict__ prob_base,
                                                     const BatchItem *__restrict__ items, int nitems, uint32_t nblocks,
                                                     const BatchPass *__restrict__ passes,
                                                     const BlkStage *__restrict__ stages,
                                                     const R *__restrict__ mats)
{
    using C2 = typename BT<R>::C2;
    using NV = typename NT2<R>::type;
    extern __shared__ __align__(16) unsigned char smem_blk[];
    C2 *s = reinterpret_cast<C2 *>(smem_blk);
    constexpr int PER = (1 << B) / 256;
    constexpr int PB = B - 8;
    // small items come first in the flat order: a workgroup runs its small circuits, then its HBM blocks
    uint32_t g = blockIdx.x;
    BatchItem cur{};
    for (; g < nblocks; g += gridDim.x) {
        cur = items[find_item(items, nitems, g)];
        if (!(cur.flags & kBatchSmall))
            break;
        batch_small<R, B>(s, cur, prob_base, passes, stages, mats);
    }
    if (g >= nblocks)
        return;
    // HBM blocks: the rotated pipeline of k_block (prefetch of the next block before the stages; waits only on the
    // prefetch loads, the previous block's stores keep draining). Complex64: the fused stage matrices of the next
    // block's pass (entry threadIdx.x of each) are fetched after the stages, before the stores, and written to LDS
    // beside the prefetched block.
    constexpr bool MF = sizeof(R) == 4;
    C2 *Ml = s + (1 << B);
    C2 mreg[kMaxMfmaStages];
    auto mfetch = [&](const BatchPass *p) {
        if constexpr (MF) {
#pragma unroll
            for (int i = 0; i < kMaxMfmaStages; ++i)
                if (i < p->mf.n) {
                    const R *src = mats + p->mf.off[i] + 2 * threadIdx.x;
                    mreg[i].x = src[0];
                    mreg[i].y = src[1];
                }
        }
    };
    auto mstore = [&](const BatchPass *p) {
        if constexpr (MF) {
#pragma unroll
            for (int i = 0; i < kMaxMfmaStages; ++i)
                if (i < p->mf.n)
                    Ml[256 * i + threadIdx.x] = mreg[i];
        }
    };
    const uint32_t sbase = slot_bytes<C2>(threadIdx.x);
    NV pre[PER];
    const BatchPass *bp = &passes[cur.pass];
    uint64_t base = ins0b(g - cur.blk_begin, bp->outer) | spread(threadIdx.x, bp->bm);
    batch_fetch<R, B>(pre, psi_base + cur.state_off, base, bp->bm);
    mfetch(bp);
    batch_to_lds<R, B>(s, pre, base, bp->bm, (cur.flags & kBatchFirst) != 0, sbase);
    mstore(bp);
    lds_barrier();
    for (;;) {
        const uint32_t nx = g + gridDim.x;
        const bool more = nx < nblocks;  // uniform
        const uint32_t ng = more ? nx : g;
        const BatchItem nt = items[find_item(items, nitems, ng)];
        const BatchPass *np = &passes[nt.pass];
        const uint64_t nbase = ins0b(ng - nt.blk_begin, np->outer) | spread(threadIdx.x, np->bm);
        if (more)
            batch_fetch<R, B>(pre, psi_base + nt.state_off, nbase, np->bm);
        for (int t = 0; t < bp->nstages; ++t) {
            const BlkStage &stg = stages[bp->stage_begin + t];
            if constexpr (MF) {
                if (stg.mfma >= 0)
                    run_stage_mfma<B, 256>(s, stg, Ml + 256 * stg.mfma);
                else
                    run_stage<R, B, 4, 256>(s, stg, mats);
            } else {
                run_stage<R, B, 4, 256>(s, stg, mats);
            }
            lds_barrier();
        }
        // issued before this block's stores, so the wait for the prefetch before the boundary covers them too
        if (more)
            mfetch(np);
        {
            uint64_t h[PB];
            batch_basis<PB>(h, bp->bm);
            const uint32_t sb = opaque_u32(sbase);
            if (cur.flags & kBatchLast) {
                double *out = prob_base + cur.prob_off + base;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const C2 v = lds_at(s, batch_slot<C2>(sb, k));
                    const double re = (double)v.x, im = (double)v.y;
                    out[batch_hi<PB>(h, k)] = re * re + im * im;
                }
            } else {
                C2 *psi = psi_base + cur.state_off + base;
#pragma unroll
                for (int k = 0; k < PER; ++k) {
                    const C2 v = lds_at(s, batch_slot<C2>(sb, k));
                    NV w;
                    w.x = v.x;
                    w.y = v.y;
                    __builtin_nontemporal_store(w, reinterpret_cast<NV *>(psi + batch_hi<PB>(h, k)));
                }
            }
        }
        if (nx >= nblocks)
            break;
        g = nx;
        cur = nt;
        bp = np;
        base = nbase;
        lds_barrier();  // every thread has read its stored values out of LDS
        batch_to_lds<R, B>(s, pre, base, bp->bm, (cur.flags & kBatchFirst) != 0, sbase);
        mstore(bp);
        lds_barrier();
    }
}

template <class R, int B>
hipError_t batch_b(void *psi, double *probs, const BatchItem *items, int nitems, uint32_t nblocks,
                   const BatchPass *passes, const BlkStage *stages, const void *mats,
                   int wg_per_cu, hipStream_t s)
{
    using C2 = typename BT<R>::C2;
    // complex64: room for a pass's fused stage matrices next to the block
    const size_t shm = (sizeof(C2) << B) + (sizeof(R) == 4 ? 256 * sizeof(C2) * kMaxMfmaStages : 0);
    if (hipError_t e = qs_allow_lds((const void *)k_batch_level<R, B>, shm))
        return e;
    uint64_t grid = (uint64_t)qs_cu_count() * wg_per_cu;
    if (grid > nblocks)
        grid = nblocks;
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL((k_batch_level<R, B>), dim3((unsigned)grid), dim3(256), shm, s, (C2 *)psi, probs, items, nitems,
                       nblocks, passes, stages, (const R *)mats);
    return hipGetLastError();
}

template <class R>
hipError_t batch_r(int b, void *psi, double *probs, const BatchItem *items, int nitems, uint32_t nblocks,
                   const BatchPass *passes, const BlkStage *stages, const void *mats,
                   int wg_per_cu, hipStream_t s)
{
    switch (b) {
    case 10: return batch_b<R, 10>(psi, probs, items, nitems, nblocks, passes, stages, mats, wg_per_cu, s);
    case 11: return batch_b<R, 11>(psi, probs, items, nitems, nblocks, passes, stages, mats, wg_per_cu, s);
    case 12: return batch_b<R, 12>(psi, probs, items, nitems, nblocks, passes, stages, mats, wg_per_cu, s);
    default: return hipErrorInvalidValue;
    }
}

// Persistent workgroups of a block pass: block_wg_per_cu counts 256-thread workgroups (smaller workgroups get
// proportionally more), at least one per CU, at most one per block.
uint64_t block_grid_nt(int nt, uint64_t nblocks)
{
    const uint64_t cus = (uint64_t)qs_cu_count();
    uint64_t grid = cus * qs_tunables().block_wg_per_cu * 256 / nt;
    if (grid < cus)
        grid = cus;
    if (grid > nblocks)
        grid = nblocks;
    return grid;
}

// One k_block variant: its LDS allowance, the absolute-addressing check, the launch.
template <class R, int B, int W, int NT, int RNF>
hipError_t launch_k_block(uint64_t grid, size_t shm, size_t shm_max, void *psi, uint64_t nblocks,
                          const InsBits &outer, const BlockMap &bm, const BlkStage *stages, int nstages,
                          const void *mats, const BlkMfma &mf, const BlkRenorm &rn, hipStream_t s)
{
    using C2 = typename BT<R>::C2;
    if (hipError_t e = qs_allow_lds((const void *)k_block<R, B, W, NT, RNF>, shm_max))
        return e;
    // the kernel addresses its LDS absolutely (lds_get / lds_put)
    if (hipError_t e = qs_check_no_static_lds((const void *)k_block<R, B, W, NT, RNF>))
        return e;
    hipLaunchKernelGGL((k_block<R, B, W, NT, RNF>), dim3((unsigned)grid), dim3(NT), shm, s, (C2 *)psi, nblocks, outer,
                       bm, stages, nstages, (const R *)mats, mf, rn.scale_norm, rn.norm_part);
    return hipGetLastError();
}

template <class R, int B, int W>
hipError_t block_b(void *psi, uint64_t nblocks, const InsBits &outer, const BlockMap &bm, const BlkStage *stages,
                   int nstages, const void *mats, const BlkMfma &mf, const BlkStageL *lstages, const BlkRenorm &rn,
                   hipStream_t s)
{
    using C2 = typename BT<R>::C2;
    constexpr int NT = BlockThreads<R, B, W>::value;
    static_assert((1 << B) >= NT, "block smaller than the workgroup");
    if (mf.n < 0 || mf.n > kMaxMfmaStages || (mf.n > 0 && (sizeof(R) != 4 || W != 4)))
        return hipErrorInvalidValue;
    const int rnf = (rn.scale_norm ? 1 : 0) | (rn.norm_part ? 2 : 0);
    if (rnf && sizeof(R) != 4)
        return hipErrorInvalidValue;  // folded renormalisation: complex64 block passes only
    const size_t data = sizeof(C2) << B;
    const size_t shm = data + 256 * sizeof(C2) * mf.n;
    const size_t shm_max = data + (sizeof(R) == 4 && W == 4 ? 256 * sizeof(C2) * kMaxMfmaStages : 0);
    // persistent workgroups (each walks several blocks so its loads can run ahead of its arithmetic)
    const uint64_t cus = (uint64_t)qs_cu_count();
    const uint64_t grid = block_grid_nt(NT, nblocks);
    if constexpr (B == 12 && W == 4 && sizeof(R) == 8) {
        if (lstages) {
            if (hipError_t e = qs_allow_lds((const void *)k_block_lanes, data))
                return e;
            if (hipError_t e = qs_check_no_static_lds((const void *)k_block_lanes))  // absolute LDS addressing
                return e;
            uint64_t g2 = cus * qs_tunables().block_wg_per_cu / 2;  // 512-thread workgroups
            if (g2 < cus)
                g2 = cus;
            if (g2 > nblocks)
                g2 = nblocks;
            hipLaunchKernelGGL(k_block_lanes, dim3((unsigned)g2), dim3(512), data, s, (double2 *)psi, nblocks, outer,
                               bm, lstages, nstages, (const double *)mats);
            return hipGetLastError();
        }
    }
    // complex128 only: a 16-byte direct-to-LDS load is one complex128 amplitude; for complex64 it would carry two
    // amplitudes into two adjacent slots, which the swizzle may need in the opposite order
    if constexpr (B == 12 && W == 4 && sizeof(R) == 8) {
        if (qs_tunables().block_async) {
            const size_t shm2 = 2 * shm;
            if (hipError_t e = qs_allow_lds((const void *)k_block_async<R, B>, shm2))
                return e;
            hipLaunchKernelGGL((k_block_async<R, B>), dim3((unsigned)grid), dim3(256), shm2, s, (C2 *)psi, nblocks,
                               outer, bm, stages, nstages, (const R *)mats);
            return hipGetLastError();
        }
    }
    if constexpr (sizeof(R) == 4) {
        switch (rnf) {
        case 1: return launch_k_block<R, B, W, NT, 1>(grid, shm, shm_max, psi, nblocks, outer, bm, stages, nstages,
                                                      mats, mf, rn, s);
        case 2: return launch_k_block<R, B, W, NT, 2>(grid, shm, shm_max, psi, nblocks, outer, bm, stages, nstages,
                                                      mats, mf, rn, s);
        case 3: return launch_k_block<R, B, W, NT, 3>(grid, shm, shm_max, psi, nblocks, outer, bm, stages, nstages,
                                                      mats, mf, rn, s);
        default: break;
        }
    }
    return launch_k_block<R, B, W, NT, 0>(grid, shm, shm_max, psi, nblocks, outer, bm, stages, nstages, mats, mf, rn,
                                          s);
}

template <class R>
hipError_t block_r(int b, int w, void *psi, uint64_t nblocks, const InsBits &outer, const BlockMap &bm,
                   const BlkStage *stages, int nstages, const void *mats, const BlkMfma &mf, const BlkStageL *lstages,
                   const BlkRenorm &rn, hipStream_t s)
{
    if (w == 3) {
        switch (b) {
        case 12: return block_b<R, 12, 3>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
        case 13: return block_b<R, 13, 3>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
        default: return hipErrorInvalidValue;
        }
    }
    if (w != 4)
        return hipErrorInvalidValue;
    switch (b) {
    case 8: return block_b<R, 8, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    case 9: return block_b<R, 9, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    case 10: return block_b<R, 10, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    case 11: return block_b<R, 11, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    case 12: return block_b<R, 12, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    case 13: return block_b<R, 13, 4>(psi, nblocks, outer, bm, stages, nstages, mats, mf, lstages, rn, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_batch_level(int dtype, int b, void *psi, double *probs, const BatchItem *items, int nitems,
                              uint32_t nblocks, const BatchPass *passes, const BlkStage *stages,
                              const void *mats, int wg_per_cu, hipStream_t s)
{
    return dtype == QS_C128 ? batch_r<double>(b, psi, probs, items, nitems, nblocks, passes, stages, mats,
                                              wg_per_cu, s)
                            : batch_r<float>(b, psi, probs, items, nitems, nblocks, passes, stages, mats,
                                             wg_per_cu, s);
}

hipError_t launch_block(int dtype, int b, int w, void *psi, uint64_t nblocks, const InsBits &outer,
                        const BlockMap &bm, const BlkStage *stages_dev, int nstages, const void *mats_dev,
                        const BlkMfma &mf, const BlkStageL *lstages_dev, hipStream_t s, const BlkRenorm &rn)
{
    return dtype == QS_C128
               ? block_r<double>(b, w, psi, nblocks, outer, bm, stages_dev, nstages, mats_dev, mf, lstages_dev, rn, s)
               : block_r<float>(b, w, psi, nblocks, outer, bm, stages_dev, nstages, mats_dev, mf, nullptr, rn, s);
}

uint64_t launch_block_grid(int dtype, int b, int w, uint64_t nblocks)
{
    int nt = 0;
    if (dtype == QS_C128) {
        switch (b) {
        case 8: nt = w == 3 ? 0 : BlockThreads<double, 8, 4>::value; break;
        case 9: nt = w == 3 ? 0 : BlockThreads<double, 9, 4>::value; break;
        case 10: nt = w == 3 ? 0 : BlockThreads<double, 10, 4>::value; break;
        case 11: nt = w == 3 ? 0 : BlockThreads<double, 11, 4>::value; break;
        case 12: nt = w == 3 ? BlockThreads<double, 12, 3>::value : BlockThreads<double, 12, 4>::value; break;
        case 13: nt = w == 3 ? BlockThreads<double, 13, 3>::value : BlockThreads<double, 13, 4>::value; break;
        default: break;
        }
    } else {
        switch (b) {
        case 8: nt = w == 3 ? 0 : BlockThreads<float, 8, 4>::value; break;
        case 9: nt = w == 3 ? 0 : BlockThreads<float, 9, 4>::value; break;
        case 10: nt = w == 3 ? 0 : BlockThreads<float, 10, 4>::value; break;
        case 11: nt = w == 3 ? 0 : BlockThreads<float, 11, 4>::value; break;
        case 12: nt = w == 3 ? BlockThreads<float, 12, 3>::value : BlockThreads<float, 12, 4>::value; break;
        case 13: nt = w == 3 ? BlockThreads<float, 13, 3>::value : BlockThreads<float, 13, 4>::value; break;
        default: break;
        }
    }
    return nt ? block_grid_nt(nt, nblocks) : 0;
}
