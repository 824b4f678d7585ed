// Index maps of libqs's kernels: which amplitude a thread loads and stores, and where it sits in LDS.
//
// Plain integer arithmetic, shared by the HIP kernels and by a host emulation in the tests (compiled there with a
// host C++ compiler), so that the maps the kernels run are the maps the emulation checks: every amplitude owned
// exactly once by the block passes, every LDS slot used once per stage, and the fused-swap forms moving amplitude
// i to sigma(i) (Sec. III-D, Listing 1: sigma exchanges bits p+j and q+j for j < s).
#pragma once

#include <cstdint>

#include "qs.h"

#if defined(__HIPCC__) || defined(__HIP__)
#define QS_HD __host__ __device__ __forceinline__
#else
#define QS_HD inline
#endif

constexpr int kMaxIns = QS_MAX_K + QS_MAX_CONTROLS + 2;
constexpr int kMaxBlockBits = 13;

// Positions (ascending) at which zero bits are inserted into a group counter, then OR-ed with `orm`.
struct InsBits {
    int np;
    uint64_t lowmask[kMaxIns];  // (1 << pos) - 1 for each position, ascending
    uint64_t orm;
};

// Target bit positions (ascending) of the group members: member a sits at base + sum_j bit_j(a) << tpos[j].
struct TPos {
    int tpos[QS_MAX_K];
};

// LDS block passes: local bit t of a block's local index <-> global bit lpos[t] (ascending).
struct BlockMap {
    int b;
    int lpos[kMaxBlockBits];
};

// Zero-bit insertion at every set bit of `mask` (at most kMaxIns of them), then `orm` OR-ed in (host side).
inline InsBits qs_make_ins(uint64_t mask, uint64_t orm)
{
    InsBits ins{};
    ins.np = 0;
    for (int p = 0; p < 64 && ins.np < kMaxIns; ++p)
        if ((mask >> p) & 1)
            ins.lowmask[ins.np++] = ((uint64_t)1 << p) - 1;
    ins.orm = orm;
    return ins;
}

// Counter g with a zero bit inserted at every position of s (ascending), then OR-ed with s.orm: the base index of
// the g-th group (Eq. 4: a group is the set of amplitudes whose indices differ only in the target bits).
QS_HD uint64_t qs_ins0(uint64_t g, const InsBits &s)
{
    for (int j = 0; j < s.np; ++j) {
        const uint64_t lo = g & s.lowmask[j];
        g = ((g ^ lo) << 1) | lo;
    }
    return g | s.orm;
}

// Offset of member a of a group: bit j of a at target position tpos[j].
template <int K>
QS_HD uint64_t qs_member_off(int a, const TPos &tp)
{
    uint64_t o = 0;
    for (int j = 0; j < K; ++j)
        o |= (uint64_t)((a >> j) & 1) << tp.tpos[j];
    return o;
}

// Local index m of a block -> global offset: bit t of m goes to global bit lpos[t].
QS_HD uint64_t qs_spread(uint32_t m, const BlockMap &bm)
{
    uint64_t o = 0;
    for (int t = 0; t < bm.b; ++t)
        o |= (uint64_t)((m >> t) & 1) << bm.lpos[t];
    return o;
}

// LDS slot of local index m in a block: its low 4 bits XOR-ed with bits 4-7, 8-11 and 12. Local position p then
// moves a 16-byte slot's bank group by the unit vector of class p mod 4, and the map is linear over XOR on indices
// with disjoint bits: slot(m | o) = slot(m) ^ slot(o).
QS_HD uint32_t blk_swz(uint32_t m) { return m ^ (((m >> 4) ^ (m >> 8) ^ (m >> 12)) & 15u); }

// Block kernel load / store phase, workgroup of NT = 2^lnt threads: thread tid handles local indices tid + NT it.
// Their global offset is the block base | spread(tid) | hi, hi the OR of h[j] = 1 << lpos[lnt + j] over the set bits
// j of it; their LDS byte slot is that of blk_swz, formed from slot_bytes(tid) with one XOR and one add (blk_swz
// folds only into the low 4 bits).
template <int PB>
QS_HD uint64_t blk_hi(const uint64_t *h, int it)
{
    uint64_t o = 0;
    for (int j = 0; j < PB; ++j)
        if ((it >> j) & 1)
            o |= h[j];
    return o;
}
QS_HD uint32_t blk_phase_slot(uint32_t sb, int it, int nt, uint32_t amp)
{
    const uint32_t m = (uint32_t)(nt * it);
    return (sb ^ ((blk_swz(m) & 15u) * amp)) + m * amp;
}

// Fused-swap launch geometry (lo < hi, s >= 1, lo + s <= hi, hi + s <= n; sz = bytes per amplitude): which form runs
// and its work decomposition.
enum { FSW_RUNS = 0, FSW_WIDE = 1, FSW_LDS = 2, FSW_PAIRS = 3 };
struct FswPlan {
    int form;
    uint64_t nwork;    // runs: exchanged elements; wide / lds: work items (one workgroup each); pairs: indices
    uint64_t npairs;   // runs: run pairs per outer index; lds: sub-tile pairs per tile
    int x;             // wide: mid bits carried along
    int ts;            // lds: log2 of the sub-tile side
    uint64_t shm;      // LDS bytes of a workgroup
};
inline FswPlan fsw_plan(int n, int lo, int hi, int s, int sz)
{
    FswPlan f{};
    // runs of at least 256 bytes, or of one 128-byte line with s <= 4: exchanged directly (measured at 28 qubits:
    // one-line runs 2.8 -> 5.3 TB/s for s = 1 against the wide-row form, but 5.4 -> 4.9 for s = 6)
    const uint64_t run = ((uint64_t)1 << lo) * (uint64_t)sz;
    if (run >= 256 || (run >= 128 && s <= 4)) {
        const uint64_t S = (uint64_t)1 << s;
        f.form = FSW_RUNS;
        f.npairs = S * (S - 1) / 2;
        f.nwork = ((uint64_t)1 << (n - 2 * s - lo)) * f.npairs * ((uint64_t)1 << lo);
        return f;
    }
    if (((uint64_t)1 << (2 * s + lo)) * (uint64_t)sz <= 32768) {
        // wide rows whenever the 2^s x 2^s tile of runs fits 32 KiB: carry x low mid bits so that a tile holds about
        // 32 KiB (or all mid bits if fewer)
        const int nmid = hi - lo - s;
        int x = (sz == 16 ? 11 : 12) - 2 * s - lo;
        if (x > nmid)
            x = nmid;
        if (x < 0)
            x = 0;
        f.form = FSW_WIDE;
        f.x = x;
        f.nwork = (uint64_t)1 << (n - 2 * s - lo - x);
        f.shm = ((uint64_t)1 << s) * (((uint64_t)1 << (x + s + lo)) + 1) * (uint64_t)sz;
        return f;
    }
    // LDS sub-tiles: the largest T = 2^ts <= 2^s with T * T * 2^lo amplitudes <= 16 KiB per tile
    int ts = s;
    while (ts > 0 && ((uint64_t)1 << (2 * ts + lo)) * (uint64_t)sz > 16384)
        --ts;
    if (((uint64_t)1 << (ts + lo)) * (uint64_t)sz >= 128 && ts >= 2) {
        const uint64_t ntile = (uint64_t)1 << (s - ts);
        f.form = FSW_LDS;
        f.ts = ts;
        f.npairs = ntile * (ntile + 1) / 2;
        f.nwork = ((uint64_t)1 << (n - 2 * s - lo)) * f.npairs;
        f.shm = 2 * ((uint64_t)1 << ts) * (((uint64_t)1 << (ts + lo)) + 1) * (uint64_t)sz;
        return f;
    }
    f.form = FSW_PAIRS;
    f.nwork = (uint64_t)1 << n;
    return f;
}

// Fused-swap, sigma(i): bits lo + j and hi + j exchanged for j < s (smask = 2^s - 1).
QS_HD uint64_t fsw_sigma(uint64_t i, int lo, int hi, uint64_t smask)
{
    const uint64_t d = ((i >> lo) ^ (i >> hi)) & smask;
    return i ^ (d << lo) ^ (d << hi);
}

// Run form: work item t -> the two indices i1 (A = a, B = b) and i2 (A = b, B = a) it exchanges, a > b, where
// B = bits [lo, lo + s) and A = bits [hi, hi + s); pr = a (a - 1) / 2 + b enumerates the pairs.
QS_HD void fsw_runs_pair(uint64_t t, int lo, int hi, int s, uint64_t npairs, uint64_t &i1, uint64_t &i2)
{
    const uint64_t E = (uint64_t)1 << lo;
    const int nmid = hi - lo - s;
    const uint64_t e = t & (E - 1);
    const uint64_t r = t >> lo;
    const uint64_t pr = r % npairs;
    const uint64_t o = r / npairs;
    uint64_t a = (uint64_t)((1.0 + __builtin_sqrt(1.0 + 8.0 * (double)pr)) * 0.5);
    while (a * (a - 1) / 2 > pr)
        --a;
    while ((a + 1) * a / 2 <= pr)
        ++a;
    const uint64_t b = pr - a * (a - 1) / 2;
    const uint64_t mid = o & (((uint64_t)1 << nmid) - 1);
    const uint64_t top = o >> nmid;
    const uint64_t common = e | (mid << (lo + s)) | (top << (hi + s));
    i1 = common | (b << lo) | (a << hi);
    i2 = common | (a << lo) | (b << hi);
}

// Wide-row form (runs too short for the direct form, tile <= 32 KiB), x low mid bits carried: work item w covers the 2^s
// rows A = a, each a contiguous segment of R = 2^(x + s + lo) amplitudes (mid_low, B, e). Load: element u of the item
// goes from global index *g to LDS row a, column c. Store: element u goes to global index *g from LDS row *ra,
// column *rc (the element at B = b of row a moves to B = a of row b).
QS_HD uint64_t fsw_wide_base(uint64_t w, int lo, int hi, int s, int x)
{
    const int nmid_hi = hi - lo - s - x;
    const uint64_t midh = w & (((uint64_t)1 << nmid_hi) - 1);
    const uint64_t top = w >> nmid_hi;
    return (top << (hi + s)) | (midh << (lo + s + x));
}
QS_HD void fsw_wide_load(uint64_t base, int u, int lo, int hi, int s, int x, uint64_t &g, int &a, int &c)
{
    const int R = 1 << (x + s + lo);
    a = u / R;
    c = u - a * R;
    g = base | ((uint64_t)a << hi) | (uint64_t)c;
    (void)lo;
    (void)s;
}
QS_HD void fsw_wide_store(uint64_t base, int u, int lo, int hi, int s, int x, uint64_t &g, int &ra, int &rc)
{
    const int R = 1 << (x + s + lo);
    const int bmask = (1 << s) - 1;
    const int b = u / R, c = u - b * R;
    ra = (c >> lo) & bmask;                // B field of the destination = the source row
    rc = (c & ~(bmask << lo)) | (b << lo);  // source column: B field = b
    g = base | ((uint64_t)b << hi) | (uint64_t)c;
}

// LDS sub-tile form: work item w -> sub-tile pair (I, J), J <= I, of one 2^s x 2^s tile of 2^lo-amplitude runs
// (T = 2^ts runs per sub-tile side), and the index bits common to the item.
QS_HD void fsw_lds_item(uint64_t w, int lo, int hi, int s, uint64_t npairs_t, uint64_t &I, uint64_t &J,
                        uint64_t &common)
{
    const uint64_t pr = w % npairs_t;
    const uint64_t o = w / npairs_t;
    I = (uint64_t)((1.0 + __builtin_sqrt(1.0 + 8.0 * (double)pr)) * 0.5) - 1;  // pr = I (I + 1) / 2 + J, J <= I
    while (I * (I + 1) / 2 > pr)
        --I;
    while ((I + 1) * (I + 2) / 2 <= pr)
        ++I;
    J = pr - I * (I + 1) / 2;
    const int nmid = hi - lo - s;
    const uint64_t mid = o & (((uint64_t)1 << nmid) - 1);
    const uint64_t top = o >> nmid;
    common = (mid << (lo + s)) | (top << (hi + s));
}
// Element (ra, rc) of sub-tile X (rows A in the I range, columns B in the J range; rc = cb 2^lo + e) and of its
// partner Y (rows A in the J range, columns B in the I range): global indices.
QS_HD uint64_t fsw_lds_x(uint64_t common, uint64_t I, uint64_t J, int ra, int rc, int lo, int hi, int ts)
{
    const int T = 1 << ts;
    const uint64_t cb = (uint64_t)(rc >> lo), e = (uint64_t)(rc & ((1 << lo) - 1));
    return common | e | ((J * T + cb) << lo) | ((I * T + (uint64_t)ra) << hi);
}
QS_HD uint64_t fsw_lds_y(uint64_t common, uint64_t I, uint64_t J, int ra, int rc, int lo, int hi, int ts)
{
    return fsw_lds_x(common, J, I, ra, rc, lo, hi, ts);
}
