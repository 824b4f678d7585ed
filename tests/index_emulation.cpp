// Host emulation of the kernels' index maps (csrc/qs_index.h, the same functions the kernels call).
//
// For small states it enumerates what every thread of every workgroup would load and store and checks:
//   * LDS block passes (k_block, k_batch_level): over all blocks, threads and load/store instructions every amplitude
//     index in [0, 2^n) is owned exactly once; within a block the load/store-phase LDS slots and, for random stages,
//     the stage slots (group slot XOR member offset) are each a permutation of the block's slots, and both phases
//     put local index m at slot blk_swz(m);
//   * fused-swap forms (runs, wide rows, LDS sub-tiles, pairs), run on an array of indices exactly as the kernels'
//     loops would (loads into an LDS copy, a barrier, stores from it): the result is psi'[sigma(i)] = psi[i] for every
//     i, and no index is written twice.
// Prints "ok <counts>" and returns 0, or prints the first failure and returns 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "qs_index.h"

static int fails = 0;
#define CHECK(cond, ...)                                                                                             \
    do {                                                                                                             \
        if (!(cond)) {                                                                                               \
            std::printf("FAIL %s:%d: ", __FILE__, __LINE__);                                                         \
            std::printf(__VA_ARGS__);                                                                                \
            std::printf("\n");                                                                                       \
            if (++fails > 5)                                                                                         \
                std::exit(1);                                                                                        \
        }                                                                                                            \
    } while (0)

template <int PB>
static void block_case(int n, int B, int nt, const std::vector<int> &L, std::mt19937_64 &rng, long &checked)
{
    // the block map as the planner builds it: L ascending, outer = zero bits inserted at L
    BlockMap bm{};
    bm.b = B;
    uint64_t lmask = 0;
    for (int t = 0; t < B; ++t) {
        bm.lpos[t] = L[t];
        lmask |= (uint64_t)1 << L[t];
    }
    const InsBits outer = qs_make_ins(lmask, 0);
    const int lnt = __builtin_ctz(nt);
    const int per = (1 << B) / nt;
    uint64_t h[16] = {};
    for (int j = 0; j < PB; ++j)
        h[j] = (uint64_t)1 << bm.lpos[lnt + j];
    const uint64_t nblocks = (uint64_t)1 << (n - B);
    std::vector<int> owner((size_t)1 << n, 0);
    const uint32_t amp = 16;
    for (uint64_t blk = 0; blk < nblocks; ++blk) {
        const uint64_t base = qs_ins0(blk, outer);
        std::vector<int> slot_seen((size_t)1 << B, 0);
        for (int tid = 0; tid < nt; ++tid) {
            const uint64_t own = qs_spread((uint32_t)tid, bm);
            const uint32_t sb = blk_swz((uint32_t)tid) * amp;
            for (int it = 0; it < per; ++it) {
                const uint32_t m = (uint32_t)(tid + nt * it);
                const uint64_t g = base | own | blk_hi<PB>(h, it);
                CHECK(g == (base | qs_spread(m, bm)), "block address of local %u", m);
                CHECK(g < owner.size(), "address %llu out of range", (unsigned long long)g);
                ++owner[g];
                const uint32_t sl = blk_phase_slot(sb, it, nt, amp);
                CHECK(sl == blk_swz(m) * amp, "phase slot of local %u", m);
                CHECK(sl / amp < slot_seen.size(), "phase slot out of range");
                ++slot_seen[sl / amp];
            }
        }
        for (size_t i = 0; i < slot_seen.size(); ++i)
            CHECK(slot_seen[i] == 1, "block %llu slot %zu used %d times", (unsigned long long)blk, i, slot_seen[i]);
    }
    for (size_t i = 0; i < owner.size(); ++i)
        CHECK(owner[i] == 1, "n=%d B=%d nt=%d: amplitude %zu owned %d times", n, B, nt, i, owner[i]);
    checked += (long)owner.size();
    // random stages: W positions in registers, the others filled by the group counter in planner order
    for (int rep = 0; rep < 8; ++rep) {
        for (int W = 3; W <= 4; ++W) {
            std::vector<int> perm(B);
            for (int t = 0; t < B; ++t)
                perm[t] = t;
            std::shuffle(perm.begin(), perm.end(), rng);
            std::vector<int> pos(perm.begin(), perm.begin() + W), order(perm.begin() + W, perm.end());
            std::sort(pos.begin(), pos.end());
            uint32_t soff[16];
            for (int a = 0; a < (1 << W); ++a) {
                uint32_t o = 0;
                for (int j = 0; j < W; ++j)
                    o |= ((uint32_t)(a >> j) & 1u) << pos[j];
                soff[a] = blk_swz(o) * amp;
            }
            std::vector<int> seen((size_t)1 << B, 0);
            for (uint32_t g = 0; g < (1u << (B - W)); ++g) {
                uint32_t m = 0;
                for (int j = 0; j < B - W; ++j)
                    m |= ((g >> j) & 1u) << order[j];
                const uint32_t sm = blk_swz(m) * amp;
                for (int a = 0; a < (1 << W); ++a) {
                    uint32_t o = 0;
                    for (int j = 0; j < W; ++j)
                        o |= ((uint32_t)(a >> j) & 1u) << pos[j];
                    const uint32_t sl = sm ^ soff[a];
                    CHECK(sl == blk_swz(m | o) * amp, "stage slot of local %u", m | o);
                    ++seen[sl / amp];
                }
            }
            for (size_t i = 0; i < seen.size(); ++i)
                CHECK(seen[i] == 1, "stage slot %zu used %d times (B=%d W=%d)", i, seen[i], B, W);
        }
    }
}

static void block_cases(std::mt19937_64 &rng, long &checked)
{
    for (int n = 8; n <= 14; ++n)
        for (int B = 8; B <= 13 && B <= n; ++B)
            for (int nt : {64, 128, 256, 512}) {
                if (nt > (1 << B))
                    continue;
                for (int w : {0, 3, 4}) {
                    // L: the w lowest qubits plus B - w others at random
                    std::vector<int> L;
                    for (int q = 0; q < w && q < B; ++q)
                        L.push_back(q);
                    std::vector<int> rest;
                    for (int q = w; q < n; ++q)
                        rest.push_back(q);
                    std::shuffle(rest.begin(), rest.end(), rng);
                    for (int q : rest)
                        if ((int)L.size() < B)
                            L.push_back(q);
                    std::sort(L.begin(), L.end());
                    switch (B - __builtin_ctz(nt)) {
                    case 0: block_case<0>(n, B, nt, L, rng, checked); break;
                    case 1: block_case<1>(n, B, nt, L, rng, checked); break;
                    case 2: block_case<2>(n, B, nt, L, rng, checked); break;
                    case 3: block_case<3>(n, B, nt, L, rng, checked); break;
                    case 4: block_case<4>(n, B, nt, L, rng, checked); break;
                    case 5: block_case<5>(n, B, nt, L, rng, checked); break;
                    case 6: block_case<6>(n, B, nt, L, rng, checked); break;
                    default: block_case<7>(n, B, nt, L, rng, checked); break;
                    }
                }
            }
}

// One fused-swap as the launched form would do it, on psi[i] = i; returns the number of writes per index.
static void fswap_case(int n, int lo, int hi, int s, int sz, long &checked, int &forms_seen, bool pairs = false)
{
    const uint64_t dim = (uint64_t)1 << n;
    const uint64_t smask = ((uint64_t)1 << s) - 1;
    std::vector<uint64_t> psi(dim);
    for (uint64_t i = 0; i < dim; ++i)
        psi[i] = i;
    std::vector<int> writes(dim, 0);
    FswPlan f = fsw_plan(n, lo, hi, s, sz);
    if (pairs) {  // the pair form, a fallback the dispatch never selects for valid arguments: run it directly
        f = FswPlan{};
        f.form = FSW_PAIRS;
        f.nwork = dim;
    }
    forms_seen |= 1 << f.form;
    if (f.form == FSW_RUNS) {
        for (uint64_t t = 0; t < f.nwork; ++t) {
            uint64_t i1, i2;
            fsw_runs_pair(t, lo, hi, s, f.npairs, i1, i2);
            CHECK(i1 < dim && i2 < dim, "runs index out of range");
            const uint64_t x1 = psi[i1], x2 = psi[i2];
            psi[i1] = x2;
            psi[i2] = x1;
            ++writes[i1];
            ++writes[i2];
        }
    } else if (f.form == FSW_WIDE) {
        const int R = 1 << (f.x + s + lo), RP = R + 1, nel = (1 << s) * R;
        std::vector<uint64_t> X((size_t)(1 << s) * RP);
        CHECK(X.size() * (size_t)sz == f.shm, "wide LDS size");
        for (uint64_t w = 0; w < f.nwork; ++w) {
            const uint64_t base = fsw_wide_base(w, lo, hi, s, f.x);
            for (int u = 0; u < nel; ++u) {
                uint64_t g;
                int a, c;
                fsw_wide_load(base, u, lo, hi, s, f.x, g, a, c);
                CHECK(g < dim && a * RP + c < (int)X.size(), "wide load out of range");
                X[(size_t)a * RP + c] = psi[g];
            }
            for (int u = 0; u < nel; ++u) {
                uint64_t g;
                int a, cs;
                fsw_wide_store(base, u, lo, hi, s, f.x, g, a, cs);
                CHECK(g < dim && a * RP + cs < (int)X.size(), "wide store out of range");
                psi[g] = X[(size_t)a * RP + cs];
                ++writes[g];
            }
        }
    } else if (f.form == FSW_LDS) {
        const int T = 1 << f.ts, E = 1 << lo, row = T * E, rstride = row + 1, nel = T * row;
        std::vector<uint64_t> X((size_t)T * rstride), Y((size_t)T * rstride);
        CHECK((X.size() + Y.size()) * (size_t)sz == f.shm, "sub-tile LDS size");
        for (uint64_t w = 0; w < f.nwork; ++w) {
            uint64_t I, J, common;
            fsw_lds_item(w, lo, hi, s, f.npairs, I, J, common);
            for (int u = 0; u < nel; ++u) {
                const int ra = u / row, rc = u % row;
                const uint64_t ix = fsw_lds_x(common, I, J, ra, rc, lo, hi, f.ts);
                CHECK(ix < dim, "sub-tile load out of range");
                X[(size_t)ra * rstride + rc] = psi[ix];
                if (I != J)
                    Y[(size_t)ra * rstride + rc] = psi[fsw_lds_y(common, I, J, ra, rc, lo, hi, f.ts)];
            }
            for (int u = 0; u < nel; ++u) {
                const int ra = u / row, rc = u % row;
                const int cb = rc / E, e = rc % E;
                const uint64_t ix = fsw_lds_x(common, I, J, ra, rc, lo, hi, f.ts);
                if (I != J) {
                    const uint64_t iy = fsw_lds_y(common, I, J, ra, rc, lo, hi, f.ts);
                    psi[ix] = Y[(size_t)cb * rstride + ra * E + e];
                    psi[iy] = X[(size_t)cb * rstride + ra * E + e];
                    ++writes[ix];
                    ++writes[iy];
                } else if (ra != cb) {
                    psi[ix] = X[(size_t)cb * rstride + ra * E + e];
                    ++writes[ix];
                }
            }
        }
    } else {
        for (uint64_t i = 0; i < f.nwork; ++i) {
            const uint64_t j = fsw_sigma(i, lo, hi, smask);
            if (j > i) {
                const uint64_t a = psi[i], b = psi[j];
                psi[i] = b;
                psi[j] = a;
                ++writes[i];
                ++writes[j];
            }
        }
    }
    for (uint64_t i = 0; i < dim; ++i) {
        const uint64_t j = fsw_sigma(i, lo, hi, smask);
        CHECK(psi[j] == i, "form %d n=%d lo=%d hi=%d s=%d sz=%d: psi'[sigma(%llu)] != psi[%llu]", f.form, n, lo, hi,
              s, sz, (unsigned long long)i, (unsigned long long)i);
        CHECK(writes[i] <= 1, "form %d: index %llu written %d times", f.form, (unsigned long long)i, writes[i]);
        if (j != i)
            CHECK(writes[i] == 1, "form %d: moved index %llu not written", f.form, (unsigned long long)i);
    }
    checked += (long)dim;
}

int main()
{
    std::mt19937_64 rng(20220330);
    long nb = 0, nf = 0;
    int forms = 0;
    block_cases(rng, nb);
    for (int sz : {16, 8})
        for (int n = 2; n <= 14; ++n)
            for (int s = 1; 2 * s <= n; ++s)
                for (int lo = 0; lo + 2 * s <= n; ++lo)
                    for (int hi = lo + s; hi + s <= n; ++hi) {
                        fswap_case(n, lo, hi, s, sz, nf, forms);
                        if (n <= 10)
                            fswap_case(n, lo, hi, s, sz, nf, forms, true);
                    }
    if (fails)
        return 1;
    if (forms != 15) {
        std::printf("FAIL: not every fused-swap form was reached (mask %d)\n", forms);
        return 1;
    }
    std::printf("ok block-amplitudes=%ld fswap-amplitudes=%ld\n", nb, nf);
    return 0;
}
