// Internal declarations shared by the host API and the HIP kernels of libqs (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qs.h"

// ------------------------------------------------------------------------------------------------------------
// error reporting (thread-local message, status code returned through the ABI)
// ------------------------------------------------------------------------------------------------------------
int qs_fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int qs_hip_fail(hipError_t e, const char *what);
void qs_clear_error();

#define QS_HIP(call)                                                                                            \
    do {                                                                                                        \
        hipError_t e_ = (call);                                                                                 \
        if (e_ != hipSuccess)                                                                                   \
            return qs_hip_fail(e_, #call);                                                                      \
    } while (0)

// ------------------------------------------------------------------------------------------------------------
// the state handle
// ------------------------------------------------------------------------------------------------------------
constexpr int kRingChunks = 16;

struct qs_state {
    int n = 0;
    int dtype = QS_C128;
    int device = 0;
    void *psi = nullptr;
    bool owns = false;
    hipStream_t stream = nullptr;
    // staging ring for matrices / tables that do not fit in kernel arguments: pinned host + device
    char *hring = nullptr;
    char *dring = nullptr;
    size_t ring_bytes = 0;
    size_t ring_head = 0;
    hipEvent_t ring_ev[kRingChunks] = {};
    bool ring_ev_live[kRingChunks] = {};
    // FP64 reduction scratch: per-block partial sums followed by the result slot
    double *red = nullptr;
    size_t red_cap = 0;
};

// Copy `bytes` of host data to the device through the staging ring (async on st->stream). Returns the device
// address, or nullptr on failure (error already recorded).
void *qs_stage(qs_state *st, const void *host, size_t bytes);

inline size_t amp_bytes(int dtype) { return dtype == QS_C128 ? 16 : 8; }

// ------------------------------------------------------------------------------------------------------------
// kernel argument blocks (passed by value)
// ------------------------------------------------------------------------------------------------------------
constexpr int kMaxIns = QS_MAX_K + QS_MAX_CONTROLS + 2;

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

// ------------------------------------------------------------------------------------------------------------
// launchers (defined in the .hip files). All enqueue on `s` and return hipError_t of the launch.
// ------------------------------------------------------------------------------------------------------------
struct PermTable {
    uint8_t src[64];    // member a receives (phase) * member src[a]
    uint8_t phase[64];  // 0: 1, 1: i, 2: -1, 3: -i
    uint64_t moving;    // bit a set when member a changes (src[a] != a or phase != 1); k <= 6 so 64 bits suffice
};

hipError_t launch_init_zero(int dtype, void *psi, uint64_t dim, hipStream_t s);
hipError_t launch_dense(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                        const double *U_host_sorted, const void *U_dev, hipStream_t s);
hipError_t launch_dense_mfma(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                             const void *U_dev, hipStream_t s);
hipError_t launch_perm(int dtype, int k, void *psi, uint64_t ngroups, const InsBits &ins, const TPos &tp,
                       const PermTable &pt, hipStream_t s);

struct DiagArgs {
    int k;
    int t[QS_MAX_DIAG_K];  // targets in matrix bit order
};
hipError_t launch_diag_full(int dtype, void *psi, uint64_t dim, const DiagArgs &da, const double *d_host,
                            const void *d_dev, const uint8_t *cls_host, const void *cls_dev, hipStream_t s);
struct DiagSparseEntry {
    uint64_t orm;  // pattern bits OR-ed into the subspace index
    double re, im;
    int cls;  // 1: negate, 2: multiply
};
constexpr int kMaxSparseDiag = 8;
hipError_t launch_diag_sparse(int dtype, void *psi, uint64_t nsub, const InsBits &ins, int m,
                              const DiagSparseEntry *ent, hipStream_t s);

hipError_t launch_fused_swap(int dtype, void *psi, int n, int lo, int hi, int s_, hipStream_t s);

hipError_t launch_probs(int dtype, const void *psi, uint64_t dim, double *out, double *partials, int nblocks,
                        double *result, hipStream_t s);
int probs_blocks(uint64_t dim);
hipError_t launch_scale(int dtype, void *psi, uint64_t dim, double f, hipStream_t s);
hipError_t launch_scale_dev(int dtype, void *psi, uint64_t dim, const double *norm_dev, hipStream_t s);

hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_probe_rmw(void *buf, size_t bytes, hipStream_t s);

// tunables (set through qs_set_option-like hooks in tests / autotuner)
struct Tunables {
    int dense_gpt = 1;       // groups per thread for k = 1, 2
    int nontemporal = 1;     // use non-temporal loads/stores in the plain gate kernels
    int mfma_wg_per_cu = 2;  // persistent workgroups per CU for the MFMA block kernel
};
Tunables &qs_tunables();
