// Internal declarations shared by the host API and the HIP kernels of libqs (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "qs.h"
#include "qs_index.h"

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
    // FP64 reduction scratch: per-block partial sums followed by the result slot and the pending-norm slot
    double *red = nullptr;
    size_t red_cap = 0;
    // per-workgroup partial sums of a norm folded into a block pass (allocated on first use)
    double *blkred = nullptr;
    size_t blkred_cap = 0;
};
// device slot holding the norm a folded renormalisation computed last (qs_plan_run_renorm)
double *qs_pending_norm(qs_state *st);
// device buffer of at least n doubles for per-workgroup partial sums (grown on demand; nullptr and the error
// recorded on failure)
double *qs_block_partials(qs_state *st, size_t n);

// Copy `bytes` of host data to the device through the staging ring (async on st->stream). Returns the device
// address, or nullptr on failure (error already recorded).
void *qs_stage(qs_state *st, const void *host, size_t bytes);

inline size_t amp_bytes(int dtype) { return dtype == QS_C128 ? 16 : 8; }

// host helpers (qs_api.hip): ascending target order, matrix in ascending target order (qs_make_ins: qs_index.h)
void qs_sort_targets(const int *t, int k, TPos &tp, int *perm);
void qs_permute_matrix(const double *U, int k, const int *perm, std::vector<double> &out);

// ------------------------------------------------------------------------------------------------------------
// kernel argument blocks (passed by value)
// ------------------------------------------------------------------------------------------------------------
// InsBits, TPos and BlockMap (index maps) are defined in qs_index.h.

// ------------------------------------------------------------------------------------------------------------
// launchers (defined in the .hip files). All enqueue on `s` and return hipError_t of the launch.
// ------------------------------------------------------------------------------------------------------------
struct PermTable {
    uint8_t src[64];    // member a receives (phase) * member src[a]
    uint8_t phase[64];  // 0: 1, 1: i, 2: -1, 3: -i
    uint64_t moving;    // bit a set when member a changes (src[a] != a or phase != 1); k <= 6 so 64 bits suffice
};

// Monomial op over a qubit set Q (at most 6 qubits, at most 2 of them outside a wave's 64 lanes of 16-byte vectors)
// whose move table is given over Q (member bit u <-> the u-th lowest qubit of Q): lane-order streaming form.
struct PermLanes {
    uint8_t src[64], phase[64];
    int nq;
    int qpos[6];  // positions of Q, ascending
};
hipError_t launch_perm_lanes(int dtype, void *psi, int n, const PermLanes &pl, hipStream_t s);

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
// *result = the sum of partials[0..nb) in a fixed order (FP64)
hipError_t launch_sum_partials(const double *partials, int nb, double *result, hipStream_t s);

// LDS block passes: local qubit set L (ascending global positions), stage table in device memory
constexpr int kMaxBlockOpK = 3;
constexpr int kStageMaxOps = 8;  // ops per stage (their masks share one 32-bit word)
struct BlkStage {
    int pos[4];    // local positions held in registers during the stage (the first W, ascending; W = 3 or 4)
    int op_begin;  // first op of the stage in the host op table
    int nops;      // <= kStageMaxOps
    // op o acts on the stage positions in bits 4o..4o+3 of masks (bit j <-> pos[j]; 1..3 bits set); its 2^k x 2^k
    // matrix starts at mat_base + the sizes of ops 0..o-1 (2 * 4^k real elements each) in the matrix pool, so a
    // kernel finds every op of the stage without a dependent load
    uint32_t masks;
    uint32_t mat_base;
    // complex64 4-position stages with several ops: slot (0..kMaxMfmaStages-1) of the stage's fused 16 x 16 complex
    // matrix among the pass's MFMA matrices, applied on the matrix cores; -1: ops applied one by one in registers
    int mfma;
    // the other local positions in the order the bits of a thread's group counter fill them: the first four cover
    // the four residue classes (mod 4) of the LDS swizzle so that 16 consecutive lanes hit 16 distinct bank groups
    int order[kMaxBlockBits - 3];
    // LDS byte offset of each register member a (bit j of a <-> pos[j]; 2^W entries used): the slot of local index
    // sum_j bit_j(a) << pos[j] (blk_swz) times the amplitude size of the plan's precision, so that a kernel forms a
    // member's address with one XOR against its group's slot
    uint32_t soff[16];
};

// Lane-pair form of a 4-position stage (complex128, 12-qubit blocks, 512 threads; passes whose ops act on one or
// two positions): a 16-amplitude group is held by two lanes of a wave (thread bit 5), 8 amplitudes each; three
// stage positions are register bits of a lane's index a (0..7), the fourth is the lane bit. An op that acts on the
// lane's position is preceded by an exchange of the lane bit with a register bit the op does not use.
struct BlkStageL {
    int order[kMaxBlockBits - 4];  // group counter bit j -> local position (as in BlkStage)
    // LDS byte offsets (slot maps are linear over XOR): member (a, l) of a group at base slot sm sits at
    // sm ^ rd[a] ^ (l ? rd_lane : 0) in the initial placement, at sm ^ wr[a] ^ (l ? wr_lane : 0) after the last op
    uint32_t rd[8], wr[8];
    uint32_t rd_lane, wr_lane;
    uint32_t masks;                // op o: register bits it acts on, bits 4o..4o+2 (its matrix in register-bit order)
    uint32_t swaps;                // op o: 0, or 1 + the register bit exchanged with the lane bit before it, bits 2o..2o+1
    uint32_t mat_base;             // pool offset of op 0's matrix; the others follow in order
    int nops;
};

struct BlkStageOp {  // host-side op table (planner statistics and batch relocation)
    int mask;          // stage positions the op acts on (bit j of the mask <-> pos[j], j < W); 1..3 bits set
    uint32_t mat_off;  // offset of its 2^k x 2^k matrix (bit order of the mask's positions) in real elements
};
// w = register stage width: 4 (256 threads, any b in 8..13) or 3 (512 threads, b = 12, 13)
// Fused stage matrices of one pass (complex64): pool offsets (real elements) of n 16 x 16 complex matrices, row-major
// and interleaved, whose stage index bit j <-> stage position pos[j]; the kernel keeps them in LDS.
constexpr int kMaxMfmaStages = 4;
struct BlkMfma {
    int n = 0;
    uint32_t off[kMaxMfmaStages] = {0, 0, 0, 0};
};
// A renormalisation folded into a complex64 block pass (both optional, device pointers): scale_norm, the state is
// scaled by 1 / sqrt(*scale_norm) as each block is loaded; norm_part, one FP64 partial sum of |amplitude|^2 per
// workgroup of the launch (launch_block_grid of them) over the amplitudes it stores.
struct BlkRenorm {
    const double *scale_norm = nullptr;
    double *norm_part = nullptr;
};
// lstages_dev: the pass's stages in lane-pair form (complex128, b = 12, 4-position stages; built for plans created
// while the tunable block_lanes is set), or null
hipError_t launch_block(int dtype, int b, int w, void *psi, uint64_t nblocks, const InsBits &outer,
                        const BlockMap &bm, const BlkStage *stages_dev, int nstages, const void *mats_dev,
                        const BlkMfma &mf, const BlkStageL *lstages_dev, hipStream_t s,
                        const BlkRenorm &rn = BlkRenorm{});
// workgroups of the block kernel's launch for nblocks blocks of 2^b amplitudes, stage width w (0: no such kernel)
uint64_t launch_block_grid(int dtype, int b, int w, uint64_t nblocks);

// batched circuits: one persistent launch per pass level (see qs_block.hip)
struct BatchCirc {
    uint64_t state_off;  // amplitude offset of the circuit's state (unused when it lives in LDS)
    uint64_t prob_off;   // offset of its 2^n FP64 probabilities
    int n;
    int pass_begin, npass;
};
struct BatchPass {
    InsBits outer;  // block number -> base index (zeros at the local positions)
    BlockMap bm;
    int stage_begin, nstages;
    BlkMfma mf;     // complex64: the pass's fused stage matrices (pool offsets in the batch's pool)
};
// one work item of a level: a whole small circuit in LDS, or one pass of a circuit held in HBM
constexpr int kBatchFirst = 1;  // first pass: generate |0..0> instead of reading the state
constexpr int kBatchLast = 2;   // last pass: write FP64 probabilities instead of amplitudes
constexpr int kBatchSmall = 4;  // whole circuit of at most B qubits, one workgroup, in LDS
struct BatchItem {
    uint64_t state_off;  // amplitude offset of the circuit's HBM state
    uint64_t prob_off;   // offset of its 2^n FP64 probabilities
    uint32_t blk_begin;  // first flat block of the item within its level (small items take one block)
    int pass;            // global index of the item's pass (small: of its first pass)
    int npass;           // small: number of passes; otherwise 1
    int n;
    int flags;
};
hipError_t launch_batch_level(int dtype, int b, void *psi, double *probs, const BatchItem *items, int nitems,
                              uint32_t nblocks, const BatchPass *passes, const BlkStage *stages, const void *mats,
                              int wg_per_cu, hipStream_t s);

hipError_t launch_probe_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
hipError_t launch_probe_rmw(void *buf, size_t bytes, hipStream_t s);

// Workgroup barrier ordering LDS only: waits for this wave's LDS accesses (lgkmcnt) but not for its global loads
// and stores, so prefetched loads and outstanding stores stay in flight across it (__syncthreads() would drain
// them). Use only where the barrier protects LDS data.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// native two-element vectors for the non-temporal builtins (which do not accept HIP_vector_type)
template <class R> struct NT2;
template <> struct NT2<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NT2<float> { typedef float type __attribute__((ext_vector_type(2))); };

// tunables (set through qs_set_tunable). Process-wide and atomic: a call on one thread may change them while
// another thread plans or launches; each launch or plan reads every tunable it uses once.
struct Tunables {
    std::atomic<int> dense_gpt{1};        // groups per thread for k = 1, 2
    std::atomic<int> nontemporal{1};      // use non-temporal loads/stores in the plain gate kernels
    std::atomic<int> mfma_wg_per_cu{2};   // persistent workgroups per CU for the MFMA block kernel
    std::atomic<int> block_wg_per_cu{32}; // persistent workgroups per CU for the LDS block kernel (256-thread units)
    std::atomic<int> block_stage_width{4}; // register stage width of new block plans: 4, or 3 (512 threads, b = 12, 13)
    std::atomic<int> plan_beam{16};       // pass formation: beam width over local-set growth (0: fewest-new greedy)
    std::atomic<int> plan_beam_search{0}; // plans (not batches): also 1.5x and 4x that width, fewest passes win
    std::atomic<int> block_async{0};      // 12-qubit block passes: double-buffered LDS with direct-to-LDS loads
    std::atomic<int> block_lanes{0};      // plans created afterwards: complex128 12-qubit lane-pair stages, 512 threads
    std::atomic<int> mfma_stage_ops{3};   // complex64 plans: stages of at least this many ops run fused on MFMA
    std::atomic<int> stage_pack{1};       // block plans: 0 greedy stage packing, 1 with one stage of lookahead
};
Tunables &qs_tunables();

// Compute units of the current device (cached per device; 256 if the query fails).
int qs_cu_count();
// Allow `fn` up to `bytes` of dynamic LDS on the current device (hipFuncSetAttribute once per device, kernel and
// larger size; thread-safe).
hipError_t qs_allow_lds(const void *fn, size_t bytes);
// hipSuccess if kernel `fn` has no static LDS (its dynamic LDS then starts at address 0), checked once per device
// and kernel; hipErrorInvalidDeviceFunction otherwise.
hipError_t qs_check_no_static_lds(const void *fn);

// input width of a cost-model MLP (qs_mlp.hip)
int qs_mlp_nin(const qs_mlp *m);
