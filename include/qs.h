/*
 * qs.h -- C ABI of libqs, an MI355X (gfx950) state-vector gate engine.
 *
 * The engine applies quantum gates to a full vector of 2^n complex amplitudes held in HBM, following the
 * state-vector method of mpiQulacs (Imamura et al., "mpiQulacs: A Distributed Quantum Computer Simulator
 * for A64FX-based Cluster Systems"):
 *   - Sec. II-A, Eq. 2: the state is 2^n complex amplitudes a_i, sum_i |a_i|^2 = 1; in double precision it
 *     takes 2^(n+4) bytes;
 *   - Sec. II-A, Eq. 4: a 1-qubit gate U on qubit q multiplies every amplitude pair whose indices differ
 *     only in bit q by the 2x2 matrix U; k-qubit gates generalise this to the 2^k amplitudes whose
 *     indices differ only in the target bits;
 *   - Sec. III-D, Listing 1: fused_swap(p, q, s) performs swap(p+i, q+i) for i < s, the two ranges
 *     [p, p+s) and [q, q+s) not overlapping.
 * On one GPU the fused-swap is an in-place permutation of HBM (the paper moves the same amplitudes
 * between processes); it exchanges high-order and low-order qubits.
 *
 * Conventions shared by every call
 *   Layout.    Amplitudes are interleaved (re, im): complex128 = 2 doubles (16 B), complex64 = 2 floats
 *              (8 B), i.e. the layout of torch.complex128 / torch.complex64. Qubit q is bit q of the index
 *              (qubit 0 = least significant bit).
 *   Matrices.  A k-qubit matrix U is a host array of 2^k x 2^k complex numbers given as interleaved FP64
 *              (re, im), row-major, with targets[j] <-> bit j of the row/column index, and psi' = U psi.
 *              FP64 is used for complex64 states too; the library rounds to FP32.
 *   Status.    Every call returns QS_OK (0) or a negative QS_E* code; qs_last_error() gives a thread-local
 *              message for the last failure on the calling thread. No C++ exception or abort crosses the ABI.
 *   Validation happens before anything is enqueued: a rejected call leaves the state unchanged.
 *   Ordering.  Calls enqueue work on the state's HIP stream and return without synchronising (except where
 *              stated). Device faults surface at qs_sync, qs_copy_out or a norm read-back.
 *   Ownership. The caller owns every host array passed in; the library copies or packs it before returning,
 *              so it may be freed on return. Device buffers passed in (dev_buf, out_dev) are the caller's and
 *              must stay alive until the work that uses them has completed on the stream.
 *   Threads.   A handle may be used by one thread at a time.
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QS_API __attribute__((visibility("default")))

enum {
    QS_OK = 0,
    QS_EINVAL = -1,       /* argument out of range, null pointer, overlapping qubits */
    QS_ENOMEM = -2,       /* device or pinned-host allocation failed */
    QS_EDEVICE = -3,      /* a HIP runtime call failed (no device, launch failure, fault) */
    QS_EUNSUPPORTED = -4  /* a valid request the library does not implement */
};

enum { QS_C128 = 0, QS_C64 = 1 };

#define QS_MAX_QUBITS 40  /* upper bound accepted by qs_alloc; HBM capacity is the practical bound */
#define QS_MAX_K 6        /* largest dense / controlled target count */
#define QS_MAX_DIAG_K 12  /* largest diagonal target count */
#define QS_MAX_CONTROLS 16

typedef struct qs_state qs_state;

/*
 * qs_alloc -- create a state of n qubits and initialise it to |0...0> (Sec. II-A, Eq. 2).
 *   out        receives the handle (must not be NULL).
 *   n          1 <= n <= QS_MAX_QUBITS.
 *   dtype      QS_C128 or QS_C64.
 *   dev_buf    NULL: the library allocates 2^n amplitudes on the current device and frees them in qs_free.
 *              Otherwise a device buffer of at least 2^n * sizeof(amplitude) bytes, 256-byte aligned, that
 *              the caller owns and keeps alive for the handle's lifetime.
 *   hip_stream the hipStream_t to enqueue on (NULL = the null stream).
 * Errors: QS_EINVAL (out NULL, n or dtype out of range, misaligned dev_buf), QS_ENOMEM, QS_EDEVICE.
 */
QS_API int qs_alloc(qs_state **out, int n, int dtype, void *dev_buf, void *hip_stream);

/* qs_free -- synchronise the stream, release library-owned memory and the handle. QS_EINVAL if st is NULL. */
QS_API int qs_free(qs_state *st);

/*
 * qs_apply_gate -- dense k-qubit gate, 1 <= k <= QS_MAX_K (Sec. II-A, Eq. 4 and its k-qubit form).
 *   targets  k distinct qubits in [0, n); targets[j] <-> bit j of U's index.
 *   U        2^k x 2^k complex FP64, row-major, interleaved.
 * Matrices whose entries are all in {0, 1, -1, i, -i} with one nonzero per row and column (X, CNOT blocks,
 * SWAP, Y up to the factor, ...) are executed as pure amplitude moves with sign/component exchange: no
 * arithmetic, bit-exact. Exactly diagonal matrices are executed as qs_apply_diag.
 * Errors: QS_EINVAL (null pointers, k out of range, target out of range or repeated).
 */
QS_API int qs_apply_gate(qs_state *st, const int *targets, int k, const double *U);

/*
 * qs_apply_diag -- diagonal gate: a_i <- d[a(i)] a_i, a(i) = the target bits of i in targets order
 * (Eq. 4 with a diagonal U; RZ, CZ, controlled phases). 1 <= k <= QS_MAX_DIAG_K.
 *   d  2^k complex FP64, interleaved. Entries exactly 1 leave their amplitudes' values bit-identical; entries
 *      exactly -1 are a sign flip (exact). When every entry is in {1, -1, i, -i} and k <= 6, the diagonal is a pure
 *      move: entries i and -i exchange the components with a sign, exactly (signed zeros kept).
 *      Access: such a diagonal that changes an amplitude in every 128-byte line (bit < 3 of the index lies inside
 *      a complex128 line, bit < 4 inside a complex64 one), with at most 2 targets at bit 6 (complex64: 7) or
 *      above and n at least 6 (7) plus that number, reads and rewrites every amplitude, the entry-1 ones
 *      unchanged. Otherwise amplitudes whose entry is exactly 1 are not accessed, except on complex64 states with
 *      k <= 2 (unless the diagonal is a pure move with an entry i or -i): there memory is accessed in 16-byte
 *      pairs of adjacent amplitudes, a pair with one entry other than 1 is read and both amplitudes are rewritten
 *      (the one with entry 1 unchanged), and a pair whose two entries are 1 is not accessed.
 * Errors: as qs_apply_gate.
 */
QS_API int qs_apply_diag(qs_state *st, const int *targets, int k, const double *d);

/*
 * qs_apply_controlled -- U on the targets, restricted to the amplitudes whose control bits are all 1
 * (CNOT, Toffoli, controlled-U). 1 <= c <= QS_MAX_CONTROLS, 1 <= k <= QS_MAX_K, c + k <= n. Permutation
 * matrices (see qs_apply_gate) are pure moves, bit-exact. When c + k <= 6, a control or target lies inside a
 * 128-byte line (bit < 3 for complex128, < 4 for complex64), every 128-byte line holds an amplitude the move
 * changes, at most 2 of the c + k qubits are at bit 6 (complex64: 7) or above and n is at least 6 (7) plus that
 * number, every amplitude is read and the unchanged ones are written back bit-identical (whole lines stream);
 * otherwise unchanged amplitudes are not accessed. The same holds for permutation matrices given to
 * qs_apply_gate.
 * Errors: QS_EINVAL (null pointers, counts out of range, qubits out of range, repeated, or a control that
 * is also a target).
 */
QS_API int qs_apply_controlled(qs_state *st, const int *controls, int c, const int *targets, int k, const double *U);

/*
 * qs_fused_swap -- fused_swap(p, q, s) of Sec. III-D, Listing 1: swap(p+i, q+i) for 0 <= i < s, in place:
 * psi'[sigma(i)] = psi[i] where sigma exchanges bit p+j with bit q+j. Pure moves, bit-exact; the 2^(n-s)
 * fixed points (sigma(i) = i) keep their values bit-identical. Whether a fixed point is accessed depends on the
 * form chosen for the run length 2^min(p,q) and the tile size: runs of at least 256 bytes, or of 128 bytes with
 * s <= 4, are exchanged directly, and short runs in tiles too small for LDS staging one index pair at a time,
 * neither accessing fixed points; the LDS tile forms read the fixed points that share a tile with moved
 * amplitudes, and the wide-row form (2^s x 2^s tiles of runs up to 32 KiB) also writes them back unchanged.
 * s = 0 is a no-op; p and q may come in either order.
 * Errors: QS_EINVAL if s < 0, p < 0, q < 0, p+s > n, q+s > n, or the ranges overlap (|p - q| < s).
 */
QS_API int qs_fused_swap(qs_state *st, int p, int q, int s);

/*
 * qs_probs -- out_dev[i] = |a_i|^2 in FP64 (complex64 components are widened first) (Sec. II-A).
 *   out_dev   device buffer of 2^n doubles (caller-owned), or NULL to compute only the norm.
 *   norm_out  host pointer, or NULL. When non-NULL the call synchronises the stream and stores
 *             sum_i |a_i|^2, reduced in FP64 in a fixed order (run-to-run bit-identical).
 * Errors: QS_EINVAL (st NULL), QS_EDEVICE.
 */
QS_API int qs_probs(qs_state *st, double *out_dev, double *norm_out);

/* ---- allocation-free entry point ----
 * qs_probs_noalloc -- qs_probs on a raw amplitude buffer, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation): it calls no hipMalloc, hipFree or
 * allocating library routine and needs no state handle. The reduction's FP64 partial sums go to a library-held
 * device array of 4096 doubles (32 KiB per GPU, resolved once per device on the first call made with that device
 * current, kept until the process ends); every call on a GPU shares it, so calls whose work overlaps on one GPU
 * (different streams) race, and calls on one stream are ordered. Results are bit-identical to qs_probs on the same
 * amplitudes (same kernels, same fixed reduction order).
 *   psi       device buffer of 2^n amplitudes in dtype's layout, 16-byte aligned (caller-owned).
 *   n, dtype  1 <= n <= QS_MAX_QUBITS; QS_C128 or QS_C64.
 *   out_dev   device buffer of 2^n doubles receiving |a_i|^2, or NULL.
 *   norm_dev  device double receiving sum_i |a_i|^2 (fixed-order FP64 reduction), or NULL; at least one of out_dev
 *             and norm_dev is non-NULL. Both 8-byte aligned.
 *   hip_stream the hipStream_t to enqueue on (NULL = the null stream); the call does not synchronise.
 * Errors: QS_EINVAL (NULL or misaligned buffers, n or dtype out of range, both outputs NULL), QS_EUNSUPPORTED (more
 * partial sums than the scratch holds; cannot happen for valid n), QS_EDEVICE. A rejected call enqueues nothing. */
QS_API int qs_probs_noalloc(const void *psi, int n, int dtype, double *out_dev, double *norm_dev, void *hip_stream);

/* ---- state management and support calls (used by tests, renormalisation and harnesses) ---- */

/* Reset to |0...0> (a fill kernel, no memset). */
QS_API int qs_init_zero(qs_state *st);
/* Copy 2^n amplitudes from / to host memory in the state's dtype layout; synchronous. */
QS_API int qs_copy_in(qs_state *st, const void *host);
QS_API int qs_copy_out(qs_state *st, void *host);
/* Wait for all work enqueued on the state's stream. */
QS_API int qs_sync(qs_state *st);
/* a_i <- f a_i with f in FP64 (complex64: product rounded to FP32). */
QS_API int qs_scale(qs_state *st, double f);
/* Synchronously compute the FP64 norm sum_i |a_i|^2 (same fixed-order reduction as qs_probs). */
QS_API int qs_norm(qs_state *st, double *norm_out);
/* Renormalise: a_i <- a_i / sqrt(sum |a|^2); the factor is formed in FP64. Optionally returns the norm
 * measured before scaling. Synchronises. */
QS_API int qs_renormalize(qs_state *st, double *norm_before);
/* Query handle properties; any output pointer may be NULL. */
QS_API int qs_get_info(qs_state *st, int *n, int *dtype, void **dev_ptr, void **hip_stream);
/* Message of the last failing call on this thread ("" if none). */
QS_API const char *qs_last_error(void);

/* ---- measurement, sampling and reset ----
 * A circuit is a sequence of gates, measurements and resets (Sec. II-A); the probability of observing basis state
 * i is |a_i|^2 relative to the total mass (Eq. 1 generalised to n qubits). Random numbers are the caller's: each
 * call takes uniforms in [0, 1), so runs are reproducible and can be checked one by one. */
/* Measure `qubit`: P0, P1 = FP64 masses with the qubit's bit 0 / 1 (fixed-order reduction), outcome = 1 iff
 * u (P0 + P1) < P1, then the state collapses: amplitudes of the observed outcome are scaled by 1/sqrt(P_outcome)
 * (factor in FP64), the others set to 0. prob_one (nullable) receives P1 / (P0 + P1). Synchronises (the outcome
 * is decided on the host). QS_EINVAL for a qubit out of range, u outside [0, 1) or a state with no finite
 * nonzero mass (then the state is unchanged). */
QS_API int qs_measure(qs_state *st, int qubit, double u, int *outcome, double *prob_one);
/* Measure `qubit` as qs_measure does, then flip it to |0> if the outcome was 1 (an exact permutation). */
QS_API int qs_reset(qs_state *st, int qubit, double u, int *outcome);
/* Draw nshots basis indices (no collapse): shot k returns the smallest i whose cumulative FP64 mass exceeds
 * u[k] x total mass (chunked deterministic prefix sums; every index returned lies in [0, 2^n)). u and out are
 * host arrays of nshots doubles / int64 (0 <= nshots <= 2^30); uses temporary device memory of about
 * 2^(n-11) doubles + 16 bytes per shot. Synchronises. QS_EINVAL for u outside [0, 1) or a state with no finite
 * nonzero mass. */
QS_API int qs_sample(qs_state *st, int64_t nshots, const double *u, int64_t *out);

/* ---- circuits and execution plans ----
 * A circuit is an ordered list of operations (Sec. II-A: a circuit applies its gates in sequence); the add
 * calls take the same arguments, with the same validation, as the qs_apply_* calls, and copy them. */
typedef struct qs_circuit qs_circuit;
typedef struct qs_plan qs_plan;

/* Create an empty circuit on n qubits (1 <= n <= QS_MAX_QUBITS). Host only; no device work. */
QS_API int qs_circuit_create(qs_circuit **out, int n);
QS_API int qs_circuit_free(qs_circuit *c);
QS_API int qs_circuit_add_gate(qs_circuit *c, const int *targets, int k, const double *U);
QS_API int qs_circuit_add_diag(qs_circuit *c, const int *targets, int k, const double *d);
QS_API int qs_circuit_add_controlled(qs_circuit *c, const int *controls, int nc, const int *targets, int k,
                                     const double *U);
QS_API int qs_circuit_add_fused_swap(qs_circuit *c, int p, int q, int s);
/* Number of operations recorded. */
QS_API int qs_circuit_size(const qs_circuit *c, int *nops);
/* Plain execution: exactly the qs_apply_* / qs_fused_swap calls of the circuit, in order (one pass each).
 * QS_EINVAL if the circuit's qubit count differs from the state's. */
QS_API int qs_circuit_run(qs_state *st, const qs_circuit *c);

enum {
    QS_PLAN_BLOCK = 0, /* LDS block passes over a qubit set of block_bits qubits (8..13) */
    QS_PLAN_FUSE = 1,  /* dense fused blocks of at most block_bits qubits (1..6) */
    QS_PLAN_REMAP = 2  /* Sec. III-B / III-D on one GPU: block passes over the lowest block_bits physical qubits only,
                        * a logical -> physical qubit map, fused-swaps inserted to bring each pass's qubits into that
                        * range, circuit fused-swaps absorbed into the map (relabel passes, no data moved), and the
                        * identity map restored by fused-swaps at the end */
};
typedef struct {
    int mode;       /* QS_PLAN_BLOCK, QS_PLAN_FUSE or QS_PLAN_REMAP */
    int block_bits; /* BLOCK: qubits local to one workgroup; FUSE: largest fused gate */
    int low_bits;   /* BLOCK: the lowest low_bits qubits are always local (whole cache lines per segment) */
    int dtype;      /* QS_C128 / QS_C64: precision the plan's matrices are uploaded in */
} qs_plan_opts;

/* Group the circuit's operations into passes (host only; the circuit may be freed afterwards). A gate joins
 * a pass only when every earlier gate on its qubits is placed, so running the plan gives the circuit's state up
 * to rounding (fused matrices are products formed in FP64 on the host). BLOCK mode on fewer than 8 qubits
 * falls back to FUSE mode with 4-qubit blocks. Errors: QS_EINVAL for out-of-range options. */
QS_API int qs_plan_create(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts);
/* Enqueue every pass (or passes [begin, end)) on the state's stream. The first run uploads the plan's matrices
 * to the current device (synchronous copy; if it fails, nothing stays allocated and a later run retries).
 * QS_EINVAL if n or dtype differ from the plan's, or if the plan was uploaded to another device. */
QS_API int qs_plan_run(qs_state *st, qs_plan *p);
QS_API int qs_plan_run_range(qs_state *st, qs_plan *p, int begin, int end);
/* Periodic renormalisation (the complex64 cadence: a state renormalised after given layers), here between plans,
 * each stretch of layers its own plan (inside one plan: qs_plan_run_range_renorm). Runs every pass of p like
 * qs_plan_run, and:
 *   QS_RUN_SCALE_FIRST  first scales the state by 1 / sqrt(N), N the state's pending norm (left by an earlier
 *                       QS_RUN_NORM_LAST run), the factor formed and applied in FP64 (complex64: rounded to FP32);
 *   QS_RUN_NORM_LAST    then sets the pending norm to sum_i |a_i|^2 (FP64, fixed-order reduction) of the state
 *                       the plan leaves.
 * Where the plan's first (last) data-moving pass is a complex64 block pass, the scaling (norm) is folded into it:
 * applied as each block is loaded (accumulated as each block is stored, one partial per workgroup); otherwise a
 * separate sweep does it. Results equal a qs_renormalize between the plans up to rounding (the norm sums in
 * another order). Asynchronous; the pending norm lives in the state's device memory. The first folded norm
 * allocates a partial-sum buffer (grown when a larger launch needs more). QS_EINVAL for unknown flags or as
 * qs_plan_run; QS_ENOMEM if that buffer cannot be allocated. */
enum { QS_RUN_SCALE_FIRST = 1, QS_RUN_NORM_LAST = 2 };
QS_API int qs_plan_run_renorm(qs_state *st, qs_plan *p, int flags);
/* The same over passes [begin, end) of one plan: the scaling folds into the range's first data-moving pass, the
 * norm into its last. A renormalisation is a scalar factor and commutes with every gate, so one plan over the
 * whole circuit can renormalise at pass boundaries (placing them is the caller's choice: the first boundary by
 * which every gate of the layers to be renormalised has run). QS_EINVAL for unknown flags, a range outside
 * [0, passes] or begin > end, or as qs_plan_run; QS_ENOMEM as qs_plan_run_renorm. An empty range with both
 * flags scales by the pending norm and then takes the norm of the scaled state, each in a sweep of its own. */
QS_API int qs_plan_run_range_renorm(qs_state *st, qs_plan *p, int begin, int end, int flags);
/* Scale the state by 1 / sqrt(N) for its pending norm N (the last renormalisation of a sequence of
 * qs_plan_run_renorm or qs_plan_run_range_renorm calls); optionally returns N. Synchronises when norm is
 * non-null. */
QS_API int qs_renormalize_pending(qs_state *st, double *norm);
/* Pass counts: all passes, LDS block passes, dense passes, others (fused-swaps, large controlled gates, relabels),
 * and the number of fused operations executed inside the block / dense passes. Any output may be NULL. */
QS_API int qs_plan_info(const qs_plan *p, int *npasses, int *nblock, int *ndense, int *nother, int *nfused_ops);
/* Pass i: type (0 block, 1 dense, 2 fused-swap, 3 other, 4 relabel: a circuit fused-swap absorbed into a remapped
 * plan's qubit map, which runs no kernel), qubits it spans and their mask, fused operations in it and circuit gates
 * it carries. Fused-swaps a remapped plan inserts carry no circuit gates. */
QS_API int qs_plan_pass_info(const qs_plan *p, int i, int *type, int *nqubits, int64_t *qmask, int *nops,
                             int *ngates);
/* The circuit gates pass i carries, in the order the pass applies them (inside a block pass: stage by stage, each
 * fused op's gates in circuit order). A gate is named by its position among the operations the circuit recorded
 * (every qs_circuit_add_* call that returned QS_OK, except fused-swaps with s = 0, which record nothing). Writes
 * min(cap, count) indices to gates (may be NULL when cap = 0) and the full count to *count (nullable). Over all
 * passes every recorded gate appears exactly once; two gates that share a qubit keep their circuit order (Sec.
 * II-A: a circuit is an ordered product of gates; gates on disjoint qubits commute). Host only.
 * QS_EINVAL for a NULL plan, a negative cap, gates NULL with cap > 0, or i out of range. */
QS_API int qs_plan_pass_gates(const qs_plan *p, int i, int *gates, int cap, int *count);
QS_API int qs_plan_free(qs_plan *p);

/* ---- learned cost model (an MLP trained on the simulator's own pass timings) ----
 * Features of plan pass i (QS_PLAN_NFEAT floats): [0-3] pass type one-hot (block, dense, fused-swap, other),
 * [4] n/40, [5] dtype (0 complex128, 1 complex64), [6] qubits spanned/16, [7] fused ops/32, [8] register
 * stages/16, [9] contiguous low qubits in the span/16, [10] lowest and [11] highest qubit/40, [12] low-4-qubit
 * count/4, [13] log2(state bytes)/40, [14] flops per amplitude/256, [15] circuit gates carried/64, [16-19] block
 * size one-hot (10..13 qubits), [20-23] dense target-count one-hot (3..6), [24] fused-swap s/16, [25] span holds
 * the 4 lowest qubits, [26-47] span mask bits 0..21. */
#define QS_PLAN_NFEAT 48
QS_API int qs_plan_features(const qs_plan *p, int i, float *features);

/* ---- learned planning: the cost model chooses every pass ----
 * Pass formation as in qs_plan_create (a gate joins a pass only when every earlier gate on its qubits is placed), but
 * at every step the planner forms candidate passes for each of the `nshapes` block shapes (block_bits, low_bits), up
 * to `per_shape` per shape (the local sets its beam search ends with, most gates first), describes each candidate by
 * its QS_PLAN_NFEAT features (qs_plan_features), lets `model` predict log(pass milliseconds) from the features
 * standardised as (f - mean) / std, and keeps the candidate with the lowest predicted time per circuit gate carried
 * among those that carry at least (the most gates any candidate carries) - gate_slack gates. With lookahead != 0 a
 * candidate is scored together with the pass that would follow it (formed with the first shape): their predicted
 * time over the gates both carry.
 * Passes of a plan may therefore differ in block size and low bits. Gates that no block pass can carry run as their
 * own passes, as in qs_plan_create. opts->mode must be QS_PLAN_BLOCK; opts->block_bits / low_bits are ignored.
 * The model runs on its own stream (one synchronising prediction per pass). Host arrays are read during the call.
 *   shape_bits[i] in [10, 13] (and <= n), shape_low[i] in [0, shape_bits[i]], 1 <= nshapes <= 16,
 *   1 <= per_shape <= 8, gate_slack >= 0; model built with nin = QS_PLAN_NFEAT; std entries > 0.
 * Errors: QS_EINVAL for NULL pointers, out-of-range fields (a shape wider than the circuit included) or a model of
 * another input width; the errors of qs_mlp_predict. */
typedef struct qs_mlp qs_mlp;
typedef struct {
    qs_mlp *model;
    const float *mean, *std; /* QS_PLAN_NFEAT each */
    int nshapes;
    const int *shape_bits, *shape_low;
    int per_shape;
    int gate_slack;
    int lookahead;
} qs_plan_model;
QS_API int qs_plan_create_learned(qs_plan **out, const qs_circuit *c, const qs_plan_opts *opts,
                                  const qs_plan_model *model);

/* An MLP nin -> hidden -> hidden -> 1 (ReLU between layers), FP32, trained with MSE loss and Adam on the GPU by
 * the library's own kernels (deterministic fixed-order reductions). Parameters are one flat array:
 * W1[hidden][nin], b1[hidden], W2[hidden][hidden], b2[hidden], W3[hidden], b3. Batches hold 1..4096 samples;
 * X is row-major (sample, feature); host arrays are copied during the call. All calls synchronise. */
QS_API int qs_mlp_create(qs_mlp **out, int nin, int hidden, void *hip_stream);
QS_API int qs_mlp_free(qs_mlp *m);
QS_API int qs_mlp_num_params(const qs_mlp *m, int *nparams);
/* Set the parameters (and reset the optimiser state) / read them back. */
QS_API int qs_mlp_set_params(qs_mlp *m, const float *params);
QS_API int qs_mlp_get_params(qs_mlp *m, float *params);
/* Y[s] = network(X[s]) for s < B. */
QS_API int qs_mlp_predict(qs_mlp *m, const float *X, int B, float *Y);
/* Forward + backward of the mean squared error against targets T: gradients (nparams floats, same layout as the
 * parameters) and loss, without updating; either output may be NULL. */
QS_API int qs_mlp_grad(qs_mlp *m, const float *X, const float *T, int B, float *grads, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the batch; loss before the step (nullable). */
QS_API int qs_mlp_train_step(qs_mlp *m, const float *X, const float *T, int B, float lr, float *loss);

/* ---- batches of independent circuits (serving form) ----
 * Many circuits (8..30 qubits each, gates on at most 3 qubits, no fused-swaps) run as one short sequence of
 * persistent launches, one per pass level: launch k runs pass k of every circuit that has more than k block passes,
 * all of their blocks forming one index space that the whole grid walks (so a large circuit is spread over every
 * compute unit). Circuits of at most block_bits qubits run start to finish inside one workgroup's LDS during the
 * first launch. Every circuit starts in |0..0>, generated in the first pass, and its last pass writes its FP64
 * output probabilities instead of amplitudes.
 *   block_bits 10..12 (the LDS block), low_bits the always-local low qubits, wg_per_cu 1..64 persistent
 *   workgroups per compute unit (tile and schedule parameters chosen by the autotuner). */
typedef struct qs_batch qs_batch;
QS_API int qs_batch_create(qs_batch **out, int dtype, int block_bits, int low_bits, int wg_per_cu, void *hip_stream);
/* Change the persistent workgroups per CU (1..64) of later runs; a captured graph is dropped (the call waits for the
 * batch's stream first) and captured again by the next graph run. Host-side only otherwise. */
QS_API int qs_batch_set_launch(qs_batch *b, int wg_per_cu);
/* Plan and append a circuit (host only). QS_EUNSUPPORTED for circuits outside the batch's scope. */
QS_API int qs_batch_add(qs_batch *b, const qs_circuit *c);
/* Build the pass levels, allocate state and probability slices, upload the tables (synchronous). QS_EUNSUPPORTED if
 * one level would exceed 2^31 blocks; QS_ENOMEM (or QS_EDEVICE) if an allocation or copy fails, in which case
 * nothing stays allocated and a later call retries. */
QS_API int qs_batch_finalize(qs_batch *b);
/* Enqueue the whole batch (one launch per level) on the batch's stream. use_graph != 0 captures the launches once
 * into a HIP graph (kernel nodes only) and replays it on later calls. Finalizes the batch if needed. */
QS_API int qs_batch_run(qs_batch *b, int use_graph);
/* Any output may be NULL: circuits, bytes of HBM state, FP64 probabilities, block passes, levels (0 before
 * finalize). */
QS_API int qs_batch_info(const qs_batch *b, int *ncirc, int64_t *state_bytes, int64_t *prob_count, int *npasses,
                         int *nlevels);
/* Circuit i's 2^n probabilities (in the order circuits were added): device pointer and/or a synchronous copy. */
QS_API int qs_batch_probs(qs_batch *b, int i, double **dev_ptr, double *host_out);
QS_API int qs_batch_free(qs_batch *b);

/* ---- bandwidth probes (the measured HBM ceiling the gate kernels are compared against) ---- */

/* dst[i] = src[i] over `bytes` (multiple of 16, both 16-byte aligned), enqueued on hip_stream. */
QS_API int qs_probe_copy(void *dst, const void *src, size_t bytes, void *hip_stream);
/* In-place read-modify-write of every 16-byte word of buf (each double multiplied by a runtime factor of 1.0,
 * so the stores are real): the traffic pattern of an in-place gate pass without its arithmetic. */
QS_API int qs_probe_rmw(void *buf, size_t bytes, void *hip_stream);

/* ---- launch tunables (autotuner / sweeps) ----
 * "dense_gpt"   groups per thread of the 1- and 2-qubit dense kernels: 1, 2 or 4 (default 1);
 * "nontemporal" 0/1: non-temporal loads and stores in the dense kernels (default 1);
 * "mfma_wg_per_cu" persistent workgroups per compute unit of the k = 5, 6 MFMA block kernel (1..16, default 2);
 * "block_wg_per_cu" persistent 256-thread workgroups per compute unit of the LDS block kernel (1..4096, default
 *               32: a grid far larger than the resident workgroups measured fastest; smaller workgroups are
 *               scaled up proportionally);
 * "block_stage_width" register stage width of block plans created afterwards: 4 (256-thread kernel, default) or
 *                     3 (512-thread kernel with 8 register amplitudes per thread, for 12- and 13-qubit blocks);
 * "block_async" 0/1: 12-qubit complex128 block passes double-buffer the next block in LDS with direct-to-LDS loads
 *               (default 0: one workgroup per CU fits, measured slower than two with register prefetch);
 * "block_lanes" 0/1: in plans created afterwards, complex128 12-qubit block passes whose ops act on one or two
 *               register positions run a 512-thread kernel that holds each 16-amplitude register group in two
 *               lanes (4 waves per SIMD instead of 2; default 0: measured 0.5 % slower, the chip's sustained
 *               clock falls as VALU activity rises);
 * "mfma_stage_ops" complex64 block plans and batches created afterwards: in each pass, up to 4 of the 4-position
 *               stages whose ops amount to at least this many 2-qubit ops' arithmetic (a k-qubit op counts
 *               2^(k-2); the stages with the most) run as one fused 16 x 16 product on the FP32 matrix cores
 *               (0..8, default 3; 0: every stage op by op on the vector ALUs);
 * "stage_pack"  0/1: how block plans created afterwards group a pass's ops into register stages. 0: repeatedly
 *               take the ready op that adds the fewest new positions until none fits. 1 (default): each stage
 *               is seeded in turn by every ready op and filled that way, and the seed whose remaining ops then
 *               need the fewest such stages wins (ties: more ops in the stage);
 * "plan_beam"   beam width of pass formation for plans created afterwards (0..64, default 16): the local set of a
 *               pass grows one ready gate at a time, keeping the candidates that take the most gates; 0 selects
 *               the fewest-new-qubits greedy. Batches always plan with 4-position stages.
 * "plan_beam_search" 0/1: plans created afterwards with qs_plan_create (not batches) also form their passes at
 *               1.5x and 4x the beam width (at most 64) and keep the formation with the fewest passes, ties to
 *               the smaller width (default 0: the learned planner prices candidate plans at several widths
 *               instead, with the single-width greedy plan as its reference).
 * Process-wide; affects launches enqueued and plans created after the call. QS_EINVAL for an unknown name or
 * value. */
QS_API int qs_set_tunable(const char *name, int64_t value);
/* The current value of a tunable named as above. QS_EINVAL for a NULL argument or an unknown name. */
QS_API int qs_get_tunable(const char *name, int64_t *value);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
