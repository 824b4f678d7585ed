// Measurement, sampling and reset (the simulator's intermediate measurement, Sec. II-A and Sec. I: the state
// vector gives the outcome probabilities directly, and a measured state collapses onto the observed outcome).
//
//  * qs_measure: one FP64 pass yields P0 and P1 (the probability mass with the qubit's bit 0 / 1), the outcome is
//    decided on the host in FP64 from a caller-supplied uniform u, and one more pass keeps the amplitudes of the
//    observed outcome, scaled by 1/sqrt(P_outcome), and zeroes the others.
//  * qs_sample: the state is cut into chunks of 4096 amplitudes (one wave each: 64 lanes x 64 consecutive
//    amplitudes); each chunk's FP64 mass is the last element of a wave-inclusive scan of its lane sums, a
//    deterministic two-level scan turns the chunk masses into an inclusive prefix, and each shot (one wave)
//    finds its chunk by binary search and its index by repeating the chunk's scan. Shot k returns the smallest
//    index i whose cumulative mass exceeds u_k x total mass, with the same additions on every path.
#include <cmath>

#include "qs_internal.h"

namespace {

template <class R> struct MT;
template <> struct MT<double> { using C2 = double2; };
template <> struct MT<float> { using C2 = float2; };

constexpr int kMeasBlocks = 2048;  // partial pairs fit the state's reduction scratch (2 x 2048 <= 4096)
constexpr int kChunkLog = 12;      // 4096 amplitudes per sampling chunk
constexpr int kTile = 2048;        // chunk masses scanned per workgroup (256 threads x 8)

template <class R>
__device__ __forceinline__ double mag2(const typename MT<R>::C2 &v)
{
    const double re = (double)v.x, im = (double)v.y;
    return re * re + im * im;
}

// Per-block FP64 masses of the amplitudes whose bit q is 0 and 1 (grid-stride, then an LDS tree in fixed order).
template <class R>
__global__ __launch_bounds__(256) void k_measure_partials(const typename MT<R>::C2 *__restrict__ psi, uint64_t dim,
                                                          int q, double *__restrict__ partials)
{
    __shared__ double r0[256], r1[256];
    double a0 = 0.0, a1 = 0.0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * 256) {
        const double p = mag2<R>(psi[i]);
        if ((i >> q) & 1)
            a1 += p;
        else
            a0 += p;
    }
    r0[threadIdx.x] = a0;
    r1[threadIdx.x] = a1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r0[0];
        partials[2 * blockIdx.x + 1] = r1[0];
    }
}

// Sum the partial pairs in a fixed order (compensated), result[0] = P0, result[1] = P1.
__global__ __launch_bounds__(64) void k_measure_total(const double *__restrict__ partials, int nb,
                                                      double *__restrict__ result)
{
    if (threadIdx.x >= 2)
        return;
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double y = partials[2 * b + threadIdx.x] - c;
        const double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    result[threadIdx.x] = s;
}

// Keep the amplitudes whose bit q equals `outcome`, scaled by `scale` in FP64; zero the others (not read).
template <class R>
__global__ __launch_bounds__(256) void k_collapse(typename MT<R>::C2 *__restrict__ psi, uint64_t dim, int q,
                                                  int outcome, double scale)
{
    using C2 = typename MT<R>::C2;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < dim; i += (uint64_t)gridDim.x * 256) {
        C2 v;
        if ((int)((i >> q) & 1) == outcome) {
            v = psi[i];
            v.x = (R)((double)v.x * scale);
            v.y = (R)((double)v.y * scale);
        } else {
            v.x = 0;
            v.y = 0;
        }
        psi[i] = v;
    }
}

// Wave-inclusive scan of one FP64 value per lane (Hillis-Steele, 6 steps, the same order on every call).
__device__ __forceinline__ double wave_incl_scan(double x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d, 64);
        if (lane >= d)
            x += y;
    }
    return x;
}

// Mass of lane `lane`'s `per` consecutive amplitudes of a chunk (sequential FP64 sum).
template <class R>
__device__ __forceinline__ double lane_mass(const typename MT<R>::C2 *__restrict__ psi, uint64_t first, int per,
                                            uint64_t dim)
{
    double s = 0.0;
    for (int j = 0; j < per; ++j) {
        const uint64_t i = first + j;
        if (i < dim)
            s += mag2<R>(psi[i]);
    }
    return s;
}

// One wave per chunk: its mass = the last element of the wave-inclusive scan of the lane masses.
template <class R>
__global__ __launch_bounds__(256) void k_chunk_mass(const typename MT<R>::C2 *__restrict__ psi, uint64_t dim,
                                                    uint64_t chunk, int per, uint64_t nchunks,
                                                    double *__restrict__ mass)
{
    const uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= nchunks)
        return;  // whole waves leave together
    const int lane = threadIdx.x & 63;
    const double incl = wave_incl_scan(lane_mass<R>(psi, c * chunk + (uint64_t)lane * per, per, dim));
    if (lane == 63)
        mass[c] = incl;
}

// Level 1 of the prefix scan: each workgroup scans a tile of kTile masses (8 sequential per thread, then an LDS
// Hillis-Steele scan of the 256 thread sums) into tile-local inclusive prefixes, and writes the tile total.
__global__ __launch_bounds__(256) void k_scan_tile(const double *__restrict__ in, uint64_t len,
                                                   double *__restrict__ out, double *__restrict__ totals)
{
    __shared__ double sh[256];
    const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * 8;
    double v[8];
    double run = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = base + j < len ? in[base + j] : 0.0;
        run += v[j];
        v[j] = run;
    }
    sh[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < 256; d <<= 1) {
        const double y = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0.0;
        __syncthreads();
        sh[threadIdx.x] += y;
        __syncthreads();
    }
    const double before = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        if (base + j < len)
            out[base + j] = before + v[j];
    if (threadIdx.x == 255)
        totals[blockIdx.x] = sh[255];
}

// Level 2: one thread turns the tile totals into exclusive tile offsets (sequential order).
__global__ void k_scan_totals(double *__restrict__ totals, uint64_t ntiles)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    double run = 0.0;
    for (uint64_t t = 0; t < ntiles; ++t) {
        const double x = totals[t];
        totals[t] = run;
        run += x;
    }
    totals[ntiles] = run;
}

// Level 3: add each tile's offset.
__global__ __launch_bounds__(256) void k_scan_add(double *__restrict__ out, uint64_t len,
                                                  const double *__restrict__ offs)
{
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < len && i >= (uint64_t)kTile)
        out[i] += offs[i / kTile];
}

// One wave per shot. total = incl[last]; target = u x total; the chunk is the smallest c with incl[c] > target
// (or, when rounding puts the target at the total, the smallest c with incl[c] >= total); the index is found by
// repeating the chunk's lane sums and wave scan. If rounding leaves no index above the residual, the chunk's last
// index with nonzero mass is taken. Every returned index lies in [0, dim).
template <class R>
__global__ __launch_bounds__(256) void k_sample(const typename MT<R>::C2 *__restrict__ psi, uint64_t dim,
                                                uint64_t chunk, int per, uint64_t nchunks,
                                                const double *__restrict__ incl, const double *__restrict__ u,
                                                int64_t nshots,
                                                int64_t *__restrict__ out)
{
    const int64_t shot = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (shot >= nshots)
        return;
    const int lane = threadIdx.x & 63;
    const double total = incl[nchunks - 1];
    double target = u[shot] * total;
    const bool clamp = !(target < total);
    uint64_t lo = 0, hi = nchunks - 1;
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        const bool right = clamp ? incl[mid] < total : incl[mid] <= target;
        if (right)
            lo = mid + 1;
        else
            hi = mid;
    }
    const uint64_t c = lo;
    const double r = target - (c > 0 ? incl[c - 1] : 0.0);
    const uint64_t first = c * chunk + (uint64_t)lane * per;
    const double mine = lane_mass<R>(psi, first, per, dim);
    const double sc = wave_incl_scan(mine);
    const unsigned long long above = __ballot(!clamp && sc > r);
    const unsigned long long nonzero = __ballot(mine > 0.0);
    int pick;
    bool exact;
    if (above) {
        pick = __ffsll(above) - 1;
        exact = true;
    } else {
        pick = nonzero ? 63 - __clzll(nonzero) : 63;
        exact = false;
    }
    // every lane takes part in both shuffles (a lane inactive in a shuffle gives undefined values to its readers)
    const double prev = __shfl_up(sc, 1, 64);
    const double before = __shfl(lane > 0 ? prev : 0.0, pick, 64);
    if (lane != pick)
        return;
    const double rr = r - (pick > 0 ? before : 0.0);
    double acc = 0.0;
    int64_t last_nz = -1, found = -1;
    for (int j = 0; j < per; ++j) {
        const uint64_t i = first + j;
        if (i >= dim)
            break;
        const double p = mag2<R>(psi[i]);
        acc += p;
        if (p > 0.0)
            last_nz = (int64_t)i;
        if (exact && found < 0 && acc > rr)
            found = (int64_t)i;
    }
    if (found < 0)
        found = last_nz >= 0 ? last_nz : (int64_t)(first + per - 1 < dim ? first + per - 1 : dim - 1);
    out[shot] = found;
}

template <class R>
hipError_t measure_r(void *psi, uint64_t dim, int q, double *partials, double *result, hipStream_t s)
{
    using C2 = typename MT<R>::C2;
    uint64_t nb = (dim + 256 * 16 - 1) / (256 * 16);
    if (nb > (uint64_t)kMeasBlocks)
        nb = kMeasBlocks;
    if (nb == 0)
        nb = 1;
    hipLaunchKernelGGL((k_measure_partials<R>), dim3((unsigned)nb), dim3(256), 0, s, (const C2 *)psi, dim, q,
                       partials);
    hipLaunchKernelGGL(k_measure_total, dim3(1), dim3(64), 0, s, (const double *)partials, (int)nb, result);
    return hipGetLastError();
}

template <class R>
hipError_t collapse_r(void *psi, uint64_t dim, int q, int outcome, double scale, hipStream_t s)
{
    using C2 = typename MT<R>::C2;
    uint64_t grid = (dim + 255) / 256;
    if (grid > ((uint64_t)1 << 20))
        grid = (uint64_t)1 << 20;
    hipLaunchKernelGGL((k_collapse<R>), dim3((unsigned)grid), dim3(256), 0, s, (C2 *)psi, dim, q, outcome, scale);
    return hipGetLastError();
}

struct SampleGeom {
    uint64_t chunk, nchunks, ntiles;
    int per;
};

SampleGeom sample_geom(uint64_t dim)
{
    SampleGeom g;
    g.chunk = dim < ((uint64_t)1 << kChunkLog) ? dim : ((uint64_t)1 << kChunkLog);
    g.per = (int)(g.chunk >= 64 ? g.chunk / 64 : 1);
    g.nchunks = dim / g.chunk;
    g.ntiles = (g.nchunks + kTile - 1) / kTile;
    return g;
}

template <class R>
hipError_t sample_r(const void *psi, uint64_t dim, const SampleGeom &g, double *mass, double *incl, double *tiles,
                    const double *u, int64_t nshots, int64_t *out, hipStream_t s)
{
    using C2 = typename MT<R>::C2;
    hipLaunchKernelGGL((k_chunk_mass<R>), dim3((unsigned)((g.nchunks + 3) / 4)), dim3(256), 0, s, (const C2 *)psi,
                       dim, g.chunk, g.per, g.nchunks, mass);
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)g.ntiles), dim3(256), 0, s, (const double *)mass, g.nchunks, incl,
                       tiles);
    hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(64), 0, s, tiles, g.ntiles);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((g.nchunks + 255) / 256)), dim3(256), 0, s, incl, g.nchunks,
                       (const double *)tiles);
    hipLaunchKernelGGL((k_sample<R>), dim3((unsigned)((nshots + 3) / 4)), dim3(256), 0, s, (const C2 *)psi, dim,
                       g.chunk, g.per, g.nchunks, (const double *)incl, u, nshots, out);
    return hipGetLastError();
}

int measure_impl(qs_state *st, int qubit, double u, int *outcome, double *prob_one)
{
    const uint64_t dim = (uint64_t)1 << st->n;
    double *partials = st->red;
    double *result = st->red + 2 * kMeasBlocks;
    QS_HIP(st->dtype == QS_C128 ? measure_r<double>(st->psi, dim, qubit, partials, result, st->stream)
                                : measure_r<float>(st->psi, dim, qubit, partials, result, st->stream));
    double P[2] = {0.0, 0.0};
    QS_HIP(hipMemcpyAsync(P, result, sizeof(P), hipMemcpyDeviceToHost, st->stream));
    QS_HIP(hipStreamSynchronize(st->stream));
    const double tot = P[0] + P[1];
    if (!(tot > 0.0) || !std::isfinite(tot))
        return qs_fail(QS_EINVAL, "qs_measure: the state has no finite nonzero mass (%g)", tot);
    const int out = (u * tot < P[1]) ? 1 : 0;
    const double keep = out ? P[1] : P[0];
    QS_HIP(st->dtype == QS_C128 ? collapse_r<double>(st->psi, dim, qubit, out, 1.0 / std::sqrt(keep), st->stream)
                                : collapse_r<float>(st->psi, dim, qubit, out, 1.0 / std::sqrt(keep), st->stream));
    if (outcome)
        *outcome = out;
    if (prob_one)
        *prob_one = P[1] / tot;
    return QS_OK;
}

}  // namespace

extern "C" {

QS_API int qs_measure(qs_state *st, int qubit, double u, int *outcome, double *prob_one)
{
    qs_clear_error();
    if (!st || !outcome)
        return qs_fail(QS_EINVAL, "qs_measure: NULL argument");
    if (qubit < 0 || qubit >= st->n)
        return qs_fail(QS_EINVAL, "qs_measure: qubit %d outside [0, %d)", qubit, st->n);
    if (!(u >= 0.0 && u < 1.0))
        return qs_fail(QS_EINVAL, "qs_measure: u = %g outside [0, 1)", u);
    if (st->red_cap < 2 * (size_t)kMeasBlocks + 2)
        return qs_fail(QS_EUNSUPPORTED, "qs_measure: reduction scratch too small");
    return measure_impl(st, qubit, u, outcome, prob_one);
}

QS_API int qs_reset(qs_state *st, int qubit, double u, int *outcome)
{
    qs_clear_error();
    int out = 0;
    if (int rc = qs_measure(st, qubit, u, &out, nullptr))
        return rc;
    if (out) {
        static const double X[8] = {0, 0, 1, 0, 1, 0, 0, 0};
        const int t = qubit;
        if (int rc = qs_apply_gate(st, &t, 1, X))
            return rc;
    }
    if (outcome)
        *outcome = out;
    return QS_OK;
}

QS_API int qs_sample(qs_state *st, int64_t nshots, const double *u, int64_t *out)
{
    qs_clear_error();
    if (!st || (nshots > 0 && (!u || !out)))
        return qs_fail(QS_EINVAL, "qs_sample: NULL argument");
    if (nshots < 0 || nshots > ((int64_t)1 << 30))
        return qs_fail(QS_EINVAL, "qs_sample: nshots = %lld outside [0, 2^30]", (long long)nshots);
    for (int64_t k = 0; k < nshots; ++k)
        if (!(u[k] >= 0.0 && u[k] < 1.0))
            return qs_fail(QS_EINVAL, "qs_sample: u[%lld] = %g outside [0, 1)", (long long)k, u[k]);
    if (nshots == 0)
        return QS_OK;
    const uint64_t dim = (uint64_t)1 << st->n;
    const SampleGeom g = sample_geom(dim);
    // scratch: chunk masses, inclusive prefix, tile totals (+ total), uniforms, outputs
    const size_t nd = 2 * g.nchunks + g.ntiles + 1;
    const size_t bytes = nd * sizeof(double) + (size_t)nshots * (sizeof(double) + sizeof(int64_t));
    char *buf = nullptr;
    QS_HIP(hipStreamSynchronize(st->stream));
    QS_HIP(hipMalloc(&buf, bytes));
    double *mass = (double *)buf;
    double *incl = mass + g.nchunks;
    double *tiles = incl + g.nchunks;
    double *du = tiles + g.ntiles + 1;
    int64_t *dout = (int64_t *)(du + nshots);
    hipError_t e = hipMemcpyAsync(du, u, (size_t)nshots * sizeof(double), hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess)
        e = st->dtype == QS_C128 ? sample_r<double>(st->psi, dim, g, mass, incl, tiles, du, nshots, dout, st->stream)
                                 : sample_r<float>(st->psi, dim, g, mass, incl, tiles, du, nshots, dout, st->stream);
    double total = 0.0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(out, dout, (size_t)nshots * sizeof(int64_t), hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, incl + (g.nchunks - 1), sizeof(double), hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st->stream);
    (void)hipFree(buf);
    if (e != hipSuccess)
        return qs_hip_fail(e, "qs_sample");
    // a state without finite nonzero mass has no distribution: its indices are meaningless
    if (!(total > 0.0) || !std::isfinite(total))
        return qs_fail(QS_EINVAL, "qs_sample: the state has no finite nonzero mass (%g)", total);
    return QS_OK;
}

}  // extern "C"
