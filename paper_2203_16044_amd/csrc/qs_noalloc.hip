// Allocation-free entry point: probabilities and norm of a caller's raw amplitude buffer.
//
// The reduction behind qs_probs needs FP64 partial sums between its two kernels (k_probs, then k_sum_partials); a
// state handle keeps them in memory allocated by qs_alloc. Callers that cannot allocate (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation) get them from the file-scope device array
// below instead: one copy per GPU, loaded with the code object and held until the process ends. Host code never
// passes the array's name to a kernel (on the host that name is only a stand-in for the symbol); it resolves the
// array's device address once per device with hipGetSymbolAddress and passes that address.
#include <mutex>

#include "qs_internal.h"

namespace {

constexpr int kScratchPartials = 4096;  // = the largest partial count of the probability reduction (probs_blocks)
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchPartials + 32];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (resolved on the first call made with the device current).
int scratch_for_current_device(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return qs_hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return qs_fail(QS_EUNSUPPORTED, "qs_probs_noalloc: device ordinal %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return qs_hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return qs_fail(QS_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return QS_OK;
}

}  // namespace

QS_API int qs_probs_noalloc(const void *psi, int n, int dtype, double *out_dev, double *norm_dev, void *hip_stream)
{
    qs_clear_error();
    if (!psi)
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: NULL amplitude buffer");
    if (reinterpret_cast<uintptr_t>(psi) % 16 != 0)
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: amplitude buffer not 16-byte aligned");
    if (n < 1 || n > QS_MAX_QUBITS)
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: n = %d outside [1, %d]", n, QS_MAX_QUBITS);
    if (dtype != QS_C128 && dtype != QS_C64)
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: unknown dtype %d", dtype);
    if (!out_dev && !norm_dev)
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: out_dev and norm_dev are both NULL");
    if ((out_dev && reinterpret_cast<uintptr_t>(out_dev) % 8 != 0) ||
        (norm_dev && reinterpret_cast<uintptr_t>(norm_dev) % 8 != 0))
        return qs_fail(QS_EINVAL, "qs_probs_noalloc: output not 8-byte aligned");
    const uint64_t dim = (uint64_t)1 << n;
    const int nb = probs_blocks(dim);
    if (nb > kScratchPartials)
        return qs_fail(QS_EUNSUPPORTED, "qs_probs_noalloc: %d partial sums exceed the %d-entry scratch", nb,
                       kScratchPartials);
    double *part = nullptr;
    const int rc = scratch_for_current_device(&part);
    if (rc != QS_OK)
        return rc;
    // without a norm output the sum still runs (its kernels are shared with qs_probs) into the scratch's spare slot
    double *result = norm_dev ? norm_dev : part + kScratchPartials;
    QS_HIP(launch_probs(dtype, psi, dim, out_dev, part, nb, result, static_cast<hipStream_t>(hip_stream)));
    return QS_OK;
}
