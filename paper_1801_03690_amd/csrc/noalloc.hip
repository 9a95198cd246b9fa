// The allocation-free variant of mm_precondition (mmncg.h): for callers that
// cannot allocate device memory during the call. The scratch of the inner
// solve of Alg. 1 (its residual, direction and product vectors, the block
// partial sums and the exit flags) lives in one static device array per GPU
// instead of context memory; the inputs, the output and the operators stay in
// the context. Every call on a GPU uses that GPU's copy of the array, so calls
// that overlap on one GPU (two streams, two threads) race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "context.h"

namespace mmncg {
namespace {

constexpr size_t kScratchBytes = (size_t)MM_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current: taken
// once per device with hipGetSymbolAddress (the array's name is a host-side
// stand-in, not a device address) and kept for later calls.
void *scratch_of(int dev) {
    if (dev < 0 || dev >= kMaxDevices) throw ApiError{MM_EINVAL, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw ApiError{MM_EDEVICE, "no device address for the static scratch"};
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace
}  // namespace mmncg

using namespace mmncg;

extern "C" int mm_precondition_noalloc(mm_ctx *c, const double *m, const double *grad, const double *gproj, int jmax,
                                       const double *dscale, double *y, int *inner_iters) {
    // guarded() makes the context's device current before the body runs
    return guarded(c, [&] {
        require_single(c);
        const size_t need = prec_scratch_bytes(c);
        if (need > kScratchBytes)
            throw ApiError{MM_EINVAL, "the inner solve needs " + std::to_string(need) +
                                          " bytes of scratch; the static array holds " +
                                          std::to_string(kScratchBytes) + " (about 460,000 magnet nodes)"};
        const PrecScratch s = prec_scratch_at(c, scratch_of(c->device));
        // the exit flags start at zero: cleared with a fill kernel (no memset
        // node if the caller captures the call in a graph)
        launch_fill(2 * (int64_t)c->ninst, (double *)s.flags, 0.0, c->stream);
        return precondition_call(c, m, grad, gproj, jmax, dscale, y, inner_iters, &s);
    });
}
