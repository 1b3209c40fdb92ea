// The march of one band with no allocation (lrt_march_noalloc): the
// per-(ray, chunk) partial sums of the spectral trapezoid, which lrt_march
// keeps in a workspace it allocates, go to a static device array instead.
// Each device the library runs on holds its own copy of the array, at its own
// address, until the process ends; the address is looked up once per device
// when a context is created there.  Calls that overlap on one device share
// the array and race.  The march writes every partial it later reads, so
// nothing has to be cleared between calls.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/lrt.h"
#include "lrt_ctx.h"
#include "lrt_internal.h"

namespace lrt {

namespace {

// 2^23 doubles (64 MiB): rays x march chunks of one band at most.
constexpr int64_t kScratchDoubles = int64_t(1) << 23;
constexpr int kMaxDevices = 64;

std::mutex g_mu;
double *g_scratch[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t noalloc_scratch_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[device] = static_cast<double *>(p);
    return hipSuccess;
}

}  // namespace lrt

using namespace lrt;

extern "C" lrt_status lrt_march_noalloc(lrt_ctx *c, int64_t band, lrt_precision prec, const void *eta,
                                        const void *kappa, const int32_t *escale, double *I_out,
                                        double *I_int_out, void *stream)
{
    if (!c) return LRT_E_ARG;
    c->err.clear();
    if (!c->have_grid) return fail(c, LRT_E_STATE, "grid not set");
    double *part = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        part = (c->device >= 0 && c->device < kMaxDevices) ? g_scratch[c->device] : nullptr;
    }
    if (!part) return fail(c, LRT_E_STATE, "no scratch address for device %d", c->device);
    int32_t k_first, n_band;
    lrt_status r;
    if ((r = band_range(c, band, k_first, n_band))) return r;
    return march_range(c, k_first, n_band, prec, eta, kappa, escale, I_out, I_int_out, (hipStream_t)stream, part,
                       kScratchDoubles);
}
