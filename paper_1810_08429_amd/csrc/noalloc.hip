// gca_energy_noalloc: the energy call of gca_energy with its workspace in a
// fixed device array instead of memory the library allocates, for callers
// that cannot allocate device memory (work under stream capture, tight
// loops, hosts that forbid allocation).
//
// The workspace of gca_energy is the dot-product partials (DOT_PARTIALS
// doubles) and, when the caller wants E only, the product G~ u (n doubles).
// Here both live in `scratch`, one array per GPU that holds the library,
// kept until the process ends.  Host code never uses the array's name as an
// address: on the first call on a device (with that device current) its
// device address is looked up once with hipGetSymbolAddress and kept per
// device; kernels receive that address like any other workspace pointer.
//
// Nothing in the array has to start at zero: the dot kernels write every
// partial they read and the product overwrites G~ u.  Calls on one GPU share
// the array, so calls that overlap in time on one GPU (different streams or
// host threads without ordering) race on it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gca_internal.h"

namespace {

// partials first, then room for the product of a handle of up to
// GCA_NOALLOC_MAX_N triangles (both in doubles)
constexpr size_t SCRATCH_DOUBLES = gca::DOT_PARTIALS + (size_t)GCA_NOALLOC_MAX_N;

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double *g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
gca_status scratch_ptr(double **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gca::set_error(GCA_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return gca::set_error(GCA_EINVAL, "device ordinal beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return gca::set_error(GCA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_ptr[dev] = (double *)p;
    }
    *out = g_ptr[dev];
    return GCA_OK;
}

}  // namespace

extern "C" gca_status gca_energy_noalloc(gca_h2 h, const double *u, const double *scale, double *e, double *g,
                                         int32_t precision, void *stream)
{
    gca::clear_error();
    GCA_TRY(gca::energy_check(h, u, e, g, precision));
    if (!g && h->n > (int64_t)GCA_NOALLOC_MAX_N)
        return gca::set_error(GCA_EINVAL, "gca_energy_noalloc: n = " + std::to_string(h->n) +
                                              " exceeds GCA_NOALLOC_MAX_N = " + std::to_string(GCA_NOALLOC_MAX_N) +
                                              " when g is NULL (pass g, which then holds G~ u)");
    double *ws = nullptr;
    GCA_TRY(scratch_ptr(&ws));
    return gca::energy_run(h, u, scale, e, g, precision, (hipStream_t)stream, ws, ws + gca::DOT_PARTIALS);
}
