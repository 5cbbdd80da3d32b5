// dirac_norm_device_static: the conserved functional of dirac_norm_device with
// its reduction partials in a library-owned device array instead of the
// caller-bound scratch, for callers that cannot allocate device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>

#include "../../include/dirac.h"
#include "ctx.h"
#include "internal.h"

using namespace dirac;

namespace {

// One workgroup partial per reduction block: kReduceBlocks x kNormVals doubles.
constexpr size_t kStaticScratchBytes = DIRAC_STATIC_SCRATCH_BYTES;
static_assert((size_t)kReduceBlocks * kNormVals * sizeof(double) <= kStaticScratchBytes,
              "the functional's partials must fit the static scratch");

// Each GPU the library runs on holds its own copy until the process ends.  In
// host code the name is only a stand-in for the symbol: kernels are given the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
hipError_t scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return hipSuccess;
}

template <typename R> ReduceArgs<R> args_for(const dirac_ctx *c, double *partial) {
    ReduceArgs<R> a;
    memset(&a, 0, sizeof a);
    const int narr = c->ndim == 3 ? 8 : 4;
    for (int q = 0; q < narr; ++q) a.f[q] = c->buf[c->cur][q];
    a.rx = (R)c->rx;
    a.ry = (R)c->ry;
    a.rz = (R)c->rz;
    a.nx = (int)c->nx;
    a.ny = (int)c->ny;
    a.nz = (int)c->nz;
    a.partial = partial;
    a.zh = c->zh;
    a.zbc = c->zbc ? 1 : 0;
    return a;
}

}  // namespace

extern "C" int dirac_norm_device_static(dirac_ctx *c, void *dev_out, void *stream) {
    if (!c) return DIRAC_E_ARG;
    if (c->is_batch) {
        c->err = "batch context: use the dirac_batch_* calls";
        return DIRAC_E_STATE;
    }
    if (!c->bound) {
        c->err = "no state bound (dirac_bind_state)";
        return DIRAC_E_STATE;
    }
    if (!dev_out) {
        c->err = "null output";
        return DIRAC_E_ARG;
    }
    const size_t need = (size_t)kReduceBlocks * kNormVals * sizeof(double);
    if (need > kStaticScratchBytes) {      // fixed by the reduction layout; kept as a run-time guard too
        c->err = "reduction partials exceed the static scratch";
        return DIRAC_E_SHAPE;
    }
    void *p = nullptr;
    hipError_t e = scratch_ptr(&p);
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)p;
    if (e == hipSuccess) {
        if (c->links_on) {
            LinkPtrs L;
            for (int q = 0; q < 24; ++q) L.u[q] = c->links[q];
            e = c->dtype == DIRAC_C64 ? launch_norm_links<float>(args_for<float>(c, part), L, c->ndim, s)
                                      : launch_norm_links<double>(args_for<double>(c, part), L, c->ndim, s);
        } else if (c->dtype == DIRAC_C64) {
            e = c->ndim == 3 ? launch_norm3<float>(args_for<float>(c, part), s)
                             : launch_norm2<float>(args_for<float>(c, part), s);
        } else {
            e = c->ndim == 3 ? launch_norm3<double>(args_for<double>(c, part), s)
                             : launch_norm2<double>(args_for<double>(c, part), s);
        }
    }
    if (e == hipSuccess) e = launch_final_sum(part, kReduceBlocks, kNormVals, (double *)dev_out, s);
    if (e != hipSuccess) {
        c->err = std::string("dirac_norm_device_static: ") + hipGetErrorString(e);
        return DIRAC_E_HIP;
    }
    return DIRAC_OK;
}
