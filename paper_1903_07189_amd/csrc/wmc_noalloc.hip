// wmc_noalloc.hip -- wmc_solve_noalloc: the solve of wmc_solve for callers
// that cannot allocate device memory (code under graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The ping-pong state of a solve of two or more sweeps lives in `scratch`, a
// file-scope device array that every device the library runs on holds until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is taken once per device with
// hipGetSymbolAddress (that device current) and only that address is ever
// passed to kernels.  Calls on one device share its array; each launch
// writes every pixel of its output plane set before the next launch reads
// it, so nothing in the array needs clearing between calls, but calls that
// overlap on one device (other streams, other threads) race on it.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "wmc.h"
#include "wmc_internal.h"

static_assert(WMC_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256 bytes");

static __device__ __align__(256) float scratch[WMC_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

std::mutex g_scratch_mu;
std::map<int, float*> g_scratch;  // device -> device address of its `scratch`

}  // namespace

extern "C" int wmc_solve_noalloc(const float* f, const float* u0, float* u_out, const float* lam,
                                 int iters, float dt, const wmc_tuning* tune, wmc_shape s,
                                 void* stream) {
    float* ws = nullptr;
    if (iters >= 2) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_scratch_mu);
            auto it = g_scratch.find(dev);
            if (it == g_scratch.end()) {
                void* p = nullptr;
                e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
                if (e == hipSuccess && p) it = g_scratch.emplace(dev, static_cast<float*>(p)).first;
            }
            if (it != g_scratch.end()) ws = it->second;
        }
        if (!ws)
            return wmc::report_error(
                WMC_EHIP, std::string("wmc_solve_noalloc: device address of the scratch: ") +
                              hipGetErrorString(e));
    }
    return wmc::solve_impl(f, u0, u_out, lam, iters, dt, nullptr, 0, tune, ws,
                           WMC_NOALLOC_SCRATCH_BYTES, s, stream, true);
}
