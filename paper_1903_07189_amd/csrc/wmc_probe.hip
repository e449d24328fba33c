// wmc_probe.hip -- streaming bandwidth probe: the achievable-bandwidth
// ceiling the update kernels are measured against.  A measurement aid, no
// part of the method: o = a (copy) or o = a + b over n floats, each lane
// moving four 16-byte vectors per round (four loads in flight before the
// stores), grid-stride.  NT makes every load and store non-temporal.
#include <hip/hip_runtime.h>

#include "wmc_internal.h"

namespace wmc {

namespace {

typedef float p4f __attribute__((ext_vector_type(4)));
constexpr int kProbeBlock = 256;
constexpr int kProbeUnroll = 4;

template <bool NT>
__device__ __forceinline__ p4f probe_ld(const p4f* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool ADD, bool NT>
__global__ __launch_bounds__(kProbeBlock) void k_bw_probe(const p4f* __restrict__ a,
                                                          const p4f* __restrict__ b,
                                                          p4f* __restrict__ o, int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock * kProbeUnroll;
    for (int64_t base = (int64_t)blockIdx.x * kProbeBlock * kProbeUnroll + threadIdx.x; base < n4;
         base += stride) {
        p4f v[kProbeUnroll];
#pragma unroll
        for (int j = 0; j < kProbeUnroll; ++j) {
            const int64_t i = base + (int64_t)j * kProbeBlock;
            if (i < n4) {
                v[j] = probe_ld<NT>(a + i);
                if constexpr (ADD) v[j] += probe_ld<NT>(b + i);
            }
        }
#pragma unroll
        for (int j = 0; j < kProbeUnroll; ++j) {
            const int64_t i = base + (int64_t)j * kProbeBlock;
            if (i < n4) {
                if constexpr (NT) __builtin_nontemporal_store(v[j], o + i);
                else o[i] = v[j];
            }
        }
    }
}

}  // namespace

hipError_t launch_bw_probe(bool add, bool nt, const float* a, const float* b, float* o,
                           int64_t n, hipStream_t st) {
    const int64_t n4 = n / 4;
    if (n4 <= 0) return hipSuccess;
    const int64_t per_block = (int64_t)kProbeBlock * kProbeUnroll;
    int64_t blocks = (n4 + per_block - 1) / per_block;
    if (blocks > (int64_t)1 << 20) blocks = (int64_t)1 << 20;
    const p4f* pa = reinterpret_cast<const p4f*>(a);
    const p4f* pb = reinterpret_cast<const p4f*>(b);
    p4f* po = reinterpret_cast<p4f*>(o);
    const dim3 g((unsigned)blocks), t(kProbeBlock);
    if (add) {
        if (nt) hipLaunchKernelGGL((k_bw_probe<true, true>), g, t, 0, st, pa, pb, po, n4);
        else hipLaunchKernelGGL((k_bw_probe<true, false>), g, t, 0, st, pa, pb, po, n4);
    } else {
        if (nt) hipLaunchKernelGGL((k_bw_probe<false, true>), g, t, 0, st, pa, pb, po, n4);
        else hipLaunchKernelGGL((k_bw_probe<false, false>), g, t, 0, st, pa, pb, po, n4);
    }
    return hipGetLastError();
}

}  // namespace wmc
