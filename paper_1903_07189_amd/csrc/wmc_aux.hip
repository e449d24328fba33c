// wmc_aux.hip -- kernels around the hot path: the conventional finite-
// difference WMC used as the paper's comparator (Sec. 5.4), and the learnable
// half-window layer of Sec. 4.3 (K learned 3x3 kernels + minimum-magnitude
// activation) with its backward pass.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

constexpr int kAX = 64, kAY = 4;

__device__ __forceinline__ int clamp_i(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// H^w of eq. (rhs) by second-order central differences (unit spacing,
// replicate border), guard eps in the denominator.  out = H^w, or
// u + dt H^w when `flow` (one explicit curvature-flow step).
__global__ __launch_bounds__(kAX* kAY) void k_fd(const float* __restrict__ u, float* __restrict__ out,
                                                int64_t ld, int64_t ps, int H, int W, float dt,
                                                float eps, int flow) {
    const int x = blockIdx.x * kAX + threadIdx.x;
    const int y = blockIdx.y * kAY + threadIdx.y;
    if (x >= W || y >= H) return;
    const float* p = u + (int64_t)blockIdx.z * ps;
    const int xm = clamp_i(x - 1, 0, W - 1), xp = clamp_i(x + 1, 0, W - 1);
    const int64_t rm = (int64_t)clamp_i(y - 1, 0, H - 1) * ld, r0 = (int64_t)y * ld,
                  rp = (int64_t)clamp_i(y + 1, 0, H - 1) * ld;
    const float c = p[r0 + x];
    const float e = p[r0 + xp], w = p[r0 + xm], s = p[rp + x], n = p[rm + x];
    const float se = p[rp + xp], ne = p[rm + xp], sw = p[rp + xm], nw = p[rm + xm];
    const float ux = 0.5f * (e - w), uy = 0.5f * (s - n);
    const float uxx = (e - 2.0f * c) + w, uyy = (s - 2.0f * c) + n;
    const float uxy = 0.25f * (((se - ne) - sw) + nw);
    const float num = (uy * uy * uyy + 2.0f * ux * uy * uxy) + ux * ux * uxx;
    const float hw = (uxx + uyy) - num / ((ux * ux + uy * uy) + eps);
    out[(int64_t)blockIdx.z * ps + r0 + x] = flow ? __builtin_fmaf(dt, hw, c) : hw;
}

int64_t kernel_slots(const void* fn, int block, size_t dyn_lds) {
    int dev = 0, ncu = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 1024;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 1024;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, dyn_lds) != hipSuccess || nb < 1)
        nb = 1;
    return (int64_t)ncu * nb * (block / 64);
}

hipError_t launch_fd(const float* u, float* out, int64_t n, int64_t h, int64_t w, int64_t ld,
                     int64_t ps, float dt, float eps, bool flow, hipStream_t st) {
    const dim3 grid((unsigned)((w + kAX - 1) / kAX), (unsigned)((h + kAY - 1) / kAY), (unsigned)n);
    hipLaunchKernelGGL(k_fd, grid, dim3(kAX, kAY), 0, st, u, out, ld, ps, (int)h, (int)w, dt, eps,
                       flow ? 1 : 0);
    return hipGetLastError();
}

}  // namespace wmc
