// wmc_aux.hip -- the conventional finite-difference WMC used as the paper's
// comparator (Sec. 5.4), and host helpers shared by the launchers.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

struct FdArgs {
    const float* u;
    float* out;
    int64_t n, h, w, ld, ps;
    float dt, eps;
    int32_t flow;  // 1: out = u + dt H^w (one explicit flow step); 0: out = H^w
    int32_t R, nstrip, nseg;
};

constexpr int kFdC = 2;                        // columns per lane
constexpr int kFdHalo = kFdC;                  // one column, rounded up to a whole lane
constexpr int kFdStep = 64 * kFdC - 2 * kFdHalo;

// H^w of eq. (rhs) by second-order central differences (unit spacing,
// replicate border), guard eps in the denominator.  One wave per work item
// (a strip of 124 owned columns, two per lane, with a halo lane on each side,
// and a segment of R rows) streaming down the rows: each row is loaded once,
// with clamped row and column indices (the replicate border), and the
// horizontal neighbours come from the adjacent lanes by DPP.
__global__ __launch_bounds__(256) void k_fd(FdArgs A) {
    constexpr int C = kFdC;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t per_plane = (int64_t)A.nseg * A.nstrip;
    const int64_t total = A.n * per_plane;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
    if (item >= total) return;
    const int p = (int)(item / per_plane);
    const int rem = (int)(item - (int64_t)p * per_plane);
    const int seg = rem / A.nstrip;
    const int strip = rem - seg * A.nstrip;
    const int H = (int)A.h, W = (int)A.w;
    const int xb = strip * kFdStep - kFdHalo + C * lane;
    const int ox0 = strip * kFdStep;
    const int ox1 = ox0 + kFdStep < W ? ox0 + kFdStep : W;
    bool own[C];
    uint32_t xc[C];
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const int x = xb + e;
        own[e] = x >= ox0 && x < ox1;
        xc[e] = (uint32_t)(x < 0 ? 0 : (x < W ? x : W - 1));
    }
    const int y0 = seg * A.R;
    const int y1 = y0 + A.R < H ? y0 + A.R : H;
    const float* u = A.u + (int64_t)p * A.ps;
    float* out = A.out + (int64_t)p * A.ps;

    // rows y-1, y, y+1: the lane's C columns with one neighbour on each side
    float v[3][C + 2];
    float pre[2][C];
    auto fetch = [&](float (&d)[C], int r) {
        const int rr = r < 0 ? 0 : (r < H ? r : H - 1);
        const float* rp = u + (int64_t)rr * A.ld;
#pragma unroll
        for (int e = 0; e < C; ++e) d[e] = ld_at<float>(rp, xc[e]);
    };
    auto put = [&](float (&d)[C + 2], const float (&c)[C]) {
        d[0] = from_lower_lane(c[0], c[C - 1]);
#pragma unroll
        for (int e = 0; e < C; ++e) d[e + 1] = c[e];
        d[C + 1] = from_upper_lane(c[C - 1], c[0]);
    };
    {
        float t[C];
        fetch(t, y0 - 1);
        put(v[0], t);
        fetch(t, y0);
        put(v[1], t);
    }
    fetch(pre[0], y0 + 1);
    fetch(pre[1], y0 + 2);
    for (int y = y0; y < y1; ++y) {
        put(v[2], pre[0]);
#pragma unroll
        for (int e = 0; e < C; ++e) pre[0][e] = pre[1][e];
        if (y + 3 < y1 + 1) fetch(pre[1], y + 3);
        float* op = out + (int64_t)y * A.ld;
#pragma unroll
        for (int e = 0; e < C; ++e) {
            const float c = v[1][e + 1];
            const float ea = v[1][e + 2], we = v[1][e], so = v[2][e + 1], no = v[0][e + 1];
            const float se = v[2][e + 2], ne = v[0][e + 2], sw = v[2][e], nw = v[0][e];
            const float ux = 0.5f * (ea - we), uy = 0.5f * (so - no);
            const float uxx = (ea - 2.0f * c) + we, uyy = (so - 2.0f * c) + no;
            const float uxy = 0.25f * (((se - ne) - sw) + nw);
            const float num = (uy * uy * uyy + 2.0f * ux * uy * uxy) + ux * ux * uxx;
            const float hw = (uxx + uyy) - num / ((ux * ux + uy * uy) + A.eps);
            if (own[e]) op[xb + e] = A.flow ? __builtin_fmaf(A.dt, hw, c) : hw;
        }
#pragma unroll
        for (int j = 0; j < C + 2; ++j) {
            v[0][j] = v[1][j];
            v[1][j] = v[2][j];
        }
    }
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
    FdArgs A{u, out, n, h, w, ld, ps, dt, eps, flow ? 1 : 0, 0, 0, 0};
    A.nstrip = (int32_t)((w + kFdStep - 1) / kFdStep);
    const int64_t slots = kernel_slots(reinterpret_cast<const void*>(k_fd), 256, 0);
    A.R = fill_rows(n * (int64_t)A.nstrip, h, slots, 8, 256);
    A.nseg = seg_count((int)h, A.R);
    const int64_t total = n * (int64_t)A.nstrip * A.nseg;
    const int64_t blocks = (total + 3) / 4;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fd, dim3((unsigned)blocks), dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace wmc
