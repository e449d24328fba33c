// wmc_adjoint.hip -- reverse-mode derivative of one WMC update for gfx950.
//
// With the selected half window m(x) held at its forward value the update
//   U'(x) = U(x) + delta [(f(x) - U(x)) + lam/12 sum_o c_{m(x)}[o] U(clamp(x+o))]
// (c_i = 12 h_i including the centre weight -12, Sec. 4.2) is affine in U, f
// and its adjoint is a transposed, data-dependent stencil:
//   g_prev(y) = keep g(y) + coef sum_{x, o: clamp(x+o) = y} c_{m(x)}[o] g(x)
// keep = 1 - delta, coef = delta lam / 12 with a data term; keep = 1,
// coef = delta / 12 for the flow.  Two kernels:
//   k_adj_select : m(x) from U^t through the same per-pixel arithmetic as the
//                  forward kernels (so it reproduces their selection bit for
//                  bit), plus per-block partial sums of dL/dlam;
//   k_adj_gather : the transposed stencil as a gather over the 3x3
//                  neighbours, with the clamped taps of border pixels folded
//                  in, plus dL/df += delta g.
// dL/dlam per plane is reduced in a fixed order (no atomics) by
// k_lam_reduce, so gradients are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

// The eight half-window kernels of Sec. 4.2 times 12, [i][row][col], row 0
// is the image row above the pixel, col 0 the column to its left.
__constant__ int8_t kHalf12[8][3][3] = {
    {{2, 2, 0}, {4, -12, 0}, {2, 2, 0}},  // h1 left
    {{2, 4, 2}, {2, -12, 2}, {0, 0, 0}},  // h2 top
    {{0, 2, 2}, {0, -12, 4}, {0, 2, 2}},  // h3 right
    {{0, 0, 0}, {2, -12, 2}, {2, 4, 2}},  // h4 bottom
    {{2, 4, 1}, {4, -12, 0}, {1, 0, 0}},  // h5 top-left
    {{1, 4, 2}, {0, -12, 4}, {0, 0, 1}},  // h6 top-right
    {{0, 0, 1}, {0, -12, 4}, {1, 4, 2}},  // h7 bottom-right
    {{1, 0, 0}, {4, -12, 0}, {2, 4, 1}},  // h8 bottom-left
};

constexpr int kTX = 64, kTY = 4;  // pixels per block: 64 columns x 4 rows

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Row quantities of one image row at column x, with the replicate border,
// computed exactly as make_row() does from the lane-neighbour values.
__device__ __forceinline__ void row_at(const float* __restrict__ row, int x, int W, float& a,
                                       float& s, float& q, float& c) {
    const float l = row[x > 0 ? x - 1 : 0];
    const float m = row[x];
    const float r = row[x + 1 < W ? x + 1 : W - 1];
    a = __builtin_fmaf(2.0f, m, l);
    s = a + r;
    q = l - r;
    c = m;
}

__global__ __launch_bounds__(kTX* kTY) void k_adj_select(AdjArgs A) {
    const int x = blockIdx.x * kTX + threadIdx.x;
    const int y = blockIdx.y * kTY + threadIdx.y;
    const int p = blockIdx.z;
    const int H = (int)A.h, W = (int)A.w;
    const bool data = A.f != nullptr;
    float contrib = 0.0f;
    if (x < W && y < H) {
        const float* u = A.u + (int64_t)p * A.ps;
        const int64_t k = (int64_t)y * A.ld + x;
        float ta, ts, tq, tc, ma, ms, mq, mc, ba, bs, bq, bc;
        row_at(u + (int64_t)clampi(y - 1, 0, H - 1) * A.ld, x, W, ta, ts, tq, tc);
        row_at(u + (int64_t)y * A.ld, x, W, ma, ms, mq, mc);
        row_at(u + (int64_t)clampi(y + 1, 0, H - 1) * A.ld, x, W, ba, bs, bq, bc);
        int idx;
        const float S = select_x12_idx(parts(ta, ts, tq, ms, mq, mc, ba, bs, bq), idx);
        A.sel[(int64_t)p * A.ps + k] = (uint8_t)idx;
        if (data) {
            const float lam = A.lam ? A.lam[p] : 0.0f;
            const Coef cf = make_coef(lam, A.dt, true);
            const float hd = to_hd(S);
            const float g = A.g[(int64_t)p * A.ps + k];
            float dudl = cf.delta * hd;
            if (!(A.dt > 0.0f)) {
                const float fv = A.f[(int64_t)p * A.ps + k];
                dudl -= cf.delta * cf.delta * ((fv - mc) + lam * hd);
            }
            contrib = g * dudl;
        }
    }
    if (!data) return;
    // fixed-order block reduction of dL/dlam
    __shared__ float red[kTX * kTY];
    const int t = threadIdx.y * kTX + threadIdx.x;
    red[t] = contrib;
    __syncthreads();
    for (int w = kTX * kTY / 2; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) {
        const int nblk = gridDim.x * gridDim.y;
        A.lam_part[(int64_t)p * nblk + blockIdx.y * gridDim.x + blockIdx.x] = red[0];
    }
}

__global__ __launch_bounds__(kTX* kTY) void k_adj_gather(AdjArgs A) {
    const int x = blockIdx.x * kTX + threadIdx.x;
    const int y = blockIdx.y * kTY + threadIdx.y;
    const int p = blockIdx.z;
    const int H = (int)A.h, W = (int)A.w;
    if (x >= W || y >= H) return;
    const bool data = A.f != nullptr;
    const float lam = (data && A.lam) ? A.lam[p] : 0.0f;
    const Coef cf = make_coef(lam, A.dt, data);
    const float keep = data ? 1.0f - cf.delta : 1.0f;
    const float coef = data ? cf.delta * cf.lam12 : cf.delta12;
    const int64_t base = (int64_t)p * A.ps;
    const float* g = A.g + base;
    const uint8_t* sel = A.sel + base;

    // For each neighbour offset d along one axis, the bit set of kernel taps o
    // (bit o+1) of the neighbour x = y + d that land on y after clamping.
    unsigned mr[3], mc[3];
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        unsigned br = 0, bc = 0;
        const int xr = y + d, xc = x + d;
#pragma unroll
        for (int o = -1; o <= 1; ++o) {
            if (xr >= 0 && xr < H && clampi(xr + o, 0, H - 1) == y) br |= 1u << (o + 1);
            if (xc >= 0 && xc < W && clampi(xc + o, 0, W - 1) == x) bc |= 1u << (o + 1);
        }
        mr[d + 1] = br;
        mc[d + 1] = bc;
    }
    float acc = 0.0f;
#pragma unroll
    for (int dr = 0; dr < 3; ++dr) {
        if (!mr[dr]) continue;
#pragma unroll
        for (int dc = 0; dc < 3; ++dc) {
            if (!mc[dc]) continue;
            const int64_t kx = (int64_t)(y + dr - 1) * A.ld + (x + dc - 1);
            const int m = sel[kx];
            int w = 0;
#pragma unroll
            for (int orr = 0; orr < 3; ++orr) {
                if (!((mr[dr] >> orr) & 1u)) continue;
#pragma unroll
                for (int oc = 0; oc < 3; ++oc)
                    if ((mc[dc] >> oc) & 1u) w += kHalf12[m][orr][oc];
            }
            acc = __builtin_fmaf((float)w, g[kx], acc);
        }
    }
    const int64_t k = (int64_t)y * A.ld + x;
    const float gy = g[k];
    A.g_prev[base + k] = __builtin_fmaf(coef, acc, keep * gy);
    if (data && A.g_f) A.g_f[base + k] += cf.delta * gy;
}

__global__ __launch_bounds__(256) void k_lam_reduce(const float* __restrict__ part, int nblk,
                                                    float* __restrict__ g_lam) {
    const int p = blockIdx.x;
    __shared__ float red[256];
    float s = 0.0f;
    for (int i = threadIdx.x; i < nblk; i += 256) s += part[(int64_t)p * nblk + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) g_lam[p] += red[0];
}

int adj_blocks_per_plane(int64_t h, int64_t w) {
    return (int)(((w + kTX - 1) / kTX) * ((h + kTY - 1) / kTY));
}

hipError_t launch_adjoint_step(const AdjArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)((a.w + kTX - 1) / kTX), (unsigned)((a.h + kTY - 1) / kTY),
                    (unsigned)a.n);
    const dim3 block(kTX, kTY);
    hipLaunchKernelGGL(k_adj_select, grid, block, 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_gather, grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lambda_reduce(const float* lam_part, int64_t n, int nblk, float* g_lam,
                                hipStream_t st) {
    hipLaunchKernelGGL(k_lam_reduce, dim3((unsigned)n), dim3(256), 0, st, lam_part, nblk, g_lam);
    return hipGetLastError();
}

}  // namespace wmc
