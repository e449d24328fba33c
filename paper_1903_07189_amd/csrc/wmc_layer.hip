// wmc_layer.hip -- the learnable half-window layer of Sec. 4.3 for gfx950.
//
// Forward: K learned 3x3 kernels w_k (K <= 16) correlated with the
// replicate-padded input, then the minimum-magnitude activation of eq. (act):
//   d_k(x) = sum_o w_k[o] Ub(x + o),  m(x) = first k with min |d_k(x)|,
//   out(x) = d_m(x).
// With the eight printed kernels this is the Half Laplace Operator (times 12
// for the integer kernel table).
//
// Backward, with the selection held fixed (the layer is linear in U and in w
// for a fixed m):
//   gU(z)   = sum_{x, o: clamp(x + o) = z} w_{m(x)}[o] g(x)
//   gW_k[o] = sum_{x: m(x) = k} g(x) Ub(x + o).
//
// Both kernels stream rows with one wave per work item (a strip of 64
// columns, one column per lane, and a segment of R rows); horizontal
// neighbours come from the adjacent lanes by DPP.  Loads use clamped row and
// column indices, so the lanes and rows beyond the image carry the replicate
// border.  The backward's strips have a two-column halo on each side; the
// first and last hold the virtual columns -1 and W, where the scatter of the
// border pixels lands, and fold them (and the virtual rows -1 and H) back
// onto the border.  gW: every lane accumulates its own products in a private
// slice of LDS indexed by (kernel, tap); a fixed-order reduction over lanes,
// then over work items, makes the result bitwise reproducible.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

#include <algorithm>

namespace wmc {

constexpr int kLayerMaxK = 16;

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
struct LayerFwdArgs {
    const float* u;
    const float* w;  // K x 3 x 3
    float* out;
    uint8_t* sel;    // may be null
    int64_t n, h, w_, ld, ps;
    int32_t K, R, nstrip, nseg;
};

constexpr int kFwdC = 2;                           // columns per lane
constexpr int kFwdHalo = kFwdC;                    // one column, rounded up to whole lanes
constexpr int kFwdStep = 64 * kFwdC - 2 * kFwdHalo;

// KT > 0: exactly KT kernels, weights held in scalar registers for the whole
// work item.  KT == 0: any K <= 16, weights read from an LDS copy.
template <int KT>
__global__ __launch_bounds__(256) void k_layer_fwd(LayerFwdArgs A) {
    constexpr int C = kFwdC;
    __shared__ float wl[KT == 0 ? 9 * kLayerMaxK : 1];
    if constexpr (KT == 0) {
        for (int i = threadIdx.x; i < 9 * A.K; i += 256) wl[i] = A.w[i];
        __syncthreads();
    }
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
    const int H = (int)A.h, W = (int)A.w_;
    const int xb = strip * kFwdStep - kFwdHalo + C * lane;
    const int ox0 = strip * kFwdStep;
    const int ox1 = ox0 + kFwdStep < W ? ox0 + kFwdStep : W;
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
    uint8_t* sel = A.sel ? A.sel + (int64_t)p * A.ps : nullptr;

    float wr[KT > 0 ? 9 * KT : 1];
    if constexpr (KT > 0) {
#pragma unroll
        for (int i = 0; i < 9 * KT; ++i) wr[i] = A.w[i];
    }

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
        fetch(pre[1], y + 3);
        float best[C];
        int bi[C];
        auto kernel = [&](int k, const float* wk) {
#pragma unroll
            for (int e = 0; e < C; ++e) {
                float d = wk[0] * v[0][e];
#pragma unroll
                for (int t = 1; t < 9; ++t) d = __builtin_fmaf(wk[t], v[t / 3][e + t % 3], d);
                if (k == 0 || __builtin_fabsf(d) < __builtin_fabsf(best[e])) {
                    best[e] = d;
                    bi[e] = k;
                }
            }
        };
        if constexpr (KT > 0) {
#pragma unroll
            for (int k = 0; k < KT; ++k) kernel(k, wr + 9 * k);
        } else {
            for (int k = 0; k < A.K; ++k) {
                float wk[9];
#pragma unroll
                for (int t = 0; t < 9; ++t) wk[t] = wl[9 * k + t];
                kernel(k, wk);
            }
        }
        float* op = out + (int64_t)y * A.ld;
#pragma unroll
        for (int e = 0; e < C; ++e)
            if (own[e]) {
                op[xb + e] = best[e];
                if (sel) sel[(int64_t)y * A.ld + xb + e] = (uint8_t)bi[e];
            }
#pragma unroll
        for (int j = 0; j < C + 2; ++j) {
            v[0][j] = v[1][j];
            v[1][j] = v[2][j];
        }
    }
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
struct LayerBwdArgs {
    const float* u;
    const float* w;
    const uint8_t* sel;
    const float* g;
    float* g_u;      // may be null
    float* part;     // per work item and chunk: KC*9 partial sums of gW, or null
    int64_t n, h, w_, ld, ps;
    int32_t K, R, nstrip, nseg;
    int32_t nchunk;  // ceil(K / KC) groups of kernels for gW
};

constexpr int kBwdHalo = 2;
constexpr int kBwdStep = 64 - 2 * kBwdHalo;
constexpr int kBwdChunk = 8;  // kernels whose gW one wave accumulates in registers

// Waves [0, items) of chunk c = wave / items accumulate gW for kernels
// [c*KC, c*KC + KC); the waves of chunk 0 also write g_u.
template <int KC>
__global__ __launch_bounds__(256) void k_layer_bwd(LayerBwdArgs A) {
    __shared__ float wt[9 * kLayerMaxK];
    const int K = A.K;
    for (int i = threadIdx.x; i < 9 * K; i += 256) wt[i] = A.w[i];
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t per_plane = (int64_t)A.nseg * A.nstrip;
    const int64_t items = A.n * per_plane;
    const int64_t wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
    if (wave >= items * A.nchunk) return;
    const int chunk = (int)(wave / items);
    const int64_t item = wave - (int64_t)chunk * items;
    const int kbase = chunk * KC;
    const bool do_gu = chunk == 0 && A.g_u != nullptr;
    const bool do_gw = A.part != nullptr;

    const int p = (int)(item / per_plane);
    const int rem = (int)(item - (int64_t)p * per_plane);
    const int seg = rem / A.nstrip;
    const int strip = rem - seg * A.nstrip;
    const int H = (int)A.h, W = (int)A.w_;
    const int x = strip * kBwdStep - kBwdHalo + lane;
    const int ox0 = strip * kBwdStep;
    const int ox1 = ox0 + kBwdStep < W ? ox0 + kBwdStep : W;
    const bool own = x >= ox0 && x < ox1;
    const bool inimg = x >= 0 && x < W;
    const bool isL = x == 0, isR = x == W - 1;
    const bool edge = (strip * kBwdStep - kBwdHalo) < 0 || (strip * kBwdStep - kBwdHalo + 64) > W;
    const uint32_t xc = (uint32_t)(x < 0 ? 0 : (x < W ? x : W - 1));
    const int y0 = seg * A.R;
    const int y1 = y0 + A.R < H ? y0 + A.R : H;
    const int64_t off = (int64_t)p * A.ps;
    const float* u = A.u + off;
    const float* g = A.g + off;
    const uint8_t* sel = A.sel + off;
    float* gu = do_gu ? A.g_u + off : nullptr;

    float acc[KC][9];
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int t = 0; t < 9; ++t) acc[k][t] = 0.0f;

    // window rows rho-1, rho, rho+1: U with neighbours (replicate), g and m
    // with neighbours (g = 0 outside the image)
    float uv[3][3], gv[3][3];
    int mv[3][3];
    struct Pre {
        float u, g;
        int m;
    } pre[2];
    auto fetch = [&](int r) {
        Pre q;
        const int rr = r < 0 ? 0 : (r < H ? r : H - 1);
        q.u = ld_at<float>(u + (int64_t)rr * A.ld, xc);
        const bool in = inimg && r >= 0 && r < H;
        q.g = in ? ld_at<float>(g + (int64_t)rr * A.ld, xc) : 0.0f;
        q.m = in ? (int)sel[(int64_t)rr * A.ld + xc] : 0;
        if (q.m >= K) q.m = K - 1;  // defensive: never index past the table
        return q;
    };
    auto put = [&](int j, const Pre& q) {
        uv[j][0] = from_lower_lane(q.u, q.u);
        uv[j][1] = q.u;
        uv[j][2] = from_upper_lane(q.u, q.u);
        gv[j][0] = from_lower_lane(0.0f, q.g);
        gv[j][1] = q.g;
        gv[j][2] = from_upper_lane(0.0f, q.g);
        mv[j][0] = __builtin_amdgcn_update_dpp(0, q.m, 0x138, 0xF, 0xF, false);
        mv[j][1] = q.m;
        mv[j][2] = __builtin_amdgcn_update_dpp(0, q.m, 0x130, 0xF, 0xF, false);
    };
    put(0, fetch(y0 - 2));
    put(1, fetch(y0 - 1));
    pre[0] = fetch(y0);
    pre[1] = fetch(y0 + 1);
    float topfold = 0.0f, pend = 0.0f;
    // rows rho = y0-1 .. y1 (the virtual rows -1 and H only at the image border)
    for (int rho = y0 - 1; rho <= y1; ++rho) {
        // window rows 0, 1 hold rho-1, rho; row rho+1 comes from the prefetch
        put(2, pre[0]);
        pre[0] = pre[1];
        pre[1] = fetch(rho + 3);

        const bool owned_row = rho >= y0 && rho < y1;
        const bool top = rho == -1 && y0 == 0;
        const bool bot = rho == H && y1 == H;
        if (do_gu && (owned_row || top || bot)) {
            // g_u at (rho, x): neighbour (dy, dx) contributes w_m[(1-dy, 1-dx)] g
            float a = 0.0f;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    a = __builtin_fmaf(wt[mv[i][j] * 9 + (2 - i) * 3 + (2 - j)], gv[i][j], a);
            if (edge) {
                // column ring: virtual column -1 onto 0, W onto W-1
                const float l = from_lower_lane(0.0f, a);
                const float r = from_upper_lane(0.0f, a);
                a += (isL ? l : 0.0f) + (isR ? r : 0.0f);
            }
            if (top) {
                topfold = a;
            } else if (bot) {
                if (own) gu[(int64_t)(H - 1) * A.ld + x] = a + pend;
            } else {
                if (rho == 0) a += topfold;
                if (rho == H - 1) pend = a;
                else if (own) gu[(int64_t)rho * A.ld + x] = a;
            }
        }
        if (do_gw && owned_row) {
            const float gc = own ? gv[1][1] : 0.0f;
            const int m = mv[1][1] - kbase;
#pragma unroll
            for (int k = 0; k < KC; ++k) {
                const float gk = (m == k) ? gc : 0.0f;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc[k][t] = __builtin_fmaf(gk, uv[t / 3][t % 3], acc[k][t]);
            }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            uv[0][j] = uv[1][j]; uv[1][j] = uv[2][j];
            gv[0][j] = gv[1][j]; gv[1][j] = gv[2][j];
            mv[0][j] = mv[1][j]; mv[1][j] = mv[2][j];
        }
    }
    if (do_gw) {
        // fixed-order butterfly over the lanes of each (kernel, tap)
        float* dst = A.part + wave * (int64_t)(9 * KC);
#pragma unroll
        for (int k = 0; k < KC; ++k)
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                float s = acc[k][t];
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
                if (lane == 0) dst[k * 9 + t] = s;
            }
    }
}

// gW[k][t] = sum over work items of the partial of chunk k / KC, in item order.
__global__ __launch_bounds__(256) void k_layer_wreduce(const float* __restrict__ part,
                                                       int64_t items, int KC, int K,
                                                       float* __restrict__ gw) {
    const int e = blockIdx.x;  // k * 9 + t
    const int k = e / 9, t = e - 9 * (e / 9);
    const int chunk = k / KC, kl = k - chunk * KC;
    const float* base = part + (int64_t)chunk * items * (9 * KC) + kl * 9 + t;
    __shared__ float red[256];
    // each thread adds items threadIdx.x, +256, +512, ... in that order; the
    // loads of eight of them are issued before the adds
    const int64_t stride = 9 * KC;
    float s = 0.0f;
    int64_t i = threadIdx.x;
    for (; i + 7 * 256 < items; i += 8 * 256) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = base[(i + j * 256) * stride];
#pragma unroll
        for (int j = 0; j < 8; ++j) s += v[j];
    }
    for (; i < items; i += 256) s += base[i * stride];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && k < K) gw[e] = red[0];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int layer_chunk(int K) { return K < kBwdChunk ? K : kBwdChunk; }

using LayerFwdFn = void (*)(LayerFwdArgs);
using LayerBwdFn = void (*)(LayerBwdArgs);

static LayerFwdFn fwd_fn(int K) {
    static const LayerFwdFn tab[9] = {k_layer_fwd<0>, k_layer_fwd<1>, k_layer_fwd<2>,
                                      k_layer_fwd<3>, k_layer_fwd<4>, k_layer_fwd<5>,
                                      k_layer_fwd<6>, k_layer_fwd<7>, k_layer_fwd<8>};
    return tab[K <= 8 ? K : 0];
}

static LayerBwdFn bwd_fn(int KC) {
    static const LayerBwdFn tab[9] = {nullptr, k_layer_bwd<1>, k_layer_bwd<2>, k_layer_bwd<3>,
                                      k_layer_bwd<4>, k_layer_bwd<5>, k_layer_bwd<6>,
                                      k_layer_bwd<7>, k_layer_bwd<8>};
    return tab[KC];
}

// Row counts that fill whole rounds of resident waves (the backward's item
// count is also the size of its partial-sum buffer, so it depends only on
// the shape and K, never on pointers).
int layer_fwd_items(int64_t n, int64_t h, int64_t w, int K, int* R, int* nstrip, int* nseg) {
    *nstrip = (int)((w + kFwdStep - 1) / kFwdStep);
    const int64_t slots = kernel_slots(reinterpret_cast<const void*>(fwd_fn(K)), 256, 0);
    *R = fill_rows(n * (int64_t)(*nstrip), h, slots, 8, 256);
    *nseg = seg_count((int)h, *R);
    return (int)std::min<int64_t>(n * (int64_t)(*nstrip) * (*nseg), 0x7fffffff);
}

int64_t layer_bwd_items(int64_t n, int64_t h, int64_t w, int K, int* R, int* nstrip, int* nseg) {
    *nstrip = (int)((w + kBwdStep - 1) / kBwdStep);
    const int KC = layer_chunk(K);
    const int nchunk = (K + KC - 1) / KC;
    const int64_t slots = kernel_slots(reinterpret_cast<const void*>(bwd_fn(KC)), 256, 0);
    *R = fill_rows(n * (int64_t)(*nstrip) * nchunk, h, slots, 8, 256);
    *nseg = seg_count((int)h, *R);
    return n * (int64_t)(*nstrip) * (*nseg);
}

int64_t layer_part_floats(int64_t n, int64_t h, int64_t w, int K) {
    int R, ns, nsg;
    const int64_t items = layer_bwd_items(n, h, w, K, &R, &ns, &nsg);
    const int KC = layer_chunk(K);
    return items * ((K + KC - 1) / KC) * 9 * KC;
}

hipError_t launch_layer_forward(const float* u, const float* w, int K, float* out, uint8_t* sel,
                                int64_t n, int64_t h, int64_t wd, int64_t ld, int64_t ps,
                                hipStream_t st) {
    if (K < 1 || K > kLayerMaxK) return hipErrorInvalidValue;
    LayerFwdArgs a{};
    a.u = u;
    a.w = w;
    a.out = out;
    a.sel = sel;
    a.n = n;
    a.h = h;
    a.w_ = wd;
    a.ld = ld;
    a.ps = ps;
    a.K = K;
    int R, ns, nsg;
    layer_fwd_items(n, h, wd, K, &R, &ns, &nsg);
    a.R = R;
    a.nstrip = ns;
    a.nseg = nsg;
    const LayerFwdFn fn = fwd_fn(K);
    const int64_t total = n * (int64_t)ns * nsg;
    hipLaunchKernelGGL(fn, dim3((unsigned)((total + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_layer_backward(const float* u, const float* w, int K, const uint8_t* sel,
                                 const float* g, float* g_u, float* part, float* g_w, int64_t n,
                                 int64_t h, int64_t wd, int64_t ld, int64_t ps, hipStream_t st) {
    if (K < 1 || K > kLayerMaxK) return hipErrorInvalidValue;
    LayerBwdArgs a{};
    a.u = u;
    a.w = w;
    a.sel = sel;
    a.g = g;
    a.g_u = g_u;
    a.part = g_w ? part : nullptr;
    a.n = n;
    a.h = h;
    a.w_ = wd;
    a.ld = ld;
    a.ps = ps;
    a.K = K;
    int R, ns, nsg;
    const int64_t items = layer_bwd_items(n, h, wd, K, &R, &ns, &nsg);
    a.R = R;
    a.nstrip = ns;
    a.nseg = nsg;
    const int KC = layer_chunk(K);
    a.nchunk = g_w ? (K + KC - 1) / KC : 1;
    const int64_t waves = items * a.nchunk;
    hipLaunchKernelGGL(bwd_fn(KC), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g_w) return e;
    hipLaunchKernelGGL(k_layer_wreduce, dim3((unsigned)(9 * K)), dim3(256), 0, st, part, items,
                       KC, K, g_w);
    return hipGetLastError();
}

}  // namespace wmc
