// wmc_3d.hip -- the half-window operator on 3-D volumes, for gfx950.
//
// The conclusion of the paper mentions the extension to 3-D images without
// giving kernels; they are built here the way Sec. 4.1 builds the 2-D ones.
// The base kernel is the tensor-product isotropic Laplacian
// K = (s (x) s (x) s - 64 delta) / 56, s = [1 2 1] (the 3-D analogue of
// k4 = (s (x) s - 16 delta) / 12).  The half windows are K reflected across
// each of the 9 mirror planes of the 3x3x3 window: normals e_x, e_y, e_z and
// e_x +- e_y, e_x +- e_z, e_y +- e_z.  Each plane gives two candidates (keep
// the side n.o <= 0, or the side n.o >= 0), 18 in all, in the order plane
// 0..8 with the "-" side first; exact magnitude ties go to the first.
//
// With c = s (x) s (x) s off the centre (1 corner, 2 edge, 4 face), every
// candidate is S = A -+ D_j (x56 domain):
//   A   = sum_o c[o] U(x + o) - 64 U(x)          (difference form, sum c = 56)
//   D_j = sum_o sign(n_j . o) c[o] U(x + o)       (odd part of plane j)
// since the two sides of a plane add up to 2K.  H = S_m / 56.
//
// Kernel: one wave per work item -- a strip of 62 owned x-columns (one halo
// lane each side, clamped loads: the replicate border), one y row, a
// segment of R z-planes -- streaming along z.  At each step the wave loads
// rows y-1, y, y+1 of the next plane, forms per-plane sums over the 3x3
// (y, x) patch with DPP neighbours, and adds them into the pending
// accumulators of the three voxels whose window contains that plane (as
// their dz = +1, 0, -1 plane).  The voxel whose window is complete is then
// finalised: candidates, selection, update, store.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

constexpr int k3Halo = 1;
constexpr int k3Step = 64 - 2 * k3Halo;

// Per-plane sums of one (x, y) column over the plane's 3x3 patch, weights
// s[dy] s[dx]: the full sum, the odd parts along x, y and the two xy
// diagonals, and the half sums needed by the x+-z, y+-z planes.
struct PlaneSums {
    float sum, ex, ey, exy, exmy, xge, xle, yge, yle, c;
};

// Accumulated parts of one voxel.
struct Acc {
    float A, dx, dy, dz, dxy, dxmy, dxz, dxmz, dyz, dymz, c, f;
};

__device__ __forceinline__ void acc_zero(Acc& a) {
    a.A = a.dx = a.dy = a.dz = a.dxy = a.dxmy = a.dxz = a.dxmz = a.dyz = a.dymz = 0.0f;
    a.c = a.f = 0.0f;
}

// rows t (y-1), m (y), b (y+1) of one plane: the lane's value and its x
// neighbours from the adjacent lanes.
__device__ __forceinline__ PlaneSums plane_sums(float t, float m, float b) {
    float l[3], r[3], v[3] = {t, m, b};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        l[i] = from_lower_lane(v[i], v[i]);
        r[i] = from_upper_lane(v[i], v[i]);
    }
    float a[3], s[3], q[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        a[i] = __builtin_fmaf(2.0f, v[i], l[i]);  // l + 2m
        s[i] = a[i] + r[i];                       // l + 2m + r
        q[i] = l[i] - r[i];
    }
    PlaneSums p;
    p.sum = __builtin_fmaf(2.0f, s[1], s[0] + s[2]);
    p.ex = -__builtin_fmaf(2.0f, q[1], q[0] + q[2]);
    p.ey = s[2] - s[0];
    const float sbl = s[2] - l[2], stl = s[0] - l[0];  // 2m + r of rows b, t
    p.exy = __builtin_fmaf(-2.0f, q[1], sbl - a[0]);
    p.exmy = __builtin_fmaf(-2.0f, q[1], stl - a[2]);
    p.xge = __builtin_fmaf(2.0f, s[1] - l[1], stl + sbl);
    p.xle = __builtin_fmaf(2.0f, a[1], a[0] + a[2]);
    p.yge = __builtin_fmaf(2.0f, s[1], s[2]);
    p.yle = __builtin_fmaf(2.0f, s[1], s[0]);
    p.c = m;
    return p;
}

// plane p as the dz = +1 plane of voxel p-1
__device__ __forceinline__ void add_up(Acc& a, const PlaneSums& p) {
    a.A += p.sum;
    a.dx += p.ex;
    a.dy += p.ey;
    a.dz += p.sum;
    a.dxy += p.exy;
    a.dxmy += p.exmy;
    a.dxz += p.xge;
    a.dxmz -= p.xle;
    a.dyz += p.yge;
    a.dymz -= p.yle;
}

// plane p as the centre plane of voxel p
__device__ __forceinline__ void add_mid(Acc& a, const PlaneSums& p) {
    a.A = __builtin_fmaf(2.0f, p.sum, a.A);
    a.dx = __builtin_fmaf(2.0f, p.ex, a.dx);
    a.dy = __builtin_fmaf(2.0f, p.ey, a.dy);
    a.dxy = __builtin_fmaf(2.0f, p.exy, a.dxy);
    a.dxmy = __builtin_fmaf(2.0f, p.exmy, a.dxmy);
    a.dxz = __builtin_fmaf(2.0f, p.ex, a.dxz);
    a.dxmz = __builtin_fmaf(2.0f, p.ex, a.dxmz);
    a.dyz = __builtin_fmaf(2.0f, p.ey, a.dyz);
    a.dymz = __builtin_fmaf(2.0f, p.ey, a.dymz);
    a.c = p.c;
}

// plane p as the dz = -1 plane of voxel p+1 (starts its accumulators)
__device__ __forceinline__ void start_down(Acc& a, const PlaneSums& p) {
    a.A = p.sum;
    a.dx = p.ex;
    a.dy = p.ey;
    a.dz = -p.sum;
    a.dxy = p.exy;
    a.dxmy = p.exmy;
    a.dxz = -p.xle;
    a.dxmz = p.xge;
    a.dyz = -p.yle;
    a.dymz = p.yge;
}

__device__ __forceinline__ float pick3(float best, float s) {
    return (__builtin_fabsf(s) < __builtin_fabsf(best)) ? s : best;
}

// Selected S (x56 domain): first of the 18 candidates with the least |S|.
__device__ __forceinline__ float select18(const Acc& a) {
    const float A = __builtin_fmaf(-64.0f, a.c, a.A);
    const float D[9] = {a.dx, a.dy, a.dz, a.dxy, a.dxmy, a.dxz, a.dxmz, a.dyz, a.dymz};
    float best = A - D[0];
    best = pick3(best, A + D[0]);
#pragma unroll
    for (int j = 1; j < 9; ++j) {
        best = pick3(best, A - D[j]);
        best = pick3(best, A + D[j]);
    }
    return best;
}

struct Vol3Args {
    const float* u;
    const float* f;  // data term or null
    float* out;
    const float* lam;
    float dt;
    int mode;        // kModeCompute / kModeData / kModeFlow
    int64_t n, d, h, w, ld, ss, vs;
    int32_t R, nstrip, nseg;
};

template <int P>
struct Phase3 {
    static constexpr int value = P;
};

__global__ __launch_bounds__(256) void k_stream3d(Vol3Args A) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t per_vol = (int64_t)A.nseg * A.h * A.nstrip;
    const int64_t total = A.n * per_vol;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
    if (item >= total) return;
    const int v = (int)(item / per_vol);
    int64_t rem = item - (int64_t)v * per_vol;
    const int seg = (int)(rem / ((int64_t)A.h * A.nstrip));
    rem -= (int64_t)seg * A.h * A.nstrip;
    const int y = (int)(rem / A.nstrip);
    const int strip = (int)(rem - (int64_t)y * A.nstrip);
    const int D = (int)A.d, H = (int)A.h, W = (int)A.w;
    const int x = strip * k3Step - k3Halo + lane;
    const int ox1 = strip * k3Step + k3Step < W ? strip * k3Step + k3Step : W;
    const bool own = x >= strip * k3Step && x < ox1;
    const uint32_t xc = (uint32_t)(x < 0 ? 0 : (x < W ? x : W - 1));
    const int z0 = seg * A.R;
    const int z1 = z0 + A.R < D ? z0 + A.R : D;
    const int64_t voff = (int64_t)v * A.vs;
    const float* u = A.u + voff;
    const float* f = A.f ? A.f + voff : nullptr;
    float* out = A.out + voff;
    const int64_t ym = (int64_t)(y > 0 ? y - 1 : 0) * A.ld;
    const int64_t y0 = (int64_t)y * A.ld;
    const int64_t yp = (int64_t)(y + 1 < H ? y + 1 : H - 1) * A.ld;
    const bool data = A.mode == kModeData;
    const float lam = (data && A.lam) ? A.lam[v] : 0.0f;
    const Coef cf = make_coef(lam, A.dt, data);
    const float lam56 = lam / 56.0f, delta56 = cf.delta / 56.0f;

    struct Rows {
        float t, m, b, f;
    };
    auto fetch = [&](int p) {
        Rows r;
        const int pc = p < 0 ? 0 : (p < D ? p : D - 1);
        const float* pl = u + (int64_t)pc * A.ss;
        r.t = ld_at<float>(pl + ym, xc);
        r.m = ld_at<float>(pl + y0, xc);
        r.b = ld_at<float>(pl + yp, xc);
        r.f = (data && p >= z0 && p < z1) ? ld_at<float>(f + (int64_t)pc * A.ss + y0, xc) : 0.0f;
        return r;
    };

    Acc acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc_zero(acc[i]);
    Rows pre[2];
    // planes p = z0-1 .. z1 (clamped: the replicate border); voxel z is
    // finished when plane z+1 has been added
    int p = z0 - 1;
    pre[0] = fetch(p);
    pre[1] = fetch(p + 1);

    auto step = [&](auto tag) {
        constexpr int Q = decltype(tag)::value;  // slot of voxel p
        constexpr int QM = (Q + 2) % 3;           // voxel p-1
        constexpr int QP = (Q + 1) % 3;           // voxel p+1
        const Rows r = pre[0];
        pre[0] = pre[1];
        pre[1] = fetch(p + 2);
        const PlaneSums ps = plane_sums(r.t, r.m, r.b);
        add_up(acc[QM], ps);
        add_mid(acc[Q], ps);
        acc[Q].f = r.f;
        start_down(acc[QP], ps);
        const int zf = p - 1;  // voxel whose window is now complete
        if (zf >= z0 && zf < z1) {
            const float S = select18(acc[QM]);
            float o;
            if (A.mode == kModeCompute) o = S * (1.0f / 56.0f);
            else if (data) o = __builtin_fmaf(cf.delta, __builtin_fmaf(lam56, S, acc[QM].f - acc[QM].c),
                                              acc[QM].c);
            else o = __builtin_fmaf(delta56, S, acc[QM].c);
            if (own) out[(int64_t)zf * A.ss + y0 + x] = o;
        }
    };
    while (true) {
        step(Phase3<0>{});
        if (++p > z1) break;
        step(Phase3<1>{});
        if (++p > z1) break;
        step(Phase3<2>{});
        if (++p > z1) break;
    }
}

// ~16K work items, 8..128 planes per item.  (Round-filling row counts, which
// help the 2-D kernels, measured slower here: this kernel hides latency
// better with more, shorter items.)
static int vol_rows(int64_t n, int64_t d, int64_t h, int64_t strips) {
    const int64_t cols = n * h * strips;
    int R = 8;
    while (R < 128 && cols * ((d + R - 1) / R) > 16384) R *= 2;
    return R;
}

hipError_t launch_stream3d(const float* u, const float* f, float* out, const float* lam, float dt,
                           int mode, int64_t n, int64_t d, int64_t h, int64_t w, int64_t ld,
                           int64_t ss, int64_t vs, hipStream_t st) {
    Vol3Args a{};
    a.u = u;
    a.f = f;
    a.out = out;
    a.lam = lam;
    a.dt = dt;
    a.mode = mode;
    a.n = n;
    a.d = d;
    a.h = h;
    a.w = w;
    a.ld = ld;
    a.ss = ss;
    a.vs = vs;
    a.nstrip = (int)((w + k3Step - 1) / k3Step);
    a.R = vol_rows(n, d, h, a.nstrip);
    a.nseg = (int)((d + a.R - 1) / a.R);
    const int64_t total = n * (int64_t)a.nseg * h * a.nstrip;
    hipLaunchKernelGGL(k_stream3d, dim3((unsigned)((total + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace wmc
