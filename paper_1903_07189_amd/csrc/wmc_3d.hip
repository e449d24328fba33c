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
// Kernel: one wave per work item -- a strip of 64 x-columns (a lane each,
// clamped loads: the replicate border), one y row, a segment of R z-planes
// -- streaming along z.  At each step the wave loads rows y-1, y, y+1 of
// the next plane (and, for lanes 0 and 63, the columns just outside the
// strip), forms per-plane sums over the 3x3 (y, x) patch with DPP
// neighbours, and adds them into the pending
// accumulators of the three voxels whose window contains that plane (as
// their dz = +1, 0, -1 plane).  The voxel whose window is complete is then
// finalised: candidates, selection, update, store.
#include <hip/hip_runtime.h>

#include <cstdlib>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

// Strips of 64 columns, one per lane, no halo lanes: lanes 0 and 63 take
// their outer x neighbour from a separate load of the adjacent columns.
constexpr int k3Step = 64;

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
// neighbours from the adjacent lanes; h (rows ht, hm, hb) holds, in lane 0,
// the column left of the strip and, in lane 63, the column right of it
// (clamped: the replicate border).
__device__ __forceinline__ PlaneSums plane_sums(float t, float m, float b, float ht, float hm,
                                                float hb) {
    float l[3], r[3], v[3] = {t, m, b}, h[3] = {ht, hm, hb};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        l[i] = from_lower_lane(h[i], v[i]);
        r[i] = from_upper_lane(h[i], v[i]);
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

// The same picks as select18, also returning the 0-based index of the
// winner (2 j for S = A - D_j, 2 j + 1 for A + D_j).
__device__ __forceinline__ float select18_idx(const Acc& a, int& idx) {
    const float A = __builtin_fmaf(-64.0f, a.c, a.A);
    const float D[9] = {a.dx, a.dy, a.dz, a.dxy, a.dxmy, a.dxz, a.dxmz, a.dyz, a.dymz};
    float best = A - D[0];
    int bi = 0;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        if (j > 0) {
            const float lo = A - D[j];
            const bool b0 = __builtin_fabsf(lo) < __builtin_fabsf(best);
            best = b0 ? lo : best;
            bi = b0 ? 2 * j : bi;
        }
        const float hi = A + D[j];
        const bool b1 = __builtin_fabsf(hi) < __builtin_fabsf(best);
        best = b1 ? hi : best;
        bi = b1 ? 2 * j + 1 : bi;
    }
    idx = bi;
    return best;
}

struct Vol3Args {
    const float* u;
    const float* f;  // data term or null
    float* out;
    uint8_t* amap;   // selection map or null
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

// One work item of the z-streaming kernels: volume v, row y, the lane's
// column x (owned when inside the volume), the clamped column xc, the
// column xh of the outer neighbour (lane 0: left of the strip, lane 63:
// right of it, clamped; others: xc), row offsets, and the segment [z0, z1)
// of voxel planes.
struct Item3 {
    int v, y, x, z0, z1;
    bool own;
    uint32_t xc, xh;
    int64_t voff, ym, y0, yp;
};

__device__ __forceinline__ Item3 item3(int64_t item, int64_t per_vol, int nstrip, int R, int D,
                                       int H, int W, int64_t ld, int64_t vs) {
    Item3 it;
    const int lane = threadIdx.x & 63;
    it.v = (int)(item / per_vol);
    int64_t rem = item - (int64_t)it.v * per_vol;
    const int seg = (int)(rem / ((int64_t)H * nstrip));
    rem -= (int64_t)seg * H * nstrip;
    it.y = (int)(rem / nstrip);
    const int strip = (int)(rem - (int64_t)it.y * nstrip);
    const int x0 = strip * k3Step;
    it.x = x0 + lane;
    it.own = it.x < W;
    it.xc = (uint32_t)(it.x < W ? it.x : W - 1);
    const int xo = lane == 0 ? x0 - 1 : (lane == 63 ? x0 + 64 : it.x);
    it.xh = (uint32_t)(xo < 0 ? 0 : (xo < W ? xo : W - 1));
    it.z0 = seg * R;
    it.z1 = it.z0 + R < D ? it.z0 + R : D;
    it.voff = (int64_t)it.v * vs;
    it.ym = (int64_t)(it.y > 0 ? it.y - 1 : 0) * ld;
    it.y0 = (int64_t)it.y * ld;
    it.yp = (int64_t)(it.y + 1 < H ? it.y + 1 : H - 1) * ld;
    return it;
}

// Streams planes z0-1 .. z1 (clamped: the replicate border) of the volume u
// through the accumulators and calls fin(z, acc) for every voxel z of the
// segment once its window is complete.  f (or null): the data term, whose
// value at the voxel is handed over in acc.f.
template <class Fin>
__device__ __forceinline__ void walk3(const float* u, const float* f, const Item3& it, int D,
                                      int64_t ss, Fin&& fin) {
    struct Rows {
        float t, m, b, f, ht, hm, hb;
    };
    auto fetch = [&](int p) {
        Rows r;
        const int pc = p < 0 ? 0 : (p < D ? p : D - 1);
        const float* pl = u + (int64_t)pc * ss;
        r.t = ld_at<float>(pl + it.ym, it.xc);
        r.m = ld_at<float>(pl + it.y0, it.xc);
        r.b = ld_at<float>(pl + it.yp, it.xc);
        r.ht = ld_at<float>(pl + it.ym, it.xh);
        r.hm = ld_at<float>(pl + it.y0, it.xh);
        r.hb = ld_at<float>(pl + it.yp, it.xh);
        r.f = (f && p >= it.z0 && p < it.z1) ? ld_at<float>(f + (int64_t)pc * ss + it.y0, it.xc) : 0.0f;
        return r;
    };

    Acc acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc_zero(acc[i]);
    Rows pre[2];
    // voxel z is finished when plane z+1 has been added
    int p = it.z0 - 1;
    pre[0] = fetch(p);
    pre[1] = fetch(p + 1);

    auto step = [&](auto tag) {
        constexpr int Q = decltype(tag)::value;  // slot of voxel p
        constexpr int QM = (Q + 2) % 3;           // voxel p-1
        constexpr int QP = (Q + 1) % 3;           // voxel p+1
        const Rows r = pre[0];
        pre[0] = pre[1];
        pre[1] = fetch(p + 2);
        const PlaneSums ps = plane_sums(r.t, r.m, r.b, r.ht, r.hm, r.hb);
        add_up(acc[QM], ps);
        add_mid(acc[Q], ps);
        acc[Q].f = r.f;
        start_down(acc[QP], ps);
        const int zf = p - 1;  // voxel whose window is now complete
        if (zf >= it.z0 && zf < it.z1) fin(zf, acc[QM]);
    };
    while (true) {
        step(Phase3<0>{});
        if (++p > it.z1) break;
        step(Phase3<1>{});
        if (++p > it.z1) break;
        step(Phase3<2>{});
        if (++p > it.z1) break;
    }
}

__global__ __launch_bounds__(256) void k_stream3d(Vol3Args A) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t per_vol = (int64_t)A.nseg * A.h * A.nstrip;
    const int64_t total = A.n * per_vol;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
    if (item >= total) return;
    const int D = (int)A.d, H = (int)A.h, W = (int)A.w;
    const Item3 it = item3(item, per_vol, A.nstrip, A.R, D, H, W, A.ld, A.vs);
    const float* u = A.u + it.voff;
    const bool data = A.mode == kModeData;
    const float* f = data ? A.f + it.voff : nullptr;
    float* out = A.out + it.voff;
    uint8_t* amap = A.amap ? A.amap + it.voff : nullptr;
    const float lam = (data && A.lam) ? A.lam[it.v] : 0.0f;
    const Coef cf = make_coef(lam, A.dt, data);
    const float lam56 = lam / 56.0f, delta56 = cf.delta / 56.0f;
    walk3(u, f, it, D, A.ss, [&](int zf, const Acc& a) {
        float S;
        int idx = 0;
        if (amap) S = select18_idx(a, idx);
        else S = select18(a);
        float o;
        if (A.mode == kModeCompute) o = S * (1.0f / 56.0f);
        else if (data) o = __builtin_fmaf(cf.delta, __builtin_fmaf(lam56, S, a.f - a.c), a.c);
        else o = __builtin_fmaf(delta56, S, a.c);
        if (it.own) {
            const int64_t q = (int64_t)zf * A.ss + it.y0 + it.x;
            out[q] = o;
            if (amap) amap[q] = (uint8_t)idx;
        }
    });
}

// ---- adjoint -----------------------------------------------------------------
// With the selection m(x) held at its forward value the update is affine in U
// and f (U' = U + delta[(f - U) + lam/56 sum_o w_m(x)[o] Ubar(x + o)], w with
// the centre weight -56), so its adjoint is
//   dL/dU(v) = keep g(v) + coef sum_{x, o : clamp(x + o) = v} w_m(x)[o] g(x)
// with keep = 1 - delta, coef = delta lam / 56 (data term) or keep = 1,
// coef = delta / 56 (flow), dL/df += delta g and
// dL/dlam = sum g (delta H - [delta = 1/(1+lam)] delta^2 ((f - U) + lam H)).
// One step is two launches.  k_adjsel3d recomputes m from U^t with the
// forward's arithmetic (bitwise the same choice, the same walk) into a byte
// map and, with a data term, updates dL/df and writes the work item's dL/dlam
// partial sum.  k_adjgather3d then gathers the sum for every voxel v from the
// selections and cotangents of its 27 neighbours, the replicate border folded
// in exactly (integer weight sums).

struct Adj3Args {
    const float* u;
    const float* f;  // data term or null (flow)
    const float* g;  // dL/dU^{t+1}
    float* g_f;      // dL/df (read unless gf_first, then written) or null
    uint8_t* sel;    // selection map out
    float* part;     // dL/dlam partial sums (slot * items + item) or null
    const float* lam;
    float dt;
    int64_t n, d, h, w, ld, ss, vs;
    int32_t R, nstrip, nseg, slot, gf_first, dlam_default;
};

__global__ __launch_bounds__(256) void k_adjsel3d(Adj3Args A) {
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t per_vol = (int64_t)A.nseg * A.h * A.nstrip;
    const int64_t total = A.n * per_vol;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wv;
    if (item >= total) return;
    const int D = (int)A.d, H = (int)A.h, W = (int)A.w;
    const Item3 it = item3(item, per_vol, A.nstrip, A.R, D, H, W, A.ld, A.vs);
    const bool data = A.f != nullptr;
    const float* u = A.u + it.voff;
    const float* f = data ? A.f + it.voff : nullptr;
    const float* g = A.g + it.voff;
    float* gfp = (data && A.g_f) ? A.g_f + it.voff : nullptr;
    uint8_t* sel = A.sel + it.voff;
    const float lam = data ? A.lam[it.v] : 0.0f;
    const Coef cf = make_coef(lam, A.dt, data);
    float contrib = 0.0f;
    walk3(u, f, it, D, A.ss, [&](int zf, const Acc& a) {
        int idx;
        const float S = select18_idx(a, idx);
        const int64_t q = (int64_t)zf * A.ss + it.y0 + it.x;
        if (it.own) sel[q] = (uint8_t)idx;
        if (data) {
            const float gv = it.own ? g[q] : 0.0f;
            const float hd = S * (1.0f / 56.0f);
            float dudl = cf.delta * hd;
            if (A.dlam_default) dudl -= cf.delta * cf.delta * ((a.f - a.c) + lam * hd);
            contrib = it.own ? __builtin_fmaf(gv, dudl, contrib) : contrib;
            if (gfp && it.own) gfp[q] = __builtin_fmaf(cf.delta, gv, A.gf_first ? 0.0f : gfp[q]);
        }
    });
    if (data && A.part) {
        // fixed-order butterfly over the wave
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
        if ((threadIdx.x & 63) == 0) A.part[(int64_t)A.slot * total + item] = contrib;
    }
}

// Normals of the 9 mirror planes (x, y, z components), plane order of the
// candidates: e_x, e_y, e_z, e_x + e_y, e_x - e_y, e_x + e_z, e_x - e_z,
// e_y + e_z, e_y - e_z.
__constant__ int8_t kPlaneN[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                                     {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

// Tap o = (ox, oy, oz) of half window i (x56 domain): -56 at the centre,
// elsewhere c[o] (1 - sign(n_j . o)) for the n.o <= 0 side (i = 2j) and
// c[o] (1 + sign(n_j . o)) for the other (i = 2j + 1), c = s (x) s (x) s:
// the kept side's weight doubled, the plane's kept, the other side's folded
// away (S = A -+ D_j).
__device__ __forceinline__ int tap3(int i, int oz, int oy, int ox) {
    if (!ox && !oy && !oz) return -56;
    const int c = (ox ? 1 : 2) * (oy ? 1 : 2) * (oz ? 1 : 2);
    const int j = i >> 1;
    const int dot = kPlaneN[j][0] * ox + kPlaneN[j][1] * oy + kPlaneN[j][2] * oz;
    const int sg = dot > 0 ? 1 : (dot < 0 ? -1 : 0);
    return (i & 1) ? c * (1 + sg) : c * (1 - sg);
}

struct Gather3Args {
    const float* g;      // dL/dU^{t+1}
    const uint8_t* sel;  // selections of step t
    float* g_prev;       // dL/dU^t out
    float* g_f;          // null, or dL/df to which dL/dU^t is added (U^0 = f)
    const float* lam;
    float dt;
    int32_t data;
    int64_t n, d, h, w, ld, ss, vs;
    int32_t R, nstrip, nseg;
};

// One wave per work item -- 64 columns of one row y of one volume (a lane
// per column, no halo) and a segment [z0, z1) of voxel planes -- streaming
// along z.  Each plane p of the walk (z0 - 1 .. z1, inside the volume) is
// loaded once as the 3x3 patch of (selection, cotangent) around the lane's
// column and feeds the three voxel planes it borders:
//   acc(v) = sum over sources s and taps o with clamp(s + o) = v of
//            w_{m(s)}[o] g(s).
// Along z the ring planes -1 and D are folded by adding their contributions
// to voxel planes 0 and D-1.  Along y and x the source in the voxel's own
// row (column) also contributes the taps of the ring rows (columns) that
// clamp onto it: o_y in {0, -1 if y = 0, +1 if y = H-1}, likewise o_x.
// Integer weights from a table of the 18 kernels in LDS; fixed summation
// order (deterministic).
__global__ __launch_bounds__(256) void k_adjgather3d(Gather3Args A) {
    // tab: the 18 kernels, tab[i * 27 + (oz+1)*9 + (oy+1)*3 + (ox+1)].
    // tabf[cy * 4 + cx]: the same with the ring folded onto the own row and
    // column for the voxel's border case (bit 0: the low ring, bit 1: the
    // high ring; cy for rows, cx for columns): entry (oz, oy, 0) adds the
    // taps (oz, oy, -1) [cx bit 0] and (oz, oy, +1) [cx bit 1], then entry
    // (oz, 0, ox) adds the x-folded (oz, -1, ox) [cy bit 0] and (oz, +1, ox)
    // [cy bit 1].  A weight is then one table read, with no branches.
    __shared__ int tab[18 * 27];
    __shared__ int tabf[16][18 * 27];
    for (int t = threadIdx.x; t < 18 * 27; t += 256) {
        const int o = t % 27;
        tab[t] = tap3(t / 27, o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1);
    }
    __syncthreads();
    auto xfold = [&](int cx, int e) {  // x-folded entry e for case cx
        int w = tab[e];
        if (e % 3 == 1) {  // ox = 0
            if (cx & 1) w += tab[e - 1];
            if (cx & 2) w += tab[e + 1];
        }
        return w;
    };
    for (int t = threadIdx.x; t < 16 * 18 * 27; t += 256) {
        const int c = t / (18 * 27), e = t % (18 * 27);
        const int cy = c >> 2, cx = c & 3;
        int w = xfold(cx, e);
        if ((e / 3) % 3 == 1) {  // oy = 0
            if (cy & 1) w += xfold(cx, e - 3);
            if (cy & 2) w += xfold(cx, e + 3);
        }
        tabf[c][e] = w;
    }
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t per_vol = (int64_t)A.nseg * A.h * A.nstrip;
    const int64_t total = A.n * per_vol;
    const int D = (int)A.d, H = (int)A.h, W = (int)A.w;
    // persistent blocks (the tables are built once per block): in round r,
    // block b takes the group of 4 items xcd_remap(b) + r * gridDim.x
    for (int64_t grp = xcd_remap(blockIdx.x, gridDim.x); grp * 4 < total; grp += gridDim.x) {
        const int64_t item = grp * 4 + wv;
        if (item >= total) break;
        const int v = (int)(item / per_vol);
        int64_t rem = item - (int64_t)v * per_vol;
        const int seg = (int)(rem / ((int64_t)H * A.nstrip));
        rem -= (int64_t)seg * H * A.nstrip;
        const int y = (int)(rem / A.nstrip);
        const int strip = (int)(rem - (int64_t)y * A.nstrip);
        const int x = strip * 64 + lane;
        const bool own = x < W;
        const int z0 = seg * A.R;
        const int z1 = z0 + A.R < D ? z0 + A.R : D;
        const int64_t base = (int64_t)v * A.vs;
        const bool data = A.data != 0;
        const float lam = data ? A.lam[v] : 0.0f;
        const Coef cf = make_coef(lam, A.dt, data);
        const float keep = data ? 1.0f - cf.delta : 1.0f;
        const float coef = data ? cf.delta * (lam / 56.0f) : cf.delta / 56.0f;

        // columns x-1, x, x+1 (clamped for the loads) and their validity
        int xs[3];
        bool xv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int xx = x + i - 1;
            xv[i] = xx >= 0 && xx < W;
            xs[i] = xx < 0 ? 0 : (xx < W ? xx : W - 1);
        }
        bool yv[3];
        int64_t yo[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int yy = y + i - 1;
            yv[i] = yy >= 0 && yy < H;
            yo[i] = (int64_t)(yy < 0 ? 0 : (yy < H ? yy : H - 1)) * A.ld;
        }
        // the voxel column's border case selects its prefolded table
        const int* tl = tabf[((y == 0 ? 1 : 0) | (y == H - 1 ? 2 : 0)) * 4 +
                             ((x == 0 ? 1 : 0) | (x == W - 1 ? 2 : 0))];

        float acc_m = 0.0f, acc_c = 0.0f, acc_n = 0.0f;  // voxel planes p-1, p, p+1
        float g_c = 0.0f;  // own cotangent of the previous plane (p-1 while plane p is added)
        const int ps = z0 - 1 > 0 ? z0 - 1 : 0;
        const int pl = z1 < D - 1 ? z1 : D - 1;
        for (int p = ps; p <= pl; ++p) {
            uint8_t ms[9];
            float gs[9];
            const int64_t pb = base + (int64_t)p * A.ss;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    ms[i * 3 + j] = A.sel[pb + yo[i] + xs[j]];
                    gs[i * 3 + j] = A.g[pb + yo[i] + xs[j]];
                }
            // weights: source (dy, dx) = (i - 1, j - 1) of plane p towards
            // target plane p + k - 1 (tap o_z = k - 1, o_y = -dy, o_x = -dx),
            // all 27 table reads issued before the products
            int wt[27];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int* row = tl + ms[i * 3 + j] * 27 + (2 - i) * 3 + (2 - j);
#pragma unroll
                    for (int k = 0; k < 3; ++k) wt[(i * 3 + j) * 3 + k] = row[k * 9];
                }
            float t[3] = {0.0f, 0.0f, 0.0f};  // towards planes p-1, p, p+1
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const bool ok = yv[i] && xv[j];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float w = ok ? (float)wt[(i * 3 + j) * 3 + k] : 0.0f;
                        t[k] = __builtin_fmaf(w, gs[i * 3 + j], t[k]);
                    }
                }
            // ring planes -1 and D fold onto planes 0 and D-1
            acc_m += p > 0 ? t[0] : 0.0f;
            acc_c += t[1];
            if (p == 0) acc_c += t[0];
            if (p == D - 1) acc_c += t[2];
            acc_n += p < D - 1 ? t[2] : 0.0f;
            // voxel plane p-1 is complete
            const int zf = p - 1;
            if (zf >= z0 && zf < z1 && own) {
                const int64_t o = base + (int64_t)zf * A.ss + yo[1] + x;
                const float gp = __builtin_fmaf(coef, acc_m, keep * g_c);
                A.g_prev[o] = gp;
                if (A.g_f) A.g_f[o] += gp;
            }
            acc_m = acc_c;
            acc_c = acc_n;
            acc_n = 0.0f;
            g_c = gs[4];
        }
        // the last plane of the volume completes with the walk
        if (pl == D - 1 && pl >= z0 && pl < z1 && own) {
            const int64_t o = base + (int64_t)pl * A.ss + yo[1] + x;
            const float gp = __builtin_fmaf(coef, acc_m, keep * g_c);
            A.g_prev[o] = gp;
            if (A.g_f) A.g_f[o] += gp;
        }
    }
}

// ~16K work items, 8..128 planes per item.  (Round-filling row counts, which
// help the 2-D kernels, measured slower here: this kernel hides latency
// better with more, shorter items.)
// WMC_VOL_ROWS=R: planes per work item, at least the default (the adjoint's
// workspace holds the dL/dlam partials of the default item count).
static int vol_rows(int64_t n, int64_t d, int64_t h, int64_t strips) {
    const int64_t cols = n * h * strips;
    int R = 8;
    while (R < 128 && cols * ((d + R - 1) / R) > 16384) R *= 2;
    if (const char* env = std::getenv("WMC_VOL_ROWS")) {
        const int r = std::atoi(env);
        if (r > R && r <= 4096) R = r;
    }
    return R;
}

hipError_t launch_stream3d(const float* u, const float* f, float* out, const float* lam, float dt,
                           int mode, int64_t n, int64_t d, int64_t h, int64_t w, int64_t ld,
                           int64_t ss, int64_t vs, hipStream_t st, uint8_t* amap) {
    Vol3Args a{};
    a.u = u;
    a.f = f;
    a.out = out;
    a.amap = amap;
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

int64_t adjsel3_items(int64_t n, int64_t d, int64_t h, int64_t w) {
    const int nstrip = (int)((w + k3Step - 1) / k3Step);
    const int R = vol_rows(n, d, h, nstrip);
    return n * ((d + R - 1) / R) * h * nstrip;
}

hipError_t launch_adjsel3d(const float* u, const float* f, const float* g, float* g_f, uint8_t* sel,
                           float* part, int slot, bool gf_first, const float* lam, float dt,
                           int64_t n, int64_t d, int64_t h, int64_t w, int64_t ld, int64_t ss,
                           int64_t vs, hipStream_t st) {
    Adj3Args a{};
    a.u = u;
    a.f = f;
    a.g = g;
    a.g_f = g_f;
    a.sel = sel;
    a.part = part;
    a.lam = lam;
    a.dt = dt;
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
    a.slot = slot;
    a.gf_first = gf_first ? 1 : 0;
    a.dlam_default = !(dt > 0.0f);
    const int64_t total = n * (int64_t)a.nseg * h * a.nstrip;
    hipLaunchKernelGGL(k_adjsel3d, dim3((unsigned)((total + 3) / 4)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_adjgather3d(const float* g, const uint8_t* sel, float* g_prev, float* g_f,
                              const float* lam, float dt, bool data, int64_t n, int64_t d, int64_t h,
                              int64_t w, int64_t ld, int64_t ss, int64_t vs, hipStream_t st) {
    Gather3Args a{};
    a.g = g;
    a.sel = sel;
    a.g_prev = g_prev;
    a.g_f = g_f;
    a.lam = lam;
    a.dt = dt;
    a.data = data ? 1 : 0;
    a.n = n;
    a.d = d;
    a.h = h;
    a.w = w;
    a.ld = ld;
    a.ss = ss;
    a.vs = vs;
    a.nstrip = (int)((w + 63) / 64);
    a.R = vol_rows(n, d, h, a.nstrip);
    a.nseg = (int)((d + a.R - 1) / a.R);
    const int64_t total = n * (int64_t)a.nseg * h * a.nstrip;
    // persistent: at most the resident blocks (4 per CU: 33 KB of LDS each)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t groups = (total + 3) / 4;
    const int64_t cap = (int64_t)4 * (cus > 0 ? cus : 256);
    hipLaunchKernelGGL(k_adjgather3d, dim3((unsigned)(groups < cap ? groups : cap)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace wmc
