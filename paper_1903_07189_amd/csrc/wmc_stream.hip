// wmc_stream.hip -- the streaming, temporally blocked WMC kernel for gfx950.
//
// One wave = one work item (a strip of 64*C columns of one plane and a
// segment of output rows).  Each lane owns C adjacent columns.  The wave walks
// down the rows; at row step n it
//   1. takes input row n (prefetched three steps earlier) and forms its row
//      quantities (a, s, q) with the horizontal neighbours fetched from the
//      adjacent lanes by DPP wave shifts -- no LDS, no barriers;
//   2. for k = 1..T computes row n-k of sweep k from the three most recent
//      rows of sweep k-1 (held in registers) and forms that row's
//      quantities for sweep k+1;
//   3. writes row n-T of sweep T.
// Image rows above 0 / below H-1 are the replicate border; segment ends that
// are not image borders are covered by T extra rows of recomputation.  The
// data term f is kept in a per-lane LDS ring of T+1 rows (written and read by
// the same lane only).
//
// Sweeps are Jacobi (every pixel of sweep k from sweep k-1 only, Sec. 3.5
// eq. (MCF)), so the result is bitwise that of T single-step launches.
#include <hip/hip_runtime.h>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

constexpr int kBlock = 256;                 // 4 independent waves per workgroup
constexpr int kWavesPerBlock = kBlock / 64;


template <int C>
struct Pref {
    float u[C];
    float f[C];
    float d[C];  // l1 mode: dual state of the input row
};

template <int C>
__device__ __forceinline__ void copy_row(RowQ<C>& d, const RowQ<C>& s) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
        d.a[e] = s.a[e];
        d.s[e] = s.s[e];
        d.q[e] = s.q[e];
        d.c[e] = s.c[e];
        d.d[e] = s.d[e];
    }
}

// A copy that stays behind a real (uniform) branch: without the barrier the
// compiler if-converts the rare border copies into selects executed at every
// row step.
template <int C>
__device__ __forceinline__ void rare_copy(RowQ<C>& d, const RowQ<C>& s) {
    __asm__ volatile("" ::: "memory");
    copy_row(d, s);
}

template <int P>
struct Phase {
    static constexpr int value = P;
};

// Everything a work item needs besides the register state.
struct Item {
    const float* src;
    const float* f;
    float* dst;
    const float* dsrc;  // l1 mode: dual state in (null: zero)
    float* ddst;        // l1 mode: dual state out
    uint8_t* amap;
    int64_t ld;
    int H, W;
    int x0, ox0, ox1;
    int y0, y1;
    bool vec;
    Coef k;
    float* traj[3];  // trajectory stores (plane offset applied), see LaunchArgs
    float* traj_in;
};


// Kinds of strip (work-item column ranges):
//   kGeneric   an image narrower than one strip, or a border strip whose
//              rows cannot be moved with vector accesses: clamped scalar
//              loads, the element holding the last image column uses itself
//              as its right neighbour, wave-edge lanes keep their own values;
//   kBorder    the first strip (starting at column 0) or the last one
//              (right-aligned, ending at column W-1): lane 0 of the first and
//              lane 63 of the last keep their own values as their missing
//              neighbour, which is the replicate border at every sweep;
//   kInterior  lanes 0 and 63 are halo lanes whose results are never stored,
//              so their missing neighbours are zero (make_row_inner, whose
//              lane shifts fold into the arithmetic).
// In a launch whose items all run at once the slowest item sets the time, so
// the border strips get their own vector-access variant.
enum StripKind : int { kGeneric = 0, kBorder = 1, kInterior = 2 };

// Runs one work item: rows of T sweeps pipelined in registers (see top of
// file).  VEC: rows are 4C-byte aligned and the strip lies inside the image,
// so every lane moves its C columns with one vector access.  TRAJ: the owned
// rows of sweeps 1..T-1 are also stored where it.traj[k-1] is set.
template <int C, int T, int MODE, bool AM, int KIND, bool VEC, bool TRAJ>
__device__ __forceinline__ void run_item(const Item it, float* __restrict__ ring) {
    constexpr bool L1 = (MODE == kL1);
    constexpr bool DATA = (MODE == kData) || L1;  // modes that read f
    constexpr int NS = T + 1;  // f ring slots
    const int lane = threadIdx.x & 63;
    const int xb = it.x0 + C * lane;
    const int H = it.H, W = it.W;
    static_assert(!(KIND == kGeneric && VEC), "the generic strip uses clamped scalar loads");

    bool last[C], ok[C];
    int xc[C];  // clamped columns for scalar loads
    bool all_ok = true;
#pragma unroll
    for (int e = 0; e < C; ++e) {
        last[e] = (xb + e == W - 1);
        ok[e] = (xb + e >= it.ox0) && (xb + e < it.ox1);
        all_ok = all_ok && ok[e];
        xc[e] = xb + e < W ? xb + e : W - 1;
    }

    // rows of sweep k live in [lo_k, hi_k); sweep k computes row rho at step rho + k
    const int lo0 = it.y0 - T > 0 ? it.y0 - T : 0;
    const int hi0 = it.y1 + T < H ? it.y1 + T : H;
    const int n_last = it.y1 - 1 + T;

    RowQ<C> win[T][3];
    Pref<C> pf[3];

    // rows whose f is ever used: those computed by sweep 1 or later
    const int lo1 = it.y0 - T + 1 > 0 ? it.y0 - T + 1 : 0;
    const int hi1 = it.y1 + T - 1 < H ? it.y1 + T - 1 : H;

    auto load = [&](Pref<C>& p, int row) {
        const float* up = it.src + (int64_t)row * it.ld;
        const float* fp = DATA ? it.f + (int64_t)row * it.ld : nullptr;
        const bool needf = DATA && row >= lo1 && row < hi1;  // wave-uniform
        if constexpr (L1) {
            if (needf && it.dsrc) {
                const float* dp = it.dsrc + (int64_t)row * it.ld;
#pragma unroll
                for (int e = 0; e < C; ++e) p.d[e] = ld_at<float>(dp, (uint32_t)xc[e]);
            } else {
#pragma unroll
                for (int e = 0; e < C; ++e) p.d[e] = 0.0f;
            }
        }
        if constexpr (VEC && C == 4) {
            const float4 v = ld_at<float4>(up, (uint32_t)xb);
            p.u[0] = v.x; p.u[1] = v.y; p.u[2] = v.z; p.u[3] = v.w;
            if (needf) {
                const float4 g = ld_at<float4>(fp, (uint32_t)xb);
                p.f[0] = g.x; p.f[1] = g.y; p.f[2] = g.z; p.f[3] = g.w;
            }
        } else if constexpr (VEC && C == 2) {
            const float2 v = ld_at<float2>(up, (uint32_t)xb);
            p.u[0] = v.x; p.u[1] = v.y;
            if (needf) {
                const float2 g = ld_at<float2>(fp, (uint32_t)xb);
                p.f[0] = g.x; p.f[1] = g.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e) {
                p.u[e] = ld_at<float>(up, (uint32_t)xc[e]);
                if (needf) p.f[e] = ld_at<float>(fp, (uint32_t)xc[e]);
            }
        }
    };

    // stores an owned row of intermediate sweep k (trajectory launches)
    auto store_traj = [&](float* base, int rho, const float (&v)[C]) {
        if (rho < it.y0 || rho >= it.y1) return;  // wave-uniform
        float* dp = base + (int64_t)rho * it.ld;
        if constexpr (VEC) {
            if (all_ok) {
                if constexpr (C == 4) st_at<float4>(dp, (uint32_t)xb, make_float4(v[0], v[1], v[2], v[3]));
                else if constexpr (C == 2) st_at<float2>(dp, (uint32_t)xb, make_float2(v[0], v[1]));
                else st_at<float>(dp, (uint32_t)xb, v[0]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ok[e]) st_at<float>(dp, (uint32_t)(xb + e), v[e]);
        }
    };

    auto store = [&](int rho, const float (&v)[C], const int (&idx)[C], const float (&dv)[C]) {
        if constexpr (L1) {
            float* qp = it.ddst + (int64_t)rho * it.ld;
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ok[e]) st_at<float>(qp, (uint32_t)(xb + e), dv[e]);
        }
        float* dp = it.dst + (int64_t)rho * it.ld;
        if constexpr (VEC) {
            if (all_ok) {  // lanes are wholly inside or wholly in a halo
                if constexpr (C == 4) st_at<float4>(dp, (uint32_t)xb, make_float4(v[0], v[1], v[2], v[3]));
                else if constexpr (C == 2) st_at<float2>(dp, (uint32_t)xb, make_float2(v[0], v[1]));
                else st_at<float>(dp, (uint32_t)xb, v[0]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ok[e]) st_at<float>(dp, (uint32_t)(xb + e), v[e]);
        }
        if constexpr (AM) {
            uint8_t* ap = it.amap + (int64_t)rho * it.ld;
#pragma unroll
            for (int e = 0; e < C; ++e)
                if (ok[e]) ap[(uint32_t)(xb + e)] = (uint8_t)idx[e];
        }
    };

    // one pixel row of sweep k from the three rows of sweep k-1
    auto sweep_row = [&](const RowQ<C>& t, const RowQ<C>& mm, const RowQ<C>& b, int rho,
                         float (&v)[C], int (&idx)[C], float (&dv)[C]) {
        float fv[C];
        if constexpr (DATA) {
            const float* slot = ring + (rho % NS) * (64 * C) + lane * C;
#pragma unroll
            for (int e = 0; e < C; ++e) fv[e] = slot[e];
        }
#pragma unroll
        for (int e = 0; e < C; ++e) {
            const Odd o = parts(t.a[e], t.s[e], t.q[e], mm.s[e], mm.q[e], mm.c[e], b.a[e], b.s[e],
                                b.q[e]);
            float S;
            if constexpr (AM) S = select_x12_idx(o, idx[e]);
            else S = select_x12(o);
            if constexpr (L1) v[e] = update_l1(mm.c[e], fv[e], mm.d[e], S, it.k, dv[e]);
            else if constexpr (MODE == kData) v[e] = update_data(mm.c[e], fv[e], S, it.k);
            else if constexpr (MODE == kFlow) v[e] = update_flow(mm.c[e], S, it.k);
            else v[e] = to_hd(S);
        }
    };

    auto put_ring = [&](int n, const Pref<C>& p) {
        if constexpr (DATA) {
            float* slot = ring + (n % NS) * (64 * C) + lane * C;
#pragma unroll
            for (int e = 0; e < C; ++e) slot[e] = p.f[e];
        }
    };

    int n = lo0;

    // ---- one row step: input row n, then row n-k of every sweep k ----------
    auto generic = [&](auto phase_tag) {
        constexpr int P = decltype(phase_tag)::value;
        constexpr int PM = (P + 2) % 3;
        constexpr int PT = (P + 1) % 3;
        if (n < hi0) {
            // take row n out of its prefetch slot before the slot is refilled
            float m[C], dm[C];
#pragma unroll
            for (int e = 0; e < C; ++e) {
                m[e] = pf[P].u[e];
                dm[e] = L1 ? pf[P].d[e] : 0.0f;
            }
            put_ring(n, pf[P]);
            if (n + 3 < hi0) load(pf[P], n + 3);
            if constexpr (TRAJ && VEC) {
                if (it.traj_in) store_traj(it.traj_in, n, m);  // the input state's owned rows
            }
            if constexpr (KIND == kGeneric) make_row<C, true>(m, last, win[0][P]);
            else if constexpr (KIND == kBorder) make_row<C, false>(m, last, win[0][P]);
            else make_row_inner<C>(m, win[0][P]);
            if constexpr (L1) {
#pragma unroll
                for (int e = 0; e < C; ++e) win[0][P].d[e] = dm[e];
            }
            if (n == 0) rare_copy(win[0][PM], win[0][P]);  // row -1 := row 0 (top border)
        }
#pragma unroll
        for (int k = 1; k <= T; ++k) {
            const int rho = n - k;
            const int lo = it.y0 - (T - k) > 0 ? it.y0 - (T - k) : 0;
            const int hi = it.y1 + (T - k) < H ? it.y1 + (T - k) : H;
            if (rho >= lo && rho < hi) {
                // bottom border: row H := row H-1; sweep k-1 produced no row this
                // step, so its newest slot is free to hold the copy
                if (rho == H - 1) rare_copy(win[k - 1][P], win[k - 1][PM]);
                float v[C], dv[C];
                int idx[C];
                sweep_row(win[k - 1][PT], win[k - 1][PM], win[k - 1][P], rho, v, idx, dv);
                if (k < T) {
                    if constexpr (TRAJ) {
                        if (it.traj[k - 1]) store_traj(it.traj[k - 1], rho, v);
                    }
                    RowQ<C>(&lv)[3] = win[k < T ? k : 0];
                    if constexpr (KIND == kGeneric) make_row<C, true>(v, last, lv[P]);
                    else if constexpr (KIND == kBorder) make_row<C, false>(v, last, lv[P]);
                    else make_row_inner<C>(v, lv[P]);
                    if constexpr (L1) {
#pragma unroll
                        for (int e = 0; e < C; ++e) lv[P].d[e] = dv[e];
                    }
                    if (rho == 0) rare_copy(lv[PM], lv[P]);  // row -1 := row 0
                } else {
                    store(rho, v, idx, dv);
                }
            }
        }
    };

#pragma unroll
    for (int j = 0; j < 3; ++j)
        if (lo0 + j < hi0) load(pf[j], lo0 + j);

    // groups of three steps: the register slot of a row is fixed by its
    // position in the group
    while (true) {
        generic(Phase<0>{});
        if (++n > n_last) return;
        generic(Phase<1>{});
        if (++n > n_last) return;
        generic(Phase<2>{});
        if (++n > n_last) return;
    }
}

// Resolves work item `item` of image d into an Item and runs it.
// VONLY: every strip of the launch moves its rows with vector accesses (the
// host checks it: aligned rows, at least two strips, the last one starting
// at a multiple of C), so the clamped scalar paths are not compiled in --
// they would otherwise set the register allocation of the whole kernel.
template <int C, int T, int MODE, bool AM, bool TRAJ = false, bool VONLY = false>
__device__ __forceinline__ void process(const ImageDesc& d, int64_t local, const LaunchArgs& a,
                                        float* ring) {
    const int64_t per_plane = (int64_t)d.nseg * d.nstrip;
    const int ch = (int)(local / per_plane);
    const int rem = (int)(local - (int64_t)ch * per_plane);
    const int seg = rem / d.nstrip;
    const int strip = rem - seg * d.nstrip;

    Item it;
    const int64_t poff = (int64_t)ch * d.ps;
    const float* srcb = a.src_sel == 0 ? d.src0 : (a.src_sel == 1 ? d.bufA : d.bufB);
    float* dstb = a.dst_sel == 1 ? d.bufA : d.bufB;
    it.src = srcb + poff;
    it.f = d.f ? d.f + poff : nullptr;
    it.dst = dstb + poff;
    it.amap = d.amap ? d.amap + poff : nullptr;
    if constexpr (MODE == kL1) {
        // l1 launches are single plane sets with the dual read from dsrc0 and
        // written to dA (the host passes explicit pointers per launch)
        it.dsrc = d.dsrc0 ? d.dsrc0 + poff : nullptr;
        it.ddst = d.dA + poff;
    } else {
        it.dsrc = nullptr;
        it.ddst = nullptr;
    }
    it.ld = d.ld;
    it.H = d.H;
    it.W = d.W;
    const int width = 64 * C, halo = halo_cols(C, T), step = width - 2 * halo;
    const bool first = strip == 0, lastS = strip == d.nstrip - 1;
    // the last of several strips is right-aligned: it ends at column W-1
    // (W <= (nstrip-1)*step + width, so its own columns keep their halo)
    it.x0 = (lastS && !first) ? d.W - width : strip * step;
    it.ox0 = first ? 0 : strip * step + halo;
    it.ox1 = lastS ? d.W : strip * step + width - halo;
    it.y0 = seg * a.R;
    it.y1 = it.y0 + a.R < d.H ? it.y0 + a.R : d.H;
    it.vec = d.vec != 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) it.traj[k] = (TRAJ && a.traj[k]) ? a.traj[k] + poff : nullptr;
    // the input state is stored by vector-only builds only (the host copies
    // it otherwise): the clamped scalar path has no registers to spare
    it.traj_in = (TRAJ && VONLY && a.traj_in) ? a.traj_in + poff : nullptr;
    const float lam = a.lam ? a.lam[d.lam_index + ch * d.lam_stride] : 0.0f;
    if constexpr (MODE == kL1) it.k = make_coef_l1(lam, a.dt, a.alpha);
    else it.k = make_coef(lam, a.dt, MODE == kData);
    if constexpr (VONLY) {
        if (first || lastS) run_item<C, T, MODE, AM, kBorder, true, TRAJ>(it, ring);
        else run_item<C, T, MODE, AM, kInterior, true, TRAJ>(it, ring);
    } else if (first || lastS) {
        if (!(first && lastS) && it.vec && it.x0 % C == 0)
            run_item<C, T, MODE, AM, kBorder, true, TRAJ>(it, ring);
        else
            run_item<C, T, MODE, AM, kGeneric, false, TRAJ>(it, ring);
    } else if (it.vec) {
        run_item<C, T, MODE, AM, kInterior, true, TRAJ>(it, ring);
    } else {
        run_item<C, T, MODE, AM, kInterior, false, TRAJ>(it, ring);
    }
}

template <int C, int T, int MODE>
constexpr int ring_floats() {
    return (MODE == kData || MODE == kL1) ? kWavesPerBlock * (T + 1) * 64 * C : 1;
}

template <int C, int T, int MODE, bool AM, bool VONLY = false>
__global__ __launch_bounds__(kBlock) void k_stream_single(ImageDesc d, LaunchArgs a) {
    __shared__ float ring[ring_floats<C, T, MODE>()];
    // wave index, made visibly wave-uniform so that all work-item bookkeeping
    // lives in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = (int64_t)d.channels * d.nseg * d.nstrip;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wv;
    if (item >= total) return;
    process<C, T, MODE, AM, false, VONLY>(
        d, item, a, ring + ((MODE == kData || MODE == kL1) ? wv * (T + 1) * 64 * C : 0));
}

// Trajectory variant of k_stream_single: also stores the states after the
// intermediate sweeps (checkpoints that fall inside a fused launch).
template <int C, int T, int MODE, bool VONLY = false>
__global__ __launch_bounds__(kBlock, (C == 2 ? 3 : 1)) void k_stream_traj(ImageDesc d, LaunchArgs a) {
    __shared__ float ring[ring_floats<C, T, MODE>()];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t total = (int64_t)d.channels * d.nseg * d.nstrip;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wv;
    if (item >= total) return;
    process<C, T, MODE, false, true, VONLY>(d, item, a,
                                            ring + (MODE == kData ? wv * (T + 1) * 64 * C : 0));
}

// Batched variant: one flat launch over the work items of many images (each
// image's items contiguous, in the order channel, segment, strip).  owner[i]
// is the image of item i, so a wave finds its descriptor with two scalar
// loads.  Items are equal-sized strips, so the hardware's dispatch of one
// wave per item balances an uneven batch as well as a work queue would,
// without a device-wide atomic per item (the 8 XCDs share no L2, so such an
// atomic goes to memory and serialises every wave of the device on one
// address).
template <int C, int T, int MODE>
__global__ __launch_bounds__(kBlock) void k_stream_batched(const ImageDesc* __restrict__ tbl,
                                                           const int32_t* __restrict__ owner,
                                                           int64_t total, LaunchArgs a) {
    __shared__ float ring[ring_floats<C, T, MODE>()];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * kWavesPerBlock + wv;
    if (item >= total) return;
    const int img = __builtin_amdgcn_readfirstlane(owner[item]);
    const ImageDesc d = tbl[img];
    process<C, T, MODE, false>(d, item - d.item_base, a,
                               ring + (MODE == kData ? wv * (T + 1) * 64 * C : 0));
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Plane-set copy and accumulate: the rows of all planes (p, y) form one list
// that the grid's y dimension strides over, so any height and plane count
// fits the launch; threads run along the row.
__global__ void k_add_planes(const float* __restrict__ src, float* __restrict__ dst, int64_t rows,
                             int64_t h, int64_t w, int64_t ld, int64_t ps) {
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const int64_t p = r / h;
        const int64_t base = p * ps + (r - p * h) * ld;
        for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < w;
             x += (int64_t)gridDim.x * blockDim.x)
            dst[base + x] += src[base + x];
    }
}

__global__ void k_copy_planes(const float* __restrict__ src, float* __restrict__ dst, int64_t rows,
                              int64_t h, int64_t w, int64_t ld, int64_t ps) {
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y) {
        const int64_t p = r / h;
        const int64_t base = p * ps + (r - p * h) * ld;
        for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < w;
             x += (int64_t)gridDim.x * blockDim.x)
            dst[base + x] = src[base + x];
    }
}

// Lane-shift self test: flags[w] = 1 iff the lane shifts of wmc_device.hpp
// (with kept and with zero edge values) move data as the kernels assume, for
// every lane of wave w.
__global__ void k_selftest(int* flags) {
    const int lane = threadIdx.x & 63;
    const float me = (float)(lane + 1);
    const float lo = from_lower_lane(-me, me);
    const float up = from_upper_lane(-me, me);
    const float want_lo = lane == 0 ? -me : (float)lane;
    const float want_up = lane == 63 ? -me : (float)(lane + 2);
    const float loz = from_lower_lane_or_zero(me);
    const float upz = from_upper_lane_or_zero(me);
    const float want_loz = lane == 0 ? 0.0f : (float)lane;
    const float want_upz = lane == 63 ? 0.0f : (float)(lane + 2);
    const bool good = (lo == want_lo) && (up == want_up) && (loz == want_loz) && (upz == want_upz);
    const unsigned long long ballot = __ballot(good);
    if (lane == 0) flags[threadIdx.x >> 6] = (ballot == ~0ull) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using SingleFn = void (*)(ImageDesc, LaunchArgs);
using BatchedFn = void (*)(const ImageDesc*, const int32_t*, int64_t, LaunchArgs);

template <int C, int T, int MODE, bool AM>
static SingleFn single_ptr() { return k_stream_single<C, T, MODE, AM>; }

static int tindex(int T) {
    switch (T) {
        case 1: return 0;
        case 2: return 1;
        case 3: return 2;
        case 4: return 3;
        case 6: return 4;
        case 8: return 5;
        default: return -1;
    }
}
static int cindex(int C) { return C == 1 ? 0 : (C == 2 ? 1 : (C == 4 ? 2 : -1)); }

#define WMC_T_LIST(X, C, M) X(C, 1, M) X(C, 2, M) X(C, 3, M) X(C, 4, M) X(C, 6, M) X(C, 8, M)

template <bool V>
static SingleFn single_table_v(int C, int T, int mode, bool am) {
    const int ci = cindex(C), ti = tindex(T);
    if (ci < 0 || ti < 0) return nullptr;
    if (mode == kModeCompute) {
        if (T != 1) return nullptr;
        static const SingleFn tab[3][2] = {
            {k_stream_single<1, 1, kCompute, false, V>, k_stream_single<1, 1, kCompute, true, V>},
            {k_stream_single<2, 1, kCompute, false, V>, k_stream_single<2, 1, kCompute, true, V>},
            {k_stream_single<4, 1, kCompute, false, V>, k_stream_single<4, 1, kCompute, true, V>}};
        return tab[ci][am ? 1 : 0];
    }
    if (am) {
        if (T != 1) return nullptr;
        static const SingleFn tab[3][2] = {
            {k_stream_single<1, 1, kData, true, V>, k_stream_single<1, 1, kFlow, true, V>},
            {k_stream_single<2, 1, kData, true, V>, k_stream_single<2, 1, kFlow, true, V>},
            {k_stream_single<4, 1, kData, true, V>, k_stream_single<4, 1, kFlow, true, V>}};
        return tab[ci][mode == kModeData ? 0 : 1];
    }
#define WMC_S(C, T, M) k_stream_single<C, T, M, false, V>,
    static const SingleFn data_tab[3][6] = {{WMC_T_LIST(WMC_S, 1, kData)},
                                            {WMC_T_LIST(WMC_S, 2, kData)},
                                            {WMC_T_LIST(WMC_S, 4, kData)}};
    static const SingleFn flow_tab[3][6] = {{WMC_T_LIST(WMC_S, 1, kFlow)},
                                            {WMC_T_LIST(WMC_S, 2, kFlow)},
                                            {WMC_T_LIST(WMC_S, 4, kFlow)}};
    if (mode == kModeL1) {
        static const SingleFn l1_tab[3][6] = {{WMC_T_LIST(WMC_S, 1, kL1)},
                                              {WMC_T_LIST(WMC_S, 2, kL1)},
                                              {WMC_T_LIST(WMC_S, 4, kL1)}};
        return l1_tab[ci][ti];
    }
#undef WMC_S
    return mode == kModeData ? data_tab[ci][ti] : flow_tab[ci][ti];
}

static SingleFn single_table(int C, int T, int mode, bool am, bool vonly = false) {
    return vonly ? single_table_v<true>(C, T, mode, am) : single_table_v<false>(C, T, mode, am);
}

static BatchedFn batched_table(int C, int T, int mode) {
    const int ci = cindex(C), ti = tindex(T);
    if (ci < 0 || ti < 0 || mode == kModeCompute) return nullptr;
#define WMC_B(C, T, M) k_stream_batched<C, T, M>,
    static const BatchedFn data_tab[3][6] = {{WMC_T_LIST(WMC_B, 1, kData)},
                                             {WMC_T_LIST(WMC_B, 2, kData)},
                                             {WMC_T_LIST(WMC_B, 4, kData)}};
    static const BatchedFn flow_tab[3][6] = {{WMC_T_LIST(WMC_B, 1, kFlow)},
                                             {WMC_T_LIST(WMC_B, 2, kFlow)},
                                             {WMC_T_LIST(WMC_B, 4, kFlow)}};
#undef WMC_B
    return mode == kModeData ? data_tab[ci][ti] : flow_tab[ci][ti];
}

bool vector_only(const ImageDesc& d, int C) {
    return d.vec != 0 && d.nstrip >= 2 && (d.W - 64 * C) % C == 0;
}

template <bool V>
static SingleFn traj_table_v(int C, int T, int mode) {
    const int ci = cindex(C);
    if (ci < 0 || T < 2 || T > kTrajMaxT || (mode != kModeData && mode != kModeFlow)) return nullptr;
#define WMC_TR(C, M) {k_stream_traj<C, 2, M, V>, k_stream_traj<C, 3, M, V>, k_stream_traj<C, 4, M, V>}
    static const SingleFn data_tab[3][3] = {WMC_TR(1, kData), WMC_TR(2, kData), WMC_TR(4, kData)};
    static const SingleFn flow_tab[3][3] = {WMC_TR(1, kFlow), WMC_TR(2, kFlow), WMC_TR(4, kFlow)};
#undef WMC_TR
    return mode == kModeData ? data_tab[ci][T - 2] : flow_tab[ci][T - 2];
}

static SingleFn traj_table(int C, int T, int mode, bool vonly) {
    return vonly ? traj_table_v<true>(C, T, mode) : traj_table_v<false>(C, T, mode);
}

hipError_t launch_stream_traj(int C, int T, int mode, const ImageDesc& d, const LaunchArgs& a,
                              hipStream_t st) {
    SingleFn fn = traj_table(C, T, mode, vector_only(d, C));
    if (!fn) return hipErrorInvalidValue;
    const int64_t total = (int64_t)d.channels * d.nseg * d.nstrip;
    const int64_t blocks = (total + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, st, d, a);
    return hipGetLastError();
}

int stream_traj_blocks_per_cu(int C, int T, int mode, bool vonly) {
    SingleFn fn = traj_table(C, T, mode, vonly);
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), kBlock,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

bool stream_variant_exists(int C, int T, int mode, bool argmin) {
    return single_table(C, T, mode, argmin) != nullptr;
}

hipError_t launch_stream_single(int C, int T, int mode, bool argmin, const ImageDesc& d,
                                const LaunchArgs& a, hipStream_t st) {
    SingleFn fn = single_table(C, T, mode, argmin, vector_only(d, C));
    if (!fn) return hipErrorInvalidValue;
    const int64_t total = (int64_t)d.channels * d.nseg * d.nstrip;
    const int64_t blocks = (total + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, st, d, a);
    return hipGetLastError();
}

int stream_single_blocks_per_cu(int C, int T, int mode, bool argmin, bool vonly) {
    SingleFn fn = single_table(C, T, mode, argmin, vonly);
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), kBlock,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

int stream_blocks_per_cu(int C, int T, int mode) {
    BatchedFn fn = batched_table(C, T, mode);
    if (!fn) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), kBlock,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_stream_batched(int C, int T, int mode, const ImageDesc* dtable,
                                 const int32_t* owner, int64_t total_items, const LaunchArgs& a,
                                 hipStream_t st) {
    BatchedFn fn = batched_table(C, T, mode);
    if (!fn) return hipErrorInvalidValue;
    const int64_t blocks = (total_items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kBlock), 0, st, dtable, owner, total_items,
                       a);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

// Grid of the plane-set copy / accumulate: up to 64 blocks along a row and
// up to 65535 along the row list (the kernels stride over the rest).
static dim3 plane_rows_grid(int64_t rows, int64_t w) {
    const int64_t gx = (w + 255) / 256 < 64 ? (w + 255) / 256 : 64;
    const int64_t gy = rows < 65535 ? rows : 65535;
    return dim3((unsigned)gx, (unsigned)gy);
}

hipError_t launch_copy_planes(const float* src, float* dst, int64_t n, int64_t h, int64_t w,
                              int64_t ld, int64_t ps, hipStream_t st) {
    if (n <= 0 || h <= 0 || w <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_planes, plane_rows_grid(n * h, w), dim3(256), 0, st, src, dst, n * h,
                       h, w, ld, ps);
    return hipGetLastError();
}

hipError_t launch_add_planes(const float* src, float* dst, int64_t n, int64_t h, int64_t w,
                             int64_t ld, int64_t ps, hipStream_t st) {
    if (n <= 0 || h <= 0 || w <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_planes, plane_rows_grid(n * h, w), dim3(256), 0, st, src, dst, n * h,
                       h, w, ld, ps);
    return hipGetLastError();
}

hipError_t launch_selftest(int* flags, hipStream_t st) {
    hipLaunchKernelGGL(k_selftest, dim3(1), dim3(256), 0, st, flags);
    return hipGetLastError();
}

}  // namespace wmc
