// wmc_adjoint.hip -- reverse-mode derivative of one WMC update for gfx950.
//
// With the selected half window m(x) held at its forward value, the update
//   U'(x) = U(x) + delta [(f(x) - U(x)) + lam/12 sum_o c_{m(x)}[o] Ub(x+o)]
// (c_i = 12 h_i with the centre weight -12, Ub the replicate-padded U,
// Sec. 4.2) is affine in U and f, and its adjoint is
//   g_prev = keep g + coef Fold(acc),   acc(z) = sum_x c_{m(x)}[z - x] g(x)
// over the padded grid z, with keep = 1 - delta, coef = delta lam / 12 (data
// term) or keep = 1, coef = delta / 12 (flow); Fold adds the one-pixel ring of
// the padded grid onto the border pixels it replicates.
//
// Every half-window kernel is c_i = a + sigma_i e_j(i): the even kernel
// a = [1 2 1; 2 -12 2; 1 2 1] plus or minus one of four odd kernels e1, e2,
// e5, e6 (the decomposition the forward evaluates, wmc_device.hpp).  With the
// fields G = g and W_j = sigma g at pixels whose selection is in family j
// (zero elsewhere), the data-dependent scatter becomes fixed stencils:
//   acc = (a (x) G) - sum_j (e_j (x) W_j),
// where (x) is the same correlation the forward computes (a is symmetric,
// the e_j antisymmetric).  The adjoint therefore runs the forward's
// column-sum form on five fields instead of gathering per-tap weights.
//
// k_adj_stream: one wave per work item -- a strip of 64*C columns with a halo
// of halo_cols(C, 2) columns on both sides (so the first strip also holds the
// virtual columns -2, -1 and the last one W, W+1) and a segment of R rows --
// streaming down the rows.  At step n it
//   - takes rows n of U, g and f (row and column indices clamped: the
//     replicate border), prefetched three steps earlier;
//   - stage A, row n-1: the selection from U rows n-2..n through the same
//     per-pixel arithmetic as the forward (bitwise the same choice), the
//     fields (zero outside the image), dL/df += delta g and the dL/dlam
//     partial sum over the pixels the item owns;
//   - stage B, row n-2: the five stencils from field rows n-3..n-1, the ring
//     folds, and g_prev.
// Fields vanish outside the image, so the stencils evaluated at the virtual
// rows -1, H and columns -1, W are exactly the ring values to fold.
//
// dL/dlam: each work item writes one partial sum per step into its slot of
// a buffer; k_lam_slot_sums and k_lam_accumulate add, per plane and in a
// fixed order, the steps of a checkpoint segment from the last to the first
// -- the same sequence of additions whatever the segment length -- so
// gradients are bitwise reproducible and independent of the checkpoint
// period.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "wmc_device.hpp"
#include "wmc_internal.h"

namespace wmc {

constexpr int kAdjBlock = 256;  // 4 independent waves per workgroup
constexpr int kAdjWaves = kAdjBlock / 64;

// Row quantities of the five fields: G (s, centre), W1 (q), W2 (s), W5 (a, q),
// W6 (a, q) -- what the stencils read.
template <int C>
struct FRow {
    float gs[C], gc[C], q1[C], s2[C], a5[C], q5[C], a6[C], q6[C];
};

template <int C>
__device__ __forceinline__ void zero_frow(FRow<C>& r) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
        r.gs[e] = 0.0f; r.gc[e] = 0.0f; r.q1[e] = 0.0f; r.s2[e] = 0.0f;
        r.a5[e] = 0.0f; r.q5[e] = 0.0f; r.a6[e] = 0.0f; r.q6[e] = 0.0f;
    }
}

// Left / right neighbours of a field row; zero beyond the wave's edge lanes
// (halo columns, whose results are not used).
template <int C>
__device__ __forceinline__ void nbrs(const float (&x)[C], float (&l)[C], float (&r)[C]) {
    const float lft = from_lower_lane_or_zero(x[C - 1]);
    const float rgt = from_upper_lane_or_zero(x[0]);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        l[e] = (e == 0) ? lft : x[e - 1];
        r[e] = (e == C - 1) ? rgt : x[e + 1];
    }
}

template <int C>
__device__ __forceinline__ void make_frow(const float (&G)[C], const float (&W1)[C],
                                          const float (&W2)[C], const float (&W5)[C],
                                          const float (&W6)[C], FRow<C>& o) {
    // l + 2x is written as l + (x + x) (2x is exact, so it rounds as
    // fma(2, x, l)): additions accept a lane-shifted operand directly
    float l[C], r[C];
    nbrs(G, l, r);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        o.gs[e] = (l[e] + (G[e] + G[e])) + r[e];
        o.gc[e] = G[e];
    }
    nbrs(W1, l, r);
#pragma unroll
    for (int e = 0; e < C; ++e) o.q1[e] = l[e] - r[e];
    nbrs(W2, l, r);
#pragma unroll
    for (int e = 0; e < C; ++e) o.s2[e] = (l[e] + (W2[e] + W2[e])) + r[e];
    nbrs(W5, l, r);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        o.a5[e] = l[e] + (W5[e] + W5[e]);
        o.q5[e] = l[e] - r[e];
    }
    nbrs(W6, l, r);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        o.a6[e] = l[e] + (W6[e] + W6[e]);
        o.q6[e] = l[e] - r[e];
    }
}

// acc at the middle row: (a (x) G) - sum_j (e_j (x) W_j), each stencil in the
// column-sum form of the forward's parts().
template <int C>
__device__ __forceinline__ float stencil(const FRow<C>& t, const FRow<C>& m, const FRow<C>& b,
                                         int e) {
    const float A = __builtin_fmaf(-16.0f, m.gc[e], __builtin_fmaf(2.0f, m.gs[e], t.gs[e] + b.gs[e]));
    const float E1 = __builtin_fmaf(2.0f, m.q1[e], t.q1[e] + b.q1[e]);
    const float E2 = t.s2[e] - b.s2[e];
    const float E5 = __builtin_fmaf(2.0f, m.q5[e], (t.a5[e] - b.a5[e]) + b.q5[e]);
    const float E6 = __builtin_fmaf(-2.0f, m.q6[e], (t.a6[e] - b.a6[e]) - t.q6[e]);
    return A - ((E1 + E2) + (E5 + E6));
}

struct AdjItem {
    const float* u;
    const float* f;
    const float* g;
    float* g_prev;
    float* g_f;
    int ld;  // row stride in elements (< 2^31: row offsets are 32 x 32 -> 64-bit products)
    int H, W;
    int x0, ox0, ox1;  // first loaded column, owned columns [ox0, ox1)
    int y0, y1;        // owned rows
    float delta, lam, keep, coef;
    bool dlam_default;  // delta = 1/(1+lam): dU'/dlam has the delta'(lam) term
    bool gf_first;      // g_f is not read (taken as zero) but written
    bool gf_fold;       // the last step of a solve from U^0 = f: dL/df also gets g_prev
};

template <int P>
struct APhase {
    static constexpr int value = P;
};

// Runs one work item; returns the item's dL/dlam partial sum (valid in lane 0
// after the wave reduction, data mode only).  EDGE: first or last strip
// (clamped scalar loads, column folds).  VEC: rows are 4C-byte aligned and the
// strip lies inside the image, so every lane moves its C columns with one
// vector access.
template <int C, bool DATA, bool EDGE, bool VEC>
__device__ __forceinline__ float run_adj(const AdjItem it) {
    const int lane = threadIdx.x & 63;
    const int xb = it.x0 + C * lane;
    const int H = it.H, W = it.W;

    bool inimg[C], own[C], isL[C], isR[C];
    int xc[C];
    bool all_own = true;
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const int x = xb + e;
        inimg[e] = x >= 0 && x < W;
        own[e] = x >= it.ox0 && x < it.ox1;
        all_own = all_own && own[e];
        isL[e] = x == 0;
        isR[e] = x == W - 1;
        xc[e] = x < 0 ? 0 : (x < W ? x : W - 1);
    }

    float pu[3][C], pg[3][C], pfv[3][C], pgf[3][C];  // prefetch slots
    RowQ<C> uw[3];                                    // U row quantities, rows n-2..n
    FRow<C> fw[3];                                    // field rows n-3..n-1
    float gr[3][C], fr[3][C], gfr[3][C];              // g, f and dL/df rows n-2..n
    float topfold[C], pend[C], pendg[C];  // row -1 fold; row H-1 held until row H is done
    float pendgf[C];                      // with gf_fold: dL/df of row H-1, held likewise
#pragma unroll
    for (int j = 0; j < 3; ++j) zero_frow(fw[j]);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        topfold[e] = 0.0f;
        pend[e] = 0.0f;
        pendg[e] = 0.0f;
        pendgf[e] = 0.0f;
    }
    float contrib = 0.0f;

    const int n0 = it.y0 - 2, nend = it.y1 + 2;

    auto load = [&](float (&u)[C], float (&g)[C], float (&fv)[C], float (&gf)[C], int row,
                    bool any_row) {
        const int rr = row < 0 ? 0 : (row < H ? row : H - 1);
        const float* up = it.u + (int64_t)rr * (int64_t)it.ld;
        const float* gp = it.g + (int64_t)rr * (int64_t)it.ld;
        const float* fp = DATA ? it.f + (int64_t)rr * (int64_t)it.ld : nullptr;
        // dL/df is read-modify-written on owned rows and columns only; with
        // any_row (steady steps) the row is loaded whether owned or not, at
        // clamped columns, and the values of rows and columns that are not
        // owned are never used
        if (DATA && it.g_f && !it.gf_first && (any_row || (row >= it.y0 && row < it.y1))) {
            const float* qp = it.g_f + (int64_t)rr * (int64_t)it.ld;
#pragma unroll
            for (int e = 0; e < C; ++e)
                gf[e] = any_row ? ld_at<float>(qp, (uint32_t)xc[e])
                                : (own[e] ? ld_at<float>(qp, (uint32_t)(xb + e)) : 0.0f);
        }
        if constexpr (VEC && C == 4) {
            const float4 a = ld_at<float4>(up, (uint32_t)xb);
            const float4 b = ld_at<float4>(gp, (uint32_t)xb);
            u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
            g[0] = b.x; g[1] = b.y; g[2] = b.z; g[3] = b.w;
            if constexpr (DATA) {
                const float4 c = ld_at<float4>(fp, (uint32_t)xb);
                fv[0] = c.x; fv[1] = c.y; fv[2] = c.z; fv[3] = c.w;
            }
        } else if constexpr (VEC && C == 2) {
            const float2 a = ld_at<float2>(up, (uint32_t)xb);
            const float2 b = ld_at<float2>(gp, (uint32_t)xb);
            u[0] = a.x; u[1] = a.y;
            g[0] = b.x; g[1] = b.y;
            if constexpr (DATA) {
                const float2 c = ld_at<float2>(fp, (uint32_t)xb);
                fv[0] = c.x; fv[1] = c.y;
            }
        } else {
#pragma unroll
            for (int e = 0; e < C; ++e) {
                u[e] = ld_at<float>(up, (uint32_t)xc[e]);
                g[e] = ld_at<float>(gp, (uint32_t)xc[e]);
                if constexpr (DATA) fv[e] = ld_at<float>(fp, (uint32_t)xc[e]);
            }
        }
    };

    // g_prev of row r; with gf_fold also dL/df(r) = gf (this step's value of
    // row r, held back by stage A) + g_prev(r), the path through U^0 = f
    auto store = [&](int r, const float (&acc)[C], const float (&gv)[C], const float (&gf)[C]) {
        float* dp = it.g_prev + (int64_t)r * (int64_t)it.ld;
        float v[C];
#pragma unroll
        for (int e = 0; e < C; ++e) v[e] = __builtin_fmaf(it.coef, acc[e], it.keep * gv[e]);
        if constexpr (DATA) {
            if (it.gf_fold) {
                float* qp = it.g_f + (int64_t)r * (int64_t)it.ld;
#pragma unroll
                for (int e = 0; e < C; ++e)
                    if (own[e]) st_at<float>(qp, (uint32_t)(xb + e), gf[e] + v[e]);
            }
        }
        if constexpr (VEC) {
            if (all_own) {
                if constexpr (C == 4) st_at<float4>(dp, (uint32_t)xb, make_float4(v[0], v[1], v[2], v[3]));
                else if constexpr (C == 2) st_at<float2>(dp, (uint32_t)xb, make_float2(v[0], v[1]));
                else st_at<float>(dp, (uint32_t)xb, v[0]);
                return;
            }
        }
#pragma unroll
        for (int e = 0; e < C; ++e)
            if (own[e]) st_at<float>(dp, (uint32_t)(xb + e), v[e]);
    };

    int n = n0;

    // One row step.  ST ("steady"): a step whose every border and ownership
    // test below is known to pass -- row n+3 is still to be prefetched, stage
    // A's row n-1 and stage B's row n-2 are owned rows, neither is the first
    // or last image row -- so that the step is straight-line code.  Steady and
    // generic steps do the same arithmetic.
    auto step = [&](auto phase_tag, auto steady_tag) {
        constexpr int P = decltype(phase_tag)::value;
        constexpr bool ST = decltype(steady_tag)::value;
        constexpr int PM = (P + 2) % 3;  // row n-1
        constexpr int PT = (P + 1) % 3;  // row n-2 (and n+1 for the prefetch)
        // row n out of its prefetch slot, then refill the slot with row n+3
        float m[C];
#pragma unroll
        for (int e = 0; e < C; ++e) {
            m[e] = pu[P][e];
            gr[P][e] = pg[P][e];
            fr[P][e] = DATA ? pfv[P][e] : 0.0f;
            gfr[P][e] = DATA ? pgf[P][e] : 0.0f;
        }
        if (ST || n + 3 <= nend) load(pu[P], pg[P], pfv[P], pgf[P], n + 3, ST);
        // lanes 0 and 63 take zero for their missing neighbour: their
        // selections only reach stencils of halo columns that are not stored
        make_row_inner<C>(m, uw[P]);

        // stage A: fields of row rho = n-1 (zero outside the image)
        const int rho = n - 1;
        if (ST || rho >= it.y0 - 1) {
            float G[C], W1[C], W2[C], W5[C], W6[C];
            if (ST || (rho >= 0 && rho < H)) {
                const bool owned_row = ST || (rho >= it.y0 && rho < it.y1);
                float* gfp = (DATA && it.g_f && owned_row) ? it.g_f + (int64_t)rho * (int64_t)it.ld : nullptr;
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    const Odd o = parts(uw[PT].a[e], uw[PT].s[e], uw[PT].q[e], uw[PM].s[e],
                                        uw[PM].q[e], uw[PM].c[e], uw[P].a[e], uw[P].s[e],
                                        uw[P].q[e]);
                    Pick pk;
                    const float S = select_x12_pick(o, pk);
                    const float gv = (!EDGE || inimg[e]) ? gr[PM][e] : 0.0f;
                    const float sg = in_mask(pk.neg) ? -gv : gv;
                    G[e] = gv;
                    W1[e] = in_mask(~pk.half & ~pk.second) ? sg : 0.0f;
                    W2[e] = in_mask(~pk.half & pk.second) ? sg : 0.0f;
                    W5[e] = in_mask(pk.half & ~pk.second) ? sg : 0.0f;
                    W6[e] = in_mask(pk.half & pk.second) ? sg : 0.0f;
                    if constexpr (DATA) {
                        if (owned_row) {
                            const float hd = to_hd(S);
                            float dudl = it.delta * hd;
                            if (it.dlam_default)
                                dudl -= it.delta * it.delta * ((fr[PM][e] - uw[PM].c[e]) + it.lam * hd);
                            const float c1 = __builtin_fmaf(gv, dudl, contrib);
                            contrib = own[e] ? c1 : contrib;
                            const float gfn =
                                __builtin_fmaf(it.delta, gv, it.gf_first ? 0.0f : gfr[PM][e]);
                            if (it.gf_fold) gfr[PM][e] = gfn;  // stored by stage B with g_prev
                            else if (gfp && own[e]) st_at<float>(gfp, (uint32_t)(xb + e), gfn);
                        }
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    G[e] = 0.0f; W1[e] = 0.0f; W2[e] = 0.0f; W5[e] = 0.0f; W6[e] = 0.0f;
                }
            }
            make_frow(G, W1, W2, W5, W6, fw[PM]);
        }

        // stage B: row r = n-2
        const int r = n - 2;
        const bool owned = ST || (r >= it.y0 && r < it.y1);
        const bool top = !ST && r == -1 && it.y0 == 0;
        const bool bot = !ST && r == H && it.y1 == H;
        if (owned || top || bot) {
            float acc[C];
#pragma unroll
            for (int e = 0; e < C; ++e) acc[e] = stencil(fw[P], fw[PT], fw[PM], e);
            if constexpr (EDGE) {
                // column ring: virtual column -1 onto column 0, W onto W-1
                const float lft = from_lower_lane_or_zero(acc[C - 1]);
                const float rgt = from_upper_lane_or_zero(acc[0]);
                float add[C];
#pragma unroll
                for (int e = 0; e < C; ++e) {
                    const float fromL = (e == 0) ? lft : acc[e - 1];
                    const float fromR = (e == C - 1) ? rgt : acc[e + 1];
                    add[e] = isL[e] ? (isR[e] ? fromL + fromR : fromL) : (isR[e] ? fromR : 0.0f);
                }
#pragma unroll
                for (int e = 0; e < C; ++e)
                    if (isL[e] || isR[e]) acc[e] += add[e];
            }
            if (top) {
#pragma unroll
                for (int e = 0; e < C; ++e) topfold[e] = acc[e];
            } else if (bot) {
#pragma unroll
                for (int e = 0; e < C; ++e) acc[e] += pend[e];
                store(H - 1, acc, pendg, pendgf);
            } else {
                if (!ST && r == 0) {
#pragma unroll
                    for (int e = 0; e < C; ++e) acc[e] += topfold[e];
                }
                if (!ST && r == H - 1) {
#pragma unroll
                    for (int e = 0; e < C; ++e) {
                        pend[e] = acc[e];
                        pendg[e] = gr[PT][e];
                        pendgf[e] = gfr[PT][e];
                    }
                } else {
                    store(r, acc, gr[PT], gfr[PT]);
                }
            }
        }
    };

#pragma unroll
    for (int j = 0; j < 3; ++j) load(pu[j], pg[j], pfv[j], pgf[j], n0 + j, false);

    // steady steps: n in [max(y0 + 2, 3), y1 - 1] (see `step`)
    const int s_lo = it.y0 + 2 > 3 ? it.y0 + 2 : 3;
    const int s_hi = it.y1 - 1;
    using Gen = std::false_type;
    using Std = std::true_type;
    // groups of three steps: the register slot of a row is fixed by its
    // position in the group
    // generic groups up to the first steady step of phase 0, steady groups,
    // then generic groups to the end
    const int ns = s_lo + (3 - (s_lo - n0) % 3) % 3;
    const int groups = s_hi >= ns + 2 ? (s_hi - ns + 1) / 3 : 0;
    if (groups > 0) {
        while (n < ns) {
            step(APhase<0>{}, Gen{});
            ++n;
            step(APhase<1>{}, Gen{});
            ++n;
            step(APhase<2>{}, Gen{});
            ++n;
        }
        for (int k = 0; k < groups; ++k) {
            step(APhase<0>{}, Std{});
            ++n;
            step(APhase<1>{}, Std{});
            ++n;
            step(APhase<2>{}, Std{});
            ++n;
        }
    }
    while (true) {
        step(APhase<0>{}, Gen{});
        if (++n > nend) break;
        step(APhase<1>{}, Gen{});
        if (++n > nend) break;
        step(APhase<2>{}, Gen{});
        if (++n > nend) break;
    }

    // fixed-order butterfly over the wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) contrib += __shfl_xor(contrib, off);
    return contrib;
}

template <int C, bool DATA>
__global__ __launch_bounds__(kAdjBlock) void k_adj_stream(AdjArgs A) {
    // wave index, made visibly wave-uniform so the item bookkeeping is scalar
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t per_plane = (int64_t)A.nseg * A.nstrip;
    const int64_t total = A.n * per_plane;
    const int64_t item = xcd_remap(blockIdx.x, gridDim.x) * kAdjWaves + wv;
    if (item >= total) return;
    const int p = (int)(item / per_plane);
    const int rem = (int)(item - (int64_t)p * per_plane);
    const int seg = rem / A.nstrip;
    const int strip = rem - seg * A.nstrip;
    const int H = (int)A.h, W = (int)A.w;

    AdjItem it;
    const int64_t off = (int64_t)p * A.ps;
    it.u = A.u + off;
    it.f = DATA ? A.f + off : nullptr;
    it.g = A.g + off;
    it.g_prev = A.g_prev + off;
    it.g_f = (DATA && A.g_f) ? A.g_f + off : nullptr;
    it.ld = (int)A.ld;
    it.H = H;
    it.W = W;
    const int hb = halo_cols(C, 2), step = 64 * C - 2 * hb;
    it.x0 = strip * step - hb;
    it.ox0 = strip * step;
    it.ox1 = it.ox0 + step < W ? it.ox0 + step : W;
    it.y0 = seg * A.R;
    it.y1 = it.y0 + A.R < H ? it.y0 + A.R : H;
    const float lam = (DATA && A.lam) ? A.lam[p] : 0.0f;
    const Coef cf = make_coef(lam, A.dt, DATA);
    it.delta = cf.delta;
    it.lam = lam;
    it.keep = DATA ? 1.0f - cf.delta : 1.0f;
    it.coef = DATA ? cf.delta * cf.lam12 : cf.delta12;
    it.dlam_default = !(A.dt > 0.0f);
    it.gf_first = A.gf_first != 0;
    it.gf_fold = DATA && it.g_f && A.gf_fold != 0;
    const bool edge = it.x0 < 0 || it.x0 + 64 * C > W;
    float c;
    if (edge) c = run_adj<C, DATA, true, false>(it);
    else if (A.vec) c = run_adj<C, DATA, false, true>(it);
    else c = run_adj<C, DATA, false, false>(it);
    if (DATA && A.part && (threadIdx.x & 63) == 0) A.part[(int64_t)A.slot * total + item] = c;
}

// The lambda gradient in two launches.  k_lam_slot_sums: one block per
// (step slot j, plane p) forms the slot's fixed-order sum over the plane's
// work items (per thread in item order, then a fixed tree over the 256
// threads) into sums[p * steps + j].  k_lam_accumulate: per plane,
// g_lam[p] += the slot sums from the last slot to the first, one addition
// at a time, starting from zero instead of g_lam[p] for the first group of
// a backward pass (0 + x = x exactly, so no separate clearing launch).  Every slot is reduced at once, so the launch fills the device
// instead of running one block per plane.
__global__ __launch_bounds__(256) void k_lam_slot_sums(const float* __restrict__ part, int64_t total,
                                                       int64_t per_plane, int steps,
                                                       float* __restrict__ sums) {
    const int j = blockIdx.x, p = blockIdx.y;
    __shared__ float red[256];
    const float* q = part + (int64_t)j * total + (int64_t)p * per_plane;
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < per_plane; i += 256) s += q[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[(int64_t)p * steps + j] = red[0];
}

__global__ __launch_bounds__(256) void k_lam_accumulate(const float* __restrict__ sums, int steps,
                                                        int64_t n, int first,
                                                        float* __restrict__ g_lam) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    float acc = first ? 0.0f : g_lam[p];
    for (int j = steps - 1; j >= 0; --j) acc += sums[p * steps + j];
    g_lam[p] = acc;
}

int adj_strip_count(int W, int C) {
    const int step = 64 * C - 2 * halo_cols(C, 2);
    return (W + step - 1) / step;
}

int adj_rows(int64_t n, int64_t h, int64_t w, int C) {
    // about 8K work items (several rounds of waves on 256 CUs), 16..128 rows
    const int64_t rows_total = n * h * adj_strip_count((int)w, C);
    int R = 16;
    while (R < 128 && rows_total / R > 8192) R *= 2;
    return R;
}

int64_t adj_items(int64_t n, int64_t h, int64_t w, int C) {
    return n * seg_count((int)h, adj_rows(n, h, w, C)) * adj_strip_count((int)w, C);
}

using AdjFn = void (*)(AdjArgs);

hipError_t launch_adjoint_step(const AdjArgs& a, hipStream_t st) {
    const bool data = a.f != nullptr;
    AdjFn fn = nullptr;
    switch (a.C) {
        case 1: fn = data ? k_adj_stream<1, true> : k_adj_stream<1, false>; break;
        case 2: fn = data ? k_adj_stream<2, true> : k_adj_stream<2, false>; break;
        case 4: fn = data ? k_adj_stream<4, true> : k_adj_stream<4, false>; break;
        default: return hipErrorInvalidValue;
    }
    const int64_t total = a.n * (int64_t)a.nseg * a.nstrip;
    const int64_t blocks = (total + kAdjWaves - 1) / kAdjWaves;
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(kAdjBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_lambda_reduce(const float* part, int steps, int64_t total, int64_t per_plane,
                                int64_t n, bool first, float* g_lam, float* sums, hipStream_t st) {
    if (steps < 1 || n < 1 || n > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_lam_slot_sums, dim3((unsigned)steps, (unsigned)n), dim3(256), 0, st, part,
                       total, per_plane, steps, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lam_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sums,
                       steps, n, first ? 1 : 0, g_lam);
    return hipGetLastError();
}

}  // namespace wmc
