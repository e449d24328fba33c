// wmc_device.hpp -- per-pixel arithmetic of the Half Laplace Operator shared by
// every GPU kernel of libwmc (gfx950, wave64).
//
// All kernels evaluate a pixel through the functions in this file, with the
// same FP32 operations in the same order, so that fused, tiled, batched and
// single-step paths produce bitwise identical results.
//
// Formulation (Sec. 4.2, eqs. (conv)/(act)): with integer weights c_i = 12 h_i,
// the eight responses S_i = 12 d_i of the printed kernels split into an even
// part A (12 times k4 of eq. (kernel3)) and odd parts:
//   S1 = A + E1, S2 = A + E2, S3 = A - E1, S4 = A - E2,
//   S5 = A + E5, S6 = A + E6, S7 = A - E5, S8 = A - E6,
// because opposite half windows are mirror images (h_i + h_i' = 2 k4 off the
// centre).  Per image row and pixel, with l, m, r the left/centre/right
// values of that row:
//   a = l + 2m,   s = l + 2m + r,   q = l - r.
// For a pixel with rows t (above), m (own), b (below):
//   A  = s_t + 2 s_m + s_b - 16 c          ([1 2 1; 2 -12 2; 1 2 1])
//   E1 = q_t + 2 q_m + q_b                 ([1 0 -1; 2 0 -2; 1 0 -1])
//   E2 = s_t - s_b                         ([1 2 1; 0 0 0; -1 -2 -1])
//   E5 = a_t - a_b + q_b + 2 q_m           ([1 2 0; 2 0 -2; 0 -2 -1])
//   E6 = a_t - a_b - q_t - 2 q_m           ([0 2 1; -2 0 2; -1 -2 0])
// A row's (a, s, q) are computed once and reused by the three output rows
// that read it.  The selection is a left-to-right tournament in which the
// right operand wins only when strictly smaller in magnitude, which equals
// "first index of the minimum" over S1..S8.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wmc {

constexpr int kWave = 64;

// Maps blockIdx.x so that the blocks the hardware places on one XCD (it deals
// blocks round-robin over the 8 XCDs) process one contiguous range of work
// items: neighbouring strips then share halo rows in that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t G) {
    const int64_t q = G / 8, r = G % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// Global memory access with a wave-uniform row pointer and a 32-bit per-lane
// byte offset, so that the loads and stores use the scalar-base addressing
// form (no 64-bit address arithmetic per lane).
template <class V>
__device__ __forceinline__ V ld_at(const float* row, uint32_t col) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(row) + col * 4u);
}
template <class V>
__device__ __forceinline__ void st_at(float* row, uint32_t col, V v) {
    *reinterpret_cast<V*>(reinterpret_cast<char*>(row) + col * 4u) = v;
}

// Lane L receives `src` of lane L-1; lane 0 keeps `old` (DPP wave_shr:1 with
// bound_ctrl off).  Passing a lane's own value as `old` makes lane 0 see its
// own value, i.e. the replicate border when lane 0 holds image column 0.
__device__ __forceinline__ float from_lower_lane(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x138, 0xF, 0xF, false));
}

// Lane L receives `src` of lane L+1; lane 63 keeps `old` (DPP wave_shl:1).
__device__ __forceinline__ float from_upper_lane(float old, float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src),
                                                      0x130, 0xF, 0xF, false));
}

// Lane L receives `src` of lane L-1 (L+1); the edge lane receives 0.  With
// no old value to preserve, the compiler can fold these shifts into the
// arithmetic that consumes them (DPP source operands).
__device__ __forceinline__ float from_lower_lane_or_zero(float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float from_upper_lane_or_zero(float src) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(src), 0x130, 0xF, 0xF, true));
}

// Per-row quantities of C consecutive columns held by one lane; d is the
// dual variable of the l1 iteration (unused by the other modes).
template <int C>
struct RowQ {
    float a[C], s[C], q[C], c[C], d[C];
};

// Builds the row quantities from the lane's C centre values.  The outer
// neighbours come from the adjacent lanes.  With RCLAMP, the element whose
// column is the last image column (flag in `last`) uses itself as its right
// neighbour (replicate border inside the wave).
template <int C, bool RCLAMP>
__device__ __forceinline__ void make_row(const float (&m)[C], const bool (&last)[C], RowQ<C>& r) {
    const float lft = from_lower_lane(m[0], m[C - 1]);
    const float rgt = from_upper_lane(m[C - 1], m[0]);
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const float l = (e == 0) ? lft : m[e - 1];
        float rr = (e == C - 1) ? rgt : m[e + 1];
        if (RCLAMP) rr = last[e] ? m[e] : rr;
        const float a = __builtin_fmaf(2.0f, m[e], l);
        r.a[e] = a;
        r.s[e] = a + rr;
        r.q[e] = l - rr;
        r.c[e] = m[e];
    }
}

// make_row for a strip whose wave-edge lanes (0 and 63) are halo lanes whose
// results are never stored: their missing neighbour may be zero.  Same
// values as make_row<C, false> on every other lane (2m is exact, so l + 2m
// rounds as fma(2, m, l)).
template <int C>
__device__ __forceinline__ void make_row_inner(const float (&m)[C], RowQ<C>& r) {
#pragma unroll
    for (int e = 0; e < C; ++e) {
        const float l = (e == 0) ? from_lower_lane_or_zero(m[C - 1]) : m[e - 1];
        const float rr = (e == C - 1) ? from_upper_lane_or_zero(m[0]) : m[e + 1];
        const float a = (e == 0) ? l + 2.0f * m[e] : __builtin_fmaf(2.0f, m[e], l);
        r.a[e] = a;
        r.s[e] = a + rr;
        r.q[e] = l - rr;
        r.c[e] = m[e];
    }
}

__device__ __forceinline__ float pick(float a, float b) {
    return (__builtin_fabsf(b) < __builtin_fabsf(a)) ? b : a;
}

struct Odd {
    float A, E1, E2, E5, E6;
};

__device__ __forceinline__ Odd parts(float ta, float ts, float tq, float ms, float mq, float mc,
                                     float ba, float bs, float bq) {
    Odd o;
    o.E2 = ts - bs;
    const float B = __builtin_fmaf(2.0f, ms, ts + bs);
    o.A = __builtin_fmaf(-16.0f, mc, B);
    // E1, E5 and E6 share 2 q_m + q_b and 2 q_m + q_t: ten operations for
    // the five parts instead of eleven
    const float yb = __builtin_fmaf(2.0f, mq, bq);
    const float yt = __builtin_fmaf(2.0f, mq, tq);
    const float da = ta - ba;
    o.E1 = tq + yb;
    o.E5 = da + yb;
    o.E6 = da - yt;
    return o;
}

// Selected response S_m (x12 domain).
__device__ __forceinline__ float select_x12(const Odd& o) {
    const float w12 = pick(o.A + o.E1, o.A + o.E2);
    const float w34 = pick(o.A - o.E1, o.A - o.E2);
    const float w56 = pick(o.A + o.E5, o.A + o.E6);
    const float w78 = pick(o.A - o.E5, o.A - o.E6);
    return pick(pick(w12, w34), pick(w56, w78));
}

// Same tournament, also returning the 0-based index of the winner.
__device__ __forceinline__ float select_x12_idx(const Odd& o, int& idx) {
    float s[8] = {o.A + o.E1, o.A + o.E2, o.A - o.E1, o.A - o.E2,
                  o.A + o.E5, o.A + o.E6, o.A - o.E5, o.A - o.E6};
    float w[4];
    int wi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const bool r = __builtin_fabsf(s[2 * j + 1]) < __builtin_fabsf(s[2 * j]);
        w[j] = r ? s[2 * j + 1] : s[2 * j];
        wi[j] = r ? 2 * j + 1 : 2 * j;
    }
    const bool r1 = __builtin_fabsf(w[1]) < __builtin_fabsf(w[0]);
    const float x0 = r1 ? w[1] : w[0];
    const int i0 = r1 ? wi[1] : wi[0];
    const bool r2 = __builtin_fabsf(w[3]) < __builtin_fabsf(w[2]);
    const float x1 = r2 ? w[3] : w[2];
    const int i1 = r2 ? wi[3] : wi[2];
    const bool r3 = __builtin_fabsf(x1) < __builtin_fabsf(x0);
    idx = r3 ? i1 : i0;
    return r3 ? x1 : x0;
}

// Lane masks of the wave (bit L = lane L): a per-lane condition as a mask and
// back.  Logic on masks runs as scalar instructions.
__device__ __forceinline__ uint64_t lanes(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool in_mask(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// Same tournament, describing the winner by lane masks instead of an index:
// `half` (S5..S8), `second` (the E2 / E6 member of its half) and `neg`
// (S = A - E); winner index = 4 half + 2 neg + second.  Called with every
// lane of the wave active.
struct Pick {
    uint64_t half, second, neg;
};
__device__ __forceinline__ float select_x12_pick(const Odd& o, Pick& p) {
    const float s0 = o.A + o.E1, s1 = o.A + o.E2, s2 = o.A - o.E1, s3 = o.A - o.E2;
    const float s4 = o.A + o.E5, s5 = o.A + o.E6, s6 = o.A - o.E5, s7 = o.A - o.E6;
    const bool r0 = __builtin_fabsf(s1) < __builtin_fabsf(s0);
    const bool r1 = __builtin_fabsf(s3) < __builtin_fabsf(s2);
    const bool r2 = __builtin_fabsf(s5) < __builtin_fabsf(s4);
    const bool r3 = __builtin_fabsf(s7) < __builtin_fabsf(s6);
    const float w0 = r0 ? s1 : s0, w1 = r1 ? s3 : s2, w2 = r2 ? s5 : s4, w3 = r3 ? s7 : s6;
    const bool q0 = __builtin_fabsf(w1) < __builtin_fabsf(w0);
    const bool q1 = __builtin_fabsf(w3) < __builtin_fabsf(w2);
    const float x0 = q0 ? w1 : w0, x1 = q1 ? w3 : w2;
    const bool h = __builtin_fabsf(x1) < __builtin_fabsf(x0);
    const uint64_t R0 = lanes(r0), R1 = lanes(r1), R2 = lanes(r2), R3 = lanes(r3);
    const uint64_t Q0 = lanes(q0), Q1 = lanes(q1), Hm = lanes(h);
    p.half = Hm;
    p.neg = (Hm & Q1) | (~Hm & Q0);
    p.second = (Hm & ((Q1 & R3) | (~Q1 & R2))) | (~Hm & ((Q0 & R1) | (~Q0 & R0)));
    return h ? x1 : x0;
}

// Output modes of the streaming kernel.
enum Mode : int { kCompute = 0, kData = 1, kFlow = 2, kL1 = 3 };

// Per-plane coefficients of the update.
struct Coef {
    float delta;   // step size
    float lam12;   // lam / 12 (data and l1 modes)
    float delta12; // delta / 12 (flow mode)
    float alpha;   // dual bound (l1 mode)
    float ainv;    // 1 / alpha (l1 mode)
};

// U' = U + delta ((f - U) + lam H_d), H_d = S / 12.
__device__ __forceinline__ float update_data(float c, float f, float S, const Coef& k) {
    return __builtin_fmaf(k.delta, __builtin_fmaf(k.lam12, S, f - c), c);
}

// U' = U + delta H_d.
__device__ __forceinline__ float update_flow(float c, float S, const Coef& k) {
    return __builtin_fmaf(k.delta12, S, c);
}

// l1 fidelity (Sec. 5.3): r = U - f + d, d' = clamp(r, -alpha, alpha),
// U' = U + delta (lam H_d - (2 d' - d) / alpha).  Returns U', writes d'.
__device__ __forceinline__ float update_l1(float c, float f, float d, float S, const Coef& k,
                                           float& dn) {
    const float r = (c - f) + d;
    dn = __builtin_amdgcn_fmed3f(r, -k.alpha, k.alpha);
    const float t = __builtin_fmaf(2.0f, dn, -d);
    return __builtin_fmaf(k.delta, __builtin_fmaf(k.lam12, S, -k.ainv * t), c);
}

__device__ __forceinline__ float to_hd(float S) { return S * (1.0f / 12.0f); }

// Resolves the step size for one plane: dt > 0 as given, otherwise
// 1/(1+lam) with a data term and 1 for the flow.
__device__ __forceinline__ Coef make_coef(float lam, float dt, bool data) {
    Coef k;
    k.delta = dt > 0.0f ? dt : (data ? 1.0f / (1.0f + lam) : 1.0f);
    k.lam12 = lam / 12.0f;
    k.delta12 = k.delta / 12.0f;
    k.alpha = 0.0f;
    k.ainv = 0.0f;
    return k;
}

// l1 mode: dt > 0 as given, otherwise 1/(lam + 2/alpha), the largest step
// for which the update is a convex combination while the dual is unclipped.
__device__ __forceinline__ Coef make_coef_l1(float lam, float dt, float alpha) {
    Coef k;
    k.alpha = alpha;
    k.ainv = 1.0f / alpha;
    k.delta = dt > 0.0f ? dt : 1.0f / (lam + 2.0f / alpha);
    k.lam12 = lam / 12.0f;
    k.delta12 = k.delta / 12.0f;
    return k;
}

}  // namespace wmc
