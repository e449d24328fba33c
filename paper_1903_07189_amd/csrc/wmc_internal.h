// wmc_internal.h -- declarations shared by the host side (wmc_api.cpp) and the
// kernels (wmc_stream.hip, wmc_adjoint.hip) of libwmc.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <string>

#include "wmc.h"

namespace wmc {

// ---------------------------------------------------------------------------
// Work decomposition of the streaming kernel.
//
// One wave processes one work item: a vertical strip of 64*C columns (C per
// lane) of one plane, streamed top to bottom over a segment of R output
// rows.  Inside the wave the rows of T consecutive Jacobi sweeps are kept in
// registers as a pipeline (sweep k lags sweep k-1 by one row), so the wave
// reads U and f once and writes U once per T sweeps.
//
// Strips overlap by a halo of round_up(T, C) columns on each side; strip j
// loads columns [j*(64C - 2*halo), j*(64C - 2*halo) + 64C) and owns the
// output columns between the halos.  The first strip starts at column 0 and
// the last one reaches column W-1, where the image border is exact, so their
// outer halos are output too.  Segments overlap by T rows (recomputed).
// ---------------------------------------------------------------------------
__host__ __device__ inline int halo_cols(int C, int T) { return ((T + C - 1) / C) * C; }

__host__ __device__ inline int strip_count(int W, int C, int T) {
    const int width = 64 * C, step = width - 2 * halo_cols(C, T);
    if (W <= width) return 1;
    return 1 + (W - width + step - 1) / step;
}

__host__ __device__ inline int seg_count(int H, int R) { return (H + R - 1) / R; }

// Rows per work item for a launch of equal one-wave items, `cols` columns of
// items (strips x planes), each covering R rows out of h: the largest R whose
// item count fills whole rounds of the `slots` resident waves (k = 1, 2, ...),
// at least rmin.  Items just past a multiple of the slots would cost a
// nearly empty extra round.
inline int fill_rows(int64_t cols, int64_t h, int64_t slots, int rmin, int rmax) {
    if (slots < 1) slots = 1;
    for (int64_t k = 1; k <= 64; ++k) {
        const int64_t nseg = (k * slots) / (cols > 0 ? cols : 1);
        if (nseg < 1) continue;
        const int64_t R = (h + nseg - 1) / nseg;
        if (R < rmin) break;
        if (R <= rmax) return (int)R;
    }
    return rmin < h ? rmin : (int)h;
}

// Resident waves of a kernel launched with `block` threads (occupancy API x CUs).
int64_t kernel_slots(const void* fn, int block, size_t dyn_lds);

// One image (all its channels) as seen by the kernels.
struct ImageDesc {
    const float* src0;  // state read by a launch with src_sel == 0
    const float* f;     // data term (null: curvature flow / compute)
    float* bufA;        // selectable buffers (dst_sel/src_sel 1 and 2)
    float* bufB;
    uint8_t* amap;      // selection map (argmin variant only)
    const float* dsrc0; // l1 mode: dual state read with src_sel == 0 (null: zero)
    float* dA;          // l1 mode: dual buffers paired with bufA / bufB
    float* dB;
    int64_t ld, ps;     // row / plane stride, elements
    int32_t H, W;
    int32_t channels;
    int32_t lam_index;  // channel c uses lam[lam_index + c*lam_stride]
    int32_t lam_stride;
    int32_t nstrip, nseg;
    int32_t vec;        // 1: every row start of every buffer is 4C-byte aligned
    int64_t item_base;  // index of the image's first work item in the launch
};

struct LaunchArgs {
    const float* lam;  // device lambda array (may be null in flow/compute mode)
    float dt;          // > 0: step size, <= 0: default
    int32_t src_sel;   // 0: src0, 1: bufA, 2: bufB
    int32_t dst_sel;   // 1: bufA, 2: bufB
    int32_t R;         // output rows per work item
    float alpha;       // l1 mode: dual bound
    // trajectory launches (k_stream_traj): the state after sweep k (1 <= k < T)
    // is also stored to traj[k-1] (a plane set with the layout of the image),
    // or not at all where traj[k-1] is null; traj_in, if set, receives the
    // launch's input state (sweep 0) the same way (vector-only builds only)
    float* traj[3];
    float* traj_in;
};

constexpr int kTrajMaxT = 4;  // trajectory launches exist for T = 2, 3, 4

enum { kModeCompute = 0, kModeData = 1, kModeFlow = 2, kModeL1 = 3 };

// Host-side launchers (wmc_stream.hip).  Return a hipError_t.
bool stream_variant_exists(int C, int T, int mode, bool argmin);
// A launch of T sweeps that also stores the states after sweeps 1..T-1 where
// a.traj[k-1] is set (data and flow modes, T <= kTrajMaxT).
hipError_t launch_stream_traj(int C, int T, int mode, const ImageDesc& d, const LaunchArgs& a,
                              hipStream_t st);
hipError_t launch_stream_single(int C, int T, int mode, bool argmin, const ImageDesc& d,
                                const LaunchArgs& a, hipStream_t st);
// One flat launch over the items of many images; owner[i] = image of item i.
hipError_t launch_stream_batched(int C, int T, int mode, const ImageDesc* dtable,
                                 const int32_t* owner, int64_t total_items, const LaunchArgs& a,
                                 hipStream_t st);
int stream_blocks_per_cu(int C, int T, int mode);
// Occupancy of a single-launch variant; vonly: the vector-only build that a
// launch whose strips all qualify uses (vector_only).
int stream_single_blocks_per_cu(int C, int T, int mode, bool argmin, bool vonly = false);
// Whether every strip of a launch over image d with C columns per lane moves
// its rows with vector accesses: aligned rows (d.vec), at least two strips,
// the last strip starting at a multiple of C.
bool vector_only(const ImageDesc& d, int C);
int stream_traj_blocks_per_cu(int C, int T, int mode, bool vonly = false);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_copy_planes(const float* src, float* dst, int64_t n, int64_t h, int64_t w,
                              int64_t ld, int64_t ps, hipStream_t st);
hipError_t launch_add_planes(const float* src, float* dst, int64_t n, int64_t h, int64_t w,
                             int64_t ld, int64_t ps, hipStream_t st);
hipError_t launch_selftest(int* out_flags, hipStream_t st);

// Adjoint launchers (wmc_adjoint.hip).
struct AdjArgs {
    const float* u;     // U^t (plane set)
    const float* f;     // data term or null (flow)
    const float* g;     // dL/dU^{t+1}
    float* g_prev;      // dL/dU^t (out)
    float* g_f;         // dL/df accumulator (data mode) or null
    float* part;        // dL/dlam partial sums, [slot][item] (data mode) or null
    const float* lam;
    float dt;
    int64_t n, h, w, ld, ps;
    int32_t C;          // columns per lane: 1, 2 or 4
    int32_t R;          // rows per work item
    int32_t nstrip, nseg;
    int32_t vec;        // 1: all row starts 4C-byte aligned
    int32_t slot;       // step slot of `part`
    int32_t gf_first;   // 1: the first adjoint step, g_f holds nothing yet (taken as zero)
    int32_t gf_fold;    // 1: the last step of a solve from U^0 = f: g_f += g_prev as well
};
int adj_strip_count(int W, int C);
int adj_rows(int64_t n, int64_t h, int64_t w, int C);
int64_t adj_items(int64_t n, int64_t h, int64_t w, int C);
hipError_t launch_adjoint_step(const AdjArgs& a, hipStream_t st);
// Adds the lambda partial sums of `steps` step slots (slot j at part +
// j * total, plane p's items at p * per_plane) into g_lam, the last slot
// first; with `first` the sum starts from zero and g_lam is not read.
// `sums` holds n * steps floats of scratch.
hipError_t launch_lambda_reduce(const float* part, int steps, int64_t total, int64_t per_plane,
                                int64_t n, bool first, float* g_lam, float* sums, hipStream_t st);

// Learnable half-window layer (wmc_layer.hip).
int64_t layer_part_floats(int64_t n, int64_t h, int64_t w, int K);
hipError_t launch_layer_forward(const float* u, const float* w, int K, float* out, uint8_t* sel,
                                int64_t n, int64_t h, int64_t wd, int64_t ld, int64_t ps,
                                hipStream_t st);
hipError_t launch_layer_backward(const float* u, const float* w, int K, const uint8_t* sel,
                                 const float* g, float* g_u, float* part, float* g_w, int64_t n,
                                 int64_t h, int64_t wd, int64_t ld, int64_t ps, hipStream_t st);

// 3-D volumes (wmc_3d.hip).  amap: null, or the selection map (1 byte per
// voxel, the layout of the volumes).
hipError_t launch_stream3d(const float* u, const float* f, float* out, const float* lam, float dt,
                           int mode, int64_t n, int64_t d, int64_t h, int64_t w, int64_t ld,
                           int64_t ss, int64_t vs, hipStream_t st, uint8_t* amap = nullptr);
// Adjoint of one 3-D step: the selection pass (selection map, dL/df, the
// dL/dlam partial sum of each of adjsel3_items() work items at
// part + slot * items) and the gather of dL/dU^t (with g_f set, dL/dU^t is
// also added into it).
int64_t adjsel3_items(int64_t n, int64_t d, int64_t h, int64_t w);
hipError_t launch_adjsel3d(const float* u, const float* f, const float* g, float* g_f, uint8_t* sel,
                           float* part, int slot, bool gf_first, const float* lam, float dt,
                           int64_t n, int64_t d, int64_t h, int64_t w, int64_t ld, int64_t ss,
                           int64_t vs, hipStream_t st);
hipError_t launch_adjgather3d(const float* g, const uint8_t* sel, float* g_prev, float* g_f,
                              const float* lam, float dt, bool data, int64_t n, int64_t d, int64_t h,
                              int64_t w, int64_t ld, int64_t ss, int64_t vs, hipStream_t st);

// Auxiliary kernels (wmc_aux.hip).
hipError_t launch_fd(const float* u, float* out, int64_t n, int64_t h, int64_t w, int64_t ld,
                     int64_t ps, float dt, float eps, bool flow, hipStream_t st);

// Streaming bandwidth probe (wmc_probe.hip): o = a, or o = a + b with `add`,
// over n floats (n a multiple of 4, 16-byte aligned); `nt` = non-temporal.
hipError_t launch_bw_probe(bool add, bool nt, const float* a, const float* b, float* o,
                           int64_t n, hipStream_t st);

// Sets the calling thread's wmc_last_error() message and returns `code`.
int report_error(int code, const std::string& msg);

// Host side of wmc_solve (wmc_api.cpp).  `noalloc`: the static-scratch entry
// point's mode -- no checkpoints, no tuning search, no graph, and `ws` is the
// scratch of ws_bytes (WMC_EINVAL if one plane set does not fit).
int solve_impl(const float* f, const float* u0, float* u_out, const float* lam, int iters,
               float dt, float* ckpt, int ckpt_every, const wmc_tuning* tune, void* ws,
               size_t ws_bytes, wmc_shape s, void* stream, bool noalloc);

}  // namespace wmc
