/*
 * wmc.h -- C ABI of libwmc: the discrete weighted mean curvature ("Half Laplace
 * Operator") of Gong & Goksel, "Weighted Mean Curvature" (arXiv 1903.07189),
 * and the iterations it drives, on AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are planes of 32-bit floats.  A plane set is described by
 *   wmc_shape: n planes of h rows by w columns; element (p, y, x) lives at
 *   ptr[p*ps + y*ld + x] (ld >= w, ps >= (h-1)*ld + w when n > 1).  x is the
 *   column, y the row (downwards).  Every array passed together with one
 *   wmc_shape uses that same layout.
 * - All data pointers are device pointers owned by the caller; the library
 *   never frees them and never keeps them after the call returns (except as
 *   keys of its launch-graph cache, see wmc_release).  `lam` is a device array
 *   too, so a learned lambda needs no host round trip.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Calls only enqueue work: a kernel fault surfaces at the caller's next
 *   synchronisation, not in the return code.
 * - Every call returns WMC_OK or a negative status; wmc_last_error() gives a
 *   thread-local message for the last failure.  Arguments are validated on the
 *   host before anything is enqueued; a rejected call enqueues nothing.
 * - Border rule: pixels outside the image take the value of the nearest image
 *   pixel (replicate), the reading of the Neumann condition of Sec. 4.1.2.
 * - Selection rule: among the eight half-window responses the one of least
 *   magnitude wins; exact ties go to the lowest index in the printed order
 *   h_1..h_8 (Sec. 4.2, eq. (act)).
 * - Step size `dt`: dt > 0 is used as given; dt <= 0 selects the default,
 *   1/(1+lam) with a data term (each update is then a convex combination of
 *   f and the 3x3 neighbourhood) and 1 for the pure curvature flow.
 * - Arithmetic is FP32; results are bitwise independent of the tiling,
 *   temporal-blocking depth and batching chosen by the library.
 * - Non-finite inputs are not checked.  A NaN response never wins a strict
 *   comparison, but the selection is evaluated as a pairwise tournament, so
 *   near a NaN (or Inf minus Inf) input the chosen response is unspecified;
 *   for finite inputs the tournament and the rule above are the same.
 * - The library runs on gfx950 only (WMC_EUNSUPPORTED elsewhere).
 */
#ifndef WMC_H
#define WMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WMC_OK 0
#define WMC_EINVAL (-1)       /* bad pointer, shape, stride, overlap or count      */
#define WMC_EHIP (-2)         /* a HIP call failed (message has hipGetErrorString) */
#define WMC_ENOMEM (-3)       /* caller workspace smaller than the size query says */
#define WMC_EUNSUPPORTED (-4) /* current device is not gfx950                      */

typedef struct wmc_shape {
    int64_t n;  /* number of planes (>= 1)                  */
    int64_t h;  /* rows per plane (>= 1)                     */
    int64_t w;  /* columns per plane (>= 1)                  */
    int64_t ld; /* row stride in elements (>= w)             */
    int64_t ps; /* plane stride in elements                  */
} wmc_shape;

/* One image of an uneven batch: `channels` planes of h x w, each with row
 * stride ld and plane stride ps (same layout for u0, f and out).  All its
 * channels use lam[lam_index] (the paper smooths each colour channel
 * separately with one setting, Sec. 5.4). */
typedef struct wmc_image {
    const float* u0; /* initial state, NULL -> start from f             */
    const float* f;  /* data term, NULL -> pure curvature flow (needs u0) */
    float* out;      /* result U^iters                                    */
    int64_t h, w, ld, ps;
    int32_t channels;
    int32_t lam_index;
} wmc_image;

/* Launch shape of the fused solver.  Zero fields mean "choose". */
typedef struct wmc_tuning {
    int32_t cols;      /* columns per lane: 1, 2 or 4                              */
    int32_t tsteps;    /* Jacobi sweeps per tile residency: 1, 2, 3, 4, 6 or 8       */
    int32_t seg_rows;  /* output rows per work item (>= 1)                           */
    int32_t use_graph; /* 1: replay a cached hipGraph of the launch sequence, 0: no  */
} wmc_tuning;

/* ---------------------------------------------------------------------------
 * wmc_compute -- H_d(U): the Half Laplace Operator, Sec. 4.2 eqs. (conv) and
 * (act).  For every pixel the eight half-window responses d_i = h_i * U are
 * formed (kernels as printed, correlation, replicate border) and the response
 * of least magnitude is written to hw.  u and hw share layout s and must not
 * overlap.  Traffic: 4 B read + 4 B written per pixel.
 * ------------------------------------------------------------------------- */
int wmc_compute(const float* u, float* hw, wmc_shape s, void* stream);

/* ---------------------------------------------------------------------------
 * wmc_step -- one synchronous (Jacobi) update, every pixel from the same U^t:
 *   f != NULL:  U' = U + dt [ (f - U) + lam H_d(U) ]   gradient descent on
 *               1/2||U - f||^2 + lam R_area with -dR/dU ~ H^w and A = I
 *               (Sec. 5.2, Sec. 3.3);
 *   f == NULL:  U' = U + dt H_d(U)                     curvature flow,
 *               Sec. 3.5 eq. (MCF) (lam is ignored and may be NULL).
 * lam: device array of s.n values, plane p uses lam[p] (lam >= 0).
 * argmin_out: NULL, or a device byte map (layout s, 1 byte per element)
 * receiving the 0-based index of the selected half window at every pixel.
 * u_out must not overlap u, f or argmin_out.  12 B/pixel with f, 8 B without.
 * ------------------------------------------------------------------------- */
int wmc_step(const float* u, const float* f, float* u_out, const float* lam, float dt,
             uint8_t* argmin_out, wmc_shape s, void* stream);

/* Bytes of workspace wmc_solve needs (one extra plane set,
 * wmc_set_stride(s) floats). */
size_t wmc_solve_workspace(wmc_shape s);

/* Elements between consecutive plane sets of a checkpoint buffer: n*ps, or
 * (n-1)*ps + (h-1)*ld + w if that is larger (0 for an invalid shape). */
int64_t wmc_set_stride(wmc_shape s);

/* Number of checkpoint plane sets a solve of `iters` steps stores with
 * checkpoints every `ckpt_every` steps: ceil(iters / ckpt_every). */
int64_t wmc_num_checkpoints(int iters, int ckpt_every);

/* ---------------------------------------------------------------------------
 * wmc_solve -- `iters` applications of wmc_step, starting from u0 (NULL ->
 * f), result in u_out.  The library fuses several sweeps per pass over
 * memory (temporal blocking) and replays the launch sequence as a cached
 * hipGraph; the result is bitwise the one of `iters` separate wmc_step calls.
 * ckpt: NULL, or a device buffer of wmc_num_checkpoints(iters, ckpt_every)
 * plane sets (plane set j at ckpt + j*wmc_set_stride(s), layout s) receiving
 * U^{j*ckpt_every} -- the states wmc_backward restarts from.
 * tune: NULL -> the autotuner's choice for this shape (cached), else used as
 * given (zero fields filled in).  ws: device workspace of at least
 * wmc_solve_workspace(s) bytes.  u_out must not overlap u0, f, ckpt or ws.
 * iters == 0 copies u0 (or f) to u_out.
 * ------------------------------------------------------------------------- */
int wmc_solve(const float* f, const float* u0, float* u_out, const float* lam, int iters,
              float dt, float* ckpt, int ckpt_every, const wmc_tuning* tune, void* ws,
              size_t ws_bytes, wmc_shape s, void* stream);

/* The launch shape wmc_solve(f, u0, ..., tune = NULL) uses for this shape:
 * the cached autotuner result, or a fresh search timed on ws (which it may
 * overwrite; nothing else is written).  Arguments as for wmc_solve.  With
 * ws_bytes >= 2 * wmc_solve_workspace(s) + 256 the search's launches
 * ping-pong between two plane sets in ws, as the solve does (the timings
 * then match the solve's more closely); with less they read U from u0 (or
 * f). */
int wmc_solve_tuning(const float* f, const float* u0, const float* lam, float dt, void* ws,
                     size_t ws_bytes, wmc_shape s, wmc_tuning* out, void* stream);

/* ---------------------------------------------------------------------------
 * wmc_solve_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same solve as wmc_solve without checkpoints (same kernels,
 * bitwise the same result), with its ping-pong state in a static device
 * array of WMC_NOALLOC_SCRATCH_BYTES that the library holds on every device
 * it runs on until the process ends, instead of a caller workspace.  It calls
 * no hipMalloc / hipFree, captures no graph and runs no tuning search: the
 * launch shape is `tune` if complete, else the autotuner's cached choice for
 * this shape (wmc_solve_tuning), else the default.  Arguments as for
 * wmc_solve; the caller owns f, u0, u_out and lam.
 * Errors: WMC_EINVAL (as wmc_solve, and when iters >= 2 and one plane set,
 * wmc_set_stride(s) floats, exceeds WMC_NOALLOC_SCRATCH_BYTES; nothing is
 * enqueued then), WMC_EHIP.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams or threads) race
 * and give wrong results.  Each launch writes the whole plane set it hands
 * to the next, so the array needs no clearing between calls.
 * ------------------------------------------------------------------------- */
#define WMC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int wmc_solve_noalloc(const float* f, const float* u0, float* u_out, const float* lam, int iters,
                      float dt, const wmc_tuning* tune, wmc_shape s, void* stream);

/* Bytes of workspace wmc_solve_l1 needs (two extra plane sets). */
size_t wmc_l1_workspace(wmc_shape s);

/* ---------------------------------------------------------------------------
 * wmc_solve_l1 -- the l1-fidelity model min ||U - f||_1 + lam R_area(U) of
 * Sec. 5.3 (A = I) by its primal-dual iteration, fused and temporally blocked
 * like wmc_solve.  Per step, with r = U - f + d:
 *   d' = clamp(r, -alpha, alpha)          (the shrinkage b is eliminated)
 *   U' = U + dt [ lam H_d(U) - (2 d' - d) / alpha ]
 * dt <= 0 selects 1/(lam + 2/alpha), the largest step for which the update is
 * a convex combination while the dual is unclipped.  u0 NULL -> f, d0 NULL ->
 * 0.  Outputs: u_out = U^iters, d_out = d^iters (layout s).  lam: device
 * array of s.n values; alpha > 0.  ws: wmc_l1_workspace(s) bytes.
 * Outputs must not overlap inputs, each other or ws.  20 B/pixel per pass.
 * ------------------------------------------------------------------------- */
int wmc_solve_l1(const float* f, const float* u0, const float* d0, float* u_out, float* d_out,
                 const float* lam, float alpha, int iters, float dt, const wmc_tuning* tune,
                 void* ws, size_t ws_bytes, wmc_shape s, void* stream);

/* Bytes of workspace wmc_solve_batched needs for this batch. */
size_t wmc_batched_workspace(const wmc_image* imgs, int n_imgs);

/* ---------------------------------------------------------------------------
 * wmc_solve_batched -- wmc_solve for many images of different sizes at once:
 * every channel of every image gets `iters` updates (each image with its own
 * lam[lam_index], channels independent, Sec. 5.4).  All tiles of all images
 * form one work list, covered by one launch (one wave per item) per fused
 * block of sweeps; the launch sequence is captured once into a hipGraph and
 * replayed.
 * imgs: HOST array of n_imgs descriptors (device pointers inside).  Outputs
 * must not overlap any input or each other.  tune: NULL -> autotuned.
 * ------------------------------------------------------------------------- */
int wmc_solve_batched(const wmc_image* imgs, int n_imgs, const float* lam, int iters, float dt,
                      const wmc_tuning* tune, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * wmc_autotune -- times candidate launch shapes (columns per lane, sweeps
 * per residency, rows per work item) on this batch, using ws as scratch and
 * writing nothing else, and returns the fastest in *out: after untimed
 * launches that let the clocks rise, every candidate is timed on single
 * launches and the six fastest again as graph replays of at least 64
 * sweeps, which decide (the same search serves wmc_solve's shapes).  Results are cached in memory and in the JSON file named by the
 * environment variable WMC_TUNE_CACHE (default ~/.cache/wmc/tune.json),
 * keyed by device architecture and a size class of the batch.  The
 * environment variable WMC_TUNE=off|cached|force selects defaults only,
 * cached results or a fresh search.  Synchronises the stream.
 * ------------------------------------------------------------------------- */
int wmc_autotune(const wmc_image* imgs, int n_imgs, int iters, wmc_tuning* out, void* ws,
                 size_t ws_bytes, void* stream);

/* Bytes of workspace wmc_backward needs. */
size_t wmc_backward_workspace(wmc_shape s, int iters, int ckpt_every);

/* ---------------------------------------------------------------------------
 * wmc_backward -- reverse-mode derivative of L(U^iters) through a solve.
 * The paper leaves the gradient of the WMC regulariser open (end of Sec. 3);
 * this is the exact derivative of the update map of wmc_step with the
 * selected half window held at its forward value:
 *   dL/dU^t(y) = k dL/dU^{t+1}(y)
 *              + c sum_{x,o : clamp(x+o) = y} h_{m(x)}[o] dL/dU^{t+1}(x)
 * with k = 1 - dt, c = dt lam (data term) or k = 1, c = dt (flow),
 * dL/df += dt dL/dU^{t+1}, and dL/dlam_p summed over the plane (including
 * the dependence of the default dt = 1/(1+lam) on lam).
 * f, u0, lam, iters, dt, ckpt_every: exactly as passed to the wmc_solve that
 * produced `ckpt` (the checkpoints are restarted from and each segment of
 * ckpt_every steps is recomputed).  g_out: dL/dU^iters.
 * Outputs (device, layout s, overwritten):
 *   g_f   (data term only; NULL allowed) dL/df, including the path through
 *         U^0 = f when u0 == NULL;
 *   g_u0  (NULL allowed) dL/dU^0 when u0 != NULL (or in flow mode);
 *   g_lam (NULL allowed) n floats, dL/dlam_p.
 * Deterministic: the lambda sums use a fixed reduction order, no atomics.
 * ws: at least wmc_backward_workspace(s, iters, ckpt_every) bytes.
 * Requires s.ld < 2^31 (WMC_EINVAL otherwise).
 * ------------------------------------------------------------------------- */
int wmc_backward(const float* f, const float* u0, const float* lam, int iters, float dt,
                 const float* ckpt, int ckpt_every, const float* g_out, float* g_f, float* g_u0,
                 float* g_lam, void* ws, size_t ws_bytes, wmc_shape s, void* stream);

/* ---------------------------------------------------------------------------
 * The learnable half-window layer of Sec. 4.3: eq. (conv) with K learned 3x3
 * kernels in place of the eight printed ones, followed by the minimum-
 * magnitude activation of eq. (act):
 *   d_k(x) = sum_o w[k][o] Ub(x + o)     (correlation, replicate border Ub)
 *   sel(x) = first k attaining min_k |d_k(x)|,   out(x) = d_sel(x)(x).
 * w: device, K x 3 x 3 floats, [k][row][col], row 0 = the image row above
 * the pixel, col 0 = the column to its left (the printed kernels' layout);
 * 1 <= K <= 16.  With the eight printed kernels times 12 the layer is 12 H_d.
 * sel: uint8, same ld/ps layout as u (nullable in the forward; the backward
 * needs the forward's).
 *
 * wmc_layer_backward -- derivative with the selection held fixed (the layer
 * is linear in u and w for a fixed sel; ties are a null set):
 *   g_u(z)     = sum_{x, o: clamp(x + o) = z} w[sel(x)][o] g_out(x)
 *   g_w[k][o]  = sum_{x: sel(x) = k} g_out(x) Ub(x + o)
 * g_u and g_w are overwritten (either may be NULL).  g_w is reduced in a
 * fixed order: bitwise reproducible.  ws: wmc_layer_workspace(s, K) bytes
 * when g_w is requested.
 * ------------------------------------------------------------------------- */
size_t wmc_layer_workspace(wmc_shape s, int K);
int wmc_layer_forward(const float* u, const float* w, int K, float* out, uint8_t* sel,
                      wmc_shape s, void* stream);
int wmc_layer_backward(const float* u, const float* w, int K, const uint8_t* sel,
                       const float* g_out, float* g_u, float* g_w, void* ws, size_t ws_bytes,
                       wmc_shape s, void* stream);

/* ---------------------------------------------------------------------------
 * wmc_fd_compute -- the conventional discretisation of the continuous WMC of
 * eq. (rhs), H^w = Lap U - (U_y^2 U_yy + 2 U_x U_y U_xy + U_x^2 U_xx) /
 * (U_x^2 + U_y^2 + eps), with second-order central differences at unit
 * spacing and the replicate border: the "deriv" comparator of Sec. 5.4.  The
 * paper gives neither the stencil nor a guard; eps >= 0 makes the normal term
 * vanish where the gradient does (H^w then tends to the Laplacian).
 * wmc_fd_flow -- iters explicit curvature-flow steps U <- U + dt H^w_fd(U)
 * from u0 (ws: wmc_solve_workspace(s) bytes when iters >= 2).
 * Comparator kernels: one wave per strip of columns streaming down the rows
 * (one sweep per launch, not temporally blocked).
 * ------------------------------------------------------------------------- */
int wmc_fd_compute(const float* u, float* hw, float eps, wmc_shape s, void* stream);
int wmc_fd_flow(const float* u0, float* u_out, int iters, float dt, float eps, void* ws,
                size_t ws_bytes, wmc_shape s, void* stream);

/* ---------------------------------------------------------------------------
 * 3-D volumes.  The conclusion of the paper mentions the extension to 3-D
 * images without giving kernels; these entry points build them the way
 * Sec. 4.1 builds the 2-D ones: the tensor-product isotropic Laplacian
 * (s x s x s - 64 delta)/56, s = [1 2 1], reflected across each of the 9
 * mirror planes of the 3x3x3 window (normals e_x, e_y, e_z, e_x +- e_y,
 * e_x +- e_z, e_y +- e_z), one candidate per plane side, 18 in all (order:
 * plane 0..8, side n.o <= 0 first); the minimum-magnitude activation with
 * first-index ties; replicate border.
 *
 * wmc_shape3: n volumes of d x h x w; element (v, z, y, x) at
 * v*vs + z*ss + y*ld + x (row stride ld >= w, slice stride
 * ss >= (h-1)*ld + w, volume stride vs >= (d-1)*ss + (h-1)*ld + w when n > 1).
 *
 * wmc3_compute -- H(u) for every voxel.
 * wmc3_step    -- one Jacobi update: u_out = u + dt[(f - u) + lam H(u)]
 *                 (f NULL: u + dt H(u)); dt <= 0 selects 1/(1+lam) (data)
 *                 or 1 (flow); lam: device array of n values (data mode).
 *                 argmin_out: NULL, or a device byte map (layout s) that
 *                 receives the 0-based index of the selected half window
 *                 (2 j for the n_j.o <= 0 side of plane j, 2 j + 1 for the
 *                 other); it must not overlap u, f or u_out.
 * wmc3_solve   -- iters such updates from u0 (NULL: f); ws: one volume set
 *                 (wmc3_set_stride(s) floats) when iters >= 2.  ckpt (or
 *                 NULL): wmc_num_checkpoints(iters, ckpt_every) volume sets,
 *                 wmc3_set_stride(s) floats apart, receiving U^{j ckpt_every}
 *                 (the restart points of wmc3_backward); ckpt must not
 *                 overlap u_out, ws or the inputs.
 * Single sweeps per launch (no temporal blocking: the sweep issues its
 * vector instructions at nearly the full rate, so it is bound by the ALUs,
 * not by the bytes a fused launch would save); the same errors as the 2-D
 * entry points.
 * ------------------------------------------------------------------------- */
typedef struct {
    int64_t n, d, h, w, ld, ss, vs;
} wmc_shape3;

int wmc3_compute(const float* u, float* hw, wmc_shape3 s, void* stream);
int wmc3_step(const float* u, const float* f, float* u_out, const float* lam, float dt,
              uint8_t* argmin_out, wmc_shape3 s, void* stream);
size_t wmc3_solve_workspace(wmc_shape3 s);
/* Elements between consecutive volume sets of a checkpoint buffer: n*vs, or
 * the extent of the set if that is larger (0 for an invalid shape). */
int64_t wmc3_set_stride(wmc_shape3 s);
int wmc3_solve(const float* f, const float* u0, float* u_out, const float* lam, int iters,
               float dt, float* ckpt, int ckpt_every, void* ws, size_t ws_bytes, wmc_shape3 s,
               void* stream);

/* Bytes of workspace wmc3_backward needs. */
size_t wmc3_backward_workspace(wmc_shape3 s, int iters, int ckpt_every);

/* ---------------------------------------------------------------------------
 * wmc3_backward -- reverse-mode derivative of L(U^iters) through wmc3_solve,
 * the 3-D counterpart of wmc_backward (the paper leaves the gradient of the
 * regulariser open, end of Sec. 3, and mentions volumes only in Sec. 6): the
 * exact derivative of the update with the selected half window held at its
 * forward value,
 *   dL/dU^t(v) = k dL/dU^{t+1}(v)
 *              + c sum_{x,o : clamp(x+o) = v} w_{m(x)}[o] dL/dU^{t+1}(x)
 * (w the 18 half windows x56, centre -56; k = 1 - dt, c = dt lam / 56 with a
 * data term, k = 1, c = dt / 56 for the flow), dL/df += dt dL/dU^{t+1}, and
 * dL/dlam_v summed over the volume (with the dependence of the default
 * dt = 1/(1+lam) on lam).  f, u0, lam, iters, dt, ckpt, ckpt_every: exactly
 * as passed to the wmc3_solve that wrote ckpt (each segment is recomputed
 * from its checkpoint).  g_out: dL/dU^iters.  Outputs (device, layout s,
 * overwritten; each may be NULL): g_f (data term) dL/df including the path
 * through U^0 = f when u0 == NULL; g_u0 dL/dU^0; g_lam n floats.
 * Deterministic: fixed summation orders, no atomics; the gradients do not
 * depend on ckpt_every.  Errors: WMC_EINVAL (shapes, NULL checkpoints with
 * iters > 0, overlapping outputs), WMC_ENOMEM (ws smaller than
 * wmc3_backward_workspace), WMC_EHIP.
 * ------------------------------------------------------------------------- */
int wmc3_backward(const float* f, const float* u0, const float* lam, int iters, float dt,
                  const float* ckpt, int ckpt_every, const float* g_out, float* g_f, float* g_u0,
                  float* g_lam, void* ws, size_t ws_bytes, wmc_shape3 s, void* stream);

/* ---------------------------------------------------------------------------
 * wmc_workspace_bytes -- one query for every workspace size:
 *   WMC_OP_SOLVE, WMC_OP_FD_FLOW   wmc_solve_workspace(s)
 *   WMC_OP_SOLVE_L1                wmc_l1_workspace(s)
 *   WMC_OP_BACKWARD                wmc_backward_workspace(s, iters, ckpt_every)
 *   WMC_OP_LAYER_BACKWARD          wmc_layer_workspace(s, K = iters)
 * 0 for an invalid shape or op.  (The batched solver's size depends on its
 * image list: wmc_batched_workspace.)
 * ------------------------------------------------------------------------- */
enum {
    WMC_OP_SOLVE = 0,
    WMC_OP_SOLVE_L1 = 1,
    WMC_OP_BACKWARD = 2,
    WMC_OP_FD_FLOW = 3,
    WMC_OP_LAYER_BACKWARD = 4
};
size_t wmc_workspace_bytes(int op, wmc_shape s, int iters, int ckpt_every);

/* ---------------------------------------------------------------------------
 * wmc_bw_probe -- a measurement aid, no part of the method: the streaming
 * bandwidth the device achieves for the access pattern of an update, as the
 * ceiling the update kernels are judged against.  op WMC_PROBE_COPY: o = a
 * (one read, one write per float); WMC_PROBE_ADD: o = a + b (two reads, one
 * write, the single update's pattern).  flags: WMC_PROBE_NONTEMPORAL makes
 * every load and store non-temporal.  n floats, a positive multiple of 4;
 * a, b, o device pointers, 16-byte aligned, o not overlapping a or b (b
 * unused for a copy).  WMC_EINVAL on bad arguments (nothing enqueued).
 * ------------------------------------------------------------------------- */
enum { WMC_PROBE_COPY = 0, WMC_PROBE_ADD = 1 };
enum { WMC_PROBE_NONTEMPORAL = 1 };
int wmc_bw_probe(int op, const float* a, const float* b, float* o, int64_t n, int flags,
                 void* stream);

/* Checks on the current device that the wavefront lane shifts the kernels
 * rely on move data as expected; returns WMC_OK or WMC_EHIP/WMC_EUNSUPPORTED.
 * Synchronises the default stream. */
int wmc_selftest(void);

/* Thread-local description of the last failure ("" if none). */
const char* wmc_last_error(void);

/* Frees cached launch graphs, device-side work tables and tuning state. */
void wmc_release(void);

#ifdef __cplusplus
}
#endif

#endif /* WMC_H */
