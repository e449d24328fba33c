/*
 * wmc_oracle.c -- plain, slow, double-precision reference ("oracle") for the
 * discrete weighted mean curvature (WMC) of Gong & Goksel, "Weighted Mean
 * Curvature" (arXiv 1903.07189), and for the iterations it drives.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it (through oracle/__init__.py).  It
 * shares no code, header, table or constant with the HIP implementation.
 *
 * Everything is FP64, single threaded, scalar loops, written to be checked
 * against the paper by eye:
 *
 *   O1  replicate (half-sample symmetric) extension of the image by one
 *       pixel -- the Neumann condition of Sec. 4.1.2 and Sec. 3.3;
 *   O2  the eight half-window responses d_i = h_i * U, Sec. 4.2 eq. (conv),
 *       with the kernels exactly as printed there (kernel overlaid on the
 *       image as printed, top row = previous image row), evaluated in the
 *       "x12" domain S_i = 12 d_i so that all weights are integers;
 *   O3  m = first index i (printed order 1..8) attaining min_i |S_i|,
 *       Sec. 4.2 eq. (act);
 *   O4  H_d = S_m / 12;
 *   O5  one Jacobi update: data mode  U' = U + delta[(f - U) + lam H_d(U)]
 *       (gradient descent of Sec. 5.2 with A = I and -dR/dU ~ H^w),
 *       MCF mode U' = U + delta H_d(U)   (Sec. 3.5, eq. (MCF));
 *   O6  a solve = iters applications of O5 starting from u0 (default f);
 *   O7  diagnostic energies (eq. (wmcr) with q = 1, and eq. (areaReg));
 *   O8  the adjoint of O5 and of a K-step solve (the paper leaves the
 *       gradient of the regulariser to future work, end of Sec. 3, so this
 *       is the exact derivative of the piecewise-linear update map with the
 *       selection m held fixed);
 *   O9  "listing mode": the Appendix A function's semantics (true 2-D
 *       convolution, zero padding, its candidate order), for cross-checks;
 *   O10 the l1-fidelity primal-dual iteration of Sec. 5.3 (A = I);
 *   O11 the conventional finite-difference WMC of eq. (rhs) and its flow
 *       (the comparator of Sec. 5.4);
 *   O12 the learnable half-window layer of Sec. 4.3: K learned 3x3 kernels
 *       (eq. (conv) with the h_i replaced by learned weights) followed by the
 *       minimum-magnitude activation of eq. (act), and its derivative with
 *       respect to the input and the kernel weights;
 *   O13 the extension to 3-D volumes that the conclusion mentions (Sec. 6);
 *       the paper gives no kernels, so they are built the way Sec. 4.1 builds
 *       the 2-D ones (see O13 below);
 *   O14 the adjoint of the 3-D iteration, derived as O8 is for 2-D.
 *
 * Images are row-major H x W arrays of doubles, x = column, y = row
 * (downwards).  Functions never allocate more than O(H W) scratch.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Sec. 4.2: the eight half-window kernels h_1..h_8, times 12.
 * [i][r][c]: r = 0 is the printed top row (image row y-1), c = 0 the
 * printed left column (image column x-1). */
static const int K12[8][3][3] = {
    {{2, 2, 0}, {4, -12, 0}, {2, 2, 0}},  /* h1: left half window   */
    {{2, 4, 2}, {2, -12, 2}, {0, 0, 0}},  /* h2: top                */
    {{0, 2, 2}, {0, -12, 4}, {0, 2, 2}},  /* h3: right              */
    {{0, 0, 0}, {2, -12, 2}, {2, 4, 2}},  /* h4: bottom             */
    {{2, 4, 1}, {4, -12, 0}, {1, 0, 0}},  /* h5: top-left           */
    {{1, 4, 2}, {0, -12, 4}, {0, 0, 1}},  /* h6: top-right          */
    {{0, 0, 1}, {0, -12, 4}, {1, 4, 2}},  /* h7: bottom-right       */
    {{1, 0, 0}, {4, -12, 0}, {2, 4, 1}},  /* h8: bottom-left        */
};

static int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Copies the 12x kernel table out (8*3*3 ints) so tests can inspect it. */
void wmco_kernel_table(int* out) {
    memcpy(out, K12, sizeof(K12));
}

/* O1: Ubar(y, x) for -1 <= y <= H, -1 <= x <= W via index clamping. */
static double ubar(const double* U, int64_t H, int64_t W, int64_t y, int64_t x) {
    return U[clampi(y, 0, H - 1) * W + clampi(x, 0, W - 1)];
}

/* O2: the eight candidates at pixel (y, x), in the difference form
 * S_i = sum_{o != 0} c_i[o] (Ubar(x+o) - Ubar(x)); since the weights of
 * every h_i sum to zero this equals sum_o c_i[o] Ubar(x+o) exactly in real
 * arithmetic, and in FP64 it makes constant images give exactly 0. */
static void candidates_at(const double* U, int64_t H, int64_t W, int64_t y, int64_t x,
                          double S[8]) {
    double c = U[y * W + x];
    double nb[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) nb[r][q] = ubar(U, H, W, y + r - 1, x + q - 1) - c;
    for (int i = 0; i < 8; ++i) {
        double s = 0.0;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) {
                if (r == 1 && q == 1) continue;
                s += (double)K12[i][r][q] * nb[r][q];
            }
        S[i] = s;
    }
}

/* O3: first index (0-based) attaining the minimum magnitude (strict '<'). */
static int select_first_min(const double S[8]) {
    int m = 0;
    for (int i = 1; i < 8; ++i)
        if (fabs(S[i]) < fabs(S[m])) m = i;
    return m;
}

/* All eight candidates S_i (x12 domain) for every pixel: S[(y*W+x)*8 + i]. */
void wmco_candidates(const double* U, int64_t H, int64_t W, double* S) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) candidates_at(U, H, W, y, x, S + (y * W + x) * 8);
}

/* O2-O4: H_d(U).  m_out (nullable) receives the 0-based selection. */
void wmco_compute(const double* U, int64_t H, int64_t W, double* Hd, int8_t* m_out) {
    double S[8];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            candidates_at(U, H, W, y, x, S);
            int m = select_first_min(S);
            Hd[y * W + x] = S[m] / 12.0;
            if (m_out) m_out[y * W + x] = (int8_t)m;
        }
}

/* O5: one Jacobi step.  f == NULL selects MCF mode.  m_forced (nullable)
 * replays a given selection instead of O3 (entries < 0 mean "use O3");
 * m_out (nullable) records the selection actually used. */
void wmco_step(const double* U, const double* f, int64_t H, int64_t W, double lam,
               double delta, const int8_t* m_forced, double* Uout, int8_t* m_out) {
    double S[8];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t k = y * W + x;
            candidates_at(U, H, W, y, x, S);
            int m = (m_forced && m_forced[k] >= 0) ? m_forced[k] : select_first_min(S);
            double hd = S[m] / 12.0;
            if (f)
                Uout[k] = U[k] + delta * ((f[k] - U[k]) + lam * hd);
            else
                Uout[k] = U[k] + delta * hd;
            if (m_out) m_out[k] = (int8_t)m;
        }
}

/* O6: iters Jacobi steps from u0 (NULL -> f).  f == NULL is MCF mode and
 * then u0 must be given.  m_forced_all (nullable) holds iters selection maps
 * back to back (H*W each) to replay. */
void wmco_solve(const double* f, const double* u0, int64_t H, int64_t W, double lam,
                double delta, int iters, const int8_t* m_forced_all, double* Uout) {
    int64_t n = H * W;
    double* a = (double*)malloc(sizeof(double) * n);
    double* b = (double*)malloc(sizeof(double) * n);
    memcpy(a, u0 ? u0 : f, sizeof(double) * n);
    for (int t = 0; t < iters; ++t) {
        wmco_step(a, f, H, W, lam, delta, m_forced_all ? m_forced_all + (int64_t)t * n : NULL, b,
                  NULL);
        double* tmp = a;
        a = b;
        b = tmp;
    }
    memcpy(Uout, a, sizeof(double) * n);
    free(a);
    free(b);
}

/* O7: eq. (wmcr) with q = 1 plus the quadratic data term (f NULL -> no data
 * term): 1/2 sum (U-f)^2 + lam sum |H_d(U)|. */
double wmco_energy_wmc(const double* U, const double* f, int64_t H, int64_t W, double lam) {
    double e = 0.0, r = 0.0, S[8];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t k = y * W + x;
            if (f) e += 0.5 * (U[k] - f[k]) * (U[k] - f[k]);
            candidates_at(U, H, W, y, x, S);
            r += fabs(S[select_first_min(S)] / 12.0);
        }
    return e + lam * r;
}

/* O7: eq. (areaReg) discretised with forward differences (zero at the last
 * column / row, i.e. replicate extension), plus the quadratic data term. */
double wmco_energy_area(const double* U, const double* f, int64_t H, int64_t W, double lam) {
    double e = 0.0, r = 0.0;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t k = y * W + x;
            if (f) e += 0.5 * (U[k] - f[k]) * (U[k] - f[k]);
            double ux = (x + 1 < W) ? U[k + 1] - U[k] : 0.0;
            double uy = (y + 1 < H) ? U[k + W] - U[k] : 0.0;
            r += sqrt(1.0 + ux * ux + uy * uy);
        }
    return e + lam * r;
}

/* O9: Appendix A semantics.  The listing builds two base kernels (the
 * left half window scaled to centre -6 and the top-left one scaled to
 * centre -12), derives six more by left-right flip, transpose, up-down
 * flip and 180-degree rotation, applies each by true 2-D convolution with
 * zero padding ("same" size), and gathers the first-index minimum.  Here
 * the eight listing kernels are derived from the two base kernels by the
 * same geometric operations and applied as a convolution,
 * out(y,x) = sum_{r,q} k[r][q] * u(y - (r-1), x - (q-1)), zero outside. */
static void flip_lr(double k[3][3]) {
    for (int r = 0; r < 3; ++r) { double t = k[r][0]; k[r][0] = k[r][2]; k[r][2] = t; }
}
static void flip_ud(double k[3][3]) {
    for (int q = 0; q < 3; ++q) { double t = k[0][q]; k[0][q] = k[2][q]; k[2][q] = t; }
}
static void transpose3(double k[3][3]) {
    for (int r = 0; r < 3; ++r)
        for (int q = r + 1; q < 3; ++q) { double t = k[r][q]; k[r][q] = k[q][r]; k[q][r] = t; }
}

void wmco_listing_kernels(double out[8][3][3]) {
    const double base1[3][3] = {{1, 1, 0}, {2, -6, 0}, {1, 1, 0}};
    const double base2[3][3] = {{2, 4, 1}, {4, -12, 0}, {1, 0, 0}};
    double k[3][3];
    for (int slot = 0; slot < 8; ++slot) {
        const double (*b)[3] = slot < 4 ? base1 : base2;
        double scale = slot < 4 ? 6.0 : 12.0;
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) k[r][q] = b[r][q] / scale;
        switch (slot) {
            case 0: break;                              /* base1            */
            case 1: flip_lr(k); break;                  /* lr-flip          */
            case 2: transpose3(k); break;               /* transpose        */
            case 3: transpose3(k); flip_ud(k); break;   /* ud-flip of transpose */
            case 4: break;                              /* base2            */
            case 5: flip_lr(k); break;                  /* lr-flip          */
            case 6: flip_ud(k); break;                  /* ud-flip          */
            case 7: flip_lr(k); flip_ud(k); break;      /* 180 degrees      */
        }
        memcpy(out[slot], k, sizeof(k));
    }
}

void wmco_listing(const double* U, int64_t H, int64_t W, double* Hd, int8_t* m_out) {
    double ks[8][3][3];
    wmco_listing_kernels(ks);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            double d[8];
            for (int s = 0; s < 8; ++s) {
                double acc = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int q = 0; q < 3; ++q) {
                        int64_t yy = y - (r - 1), xx = x - (q - 1);
                        if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                        acc += ks[s][r][q] * U[yy * W + xx];
                    }
                d[s] = acc;
            }
            int m = select_first_min(d);
            Hd[y * W + x] = d[m];
            if (m_out) m_out[y * W + x] = (int8_t)m;
        }
}

/* O8: adjoint of one step (scatter-add form).  With m held fixed the step
 * is affine in (U, f):
 *   U'(x) = U(x) + delta[(f(x) - U(x)) + lam/12 sum_o c_m(x)[o] Ubar(x+o)]
 * where c[o] includes the centre weight -12 and Ubar(x+o) is the clamped
 * pixel.  Given gbar = dL/dU' this writes gU = dL/dU, adds delta*gbar into
 * gf (nullable) and adds dL/dlam into *glam (nullable).  When
 * delta_from_lam != 0 the step size is delta = 1/(1+lam) and its
 * derivative -delta^2 enters dL/dlam.  f == NULL is MCF mode
 * (U' = U + delta H_d, no lam).  m_forced as in wmco_step. */
void wmco_step_adjoint(const double* U, const double* f, int64_t H, int64_t W, double lam,
                       double delta, int delta_from_lam, const int8_t* m_forced,
                       const double* gbar, double* gU, double* gf, double* glam) {
    int64_t n = H * W;
    double S[8];
    double coef = f ? delta * lam / 12.0 : delta / 12.0;
    double keep = f ? 1.0 - delta : 1.0;
    for (int64_t k = 0; k < n; ++k) gU[k] = keep * gbar[k];
    double gl = 0.0;
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t k = y * W + x;
            candidates_at(U, H, W, y, x, S);
            int m = (m_forced && m_forced[k] >= 0) ? m_forced[k] : select_first_min(S);
            for (int r = 0; r < 3; ++r)
                for (int q = 0; q < 3; ++q) {
                    int64_t yy = clampi(y + r - 1, 0, H - 1), xx = clampi(x + q - 1, 0, W - 1);
                    gU[yy * W + xx] += coef * (double)K12[m][r][q] * gbar[k];
                }
            if (f) {
                double hd = S[m] / 12.0;
                if (gf) gf[k] += delta * gbar[k];
                double du_dlam = delta * hd;
                if (delta_from_lam) du_dlam += -delta * delta * ((f[k] - U[k]) + lam * hd);
                gl += gbar[k] * du_dlam;
            }
        }
    if (glam) *glam += gl;
}

/* O8: adjoint of a K-step solve.  All K states are kept (small images
 * only).  Outputs: gu0 = dL/dU^0 (nullable), gf = dL/df through the data
 * term only (nullable; if the solve started from u0 = f the caller adds
 * gu0), glam = dL/dlam (nullable).  UK (nullable) receives U^K. */
void wmco_solve_adjoint(const double* f, const double* u0, int64_t H, int64_t W, double lam,
                        double delta, int delta_from_lam, int K, const int8_t* m_forced_all,
                        const double* gK, double* gu0, double* gf, double* glam, double* UK) {
    int64_t n = H * W;
    double* states = (double*)malloc(sizeof(double) * n * (size_t)(K + 1));
    memcpy(states, u0 ? u0 : f, sizeof(double) * n);
    for (int t = 0; t < K; ++t)
        wmco_step(states + (int64_t)t * n, f, H, W, lam, delta,
                  m_forced_all ? m_forced_all + (int64_t)t * n : NULL,
                  states + (int64_t)(t + 1) * n, NULL);
    if (UK) memcpy(UK, states + (int64_t)K * n, sizeof(double) * n);
    double* g = (double*)malloc(sizeof(double) * n);
    double* g2 = (double*)malloc(sizeof(double) * n);
    memcpy(g, gK, sizeof(double) * n);
    if (gf) memset(gf, 0, sizeof(double) * n);
    double gl = 0.0;
    for (int t = K - 1; t >= 0; --t) {
        wmco_step_adjoint(states + (int64_t)t * n, f, H, W, lam, delta, delta_from_lam,
                          m_forced_all ? m_forced_all + (int64_t)t * n : NULL, g, g2, gf, &gl);
        double* tmp = g;
        g = g2;
        g2 = tmp;
    }
    if (gu0) memcpy(gu0, g, sizeof(double) * n);
    if (glam) *glam = gl;
    free(states);
    free(g);
    free(g2);
}

/* Sec. 5.3: l1 data fidelity min ||U - f||_1 + lam R(U), A = I, solved by the
 * primal-dual iteration: with r = U^t - f + d^t the dual update is the
 * clamp d^{t+1} = min(max(r, -alpha), alpha) (b = shrink(r, alpha) eliminated)
 * and the primal update is
 *   U^{t+1} = U^t + delta [ lam H_d(U^t) - (2 d^{t+1} - d^t) / alpha ].
 * Jacobi in U (H_d from U^t only); d is pointwise.  m_forced as in
 * wmco_step. */
void wmco_l1_step(const double* U, const double* d, const double* f, int64_t H, int64_t W,
                  double lam, double alpha, double delta, const int8_t* m_forced, double* Uout,
                  double* dout, int8_t* m_out) {
    double S[8];
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            int64_t k = y * W + x;
            candidates_at(U, H, W, y, x, S);
            int m = (m_forced && m_forced[k] >= 0) ? m_forced[k] : select_first_min(S);
            double hd = S[m] / 12.0;
            double r = U[k] - f[k] + d[k];
            double dn = r > alpha ? alpha : (r < -alpha ? -alpha : r);
            Uout[k] = U[k] + delta * (lam * hd - (2.0 * dn - d[k]) / alpha);
            dout[k] = dn;
            if (m_out) m_out[k] = (int8_t)m;
        }
}

/* iters l1 steps from (u0, d0); u0 NULL -> f, d0 NULL -> 0. */
void wmco_l1_solve(const double* f, const double* u0, const double* d0, int64_t H, int64_t W,
                   double lam, double alpha, double delta, int iters, double* Uout,
                   double* dout) {
    int64_t n = H * W;
    double* ua = (double*)malloc(sizeof(double) * n);
    double* ub = (double*)malloc(sizeof(double) * n);
    double* da = (double*)malloc(sizeof(double) * n);
    double* db = (double*)malloc(sizeof(double) * n);
    memcpy(ua, u0 ? u0 : f, sizeof(double) * n);
    if (d0) memcpy(da, d0, sizeof(double) * n);
    else memset(da, 0, sizeof(double) * n);
    for (int t = 0; t < iters; ++t) {
        wmco_l1_step(ua, da, f, H, W, lam, alpha, delta, NULL, ub, db, NULL);
        double* tu = ua; ua = ub; ub = tu;
        double* td = da; da = db; db = td;
    }
    memcpy(Uout, ua, sizeof(double) * n);
    memcpy(dout, da, sizeof(double) * n);
    free(ua); free(ub); free(da); free(db);
}

/* O11: the conventional ("deriv") discretisation of the continuous WMC,
 * eq. (rhs): H^w = Lap U - (U_y^2 U_yy + 2 U_x U_y U_xy + U_x^2 U_xx) /
 * (U_x^2 + U_y^2), with second-order central differences at unit spacing and
 * the replicate border.  The paper does not give its stencil or the guard at
 * a vanishing gradient; here the denominator is U_x^2 + U_y^2 + eps, so that
 * the normal term vanishes where the gradient does and H^w tends to the
 * Laplacian there (cf. Sec. 3.3). */
void wmco_fd_compute(const double* U, int64_t H, int64_t W, double eps, double* Hw) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            double c = U[y * W + x];
            double e = ubar(U, H, W, y, x + 1), w = ubar(U, H, W, y, x - 1);
            double s = ubar(U, H, W, y + 1, x), n = ubar(U, H, W, y - 1, x);
            double se = ubar(U, H, W, y + 1, x + 1), ne = ubar(U, H, W, y - 1, x + 1);
            double sw = ubar(U, H, W, y + 1, x - 1), nw = ubar(U, H, W, y - 1, x - 1);
            double ux = 0.5 * (e - w), uy = 0.5 * (s - n);
            double uxx = e - 2.0 * c + w, uyy = s - 2.0 * c + n;
            double uxy = 0.25 * (se - ne - sw + nw);
            double num = uy * uy * uyy + 2.0 * ux * uy * uxy + ux * ux * uxx;
            Hw[y * W + x] = (uxx + uyy) - num / (ux * ux + uy * uy + eps);
        }
}

/* iters curvature-flow steps U <- U + delta H^w_fd(U) from u0 (Sec. 3.5 with
 * the conventional discretisation; the comparator of Sec. 5.4). */
void wmco_fd_flow(const double* u0, int64_t H, int64_t W, double delta, double eps, int iters,
                  double* Uout) {
    int64_t n = H * W;
    double* a = (double*)malloc(sizeof(double) * n);
    double* h = (double*)malloc(sizeof(double) * n);
    memcpy(a, u0, sizeof(double) * n);
    for (int t = 0; t < iters; ++t) {
        wmco_fd_compute(a, H, W, eps, h);
        for (int64_t k = 0; k < n; ++k) a[k] += delta * h[k];
    }
    memcpy(Uout, a, sizeof(double) * n);
    free(a);
    free(h);
}

/* O12: the learnable layer of Sec. 4.3.  d_k(x) = sum_o w_k[o] Ubar(x + o)
 * for k = 0..K-1 (w: K x 3 x 3, [k][r][c] with r = 0 the row above, c = 0 the
 * column to the left, like the printed kernels), m(x) = first k attaining
 * min_k |d_k(x)| (eq. (act)), out(x) = d_m(x).  m_out (nullable) receives m. */
void wmco_layer_forward(const double* U, int64_t H, int64_t W, int K, const double* w,
                        double* out, int8_t* m_out) {
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            double best = 0.0;
            int bi = 0;
            for (int k = 0; k < K; ++k) {
                double d = 0.0;
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c)
                        d += w[(k * 3 + r) * 3 + c] * ubar(U, H, W, y + r - 1, x + c - 1);
                if (k == 0 || fabs(d) < fabs(best)) {
                    best = d;
                    bi = k;
                }
            }
            out[y * W + x] = best;
            if (m_out) m_out[y * W + x] = (int8_t)bi;
        }
}

/* O12: derivative of the layer with the selection m held fixed (the layer is
 * linear in U and in w for a fixed m).  g = dL/dout.
 *   gU(z)      = sum_{x, o : clamp(x + o) = z} w_{m(x)}[o] g(x)   (scatter)
 *   gW_k[o]    = sum_{x : m(x) = k} g(x) Ubar(x + o)
 * gU and gW (K x 3 x 3) are overwritten. */
void wmco_layer_backward(const double* U, int64_t H, int64_t W, int K, const double* w,
                         const int8_t* m, const double* g, double* gU, double* gW) {
    memset(gU, 0, sizeof(double) * H * W);
    memset(gW, 0, sizeof(double) * K * 9);
    for (int64_t y = 0; y < H; ++y)
        for (int64_t x = 0; x < W; ++x) {
            const int k = m[y * W + x];
            const double gv = g[y * W + x];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    const int64_t zy = clampi(y + r - 1, 0, H - 1), zx = clampi(x + c - 1, 0, W - 1);
                    gU[zy * W + zx] += w[(k * 3 + r) * 3 + c] * gv;
                    gW[(k * 3 + r) * 3 + c] += gv * U[zy * W + zx];
                }
        }
}

/* O13: half-window WMC of a 3-D volume U (D x H x W, z slowest).
 *
 * Sec. 4.1 builds the 2-D operator from the isotropic Laplacian k4 and a
 * Neumann reflection of k4 across each cut line through the centre; k4 is
 * (s x s - 16 delta)/12 with s = [1 2 1].  The 3-D construction here follows
 * the same two steps (the paper does not specify one):
 *   K = (s x s x s - 64 delta)/56  (off-centre weights 1 at corners, 2 on
 *       edges, 4 on faces of the 3x3x3 window, centre -1 after / 56);
 *   the cut planes are the 9 mirror planes of the cube (normals e_x, e_y,
 *   e_z and the 6 face diagonals e_x +- e_y, e_x +- e_z, e_y +- e_z), so the
 *   reflection maps the window onto itself as in 2-D; for each plane and
 *   side the half window keeps the weights on the kept side and on the
 *   plane and adds the reflected weights of the other side.
 * The 18 responses S_i (x56 domain) are evaluated in the difference form
 * sum_{o != 0} w_i[o] (Ubar(x + o) - U(x)) with the replicate border;
 * m = first index with the least |S_i| in the order plane 0..8, side
 * "-" (keep n.o <= 0) before side "+"; H = S_m / 56. */
static const int N3[9][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, -1, 0},
                             {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

static int s121(int o) { return o == 0 ? 2 : 1; }

/* w[i][dz+1][dy+1][dx+1] for i = 2*plane + side (side 0: keep n.o <= 0). */
void wmco3_kernels(int* w) {
    for (int j = 0; j < 9; ++j)
        for (int side = 0; side < 2; ++side) {
            int* k = w + (2 * j + side) * 27;
            for (int t = 0; t < 27; ++t) k[t] = 0;
            const int sg = side == 0 ? 1 : -1;  /* kept side: sg * n.o <= 0 */
            for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dx = -1; dx <= 1; ++dx) {
                        if (!dx && !dy && !dz) continue;
                        const int c = s121(dx) * s121(dy) * s121(dz);
                        const int d = sg * (N3[j][0] * dx + N3[j][1] * dy + N3[j][2] * dz);
                        const int nn = N3[j][0] * N3[j][0] + N3[j][1] * N3[j][1] + N3[j][2] * N3[j][2];
                        int tx = dx, ty = dy, tz = dz;
                        if (d > 0) { /* reflect across the plane onto the kept side */
                            const int dot = N3[j][0] * dx + N3[j][1] * dy + N3[j][2] * dz;
                            tx = dx - 2 * dot * N3[j][0] / nn;
                            ty = dy - 2 * dot * N3[j][1] / nn;
                            tz = dz - 2 * dot * N3[j][2] / nn;
                        }
                        k[((tz + 1) * 3 + (ty + 1)) * 3 + (tx + 1)] += c;
                    }
            k[13] = -56;
        }
}

static double ubar3(const double* U, int64_t D, int64_t H, int64_t W, int64_t z, int64_t y,
                    int64_t x) {
    return U[(clampi(z, 0, D - 1) * H + clampi(y, 0, H - 1)) * W + clampi(x, 0, W - 1)];
}

/* The 18 responses S_i (x56 domain) at voxel (z, y, x), difference form. */
static void cands3_at(const double* U, int64_t D, int64_t H, int64_t W, int64_t z, int64_t y,
                      int64_t x, const int* w, double S[18]) {
    const double c = U[(z * H + y) * W + x];
    for (int i = 0; i < 18; ++i) {
        double acc = 0.0;
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int t = ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1);
                    if (t == 13 || !w[i * 27 + t]) continue;
                    acc += w[i * 27 + t] * (ubar3(U, D, H, W, z + dz, y + dy, x + dx) - c);
                }
        S[i] = acc;
    }
}

/* First index attaining the least |S_i| (strict '<'). */
static int first_min18(const double S[18]) {
    int m = 0;
    for (int i = 1; i < 18; ++i)
        if (fabs(S[i]) < fabs(S[m])) m = i;
    return m;
}

void wmco3_compute(const double* U, int64_t D, int64_t H, int64_t W, double* Hd, int8_t* m_out) {
    int w[18 * 27];
    double S[18];
    wmco3_kernels(w);
    for (int64_t z = 0; z < D; ++z)
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                cands3_at(U, D, H, W, z, y, x, w, S);
                const int m = first_min18(S);
                Hd[(z * H + y) * W + x] = S[m] / 56.0;
                if (m_out) m_out[(z * H + y) * W + x] = (int8_t)m;
            }
}

/* O13: Jacobi steps of the data or flow iteration (O5) with the 3-D operator. */
void wmco3_solve(const double* f, const double* u0, int64_t D, int64_t H, int64_t W, double lam,
                 double delta, int iters, double* Uout) {
    const int64_t n = D * H * W;
    double* a = (double*)malloc(sizeof(double) * n);
    double* h = (double*)malloc(sizeof(double) * n);
    memcpy(a, u0 ? u0 : f, sizeof(double) * n);
    for (int t = 0; t < iters; ++t) {
        wmco3_compute(a, D, H, W, h, NULL);
        for (int64_t k = 0; k < n; ++k)
            a[k] = f ? a[k] + delta * ((f[k] - a[k]) + lam * h[k]) : a[k] + delta * h[k];
    }
    memcpy(Uout, a, sizeof(double) * n);
    free(a);
    free(h);
}

/* O14: one Jacobi step of the 3-D iteration (O13) with the selection
 * replayable as in O5: m_forced (nullable) entries >= 0 replace the
 * first-minimum rule; m_out (nullable) records the selection used.
 * f == NULL is the flow U' = U + delta H. */
void wmco3_step(const double* U, const double* f, int64_t D, int64_t H, int64_t W, double lam,
                double delta, const int8_t* m_forced, double* Uout, int8_t* m_out) {
    int w[18 * 27];
    double S[18];
    wmco3_kernels(w);
    for (int64_t z = 0; z < D; ++z)
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                const int64_t k = (z * H + y) * W + x;
                cands3_at(U, D, H, W, z, y, x, w, S);
                const int m = (m_forced && m_forced[k] >= 0) ? m_forced[k] : first_min18(S);
                const double h = S[m] / 56.0;
                Uout[k] = f ? U[k] + delta * ((f[k] - U[k]) + lam * h) : U[k] + delta * h;
                if (m_out) m_out[k] = (int8_t)m;
            }
}

/* O14: adjoint of one 3-D step, the counterpart of O8.  With m held fixed
 * the step is affine in (U, f):
 *   U'(x) = U(x) + delta[(f(x) - U(x)) + lam/56 sum_o w_m(x)[o] Ubar(x+o)]
 * (w_i with its centre weight -56, Ubar the replicate-clamped voxel), so
 * dL/dU(v) = keep gbar(v) + coef sum_{x, o : clamp(x+o) = v} w_m(x)[o] gbar(x)
 * with keep = 1 - delta, coef = delta lam / 56 (data) or keep = 1,
 * coef = delta / 56 (flow).  gf (nullable) += delta gbar; *glam (nullable)
 * += sum gbar dU'/dlam with dU'/dlam = delta H, plus -delta^2((f - U) + lam H)
 * when delta_from_lam (delta = 1/(1+lam)).  gU is overwritten. */
void wmco3_step_adjoint(const double* U, const double* f, int64_t D, int64_t H, int64_t W,
                        double lam, double delta, int delta_from_lam, const int8_t* m_forced,
                        const double* gbar, double* gU, double* gf, double* glam) {
    int w[18 * 27];
    double S[18];
    wmco3_kernels(w);
    const int64_t n = D * H * W;
    const double coef = f ? delta * lam / 56.0 : delta / 56.0;
    const double keep = f ? 1.0 - delta : 1.0;
    for (int64_t k = 0; k < n; ++k) gU[k] = keep * gbar[k];
    double gl = 0.0;
    for (int64_t z = 0; z < D; ++z)
        for (int64_t y = 0; y < H; ++y)
            for (int64_t x = 0; x < W; ++x) {
                const int64_t k = (z * H + y) * W + x;
                cands3_at(U, D, H, W, z, y, x, w, S);
                const int m = (m_forced && m_forced[k] >= 0) ? m_forced[k] : first_min18(S);
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int t = ((dz + 1) * 3 + (dy + 1)) * 3 + (dx + 1);
                            const int64_t v = (clampi(z + dz, 0, D - 1) * H + clampi(y + dy, 0, H - 1)) * W +
                                              clampi(x + dx, 0, W - 1);
                            gU[v] += coef * (double)w[m * 27 + t] * gbar[k];
                        }
                if (f) {
                    const double h = S[m] / 56.0;
                    if (gf) gf[k] += delta * gbar[k];
                    double du = delta * h;
                    if (delta_from_lam) du += -delta * delta * ((f[k] - U[k]) + lam * h);
                    gl += gbar[k] * du;
                }
            }
    if (glam) *glam += gl;
}

/* O14: adjoint of a K-step 3-D solve, all K states kept (small volumes).
 * Outputs as O8: gu0 = dL/dU^0, gf = dL/df through the data term only (if
 * the solve started from u0 = f the caller adds gu0), glam, UK = U^K; all
 * nullable.  m_forced_all (nullable): K selection maps back to back. */
void wmco3_solve_adjoint(const double* f, const double* u0, int64_t D, int64_t H, int64_t W,
                         double lam, double delta, int delta_from_lam, int K,
                         const int8_t* m_forced_all, const double* gK, double* gu0, double* gf,
                         double* glam, double* UK) {
    const int64_t n = D * H * W;
    double* states = (double*)malloc(sizeof(double) * n * (size_t)(K + 1));
    memcpy(states, u0 ? u0 : f, sizeof(double) * n);
    for (int t = 0; t < K; ++t)
        wmco3_step(states + (int64_t)t * n, f, D, H, W, lam, delta,
                   m_forced_all ? m_forced_all + (int64_t)t * n : NULL,
                   states + (int64_t)(t + 1) * n, NULL);
    if (UK) memcpy(UK, states + (int64_t)K * n, sizeof(double) * n);
    double* g = (double*)malloc(sizeof(double) * n);
    double* g2 = (double*)malloc(sizeof(double) * n);
    memcpy(g, gK, sizeof(double) * n);
    if (gf) memset(gf, 0, sizeof(double) * n);
    double gl = 0.0;
    for (int t = K - 1; t >= 0; --t) {
        wmco3_step_adjoint(states + (int64_t)t * n, f, D, H, W, lam, delta, delta_from_lam,
                           m_forced_all ? m_forced_all + (int64_t)t * n : NULL, g, g2, gf, &gl);
        double* tmp = g;
        g = g2;
        g2 = tmp;
    }
    if (gu0) memcpy(gu0, g, sizeof(double) * n);
    if (glam) *glam = gl;
    free(states);
    free(g);
    free(g2);
}
