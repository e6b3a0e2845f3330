/*
 * fe_oracle.c -- plain FP64 CPU reference of the Anscombe-domain
 * Fields-of-Experts Poisson denoiser (Feng, Qiao & Chen, "Poisson Noise
 * Reduction with Higher-order Natural Image Prior Model").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Every routine is written from the paper's definitions, in double
 * precision, with plain loops and no blocking or fusion:
 *   - Anscombe transform                         eq. 2.3
 *   - closed-form unbiased inverse I_C           eq. 2.4
 *   - FoE prior energy, Student-t potential      eq. 2.5, 2.6
 *   - influence rho'(z) = 2z/(1+z^2)             Section 2.5 (below eq. 2.13)
 *   - K_i as a sparse N x N matrix, K_i^T its    Section 2.5 (Hessian text)
 *     exact transpose
 *   - gradient of the prior term                 eq. 3.2
 *   - iPiano inertial forward-backward step      eq. 2.8, prox eq. 2.9
 *   - quadratic data term and its prox           eq. 3.4, 3.5
 *   - I-divergence data term and its prox        eq. 2.2, 3.3, 3.6
 *   - final adaptive scheme                      eq. 3.7
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - k_i * u is a correlation with taps k[a][b] applied at offset
 *     (a - r, b - r), r = (m - 1) / 2;
 *   - the image is extended half-sample symmetrically (u(-1-i) = u(i),
 *     u(n + i) = u(n - 1 - i)); K_i is "extend, then correlate", and K_i^T
 *     is its exact transpose: full correlation with the rotated filter on
 *     the zero-extended input, then the ghost rows and columns are added
 *     back onto the pixels they mirror;
 *   - u^0 = u^{-1} = v; a fixed iteration count; no stopping test;
 *   - x_hat = I_C(u_hat) for u_hat >= sqrt(3/2), else 0 (I_C vanishes
 *     exactly at sqrt(3/2) and is negative or singular below);
 *   - eq. 3.6 is taken with the weights alpha_i of eq. 3.7.
 *
 * Inputs arrive as float32 values widened exactly to double, so parity
 * against the GPU measures arithmetic error only.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define DATA_QUADRATIC 1
#define DATA_IDIV 2

/* Rows are shared among threads only for images big enough to pay for it;
 * every row is computed by one thread in the same order either way, so the
 * results do not depend on the thread count. */
#define PARALLEL(H, W) ((long)(H) * (long)(W) >= 16384)

/* Half-sample symmetric index into [0, n): -1 -> 0, -2 -> 1, n -> n-1.
 * One reflection only, which is valid whenever the offset is at most n. */
static long sym_index(long i, long n)
{
    if (i < 0) i = -1 - i;
    if (i >= n) i = 2 * n - 1 - i;
    return i;
}

/* eq. 2.3: v = 2 sqrt(y + 3/8). */
void oracle_anscombe(const double *y, double *v, long n)
{
    for (long p = 0; p < n; ++p) v[p] = 2.0 * sqrt(y[p] + 3.0 / 8.0);
}

/* eq. 2.4: closed-form approximation of the exact unbiased inverse,
 * clamped to 0 below sqrt(3/2), where I_C is exactly zero. */
double oracle_inverse_anscombe_scalar(double z)
{
    const double c = sqrt(1.5);
    if (!(z >= c)) return 0.0;
    return 0.25 * z * z + 0.25 * c / z - (11.0 / 8.0) / (z * z)
           + (5.0 / 8.0) * c / (z * z * z) - 0.125;
}

void oracle_inverse_anscombe(const double *u, double *x, long n)
{
    for (long p = 0; p < n; ++p) x[p] = oracle_inverse_anscombe_scalar(u[p]);
}

/* Extension e of size (H + 2r) x (W + 2r): e(i, j) = u(sym(i - r), sym(j - r)). */
void oracle_extend_symmetric(const double *u, int H, int W, int r, double *e)
{
    const long We = W + 2 * r;
    for (long i = 0; i < H + 2 * r; ++i)
        for (long j = 0; j < We; ++j)
            e[i * We + j] = u[sym_index(i - r, H) * W + sym_index(j - r, W)];
}

/* Forward filter bank z_i = K_i u for i = 0..nf-1 (eq. 2.5 with the
 * correlation reading): z_i(y, x) = sum_{a,b} k_i[a][b] e(y + a, x + b),
 * taps summed in (a, b) row-major order for every pixel.
 * z has layout [nf][H][W]. */
void oracle_filter(const double *u, int H, int W, const double *k, int m,
                   int nf, double *z)
{
    const int r = (m - 1) / 2;
    const long We = W + 2 * r;
    double *e = (double *)malloc(sizeof(double) * (size_t)(H + 2 * r) * We);
    oracle_extend_symmetric(u, H, W, r, e);
    for (int i = 0; i < nf; ++i) {
        const double *ki = k + (size_t)i * m * m;
        double *zi = z + (size_t)i * H * W;
#pragma omp parallel for schedule(static) if (PARALLEL(H, W))
        for (long y = 0; y < H; ++y) {
            double *row = zi + y * W;
            for (long x = 0; x < W; ++x) row[x] = 0.0;
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < m; ++b) {
                    const double kab = ki[a * m + b];
                    const double *er = e + (y + a) * We + b;
                    for (long x = 0; x < W; ++x) row[x] += kab * er[x];
                }
        }
    }
    free(e);
}

/* Adjoint g = sum_i K_i^T w_i, the exact transpose of oracle_filter.
 * Step 1 (transpose of the correlation, on the extended grid):
 *   G_i(s, t) = sum_{a,b} k_i[a][b] w_i(s - a, t - b),  s in [0, H+2r),
 *   t in [0, W+2r) (extended coordinates), w_i = 0 outside the image;
 *   G = sum_i G_i.
 * Step 2 (transpose of the symmetric extension): each extended position
 *   (s, t) adds G_i(s, t) onto the pixel it was copied from,
 *   (sym(s - r), sym(t - r)).
 * w has layout [nf][H][W]; g is H x W and is overwritten. */
void oracle_filter_adjoint(const double *w, int H, int W, const double *k,
                           int m, int nf, double *g)
{
    const int r = (m - 1) / 2;
    const long He = H + 2 * r, We = W + 2 * r;
    /* w_i zero-extended by m - 1 on every side, so that w_i(s - a, t - b)
     * is wz[s - a + m - 1][t - b + m - 1] for every extended (s, t). */
    const long P = m - 1, Hz = H + 2 * P, Wz = W + 2 * P;
    double *G = (double *)calloc((size_t)He * We, sizeof(double));
    double *wz = (double *)calloc((size_t)Hz * Wz, sizeof(double));
    for (int i = 0; i < nf; ++i) {
        const double *ki = k + (size_t)i * m * m;
        const double *wi = w + (size_t)i * H * W;
        for (long y = 0; y < H; ++y)
            for (long x = 0; x < W; ++x) wz[(y + P) * Wz + x + P] = wi[y * W + x];
#pragma omp parallel if (PARALLEL(H, W))
        {
            double *acc = (double *)malloc(sizeof(double) * (size_t)We);
#pragma omp for schedule(static)
            for (long s = 0; s < He; ++s) {
                for (long t = 0; t < We; ++t) acc[t] = 0.0;
                for (int a = 0; a < m; ++a)
                    for (int b = 0; b < m; ++b) {
                        const double kab = ki[a * m + b];
                        const double *wr = wz + (s - a + P) * Wz + (P - b);
                        for (long t = 0; t < We; ++t) acc[t] += kab * wr[t];
                    }
                for (long t = 0; t < We; ++t) G[s * We + t] += acc[t];
            }
            free(acc);
        }
    }
    free(wz);
    /* Fold: g(p) = sum of G over every extended position mirroring p.
     * Gathered per output row so rows can run in parallel.  With a single
     * reflection, the extended rows s with sym(s - r) == y are among
     * r - 1 - y (mirror above), y + r (the row itself) and 2H - 1 - y + r
     * (mirror below), in increasing order; each is checked explicitly. */
#pragma omp parallel for schedule(static) if (PARALLEL(H, W))
    for (long y = 0; y < H; ++y) {
        const long cand[3] = { r - 1 - y, y + r, 2 * (long)H - 1 - y + r };
        for (long x = 0; x < W; ++x) g[y * W + x] = 0.0;
        for (int c = 0; c < 3; ++c) {
            const long s = cand[c];
            if (s < 0 || s >= He || sym_index(s - r, H) != y) continue;
            for (long t = 0; t < We; ++t)
                g[y * W + sym_index(t - r, W)] += G[s * We + t];
        }
    }
    free(G);
}

/* Influence of the weighted Student-t potential: alpha_i rho'(z),
 * rho'(z) = 2 z / (1 + z^2) (derivative of eq. 2.6). */
double oracle_rho(double z) { return log(1.0 + z * z); }
double oracle_rho_prime(double z) { return 2.0 * z / (1.0 + z * z); }

/* eq. 3.2: grad F(u) = sum_i alpha_i K_i^T rho'(K_i u). */
void oracle_grad_prior(const double *u, int H, int W, const double *k,
                       const double *alpha, int m, int nf, double *g)
{
    const long n = (long)H * W;
    double *z = (double *)malloc(sizeof(double) * (size_t)nf * n);
    oracle_filter(u, H, W, k, m, nf, z);
    for (int i = 0; i < nf; ++i)
        for (long p = 0; p < n; ++p)
            z[(size_t)i * n + p] = alpha[i] * oracle_rho_prime(z[(size_t)i * n + p]);
    oracle_filter_adjoint(z, H, W, k, m, nf, g);
    free(z);
}

/* Ordered sum of a row-major H x W array: each row left to right, then
 * the row sums top to bottom, so the result does not depend on threads. */
static double ordered_sum(const double *a, long H, long W)
{
    double *rows = (double *)malloc(sizeof(double) * (size_t)H);
#pragma omp parallel for schedule(static) if (PARALLEL(H, W))
    for (long y = 0; y < H; ++y) {
        double s = 0.0;
        for (long x = 0; x < W; ++x) s += a[y * W + x];
        rows[y] = s;
    }
    double s = 0.0;
    for (long y = 0; y < H; ++y) s += rows[y];
    free(rows);
    return s;
}

/* eq. 2.5 with eq. 2.6: E_FoE(u) = sum_i alpha_i sum_p log(1 + (K_i u)_p^2). */
double oracle_energy_prior(const double *u, int H, int W, const double *k,
                           const double *alpha, int m, int nf)
{
    const long n = (long)H * W;
    double *z = (double *)malloc(sizeof(double) * (size_t)nf * n);
    oracle_filter(u, H, W, k, m, nf, z);
    double e = 0.0;
    for (int i = 0; i < nf; ++i) {
        double *zi = z + (size_t)i * n;
        for (long p = 0; p < n; ++p) zi[p] = oracle_rho(zi[p]);
        e += alpha[i] * ordered_sum(zi, H, W);
    }
    free(z);
    return e;
}

/* Data terms D(u, v):
 *   quadratic (eq. 3.4):     lambda/2 * sum (u - v)^2
 *   I-divergence (eq. 3.6):  lambda * sum (u - v log u), +inf if any u <= 0. */
double oracle_energy_data(const double *u, const double *v, long n,
                          double lam, int data_term)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    int bad = 0;
    for (long p = 0; p < n; ++p) {
        if (data_term == DATA_QUADRATIC) {
            const double d = u[p] - v[p];
            t[p] = 0.5 * d * d;
        } else {
            if (!(u[p] > 0.0)) bad = 1;
            t[p] = u[p] - v[p] * log(u[p]);
        }
    }
    double s = bad ? INFINITY : lam * ordered_sum(t, 1, n);
    free(t);
    return s;
}

/* Gradient of the data term: lambda (u - v) or lambda (1 - v / u). */
void oracle_grad_data(const double *u, const double *v, long n, double lam,
                      int data_term, double *g)
{
    for (long p = 0; p < n; ++p)
        g[p] = (data_term == DATA_QUADRATIC) ? lam * (u[p] - v[p])
                                             : lam * (1.0 - v[p] / u[p]);
}

/* Proximal map of tau*G (eq. 2.9) for the two data terms.
 *   quadratic, eq. 3.5:     (u~ + tau lam v) / (1 + tau lam)
 *   I-divergence, eq. 3.3 with y replaced by v as eq. 3.6 prescribes:
 *     (u~ - tau lam + sqrt((u~ - tau lam)^2 + 4 tau lam v)) / 2 */
double oracle_prox_scalar(double ut, double v, double tau, double lam,
                          int data_term)
{
    const double tl = tau * lam;
    if (data_term == DATA_QUADRATIC) return (ut + tl * v) / (1.0 + tl);
    const double a = ut - tl;
    return 0.5 * (a + sqrt(a * a + 4.0 * tl * v));
}

void oracle_prox(const double *ut, const double *v, long n, double tau,
                 double lam, int data_term, double *out)
{
    for (long p = 0; p < n; ++p)
        out[p] = oracle_prox_scalar(ut[p], v[p], tau, lam, data_term);
}

/* One iPiano step, eq. 2.8, for F = E_FoE and G = the data term:
 *   u~ = u^n - tau grad F(u^n) + gamma (u^n - u^{n-1});  u^{n+1} = prox(u~).
 * u_next may not alias u or u_prev. */
void oracle_ipiano_step(const double *u, const double *u_prev,
                        const double *v, int H, int W, const double *k,
                        const double *alpha, int m, int nf, double lam,
                        double tau, double gamma, int data_term,
                        double *u_next)
{
    const long n = (long)H * W;
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_grad_prior(u, H, W, k, alpha, m, nf, g);
    for (long p = 0; p < n; ++p) {
        const double ut = u[p] - tau * g[p] + gamma * (u[p] - u_prev[p]);
        u_next[p] = oracle_prox_scalar(ut, v[p], tau, lam, data_term);
    }
    free(g);
}

/* The whole scheme (eq. 3.7): v = f_A(y); iters iPiano steps from
 * u^0 = u^{-1} = v; x_hat = I_C(u_hat).  u_hat and x_hat are H x W. */
void oracle_denoise(const double *counts, int H, int W, const double *k,
                    const double *alpha, int m, int nf, double lam,
                    double tau, double gamma, int iters, int data_term,
                    double *u_hat, double *x_hat)
{
    const long n = (long)H * W;
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *a = (double *)malloc(sizeof(double) * (size_t)n);
    double *b = (double *)malloc(sizeof(double) * (size_t)n);
    double *c = (double *)malloc(sizeof(double) * (size_t)n);
    oracle_anscombe(counts, v, n);
    memcpy(a, v, sizeof(double) * (size_t)n); /* u^n     */
    memcpy(b, v, sizeof(double) * (size_t)n); /* u^{n-1} */
    for (int it = 0; it < iters; ++it) {
        oracle_ipiano_step(a, b, v, H, W, k, alpha, m, nf, lam, tau, gamma,
                           data_term, c);
        double *t = b; b = a; a = c; c = t;
    }
    memcpy(u_hat, a, sizeof(double) * (size_t)n);
    oracle_inverse_anscombe(u_hat, x_hat, n);
    free(v); free(a); free(b); free(c);
}

/* Full energy E(u) = E_FoE(u) + D(u, v) and its gradient (grad may be NULL). */
double oracle_energy_grad(const double *u, const double *v, int H, int W,
                          const double *k, const double *alpha, int m, int nf,
                          double lam, int data_term, double *grad)
{
    const long n = (long)H * W;
    double e = oracle_energy_prior(u, H, W, k, alpha, m, nf)
               + oracle_energy_data(u, v, n, lam, data_term);
    if (grad) {
        double *gd = (double *)malloc(sizeof(double) * (size_t)n);
        oracle_grad_prior(u, H, W, k, alpha, m, nf, grad);
        oracle_grad_data(u, v, n, lam, data_term, gd);
        for (long p = 0; p < n; ++p) grad[p] += gd[p];
        free(gd);
    }
    return e;
}

/* Largest eigenvalue of M = sum_i alpha_i K_i^T K_i by power iteration from
 * the caller's start vector x0 (H x W).  The Lipschitz constant of grad F
 * is then at most 2 * lambda_max(M), since |rho''| <= 2. */
double oracle_power_iteration(const double *x0, int H, int W, const double *k,
                              const double *alpha, int m, int nf, int iters)
{
    const long n = (long)H * W;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)nf * n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(x, x0, sizeof(double) * (size_t)n);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        double nx = 0.0;
        for (long p = 0; p < n; ++p) nx += x[p] * x[p];
        nx = sqrt(nx);
        for (long p = 0; p < n; ++p) x[p] /= nx;
        oracle_filter(x, H, W, k, m, nf, z);
        for (int i = 0; i < nf; ++i)
            for (long p = 0; p < n; ++p) z[(size_t)i * n + p] *= alpha[i];
        oracle_filter_adjoint(z, H, W, k, m, nf, y);
        double xy = 0.0;
        for (long p = 0; p < n; ++p) xy += x[p] * y[p];
        lam = xy;
        memcpy(x, y, sizeof(double) * (size_t)n);
    }
    free(x); free(z); free(y);
    return lam;
}

/* ---- binning variant (Section 4: 3 x 3 ones kernel, peak x 9, bilinear
 * upscaling; eq. 3.7 with the peak of the binned image) ---------------------
 * Readings: bins are the non-overlapping 3 x 3 blocks starting at (0, 0);
 * an image whose side is not a multiple of 3 is first extended half-sample
 * symmetrically, so every bin sums nine counts; the denoised bin value
 * estimates the sum of nine intensities, so the per-pixel estimate is the
 * bin value / 9, placed at the bin centre (3i + 1, 3j + 1) and interpolated
 * bilinearly, constant beyond the outermost centres. */

/* yb[i][j] = sum of the 3 x 3 block (3i.., 3j..) of the extended image;
 * yb is ceil(H/3) x ceil(W/3). */
void oracle_bin3(const double *y, int H, int W, double *yb)
{
    const long Hb = (H + 2) / 3, Wb = (W + 2) / 3;
    for (long i = 0; i < Hb; ++i)
        for (long j = 0; j < Wb; ++j) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    s += y[sym_index(3 * i + a, H) * W + sym_index(3 * j + b, W)];
            yb[i * Wb + j] = s;
        }
}

/* Bilinear upscaling of the per-pixel estimate xb / 9 to H x W. */
void oracle_upsample3(const double *xb, int Hb, int Wb, int H, int W, double *x)
{
    for (long y = 0; y < H; ++y) {
        double fy = (y - 1) / 3.0;
        if (fy < 0.0) fy = 0.0;
        if (fy > Hb - 1) fy = Hb - 1;
        long i0 = (long)floor(fy);
        if (i0 > Hb - 1) i0 = Hb - 1;
        const long i1 = i0 + 1 < Hb ? i0 + 1 : Hb - 1;
        const double wy = fy - i0;
        for (long xx = 0; xx < W; ++xx) {
            double fx = (xx - 1) / 3.0;
            if (fx < 0.0) fx = 0.0;
            if (fx > Wb - 1) fx = Wb - 1;
            long j0 = (long)floor(fx);
            if (j0 > Wb - 1) j0 = Wb - 1;
            const long j1 = j0 + 1 < Wb ? j0 + 1 : Wb - 1;
            const double wx = fx - j0;
            const double v = (1.0 - wy) * ((1.0 - wx) * xb[i0 * Wb + j0] + wx * xb[i0 * Wb + j1])
                             + wy * ((1.0 - wx) * xb[i1 * Wb + j0] + wx * xb[i1 * Wb + j1]);
            x[y * W + xx] = v / 9.0;
        }
    }
}
