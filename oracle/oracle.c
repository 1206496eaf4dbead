/*
 * FP64 CPU oracle for the Gauss-polynomial (GP) bilateral filter of
 * Chaudhury, "Fast and Accurate Bilateral Filtering using Gauss-Polynomial
 * Decomposition" (arXiv 1505.00077).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file.  It exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the GPU path with a plain, slow,
 * obviously correct implementation.  It shares no code, header, table or
 * constant generator with the GPU path.
 *
 * Every routine works in double precision on row-major H x W images.
 *
 * Spatial kernels are passed as symmetric 1-D tables k[0..R] (k[d] is the
 * weight at offset +d and -d).  The 2-D spatial weight is k[|dy|] * k[|dx|]
 * (the Gaussian of eq. (2) is separable).  Two tables are provided:
 *   - or_gauss_table:   the sampled Gaussian of eq. (2), exp(-d^2 / 2 s^2);
 *   - or_deriche_table: the closed-form impulse response of Deriche's
 *     fourth-order recursive Gaussian, which the paper's experiments use for
 *     the spatial filtering of the GP method (Experiments section).
 * Offsets outside the image are skipped in every sum (zero extension); the
 * paper does not state a boundary rule.
 *
 * Parity status: every routine below is pinned by tests against a brute
 * force, a closed form, a library routine or finite differences; none is
 * "parity unpinned".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

/* Centre modes of the centring (Section 2, the Proposition eq. (6),
 * Algorithm 1).  The paper uses the mean; the others are there so
 * that tests can exercise eq. (6) with other centres. */
#define OR_CENTER_MEAN 0
#define OR_CENTER_MIDRANGE 1
#define OR_CENTER_NONE 2

/* ------------------------------------------------------------------------ */
/* Spatial kernel tables                                                     */
/* ------------------------------------------------------------------------ */

/* Eq. (2): g_s(d) = exp(-d^2 / (2 s^2)), unnormalised, sampled at integers. */
void or_gauss_table(double sigma_s, int R, double *k)
{
    for (int d = 0; d <= R; ++d)
        k[d] = exp(-(double)d * (double)d / (2.0 * sigma_s * sigma_s));
}

/* d/d(log sigma_s) of the table above: (d^2 / s^2) * g_s(d). */
void or_gauss_dtable(double sigma_s, int R, double *kt)
{
    for (int d = 0; d <= R; ++d) {
        double t2 = (double)d * (double)d / (sigma_s * sigma_s);
        kt[d] = t2 * exp(-0.5 * t2);
    }
}

/* Deriche's fourth-order approximation of the Gaussian (R. Deriche,
 * "Recursively implementing the Gaussian and its derivatives", 1993): for
 * t = |d| / s,
 *   h(t) = (a0 cos(w0 t) + a1 sin(w0 t)) exp(-b0 t)
 *        + (c0 cos(w1 t) + c1 sin(w1 t)) exp(-b1 t),
 * which approximates exp(-t^2 / 2) (the overall gain 1/(s sqrt(2 pi)) of the
 * published normalised form is dropped; the filter output is a ratio and does
 * not depend on the gain).  Constants as published. */
static const double DER_A0 = 1.680, DER_A1 = 3.735;
static const double DER_B0 = 1.783, DER_B1 = 1.723;
static const double DER_C0 = -0.6803, DER_C1 = -0.2598;
static const double DER_W0 = 0.6318, DER_W1 = 1.997;

double or_deriche_h(double t)
{
    t = fabs(t);
    return (DER_A0 * cos(DER_W0 * t) + DER_A1 * sin(DER_W0 * t)) * exp(-DER_B0 * t) +
           (DER_C0 * cos(DER_W1 * t) + DER_C1 * sin(DER_W1 * t)) * exp(-DER_B1 * t);
}

/* dh/dt for t >= 0, from the product rule on each damped sinusoid. */
static double deriche_dh(double t)
{
    double e0 = exp(-DER_B0 * t), e1 = exp(-DER_B1 * t);
    double c0 = cos(DER_W0 * t), s0 = sin(DER_W0 * t);
    double c1 = cos(DER_W1 * t), s1 = sin(DER_W1 * t);
    double d0 = (-DER_A0 * DER_W0 * s0 + DER_A1 * DER_W0 * c0) - DER_B0 * (DER_A0 * c0 + DER_A1 * s0);
    double d1 = (-DER_C0 * DER_W1 * s1 + DER_C1 * DER_W1 * c1) - DER_B1 * (DER_C0 * c1 + DER_C1 * s1);
    return d0 * e0 + d1 * e1;
}

void or_deriche_table(double sigma_s, int R, double *k)
{
    for (int d = 0; d <= R; ++d)
        k[d] = or_deriche_h((double)d / sigma_s);
}

/* d/d(log sigma_s) of h(|d| / s) = -(t) h'(t), t = |d| / s. */
void or_deriche_dtable(double sigma_s, int R, double *kt)
{
    for (int d = 0; d <= R; ++d) {
        double t = (double)d / sigma_s;
        kt[d] = -t * deriche_dh(t);
    }
}

/* ------------------------------------------------------------------------ */
/* Separable spatial filtering, eq. (8)                                      */
/* ------------------------------------------------------------------------ */

/* One 1-D pass along rows (dir 0) or columns (dir 1):
 *   out(y,x) = sum_{|d|<=R, in-domain} k[|d|] in(y, x-d)   (rows)
 *   out(y,x) = sum_{|d|<=R, in-domain} k[|d|] in(y-d, x)   (columns) */
static void pass_1d(const double *in, double *out, int H, int W, const double *k, int R, int dir)
{
#pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double acc = 0.0;
            for (int d = -R; d <= R; ++d) {
                int yy = dir ? y - d : y;
                int xx = dir ? x : x - d;
                if (yy < 0 || yy >= H || xx < 0 || xx >= W)
                    continue;
                acc += k[d < 0 ? -d : d] * in[(size_t)yy * W + xx];
            }
            out[(size_t)y * W + x] = acc;
        }
    }
}

/* Eq. (8) with the separable weight ky[|dy|] * kx[|dx|]: a column pass with
 * ky followed by a row pass with kx.  tmp has H*W entries. */
static void spatial_sep(const double *in, double *out, double *tmp, int H, int W,
                        const double *ky, const double *kx, int R)
{
    pass_1d(in, tmp, H, W, ky, R, 1);
    pass_1d(tmp, out, H, W, kx, R, 0);
}

int or_spatial(const double *in, double *out, int H, int W, const double *k, int R)
{
    if (!in || !out || !k || H < 1 || W < 1 || R < 0)
        return OR_EINVAL;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)H * W);
    if (!tmp)
        return OR_ENOMEM;
    spatial_sep(in, out, tmp, H, W, k, k, R);
    free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Eq. (1): the bilateral filter computed directly                           */
/* ------------------------------------------------------------------------ */

int or_direct(const double *f, double *out, int H, int W, const double *k, int R, double sigma_r)
{
    if (!f || !out || !k || H < 1 || W < 1 || R < 0 || !(sigma_r > 0))
        return OR_EINVAL;
    const double inv2r2 = 1.0 / (2.0 * sigma_r * sigma_r);
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const double fi = f[(size_t)y * W + x];
            double num = 0.0, den = 0.0;
            for (int dy = -R; dy <= R; ++dy) {
                int yy = y - dy;
                if (yy < 0 || yy >= H)
                    continue;
                const double ky = k[dy < 0 ? -dy : dy];
                for (int dx = -R; dx <= R; ++dx) {
                    int xx = x - dx;
                    if (xx < 0 || xx >= W)
                        continue;
                    const double fj = f[(size_t)yy * W + xx];
                    const double t = fj - fi;
                    const double w = ky * k[dx < 0 ? -dx : dx] * exp(-t * t * inv2r2);
                    num += w * fj;
                    den += w;
                }
            }
            out[(size_t)y * W + x] = num / den;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Centre of the intensity range (Section 2, eq. (6); Algorithm 1: the mean)*/
/* ------------------------------------------------------------------------ */

double or_center(const double *f, int H, int W, int mode)
{
    size_t n = (size_t)H * W;
    if (mode == OR_CENTER_NONE)
        return 0.0;
    if (mode == OR_CENTER_MIDRANGE) {
        double lo = f[0], hi = f[0];
        for (size_t i = 1; i < n; ++i) {
            if (f[i] < lo)
                lo = f[i];
            if (f[i] > hi)
                hi = f[i];
        }
        return 0.5 * (lo + hi);
    }
    double s = 0.0;
    for (size_t i = 0; i < n; ++i)
        s += f[i];
    return s / (double)n;
}

/* ------------------------------------------------------------------------ */
/* The Gauss-polynomial filter of Section 3 (Algorithm 1 summarises it)      */
/* ------------------------------------------------------------------------ */

/* Inputs: image f, range parameter sigma_r, degree N, spatial table k[0..R].
 *
 * Section 3 states the method on an image whose intensity range is centred
 * (the Proposition, eq. (6)): with h = f - t_c and x = h / sigma_r,
 *   G_n = x^n,  F_n = exp(-x^2 / 2) G_n,  n = 0..N+1        (eq. (7) on h)
 *   Fbar_n = F_n filtered with the spatial table              (eq. (8))
 *   P = sigma_r sum_{n=0..N} G_n Fbar_{n+1} / n!              (eq. (9))
 *   Q = sum_{n=0..N} G_n Fbar_n / n!                          (eq. (10))
 * and the filtered image is P / Q (eq. (11)) plus the centre t_c (eq. (6)).
 * Each Fbar_n is computed once and enters Q as its n-th term and P as its
 * (n-1)-th term, so that only one filtered image is held at a time. */
int or_gp_alg1(const double *f, double *out, int H, int W, double sigma_r, int N,
               const double *k, int R, int center_mode)
{
    if (!f || !out || !k || H < 1 || W < 1 || R < 0 || !(sigma_r > 0) || N < 0)
        return OR_EINVAL;
    const size_t n = (size_t)H * W;
    double *x = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *G = malloc(sizeof(double) * n), *Gprev = malloc(sizeof(double) * n);
    double *Fn = malloc(sizeof(double) * n), *Fb = malloc(sizeof(double) * n);
    double *P = malloc(sizeof(double) * n), *Q = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    double *inv_fact = malloc(sizeof(double) * (size_t)(N + 2));
    if (!x || !E || !G || !Gprev || !Fn || !Fb || !P || !Q || !tmp || !inv_fact) {
        free(x); free(E); free(G); free(Gprev); free(Fn); free(Fb); free(P); free(Q); free(tmp); free(inv_fact);
        return OR_ENOMEM;
    }
    inv_fact[0] = 1.0;                                     /* 1 / n! */
    for (int m = 1; m <= N + 1; ++m)
        inv_fact[m] = inv_fact[m - 1] / (double)m;
    const double tc = or_center(f, H, W, center_mode);
    for (size_t i = 0; i < n; ++i) {
        x[i] = (f[i] - tc) / sigma_r;
        E[i] = exp(-0.5 * x[i] * x[i]);
        G[i] = 1.0;                                        /* G_0 */
        P[i] = 0.0;
        Q[i] = 0.0;
    }
    for (int m = 0; m <= N + 1; ++m) {
        /* G holds G_m = x^m and Gprev holds G_{m-1} */
        for (size_t i = 0; i < n; ++i)
            Fn[i] = E[i] * G[i];                           /* F_m, eq. (7) */
        spatial_sep(Fn, Fb, tmp, H, W, k, k, R);           /* Fbar_m, eq. (8) */
        for (size_t i = 0; i < n; ++i) {
            if (m <= N)
                Q[i] += inv_fact[m] * G[i] * Fb[i];        /* eq. (10), term m */
            if (m >= 1)
                P[i] += sigma_r * inv_fact[m - 1] * Gprev[i] * Fb[i];  /* eq. (9), term m-1 */
            Gprev[i] = G[i];
            G[i] = G[i] * x[i];                            /* G_{m+1} */
        }
    }
    for (size_t i = 0; i < n; ++i)
        out[i] = P[i] / Q[i] + tc;                         /* eq. (11), then eq. (6) */
    free(x); free(E); free(G); free(Gprev); free(Fn); free(Fb); free(P); free(Q); free(tmp); free(inv_fact);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Joint (cross) bilateral filter                                            */
/* ------------------------------------------------------------------------ */

/* The extension the paper's conclusion names: the range kernel is evaluated
 * on a guide image g and the average is taken of a data image f,
 *   out(i) = sum_j k(j) g_r(g(i-j) - g(i)) f(i-j) / sum_j k(j) g_r(g(i-j) - g(i)),
 * i.e. eq. (1) with the range argument taken from g (g = f gives eq. (1)). */
int or_joint_direct(const double *g, const double *f, double *out, int H, int W, const double *k, int R,
                    double sigma_r)
{
    if (!g || !f || !out || !k || H < 1 || W < 1 || R < 0 || !(sigma_r > 0))
        return OR_EINVAL;
    const double inv2r2 = 1.0 / (2.0 * sigma_r * sigma_r);
#pragma omp parallel for schedule(dynamic, 4)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const double gi = g[(size_t)y * W + x];
            double num = 0.0, den = 0.0;
            for (int dy = -R; dy <= R; ++dy) {
                int yy = y - dy;
                if (yy < 0 || yy >= H)
                    continue;
                const double ky = k[dy < 0 ? -dy : dy];
                for (int dx = -R; dx <= R; ++dx) {
                    int xx = x - dx;
                    if (xx < 0 || xx >= W)
                        continue;
                    const size_t j = (size_t)yy * W + xx;
                    const double t = g[j] - gi;
                    const double w = ky * k[dx < 0 ? -dx : dx] * exp(-t * t * inv2r2);
                    num += w * f[j];
                    den += w;
                }
            }
            out[(size_t)y * W + x] = num / den;
        }
    }
    return OR_OK;
}

/* The Gauss-polynomial approximation of the joint filter.  With t_c the
 * centre of the guide g, x = (g - t_c) / sigma_r, G_n = x^n and
 * F_n = exp(-x^2 / 2) G_n (eq. (7) on the guide), the range weight of a pair
 * factors as g_r(g_j - g_i) = F_0(i) F_0(j) exp(x_i x_j), and truncating the
 * exponential as in eqs. (4)-(5) gives, after the F_0(i) cancel,
 *   Q = sum_{n=0..N} G_n (F_n * g_s) / n!,   P = sum_{n=0..N} G_n ((F_n f) * g_s) / n!,
 * and out = P / Q (eqs. (8)-(11) with the data f in the numerator's images).
 * With g = f, F_n f = t_c F_n + sigma_r F_{n+1}, so P = t_c Q + sigma_r P_eq9
 * and the output is that of the image filter. */
int or_joint_gp(const double *g, const double *f, double *out, int H, int W, double sigma_r, int N,
                const double *k, int R, int center_mode)
{
    if (!g || !f || !out || !k || H < 1 || W < 1 || R < 0 || !(sigma_r > 0) || N < 0)
        return OR_EINVAL;
    const size_t n = (size_t)H * W;
    double *x = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *G = malloc(sizeof(double) * n), *Fn = malloc(sizeof(double) * n);
    double *Fb = malloc(sizeof(double) * n), *P = malloc(sizeof(double) * n);
    double *Q = malloc(sizeof(double) * n), *tmp = malloc(sizeof(double) * n);
    if (!x || !E || !G || !Fn || !Fb || !P || !Q || !tmp) {
        free(x); free(E); free(G); free(Fn); free(Fb); free(P); free(Q); free(tmp);
        return OR_ENOMEM;
    }
    const double tc = or_center(g, H, W, center_mode);
    for (size_t i = 0; i < n; ++i) {
        x[i] = (g[i] - tc) / sigma_r;
        E[i] = exp(-0.5 * x[i] * x[i]);
        G[i] = 1.0;
        P[i] = 0.0;
        Q[i] = 0.0;
    }
    double inv_fact = 1.0;                                 /* 1 / m! */
    for (int m = 0; m <= N; ++m) {
        for (size_t i = 0; i < n; ++i)
            Fn[i] = E[i] * G[i];                           /* F_m of the guide */
        spatial_sep(Fn, Fb, tmp, H, W, k, k, R);
        for (size_t i = 0; i < n; ++i) {
            Q[i] += inv_fact * G[i] * Fb[i];
            Fn[i] = Fn[i] * f[i];                          /* F_m f */
        }
        spatial_sep(Fn, Fb, tmp, H, W, k, k, R);
        for (size_t i = 0; i < n; ++i) {
            P[i] += inv_fact * G[i] * Fb[i];
            G[i] = G[i] * x[i];                            /* G_{m+1} */
        }
        inv_fact /= (double)(m + 1);
    }
    for (size_t i = 0; i < n; ++i)
        out[i] = P[i] / Q[i];
    free(x); free(E); free(G); free(Fn); free(Fb); free(P); free(Q); free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Volumes and video                                                         */
/* ------------------------------------------------------------------------ */

/* The extension to higher-dimensional signals the introduction and the
 * Conclusion name, for a T x H x W volume (frames t, rows y, columns x) with
 * the separable spatial weight kt[|dt|] * ks[|dy|] * ks[|dx|] (the third axis
 * may have its own scale, e.g. time in a video).  Offsets outside the volume
 * are skipped (zero extension). */

/* One 1-D pass along t (axis 0), y (axis 1) or x (axis 2). */
static void pass_1d_3(const double *in, double *out, int T, int H, int W, const double *k, int R, int axis)
{
#pragma omp parallel for schedule(static)
    for (int t = 0; t < T; ++t) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int d = -R; d <= R; ++d) {
                    int tt = axis == 0 ? t - d : t, yy = axis == 1 ? y - d : y, xx = axis == 2 ? x - d : x;
                    if (tt < 0 || tt >= T || yy < 0 || yy >= H || xx < 0 || xx >= W)
                        continue;
                    acc += k[d < 0 ? -d : d] * in[((size_t)tt * H + yy) * W + xx];
                }
                out[((size_t)t * H + y) * W + x] = acc;
            }
        }
    }
}

static void spatial_sep3(const double *in, double *out, double *tmp, int T, int H, int W, const double *kt,
                         int Rt, const double *ks, int Rs)
{
    pass_1d_3(in, out, T, H, W, kt, Rt, 0);
    pass_1d_3(out, tmp, T, H, W, ks, Rs, 1);
    pass_1d_3(tmp, out, T, H, W, ks, Rs, 2);
}

int or_spatial3(const double *in, double *out, int T, int H, int W, const double *kt, int Rt, const double *ks,
                int Rs)
{
    if (!in || !out || !kt || !ks || T < 1 || H < 1 || W < 1 || Rt < 0 || Rs < 0)
        return OR_EINVAL;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)T * H * W);
    if (!tmp)
        return OR_ENOMEM;
    spatial_sep3(in, out, tmp, T, H, W, kt, Rt, ks, Rs);
    free(tmp);
    return OR_OK;
}

/* Eq. (1) over a volume, computed directly. */
int or_volume_direct(const double *f, double *out, int T, int H, int W, const double *kt, int Rt,
                     const double *ks, int Rs, double sigma_r)
{
    if (!f || !out || !kt || !ks || T < 1 || H < 1 || W < 1 || Rt < 0 || Rs < 0 || !(sigma_r > 0))
        return OR_EINVAL;
    const double inv2r2 = 1.0 / (2.0 * sigma_r * sigma_r);
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < T; ++t) {
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                const double fi = f[((size_t)t * H + y) * W + x];
                double num = 0.0, den = 0.0;
                for (int dt = -Rt; dt <= Rt; ++dt) {
                    int tt = t - dt;
                    if (tt < 0 || tt >= T)
                        continue;
                    for (int dy = -Rs; dy <= Rs; ++dy) {
                        int yy = y - dy;
                        if (yy < 0 || yy >= H)
                            continue;
                        for (int dx = -Rs; dx <= Rs; ++dx) {
                            int xx = x - dx;
                            if (xx < 0 || xx >= W)
                                continue;
                            const double fj = f[((size_t)tt * H + yy) * W + xx];
                            const double d = fj - fi;
                            const double w = kt[dt < 0 ? -dt : dt] * ks[dy < 0 ? -dy : dy] * ks[dx < 0 ? -dx : dx] *
                                             exp(-d * d * inv2r2);
                            num += w * fj;
                            den += w;
                        }
                    }
                }
                out[((size_t)t * H + y) * W + x] = num / den;
            }
        }
    }
    return OR_OK;
}

/* The Gauss-polynomial filter of Section 3 over a volume: eqs. (7)-(11) as
 * in or_gp_alg1, with eq. (8) the separable filtering over all three axes and
 * the centre taken over the whole volume. */
int or_volume_gp(const double *f, double *out, int T, int H, int W, double sigma_r, int N, const double *kt,
                 int Rt, const double *ks, int Rs, int center_mode)
{
    if (!f || !out || !kt || !ks || T < 1 || H < 1 || W < 1 || Rt < 0 || Rs < 0 || !(sigma_r > 0) || N < 0)
        return OR_EINVAL;
    const size_t n = (size_t)T * H * W;
    double *x = malloc(sizeof(double) * n), *E = malloc(sizeof(double) * n);
    double *G = malloc(sizeof(double) * n), *Gprev = malloc(sizeof(double) * n);
    double *Fn = malloc(sizeof(double) * n), *Fb = malloc(sizeof(double) * n);
    double *P = malloc(sizeof(double) * n), *Q = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * n);
    if (!x || !E || !G || !Gprev || !Fn || !Fb || !P || !Q || !tmp) {
        free(x); free(E); free(G); free(Gprev); free(Fn); free(Fb); free(P); free(Q); free(tmp);
        return OR_ENOMEM;
    }
    /* the centre over the whole volume (a T H x W image) */
    const double tc = or_center(f, T * H, W, center_mode);
    for (size_t i = 0; i < n; ++i) {
        x[i] = (f[i] - tc) / sigma_r;
        E[i] = exp(-0.5 * x[i] * x[i]);
        G[i] = 1.0;
        P[i] = 0.0;
        Q[i] = 0.0;
    }
    double inv_fact = 1.0;                                 /* 1 / m! */
    for (int m = 0; m <= N + 1; ++m) {
        for (size_t i = 0; i < n; ++i)
            Fn[i] = E[i] * G[i];                           /* F_m, eq. (7) */
        spatial_sep3(Fn, Fb, tmp, T, H, W, kt, Rt, ks, Rs);
        for (size_t i = 0; i < n; ++i) {
            if (m <= N)
                Q[i] += inv_fact * G[i] * Fb[i];           /* eq. (10), term m */
            if (m >= 1)
                P[i] += sigma_r * inv_fact * (double)m * Gprev[i] * Fb[i];  /* eq. (9), term m-1: 1/(m-1)! = m/m! */
            Gprev[i] = G[i];
            G[i] = G[i] * x[i];
        }
        inv_fact /= (double)(m + 1);
    }
    for (size_t i = 0; i < n; ++i)
        out[i] = P[i] / Q[i] + tc;
    free(x); free(E); free(G); free(Gprev); free(Fn); free(Fb); free(P); free(Q); free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* The same approximation in rescaled channels                               */
/* ------------------------------------------------------------------------ */

/* With x = (f - t_c) / sigma_r and u_n(x) = exp(-x^2/2) x^n / sqrt(n!), the
 * auxiliary images of eq. (7) are F_n = sqrt(n!) u_n(x).  Writing
 * Ubar_n = u_n(x) * g_s, eqs. (9)-(11) become, after cancelling the common
 * factor exp(-tau^2/2) with tau = x(i),
 *   Q(i) ~ D(i) = sum_{n<=N} u_n(tau) Ubar_n(i),
 *   P(i) ~ sigma_r M(i),  M(i) = sum_{n<=N} u_n(tau) sqrt(n+1) Ubar_{n+1}(i),
 * and the output is t_c + sigma_r M / D.  The u_n stay bounded by one, which
 * is why the GPU path stores these channels.  Optional outputs D and M
 * (may be NULL). */
int or_gp_rescaled(const double *f, double *out, double *Dout, double *Mout, int H, int W,
                   double sigma_r, int N, const double *k, int R, int center_mode)
{
    if (!f || !out || !k || H < 1 || W < 1 || R < 0 || !(sigma_r > 0) || N < 0)
        return OR_EINVAL;
    const size_t n = (size_t)H * W;
    const int C = N + 2;
    double *U = malloc(sizeof(double) * n), *Ub = malloc(sizeof(double) * n * C);
    double *x = malloc(sizeof(double) * n), *tmp = malloc(sizeof(double) * n);
    if (!U || !Ub || !x || !tmp) {
        free(U); free(Ub); free(x); free(tmp);
        return OR_ENOMEM;
    }
    const double tc = or_center(f, H, W, center_mode);
    for (size_t i = 0; i < n; ++i)
        x[i] = (f[i] - tc) / sigma_r;
    for (int m = 0; m < C; ++m) {
        for (size_t i = 0; i < n; ++i) {
            /* u_m(x) = exp(-x^2/2 + m log|x| - log(m!)/2) sign(x)^m */
            double v;
            if (m == 0)
                v = exp(-0.5 * x[i] * x[i]);
            else if (x[i] == 0.0)
                v = 0.0;
            else {
                v = exp(-0.5 * x[i] * x[i] + m * log(fabs(x[i])) - 0.5 * lgamma(m + 1.0));
                if (x[i] < 0 && (m & 1))
                    v = -v;
            }
            U[i] = v;
        }
        spatial_sep(U, Ub + (size_t)m * n, tmp, H, W, k, k, R);
    }
    for (size_t i = 0; i < n; ++i) {
        double D = 0.0, M = 0.0, u = exp(-0.5 * x[i] * x[i]);
        for (int m = 0; m <= N; ++m) {
            D += u * Ub[(size_t)m * n + i];
            M += u * sqrt(m + 1.0) * Ub[(size_t)(m + 1) * n + i];
            u = u * x[i] / sqrt(m + 1.0);
        }
        out[i] = tc + sigma_r * M / D;
        if (Dout)
            Dout[i] = D;
        if (Mout)
            Mout[i] = M;
    }
    free(U); free(Ub); free(x); free(tmp);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Gradients of the rescaled form (the paper has no gradient; this is the    */
/* plain chain rule through eqs. (7)-(11) and the mean used as centre)    */
/* ------------------------------------------------------------------------ */

/* Given upstream gout = dL/dout, returns dL/df (grad_f, may be NULL),
 * dL/d(log sigma_s) and dL/d(log sigma_r) (pointers may be NULL).
 * kt is d k / d(log sigma_s) on the same radius R (the radius is held fixed).
 * Centre mode must be mean or none. */
int or_gp_grad(const double *f, const double *gout, int H, int W, double sigma_r, int N,
               const double *k, const double *kt, int R, int center_mode,
               double *grad_f, double *grad_log_ss, double *grad_log_sr)
{
    if (!f || !gout || !k || !kt || H < 1 || W < 1 || R < 0 || !(sigma_r > 0) || N < 0)
        return OR_EINVAL;
    if (center_mode != OR_CENTER_MEAN && center_mode != OR_CENTER_NONE)
        return OR_EINVAL;
    const size_t n = (size_t)H * W;
    const int C = N + 2;      /* channels u_0..u_{N+1} */
    const int CU = N + 3;     /* u_0..u_{N+2}: the derivative of u_{N+1} needs u_{N+2} */
    double *x = malloc(sizeof(double) * n), *U = malloc(sizeof(double) * n * CU);
    double *Ub = malloc(sizeof(double) * n * C), *tmp = malloc(sizeof(double) * n);
    double *alpha = malloc(sizeof(double) * n), *beta = malloc(sizeof(double) * n);
    double *gH = malloc(sizeof(double) * n), *V = malloc(sizeof(double) * n);
    double *Wn = malloc(sizeof(double) * n), *KtU = malloc(sizeof(double) * n);
    double *t1 = malloc(sizeof(double) * n);
    double *outv = malloc(sizeof(double) * n);
    if (!x || !U || !Ub || !tmp || !alpha || !beta || !gH || !V || !Wn || !KtU || !t1 || !outv) {
        free(x); free(U); free(Ub); free(tmp); free(alpha); free(beta); free(gH);
        free(V); free(Wn); free(KtU); free(t1); free(outv);
        return OR_ENOMEM;
    }
    const double tc = or_center(f, H, W, center_mode);
    for (size_t i = 0; i < n; ++i)
        x[i] = (f[i] - tc) / sigma_r;
    /* U_m = u_m(x), m = 0..N+2 */
    for (size_t i = 0; i < n; ++i) {
        double u = exp(-0.5 * x[i] * x[i]);
        for (int m = 0; m < CU; ++m) {
            U[(size_t)m * n + i] = u;
            u = u * x[i] / sqrt(m + 1.0);
        }
    }
    for (int m = 0; m < C; ++m)
        spatial_sep(U + (size_t)m * n, Ub + (size_t)m * n, tmp, H, W, k, k, R);

    /* forward quantities D, M and their tau-derivatives D', M' */
    double sum_g = 0.0;
    for (size_t i = 0; i < n; ++i) {
        double D = 0.0, M = 0.0, Dp = 0.0, Mp = 0.0;
        for (int m = 0; m <= N; ++m) {
            const double um = U[(size_t)m * n + i];
            /* u_m'(x) = sqrt(m) u_{m-1}(x) - sqrt(m+1) u_{m+1}(x) */
            const double dum = (m > 0 ? sqrt((double)m) * U[(size_t)(m - 1) * n + i] : 0.0) -
                               sqrt(m + 1.0) * U[(size_t)(m + 1) * n + i];
            const double a = Ub[(size_t)m * n + i];
            const double b = sqrt(m + 1.0) * Ub[(size_t)(m + 1) * n + i];
            D += um * a;
            M += um * b;
            Dp += dum * a;
            Mp += dum * b;
        }
        outv[i] = tc + sigma_r * M / D;
        alpha[i] = gout[i] * sigma_r / D;          /* dL/dM */
        beta[i] = -alpha[i] * M / D;               /* dL/dD */
        gH[i] = alpha[i] * Mp + beta[i] * Dp;      /* through tau = x(i) */
        sum_g += gout[i];
    }
    double g_lss = 0.0;
    for (int m = 0; m < C; ++m) {
        /* V_m = dL/dUbar_m */
        for (size_t i = 0; i < n; ++i) {
            double v = 0.0;
            if (m <= N)
                v += beta[i] * U[(size_t)m * n + i];
            if (m >= 1)
                v += alpha[i] * sqrt((double)m) * U[(size_t)(m - 1) * n + i];
            V[i] = v;
        }
        /* W_m = K^T V_m = K V_m (the zero-extended symmetric kernel is
         * self-adjoint) */
        spatial_sep(V, Wn, tmp, H, W, k, k, R);
        for (size_t i = 0; i < n; ++i) {
            const double dum = (m > 0 ? sqrt((double)m) * U[(size_t)(m - 1) * n + i] : 0.0) -
                               sqrt(m + 1.0) * U[(size_t)(m + 1) * n + i];
            gH[i] += Wn[i] * dum;
        }
        /* d K / d log sigma_s = kt (x) k + k (x) kt; contribution <V_m, Kt U_m> */
        spatial_sep(U + (size_t)m * n, KtU, tmp, H, W, kt, k, R);
        spatial_sep(U + (size_t)m * n, t1, tmp, H, W, k, kt, R);
        for (size_t i = 0; i < n; ++i)
            g_lss += V[i] * (KtU[i] + t1[i]);
    }
    double sum_gh = 0.0, g_lsr = 0.0;
    for (size_t i = 0; i < n; ++i) {
        sum_gh += gH[i] / sigma_r;
        /* out = tc + sigma_r M/D: d/dlog sigma_r at fixed x is (out - tc);
         * x = (f - tc)/sigma_r gives dx/dlog sigma_r = -x */
        g_lsr += gout[i] * (outv[i] - tc) - x[i] * gH[i];
    }
    if (grad_f) {
        const double corr = center_mode == OR_CENTER_MEAN ? (sum_g - sum_gh) / (double)n : 0.0;
        for (size_t i = 0; i < n; ++i)
            grad_f[i] = gH[i] / sigma_r + corr;
    }
    if (grad_log_ss)
        *grad_log_ss = g_lss;
    if (grad_log_sr)
        *grad_log_sr = g_lsr;
    free(x); free(U); free(Ub); free(tmp); free(alpha); free(beta); free(gH);
    free(V); free(Wn); free(KtU); free(t1); free(outv);
    return OR_OK;
}

/* Eq. (5): the Gauss-polynomial approximation of g_r(t - tau), i.e.
 * exp(-tau^2/2r^2) exp(-t^2/2r^2) sum_{n<=N} (tau t / r^2)^n / n!. */
double or_gauss_poly(double t, double tau, double sigma_r, int N)
{
    const double r2 = sigma_r * sigma_r, z = tau * t / r2;
    double term = 1.0, s = 0.0;
    for (int m = 0; m <= N; ++m) {
        s += term;
        term = term * z / (double)(m + 1);
    }
    return exp(-tau * tau / (2.0 * r2)) * exp(-t * t / (2.0 * r2)) * s;
}
