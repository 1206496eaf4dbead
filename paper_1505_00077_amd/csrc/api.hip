// C ABI of libbfgp: argument checks, workspace layout, coefficient set-up and
// kernel launches.  Everything here runs on the host.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <string>

#include "../../include/bfgp.h"
#include "launch.hpp"
#include "fir.hpp"
#include "iir.hpp"
#include "hrow.hpp"
#include "direct.hpp"
#include "box.hpp"
#include "bwd.hpp"
#include "iir_bwd.hpp"

using namespace bfgp;

namespace {

thread_local std::string g_err;
std::atomic<int> g_fir_crossover{9};  // FIR while ceil(3 sigma_s) <= this radius

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(BF_EHIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// Window half-width of eq. (1): W = 3 sigma_s rounded up, at least 1.  A
// relative excess below 1e-6 (e.g. sigma_s = exp(float32 log 2)) does not
// round up.
int fir_radius(double sigma_s) {
    int r = (int)ceil(3.0 * sigma_s * (1.0 - 1e-6));
    return r < 1 ? 1 : r;
}

// Size-dependent crossover (set by a tuner): the first entry whose pixel
// count bounds the image gives the radius; larger images use the process-wide
// radius.
constexpr int kMaxCrossTable = 8;
std::mutex g_cross_mu;
int g_cross_n = 0;
long long g_cross_px[kMaxCrossTable];
int g_cross_r[kMaxCrossTable];

int crossover_for(long long px) {
    if (px > 0) {
        std::lock_guard<std::mutex> g(g_cross_mu);
        for (int k = 0; k < g_cross_n; ++k)
            if (px <= g_cross_px[k]) return g_cross_r[k];
    }
    return g_fir_crossover.load();
}

// px = H * W of the image, or 0 when unknown (the process-wide radius).
unsigned resolve_spatial(long long px, double sigma_s, unsigned flags) {
    unsigned m = flags & BF_SPATIAL_MASK;
    if (m != BF_SPATIAL_AUTO) return m;
    return fir_radius(sigma_s) <= crossover_for(px) ? BF_SPATIAL_FIR : BF_SPATIAL_IIR;
}

int center_code(unsigned flags) {
    switch (flags & BF_CENTER_MASK) {
        case BF_CENTER_MIDRANGE: return 1;
        case BF_CENTER_NONE: return 2;
        default: return 0;
    }
}

// Largest |x| for which the largest channel max_n u_n(x), n <= N+1, is still at
// least exp(-80) (well inside the FP32 normal range).  ln u_n(x) =
// -x^2/2 + n ln x - ln(n!)/2.
double range_limit(int N) {
    auto ok = [N](double x) {
        double best = -1e300;
        for (int n = 0; n <= N + 1; ++n) {
            double l = -0.5 * x * x + (n > 0 ? n * log(x) : 0.0) - 0.5 * lgamma(n + 1.0);
            if (l > best) best = l;
        }
        return best >= -80.0;
    };
    double lo = 0.0, hi = 64.0;
    for (int it = 0; it < 80; ++it) {
        double mid = 0.5 * (lo + hi);
        if (ok(mid)) lo = mid; else hi = mid;
    }
    return lo;
}

// Launch-shape overrides of the IIR passes (0 = automatic), for tuning.
std::atomic<int> g_band_rows{0}, g_col_groups{0}, g_row_groups{0};
// Waves the column passes aim for: a few per SIMD of the 1024 on the device.
constexpr long kTargetWaves = 2048, kBand64Waves = 1024, kRowTargetWaves = 3072;
constexpr int kIirMaxW = 8192;       // IIR widths of the saved terms, joint, volume, batched and stacked calls
constexpr int kIirMaxWide = 2 * kRowSeg;  // IIR widths of the plain forward (row segments)

struct Layout {
    size_t parts, status, stats, carry, stack, segst, total;
};

// Box mode: samples per row-pass thread, threads per row and stack pitch.
int box_L(int W) { return W <= 4096 ? 4 : W <= 8192 ? 16 : 32; }
int box_T(int W) { return ((W + box_L(W) - 1) / box_L(W) + 63) / 64 * 64; }
int box_pitch(int W) { return box_T(W) * box_L(W); }

// Radius of the box window: that of eq. (1), capped at max(H, W) (a wider
// window covers the same pixels).
int box_radius(double sigma_s, int H, int W) {
    double r = ceil(3.0 * sigma_s * (1.0 - 1e-6));
    const int m = H > W ? H : W;
    if (r < 1.0) r = 1.0;
    return r > (double)m ? m : (int)r;
}

// Box launch shape: bands of at least two radii (the start-up window costs at
// most one band), then channel groups until the column pass has a few waves
// per SIMD (each thread holds at most kBoxKC running sums).
BoxShape box_shape(int H, int W, int C, int R) {
    BoxShape sh;
    sh.R = R;
    const long twoR = 2L * R;
    long Bb = ((twoR + 31) / 32) * 32;
    if (Bb < 32) Bb = 32;
    if (Bb > H) Bb = H;
    sh.Bb = (int)Bb;
    sh.nb = (int)((H + Bb - 1) / Bb);
    const long waves = (long)((W + 63) / 64) * sh.nb;
    int G = (int)((kTargetWaves + waves - 1) / waves);
    if (G > 8) G = 8;
    const int gmin = (C + kBoxKC - 1) / kBoxKC;
    if (G < gmin) G = gmin;
    if (G > C) G = C;
    sh.G = G;
    const int per = (C + G - 1) / G;
    sh.NC = per <= 4 ? 4 : per <= 6 ? 6 : per <= 8 ? 8 : per <= 12 ? 12 : per <= 16 ? 16 : 24;
    sh.L = box_L(W);
    sh.T = box_T(W);
    sh.P = box_pitch(W);
    return sh;
}

// C: channels of the stack (N + 2 for the filter, 2 (N + 1) for the joint
// filter).
Layout gp_layout_c(int H, int W, int C, unsigned spatial, bool rows32) {
    Layout L;
    size_t off = 0;
    L.parts = off;
    off = align256(off + sizeof(Partial) * kMaxParts);
    L.status = off;
    off = align256(off + 16);
    L.stats = off;
    off = align256(off + sizeof(Stats));
    L.carry = L.stack = L.segst = off;
    if (spatial == BF_SPATIAL_IIR) {
        const IirShape sh = iir_shape(H, W, C, false, rows32);
        const size_t nb = ((size_t)H + sh.B - 1) / sh.B;
        L.carry = off;
        off = align256(off + sizeof(float) * nb * (size_t)C * 8 * (size_t)W);
        L.stack = off;
        off = align256(off + sizeof(float) * (size_t)C * (size_t)sh.Hs * (size_t)sh.P);
        L.segst = off;
        if (sh.nseg > 1) off = align256(off + sizeof(float) * (size_t)H * sh.nseg * C * 8);
    } else if (spatial == BF_SPATIAL_BOX) {
        L.stack = off;
        off = align256(off + sizeof(float) * (size_t)C * (size_t)H * (size_t)box_pitch(W));
    }
    L.total = off;
    return L;
}

Layout gp_layout(int H, int W, int N, unsigned spatial) { return gp_layout_c(H, W, N + 2, spatial, false); }

int check_image(const void *img, const void *out, int H, int W, int pitch) {
    if (!img || !out) return fail(BF_EINVAL, "null image pointer");
    if (H < 1 || W < 1) return fail(BF_EINVAL, "image size %dx%d must be at least 1x1", H, W);
    if (pitch < W) return fail(BF_EINVAL, "pitch %d is smaller than the width %d", pitch, W);
    if ((size_t)H * (size_t)pitch >= ((size_t)1 << 40)) return fail(BF_EINVAL, "image too large");
    return BF_OK;
}

int check_params(double sigma_s, double sigma_r, int N) {
    if (!finite_pos(sigma_s)) return fail(BF_EINVAL, "sigma_s must be finite and > 0");
    if (!finite_pos(sigma_r)) return fail(BF_EINVAL, "sigma_r must be finite and > 0");
    if (N < 0 || N > BF_MAX_DEGREE) return fail(BF_EINVAL, "degree N=%d outside 0..%d", N, BF_MAX_DEGREE);
    return BF_OK;
}

int check_spatial(unsigned spatial, double sigma_s, int W) {
    if (spatial == BF_SPATIAL_FIR && fir_radius(sigma_s) > BF_FIR_MAX_RADIUS)
        return fail(BF_EUNSUPPORTED, "FIR radius %d exceeds %d (use the IIR mode)", fir_radius(sigma_s),
                    BF_FIR_MAX_RADIUS);
    if (spatial == BF_SPATIAL_IIR && W > kIirMaxWide)
        return fail(BF_EUNSUPPORTED, "IIR mode supports widths up to %d", kIirMaxWide);
    if (spatial == BF_SPATIAL_BOX && W > kBoxMaxW)
        return fail(BF_EUNSUPPORTED, "box mode supports widths up to %d", kBoxMaxW);
    return BF_OK;
}

GPParams make_params(const float *img, float *out, int H, int W, int pitch, double sigma_r, int N,
                     unsigned flags, char *ws, const Layout &L, void *saved) {
    GPParams p;
    memset(&p, 0, sizeof p);
    p.img = img;
    p.out = out;
    p.H = H;
    p.W = W;
    p.pitch = pitch;
    p.N = N;
    p.C = N + 2;
    p.center = center_code(flags);
    p.sigma_r = sigma_r;
    p.inv_sigma_r = 1.0 / sigma_r;
    p.xlim = range_limit(N);
    p.parts = (const Partial *)(ws + L.parts);
    p.nparts = H < kMaxParts ? H : kMaxParts;
    p.status = (int *)(ws + L.status);
    p.stats = (Stats *)(ws + L.stats);
    p.saved = saved;
    for (int n = 0; n < kMaxC + 3; ++n) {
        p.sq[n] = sqrt((double)n);
        p.isq[n] = n > 0 ? 1.0 / sqrt((double)n) : 0.0;
        p.rm[n] = n > 0 ? sqrt((double)n + 1.0) / (double)n : 0.0;
        p.inv[n] = n > 0 ? 1.0 / (double)n : 0.0;
    }
    return p;
}

FirTaps make_taps(double sigma_s, int R) {
    FirTaps t;
    memset(&t, 0, sizeof t);
    for (int d = 0; d <= R; ++d) t.k[d] = (float)exp(-(double)d * d / (2.0 * sigma_s * sigma_s));
    return t;
}

// Deriche's fourth-order recursive Gaussian (published constants): for t >= 0,
//   h(t) = (a0 cos(w0 t) + a1 sin(w0 t)) e^{-b0 t} + (c0 cos(w1 t) + c1 sin(w1 t)) e^{-b1 t},
// t = |d| / sigma_s.  Each damped sinusoid alpha cos(w t) + beta sin(w t) e^{-l t}
// sampled at integers is the impulse response of the second-order section
//   y_n = alpha x_n + r (beta sin th - alpha cos th) x_{n-1} + 2 r cos th y_{n-1} - r^2 y_{n-2},
// th = w / sigma_s, r = e^{-l / sigma_s}; its strictly anticausal half uses
// m1 = n1 - n0 d1, m2 = -n0 d2.
void mat2_mul(const double *A, const double *B, double *C) {
    double c0 = A[0] * B[0] + A[1] * B[2], c1 = A[0] * B[1] + A[1] * B[3];
    double c2 = A[2] * B[0] + A[3] * B[2], c3 = A[2] * B[1] + A[3] * B[3];
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}
void mat2_pow(const double *A, long m, double *R) {
    double base[4] = {A[0], A[1], A[2], A[3]};
    R[0] = 1; R[1] = 0; R[2] = 0; R[3] = 1;
    while (m > 0) {
        if (m & 1) mat2_mul(R, base, R);
        mat2_mul(base, base, base);
        m >>= 1;
    }
}

IirCoef make_iir(double sigma_s, int B, int L) {
    static const double al[2] = {1.680, -0.6803}, be[2] = {3.735, -0.2598};
    static const double la[2] = {1.783, 1.723}, om[2] = {0.6318, 1.997};
    IirCoef c;
    memset(&c, 0, sizeof c);
    for (int s = 0; s < 2; ++s) {
        const double th = om[s] / sigma_s, r = exp(-la[s] / sigma_s);
        const double n0 = al[s], n1 = r * (be[s] * sin(th) - al[s] * cos(th));
        const double d1 = -2.0 * r * cos(th), d2 = r * r;
        c.n0[s] = (float)n0;
        c.n1[s] = (float)n1;
        c.d1[s] = (float)d1;
        c.d2[s] = (float)d2;
        c.m1[s] = (float)(n1 - n0 * d1);
        c.m2[s] = (float)(-n0 * d2);
        const double Phi[4] = {-d1, -d2, 1.0, 0.0};
        double M[4];
        mat2_pow(Phi, B, M);
        for (int q = 0; q < 4; ++q) c.phiB[s][q] = (float)M[q];
        for (int j = 0; j < 6; ++j) {
            mat2_pow(Phi, (long)L << j, M);
            for (int q = 0; q < 4; ++q) c.phiL[s][j][q] = (float)M[q];
        }
        mat2_pow(Phi, 64L * L, M);
        for (int q = 0; q < 4; ++q) c.phiW[s][q] = (float)M[q];

    }
    return c;
}

// Coefficients of the row pass (hrow2) for chunks of L samples: the section
// coefficients of make_iir and Phi^(L 2^j), j = 0..9.
RowCoef make_row_coef(double sigma_s, int L) {
    const IirCoef ic = make_iir(sigma_s, 32, L);
    RowCoef c;
    memset(&c, 0, sizeof c);
    for (int s = 0; s < 2; ++s) {
        c.n0[s] = ic.n0[s];
        c.n1[s] = ic.n1[s];
        c.m1[s] = ic.m1[s];
        c.m2[s] = ic.m2[s];
        c.d1[s] = ic.d1[s];
        c.d2[s] = ic.d2[s];
        const double Phi[4] = {-(double)ic.d1[s], -(double)ic.d2[s], 1.0, 0.0};
        for (int j = 0; j < 10; ++j) {
            double M[4];
            mat2_pow(Phi, (long)L << j, M);
            for (int q = 0; q < 4; ++q) c.pw[s][j][q] = (float)M[q];
        }
        for (int i = 0; i < kRowMaxL; ++i) {
            double M[4];
            mat2_pow(Phi, i + 1, M);
            c.hom[i][2 * s] = (float)M[0];
            c.hom[i][2 * s + 1] = (float)M[1];
        }
    }
    return c;
}

// The same recursion differentiated in log sigma_s (theta = w / s and
// r = e^{-l / s} give theta' = -theta, r' = r l / s), and the band transfer
// blocks of the tangent system [[Phi, 0], [Phi', Phi]] over the band lengths of
// the backward passes (Phi' = [[-d1', -d2'], [0, 0]]).
IirTan make_iir_tan(double sigma_s) {
    static const double al[2] = {1.680, -0.6803}, be[2] = {3.735, -0.2598};
    static const double la[2] = {1.783, 1.723}, om[2] = {0.6318, 1.997};
    IirTan c;
    memset(&c, 0, sizeof c);
    for (int s = 0; s < 2; ++s) {
        const double th = om[s] / sigma_s, r = exp(-la[s] / sigma_s);
        const double dth = -th, dr = r * la[s] / sigma_s;
        const double cs = cos(th), sn = sin(th);
        const double n0 = al[s], n1 = r * (be[s] * sn - al[s] * cs);
        const double d1 = -2.0 * r * cs, d2 = r * r;
        const double dn1 = dr * (be[s] * sn - al[s] * cs) + r * dth * (be[s] * cs + al[s] * sn);
        const double dd1 = -2.0 * dr * cs + 2.0 * r * sn * dth;
        const double dd2 = 2.0 * r * dr;
        c.n0[s] = (float)n0;
        c.n1[s] = (float)n1;
        c.d1[s] = (float)d1;
        c.d2[s] = (float)d2;
        c.m1[s] = (float)(n1 - n0 * d1);
        c.m2[s] = (float)(-n0 * d2);
        c.tn1[s] = (float)dn1;
        c.td1[s] = (float)dd1;
        c.td2[s] = (float)dd2;
        c.tm1[s] = (float)(dn1 - n0 * dd1);
        c.tm2[s] = (float)(-n0 * dd2);
        const double A[16] = {-d1, -d2, 0, 0, 1, 0, 0, 0, -dd1, -dd2, -d1, -d2, 0, 0, 1, 0};
        for (int which = 0; which < 2; ++which) {
            const int B = which == 0 ? kBwdBV : kBwdBH;
            double M[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
            for (int k = 0; k < B; ++k) {
                double T[16];
                for (int i = 0; i < 4; ++i)
                    for (int j = 0; j < 4; ++j) {
                        double v = 0.0;
                        for (int q = 0; q < 4; ++q) v += A[4 * i + q] * M[4 * q + j];
                        T[4 * i + j] = v;
                    }
                memcpy(M, T, sizeof M);
            }
            float *phi = which == 0 ? c.phiV[s] : c.phiH[s];
            float *psi = which == 0 ? c.psiV[s] : c.psiH[s];
            phi[0] = (float)M[0]; phi[1] = (float)M[1]; phi[2] = (float)M[4]; phi[3] = (float)M[5];
            psi[0] = (float)M[8]; psi[1] = (float)M[9]; psi[2] = (float)M[12]; psi[3] = (float)M[13];
        }
    }
    return c;
}

struct BwdLayout {
    size_t parts, status, stats, bparts, corr, cv, pt, qt, chz, total;
    int Hp;
};

BwdLayout bwd_layout(int H, int W, int N, unsigned spatial) {
    BwdLayout L;
    memset(&L, 0, sizeof L);
    const bool iir = spatial == BF_SPATIAL_IIR;
    size_t off = 0;
    L.parts = off;
    off = align256(off + sizeof(Partial) * kMaxParts);
    L.status = off;
    off = align256(off + 16);
    L.stats = off;
    off = align256(off + sizeof(Stats));
    L.bparts = off;
    off = align256(off + sizeof(BwdPartial) * (size_t)(iir ? bwd_iir_parts(H, W) : bwd_tiles(H, W)));
    L.corr = off;
    off = align256(off + sizeof(double));
    if (iir) {
        const size_t C = (size_t)N + 2;
        L.Hp = ((H + 63) / 64) * 64;
        const size_t nbv = ((size_t)H + kBwdBV - 1) / kBwdBV, nbh = ((size_t)W + kBwdBH - 1) / kBwdBH;
        L.cv = off;
        off = align256(off + sizeof(float) * nbv * C * 16 * (size_t)W);
        L.pt = off;
        off = align256(off + sizeof(float) * C * (size_t)W * (size_t)L.Hp);
        L.qt = off;
        off = align256(off + sizeof(float) * C * (size_t)W * (size_t)L.Hp);
        L.chz = off;
        off = align256(off + sizeof(float) * nbh * C * 16 * (size_t)L.Hp);
    }
    L.total = off;
    return L;
}

}  // namespace

// Helpers shared with the batched path (batched.hip).
namespace bfgp {
IirShape iir_shape(int H, int W, int C, bool batch, bool rows32) {
    IirShape sh;
    const long cols = (W + 63) / 64;  // one wave per 64 columns of one band
    // band height: 64 rows once the image gives at least kBand64Waves column
    // waves at that height (half the band carries of 32 rows: 11 instead of 22
    // bytes per pixel written by the end-state pass and read by the column
    // pass, and half the resolve's traffic; measured on MI355X: 4096^2 1.30 ->
    // 1.21 ms, 2048^2 0.35 -> 0.34 ms), else 32 (more waves: 1024^2 is 0.11
    // ms at 32 rows and 0.12 at 64).  A batch plan keeps 32 for all images,
    // and so do the callers that run 32-row bands only (rows32: the joint
    // filter, whose three arrays of band samples would not fit the registers
    // of 64-row bands, and the volume filter).
    int B = g_band_rows.load();
    if (B != 32 && B != 64) B = (!batch && !rows32 && cols * ((H + 63) / 64) >= kBand64Waves) ? 64 : 32;
    sh.B = B;
    // channel groups of the column passes: each repeats the band's channel
    // generation up to its first channel, so only images with too few waves
    // are split
    int G = g_col_groups.load();
    if (G < 1 && batch) G = 1;
    if (G < 1) {
        const long waves = cols * ((H + B - 1) / B);
        G = (int)((kTargetWaves + waves - 1) / waves);
        if (G > 8) G = 8;
    }
    if (G < 1) G = 1;
    if (G > C) G = C;
    sh.G = G;
    // row pass: the fewest waves that hold the row at 16 samples per thread,
    // then the shortest chunk (a multiple of 4 samples) that still covers it
    // (fewer idle lanes), and channel groups until the rows give enough waves
    // (each group adds an LDS hand-over, so no more than needed)
    sh.nseg = 1;
    sh.T = (int)(((W + kRowMaxL * 64 - 1) / (kRowMaxL * 64)) * 64);
    sh.L = kRowMaxL;
    for (int l = 4; l < kRowMaxL; l += 4)
        if (sh.T * l >= W) {
            sh.L = l;
            break;
        }
    if (sh.T > 512) {
        // rows wider than 8192: segments of 512 threads x 16 samples
        sh.T = 512;
        sh.L = kRowMaxL;
        sh.nseg = (W + kRowSeg - 1) / kRowSeg;
    }
    int Gr = g_row_groups.load();
    if (Gr < 1 && batch) Gr = 1;
    if (Gr < 1) {
        // the row pass holds three waves per SIMD (its registers): as many
        // channel groups as fill that once, and no more (a second, partial
        // round costs more than the groups gain: 1024^2 takes 104 us for the
        // forward with three groups, 110 with two and 116 with four)
        const long waves = (long)H * (sh.T / 64);
        Gr = (int)(kRowTargetWaves / waves);
        if (Gr > 4) Gr = 4;
    }
    if (Gr > 512 / sh.T) Gr = 512 / sh.T;
    if (Gr > C) Gr = C;
    if (Gr < 1 || sh.nseg > 1) Gr = 1;
    while (Gr > 1 && hrow2_smem_bytes(sh.T, Gr, sh.L) > 65536) --Gr;
    sh.Gr = Gr;
    // the row pass that stores the saved terms, the joint filter's and the
    // batched path's: at most 16 samples per thread
    sh.To = (((W + 15) / 16 + 63) / 64) * 64;
    sh.Lo = 16;
    for (int l = 4; l < 16; l += 4)
        if (sh.To * l >= W) {
            sh.Lo = l;
            break;
        }
    int Gro = g_row_groups.load();
    if (Gro < 1 && batch) Gro = 1;
    if (Gro < 1) {
        const long waves = (long)H * (sh.To / 64);
        Gro = (int)((kTargetWaves + waves - 1) / waves);
        if (Gro > 4) Gro = 4;
    }
    if (sh.To <= 512 && Gro > 512 / sh.To) Gro = 512 / sh.To;
    if (Gro > C) Gro = C;
    if (Gro < 1) Gro = 1;
    while (Gro > 1 && hrow_smem_bytes(sh.To, Gro, sh.Lo) > 65536) --Gro;
    sh.Gro = Gro;
    // stack pitch: the image columns rounded up to 4, then the zero pad that
    // the loads of either row pass reach (a chunk that straddles the row end
    // reads L + 2 columns past it; chunks wholly past the row end read the pad
    // at the rounded width), rounded up to a 128-byte line so that every stack
    // row starts on a line
    const int W4 = (W + 3) & ~3;
    const int Lm = sh.L > sh.Lo ? sh.L : sh.Lo;
    sh.P = ((W4 + Lm + 2 + 31) / 32) * 32;
    sh.Hs = ((H + B - 1) / B) * B;
    return sh;
}
GPParams gp_params_for(const float *img, float *out, int H, int W, int pitch, double sigma_r, int N, unsigned flags,
                       const Partial *parts, int nparts, int *status, Stats *stats) {
    Layout L;
    L.parts = 0;
    L.status = 0;
    L.stats = 0;
    GPParams p = make_params(img, out, H, W, pitch, sigma_r, N, flags, (char *)0, L, nullptr);
    p.parts = parts;
    p.nparts = nparts;
    p.status = status;
    p.stats = stats;
    return p;
}
int gp_forward_check(const float *img, const float *out, int H, int W, int pitch, double sigma_s, double sigma_r,
                     int N, unsigned flags, const void *saved, size_t *ws_need) {
    int rc;
    if ((rc = check_image(img, out, H, W, pitch))) return rc;
    if ((rc = check_params(sigma_s, sigma_r, N))) return rc;
    if (flags & ~(BF_SPATIAL_MASK | BF_CENTER_MASK)) return fail(BF_EINVAL, "unknown flag bits 0x%x", flags);
    if ((flags & BF_CENTER_MASK) == 12u) return fail(BF_EINVAL, "invalid flag combination");
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if ((rc = check_spatial(spatial, sigma_s, W))) return rc;
    if (spatial == BF_SPATIAL_BOX && saved)
        return fail(BF_EUNSUPPORTED, "the box mode has no backward pass (pass saved = NULL)");
    if (spatial == BF_SPATIAL_IIR && saved && W > kIirMaxW)
        return fail(BF_EUNSUPPORTED, "the saved terms of the IIR mode need widths up to %d", kIirMaxW);
    if ((const void *)img == (const void *)out) return fail(BF_EINVAL, "img and out must not alias");
    *ws_need = gp_layout(H, W, N, spatial).total;
    return BF_OK;
}
IirCoef iir_coef_for(double sigma_s, int B, int L) { return make_iir(sigma_s, B, L); }
RowCoef row_coef_for(double sigma_s, int L) { return make_row_coef(sigma_s, L); }
FirTaps fir_taps_for(double sigma_s, int R) { return make_taps(sigma_s, R); }
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace bfgp

extern "C" {

int bf_version(void) { return 10000; }

const char *bf_last_error(void) { return g_err.c_str(); }

unsigned bf_gp_resolve_spatial(double sigma_s, unsigned flags) { return resolve_spatial(0, sigma_s, flags); }

unsigned bf_gp_resolve_spatial_for(int H, int W, double sigma_s, unsigned flags) {
    return resolve_spatial(H > 0 && W > 0 ? (long long)H * W : 0, sigma_s, flags);
}

int bf_gp_set_fir_crossover_table(const long long *max_pixels, const int *radius, int count) {
    if (count < 0 || count > kMaxCrossTable) return fail(BF_EINVAL, "crossover table of %d entries (0..%d)", count, kMaxCrossTable);
    if (count > 0 && (!max_pixels || !radius)) return fail(BF_EINVAL, "null crossover table");
    for (int k = 0; k < count; ++k) {
        if (max_pixels[k] < 1 || (k > 0 && max_pixels[k] <= max_pixels[k - 1]))
            return fail(BF_EINVAL, "crossover table pixel counts must be positive and increasing");
        if (radius[k] < 0 || radius[k] > BF_FIR_MAX_RADIUS)
            return fail(BF_EINVAL, "crossover radius %d outside 0..%d", radius[k], BF_FIR_MAX_RADIUS);
    }
    std::lock_guard<std::mutex> g(g_cross_mu);
    for (int k = 0; k < count; ++k) {
        g_cross_px[k] = max_pixels[k];
        g_cross_r[k] = radius[k];
    }
    g_cross_n = count;
    return BF_OK;
}

int bf_gp_get_fir_crossover_table(long long *max_pixels, int *radius, int max) {
    if (max < 0 || (max > 0 && (!max_pixels || !radius))) return fail(BF_EINVAL, "bad table buffers");
    std::lock_guard<std::mutex> g(g_cross_mu);
    const int n = g_cross_n < max ? g_cross_n : max;
    for (int k = 0; k < n; ++k) {
        max_pixels[k] = g_cross_px[k];
        radius[k] = g_cross_r[k];
    }
    return g_cross_n;
}

int bf_gp_set_fir_crossover(int radius) {
    if (radius < 0 || radius > BF_FIR_MAX_RADIUS) return fail(BF_EINVAL, "crossover radius %d outside 0..%d", radius, BF_FIR_MAX_RADIUS);
    g_fir_crossover.store(radius);
    return BF_OK;
}

int bf_gp_get_fir_crossover(void) { return g_fir_crossover.load(); }

int bf_gp_set_iir_tuning(int band_rows, int col_groups, int row_groups) {
    if (band_rows != 0 && band_rows != 32 && band_rows != 64) return fail(BF_EINVAL, "band rows %d not 0, 32 or 64", band_rows);
    if (col_groups < 0 || col_groups > 8) return fail(BF_EINVAL, "column groups %d outside 0..8", col_groups);
    if (row_groups < 0 || row_groups > 8) return fail(BF_EINVAL, "row groups %d outside 0..8", row_groups);
    g_band_rows.store(band_rows);
    g_col_groups.store(col_groups);
    g_row_groups.store(row_groups);
    return BF_OK;
}

int bf_gp_iir_shape(int H, int W, int N, int *shape) {
    if (!shape) return fail(BF_EINVAL, "null shape");
    if (H < 1 || W < 1 || W > kIirMaxWide || N < 0 || N > BF_MAX_DEGREE) return fail(BF_EINVAL, "bad image size or degree");
    const IirShape sh = iir_shape(H, W, N + 2);
    shape[0] = sh.B;
    shape[1] = sh.G;
    shape[2] = sh.L;
    shape[3] = sh.T;
    shape[4] = sh.Gr;
    return BF_OK;
}

size_t bf_gp_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags) {
    if (H < 1 || W < 1 || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s)) return 0;
    return gp_layout(H, W, N, resolve_spatial((long long)H * W, sigma_s, flags)).total;
}

int bf_gp_forward(const float *img, float *out, int H, int W, int pitch, double sigma_s, double sigma_r, int N,
                  unsigned flags, void *saved, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    size_t need = 0;
    if ((rc = gp_forward_check(img, out, H, W, pitch, sigma_s, sigma_r, N, flags, saved, &need))) return rc;
    if (!ws) return fail(BF_EINVAL, "null workspace");
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    const Layout L = gp_layout(H, W, N, spatial);
    if (ws_bytes < L.total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    GPParams p = make_params(img, out, H, W, pitch, sigma_r, N, flags, w, L, saved);
    hipError_t e = launch_stats(p, false, s);
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    if (spatial == BF_SPATIAL_FIR) {
        const int R = fir_radius(sigma_s);
        e = launch_fir(p, make_taps(sigma_s, R), R, saved != nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "FIR launch");
    } else if (spatial == BF_SPATIAL_BOX) {
        const BoxShape sh = box_shape(H, W, N + 2, box_radius(sigma_s, H, W));
        e = launch_box(p, sh, (float *)(w + L.stack), s);
        if (e != hipSuccess) return hip_fail(e, "box launch");
    } else {
        const IirShape sh = iir_shape(H, W, N + 2);
        e = launch_iir(p, make_iir(sigma_s, sh.B, sh.Lo), make_row_coef(sigma_s, sh.L), sh, (float *)(w + L.carry),
                       (float *)(w + L.stack), saved != nullptr, false, s, (float *)(w + L.segst));
        if (e != hipSuccess) return hip_fail(e, "IIR launch");
    }
    return BF_OK;
}

size_t bf_gp_joint_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags) {
    if (H < 1 || W < 1 || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s)) return 0;
    if ((flags & BF_SPATIAL_MASK) == BF_SPATIAL_FIR || (flags & BF_SPATIAL_MASK) == BF_SPATIAL_BOX) return 0;
    return gp_layout_c(H, W, 2 * (N + 1), BF_SPATIAL_IIR, true).total;
}

int bf_gp_joint_forward(const float *guide, const float *data, float *out, int H, int W, int pitch, double sigma_s,
                        double sigma_r, int N, unsigned flags, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if ((rc = check_image(guide, out, H, W, pitch))) return rc;
    if (!data) return fail(BF_EINVAL, "null data pointer");
    if ((rc = check_params(sigma_s, sigma_r, N))) return rc;
    if (!ws) return fail(BF_EINVAL, "null workspace");
    if (flags & ~(BF_SPATIAL_MASK | BF_CENTER_MASK)) return fail(BF_EINVAL, "unknown flag bits 0x%x", flags);
    if ((flags & BF_CENTER_MASK) == 12u) return fail(BF_EINVAL, "invalid flag combination");
    if ((const void *)out == (const void *)guide || (const void *)out == (const void *)data)
        return fail(BF_EINVAL, "out must not alias the guide or the data");
    if ((flags & BF_SPATIAL_MASK) == BF_SPATIAL_FIR || (flags & BF_SPATIAL_MASK) == BF_SPATIAL_BOX)
        return fail(BF_EUNSUPPORTED, "the joint filter runs in the recursive (IIR) spatial mode");
    if ((rc = check_spatial(BF_SPATIAL_IIR, sigma_s, W))) return rc;
    if (W > kIirMaxW) return fail(BF_EUNSUPPORTED, "the joint filter supports widths up to %d", kIirMaxW);
    const int C = 2 * (N + 1);
    const Layout L = gp_layout_c(H, W, C, BF_SPATIAL_IIR, true);
    if (ws_bytes < L.total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    GPParams p = make_params(guide, out, H, W, pitch, sigma_r, N, flags, w, L, nullptr);
    p.C = C;
    p.data = data;
    // the channels reach degree N only (not N + 1)
    p.xlim = range_limit(N - 1);
    hipError_t e = launch_stats(p, false, s);
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    const IirShape sh = iir_shape(H, W, C, false, true);
    e = launch_iir(p, make_iir(sigma_s, sh.B, sh.Lo), make_row_coef(sigma_s, sh.L), sh, (float *)(w + L.carry),
                   (float *)(w + L.stack), false, true,
                   s);
    if (e != hipSuccess) return hip_fail(e, "IIR launch");
    return BF_OK;
}

// Workspace of a volume forward (recursive mode): statistics, then the time
// carries and stack S1, the per-frame column carries and the row-pass stack S2.
struct VolLayout {
    size_t parts, status, stats, carry_z, s1, carry_y, s2, total;
    IirShape shz, shs;
    int Hs;
};

VolLayout vol_layout(int T, int H, int W, int N) {
    VolLayout L;
    memset(&L, 0, sizeof L);
    const size_t C = (size_t)N + 2, HW = (size_t)H * W;
    // the volume kernels run 32-row bands only (also under a band-rows override)
    L.shz = iir_shape(T, (int)HW, (int)C, false, true);
    L.shz.B = 32;
    L.shs = iir_shape(T * H, W, (int)C, false, true);
    L.shs.B = 32;
    L.Hs = ((H + 31) / 32) * 32;
    const size_t nbz = ((size_t)T + 31) / 32, nby = ((size_t)H + 31) / 32;
    size_t off = 0;
    L.parts = off;
    off = align256(off + sizeof(Partial) * kMaxParts);
    L.status = off;
    off = align256(off + 16);
    L.stats = off;
    off = align256(off + sizeof(Stats));
    L.carry_z = off;
    off = align256(off + sizeof(float) * nbz * C * 8 * HW);
    L.s1 = off;
    off = align256(off + sizeof(float) * C * nbz * 32 * HW);
    L.carry_y = off;
    off = align256(off + sizeof(float) * (size_t)T * nby * C * 8 * (size_t)W);
    L.s2 = off;
    off = align256(off + sizeof(float) * (size_t)T * C * (size_t)L.Hs * (size_t)L.shs.P);
    L.total = off;
    return L;
}

bool vol_size_ok(int T, int H, int W) {
    return T >= 1 && H >= 1 && W >= 1 && W <= kIirMaxW && (long long)H * W < (1LL << 31) &&
           (long long)T * H < (1LL << 31) && (double)T * H * W < (double)(1LL << 40);
}

size_t bf_gp_volume_workspace_bytes(int T, int H, int W, int N, double sigma_s, double sigma_t, unsigned flags) {
    if (!vol_size_ok(T, H, W) || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s) || !finite_pos(sigma_t)) return 0;
    if ((flags & BF_SPATIAL_MASK) == BF_SPATIAL_FIR || (flags & BF_SPATIAL_MASK) == BF_SPATIAL_BOX) return 0;
    return vol_layout(T, H, W, N).total;
}

int bf_gp_volume_forward(const float *vol, float *out, int T, int H, int W, double sigma_s, double sigma_t,
                         double sigma_r, int N, unsigned flags, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    if (!vol || !out) return fail(BF_EINVAL, "null volume pointer");
    if (T < 1 || H < 1 || W < 1) return fail(BF_EINVAL, "volume size %dx%dx%d must be at least 1x1x1", T, H, W);
    if (!vol_size_ok(T, H, W)) return fail(BF_EUNSUPPORTED, "volume %dx%dx%d too large (rows up to %d wide)", T, H, W, kIirMaxW);
    if ((rc = check_params(sigma_s, sigma_r, N))) return rc;
    if (!finite_pos(sigma_t)) return fail(BF_EINVAL, "sigma_t must be finite and > 0");
    if (!ws) return fail(BF_EINVAL, "null workspace");
    if (flags & ~(BF_SPATIAL_MASK | BF_CENTER_MASK)) return fail(BF_EINVAL, "unknown flag bits 0x%x", flags);
    if ((flags & BF_CENTER_MASK) == 12u) return fail(BF_EINVAL, "invalid flag combination");
    if ((const void *)vol == (const void *)out) return fail(BF_EINVAL, "vol and out must not alias");
    if ((flags & BF_SPATIAL_MASK) == BF_SPATIAL_FIR || (flags & BF_SPATIAL_MASK) == BF_SPATIAL_BOX)
        return fail(BF_EUNSUPPORTED, "volumes run in the recursive (IIR) spatial mode");
    const VolLayout L = vol_layout(T, H, W, N);
    if (ws_bytes < L.total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    Layout fl;
    memset(&fl, 0, sizeof fl);
    fl.parts = L.parts;
    fl.status = L.status;
    fl.stats = L.stats;
    // the volume as a (T H) x W image (statistics, and each frame's passes)
    GPParams ps = make_params(vol, out, T * H, W, W, sigma_r, N, flags, w, fl, nullptr);
    // the volume as a T x (H W) image (time direction)
    GPParams pz = ps;
    pz.H = T;
    pz.W = H * W;
    pz.pitch = H * W;
    VolumeBuffers vb;
    vb.carry_z = (float *)(w + L.carry_z);
    vb.S1 = (float *)(w + L.s1);
    vb.carry_y = (float *)(w + L.carry_y);
    vb.S2 = (float *)(w + L.s2);
    vb.Hs = L.Hs;
    hipError_t e = launch_volume(pz, ps, make_iir(sigma_t, 32, L.shz.Lo), make_iir(sigma_s, 32, L.shs.Lo),
                                 make_row_coef(sigma_s, L.shs.L), L.shz,
                                 L.shs, T, vb, s);
    if (e != hipSuccess) return hip_fail(e, "volume launch");
    return BF_OK;
}

// P(Poisson(lam) > N), summed from the tail side in log space (no
// cancellation when the tail is small).
static double poisson_tail(int N, double lam) {
    if (lam <= 0.0) return 0.0;
    const double ll = log(lam);
    double sum = 0.0;
    for (int k = N + 1; k < N + 4000; ++k) {
        const double term = exp(-lam + k * ll - lgamma(k + 1.0));
        sum += term;
        if (k > lam && term < 1e-18 * sum) break;
    }
    return sum;
}

int bf_gp_degree_for(double xmax, double eps) {
    if (!isfinite(xmax) || xmax < 0.0) return fail(BF_EINVAL, "xmax must be finite and >= 0");
    if (!(eps > 0.0 && eps < 1.0)) return fail(BF_EINVAL, "eps must lie in (0, 1)");
    const double lam = xmax * xmax;
    int n0 = (int)ceil(lam - 1.0);
    if (n0 < 0) n0 = 0;
    if (n0 & 1) ++n0;
    for (int N = n0; N <= BF_MAX_DEGREE; N += 2)
        if (poisson_tail(N, lam) <= eps) return N;
    return fail(BF_ERANGE, "no even degree up to %d bounds the weight error by %g at xmax %g", BF_MAX_DEGREE, eps, xmax);
}

int bf_gp_status(const void *ws, void *stream, int *status) {
    if (!ws || !status) return fail(BF_EINVAL, "null pointer");
    int v = 0;
    const Layout L = gp_layout(1, 1, 0, BF_SPATIAL_FIR);
    hipError_t e = hipMemcpyAsync(&v, (const char *)ws + L.status, sizeof v, hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "status copy");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "status sync");
    *status = v;
    return BF_OK;
}


size_t bf_gp_backward_workspace_bytes(int H, int W, int N, double sigma_s, unsigned flags) {
    if (H < 1 || W < 1 || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s)) return 0;
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if (spatial == BF_SPATIAL_BOX) return 0;
    return bwd_layout(H, W, N, spatial).total;
}

static int bwd_check(const float *img, const float *grad_out, const void *saved, int H, int W, int pitch,
                     double sigma_s, double sigma_r, int N, unsigned flags, const float *grad_img, const void *ws,
                     unsigned *spatial_out) {
    int rc;
    if ((rc = check_image(img, grad_out, H, W, pitch))) return rc;
    if ((rc = check_params(sigma_s, sigma_r, N))) return rc;
    if (!saved) return fail(BF_EINVAL, "null saved buffer");
    if (!ws) return fail(BF_EINVAL, "null workspace");
    if (flags & ~(BF_SPATIAL_MASK | BF_CENTER_MASK)) return fail(BF_EINVAL, "unknown flag bits 0x%x", flags);
    if ((flags & BF_CENTER_MASK) == 12u) return fail(BF_EINVAL, "invalid flag combination");
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if (spatial == BF_SPATIAL_BOX) return fail(BF_EUNSUPPORTED, "the box mode has no backward pass");
    if ((rc = check_spatial(spatial, sigma_s, W))) return rc;
    if (spatial == BF_SPATIAL_IIR && W > kIirMaxW)
        return fail(BF_EUNSUPPORTED, "the IIR backward supports widths up to %d", kIirMaxW);
    if ((flags & BF_CENTER_MASK) == BF_CENTER_MIDRANGE)
        return fail(BF_EUNSUPPORTED, "the backward pass supports the mean centre or no centring");
    if (grad_img && ((const void *)grad_img == (const void *)img || (const void *)grad_img == (const void *)grad_out))
        return fail(BF_EINVAL, "grad_img must not alias img or grad_out");
    *spatial_out = spatial;
    return BF_OK;
}

// The IIR backward's buffers and channel groups for image buffers at the given
// pointers and the workspace layout L at w; nimg: the images of a stacked call.
static BwdIir bwd_iir_args(const float *grad_out, const void *saved, float *grad_img, char *w, const BwdLayout &L,
                           int H, int W, int N, int nimg = 1) {
    const size_t npx = (size_t)H * W;
    BwdIir b;
    memset(&b, 0, sizeof b);
    b.grad_out = grad_out;
    b.rho = (const float *)saved;
    b.drho = (const float *)saved + npx;
    b.Dp = (const double *)((const float *)saved + 2 * npx);
    b.grad_img = grad_img;
    b.cv = (float *)(w + L.cv);
    b.PT = (float *)(w + L.pt);
    b.QT = (float *)(w + L.qt);
    b.chz = (float *)(w + L.chz);
    b.bparts = (BwdPartial *)(w + L.bparts);
    b.Hp = L.Hp;
    bwd_iir_groups(H, W, N + 2, nimg, &b.Gv, &b.Gh);
    // the tuning overrides of the column and row channel groups apply here too
    if (g_col_groups.load() > 0) b.Gv = g_col_groups.load() < N + 2 ? g_col_groups.load() : N + 2;
    if (g_row_groups.load() > 0) {
        const int gr = g_row_groups.load() < 4 ? g_row_groups.load() : 4;
        b.Gh = gr < N + 2 ? gr : N + 2;
    }
    return b;
}

static FirTaps2 bwd_taps(double sigma_s, int R) {
    FirTaps2 t;
    memset(&t, 0, sizeof t);
    for (int d = 0; d <= R; ++d) {
        const double q = (double)d * d / (sigma_s * sigma_s);
        t.k[d] = (float)exp(-0.5 * q);
        t.kt[d] = (float)(q * exp(-0.5 * q));
    }
    return t;
}

int bf_gp_backward(const float *img, const float *grad_out, const void *saved, int H, int W, int pitch,
                   double sigma_s, double sigma_r, int N, unsigned flags, float *grad_img, double *grad_log_sigma_s,
                   double *grad_log_sigma_r, void *ws, size_t ws_bytes, void *stream) {
    int rc;
    unsigned spatial = 0;
    if ((rc = bwd_check(img, grad_out, saved, H, W, pitch, sigma_s, sigma_r, N, flags, grad_img, ws, &spatial)))
        return rc;
    const BwdLayout L = bwd_layout(H, W, N, spatial);
    if (ws_bytes < L.total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    Layout fl;
    fl.parts = L.parts;
    fl.status = L.status;
    fl.stats = L.stats;
    GPParams p = make_params(img, nullptr, H, W, pitch, sigma_r, N, flags, w, fl, const_cast<void *>(saved));
    hipError_t e = launch_stats(p, true, s);
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    if (spatial == BF_SPATIAL_IIR) {
        const BwdIir b = bwd_iir_args(grad_out, saved, grad_img, w, L, H, W, N);
        e = launch_bwd_iir(p, b, make_iir_tan(sigma_s), (double *)(w + L.corr), grad_log_sigma_s, grad_log_sigma_r, s);
        if (e != hipSuccess) return hip_fail(e, "backward launch");
        return BF_OK;
    }
    const int R = fir_radius(sigma_s);
    const FirTaps2 t = bwd_taps(sigma_s, R);
    BwdParams b;
    b.grad_out = grad_out;
    b.saved = (const float *)saved;
    b.grad_img = grad_img;
    b.bparts = (BwdPartial *)(w + L.bparts);
    e = launch_bwd(p, b, t, R, (double *)(w + L.corr), grad_log_sigma_s, grad_log_sigma_r, s);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return BF_OK;
}

// ---- stacked batch --------------------------------------------------------------

// Per-image workspace slice and descriptor block of a stacked call.
static size_t stk_desc_bytes(int B) { return align256(sizeof(GPParams) * (size_t)B); }

static int stk_check(int B, int H, int pitch, size_t img_stride, const void *a, const void *b) {
    if (B < 1) return fail(BF_EINVAL, "batch of %d images", B);
    if (img_stride < (size_t)H * (size_t)pitch) return fail(BF_EINVAL, "image stride smaller than an image");
    if ((double)img_stride * B >= (double)((size_t)1 << 40)) return fail(BF_EINVAL, "batch too large");
    // the two batches' element ranges must not overlap
    if (a && b) {
        const char *a0 = (const char *)a, *b0 = (const char *)b;
        const size_t span = sizeof(float) * (img_stride * (size_t)(B - 1) + (size_t)H * pitch);
        if (a0 < b0 + span && b0 < a0 + span) return fail(BF_EINVAL, "batches overlap");
    }
    return BF_OK;
}

size_t bf_gp_forward_stacked_workspace_bytes(int B, int H, int W, int N, double sigma_s, unsigned flags) {
    if (B < 1 || H < 1 || W < 1 || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s)) return 0;
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if (spatial == BF_SPATIAL_BOX) return 0;
    return stk_desc_bytes(B) + (size_t)B * align256(gp_layout(H, W, N, spatial).total);
}

int bf_gp_forward_stacked(const float *img, float *out, int B, int H, int W, int pitch, size_t img_stride,
                          double sigma_s, double sigma_r, int N, unsigned flags, void *saved, void *ws,
                          size_t ws_bytes, void *stream) {
    int rc;
    size_t need = 0;
    if ((rc = gp_forward_check(img, out, H, W, pitch, sigma_s, sigma_r, N, flags, saved, &need))) return rc;
    if ((rc = stk_check(B, H, pitch, img_stride, img, out))) return rc;
    if (!ws) return fail(BF_EINVAL, "null workspace");
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if (spatial == BF_SPATIAL_BOX) return fail(BF_EUNSUPPORTED, "the stacked path runs the FIR and IIR modes");
    if (spatial == BF_SPATIAL_IIR && W > kIirMaxW)
        return fail(BF_EUNSUPPORTED, "the stacked IIR path supports widths up to %d", kIirMaxW);
    const Layout L = gp_layout(H, W, N, spatial);
    const size_t slice = align256(L.total), total = stk_desc_bytes(B) + (size_t)B * slice;
    if (ws_bytes < total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, total);
    hipStream_t s = (hipStream_t)stream;
    char *w0 = (char *)ws + stk_desc_bytes(B);
    GPParams *pd = (GPParams *)ws;
    const GPParams p0 = make_params(img, out, H, W, pitch, sigma_r, N, flags, w0, L, saved);
    StkOfs o;
    o.img = img_stride;
    o.ws = slice;
    o.saved = (size_t)16 * H * W;
    o.B = B;
    hipError_t e = launch_stk_setup(p0, o, pd, s);
    if (e == hipSuccess) e = launch_stk_stats(p0, pd, o, false, s);
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    if (spatial == BF_SPATIAL_FIR) {
        const int R = fir_radius(sigma_s);
        e = launch_stk_fir(p0, pd, o, make_taps(sigma_s, R), R, saved != nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "FIR launch");
    } else {
        const IirShape sh = iir_shape(H, W, N + 2);
        e = launch_stk_iir(p0, pd, o, make_iir(sigma_s, sh.B, sh.Lo), make_row_coef(sigma_s, sh.L), sh,
                           (float *)(w0 + L.carry), (float *)(w0 + L.stack), saved != nullptr, s);
        if (e != hipSuccess) return hip_fail(e, "IIR launch");
    }
    return BF_OK;
}

size_t bf_gp_backward_stacked_workspace_bytes(int B, int H, int W, int N, double sigma_s, unsigned flags) {
    if (B < 1 || H < 1 || W < 1 || N < 0 || N > BF_MAX_DEGREE || !finite_pos(sigma_s)) return 0;
    const unsigned spatial = resolve_spatial((long long)H * W, sigma_s, flags);
    if (spatial == BF_SPATIAL_BOX) return 0;
    return stk_desc_bytes(B) + align256(sizeof(double) * (size_t)B) +
           (size_t)B * align256(bwd_layout(H, W, N, spatial).total);
}

int bf_gp_backward_stacked(const float *img, const float *grad_out, const void *saved, int B, int H, int W, int pitch,
                           size_t img_stride, double sigma_s, double sigma_r, int N, unsigned flags, float *grad_img,
                           double *grad_log_sigma_s, double *grad_log_sigma_r, void *ws, size_t ws_bytes,
                           void *stream) {
    int rc;
    unsigned spatial = 0;
    if ((rc = bwd_check(img, grad_out, saved, H, W, pitch, sigma_s, sigma_r, N, flags, grad_img, ws, &spatial)))
        return rc;
    if ((rc = stk_check(B, H, pitch, img_stride, img, grad_img))) return rc;
    if ((rc = stk_check(B, H, pitch, img_stride, grad_out, grad_img))) return rc;
    const BwdLayout L = bwd_layout(H, W, N, spatial);
    const size_t slice = align256(L.total);
    const size_t total = stk_desc_bytes(B) + align256(sizeof(double) * (size_t)B) + (size_t)B * slice;
    if (ws_bytes < total) return fail(BF_ENOMEM, "workspace of %zu bytes, %zu needed", ws_bytes, total);
    hipStream_t s = (hipStream_t)stream;
    GPParams *pd = (GPParams *)ws;
    double *corr = (double *)((char *)ws + stk_desc_bytes(B));
    char *w0 = (char *)ws + stk_desc_bytes(B) + align256(sizeof(double) * (size_t)B);
    Layout fl;
    fl.parts = L.parts;
    fl.status = L.status;
    fl.stats = L.stats;
    const GPParams p0 = make_params(img, nullptr, H, W, pitch, sigma_r, N, flags, w0, fl, const_cast<void *>(saved));
    StkOfs o;
    o.img = img_stride;
    o.ws = slice;
    o.saved = (size_t)16 * H * W;
    o.B = B;
    hipError_t e = launch_stk_setup(p0, o, pd, s);
    if (e == hipSuccess) e = launch_stk_stats(p0, pd, o, true, s);
    if (e != hipSuccess) return hip_fail(e, "statistics launch");
    if (spatial == BF_SPATIAL_IIR) {
        const BwdIir b = bwd_iir_args(grad_out, saved, grad_img, w0, L, H, W, N, B);
        e = launch_stk_bwd_iir(p0, pd, b, o, make_iir_tan(sigma_s), corr, grad_log_sigma_s, grad_log_sigma_r, s);
    } else {
        const int R = fir_radius(sigma_s);
        BwdParams b;
        b.grad_out = grad_out;
        b.saved = (const float *)saved;
        b.grad_img = grad_img;
        b.bparts = (BwdPartial *)(w0 + L.bparts);
        e = launch_stk_bwd(p0, pd, b, o, bwd_taps(sigma_s, R), R, corr, grad_log_sigma_s, grad_log_sigma_r, s);
    }
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return BF_OK;
}

int bf_direct_forward(const float *img, float *out, int H, int W, int pitch, double sigma_s, double sigma_r,
                      int window, void *stream) {
    int rc;
    if ((rc = check_image(img, out, H, W, pitch))) return rc;
    if (!finite_pos(sigma_s) || !finite_pos(sigma_r)) return fail(BF_EINVAL, "sigma_s and sigma_r must be finite and > 0");
    const int win = window < 0 ? fir_radius(sigma_s) : window;
    if (win > kDirectMaxW) return fail(BF_EUNSUPPORTED, "window %d exceeds %d", win, kDirectMaxW);
    if ((const void *)img == (const void *)out) return fail(BF_EINVAL, "img and out must not alias");
    DirectArgs a;
    memset(&a, 0, sizeof a);
    a.img = img;
    a.out = out;
    a.H = H;
    a.W = W;
    a.pitch = pitch;
    a.win = win;
    const double log2e = 1.4426950408889634;
    a.cr = (float)(-log2e / (2.0 * sigma_r * sigma_r));
    for (int d = 0; d <= win; ++d) a.lk[d] = (float)(-log2e * (double)d * d / (2.0 * sigma_s * sigma_s));
    hipError_t e = launch_direct(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "direct launch");
    return BF_OK;
}

}  // extern "C"
