// Recursive (IIR) spatial Gaussian for the GP forward: Deriche's 4th-order
// approximation in parallel form, run causally and anticausally along columns
// and then along rows, with the FP64 recombination fused into the row pass.
//
// Each of the two second-order sections s of one direction computes
//   causal:      y_n = n0 x_n + n1 x_{n-1} - d1 y_{n-1} - d2 y_{n-2}
//   anticausal:  z_n = m1 x_{n+1} + m2 x_{n+2} - d1 z_{n+1} - d2 z_{n+2}
// from rest with zero input outside the image, and the 1-D output is the sum of
// the four recursions.  Its impulse response is Deriche's h(|d| / sigma_s) at
// every offset, so the filter is an exact zero-extended convolution with h.
//
// Column direction (lines = image columns, up to H long): lines are cut into
// bands of B rows.  Pass A runs each band from rest and stores the band's end
// states; pass B resolves the true incoming state of every band with the 2x2
// band transfer matrix; pass C reruns each band from its true state and writes
// the column-filtered channel stack.  Lanes own columns, so every load and store
// is a coalesced row segment.
//
// Row direction (fused with the recombination): one workgroup owns a full row;
// each thread owns a chunk of L samples.  Chunks run from rest, the chunk
// states are combined by a wave-level scan plus a cross-wave step, and the
// homogeneous response of the true incoming states is added back.
#pragma once
#include "common.hpp"

namespace bfgp {

constexpr int kIirMaxL = 16;
// End states by weighted sums: channel groups of at most kAggG channels, for
// stacks of at most kAggMaxC channels (unnormalised powers stay in FP32 up
// to degree 47; 4 groups of at most 12 channels).
constexpr int kAggG = 12, kAggMaxC = 48;

struct IirCoef {
    float n0[2], n1[2], m1[2], m2[2], d1[2], d2[2];
    float phiB[2][4];     // Phi^B, Phi = [[-d1, -d2], [1, 0]], row-major
    float phiL[2][6][4];  // Phi^(L 2^j), j = 0..5
    float phiW[2][4];     // Phi^(64 L)
};

// Weights of the band end states as sums over the band's inputs (the
// recursions' responses to unit inputs, agg_weight_task), computed once per
// call on the host for bands of up to kAggMaxB rows and passed by value: the
// kernels read them with scalar loads.  w[i * 8 + k]; one more row of eight
// as the read-ahead pad.
constexpr int kAggMaxB = 64;
struct AggW {
    float w[(kAggMaxB + 4) * 8];
};

// x^e for a small non-negative integer e (binary powering)
__device__ __forceinline__ double ipow(double x, int e) {
    double r = 1.0;
    while (e > 0) {
        if (e & 1) r *= x;
        x *= x;
        e >>= 1;
    }
    return r;
}

// One band of B rows in one column.  AGG: run from rest, write the band's end
// states (causal end, anticausal start).  !AGG: run from the resolved
// incoming states and write the column-filtered channel stack S[n][row][col].
//
// carry layout: carry[((band * C + n) * 8 + k) * W + col], k = 0..3 causal
// (section 0: y_{e}, y_{e-1}; section 1: same), k = 4..7 anticausal
// (section 0: z_a, z_{a+1}; section 1: same).
// sacc: LDS scratch of B * 64 floats (the causal outputs of the wave's 64
// columns while the anticausal pass runs), used only when !AGG.
// Channels [cb, ce) only: the channel recurrence still starts from u_0, so the
// values do not depend on how the channels are split across workgroups.
// JOINT (joint filter, range kernel on the guide p.img, average of p.data):
// stack channel 2n holds u_n(x) of the guide and 2n+1 holds u_n(x) f of the
// data, n = 0..N.
// STACKIN (a volume's row-direction pass): the channel values are read from a
// stack that an earlier pass filtered, channel n at src + n * src_cstride with
// rows of p.pitch, instead of being generated from the image.
// SHARED (G >= 2 channel groups of one band in one workgroup, this wave group
// g): the waves split the band's B + 3 rows of centred intensities and
// exp(-x^2/2) (and the joint data) between them and exchange them through
// `pro` in LDS, instead of each computing all of them.
template <int B, bool AGG, bool BIG, bool JOINT = false, bool STACKIN = false, bool SHARED = false>
__device__ __forceinline__ void vband(const GPParams &p, const IirCoef &c, const Stats &st, int col, int band,
                                      float *__restrict__ carry, float *__restrict__ S, int sp_pitch, float *sacc,
                                      int cb, int ce, const float *__restrict__ src = nullptr,
                                      size_t src_cstride = 0, float *pro = nullptr, int G = 1, int g = 0) {
    const int lane = threadIdx.x & 63;
    const int a = band * B;
    constexpr int NR = B + 3;  // rows a-1 .. a+B+1
    if constexpr (SHARED && !STACKIN) {
        // a column group lying wholly in the pad has nothing to share (the
        // test is uniform over the workgroup: its waves share the columns)
        if (col - lane < p.W) {
            // this wave's rows g, g + G, ... (at most (NR + 1) / 2 of them for
            // G >= 2), six loads in flight at a time
            constexpr int PER = (NR + 1) / 2, CH = 6;
            const int colc = col < p.W ? col : p.W - 1;
            for (int k0 = 0; k0 < PER; k0 += CH) {
                float f[CH], fd[JOINT ? CH : 1];
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int r = g + (k0 + k) * G;
                    const int row = a - 1 + (r < NR ? r : NR - 1);
                    const int rc = row < 0 ? 0 : (row >= p.H ? p.H - 1 : row);
                    f[k] = p.img[(size_t)rc * p.pitch + colc];
                    if constexpr (JOINT) fd[k] = p.data[(size_t)rc * p.pitch + colc];
                }
#pragma unroll
                for (int k = 0; k < CH; ++k) {
                    const int r = g + (k0 + k) * G;
                    if (r < NR) {
                        const float x = centred(f[k], st, p.inv_sigma_r);
                        pro[r * 64 + lane] = x;
                        pro[(NR + r) * 64 + lane] = gauss_u0(x, BIG ? big_shift(x) : 0);
                        if constexpr (JOINT) pro[(2 * NR + r) * 64 + lane] = fd[k];
                    }
                }
            }
            __syncthreads();
        }
    }
    // the stack holds every channel as rows(H) = H rounded up to a whole band
    // of rows with pitch sp_pitch, so every band stores all of its rows
    const int srows = ((p.H + B - 1) / B) * B;
    // lanes own columns and never exchange data.  Lanes on the stack's pad
    // columns [W, sp_pitch) store zeros there (the row pass reads them as the
    // zero extension of the image), lanes past the pad leave at once.
    if (col >= p.W) {
        if (!AGG && col < sp_pitch) {
            for (int n = cb; n < ce; ++n) {
                float *sp = S + ((size_t)n * srows + a) * sp_pitch + col;
#pragma unroll
                for (int i = 0; i < B; ++i) sp[(size_t)i * sp_pitch] = 0.f;
            }
        }
        return;
    }
    // rows a-1 .. a+B+1: every load is issued unconditionally from a clamped
    // row (so that all of them are in flight together), and samples outside
    // the image are zeroed afterwards
    constexpr int NG = STACKIN ? 1 : B + 3;  // samples of the generated channels
    float xv[NG], u[NG], dv[JOINT ? B + 3 : 1];
    if constexpr (!STACKIN) {
        if constexpr (SHARED) {
#pragma unroll
            for (int i = 0; i < NR; ++i) {
                xv[i] = pro[i * 64 + lane];
                u[i] = pro[(NR + i) * 64 + lane];
                if constexpr (JOINT) dv[i] = pro[(2 * NR + i) * 64 + lane];
            }
        } else {
#pragma unroll
            for (int i = 0; i < B + 3; ++i) {
                const int row = a - 1 + i;
                const int rc = row < 0 ? 0 : (row >= p.H ? p.H - 1 : row);
                xv[i] = p.img[(size_t)rc * p.pitch + col];
                if constexpr (JOINT) dv[i] = p.data[(size_t)rc * p.pitch + col];
            }
#pragma unroll
            for (int i = 0; i < B + 3; ++i) {
                xv[i] = centred(xv[i], st, p.inv_sigma_r);
                u[i] = gauss_u0(xv[i], BIG ? big_shift(xv[i]) : 0);
            }
        }
        // rows outside the image (a uniform test per row: only the first and
        // the last bands have any)
        if (a == 0) {
            xv[0] = 0.f;
            u[0] = 0.f;
        }
        if (a + B + 2 > p.H) {
#pragma unroll
            for (int i = 1; i < B + 3; ++i)
                if (a - 1 + i >= p.H) {
                    xv[i] = 0.f;
                    u[i] = 0.f;
                }
        }
        // advance u to the first channel's degree (the loop below advances it
        // on entering every degree n > 0: channel n, or channel 2n of a joint
        // stack)
        const int pre = JOINT ? ((cb & 1) ? cb >> 1 : (cb >> 1) - 1) : cb - 1;
        for (int n = 1; n <= pre; ++n) {
            const float isq = (float)p.isq[n];
#pragma unroll
            for (int i = 0; i < B + 3; ++i) u[i] *= xv[i] * isq;
        }
    }
    const size_t cstride = (size_t)p.W;
    // the rerun reads the next channel's incoming states while the current
    // one is filtered
    float in8n[AGG ? 1 : 8];
    auto load_in = [&](int n) {
        const float *cq = carry + ((size_t)(band * p.C + n) * 8) * cstride + col;
#pragma unroll
        for (int k = 0; k < 8; ++k) in8n[k] = cq[k * cstride];
    };
    if (!AGG && ce > cb) load_in(cb);
    for (int n = cb; n < ce; ++n) {
        const int deg = JOINT ? n >> 1 : n;
        const bool dat = JOINT && (n & 1);  // a joint data channel (uniform)
        float sv[STACKIN ? B + 3 : 1];
        if constexpr (STACKIN) {
            // rows a-1 .. a+B+1 of channel n of the source stack (clamped
            // loads, rows outside the image zeroed)
            const float *sn = src + (size_t)n * src_cstride + col;
#pragma unroll
            for (int i = 0; i < B + 3; ++i) {
                const int row = a - 1 + i;
                const int rc = row < 0 ? 0 : (row >= p.H ? p.H - 1 : row);
                sv[i] = sn[(size_t)rc * p.pitch];
            }
            if (a == 0) sv[0] = 0.f;
            if (a + B + 2 > p.H) {
#pragma unroll
                for (int i = 1; i < B + 3; ++i)
                    if (a - 1 + i >= p.H) sv[i] = 0.f;
            }
        } else {
            const float isq = (float)p.isq[deg];
            if (deg > 0 && !dat) {
#pragma unroll
                for (int i = 0; i < B + 3; ++i) u[i] *= xv[i] * isq;
            }
        }
        // channel value of sample i (undoing the range shift of BIG images;
        // times the data for a joint data channel)
        auto V = [&](int i) -> float {
            if constexpr (STACKIN) {
                return sv[i];
            } else {
                const float v = BIG ? ldexpf(u[i], -big_shift(xv[i])) : u[i];
                if constexpr (JOINT) return dat ? v * dv[i] : v;
                return v;
            }
        };
        float *cp = carry + ((size_t)(band * p.C + n) * 8) * cstride + col;
        // incoming states of both directions
        float in8[8];
        if constexpr (!AGG) {
#pragma unroll
            for (int k = 0; k < 8; ++k) in8[k] = in8n[k];
            if (n + 1 < ce) load_in(n + 1);
        }
        // causal: both sections advance together; the sum is staged in LDS
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    y1[s] = in8[2 * s];
                    y2[s] = in8[2 * s + 1];
                }
            }
            float xp = V(0);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const float vi = V(i + 1);
                float yv[2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.n0[s], vi, fmaf(c.n1[s], xp, -c.d2[s] * y2[s]));
                    yv[s] = fmaf(-c.d1[s], y1[s], b);
                    y2[s] = y1[s];
                    y1[s] = yv[s];
                }
                xp = vi;
                if (!AGG) sacc[i * 64 + lane] = yv[0] + yv[1];
            }
            if (AGG) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    cp[(2 * s) * cstride] = y1[s];
                    cp[(2 * s + 1) * cstride] = y2[s];
                }
            }
        }
        // anticausal: both sections advance together, and the finished
        // sample (causal + anticausal) is stored as soon as it is known
        {
            float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    z1[s] = in8[4 + 2 * s];
                    z2[s] = in8[5 + 2 * s];
                }
            }
            float xn1 = V(B + 1), xn2 = V(B + 2);
            float *sp = S + ((size_t)n * srows + a) * sp_pitch + col;
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                float zv[2];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.m1[s], xn1, fmaf(c.m2[s], xn2, -c.d2[s] * z2[s]));
                    zv[s] = fmaf(-c.d1[s], z1[s], b);
                    z2[s] = z1[s];
                    z1[s] = zv[s];
                }
                xn2 = xn1;
                xn1 = V(i + 1);
                if (!AGG) sp[(size_t)i * sp_pitch] = sacc[i * 64 + lane] + (zv[0] + zv[1]);
            }
            if (AGG) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    cp[(4 + 2 * s) * cstride] = z1[s];
                    cp[(5 + 2 * s) * cstride] = z2[s];
                }
            }
        }
    }
}

// Band end states as weighted sums ("moments").  The end states that vband
// <B, AGG> leaves for a band (causal y_{a+B-1}, y_{a+B-2} and anticausal z_a,
// z_{a+1} of both sections, from rest, with the true halo inputs) are linear
// in the band's B + 3 input samples (rows a-1 .. a+B+1):
//     e_k = sum_i w_k(i) u_n(x_i),   k = 0..7.
// The weights are the recursion's responses to unit inputs (agg_weight_task
// runs the same recursions on e_i; the table is made once per call on the
// host).  Per sample and channel this costs one multiply (the next power)
// and eight FMAs instead of both recursions.  The channels are taken
// unnormalised, p_n = exp(-x^2/2) x^n, and the end states are scaled by
// 1/sqrt(n!) at the store; the powers stay in the FP32 range up to degree 47
// (N <= 46), which the caller checks.

// One of the 4 (B + 3) responses (position i, section s, direction anti):
// the two end states that the recursion from rest leaves for a unit input at
// band position i (causal: rows a-1 (i = 0) .. a+B-1 (i = B); anticausal:
// rows a+1 (i = 2) .. a+B+1 (i = B+2)), into wts[i * 8 + ...].
__host__ __device__ inline void agg_weight_task(const IirCoef &c, int B, int task, float *wts) {
    const int i = task % (B + 3), s = (task / (B + 3)) & 1, anti = task / (2 * (B + 3));
    if (!anti) {
        float y1 = 0.f, y2 = 0.f, xp = i == 0 ? 1.f : 0.f;
        for (int j = 0; j < B; ++j) {
            const float v = (j + 1 == i) ? 1.f : 0.f;
            const float b = fmaf(c.n0[s], v, fmaf(c.n1[s], xp, -c.d2[s] * y2));
            const float y = fmaf(-c.d1[s], y1, b);
            y2 = y1;
            y1 = y;
            xp = v;
        }
        wts[i * 8 + 2 * s] = y1;
        wts[i * 8 + 2 * s + 1] = y2;
    } else {
        float z1 = 0.f, z2 = 0.f;
        float xn1 = (B + 1 == i) ? 1.f : 0.f, xn2 = (B + 2 == i) ? 1.f : 0.f;
        for (int j = B - 1; j >= 0; --j) {
            const float b = fmaf(c.m1[s], xn1, fmaf(c.m2[s], xn2, -c.d2[s] * z2));
            const float z = fmaf(-c.d1[s], z1, b);
            z2 = z1;
            z1 = z;
            xn2 = xn1;
            xn1 = (j + 1 == i) ? 1.f : 0.f;
        }
        wts[i * 8 + 4 + 2 * s] = z1;
        wts[i * 8 + 5 + 2 * s] = z2;
    }
}

// The whole table for bands of B <= kAggMaxB rows (pad row zeroed).
inline AggW make_agg_w(const IirCoef &c, int B) {
    AggW a;
    for (int k = 0; k < (kAggMaxB + 4) * 8; ++k) a.w[k] = 0.f;
    for (int task = 0; task < 4 * (B + 3); ++task) agg_weight_task(c, B, task, a.w);
    return a;
}

// Prologue of vagg_moments for the band's rows a-1 .. a+B+1 of one column
// group: the centred intensity x and exp(-x^2/2) (times the power-of-two
// shift of big_shift(x) when BIG) of rows r = g0, g0 + G, ... into pro
// (pro[r * 64 + lane] and pro[(B + 3 + r) * 64 + lane]), zeros for rows
// outside the image.  The G waves of a band each store their share.
template <int B, bool BIG>
__device__ __forceinline__ void vagg_prologue(const GPParams &p, const Stats &st, int col, int band, int g0, int G,
                                              float *pro) {
    const int lane = threadIdx.x & 63;
    const int a = band * B;
    const int colc = col < p.W ? col : p.W - 1;
    constexpr int NR = B + 3, CH = 6;
    for (int r0 = g0; r0 < NR; r0 += CH * G) {
        float f[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = r0 + k * G;
            const int row = a - 1 + (r < NR ? r : NR - 1);
            const int rc = row < 0 ? 0 : (row >= p.H ? p.H - 1 : row);
            f[k] = p.img[(size_t)rc * p.pitch + colc];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            const int r = r0 + k * G;
            if (r < NR) {
                const int row = a - 1 + r;
                const bool in = row >= 0 && row < p.H;
                const float x = in ? centred(f[k], st, p.inv_sigma_r) : 0.f;
                pro[r * 64 + lane] = x;
                pro[(NR + r) * 64 + lane] = in ? gauss_u0(x, BIG ? big_shift(x) : 0) : 0.f;
            }
        }
    }
}

// End states of one band of B rows in one column for the channels g, g + G,
// g + 2 G, ... < C (at most MAXG of them), by weighted sums, into carry (the
// layout of vband), from the band's prologue in pro (vagg_prologue).  The
// powers advance by x^G per channel.
// BIG: exp(-x^2/2) leaves the FP32 range (|x| > 12): it is carried with the
// per-sample power-of-two shift of vband, and every term is unscaled before
// it is accumulated (the channel values themselves are in range where they
// matter, as in the recursion).
template <int B, int MAXG, bool BIG>
__device__ __forceinline__ void vagg_moments(const GPParams &p, int col, int band, float *__restrict__ carry, int g,
                                             int G, const float *wts, const float *pro) {
    const int lane = threadIdx.x & 63;
    const int ng = (p.C - g + G - 1) / G;
    float acc[MAXG][8];
#pragma unroll
    for (int n = 0; n < MAXG; ++n)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[n][k] = 0.f;
    constexpr int NR = B + 3;
    // the next sample's prologue and weights are read one step ahead; past
    // the band's last sample these reads land in the weight table's pad row
    // (or, for a table in LDS, in the prologue after it) and in the next
    // prologue array or the LDS pad row, and are not used
    float xn = pro[lane], gn = pro[NR * 64 + lane];
    float4 w0n = *(const float4 *)wts, w1n = *(const float4 *)(wts + 4);
#pragma unroll 1
    for (int i = 0; i < NR; ++i) {
        const float x = xn, g0 = gn;
        const float4 w0 = w0n, w1 = w1n;
        const int in = i + 1;
        xn = pro[in * 64 + lane];
        gn = pro[(NR + in) * 64 + lane];
        w0n = *(const float4 *)(wts + in * 8);
        w1n = *(const float4 *)(wts + in * 8 + 4);
        const int sh = BIG ? big_shift(x) : 0;
        // exp(-x^2/2) x^g and the step x^G (g < G <= 4, uniform)
        float pw = g0, xg = x;
        for (int e = 0; e < g; ++e) pw *= x;
        for (int e = 1; e < G; ++e) xg *= x;
#pragma unroll
        for (int n = 0; n < MAXG; ++n) {
            if (n < ng) {
                const float v = BIG ? ldexpf(pw, -sh) : pw;
                acc[n][0] = fmaf(w0.x, v, acc[n][0]);
                acc[n][1] = fmaf(w0.y, v, acc[n][1]);
                acc[n][2] = fmaf(w0.z, v, acc[n][2]);
                acc[n][3] = fmaf(w0.w, v, acc[n][3]);
                acc[n][4] = fmaf(w1.x, v, acc[n][4]);
                acc[n][5] = fmaf(w1.y, v, acc[n][5]);
                acc[n][6] = fmaf(w1.z, v, acc[n][6]);
                acc[n][7] = fmaf(w1.w, v, acc[n][7]);
                pw *= xg;
            }
        }
    }
    if (col >= p.W) return;
    // 1/sqrt(n!) for n = g, then over G factors per channel
    double kap = 1.0;
    for (int j = 2; j <= g; ++j) kap *= p.isq[j];
    const size_t cstride = (size_t)p.W;
#pragma unroll
    for (int m = 0; m < MAXG; ++m) {
        if (m < ng) {
            const int n = g + m * G;
            const float kf = (float)kap;
            float *cp = carry + ((size_t)(band * p.C + n) * 8) * cstride + col;
#pragma unroll
            for (int k = 0; k < 8; ++k) cp[k * cstride] = acc[m][k] * kf;
            for (int j = 1; j <= G; ++j) kap *= p.isq[n + j];
        }
    }
}

// Channel groups of the weighted-sum end states for an image: 2 (the two
// waves of a band take the even and the odd channels) when the image gives
// at least kTargetAggWaves waves that way and C <= 2 kAggG, else 4.  Depends on
// the image size and channel count only, so that single and batched calls
// group alike (the grouping decides the rounding of the powers).
constexpr long kTargetAggWaves = 2048;
__host__ __device__ inline int agg_groups(int H, int W, int C) {
    const long bands = (long)((W + 63) / 64) * ((H + 31) / 32);
    return (2 * bands >= kTargetAggWaves && C <= 2 * kAggG) ? 2 : 4;
}

// LDS floats of one workgroup of the weighted-sum end states holding NBW
// bands: the weights (the batched kernel's copy), one prologue per band and a
// pad row.
__host__ __device__ constexpr int vagg_smem_floats(int B, int NBW) {
    return (B + 3) * 8 + NBW * 2 * (B + 3) * 64 + 64;  // + the pad row of the read-ahead
}

// Resolves, for one (column, channel) and one direction (dir 0 causal, top to
// bottom; dir 1 anticausal, bottom to top), the true incoming states of every
// band from the band end states, in place.  The end states are read 16 bands
// at a time so that the loads overlap.
__device__ __forceinline__ void vresolve(const GPParams &p, const IirCoef &c, int nb, int col, int n, int dir,
                                         float *__restrict__ carry) {
    constexpr int K = 16;
    const size_t cs = (size_t)p.W;
    float st4[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < nb; k0 += K) {
        float l[K][4];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int kk = k0 + q;
            const int k = dir == 0 ? kk : nb - 1 - kk;
            if (kk < nb) {
                const float *cp = carry + ((size_t)(k * p.C + n) * 8 + 4 * dir) * cs + col;
#pragma unroll
                for (int j = 0; j < 4; ++j) l[q][j] = cp[j * cs];
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int kk = k0 + q;
            if (kk >= nb) break;
            const int k = dir == 0 ? kk : nb - 1 - kk;
            float *cp = carry + ((size_t)(k * p.C + n) * 8 + 4 * dir) * cs + col;
#pragma unroll
            for (int j = 0; j < 4; ++j) cp[j * cs] = st4[j];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const float *P = c.phiB[s];
                const float a0 = st4[2 * s], a1 = st4[2 * s + 1];
                st4[2 * s] = fmaf(P[0], a0, fmaf(P[1], a1, l[q][2 * s]));
                st4[2 * s + 1] = fmaf(P[2], a0, fmaf(P[3], a1, l[q][2 * s + 1]));
            }
        }
    }
}

// 2x2 helpers (row-major)
// (explicit fmaf throughout the shared kernels: the result must not depend on
// how the compiler contracts multiply-adds in different calling kernels)
__device__ __forceinline__ void mat_mul(const float *A, const float *B, float *C) {
    const float c0 = fmaf(A[0], B[0], A[1] * B[2]), c1 = fmaf(A[0], B[1], A[1] * B[3]);
    const float c2 = fmaf(A[2], B[0], A[3] * B[2]), c3 = fmaf(A[2], B[1], A[3] * B[3]);
    C[0] = c0; C[1] = c1; C[2] = c2; C[3] = c3;
}
__device__ __forceinline__ void mat_pow_chunks(const IirCoef &c, int s, int m, float *G) {
    // G = Phi^(m L) for 1 <= m <= 64
    if (m >= 64) {
        for (int j = 0; j < 4; ++j) G[j] = c.phiW[s][j];
        return;
    }
    G[0] = 1.f; G[1] = 0.f; G[2] = 0.f; G[3] = 1.f;
    for (int j = 0; j < 6; ++j)
        if (m & (1 << j)) mat_mul(G, c.phiL[s][j], G);
}

// LDS bytes used by hrow for rows of T threads split into `groups` channel
// groups: the per-lane chunk-power tables, the wave totals of every group
// (double-buffered), and the FP64 partial sums that groups 1.. hand to group 0.
__host__ __device__ constexpr size_t hrow_smem_bytes(int T, int groups, int L) {
    return sizeof(float) * (size_t)(16 * 64 + groups * 16 * (T / 64)) +
           sizeof(double) * 2 * (size_t)(groups - 1) * (size_t)T * (size_t)L;
}

// Lane shifts through DPP (no LDS round trip).  Lanes whose source is outside
// the row (or wave) read 0.
constexpr int kDppRowShl = 0x100, kDppRowShr = 0x110, kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_f(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
// s[0..1] += P * (v0, v1), P 2x2 row-major
__device__ __forceinline__ void acc2(float *s, const float *P, float v0, float v1) {
    s[0] = fmaf(P[0], v0, fmaf(P[1], v1, s[0]));
    s[1] = fmaf(P[2], v0, fmaf(P[3], v1, s[1]));
}
// r = v + P * w (2-vectors)
__device__ __forceinline__ void affine2(float *r, const float *v, const float *P, const float *w) {
    const float a = w[0], b = w[1];
    r[0] = fmaf(P[0], a, fmaf(P[1], b, v[0]));
    r[1] = fmaf(P[2], a, fmaf(P[3], b, v[1]));
}

// One image row: row pass of eq. (8) on every channel of the column-filtered
// stack, fused with the recombination of eqs. (9)-(11).  The workgroup holds
// `groups` channel groups of T threads each (T a multiple of 64, T * L >= W);
// thread t of a group owns samples [t L, t L + L), and group g filters the
// channels [C g / groups, C (g + 1) / groups).  Threads past the last group
// only take part in the barriers.  Per channel:
//   1. each chunk runs causally and anticausally from rest (true halo inputs),
//      giving local outputs and its end states;
//   2. the chunk states are combined in order: a DPP scan inside each row of
//      16 lanes, the row totals across the wave by readlane, the wave totals
//      across the group through LDS;
//   3. each chunk adds the homogeneous response of its true incoming states.
// Channels are visited from the top of the group's range down, so that the
// recombination is a Horner evaluation in tau with two FP64 accumulators per
// pixel:
//   bD <- Ubar_n + bD tau / sqrt(n+1)  (n <= N),
//   bM <- Ubar_n + bM tau sqrt(n+1) / n  (n >= 1),
// which over all channels ends with bD = D exp(tau^2/2) and bM = M exp(tau^2/2)
// (the second is the Horner form of sum_k sqrt(k) p_{k-1} Ubar_k with sqrt(k)
// divided out).  A group that starts at channel cb > 0 holds the tail of both
// Horner sums; its share of the full sums is its value times
//   tau^cb / sqrt(cb!)                                  (bD),
//   prod_{j=1}^{cb-1} tau sqrt(j+1) / j = tau^(cb-1) sqrt(cb!) / (cb-1)!  (bM),
// and group 0 adds the shares of groups 1, 2, ... in that order.
// (The plain forward, its saved terms and the batches take the row pass of
// hrow.hpp; this one serves the joint filter.)
// sm: hrow_smem_bytes(T, groups, L) bytes.
// foff: element offset of the image and output rows (a volume's frame).
template <int L, bool JOINT = false>
__device__ __forceinline__ void hrow(const GPParams &p, const IirCoef &c, const Stats &st, int y,
                                     const float *__restrict__ S, int sp_rows, int sp_pitch, float *sm, int T,
                                     int groups, size_t foff = 0) {
    const int g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / T);  // whole waves share a group
    const int t = threadIdx.x - g * T;
    const int lane = threadIdx.x & 63, wave = t >> 6, nw = T >> 6;
    const int r16 = lane >> 4, j16 = lane & 15;
    const int x0 = t * L;
    const int xl = x0 < p.W ? x0 : ((p.W + 3) & ~3);  // chunks past the row end read the zero pad
    const bool member = g < groups;
    const int cb = member ? (p.C * g) / groups : p.C;
    const int ce = member ? (p.C * (g + 1)) / groups : p.C;
    const int steps = (p.C + groups - 1) / groups;  // largest group
    float *G64 = sm;                                // G64[k * 64 + lane], k = 0..15
    float *tot = sm + 16 * 64 + (member ? g : 0) * (16 * nw);  // wave totals, double-buffered
    double *comb = (double *)(sm + 16 * 64 + groups * 16 * nw);
    if (nw > 1) {
        if (threadIdx.x < 64) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                float gm[4];
                mat_pow_chunks(c, s, lane + 1, gm);
                for (int q = 0; q < 4; ++q) G64[(4 * s + q) * 64 + lane] = gm[q];
                mat_pow_chunks(c, s, 64 - lane, gm);
                for (int q = 0; q < 4; ++q) G64[(8 + 4 * s + q) * 64 + lane] = gm[q];
            }
        }
        __syncthreads();
    }
    // per-lane multipliers across a row of 16 chunks
    float G16c[2][4], G16a[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        mat_pow_chunks(c, s, j16 + 1, G16c[s]);
        mat_pow_chunks(c, s, 16 - j16, G16a[s]);
    }

    float tau[L];
    double bD[L], bM[L];
    {
        // unconditional loads from clamped columns, zeroed past the row end
        const float *irow = p.img + foff + (size_t)y * p.pitch;
#pragma unroll
        for (int i = 0; i < L; ++i) tau[i] = irow[x0 + i < p.W ? x0 + i : p.W - 1];
#pragma unroll
        for (int i = 0; i < L; ++i) {
            tau[i] = x0 + i < p.W ? centred(tau[i], st, p.inv_sigma_r) : 0.f;
            bD[i] = 0.0;
            bM[i] = 0.0;
        }
    }
    for (int it = 0; it < steps; ++it) {
        const int n = ce - 1 - it;
        const bool act = n >= cb;  // uniform over the group
        float o[L];
        float sc[4], sa[4];
        if (act) {
            // samples x0-1 .. x0+L+1 of the stack row: columns W .. pitch-1
            // are zero pad, so only the sample left of the row start needs a
            // mask (the pitch is a multiple of 4 and the rows 16-byte aligned)
            const float *row = S + ((size_t)n * sp_rows + y) * sp_pitch;
            float z[L + 3];
            z[0] = row[xl > 0 ? xl - 1 : 0];
#pragma unroll
            for (int i = 0; i < L; i += 4) {
                const float4 q = *(const float4 *)(row + xl + i);
                z[1 + i] = q.x; z[2 + i] = q.y; z[3 + i] = q.z; z[4 + i] = q.w;
            }
            z[L + 1] = row[xl + L];
            z[L + 2] = row[xl + L + 1];
            z[0] = x0 > 0 ? z[0] : 0.f;

            // 1. chunk from rest
            {
                float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    float v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float b = fmaf(c.n0[s], z[i + 1], fmaf(c.n1[s], z[i], -c.d2[s] * y2[s]));
                        v[s] = fmaf(-c.d1[s], y1[s], b);
                        y2[s] = y1[s];
                        y1[s] = v[s];
                    }
                    o[i] = v[0] + v[1];
                }
                sc[0] = y1[0]; sc[1] = y2[0]; sc[2] = y1[1]; sc[3] = y2[1];
            }
            {
                float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f};
#pragma unroll
                for (int i = L - 1; i >= 0; --i) {
                    float v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float b = fmaf(c.m1[s], z[i + 2], fmaf(c.m2[s], z[i + 3], -c.d2[s] * z2[s]));
                        v[s] = fmaf(-c.d1[s], z1[s], b);
                        z2[s] = z1[s];
                        z1[s] = v[s];
                    }
                    o[i] += v[0] + v[1];
                }
                sa[0] = z1[0]; sa[1] = z2[0]; sa[2] = z1[1]; sa[3] = z2[1];
            }
            // 2a. scans inside each row of 16 lanes (distances 1, 2, 4, 8 chunks)
#define BF_ROWSTEP(J, D)                                                                   \
            {                                                                              \
                float pc[4], pa[4];                                                        \
                _Pragma("unroll") for (int q = 0; q < 4; ++q) {                            \
                    pc[q] = dpp_f<kDppRowShr + D>(sc[q]);                                  \
                    pa[q] = dpp_f<kDppRowShl + D>(sa[q]);                                  \
                }                                                                          \
                _Pragma("unroll") for (int s = 0; s < 2; ++s) {                            \
                    acc2(&sc[2 * s], c.phiL[s][J], pc[2 * s], pc[2 * s + 1]);              \
                    acc2(&sa[2 * s], c.phiL[s][J], pa[2 * s], pa[2 * s + 1]);              \
                }                                                                          \
            }
            BF_ROWSTEP(0, 1)
            BF_ROWSTEP(1, 2)
            BF_ROWSTEP(2, 4)
            BF_ROWSTEP(3, 8)
#undef BF_ROWSTEP
            // 2b. across the four rows of the wave
            {
                float C1[4], C2[4], C3[4], A0[4], A1[4], A2[4];
                float t0[4], t1[4], t2[4], h1[4], h2[4], h3[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    t0[q] = lane_f(sc[q], 15);
                    t1[q] = lane_f(sc[q], 31);
                    t2[q] = lane_f(sc[q], 47);
                    h1[q] = lane_f(sa[q], 16);
                    h2[q] = lane_f(sa[q], 32);
                    h3[q] = lane_f(sa[q], 48);
                }
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float *P16 = c.phiL[s][4];
                    C1[2 * s] = t0[2 * s];
                    C1[2 * s + 1] = t0[2 * s + 1];
                    affine2(&C2[2 * s], &t1[2 * s], P16, &C1[2 * s]);
                    affine2(&C3[2 * s], &t2[2 * s], P16, &C2[2 * s]);
                    A2[2 * s] = h3[2 * s];
                    A2[2 * s + 1] = h3[2 * s + 1];
                    affine2(&A1[2 * s], &h2[2 * s], P16, &A2[2 * s]);
                    affine2(&A0[2 * s], &h1[2 * s], P16, &A1[2 * s]);
                }
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    float cr0 = 0.f, cr1 = 0.f, ar0 = 0.f, ar1 = 0.f;
                    if (r16 == 1) { cr0 = C1[2 * s]; cr1 = C1[2 * s + 1]; }
                    if (r16 == 2) { cr0 = C2[2 * s]; cr1 = C2[2 * s + 1]; }
                    if (r16 == 3) { cr0 = C3[2 * s]; cr1 = C3[2 * s + 1]; }
                    if (r16 == 0) { ar0 = A0[2 * s]; ar1 = A0[2 * s + 1]; }
                    if (r16 == 1) { ar0 = A1[2 * s]; ar1 = A1[2 * s + 1]; }
                    if (r16 == 2) { ar0 = A2[2 * s]; ar1 = A2[2 * s + 1]; }
                    acc2(&sc[2 * s], G16c[s], cr0, cr1);
                    acc2(&sa[2 * s], G16a[s], ar0, ar1);
                }
            }
        }
        // 2c. across the waves of the group (every wave of the workgroup meets
        // the barrier, active or not)
        float cc[4] = {0.f, 0.f, 0.f, 0.f}, ca[4] = {0.f, 0.f, 0.f, 0.f};
        if (nw > 1) {
            float *buf = tot + (it & 1) * (2 * nw * 4);
            if (act) {
                float wc[4], wa[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    wc[q] = lane_f(sc[q], 63);
                    wa[q] = lane_f(sa[q], 0);
                }
                if (lane == 0) {
                    for (int q = 0; q < 4; ++q) {
                        buf[wave * 4 + q] = wc[q];
                        buf[(nw + wave) * 4 + q] = wa[q];
                    }
                }
            }
            __syncthreads();
            if (act) {
                for (int w2 = 0; w2 < wave; ++w2) {
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        float r[2];
                        affine2(r, &buf[w2 * 4 + 2 * s], c.phiW[s], &cc[2 * s]);
                        cc[2 * s] = r[0];
                        cc[2 * s + 1] = r[1];
                    }
                }
                for (int w2 = nw - 1; w2 > wave; --w2) {
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        float r[2];
                        affine2(r, &buf[(nw + w2) * 4 + 2 * s], c.phiW[s], &ca[2 * s]);
                        ca[2 * s] = r[0];
                        ca[2 * s + 1] = r[1];
                    }
                }
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    float gm[4], hm[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        gm[q] = G64[(4 * s + q) * 64 + lane];
                        hm[q] = G64[(8 + 4 * s + q) * 64 + lane];
                    }
                    acc2(&sc[2 * s], gm, cc[2 * s], cc[2 * s + 1]);
                    acc2(&sa[2 * s], hm, ca[2 * s], ca[2 * s + 1]);
                }
            }
        }
        if (!act) continue;
        // exclusive states: incoming causal from the previous chunk, incoming
        // anticausal from the next chunk
        float ic[4], ia[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float up = dpp_f<kDppWaveShr1>(sc[q]);
            const float dn = dpp_f<kDppWaveShl1>(sa[q]);
            ic[q] = lane == 0 ? cc[q] : up;
            ia[q] = lane == 63 ? ca[q] : dn;
        }
        // 3. homogeneous responses of the incoming states (by recursion)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float d1 = c.d1[s], d2 = c.d2[s];
            float a1 = ic[2 * s], a2 = ic[2 * s + 1];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const float h = fmaf(-d1, a1, -d2 * a2);
                o[i] += h;
                a2 = a1;
                a1 = h;
            }
            float b1 = ia[2 * s], b2 = ia[2 * s + 1];
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                const float h = fmaf(-d1, b1, -d2 * b2);
                o[i] += h;
                b2 = b1;
                b1 = h;
            }
        }
        // recombination: Horner in tau, double precision.  With
        // m_k = bM_k / sqrt(k): m_k = Ubar_k + m_{k+1} tau sqrt(k+1) / k.
        // (channel N+1 enters only bM, channel 0 only bD: uniform branches,
        // so that the common case carries no per-sample selects)
        if constexpr (JOINT) {
            // joint stack: channel 2k + 1 (data) into bM, channel 2k (guide)
            // into bD, both with the Horner factor tau / sqrt(k + 1): bD ends
            // as sum_k p_k(tau) Ubar_2k, bM as sum_k p_k(tau) Ubar_2k+1
            const double r = p.isq[(n >> 1) + 1];
            if (n & 1) {
#pragma unroll
                for (int i = 0; i < L; ++i) bM[i] = fma(bM[i], (double)tau[i] * r, (double)o[i]);
            } else {
#pragma unroll
                for (int i = 0; i < L; ++i) bD[i] = fma(bD[i], (double)tau[i] * r, (double)o[i]);
            }
            continue;
        }
        const double rD = p.isq[n + 1];
        const double rM = p.rm[n];
        if (n <= p.N && n >= 1) {
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const double ub = (double)o[i];
                const double tv = (double)tau[i];
                bD[i] = fma(bD[i], tv * rD, ub);
                bM[i] = fma(bM[i], tv * rM, ub);
            }
        } else if (n >= 1) {
#pragma unroll
            for (int i = 0; i < L; ++i) {
                bM[i] = fma(bM[i], (double)tau[i] * rM, (double)o[i]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < L; ++i) {
                bD[i] = fma(bD[i], (double)tau[i] * rD, (double)o[i]);
            }
        }
    }
    if (!JOINT && groups > 1) {
        // shares of groups 1.. in the full Horner sums, through LDS
        if (member && g > 0) {
            double kD = 1.0, kM = 1.0;
            for (int j = 0; j < cb; ++j) kD *= p.isq[j + 1];
            for (int j = 1; j < cb; ++j) kM *= p.rm[j];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const double tv = (double)tau[i];
                const double tp = ipow(tv, cb - 1);
                comb[((size_t)(g - 1) * 2 * L + 2 * i) * T + t] = bD[i] * (tp * tv * kD);
                comb[((size_t)(g - 1) * 2 * L + 2 * i + 1) * T + t] = bM[i] * (tp * kM);
            }
        }
        __syncthreads();
        if (g == 0) {
            for (int gg = 1; gg < groups; ++gg) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    bD[i] += comb[((size_t)(gg - 1) * 2 * L + 2 * i) * T + t];
                    bM[i] += comb[((size_t)(gg - 1) * 2 * L + 2 * i + 1) * T + t];
                }
            }
        }
    }
    if (g == 0 && y < p.H) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int x = x0 + i;
            if (x < p.W) {
                const double rho = bM[i] / bD[i];
                if constexpr (JOINT) {
                    p.out[foff + (size_t)y * p.pitch + x] = st.ok ? (float)rho : __builtin_nanf("");
                    continue;
                }
                p.out[foff + (size_t)y * p.pitch + x] = st.ok ? (float)fma(p.sigma_r, rho, st.tc) : __builtin_nanf("");
            }
        }
    }
}

}  // namespace bfgp
