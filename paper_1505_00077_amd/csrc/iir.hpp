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

struct IirCoef {
    float n0[2], n1[2], m1[2], m2[2], d1[2], d2[2];
    float phiB[2][4];     // Phi^B, Phi = [[-d1, -d2], [1, 0]], row-major
    float phiL[2][6][4];  // Phi^(L 2^j), j = 0..5
    float phiW[2][4];     // Phi^(64 L)
};

// Centred intensity of column `col`, row `row`, or 0 outside the image.
__device__ __forceinline__ float xval(const GPParams &p, const Stats &st, int row, int col) {
    if (row < 0 || row >= p.H || col >= p.W) return 0.f;
    return centred(p.img[(size_t)row * p.pitch + col], st, p.inv_sigma_r);
}
__device__ __forceinline__ bool inimg(const GPParams &p, int row, int col) {
    return row >= 0 && row < p.H && col < p.W;
}

// Scale exponent used when exp(-x^2/2) would leave the FP32 range: the channel
// is carried as uh = u * 2^s and stored as u = uh * 2^-s.
__device__ __forceinline__ int big_shift(float x) {
    const float t = x * x;
    return t > 144.f ? (int)(t * 0.72134752f) - 60 : 0;
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
template <int B, bool AGG, bool BIG>
__device__ __forceinline__ void vband(const GPParams &p, const IirCoef &c, const Stats &st, int col, int band,
                                      float *__restrict__ carry, float *__restrict__ S, float *sacc, int cb,
                                      int ce) {
    const int lane = threadIdx.x & 63;
    const int a = band * B;
    float xv[B + 3], u[B + 3];
#pragma unroll
    for (int i = 0; i < B + 3; ++i) {
        const int row = a - 1 + i;
        const float x = xval(p, st, row, col);
        xv[i] = x;
        u[i] = inimg(p, row, col) ? gauss_u0(x, BIG ? big_shift(x) : 0) : 0.f;
    }
    const size_t cstride = (size_t)p.W;
    for (int n = 1; n < cb; ++n) {
        const float isq = (float)p.isq[n];
#pragma unroll
        for (int i = 0; i < B + 3; ++i) u[i] *= xv[i] * isq;
    }
    for (int n = cb; n < ce; ++n) {
        const float isq = (float)p.isq[n];
        if (n > 0) {
#pragma unroll
            for (int i = 0; i < B + 3; ++i) u[i] *= xv[i] * isq;
        }
        // channel value of sample i (undoing the range shift of BIG images)
        auto V = [&](int i) -> float { return BIG ? ldexpf(u[i], -big_shift(xv[i])) : u[i]; };
        float *cp = carry + ((size_t)(band * p.C + n) * 8) * cstride + col;
        // causal: both sections advance together; the sum is staged in LDS
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
            if (!AGG && col < p.W) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    y1[s] = cp[(2 * s) * cstride];
                    y2[s] = cp[(2 * s + 1) * cstride];
                }
            }
            float xp = V(0);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const float vi = V(i + 1);
                float tot = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.n0[s], vi, fmaf(c.n1[s], xp, -c.d2[s] * y2[s]));
                    const float y = fmaf(-c.d1[s], y1[s], b);
                    y2[s] = y1[s];
                    y1[s] = y;
                    tot += y;
                }
                xp = vi;
                if (!AGG) sacc[i * 64 + lane] = tot;
            }
            if (AGG && col < p.W) {
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
            if (!AGG && col < p.W) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    z1[s] = cp[(4 + 2 * s) * cstride];
                    z2[s] = cp[(5 + 2 * s) * cstride];
                }
            }
            float xn1 = V(B + 1), xn2 = V(B + 2);
            float *sp = S + ((size_t)n * p.H + a) * p.W + col;
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                float tot = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.m1[s], xn1, fmaf(c.m2[s], xn2, -c.d2[s] * z2[s]));
                    const float z = fmaf(-c.d1[s], z1[s], b);
                    z2[s] = z1[s];
                    z1[s] = z;
                    tot += z;
                }
                xn2 = xn1;
                xn1 = V(i + 1);
                if (!AGG && col < p.W && a + i < p.H) sp[(size_t)i * p.W] = sacc[i * 64 + lane] + tot;
            }
            if (AGG && col < p.W) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    cp[(4 + 2 * s) * cstride] = z1[s];
                    cp[(5 + 2 * s) * cstride] = z2[s];
                }
            }
        }
    }
}

// Resolves, for one (column, channel) and one direction (dir 0 causal, top to
// bottom; dir 1 anticausal, bottom to top), the true incoming states of every
// band from the band end states, in place.
__device__ __forceinline__ void vresolve(const GPParams &p, const IirCoef &c, int nb, int col, int n, int dir,
                                         float *__restrict__ carry) {
    const size_t cs = (size_t)p.W;
    float st4[4] = {0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < nb; ++kk) {
        const int k = dir == 0 ? kk : nb - 1 - kk;
        float *cp = carry + ((size_t)(k * p.C + n) * 8 + 4 * dir) * cs + col;
        float l[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) l[j] = cp[j * cs];
#pragma unroll
        for (int j = 0; j < 4; ++j) cp[j * cs] = st4[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float *P = c.phiB[s];
            const float a0 = st4[2 * s], a1 = st4[2 * s + 1];
            st4[2 * s] = fmaf(P[0], a0, fmaf(P[1], a1, l[2 * s]));
            st4[2 * s + 1] = fmaf(P[2], a0, fmaf(P[3], a1, l[2 * s + 1]));
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

// LDS floats used by hrow for a workgroup of nw waves.
__host__ __device__ constexpr int hrow_smem_floats(int nw) {
    return 2 * 2 * nw * 4 + 16 * 64;
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
// stack, fused with the recombination of eqs. (9)-(11).  Workgroup of T
// threads (T a multiple of 64, T * L >= W); thread t owns samples
// [t L, t L + L).  Per channel:
//   1. each chunk runs causally and anticausally from rest (true halo inputs),
//      giving local outputs and its end states;
//   2. the chunk states are combined in order: a DPP scan inside each row of
//      16 lanes, the row totals across the wave by readlane, the wave totals
//      across the workgroup through LDS;
//   3. each chunk adds the homogeneous response of its true incoming states.
// Channels are visited from N+1 down to 0 so that the recombination is a
// Horner evaluation in tau with two FP64 accumulators per pixel:
//   bD <- Ubar_n + bD tau / sqrt(n+1)  (n <= N),
//   bM <- Ubar_n + bM tau sqrt(n+1) / n  (n >= 1),
// ending with bD = D exp(tau^2/2) and bM = M exp(tau^2/2) (the second is the
// Horner form of sum_k sqrt(k) p_{k-1} Ubar_k with sqrt(k) divided out).
// sm: hrow_smem_floats(T / 64) floats.
template <int L>
__device__ __forceinline__ void hrow(const GPParams &p, const IirCoef &c, const Stats &st, int y,
                                     const float *__restrict__ S, float *sm) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
    const int r16 = lane >> 4, j16 = lane & 15;
    const int x0 = t * L;
    float *tot = sm;                 // wave totals, double-buffered
    float *G64 = sm + 2 * 2 * nw * 4;  // G64[k * 64 + lane], k = 0..15
    if (nw > 1) {
        if (wave == 0) {
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                float g[4];
                mat_pow_chunks(c, s, lane + 1, g);
                for (int q = 0; q < 4; ++q) G64[(4 * s + q) * 64 + lane] = g[q];
                mat_pow_chunks(c, s, 64 - lane, g);
                for (int q = 0; q < 4; ++q) G64[(8 + 4 * s + q) * 64 + lane] = g[q];
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
#pragma unroll
    for (int i = 0; i < L; ++i) {
        tau[i] = xval(p, st, y, x0 + i);
        bD[i] = 0.0;
        bM[i] = 0.0;
    }
    for (int n = p.C - 1; n >= 0; --n) {
        const float *row = S + ((size_t)n * p.H + y) * p.W;
        float z[L + 3];
        z[0] = (x0 - 1 >= 0 && x0 - 1 < p.W) ? row[x0 - 1] : 0.f;
        if (x0 + L <= p.W && ((((size_t)(row + x0)) & 15) == 0) && (L % 4) == 0) {
#pragma unroll
            for (int i = 0; i < L; i += 4) {
                const float4 q = *(const float4 *)(row + x0 + i);
                z[1 + i] = q.x; z[2 + i] = q.y; z[3 + i] = q.z; z[4 + i] = q.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < L; ++i) z[1 + i] = (x0 + i < p.W) ? row[x0 + i] : 0.f;
        }
        z[L + 1] = (x0 + L < p.W) ? row[x0 + L] : 0.f;
        z[L + 2] = (x0 + L + 1 < p.W) ? row[x0 + L + 1] : 0.f;

        // 1. chunk from rest
        float o[L];
        float sc[4], sa[4];
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
#pragma unroll
            for (int i = 0; i < L; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.n0[s], z[i + 1], fmaf(c.n1[s], z[i], -c.d2[s] * y2[s]));
                    const float v = fmaf(-c.d1[s], y1[s], b);
                    y2[s] = y1[s];
                    y1[s] = v;
                    acc += v;
                }
                o[i] = acc;
            }
            sc[0] = y1[0]; sc[1] = y2[0]; sc[2] = y1[1]; sc[3] = y2[1];
        }
        {
            float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f};
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float b = fmaf(c.m1[s], z[i + 2], fmaf(c.m2[s], z[i + 3], -c.d2[s] * z2[s]));
                    const float v = fmaf(-c.d1[s], z1[s], b);
                    z2[s] = z1[s];
                    z1[s] = v;
                    acc += v;
                }
                o[i] += acc;
            }
            sa[0] = z1[0]; sa[1] = z2[0]; sa[2] = z1[1]; sa[3] = z2[1];
        }
        // 2a. scans inside each row of 16 lanes (distances 1, 2, 4, 8 chunks)
#define BF_ROWSTEP(J, D)                                                                   \
        {                                                                                  \
            float pc[4], pa[4];                                                            \
            _Pragma("unroll") for (int q = 0; q < 4; ++q) {                                \
                pc[q] = dpp_f<kDppRowShr + D>(sc[q]);                                      \
                pa[q] = dpp_f<kDppRowShl + D>(sa[q]);                                      \
            }                                                                              \
            _Pragma("unroll") for (int s = 0; s < 2; ++s) {                                \
                acc2(&sc[2 * s], c.phiL[s][J], pc[2 * s], pc[2 * s + 1]);                  \
                acc2(&sa[2 * s], c.phiL[s][J], pa[2 * s], pa[2 * s + 1]);                  \
            }                                                                              \
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
        // 2c. across the waves of the workgroup
        float cc[4] = {0.f, 0.f, 0.f, 0.f}, ca[4] = {0.f, 0.f, 0.f, 0.f};
        if (nw > 1) {
            float *buf = tot + (n & 1) * (2 * nw * 4);
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
            __syncthreads();
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
                float g[4], h[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    g[q] = G64[(4 * s + q) * 64 + lane];
                    h[q] = G64[(8 + 4 * s + q) * 64 + lane];
                }
                acc2(&sc[2 * s], g, cc[2 * s], cc[2 * s + 1]);
                acc2(&sa[2 * s], h, ca[2 * s], ca[2 * s + 1]);
            }
        }
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
        const bool inD = n <= p.N;
        const double rD = p.isq[n + 1];
        const double rM = n >= 1 ? p.sq[n + 1] / (double)n : 0.0;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const double ub = (double)o[i];
            const double tv = (double)tau[i];
            if (inD) bD[i] = fma(bD[i], tv * rD, ub);
            if (n >= 1) bM[i] = fma(bM[i], tv * rM, ub);
        }
    }
    if (y < p.H) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int x = x0 + i;
            if (x < p.W) {
                const double rho = bM[i] / bD[i];
                p.out[(size_t)y * p.pitch + x] = st.ok ? (float)fma(p.sigma_r, rho, st.tc) : __builtin_nanf("");
            }
        }
    }
}

}  // namespace bfgp
