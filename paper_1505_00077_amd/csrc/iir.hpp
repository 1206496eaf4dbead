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
    float fix1[2][kIirMaxL], fix2[2][kIirMaxL];  // (Phi^(i+1))[0][0], [0][1]
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
template <int B, bool AGG, bool BIG>
__device__ __forceinline__ void vband(const GPParams &p, const IirCoef &c, const Stats &st, int col, int band,
                                      float *__restrict__ carry, float *__restrict__ S, float *sacc) {
    const int lane = threadIdx.x & 63;
    const int a = band * B;
    float xv[B + 3], u[B + 3];
#pragma unroll
    for (int i = 0; i < B + 3; ++i) {
        const int row = a - 1 + i;
        const float x = xval(p, st, row, col);
        xv[i] = x;
        double lu = -0.5 * (double)x * (double)x;
        if (BIG) lu += (double)big_shift(x) * 0.69314718055994531;
        u[i] = inimg(p, row, col) ? (float)exp(lu) : 0.f;
    }
    const size_t cstride = (size_t)p.W;
    for (int n = 0; n < p.C; ++n) {
        const float isq = (float)p.isq[n];
        if (n > 0) {
#pragma unroll
            for (int i = 0; i < B + 3; ++i) u[i] *= xv[i] * isq;
        }
        // channel value of sample i (undoing the range shift of BIG images)
        auto V = [&](int i) -> float { return BIG ? ldexpf(u[i], -big_shift(xv[i])) : u[i]; };
        float *cp = carry + ((size_t)(band * p.C + n) * 8) * cstride + col;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float n0 = c.n0[s], n1 = c.n1[s], d1 = c.d1[s], d2 = c.d2[s];
            float y1 = 0.f, y2 = 0.f;
            if (!AGG && col < p.W) {
                y1 = cp[(2 * s) * cstride];
                y2 = cp[(2 * s + 1) * cstride];
            }
            float xp = V(0);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const float vi = V(i + 1);
                const float y = fmaf(n0, vi, fmaf(n1, xp, fmaf(-d1, y1, -d2 * y2)));
                y2 = y1;
                y1 = y;
                xp = vi;
                if (!AGG) sacc[i * 64 + lane] = (s == 0) ? y : sacc[i * 64 + lane] + y;
            }
            if (AGG && col < p.W) {
                cp[(2 * s) * cstride] = y1;
                cp[(2 * s + 1) * cstride] = y2;
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
                    const float z = fmaf(c.m1[s], xn1, fmaf(c.m2[s], xn2, fmaf(-c.d1[s], z1[s], -c.d2[s] * z2[s])));
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

// Resolves, for one (column, channel), the true incoming states of every band
// from the band end states, in place.
__device__ __forceinline__ void vresolve(const GPParams &p, const IirCoef &c, int nb, int col, int n,
                                         float *__restrict__ carry) {
    const size_t cs = (size_t)p.W;
    float sc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < nb; ++k) {
        float *cp = carry + ((size_t)(k * p.C + n) * 8) * cs + col;
        float l[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) l[j] = cp[j * cs];
#pragma unroll
        for (int j = 0; j < 4; ++j) cp[j * cs] = sc[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float *P = c.phiB[s];
            const float a0 = sc[2 * s], a1 = sc[2 * s + 1];
            sc[2 * s] = l[2 * s] + P[0] * a0 + P[1] * a1;
            sc[2 * s + 1] = l[2 * s + 1] + P[2] * a0 + P[3] * a1;
        }
    }
    float sa[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = nb - 1; k >= 0; --k) {
        float *cp = carry + ((size_t)(k * p.C + n) * 8 + 4) * cs + col;
        float l[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) l[j] = cp[j * cs];
#pragma unroll
        for (int j = 0; j < 4; ++j) cp[j * cs] = sa[j];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const float *P = c.phiB[s];
            const float a0 = sa[2 * s], a1 = sa[2 * s + 1];
            sa[2 * s] = l[2 * s] + P[0] * a0 + P[1] * a1;
            sa[2 * s + 1] = l[2 * s + 1] + P[2] * a0 + P[3] * a1;
        }
    }
}

// 2x2 helpers (row-major)
__device__ __forceinline__ void mat_mul(const float *A, const float *B, float *C) {
    const float c0 = A[0] * B[0] + A[1] * B[2], c1 = A[0] * B[1] + A[1] * B[3];
    const float c2 = A[2] * B[0] + A[3] * B[2], c3 = A[2] * B[1] + A[3] * B[3];
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
    return 2 * 2 * nw * 4 + 4 * kIirMaxL + 16 * 64;
}

// One image row: row pass of eq. (8) on every channel of the column-filtered
// stack, fused with the recombination of eqs. (9)-(11).  Workgroup of T
// threads (T a multiple of 64, T * L >= W); thread t owns samples
// [t L, t L + L).  sm: hrow_smem_floats(T / 64) floats.
template <int L>
__device__ __forceinline__ void hrow(const GPParams &p, const IirCoef &c, const Stats &st, int y,
                                     const float *__restrict__ S, float *sm) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
    const int x0 = t * L;
    float *tot = sm;                          // wave totals, double-buffered
    float *fix = sm + 2 * 2 * nw * 4;         // fix[(2 s + k) * L + i]
    float *G = fix + 4 * kIirMaxL;            // G[k * 64 + lane], k = 0..15
    for (int i = t; i < 4 * L; i += blockDim.x) {
        const int s = i / (2 * L), k = (i / L) & 1, j = i % L;
        fix[i] = k == 0 ? c.fix1[s][j] : c.fix2[s][j];
    }
    if (wave == 0) {
        // carry-in multipliers Phi^((lane+1) L) (causal) and Phi^((64-lane) L)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float g[4];
            mat_pow_chunks(c, s, lane + 1, g);
            for (int q = 0; q < 4; ++q) G[(4 * s + q) * 64 + lane] = g[q];
            mat_pow_chunks(c, s, 64 - lane, g);
            for (int q = 0; q < 4; ++q) G[(8 + 4 * s + q) * 64 + lane] = g[q];
        }
    }
    __syncthreads();

    float tau[L];
    double D[L], M[L], P[L];
#pragma unroll
    for (int i = 0; i < L; ++i) {
        tau[i] = xval(p, st, y, x0 + i);
        D[i] = 0.0;
        M[i] = 0.0;
        P[i] = 0.0;
    }
    for (int n = 0; n < p.C; ++n) {
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

        // chunk from rest: causal and anticausal, both sections together
        float o[L];
        float sc[4], sa[4];
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
            float xp = z[0];
#pragma unroll
            for (int i = 0; i < L; ++i) {
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float v = fmaf(c.n0[s], z[i + 1], fmaf(c.n1[s], xp, fmaf(-c.d1[s], y1[s], -c.d2[s] * y2[s])));
                    y2[s] = y1[s];
                    y1[s] = v;
                    acc += v;
                }
                xp = z[i + 1];
                o[i] = acc;
            }
            sc[0] = y1[0]; sc[1] = y2[0]; sc[2] = y1[1]; sc[3] = y2[1];
        }
        {
            float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f};
            float xn1 = z[L + 1], xn2 = z[L + 2];
#pragma unroll
            for (int i = L - 1; i >= 0; --i) {
                float acc = 0.f;
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float v = fmaf(c.m1[s], xn1, fmaf(c.m2[s], xn2, fmaf(-c.d1[s], z1[s], -c.d2[s] * z2[s])));
                    z2[s] = z1[s];
                    z1[s] = v;
                    acc += v;
                }
                xn2 = xn1;
                xn1 = z[i + 1];
                o[i] += acc;
            }
            sa[0] = z1[0]; sa[1] = z2[0]; sa[2] = z1[1]; sa[3] = z2[1];
        }
        // wave-level scans: causal prefix, anticausal suffix
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const int d = 1 << j;
            float pc[4], pa[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                pc[q] = __shfl_up(sc[q], d, 64);
                pa[q] = __shfl_down(sa[q], d, 64);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const float *Pm = c.phiL[s][j];
                if (lane >= d) {
                    sc[2 * s] += Pm[0] * pc[2 * s] + Pm[1] * pc[2 * s + 1];
                    sc[2 * s + 1] += Pm[2] * pc[2 * s] + Pm[3] * pc[2 * s + 1];
                }
                if (lane + d < 64) {
                    sa[2 * s] += Pm[0] * pa[2 * s] + Pm[1] * pa[2 * s + 1];
                    sa[2 * s + 1] += Pm[2] * pa[2 * s] + Pm[3] * pa[2 * s + 1];
                }
            }
        }
        // cross-wave carries
        float cc[4] = {0.f, 0.f, 0.f, 0.f}, ca[4] = {0.f, 0.f, 0.f, 0.f};
        if (nw > 1) {
            float *buf = tot + (n & 1) * (2 * nw * 4);
            if (lane == 63)
                for (int q = 0; q < 4; ++q) buf[wave * 4 + q] = sc[q];
            if (lane == 0)
                for (int q = 0; q < 4; ++q) buf[(nw + wave) * 4 + q] = sa[q];
            __syncthreads();
            for (int w2 = 0; w2 < wave; ++w2) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float *Pm = c.phiW[s];
                    const float a0 = cc[2 * s], a1 = cc[2 * s + 1];
                    cc[2 * s] = buf[w2 * 4 + 2 * s] + Pm[0] * a0 + Pm[1] * a1;
                    cc[2 * s + 1] = buf[w2 * 4 + 2 * s + 1] + Pm[2] * a0 + Pm[3] * a1;
                }
            }
            for (int w2 = nw - 1; w2 > wave; --w2) {
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const float *Pm = c.phiW[s];
                    const float a0 = ca[2 * s], a1 = ca[2 * s + 1];
                    ca[2 * s] = buf[(nw + w2) * 4 + 2 * s] + Pm[0] * a0 + Pm[1] * a1;
                    ca[2 * s + 1] = buf[(nw + w2) * 4 + 2 * s + 1] + Pm[2] * a0 + Pm[3] * a1;
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const float g0 = G[(4 * s + 0) * 64 + lane], g1 = G[(4 * s + 1) * 64 + lane];
                const float g2 = G[(4 * s + 2) * 64 + lane], g3 = G[(4 * s + 3) * 64 + lane];
                const float a0 = cc[2 * s], a1 = cc[2 * s + 1];
                sc[2 * s] += g0 * a0 + g1 * a1;
                sc[2 * s + 1] += g2 * a0 + g3 * a1;
                const float h0 = G[(8 + 4 * s + 0) * 64 + lane], h1 = G[(8 + 4 * s + 1) * 64 + lane];
                const float h2 = G[(8 + 4 * s + 2) * 64 + lane], h3 = G[(8 + 4 * s + 3) * 64 + lane];
                const float b0 = ca[2 * s], b1 = ca[2 * s + 1];
                sa[2 * s] += h0 * b0 + h1 * b1;
                sa[2 * s + 1] += h2 * b0 + h3 * b1;
            }
        }
        // exclusive states: incoming causal from the previous chunk, incoming
        // anticausal from the next chunk
        float ic[4], ia[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float up = __shfl_up(sc[q], 1, 64);
            const float dn = __shfl_down(sa[q], 1, 64);
            ic[q] = lane == 0 ? cc[q] : up;
            ia[q] = lane == 63 ? ca[q] : dn;
        }
        // homogeneous responses of the incoming states, then the recombination
        // in double precision
        const double sqn = p.sq[n], isqn = p.isq[n];
        const bool inD = n <= p.N;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            float v = o[i];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                v = fmaf(fix[(2 * s) * L + i], ic[2 * s], v);
                v = fmaf(fix[(2 * s + 1) * L + i], ic[2 * s + 1], v);
                v = fmaf(fix[(2 * s) * L + (L - 1 - i)], ia[2 * s], v);
                v = fmaf(fix[(2 * s + 1) * L + (L - 1 - i)], ia[2 * s + 1], v);
            }
            const double ub = (double)v;
            if (n >= 1) M[i] = fma(P[i] * sqn, ub, M[i]);
            if (inD) {
                P[i] = (n == 0) ? 1.0 : P[i] * (double)tau[i] * isqn;
                D[i] = fma(P[i], ub, D[i]);
            }
        }
    }
    if (y < p.H) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int x = x0 + i;
            if (x < p.W) {
                const double rho = M[i] / D[i];
                p.out[(size_t)y * p.pitch + x] = st.ok ? (float)(st.tc + p.sigma_r * rho) : __builtin_nanf("");
            }
        }
    }
}

}  // namespace bfgp
