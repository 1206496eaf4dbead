// Backward of the GP forward (FIR spatial mode), derived by the chain rule
// through eqs. (7)-(11) and the mean that Algorithm 1 takes as the centre.
//
// With tau = x(i), rho = M/D, upstream g = dL/dout and the forward's saved
// rho, drho/dtau and D' = exp(tau^2/2) D (double):
//   adjoint of the filtered channels (n = 0..N+1):
//     V_n(i) = a(i) [ sqrt(n) p_{n-1}(tau) - rho p_n(tau) [n <= N] ],
//     a = g sigma_r / D',  p_n = tau^n / sqrt(n!)
//   (equal to dL/dM * sqrt(n) u_{n-1}(tau) + dL/dD * u_n(tau), the common
//   exp(-tau^2/2) cancelling);
//   the filter is symmetric with zero extension, so the adjoint of K is K:
//     W_n = K V_n,   Z_n = Kt V_n,  Kt = dK/dlog(sigma_s) = kt (x) k + k (x) kt,
//     kt(d) = (d^2 / sigma_s^2) k(d)  (radius held fixed);
//   per pixel j, with u_n' = sqrt(n) u_{n-1} - sqrt(n+1) u_{n+1}:
//     gH(j) = sum_n W_n(j) u_n'(x_j) + g(j) sigma_r drho/dtau(j),
//     dL/dlog sigma_s = sum_n sum_j Z_n(j) u_n(x_j),
//     dL/dlog sigma_r = sum_j g(j) sigma_r rho(j) - sum_j x_j gH(j),
//     dL/df_j = gH(j)/sigma_r + [mean centre] (sum g - sum gH/sigma_r) / |I|.
// One workgroup handles a 32 x 32 tile; per channel it forms V_n on the
// (32+2R)^2 region in LDS, runs the column pass with k and kt, the row pass
// (k on both, kt on the k-column result) and contracts at its 4 pixels.
#pragma once
#include "common.hpp"

namespace bfgp {

struct FirTaps2 {
    float k[kFirMaxR + 1];
    float kt[kFirMaxR + 1];
};

// Per-workgroup partial sums of the backward reductions.
struct BwdPartial {
    double sum_gh;    // sum of gH / sigma_r
    double sum_xgH;   // sum of x gH
    double sum_grho;  // sum of g sigma_r rho
    double sum_zu;    // sigma_s gradient
    double sum_g;     // sum of g
};

struct BwdParams {
    const float *grad_out;
    const float *saved;   // rho[HW], drho[HW], then D'[HW] as double
    float *grad_img;      // nullable; receives gH / sigma_r (+ correction later)
    BwdPartial *bparts;
};

template <int R>
struct BwdShape {
    static constexpr int TY = 32, TX = 32;
    static constexpr int RY = TY + 2 * R, RX = TX + 2 * R;
    static constexpr int REG = RY * RX;
    static constexpr int PER = (REG + kBlock - 1) / kBlock;
    static constexpr int SV = 4;
    static constexpr int BP = RX + 1;
    static constexpr int PX = 4;
    static constexpr int SMEM_FLOATS = REG + 2 * TY * BP;
};

template <int R>
__device__ __forceinline__ void bwd_tile(const GPParams &p, const BwdParams &b, const FirTaps2 &taps,
                                         const Stats &st, int ty0, int tx0, int tile, float *smem) {
    using S = BwdShape<R>;
    float *A = smem;
    float *B1 = smem + S::REG;
    float *B2 = B1 + S::TY * S::BP;
    const int tid = threadIdx.x;
    const size_t npx = (size_t)p.H * p.W;
    const float *rho_s = b.saved;
    const float *drho_s = b.saved + npx;
    const double *Dp_s = (const double *)(b.saved + 2 * npx);

    // region: s = a p_{n-1} (double), rho, tau
    double sr[S::PER];
    float rr[S::PER], xr[S::PER];
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
        const int e = tid + i * kBlock;
        sr[i] = 0.0;
        rr[i] = 0.f;
        xr[i] = 0.f;
        if (e < S::REG) {
            const int gy = ty0 - R + e / S::RX;
            const int gx = tx0 - R + e % S::RX;
            if (gy >= 0 && gy < p.H && gx >= 0 && gx < p.W) {
                const size_t idx = (size_t)gy * p.W + gx;
                xr[i] = centred(p.img[(size_t)gy * p.pitch + gx], st, p.inv_sigma_r);
                rr[i] = rho_s[idx];
                sr[i] = (double)b.grad_out[(size_t)gy * p.pitch + gx] * p.sigma_r / Dp_s[idx];  // a
            }
        }
    }

    // owned pixels: row oy, columns ox0..ox0+3
    const int oy = tid >> 3;
    const int ox0 = (tid & 7) * S::PX;
    double gH[S::PX], zu[S::PX], um[S::PX], u0[S::PX], up[S::PX];
    float tau[S::PX];
    const int gy = ty0 + oy;
#pragma unroll
    for (int i = 0; i < S::PX; ++i) {
        const int gx = tx0 + ox0 + i;
        float x = 0.f;
        if (gy < p.H && gx < p.W) x = centred(p.img[(size_t)gy * p.pitch + gx], st, p.inv_sigma_r);
        tau[i] = x;
        gH[i] = 0.0;
        zu[i] = 0.0;
        um[i] = 0.0;
        u0[i] = exp(-0.5 * (double)x * (double)x);
        up[i] = u0[i] * (double)x;  // u_1 = x u_0
    }

    for (int n = 0; n < p.C; ++n) {
        // 1. V_n on the region
        const double sqn = p.sq[n], isqn = p.isq[n];
        const bool inD = n <= p.N;
#pragma unroll
        for (int i = 0; i < S::PER; ++i) {
            const int e = tid + i * kBlock;
            if (e < S::REG) {
                double v;
                if (n == 0) {
                    v = -(double)rr[i] * sr[i];           // -rho a p_0
                } else {
                    // a p_{n-1} (sqrt(n) - rho tau / sqrt(n) [n <= N])
                    const double f = inD ? sqn - (double)rr[i] * (double)xr[i] * isqn : sqn;
                    v = sr[i] * f;
                    sr[i] *= (double)xr[i] * isqn;        // -> a p_n
                }
                A[e] = (float)v;
            }
        }
        __syncthreads();
        // 2. column pass with k and kt
        for (int it = tid; it < S::RX * (S::TY / S::SV); it += kBlock) {
            const int xx = it % S::RX, sy = it / S::RX;
            const float *col = A + sy * S::SV * S::RX + xx;
            float a1[S::SV], a2[S::SV];
#pragma unroll
            for (int i = 0; i < S::SV; ++i) {
                a1[i] = 0.f;
                a2[i] = 0.f;
            }
#pragma unroll
            for (int j = 0; j < S::SV + 2 * R; ++j) {
                const float v = col[j * S::RX];
#pragma unroll
                for (int i = 0; i < S::SV; ++i) {
                    const int d = j - i;
                    if (d >= 0 && d <= 2 * R) {
                        const int ad = d >= R ? d - R : R - d;
                        a1[i] = fmaf(taps.k[ad], v, a1[i]);
                        a2[i] = fmaf(taps.kt[ad], v, a2[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < S::SV; ++i) {
                B1[(sy * S::SV + i) * S::BP + xx] = a1[i];
                B2[(sy * S::SV + i) * S::BP + xx] = a2[i];
            }
        }
        __syncthreads();
        // 3. row pass at the owned pixels: W = k(B1), Z = kt(B1) + k(B2)
        float w[S::PX], z[S::PX];
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            w[i] = 0.f;
            z[i] = 0.f;
        }
        {
            const float *r1 = B1 + oy * S::BP + ox0;
            const float *r2 = B2 + oy * S::BP + ox0;
#pragma unroll
            for (int j = 0; j < S::PX + 2 * R; ++j) {
                const float v1 = r1[j], v2 = r2[j];
#pragma unroll
                for (int i = 0; i < S::PX; ++i) {
                    const int d = j - i;
                    if (d >= 0 && d <= 2 * R) {
                        const int ad = d >= R ? d - R : R - d;
                        w[i] = fmaf(taps.k[ad], v1, w[i]);
                        z[i] = fmaf(taps.kt[ad], v1, fmaf(taps.k[ad], v2, z[i]));
                    }
                }
            }
        }
        // 4. contraction with u_n' and u_n at the owned pixels
        const double sqn1 = p.sq[n + 1], isqn2 = p.isq[n + 2];
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            const double du = sqn * um[i] - sqn1 * up[i];
            gH[i] = fma((double)w[i], du, gH[i]);
            zu[i] = fma((double)z[i], u0[i], zu[i]);
            um[i] = u0[i];
            u0[i] = up[i];
            up[i] = up[i] * (double)tau[i] * isqn2;  // u_{n+2}
        }
    }

    // ---- per-pixel gradient and per-workgroup sums ----
    double s_gh = 0.0, s_xgH = 0.0, s_grho = 0.0, s_zu = 0.0, s_g = 0.0;
    if (gy < p.H) {
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            const int gx = tx0 + ox0 + i;
            if (gx < p.W) {
                const size_t idx = (size_t)gy * p.W + gx;
                const double g = (double)b.grad_out[(size_t)gy * p.pitch + gx];
                const double h = gH[i] + g * p.sigma_r * (double)drho_s[idx];
                const double gh = h * p.inv_sigma_r;
                if (b.grad_img) b.grad_img[(size_t)gy * p.pitch + gx] = (float)gh;
                s_gh += gh;
                s_xgH += (double)tau[i] * h;
                s_grho += g * p.sigma_r * (double)rho_s[idx];
                s_zu += zu[i];
                s_g += g;
            }
        }
    }
    // block reduction in a fixed order
    __shared__ double red[5][kBlock / 64];
    double v[5] = {s_gh, s_xgH, s_grho, s_zu, s_g};
#pragma unroll
    for (int q = 0; q < 5; ++q) v[q] = wave_sum(v[q]);
    __syncthreads();
    if ((tid & 63) == 0)
        for (int q = 0; q < 5; ++q) red[q][tid >> 6] = v[q];
    __syncthreads();
    if (tid == 0) {
        double o[5];
        for (int q = 0; q < 5; ++q) {
            o[q] = 0.0;
            for (int w2 = 0; w2 < kBlock / 64; ++w2) o[q] += red[q][w2];
        }
        BwdPartial bp;
        bp.sum_gh = o[0];
        bp.sum_xgH = o[1];
        bp.sum_grho = o[2];
        bp.sum_zu = o[3];
        bp.sum_g = o[4];
        b.bparts[tile] = bp;
    }
}

}  // namespace bfgp
