// Fused FIR forward: channel generation, both spatial passes and the FP64
// recombination for one output tile, all in LDS / registers.
//
// Per tile (TY x TX outputs) and per channel n = 0..N+1 (eq. (7), rescaled):
//   1. every thread updates its share of the (TY+2R) x (TX+2R) input region,
//      u_n = u_{n-1} * x / sqrt(n) (double), and stores it to LDS as float;
//   2. the column pass of eq. (8): B = k (*) A along y, (TY) x (TX+2R);
//   3. the row pass of eq. (8): Ubar_n at the thread's PX output pixels;
//   4. the recombination of eqs. (9)-(11) as power sums in tau (double):
//        D' += p_n Ubar_n (n <= N),  M' += sqrt(n) p_{n-1} Ubar_n (n >= 1),
//      p_n = tau^n / sqrt(n!).  D' = exp(tau^2/2) D and M' = exp(tau^2/2) M,
//      so M'/D' = M/D.
// Steps 1-2 and 3-4 each run for CH channels between barriers.  The channel
// buffer never leaves the chip: HBM traffic is the input region and the
// output tile.
#pragma once
#include "common.hpp"

namespace bfgp {

// Two variants share each kernel.  The register-column variant (radii up to
// kFirRegMaxR, kFirRegMaxRSave with the saved terms) gives every thread one column
// of the input region: its channel values stay in registers and its column
// pass runs from them, so LDS only carries the column-filtered rows to the row
// pass.  The region variant (below) stages the region in LDS; it serves wider
// radii, the saved terms, and images the register variant cannot represent
// (|x| > 12, degree above kFirRegMaxN), with the same tile shape.
constexpr int kFirRegMaxR = 16;
constexpr int kFirRegMaxRSave = 12;  // with the saved terms (two more FP64 sums per pixel)
constexpr int kFirXcStride = 36;     // floats per thread of the x rows kept in LDS with the saved terms
constexpr int kFirRegMaxN = 46;
__host__ __device__ constexpr bool fir_reg(int R, bool save) { return R <= (save ? kFirRegMaxRSave : kFirRegMaxR); }

// Output tile of a FIR launch: fir_tx(R, save) columns by fir_ty(R, save)
// rows.  Kernels that can take the register variant use 8 x 224 tiles: the
// region's 224 + 2R columns (R <= 16) give every one of the four waves a
// column-pass share (fewer than 193 columns would leave a wave idle through
// the heaviest phase); the region variant then covers such a tile as four
// 8 x 64 pieces, the last one cut at the tile's edge.  Other kernels use the
// region variant's own tile, 64 columns wide: 16-row tiles give twice the
// workgroups and fewer registers per thread; they were measured faster except
// for radii 10..17 without the saved terms, where the halo rows of a 16-row
// tile cost more than the extra parallelism gains.  With the saved terms (more
// accumulators) 16 rows keep two waves per SIMD.
constexpr int kFirRegTY = 8, kFirRegTX = 224;
__host__ __device__ constexpr int fir_region_ty(int R, bool save = false) {
    return (!fir_reg(R, save) && !save && R >= 10 && R <= 17) ? 32 : 16;
}
__host__ __device__ constexpr int fir_tx(int R, bool save = false) { return fir_reg(R, save) ? kFirRegTX : 64; }
__host__ __device__ constexpr int fir_ty(int R, bool save = false) {
    return fir_reg(R, save) ? kFirRegTY : fir_region_ty(R, save);
}

// LDS floats of one channel stage of the region variant with TY-row tiles:
// the region, then the column-pass output (odd pitch).
__host__ __device__ constexpr int fir_stage_floats(int R, int TY) {
    return (TY + 2 * R) * (64 + 2 * R) + TY * (64 + 2 * R + 1);
}
// Channels processed between two barrier pairs by the region variant: two
// (twice the independent work per barrier) where the LDS stages of two
// channels fit in 64 KB.
__host__ __device__ constexpr int fir_ch_ty(int R, int TY, bool save) {
    return (!save && 2 * fir_stage_floats(R, TY) <= 16384) ? 2 : 1;
}
__host__ __device__ constexpr int fir_ch(int R, bool save = false) { return fir_ch_ty(R, fir_region_ty(R, save), save); }

// Shape of the region variant's tile (64 columns, TYO rows).
template <int R, bool SAVE = false, int TYO = fir_region_ty(R, SAVE)>
struct FirShape {
    static constexpr int TY = TYO, TX = 64;       // output tile
    static constexpr int RY = TY + 2 * R, RX = TX + 2 * R;
    static constexpr int REG = RY * RX;           // region elements
    static constexpr int PER = (REG + kBlock - 1) / kBlock;
    static constexpr int SV = 4;                  // column-pass outputs per item
    static constexpr int BP = RX + 1;             // odd pitch of the row-pass input
    static constexpr int PX = TY * TX / kBlock;   // output pixels per thread (one row segment)
    static constexpr int CH = fir_ch_ty(R, TY, SAVE);  // channels per barrier pair
    static constexpr int STAGE = REG + TY * BP;   // LDS floats per channel
    static constexpr int SMEM_FLOATS = CH * STAGE;
};

// Number of LDS floats needed by fir_tile_auto<R, save> (either variant).
__host__ __device__ constexpr int fir_smem_floats(int R, bool save = false) {
    return fir_reg(R, save)
               ? (fir_ch_ty(R, kFirRegTY, save) * fir_stage_floats(R, kFirRegTY) >
                          4 * kFirRegTY * (kFirRegTX + 2 * R + 1) + (save ? kBlock * kFirXcStride : 0)
                      ? fir_ch_ty(R, kFirRegTY, save) * fir_stage_floats(R, kFirRegTY)
                      : 4 * kFirRegTY * (kFirRegTX + 2 * R + 1) + (save ? kBlock * kFirXcStride : 0))
               : fir_ch(R, save) * fir_stage_floats(R, fir_region_ty(R, save));
}

// Region variant; outputs at columns >= xlim are left to the tile that owns
// them.
template <int R, bool SAVE, int TYO = fir_region_ty(R, SAVE)>
__device__ __forceinline__ void fir_tile(const GPParams &p, const FirTaps &taps, const Stats &st,
                                         int ty0, int tx0, float *smem, int xlim = 0x7fffffff) {
    using S = FirShape<R, SAVE, TYO>;
    // stage c (one per channel in flight): region A_c (RY x RX), then the
    // column-pass output B_c (TY x BP)
    auto A = [&](int c) { return smem + c * S::STAGE; };
    auto Bc = [&](int c) { return smem + c * S::STAGE + S::REG; };
    const int tid = threadIdx.x;

    // ---- region: centred intensities and u_0 = exp(-x^2/2) ----
    // every load is issued unconditionally from a clamped address, so that
    // all of them are in flight together; samples outside the image (or past
    // the region) are zeroed afterwards
    float xr[S::PER];
    double u[S::PER];
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
        const int e = tid + i * kBlock;
        const int gy = ty0 - R + e / S::RX;
        const int gx = tx0 - R + e % S::RX;
        const int yc = gy < 0 ? 0 : (gy >= p.H ? p.H - 1 : gy);
        const int xc = gx < 0 ? 0 : (gx >= p.W ? p.W - 1 : gx);
        xr[i] = p.img[(size_t)yc * p.pitch + xc];
    }
#pragma unroll
    for (int i = 0; i < S::PER; ++i) {
        const int e = tid + i * kBlock;
        const int gy = ty0 - R + e / S::RX;
        const int gx = tx0 - R + e % S::RX;
        const bool in = e < S::REG && gy >= 0 && gy < p.H && gx >= 0 && gx < p.W;
        const float x = in ? centred(xr[i], st, p.inv_sigma_r) : 0.f;
        xr[i] = x;
        // exp(-x^2/2) formed with a range shift and taken to double exactly,
        // so that it does not underflow where |x| > 13 (double carries it)
        const int sh = big_shift(x);
        u[i] = in ? ldexp((double)gauss_u0(x, sh), -sh) : 0.0;
    }

    // ---- output ownership: row oy, PX consecutive columns from ox0 ----
    const int oy = tid % S::TY;
    const int ox0 = (tid / S::TY) * S::PX;
    double tau[S::PX], Dp[S::PX], Mp[S::PX], pw[S::PX];
    double Dt[SAVE ? S::PX : 1], Mt[SAVE ? S::PX : 1], pm[SAVE ? S::PX : 1];
    {
        const int gy = ty0 + oy;
        const int yc = gy < p.H ? gy : p.H - 1;
        float f[S::PX];
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            const int gx = tx0 + ox0 + i;
            f[i] = p.img[(size_t)yc * p.pitch + (gx < p.W ? gx : p.W - 1)];
        }
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            const int gx = tx0 + ox0 + i;
            const float x = (gy < p.H && gx < p.W) ? centred(f[i], st, p.inv_sigma_r) : 0.f;
            tau[i] = (double)x;
            Dp[i] = 0.0;
            Mp[i] = 0.0;
            pw[i] = 0.0;
            if (SAVE) {
                Dt[i] = 0.0;
                Mt[i] = 0.0;
                pm[i] = 0.0;
            }
        }
    }

    for (int n0 = 0; n0 < p.C; n0 += S::CH) {
        const int nc = p.C - n0 < S::CH ? p.C - n0 : S::CH;  // channels this round
        // 1. channels n0 .. n0+nc-1 on the region
#pragma unroll
        for (int c = 0; c < S::CH; ++c) {
            if (c < nc) {
                const int n = n0 + c;
                const double isq = p.isq[n];
                float *Ac = A(c);
#pragma unroll
                for (int i = 0; i < S::PER; ++i) {
                    const int e = tid + i * kBlock;
                    if (e < S::REG) {
                        if (n > 0) u[i] *= (double)xr[i] * isq;
                        Ac[e] = (float)u[i];
                    }
                }
            }
        }
        __syncthreads();
        // 2. column pass
        for (int it = tid; it < S::RX * (S::TY / S::SV); it += kBlock) {
            const int xx = it % S::RX, sy = it / S::RX;
#pragma unroll
            for (int c = 0; c < S::CH; ++c) {
                if (c < nc) {
                    const float *col = A(c) + sy * S::SV * S::RX + xx;
                    float acc[S::SV];
#pragma unroll
                    for (int i = 0; i < S::SV; ++i) acc[i] = 0.f;
#pragma unroll
                    for (int j = 0; j < S::SV + 2 * R; ++j) {
                        const float v = col[j * S::RX];
#pragma unroll
                        for (int i = 0; i < S::SV; ++i) {
                            const int d = j - i;
                            if (d >= 0 && d <= 2 * R) acc[i] = fmaf(taps.k[d >= R ? d - R : R - d], v, acc[i]);
                        }
                    }
                    float *Bo = Bc(c);
#pragma unroll
                    for (int i = 0; i < S::SV; ++i) Bo[(sy * S::SV + i) * S::BP + xx] = acc[i];
                }
            }
        }
        __syncthreads();
        // 3. row pass at the owned pixels, 4. recombination per channel
#pragma unroll
        for (int c = 0; c < S::CH; ++c) {
            if (c < nc) {
                const int n = n0 + c;
                float h[S::PX];
#pragma unroll
                for (int i = 0; i < S::PX; ++i) h[i] = 0.f;
                {
                    const float *row = Bc(c) + oy * S::BP + ox0;
#pragma unroll
                    for (int j = 0; j < S::PX + 2 * R; ++j) {
                        const float v = row[j];
#pragma unroll
                        for (int i = 0; i < S::PX; ++i) {
                            const int d = j - i;
                            if (d >= 0 && d <= 2 * R) h[i] = fmaf(taps.k[d >= R ? d - R : R - d], v, h[i]);
                        }
                    }
                }
                // recombination, double precision.  Channel 0 only starts D'
                // (p_0 = 1) and channel N+1 only enters M': uniform branches,
                // so that the common case carries no per-pixel selects.
                const double isq = p.isq[n];
                const double sqn = p.sq[n];
                const double sqm = n >= 1 ? p.sq[n - 1] : 0.0;
                if (n >= 1 && n <= p.N) {
#pragma unroll
                    for (int i = 0; i < S::PX; ++i) {
                        const double ub = (double)h[i];
                        const double q = pw[i] * sqn;  // sqrt(n) p_{n-1}
                        Mp[i] = fma(q, ub, Mp[i]);
                        if (SAVE) {
                            Dt[i] = fma(q, ub, Dt[i]);
                            Mt[i] = fma(sqn * sqm * pm[i], ub, Mt[i]);
                            pm[i] = pw[i];
                        }
                        pw[i] = pw[i] * tau[i] * isq;
                        Dp[i] = fma(pw[i], ub, Dp[i]);
                    }
                } else if (n == 0) {
#pragma unroll
                    for (int i = 0; i < S::PX; ++i) {
                        if (SAVE) pm[i] = pw[i];
                        pw[i] = 1.0;
                        Dp[i] = fma(pw[i], (double)h[i], Dp[i]);
                    }
                } else {
#pragma unroll
                    for (int i = 0; i < S::PX; ++i) {
                        const double ub = (double)h[i];
                        Mp[i] = fma(pw[i] * sqn, ub, Mp[i]);
                        if (SAVE) Mt[i] = fma(sqn * sqm * pm[i], ub, Mt[i]);
                    }
                }
            }
        }
    }

    // ---- outputs ----
    const int gy = ty0 + oy;
    if (gy < p.H) {
        const size_t npx = (size_t)p.H * p.W;
#pragma unroll
        for (int i = 0; i < S::PX; ++i) {
            const int gx = tx0 + ox0 + i;
            if (gx < p.W && gx < xlim) {
                const double rho = Mp[i] / Dp[i];
                const float o = st.ok ? (float)fma(p.sigma_r, rho, st.tc) : __builtin_nanf("");
                p.out[(size_t)gy * p.pitch + gx] = o;
                if (SAVE) {
                    const size_t idx = (size_t)gy * p.W + gx;
                    float *sv = (float *)p.saved;
                    sv[idx] = (float)rho;
                    sv[npx + idx] = (float)(Mt[i] / Dp[i] - rho * Dt[i] / Dp[i]);
                    ((double *)(sv + 2 * npx))[idx] = Dp[i];
                }
            }
        }
    }
}

// Register-column variant (8 x 224 tile, radius R <= kFirRegMaxR).  The
// channels are carried unnormalised, w_n = exp(-x^2/2) x^n = sqrt(n!) u_n
// (one multiply per sample and channel); the 1/sqrt(n!) goes into the
// recombination weights: with q_n = tau^n / n!,
//   D' = sum_{n<=N} q_n (k * w_n),   M' = sum_{n=1}^{N+1} q_{n-1} (k * w_n),
// the same D' = exp(tau^2/2) D and M' = exp(tau^2/2) M as the region variant.
// w_n stays in the FP32 range for |x| <= 12 and n <= kFirRegMaxN + 1.
// Per pair of channels: threads 0 .. 223+2R update their region column and
// run its column pass from registers into LDS (two pairs of buffers, one
// barrier per pair), then every thread runs the row pass at its 7 pixels (one
// row segment; the 32 threads of a row read LDS at a stride of 7 words, on
// distinct banks) and accumulates D', M' in double.
// SAVE: the terms the backward pass needs are stored as well: rho = M'/D',
// drho/dtau = (dM'/dtau - rho dD'/dtau) / D' and D', with (filtered channels
// held fixed) dD'/dtau = sum_{1<=n<=N} q_{n-1} (k * w_n) (M' without its
// N+1 term) and dM'/dtau = sum_{n>=2} q_{n-2} (k * w_n).
template <int R, bool SAVE = false>
__device__ __forceinline__ void fir_tile_reg(const GPParams &p, const FirTaps &taps, const Stats &st, int ty0,
                                             int tx0, float *smem) {
    constexpr int TY = kFirRegTY, TX = kFirRegTX, RX = TX + 2 * R, RY = TY + 2 * R, BP = RX + 1;
    constexpr int PX = TY * TX / kBlock, RT = TX / PX;  // pixels per thread, threads per output row
    static_assert(RX <= kBlock, "one region column per thread");
    static_assert(PX * RT == TX && RT * TY == kBlock, "row segments cover the tile");
    const int tid = threadIdx.x;
    const bool colt = tid < RX;

    // ---- region column tid: centred x and w_0 = exp(-x^2/2) ----
    // SAVE: the column's x values wait in LDS (a row of kFirXcStride floats per
    // thread after the four row-pass buffers; the stride is 4 more than a
    // multiple of 32, so eight lanes' 16-byte reads fall on distinct banks),
    // which leaves the registers to the two more FP64 sums per pixel
    static_assert(!SAVE || RY <= kFirXcStride, "x row fits");
    float w[RY], xc[SAVE ? 1 : RY];
    float *xcs = smem + 4 * TY * BP + tid * kFirXcStride;
    {
        const int gx = tx0 - R + tid;
        const int xcl = gx < 0 ? 0 : (gx >= p.W ? p.W - 1 : gx);
        const bool inx = colt && gx >= 0 && gx < p.W;
        float f[RY];
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = ty0 - R + j;
            const int yc = gy < 0 ? 0 : (gy >= p.H ? p.H - 1 : gy);
            f[j] = p.img[(size_t)yc * p.pitch + xcl];
        }
#pragma unroll
        for (int j = 0; j < RY; ++j) {
            const int gy = ty0 - R + j;
            const bool in = inx && gy >= 0 && gy < p.H;
            const float x = in ? centred(f[j], st, p.inv_sigma_r) : 0.f;
            if constexpr (SAVE) {
                if (colt) xcs[j] = x;
            } else {
                xc[j] = x;
            }
            w[j] = in ? gauss_u0(x, 0) : 0.f;
        }
    }

    // ---- output ownership: row oy, PX consecutive columns from ox0 ----
    const int oy = tid / RT;
    const int ox0 = (tid % RT) * PX;
    double tau[PX], Dp[PX], Mp[PX], q[PX];
    double Mt[SAVE ? PX : 1], qq[SAVE ? PX : 1], Dt[SAVE ? PX : 1];  // dM'/dtau, q_{n-2}, dD'/dtau
    {
        const int gy = ty0 + oy;
        const int yc = gy < p.H ? gy : p.H - 1;
        float f[PX];
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            const int gx = tx0 + ox0 + i;
            f[i] = p.img[(size_t)yc * p.pitch + (gx < p.W ? gx : p.W - 1)];
        }
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            const int gx = tx0 + ox0 + i;
            tau[i] = (gy < p.H && gx < p.W) ? (double)centred(f[i], st, p.inv_sigma_r) : 0.0;
            Dp[i] = 0.0;
            Mp[i] = 0.0;
            q[i] = 1.0;
            if constexpr (SAVE) {
                Mt[i] = 0.0;
                qq[i] = 0.0;
                Dt[i] = 0.0;
            }
        }
    }

    // column pass of the next channel from registers into B
    auto column = [&](int n, float *B) {
        if (n > 0) {
            if constexpr (SAVE) {
#pragma unroll
                for (int j = 0; j + 3 < RY; j += 4) {
                    const float4 v = *(const float4 *)(xcs + j);
                    w[j] *= v.x; w[j + 1] *= v.y; w[j + 2] *= v.z; w[j + 3] *= v.w;
                }
#pragma unroll
                for (int j = RY & ~3; j < RY; ++j) w[j] *= xcs[j];
            } else {
#pragma unroll
                for (int j = 0; j < RY; ++j) w[j] *= xc[j];
            }
        }
        float acc[TY];
#pragma unroll
        for (int i = 0; i < TY; ++i) {
            float a = 0.f;
#pragma unroll
            for (int d = -R; d <= R; ++d) a = fmaf(taps.k[d < 0 ? -d : d], w[i + R + d], a);
            acc[i] = a;
        }
#pragma unroll
        for (int i = 0; i < TY; ++i) B[i * BP + tid] = acc[i];
    };
    // row pass of channel n at the owned pixels, then the recombination
    // (double): M' takes q_{n-1}, D' takes q_n; channel 0 only starts D',
    // channel N+1 only ends M' (uniform branches)
    auto row = [&](int n, const float *B) {
        float h[PX];
#pragma unroll
        for (int i = 0; i < PX; ++i) h[i] = 0.f;
        {
            const float *r = B + oy * BP + ox0;
#pragma unroll
            for (int j = 0; j < PX + 2 * R; ++j) {
                const float v = r[j];
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    const int d = j - i;
                    if (d >= 0 && d <= 2 * R) h[i] = fmaf(taps.k[d >= R ? d - R : R - d], v, h[i]);
                }
            }
        }
        if (n == 0) {
#pragma unroll
            for (int i = 0; i < PX; ++i) Dp[i] = (double)h[i];
        } else {
            const double rn = p.inv[n];
            if (n <= p.N) {
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    const double hd = (double)h[i];
                    if constexpr (SAVE) {
                        Mt[i] = fma(qq[i], hd, Mt[i]);  // q_{n-2} (0 at n = 1)
                        qq[i] = q[i];
                    }
                    Mp[i] = fma(q[i], hd, Mp[i]);
                    q[i] *= tau[i] * rn;
                    Dp[i] = fma(q[i], hd, Dp[i]);
                }
            } else {
#pragma unroll
                for (int i = 0; i < PX; ++i) {
                    const double hd = (double)h[i];
                    if constexpr (SAVE) {
                        Mt[i] = fma(qq[i], hd, Mt[i]);
                        Dt[i] = Mp[i];  // M' without the N+1 term
                    }
                    Mp[i] = fma(q[i], hd, Mp[i]);
                }
            }
        }
    };
    // two channels per step between barriers (pairs of buffers, alternating
    // between steps): half the barriers, and each phase has two channels'
    // independent work in flight
    for (int n = 0; n < p.C; n += 2) {
        const bool two = n + 1 < p.C;  // uniform
        float *B0 = smem + ((n >> 1) & 1) * (2 * TY * BP);
        float *B1 = B0 + TY * BP;
        if (colt) {
            column(n, B0);
            if (two) column(n + 1, B1);
        }
        __syncthreads();
        row(n, B0);
        if (two) row(n + 1, B1);
    }

    const int gy = ty0 + oy;
    if (gy < p.H) {
        const size_t npx = (size_t)p.H * p.W;
#pragma unroll
        for (int i = 0; i < PX; ++i) {
            const int gx = tx0 + ox0 + i;
            if (gx < p.W) {
                const double rho = Mp[i] / Dp[i];
                p.out[(size_t)gy * p.pitch + gx] = st.ok ? (float)fma(p.sigma_r, rho, st.tc) : __builtin_nanf("");
                if constexpr (SAVE) {
                    const size_t idx = (size_t)gy * p.W + gx;
                    float *sv = (float *)p.saved;
                    sv[idx] = (float)rho;
                    sv[npx + idx] = (float)(Mt[i] / Dp[i] - rho * Dt[i] / Dp[i]);
                    ((double *)(sv + 2 * npx))[idx] = Dp[i];
                }
            }
        }
    }
}

// The FIR tile with the variant this image can take (the choice is uniform
// over the launch: it depends on the image statistics and the degree only).
template <int R, bool SAVE>
__device__ __forceinline__ void fir_tile_auto(const GPParams &p, const FirTaps &taps, const Stats &st, int ty0,
                                              int tx0, float *smem) {
    if constexpr (fir_reg(R, SAVE)) {
        if (st.xmax <= 12.0 && p.N <= kFirRegMaxN) {
            fir_tile_reg<R, SAVE>(p, taps, st, ty0, tx0, smem);
        } else {
            for (int k = 0; k < kFirRegTX; k += 64) {
                fir_tile<R, SAVE, kFirRegTY>(p, taps, st, ty0, tx0 + k, smem, tx0 + kFirRegTX);
                __syncthreads();  // the next piece reuses the LDS stages
            }
        }
    } else {
        fir_tile<R, SAVE>(p, taps, st, ty0, tx0, smem);
    }
}

}  // namespace bfgp
