// Box spatial kernel: eq. (8) with uniform weights over the window of eq. (1),
// |dy|, |dx| <= R.  Section 3 notes, after eq. (11), that the derivation holds
// for any spatial filter with a constant-time implementation, a box filter for
// instance; a box has one: running sums.  Two passes over the channel stack,
// both O(1) per pixel and channel whatever R is:
//
//   column pass: one thread per column, band of rows and group of channels;
//     the channels of the row entering the window are added to FP64 running
//     sums and those of the row leaving it subtracted, so each band costs its
//     rows plus one window of start-up.  Channels are generated in double as
//     e^{-x^2/2} x^n and normalised by 1/sqrt(n!) at the store, as FP32, into
//     the stack S[n][y][x] (row pitch P >= W, rows 16-byte aligned).
//   row pass: one workgroup per image row; per channel, the row's FP64
//     exclusive prefix sums go to LDS (chunk sums in registers, a DPP wave
//     scan, wave totals through LDS), and every pixel's window sum is the
//     difference of two prefix values; the recombination of eqs. (9)-(11) follows as a
//     Horner evaluation in tau (double), channels taken from the top down.
//
// Prefix sums and running sums are FP64: a window sum is then off by at most
// about 1e-16 of the row's (column's) absolute channel mass, which the
// recombination weighs below 1e-9 of the pixel's own weight.  In FP32 the same
// differences would lose the small window sums of a row with large ones
// elsewhere.
#pragma once
#include "common.hpp"

namespace bfgp {

constexpr int kBoxKC = 24;      // most channels one column-pass thread accumulates
constexpr int kBoxMaxW = 16384;  // widest row of the row pass (T L >= W, L 4, 16 or 32)

// Launch shape of the box passes.
struct BoxShape {
    int R;   // window radius (at most max(H, W): a wider window changes nothing)
    int Bb;  // rows per band of the column pass
    int nb;  // bands
    int G;   // channel groups of the column pass
    int NC;  // channels one column-pass thread accumulates (4, 6, 8, 12, 16 or 24),
             // at least ceil(C / G)
    int L;   // samples per thread of the row pass: 4 (W <= 4096) or 16
    int T;   // threads per row (a multiple of 64, T L >= W; at most 1024 for
             // L = 4, 512 for L = 16)
    int P;   // row pitch of the stack: T L
};

// 1 / sqrt(n!), n = 0 .. kMaxC - 1 (host-built): the column pass accumulates
// e^{-x^2/2} x^n and normalises at the store.
struct BoxFact {
    double ifs[kMaxC];
};

// x^e for a small non-negative integer e (binary powering)
__device__ __forceinline__ double box_ipow(double x, int e) {
    double r = 1.0;
    while (e > 0) {
        if (e & 1) r *= x;
        x *= x;
        e >>= 1;
    }
    return r;
}

// exp(-x^2/2) x^cb in double: exp(-x^2/2) is formed at a power-of-two shift
// where it would leave the FP32 range, and taken to double exactly.
__device__ __forceinline__ double box_lead(float xf, int cb) {
    const int sh = big_shift(xf);
    return ldexp((double)gauss_u0(xf, sh), -sh) * box_ipow((double)xf, cb);
}

// Column pass for column `col` (< W), rows [y0, y1), channels [cb, cb + nch),
// nch <= NC.  acc[k] holds the window sum of e^{-x^2/2} x^(cb+k); every row
// adds the channels of the row entering the window and subtracts those of the
// row leaving it in one update (two independent power chains), and stores
// acc[k] / sqrt((cb+k)!).  Channels k >= nch are accumulated but not stored.
// Rows are loaded eight at a time, the next eight issued before the current
// ones are used (in the start-up window too).
template <int NC>
__device__ __forceinline__ void boxcol(const GPParams &p, const BoxFact &bfct, const Stats &st, int R, int col,
                                       int y0, int y1, int cb, int nch, float *__restrict__ S, int P) {
    double acc[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) acc[k] = 0.0;
    const float *img = p.img + col;
    const size_t pitch = (size_t)p.pitch;
    const int H = p.H;
    auto clampy = [H](int y) { return y < 0 ? 0 : (y < H ? y : H - 1); };
    // start-up: rows y0 - R - 1 .. y0 + R - 1 (inside the image), the window of
    // row y0 before its update
    {
        const int a = y0 - R - 1 > 0 ? y0 - R - 1 : 0;
        const int b = y0 + R < H ? y0 + R : H;  // exclusive
        float f[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) f[i] = img[(size_t)clampy(a + i) * pitch];
        for (int y = a; y < b; y += 8) {
            float fn[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) fn[i] = img[(size_t)clampy(y + 8 + i) * pitch];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                if (y + i < b) {
                    const float x = centred(f[i], st, p.inv_sigma_r);
                    double u = box_lead(x, cb);
#pragma unroll
                    for (int k = 0; k < NC; ++k) {
                        acc[k] += u;
                        u *= (double)x;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) f[i] = fn[i];
        }
    }
    float *out = S + ((size_t)cb * H) * P + col;
    const size_t cstride = (size_t)H * P;
    float fe[8], fl[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        fe[i] = img[(size_t)clampy(y0 + i + R) * pitch];
        fl[i] = img[(size_t)clampy(y0 + i - R - 1) * pitch];
    }
    for (int y = y0; y < y1; y += 8) {
        float ne[8], nl[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            ne[i] = img[(size_t)clampy(y + 8 + i + R) * pitch];
            nl[i] = img[(size_t)clampy(y + 8 + i - R - 1) * pitch];
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int yy = y + i;
            if (yy < y1) {
                const float xe = centred(fe[i], st, p.inv_sigma_r);
                const float xl = centred(fl[i], st, p.inv_sigma_r);
                double ue = yy + R < H ? box_lead(xe, cb) : 0.0;
                double ul = yy - R - 1 >= 0 ? box_lead(xl, cb) : 0.0;
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    acc[k] += ue - ul;
                    ue *= (double)xe;
                    ul *= (double)xl;
                }
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    if (k < nch)
                        out[k * cstride + (size_t)yy * P] = (float)(acc[k] * bfct.ifs[min(cb + k, kMaxC - 1)]);
            }
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            fe[i] = ne[i];
            fl[i] = nl[i];
        }
    }
}

// DPP lane shifts of a double (both halves moved alike); lanes whose source
// is outside the row (wave) read 0.
constexpr int kBoxRowShr = 0x110, kBoxWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ double box_dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double box_lane(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}
// Inclusive sum of v over lanes 0 .. lane of the wave: scans inside each row
// of 16 lanes (shifts 1, 2, 4, 8), then the row totals read by readlane.
__device__ __forceinline__ double box_wave_scan(double v, int lane) {
    v += box_dpp<kBoxRowShr + 1>(v);
    v += box_dpp<kBoxRowShr + 2>(v);
    v += box_dpp<kBoxRowShr + 4>(v);
    v += box_dpp<kBoxRowShr + 8>(v);
    const double r0 = box_lane(v, 15), r1 = box_lane(v, 31), r2 = box_lane(v, 47);
    const int r = lane >> 4;
    if (r >= 1) v += r0;
    if (r >= 2) v += r1;
    if (r >= 3) v += r2;
    return v;
}

// LDS of the row pass: per channel of a step, the T L + 1 exclusive prefix
// values with one pad slot after every chunk of L (T L + T + 2 slots), and the
// wave totals.
__host__ __device__ constexpr size_t boxrow_pe_stride(int T, int L) { return (size_t)T * L + T + 2; }
__host__ __device__ constexpr size_t boxrow_smem_bytes(int T, int L, int K) {
    return sizeof(double) * (size_t)K * (boxrow_pe_stride(T, L) + (size_t)(T / 64));
}

// Row pass and recombination of image row y.  Thread t holds the contiguous
// chunk [t L, t L + L) of the prefix scan and the output pixels t + k T,
// k < L (consecutive lanes read consecutive prefix values).  K channels are
// scanned per step (one pair of barriers for all of them, their chains
// independent); the next step's chunks are in flight meanwhile (two steps
// ahead measured no faster).
// Horner in tau over the channels from the top down, as
//   bD <- Ubar_n + bD tau / sqrt(n+1)  (n <= N),
//   bM <- Ubar_n + bM tau sqrt(n+1) / n  (n >= 1),
// ends with bD = exp(tau^2/2) D and bM = exp(tau^2/2) M, so M/D = bM/bD.
// sm: boxrow_smem_bytes(T, L, K) bytes.  Every thread of the workgroup takes
// part in every barrier.
// LO < L: the workgroup scans the whole row but evaluates only the outputs
// t + k T for k in [ob, ob + LO) (rows too wide for L accumulators a thread:
// two workgroups per row share the outputs).
template <int L, int K, int LO = L>
__device__ __forceinline__ void boxrow(const GPParams &p, const Stats &st, int R, int y, const float *__restrict__ S,
                                       int P, int T, double *sm, int ob = 0) {
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int TL = T * L, x0 = t * L;
    // channel j of a step: prefix values at Pe + j PS (the sum of the row's
    // samples 0 .. m-1 at slot m + m / L: a thread's chunk is written at a
    // stride of L + 1 doubles across lanes, which spreads it over the LDS
    // banks, and consecutive m stay consecutive for the reads), wave totals
    // at wt + j nw
    const size_t PS = boxrow_pe_stride(T, L);
    double *Pe = sm;
    double *wt = sm + (size_t)K * PS;
    float tau[LO];
    double bD[LO], bM[LO];
    {
        const float *irow = p.img + (size_t)y * p.pitch;
#pragma unroll
        for (int k = 0; k < LO; ++k) {
            const int x = t + (ob + k) * T;
            tau[k] = x < p.W ? centred(irow[x], st, p.inv_sigma_r) : 0.f;
            bD[k] = 0.0;
            bM[k] = 0.0;
        }
    }
    auto load = [&](int n, float *d) {
        const float *row = S + ((size_t)(n > 0 ? n : 0) * p.H + y) * P + x0;
#pragma unroll
        for (int i = 0; i < L; i += 4) {
            const float4 q = *(const float4 *)(row + i);
            d[i] = q.x; d[i + 1] = q.y; d[i + 2] = q.z; d[i + 3] = q.w;
        }
    };
    // the next step's chunks are loaded at the top of each step
    float z[K][L];
#pragma unroll
    for (int j = 0; j < K; ++j) load(p.C - 1 - j, z[j]);
    for (int n0 = p.C - 1; n0 >= 0; n0 -= K) {
        float zn[K][L];
#pragma unroll
        for (int j = 0; j < K; ++j) load(n0 - K - j, zn[j]);
        double run[K], ex[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            run[j] = 0.0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                z[j][i] = x0 + i < p.W ? z[j][i] : 0.f;  // pad columns hold no data
                run[j] += (double)z[j][i];
            }
            const double s = box_wave_scan(run[j], lane);
            ex[j] = box_dpp<kBoxWaveShr1>(s);
            if (lane == 63) wt[j * nw + wave] = s;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K; ++j) {
            // totals of the waves before this one: lane l < nw (<= 16) reads
            // wave l's total, a scan inside the first row of 16 lanes sums
            // them, and lane wave - 1 holds the offset
            double v = lane < nw ? wt[j * nw + lane] : 0.0;
            v += box_dpp<kBoxRowShr + 1>(v);
            v += box_dpp<kBoxRowShr + 2>(v);
            v += box_dpp<kBoxRowShr + 4>(v);
            v += box_dpp<kBoxRowShr + 8>(v);
            const double base = ex[j] + (wave > 0 ? box_lane(v, wave > 0 ? wave - 1 : 0) : 0.0);
            double *pe = Pe + (size_t)j * PS;
            // the chunk's exclusive prefix (the same additions in the same
            // order as its total); slot of m = x0 + i is m + t
            double c = 0.0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                pe[x0 + t + i] = base + c;
                c += (double)z[j][i];
            }
            if (t == T - 1) pe[TL + T] = base + run[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int n = n0 - j;
            if (n < 0) break;
            const double *pe = Pe + (size_t)j * PS;
            const double rD = p.isq[n + 1];
            const double rM = p.rm[n];
            const bool inD = n <= p.N, inM = n >= 1;
#pragma unroll
            for (int k = 0; k < LO; ++k) {
                const int x = t + (ob + k) * T;
                const int hi = x + R + 1 < p.W ? x + R + 1 : p.W;
                const int lo = x - R > 0 ? x - R : 0;
                const double ub = x < p.W ? pe[hi + hi / L] - pe[lo + lo / L] : 0.0;
                const double tv = (double)tau[k];
                if (inD) bD[k] = fma(bD[k], tv * rD, ub);
                if (inM) bM[k] = fma(bM[k], tv * rM, ub);
            }
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int i = 0; i < L; ++i) z[j][i] = zn[j][i];
    }
    float *orow = p.out + (size_t)y * p.pitch;
#pragma unroll
    for (int k = 0; k < LO; ++k) {
        const int x = t + (ob + k) * T;
        if (x < p.W) orow[x] = (float)fma(p.sigma_r, bM[k] / bD[k], st.tc);
    }
}

}  // namespace bfgp
