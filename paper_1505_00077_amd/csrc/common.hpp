// Device-side building blocks shared by the GP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfgp {

constexpr int kBlock = 256;          // threads per workgroup for every GP kernel
constexpr int kMaxN = 64;            // largest Gauss-polynomial degree
constexpr int kMaxC = kMaxN + 2;     // channels u_0..u_{N+1}
constexpr int kFirMaxR = 24;         // largest FIR radius compiled
constexpr int kMaxParts = 256;       // partial sums of the statistics pass
constexpr int kDirectMaxW = 64;      // largest direct-filter window

// Workgroups are handed to the eight XCDs in turn (linear workgroup i runs on
// XCD i mod 8), and each XCD has its own L2.  xcd_block maps the linear index
// i of a grid of n workgroups to a tile index such that every XCD receives a
// contiguous run of tiles (XCD k the k-th eighth, in tile order): tiles that
// share halo samples then meet in one L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_block(int i, int n) {
    const int q = n >> 3, r = n & 7, x = i & 7, j = i >> 3;
    return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// One workgroup's share of the image statistics.
struct Partial {
    double sum;
    float lo;
    float hi;
};

// Per-image statistics: the centre t_c of Algorithm 1 (the mean), plus the
// extremes used for the FP32 range check.  Written once per call by the
// statistics pass, read by every later kernel.
struct Stats {
    double tc;
    double xmax;  // max |f - t_c| / sigma_r
    int ok;       // 1 when xmax is within the representable bound
    int pad;
};

// Coefficients for one image that every GP kernel needs.
struct GPParams {
    const float *img;
    float *out;
    int H, W, pitch;
    int N, C;            // degree and channel count C = N + 2
    int center;          // 0 mean, 1 midrange, 2 none
    double sigma_r, inv_sigma_r;
    double xlim;         // largest |x| whose channels stay in FP32 range
    const Partial *parts;
    int nparts;
    int *status;         // device status word (BF_OK / BF_ERANGE)
    Stats *stats;        // written by the first kernel after the statistics pass
    void *saved;         // nullable, 16 B per pixel (see bf_gp_forward)
    const float *data;   // joint filter: the image averaged (img is the guide); else null
    double sq[kMaxC + 3];   // sqrt(n)
    double isq[kMaxC + 3];  // 1 / sqrt(n)
    double rm[kMaxC + 3];   // sqrt(n + 1) / n (n >= 1; 0 at n = 0)
    double inv[kMaxC + 3];  // 1 / n (n >= 1; 0 at n = 0)
};

// Spatial taps of the FIR mode: k[d] = exp(-d^2 / 2 sigma_s^2), d = 0..R.
struct FirTaps {
    float k[kFirMaxR + 1];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// Statistics pass: workgroup b reduces rows b, b + G, ... into parts[b].
// The sum is accumulated in double, in a fixed order (deterministic).  Loads
// are issued eight at a time (four rows by two 4-column groups per thread,
// from clamped addresses, masked afterwards) so that enough are in flight.
__device__ __forceinline__ void stats_rows(const float *__restrict__ img, int H, int W, int pitch,
                                           int b, int G, Partial *__restrict__ parts) {
    __shared__ double s_sum[kBlock / 64];
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    double s = 0.0, s2 = 0.0;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    const int nr = (H - b + G - 1) / G;  // rows of this workgroup
    const bool vec = ((((size_t)img) & 15) == 0) && (pitch & 3) == 0;
    const int W4 = vec ? (W & ~3) : 0;
    const int nch = (W4 + 4 * kBlock - 1) / (4 * kBlock);  // 4-column groups per thread and row
    for (int r0 = 0; r0 < nr; r0 += 4) {
        for (int j0 = 0; j0 < nch; j0 += 2) {
            float4 v[8];
            bool ok[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int r = r0 + (k >> 1), x = 4 * ((int)threadIdx.x + (j0 + (k & 1)) * kBlock);
                ok[k] = r < nr && x < W4;
                const int y = b + (ok[k] ? r : 0) * G;
                v[k] = *(const float4 *)(img + (size_t)y * pitch + (ok[k] ? x : 0));
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (ok[k]) {
                    s += (double)v[k].x + (double)v[k].y;
                    s2 += (double)v[k].z + (double)v[k].w;
                    lo = fminf(lo, fminf(fminf(v[k].x, v[k].y), fminf(v[k].z, v[k].w)));
                    hi = fmaxf(hi, fmaxf(fmaxf(v[k].x, v[k].y), fmaxf(v[k].z, v[k].w)));
                }
            }
        }
    }
    // columns W4 .. W-1 (all of them when rows are not 16-byte aligned)
    const int tw = W - W4;
    for (int r = 0; r < nr; ++r) {
        const float *row = img + (size_t)(b + r * G) * pitch + W4;
        for (int x = threadIdx.x; x < tw; x += kBlock) {
            const float f = row[x];
            s += (double)f;
            lo = fminf(lo, f);
            hi = fmaxf(hi, f);
        }
    }
    s += s2;
    s = wave_sum(s);
    lo = wave_min(lo);
    hi = wave_max(hi);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_sum[w] = s;
        s_lo[w] = lo;
        s_hi[w] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        float l = __builtin_inff(), h = -__builtin_inff();
        for (int i = 0; i < kBlock / 64; ++i) {
            t += s_sum[i];
            l = fminf(l, s_lo[i]);
            h = fmaxf(h, s_hi[i]);
        }
        parts[b].sum = t;
        parts[b].lo = l;
        parts[b].hi = h;
    }
    __syncthreads();
}

// Reduces the partials of the statistics pass inside one wave, in a fixed
// order (the sum is the one lane 0 forms, so every wave that calls this gets
// the same bits), and derives the centre and the range check.  The first
// kernel after the statistics pass calls it in every wave instead of reading
// a result, which saves a launch; its first workgroup publishes the result.
__device__ __forceinline__ Stats reduce_stats(const GPParams &p) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    // all of a lane's partials (at most kMaxParts / 64) are loaded at once from
    // clamped indices, then summed in index order
    Partial q[kMaxParts / 64];
#pragma unroll
    for (int k = 0; k < kMaxParts / 64; ++k) {
        const int i = lane + 64 * k;
        q[k] = p.parts[i < p.nparts ? i : 0];
    }
#pragma unroll
    for (int k = 0; k < kMaxParts / 64; ++k) {
        if (lane + 64 * k < p.nparts) {
            s += q[k].sum;
            lo = fminf(lo, q[k].lo);
            hi = fmaxf(hi, q[k].hi);
        }
    }
    s = __shfl(wave_sum(s), 0, 64);
    lo = wave_min(lo);
    hi = wave_max(hi);
    double tc;
    if (p.center == 1)
        tc = 0.5 * ((double)lo + (double)hi);
    else if (p.center == 2)
        tc = 0.0;
    else
        tc = s / ((double)p.H * (double)p.W);
    const double a = fabs((double)lo - tc) * p.inv_sigma_r;
    const double b = fabs((double)hi - tc) * p.inv_sigma_r;
    Stats st;
    st.tc = tc;
    st.xmax = a > b ? a : b;
    st.ok = (st.xmax <= p.xlim) ? 1 : 0;
    st.pad = 0;
    return st;
}

// Stores the statistics and the status word for the kernels and calls that
// follow (one thread).
__device__ __forceinline__ void publish_stats(const GPParams &p, const Stats &st) {
    *p.stats = st;
    *p.status = st.ok ? 0 : -3;
}

// Statistics of an image as a kernel of its own (one wave publishes).
__device__ __forceinline__ void stats_final(const GPParams &p) {
    if (threadIdx.x >= 64) return;
    const Stats st = reduce_stats(p);
    if (threadIdx.x == 0) publish_stats(p, st);
}

// The statistics of the image (written earlier in the same stream).
__device__ __forceinline__ Stats load_stats(const GPParams &p) { return *p.stats; }

// exp(-x^2/2) * 2^shift as float, to about one ulp: the base-2 exponent is
// formed in double and split into an integer part (applied by ldexp) and a
// fraction in [-1/2, 1/2] (exp2 in float).  Much cheaper than a double exp.
__device__ __forceinline__ float gauss_u0(float x, int shift) {
    const double a = fma(-0.72134752044448170, (double)x * (double)x, (double)shift);  // log2(e)/2
    const double ah = rint(a);
    return ldexpf(exp2f((float)(a - ah)), (int)ah);
}

// Scale exponent used when exp(-x^2/2) would leave the FP32 range (|x| > 12):
// the channel is carried as uh = u * 2^s (u_0 = gauss_u0(x, s) stays near
// 2^-60) and u is recovered as uh * 2^-s.
__device__ __forceinline__ int big_shift(float x) {
    const float t = x * x;
    return t > 144.f ? (int)(t * 0.72134752f) - 60 : 0;
}

// x = (f - t_c) / sigma_r, computed in double and rounded once to float.
__device__ __forceinline__ float centred(float f, const Stats &st, double inv_sr) {
    return (float)(((double)f - st.tc) * inv_sr);
}

}  // namespace bfgp
