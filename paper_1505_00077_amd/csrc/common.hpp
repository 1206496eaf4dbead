// Device-side building blocks shared by the GP kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfgp {

constexpr int kBlock = 256;          // threads per workgroup for every GP kernel
constexpr int kMaxN = 64;            // largest Gauss-polynomial degree
constexpr int kMaxC = kMaxN + 2;     // channels u_0..u_{N+1}
constexpr int kFirMaxR = 24;         // largest FIR radius compiled
constexpr int kMaxParts = 1024;      // partial sums of the statistics pass
constexpr int kDirectMaxW = 64;      // largest direct-filter window

// One workgroup's share of the image statistics.
struct Partial {
    double sum;
    float lo;
    float hi;
};

// Per-image statistics: the centre t_c of Algorithm 1's first step, plus the
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
    Stats *stats;        // written by stats_final
    void *saved;         // nullable, 16 B per pixel (see bf_gp_forward)
    double sq[kMaxC + 3];   // sqrt(n)
    double isq[kMaxC + 3];  // 1 / sqrt(n)
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
// The sum is accumulated in double, in a fixed order (deterministic).
__device__ __forceinline__ void stats_rows(const float *__restrict__ img, int H, int W, int pitch,
                                           int b, int G, Partial *__restrict__ parts) {
    __shared__ double s_sum[kBlock / 64];
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    double s = 0.0, s2 = 0.0;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int y = b; y < H; y += G) {
        const float *row = img + (size_t)y * pitch;
        int x0 = 0;
        if ((((size_t)row) & 15) == 0) {
            // four columns per load; two independent double accumulators
            const int W4 = W & ~3;
            for (int x = 4 * (int)threadIdx.x; x < W4; x += 4 * kBlock) {
                const float4 v = *(const float4 *)(row + x);
                s += (double)v.x + (double)v.y;
                s2 += (double)v.z + (double)v.w;
                lo = fminf(lo, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
                hi = fmaxf(hi, fmaxf(fmaxf(v.x, v.y), fmaxf(v.z, v.w)));
            }
            x0 = W4;
        }
        for (int x = x0 + threadIdx.x; x < W; x += kBlock) {
            const float v = row[x];
            s += (double)v;
            lo = fminf(lo, v);
            hi = fmaxf(hi, v);
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

// Reduces the partials in a fixed order (one workgroup), derives the centre and
// the range check, and stores them with the status word.
__device__ __forceinline__ void stats_final(const GPParams &p) {
    __shared__ double s_sum[kBlock / 64];
    __shared__ float s_lo[kBlock / 64], s_hi[kBlock / 64];
    double s = 0.0;
    float lo = __builtin_inff(), hi = -__builtin_inff();
    for (int i = threadIdx.x; i < p.nparts; i += kBlock) {
        s += p.parts[i].sum;
        lo = fminf(lo, p.parts[i].lo);
        hi = fmaxf(hi, p.parts[i].hi);
    }
    s = wave_sum(s);
    lo = wave_min(lo);
    hi = wave_max(hi);
    if ((threadIdx.x & 63) == 0) {
        s_sum[threadIdx.x >> 6] = s;
        s_lo[threadIdx.x >> 6] = lo;
        s_hi[threadIdx.x >> 6] = hi;
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
        double tc;
        if (p.center == 1)
            tc = 0.5 * ((double)l + (double)h);
        else if (p.center == 2)
            tc = 0.0;
        else
            tc = t / ((double)p.H * (double)p.W);
        const double a = fabs((double)l - tc) * p.inv_sigma_r;
        const double b = fabs((double)h - tc) * p.inv_sigma_r;
        Stats st;
        st.tc = tc;
        st.xmax = a > b ? a : b;
        st.ok = (st.xmax <= p.xlim) ? 1 : 0;
        st.pad = 0;
        *p.stats = st;
        *p.status = st.ok ? 0 : -3;
    }
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

// x = (f - t_c) / sigma_r, computed in double and rounded once to float.
__device__ __forceinline__ float centred(float f, const Stats &st, double inv_sr) {
    return (float)(((double)f - st.tc) * inv_sr);
}

}  // namespace bfgp
