// Stacked batch: B images of one size, filtered with one (sigma_s, sigma_r,
// N), every stage one launch over all images (blockIdx.z carries the image).
// For training loops over a batch of equal-size images: the forward with the
// saved terms and the backward run the same device functions as the
// single-image kernels, on image b's parameters, buffers and workspace slice,
// so every image's outputs equal those of a single call bit for bit.
//
// Per-image parameters: a setup kernel writes B copies of the image-0
// GPParams into the workspace with the image pointers (image, output, saved
// terms) and the workspace pointers (statistics, status) moved to image b;
// the stage kernels read image b's copy from there.  Other buffers (carries,
// stacks, gradients) are moved by b times a per-image stride in the kernels.
#include "launch.hpp"
#include "fir.hpp"
#include "iir.hpp"
#include "hrow.hpp"
#include "bwd.hpp"
#include "iir_bwd.hpp"

namespace bfgp {

namespace {

template <class T>
__device__ __forceinline__ T *shifted(T *q, size_t bytes) {
    return q ? (T *)((char *)q + bytes) : q;
}

__device__ __forceinline__ BwdParams bwd_for(const BwdParams &b0, const StkOfs &o, int b) {
    BwdParams r = b0;
    r.grad_out = shifted(b0.grad_out, sizeof(float) * o.img * b);
    r.saved = shifted(b0.saved, o.saved * b);
    r.grad_img = shifted(b0.grad_img, sizeof(float) * o.img * b);
    r.bparts = shifted(b0.bparts, o.ws * b);
    return r;
}

__device__ __forceinline__ BwdIir bwd_for(const BwdIir &b0, const StkOfs &o, int b) {
    BwdIir r = b0;
    r.grad_out = shifted(b0.grad_out, sizeof(float) * o.img * b);
    r.rho = shifted(b0.rho, o.saved * b);
    r.drho = shifted(b0.drho, o.saved * b);
    r.Dp = shifted(b0.Dp, o.saved * b);
    r.grad_img = shifted(b0.grad_img, sizeof(float) * o.img * b);
    r.cv = shifted(b0.cv, o.ws * b);
    r.PT = shifted(b0.PT, o.ws * b);
    r.QT = shifted(b0.QT, o.ws * b);
    r.chz = shifted(b0.chz, o.ws * b);
    r.bparts = shifted(b0.bparts, o.ws * b);
    return r;
}

}  // namespace

// One workgroup per image: the image-0 parameters copied word by word, then
// the pointers of image blockIdx.x moved.
__global__ __launch_bounds__(64) void ks_setup(GPParams p0, StkOfs o, GPParams *pd) {
    const int b = blockIdx.x;
    const int *src = (const int *)&p0;
    int *dst = (int *)(pd + b);
    for (int k = threadIdx.x; k < (int)(sizeof(GPParams) / sizeof(int)); k += 64) dst[k] = src[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        GPParams &p = pd[b];
        p.img = p0.img + o.img * b;
        p.out = p0.out ? p0.out + o.img * b : nullptr;
        p.parts = shifted(p0.parts, o.ws * b);
        p.status = shifted(p0.status, o.ws * b);
        p.stats = shifted(p0.stats, o.ws * b);
        p.saved = shifted(p0.saved, o.saved * b);
    }
}

__global__ __launch_bounds__(kBlock) void ks_stats(const GPParams *pd) {
    const GPParams &p = pd[blockIdx.z];
    stats_rows(p.img, p.H, p.W, p.pitch, blockIdx.x, gridDim.x, const_cast<Partial *>(p.parts));
}

__global__ __launch_bounds__(kBlock) void ks_stats_final(const GPParams *pd) { stats_final(pd[blockIdx.z]); }

template <int R, bool SAVE>
__global__ __launch_bounds__(kBlock) void ks_fir(const GPParams *pd, FirTaps taps) {
    extern __shared__ float smem[];
    const GPParams &p = pd[blockIdx.z];
    const Stats st = reduce_stats(p);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) publish_stats(p, st);
    fir_tile_auto<R, SAVE>(p, taps, st, blockIdx.y * fir_ty(R, SAVE), blockIdx.x * fir_tx(R, SAVE), smem);
}

// ---- recursive passes (the kernels of launch_iir, image blockIdx.z) -------------

template <int B, int G>
__global__ __launch_bounds__(256) void ks_vagg(const GPParams *pd, AggW aw, float *carry0, StkOfs o, int cgr) {
    __shared__ float sm[vagg_smem_floats(B, 4 / G)];
    const GPParams &p = pd[blockIdx.z];
    float *carry = shifted(carry0, o.ws * blockIdx.z);
    const Stats st = reduce_stats(p);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    if (!st.ok) return;
    const int nb = (p.H + B - 1) / B;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int pr = wave / G, gw = wave % G;
    const int pair = blockIdx.x * (4 / G) + pr;
    const bool live = pair < cgr * nb;
    const int cg = pair % cgr, band = pair / cgr;
    const int col = cg * 64 + (threadIdx.x & 63);
    float *pro = sm + pr * 2 * (B + 3) * 64;
    const bool big = st.xmax > 12.0;
    if (live) {
        if (big)
            vagg_prologue<B, true>(p, st, col, band, gw, G, pro);
        else
            vagg_prologue<B, false>(p, st, col, band, gw, G, pro);
    }
    __syncthreads();
    if (!live) return;
    if (big)
        vagg_moments<B, kAggG, true>(p, col, band, carry, gw, G, aw.w, pro);
    else
        vagg_moments<B, kAggG, false>(p, col, band, carry, gw, G, aw.w, pro);
}

template <int B, bool AGG>
__global__ __launch_bounds__(64, (B == 32 ? 3 : 2)) void ks_vband(const GPParams *pd, IirCoef c, float *carry0, float *S0, StkOfs o,
                                                  int sp, int groups, int cgr, int cgp) {
    __shared__ float sacc[AGG ? 1 : B * 64];
    const GPParams &p = pd[blockIdx.z];
    float *carry = shifted(carry0, o.ws * blockIdx.z), *S = shifted(S0, o.ws * blockIdx.z);
    Stats st;
    if (AGG) {
        st = reduce_stats(p);
        if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    } else {
        st = load_stats(p);
    }
    if (!st.ok) return;
    const int nb = (p.H + B - 1) / B;
    const int nreal = cgr * nb * groups;
    int idx = blockIdx.x, cg;
    if (idx < nreal) {
        cg = idx % cgr;
        idx /= cgr;
    } else {
        idx -= nreal;
        cg = cgr + idx % cgp;
        idx /= cgp;
    }
    const int band = idx % nb, grp = idx / nb;
    const int col = cg * 64 + threadIdx.x;
    const int cb = (p.C * grp) / groups, ce = (p.C * (grp + 1)) / groups;
    if (st.xmax > 12.0)
        vband<B, AGG, true>(p, c, st, col, band, carry, S, sp, sacc, cb, ce);
    else
        vband<B, AGG, false>(p, c, st, col, band, carry, S, sp, sacc, cb, ce);
}

template <int B, bool AGG>
__global__ __launch_bounds__(512, 3) void ks_vbandg(const GPParams *pd, IirCoef c, float *carry0, float *S0, StkOfs o,
                                                    int sp, int groups, int cgr, int cgp) {
    extern __shared__ float sm[];
    const GPParams &p = pd[blockIdx.z];
    float *carry = shifted(carry0, o.ws * blockIdx.z), *S = shifted(S0, o.ws * blockIdx.z);
    Stats st;
    if (AGG) {
        st = reduce_stats(p);
        if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    } else {
        st = load_stats(p);
    }
    if (!st.ok) return;
    const int nb = (p.H + B - 1) / B;
    int idx = blockIdx.x, cg;
    if (idx < cgr * nb) {
        cg = idx % cgr;
        idx /= cgr;
    } else {
        idx -= cgr * nb;
        cg = cgr + idx % cgp;
        idx /= cgp;
    }
    const int band = idx;
    const int grp = threadIdx.x >> 6;
    const int col = cg * 64 + (threadIdx.x & 63);
    const int cb = (p.C * grp) / groups, ce = (p.C * (grp + 1)) / groups;
    float *sacc = sm + grp * B * 64;
    float *pro = sm + (AGG ? 0 : groups * B * 64);
    if (st.xmax > 12.0)
        vband<B, AGG, true, false, false, true>(p, c, st, col, band, carry, S, sp, sacc, cb, ce, nullptr, 0, pro,
                                                 groups, grp);
    else
        vband<B, AGG, false, false, false, true>(p, c, st, col, band, carry, S, sp, sacc, cb, ce, nullptr, 0, pro,
                                                  groups, grp);
}

__global__ __launch_bounds__(64) void ks_vresolve(const GPParams *pd, IirCoef c, int nb, float *carry0, StkOfs o) {
    const int b = blockIdx.z >> 1;
    const GPParams &p = pd[b];
    const int col = blockIdx.x * 64 + threadIdx.x;
    if (col < p.W) vresolve(p, c, nb, col, blockIdx.y, blockIdx.z & 1, shifted(carry0, o.ws * b));
}

template <int L, bool SAVE>
__global__ __launch_bounds__(512) void ks_hrow2(const GPParams *pd, RowCoef c, const float *S0, StkOfs o, int srows,
                                                int sp, int T, int groups) {
    extern __shared__ float sm[];
    const GPParams &p = pd[blockIdx.z];
    const float *S = shifted(S0, o.ws * blockIdx.z);
    const Stats st = load_stats(p);
    if (!st.ok) {
        for (int x = threadIdx.x; x < p.W; x += blockDim.x) p.out[(size_t)blockIdx.x * p.pitch + x] = __builtin_nanf("");
        return;
    }
    hrow2<L, 0, SAVE>(p, c, st, blockIdx.x, S, srows, sp, sm, T, SAVE ? 1 : groups);
}

// ---- backward -------------------------------------------------------------------

template <int R>
__global__ __launch_bounds__(kBlock) void ks_bwd(const GPParams *pd, BwdParams b0, StkOfs o, FirTaps2 taps) {
    extern __shared__ float smem[];
    const GPParams &p = pd[blockIdx.z];
    const BwdParams b = bwd_for(b0, o, blockIdx.z);
    const Stats st = load_stats(p);
    bwd_tile<R>(p, b, taps, st, blockIdx.y * BwdShape<R>::TY, blockIdx.x * BwdShape<R>::TX,
                blockIdx.y * gridDim.x + blockIdx.x, smem);
}

// Per image: the partials summed in a fixed order (as k_bwd_finalize), the
// scalar gradients into g_lss[b], g_lsr[b] and the mean correction into
// corr[b].
__global__ __launch_bounds__(64) void ks_bwd_finalize(const GPParams *pd, const BwdPartial *bp0, StkOfs o, int ntiles,
                                                      double *corr, double *g_lss, double *g_lsr) {
    const int b = blockIdx.z;
    const GPParams &p = pd[b];
    const BwdPartial *bp = shifted(bp0, o.ws * b);
    double v[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < ntiles; i += 64) {
        v[0] += bp[i].sum_gh;
        v[1] += bp[i].sum_xgH;
        v[2] += bp[i].sum_grho;
        v[3] += bp[i].sum_zu;
        v[4] += bp[i].sum_g;
    }
    for (int q = 0; q < 5; ++q) v[q] = wave_sum(v[q]);
    if (threadIdx.x == 0) {
        const double n = (double)p.H * (double)p.W;
        corr[b] = p.center == 0 ? (v[4] - v[0]) / n : 0.0;
        if (g_lss) g_lss[b] = v[3];
        if (g_lsr) g_lsr[b] = v[2] - v[1];
    }
}

__global__ __launch_bounds__(kBlock) void ks_bwd_apply(float *grad0, int H, int W, int pitch, StkOfs o,
                                                       const double *corr) {
    const int b = blockIdx.z;
    float *grad = grad0 + o.img * b;
    const float c = (float)corr[b];
    for (int y = blockIdx.x; y < H; y += gridDim.x)
        for (int x = threadIdx.x; x < W; x += kBlock) grad[(size_t)y * pitch + x] += c;
}

template <bool AGG>
__global__ __launch_bounds__(64) void ks_bwd_vband(const GPParams *pd, BwdIir b0, StkOfs o, IirTan c) {
    __shared__ float tile[AGG ? 1 : 2 * kBwdBV * 65];
    const int b = blockIdx.z / b0.Gv, g = blockIdx.z % b0.Gv;
    const GPParams &p = pd[b];
    const BwdIir bb = bwd_for(b0, o, b);
    const Stats st = load_stats(p);
    bvband<kBwdBV, AGG>(p, bb, c, st, blockIdx.x * 64, blockIdx.y, (p.C * g) / bb.Gv, (p.C * (g + 1)) / bb.Gv, tile);
}

__global__ __launch_bounds__(64) void ks_bwd_resolve(const GPParams *pd, IirTan c, float *carry0, StkOfs o, int nb,
                                                     int lines, int stride, int horiz) {
    const int b = blockIdx.z >> 1;
    const GPParams &p = pd[b];
    const int line = blockIdx.x * 64 + threadIdx.x;
    if (line < lines)
        bresolve(horiz ? c.phiH : c.phiV, horiz ? c.psiH : c.psiV, nb, p.C, blockIdx.y, blockIdx.z & 1, (size_t)stride,
                 (size_t)line, shifted(carry0, o.ws * b));
}

__global__ __launch_bounds__(64) void ks_bwd_hband_agg(const GPParams *pd, BwdIir b0, StkOfs o, IirTan c) {
    const int b = blockIdx.z / b0.Gh, g = blockIdx.z % b0.Gh;
    const GPParams &p = pd[b];
    const BwdIir bb = bwd_for(b0, o, b);
    const Stats st = load_stats(p);
    bhband<kBwdBH, true>(p, bb, c, st, blockIdx.x * 64 + threadIdx.x, blockIdx.y, (p.C * g) / bb.Gh,
                         (p.C * (g + 1)) / bb.Gh, g, bb.Gh, nullptr, nullptr);
}

__global__ __launch_bounds__(256) void ks_bwd_hband(const GPParams *pd, BwdIir b0, StkOfs o, IirTan c) {
    extern __shared__ double red[];
    const int b = blockIdx.z;
    const GPParams &p = pd[b];
    const BwdIir bb = bwd_for(b0, o, b);
    const Stats st = load_stats(p);
    const int g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);
    bhband<kBwdBH, false>(p, bb, c, st, blockIdx.x * 64 + (threadIdx.x & 63), blockIdx.y, (p.C * g) / bb.Gh,
                          (p.C * (g + 1)) / bb.Gh, g, bb.Gh, bb.bparts + (size_t)blockIdx.y * gridDim.x + blockIdx.x,
                          red);
}

// ---- host launchers ---------------------------------------------------------------

hipError_t launch_stk_setup(const GPParams &p0, const StkOfs &o, GPParams *pd, hipStream_t s) {
    BF_LAUNCH("k_stk_setup", ks_setup, dim3(o.B), dim3(64), 0, s, p0, o, pd);
    return hipGetLastError();
}

hipError_t launch_stk_stats(const GPParams &p0, const GPParams *pd, const StkOfs &o, bool final_kernel,
                            hipStream_t s) {
    BF_LAUNCH("k_stats", ks_stats, dim3(p0.nparts, 1, o.B), dim3(kBlock), 0, s, pd);
    if (final_kernel) BF_LAUNCH("k_stats_final", ks_stats_final, dim3(1, 1, o.B), dim3(64), 0, s, pd);
    return hipGetLastError();
}

template <int R, bool SAVE>
static hipError_t stk_fir_rs(const GPParams &p0, const GPParams *pd, const StkOfs &o, const FirTaps &t, hipStream_t s) {
    dim3 grid((p0.W + fir_tx(R, SAVE) - 1) / fir_tx(R, SAVE), (p0.H + fir_ty(R, SAVE) - 1) / fir_ty(R, SAVE), o.B);
    BF_LAUNCH("k_fir", (ks_fir<R, SAVE>), grid, dim3(kBlock), sizeof(float) * fir_smem_floats(R, SAVE), s, pd, t);
    return hipGetLastError();
}

hipError_t launch_stk_fir(const GPParams &p0, const GPParams *pd, const StkOfs &o, const FirTaps &t, int R, bool save,
                          hipStream_t s) {
    switch (R) {
#define BF_CASE(r) \
    case r: return save ? stk_fir_rs<r, true>(p0, pd, o, t, s) : stk_fir_rs<r, false>(p0, pd, o, t, s);
        BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
        BF_CASE(9) BF_CASE(10) BF_CASE(11) BF_CASE(12) BF_CASE(13) BF_CASE(14) BF_CASE(15) BF_CASE(16)
        BF_CASE(17) BF_CASE(18) BF_CASE(19) BF_CASE(20) BF_CASE(21) BF_CASE(22) BF_CASE(23) BF_CASE(24)
#undef BF_CASE
        default: return hipErrorInvalidValue;
    }
}

// The stages of launch_iir (same choices: end states by weighted sums for
// bands of at most kAggMaxC channels, the grouped column passes for 32-row
// bands in 2..8 channel groups, the row pass of the saved terms or hrow2),
// image blockIdx.z.
hipError_t launch_stk_iir(const GPParams &p0, const GPParams *pd, const StkOfs &o, const IirCoef &c,
                          const RowCoef &rc, const IirShape &sh, float *carry, float *S, bool save, hipStream_t s) {
    const int nb = (p0.H + sh.B - 1) / sh.B;
    const int cgr = (p0.W + 63) / 64, cgp = (sh.P + 63) / 64 - cgr;
    const bool grouped = sh.B == 32 && sh.G >= 2 && sh.G <= 8;
    const unsigned B = (unsigned)o.B;
    if (sh.B != 32 && sh.B != 64) return hipErrorInvalidValue;
    if (sh.B == 64 && p0.C <= kAggMaxC) {
        BF_LAUNCH("k_vband_agg", (ks_vagg<64, 4>), dim3((unsigned)(cgr * nb), 1, B), dim3(256), 0, s, pd,
                  make_agg_w(c, 64), carry, o, cgr);
    } else if (sh.B == 64) {
        BF_LAUNCH("k_vband_agg", (ks_vband<64, true>), dim3(cgr * nb * sh.G, 1, B), dim3(64), 0, s, pd, c, carry, S, o,
                  sh.P, sh.G, cgr, cgp);
    } else if (p0.C <= kAggMaxC) {
        const int G = agg_groups(p0.H, p0.W, p0.C);
        const long bands = (long)cgr * nb;
        if (G == 2)
            BF_LAUNCH("k_vband_agg", (ks_vagg<32, 2>), dim3((unsigned)((bands + 1) / 2), 1, B), dim3(256), 0, s, pd,
                      make_agg_w(c, 32), carry, o, cgr);
        else
            BF_LAUNCH("k_vband_agg", (ks_vagg<32, 4>), dim3((unsigned)bands, 1, B), dim3(256), 0, s, pd,
                      make_agg_w(c, 32), carry, o, cgr);
    } else if (grouped) {
        static hipError_t attr = hipFuncSetAttribute((const void *)ks_vbandg<32, true>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(float) * (size_t)35 * 64 * 2));
        if (attr != hipSuccess) return attr;
        BF_LAUNCH("k_vband_agg", (ks_vbandg<32, true>), dim3(cgr * nb, 1, B), dim3(64 * sh.G),
                  sizeof(float) * (size_t)35 * 64 * 2, s, pd, c, carry, S, o, sh.P, sh.G, cgr, cgp);
    } else {
        BF_LAUNCH("k_vband_agg", (ks_vband<32, true>), dim3(cgr * nb * sh.G, 1, B), dim3(64), 0, s, pd, c, carry, S, o,
                  sh.P, sh.G, cgr, cgp);
    }
    BF_LAUNCH("k_vresolve", ks_vresolve, dim3(cgr, p0.C, 2 * B), dim3(64), 0, s, pd, c, nb, carry, o);
    if (grouped) {
        const size_t smb = sizeof(float) * ((size_t)sh.G * 32 * 64 + (size_t)35 * 64 * 2);
        static hipError_t attr = hipFuncSetAttribute((const void *)ks_vbandg<32, false>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)(sizeof(float) * ((size_t)8 * 32 * 64 + (size_t)35 * 64 * 2)));
        if (attr != hipSuccess) return attr;
        BF_LAUNCH("k_vband", (ks_vbandg<32, false>), dim3((cgr + cgp) * nb, 1, B), dim3(64 * sh.G), smb, s, pd, c,
                  carry, S, o, sh.P, sh.G, cgr, cgp);
    } else if (sh.B == 64) {
        BF_LAUNCH("k_vband", (ks_vband<64, false>), dim3((cgr + cgp) * nb * sh.G, 1, B), dim3(64), 0, s, pd, c, carry, S,
                  o, sh.P, sh.G, cgr, cgp);
    } else {
        BF_LAUNCH("k_vband", (ks_vband<32, false>), dim3((cgr + cgp) * nb * sh.G, 1, B), dim3(64), 0, s, pd, c, carry, S,
                  o, sh.P, sh.G, cgr, cgp);
    }
    {
        // the row pass and the recombination (the saved terms in one channel
        // group)
        const int gr = save ? 1 : sh.Gr;
        const size_t sm = hrow2_smem_bytes(sh.T, gr, sh.L);
        switch (sh.L) {
#define BF_CASE2(l, sv)                                                                                           \
    {                                                                                                             \
        if (sm > 65536) {                                                                                         \
            static hipError_t attr = hipFuncSetAttribute((const void *)ks_hrow2<l, sv>,                           \
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
            if (attr != hipSuccess) return attr;                                                                  \
        }                                                                                                         \
        BF_LAUNCH("k_hrow", (ks_hrow2<l, sv>), dim3(p0.H, 1, B), dim3(sh.T * gr), sm, s, pd, rc, (const float *)S, \
                  o, sh.Hs, sh.P, sh.T, gr);                                                                      \
    }
#define BF_CASE(l)                        \
    case l:                               \
        if (save) BF_CASE2(l, true)       \
        else BF_CASE2(l, false)           \
        break;
            BF_CASE(4) BF_CASE(8) BF_CASE(12) BF_CASE(16)
#undef BF_CASE
#undef BF_CASE2
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

template <int R>
static hipError_t stk_bwd_r(const GPParams &p0, const GPParams *pd, const BwdParams &b, const StkOfs &o,
                            const FirTaps2 &t, hipStream_t s) {
    using Sh = BwdShape<R>;
    dim3 grid((p0.W + Sh::TX - 1) / Sh::TX, (p0.H + Sh::TY - 1) / Sh::TY, o.B);
    BF_LAUNCH("k_bwd", (ks_bwd<R>), grid, dim3(kBlock), sizeof(float) * Sh::SMEM_FLOATS, s, pd, b, o, t);
    return hipGetLastError();
}

static hipError_t stk_finish(const GPParams &p0, const GPParams *pd, const BwdPartial *bparts, float *grad_img,
                             const StkOfs &o, int nparts, double *corr, double *g_lss, double *g_lsr, hipStream_t s) {
    BF_LAUNCH("k_bwd_finalize", ks_bwd_finalize, dim3(1, 1, o.B), dim3(64), 0, s, pd, bparts, o, nparts, corr, g_lss,
              g_lsr);
    if (grad_img && p0.center == 0) {
        const int g = p0.H < 1024 ? p0.H : 1024;
        BF_LAUNCH("k_bwd_apply", ks_bwd_apply, dim3(g, 1, o.B), dim3(kBlock), 0, s, grad_img, p0.H, p0.W, p0.pitch, o,
                  (const double *)corr);
    }
    return hipGetLastError();
}

hipError_t launch_stk_bwd(const GPParams &p0, const GPParams *pd, const BwdParams &b, const StkOfs &o,
                          const FirTaps2 &t, int R, double *corr, double *g_lss, double *g_lsr, hipStream_t s) {
    hipError_t e;
    switch (R) {
#define BF_CASE(r) case r: e = stk_bwd_r<r>(p0, pd, b, o, t, s); break;
        BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
        BF_CASE(9) BF_CASE(10) BF_CASE(11) BF_CASE(12) BF_CASE(13) BF_CASE(14) BF_CASE(15) BF_CASE(16)
        BF_CASE(17) BF_CASE(18) BF_CASE(19) BF_CASE(20) BF_CASE(21) BF_CASE(22) BF_CASE(23) BF_CASE(24)
#undef BF_CASE
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    return stk_finish(p0, pd, b.bparts, b.grad_img, o, bwd_tiles(p0.H, p0.W), corr, g_lss, g_lsr, s);
}

hipError_t launch_stk_bwd_iir(const GPParams &p0, const GPParams *pd, const BwdIir &b, const StkOfs &o,
                              const IirTan &c, double *corr, double *g_lss, double *g_lsr, hipStream_t s) {
    if (b.Gv < 1 || b.Gv > p0.C || b.Gh < 1 || b.Gh > 4 || b.Gh > p0.C) return hipErrorInvalidValue;
    const unsigned B = (unsigned)o.B;
    const int nbv = (p0.H + kBwdBV - 1) / kBwdBV, nbh = (p0.W + kBwdBH - 1) / kBwdBH;
    const dim3 gv((p0.W + 63) / 64, nbv, b.Gv * B);
    BF_LAUNCH("k_bwd_vband_agg", ks_bwd_vband<true>, gv, dim3(64), 0, s, pd, b, o, c);
    BF_LAUNCH("k_bwd_resolve", ks_bwd_resolve, dim3((p0.W + 63) / 64, p0.C, 2 * B), dim3(64), 0, s, pd, c, b.cv, o,
              nbv, p0.W, p0.W, 0);
    BF_LAUNCH("k_bwd_vband", ks_bwd_vband<false>, gv, dim3(64), 0, s, pd, b, o, c);
    BF_LAUNCH("k_bwd_hband_agg", ks_bwd_hband_agg, dim3(b.Hp / 64, nbh, b.Gh * B), dim3(64), 0, s, pd, b, o, c);
    BF_LAUNCH("k_bwd_resolve", ks_bwd_resolve, dim3((p0.H + 63) / 64, p0.C, 2 * B), dim3(64), 0, s, pd, c, b.chz, o,
              nbh, p0.H, b.Hp, 1);
    BF_LAUNCH("k_bwd_hband", ks_bwd_hband, dim3(b.Hp / 64, nbh, B), dim3(64 * b.Gh), bhband_smem_bytes(b.Gh, kBwdBH), s,
              pd, b, o, c);
    return stk_finish(p0, pd, b.bparts, b.grad_img, o, bwd_iir_parts(p0.H, p0.W), corr, g_lss, g_lsr, s);
}

}  // namespace bfgp
