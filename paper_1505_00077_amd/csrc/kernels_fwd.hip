// __global__ entry points of the single-image forward path (statistics, fused
// FIR, recursive IIR passes, direct filter) and their host-side launchers.
#include "launch.hpp"
#include "fir.hpp"
#include "iir.hpp"
#include "hrow.hpp"
#include "direct.hpp"
#include "box.hpp"

namespace bfgp {

__global__ __launch_bounds__(kBlock) void k_stats(const float *img, int H, int W, int pitch, Partial *parts) {
    stats_rows(img, H, W, pitch, blockIdx.x, gridDim.x, parts);
}

__global__ __launch_bounds__(kBlock) void k_stats_final(GPParams p) { stats_final(p); }

template <int R, bool SAVE>
__global__ __launch_bounds__(kBlock) void k_fir(GPParams p, FirTaps taps) {
    extern __shared__ float smem[];
    const Stats st = reduce_stats(p);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) publish_stats(p, st);
    const int t = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int tx = t % gridDim.x, ty = t / gridDim.x;
    fir_tile_auto<R, SAVE>(p, taps, st, ty * fir_ty(R, SAVE), tx * fir_tx(R, SAVE), smem);
}

__global__ __launch_bounds__(kBlock) void k_direct(DirectArgs a) {
    extern __shared__ float smem[];
    direct_tile(a, blockIdx.y * kDirTY, blockIdx.x * kDirTX, smem);
}


// ---- recursive (IIR) passes ----------------------------------------------------

// One kernel per pass covers both channel representations: images whose
// range needs the per-sample shift (xmax > 12) take the BIG branch, which is
// uniform over the launch.  The launch bound keeps the common branch at three
// waves per SIMD (the rare BIG branch may spill).  The end-state pass is the
// first kernel after the statistics pass: it reduces the partials itself.
// One-dimensional grid: the workgroups of the image's column groups (cgr of
// them per band and channel group) come first, those of the stack's pad-only
// column groups (cgp, column pass only: they store zeros) last, so that the
// light pad workgroups fill in behind the full ones.
template <int B, bool AGG, bool JOINT>
__global__ __launch_bounds__(64, (B == 32 ? 3 : 2)) void k_vband(GPParams p, IirCoef c, float *carry, float *S, int sp, int groups,
                                                 int cgr, int cgp) {
    __shared__ float sacc[AGG ? 1 : B * 64];
    Stats st;
    if (AGG) {
        st = reduce_stats(p);
        if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && threadIdx.x == 0) publish_stats(p, st);
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
    // channel group grp of `groups` nearly equal groups
    const int cb = (p.C * grp) / groups, ce = (p.C * (grp + 1)) / groups;
    if (st.xmax > 12.0)
        vband<B, AGG, true, JOINT>(p, c, st, col, band, carry, S, sp, sacc, cb, ce);
    else
        vband<B, AGG, false, JOINT>(p, c, st, col, band, carry, S, sp, sacc, cb, ce);
}

// The same passes with all `groups` (>= 2) channel groups of a band in one
// workgroup, one wave per group: the band's centred intensities and
// exp(-x^2/2) are computed once for the workgroup and shared through LDS
// (dynamic: groups * B * 64 floats of staging for the column pass, then
// (B + 3) * 64 * (JOINT ? 3 : 2) floats).  Grid: the image's column groups per
// band first, then the pad-only ones (column pass).
template <int B, bool AGG, bool JOINT>
__global__ __launch_bounds__(512, 3) void k_vbandg(GPParams p, IirCoef c, float *carry, float *S, int sp, int groups,
                                                   int cgr, int cgp) {
    extern __shared__ float sm[];
    Stats st;
    if (AGG) {
        st = reduce_stats(p);
        if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    } else {
        st = load_stats(p);
    }
    if (!st.ok) return;  // uniform over the launch
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
        vband<B, AGG, true, JOINT, false, true>(p, c, st, col, band, carry, S, sp, sacc, cb, ce, nullptr, 0, pro,
                                                 groups, grp);
    else
        vband<B, AGG, false, JOINT, false, true>(p, c, st, col, band, carry, S, sp, sacc, cb, ce, nullptr, 0, pro,
                                                  groups, grp);
}

// Band end states by weighted sums (vagg_moments): G NBW waves per
// workgroup, NBW bands (64-column group and band of B rows), the G waves of
// a band taking the channels g, g + G, ... (g = 0..G-1) and sharing its prologue
// through LDS; the
// workgroup computes the weight table in LDS.  Images whose range needs the
// per-sample shift (xmax > 12) take the BIG branch, uniform over the launch.
// The first kernel after the statistics pass: it reduces the partials itself.
template <int B, int G, int NBW = 4 / G>
__global__ __launch_bounds__(64 * G * NBW) void k_vagg(GPParams p, AggW aw, float *carry, int cgr) {
    __shared__ float sm[vagg_smem_floats(B, NBW)];
    const Stats st = reduce_stats(p);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    if (!st.ok) return;  // uniform over the launch
    const int nb = (p.H + B - 1) / B;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int pr = wave / G, gw = wave % G;
    const int pair = blockIdx.x * NBW + pr;
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

__global__ __launch_bounds__(64) void k_vresolve(GPParams p, IirCoef c, int nb, float *carry) {
    const int col = blockIdx.x * 64 + threadIdx.x;
    if (col < p.W) vresolve(p, c, nb, col, blockIdx.y, blockIdx.z, carry);
}

template <int L, bool JOINT>
__global__ __launch_bounds__(512, 1) void k_hrow(GPParams p, IirCoef c, const float *S, int srows, int sp, int T,
                                                 int groups) {
    extern __shared__ float sm[];
    const Stats st = load_stats(p);
    if (!st.ok) {
        for (int x = threadIdx.x; x < p.W; x += blockDim.x) p.out[(size_t)blockIdx.x * p.pitch + x] = __builtin_nanf("");
        return;
    }
    hrow<L, JOINT>(p, c, st, blockIdx.x, S, srows, sp, sm, T, groups);
}

// Row pass + recombination of one image row (hrow2): T threads per channel
// group, `groups` groups, T * groups <= 512 (SAVE: one group, the saved
// terms stored too).
template <int L, bool SAVE = false>
__global__ __launch_bounds__(512) void k_hrow2(GPParams p, RowCoef c, const float *S, int srows, int sp, int T,
                                               int groups) {
    extern __shared__ float sm[];
    const Stats st = load_stats(p);
    if (!st.ok) {
        for (int x = threadIdx.x; x < p.W; x += blockDim.x) p.out[(size_t)blockIdx.x * p.pitch + x] = __builtin_nanf("");
        return;
    }
    hrow2<L, 0, SAVE>(p, c, st, blockIdx.x, S, srows, sp, sm, T, SAVE ? 1 : groups);
}

// Row pass of rows wider than one workgroup: segment blockIdx.y of row
// blockIdx.x (512 threads, 16 samples each); MODE 1 stores the segments' end
// states, MODE 2 filters the segments with them.
template <int MODE>
__global__ __launch_bounds__(512) void k_hrow2seg(GPParams p, RowCoef c, const float *S, int srows, int sp,
                                                  float *segst) {
    extern __shared__ float sm[];
    const Stats st = load_stats(p);
    if (!st.ok) {
        if (MODE == 2)
            for (int x = blockIdx.y * kRowSeg + threadIdx.x; x < p.W && x < (blockIdx.y + 1) * kRowSeg; x += blockDim.x)
                p.out[(size_t)blockIdx.x * p.pitch + x] = __builtin_nanf("");
        return;
    }
    hrow2<kRowMaxL, MODE>(p, c, st, blockIdx.x, S, srows, sp, sm, 512, 1, 0, blockIdx.y, gridDim.y, segst);
}

// ---- volumes: the row-direction pass per frame and the frame-wise row pass ----

// Column pass of every frame over the time-filtered stack S1 (channel n, frame
// t at S1 + n * s1_cstride + t * H * W, rows of W): grid x as k_vband, y the
// frame.  The statistics were published by the time pass.
template <int B, bool AGG>
__global__ __launch_bounds__(64, 3) void k_vband3(GPParams p, IirCoef c, float *carry, float *S, int sp, int groups,
                                                  int cgr, int cgp, const float *S1, size_t s1_cstride,
                                                  size_t carry_fstride, size_t s_fstride) {
    __shared__ float sacc[AGG ? 1 : B * 64];
    const Stats st = load_stats(p);
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
    const size_t t = blockIdx.y;
    vband<B, AGG, false, false, true>(p, c, st, col, band, carry + t * carry_fstride, S + t * s_fstride, sp, sacc, cb,
                                      ce, S1 + t * (size_t)p.H * p.W, s1_cstride);
}

__global__ __launch_bounds__(64) void k_vresolve3(GPParams p, IirCoef c, int nb, float *carry, size_t carry_fstride) {
    const int col = blockIdx.x * 64 + threadIdx.x;
    const size_t t = blockIdx.z >> 1;
    if (col < p.W) vresolve(p, c, nb, col, blockIdx.y, blockIdx.z & 1, carry + t * carry_fstride);
}

// Row pass of frame blockIdx.x / H, row blockIdx.x % H.
template <int L>
__global__ __launch_bounds__(512) void k_hrow3(GPParams p, RowCoef c, const float *S, int srows, int sp, int T,
                                               int groups, size_t s_fstride) {
    extern __shared__ float sm[];
    const Stats st = load_stats(p);
    const size_t t = blockIdx.x / p.H;
    const int y = blockIdx.x % p.H;
    const size_t foff = t * (size_t)p.H * p.pitch;
    if (!st.ok) {
        for (int x = threadIdx.x; x < p.W; x += blockDim.x) p.out[foff + (size_t)y * p.pitch + x] = __builtin_nanf("");
        return;
    }
    hrow2<L>(p, c, st, y, S + t * s_fstride, srows, sp, sm, T, groups, foff);
}

// ---- box spatial kernel ----------------------------------------------------------

// Column pass: one 64-column wave per band and channel group (workgroups of
// the same band and group are adjacent).  The first kernel after the
// statistics pass: it reduces the partials itself.
template <int NC>
__global__ __launch_bounds__(64) void k_boxcol(GPParams p, BoxFact bfct, float *S, int R, int Bb, int nb, int G,
                                               int cgr, int P) {
    const Stats st = reduce_stats(p);
    if (blockIdx.x == 0 && threadIdx.x == 0) publish_stats(p, st);
    if (!st.ok) return;
    int idx = blockIdx.x;
    const int cg = idx % cgr;
    idx /= cgr;
    const int band = idx % nb, grp = idx / nb;
    const int col = cg * 64 + threadIdx.x;
    if (col >= p.W) return;
    const int cb = (p.C * grp) / G, ce = (p.C * (grp + 1)) / G;
    const int y0 = band * Bb, y1 = y0 + Bb < p.H ? y0 + Bb : p.H;
    boxcol<NC>(p, bfct, st, R, col, y0, y1, cb, ce - cb, S, P);
}

// Row pass + recombination: one workgroup of T threads per image row, K
// channels per step; LO < L: blockIdx.y selects the row's LO-th part of the
// outputs.
template <int L, int K, int LO = L>
__global__ __launch_bounds__(L == 4 ? 1024 : 512) void k_boxrow(GPParams p, const float *S, int R, int P, int T) {
    extern __shared__ float sm[];
    const Stats st = load_stats(p);
    if (!st.ok) {
        if (blockIdx.y == 0)
            for (int x = threadIdx.x; x < p.W; x += blockDim.x) p.out[(size_t)blockIdx.x * p.pitch + x] = __builtin_nanf("");
        return;
    }
    boxrow<L, K, LO>(p, st, R, blockIdx.x, S, P, T, (double *)sm, blockIdx.y * LO);
}

// ---- host launchers ----------------------------------------------------------

hipError_t launch_stats(const GPParams &p, bool final_kernel, hipStream_t s) {
    BF_LAUNCH("k_stats", k_stats, dim3(p.nparts), dim3(kBlock), 0, s, p.img, p.H, p.W, p.pitch,
              const_cast<Partial *>(p.parts));
    if (final_kernel) BF_LAUNCH("k_stats_final", k_stats_final, dim3(1), dim3(64), 0, s, p);
    return hipGetLastError();
}

template <int R, bool SAVE>
static hipError_t fir_launch_rs(const GPParams &p, const FirTaps &t, hipStream_t s) {
    dim3 grid((p.W + fir_tx(R, SAVE) - 1) / fir_tx(R, SAVE), (p.H + fir_ty(R, SAVE) - 1) / fir_ty(R, SAVE));
    BF_LAUNCH("k_fir", (k_fir<R, SAVE>), grid, dim3(kBlock), sizeof(float) * fir_smem_floats(R, SAVE), s, p, t);
    return hipGetLastError();
}

template <int R>
static hipError_t fir_launch_r(const GPParams &p, const FirTaps &t, bool save, hipStream_t s) {
    return save ? fir_launch_rs<R, true>(p, t, s) : fir_launch_rs<R, false>(p, t, s);
}

hipError_t launch_fir(const GPParams &p, const FirTaps &t, int R, bool save, hipStream_t s) {
    switch (R) {
#define BF_CASE(r) case r: return fir_launch_r<r>(p, t, save, s);
        BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
        BF_CASE(9) BF_CASE(10) BF_CASE(11) BF_CASE(12) BF_CASE(13) BF_CASE(14) BF_CASE(15) BF_CASE(16)
        BF_CASE(17) BF_CASE(18) BF_CASE(19) BF_CASE(20) BF_CASE(21) BF_CASE(22) BF_CASE(23) BF_CASE(24)
#undef BF_CASE
        default: return hipErrorInvalidValue;
    }
}


// The row pass that recombines the joint filter (chunks of sh.Lo samples, one
// channel group).
template <int L>
static void hrow_launch_joint(const GPParams &p, const IirCoef &c, const IirShape &sh, const float *S, hipStream_t s) {
    const dim3 rb(sh.To);
    const size_t sm = hrow_smem_bytes(sh.To, 1, sh.Lo);
    BF_LAUNCH("k_hrow", (k_hrow<L, true>), dim3(p.H), rb, sm, s, p, c, S, sh.Hs, sh.P, sh.To, 1);
}

// The row pass of the plain forward (chunks of sh.L samples); with the saved
// terms in one channel group.
template <int L, bool SAVE>
static hipError_t hrow2_launch_s(const GPParams &p, const RowCoef &c, const IirShape &sh, const float *S,
                                 hipStream_t s) {
    const int gr = SAVE ? 1 : sh.Gr;
    const size_t sm = hrow2_smem_bytes(sh.T, gr, sh.L);
    if (sm > 65536) {
        static hipError_t attr = hipFuncSetAttribute((const void *)k_hrow2<L, SAVE>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (attr != hipSuccess) return attr;
    }
    BF_LAUNCH("k_hrow", (k_hrow2<L, SAVE>), dim3(p.H), dim3(sh.T * gr), sm, s, p, c, S, sh.Hs, sh.P, sh.T, gr);
    return hipSuccess;
}
template <int L>
static hipError_t hrow2_launch(const GPParams &p, const RowCoef &c, const IirShape &sh, const float *S, bool save,
                               hipStream_t s) {
    return save ? hrow2_launch_s<L, true>(p, c, sh, S, s) : hrow2_launch_s<L, false>(p, c, sh, S, s);
}

#define BF_ROW2_SWITCH(Lv, CALL)                                                         \
    switch (Lv) {                                                                        \
        case 4: CALL(4); break;                                                          \
        case 8: CALL(8); break;                                                          \
        case 12: CALL(12); break;                                                        \
        case 16: CALL(16); break;                                                        \
        default: return hipErrorInvalidValue;                                            \
    }

template <int B, bool AGG>
static void vband_launch(const GPParams &p, const IirCoef &c, const IirShape &sh, dim3 grid, float *carry, float *S,
                         int cgr, int cgp, bool joint, hipStream_t s) {
    const char *name = AGG ? "k_vband_agg" : "k_vband";
    if (joint)
        BF_LAUNCH(name, (k_vband<B, AGG, true>), grid, dim3(64), 0, s, p, c, carry, S, sh.P, sh.G, cgr, cgp);
    else
        BF_LAUNCH(name, (k_vband<B, AGG, false>), grid, dim3(64), 0, s, p, c, carry, S, sh.P, sh.G, cgr, cgp);
}

// Dynamic LDS of k_vbandg.
constexpr size_t vbandg_smem_bytes(int B, bool agg, bool joint, int groups) {
    return sizeof(float) * ((agg ? 0 : (size_t)groups * B * 64) + (size_t)(B + 3) * 64 * (joint ? 3 : 2));
}

// The grouped passes (32-row bands, 2..8 channel groups): grid = the column
// groups of every band, `groups` waves per workgroup.
template <bool AGG>
static hipError_t vbandg_launch(const GPParams &p, const IirCoef &c, const IirShape &sh, float *carry, float *S, int cgr,
                                int cgp, hipStream_t s) {
    // more than 64 KiB of LDS for 7..8 groups in the column pass: the
    // attribute is set once, to the largest size
    static hipError_t attr = hipFuncSetAttribute((const void *)k_vbandg<32, AGG, false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)vbandg_smem_bytes(32, AGG, false, 8));
    if (attr != hipSuccess) return attr;
    const int nb = (p.H + 31) / 32;
    const dim3 grid((AGG ? cgr : cgr + cgp) * nb);
    const char *name = AGG ? "k_vband_agg" : "k_vband";
    BF_LAUNCH(name, (k_vbandg<32, AGG, false>), grid, dim3(64 * sh.G), vbandg_smem_bytes(32, AGG, false, sh.G), s, p,
              c, carry, S, sh.P, sh.G, cgr, cgp);
    return hipSuccess;
}

hipError_t launch_iir(const GPParams &p, const IirCoef &c, const RowCoef &rc, const IirShape &shape, float *carry,
                      float *S, bool save, bool joint, hipStream_t s, float *segst) {
    IirShape sh = shape;
    const int nb = (p.H + sh.B - 1) / sh.B;
    // the end-state pass has nothing to do on the stack's pad columns: its
    // grid covers the image columns only (an even number of waves per SIMD
    // where the column pass has one extra, nearly empty, column group)
    const int cgr = (p.W + 63) / 64, cgp = (sh.P + 63) / 64 - cgr;
    const dim3 ga(cgr * nb * sh.G), gv((cgr + cgp) * nb * sh.G);
    // bands of 32 rows split into 2..8 channel groups share each band's
    // prologue inside one workgroup (not the joint filter: its grouped
    // passes spill registers and measured slower)
    const bool grouped = !joint && sh.B == 32 && sh.G >= 2 && sh.G <= 8;
    hipError_t e = hipSuccess;
    if (!joint && sh.B == 64 && p.C <= kAggMaxC) {
        // 64-row bands (large images): four channel groups per band, one
        // band per workgroup (two groups in a workgroup of two waves measured
        // 2.5 % slower at 4096^2: half the waves per CU for the same LDS)
        const long bands = (long)cgr * nb;
        BF_LAUNCH("k_vband_agg", (k_vagg<64, 4>), dim3((unsigned)bands), dim3(256), 0, s, p, make_agg_w(c, 64), carry,
                  cgr);
    } else if (!joint && sh.B == 32 && p.C <= kAggMaxC) {
        // end states by weighted sums, 2 or 4 channel groups per band
        const int G = agg_groups(p.H, p.W, p.C);
        const long bands = (long)cgr * nb;
        if (G == 2)
            BF_LAUNCH("k_vband_agg", (k_vagg<32, 2>), dim3((unsigned)((bands + 1) / 2)), dim3(256), 0, s, p,
                      make_agg_w(c, 32), carry, cgr);
        else
            BF_LAUNCH("k_vband_agg", (k_vagg<32, 4>), dim3((unsigned)bands), dim3(256), 0, s, p, make_agg_w(c, 32),
                      carry, cgr);
    } else if (grouped)
        e = vbandg_launch<true>(p, c, sh, carry, S, cgr, cgp, s);
    else if (sh.B == 64)
        vband_launch<64, true>(p, c, sh, ga, carry, S, cgr, cgp, joint, s);
    else if (sh.B == 32)
        vband_launch<32, true>(p, c, sh, ga, carry, S, cgr, cgp, joint, s);
    else
        return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    BF_LAUNCH("k_vresolve", k_vresolve, dim3((p.W + 63) / 64, p.C, 2), dim3(64), 0, s, p, c, nb, carry);
    if (grouped)
        e = vbandg_launch<false>(p, c, sh, carry, S, cgr, cgp, s);
    else if (sh.B == 64)
        vband_launch<64, false>(p, c, sh, gv, carry, S, cgr, cgp, joint, s);
    else
        vband_launch<32, false>(p, c, sh, gv, carry, S, cgr, cgp, joint, s);
    if (e != hipSuccess) return e;
    if (joint) {
        // the joint recombination: the row pass with the whole Horner sums of
        // the channel pairs in one group
        switch (sh.Lo) {
            case 4: hrow_launch_joint<4>(p, c, sh, S, s); break;
            case 8: hrow_launch_joint<8>(p, c, sh, S, s); break;
            case 12: hrow_launch_joint<12>(p, c, sh, S, s); break;
            case 16: hrow_launch_joint<16>(p, c, sh, S, s); break;
            default: return hipErrorInvalidValue;
        }
    } else if (sh.nseg > 1) {
        if (save) return hipErrorInvalidValue;  // the saved terms stop at 8192 columns
        if (sh.T != 512 || sh.L != kRowMaxL || !segst) return hipErrorInvalidValue;
        const size_t sm = hrow2_smem_bytes(512, 1, kRowMaxL);
        static hipError_t attr = [] {
            hipError_t a = hipFuncSetAttribute((const void *)k_hrow2seg<1>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
            if (a == hipSuccess)
                a = hipFuncSetAttribute((const void *)k_hrow2seg<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        160 * 1024);
            return a;
        }();
        if (attr != hipSuccess) return attr;
        const dim3 grid(p.H, sh.nseg);
        BF_LAUNCH("k_hrow_seg", k_hrow2seg<1>, grid, dim3(512), sm, s, p, rc, S, sh.Hs, sh.P, segst);
        BF_LAUNCH("k_hrow", k_hrow2seg<2>, grid, dim3(512), sm, s, p, rc, S, sh.Hs, sh.P, segst);
    } else {
#define BF_CALL(l) e = hrow2_launch<l>(p, rc, sh, S, save, s)
        BF_ROW2_SWITCH(sh.L, BF_CALL)
#undef BF_CALL
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

hipError_t launch_direct(const DirectArgs &a, hipStream_t s) {
    dim3 grid((a.W + kDirTX - 1) / kDirTX, (a.H + kDirTY - 1) / kDirTY);
    BF_LAUNCH("k_direct", k_direct, grid, dim3(kBlock), sizeof(float) * direct_smem_floats(), s, a);
    return hipGetLastError();
}

hipError_t launch_volume(const GPParams &pz, const GPParams &ps, const IirCoef &ct, const IirCoef &cs,
                         const RowCoef &rcs, const IirShape &shz, const IirShape &shs, int T, const VolumeBuffers &vb,
                         hipStream_t s) {
    // 1. statistics of the volume seen as a (T H) x W image (ps)
    hipError_t e = launch_stats(ps, false, s);
    if (e != hipSuccess) return e;
    // 2. time direction: the column passes over the volume seen as a T x (H W)
    // image (pz); its stack S1 has rows of H W and no pad
    const int nbz = (pz.H + shz.B - 1) / shz.B;
    const int cgz = (pz.W + 63) / 64;
    const dim3 gz(cgz * nbz * shz.G);
    if (shz.B != 32) return hipErrorInvalidValue;
    BF_LAUNCH("k_vband_agg", (k_vband<32, true, false>), gz, dim3(64), 0, s, pz, ct, vb.carry_z, vb.S1, pz.W, shz.G,
              cgz, 0);
    BF_LAUNCH("k_vresolve", k_vresolve, dim3(cgz, pz.C, 2), dim3(64), 0, s, pz, ct, nbz, vb.carry_z);
    BF_LAUNCH("k_vband", (k_vband<32, false, false>), gz, dim3(64), 0, s, pz, ct, vb.carry_z, vb.S1, pz.W, shz.G,
              cgz, 0);
    // 3. column direction in every frame, from S1 into the row-pass stack S2
    GPParams py = ps;
    py.H = ps.H / T;
    const int nby = (py.H + shs.B - 1) / shs.B;
    const int cgr = (py.W + 63) / 64, cgp = (shs.P + 63) / 64 - cgr;
    const size_t s1_cstride = (size_t)((pz.H + shz.B - 1) / shz.B) * shz.B * (size_t)pz.W;
    const size_t carry_fstride = (size_t)nby * py.C * 8 * py.W;
    const size_t s_fstride = (size_t)py.C * vb.Hs * shs.P;
    if (shs.B != 32) return hipErrorInvalidValue;
    BF_LAUNCH("k_vband_agg", (k_vband3<32, true>), dim3(cgr * nby * shs.G, T), dim3(64), 0, s, py, cs, vb.carry_y,
              vb.S2, shs.P, shs.G, cgr, cgp, (const float *)vb.S1, s1_cstride, carry_fstride, s_fstride);
    BF_LAUNCH("k_vresolve", k_vresolve3, dim3(cgr, py.C, 2 * T), dim3(64), 0, s, py, cs, nby, vb.carry_y,
              carry_fstride);
    BF_LAUNCH("k_vband", (k_vband3<32, false>), dim3((cgr + cgp) * nby * shs.G, T), dim3(64), 0, s, py, cs,
              vb.carry_y, vb.S2, shs.P, shs.G, cgr, cgp, (const float *)vb.S1, s1_cstride, carry_fstride, s_fstride);
    // 4. row direction and the recombination, frame by frame
    const dim3 rb(shs.T * shs.Gr);
    const size_t sm = hrow2_smem_bytes(shs.T, shs.Gr, shs.L);
    const dim3 gr((unsigned)(T * py.H));
#define BF_CALL(l)                                                                                               \
    {                                                                                                            \
        if (sm > 65536) {                                                                                        \
            static hipError_t attr = hipFuncSetAttribute((const void *)k_hrow3<l>,                               \
                                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024); \
            if (attr != hipSuccess) return attr;                                                                 \
        }                                                                                                        \
        BF_LAUNCH("k_hrow", (k_hrow3<l>), gr, rb, sm, s, py, rcs, (const float *)vb.S2, vb.Hs, shs.P, shs.T,      \
                  shs.Gr, s_fstride);                                                                            \
    }
    BF_ROW2_SWITCH(shs.L, BF_CALL)
#undef BF_CALL
    return hipGetLastError();
}

hipError_t launch_box(const GPParams &p, const BoxShape &sh, float *S, hipStream_t s) {
    const int cgr = (p.W + 63) / 64;
    if ((long)cgr * sh.nb * sh.G > 0x7fffffffL || sh.T > (sh.L == 4 ? 1024 : 512) || sh.T % 64 ||
        (long)sh.T * sh.L < p.W || sh.P != sh.T * sh.L)
        return hipErrorInvalidValue;
    BoxFact bfct;
    double v = 1.0;
    for (int n = 0; n < kMaxC; ++n) {
        if (n > 0) v *= p.isq[n];
        bfct.ifs[n] = v;
    }
    const dim3 cgrid(cgr * sh.nb * sh.G);
    switch (sh.NC) {
#define BF_CASE(nc)                                                                                            \
    case nc:                                                                                                   \
        BF_LAUNCH("k_boxcol", k_boxcol<nc>, cgrid, dim3(64), 0, s, p, bfct, S, sh.R, sh.Bb, sh.nb, sh.G, cgr, sh.P); \
        break;
        BF_CASE(4) BF_CASE(6) BF_CASE(8) BF_CASE(12) BF_CASE(16) BF_CASE(24)
#undef BF_CASE
        default: return hipErrorInvalidValue;
    }
    // two channels per step, one for the widest rows (registers); rows past
    // about 3000 samples need more than 64 KiB of LDS (the attribute is set
    // once per instantiation, to its largest row)
    if (sh.L == 4) {
        static hipError_t attr = hipFuncSetAttribute((const void *)k_boxrow<4, 2>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)boxrow_smem_bytes(1024, 4, 2));
        if (attr != hipSuccess) return attr;
        const size_t sm = boxrow_smem_bytes(sh.T, 4, 2);
        BF_LAUNCH("k_boxrow", (k_boxrow<4, 2>), dim3(p.H), dim3(sh.T), sm, s, p, S, sh.R, sh.P, sh.T);
    } else if (sh.L == 16) {
        static hipError_t attr = hipFuncSetAttribute((const void *)k_boxrow<16, 1>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)boxrow_smem_bytes(512, 16, 1));
        if (attr != hipSuccess) return attr;
        const size_t sm = boxrow_smem_bytes(sh.T, 16, 1);
        BF_LAUNCH("k_boxrow", (k_boxrow<16, 1>), dim3(p.H), dim3(sh.T), sm, s, p, S, sh.R, sh.P, sh.T);
    } else if (sh.L == 32) {
        // rows past 8192 samples: the row's prefix fills 135 KiB of LDS, and
        // two workgroups per row each evaluate half of the outputs
        static hipError_t attr = hipFuncSetAttribute((const void *)k_boxrow<32, 1, 16>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                                     (int)boxrow_smem_bytes(512, 32, 1));
        if (attr != hipSuccess) return attr;
        const size_t sm = boxrow_smem_bytes(sh.T, 32, 1);
        BF_LAUNCH("k_boxrow", (k_boxrow<32, 1, 16>), dim3(p.H, 2), dim3(sh.T), sm, s, p, S, sh.R, sh.P, sh.T);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace bfgp
