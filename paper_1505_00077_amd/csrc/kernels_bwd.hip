// __global__ entry points of the backward pass and their launchers.
#include "launch.hpp"
#include "bwd.hpp"
#include "iir_bwd.hpp"

namespace bfgp {

template <int R>
__global__ __launch_bounds__(kBlock) void k_bwd(GPParams p, BwdParams b, FirTaps2 taps) {
    extern __shared__ float smem[];
    const Stats st = load_stats(p);
    bwd_tile<R>(p, b, taps, st, blockIdx.y * BwdShape<R>::TY, blockIdx.x * BwdShape<R>::TX,
                blockIdx.y * gridDim.x + blockIdx.x, smem);
}

// Sums the per-tile partials in a fixed order and writes the scalar gradients
// and the mean-centring correction of the image gradient.
__global__ __launch_bounds__(64) void k_bwd_finalize(GPParams p, const BwdPartial *bp, int ntiles, double *corr,
                                                     double *g_lss, double *g_lsr) {
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
        *corr = p.center == 0 ? (v[4] - v[0]) / n : 0.0;
        if (g_lss) *g_lss = v[3];
        if (g_lsr) *g_lsr = v[2] - v[1];
    }
}

__global__ __launch_bounds__(kBlock) void k_bwd_apply(float *grad, int H, int W, int pitch, const double *corr) {
    const float c = (float)*corr;
    for (int y = blockIdx.x; y < H; y += gridDim.x)
        for (int x = threadIdx.x; x < W; x += kBlock) grad[(size_t)y * pitch + x] += c;
}

template <int R>
static hipError_t bwd_launch_r(const GPParams &p, const BwdParams &b, const FirTaps2 &t, hipStream_t s) {
    using S = BwdShape<R>;
    dim3 grid((p.W + S::TX - 1) / S::TX, (p.H + S::TY - 1) / S::TY);
    BF_LAUNCH("k_bwd", (k_bwd<R>), grid, dim3(kBlock), sizeof(float) * S::SMEM_FLOATS, s, p, b, t);
    return hipGetLastError();
}

int bwd_tiles(int H, int W) { return ((W + 31) / 32) * ((H + 31) / 32); }

hipError_t launch_bwd(const GPParams &p, const BwdParams &b, const FirTaps2 &t, int R, double *corr, double *g_lss,
                      double *g_lsr, hipStream_t s) {
    hipError_t e;
    switch (R) {
#define BF_CASE(r) case r: e = bwd_launch_r<r>(p, b, t, s); break;
        BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6) BF_CASE(7) BF_CASE(8)
        BF_CASE(9) BF_CASE(10) BF_CASE(11) BF_CASE(12) BF_CASE(13) BF_CASE(14) BF_CASE(15) BF_CASE(16)
        BF_CASE(17) BF_CASE(18) BF_CASE(19) BF_CASE(20) BF_CASE(21) BF_CASE(22) BF_CASE(23) BF_CASE(24)
#undef BF_CASE
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    BF_LAUNCH("k_bwd_finalize", k_bwd_finalize, dim3(1), dim3(64), 0, s, p, b.bparts, bwd_tiles(p.H, p.W), corr,
              g_lss, g_lsr);
    if (b.grad_img && p.center == 0) {
        const int g = p.H < 1024 ? p.H : 1024;
        BF_LAUNCH("k_bwd_apply", k_bwd_apply, dim3(g), dim3(kBlock), 0, s, b.grad_img, p.H, p.W, p.pitch, corr);
    }
    return hipGetLastError();
}

// ---- recursive (IIR) mode ------------------------------------------------------

template <bool AGG>
__global__ __launch_bounds__(64) void k_bwd_vband(GPParams p, BwdIir b, IirTan c) {
    __shared__ float tile[AGG ? 1 : 2 * kBwdBV * 65];
    const Stats st = load_stats(p);
    const int g = blockIdx.z;
    bvband<kBwdBV, AGG>(p, b, c, st, blockIdx.x * 64, blockIdx.y, (p.C * g) / b.Gv, (p.C * (g + 1)) / b.Gv, tile);
}

// lines: lines to resolve; stride: line stride of the carry array; horiz
// selects the band transfer blocks of the row pass.
__global__ __launch_bounds__(64) void k_bwd_resolve(GPParams p, IirTan c, float *carry, int nb, int lines, int stride,
                                                    int horiz) {
    const int line = blockIdx.x * 64 + threadIdx.x;
    if (line < lines)
        bresolve(horiz ? c.phiH : c.phiV, horiz ? c.psiH : c.psiV, nb, p.C, blockIdx.y, blockIdx.z, (size_t)stride,
                 (size_t)line, carry);
}

// End states: one wave per (64 rows, band, channel group).
__global__ __launch_bounds__(64) void k_bwd_hband_agg(GPParams p, BwdIir b, IirTan c) {
    const Stats st = load_stats(p);
    const int g = blockIdx.z;
    bhband<kBwdBH, true>(p, b, c, st, blockIdx.x * 64 + threadIdx.x, blockIdx.y, (p.C * g) / b.Gh,
                         (p.C * (g + 1)) / b.Gh, g, b.Gh, nullptr, nullptr);
}

// Rerun and contraction: one workgroup of Gh waves per (64 rows, band).
__global__ __launch_bounds__(256) void k_bwd_hband(GPParams p, BwdIir b, IirTan c) {
    extern __shared__ double red[];
    const Stats st = load_stats(p);
    const int g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);
    bhband<kBwdBH, false>(p, b, c, st, blockIdx.x * 64 + (threadIdx.x & 63), blockIdx.y, (p.C * g) / b.Gh,
                          (p.C * (g + 1)) / b.Gh, g, b.Gh, b.bparts + (size_t)blockIdx.y * gridDim.x + blockIdx.x, red);
}

static int iir_hp(int H) { return ((H + 63) / 64) * 64; }
int bwd_iir_parts(int H, int W) { return (iir_hp(H) / 64) * ((W + kBwdBH - 1) / kBwdBH); }

// Channel groups of the backward passes: enough waves for the device (about
// two per SIMD), at most 8 (column pass) and 4 (row pass, one workgroup).
// The column groups count the waves of all nimg images of a stacked call (the
// grouping does not change the column pass's rounding); the row groups, whose
// partial sums are added per group, count one image's, so that a stacked call
// and single calls give the same bits.
void bwd_iir_groups(int H, int W, int C, int nimg, int *Gv, int *Gh) {
    const long target = 2048;
    const long wv = (long)((W + 63) / 64) * ((H + kBwdBV - 1) / kBwdBV) * (nimg > 1 ? nimg : 1);
    const long wh = (long)(iir_hp(H) / 64) * ((W + kBwdBH - 1) / kBwdBH);
    long gv = (target + wv - 1) / wv, gh = (target + wh - 1) / wh;
    gv = gv < 1 ? 1 : (gv > 8 ? 8 : gv);
    gh = gh < 1 ? 1 : (gh > 4 ? 4 : gh);
    *Gv = (int)(gv > C ? C : gv);
    *Gh = (int)(gh > C ? C : gh);
}

hipError_t launch_bwd_iir(const GPParams &p, const BwdIir &b, const IirTan &c, double *corr, double *g_lss,
                          double *g_lsr, hipStream_t s) {
    if (b.Hp != iir_hp(p.H) || b.Gv < 1 || b.Gv > p.C || b.Gh < 1 || b.Gh > 4 || b.Gh > p.C)
        return hipErrorInvalidValue;
    const int nbv = (p.H + kBwdBV - 1) / kBwdBV, nbh = (p.W + kBwdBH - 1) / kBwdBH;
    const dim3 gv((p.W + 63) / 64, nbv, b.Gv);
    BF_LAUNCH("k_bwd_vband_agg", k_bwd_vband<true>, gv, dim3(64), 0, s, p, b, c);
    BF_LAUNCH("k_bwd_resolve", k_bwd_resolve, dim3((p.W + 63) / 64, p.C, 2), dim3(64), 0, s, p, c, b.cv, nbv, p.W,
              p.W, 0);
    BF_LAUNCH("k_bwd_vband", k_bwd_vband<false>, gv, dim3(64), 0, s, p, b, c);
    BF_LAUNCH("k_bwd_hband_agg", k_bwd_hband_agg, dim3(b.Hp / 64, nbh, b.Gh), dim3(64), 0, s, p, b, c);
    BF_LAUNCH("k_bwd_resolve", k_bwd_resolve, dim3((p.H + 63) / 64, p.C, 2), dim3(64), 0, s, p, c, b.chz, nbh, p.H,
              b.Hp, 1);
    BF_LAUNCH("k_bwd_hband", k_bwd_hband, dim3(b.Hp / 64, nbh), dim3(64 * b.Gh), bhband_smem_bytes(b.Gh, kBwdBH), s,
              p, b, c);
    BF_LAUNCH("k_bwd_finalize", k_bwd_finalize, dim3(1), dim3(64), 0, s, p, b.bparts, bwd_iir_parts(p.H, p.W), corr,
              g_lss, g_lsr);
    if (b.grad_img && p.center == 0) {
        const int g = p.H < 1024 ? p.H : 1024;
        BF_LAUNCH("k_bwd_apply", k_bwd_apply, dim3(g), dim3(kBlock), 0, s, b.grad_img, p.H, p.W, p.pitch, corr);
    }
    return hipGetLastError();
}

}  // namespace bfgp
