// Batched GP forward: many images of uneven size, each with its own sigma_s and
// sigma_r, in one graph of grouped launches.
//
// The host builds, per stage, one work list that covers every image of the
// batch.  Each stage is one grouped launch with one workgroup per item; stage
// order is kept by the launch order on the stream, so no workgroup ever waits
// for another and the grid always drains.  Stages: statistics (all images),
// fused FIR tiles (FIR images), then for IIR images the column-band end states,
// the band carry resolution, the column pass and the row pass with the FP64
// recombination.  The whole sequence is captured into a hipGraph by the caller
// and replayed.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/bfgp.h"
#include "launch.hpp"
#include "fir.hpp"
#include "iir.hpp"
#include "hrow.hpp"

namespace bfgp {

// kStRow + k: row items whose workgroup has 64 (k + 1) threads (k = 0..7)
// kStFir: FIR images with radius up to kBatchFirSplit; kStFirWide: the rest
// (separate launches, so that wide radii do not set the register budget of
// narrow ones)
// kStAggM: end states by weighted sums (stacks of at most kAggMaxC channels),
// four items of one image per workgroup; kStAgg: by the recursion (wider
// stacks), one item per workgroup.
enum { kStStats = 0, kStFir, kStFirWide, kStAggM, kStAgg, kStResolve, kStBand, kStRow, kNumStages = kStRow + 8 };
constexpr int kBatchFirSplit = 12;
// same partial count as the single-image path, so that both reduce the image
// sum in the same order and produce bit-identical centres and outputs
constexpr int kBatchStatsParts = kMaxParts;
constexpr int kBatchFirMaxR = kFirMaxR;
constexpr int kBatchMaxW = 8192;

struct BatchImage {
    GPParams p;
    IirCoef c;
    AggW aw;  // end-state weights for the image's band height
    RowCoef rc;
    FirTaps taps;
    int iir;       // 0 FIR, 1 IIR
    int R;         // FIR radius
    int Bh;        // IIR band rows (32 or 64)
    int nb;        // IIR bands
    int G;         // channel groups of the column passes
    int L;         // IIR row chunk
    int T;         // row threads per channel group
    int Gr;        // channel groups of the row pass
    int Sp;        // row pitch of the channel stack
    int Sr;        // rows per channel of the stack
    float *carry;
    float *S;
};

struct BatchItem {
    int img, idx;
};

__global__ __launch_bounds__(kBlock) void k_bstats(const BatchImage *imgs, const BatchItem *items) {
    const BatchItem w = items[blockIdx.x];
    const GPParams &p = imgs[w.img].p;
    stats_rows(p.img, p.H, p.W, p.pitch, w.idx, p.nparts, const_cast<Partial *>(p.parts));
}


template <int R>
__device__ __forceinline__ void fir_item(const BatchImage &B, const Stats &st, int idx, float *smem) {
    const int tx = (B.p.W + fir_tx(R) - 1) / fir_tx(R);
    fir_tile_auto<R, false>(B.p, B.taps, st, (idx / tx) * fir_ty(R), (idx % tx) * fir_tx(R), smem);
}

template <bool WIDE>
__global__ __launch_bounds__(kBlock) void k_bfir(const BatchImage *imgs, const BatchItem *items) {
    extern __shared__ float smem[];
    const BatchItem w = items[blockIdx.x];
    const BatchImage &B = imgs[w.img];
    // first kernel after the statistics pass for FIR images
    const Stats st = reduce_stats(B.p);
    if (w.idx == 0 && threadIdx.x == 0) publish_stats(B.p, st);
#define BF_CASE(r) case r: fir_item<r>(B, st, w.idx, smem); break;
    if (!WIDE) {
        switch (B.R) {
            BF_CASE(1) BF_CASE(2) BF_CASE(3) BF_CASE(4) BF_CASE(5) BF_CASE(6)
            BF_CASE(7) BF_CASE(8) BF_CASE(9) BF_CASE(10) BF_CASE(11) BF_CASE(12)
            default: break;
        }
    } else {
        switch (B.R) {
            BF_CASE(13) BF_CASE(14) BF_CASE(15) BF_CASE(16) BF_CASE(17) BF_CASE(18)
            BF_CASE(19) BF_CASE(20) BF_CASE(21) BF_CASE(22) BF_CASE(23) BF_CASE(24)
            default: break;
        }
    }
#undef BF_CASE
}

// One item = one channel group of one band of one 64-column group (one wave,
// as in the single-image launch).  The end-state pass is the first kernel
// after the statistics pass for IIR images.  The band height is the same for
// every image of a plan (it depends on no image property).
template <int BH, bool AGG>
__global__ __launch_bounds__(64, (BH == 32 ? 3 : 2)) void k_bband(const BatchImage *imgs, const BatchItem *items) {
    __shared__ float sacc[AGG ? 1 : BH * 64];
    const BatchItem w = items[blockIdx.x];
    const BatchImage &B = imgs[w.img];
    Stats st;
    if (AGG) {
        st = reduce_stats(B.p);
        if (w.idx == 0 && threadIdx.x == 0) publish_stats(B.p, st);
    } else {
        st = load_stats(B.p);
    }
    if (!st.ok) return;
    const bool big = st.xmax > 12.0;
    const int lane = threadIdx.x & 63;
    const int ncg = (B.Sp + 63) / 64;
    const int g = w.idx % B.G, rest = w.idx / B.G;
    const int band = rest / ncg, cg = rest % ncg;
    const int cb = (B.p.C * g) / B.G, ce = (B.p.C * (g + 1)) / B.G;
    float *sa = sacc;
    const int col = cg * 64 + lane;
    if (big)
        vband<BH, AGG, true>(B.p, B.c, st, col, band, B.carry, B.S, B.Sp, sa, cb, ce);
    else
        vband<BH, AGG, false>(B.p, B.c, st, col, band, B.carry, B.S, B.Sp, sa, cb, ce);
}

// End states by weighted sums (as the single-image k_vagg, with the same
// channel groups, so that both give the same bits): item idx of an image
// covers its bands 4 idx / G .. 4 (idx + 1) / G - 1, G waves per band
// (bands of 64 rows: four groups, one band per item).
template <int BH>
__global__ __launch_bounds__(256) void k_bagg(const BatchImage *imgs, const BatchItem *items) {
    constexpr int NR = BH + 3;
    __shared__ float sm[vagg_smem_floats(BH, BH == 32 ? 2 : 1)];  // at most two bands (G >= 2) of 32 rows
    float *wts = sm;
    const BatchItem w = items[blockIdx.x];
    const BatchImage &B = imgs[w.img];
    const Stats st = reduce_stats(B.p);
    if (w.idx == 0 && threadIdx.x == 0) publish_stats(B.p, st);
    if (!st.ok) return;
    for (int k = threadIdx.x; k < (BH + 3) * 8; k += blockDim.x) wts[k] = B.aw.w[k];
    const int G = BH == 32 ? agg_groups(B.p.H, B.p.W, B.p.C) : 4;
    const int cgr = (B.p.W + 63) / 64;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int pr = wave / G, gw = wave % G;
    const int pair = w.idx * (4 / G) + pr;
    const bool live = pair < cgr * B.nb;
    const int cg = pair % cgr, band = pair / cgr;
    const int col = cg * 64 + (threadIdx.x & 63);
    float *pro = sm + NR * 8 + pr * 2 * NR * 64;
    const bool big = st.xmax > 12.0;
    if (live) {
        if (big)
            vagg_prologue<BH, true>(B.p, st, col, band, gw, G, pro);
        else
            vagg_prologue<BH, false>(B.p, st, col, band, gw, G, pro);
    }
    __syncthreads();
    if (!live) return;
    if (big)
        vagg_moments<BH, kAggG, true>(B.p, col, band, B.carry, gw, G, wts, pro);
    else
        vagg_moments<BH, kAggG, false>(B.p, col, band, B.carry, gw, G, wts, pro);
}

__global__ __launch_bounds__(kBlock) void k_bresolve(const BatchImage *imgs, const BatchItem *items) {
    const BatchItem w = items[blockIdx.x];
    const BatchImage &B = imgs[w.img];
    const int ng = (B.p.W + kBlock - 1) / kBlock;
    const int dir = w.idx & 1, rest = w.idx >> 1;
    const int n = rest / ng, col = (rest % ng) * kBlock + threadIdx.x;
    if (col < B.p.W) vresolve(B.p, B.c, B.nb, col, n, dir, B.carry);
}

// blockDim: T * Gr of every image in the launch (images are launched in
// classes of equal workgroup size).
__global__ __launch_bounds__(512) void k_brow(const BatchImage *imgs, const BatchItem *items) {
    extern __shared__ float sm[];
    const BatchItem w = items[blockIdx.x];
    const BatchImage &B = imgs[w.img];
    const Stats st = load_stats(B.p);
    if (!st.ok) {
        for (int x = threadIdx.x; x < B.p.W; x += blockDim.x) B.p.out[(size_t)w.idx * B.p.pitch + x] = __builtin_nanf("");
        return;
    }
    switch (B.L) {
        case 4: hrow2<4>(B.p, B.rc, st, w.idx, B.S, B.Sr, B.Sp, sm, B.T, B.Gr); break;
        case 8: hrow2<8>(B.p, B.rc, st, w.idx, B.S, B.Sr, B.Sp, sm, B.T, B.Gr); break;
        case 12: hrow2<12>(B.p, B.rc, st, w.idx, B.S, B.Sr, B.Sp, sm, B.T, B.Gr); break;
        default: hrow2<16>(B.p, B.rc, st, w.idx, B.S, B.Sr, B.Sp, sm, B.T, B.Gr); break;
    }
}

// ---- host side -------------------------------------------------------------

struct Plan {
    std::vector<bf_gp_item> items;
    std::vector<BatchImage> imgs;
    std::vector<BatchItem> work;           // all stages, concatenated
    int first[kNumStages + 1];             // stage s items: work[first[s] .. first[s+1])
    std::vector<int> iir, R;
    std::vector<IirShape> shape;
    size_t off_imgs, off_items, total;
    std::vector<size_t> off_parts, off_status, off_stats, off_carry, off_S;
    size_t fir_smem[2], row_smem[8];
    int band_rows;
    unsigned flags;
    bool uploaded;
    void *ws;
};

}  // namespace bfgp

using namespace bfgp;

namespace {

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

int fir_radius_b(double sigma_s) {
    int r = (int)ceil(3.0 * sigma_s * (1.0 - 1e-6));
    return r < 1 ? 1 : r;
}

}  // namespace

// defined in api.hip
namespace bfgp {
GPParams gp_params_for(const float *img, float *out, int H, int W, int pitch, double sigma_r, int N, unsigned flags,
                       const Partial *parts, int nparts, int *status, Stats *stats);
IirCoef iir_coef_for(double sigma_s, int B, int L);
RowCoef row_coef_for(double sigma_s, int L);
FirTaps fir_taps_for(double sigma_s, int R);
int set_error(int code, const char *msg);
}  // namespace bfgp

extern "C" {

int bf_gp_plan_batched(const bf_gp_item *items, int count, unsigned flags, void **plan_out) {
    if (!plan_out) return set_error(BF_EINVAL, "null plan_out");
    *plan_out = nullptr;
    if (!items || count < 1) return set_error(BF_EINVAL, "empty batch");
    if (flags & ~(BF_SPATIAL_MASK | BF_CENTER_MASK)) return set_error(BF_EINVAL, "unknown flag bits");
    if ((flags & BF_CENTER_MASK) == 12u) return set_error(BF_EINVAL, "invalid flags");
    if ((flags & BF_SPATIAL_MASK) == BF_SPATIAL_BOX)
        return set_error(BF_EUNSUPPORTED, "the batched path runs the FIR and IIR modes");
    for (int i = 0; i < count; ++i) {
        const bf_gp_item &it = items[i];
        if (!it.img || !it.out || it.img == it.out) return set_error(BF_EINVAL, "bad image pointers in the batch");
        if (it.H < 1 || it.W < 1 || it.pitch < it.W) return set_error(BF_EINVAL, "bad image size in the batch");
        if (!(it.sigma_s > 0) || !(it.sigma_r > 0) || !std::isfinite((double)it.sigma_s) ||
            !std::isfinite((double)it.sigma_r))
            return set_error(BF_EINVAL, "bad sigma in the batch");
        if (it.N < 0 || it.N > BF_MAX_DEGREE) return set_error(BF_EINVAL, "bad degree in the batch");
        if (it.W > kBatchMaxW) return set_error(BF_EUNSUPPORTED, "batched images are limited to 8192 columns");
    }
    Plan *P = new (std::nothrow) Plan();
    if (!P) return set_error(BF_EHIP, "out of host memory");
    P->items.assign(items, items + count);
    P->flags = flags;
    P->uploaded = false;
    P->ws = nullptr;
    size_t off = 0;
    P->off_imgs = off;
    off = al(off + sizeof(BatchImage) * count);
    size_t fir_smem[2] = {0, 0};
    std::vector<std::vector<BatchItem>> per(kNumStages);
    P->off_parts.resize(count);
    P->off_status.resize(count);
    P->off_stats.resize(count);
    P->off_carry.resize(count);
    P->off_S.resize(count);
    P->iir.resize(count);
    P->R.resize(count);
    P->shape.assign(count, IirShape{64, 1, 16, 64, 1});
    size_t row_smem[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    P->band_rows = 32;
    for (int i = 0; i < count; ++i) {
        const bf_gp_item &it = items[i];
        unsigned m = flags & BF_SPATIAL_MASK;
        if (m == BF_SPATIAL_AUTO) m = bf_gp_resolve_spatial_for(it.H, it.W, it.sigma_s, flags);
        const int R = fir_radius_b(it.sigma_s);
        const bool iir = (m == BF_SPATIAL_IIR) || R > kBatchFirMaxR;
        P->iir[i] = iir;
        P->R[i] = R;
        const int nparts = std::min(it.H, kBatchStatsParts);
        P->off_parts[i] = off;
        off = al(off + sizeof(Partial) * nparts);
        P->off_status[i] = off;
        off = al(off + 16);
        P->off_stats[i] = off;
        off = al(off + sizeof(Stats));
        for (int b = 0; b < nparts; ++b) per[kStStats].push_back({i, b});
        if (!iir) {
            const int tiles = ((it.W + fir_tx(R) - 1) / fir_tx(R)) * ((it.H + fir_ty(R) - 1) / fir_ty(R));
            const int wide = R > kBatchFirSplit;
            for (int t = 0; t < tiles; ++t) per[wide ? kStFirWide : kStFir].push_back({i, t});
            fir_smem[wide] = std::max(fir_smem[wide], sizeof(float) * (size_t)fir_smem_floats(R));
            P->off_carry[i] = P->off_S[i] = 0;
        } else {
            const size_t C = (size_t)it.N + 2;
            const IirShape sh = iir_shape(it.H, it.W, (int)C, true);
            P->shape[i] = sh;
            P->band_rows = sh.B;  // the same for every image
            const int nb = (it.H + sh.B - 1) / sh.B;
            P->off_carry[i] = off;
            off = al(off + sizeof(float) * nb * C * 8 * (size_t)it.W);
            P->off_S[i] = off;
            off = al(off + sizeof(float) * C * (size_t)sh.Hs * sh.P);
            const int ncg = (sh.P + 63) / 64;
            const int G = sh.G;
            const int cls = sh.T * sh.Gr / 64 - 1;  // T * Gr is a multiple of 64, at most 512
            row_smem[cls] = std::max(row_smem[cls], hrow2_smem_bytes(sh.T, sh.Gr, sh.L));
            if ((int)C <= kAggMaxC) {
                const int G = sh.B == 32 ? agg_groups(it.H, it.W, (int)C) : 4;
                const int nbands = (it.W + 63) / 64 * nb;
                for (int t = 0; t < (nbands * G + 3) / 4; ++t) per[kStAggM].push_back({i, t});
            } else {
                for (int t = 0; t < nb * ncg * G; ++t) per[kStAgg].push_back({i, t});
            }
            const int ng = (it.W + kBlock - 1) / kBlock;
            for (int t = 0; t < (int)C * ng * 2; ++t) per[kStResolve].push_back({i, t});
            for (int t = 0; t < nb * ncg * G; ++t) per[kStBand].push_back({i, t});
            for (int y = 0; y < it.H; ++y) per[kStRow + cls].push_back({i, y});
        }
    }
    for (int s = 0; s < kNumStages; ++s) {
        P->first[s] = (int)P->work.size();
        P->work.insert(P->work.end(), per[s].begin(), per[s].end());
    }
    P->first[kNumStages] = (int)P->work.size();
    P->off_items = off;
    off = al(off + sizeof(BatchItem) * P->work.size());
    P->total = off;
    P->fir_smem[0] = fir_smem[0];
    P->fir_smem[1] = fir_smem[1];
    for (int k = 0; k < 8; ++k) P->row_smem[k] = row_smem[k];
    P->imgs.resize(count);
    *plan_out = P;
    return BF_OK;
}

size_t bf_gp_plan_workspace_bytes(const void *plan) {
    return plan ? ((const Plan *)plan)->total : 0;
}

int bf_gp_plan_upload(void *plan, void *ws, size_t ws_bytes, void *stream) {
    Plan *P = (Plan *)plan;
    if (!P || !ws) return set_error(BF_EINVAL, "null plan or workspace");
    if (ws_bytes < P->total) return set_error(BF_ENOMEM, "workspace too small for the batch plan");
    char *w = (char *)ws;
    const int count = (int)P->items.size();
    for (int i = 0; i < count; ++i) {
        const bf_gp_item &it = P->items[i];
        BatchImage &B = P->imgs[i];
        memset(&B, 0, sizeof B);
        const int nparts = std::min(it.H, kBatchStatsParts);
        B.p = gp_params_for(it.img, it.out, it.H, it.W, it.pitch, it.sigma_r, it.N, P->flags,
                            (const Partial *)(w + P->off_parts[i]), nparts, (int *)(w + P->off_status[i]),
                            (Stats *)(w + P->off_stats[i]));
        B.iir = P->iir[i];
        B.R = P->R[i];
        const IirShape &sh = P->shape[i];
        B.Bh = sh.B;
        B.nb = (it.H + sh.B - 1) / sh.B;
        B.G = sh.G;
        B.L = sh.L;
        B.T = sh.T;
        B.Gr = sh.Gr;
        B.Sp = sh.P;
        B.Sr = sh.Hs;
        if (B.iir) {
            B.c = iir_coef_for(it.sigma_s, sh.B, sh.Lo);
            B.aw = make_agg_w(B.c, sh.B);
            B.rc = row_coef_for(it.sigma_s, sh.L);
            B.carry = (float *)(w + P->off_carry[i]);
            B.S = (float *)(w + P->off_S[i]);
        } else {
            B.taps = fir_taps_for(it.sigma_s, B.R);
        }
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(w + P->off_imgs, P->imgs.data(), sizeof(BatchImage) * count,
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + P->off_items, P->work.data(), sizeof(BatchItem) * P->work.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return set_error(BF_EHIP, hipGetErrorString(e));
    P->uploaded = true;
    P->ws = ws;
    return BF_OK;
}

int bf_gp_forward_batched(void *plan, void *ws, size_t ws_bytes, void *stream) {
    Plan *P = (Plan *)plan;
    if (!P || !ws) return set_error(BF_EINVAL, "null plan or workspace");
    if (!P->uploaded || P->ws != ws) return set_error(BF_EINVAL, "plan not uploaded to this workspace");
    if (ws_bytes < P->total) return set_error(BF_ENOMEM, "workspace too small for the batch plan");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const BatchImage *imgs = (const BatchImage *)(w + P->off_imgs);
    const BatchItem *work = (const BatchItem *)(w + P->off_items);
    auto n = [P](int st) { return P->first[st + 1] - P->first[st]; };
    auto at = [P, work](int st) { return work + P->first[st]; };
    if (n(kStStats)) BF_LAUNCH("k_bstats", k_bstats, dim3(n(kStStats)), dim3(kBlock), 0, s, imgs, at(kStStats));
    if (n(kStFir))
        BF_LAUNCH("k_bfir", k_bfir<false>, dim3(n(kStFir)), dim3(kBlock), P->fir_smem[0], s, imgs, at(kStFir));
    if (n(kStFirWide))
        BF_LAUNCH("k_bfir", k_bfir<true>, dim3(n(kStFirWide)), dim3(kBlock), P->fir_smem[1], s, imgs, at(kStFirWide));
    if (n(kStAggM) || n(kStAgg)) {
        if (n(kStAggM)) {
            if (P->band_rows == 32)
                BF_LAUNCH("k_bband_agg", k_bagg<32>, dim3(n(kStAggM)), dim3(256), 0, s, imgs, at(kStAggM));
            else
                BF_LAUNCH("k_bband_agg", k_bagg<64>, dim3(n(kStAggM)), dim3(256), 0, s, imgs, at(kStAggM));
        }
        if (n(kStAgg)) {
            if (P->band_rows == 32)
                BF_LAUNCH("k_bband_agg", (k_bband<32, true>), dim3(n(kStAgg)), dim3(64), 0, s, imgs, at(kStAgg));
            else
                BF_LAUNCH("k_bband_agg", (k_bband<64, true>), dim3(n(kStAgg)), dim3(64), 0, s, imgs, at(kStAgg));
        }
        BF_LAUNCH("k_bresolve", k_bresolve, dim3(n(kStResolve)), dim3(kBlock), 0, s, imgs, at(kStResolve));
        if (P->band_rows == 32)
            BF_LAUNCH("k_bband", (k_bband<32, false>), dim3(n(kStBand)), dim3(64), 0, s, imgs, at(kStBand));
        else
            BF_LAUNCH("k_bband", (k_bband<64, false>), dim3(n(kStBand)), dim3(64), 0, s, imgs, at(kStBand));
        for (int k = 0; k < 8; ++k) {
            if (n(kStRow + k) && P->row_smem[k] > 65536) {
                static hipError_t attr = hipFuncSetAttribute((const void *)k_brow,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
                if (attr != hipSuccess) return set_error(BF_EHIP, hipGetErrorString(attr));
            }
        }
        for (int k = 0; k < 8; ++k)
            if (n(kStRow + k))
                BF_LAUNCH("k_brow", k_brow, dim3(n(kStRow + k)), dim3(64 * (k + 1)), P->row_smem[k], s, imgs,
                          at(kStRow + k));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(BF_EHIP, hipGetErrorString(e));
    return BF_OK;
}

void bf_gp_plan_free(void *plan) { delete (Plan *)plan; }

}  // extern "C"
