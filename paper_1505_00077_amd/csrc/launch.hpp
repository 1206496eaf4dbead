// Host-side launchers of the forward, backward and batched kernels.
#pragma once
#include "common.hpp"

namespace bfgp {

struct IirCoef;
struct RowCoef;
struct DirectArgs;
struct BwdParams;
struct FirTaps2;

// stage timing hooks (no-ops unless bf_profile_enable(1))
void prof_begin(hipStream_t s, const char *name, long long threads);
void prof_end(hipStream_t s);

// Launches a kernel between the two profiling marks.
#define BF_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                   \
    do {                                                                           \
        ::bfgp::prof_begin(stream, name, (long long)dim3(grid).x * dim3(grid).y * dim3(grid).z * \
                                             dim3(block).x * dim3(block).y * dim3(block).z);   \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);       \
        ::bfgp::prof_end(stream);                                                  \
    } while (0)

// Statistics partials; with final_kernel also a kernel that reduces them
// (otherwise the next kernel reduces them itself).
hipError_t launch_stats(const GPParams &p, bool final_kernel, hipStream_t s);
hipError_t launch_fir(const GPParams &p, const FirTaps &t, int R, bool save, hipStream_t s);
// Launch shape of the IIR passes for one image.  The single-image and the
// batched path take it from the same function, so both round identically.
struct IirShape {
    int B;   // band height of the column passes (32 or 64 rows)
    int G;   // channel groups of the column passes
    int L;   // samples per thread in the row pass (4, 8, 12 or 16)
    int T;   // threads per channel group of the row pass (T L >= W, T Gr <= 512)
    int Gr;  // channel groups of the row pass
    int Lo;  // the same for the row pass with the saved terms and the joint
    int To;  // filter (and the batched path): L 4, 8, 12 or 16, T <= 512
    int Gro;
    int P;   // row pitch of the channel stack, >= W rounded up to 4 plus
             // max(L, Lo) + 2, a multiple of 32 (columns W .. P-1 are zero;
             // row-pass chunks past the row end read them)
    int Hs;  // rows per channel of the stack: H rounded up to a multiple of B
    int nseg;  // segments of T L = 8192 columns per row in the row pass (rows
               // wider than 8192, the plain forward only); 1 otherwise
};
// batch: the image is one of many filtered together, which fill the device by
// themselves: no channel groups unless the tuning overrides ask for them.
IirShape iir_shape(int H, int W, int C, bool batch = false, bool rows32 = false);
// save: also store the terms bf_gp_backward needs (p.saved), with the row pass
// in one channel group.  joint: the joint filter (p.img the guide, p.data the
// data, p.C = 2 (N + 1) stack channels), row pass in one channel group.
// c: the column passes' coefficients (and the row pass of the saved terms and
// the joint filter, chunks of sh.Lo); rc: the row pass's (chunks of sh.L).
// segst: the segments' end states of rows wider than 8192 (sh.nseg > 1).
hipError_t launch_iir(const GPParams &p, const IirCoef &c, const RowCoef &rc, const IirShape &sh, float *carry,
                      float *S, bool save, bool joint, hipStream_t s, float *segst = nullptr);
hipError_t launch_direct(const DirectArgs &a, hipStream_t s);
struct BoxShape;
// Box spatial mode: column pass (running sums) into the stack S, then the row
// pass with the recombination.
hipError_t launch_box(const GPParams &p, const BoxShape &sh, float *S, hipStream_t s);
// Buffers of a volume forward: the time-direction carries and stack S1
// (C x rows_B(T) x (H W)), the per-frame column carries and the row-pass stack
// S2 (T x C x Hs x P), Hs = H rounded up to the band.
struct VolumeBuffers {
    float *carry_z, *S1, *carry_y, *S2;
    int Hs;
};
// pz: the volume as a T x (H W) image (coefficients ct, shape shz); ps: the
// volume as a (T H) x W image (statistics; coefficients cs and shape shs of
// each H x W frame).
hipError_t launch_volume(const GPParams &pz, const GPParams &ps, const IirCoef &ct, const IirCoef &cs,
                         const RowCoef &rcs, const IirShape &shz, const IirShape &shs, int T, const VolumeBuffers &vb,
                         hipStream_t s);
// Stacked batch (B images of one size): image b at img + b * img elements
// (image, output, gradients), workspace slice ws0 + b * ws bytes, saved terms
// saved0 + b * saved bytes.
struct StkOfs {
    size_t img, ws, saved;
    int B;
};
struct RowCoef;
struct FirTaps2;
struct BwdParams;
struct BwdIir;
struct IirTan;
hipError_t launch_stk_setup(const GPParams &p0, const StkOfs &o, GPParams *pd, hipStream_t s);
hipError_t launch_stk_stats(const GPParams &p0, const GPParams *pd, const StkOfs &o, bool final_kernel, hipStream_t s);
hipError_t launch_stk_fir(const GPParams &p0, const GPParams *pd, const StkOfs &o, const FirTaps &t, int R, bool save,
                          hipStream_t s);
hipError_t launch_stk_iir(const GPParams &p0, const GPParams *pd, const StkOfs &o, const IirCoef &c,
                          const RowCoef &rc, const IirShape &sh, float *carry, float *S, bool save, hipStream_t s);
hipError_t launch_stk_bwd(const GPParams &p0, const GPParams *pd, const BwdParams &b, const StkOfs &o,
                          const FirTaps2 &t, int R, double *corr, double *g_lss, double *g_lsr, hipStream_t s);
hipError_t launch_stk_bwd_iir(const GPParams &p0, const GPParams *pd, const BwdIir &b, const StkOfs &o,
                              const IirTan &c, double *corr, double *g_lss, double *g_lsr, hipStream_t s);
int bwd_tiles(int H, int W);
hipError_t launch_bwd(const GPParams &p, const BwdParams &b, const FirTaps2 &t, int R, double *corr, double *g_lss,
                      double *g_lsr, hipStream_t s);
struct BwdIir;
struct IirTan;
int bwd_iir_parts(int H, int W);
void bwd_iir_groups(int H, int W, int C, int nimg, int *Gv, int *Gh);
hipError_t launch_bwd_iir(const GPParams &p, const BwdIir &b, const IirTan &c, double *corr, double *g_lss,
                          double *g_lsr, hipStream_t s);

}  // namespace bfgp
