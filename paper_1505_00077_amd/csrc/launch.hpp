// Host-side launchers of the forward, backward and batched kernels.
#pragma once
#include "common.hpp"

namespace bfgp {

struct IirCoef;
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

hipError_t launch_stats(const GPParams &p, hipStream_t s);
hipError_t launch_fir(const GPParams &p, const FirTaps &t, int R, bool save, hipStream_t s);
hipError_t launch_iir(const GPParams &p, const IirCoef &c, int B, int L, int T, int G, float *carry, float *S,
                      hipStream_t s);
// Channel groups of the column passes for an image (enough workgroups to fill
// the device several times over).
int column_groups(int H, int W, int C);
hipError_t launch_direct(const DirectArgs &a, hipStream_t s);
int bwd_tiles(int H, int W);
hipError_t launch_bwd(const GPParams &p, const BwdParams &b, const FirTaps2 &t, int R, double *corr, double *g_lss,
                      double *g_lsr, hipStream_t s);

}  // namespace bfgp
