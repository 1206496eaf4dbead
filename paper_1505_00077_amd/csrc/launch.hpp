// Host-side launchers of the forward, backward and batched kernels.
#pragma once
#include "common.hpp"

namespace bfgp {

struct IirCoef;
struct DirectArgs;

hipError_t launch_stats(const float *img, int H, int W, int pitch, Partial *parts, int nparts, hipStream_t s);
hipError_t launch_fir(const GPParams &p, const FirTaps &t, int R, bool save, hipStream_t s);
hipError_t launch_iir(const GPParams &p, const IirCoef &c, int B, int L, int T, float *carry, float *S, hipStream_t s);
hipError_t launch_direct(const DirectArgs &a, hipStream_t s);

}  // namespace bfgp
