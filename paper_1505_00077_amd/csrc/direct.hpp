// Eq. (1) evaluated directly, for the O(sigma_s^2) comparison.
//
// One workgroup computes a TY x TX output tile.  The (TY + 2W) input rows
// around the tile are streamed through LDS in slabs of SLAB rows, each slab
// (SLAB x (TX + 2W)) loaded once; every output pixel walks the slab rows
// inside its window and all 2W+1 columns, with one exp2 per tap.  Spatial
// weights enter as log2 values so that each tap costs one exp2:
//   w = exp2(c_r (f_j - f_i)^2 + l(dy) + l(dx)),  c_r = -log2(e) / (2 sigma_r^2),
//   l(d) = -log2(e) d^2 / (2 sigma_s^2).
// Numerator and denominator accumulate in double.
#pragma once
#include "common.hpp"

namespace bfgp {

struct DirectArgs {
    const float *img;
    float *out;
    int H, W, pitch;
    int win;            // window half-width
    float cr;           // -log2(e) / (2 sigma_r^2)
    float lk[kDirectMaxW + 1];  // -log2(e) d^2 / (2 sigma_s^2)
};

constexpr int kDirTY = 16, kDirTX = 64, kDirSlab = 16;
__host__ __device__ constexpr int direct_smem_floats() {
    return kDirSlab * (kDirTX + 2 * kDirectMaxW) + (2 * kDirectMaxW + 1);
}

__device__ __forceinline__ void direct_tile(const DirectArgs &a, int ty0, int tx0, float *smem) {
    const int Wn = a.win;
    const int SX = kDirTX + 2 * Wn;  // slab row length
    float *slab = smem;
    float *lkx = smem + kDirSlab * (kDirTX + 2 * kDirectMaxW);
    const int tid = threadIdx.x;
    for (int i = tid; i <= 2 * Wn; i += kBlock) lkx[i] = a.lk[i >= Wn ? i - Wn : Wn - i];

    const int ox = tid & 63;
    const int oyb = tid >> 6;  // rows oyb, oyb+4, oyb+8, oyb+12
    constexpr int PY = kDirTY / (kBlock / 64);
    float fi[PY];
    double num[PY], den[PY];
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const int gy = ty0 + oyb + 4 * j, gx = tx0 + ox;
        fi[j] = (gy < a.H && gx < a.W) ? a.img[(size_t)gy * a.pitch + gx] : 0.f;
        num[j] = 0.0;
        den[j] = 0.0;
    }
    const int rows = kDirTY + 2 * Wn;
    for (int s0 = 0; s0 < rows; s0 += kDirSlab) {
        __syncthreads();
        const int ns = min(kDirSlab, rows - s0);
        for (int e = tid; e < ns * SX; e += kBlock) {
            const int r = e / SX, c = e % SX;
            const int gy = ty0 - Wn + s0 + r, gx = tx0 - Wn + c;
            // out-of-image neighbours are marked with NaN and skipped
            slab[r * SX + c] = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W)
                                   ? a.img[(size_t)gy * a.pitch + gx] : __builtin_nanf("");
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < PY; ++j) {
            const int oy = oyb + 4 * j;
            // slab row r holds input row ty0 - Wn + s0 + r; offset dy = row - (ty0 + oy)
            const int rlo = max(0, oy - s0), rhi = min(ns - 1, oy + 2 * Wn - s0);
            for (int r = rlo; r <= rhi; ++r) {
                const int dy = s0 + r - oy - Wn;
                const float ly = a.lk[dy >= 0 ? dy : -dy];
                const float *row = slab + r * SX + ox;
                float sn = 0.f, sd = 0.f;
                for (int dx = 0; dx <= 2 * Wn; ++dx) {
                    const float v = row[dx];
                    const float t = v - fi[j];
                    const float w = exp2f(fmaf(t * t, a.cr, ly + lkx[dx]));
                    // NaN (outside the image) fails the comparison and is skipped
                    const bool in = v == v;
                    sn += in ? w * v : 0.f;
                    sd += in ? w : 0.f;
                }
                num[j] += (double)sn;
                den[j] += (double)sd;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < PY; ++j) {
        const int gy = ty0 + oyb + 4 * j, gx = tx0 + ox;
        if (gy < a.H && gx < a.W) a.out[(size_t)gy * a.pitch + gx] = (float)(num[j] / den[j]);
    }
}

}  // namespace bfgp
