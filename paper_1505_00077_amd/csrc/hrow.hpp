// Row pass of the recursive (IIR) spatial filter fused with the FP64
// recombination (eqs. (8)-(11)): one workgroup owns one image row and filters
// every channel of the column-filtered stack along it.
//
// Thread t of a channel group owns the chunk of L samples [t L, t L + L).  Per
// channel:
//   1. the chunk runs causally and anticausally from rest (with its true halo
//      inputs), giving local outputs and the chunk's end states;
//   2. the chunk states are combined in order in three levels: a Kogge-Stone
//      scan inside each row of 16 lanes (DPP shifts, distances 1, 2, 4, 8
//      chunks), a scan over the wave's four row totals (gathered into four
//      lanes by cross-lane permutes), and, when a row spans several waves, a
//      scan over the wave totals that the waves leave in LDS (one barrier per
//      channel);
//   3. each chunk adds the homogeneous response of its true incoming states.
// The states are those of Deriche's second-order sections (two per
// direction), y_n = n0 x_n + n1 x_{n-1} - d1 y_{n-1} - d2 y_{n-2} and its
// anticausal mirror; a state (y_{n-1}, y_{n-2}) moves over m samples without
// input by Phi^m, Phi = [[-d1, -d2], [1, 0]].
//
// Recombination.  With a_k = Ubar_k / sqrt(k!) (the filtered channel k, in
// double) and P(tau) = sum_{k=0}^{N+1} a_k tau^k, the two sums of eq. (11)
// times exp(tau^2/2) are
//     D = sum_{k<=N} a_k tau^k = P(tau) - a_{N+1} tau^(N+1),
//     M = sum_{k=1}^{N+1} k a_k tau^{k-1} = P'(tau)
// (M is the derivative of the channel polynomial: sqrt(n+1) u_n(tau) /
// exp(-tau^2/2) = (n+1) tau^n / sqrt((n+1)!)).  Channels are visited from the
// top down and P and P' are evaluated together by Horner in tau, the same
// step for every channel:
//     c <- c tau + b,   b <- b tau + a_k,
// and the top term is taken out of D at the end (from the top channel's
// filtered row, kept in LDS).  Where |x| is large that term dominates P, and
// the difference loses about log10(P / D) of the sixteen digits of the
// double sums: one or two.  A channel group that starts at channel cb > 0
// evaluates its part relative to tau^cb; the groups' parts are added by
// group 0 in order:
//     D = sum_g tau^cb_g d_g,  M = sum_g (cb_g tau^(cb_g - 1) b_g + tau^cb_g c_g),
// with d_g = b_g except in the group holding channel N+1.
#pragma once
#include "iir.hpp"

namespace bfgp {

// Coefficients of the row pass for one sigma_s and chunk length L.
constexpr int kRowMaxL = 16;  // samples per thread
constexpr int kRowSeg = 512 * kRowMaxL;  // columns of a row segment (rows wider than one workgroup)
struct RowCoef {
    float n0[2], n1[2], m1[2], m2[2], d1[2], d2[2];
    float pw[2][10][4];        // Phi^(L 2^j), j = 0..9, row-major (chunk distances 1 .. 512)
    float hom[kRowMaxL][4];    // first rows of Phi_0^(i+1) and Phi_1^(i+1): the homogeneous
                               // response i samples after a state, (alpha_0, beta_0, alpha_1, beta_1)
};

// LDS of hrow2 in floats: the power matrices Phi^(L 2^j) (2 x 10 x 4), the
// homogeneous-response table (16 x 4), the per-lane power table (16 x 8), the
// per-row power table (4 x 8), the wave totals of every group
// (double-buffered, 2 x 8 x 8 each); then as doubles the centred intensities
// of the row (T rows of L + 1, one pad) and, with groups, the hand-over of one
// group at a time to group 0 (2 per pixel); then the top channel's filtered
// row (T rows of L + 1 floats).
constexpr int kRowSmemHead = 80 + 4 * kRowMaxL + 128 + 32;
__host__ __device__ constexpr size_t hrow2_smem_bytes(int T, int groups, int L) {
    return sizeof(float) * ((size_t)kRowSmemHead + (size_t)groups * 128 + (size_t)T * (L + 1)) +
           sizeof(double) * ((size_t)T * (L + 1) + (groups > 1 ? 2 * (size_t)T * (size_t)L : 0));
}

// s[0..1] += P * (v0, v1), P a 2x2 matrix (row-major) in LDS
__device__ __forceinline__ void acc2v(float *s, const float *P, float v0, float v1) {
    const float4 m = *(const float4 *)P;
    s[0] = fmaf(m.x, v0, fmaf(m.y, v1, s[0]));
    s[1] = fmaf(m.z, v0, fmaf(m.w, v1, s[1]));
}

__device__ __forceinline__ float bperm_f(float v, int src_lane) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}

// One image row (see the file comment).  The workgroup holds `groups` channel
// groups of T threads (T a multiple of 64, T L >= W, groups * T <= 512,
// T <= 512, L <= kRowMaxL);
// group g filters channels [C g / groups, C (g + 1) / groups).
// S: the column-filtered stack, channel n row r at S + (n * sp_rows + r) *
// sp_pitch; columns W .. sp_pitch - 1 hold zeros and sp_pitch >= T L + 2.
// sm: hrow2_smem_bytes(T, groups, L) bytes.  foff: element offset of the image
// and output rows (a volume's frame).
//
// Rows wider than one workgroup's T L samples are cut into segments of T L
// (T = 512, L = 16): MODE 1 runs a segment from rest and stores its end states
// (the causal state at its end and the anticausal one at its start, per
// channel) in segst; MODE 2 then filters each segment with the incoming
// states of the segments before and after it (the end states moved over the
// segments between by Phi^(T L)), added to the states its waves hand over.
// segst: [row][segment][channel][8].  MODE 0: one segment per row.
//
// SAVE (one channel group, MODE 0): the Horner scheme carries a third chain,
// e <- e tau + c, which ends at P''/2, and the terms the backward pass needs
// are stored: rho = M/D, drho/dtau = (M' - rho D') / D with M' = P'' and
// D' = P' - (N+1) a_{N+1} tau^N (the derivatives in tau with the filtered
// channels held fixed), and D itself (= exp(tau^2/2) times eq. (11)'s
// denominator).
template <int L, int MODE = 0, bool SAVE = false>
__device__ __forceinline__ void hrow2(const GPParams &p, const RowCoef &c, const Stats &st, int y,
                                      const float *__restrict__ S, int sp_rows, int sp_pitch, float *sm, int T,
                                      int groups, size_t foff = 0, int seg = 0, int nseg = 1,
                                      float *segst = nullptr) {
    const int g = __builtin_amdgcn_readfirstlane((int)threadIdx.x / T);  // whole waves share a group
    const int t = threadIdx.x - g * T;
    const int lane = threadIdx.x & 63, jj = lane & 15;
    const int nw = T >> 6;  // waves in a group
    const int wv = t >> 6;  // this chunk's wave in the group
    const int r16 = lane >> 4;  // this chunk's row of 16 lanes in the wave
    const int x0 = (seg * T + t) * L;
    // where the chunk's stack samples are read: chunks wholly past the row end
    // read the zero pad at the row width rounded up to 4 (the stack is no
    // wider than the row plus that pad)
    const int xl = x0 < p.W ? x0 : ((p.W + 3) & ~3);
    const int cb = (p.C * g) / groups, ce = (p.C * (g + 1)) / groups;
    const int steps = (p.C + groups - 1) / groups;  // channels of the largest group
    float *pws = sm;                      // pws[(10 s + j) * 4 + q] = Phi_s^(L 2^j)
    float *homs = sm + 80;                // homs[i * 4 + q] = c.hom[i][q]
    float *Gt = homs + 4 * kRowMaxL;      // Gt[jj * 8 + 4 s + q] = Phi_s^(L jj)
    float *Gw = Gt + 128;                 // Gw[r * 8 + 4 s + q] = Phi_s^(16 L r), r = 0..3
    float *wtot = sm + kRowSmemHead + (size_t)g * 128;  // [2][8 waves][8]
    // per-thread rows of L + 1 (the odd stride puts the lanes of a wave on
    // distinct banks; a thread's L values sit at immediate offsets)
    double *taus = (double *)(sm + kRowSmemHead + (size_t)groups * 128) + (size_t)t * (L + 1);  // taus[i]
    double *comb = (double *)(sm + kRowSmemHead + (size_t)groups * 128) + (size_t)T * (L + 1);
    float *otop = (float *)(comb + (groups > 1 ? 2 * (size_t)T * L : 0)) + (size_t)t * (L + 1);  // otop[i]

    // the coefficient tables go through LDS (as kernel arguments held in
    // scalar registers they would spill)
    for (int k = threadIdx.x; k < 80 + 4 * kRowMaxL; k += blockDim.x)
        sm[k] = k < 80 ? (&c.pw[0][0][0])[k] : (&c.hom[0][0])[k - 80];
    if (threadIdx.x < 16) {
        const int k = threadIdx.x;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            float G[4] = {1.f, 0.f, 0.f, 1.f};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (k & (1 << j)) mat_mul(G, c.pw[s][j], G);
#pragma unroll
            for (int q = 0; q < 4; ++q) Gt[k * 8 + 4 * s + q] = G[q];
            if (k < 4) {
                float H[4] = {1.f, 0.f, 0.f, 1.f};
                if (k & 1) mat_mul(H, c.pw[s][4], H);
                if (k & 2) mat_mul(H, c.pw[s][5], H);
#pragma unroll
                for (int q = 0; q < 4; ++q) Gw[k * 8 + 4 * s + q] = H[q];
            }
        }
    }
    if (g == 0) {
        // centred intensities of the row (unconditional loads from clamped
        // columns, zero past the row end)
        const float *irow = p.img + foff + (size_t)y * p.pitch;
        float f[L];
#pragma unroll
        for (int i = 0; i < L; ++i) f[i] = irow[x0 + i < p.W ? x0 + i : p.W - 1];
#pragma unroll
        for (int i = 0; i < L; ++i)
            taus[i] = x0 + i < p.W ? (double)centred(f[i], st, p.inv_sigma_r) : 0.0;
    }
    __syncthreads();

    double bP[L], bC[L];  // Horner accumulators of P and P' (relative to tau^cb)
    double bS[SAVE ? L : 1];  // SAVE: P''/2
#pragma unroll
    for (int i = 0; i < L; ++i) {
        bP[i] = 0.0;
        bC[i] = 0.0;
        if constexpr (SAVE) bS[i] = 0.0;
    }
    // 1 / sqrt(n!) of the group's first (highest) channel, then divided by
    // sqrt(n) at every step down
    double kap = 1.0;
    for (int n = 2; n < ce; ++n) kap *= p.isq[n];
    const double ktop = kap;  // 1 / sqrt((N+1)!) in the group holding channel N+1

    // samples x0-1 .. x0+L+1 of channel n's stack row (columns W .. pitch-1
    // are zero pad; only the sample left of the row start is masked).  The
    // next channel's samples are loaded while the current one is filtered.
    auto load = [&](float *z, int n) {
        const float *srow = S + ((size_t)n * sp_rows + y) * sp_pitch;
        z[0] = srow[xl > 0 ? xl - 1 : 0];
#pragma unroll
        for (int i = 0; i < L; i += 4) {
            const float4 q = *(const float4 *)(srow + xl + i);
            z[1 + i] = q.x; z[2 + i] = q.y; z[3 + i] = q.z; z[4 + i] = q.w;
        }
        z[L + 1] = srow[xl + L];
        z[L + 2] = srow[xl + L + 1];
    };
    // one channel step: z holds channel n = ce - 1 - it, zn receives n - 1
    auto step = [&](float *z, float *zn, int it) {
        const int n = ce - 1 - it;
        const bool act = n >= cb;  // uniform over the group
        float o[L];
        float sc[4], sa[4];
        if (act) {
            if (n - 1 >= cb) load(zn, n - 1);
            z[0] = x0 > 0 ? z[0] : 0.f;
            // 1. the chunk from rest
            {
                float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f};
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    float v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float b = fmaf(c.n0[s], z[i + 1], fmaf(c.n1[s], z[i], -c.d2[s] * y2[s]));
                        v[s] = fmaf(-c.d1[s], y1[s], b);
                        y2[s] = y1[s];
                        y1[s] = v[s];
                    }
                    o[i] = v[0] + v[1];
                }
                sc[0] = y1[0]; sc[1] = y2[0]; sc[2] = y1[1]; sc[3] = y2[1];
            }
            {
                float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f};
#pragma unroll
                for (int i = L - 1; i >= 0; --i) {
                    float v[2];
#pragma unroll
                    for (int s = 0; s < 2; ++s) {
                        const float b = fmaf(c.m1[s], z[i + 2], fmaf(c.m2[s], z[i + 3], -c.d2[s] * z2[s]));
                        v[s] = fmaf(-c.d1[s], z1[s], b);
                        z2[s] = z1[s];
                        z1[s] = v[s];
                    }
                    o[i] += v[0] + v[1];
                }
                sa[0] = z1[0]; sa[1] = z2[0]; sa[2] = z1[1]; sa[3] = z2[1];
            }
            // 2a. inclusive scans inside each row of 16 lanes: causal from the
            // left (row_shr), anticausal from the right (row_shl)
#define BF_ROWSTEP2(J, D)                                                                  \
            {                                                                              \
                float pc[4], pa[4];                                                        \
                _Pragma("unroll") for (int q = 0; q < 4; ++q) {                            \
                    pc[q] = dpp_f<kDppRowShr + D>(sc[q]);                                  \
                    pa[q] = dpp_f<kDppRowShl + D>(sa[q]);                                  \
                }                                                                          \
                _Pragma("unroll") for (int s = 0; s < 2; ++s) {                            \
                    acc2v(&sc[2 * s], pws + (10 * s + J) * 4, pc[2 * s], pc[2 * s + 1]);   \
                    acc2v(&sa[2 * s], pws + (10 * s + J) * 4, pa[2 * s], pa[2 * s + 1]);   \
                }                                                                          \
            }
            BF_ROWSTEP2(0, 1)
            BF_ROWSTEP2(1, 2)
            BF_ROWSTEP2(2, 4)
            BF_ROWSTEP2(3, 8)
#undef BF_ROWSTEP2
        }
        // 2b. the four rows of the wave: lane r (r < 4) takes row r's totals
        // (the causal one ends at its lane 15, the anticausal one at its lane
        // 0) and the lanes scan them (DPP, distances 1 and 2 rows)
        float rc[4], ra[4];
        if (act) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rc[q] = bperm_f(sc[q], (lane & 3) * 16 + 15);
                ra[q] = bperm_f(sa[q], (lane & 3) * 16);
                rc[q] = lane < 4 ? rc[q] : 0.f;
                ra[q] = lane < 4 ? ra[q] : 0.f;
            }
#define BF_L2STEP(J, D)                                                                      \
            {                                                                                \
                float pc[4], pa[4];                                                          \
                _Pragma("unroll") for (int q = 0; q < 4; ++q) {                              \
                    pc[q] = dpp_f<kDppRowShr + D>(rc[q]);                                    \
                    pa[q] = dpp_f<kDppRowShl + D>(ra[q]);                                    \
                }                                                                            \
                _Pragma("unroll") for (int s = 0; s < 2; ++s) {                              \
                    acc2v(&rc[2 * s], pws + (10 * s + J) * 4, pc[2 * s], pc[2 * s + 1]);     \
                    acc2v(&ra[2 * s], pws + (10 * s + J) * 4, pa[2 * s], pa[2 * s + 1]);     \
                }                                                                            \
            }
            BF_L2STEP(4, 1)
            BF_L2STEP(5, 2)
        }
        // 2c. across the waves of the group: wave totals through LDS (lane 3
        // holds the causal total of the wave, lane 0 the anticausal one), a
        // DPP scan over the waves (distances 1, 2, 4), and the wave's
        // incoming states (uniform).  Every wave meets the barrier.
        float wc[4] = {0.f, 0.f, 0.f, 0.f}, wa[4] = {0.f, 0.f, 0.f, 0.f};
        if (nw > 1) {
            float *tb = wtot + (it & 1) * 64;
            if (act && lane == 3) *(float4 *)(tb + wv * 8) = make_float4(rc[0], rc[1], rc[2], rc[3]);
            if (act && lane == 0) *(float4 *)(tb + wv * 8 + 4) = make_float4(ra[0], ra[1], ra[2], ra[3]);
            __syncthreads();
            if (act) {
                const int l = lane < nw ? lane : 0;
                const float4 c4 = *(const float4 *)(tb + l * 8), a4 = *(const float4 *)(tb + l * 8 + 4);
                const bool in = lane < nw;
                float xc[4] = {in ? c4.x : 0.f, in ? c4.y : 0.f, in ? c4.z : 0.f, in ? c4.w : 0.f};
                float xa[4] = {in ? a4.x : 0.f, in ? a4.y : 0.f, in ? a4.z : 0.f, in ? a4.w : 0.f};
#define BF_WSTEP(J, D)                                                                       \
                if (D < nw) {                                                                \
                    float pc[4], pa[4];                                                      \
                    _Pragma("unroll") for (int q = 0; q < 4; ++q) {                          \
                        pc[q] = dpp_f<kDppRowShr + D>(xc[q]);                                \
                        pa[q] = dpp_f<kDppRowShl + D>(xa[q]);                                \
                    }                                                                        \
                    _Pragma("unroll") for (int s = 0; s < 2; ++s) {                          \
                        acc2v(&xc[2 * s], pws + (10 * s + J) * 4, pc[2 * s], pc[2 * s + 1]); \
                        acc2v(&xa[2 * s], pws + (10 * s + J) * 4, pa[2 * s], pa[2 * s + 1]); \
                    }                                                                        \
                }
                BF_WSTEP(6, 1)
                BF_WSTEP(7, 2)
                BF_WSTEP(8, 4)
#undef BF_WSTEP
                if constexpr (MODE == 1) {
                    // the segment's end states: the causal one after its
                    // last wave, the anticausal one before its first
                    float *sg = segst + (((size_t)y * nseg + seg) * p.C + n) * 8;
                    if (wv == 0 && lane == nw - 1) *(float4 *)sg = make_float4(xc[0], xc[1], xc[2], xc[3]);
                    if (wv == 0 && lane == 0) *(float4 *)(sg + 4) = make_float4(xa[0], xa[1], xa[2], xa[3]);
                }
                // exclusive: the waves before (causal) and after (anticausal)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    xc[q] = dpp_f<kDppRowShr + 1>(xc[q]);
                    xa[q] = dpp_f<kDppRowShl + 1>(xa[q]);
                    wc[q] = lane_f(xc[q], wv);
                    wa[q] = lane_f(xa[q], wv);
                }
                if constexpr (MODE == 2) {
                    // the segment's incoming states from the segments before
                    // and after it, moved over this wave's place in it
                    float ci[4] = {0.f, 0.f, 0.f, 0.f}, ai[4] = {0.f, 0.f, 0.f, 0.f};
                    const float *sr = segst + ((size_t)y * nseg * p.C + n) * 8;
                    const size_t sstep = (size_t)p.C * 8;
                    for (int j = 0; j < seg; ++j) {
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2) {
                            float r2[2];
                            affine2(r2, sr + j * sstep + 2 * s2, pws + (10 * s2 + 9) * 4, &ci[2 * s2]);
                            ci[2 * s2] = r2[0];
                            ci[2 * s2 + 1] = r2[1];
                        }
                    }
                    for (int j = nseg - 1; j > seg; --j) {
#pragma unroll
                        for (int s2 = 0; s2 < 2; ++s2) {
                            float r2[2];
                            affine2(r2, sr + j * sstep + 4 + 2 * s2, pws + (10 * s2 + 9) * 4, &ai[2 * s2]);
                            ai[2 * s2] = r2[0];
                            ai[2 * s2 + 1] = r2[1];
                        }
                    }
#pragma unroll
                    for (int s2 = 0; s2 < 2; ++s2) {
                        float Mc[4] = {1.f, 0.f, 0.f, 1.f}, Ma[4] = {1.f, 0.f, 0.f, 1.f};
                        const int wa_ = nw - 1 - wv;
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            if (wv & (1 << b)) mat_mul(Mc, pws + (10 * s2 + 6 + b) * 4, Mc);
                            if (wa_ & (1 << b)) mat_mul(Ma, pws + (10 * s2 + 6 + b) * 4, Ma);
                        }
                        acc2(&wc[2 * s2], Mc, ci[2 * s2], ci[2 * s2 + 1]);
                        acc2(&wa[2 * s2], Ma, ai[2 * s2], ai[2 * s2 + 1]);
                    }
                }
            }
        }
        if constexpr (MODE == 1) return;
        if (!act) return;
        // row-exclusive incoming states of the wave's rows (lanes 0..3): the
        // rows before (after) inside the wave plus the wave's incoming state
        // moved over the rows between; then each chunk fetches its row's
        float qc[4], qa[4];
        {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                qc[q] = dpp_f<kDppRowShr + 1>(rc[q]);
                qa[q] = dpp_f<kDppRowShl + 1>(ra[q]);
            }
            const int rr = lane & 3;
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                acc2v(&qc[2 * s], Gw + rr * 8 + 4 * s, wc[2 * s], wc[2 * s + 1]);
                acc2v(&qa[2 * s], Gw + (3 - rr) * 8 + 4 * s, wa[2 * s], wa[2 * s + 1]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                qc[q] = bperm_f(qc[q], r16);
                qa[q] = bperm_f(qa[q], r16);
            }
        }
        // incoming states of this chunk: the row-exclusive prefix inside the
        // row (a shift by one lane) plus the row's incoming state moved over
        // the chunks between
        float ic[4], ia[4];
        // (the power tables are read from LDS at their use: an opaque zero
        // keeps the reads from being hoisted out of the channel loop, where
        // they would hold 16 registers)
        int jz0 = 0;
        asm volatile("" : "+s"(jz0));
        const int jz = jj + jz0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ic[q] = dpp_f<kDppRowShr + 1>(sc[q]);
            ia[q] = dpp_f<kDppRowShl + 1>(sa[q]);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            acc2v(&ic[2 * s], Gt + jz * 8 + 4 * s, qc[2 * s], qc[2 * s + 1]);
            acc2v(&ia[2 * s], Gt + (15 - jj + jz0) * 8 + 4 * s, qa[2 * s], qa[2 * s + 1]);
        }
        // 3. homogeneous responses of the incoming states: the response i
        // samples after a state (a1, a2) of section s is alpha a1 + beta a2,
        // (alpha, beta) the first row of Phi_s^(i+1) (four table entries per
        // i; the anticausal states act from the chunk's right end).  The
        // opaque zero keeps the table reads at their use (hoisted out of the
        // loop they would hold 64 registers).
        {
            int z0 = 0;
            asm volatile("" : "+s"(z0));
            const float *hp = homs + z0;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const float4 h = *(const float4 *)(hp + 4 * i);
                o[i] = fmaf(h.x, ic[0], fmaf(h.y, ic[1], o[i]));
                o[i] = fmaf(h.z, ic[2], fmaf(h.w, ic[3], o[i]));
                o[L - 1 - i] = fmaf(h.x, ia[0], fmaf(h.y, ia[1], o[L - 1 - i]));
                o[L - 1 - i] = fmaf(h.z, ia[2], fmaf(h.w, ia[3], o[L - 1 - i]));
            }
        }
        // the top channel's row is kept for taking its term out of D
        if (n == p.N + 1) {
#pragma unroll
            for (int i = 0; i < L; ++i) otop[i] = o[i];
        }
        // Horner step of P and P' (the same for every channel)
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const double tv = taus[i];
            if constexpr (SAVE) bS[i] = fma(bS[i], tv, bC[i]);
            bC[i] = fma(bC[i], tv, bP[i]);
            // bP tau + kap o with the product bP tau rounded: both updates
            // then stay in their own registers
            bP[i] = fma(kap, (double)o[i], bP[i] * tv);
        }
        kap *= p.sq[n];  // 1 / sqrt((n-1)!)
    };
    float zn[L + 3];
    if (ce - 1 >= cb) load(zn, ce - 1);
    for (int it = 0; it < steps; ++it) {
        float z[L + 3];
#pragma unroll
        for (int i = 0; i < L + 3; ++i) z[i] = zn[i];
        step(z, zn, it);
    }
    if constexpr (MODE == 1) return;
    // D of this group: P without the top channel's term (the group holding
    // channel N+1 subtracts a_{N+1} tau^(N+1-cb); uniform branch)
    double bD[L];
#pragma unroll
    for (int i = 0; i < L; ++i) bD[i] = bP[i];
    if (ce == p.C) {
        const int e = p.N + 1 - cb;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const double tv = taus[i];
            bD[i] = fma(-(ktop * (double)otop[i]), ipow(tv, e), bP[i]);
        }
    }
    if (groups > 1) {
        // the parts of groups 1.. in the full sums, handed to group 0 one
        // group at a time through one LDS buffer and added in group order
        for (int gg = 1; gg < groups; ++gg) {
            if (g == gg) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    const double tv = taus[i];
                    const double tp = ipow(tv, cb - 1);  // tau^(cb - 1)
                    comb[(size_t)(2 * i) * T + t] = bD[i] * (tp * tv);
                    comb[(size_t)(2 * i + 1) * T + t] = (double)cb * tp * bP[i] + tp * tv * bC[i];
                }
            }
            __syncthreads();
            if (g == 0) {
#pragma unroll
                for (int i = 0; i < L; ++i) {
                    bD[i] += comb[(size_t)(2 * i) * T + t];
                    bC[i] += comb[(size_t)(2 * i + 1) * T + t];
                }
            }
            __syncthreads();
        }
    }
    if (g == 0 && y < p.H) {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            const int x = x0 + i;
            if (x < p.W) {
                const double rho = bC[i] / bD[i];
                p.out[foff + (size_t)y * p.pitch + x] = st.ok ? (float)fma(p.sigma_r, rho, st.tc) : __builtin_nanf("");
                if constexpr (SAVE) {
                    // one group (cb = 0): D' = P' - (N+1) a_{N+1} tau^N
                    const double tv = taus[i];
                    const double a = ktop * (double)otop[i];
                    const double dD = fma(-(double)(p.N + 1) * a, ipow(tv, p.N), bC[i]);
                    const size_t npx = (size_t)p.H * p.W, idx = (size_t)y * p.W + x;
                    float *sv = (float *)p.saved;
                    sv[idx] = (float)rho;
                    sv[npx + idx] = (float)((2.0 * bS[i] - rho * dD) / bD[i]);
                    ((double *)(sv + 2 * npx))[idx] = bD[i];
                }
            }
        }
    }
}

}  // namespace bfgp
