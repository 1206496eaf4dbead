// Backward of the GP forward in the recursive (IIR) spatial mode.
//
// The chain rule is the one of the FIR backward (eqs. (7)-(11) and the mean
// that Algorithm 1 takes as the centre): with a = g sigma_r / D' and p_n = tau^n / sqrt(n!),
//   V_n = a [ sqrt(n) p_{n-1}(tau) - rho p_n(tau) [n <= N] ],  n = 0..N+1,
//   W_n = K V_n,   Z_n = dK/dlog(sigma_s) V_n,
//   gH(j) = sum_n W_n(j) u_n'(x_j) + g(j) sigma_r drho/dtau(j),
//   dL/dlog sigma_s = sum_n sum_j Z_n(j) u_n(x_j).
// K is Deriche's zero-extended convolution with h(|d| / sigma_s) along each
// axis; h is even, so K is symmetric and its adjoint is K itself.  Its
// derivative in log sigma_s is obtained by differentiating the recursion:
// every second-order section carries, beside its state (y_{n-1}, y_{n-2}), the
// tangent state (y'_{n-1}, y'_{n-2}) of
//   y'_n = n0 x'_n + n1 x'_{n-1} + n1' x_{n-1} - d1' y_{n-1} - d2' y_{n-2}
//          - d1 y'_{n-1} - d2 y'_{n-2},
// whose impulse response is d h(|d| / sigma_s) / d log sigma_s (n0 does not
// depend on sigma_s).  Along columns the input has no tangent (x' = 0): the
// pass yields P = k_y V and Q = k_y' V.  Along rows the input is the pair
// (P, Q): the pass yields W = k_x P and Z = k_x' P + k_x Q.
//
// Both axes use the band scheme of the forward column pass (bands from rest,
// a sequential resolve of the band carries with the band transfer matrix
// [[Phi^B, 0], [Psi_B, Phi^B]], bands rerun from their true states) with one
// lane per line, so the column pass writes P and Q transposed (PT[n][x][y])
// and the row pass reads them with lanes along y, coalesced.
//
// The contraction uses u_n' = sqrt(n) u_{n-1} - sqrt(n+1) u_{n+1}, u_n =
// e^{-tau^2/2} p_n, so that
//   sum_n W_n u_n' = e^{-tau^2/2} (S1 - tau S2),  sum_n Z_n u_n = e^{-tau^2/2} S3,
//   S1 = sum_{n>=1} sqrt(n) W_n p_{n-1},  S2 = sum_n W_n p_n,  S3 = sum_n Z_n p_n,
// three power series in tau, each evaluated by Horner (double) over the
// channels of a group in descending order; group g (channels cb..ce-1) holds
// its sums relative to p_cb (p_{cb-1} for S1) and is scaled by p_cb(tau) =
// tau^cb / sqrt(cb!) before the groups are added in a fixed order.  Channel
// groups split both passes when the image gives too few waves; the channel
// recurrence of the column pass then starts from p_{cb-1} directly.
#pragma once
#include "common.hpp"
#include "bwd.hpp"
#include "iir.hpp"

namespace bfgp {

constexpr int kBwdBV = 16;  // band rows of the column pass
constexpr int kBwdBH = 16;  // band columns of the row pass

// Section coefficients (as in IirCoef), their derivatives in log sigma_s, and
// the band transfer blocks for both band lengths (row-major 2x2).
struct IirTan {
    float n0[2], n1[2], m1[2], m2[2], d1[2], d2[2];
    float tn1[2], tm1[2], tm2[2], td1[2], td2[2];
    float phiV[2][4], psiV[2][4];  // bands of kBwdBV
    float phiH[2][4], psiH[2][4];  // bands of kBwdBH
};

// Per-call arguments of the IIR backward.
struct BwdIir {
    const float *grad_out;  // H x W, image pitch
    const float *rho;       // saved: M/D, H x W packed
    const float *drho;      // saved: d(M/D)/dtau, packed
    const double *Dp;       // saved: exp(tau^2/2) D, packed
    float *grad_img;        // nullable, image pitch
    float *cv;              // column carries [nbv][C][16][W]
    float *PT, *QT;         // transposed stacks [C][W][Hp]
    float *chz;             // row carries [nbh][C][16][Hp]
    BwdPartial *bparts;     // one per row-pass workgroup
    int Hp;                 // rows of the transposed stacks: H rounded up to 64
    int Gv, Gh;             // channel groups of the column and the row passes
};

// 1 / sqrt(k!) (k uniform over the wave); p_k(x) = x^k / sqrt(k!) is
// ipow(x, k) times it.
__device__ __forceinline__ double inv_sqrt_fact(const GPParams &p, int k) {
    double c = 1.0;
    for (int j = 1; j <= k; ++j) c *= p.isq[j];
    return c;
}

// LDS bytes of the row pass with G channel groups in one workgroup: the
// scaled sums (S1, S2, S3) of groups 1..G-1 for every lane and sample.
__host__ __device__ constexpr size_t bhband_smem_bytes(int G, int B) {
    return sizeof(double) * 3 * (size_t)(G > 1 ? G - 1 : 0) * (size_t)B * 64;
}

// One step of a causal section with its tangent.  (y1, y2, t1, t2) is the
// state; xc, xp are the current and previous inputs, tc, tp their tangents.
template <bool TIN>
__device__ __forceinline__ void tstep(const IirTan &c, int s, float xc, float xp, float tc, float tp, float &y1,
                                      float &y2, float &t1, float &t2, float &yo, float &to) {
    const float y = fmaf(-c.d1[s], y1, fmaf(c.n0[s], xc, fmaf(c.n1[s], xp, -c.d2[s] * y2)));
    float t = fmaf(c.tn1[s], xp, fmaf(-c.td1[s], y1, fmaf(-c.td2[s], y2, fmaf(-c.d1[s], t1, -c.d2[s] * t2))));
    if (TIN) t = fmaf(c.n0[s], tc, fmaf(c.n1[s], tp, t));
    y2 = y1;
    y1 = y;
    t2 = t1;
    t1 = t;
    yo = y;
    to = t;
}
// The same for an anticausal section: x1, x2 are the inputs one and two
// samples ahead, s1, s2 their tangents.
template <bool TIN>
__device__ __forceinline__ void astep(const IirTan &c, int s, float x1, float x2, float s1, float s2, float &z1,
                                      float &z2, float &t1, float &t2, float &zo, float &to) {
    const float z = fmaf(-c.d1[s], z1, fmaf(c.m1[s], x1, fmaf(c.m2[s], x2, -c.d2[s] * z2)));
    float t = fmaf(c.tm1[s], x1, fmaf(c.tm2[s], x2, fmaf(-c.td1[s], z1, fmaf(-c.td2[s], z2, fmaf(-c.d1[s], t1, -c.d2[s] * t2)))));
    if (TIN) t = fmaf(c.m1[s], s1, fmaf(c.m2[s], s2, t));
    z2 = z1;
    z1 = z;
    t2 = t1;
    t1 = t;
    zo = z;
    to = t;
}

// Column pass over the adjoint channels V_n of one band of B rows in one
// column.  AGG: run from rest and store the band's end states.  !AGG: run
// from the resolved states and write P_n, Q_n transposed.
// Carry layout: cv[((band * C + n) * 16 + k) * W + col]; k = 4 s + {0,1,2,3}
// = (y_{e}, y_{e-1}, y'_{e}, y'_{e-1}) of causal section s, k = 8 + 4 s + ..
// the same for the anticausal section (z_a, z_{a+1}, z'_a, z'_{a+1}).
// tile: LDS of 2 * B * 65 floats (the band of P and Q for the wave's 64
// columns, used for the transposed store).
template <int B, bool AGG>
__device__ __forceinline__ void bvband(const GPParams &p, const BwdIir &b, const IirTan &c, const Stats &st, int col0,
                                       int band, int cb, int ce, float *tile) {
    const int lane = threadIdx.x & 63;
    const int col = col0 + lane;
    const bool live = col < p.W;
    const int cl = live ? col : p.W - 1;
    const int a = band * B;
    // per-sample terms of rows a-1 .. a+B+1 (loads from clamped rows, masked):
    // x, rho and s = a p_{n-1} (double; a itself can leave the float range)
    double s[B + 3];
    float xr[B + 3], rr[B + 3];
#pragma unroll
    for (int i = 0; i < B + 3; ++i) {
        const int row = a - 1 + i;
        const int rc = row < 0 ? 0 : (row >= p.H ? p.H - 1 : row);
        const size_t pi = (size_t)rc * p.pitch + cl, qi = (size_t)rc * p.W + cl;
        const float f = p.img[pi];
        const float g = b.grad_out[pi];
        const float r = b.rho[qi];
        const double dp = b.Dp[qi];
        const bool in = live && row >= 0 && row < p.H;
        xr[i] = in ? centred(f, st, p.inv_sigma_r) : 0.f;
        rr[i] = in ? r : 0.f;
        s[i] = in ? (double)g * p.sigma_r / dp : 0.0;
    }
    // a p_{cb-1} by the products the channels 1 .. cb-1 would apply in turn,
    // so that every column grouping rounds the adjoint channels alike
    for (int j = 1; j < cb; ++j) {
        const double isqj = p.isq[j];
#pragma unroll
        for (int i = 0; i < B + 3; ++i) s[i] *= (double)xr[i] * isqj;
    }
    float *tp = tile, *tq = tile + B * 65;
    // the incoming states of the next channel are read while the current one
    // is filtered (the rerun only)
    float cinn[AGG ? 1 : 16];
    auto load_in = [&](int n) {
        const float *cq = b.cv + ((size_t)(band * p.C + n) * 16) * p.W + cl;
#pragma unroll
        for (int k = 0; k < 16; ++k) cinn[k] = cq[(size_t)k * p.W];
    };
    if (!AGG && ce > cb) load_in(cb);
    for (int n = cb; n < ce; ++n) {
        float cin[AGG ? 1 : 16];
        if constexpr (!AGG) {
#pragma unroll
            for (int k = 0; k < 16; ++k) cin[k] = cinn[k];
            if (n + 1 < ce) load_in(n + 1);
        }
        float v[B + 3];
        if (n == 0) {
#pragma unroll
            for (int i = 0; i < B + 3; ++i) v[i] = (float)(-(double)rr[i] * s[i]);  // -rho a p_0
        } else {
            // a p_{n-1} (sqrt(n) - rho x / sqrt(n) [n <= N]), then s -> a p_n
            const double sqn = p.sq[n], isqn = p.isq[n];
            const bool inD = n <= p.N;
#pragma unroll
            for (int i = 0; i < B + 3; ++i) {
                const double f = inD ? fma(-(double)rr[i] * (double)xr[i], isqn, sqn) : sqn;
                v[i] = (float)(s[i] * f);
                s[i] *= (double)xr[i] * isqn;
            }
        }
        float *cp = b.cv + ((size_t)(band * p.C + n) * 16) * p.W + cl;
        const size_t cs = (size_t)p.W;
        // causal
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f}, t1[2] = {0.f, 0.f}, t2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    y1[q] = cin[4 * q + 0];
                    y2[q] = cin[4 * q + 1];
                    t1[q] = cin[4 * q + 2];
                    t2[q] = cin[4 * q + 3];
                }
            }
#pragma unroll
            for (int i = 0; i < B; ++i) {
                float yo[2], to[2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    tstep<false>(c, q, v[i + 1], v[i], 0.f, 0.f, y1[q], y2[q], t1[q], t2[q], yo[q], to[q]);
                if constexpr (!AGG) {
                    tp[i * 65 + lane] = yo[0] + yo[1];
                    tq[i * 65 + lane] = to[0] + to[1];
                }
            }
            if (AGG && live) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    cp[(4 * q + 0) * cs] = y1[q];
                    cp[(4 * q + 1) * cs] = y2[q];
                    cp[(4 * q + 2) * cs] = t1[q];
                    cp[(4 * q + 3) * cs] = t2[q];
                }
            }
        }
        // anticausal
        {
            float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f}, t1[2] = {0.f, 0.f}, t2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    z1[q] = cin[8 + 4 * q + 0];
                    z2[q] = cin[8 + 4 * q + 1];
                    t1[q] = cin[8 + 4 * q + 2];
                    t2[q] = cin[8 + 4 * q + 3];
                }
            }
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                float zo[2], to[2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    astep<false>(c, q, v[i + 2], v[i + 3], 0.f, 0.f, z1[q], z2[q], t1[q], t2[q], zo[q], to[q]);
                if constexpr (!AGG) {
                    tp[i * 65 + lane] += zo[0] + zo[1];
                    tq[i * 65 + lane] += to[0] + to[1];
                }
            }
            if (AGG && live) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    cp[(8 + 4 * q + 0) * cs] = z1[q];
                    cp[(8 + 4 * q + 1) * cs] = z2[q];
                    cp[(8 + 4 * q + 2) * cs] = t1[q];
                    cp[(8 + 4 * q + 3) * cs] = t2[q];
                }
            }
        }
        if (!AGG) {
            // transposed store: stack row x = col0 + j holds rows a .. a+B-1
            // of the band; 8 lanes cover one row segment with 16-byte stores
            __syncthreads();
            constexpr int SEG = B / 4;        // lanes per row segment
            constexpr int RPI = 64 / SEG;     // row segments per instruction
            const int q4 = (lane % SEG) * 4;
#pragma unroll
            for (int k = 0; k < 64 / RPI; ++k) {
                const int j = lane / SEG + k * RPI;
                const int x = col0 + j;
                if (x < p.W) {
                    float4 P4, Q4;
                    P4.x = tp[(q4 + 0) * 65 + j]; P4.y = tp[(q4 + 1) * 65 + j];
                    P4.z = tp[(q4 + 2) * 65 + j]; P4.w = tp[(q4 + 3) * 65 + j];
                    Q4.x = tq[(q4 + 0) * 65 + j]; Q4.y = tq[(q4 + 1) * 65 + j];
                    Q4.z = tq[(q4 + 2) * 65 + j]; Q4.w = tq[(q4 + 3) * 65 + j];
                    const size_t o = ((size_t)n * p.W + x) * (size_t)b.Hp + a + q4;
                    *(float4 *)(b.PT + o) = P4;
                    *(float4 *)(b.QT + o) = Q4;
                }
            }
            __syncthreads();
        }
    }
}

// Resolves the true incoming states of every band for one line, one channel
// and one direction (dir 0 causal, bands in order; dir 1 anticausal, bands in
// reverse), in place: state_{k+1} = A^B state_k + rest_k per section, with
// A^B = [[phi, 0], [psi, phi]] acting on (y1, y2, t1, t2).
__device__ __forceinline__ void bresolve(const float (*phi)[4], const float (*psi)[4], int nb, int C, int n,
                                         int dir, size_t lines, size_t line, float *__restrict__ carry) {
    float st[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int kk = 0; kk < nb; ++kk) {
        const int k = dir == 0 ? kk : nb - 1 - kk;
        float *cp = carry + ((size_t)(k * C + n) * 16 + 8 * dir) * lines + line;
        float l[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) l[j] = cp[j * lines];
#pragma unroll
        for (int j = 0; j < 8; ++j) cp[j * lines] = st[j];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const float *P = phi[q], *S = psi[q];
            const float y1 = st[4 * q], y2 = st[4 * q + 1], t1 = st[4 * q + 2], t2 = st[4 * q + 3];
            st[4 * q + 0] = fmaf(P[0], y1, fmaf(P[1], y2, l[4 * q + 0]));
            st[4 * q + 1] = fmaf(P[2], y1, fmaf(P[3], y2, l[4 * q + 1]));
            st[4 * q + 2] = fmaf(S[0], y1, fmaf(S[1], y2, fmaf(P[0], t1, fmaf(P[1], t2, l[4 * q + 2]))));
            st[4 * q + 3] = fmaf(S[2], y1, fmaf(S[3], y2, fmaf(P[2], t1, fmaf(P[3], t2, l[4 * q + 3]))));
        }
    }
}

// Row pass over the transposed stacks for one band of B columns in one image
// row y (lane), channels cb..ce-1.  AGG: end states from rest into b.chz.
// !AGG: rerun from the resolved states and accumulate the group's Horner sums
// (descending channels); the workgroup holds the G groups of the same rows and
// band (wave g = group g), groups 1.. hand their scaled sums to group 0
// through `red`, and group 0 forms the image gradient and this workgroup's
// partial sums (bp).
template <int B, bool AGG>
__device__ __forceinline__ void bhband(const GPParams &p, const BwdIir &b, const IirTan &c, const Stats &st, int y,
                                       int band, int cb, int ce, int g, int G, BwdPartial *bp, double *red) {
    const int lane = threadIdx.x & 63;
    const bool live = y < p.H;
    const int yl = live ? y : p.H - 1;  // rows past the image read a real row, results discarded
    const int a = band * B;
    const size_t Hp = (size_t)b.Hp;
    double h1[AGG ? 1 : B], h2[AGG ? 1 : B], h3[AGG ? 1 : B];
    float xf[AGG ? 1 : B];
    if constexpr (!AGG) {
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int x = a + i;
            const float f = p.img[(size_t)yl * p.pitch + (x < p.W ? x : p.W - 1)];
            xf[i] = x < p.W ? centred(f, st, p.inv_sigma_r) : 0.f;
            h1[i] = 0.0;
            h2[i] = 0.0;
            h3[i] = 0.0;
        }
    }
    // channel order of the pass: ascending for the end states, descending for
    // the Horner sums; the rerun reads the incoming states of the next channel
    // while the current one is filtered (reading the stack rows ahead as well
    // measured slower: the registers cost the pass half its waves)
    auto chan = [&](int it) { return AGG ? cb + it : ce - 1 - it; };
    float cinn[AGG ? 1 : 16];
    auto load_in = [&](int n) {
        const float *cq = b.chz + ((size_t)(band * p.C + n) * 16) * Hp + yl;
#pragma unroll
        for (int k = 0; k < 16; ++k) cinn[k] = cq[k * Hp];
    };
    if (!AGG && ce > cb) load_in(chan(0));
    for (int it = 0; it < ce - cb; ++it) {
        const int n = chan(it);
        float cin[AGG ? 1 : 16];
        if constexpr (!AGG) {
#pragma unroll
            for (int k = 0; k < 16; ++k) cin[k] = cinn[k];
            if (it + 1 < ce - cb) load_in(chan(it + 1));
        }
        // samples a-1 .. a+B+1 of stack row n (clamped loads, masked)
        float P[B + 3], Q[B + 3];
        const float *pt = b.PT + (size_t)n * p.W * Hp + yl;
        const float *qt = b.QT + (size_t)n * p.W * Hp + yl;
#pragma unroll
        for (int i = 0; i < B + 3; ++i) {
            const int x = a - 1 + i;
            const int xc = x < 0 ? 0 : (x >= p.W ? p.W - 1 : x);
            P[i] = pt[(size_t)xc * Hp];
            Q[i] = qt[(size_t)xc * Hp];
        }
        if (a == 0) {
            P[0] = 0.f;
            Q[0] = 0.f;
        }
        if (a + B + 2 > p.W) {
#pragma unroll
            for (int i = 1; i < B + 3; ++i)
                if (a - 1 + i >= p.W) {
                    P[i] = 0.f;
                    Q[i] = 0.f;
                }
        }
        float *cp = b.chz + ((size_t)(band * p.C + n) * 16) * Hp + yl;
        float wc[AGG ? 1 : B], zc[AGG ? 1 : B];
        {
            float y1[2] = {0.f, 0.f}, y2[2] = {0.f, 0.f}, t1[2] = {0.f, 0.f}, t2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    y1[q] = cin[4 * q + 0];
                    y2[q] = cin[4 * q + 1];
                    t1[q] = cin[4 * q + 2];
                    t2[q] = cin[4 * q + 3];
                }
            }
#pragma unroll
            for (int i = 0; i < B; ++i) {
                float yo[2], to[2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    tstep<true>(c, q, P[i + 1], P[i], Q[i + 1], Q[i], y1[q], y2[q], t1[q], t2[q], yo[q], to[q]);
                if constexpr (!AGG) {
                    wc[i] = yo[0] + yo[1];
                    zc[i] = to[0] + to[1];
                }
            }
            if (AGG && live) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    cp[(4 * q + 0) * Hp] = y1[q];
                    cp[(4 * q + 1) * Hp] = y2[q];
                    cp[(4 * q + 2) * Hp] = t1[q];
                    cp[(4 * q + 3) * Hp] = t2[q];
                }
            }
        }
        {
            float z1[2] = {0.f, 0.f}, z2[2] = {0.f, 0.f}, t1[2] = {0.f, 0.f}, t2[2] = {0.f, 0.f};
            if (!AGG) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    z1[q] = cin[8 + 4 * q + 0];
                    z2[q] = cin[8 + 4 * q + 1];
                    t1[q] = cin[8 + 4 * q + 2];
                    t2[q] = cin[8 + 4 * q + 3];
                }
            }
#pragma unroll
            for (int i = B - 1; i >= 0; --i) {
                float zo[2], to[2];
#pragma unroll
                for (int q = 0; q < 2; ++q)
                    astep<true>(c, q, P[i + 2], P[i + 3], Q[i + 2], Q[i + 3], z1[q], z2[q], t1[q], t2[q], zo[q], to[q]);
                if constexpr (!AGG) {
                    wc[i] += zo[0] + zo[1];
                    zc[i] += to[0] + to[1];
                }
            }
            if (AGG && live) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    cp[(8 + 4 * q + 0) * Hp] = z1[q];
                    cp[(8 + 4 * q + 1) * Hp] = z2[q];
                    cp[(8 + 4 * q + 2) * Hp] = t1[q];
                    cp[(8 + 4 * q + 3) * Hp] = t2[q];
                }
            }
        }
        if constexpr (!AGG) {
            // Horner steps of S2, S3 (ratio tau / sqrt(n+1)) and of S1 (ratio
            // tau / sqrt(n), channels n >= 1)
            const double r2 = p.isq[n + 1], r1 = p.isq[n], sq = p.sq[n];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const double xd = (double)xf[i], wd = (double)wc[i];
                h2[i] = fma(h2[i], xd * r2, wd);
                h3[i] = fma(h3[i], xd * r2, (double)zc[i]);
                if (n >= 1) h1[i] = fma(h1[i], xd * r1, sq * wd);
            }
        }
    }
    if constexpr (AGG) {
        return;
    } else {
        // scale to the full sums: S1 by p_{cb-1}, S2 and S3 by p_cb
        // (group 0 needs none: its S1 ran over n >= 1 relative to p_0 = 1)
        if (cb > 0) {
            const double c1 = inv_sqrt_fact(p, cb - 1);
#pragma unroll
            for (int i = 0; i < B; ++i) {
                const double xd = (double)xf[i];
                const double q1 = ipow(xd, cb - 1) * c1;  // p_{cb-1}
                const double q2 = q1 * xd * p.isq[cb];    // p_cb
                h1[i] *= q1;
                h2[i] *= q2;
                h3[i] *= q2;
            }
        }
        if (G > 1) {
            if (g > 0) {
                double *r = red + (size_t)(g - 1) * 3 * B * 64;
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    r[(0 * B + i) * 64 + lane] = h1[i];
                    r[(1 * B + i) * 64 + lane] = h2[i];
                    r[(2 * B + i) * 64 + lane] = h3[i];
                }
            }
            __syncthreads();
            if (g > 0) return;
            for (int gg = 1; gg < G; ++gg) {
                const double *r = red + (size_t)(gg - 1) * 3 * B * 64;
#pragma unroll
                for (int i = 0; i < B; ++i) {
                    h1[i] += r[(0 * B + i) * 64 + lane];
                    h2[i] += r[(1 * B + i) * 64 + lane];
                    h3[i] += r[(2 * B + i) * 64 + lane];
                }
            }
        }
        double s_gh = 0.0, s_xgH = 0.0, s_grho = 0.0, s_zu = 0.0, s_g = 0.0;
#pragma unroll
        for (int i = 0; i < B; ++i) {
            const int x = a + i;
            if (live && x < p.W) {
                const double xd = (double)xf[i];
                const double e = exp(-0.5 * xd * xd);
                const size_t pi = (size_t)y * p.pitch + x, qi = (size_t)y * p.W + x;
                const double gv = (double)b.grad_out[pi];
                const double h = fma(e, fma(-xd, h2[i], h1[i]), gv * p.sigma_r * (double)b.drho[qi]);
                const double gh = h * p.inv_sigma_r;
                if (b.grad_img) b.grad_img[pi] = (float)gh;
                s_gh += gh;
                s_xgH += xd * h;
                s_grho += gv * p.sigma_r * (double)b.rho[qi];
                s_zu += e * h3[i];
                s_g += gv;
            }
        }
        s_gh = wave_sum(s_gh);
        s_xgH = wave_sum(s_xgH);
        s_grho = wave_sum(s_grho);
        s_zu = wave_sum(s_zu);
        s_g = wave_sum(s_g);
        if (lane == 0) {
            BwdPartial o;
            o.sum_gh = s_gh;
            o.sum_xgH = s_xgH;
            o.sum_grho = s_grho;
            o.sum_zu = s_zu;
            o.sum_g = s_g;
            *bp = o;
        }
    }
}

}  // namespace bfgp
