// Local Fourier analysis of the frozen-coefficient smoothers over a whole
// image (Sec. 3.3; Table 1's mu~_max and mu~_avg).  At a pixel with frozen
// couplings A, B, C, D (to i+1, i-1, j+1, j-1) a smoother that takes the
// couplings of the set `new` at the updated iterate and the others at the
// old one amplifies the Fourier mode exp(i(a1 i + a2 j)) by
//   mu(a1, a2) = |sum_{old} c E_c| / |S + Q' - sum_{new} c E_c|,
// E_A = e^{i a1}, E_B = e^{-i a1}, E_C = e^{i a2}, E_D = e^{-i a2}, S the sum
// of the couplings and Q' the NEWT term (zero otherwise).  The pixel's rate
// mu^ is the maximum over the high frequencies of the grid a = 2 pi t / 128,
// t = -64 .. 64, max(|a1|, |a2|) > pi / 2.  mu(-a1, -a2) = mu(a1, a2), so
// a1 >= 0 suffices.
//
// One thread per pixel; the 129 angles' cosines and sines sit in LDS.  The
// terms in a1 (couplings A, B) are formed once per a1 and the terms in a2
// (C, D) per point: about 15 FP32 operations per frequency, ALU-bound.
#pragma once
#include "mgseg_device.h"

#define LFA_T 64          // frequencies t = -LFA_T .. LFA_T on a grid of 2 LFA_T
#define LFA_NB 256        // threads per block

// new-coupling masks: bit 0 A, 1 B, 2 C, 3 D
enum { LFA_GSLEX = 0xA, LFA_GSLINE = 0xB };

struct LfaArgs {
    const float4 *cf;          // frozen couplings (A, B, C, D up to a common positive factor), pitch p
    const float *qd;           // NEWT diagonal term (null: none), pitch p
    const uint8_t *lab;        // jump-set labels (mode 2), pitch p
    int p, n, m;
    int mode;                  // 0 GSLEX, 1 GSLINE (column lines), 2 Hybrid Smoother 2
    float *mu;                 // per-pixel rate (may be null), pitch mp
    int mp;
    double *partial;           // per block: max, sum over all pixels, max, sum, count over the jump set
};

__device__ __forceinline__ float lfa_rate(float A, float B, float C, float D, float qd, unsigned nw,
                                          const float *cs, const float *sn)
{
    const float S = A + B + C + D + qd;
    // coefficient of each coupling in the numerator (old) or the denominator (new)
    const float oA = (nw & 1u) ? 0.0f : A, oB = (nw & 2u) ? 0.0f : B;
    const float oC = (nw & 4u) ? 0.0f : C, oD = (nw & 8u) ? 0.0f : D;
    const float nA = A - oA, nB = B - oB, nC = C - oC, nD = D - oD;
    float best_n = 0.0f, best_d = 1.0f;     // best ratio kept as a fraction (no division in the loop)
    for (int t1 = 0; t1 <= LFA_T; t1++) {
        const float c1 = cs[t1 + LFA_T], s1 = sn[t1 + LFA_T];
        // a1 terms: A E_A + B E_B = (A + B) cos + i (A - B) sin
        const float n1r = (oA + oB) * c1, n1i = (oA - oB) * s1;
        const float d1r = S - (nA + nB) * c1, d1i = -(nA - nB) * s1;
        const bool all = t1 > LFA_T / 2;
#pragma unroll 4
        for (int t2 = -LFA_T; t2 <= LFA_T; t2++) {
            if (!all && t2 >= -LFA_T / 2 && t2 <= LFA_T / 2) continue;
            const float c2 = cs[t2 + LFA_T], s2 = sn[t2 + LFA_T];
            const float nr = fmaf(oC + oD, c2, n1r), ni = fmaf(oC - oD, s2, n1i);
            const float dr = fmaf(-(nC + nD), c2, d1r), di = fmaf(-(nC - nD), s2, d1i);
            const float num = fmaf(nr, nr, ni * ni), den = fmaf(dr, dr, di * di);
            if (num * best_d > best_n * den) { best_n = num; best_d = den; }
        }
    }
    return sqrtf(best_n / best_d);
}

__global__ void __launch_bounds__(LFA_NB) k_lfa_rates(LfaArgs L)
{
    __shared__ float cs[2 * LFA_T + 1], sn[2 * LFA_T + 1];
    __shared__ double red[5][LFA_NB];
    const int tid = threadIdx.x;
    for (int t = tid; t <= 2 * LFA_T; t += LFA_NB) {
        // angle 2 pi (t - T) / (2 T) in FP64, then rounded: the same table on every block
        double s, c;
        sincospi((double)(t - LFA_T) / (double)LFA_T, &s, &c);
        cs[t] = (float)c;
        sn[t] = (float)s;
    }
    __syncthreads();
    const long long N = (long long)L.n * L.m;
    const long long q = (long long)blockIdx.x * LFA_NB + tid;
    double mx = 0.0, sm = 0.0, mxd = 0.0, smd = 0.0, cntd = 0.0;
    if (q < N) {
        const int i = (int)(q / L.m), j = (int)(q % L.m);
        const long long o = (long long)i * L.p + j;
        const float4 g = L.cf[o];
        const float qd = L.qd ? L.qd[o] : 0.0f;
        unsigned nw = L.mode == 1 ? LFA_GSLINE : LFA_GSLEX;
        const uint8_t b = L.lab ? L.lab[o] : 0;
        if (L.mode == 2 && b) nw = 0xFu & ~(unsigned)b;     // the sweep that lags the labelled coupling
        float mu = 0.0f;
        if (g.x + g.y + g.z + g.w + qd > 0.0f) mu = lfa_rate(g.x, g.y, g.z, g.w, qd, nw, cs, sn);
        if (L.mu) L.mu[(long long)i * L.mp + j] = mu;
        mx = sm = mu;
        if (b) { mxd = smd = mu; cntd = 1.0; }
    }
    red[0][tid] = mx; red[1][tid] = sm; red[2][tid] = mxd; red[3][tid] = smd; red[4][tid] = cntd;
    __syncthreads();
    for (int s = LFA_NB / 2; s > 0; s >>= 1) {
        if (tid < s) {
            red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
            red[1][tid] += red[1][tid + s];
            red[2][tid] = fmax(red[2][tid], red[2][tid + s]);
            red[3][tid] += red[3][tid + s];
            red[4][tid] += red[4][tid + s];
        }
        __syncthreads();
    }
    if (tid == 0)
        for (int k = 0; k < 5; k++) L.partial[5 * (long long)blockIdx.x + k] = red[k][0];
}

// the blocks' partials, in block order (deterministic): out = max, sum, max, sum, count
__global__ void k_lfa_final(const double *partial, int nb, double *out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = 0; b < nb; b++) {
        const double *p = partial + 5 * (long long)b;
        r[0] = fmax(r[0], p[0]); r[1] += p[1]; r[2] = fmax(r[2], p[2]); r[3] += p[3]; r[4] += p[4];
    }
    for (int k = 0; k < 5; k++) out[k] = r[k];
}
