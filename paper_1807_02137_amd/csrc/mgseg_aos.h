// AOS (additive operator splitting) on the finest grid, in FP64: the
// semi-implicit time stepper the paper measures its multigrid against
// (Sec. 5, Table 4) and names as an "exact" solver of the coarsest grid
// (Algorithm 1).  For phi_t = N(phi) with the coefficients of eq. abcdrc
// frozen at phi^k, one step is
//   r   = phi^k - tau f,
//   y_1 = (I - 2 tau A_1)^{-1} r   (couplings A, B along i: one system per column),
//   y_2 = (I - 2 tau A_2)^{-1} r   (couplings C, D along j: one system per row),
//   phi^{k+1} = clamp((y_1 + y_2) / 2, -M, M),
// with tau = tau_hat h / mu, so that 2 tau times a coupling is 2 tau_hat
// times the face value.
//
// Data: five dense n x m FP64 planes hold 2 tau s g for the faces to i+1,
// i-1, j+1, j-1 (s = kappa delta, or kappa for the scaled rows) and r; the
// column solves put y_1 in a sixth.  A column is one thread (consecutive
// threads take consecutive columns, so every row step is one coalesced
// access); a row is one thread walking along its row (the accesses of a wave
// are one element of each of 64 rows; each 128-byte line serves 16 steps
// from the cache).  Both are Thomas eliminations (the rows are strictly
// diagonally dominant M-matrix rows: positive pivots, no pivoting).
#pragma once
#include "mgseg_device.h"

struct AosArgs {
    const double *phi64, *w64, *d64;   // dense n x m
    const float *z32; int p32;         // image (pitch p32)
    const double *c12, *area;          // region means; area term (Rada-Chen) or null
    double kap, e2, eps, l1, l2, theta, tau;
    int model, scaled, n, m;
    double *uA, *uB, *uC, *uD, *r;     // outputs, dense n x m
};

// the four face values w_face / |grad phi|_eps of cell (i, j) (zero on boundary faces)
__device__ __forceinline__ void aos_faces(const AosArgs &A, int i, int j, double (&g)[4])
{
    const int n = A.n, m = A.m;
    const int im = mg_mirror(i - 1, n), ip = mg_mirror(i + 1, n), jm = mg_mirror(j - 1, m), jp = mg_mirror(j + 1, m);
    auto P = [&](int a, int b) { return A.phi64[(long long)a * m + b]; };
    auto W = [&](int a, int b) { return A.w64[(long long)a * m + b]; };
    const double p0 = P(i, j);
    g[0] = i + 1 < n ? mg_face64(p0, P(i + 1, j), P(i, jp), P(i + 1, jp), P(i, jm), P(i + 1, jm), W(i, j), W(i + 1, j), A.e2) : 0.0;
    g[1] = i > 0 ? mg_face64(P(i - 1, j), p0, P(i - 1, jp), P(i, jp), P(i - 1, jm), P(i, jm), W(i - 1, j), W(i, j), A.e2) : 0.0;
    g[2] = j + 1 < m ? mg_face64(p0, P(i, j + 1), P(ip, j), P(ip, j + 1), P(im, j), P(im, j + 1), W(i, j), W(i, j + 1), A.e2) : 0.0;
    g[3] = j > 0 ? mg_face64(P(i, j - 1), p0, P(ip, j - 1), P(ip, j), P(im, j - 1), P(im, j), W(i, j - 1), W(i, j), A.e2) : 0.0;
}

// the scaled couplings and the right-hand side of every cell
__global__ void __launch_bounds__(256) k_aos_coef(AosArgs A)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= A.m || i >= A.n) return;
    const long long q = (long long)i * A.m + j;
    double g[4];
    aos_faces(A, i, j, g);
    const double p0 = A.phi64[q];
    const double dl = A.scaled ? 1.0 : mg_delta64(p0, A.eps);
    const double t2 = 2.0 * A.tau * A.kap * dl;
    const double z = (double)A.z32[(long long)i * A.p32 + j];
    const double fa = z - A.c12[0], fb = z - A.c12[1];
    double fit = A.l1 * fa * fa - A.l2 * fb * fb;
    if (A.model == 0) fit += A.theta * A.d64[q];
    const double f = dl * (fit + (A.area ? *A.area : 0.0));
    A.uA[q] = t2 * g[0];
    A.uB[q] = t2 * g[1];
    A.uC[q] = t2 * g[2];
    A.uD[q] = t2 * g[3];
    A.r[q] = p0 - A.tau * f;
}

// Thomas elimination of one line of len cells at base + k * step:
//   -lo_k y_{k-1} + (1 + up_k + lo_k) y_k - up_k y_{k+1} = r_k.
// Forward: y_k = e_k y_{k+1} + t_k with e_k = up_k / d_k, t_k = (r_k + lo_k t_{k-1}) / d_k,
// d_k = 1 + up_k + lo_k (1 - e_{k-1}); e goes over up, t over y; back substitution in y.
__device__ __forceinline__ void aos_line(double *up, const double *lo, const double *r, double *y, long long base,
                                         long long step, int len)
{
    double e = 0.0, t = 0.0;
    for (int k = 0; k < len; k++) {
        const long long q = base + k * step;
        const double a = up[q], b = lo[q];
        const double inv = 1.0 / (1.0 + a + b * (1.0 - e));
        e = a * inv;
        t = (r[q] + b * t) * inv;
        up[q] = e;
        y[q] = t;
    }
    for (int k = len - 2; k >= 0; k--) {
        const long long q = base + k * step;
        t = fma(up[q], t, y[q]);
        y[q] = t;
    }
}

// one thread per column: couplings to i+1 (uA) and i-1 (uB); y_1 -> y
__global__ void __launch_bounds__(64) k_aos_cols(double *uA, const double *uB, const double *r, double *y, int n, int m)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    aos_line(uA, uB, r, y, j, m, n);
}

// one thread per row: couplings to j+1 (uC) and j-1 (uD); y_2 -> uD (each
// element is read before it is overwritten, by the same thread)
__global__ void __launch_bounds__(64) k_aos_rows(double *uC, double *uD, const double *r, int n, int m)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    aos_line(uC, uD, r, uD, (long long)i * m, 1, m);
}

// phi = clamp((y_1 + y_2) / 2, -M, M)
__global__ void k_aos_combine(double *phi64, const double *y1, const double *y2, long long N, double M)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const double v = 0.5 * (y1[q] + y2[q]);
    phi64[q] = v < -M ? -M : (v > M ? M : v);
}
