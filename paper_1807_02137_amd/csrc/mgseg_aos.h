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
// column solves put y_1 in a sixth, the row solves y_2 over a coupling
// plane.  Every line (column or row) is one wave (k_aos_lines); the rows are
// strictly diagonally dominant M-matrix rows (positive pivots, no pivoting).
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

// One line of len cells per wave, chunks of C = ceil(len / 64) consecutive
// cells per lane, for the rows
//   -lo_k y_{k-1} + (1 + up_k + lo_k) y_k - up_k y_{k+1} = r_k
// (lo_0 = up_{len-1} = 0: the couplings across the grid edge vanish), cell k
// of line L at L * ls + k * cs.  The backward elimination y_k = P_k y_{k-1} +
// Q_k is the linear-fractional map of the elimination scan (Elim, FP64):
//  1. each lane composes its chunk's steps into one map;
//  2. a wave scan of the chunk maps from the line's end gives each lane the
//     state (P, Q) just after its chunk;
//  3. each lane runs the plain backward recursion over its own cells from
//     that state, and stores P_k, Q_k over up_k, lo_k;
//  4. the forward substitution: each lane composes its cells' affine maps
//     y -> P_k y + Q_k, a wave scan in line order gives the value entering
//     its chunk, and the lane writes its cells' y.
// The recursions inside a chunk are the sequential elimination; only the 6
// scan levels compose maps.  A workgroup of 4 waves takes 4 neighbouring
// lines.
__device__ __forceinline__ Elim elim_step_d(double a, double c, double r) { return Elim{c, 0.0, -r, 0.0, a, -c}; }

struct Aff {
    double a, b;               // y -> a y + b
};
__device__ __forceinline__ Aff aff_comp(const Aff &g, const Aff &f) { return Aff{g.a * f.a, fma(g.a, f.b, g.b)}; }
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ Aff dpp_aff(const Aff &v)
{
    return Aff{dpp_d<CTRL, ROWM>(1.0, v.a), dpp_d<CTRL, ROWM>(0.0, v.b)};
}
__device__ __forceinline__ Aff wave_scan_aff(Aff v)
{
    v = aff_comp(v, dpp_aff<0x111>(v));
    v = aff_comp(v, dpp_aff<0x112>(v));
    v = aff_comp(v, dpp_aff<0x114>(v));
    v = aff_comp(v, dpp_aff<0x118>(v));
    v = aff_comp(v, dpp_aff<0x142, 0xa>(v));
    v = aff_comp(v, dpp_aff<0x143, 0xc>(v));
    return v;
}
__device__ __forceinline__ double shfl_d(double x, int src)
{
    return __shfl(x, src, 64);
}
__device__ __forceinline__ Elim shfl_elim(const Elim &e, int src)
{
    return Elim{shfl_d(e.al, src), shfl_d(e.b0, src), shfl_d(e.b1, src), shfl_d(e.m00, src), shfl_d(e.m01, src),
                shfl_d(e.m10, src)};
}

// the elimination map of the chunk's steps (each row normalised by its diagonal)
__device__ __forceinline__ Elim aos_step_map(double a, double b, double r)
{
    const double inv = 1.0 / (1.0 + a + b);
    return elim_step_d(b * inv, a * inv, -r * inv);
}
// the chunk maps of the chunks after this one (lanes reversed, so that a later chunk sits on a
// lower lane and is applied first; exclusive), applied to the end state: (P, Q) after the chunk
__device__ __forceinline__ void aos_after(const Elim &E, int lane, double &P, double &Q)
{
    Elim R = shfl_elim(E, 63 - lane);
    R = wave_scan_elim<64>(R);
    const Elim id = elim_id();
    R = Elim{dpp_d<0x138>(id.al, R.al), dpp_d<0x138>(id.b0, R.b0), dpp_d<0x138>(id.b1, R.b1),
             dpp_d<0x138>(id.m00, R.m00), dpp_d<0x138>(id.m01, R.m01), dpp_d<0x138>(id.m10, R.m10)};
    const Elim S = shfl_elim(R, 63 - lane);
    P = S.m01;
    Q = S.b1;
}
// the value entering each lane's chunk from the chunks' affine maps (exclusive, line order)
__device__ __forceinline__ double aos_entering(const Aff &F)
{
    const Aff inc = wave_scan_aff(F);
    return dpp_d<0x138>(0.0, inc.b);                  // y_{-1} = 0
}

// Each pass over a chunk reads its cells in blocks of G whose loads are issued
// together before any of the block's stores (the recursion itself is a chain
// in registers), so that one memory latency is paid per block, not per cell.
template <int G>
__global__ void __launch_bounds__(256) k_aos_lines(double *up, double *lo, const double *r, double *y, int nlines,
                                                   int len, long long ls, long long cs)
{
    const int lane = threadIdx.x & 63;
    const int line = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (line >= nlines) return;                        // whole waves
    const long long base = (long long)line * ls;
    const int C = (len + 63) / 64;
    const int k0 = min(lane * C, len), k1 = min(k0 + C, len);
    auto at = [&](int k) { return base + (long long)k * cs; };
    double a[G], b[G], rv[G];
    // backward over the chunk in blocks: k = kb, kb - 1, ..., kb - G + 1
    auto load_back = [&](int kb, bool with_r) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            const int k = kb - j;
            if (k >= k0) {
                const long long q = at(k);
                a[j] = up[q]; b[j] = lo[q];
                if (with_r) rv[j] = r[q];
            }
        }
    };
    // 1. the chunk's elimination map, from its last cell to its first
    Elim E = elim_id();
    for (int kb = k1 - 1; kb >= k0; kb -= G) {
        load_back(kb, true);
#pragma unroll
        for (int j = 0; j < G; j++)
            if (kb - j >= k0) E = elim_comp(aos_step_map(a[j], b[j], rv[j]), E);
    }
    // 2. the state after the chunk; 3. the backward recursion, P over up and Q over lo
    double P, Q;
    aos_after(E, lane, P, Q);
    for (int kb = k1 - 1; kb >= k0; kb -= G) {
        load_back(kb, true);
#pragma unroll
        for (int j = 0; j < G; j++) {
            const int k = kb - j;
            if (k < k0) continue;
            const double inv = 1.0 / (1.0 + a[j] + b[j] - a[j] * P);
            Q = fma(a[j], Q, rv[j]) * inv;
            P = b[j] * inv;
            const long long q = at(k);
            up[q] = P;
            lo[q] = Q;
        }
    }
    // 4. forward substitution: the chunk's affine map, the value entering it, the cells
    auto load_fwd = [&](int kb) {
#pragma unroll
        for (int j = 0; j < G; j++) {
            const int k = kb + j;
            if (k < k1) {
                const long long q = at(k);
                a[j] = up[q]; b[j] = lo[q];
            }
        }
    };
    Aff F{1.0, 0.0};
    for (int kb = k0; kb < k1; kb += G) {
        load_fwd(kb);
#pragma unroll
        for (int j = 0; j < G; j++)
            if (kb + j < k1) F = aff_comp(Aff{a[j], b[j]}, F);
    }
    double v = aos_entering(F);
    for (int kb = k0; kb < k1; kb += G) {
        load_fwd(kb);
#pragma unroll
        for (int j = 0; j < G; j++) {
            if (kb + j >= k1) continue;
            v = fma(a[j], v, b[j]);
            y[at(kb + j)] = v;
        }
    }
}

// phi = clamp((y_1 + y_2) / 2, -M, M)
__global__ void k_aos_combine(double *phi64, const double *y1, const double *y2, long long N, double M)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N) return;
    const double v = 0.5 * (y1[q] + y2[q]);
    phi64[q] = v < -M ? -M : (v > M ? M : v);
}
