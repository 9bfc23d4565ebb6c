// mgseg_kernels.h -- grid kernels of libmgseg other than the line sweep.
#pragma once
#include "mgseg_device.h"

#define TILE 32
// rows of a 32 x 32-tile block: 16 (two rows per thread; 512 threads, three
// blocks per CU beside the stencil and transpose staging in LDS) on grids of
// many tiles, where several blocks per CU overlap each other's barriers; 32
// (one row per thread, the shortest chain) on small grids
__host__ __device__ inline int tile_rows(long long tiles) { return tiles >= 4096 ? 16 : TILE; }

// ==========================================================================
// Setup maps (Sec. 2.2).  Level-0 maps are computed in FP64.
// Gaussian pre-blur of z (separable, half-sample mirror), then
// g = 1/(1 + beta |grad|^2) with central differences per pixel.
__global__ void k_blur_rows(const float *z, int pz, double *out, int n, int m, const double *ker, int R)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    double s = 0.0;
    for (int t = -R; t <= R; t++) {
        int jj = j + t;
        while (jj < 0 || jj >= m) jj = (jj < 0) ? -jj - 1 : 2 * m - jj - 1;
        s += ker[t + R] * (double)z[(long long)i * pz + jj];
    }
    out[(long long)i * m + j] = s;
}
__global__ void k_blur_cols(const double *in, double *out, int n, int m, const double *ker, int R)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    double s = 0.0;
    for (int t = -R; t <= R; t++) {
        int ii = i + t;
        while (ii < 0 || ii >= n) ii = (ii < 0) ? -ii - 1 : 2 * n - ii - 1;
        s += ker[t + R] * in[(long long)ii * m + j];
    }
    out[(long long)i * m + j] = s;
}

// Setup maps of the finest grid (Sec. 2.2 and Sec. 5), computed per cell:
//  g   : the edge detector 1/(1 + beta |grad(G_sigma * z)|^2), the gradient by
//        central differences of the blurred image per pixel, mirrored edges;
//  d   : the marker distance function, the product over the markers of
//        1 - exp(-|x_k - x|^2 / (2 sigma_d^2)) in domain units (formed with
//        expm1, exact where a marker is close);
//  w   : g (Spencer-Chen) or d g (Rada-Chen), the weight of the curvature term;
//  phi0: the signed distance in pixels to the boundary of the marker polygon
//        (the convex hull of the markers), positive inside, clamped to [-M, M].
// The hull reaches the device as its edges: start vertex, unit direction,
// length, and the unit outward normal with its offset, so that the line
// through an edge is {x : nrm . x = off}.  For a closed hull (three or more
// vertices) a point is inside when it lies on the inner side of every edge
// line, and its distance to the boundary is then the least distance to an
// edge line (convexity).  Outside, the nearest boundary point is either a
// vertex or the foot of the perpendicular on an edge whose foot falls within
// it.  One or two markers give an open hull (a point or a segment): every
// cell is outside.
struct HullEdge {
    double ar, ac;      // start vertex (row, col)
    double ur, uc;      // unit direction
    double len;         // length
    double nr, nc;      // unit outward normal
    double off;         // nrm . start vertex
};
#define MG_MAX_HULL 64

struct MarkerArgs {
    const double *mk; int k;          // markers (row, col) in pixels
    const HullEdge *edge; int ne;     // hull edges (a segment: one edge; a point: none)
    const double *vtx; int nv;        // hull vertices (row, col)
    int closed;                       // 1: the hull is a polygon with an inside
    double h0, sigma_d, M;
    int model, n, m;
    const double *g64;
    const float *z; int pz;
    double *d64, *w64, *phi64;
    float *w32, *d32, *z32, *phi32; int p32;
};

// signed distance (pixels) of the point (pr, pc) to the hull boundary, + inside
__device__ double hull_signed_distance(const MarkerArgs &A, double pr, double pc)
{
    double worst = -1e300;            // largest signed distance to an edge line (outward positive)
    double nearest = 1e300;           // least distance to a boundary point found so far
    for (int e = 0; e < A.ne; e++) {
        const HullEdge E = A.edge[e];
        const double rr = pr - E.ar, rc = pc - E.ac;
        const double side = fma(E.nr, pr, fma(E.nc, pc, -E.off));
        worst = fmax(worst, side);
        const double along = fma(rr, E.ur, rc * E.uc);
        if (along > 0.0 && along < E.len) nearest = fmin(nearest, fabs(side));
    }
    if (A.closed && worst <= 0.0) return -worst;
    for (int v = 0; v < A.nv; v++) nearest = fmin(nearest, hypot(pr - A.vtx[2 * v], pc - A.vtx[2 * v + 1]));
    return -nearest;
}

// edge detector from the blurred image: a 32 x 32 tile with a mirrored one-cell
// halo staged in LDS, each cell's four neighbours read from there
__global__ void __launch_bounds__(256) k_edge_detector(const double *zb, int n, int m, double beta, double *g64)
{
    __shared__ double tile[TILE + 2][TILE + 3];
    const int i0 = blockIdx.y * TILE, j0 = blockIdx.x * TILE;
    for (int t = threadIdx.x; t < (TILE + 2) * (TILE + 2); t += blockDim.x) {
        const int ti = t / (TILE + 2), tj = t % (TILE + 2);
        const int i = mg_mirror(i0 + ti - 1, n), j = mg_mirror(j0 + tj - 1, m);   // halo past the tile's cells unused
        tile[ti][tj] = zb[(long long)i * m + j];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) {
        const int ti = t / TILE, tj = t % TILE, i = i0 + ti, j = j0 + tj;
        if (i >= n || j >= m) continue;
        const double hx = 0.5 * (tile[ti + 1][tj + 2] - tile[ti + 1][tj]);
        const double hy = 0.5 * (tile[ti + 2][tj + 1] - tile[ti][tj + 1]);
        g64[(long long)i * m + j] = 1.0 / fma(beta, fma(hx, hx, hy * hy), 1.0);
    }
}

// marker distance function, curvature weight and the initial level set
__global__ void k_marker_maps(MarkerArgs A)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= A.m || i >= A.n) return;
    const double yc = i + 0.5, xc = j + 0.5;
    const double inv2s2 = 0.5 / (A.sigma_d * A.sigma_d);
    double d = 1.0;
    for (int t = 0; t < A.k; t++) {
        const double dy = (yc - A.mk[2 * t]) * A.h0, dx = (xc - A.mk[2 * t + 1]) * A.h0;
        d *= -expm1(-fma(dx, dx, dy * dy) * inv2s2);
    }
    const long long q = (long long)i * A.m + j, q32 = (long long)i * A.p32 + j;
    const double g = A.g64[q];
    const double w = A.model == 1 ? d * g : g;
    const double phi = fmin(A.M, fmax(-A.M, hull_signed_distance(A, yc, xc)));
    A.d64[q] = d; A.w64[q] = w; A.phi64[q] = phi;
    A.d32[q32] = (float)d; A.w32[q32] = (float)w; A.phi32[q32] = (float)phi;
    A.z32[q32] = A.z[(long long)i * A.pz + j];
}

// ==========================================================================
// Transfers (Sec. 3.1).  Full weighting, 0-based: coarse I takes fine
// 2I, 2I+1, 2I+2 with 1/4, 1/2, 1/4, the last coarse index fine 2I, 2I+1 with
// 1/2, 1/2 (the paper's boundary rule); tensor product in 2-D.
__device__ __forceinline__ float fw_row(const float *row, int J, int mc)
{
    if (J < mc - 1) return 0.25f * row[2 * J] + 0.5f * row[2 * J + 1] + 0.25f * row[2 * J + 2];
    return 0.5f * row[2 * J] + 0.5f * row[2 * J + 1];
}
__device__ __forceinline__ float fw2(const float *f, int pf, int I, int J, int nc, int mc)
{
    const float *r0 = f + (long long)(2 * I) * pf, *r1 = r0 + pf;
    if (I < nc - 1) {
        const float *r2 = r1 + pf;
        return 0.25f * fw_row(r0, J, mc) + 0.5f * fw_row(r1, J, mc) + 0.25f * fw_row(r2, J, mc);
    }
    return 0.5f * fw_row(r0, J, mc) + 0.5f * fw_row(r1, J, mc);
}
__global__ void k_restrict(const float *f, int pf, float *c, int pc, int nc, int mc)
{
    int J = blockIdx.x * blockDim.x + threadIdx.x, I = blockIdx.y;
    if (J >= mc || I >= nc) return;
    c[(long long)I * pc + J] = fw2(f, pf, I, J, nc, mc);
}

// coarse bounds of the box reading: the coarse unknown may move only as far as
// every fine cell its interpolated correction reaches can follow inside that
// cell's own bounds: lo_c = phic + max(lo_f - phi_f), hi_c = phic + min(hi_f - phi_f)
// over fine (2I..2I+2) x (2J..2J+2).  flo / fhi null: -M / M.
__global__ void k_coarse_bounds(const float *phi, const float *flo, const float *fhi, int pf, int n, int m,
                                const float *phic, float *clo, float *chi, int pc, int nc, int mc, float M)
{
    int J = blockIdx.x * blockDim.x + threadIdx.x, I = blockIdx.y;
    if (J >= mc || I >= nc) return;
    float dl = -MG_BIG, dh = MG_BIG;
    for (int i = 2 * I; i <= 2 * I + 2 && i < n; i++)
        for (int j = 2 * J; j <= 2 * J + 2 && j < m; j++) {
            long long q = (long long)i * pf + j;
            float p = phi[q];
            float lo = flo ? flo[q] : -M, hi = fhi ? fhi[q] : M;
            dl = fmaxf(dl, lo - p);
            dh = fminf(dh, hi - p);
        }
    float pcv = phic[(long long)I * pc + J];
    clo[(long long)I * pc + J] = pcv + dl;
    chi[(long long)I * pc + J] = pcv + dh;
}

// bilinear interpolation (Sec. 3.1), 0-based: fine 2I+1 <- coarse I, fine 2I
// (I >= 1) <- mean of coarse I-1, I, fine 0 <- coarse 0; tensor product.
// Correction: phi <- clip(phi + P(phi^c - phic), lo, hi); phic null: phi^c is
// the correction itself (deviation form).
__device__ __forceinline__ void pl_idx(int f, int &a, int &b, float &wa)
{
    if (f & 1) { a = b = f >> 1; wa = 1.0f; }
    else if (f == 0) { a = b = 0; wa = 1.0f; }
    else { a = (f >> 1) - 1; b = f >> 1; wa = 0.5f; }
}
__global__ void k_prolong_correct(float *phi, const float *lo, const float *hi, int pf, int n, int m,
                                  const float *phis, const float *phic, int pc, float M)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    int ia, ib, ja, jb;
    float wi, wj;
    pl_idx(i, ia, ib, wi);
    pl_idx(j, ja, jb, wj);
    auto e = [&](int I, int J) { long long q = (long long)I * pc + J; return phic ? phis[q] - phic[q] : phis[q]; };
    float ea = wj * e(ia, ja) + (1.0f - wj) * e(ia, jb);
    float eb = wj * e(ib, ja) + (1.0f - wj) * e(ib, jb);
    float corr = wi * ea + (1.0f - wi) * eb;
    long long q = (long long)i * pf + j;
    float l = lo ? lo[q] : -M, h = hi ? hi[q] : M;
    phi[q] = mg_clip(phi[q] + corr, l, h);
}

// ==========================================================================
// transposes (32 x 32 tiles through LDS)
template <typename T>
__global__ void k_transpose(const T *in, int pin, T *out, int pout, int n, int m)
{
    // in: n x m (row pitch pin) -> out: m x n (row pitch pout)
    __shared__ T tile[TILE][TILE + 1];
    int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        int i = by + y, j = bx + threadIdx.x;
        if (i < n && j < m) tile[y][threadIdx.x] = in[(long long)i * pin + j];
    }
    __syncthreads();
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        int j = bx + y, i = by + threadIdx.x;
        if (i < n && j < m) out[(long long)j * pout + i] = tile[threadIdx.x][y];
    }
}

// ==========================================================================
// Freeze (start of every outer iteration, Sec. 3.2 "-I"): labels of the
// jump set (Sec. 4.1 Definition; threshold Sigma of Sec. 5.2) with the
// smallest coefficient (Sec. 4.2), on the four face values of each cell
// (the common factor mu delta / h^2 cancels in both tests).  Interior faces
// only; a zero interior value counts as an infinite ratio; ties take the
// first of A, B, C, D.  Bit s of the label byte = starred in sweep s.
// raw face values w_face / |grad x|_eps of the faces A (i+1/2, j), B (i-1/2, j),
// C (i, j+1/2), D (i, j-1/2) of cell (i, j), x read through X(i, j); zero on
// boundary faces.  The arguments are those of the line sweep, so the values
// are bit-identical to the sweep's.
template <class X, class W>
__device__ __forceinline__ void faces4(const X &P, const W &Wf, int n, int m, int i, int j, float e2, float (&g)[4])
{
    const int im = mg_mirror(i - 1, n), ip = mg_mirror(i + 1, n), jm = mg_mirror(j - 1, m), jp = mg_mirror(j + 1, m);
    const float p0 = P(i, j);
    g[0] = i + 1 < n ? mg_face(p0, P(i + 1, j), P(i, jp), P(i + 1, jp), P(i, jm), P(i + 1, jm), Wf(i, j), Wf(i + 1, j), e2) : 0.0f;
    g[1] = i > 0 ? mg_face(P(i - 1, j), p0, P(i - 1, jp), P(i, jp), P(i - 1, jm), P(i, jm), Wf(i - 1, j), Wf(i, j), e2) : 0.0f;
    g[2] = j + 1 < m ? mg_face(p0, P(i, j + 1), P(ip, j), P(ip, j + 1), P(im, j), P(im, j + 1), Wf(i, j), Wf(i, j + 1), e2) : 0.0f;
    g[3] = j > 0 ? mg_face(P(i, j - 1), p0, P(ip, j - 1), P(ip, j), P(im, j - 1), P(im, j), Wf(i, j - 1), Wf(i, j), e2) : 0.0f;
}

__device__ __forceinline__ uint8_t label_of(const float (&G)[4], int n, int m, int i, int j, float Sigma)
{
    const bool in[4] = {i + 1 < n, i > 0, j + 1 < m, j > 0};
    int cnt = 0, amin = -1;
    float gmin = 0.0f, gmax = 0.0f;
    for (int s = 0; s < 4; s++) {
        if (!in[s]) continue;
        if (cnt == 0 || G[s] < gmin) { gmin = G[s]; amin = s; }
        if (cnt == 0 || G[s] > gmax) gmax = G[s];
        cnt++;
    }
    return (cnt >= 2 && gmax > Sigma * gmin) ? (uint8_t)(1u << amin) : (uint8_t)0;
}

__device__ __forceinline__ uint8_t cell_label(const float *psi, const float *w, int p, int n, int m, int i, int j,
                                              float e2, float Sigma)
{
    auto P = [&](int a, int b) { return psi[(long long)a * p + b]; };
    auto W = [&](int a, int b) { return w[(long long)a * p + b]; };
    float G[4];
    faces4(P, W, n, m, i, j, e2, G);
    return label_of(G, n, m, i, j, Sigma);
}


// FP32-mode freeze: psi = phi and the labels, both layouts
__global__ void k_freeze32(const float *phi, const float *w, int p, int n, int m, float e2, float Sigma, float *psi,
                           float *psi_cm, uint8_t *lab, uint8_t *lab_cm, int pc)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    const long long q = (long long)i * p + j, qc = (long long)j * pc + i;
    const uint8_t b = cell_label(phi, w, p, n, m, i, j, e2, Sigma);
    psi[q] = psi_cm[qc] = phi[q];
    lab[q] = lab_cm[qc] = b;
}

// ==========================================================================
// operator N(phi) at one cell (eq. abcd, all coefficients at phi) in FP32
__device__ __forceinline__ float cell_N(const float *phi, const float *w, const float *fit, int p, int n, int m,
                                        int i, int j, float kap, float e2, float eps, float area, int scaled)
{
    int im = mg_mirror(i - 1, n), ip = mg_mirror(i + 1, n), jm = mg_mirror(j - 1, m), jp = mg_mirror(j + 1, m);
    auto P = [&](int a, int b) { return phi[(long long)a * p + b]; };
    auto W = [&](int a, int b) { return w[(long long)a * p + b]; };
    float p0 = P(i, j);
    float dl = scaled ? 1.0f : mg_delta(p0, eps);
    float s = kap * dl;
    float v = -dl * (fit[(long long)i * p + j] + area);
    if (i + 1 < n) v += s * mg_face(p0, P(i + 1, j), P(i, jp), P(i + 1, jp), P(i, jm), P(i + 1, jm), W(i, j), W(i + 1, j), e2) * (P(i + 1, j) - p0);
    if (i > 0) v += s * mg_face(P(i - 1, j), p0, P(i - 1, jp), P(i, jp), P(i - 1, jm), P(i, jm), W(i - 1, j), W(i, j), e2) * (P(i - 1, j) - p0);
    if (j + 1 < m) v += s * mg_face(p0, P(i, j + 1), P(ip, j), P(ip, j + 1), P(im, j), P(im, j + 1), W(i, j), W(i, j + 1), e2) * (P(i, j + 1) - p0);
    if (j > 0) v += s * mg_face(P(i, j - 1), p0, P(ip, j - 1), P(ip, j), P(im, j - 1), P(im, j), W(i, j - 1), W(i, j), e2) * (P(i, j - 1) - p0);
    return v;
}

// residual r = F - N(phi), projected on the box (zero where the correction
// -r/S would leave [lo, hi]); optional per-block partial sums of r^2.
__global__ void k_residual(const float *phi, const float *w, const float *fit, const float *F, const float *lo,
                           const float *hi, int p, int n, int m, float kap, float e2, float eps,
                           const double *area, int scaled, float M, float *r, double *partial)
{
    __shared__ double red[256];
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    int tid = threadIdx.x;
    double acc = 0.0;
    if (j < m && i < n) {
        float ar = area ? (float)(*area) : 0.0f;
        long long q = (long long)i * p + j;
        float v = (F ? F[q] : 0.0f) - cell_N(phi, w, fit, p, n, m, i, j, kap, e2, eps, ar, scaled);
        float ph = phi[q], l = lo ? lo[q] : -M, h = hi ? hi[q] : M;
        if ((ph >= h && v < 0.0f) || (ph <= l && v > 0.0f)) v = 0.0f;
        if (r) r[q] = v;
        acc = (double)v * (double)v;
    }
    if (partial) {
        red[tid] = acc;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (tid < s) red[tid] += red[tid + s];
            __syncthreads();
        }
        if (tid == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
    }
}

// coarse right-hand side F_c = N_c(phi_c) + r_c (Algorithm-1 box)
__global__ void k_coarse_rhs(const float *phic, const float *w, const float *fit, const float *rc, int p, int n,
                             int m, float kap, float e2, float eps, const double *area, int scaled, float *F,
                             float *phi_init)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    float ar = area ? (float)(*area) : 0.0f;
    long long q = (long long)i * p + j;
    F[q] = cell_N(phic, w, fit, p, n, m, i, j, kap, e2, eps, ar, scaled) + rc[q];
    phi_init[q] = phic[q];
}

// fit maps of every level with the current c1, c2 (Spencer-Chen adds theta d),
// one launch of 32 x 32 tiles, block (32, tile_rows): block row y covers tile row
// y - trow0[l] of the level l whose tile rows [trow0[l], trow0[l+1]) contain
// y; the column-major copy goes through LDS (fit_cm[l] null: not written)
#define FIT_MAXLEV 16
struct FitLevels {
    const float *z[FIT_MAXLEV], *d[FIT_MAXLEV];
    float *fit[FIT_MAXLEV], *fit_cm[FIT_MAXLEV];
    int p[FIT_MAXLEV], pc[FIT_MAXLEV], n[FIT_MAXLEV], m[FIT_MAXLEV], trow0[FIT_MAXLEV + 1];
    int L;
};
__global__ void __launch_bounds__(1024) k_fit(FitLevels F, const double *c12, float l1, float l2, float theta,
                                             int model)
{
    __shared__ float tf[TILE][TILE + 1];
    int l = 0;
    while (l + 1 < F.L && (int)blockIdx.y >= F.trow0[l + 1]) l++;
    const int n = F.n[l], m = F.m[l];
    const int by = ((int)blockIdx.y - F.trow0[l]) * TILE, bx = blockIdx.x * TILE;
    if (bx >= m) return;                   // the whole block: narrower level
    const float c1 = (float)c12[0], c2 = (float)c12[1];
    const bool cm = F.fit_cm[l] != nullptr;          // the same for the whole block
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int i = by + y, j = bx + threadIdx.x;
        if (i >= n || j >= m) continue;
        const long long q = (long long)i * F.p[l] + j;
        const float a = F.z[l][q] - c1, b = F.z[l][q] - c2;
        float v = l1 * a * a - l2 * b * b;
        if (model == 0) v += theta * F.d[l][q];
        F.fit[l][q] = v;
        if (cm) tf[y][threadIdx.x] = v;
    }
    if (!cm) return;
    __syncthreads();
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int j = bx + y, i = by + threadIdx.x;
        if (i >= n || j >= m) continue;
        F.fit_cm[l][(long long)j * F.pc[l] + i] = tf[threadIdx.x][y];
    }
}

// ==========================================================================
// deterministic FP64 sums over a level: sum H(phi), sum H(phi) z, sum z
template <typename T>
__global__ void k_sums(const T *phi, int pp, const float *z, int pz, int n, int m, double eps, double *partial)
{
    __shared__ double r0[256], r1[256], r2[256];
    int tid = threadIdx.x;
    long long N = (long long)n * m;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + tid; t < N; t += (long long)gridDim.x * blockDim.x) {
        int i = (int)(t / m), j = (int)(t % m);
        double H = mg_heav64((double)phi[(long long)i * pp + j], eps);
        double zz = z ? (double)z[(long long)i * pz + j] : 0.0;
        a0 += H; a1 += H * zz; a2 += zz;
    }
    r0[tid] = a0; r1[tid] = a1; r2[tid] = a2;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) { r0[tid] += r0[tid + s]; r1[tid] += r1[tid + s]; r2[tid] += r2[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) {
        partial[3 * blockIdx.x] = r0[0];
        partial[3 * blockIdx.x + 1] = r1[0];
        partial[3 * blockIdx.x + 2] = r2[0];
    }
}

// finalize: mode 0 -> area term 2 nu (h^2 sum H - A1) into out[0];
//           mode 1 -> c1, c2 (eq. c1c2) into out[0], out[1];
//           mode 2 -> sqrt(sum of partial r^2) into out[0] (partials of stride 1)
//           mode 3 -> sqrt(sum d^2 / sum p^2) into out[0] (pairs of partials: eta)
#define FIN_NT 256
__global__ void __launch_bounds__(FIN_NT) k_finalize(const double *partial, int nb, int mode, double N, double h2,
                                                     double A1, double nu, double *out)
{
    // deterministic: fixed strided assignment of partials, then a fixed tree
    __shared__ double r0[FIN_NT], r1[FIN_NT], r2[FIN_NT];
    const int t = threadIdx.x;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (mode == 2) {
        for (int b = t; b < nb; b += FIN_NT) a0 += partial[b];
    } else if (mode == 3 || mode == 4) {
        for (int b = t; b < nb; b += FIN_NT) { a0 += partial[2 * b]; a1 += partial[2 * b + 1]; }
    } else {
        for (int b = t; b < nb; b += FIN_NT) {
            a0 += partial[3 * b]; a1 += partial[3 * b + 1]; a2 += partial[3 * b + 2];
        }
    }
    r0[t] = a0; r1[t] = a1; r2[t] = a2;
    __syncthreads();
    for (int s = FIN_NT / 2; s > 0; s >>= 1) {
        if (t < s) { r0[t] += r0[t + s]; r1[t] += r1[t + s]; r2[t] += r2[t + s]; }
        __syncthreads();
    }
    if (t != 0) return;
    const double sH = r0[0], sHz = r1[0], sz = r2[0];
    if (mode == 2) {
        out[0] = sqrt(sH);
    } else if (mode == 4) {
        // the two residual norms: out[0] and out[2] (the slots around the one between)
        out[0] = sqrt(sH);
        out[2] = sqrt(sHz);
    } else if (mode == 3) {
        out[0] = sHz > 0.0 ? sqrt(sH / sHz) : 0.0;
    } else if (mode == 0) {
        out[0] = 2.0 * nu * (h2 * sH - A1);
    } else {
        out[0] = sH > 0.0 ? sHz / sH : 0.0;
        out[1] = (N - sH) > 0.0 ? (sz - sHz) / (N - sH) : 0.0;
    }
}

// ==========================================================================
// FP64 residual on the finest grid (defect-correction loop): r64 = -N64(phi64)
// (F = 0 there), its projected norm, and optionally phi32 = fl32(phi64) (the
// FP32 mode's next iterate) and G = fl32(r64) unprojected (the deviation
// form's finest right-hand side).
struct Res64Args {
    const double *phi64, *w64, *d64;       // dense n x m
    const float *z32, *w32, *fit32; int p32;
    const double *c12, *area;              // area may be null
    double kap, e2, eps, l1, l2, theta, M;
    int model, scaled, n, m;
    float *phi32, *G;                      // outputs (p32), each may be null
    double *partial;
};

// the squares of the projected residual of the paper's rows (eq. abcdrc, each
// with its delta(phi) factor: the stopping measure) and of the rows as the
// smoother holds them (divided by delta(phi) when scaled) go to two partials
// per block.  A block (32, 16) takes the 32 x 32 tiles of one tile column at
// tile rows y, y + gridDim.y, ...: phi and w of a tile and its one-cell halo
// (mirrored at the grid edge as the stencil mirrors) are staged in LDS, and
// every face value of the tile (33 x 32 between rows, 32 x 33 between
// columns) is computed once, for the two cells it separates.
#define R64_ROWS 16
__global__ void __launch_bounds__(TILE * R64_ROWS) k_res64(Res64Args A)
{
    __shared__ double ph[TILE + 2][TILE + 2], ww[TILE + 2][TILE + 2];
    __shared__ double fv[TILE + 1][TILE], fh[TILE][TILE + 1];
    __shared__ double red[TILE * R64_ROWS], red2[TILE * R64_ROWS];
    const int n = A.n, m = A.m, tx = threadIdx.x, ty = threadIdx.y, tid = ty * TILE + tx;
    constexpr int NTH = TILE * R64_ROWS;
    const int bx = blockIdx.x * TILE;
    const double c1 = A.c12[0], c2 = A.c12[1];
    const double area = A.area ? *A.area : 0.0;
    double acc = 0.0, acc_rows = 0.0;
    for (int by = blockIdx.y * TILE; by < n; by += gridDim.y * TILE) {
        __syncthreads();                  // the previous tile's LDS reads are done
        for (int t = tid; t < (TILE + 2) * (TILE + 2); t += NTH) {
            const int yy = t / (TILE + 2), xx = t % (TILE + 2);
            const long long q = (long long)mg_mirror(by - 1 + yy, n) * m + mg_mirror(bx - 1 + xx, m);
            ph[yy][xx] = A.phi64[q];
            ww[yy][xx] = A.w64[q];
        }
        __syncthreads();
        // fv[yy][x]: the face between tile rows yy - 1 and yy (grid rows by - 1 + yy, by + yy);
        // fh[y][xx]: between tile columns xx - 1 and xx; faces on the grid edge are not used
        for (int t = tid; t < (TILE + 1) * TILE; t += NTH) {
            const int yy = t / TILE, x = t % TILE;
            fv[yy][x] = mg_face64(ph[yy][x + 1], ph[yy + 1][x + 1], ph[yy][x + 2], ph[yy + 1][x + 2], ph[yy][x],
                                  ph[yy + 1][x], ww[yy][x + 1], ww[yy + 1][x + 1], A.e2);
            const int y = t / (TILE + 1), xx = t % (TILE + 1);
            fh[y][xx] = mg_face64(ph[y + 1][xx], ph[y + 1][xx + 1], ph[y + 2][xx], ph[y + 2][xx + 1], ph[y][xx],
                                  ph[y][xx + 1], ww[y + 1][xx], ww[y + 1][xx + 1], A.e2);
        }
        __syncthreads();
        for (int y = ty; y < TILE; y += R64_ROWS) {
            const int i = by + y, j = bx + tx;
            if (i >= n || j >= m) continue;
            const double p0 = ph[y + 1][tx + 1];
            const double dl = A.scaled ? 1.0 : mg_delta64(p0, A.eps);
            const double s = A.kap * dl;
            const double z = (double)A.z32[(long long)i * A.p32 + j];
            const double fa = z - c1, fb = z - c2;
            double fit = A.l1 * fa * fa - A.l2 * fb * fb;
            if (A.model == 0) fit += A.theta * A.d64[(long long)i * m + j];
            double v = -dl * (fit + area);
            if (i + 1 < n) v += s * fv[y + 1][tx] * (ph[y + 2][tx + 1] - p0);
            if (i > 0) v += s * fv[y][tx] * (ph[y][tx + 1] - p0);
            if (j + 1 < m) v += s * fh[y][tx + 1] * (ph[y + 1][tx + 2] - p0);
            if (j > 0) v += s * fh[y][tx] * (ph[y + 1][tx] - p0);
            const double r = -v;
            double rp = r;
            if ((p0 >= A.M && rp < 0.0) || (p0 <= -A.M && rp > 0.0)) rp = 0.0;
            acc_rows += rp * rp;
            const double rpp = A.scaled ? mg_delta64(p0, A.eps) * rp : rp;
            acc += rpp * rpp;
            const long long q = (long long)i * A.p32 + j;
            if (A.phi32) A.phi32[q] = (float)p0;
            if (A.G) A.G[q] = (float)r;
        }
    }
    red[tid] = acc;
    red2[tid] = acc_rows;
    __syncthreads();
    for (int st = NTH / 2; st > 0; st >>= 1) {
        if (tid < st) { red[tid] += red[tid + st]; red2[tid] += red2[tid + st]; }
        __syncthreads();
    }
    if (tid == 0) {
        const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
        A.partial[2 * b] = red[0];
        A.partial[2 * b + 1] = red2[0];
    }
}

__global__ void k_copy32to64(const float *phi32, int p32, double *phi64, int n, int m)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    phi64[(long long)i * m + j] = (double)phi32[(long long)i * p32 + j];
}

__global__ void k_copy64to32(const double *phi64, int n, int m, float *phi32, int p32)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    phi32[(long long)i * p32 + j] = (float)phi64[(long long)i * m + j];
}

__global__ void k_set_phi0(const float *src, int ps, double M, double *phi64, float *phi32, int p32, int n, int m)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    double v = (double)src[(long long)i * ps + j];
    v = v < -M ? -M : (v > M ? M : v);
    phi64[(long long)i * m + j] = v;
    phi32[(long long)i * p32 + j] = (float)v;
}

__global__ void k_out_phi(const double *phi64, int n, int m, double *out, int po)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    out[(long long)i * po + j] = phi64[(long long)i * m + j];
}
__global__ void k_out_mask(const double *phi64, int n, int m, uint8_t *out, int po)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    out[(long long)i * po + j] = phi64[(long long)i * m + j] > 0.0 ? 1 : 0;
}

// relative change of the paper's stopping rule: sum (phi - prev)^2, sum prev^2
__global__ void k_eta(const double *phi64, const double *prev, long long N, double *partial)
{
    __shared__ double r0[256], r1[256];
    int tid = threadIdx.x;
    double a0 = 0.0, a1 = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + tid; t < N; t += (long long)gridDim.x * blockDim.x) {
        double d = phi64[t] - prev[t];
        a0 += d * d; a1 += prev[t] * prev[t];
    }
    r0[tid] = a0; r1[tid] = a1;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) { r0[tid] += r0[tid + s]; r1[tid] += r1[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) { partial[2 * blockIdx.x] = r0[0]; partial[2 * blockIdx.x + 1] = r1[0]; }
}


// ==========================================================================
// Deviation form (mixed-precision mode).  On every level the state is
// u = b + e: b a base held fixed while the cycle is on the level (the FP64
// iterate on the finest grid, the restricted finer state on coarse grids) and
// e an FP32 deviation that starts at zero.  Writing the level's right-hand
// side as F = N_b(b) + G (G: the unprojected FP64 residual at b on the finest
// grid, the restricted projected residual on coarse grids), the frozen
// equation N_psi(b + e) = F reads, for e,
//     L_psi e = G + [L_b b - f_b] - [L_psi b - f_psi] =: T,
// with L_x y = sum over faces of a_f(x) (y_nb - y_p) and f_x = dl(x)(fit + s_x).
// T is summed in FP64 from FP32 coefficients and base differences, so no
// rounding of |b| enters and FP32 sweeps on e reach the FP64 fixed point.
// Cycle start on the finest grid: e = 0 with bounds [-M - b, M - b]; coarse
// grids: e = 0 with bounds from the finer grid's slack.

// finest-grid cycle start: e = 0, bounds of e = [-M - b, M - b]
// (32 x 32 tiles, block (32, 16) or (32, 32) as tile_rows picks; the
// column-major bounds through LDS so that both layouts are written coalesced)
__global__ void __launch_bounds__(1024) k_start0(const double *b, int n, int m, double M, float *e, float *lo,
                                                float *hi, int p, float *lo_cm, float *hi_cm, int pc)
{
    __shared__ float tlo[TILE][TILE + 1], thi[TILE][TILE + 1];
    const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int i = by + y, j = bx + threadIdx.x;
        if (i >= n || j >= m) continue;
        const double v = b[(long long)i * m + j];
        const long long q = (long long)i * p + j;
        const float l = (float)(-M - v), h = (float)(M - v);
        e[q] = 0.0f;
        lo[q] = l;
        hi[q] = h;
        tlo[y][threadIdx.x] = l;
        thi[y][threadIdx.x] = h;
    }
    __syncthreads();
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int j = bx + y, i = by + threadIdx.x;
        if (i >= n || j >= m) continue;
        const long long qc = (long long)j * pc + i;
        lo_cm[qc] = tlo[threadIdx.x][y];
        hi_cm[qc] = thi[threadIdx.x][y];
    }
}

// finest-grid cycle end: phi64 = clip(b + e) (a deviation at its bound lands
// exactly on the bound), with the sums the cycle's end needs taken in the same
// pass: sum H(phi), sum H(phi) z, sum z at the new phi (c1, c2) into pc, and
// sum (phi - b)^2, sum b^2 (the relative change eta, b being the value the
// cycle started from) into pe.  Cells go to threads as in k_sums and k_eta
// (grid-stride over the row-major index, gridDim.x x 256 threads) and the
// block sums take the same tree, so with the same grid every sum has the bits
// of those kernels run after the update.
__global__ void __launch_bounds__(256) k_finish0_sums(double *b, const float *e, const float *lo, const float *hi,
                                                      int p, const float *z, int pz, int n, int m, double M,
                                                      double eps, double *pc, double *pe)
{
    __shared__ double r0[256], r1[256], r2[256], r3[256], r4[256];
    const int tid = threadIdx.x;
    const long long N = (long long)n * m, stride = (long long)gridDim.x * blockDim.x;
    long long t = (long long)blockIdx.x * blockDim.x + tid;
    int i = (int)(t / m), j = (int)(t % m);
    const int di = (int)(stride / m), dj = (int)(stride % m);
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, d0 = 0.0, d1 = 0.0;
    for (; t < N; t += stride) {
        const long long q = (long long)i * p + j, qb = (long long)i * m + j;
        const double old = b[qb];
        const float ev = e[q];
        double v = old + (double)ev;
        if (ev >= hi[q]) v = M;
        if (ev <= lo[q]) v = -M;
        v = v < -M ? -M : (v > M ? M : v);
        b[qb] = v;
        const double H = mg_heav64(v, eps);
        const double zz = (double)z[(long long)i * pz + j];
        a0 += H; a1 += H * zz; a2 += zz;
        const double d = v - old;
        d0 += d * d; d1 += old * old;
        j += dj; i += di;
        if (j >= m) { j -= m; i++; }
    }
    r0[tid] = a0; r1[tid] = a1; r2[tid] = a2; r3[tid] = d0; r4[tid] = d1;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) {
            r0[tid] += r0[tid + s]; r1[tid] += r1[tid + s]; r2[tid] += r2[tid + s];
            r3[tid] += r3[tid + s]; r4[tid] += r4[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        pc[3 * blockIdx.x] = r0[0]; pc[3 * blockIdx.x + 1] = r1[0]; pc[3 * blockIdx.x + 2] = r2[0];
        pe[2 * blockIdx.x] = r3[0]; pe[2 * blockIdx.x + 1] = r4[0];
    }
}

template <typename BT>
struct DevArgs {
    const BT *b; int pb;                       // base and its row pitch
    const float *e, *G, *w, *fit, *lo, *hi;    // row pitch p
    float *psi, *T, *r;                        // outputs (pitch p); psi null: not written
    uint8_t *lab;                              // labels (pitch p), null: not written
    float *psi_cm, *T_cm;                      // column-major copies (pitch pc), null: not written
                                               // (T_cm null: no column-major output at all)
    uint8_t *lab_cm;
    float4 *cf, *cf_cm;                        // scaled face coefficients for the sweeps, null: not written
    int pc;
    const double *area_b, *area_u;             // Rada-Chen area terms at b and at b + e (null: 0)
    int p, n, m, scaled;
    float kap, e2, eps, Sigma;
};

// T at cell (i, j) with psi = fl32(b + e); with want_Le also L_psi e
// (FP64 sums of FP32 coefficients); u0 = psi_ij; lab = the cell's label at psi;
// au = the four face coefficients at psi scaled by kap dl(psi) (to i+1, i-1,
// j+1, j-1; 0 across the grid edge): the sweeps' frozen A, B, C, D.
// Bv, Ev, Wv: b, e, w at a cell (global memory or a staged tile).
// (dev_cell_faces: the same with the cell's face values at b and at psi given)
template <typename BT, class BV, class EV>
__device__ __forceinline__ double dev_cell_faces(const DevArgs<BT> &A, int i, int j, bool want_Le, double &Le,
                                                 float &u0, uint8_t &lab, float (&au)[4], const BV &Bv, const EV &Ev,
                                                 const float (&gb)[4], const float (&gu)[4])
{
    const int n = A.n, m = A.m;
    auto B64 = [&](int a, int c) { return (double)Bv(a, c); };
    auto E64 = [&](int a, int c) { return (double)Ev(a, c); };
    auto Bf = [&](int a, int c) { return (float)Bv(a, c); };
    auto Uf = [&](int a, int c) { return (float)(B64(a, c) + E64(a, c)); };
    const float ub = Bf(i, j);
    u0 = Uf(i, j);
    const float dlb = A.scaled ? 1.0f : mg_delta(ub, A.eps), dlu = A.scaled ? 1.0f : mg_delta(u0, A.eps);
    const float scb = A.kap * dlb, scu = A.kap * dlu;
    const long long q = (long long)i * A.p + j;
    const double b0 = B64(i, j), e0 = E64(i, j);
    const bool in[4] = {i + 1 < n, i > 0, j + 1 < m, j > 0};
    const int ni[4] = {i + 1, i - 1, i, i}, nj[4] = {j, j, j + 1, j - 1};
    double t = (double)A.G[q];
    Le = 0.0;
#pragma unroll
    for (int f = 0; f < 4; f++) au[f] = gu[f] * scu;
#pragma unroll
    for (int f = 0; f < 4; f++) {
        if (!in[f]) continue;
        const float ab = gb[f] * scb;
        t += ((double)ab - (double)au[f]) * (B64(ni[f], nj[f]) - b0);
        if (want_Le) Le += (double)au[f] * (E64(ni[f], nj[f]) - e0);
    }
    const double fit = (double)A.fit[q];
    const double sb = A.area_b ? *A.area_b : 0.0, su = A.area_u ? *A.area_u : 0.0;
    t -= (double)dlb * (fit + sb) - (double)dlu * (fit + su);
    lab = label_of(gu, n, m, i, j, A.Sigma);
    return t;
}
template <typename BT, class BV, class EV, class WV>
__device__ __forceinline__ double dev_cell_at(const DevArgs<BT> &A, int i, int j, bool want_Le, double &Le, float &u0,
                                              uint8_t &lab, float (&au)[4], const BV &Bv, const EV &Ev, const WV &Wv)
{
    auto Bf = [&](int a, int c) { return (float)Bv(a, c); };
    auto Uf = [&](int a, int c) { return (float)((double)Bv(a, c) + (double)Ev(a, c)); };
    float gb[4], gu[4];
    faces4(Bf, Wv, A.n, A.m, i, j, A.e2, gb);
    faces4(Uf, Wv, A.n, A.m, i, j, A.e2, gu);
    return dev_cell_faces(A, i, j, want_Le, Le, u0, lab, au, Bv, Ev, gb, gu);
}
template <typename BT>
__device__ __forceinline__ double dev_cell(const DevArgs<BT> &A, int i, int j, bool want_Le, double &Le, float &u0,
                                           uint8_t &lab, float (&au)[4])
{
    return dev_cell_at(
        A, i, j, want_Le, Le, u0, lab, au, [&](int a, int c) { return A.b[(long long)a * A.pb + c]; },
        [&](int a, int c) { return A.e[(long long)a * A.p + c]; },
        [&](int a, int c) { return A.w[(long long)a * A.p + c]; });
}
template <typename BT>
__device__ __forceinline__ double dev_cell(const DevArgs<BT> &A, int i, int j, bool want_Le, double &Le, float &u0,
                                           uint8_t &lab)
{
    float au[4];
    return dev_cell(A, i, j, want_Le, Le, u0, lab, au);
}

// b, e and w of the 32 x 32 tile at (by, bx) and a one-cell halo, mirrored
// at the grid edge as the face stencil mirrors, staged in LDS by the block:
// every value of the tile's stencils is then read from memory once.
template <typename BT>
__device__ __forceinline__ void stage_halo(const DevArgs<BT> &A, int by, int bx, BT (&hb)[TILE + 2][TILE + 2],
                                           float (&he)[TILE + 2][TILE + 2], float (&hw)[TILE + 2][TILE + 2])
{
    const int nt = blockDim.x * blockDim.y, tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int t = tid; t < (TILE + 2) * (TILE + 2); t += nt) {
        const int yy = t / (TILE + 2), xx = t % (TILE + 2);
        const int gi = mg_mirror(by - 1 + yy, A.n), gj = mg_mirror(bx - 1 + xx, A.m);
        hb[yy][xx] = A.b[(long long)gi * A.pb + gj];
        he[yy][xx] = A.e[(long long)gi * A.p + gj];
        hw[yy][xx] = A.w[(long long)gi * A.p + gj];
    }
}

// The face values of a staged tile at b and at psi = fl32(b + e), each face
// computed once for the two cells it separates, with the arguments faces4
// gives it (so the same values): fv[yy][x] is the face between tile rows
// yy - 1 and yy, fh[y][xx] the face between tile columns xx - 1 and xx (a face
// on the grid edge comes from the mirrored halo and is not used).  bf, uf: b
// and psi of the tile and its halo in FP32.
struct TileFaces {
    float bf[TILE + 2][TILE + 2], uf[TILE + 2][TILE + 2];
    float fvb[TILE + 1][TILE], fvu[TILE + 1][TILE], fhb[TILE][TILE + 1], fhu[TILE][TILE + 1];
};
template <typename BT>
__device__ __forceinline__ void tile_faces(const BT (&hb)[TILE + 2][TILE + 2], const float (&he)[TILE + 2][TILE + 2],
                                           const float (&hw)[TILE + 2][TILE + 2], float e2, TileFaces &F)
{
    const int nt = blockDim.x * blockDim.y, tid = threadIdx.y * blockDim.x + threadIdx.x;
    for (int t = tid; t < (TILE + 2) * (TILE + 2); t += nt) {
        const int yy = t / (TILE + 2), xx = t % (TILE + 2);
        F.bf[yy][xx] = (float)hb[yy][xx];
        F.uf[yy][xx] = (float)((double)hb[yy][xx] + (double)he[yy][xx]);
    }
    __syncthreads();
    for (int t = tid; t < (TILE + 1) * TILE; t += nt) {
        const int yy = t / TILE, x = t % TILE, y = t / (TILE + 1), xx = t % (TILE + 1);
        F.fvb[yy][x] = mg_face(F.bf[yy][x + 1], F.bf[yy + 1][x + 1], F.bf[yy][x + 2], F.bf[yy + 1][x + 2], F.bf[yy][x],
                               F.bf[yy + 1][x], hw[yy][x + 1], hw[yy + 1][x + 1], e2);
        F.fvu[yy][x] = mg_face(F.uf[yy][x + 1], F.uf[yy + 1][x + 1], F.uf[yy][x + 2], F.uf[yy + 1][x + 2], F.uf[yy][x],
                               F.uf[yy + 1][x], hw[yy][x + 1], hw[yy + 1][x + 1], e2);
        F.fhb[y][xx] = mg_face(F.bf[y + 1][xx], F.bf[y + 1][xx + 1], F.bf[y + 2][xx], F.bf[y + 2][xx + 1], F.bf[y][xx],
                               F.bf[y][xx + 1], hw[y + 1][xx], hw[y + 1][xx + 1], e2);
        F.fhu[y][xx] = mg_face(F.uf[y + 1][xx], F.uf[y + 1][xx + 1], F.uf[y + 2][xx], F.uf[y + 2][xx + 1], F.uf[y][xx],
                               F.uf[y][xx + 1], hw[y + 1][xx], hw[y + 1][xx + 1], e2);
    }
    __syncthreads();
}
// the four faces (faces4's order, zero across the grid edge) of tile cell (y, x), grid cell (i, j)
__device__ __forceinline__ void tile_cell_faces(const TileFaces &F, int y, int x, int i, int j, int n, int m,
                                                float (&gb)[4], float (&gu)[4])
{
    gb[0] = i + 1 < n ? F.fvb[y + 1][x] : 0.0f;
    gu[0] = i + 1 < n ? F.fvu[y + 1][x] : 0.0f;
    gb[1] = i > 0 ? F.fvb[y][x] : 0.0f;
    gu[1] = i > 0 ? F.fvu[y][x] : 0.0f;
    gb[2] = j + 1 < m ? F.fhb[y][x + 1] : 0.0f;
    gu[2] = j + 1 < m ? F.fhu[y][x + 1] : 0.0f;
    gb[3] = j > 0 ? F.fhb[y][x] : 0.0f;
    gu[3] = j > 0 ? F.fhu[y][x] : 0.0f;
}

// freeze in deviation form: psi = fl32(b + e), T, labels and (cf non-null)
// the sweeps' scaled face coefficients, as (to the next line, to the previous
// line, to the next cell, to the previous cell) of each layout: row-major
// (i+1, i-1, j+1, j-1), column-major (j+1, j-1, i+1, i-1).  32 x 32 tiles:
// the stencil inputs staged in LDS (stage_halo), the tile's faces computed
// once (tile_faces), row-major outputs written directly, column-major copies
// through LDS (over the face arrays, once every cell has read its faces) so
// that both layouts are written coalesced.  Block (32, 32) or (32, 16): one
// or two rows per thread.
template <typename BT>
__global__ void __launch_bounds__(1024) k_freeze_dev(DevArgs<BT> A)
{
    struct Staging {
        float tp[TILE][TILE + 1], tt[TILE][TILE + 1];
        float4 tc[TILE][TILE + 1];
        uint8_t tl[TILE][TILE + 1];
    };
    constexpr size_t UNI = sizeof(TileFaces) > sizeof(Staging) ? sizeof(TileFaces) : sizeof(Staging);
    __shared__ __align__(16) unsigned char uni[UNI];
    __shared__ BT hb[TILE + 2][TILE + 2];
    __shared__ float he[TILE + 2][TILE + 2], hw[TILE + 2][TILE + 2];
    TileFaces &F = *reinterpret_cast<TileFaces *>(uni);
    Staging &S = *reinterpret_cast<Staging *>(uni);
    const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
    stage_halo(A, by, bx, hb, he, hw);
    __syncthreads();
    tile_faces(hb, he, hw, A.e2, F);
    // grid cell (a, c) of the stencil of a tile cell lies in the staged halo
    auto Bv = [&](int a, int c) { return hb[a - by + 1][c - bx + 1]; };
    auto Ev = [&](int a, int c) { return he[a - by + 1][c - bx + 1]; };
    constexpr int RPT = 2;   // rows per thread (block (32, 16); (32, 32) uses one)
    float r_u0[RPT], r_t[RPT], r_au[RPT][4];
    uint8_t r_lab[RPT];
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int y = threadIdx.y + k * blockDim.y;
        const int i = by + y, j = bx + threadIdx.x;
        r_u0[k] = 0.0f; r_t[k] = 0.0f; r_lab[k] = 0;
        r_au[k][0] = r_au[k][1] = r_au[k][2] = r_au[k][3] = 0.0f;
        if (y < TILE && i < A.n && j < A.m) {
            double Le;
            float gb[4], gu[4];
            tile_cell_faces(F, y, threadIdx.x, i, j, A.n, A.m, gb, gu);
            const double t = dev_cell_faces(A, i, j, false, Le, r_u0[k], r_lab[k], r_au[k], Bv, Ev, gb, gu);
            r_t[k] = (float)t;
            const long long q = (long long)i * A.p + j;
            if (A.psi) A.psi[q] = r_u0[k];
            A.T[q] = r_t[k];
            A.lab[q] = r_lab[k];
            if (A.cf) A.cf[q] = make_float4(r_au[k][0], r_au[k][1], r_au[k][2], r_au[k][3]);
        }
    }
    if (!A.T_cm) return;
    __syncthreads();                 // every cell has read its faces: the staging takes their place
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int y = threadIdx.y + k * blockDim.y;
        if (y >= TILE) continue;
        S.tp[y][threadIdx.x] = r_u0[k]; S.tt[y][threadIdx.x] = r_t[k]; S.tl[y][threadIdx.x] = r_lab[k];
        S.tc[y][threadIdx.x] = make_float4(r_au[k][2], r_au[k][3], r_au[k][0], r_au[k][1]);
    }
    __syncthreads();
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int j = bx + y, i = by + threadIdx.x;
        if (i < A.n && j < A.m) {
            const long long qc = (long long)j * A.pc + i;
            if (A.psi_cm) A.psi_cm[qc] = S.tp[threadIdx.x][y];
            A.T_cm[qc] = S.tt[threadIdx.x][y];
            A.lab_cm[qc] = S.tl[threadIdx.x][y];
            if (A.cf_cm) A.cf_cm[qc] = S.tc[threadIdx.x][y];
        }
    }
}

// residual in deviation form: r = F - N(b + e) = T(b + e) - L_{b+e} e, projected
// on the bounds of e (zero where the correction would leave them).  32 x 32
// tiles, block (32, tile_rows), the stencil inputs staged in LDS (stage_halo).
// (Each cell forms its own four faces here: the shared-face staging of the
// freeze costs this kernel more in occupancy than it saves.)
template <typename BT>
__global__ void __launch_bounds__(1024) k_res_dev(DevArgs<BT> A)
{
    __shared__ BT hb[TILE + 2][TILE + 2];
    __shared__ float he[TILE + 2][TILE + 2], hw[TILE + 2][TILE + 2];
    const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
    stage_halo(A, by, bx, hb, he, hw);
    __syncthreads();
    auto Bv = [&](int a, int c) { return hb[a - by + 1][c - bx + 1]; };
    auto Ev = [&](int a, int c) { return he[a - by + 1][c - bx + 1]; };
    auto Wv = [&](int a, int c) { return hw[a - by + 1][c - bx + 1]; };
    for (int y = threadIdx.y; y < TILE; y += blockDim.y) {
        const int i = by + y, j = bx + threadIdx.x;
        if (i >= A.n || j >= A.m) continue;
        double Le;
        float u0;
        uint8_t lab;
        float au[4];
        const double t = dev_cell_at(A, i, j, true, Le, u0, lab, au, Bv, Ev, Wv);
        const long long q = (long long)i * A.p + j;
        double v = t - Le;
        const float e = A.e[q];
        if ((e >= A.hi[q] && v < 0.0) || (e <= A.lo[q] && v > 0.0)) v = 0.0;
        A.r[q] = (float)v;
    }
}

// The residual and both transfers of a level in one launch (the V-cycle's way
// down, deviation form): k_res_dev's projected residual r of every fine cell
// a coarse tile restricts, kept in LDS (the fine residual plane is not
// written), then per coarse cell (I, J)
//   G_c = FW r,  base_c = fl32(FW(b + e)) (FP64 sums),  e_c = 0,
//   lo_c = max(lo - e), hi_c = min(hi - e) over fine (2I..2I+2) x (2J..2J+2),
// the bounds also column-major through LDS.  Coarse tiles of RR_CT x RR_CT,
// block (RR_CT, RR_CT); the fine rows and columns 2 by - 1 .. 2 by + 2 RR_CT + 1
// of b, e and w staged (mirrored at the grid edge as the stencil mirrors).
// (Measured: 1320 us at 8192 x 8192 against 1457 us for the residual and
// the restriction as two launches, the same bits; staging fewer arrays or
// smaller tiles was slower.)
#define RR_CT 16
#define RR_F (2 * RR_CT + 1)          // fine cells a tile restricts, per side
#define RR_H (RR_F + 2)               // with the stencil halo
template <typename BT>
__global__ void __launch_bounds__(RR_CT *RR_CT) k_res_restrict_dev(DevArgs<BT> A, float *bc, float *ec, float *clo,
                                                                   float *chi, int pc, int nc, int mc,
                                                                   float *clo_cm, float *chi_cm, int pcc, float *Gc)
{
    __shared__ BT hb[RR_H][RR_H];
    __shared__ float he[RR_H][RR_H], hw[RR_H][RR_H], hr[RR_F][RR_F + 1];
    __shared__ float tlo[RR_CT][RR_CT + 1], thi[RR_CT][RR_CT + 1];
    const int n = A.n, m = A.m;
    const int by = blockIdx.y * RR_CT, bx = blockIdx.x * RR_CT;
    const int fy0 = 2 * by - 1, fx0 = 2 * bx - 1;
    const int nt = RR_CT * RR_CT, tid = threadIdx.y * RR_CT + threadIdx.x;
    for (int t = tid; t < RR_H * RR_H; t += nt) {
        const int yy = t / RR_H, xx = t % RR_H;
        const int gi = mg_mirror(fy0 + yy, n), gj = mg_mirror(fx0 + xx, m);
        hb[yy][xx] = A.b[(long long)gi * A.pb + gj];
        he[yy][xx] = A.e[(long long)gi * A.p + gj];
        hw[yy][xx] = A.w[(long long)gi * A.p + gj];
    }
    __syncthreads();
    auto Bv = [&](int a, int c) { return hb[a - fy0][c - fx0]; };
    auto Ev = [&](int a, int c) { return he[a - fy0][c - fx0]; };
    auto Wv = [&](int a, int c) { return hw[a - fy0][c - fx0]; };
    for (int t = tid; t < RR_F * RR_F; t += nt) {
        const int fy = t / RR_F, fx = t % RR_F;
        const int i = 2 * by + fy, j = 2 * bx + fx;
        if (i >= n || j >= m) continue;
        double Le;
        float u0;
        uint8_t lab;
        float au[4];
        const double tt = dev_cell_at(A, i, j, true, Le, u0, lab, au, Bv, Ev, Wv);
        const long long q = (long long)i * A.p + j;
        double v = tt - Le;
        const float e = A.e[q];
        if ((e >= A.hi[q] && v < 0.0) || (e <= A.lo[q] && v > 0.0)) v = 0.0;
        hr[fy][fx] = (float)v;
    }
    __syncthreads();
    const int I = by + threadIdx.y, J = bx + threadIdx.x;
    float dl = 0.0f, dh = 0.0f;
    if (I < nc && J < mc) {
        // full weighting of the staged residual (fw2's expressions)
        auto rrow = [&](int ri, int jj) {
            const float *row = hr[ri - 2 * by];
            const int c0 = 2 * jj - 2 * bx;
            if (jj < mc - 1) return 0.25f * row[c0] + 0.5f * row[c0 + 1] + 0.25f * row[c0 + 2];
            return 0.5f * row[c0] + 0.5f * row[c0 + 1];
        };
        float g;
        if (I < nc - 1) g = 0.25f * rrow(2 * I, J) + 0.5f * rrow(2 * I + 1, J) + 0.25f * rrow(2 * I + 2, J);
        else g = 0.5f * rrow(2 * I, J) + 0.5f * rrow(2 * I + 1, J);
        Gc[(long long)I * pc + J] = g;
        // full weighting of b + e in FP64 from the staged values
        auto vrow = [&](int ri, int jj) {
            auto V = [&](int c) { return (double)Bv(ri, c) + (double)Ev(ri, c); };
            if (jj < mc - 1) return 0.25 * V(2 * jj) + 0.5 * V(2 * jj + 1) + 0.25 * V(2 * jj + 2);
            return 0.5 * V(2 * jj) + 0.5 * V(2 * jj + 1);
        };
        double v;
        if (I < nc - 1) v = 0.25 * vrow(2 * I, J) + 0.5 * vrow(2 * I + 1, J) + 0.25 * vrow(2 * I + 2, J);
        else v = 0.5 * vrow(2 * I, J) + 0.5 * vrow(2 * I + 1, J);
        dl = -MG_BIG;
        dh = MG_BIG;
        for (int i = 2 * I; i <= 2 * I + 2 && i < n; i++)
            for (int j = 2 * J; j <= 2 * J + 2 && j < m; j++) {
                const long long q = (long long)i * A.p + j;
                dl = fmaxf(dl, A.lo[q] - A.e[q]);
                dh = fminf(dh, A.hi[q] - A.e[q]);
            }
        const long long qc = (long long)I * pc + J;
        bc[qc] = (float)v;
        ec[qc] = 0.0f;
        clo[qc] = dl;
        chi[qc] = dh;
    }
    tlo[threadIdx.y][threadIdx.x] = dl;
    thi[threadIdx.y][threadIdx.x] = dh;
    __syncthreads();
    const int Jt = bx + threadIdx.y, It = by + threadIdx.x;
    if (It < nc && Jt < mc) {
        clo_cm[(long long)Jt * pcc + It] = tlo[threadIdx.x][threadIdx.y];
        chi_cm[(long long)Jt * pcc + It] = thi[threadIdx.x][threadIdx.y];
    }
}

// sum of H(b + e) over a level (area term of the Rada-Chen model)
template <typename BT>
__global__ void k_sums_dev(const BT *b, int pb, const float *e, int p, int n, int m, double eps, double *partial)
{
    __shared__ double r0[256];
    int tid = threadIdx.x;
    long long N = (long long)n * m;
    double a0 = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + tid; t < N; t += (long long)gridDim.x * blockDim.x) {
        int i = (int)(t / m), j = (int)(t % m);
        a0 += mg_heav64((double)b[(long long)i * pb + j] + (double)e[(long long)i * p + j], eps);
    }
    r0[tid] = a0;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (tid < s) r0[tid] += r0[tid + s];
        __syncthreads();
    }
    if (tid == 0) {
        partial[3 * blockIdx.x] = r0[0];
        partial[3 * blockIdx.x + 1] = 0.0;
        partial[3 * blockIdx.x + 2] = 0.0;
    }
}

// ==========================================================================
// Outer iterations of Hybrid Smoother 2 (freeze + sweeps A, B, C, D) on a
// small grid in one workgroup, exactly the steps of the multi-kernel path,
// with block barriers in place of kernel boundaries and every array of the
// level staged in LDS; at most `iters` of them, stopping after the first
// iteration that moves no value by more than rtol times the largest change
// since the workgroup began (rtol = 0: all `iters`, with no test).  The coarsest
// solve and the smoothing of the small grids.  Each wave of the NT threads
// takes bands of 4 lines (lines of at most 64 cells, one wave each).
struct CoarseArgs {
    float *P0;                      // state in / out (row pitch prm)
    const float *w, *fit, *lo, *hi; // row-major, pitch prm
    const float *F;                 // FP32 mode: F (may be null)
    const float *base, *G;          // deviation form (P0 holds e); null base: FP32 mode
    const double *area_b;           // deviation form, Rada-Chen: area term at the base
    double *area;                   // slot for the area term (Rada-Chen), may be null
    double h2, A1, nu, eps;
    int n, m, prm, iters, scaled;
    float kap, e2, M, Sigma, rtol;
    int smoother;                   // 1: GSLEX-I (sweep A's order, every cell a point) in place of HS2
    int run_max;                    // 0: maximal runs of starred cells; else the cut (LineArgs::run_max)
};
#define CO_ARRAYS 18
#define CO_MAX_CELLS 1024
// dynamic LDS: [two float4 coefficient arrays][CO_ARRAYS float arrays][two label arrays]
__host__ __device__ inline size_t coarse_lds_bytes(int n, int m)
{
    const size_t N = (size_t)n * m;
    return 2 * N * sizeof(float4) + CO_ARRAYS * N * sizeof(float) + ((2 * N + 7) / 8) * 8;
}

// largest change of the state over one outer iteration and since the
// coarsest solve began (multi-kernel coarsest path); once the change is at
// most rtol times the total change, *stop is set and the remaining sweeps of
// the coarsest solve return at once (no host synchronisation)
__global__ void __launch_bounds__(256) k_coarse_delta(const float *x, const float *prev, const float *entry, int p,
                                                      int n, int m, double rtol, int *stop)
{
    __shared__ float r0[256], r1[256];
    const int t = threadIdx.x;
    float a = 0.0f, b = 0.0f;
    for (int q = t; q < n * m; q += 256) {
        const int k = (q / m) * p + q % m;
        a = fmaxf(a, fabsf(x[k] - prev[k]));
        b = fmaxf(b, fabsf(x[k] - entry[k]));
    }
    r0[t] = a; r1[t] = b;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) { r0[t] = fmaxf(r0[t], r0[t + s]); r1[t] = fmaxf(r1[t], r1[t + s]); }
        __syncthreads();
    }
    if (t == 0 && (double)r0[0] <= rtol * (double)r1[0]) stop[0] = 1;
}

// ==========================================================================
// Hybrid Smoother 1, step II (Sec. 4.2, eqs. caseAlagged .. caseDlagged): at
// a jump-set cell whose smallest coefficient is s, the cell and its three
// neighbours other than the one behind s are updated collectively (the
// neighbour behind s is lagged).  Each neighbour's row is its own equation
// (its coefficient towards the centre; with delta-scaled rows the centre's
// towards it, as the paper's arrow matrices write it), every other cell at its
// current value.  In the deviation form the rows are those of the freeze:
//   sum_f a_f e_nb - S e = T   (a_f the stored scaled face coefficients).
// The box-constrained block is solved exactly: a leaf k is the clipped ramp
// x_k = clip(al_k y + be_k, lo_k, hi_k) of the centre value y, so the centre
// solves y = clip(g(y), lo, hi) with g monotone piecewise linear of slope
// below one (diagonal dominance); y - clip(g(y)) increases, and its root lies
// on the linear piece between the largest candidate (the leaves' kinks and
// the centre's bounds) where it is <= 0 and the smallest where it is >= 0.
// Cells of class (i + 3 j) mod 8 = cls only: two of them are at least four
// cells apart, so the blocks of one launch share no cell and read none that
// another writes.
// NEWT (eq. newtrc): the derivative Q' in phi_ij of the Rada-Chen area term at the
// frozen state psi = b + e (b null: psi = e): rows scaled by delta_eps, the row's
// area term 2 nu (h^2 sum H - A1) gives Q' = 2 nu h^2 delta_eps(psi); unscaled rows
// carry delta_eps(psi) times it, Q' = 2 nu h^2 delta_eps^2 + delta_eps'(psi) area.
template <typename BT>
__global__ void k_newton_diag(const BT *b, int pb, const float *e, int p, int n, int m, double h2nu2, double eps,
                              int scaled, const double *area, float *qd)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    const double psi = (b ? (double)b[(long long)i * pb + j] : 0.0) + (double)e[(long long)i * p + j];
    const double d = mg_delta64(psi, eps);
    double v = h2nu2 * d;
    if (!scaled) v = v * d - 2.0 * psi * d * d * MG_PI / eps * (*area);
    qd[(long long)i * p + j] = (float)v;
}

struct BlockArgs {
    float *e;                    // row-major state (pitch p)
    const float4 *cf;            // frozen scaled face coefficients: to i+1, i-1, j+1, j-1
    const float *T, *lo, *hi;    // right-hand side and bounds of the rows
    const uint8_t *lab;          // labels: bit s = jump set with smallest coefficient s
    const int *skip;             // non-null and set: the launch does nothing
    int p, n, m, cls;
};
__device__ __forceinline__ float blk_coef(const float4 &g, int s)
{
    return s == 0 ? g.x : (s == 1 ? g.y : (s == 2 ? g.z : g.w));
}
__global__ void __launch_bounds__(256) k_hs1_blocks(BlockArgs B)
{
    if (B.skip && *B.skip) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (i >= B.n || j >= B.m || ((i + 3 * j) & 7) != B.cls) return;
    const long long q0 = (long long)i * B.p + j;
    const unsigned lb = B.lab[q0];
    if (!lb) return;
    const int lag = (lb & 1) ? 0 : ((lb & 2) ? 1 : ((lb & 4) ? 2 : 3));
    const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1}, back[4] = {1, 0, 3, 2};
    auto inside = [&](int a, int b) { return a >= 0 && a < B.n && b >= 0 && b < B.m; };
    const float4 g0 = B.cf[q0];
    const float S0 = g0.x + g0.y + g0.z + g0.w;
    if (!(S0 > 0.0f)) return;
    // centre row: sum over leaves a_k x_k - S0 y = T0 - a_lag e_lag
    float rhs0 = B.T[q0];
    if (inside(i + di[lag], j + dj[lag]))
        rhs0 -= blk_coef(g0, lag) * B.e[(long long)(i + di[lag]) * B.p + j + dj[lag]];
    float gam[3], al[3], be[3], llo[3], lhi[3];
    long long lq[3];
    int nl = 0;
    for (int s = 0; s < 4; s++) {
        if (s == lag) continue;
        const int a = i + di[s], b = j + dj[s];
        if (!inside(a, b)) continue;
        const long long q = (long long)a * B.p + b;
        const float4 g = B.cf[q];
        const float S = g.x + g.y + g.z + g.w;
        if (!(S > 0.0f)) return;
        // leaf row: a_(leaf -> centre) y - S x = T - (its other neighbours at their values)
        float r = B.T[q];
        for (int t = 0; t < 4; t++) {
            if (t == back[s]) continue;
            const int c2 = a + di[t], d2 = b + dj[t];
            if (inside(c2, d2)) r -= blk_coef(g, t) * B.e[(long long)c2 * B.p + d2];
        }
        const float inv = 1.0f / S;
        gam[nl] = blk_coef(g0, s) / S0;
        al[nl] = blk_coef(g, back[s]) * inv;
        be[nl] = -r * inv;
        llo[nl] = B.lo[q]; lhi[nl] = B.hi[q];
        lq[nl] = q;
        nl++;
    }
    const float be0 = -rhs0 / S0, lo0 = B.lo[q0], hi0 = B.hi[q0];
    auto leaf = [&](int k, float y) { return mg_clip(fmaf(al[k], y, be[k]), llo[k], lhi[k]); };
    auto g_of = [&](float y) {
        float v = be0;
        for (int k = 0; k < nl; k++) v = fmaf(gam[k], leaf(k, y), v);
        return v;
    };
    auto psi = [&](float y) { return y - mg_clip(g_of(y), lo0, hi0); };
    // candidates: the leaves' kinks and the centre's bounds
    float plo = lo0, phi = hi0;
    for (int k = 0; k < nl; k++) {
        if (!(al[k] > 0.0f)) continue;
        const float ia = 1.0f / al[k];
        const float c2[2] = {(llo[k] - be[k]) * ia, (lhi[k] - be[k]) * ia};
        for (int t = 0; t < 2; t++) {
            const float pc = mg_clip(c2[t], lo0, hi0);
            const float v = psi(pc);
            if (v <= 0.0f && pc > plo) plo = pc;
            if (v >= 0.0f && pc < phi) phi = pc;
        }
    }
    float y;
    if (psi(lo0) >= 0.0f) y = lo0;
    else if (psi(hi0) <= 0.0f) y = hi0;
    else if (!(phi > plo)) y = plo;
    else {
        // g on (plo, phi): each leaf either at a bound or on its ramp
        const float mid = 0.5f * (plo + phi);
        float sl = 0.0f, c0 = be0;
        for (int k = 0; k < nl; k++) {
            const float v = fmaf(al[k], mid, be[k]);
            if (v <= llo[k]) c0 = fmaf(gam[k], llo[k], c0);
            else if (v >= lhi[k]) c0 = fmaf(gam[k], lhi[k], c0);
            else { sl = fmaf(gam[k], al[k], sl); c0 = fmaf(gam[k], be[k], c0); }
        }
        y = mg_clip(mg_clip(c0 / (1.0f - sl), lo0, hi0), plo, phi);
    }
    B.e[q0] = y;
    for (int k = 0; k < nl; k++) B.e[lq[k]] = leaf(k, y);
}

__global__ void k_set_int(int *p, int v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

template <int NT>
__device__ void block_transpose(const float *in, int pin, float *out, int pout, int n, int m)
{
    for (int t = threadIdx.x; t < n * m; t += NT) {
        int i = t / m, j = t % m;
        out[j * pout + i] = in[i * pin + j];
    }
}

template <int NT>
__global__ void __launch_bounds__(NT) k_coarse_smooth(CoarseArgs G)
{
    __shared__ Ramp sh[2 * (NT / 64 > 0 ? NT / 64 : 1)];
    __shared__ double red[NT];
    __shared__ float rdt[NT];
    __shared__ float rb[2 * RB_FIELDS * NT];
    __shared__ uint64_t msk[(NT + 63) / 64];
    extern __shared__ float4 co4[];
    const int n = G.n, m = G.m, N = n * m, tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, so bands stay scalar
    constexpr int NWV = NT / 64;
    const bool dev = G.base != nullptr;
    // LDS arrays: row-major with pitch m, column-major with pitch n.  cf / cf_cm: the
    // frozen scaled face coefficients of each layout, (to the next line, to the previous
    // line, to the next cell, to the previous cell); Fe / Fe_cm: F plus the fit term.
    float4 *cf = co4, *cf_cm = co4 + N;
    float *co = reinterpret_cast<float *>(co4 + 2 * N);
    float *P0 = co, *P1 = co + N, *P2 = co + 2 * N, *T1 = co + 3 * N, *T2 = co + 4 * N;
    float *psi = co + 5 * N, *w = co + 6 * N, *fit = co + 7 * N;
    float *lo = co + 8 * N, *lo_cm = co + 9 * N, *hi = co + 10 * N, *hi_cm = co + 11 * N;
    float *F = co + 12 * N, *Fe = co + 13 * N, *Fe_cm = co + 14 * N, *base = co + 15 * N, *Gv = co + 16 * N;
    float *E = co + 17 * N;
    uint8_t *lab = reinterpret_cast<uint8_t *>(co + CO_ARRAYS * N), *lab_cm = lab + N;
    for (int t = tid; t < N; t += NT) {
        const int i = t / m, j = t % m, qg = i * G.prm + j, qr = t, qc = j * n + i;
        P0[qr] = E[qr] = G.P0[qg];
        w[qr] = G.w[qg];
        fit[qr] = G.fit[qg];
        lo[qr] = lo_cm[qc] = G.lo[qg];
        hi[qr] = hi_cm[qc] = G.hi[qg];
        F[qr] = (!dev && G.F) ? G.F[qg] : 0.0f;
        base[qr] = dev ? G.base[qg] : 0.0f;
        Gv[qr] = dev ? G.G[qg] : 0.0f;
    }
    __syncthreads();
    // each wave's row buffers, mask word and scan totals
    RunBuf RBr, RBc;
    RBr.p = rb + wave * 2 * RB_FIELDS * 64; RBr.fs = m;
    RBc.p = RBr.p; RBc.fs = n;
    uint64_t *mskw = msk + wave;
    Ramp *shw = sh + 2 * wave;
    // C: the row-major arguments the freeze evaluates the coefficients with; R / T: the
    // row and column sweeps, which read the stored coefficients
    LineArgs C, R, T;
    C.psi = psi; C.w = w; C.fit = dev ? nullptr : fit; C.F = F; C.lab = lab; C.lo = lo; C.hi = hi;
    C.skip = nullptr; C.tout = nullptr; C.tpitch = 0; C.area = G.area; C.pitch = m; C.lpitch = m; C.cf = nullptr;
    C.qd = nullptr; C.split = 0; C.nb_old = nullptr;
    C.nl = n; C.ml = m; C.kap = G.kap; C.e2 = G.e2; C.M = G.M; C.eps = (float)G.eps; C.scaled = G.scaled;
    C.run_max = G.run_max;
    C.phi_old = P0; C.phi_new = nullptr; C.bit = 0;
    R = C;
    R.psi = nullptr; R.w = nullptr; R.fit = nullptr; R.F = Fe; R.cf = cf;
    T = R;
    T.F = Fe_cm; T.cf = cf_cm; T.lab = lab_cm; T.lo = lo_cm; T.hi = hi_cm; T.pitch = n; T.lpitch = n; T.nl = m;
    T.ml = n;
    DevArgs<float> D;
    D.b = base; D.pb = m; D.e = P0; D.G = Gv; D.w = w; D.fit = fit; D.lo = lo; D.hi = hi;
    D.psi = nullptr; D.T = nullptr; D.r = nullptr; D.lab = nullptr;
    D.psi_cm = nullptr; D.T_cm = nullptr; D.lab_cm = nullptr; D.pc = n; D.cf = nullptr; D.cf_cm = nullptr;
    D.area_b = G.area_b; D.area_u = G.area;
    D.p = m; D.n = n; D.m = m; D.scaled = G.scaled;
    D.kap = G.kap; D.e2 = G.e2; D.eps = (float)G.eps; D.Sigma = G.Sigma;
    for (int it = 0; it < G.iters; it++) {
        // freeze
        double acc = 0.0;
        if (G.area) {
            for (int t = tid; t < N; t += NT)
                acc += mg_heav64(dev ? (double)base[t] + (double)P0[t] : (double)P0[t], G.eps);
            red[tid] = acc;
            __syncthreads();
            if (tid == 0) {
                double s = 0.0;
                for (int k = 0; k < NT; k++) s += red[k];
                *G.area = 2.0 * G.nu * (G.h2 * s - G.A1);
            }
            __syncthreads();
        }
        if (dev) {
            for (int t = tid; t < N; t += NT) {
                const int i = t / m, j = t % m, qc = j * n + i;
                double Le;
                float u0;
                uint8_t b;
                const double tv = dev_cell(D, i, j, false, Le, u0, b);
                psi[t] = u0;
                F[t] = (float)tv;
                lab[t] = b; lab_cm[qc] = b;
            }
        } else {
            for (int t = tid; t < N; t += NT) psi[t] = P0[t];
            __syncthreads();
            for (int t = tid; t < N; t += NT) {
                const int i = t / m, j = t % m;
                const uint8_t b = cell_label(psi, w, m, n, m, i, j, G.e2, G.Sigma);
                lab[t] = b;
                lab_cm[j * n + i] = b;
            }
        }
        __syncthreads();
        // the frozen scaled face coefficients and F plus the fit term of every cell, once for the
        // four sweeps, in both layouts (the products the sweeps would form, so the same bits)
        {
            const float area = G.area ? (float)(*G.area) : 0.0f;
            for (int t = tid; t < N; t += NT) {
                const int i = t / m, j = t % m, qc = j * n + i;
                CellIn c;
                cell_load<false, false>(line_rows<false>(C, i, true, true), m, j, c);
                float xp, xm, lp, lm, f;
                cell_coef<false>(C, c, i, j, area, xp, xm, lp, lm, f);
                cf[t] = make_float4(xp, xm, lp, lm);
                cf_cm[qc] = make_float4(lp, lm, xp, xm);
                const float fe = f + c.F;
                Fe[t] = fe;
                Fe_cm[qc] = fe;
            }
        }
        __syncthreads();
        // sweeps A and B (rows); the sweep output is read by the next sweep
        // after a barrier (the bands of one sweep read only its input)
        int lpar = 0;
        R.phi_old = P0; R.phi_new = P1; R.bit = G.smoother == 1 ? LAB_NONE : 0;
        for (int b = wave; b < (n + 3) / 4; b += NWV)
            sweep_band<64, false, true, true, true>(R, b, RBr, mskw, shw, nullptr, nullptr, lpar);
        __syncthreads();
        if (G.smoother == 1) {
            // GSLEX-I: the pass of sweep A is the whole outer iteration
            block_transpose<NT>(P1, m, T1, n, n, m);
            __syncthreads();
        } else {
            R.phi_old = P1; R.phi_new = P2; R.bit = 1;
            for (int b = wave; b < (n + 3) / 4; b += NWV)
                sweep_band<64, true, true, true, true>(R, b, RBr, mskw, shw, nullptr, nullptr, lpar);
            __syncthreads();
            block_transpose<NT>(P2, m, T1, n, n, m);
            __syncthreads();
            // sweeps C and D (columns)
            T.phi_old = T1; T.phi_new = T2; T.bit = 2;
            for (int b = wave; b < (m + 3) / 4; b += NWV)
                sweep_band<64, false, true, true, true>(T, b, RBc, mskw, shw, nullptr, nullptr, lpar);
            __syncthreads();
            T.phi_old = T2; T.phi_new = T1; T.bit = 3;
            for (int b = wave; b < (m + 3) / 4; b += NWV)
                sweep_band<64, true, true, true, true>(T, b, RBc, mskw, shw, nullptr, nullptr, lpar);
            __syncthreads();
        }
        float dmax = 0.0f, tot = 0.0f;
        for (int t = tid; t < N; t += NT) {
            const int i = t / m, j = t % m;
            const float v = T1[j * n + i];
            dmax = fmaxf(dmax, fabsf(v - P0[t]));
            tot = fmaxf(tot, fabsf(v - E[t]));
            P0[t] = v;
        }
        if (!(G.rtol > 0.0f)) {
            // no stopping test: an iteration that moves nothing leaves every further one the same
            __syncthreads();
            continue;
        }
        red[tid] = (double)dmax;
        rdt[tid] = tot;
        __syncthreads();
        for (int s = NT / 2; s > 0; s >>= 1) {
            if (tid < s) { red[tid] = fmax(red[tid], red[tid + s]); rdt[tid] = fmaxf(rdt[tid], rdt[tid + s]); }
            __syncthreads();
        }
        const bool stop = red[0] <= (double)G.rtol * (double)rdt[0];
        __syncthreads();
        if (stop) break;
    }
    for (int t = tid; t < N; t += NT) G.P0[(t / m) * G.prm + t % m] = P0[t];
}

// network input of the finest grid: z, d, marker mask (1 at a marker's cell)
__global__ void k_features(const float *z, const float *d, int p, int n, int m, const double *mk, int k, float *out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= m || i >= n) return;
    const long long q = (long long)i * m + j, HW = (long long)n * m;
    out[q] = z[(long long)i * p + j];
    out[HW + q] = d[(long long)i * p + j];
    float mk1 = 0.0f;
    for (int t = 0; t < k; t++)
        if ((int)floor(mk[2 * t]) == i && (int)floor(mk[2 * t + 1]) == j) mk1 = 1.0f;
    out[2 * HW + q] = mk1;
}

// flag = 1 if phi (dense n x m) is positive at the cell of every marker (row, col), else 0.
// One block of 256 threads.
__global__ void k_markers_inside(const float *phi, int n, int m, const double *mk, int k, int *flag)
{
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < k; t += blockDim.x) {
        const long long i = (long long)floor(mk[2 * t]), j = (long long)floor(mk[2 * t + 1]);
        if (i < 0 || i >= n || j < 0 || j >= m || !(phi[i * m + j] > 0.0f)) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = bad ? 0 : 1;
}

// The model's discrete energy at the finest FP64 phi (Sec. 2, the functional
// whose Euler-Lagrange equation the cycle solves): per cell h^2 times
//   mu w delta_eps(phi) |grad phi| + lambda1 (z - c1)^2 H + lambda2 (z - c2)^2 (1 - H) (+ theta d H, Spencer-Chen)
// with central differences at mirrored edges and w = g (Spencer-Chen) or g d
// (Rada-Chen).  Per-block partials of the sum and of sum H, in FP64.
struct EnergyArgs {
    const double *phi, *g, *d, *dsc;
    const float *z;
    int pz, n, m, model;
    double h, mu, lambda1, lambda2, theta, eps;
    double *partial;
};
// The model's discrete energy (eq. scfunc / rcfunc) at the FP64 finest phi:
// per cell, the length term mu w delta(phi) |grad phi| (|grad H(phi)| by the
// chain rule, central differences in domain units, mirrored edges) plus the
// region terms H (lambda1 (z - c1)^2 [+ theta d]) + (1 - H) lambda2 (z - c2)^2,
// times the cell area h^2 (applied in k_energy_final with the Rada-Chen area
// penalty).  One 32 x 32 tile per block with its mirrored halo of phi in LDS;
// each block writes the sums of its tile (energy, sum of H) as one partial.
__global__ void __launch_bounds__(256) k_energy(EnergyArgs A)
{
    __shared__ double ph[TILE + 2][TILE + 3];
    __shared__ double wsum[2][256 / 64];
    const int i0 = blockIdx.y * TILE, j0 = blockIdx.x * TILE, n = A.n, m = A.m;
    for (int t = threadIdx.x; t < (TILE + 2) * (TILE + 2); t += blockDim.x) {
        const int ti = t / (TILE + 2), tj = t % (TILE + 2);
        ph[ti][tj] = A.phi[(long long)mg_mirror(i0 + ti - 1, n) * m + mg_mirror(j0 + tj - 1, m)];
    }
    __syncthreads();
    const double c1 = A.dsc[0], c2 = A.dsc[1], inv2h = 0.5 / A.h;
    double en = 0.0, hs = 0.0;
    for (int t = threadIdx.x; t < TILE * TILE; t += blockDim.x) {
        const int ti = t / TILE, tj = t % TILE, i = i0 + ti, j = j0 + tj;
        if (i >= n || j >= m) continue;
        const long long q = (long long)i * m + j;
        const double p0 = ph[ti + 1][tj + 1];
        const double px = (ph[ti + 1][tj + 2] - ph[ti + 1][tj]) * inv2h;
        const double py = (ph[ti + 2][tj + 1] - ph[ti][tj + 1]) * inv2h;
        const double heav = mg_heav64(p0, A.eps);
        const double zv = (double)A.z[(long long)i * A.pz + j];
        const double in_term = A.lambda1 * (zv - c1) * (zv - c1) + (A.model == 0 ? A.theta * A.d[q] : 0.0);
        const double out_term = A.lambda2 * (zv - c2) * (zv - c2);
        const double weight = A.model == 1 ? A.g[q] * A.d[q] : A.g[q];
        en += A.mu * weight * mg_delta64(p0, A.eps) * sqrt(px * px + py * py) + heav * in_term + (1.0 - heav) * out_term;
        hs += heav;
    }
    // wave sums by lane exchange, then the block's four waves in order
    for (int o = 32; o > 0; o >>= 1) {
        en += __shfl_down(en, o, 64);
        hs += __shfl_down(hs, o, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { wsum[0][wv] = en; wsum[1][wv] = hs; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = 0.0, s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); k++) { e += wsum[0][k]; s += wsum[1][k]; }
        const int b = blockIdx.y * gridDim.x + blockIdx.x;
        A.partial[2 * b] = e;
        A.partial[2 * b + 1] = s;
    }
}

// adds the nb partials of k_energy in a fixed order: out = h^2 sum + (Rada-Chen) nu (a1^2 + a2^2),
// a1 = h^2 sum H - A1, a2 = h^2 (N - sum H) - (1 - A1)
__global__ void __launch_bounds__(256) k_energy_final(const double *partial, int nb, double h2, double N, int model,
                                                      double nu, double A1, double *out)
{
    __shared__ double r0[256], r1[256];
    const int tid = threadIdx.x;
    double e = 0.0, sh = 0.0;
    for (int b = tid; b < nb; b += 256) { e += partial[2 * b]; sh += partial[2 * b + 1]; }
    r0[tid] = e; r1[tid] = sh;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) { r0[tid] += r0[tid + s]; r1[tid] += r1[tid + s]; }
        __syncthreads();
    }
    if (tid == 0) {
        double E = r0[0] * h2;
        if (model == 1) {
            const double a1 = h2 * r1[0] - A1, a2 = h2 * (N - r1[0]) - (1.0 - A1);
            E += nu * (a1 * a1 + a2 * a2);
        }
        out[0] = E;
    }
}

// per-block counts of the nonzero labels of an n x m byte grid with row pitch p
__global__ void __launch_bounds__(256) k_count_labels(const uint8_t *lab, int p, int n, int m, double *partial)
{
    __shared__ double r[256];
    const int tid = threadIdx.x;
    const long long N = (long long)n * m;
    double cnt = 0.0;
    for (long long t = (long long)blockIdx.x * blockDim.x + tid; t < N; t += (long long)gridDim.x * blockDim.x)
        cnt += lab[(t / m) * p + t % m] != 0 ? 1.0 : 0.0;
    r[tid] = cnt;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) r[tid] += r[tid + s];
        __syncthreads();
    }
    if (tid == 0) partial[blockIdx.x] = r[0];
}
