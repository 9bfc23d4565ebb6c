// The local ("-II") smoothers of Sec. 3.2: a pixel's (GSLEX-II) or a
// column's (GSLINE-II) coefficients of eq. abcdrc are refreshed from the
// current iterate right before they are used, instead of once per outer
// iteration.  Deviation form (psi = b + e), Spencer-Chen rows (no global
// area sum, whose running refresh would order every pixel after every other).
//
// Order: the lines of the four classes (index mod 4) of the parallel sweeps,
// class after class.  The lines of one class share no stencil cell (a
// pixel's coefficients and update read its 3 x 3 neighbourhood), so every
// line of a class is updated at once and the result equals the sequential
// order line by line.
//
// GSLEX-II: one thread per row of the class, walking its row left to right:
// at each pixel the refreshed row (the face coefficients au and the
// right-hand side T at the current b + e) and the point update
//   e_ij <- clip((sum au e_nb - T) / sum au, lo, hi),
// the left neighbour already updated.  A row is inherently sequential (the
// next pixel's coefficients depend on this pixel's new value), so the pass
// costs one pixel-step per column of every class, latency-bound.
//
// GSLINE-II: one workgroup per column of the class, one thread per cell: the
// column's refreshed rows, then the column's box-constrained tridiagonal
// system through the whole-line path of the directional sweep (every cell
// starred), written in place.
#pragma once
#include "mgseg_kernels.h"

// skip: non-null and set, the launch does nothing (the coarsest solve's stop)
//
// The thread keeps b, e and w of its 3 x 3 stencil in registers (columns
// j-1, j, j+1 of rows i-1, i, i+1; the half-sample mirror at the grid edge
// names the cell itself, so an edge never needs the slot beyond it) and
// reads column j+2 one step ahead, so a step waits on no memory: its own
// row's left neighbour is the value it has just written.  The values are
// those of global memory at that point of the walk, so the result is the
// same bit for bit as reading them there.
// (Named scalars rather than arrays, whose selects the compiler turned into
// indexed loads from scratch memory; the FP32 build keeps the window in
// registers, the FP64 one of the finest grid still holds 40 bytes of it in
// scratch.)
template <typename T>
struct Win3 {
    T u0, u1, u2, c0, c1, c2, d0, d1, d2;    // rows i-1, i, i+1 (mirrored) x columns j-1, j, j+1
    __device__ __forceinline__ T at(int a, int c, int i, int j) const
    {
        const T vu = c < j ? u0 : (c == j ? u1 : u2);
        const T vc = c < j ? c0 : (c == j ? c1 : c2);
        const T vd = c < j ? d0 : (c == j ? d1 : d2);
        return a < i ? vu : (a == i ? vc : vd);
    }
    __device__ __forceinline__ void shift(T nu, T nc, T nd)
    {
        u0 = u1; u1 = u2; u2 = nu;
        c0 = c1; c1 = c2; c2 = nc;
        d0 = d1; d1 = d2; d2 = nd;
    }
};

template <typename BT>
__global__ void __launch_bounds__(64) k_gslex_local(DevArgs<BT> A, int cls, const int *skip)
{
    if (skip && *skip) return;
    const int i = cls + 4 * (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= A.n) return;
    float *e = const_cast<float *>(A.e);
    const int n = A.n, m = A.m;
    const long long row = (long long)i * A.p;
    const long long ru = (long long)mg_mirror(i - 1, n), rd = (long long)mg_mirror(i + 1, n);
    const long long pu = ru * A.p, pd = rd * A.p, bu = ru * A.pb, bc = (long long)i * A.pb, bd = rd * A.pb;
    Win3<BT> wb;
    Win3<float> we, ww;
    // column c of the three rows (past the edge: a column that is never read)
    BT nbu, nbc, nbd;
    float neu, nec, ned, nwu, nwc, nwd;
    auto fetch = [&](int c) {
        const int cc = c < m ? c : m - 1;
        nbu = A.b[bu + cc]; nbc = A.b[bc + cc]; nbd = A.b[bd + cc];
        neu = e[pu + cc]; nec = e[row + cc]; ned = e[pd + cc];
        nwu = A.w[pu + cc]; nwc = A.w[row + cc]; nwd = A.w[pd + cc];
    };
    fetch(0);
    wb.shift(nbu, nbc, nbd); we.shift(neu, nec, ned); ww.shift(nwu, nwc, nwd);
    wb.shift(nbu, nbc, nbd); we.shift(neu, nec, ned); ww.shift(nwu, nwc, nwd);
    fetch(1);
    wb.shift(nbu, nbc, nbd); we.shift(neu, nec, ned); ww.shift(nwu, nwc, nwd);
    for (int j = 0; j < m; j++) {
        fetch(j + 2);
        // stencil cell (a, c): after mirroring one of (i - 1 | i | i + 1) x (j - 1 | j | j + 1)
        auto Bv = [&](int a, int c) { return wb.at(a, c, i, j); };
        auto Ev = [&](int a, int c) { return we.at(a, c, i, j); };
        auto Wv = [&](int a, int c) { return ww.at(a, c, i, j); };
        double Le;
        float u0, au[4];
        uint8_t lab;
        const double t = dev_cell_at(A, i, j, false, Le, u0, lab, au, Bv, Ev, Wv);
        const float S = au[0] + au[1] + au[2] + au[3];
        if (S > 0.0f) {
            float v = -(float)t;
            if (i + 1 < n) v = fmaf(au[0], we.d1, v);
            if (i > 0) v = fmaf(au[1], we.u1, v);
            if (j + 1 < m) v = fmaf(au[2], we.c2, v);
            if (j > 0) v = fmaf(au[3], we.c0, v);
            we.c1 = mg_clip(v / S, A.lo[row + j], A.hi[row + j]);
            e[row + j] = we.c1;
        }
        wb.shift(nbu, nbc, nbd); we.shift(neu, nec, ned); ww.shift(nwu, nwc, nwd);
    }
}

// L: the column sweep's arguments (nl = m lines of ml = n cells, bit LAB_ALL,
// tout = e row-major); one workgroup of NT >= n threads per column
template <int NT, typename BT>
__global__ void __launch_bounds__(NT) k_gsline_local(DevArgs<BT> A, LineArgs L, int cls)
{
    if (L.skip && *L.skip) return;
    extern __shared__ uint64_t smem64[];
    __shared__ Ramp wtot[2 * (NT / 64)];
    __shared__ unsigned wbad[NT / 64];
    __shared__ Elim etot[NT / 64];
    const int j = cls + 4 * (int)blockIdx.x;
    if (j >= A.m) return;
    const int i = threadIdx.x;
    uint64_t *msk = smem64;
    RunBuf B;
    B.fs = A.n;
    B.p = reinterpret_cast<float *>(smem64 + sweep_mask_words(A.n));
    CellIn c{};
    if (i < A.n) {
        double Le;
        float u0, au[4];
        uint8_t lab;
        const double t = dev_cell(A, i, j, false, Le, u0, lab, au);
        const long long q = (long long)i * A.p + j;
        // (to the next line j+1, the previous line j-1, the next cell i+1, the previous cell i-1)
        c.g = make_float4(au[2], au[3], au[0], au[1]);
        c.F = (float)t;
        c.vu = j > 0 ? A.e[q - 1] : 0.0f;
        c.vd = j + 1 < A.m ? A.e[q + 1] : 0.0f;
        c.sig = i + 1 < A.n ? A.e[q + A.p] : 0.0f;
        c.pold = A.e[q];
        c.lo = A.lo[q];
        c.hi = A.hi[q];
        c.lab = 0;
        c.qd = 0.0f;
    }
    sweep_line<NT, false, true, NT == 64, true>(L, j, B, msk, true, 0.0f, false, 0.0f, false, wtot, wbad, etot, c,
                                                i, true);
}

inline size_t gsline_local_lds(int n)
{
    return sizeof(uint64_t) * (size_t)sweep_mask_words(n) + sizeof(float) * (size_t)RB_FIELDS * n;
}
