// mgseg_device.h -- device code of libmgseg (gfx950, wave64).
//
// Grid arrays are FP32 in one of two layouts: row-major ("rm": element
// (i, j) at i*pitch + j) and column-major ("cm": element (i, j) at
// j*pitch + i).  The smoother works on "lines": in rm the lines are rows and
// the in-line index is j, in cm the lines are columns and the in-line index
// is i; a single line kernel serves all four directional sweeps of Hybrid
// Smoother 2 by reading the arrays of the matching layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MG_PI 3.14159265358979323846
#define MG_BIG 1.0e30f

// --------------------------------------------------------------------------
// smoothed Heaviside and delta (Sec. 2: H = 1/2 + atan(phi/eps)/pi)
__device__ __forceinline__ float mg_delta(float phi, float eps)
{
    return eps / ((float)MG_PI * (eps * eps + phi * phi));
}
__device__ __forceinline__ double mg_delta64(double phi, double eps)
{
    return eps / (MG_PI * (eps * eps + phi * phi));
}
__device__ __forceinline__ double mg_heav64(double phi, double eps)
{
    return 0.5 + atan(phi / eps) / MG_PI;
}
__device__ __forceinline__ int mg_mirror(int t, int n)
{
    // half-sample mirror of the cell-centred Neumann boundary (|t| < 2n)
    if (t < 0) t = -t - 1;
    if (t >= n) t = 2 * n - t - 1;
    return t < 0 ? 0 : (t >= n ? n - 1 : t);
}
// clip(x, lo, hi) for lo <= hi: the median of the three (one instruction)
__device__ __forceinline__ float mg_clip(float x, float lo, float hi)
{
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}

// Face coefficient between cells P and Q (eq. abcdrc with the conservative
// face form): w_face / sqrt(dn^2 + dt^2 + e2), dn = psiQ - psiP, dt the
// tangential central difference averaged over P and Q:
// (tpP + tpQ - tmP - tmQ)/4.  Written once and used by every caller in the
// same operand order so that the two orientations give identical bits.
__device__ __forceinline__ float mg_face(float psiP, float psiQ, float tpP, float tpQ,
                                         float tmP, float tmQ, float wP, float wQ, float e2)
{
#pragma clang fp contract(off)
    float dn = psiQ - psiP;
    float dt = ((tpP + tpQ) - (tmP + tmQ)) * 0.25f;
    float wf = 0.5f * (wP + wQ);
    return wf * __builtin_amdgcn_rsqf(dn * dn + dt * dt + e2);
}
__device__ __forceinline__ double mg_face64(double psiP, double psiQ, double tpP, double tpQ,
                                            double tmP, double tmQ, double wP, double wQ, double e2)
{
#pragma clang fp contract(off)
    double dn = psiQ - psiP;
    double dt = ((tpP + tpQ) - (tmP + tmQ)) * 0.25;
    double wf = 0.5 * (wP + wQ);
    return wf / sqrt(dn * dn + dt * dt + e2);
}

// --------------------------------------------------------------------------
// clipped ramps x -> clip(a x + b, lo, hi) with a >= 0: the map from the
// fresh value of a unit's in-line predecessor to the unit's last value.
// Closed under composition, so a line of units is a scan.
struct Ramp {
    float a, b, lo, hi;
};
__device__ __forceinline__ Ramp ramp_id() { return Ramp{1.0f, 0.0f, -MG_BIG, MG_BIG}; }
__device__ __forceinline__ float ramp_eval(const Ramp &r, float x)
{
    return mg_clip(fmaf(r.a, x, r.b), r.lo, r.hi);
}
// g o f
__device__ __forceinline__ Ramp ramp_comp(const Ramp &g, const Ramp &f)
{
    Ramp o;
    o.a = g.a * f.a;
    o.b = fmaf(g.a, f.b, g.b);
    o.lo = mg_clip(fmaf(g.a, f.lo, g.b), g.lo, g.hi);
    o.hi = mg_clip(fmaf(g.a, f.hi, g.b), g.lo, g.hi);
    return o;
}

// a label bit no cell carries (the labels use bits 0-3, one per sweep): a
// sweep with it has no starred cell, every cell a point update
#define LAB_NONE 4
// every cell starred: each line is one system (line Gauss-Seidel, GSLINE-I of
// Sec. 3.2), solved with the box; no cut of the run other than the kernel's
#define LAB_ALL 5

// --------------------------------------------------------------------------
// Line-sweep arguments.  All arrays are in the layout of the sweep; `lab`
// holds one byte per cell with bit s set when the cell is starred in sweep
// s (jump set and smallest coefficient s).  lo/hi may be null (then -M, M).
struct LineArgs {
    const float *phi_old;
    float *phi_new;
    const float *psi, *w, *fit, *F;     // F may be null (zero)
    const uint8_t *lab;
    const float *lo, *hi;
    const int *skip;                    // non-null and set: the launch does nothing
    float *tout;                        // non-null: new values written transposed,
    int tpitch;                         //   cell q of line r at tout[q * tpitch + r]
    const double *area;                 // Rada-Chen area term (null: 0)
    const float4 *cf;                   // frozen scaled face coefficients (sweeps with CF; fit null)
    const float *qd = nullptr;          // NEWT: the Newton term Q' added to each cell's diagonal (null: none)
    // sweeps written in their own layout: 0 every line of a band in one launch; 1 the band's
    // first three lines only; 2 its fourth line only, its cross-line neighbours (final after
    // the split-1 launch) read from nb_old
    int split = 0;
    const float *nb_old = nullptr;
    // split long-line sweeps: the plane (line layout, pitch) holding the previous own line's final
    // values (phi_new), read in place of a copy in LDS
    const float *fresh = nullptr;
    int pitch, lpitch, nl, ml;
    float kap, e2, M, eps;
    int bit, scaled;
    int run_max;                        // 0: maximal runs; else runs cut into pieces of at most run_max
};

// --------------------------------------------------------------------------
// Collective units of Hybrid Smoother 2 (Sec. 4.3, Fig. 3).  A maximal run
// of starred cells along the line (the paper's superpixel) is solved as one
// box-constrained tridiagonal system; a single starred cell takes the next
// cell of the line into its unit (a single starred cell at the line end
// stays alone).  With LineArgs::run_max > 0 runs longer than run_max are cut
// into ceil(len / run_max) pieces of near-equal length (the longer pieces
// first), each solved as its own unit; lines longer than one workgroup cut
// runs at the workgroup size (their row ring holds two rounds).
//
// Row buffer of the line being swept, indexed by visit position p:
//   a y_{p-1} - y_p + c y_{p+1} = r  (a = NaN marks S = 0), box [lo, hi],
// x = old value.  Units of more than three cells also use P, Q (their
// elimination, then scratch of the exact solve) and O (their new values).
// In LDS: two buffers of the whole line (RB_FIELDS fields each) for lines of
// one workgroup, a ring of two rounds (RF_COUNT fields) for longer lines.
enum { RF_A = 0, RF_C, RF_R, RF_LO, RF_HI, RF_X, RF_P, RF_Q, RF_O, RB_FIELDS };

struct RunBuf {
    float *p;
    int fs;            // elements between fields (>= line length)
    __device__ __forceinline__ float &at(int f, int q) const { return p[f * fs + q]; }
    // old value of the cell after position `last` (0 past the line end)
    __device__ __forceinline__ float sig_after(int last, int ml) const
    {
        return last + 1 < ml ? at(RF_X, last + 1) : 0.0f;
    }
    // the other of the two buffers of a line
    __device__ __forceinline__ RunBuf other(int k) const { return RunBuf{p + k * RB_FIELDS * fs, fs}; }
};

// 64-bit starred-mask words of a line of ml cells
__host__ __device__ inline int sweep_mask_words(int ml) { return (ml + 63) / 64; }

// Row buffer of lines longer than one workgroup: a ring of SLOTS positions
// (two rounds of the line).  Only unit cells are stored; the successor's old
// value sits beside each cell (RG_S), and a unit's new values go to RF_O,
// which shares the storage of RF_X: a unit's new values are written only by
// its own solve, after that solve has read the unit's rows, and the one later
// read of RF_X inside the solve (a cell of S = 0, held at its old value) finds
// that value there, as the substitution leaves it (such cells occur in units
// of more than three cells only in whole-line systems, which these lines do
// not take).  Nine fields instead of ten let two workgroups share a CU.
enum { RG_S = RB_FIELDS, RF_COUNT };
constexpr int RING_FIELDS = RF_COUNT - 1;
template <int SLOTS>
struct RingBuf {
    float *p;
    __device__ __forceinline__ static constexpr int slot(int f) { return f == RF_O ? RF_X : (f == RG_S ? RF_O : f); }
    __device__ __forceinline__ float &at(int f, int q) const { return p[slot(f) * SLOTS + (q & (SLOTS - 1))]; }
    __device__ __forceinline__ float sig_after(int last, int) const { return at(RG_S, last); }
    __device__ __forceinline__ float &y(int q) const { return at(RF_O, q); }
};

// Units of one or two cells in closed form.  The box-constrained problem of
// an M-matrix row set is the projected one: every cell sits at the projection
// of its row.  One cell: y0 = clip(a0 x + c0 sig - r0, lo0, hi0), a clipped
// ramp of x.  Two cells: y0 = clip(a0 x - r0 + c0 y1, lo0, hi0) and
// y1 = clip(a1 y0 + c1 sig - r1, lo1, hi1) compose into
// y1 = clip(a1 c0 y1 + b, L', U') (ramp composition), whose unique fixed point
// for 0 <= a1 c0 < 1 is clip(b / (1 - a1 c0), L', U'); y0 then follows.
struct PairRows {
    float a0, c0, r0, lo0, hi0, x0, a1, al1, lo1, hi1, x1;   // al1 = c1 sig - r1
    bool ok;
};
template <class Buf>
__device__ __forceinline__ void pair_load(const Buf &B, int ps, int L, int ml, PairRows &P)
{
    P.a0 = B.at(RF_A, ps); P.c0 = B.at(RF_C, ps); P.r0 = B.at(RF_R, ps);
    P.lo0 = B.at(RF_LO, ps); P.hi0 = B.at(RF_HI, ps); P.x0 = B.at(RF_X, ps);
    P.ok = !isnan(P.a0);
    if (L == 2) {
        P.a1 = B.at(RF_A, ps + 1);
        const float sig = B.sig_after(ps + 1, ml);
        P.al1 = B.at(RF_C, ps + 1) * sig - B.at(RF_R, ps + 1);
        P.lo1 = B.at(RF_LO, ps + 1); P.hi1 = B.at(RF_HI, ps + 1); P.x1 = B.at(RF_X, ps + 1);
        P.ok = P.ok && !isnan(P.a1) && (1.0f - P.a1 * P.c0) > 0.0f;
    } else {
        const float sig = B.sig_after(ps, ml);
        P.r0 -= P.c0 * sig;            // one cell: the successor's old value is known
        P.c0 = 0.0f;
        P.a1 = 0.0f; P.al1 = 0.0f; P.lo1 = 0.0f; P.hi1 = 0.0f; P.x1 = 0.0f;
    }
}
// chain ramp x -> value of the unit's last cell
__device__ __forceinline__ Ramp pair_ramp(const PairRows &P, int L)
{
    if (!P.ok) {
        const float yo = L == 2 ? P.x1 : P.x0;
        return Ramp{0.0f, yo, yo, yo};
    }
    if (L == 1) return Ramp{P.a0, -P.r0, P.lo0, P.hi0};
    const float inv = __builtin_amdgcn_rcpf(1.0f - P.a1 * P.c0);
    const float Lp = mg_clip(fmaf(P.a1, P.lo0, P.al1), P.lo1, P.hi1);
    const float Up = mg_clip(fmaf(P.a1, P.hi0, P.al1), P.lo1, P.hi1);
    return Ramp{P.a1 * P.a0 * inv, (P.al1 - P.a1 * P.r0) * inv, Lp, Up};
}
// the unit's values at the entering value x
__device__ __forceinline__ void pair_solve(const PairRows &P, int L, float x, float &y0, float &y1)
{
    if (!P.ok) { y0 = P.x0; y1 = P.x1; return; }
    if (L == 1) { y0 = mg_clip(fmaf(P.a0, x, -P.r0), P.lo0, P.hi0); y1 = 0.0f; return; }
    y1 = ramp_eval(pair_ramp(P, 2), x);
    y0 = mg_clip(fmaf(P.c0, y1, fmaf(P.a0, x, -P.r0)), P.lo0, P.hi0);
}

// Units of three cells.  With the middle value y1 given, the end cells are
// the clipped ramps y0 = R0(y1) = clip(a0 x - r0 + c0 y1, lo0, hi0) and
// y2 = R2(y1) = clip(c2 sig - r2 + a2 y1, lo2, hi2), so the middle cell solves
// y1 = clip(h(y1), lo1, hi1) with h = -r1 + a1 R0 + c1 R2 monotone piecewise
// linear of slope < 1.  psi(y) = y - clip(h(y)) increases: its root lies between
// the largest candidate point (lo1, hi1, the ramps' kinks) with psi <= 0 and the
// smallest with psi >= 0, where h is linear, so it is the fixed point of that
// linear piece.  As a map of x the last cell is the clipped ramp
// clip(u + v x, y-, y+): u + v x the all-free solution, y-/y+ the two-cell
// solutions of cells 1, 2 with cell 0 held at lo0 / hi0.
struct TriRows {
    float a0, c0, r0, lo0, hi0, a1, c1, r1, lo1, hi1, a2, al2, lo2, hi2, x0, x1, x2;   // al2 = c2 sig - r2
    bool ok;
};
template <class Buf>
__device__ __forceinline__ void tri_load(const Buf &B, int ps, int ml, TriRows &T)
{
    T.a0 = B.at(RF_A, ps); T.c0 = B.at(RF_C, ps); T.r0 = B.at(RF_R, ps);
    T.lo0 = B.at(RF_LO, ps); T.hi0 = B.at(RF_HI, ps); T.x0 = B.at(RF_X, ps);
    T.a1 = B.at(RF_A, ps + 1); T.c1 = B.at(RF_C, ps + 1); T.r1 = B.at(RF_R, ps + 1);
    T.lo1 = B.at(RF_LO, ps + 1); T.hi1 = B.at(RF_HI, ps + 1); T.x1 = B.at(RF_X, ps + 1);
    T.a2 = B.at(RF_A, ps + 2);
    const float sig = B.sig_after(ps + 2, ml);
    T.al2 = B.at(RF_C, ps + 2) * sig - B.at(RF_R, ps + 2);
    T.lo2 = B.at(RF_LO, ps + 2); T.hi2 = B.at(RF_HI, ps + 2); T.x2 = B.at(RF_X, ps + 2);
    T.ok = !isnan(T.a0) && !isnan(T.a1) && !isnan(T.a2) && (1.0f - T.a1 * T.c0 - T.c1 * T.a2) > 0.0f &&
           (1.0f - T.a2 * T.c1) > 0.0f;
}
__device__ __forceinline__ void tri_solve(const TriRows &T, float x, float &y0, float &y1, float &y2)
{
    if (!T.ok) { y0 = T.x0; y1 = T.x1; y2 = T.x2; return; }
    const float al0 = fmaf(T.a0, x, -T.r0);
    auto R0 = [&](float y) { return mg_clip(fmaf(T.c0, y, al0), T.lo0, T.hi0); };
    auto R2 = [&](float y) { return mg_clip(fmaf(T.a2, y, T.al2), T.lo2, T.hi2); };
    auto psi = [&](float y) {
        return y - mg_clip(fmaf(T.c1, R2(y), fmaf(T.a1, R0(y), -T.r1)), T.lo1, T.hi1);
    };
    float cand[4];
    const float big = 3.0e38f;
    cand[0] = T.c0 > 0.0f ? (T.lo0 - al0) * __builtin_amdgcn_rcpf(T.c0) : big;
    cand[1] = T.c0 > 0.0f ? (T.hi0 - al0) * __builtin_amdgcn_rcpf(T.c0) : big;
    cand[2] = T.a2 > 0.0f ? (T.lo2 - T.al2) * __builtin_amdgcn_rcpf(T.a2) : big;
    cand[3] = T.a2 > 0.0f ? (T.hi2 - T.al2) * __builtin_amdgcn_rcpf(T.a2) : big;
    float plo = T.lo1, phi = T.hi1;
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const float p = mg_clip(cand[k], T.lo1, T.hi1);
        const float v = psi(p);
        if (v <= 0.0f && p > plo) plo = p;
        if (v >= 0.0f && p < phi) phi = p;
    }
    if (!(phi > plo)) {
        y1 = plo;
    } else {
        // the linear piece of h on (plo, phi)
        const float m = 0.5f * (plo + phi);
        float sl = 0.0f, t = -T.r1;
        const float v0 = fmaf(T.c0, m, al0), v2 = fmaf(T.a2, m, T.al2);
        if (v0 <= T.lo0) t = fmaf(T.a1, T.lo0, t);
        else if (v0 >= T.hi0) t = fmaf(T.a1, T.hi0, t);
        else { sl = fmaf(T.a1, T.c0, sl); t = fmaf(T.a1, al0, t); }
        if (v2 <= T.lo2) t = fmaf(T.c1, T.lo2, t);
        else if (v2 >= T.hi2) t = fmaf(T.c1, T.hi2, t);
        else { sl = fmaf(T.c1, T.a2, sl); t = fmaf(T.c1, T.al2, t); }
        y1 = mg_clip(mg_clip(t * __builtin_amdgcn_rcpf(1.0f - sl), T.lo1, T.hi1), plo, phi);
    }
    y0 = R0(y1);
    y2 = R2(y1);
}
// two-cell solution of cells 1, 2 with cell 0 fixed at y0: value of cell 2
__device__ __forceinline__ float tri_tail(const TriRows &T, float y0)
{
    const float al1 = fmaf(T.a1, y0, -T.r1);
    const float Lp = mg_clip(fmaf(T.a2, T.lo1, T.al2), T.lo2, T.hi2);
    const float Up = mg_clip(fmaf(T.a2, T.hi1, T.al2), T.lo2, T.hi2);
    return mg_clip(fmaf(T.a2, al1, T.al2) * __builtin_amdgcn_rcpf(1.0f - T.a2 * T.c1), Lp, Up);
}
__device__ __forceinline__ Ramp tri_ramp(const TriRows &T)
{
    if (!T.ok) return Ramp{0.0f, T.x2, T.x2, T.x2};
    if (!(T.a0 > 0.0f)) {
        float y0, y1, y2;
        tri_solve(T, 0.0f, y0, y1, y2);
        return Ramp{0.0f, y2, y2, y2};
    }
    // all cells free: y1 = (-r1 + a1 (a0 x - r0) + c1 al2) / D, y2 = al2 + a2 y1
    const float invD = __builtin_amdgcn_rcpf(1.0f - T.a1 * T.c0 - T.c1 * T.a2);
    const float u1 = (fmaf(T.c1, T.al2, -T.r1) - T.a1 * T.r0) * invD;
    const float v1 = T.a1 * T.a0 * invD;
    const float ym = tri_tail(T, T.lo0), yp = tri_tail(T, T.hi0);
    return Ramp{T.a2 * v1, fmaf(T.a2, u1, T.al2), fminf(ym, yp), fmaxf(ym, yp)};
}

// starred-cell bit masks of the line (LDS): bit p of word p / 64
__device__ __forceinline__ bool mask_bit(const uint64_t *msk, int p)
{
    return ((msk[p >> 6] >> (p & 63)) & 1ull) != 0ull;
}
// first / last position of the maximal starred run through the starred position p
__device__ __forceinline__ int run_first(const uint64_t *msk, int p)
{
    int wi = p >> 6;
    uint64_t z = ~msk[wi] & ((1ull << (p & 63)) - 1ull);
    while (z == 0ull) {
        if (wi == 0) return 0;
        wi--;
        z = ~msk[wi];
    }
    return (wi << 6) + 64 - __builtin_clzll(z);
}
__device__ __forceinline__ int run_last(const uint64_t *msk, int nw, int p)
{
    int wi = p >> 6;
    uint64_t z = ~msk[wi] & ~((2ull << (p & 63)) - 1ull);
    while (z == 0ull) {
        if (++wi >= nw) return (nw << 6) - 1;
        z = ~msk[wi];
    }
    return (wi << 6) + __builtin_ctzll(z) - 1;
}
// unit of the starred position p of the maximal starred run t0..e: first
// position ps and length L; cap > 0 cuts runs longer than cap into
// ceil(len / cap) near-equal pieces, the longer ones first
__device__ __forceinline__ void unit_of_run(int t0, int e, int ml, int p, int cap, int &ps, int &L)
{
    const int rl = e - t0 + 1;
    if (rl == 1) { ps = p; L = p + 1 < ml ? 2 : 1; return; }
    if (cap <= 0 || rl <= cap) { ps = t0; L = rl; return; }
    const int np = (rl + cap - 1) / cap, base = rl / np, extra = rl % np;
    const int o = p - t0, big = extra * (base + 1);
    if (o < big) { ps = t0 + (o / (base + 1)) * (base + 1); L = base + 1; }
    else { ps = t0 + big + ((o - big) / base) * base; L = base; }
}
__device__ __forceinline__ void unit_of(const uint64_t *msk, int nw, int ml, int p, int cap, int &ps, int &L)
{
    unit_of_run(run_first(msk, p), run_last(msk, nw, p), ml, p, cap, ps, L);
}
// the same on a line of at most 64 cells whose starred mask is the word bm
__device__ __forceinline__ void unit_of1(uint64_t bm, int ml, int p, int cap, int &ps, int &L)
{
    const uint64_t zb = ~bm & ((1ull << p) - 1ull), za = ~bm & ~((2ull << p) - 1ull);
    unit_of_run(zb ? 64 - __builtin_clzll(zb) : 0, za ? __builtin_ctzll(za) - 1 : 63, ml, p, cap, ps, L);
}
// a maximal starred run of at least four cells in the mask words w0 (then
// w1, the next word): units of more than three cells are possible
__device__ __forceinline__ bool has_run4(uint64_t w0, uint64_t w1)
{
    const uint64_t s1 = (w0 >> 1) | (w1 << 63), s2 = (w0 >> 2) | (w1 << 62), s3 = (w0 >> 3) | (w1 << 61);
    return (w0 & s1 & s2 & s3) != 0ull;
}
// the cut of the sweep's runs: units of more than three cells exist unless
// runs are cut into pieces of at most three
__device__ __forceinline__ bool long_units_possible(const LineArgs &A)
{
    return A.bit == LAB_ALL || (A.bit != LAB_NONE && !(A.run_max >= 1 && A.run_max <= 3));
}
// the cut of the runs of a sweep (0: none); whole-line systems are never cut
__device__ __forceinline__ int run_cut(const LineArgs &A) { return A.bit == LAB_ALL ? 0 : A.run_max; }
__device__ __forceinline__ bool starred(const LineArgs &A, unsigned lab)
{
    return A.bit == LAB_ALL || ((lab >> A.bit) & 1) != 0;
}

// Units of more than three cells.  Rows k = 0..L-1 of the unit (positions
// ps + k):  y_k = a_k y_{k-1} + c_k y_{k+1} - r_k  on [lo_k, hi_k], with
// y_{-1} = x (the entering value) and y_L = s (the successor's old value).
//
// Eliminating the unit from its far end without the box gives
// y_k = P_k y_{k-1} + Q_k (P_{L-1} = a, Q_{L-1} = c s - r, then
// P_k = a_k / (1 - c_k P_{k+1}), Q_k = (c_k Q_{k+1} - r_k) / (1 - c_k P_{k+1})).
// For the box-constrained unit the last value is a monotone function of x
// that is affine (slope P_0 ... P_{L-1}) where no cell is at a bound and
// constant elsewhere, because a cell at a bound separates the cells after it
// from x.  Writing Z_k(t) = clip(P_k t + Q_k, lo_k, hi_k), the composition
// Z_{L-1} o ... o Z_0 is such a clipped ramp, and it has the right limits:
// as x -> -inf (+inf) cell 0 goes to lo_0 (hi_0) and the composition of the
// remaining Z's gives the tail's last value with cell 0 held there (the same
// argument one cell further on).  So in the line scan every cell of such a
// unit contributes its Z_k, and the scan carries the exact last value of the
// unit on to the cells after it.  (A cell with a_k = 0 is the limit of small
// a_k, where both sides are continuous.)
//
// Values inside the unit.  The scan's values z_k = Z_k(z_{k-1}) (z_{-1} = x)
// are the unit's values wherever no cell after k is held at a bound by the
// true solution; they are checked row by row (every cell must be the
// projection of its own row).  A unit that fails the check is finished by a
// primal-dual active-set iteration: cells held at a bound are fixed there,
// the free chains between them are solved exactly (one forward elimination
// and one back substitution over the unit), free cells that leave the box are
// held, held cells whose row points back into the box are released, until no
// cell changes (Hintermueller, Ito & Kunisch: finite for M-matrices).  One
// thread takes such a unit.
//
// Rows of S = 0 cannot be starred (the jump test needs a non-zero interior
// coefficient), so units of more than three cells have none; a cell of S = 0
// placed in one anyway keeps its old value inside the elimination.  The
// pivots are positive: the rows are strictly diagonally dominant through the
// coefficients across the line.

// P_k, Q_k of position p by elimination from the unit's last position down to
// p; P1 / Q1 are P_{k+1}, Q_{k+1} (for the last cell: 0 and s)
template <class Buf>
__device__ __forceinline__ void long_elim(const Buf &B, int p, int last, float s, float &P, float &Q, float &P1,
                                          float &Q1)
{
    float Pn = 0.0f, Qn = s, Pp = 0.0f, Qp = s;
    // four rows per step: their reads are issued together, ahead of the dependent chain
    for (int q = last; q >= p; q -= 4) {
        float a[4], c[4], r[4];
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int qq = q - j >= p ? q - j : p;
            a[j] = B.at(RF_A, qq); c[j] = B.at(RF_C, qq); r[j] = B.at(RF_R, qq);
        }
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (q - j < p) break;
            Pp = Pn; Qp = Qn;
            if (isnan(a[j])) {
                Pn = 0.0f; Qn = B.at(RF_X, q - j);
            } else {
                const float inv = __builtin_amdgcn_rcpf(fmaf(-c[j], Pn, 1.0f));
                Pn = a[j] * inv;
                Qn = fmaf(c[j], Qn, -r[j]) * inv;
            }
        }
    }
    P = Pn; Q = Qn; P1 = Pp; Q1 = Qp;
}

// the unit's row at position q evaluated at its neighbours' values in RF_O
// (the value the cell would take free of its box); mag: the size of its
// terms, the scale of its rounding
template <class Buf>
__device__ __forceinline__ float long_row(const Buf &B, int q, int ps, int last, float x, float s, float &mag)
{
    const float yp = q == ps ? x : B.at(RF_O, q - 1);
    const float yn = q == last ? s : B.at(RF_O, q + 1);
    const float ta = B.at(RF_A, q) * yp, tc = B.at(RF_C, q) * yn, r = B.at(RF_R, q);
    mag = fabsf(ta) + fabsf(tc) + fabsf(r);
    return (ta + tc) - r;
}
// does z_q (in RF_O) sit at the projection of its row?
__device__ __forceinline__ bool long_row_ok(float z, float v, float mag, float lo, float hi)
{
    return fabsf(mg_clip(v, lo, hi) - z) <= 1e-5f * mag;
}

// The active-set iteration of a unit from the values in RF_O (its starting
// held set: the cells there at a bound); the result replaces RF_O.  RF_P
// holds the held state between passes (-1 held at lo, -2 held at hi, -3 a
// cell of S = 0 held at its old value, else free) and the elimination factor
// E >= 0 of a free cell within a pass; RF_Q the elimination's F (a held cell:
// its value).
template <class Buf>
__device__ __forceinline__ void long_active_set(const Buf &B, int ps, int L, int ml, float x)
{
    const int last = ps + L - 1;
    const float s = B.sig_after(last, ml);
#pragma nounroll
    for (int q = ps; q <= last; q++) {
        const float v = B.at(RF_O, q);
        B.at(RF_P, q) = isnan(B.at(RF_A, q)) ? -3.0f
                        : (v <= B.at(RF_LO, q) ? -1.0f : (v >= B.at(RF_HI, q) ? -2.0f : 0.0f));
    }
#pragma nounroll
    for (int it = 0; it < L + 8; it++) {
        // forward elimination of the free chains: y_q = E_q y_{q+1} + F_q
        float Ep = 0.0f, Fp = x;
#pragma nounroll
        for (int q = ps; q <= last; q++) {
            const float st = B.at(RF_P, q);
            if (st < 0.0f) {
                Ep = 0.0f;
                Fp = st == -1.0f ? B.at(RF_LO, q) : (st == -2.0f ? B.at(RF_HI, q) : B.at(RF_X, q));
            } else {
                const float a = B.at(RF_A, q);
                const float inv = __builtin_amdgcn_rcpf(fmaf(-a, Ep, 1.0f));
                Ep = B.at(RF_C, q) * inv;
                Fp = fmaf(a, Fp, -B.at(RF_R, q)) * inv;
                B.at(RF_P, q) = Ep;
            }
            B.at(RF_Q, q) = Fp;
        }
        float yn = s;
#pragma nounroll
        for (int q = last; q >= ps; q--) {
            const float e = B.at(RF_P, q);
            yn = e < 0.0f ? B.at(RF_Q, q) : fmaf(e, yn, B.at(RF_Q, q));
            B.at(RF_O, q) = yn;
        }
        // new held state: free cells outside the box are held; a held cell is
        // released where its row points back into the box (beyond rounding)
        bool changed = false;
#pragma nounroll
        for (int q = ps; q <= last; q++) {
            const float lo = B.at(RF_LO, q), hi = B.at(RF_HI, q), yv = B.at(RF_O, q), was = B.at(RF_P, q);
            float st = 0.0f;
            if (was == -3.0f) {
                st = -3.0f;
            } else if (was < 0.0f) {
                float mag;
                const float v = long_row(B, q, ps, last, x, s, mag);
                const float tol = 2e-6f * (mag + fabsf(was == -1.0f ? lo : hi));
                if (was == -1.0f) st = v > lo + tol ? 0.0f : -1.0f;
                else st = v < hi - tol ? 0.0f : -2.0f;
            } else if (yv < lo) {
                st = -1.0f;
            } else if (yv > hi) {
                st = -2.0f;
            }
            changed |= (st < 0.0f) != (was < 0.0f);
            B.at(RF_P, q) = st;
        }
        if (!changed) break;
    }
#pragma nounroll
    for (int q = ps; q <= last; q++) B.at(RF_O, q) = mg_clip(B.at(RF_O, q), B.at(RF_LO, q), B.at(RF_HI, q));
}

// One thread per unit (lines longer than one workgroup).  The chain ramp:
// the composition of the unit's Z_k, built during one elimination that also
// stores P_k, Q_k.
template <class Buf>
__device__ __forceinline__ Ramp long_ramp(const Buf &B, int ps, int L, int ml)
{
    const int last = ps + L - 1;
    float Pn = 0.0f, Qn = B.sig_after(last, ml);
    Ramp T = ramp_id();
#pragma nounroll
    for (int q = last; q >= ps; q--) {
        const float a = B.at(RF_A, q), c = B.at(RF_C, q), r = B.at(RF_R, q);
        if (isnan(a)) {
            Pn = 0.0f; Qn = B.at(RF_X, q);
        } else {
            const float inv = __builtin_amdgcn_rcpf(fmaf(-c, Pn, 1.0f));
            Pn = a * inv;
            Qn = fmaf(c, Qn, -r) * inv;
        }
        B.at(RF_P, q) = Pn;
        B.at(RF_Q, q) = Qn;
        T = ramp_comp(T, Ramp{Pn, Qn, B.at(RF_LO, q), B.at(RF_HI, q)});
    }
    return T;
}
// the unit's values at x into RF_O: forward substitution through the Z_k,
// the row check, the active-set iteration where it fails
template <class Buf>
__device__ __forceinline__ void long_solve(const Buf &B, int ps, int L, int ml, float x)
{
    const int last = ps + L - 1;
    const float s = B.sig_after(last, ml);
    float y = x;
#pragma nounroll
    for (int q = ps; q <= last; q++) {
        y = mg_clip(fmaf(B.at(RF_P, q), y, B.at(RF_Q, q)), B.at(RF_LO, q), B.at(RF_HI, q));
        B.at(RF_O, q) = y;
    }
    bool good = true;
#pragma nounroll
    for (int q = ps; q <= last && good; q++) {
        float mag;
        const float v = long_row(B, q, ps, last, x, s, mag);
        good = long_row_ok(B.at(RF_O, q), v, mag, B.at(RF_LO, q), B.at(RF_HI, q));
    }
    if (!good) long_active_set(B, ps, L, ml, x);
}

// --------------------------------------------------------------------------
// Block-wide exclusive scan of ramps in thread order.  Within a wave:
// Hillis-Steele over rows of 16 lanes with DPP row shifts, then the row
// totals with DPP row broadcasts (lanes whose source is outside the pattern
// take the identity).  Across waves: the wave totals go through LDS and one
// wave-level scan of them gives every wave its prefix.  wtot holds two sets
// of NT/64 totals used alternately (parity), so consecutive scans need one
// barrier each.
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ float dpp_f(float old, float src)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(src), CTRL, ROWM, 0xf,
                                                      false));
}
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ Ramp dpp_ramp(const Ramp &r)
{
    const Ramp id = ramp_id();
    return Ramp{dpp_f<CTRL, ROWM>(id.a, r.a), dpp_f<CTRL, ROWM>(id.b, r.b), dpp_f<CTRL, ROWM>(id.lo, r.lo),
                dpp_f<CTRL, ROWM>(id.hi, r.hi)};
}
// inclusive scan in lane order, complete on the first LANES lanes of the wave
// (the stages that only reach lanes at or above LANES are left out)
template <int LANES = 64>
__device__ __forceinline__ Ramp wave_scan_incl(Ramp v)
{
    if (LANES > 1) v = ramp_comp(v, dpp_ramp<0x111>(v));          // row_shr:1
    if (LANES > 2) v = ramp_comp(v, dpp_ramp<0x112>(v));          // row_shr:2
    if (LANES > 4) v = ramp_comp(v, dpp_ramp<0x114>(v));          // row_shr:4
    if (LANES > 8) v = ramp_comp(v, dpp_ramp<0x118>(v));          // row_shr:8
    if (LANES > 16) v = ramp_comp(v, dpp_ramp<0x142, 0xa>(v));    // row_bcast:15 into rows 1, 3
    if (LANES > 32) v = ramp_comp(v, dpp_ramp<0x143, 0xc>(v));    // row_bcast:31 into rows 2, 3
    return v;
}
__device__ __forceinline__ Ramp readlane_ramp(const Ramp &r, int lane)
{
    return Ramp{__int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.a), lane)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.b), lane)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.lo), lane)),
                __int_as_float(__builtin_amdgcn_readlane(__float_as_int(r.hi), lane))};
}

// t: the thread's index in the group of NT threads that takes the scan.
// want (one wave): only the first `want` prefixes are needed (total is then
// not the line's).
template <int NT>
__device__ __forceinline__ Ramp block_scan_excl(Ramp mine, Ramp *wtot, int parity, Ramp &total, int t,
                                                int want = 64)
{
    const int lane = t & 63, wave = t >> 6;
    constexpr int NW = NT / 64;
    const Ramp inc = NW > 1 || want > 32 ? wave_scan_incl<64>(mine)
                     : want > 16         ? wave_scan_incl<32>(mine)
                                         : wave_scan_incl<16>(mine);
    Ramp ex = dpp_ramp<0x138>(inc);                 // wave_shr:1 (lane 0: identity)
    if (NW > 1) {
        Ramp *wt = wtot + parity * NW;
        if (lane == 63) wt[wave] = inc;
        __syncthreads();
        const Ramp ws = wave_scan_incl<NW>(lane < NW ? wt[lane] : ramp_id());
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        if (wv > 0) ex = ramp_comp(ex, readlane_ramp(ws, wv - 1));
        total = readlane_ramp(ws, NW - 1);
    } else {
        total = readlane_ramp(inc, 63);
    }
    return ex;
}

// --------------------------------------------------------------------------
// The backward elimination of a whole line as a scan.  The step
//   P_k = a_k / (1 - c_k P_{k+1}),  Q_k = (c_k Q_{k+1} - r_k) / (1 - c_k P_{k+1})
// is linear-fractional in (P, Q): on the homogeneous vector (Q, P, 1) it acts
// as the block upper-triangular matrix [[c, 0, -r], [0, 0, a], [0, -c, 1]],
// and products of such matrices keep the form [[al, b0, b1], [0, B]] (B 2x2):
// seven numbers.  A scan over the positions from the line's end composes them;
// position k's prefix applied to the end vector (0, 0, 1) (no successor beyond
// the line end, where c = 0) gives (Q_k, P_k, 1) up to a common factor.  Each
// composition is rescaled by its denominator entry B11 (positive: a product of
// the pivots 1 - c P), which leaves the ratios unchanged and keeps long lines
// in range; B11 = 1 is then implicit and six numbers are kept, and the
// prefix's P_k = m01, Q_k = b1.  The compositions run in FP64: composing
// near-singular steps (strong coupling along the line) in FP32 loses several
// bits against the sequential elimination, while FP64 leaves P, Q correct to
// their FP32 rounding.
struct Elim {
    double al, b0, b1, m00, m01, m10;
};
__device__ __forceinline__ Elim elim_id() { return Elim{1.0, 0.0, 0.0, 1.0, 0.0, 0.0}; }
__device__ __forceinline__ Elim elim_step(float a, float c, float r)
{
    return Elim{(double)c, 0.0, -(double)r, 0.0, (double)a, -(double)c};
}
// a fixed value y (P = 0, Q = y)
__device__ __forceinline__ Elim elim_fixed(float y) { return Elim{0.0, 0.0, (double)y, 0.0, 0.0, 0.0}; }
// g o f (f applied first), rescaled to B11 = 1
__device__ __forceinline__ Elim elim_comp(const Elim &g, const Elim &f)
{
    // the denominator lies in (0, 2]: the hardware reciprocal and one Newton step
    const double den = fma(g.m10, f.m01, 1.0);
    double sc = __builtin_amdgcn_rcp(den);
    sc = fma(sc, fma(-den, sc, 1.0), sc);
    Elim o;
    o.al = g.al * f.al * sc;
    o.b0 = fma(g.al, f.b0, fma(g.b0, f.m00, g.b1 * f.m10)) * sc;
    o.b1 = fma(g.al, f.b1, fma(g.b0, f.m01, g.b1)) * sc;
    o.m00 = fma(g.m00, f.m00, g.m01 * f.m10) * sc;
    o.m01 = fma(g.m00, f.m01, g.m01) * sc;
    o.m10 = fma(g.m10, f.m00, f.m10) * sc;
    return o;
}
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ double dpp_d(double old, double src)
{
    const long long o = __double_as_longlong(old), v = __double_as_longlong(src);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)v, CTRL, ROWM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, ROWM, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROWM = 0xf>
__device__ __forceinline__ Elim dpp_elim(const Elim &e)
{
    return Elim{dpp_d<CTRL, ROWM>(1.0, e.al), dpp_d<CTRL, ROWM>(0.0, e.b0), dpp_d<CTRL, ROWM>(0.0, e.b1),
                dpp_d<CTRL, ROWM>(1.0, e.m00), dpp_d<CTRL, ROWM>(0.0, e.m01), dpp_d<CTRL, ROWM>(0.0, e.m10)};
}
template <int LANES = 64>
__device__ __forceinline__ Elim wave_scan_elim(Elim v)
{
    if (LANES > 1) v = elim_comp(v, dpp_elim<0x111>(v));
    if (LANES > 2) v = elim_comp(v, dpp_elim<0x112>(v));
    if (LANES > 4) v = elim_comp(v, dpp_elim<0x114>(v));
    if (LANES > 8) v = elim_comp(v, dpp_elim<0x118>(v));
    if (LANES > 16) v = elim_comp(v, dpp_elim<0x142, 0xa>(v));
    if (LANES > 32) v = elim_comp(v, dpp_elim<0x143, 0xc>(v));
    return v;
}
__device__ __forceinline__ Elim readlane_elim(const Elim &e, int lane)
{
    auto rl = [&](double x) {
        const long long b = __double_as_longlong(x);
        const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    };
    return Elim{rl(e.al), rl(e.b0), rl(e.b1), rl(e.m00), rl(e.m01), rl(e.m10)};
}
// inclusive scan in thread order over the NT threads of the group (t: index in
// the group); several waves: one barrier (wave totals through LDS)
template <int NT>
__device__ __forceinline__ Elim block_scan_elim(Elim mine, Elim *etot, int t)
{
    const int lane = t & 63, wave = t >> 6;
    constexpr int NW = NT / 64;
    Elim inc = wave_scan_elim<64>(mine);
    if (NW > 1) {
        if (lane == 63) etot[wave] = inc;
        __syncthreads();
        const Elim ws = wave_scan_elim<NW>(lane < NW ? etot[lane] : elim_id());
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        if (wv > 0) inc = elim_comp(inc, readlane_elim(ws, wv - 1));
    }
    return inc;
}

// Global inputs of one cell of a line (the frozen state of the sweep and the
// old values): everything phase 1 of a line step reads from memory, so that
// the next line's reads can be issued before the current line is computed
// (sweep_band) or the next round's (long_band).
struct CellIn {
    float p0, pp, pm, p0p, p0m, ppp, ppm, pmp, pmm;   // psi at (r,q), (r+1,q), (r-1,q), (r,q+), (r,q-), (r+1,q+), (r+1,q-), (r-1,q+), (r-1,q-)
    float w00, wp, wm, w0p, w0m;                      // w at (r,q), (r+1,q), (r-1,q), (r,q+), (r,q-)
    float fit, F, vu, vd, sig, pold, lo, hi, qd;
    float4 g;                                         // stored coefficients (CF): to r+1, r-1, q+1, q-1
    unsigned lab;
};

// Rows of line r that its cells read (rows mirrored at the grid edge); vu / vd
// are set only where the neighbour line exists and is not supplied fresh by
// the caller, fit / F / lo / hi where the arrays exist.
struct LineRows {
    const float *ps0, *psm, *psp, *w0, *wm, *wp, *old, *fit, *F, *lo, *hi, *vu, *vd;
    const float4 *cf;
    const float *qd;
    const uint8_t *lab;
    float M;
};
template <bool REV>
__device__ __forceinline__ LineRows line_rows(const LineArgs &A, int r, bool up_fresh, bool dn_fresh)
{
    const int nl = A.nl, P = A.pitch;
    const int ru = REV ? r + 1 : r - 1, rd = REV ? r - 1 : r + 1;
    const int rm1 = mg_mirror(r - 1, nl), rp1 = mg_mirror(r + 1, nl);
    const long long ro = (long long)r * P;
    LineRows R;
    R.ps0 = A.psi + ro; R.psm = A.psi + (long long)rm1 * P; R.psp = A.psi + (long long)rp1 * P;
    R.w0 = A.w + ro; R.wm = A.w + (long long)rm1 * P; R.wp = A.w + (long long)rp1 * P;
    R.old = A.phi_old + ro;
    R.fit = A.fit ? A.fit + ro : nullptr;
    R.F = A.F ? A.F + ro : nullptr;
    R.lo = A.lo ? A.lo + ro : nullptr;
    R.hi = A.lo ? A.hi + ro : nullptr;
    const float *nbs = A.nb_old ? A.nb_old : A.phi_old;
    R.vu = ru >= 0 && ru < nl && !up_fresh ? nbs + (long long)ru * P : nullptr;
    R.vd = rd >= 0 && rd < nl && !dn_fresh ? nbs + (long long)rd * P : nullptr;
    R.cf = A.cf ? A.cf + ro : nullptr;
    R.qd = A.qd ? A.qd + ro : nullptr;
    R.lab = A.lab + (long long)r * A.lpitch;
    R.M = A.M;
    return R;
}
// Reads the inputs of visit position p (q+ / q- the mirrored in-line neighbours);
// CF: the stored coefficients instead of psi and w.
template <bool REV, bool CF = false>
__device__ __forceinline__ void cell_load(const LineRows &R, int ml, int p, CellIn &c)
{
    const int q = REV ? ml - 1 - p : p;
    c.lab = R.lab[q];
    if (CF) {
        c.g = R.cf[q];
    } else {
        const int qm = mg_mirror(q - 1, ml), qp = mg_mirror(q + 1, ml);
        c.p0 = R.ps0[q]; c.pp = R.psp[q]; c.pm = R.psm[q];
        c.p0p = R.ps0[qp]; c.p0m = R.ps0[qm];
        c.ppp = R.psp[qp]; c.ppm = R.psp[qm]; c.pmp = R.psm[qp]; c.pmm = R.psm[qm];
        c.w00 = R.w0[q]; c.wp = R.wp[q]; c.wm = R.wm[q]; c.w0p = R.w0[qp]; c.w0m = R.w0[qm];
    }
    c.fit = R.fit ? R.fit[q] : 0.0f;
    c.F = R.F ? R.F[q] : 0.0f;
    c.vu = R.vu ? R.vu[q] : 0.0f;
    c.vd = R.vd ? R.vd[q] : 0.0f;
    c.sig = p + 1 < ml ? R.old[REV ? ml - 2 - p : p + 1] : 0.0f;
    c.lo = R.lo ? R.lo[q] : -R.M;
    c.hi = R.lo ? R.hi[q] : R.M;
    c.pold = R.old[q];
    c.qd = R.qd ? R.qd[q] : 0.0f;
}

// The frozen coefficients of cell (r, q) (eq. abcdrc) as the row
// a y_prev - y + c y_next = rr of its line, with the cross-line neighbours at
// vu / vd moved into rr; pb = c sig - rr is the point update's offset with the
// successor at its old value.  ok = false where S = 0 (the cell keeps x).
struct CellRow {
    float a, c, rr, pb, lo, hi, x;
    bool ok;
};
// CF: the scaled face coefficients come from the freeze (the same products,
// so the same bits) and the fit term is part of F.
// The scaled face coefficients of cell (r, q) to lines r+1, r-1 and cells
// q+1, q-1 (zero across the grid edge) and the fit term f (eq. abcdrc); CF:
// the coefficients stored by the freeze (the fit term is then part of F).
template <bool CF = false>
__device__ __forceinline__ void cell_coef(const LineArgs &A, const CellIn &c, int r, int q, float area, float &xp,
                                          float &xm, float &lp, float &lm, float &f)
{
    const int nl = A.nl, ml = A.ml;
    xp = 0.0f; xm = 0.0f; lp = 0.0f; lm = 0.0f; f = 0.0f;
    if (CF) {
        xp = c.g.x; xm = c.g.y; lp = c.g.z; lm = c.g.w;
    } else {
        const float e2 = A.e2;
        const float p0 = c.p0;
        if (r + 1 < nl) xp = mg_face(p0, c.pp, c.p0p, c.ppp, c.p0m, c.ppm, c.w00, c.wp, e2);
        if (r > 0) xm = mg_face(c.pm, p0, c.pmp, c.p0p, c.pmm, c.p0m, c.wm, c.w00, e2);
        if (q + 1 < ml) lp = mg_face(p0, c.p0p, c.pp, c.ppp, c.pm, c.pmp, c.w00, c.w0p, e2);
        if (q > 0) lm = mg_face(c.p0m, p0, c.ppm, c.pp, c.pmm, c.pm, c.w0m, c.w00, e2);
        const float dl = A.scaled ? 1.0f : mg_delta(p0, A.eps);
        const float sc = A.kap * dl;
        xp *= sc; xm *= sc; lp *= sc; lm *= sc;
        f = A.fit ? dl * (c.fit + area) : 0.0f;   // null fit: f is part of F
    }
}
template <bool REV, bool CF = false>
__device__ __forceinline__ CellRow cell_row(const LineArgs &A, const CellIn &c, int r, int q, float vu, float vd,
                                            float area)
{
    float xp, xm, lp, lm, f;
    cell_coef<CF>(A, c, r, q, area, xp, xm, lp, lm, f);
    // NEWT (eq. newtrc): the Newton term Q' joins the diagonal, and Q' times the old value the
    // right-hand side (zero for the other smoothers)
    const float S = xp + xm + lp + lm + c.qd;
    const float Xu = REV ? xp : xm, Xd = REV ? xm : xp;
    const float Lp = REV ? lp : lm, Ls = REV ? lm : lp;
    const float rhs = f + c.F - Xu * vu - Xd * vd - c.qd * c.pold;
    CellRow w;
    w.ok = S > 0.0f;
    const float inv = w.ok ? __builtin_amdgcn_rcpf(S) : 0.0f;
    w.a = Lp * inv;
    w.c = Ls * inv;
    w.rr = rhs * inv;
    w.pb = (Ls * c.sig - rhs) * inv;
    w.lo = c.lo;
    w.hi = c.hi;
    w.x = c.pold;
    return w;
}
// the point update as a clipped ramp of the entering value
__device__ __forceinline__ Ramp cell_ramp(const CellRow &w)
{
    return w.ok ? Ramp{w.a, w.pb, w.lo, w.hi} : Ramp{0.0f, w.x, w.x, w.x};
}
// the row stored for the unit solves (a = NaN marks S = 0)
template <class Buf>
__device__ __forceinline__ void row_store(const Buf &B, int p, const CellRow &w)
{
    B.at(RF_A, p) = w.ok ? w.a : __builtin_nanf("");
    B.at(RF_C, p) = w.ok ? w.c : 0.0f;
    B.at(RF_R, p) = w.ok ? w.rr : 0.0f;
    B.at(RF_LO, p) = w.lo;
    B.at(RF_HI, p) = w.hi;
    B.at(RF_X, p) = w.x;
}
// the row back from LDS (as row_store left it; pb is not kept, the cell being a unit cell)
template <class Buf>
__device__ __forceinline__ CellRow row_load(const Buf &B, int p)
{
    CellRow w;
    const float a = B.at(RF_A, p);
    w.ok = !isnan(a);
    w.a = w.ok ? a : 0.0f;
    w.c = B.at(RF_C, p);
    w.rr = B.at(RF_R, p);
    w.pb = 0.0f;
    w.lo = B.at(RF_LO, p);
    w.hi = B.at(RF_HI, p);
    w.x = B.at(RF_X, p);
    return w;
}

// --------------------------------------------------------------------------
// One line of one directional sweep, one thread per cell (visit position
// p = t, the thread's index in the group of NT threads that takes the line;
// REV: q = ml-1 down to 0), lines of at most NT cells.  REV takes the upstream
// line at r+1.  up_fresh / dn_fresh: the cross-line neighbour values are the
// caller's registers (same thread = same cell) instead of phi_old.  act =
// false: the group takes the step's barriers on no cells.  Returns the
// thread's new value.  WS: the group is one wave that needs no block barrier
// (a wave-level fence makes the rows and masks visible to its lanes).
//
// Every point and every unit is a clipped ramp of the value entering it, so
// the line is one block scan.  A unit's chain ramp sits at its LAST cell and
// its other cells take the identity, so that the scan's exclusive prefix at
// every cell of a unit is the value entering the unit: each unit cell then
// solves its unit from the rows in LDS and keeps its own value, with no
// exchange of results.  Barriers: one after the rows and masks are written,
// one inside the scan (several waves).  The rows live in one of two buffers
// chosen by the caller's line parity, so that the next line can write the
// other while this one's cells still read theirs after the scan; the masks
// are read before the scan only.
// OR of the per-wave flags of the workgroup (after the barrier that published them)
// Passes of the parallel active-set repair before a failed unit is finished by
// its first cell's serial iteration.  The held set of a whole-line system can
// move along the line a few cells per pass, and its serial finish costs
// milliseconds on a line of hundreds of cells, so whole lines take more passes.
// (Both halves of a two-half workgroup count the passes with this.)
__device__ __forceinline__ constexpr int repair_passes(bool whole) { return whole ? 256 : 8; }
__device__ __forceinline__ bool block_flag(const unsigned *wflag)
{
    const int ln = threadIdx.x & 63;
    return __ballot(ln < (int)(blockDim.x >> 6) && wflag[ln] != 0u) != 0ull;
}
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int NT, bool REV, bool CF = false, bool WS = false, bool WH = false>
__device__ __forceinline__ float sweep_line(const LineArgs &A, int r, const RunBuf &B, uint64_t *msk, bool write,
                                            float upv, bool up_fresh, float dnv, bool dn_fresh, Ramp *wtot,
                                            unsigned *wbad, Elim *etot, const CellIn &c, int t, bool act)
{
    static_assert(!WS || NT == 64, "a wave-synchronous line is one wave");
    if (WS) wave_lds_sync();
    const int lane = t & 63, wave = t >> 6;
    const int nl = A.nl, ml = A.ml, nw = (ml + 63) >> 6;
    const int ru = REV ? r + 1 : r - 1;      // upstream line
    const int rd = REV ? r - 1 : r + 1;      // downstream line
    const float area = A.area ? (float)(*A.area) : 0.0f;
    const bool has_up = ru >= 0 && ru < nl, has_dn = rd >= 0 && rd < nl;
    const int p = t;
    const bool in = act && p < ml;
    const int q = REV ? ml - 1 - p : p;

    // phase 1: frozen coefficients (eq. abcdrc), the row of the cell, starred masks
    CellRow w;
    w.ok = false; w.x = 0.0f;
    bool s0 = false;
    if (in) {
        s0 = starred(A, c.lab);
        float vu = 0.0f, vd = 0.0f;
        if (has_up) vu = up_fresh ? upv : c.vu;
        if (has_dn) vd = dn_fresh ? dnv : c.vd;
        w = cell_row<REV, CF>(A, c, r, q, vu, vd, area);
        row_store(B, p, w);
    }
    // a line of one wave keeps its starred mask in the ballot word (bm)
    const unsigned long long bm = __ballot(s0);
    if (NT > 64 && lane == 0 && wave * 64 < ml) msk[wave] = bm;
    bool any_star, any_long = false;
    const bool lmode = long_units_possible(A);
    if (NT == 64) {
        any_star = bm != 0ull;
        any_long = lmode && has_run4(bm, 0ull);
        if (WS) wave_lds_sync();
        else __syncthreads();
    } else {
        // one barrier makes the rows and masks visible; a line has a starred cell iff a mask word is non-zero
        __syncthreads();
        const uint64_t w0 = lane < nw ? msk[lane] : 0ull;
        any_star = __ballot(w0 != 0ull) != 0ull;
        if (lmode) any_long = __ballot(has_run4(w0, lane + 1 < nw ? msk[lane + 1] : 0ull)) != 0ull;
    }

    // phase 1b: a whole-line system (every cell starred, more than three cells) is eliminated by
    // one scan from the line's end: the thread of index t takes position ml - 1 - t and leaves
    // that position's P, Q in RF_P, RF_Q
    const bool whole = WH && ml > 3;
    if (whole) {
        const int pr = ml - 1 - t;
        Elim e = elim_id();
        if (act && pr >= 0) {
            const float a = B.at(RF_A, pr);
            e = isnan(a) ? elim_fixed(B.at(RF_X, pr)) : elim_step(a, B.at(RF_C, pr), B.at(RF_R, pr));
        }
        const Elim pre = block_scan_elim<NT>(e, etot, t);
        if (act && pr >= 0) {
            B.at(RF_P, pr) = (float)pre.m01;
            B.at(RF_Q, pr) = (float)pre.b1;
        }
        if (NT == 64 && WS) wave_lds_sync();
        else __syncthreads();
        // the row is taken again from LDS, so that no register holds it across the scan
        if (in) w = row_load(B, p);
    }

    // phase 2: the cell's unit (ps, L; L = 0: a point); the chain ramp of a unit of at most three
    // cells at its last cell; every cell of a longer unit its own Z_k
    int ps = p, Lu = 0;
    Ramp u = ramp_id();
    float lP1 = 0.0f, lQ1 = 0.0f;
    if (in) {
        if (any_star) {
            if (NT == 64) {
                if (s0) unit_of1(bm, ml, p, run_cut(A), ps, Lu);
                else if (p >= 1 && ((bm >> (p - 1)) & 1ull) && (p < 2 || !((bm >> (p - 2)) & 1ull))) {
                    ps = p - 1; Lu = 2;
                }
            } else {
                if (s0) unit_of(msk, nw, ml, p, run_cut(A), ps, Lu);
                else if (p >= 1 && mask_bit(msk, p - 1) && (p < 2 || !mask_bit(msk, p - 2))) { ps = p - 1; Lu = 2; }
            }
        }
        if (Lu == 0) {
            u = cell_ramp(w);
        } else if (Lu > 3) {
            const int last = ps + Lu - 1;
            float P, Q;
            if (whole) {
                P = B.at(RF_P, p); Q = B.at(RF_Q, p);
                if (p < last) { lP1 = B.at(RF_P, p + 1); lQ1 = B.at(RF_Q, p + 1); }
                else { lP1 = 0.0f; lQ1 = B.sig_after(last, ml); }
            } else {
                long_elim(B, p, last, B.sig_after(last, ml), P, Q, lP1, lQ1);
            }
            u = Ramp{P, Q, w.lo, w.hi};
            if (p == ps) B.at(RF_P, ps) = 0.0f;      // the unit's failed-check flag
        } else if (ps + Lu - 1 == p) {
            if (Lu <= 2) {
                PairRows Q;
                pair_load(B, ps, Lu, ml, Q);
                u = pair_ramp(Q, Lu);
            } else {
                TriRows T3;
                tri_load(B, ps, ml, T3);
                u = tri_ramp(T3);
            }
        }
    }

    // phase 3: the scan gives every cell the value entering it (a cell of a unit of at most three
    // cells: entering its unit; of a longer unit: its predecessor's value z in the unit's Z chain)
    Ramp tot;
    const Ramp ex = block_scan_excl<NT>(u, wtot, 0, tot, t, ml);
    const float x = ramp_eval(ex, 0.0f);
    float v = 0.0f;
    bool lbad = false;
    if (in) {
        if (Lu == 0) {
            v = ramp_eval(u, x);
        } else if (Lu > 3) {
            // z_k, and the check of the cell's row at z_{k-1} (= x) and z_{k+1} = Z_{k+1}(z_k)
            v = ramp_eval(u, x);
            const int last = ps + Lu - 1;
            const float yn = p == last ? lQ1 : mg_clip(fmaf(lP1, v, lQ1), B.at(RF_LO, p + 1), B.at(RF_HI, p + 1));
            const float ta = w.a * x, tc = w.c * yn;
            lbad = w.ok && !long_row_ok(v, (ta + tc) - w.rr, fabsf(ta) + fabsf(tc) + fabsf(w.rr), w.lo, w.hi);
            B.at(RF_O, p) = v;
            B.at(RF_Q, p) = v <= w.lo ? -1.0f : (v >= w.hi ? -2.0f : 0.0f);   // held state of z
            if (lbad) B.at(RF_P, ps) = 1.0f;
        } else if (Lu <= 2) {
            PairRows Q;
            pair_load(B, ps, Lu, ml, Q);
            float y0, y1;
            pair_solve(Q, Lu, x, y0, y1);
            v = p == ps ? y0 : y1;
        } else {
            TriRows T3;
            tri_load(B, ps, ml, T3);
            float y0, y1, y2;
            tri_solve(T3, x, y0, y1, y2);
            v = p == ps ? y0 : (p == ps + 1 ? y1 : y2);
        }
    }
    // A unit of more than three cells that fails the check is repaired by the active-set
    // iteration run in parallel: the held state of every cell of such a unit lives in RF_Q (-1 at
    // lo, -2 at hi, 0 free; at first the state of z), every cell eliminates its free chain up to
    // the next held cell, a second scan substitutes, and the cells update their held states, until
    // none changes.  After repair_passes such passes the thread of the unit's first cell (which
    // holds the entering value) finishes the unit with the serial iteration.  One-wave lines synchronise
    // only where a unit failed; wider lines publish one flag per wave and take one barrier (the
    // other half of a two-half workgroup takes it too), and the repair's barriers only where a
    // unit failed.
    bool repair = false;
    if (NT == 64 && WS) {
        repair = any_long && __ballot(lbad) != 0ull;
        if (repair) wave_lds_sync();
    } else if (lmode) {
        const unsigned long long bb = __ballot(lbad);
        if (lane == 0) wbad[threadIdx.x >> 6] = bb != 0ull ? 1u : 0u;
        __syncthreads();
        repair = block_flag(wbad);
    }
    if (repair) {
        const int last = ps + Lu - 1;
        const bool fu = in && Lu > 3 && B.at(RF_P, ps) != 0.0f;
        const float su = fu ? B.sig_after(last, ml) : 0.0f;
        float yv = v;
        for (int pass = 0;; pass++) {
            Ramp u2 = ramp_id();
            float st = 0.0f;
            if (whole) {
                // the free chains of the whole line eliminated by one scan (held cells fixed at
                // their bounds); P into RF_P, Q into RF_O (the values are not read again before
                // the substitution writes them)
                const int pr = ml - 1 - t;
                Elim e = elim_id();
                if (act && pr >= 0) {
                    // a cell of S = 0 keeps its old value, a held cell its bound
                    const float sq = B.at(RF_Q, pr), a = B.at(RF_A, pr);
                    if (isnan(a) || sq < 0.0f) {
                        const float y = isnan(a) ? B.at(RF_X, pr) : (sq == -1.0f ? B.at(RF_LO, pr) : B.at(RF_HI, pr));
                        e = elim_fixed(y);
                    } else {
                        e = elim_step(a, B.at(RF_C, pr), B.at(RF_R, pr));
                    }
                }
                const Elim pre = block_scan_elim<NT>(e, etot, t);
                if (act && pr >= 0) {
                    B.at(RF_P, pr) = (float)pre.m01;
                    B.at(RF_O, pr) = (float)pre.b1;
                }
                if (NT == 64 && WS) wave_lds_sync();
                else __syncthreads();
                if (in) w = row_load(B, p);
            }
            if (fu && whole) {
                st = B.at(RF_Q, p);
                const float P2 = B.at(RF_P, p), Q2 = B.at(RF_O, p);
                if (st < 0.0f) {
                    u2 = Ramp{0.0f, Q2, Q2, Q2};
                } else if (p == ps) {
                    const float y0 = fmaf(P2, x, Q2);
                    u2 = Ramp{0.0f, y0, y0, y0};
                } else {
                    u2 = Ramp{P2, Q2, -MG_BIG, MG_BIG};
                }
            } else if (fu) {
                st = B.at(RF_Q, p);
                float P2 = 0.0f, Q2 = su;
#pragma nounroll
                for (int qq = last; qq >= p; qq--) {
                    const float sq = B.at(RF_Q, qq);
                    if (sq < 0.0f) {
                        P2 = 0.0f;
                        Q2 = sq == -1.0f ? B.at(RF_LO, qq) : B.at(RF_HI, qq);
                    } else {
                        const float cq = B.at(RF_C, qq);
                        const float inv = __builtin_amdgcn_rcpf(fmaf(-cq, P2, 1.0f));
                        P2 = B.at(RF_A, qq) * inv;
                        Q2 = fmaf(cq, Q2, -B.at(RF_R, qq)) * inv;
                    }
                }
                if (st < 0.0f) {
                    u2 = Ramp{0.0f, Q2, Q2, Q2};
                } else if (p == ps) {
                    const float y0 = fmaf(P2, x, Q2);
                    u2 = Ramp{0.0f, y0, y0, y0};
                } else {
                    u2 = Ramp{P2, Q2, -MG_BIG, MG_BIG};
                }
            }
            Ramp tot2;
            const Ramp ex2 = block_scan_excl<NT>(u2, wtot, 0, tot2, t, ml);
            if (fu) {
                yv = ramp_eval(u2, ramp_eval(ex2, 0.0f));
                B.at(RF_O, p) = yv;
            }
            if (NT == 64 && WS) wave_lds_sync();
            else __syncthreads();
            // new held state: a free cell outside its box is held; a held cell is released where
            // its row points back into the box (beyond rounding)
            bool chg = false;
            if (fu) {
                float ns = st;
                if (!w.ok) {
                    // a cell of S = 0 (whole lines only) stays at its old value
                } else if (st == 0.0f) {
                    ns = yv < w.lo ? -1.0f : (yv > w.hi ? -2.0f : 0.0f);
                } else {
                    const float yp = p == ps ? x : B.at(RF_O, p - 1);
                    const float yn = p == last ? su : B.at(RF_O, p + 1);
                    const float ta = w.a * yp, tc = w.c * yn;
                    const float vr = (ta + tc) - w.rr;
                    const float tol = 2e-6f * (fabsf(ta) + fabsf(tc) + fabsf(w.rr) + fabsf(yv));
                    ns = st == -1.0f ? (vr > w.lo + tol ? 0.0f : -1.0f) : (vr < w.hi - tol ? 0.0f : -2.0f);
                }
                chg = (ns < 0.0f) != (st < 0.0f);
                B.at(RF_Q, p) = ns;
            }
            bool more;
            if (NT == 64 && WS) {
                more = __ballot(chg) != 0ull;
                if (more) wave_lds_sync();
            } else {
                const unsigned long long bc = __ballot(chg);
                if (lane == 0) wbad[threadIdx.x >> 6] = bc != 0ull ? 1u : 0u;
                __syncthreads();
                more = block_flag(wbad);
            }
            if (!more) break;
            if (pass + 1 == repair_passes(whole)) {
                if (fu && p == ps) long_active_set(B, ps, Lu, ml, x);
                if (NT == 64 && WS) wave_lds_sync();
                else __syncthreads();
                if (fu) yv = B.at(RF_O, p);
                break;
            }
        }
        if (fu) v = mg_clip(yv, w.lo, w.hi);
    }
    if (write && in) {
        if (A.tout) A.tout[(long long)q * A.tpitch + r] = v;
        else A.phi_new[(long long)r * A.pitch + q] = v;
    }
    return v;
}

// One band of four lines (one per class r mod 4) of a directional sweep,
// processed in the class order 0,1,2,3 (forward) or 3,2,1,0 (reverse); the
// neighbouring band's first-processed line is recomputed (not written) where
// a line of this band needs it fresh.
//
// Step st of the band (0..4): its line, whether it is the recomputed
// neighbour, and whether its up / down neighbour values are fresh registers.
// Forward order: r0, r0+1, r0+2, [r0+4 recomputed], r0+3.
// Reverse order: r0+3, r0+2, r0+1, [r0-1 recomputed], r0.
template <bool REV>
__device__ __forceinline__ int band_line(int r0, int st)
{
    if (!REV) return (st < 3) ? r0 + st : (st == 3 ? r0 + 4 : r0 + 3);
    return (st < 3) ? r0 + 3 - st : (st == 3 ? r0 - 1 : r0);
}
template <bool REV>
__device__ __forceinline__ void band_step(int r0, int nl, int st, int &r, bool &redundant, bool &up_fresh,
                                          bool &dn_fresh)
{
    r = band_line<REV>(r0, st);
    redundant = st == 3;
    // an own line processed before this step (steps 0, 1, 2 are own lines)
    bool have_prev = false;
    for (int s2 = 0; s2 < 3 && s2 < st; s2++) {
        const int rr = band_line<REV>(r0, s2);
        have_prev |= rr >= 0 && rr < nl;
    }
    if (redundant) { up_fresh = false; dn_fresh = false; }
    else if (st < 3) { up_fresh = have_prev; dn_fresh = false; }
    else {
        // the last own line: upstream = the line processed just before it,
        // downstream = the recomputed neighbour line (if it exists)
        up_fresh = have_prev;
        const int rn = REV ? r0 - 1 : r0 + 4;
        dn_fresh = rn >= 0 && rn < nl;
    }
}

// One band of a sweep with lines of at most NT cells, one cell per thread.
// PF: read the next step's inputs before computing the current line, so that
// their latency overlaps the current line's phases (the registers of one more
// CellIn).  B: the first of two row buffers; lpar: the caller's running line
// count, whose parity picks the buffer of each line (it continues across
// bands that one workgroup takes one after another).
template <int NT, bool REV, bool PF = false, bool CF = false, bool WS = false, bool WH = false>
__device__ __forceinline__ void sweep_band(const LineArgs &A, int b, const RunBuf &B, uint64_t *msk, Ramp *wtot,
                                           unsigned *wbad, Elim *etot, int &lpar)
{
    // transposed output of a full band: the band's 4 lines are 4 consecutive
    // floats of the output layout, written as one 16-byte store per cell
    float prev = 0.0f, red = 0.0f, o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
    // t: the thread's cell in the group of NT threads that takes the band
    const int nl = A.nl, ml = A.ml, t = threadIdx.x % NT;
    const int r0 = 4 * b;
    const bool pack = A.tout != nullptr && r0 + 3 < nl;
    // a split sweep takes the band's first three lines, or its fourth with both neighbours in memory
    auto valid = [&](int st) {
        const int r = band_line<REV>(r0, st);
        return r >= 0 && r < nl && !((A.split == 1 && st >= 3) || (A.split == 2 && st != 4));
    };
    auto load = [&](int r, bool uf, bool df, CellIn &c) {
        if (t < ml) cell_load<REV, CF>(line_rows<REV>(A, r, uf, df), ml, t, c);
    };
    CellIn la, lb;
    int st = 0;
    while (st < 5 && !valid(st)) st++;
    if (PF && st < 5) {
        int r; bool rdd, uf, df;
        band_step<REV>(r0, nl, st, r, rdd, uf, df);
        if (A.split == 2) { uf = false; df = false; }
        load(r, uf, df, la);
    }
#pragma nounroll
    while (st < 5) {
        int r; bool redundant, up_fresh, dn_fresh;
        band_step<REV>(r0, nl, st, r, redundant, up_fresh, dn_fresh);
        if (A.split == 2) { up_fresh = false; dn_fresh = false; }
        int nx = st + 1;
        while (nx < 5 && !valid(nx)) nx++;
        if (PF) {
            if (nx < 5) {
                int r2; bool rd2, uf2, df2;
                band_step<REV>(r0, nl, nx, r2, rd2, uf2, df2);
                if (A.split == 2) { uf2 = false; df2 = false; }
                load(r2, uf2, df2, lb);
            }
        } else {
            load(r, up_fresh, dn_fresh, la);
        }
        const float cur = sweep_line<NT, REV, CF, WS, WH>(A, r, B.other(lpar & 1), msk, !redundant && !pack, prev,
                                                      up_fresh, red, dn_fresh, wtot, wbad, etot, la, t, true);
        lpar++;
        const int li = r - r0;
        if (redundant) red = cur;
        else prev = cur;
        if (!redundant) {
            if (li == 0) o0 = cur;
            else if (li == 1) o1 = cur;
            else if (li == 2) o2 = cur;
            else o3 = cur;
        }
        if (PF) la = lb;
        st = nx;
    }
    if (pack && t < ml) {
        const int q = REV ? ml - 1 - t : t;
        *reinterpret_cast<float4 *>(A.tout + (long long)q * A.tpitch + r0) = make_float4(o0, o1, o2, o3);
    }
}

// One band of a sweep with lines of at most NT cells in a workgroup of 2 NT
// threads.  The neighbouring band's line that the band recomputes reads old
// values only (both of its cross-line neighbours are processed after it), so
// the upper half computes it beside the band's first line and leaves it in
// LDS (redl, by visit position), while the lower half takes the band's own
// lines: four line steps instead of five.  Both halves take four steps (a
// half with no line in a step takes only that step's barriers), so every
// block barrier is reached by all waves.  Each half has its own masks, row
// buffers and scan totals.  Lines of one wave (NT = 64) take no block barrier
// inside a step: each half runs its own steps, and one block barrier before
// the last step publishes the recomputed line.
template <int NT, bool REV, bool PF, bool CF, bool WH>
__device__ __forceinline__ void sweep_band2(const LineArgs &A, int b, const RunBuf &B0, const RunBuf &B1,
                                            uint64_t *msk0, uint64_t *msk1, Ramp *wtot0, Ramp *wtot1, float *redl,
                                            unsigned *wbad, Elim *etot0, Elim *etot1)
{
    constexpr bool WS = NT == 64;
    // read all four steps' inputs at the start where the registers allow it
    constexpr bool DEEP = PF && (WS || (CF && NT <= 512));
    const int nl = A.nl, ml = A.ml;
    const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT);
    const int t = threadIdx.x - half * NT;
    const int r0 = 4 * b;
    const bool pack = A.tout != nullptr && r0 + 3 < nl;
    const RunBuf B = half ? B1 : B0;
    uint64_t *msk = half ? msk1 : msk0;
    Ramp *wtot = half ? wtot1 : wtot0;
    Elim *etot = half ? etot1 : etot0;
    auto valid = [&](int st) { const int r = band_line<REV>(r0, st); return r >= 0 && r < nl; };
    // the band step of this half's k-th call (-1: none): lower 0, 1, 2, 4; upper 3
    auto step_of = [&](int k) { return half == 0 ? (k < 3 ? k : 4) : (k == 0 ? 3 : -1); };
    auto load = [&](int k, CellIn &c) {
        const int st = step_of(k);
        if (st < 0 || !valid(st) || t >= ml) return;
        int r; bool rdd, uf, df;
        band_step<REV>(r0, nl, st, r, rdd, uf, df);
        cell_load<REV, CF>(line_rows<REV>(A, r, uf, df), ml, t, c);
    };
    float prev = 0.0f, o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
    // read-ahead: the next step's inputs, or (DEEP) all four steps' inputs at once
    CellIn la{}, lb{}, lc{}, ld{};
    if (PF) {
        load(0, la);
        if (DEEP) { load(1, lb); load(2, lc); load(3, ld); }
    }
#pragma nounroll
    for (int k = 0; k < 4; k++) {
        const int st = step_of(k);
        const bool act = st >= 0 && valid(st);
        int r = r0; bool redundant = false, up_fresh = false, dn_fresh = false;
        if (act) band_step<REV>(r0, nl, st, r, redundant, up_fresh, dn_fresh);
        if (PF) {
            if (!DEEP && k + 1 < 4) load(k + 1, lb);
        } else {
            load(k, la);
        }
        // the recomputed line was left in LDS by the upper half at k = 0 (barriers of the calls between,
        // or the one below for one-wave lines)
        if (WS && k == 3) __syncthreads();
        const float dnv = act && dn_fresh && t < ml ? redl[t] : 0.0f;
        float cur = 0.0f;
        if (act) {
            cur = sweep_line<NT, REV, CF, WS, WH>(A, r, B.other(k & 1), msk, !redundant && !pack, prev, up_fresh, dnv,
                                              dn_fresh, wtot, wbad, etot, la, t, true);
        } else if (!WS) {
            // a half with no line takes the line step's barriers only: the one after the rows and
            // masks, the scan's (several waves), and those of the long-unit check (its waves
            // publish no failure)
            const bool whole = WH && ml > 3;
            __syncthreads();
            if (whole) {
                if (NT > 64) __syncthreads();
                __syncthreads();
            }
            if (NT > 64) __syncthreads();
            if (long_units_possible(A)) {
                const bool l0 = (threadIdx.x & 63) == 0;
                if (l0) wbad[threadIdx.x >> 6] = 0u;
                __syncthreads();
                if (block_flag(wbad)) {
                    // the repair's passes: [whole lines: elimination scan and its publication,]
                    // scan, values, flags (and the serial finish after repair_passes)
                    for (int pass = 0;; pass++) {
                        if (whole) {
                            if (NT > 64) __syncthreads();
                            __syncthreads();
                        }
                        if (NT > 64) __syncthreads();
                        __syncthreads();
                        if (l0) wbad[threadIdx.x >> 6] = 0u;
                        __syncthreads();
                        if (!block_flag(wbad)) break;
                        if (pass + 1 == repair_passes(whole)) {
                            __syncthreads();
                            break;
                        }
                    }
                }
            }
        }
        if (act) {
            if (redundant) {
                if (t < ml) redl[t] = cur;
            } else {
                prev = cur;
                const int li = r - r0;
                if (li == 0) o0 = cur;
                else if (li == 1) o1 = cur;
                else if (li == 2) o2 = cur;
                else o3 = cur;
            }
        }
        if (PF) {
            la = lb;
            if (DEEP) { lb = lc; lc = ld; }
        }
    }
    if (half == 0 && pack && t < ml) {
        const int q = REV ? ml - 1 - t : t;
        *reinterpret_cast<float4 *>(A.tout + (long long)q * A.tpitch + r0) = make_float4(o0, o1, o2, o3);
    }
}

// --------------------------------------------------------------------------
// Lines longer than one workgroup: NT threads take K rounds of NT cells, one
// round after another, so that only one round's inputs are held at a time.
// A unit of at most three cells, or one that crosses into the next round,
// has its chain ramp at its LAST position (its other cells take the
// identity): the scan's exclusive prefix there is the value entering the
// unit, and a unit that begins in one round and ends in the next is solved
// in the next round, where all of its rows are known (units are at most one
// round long, so the ring of two rounds holds every row of a unit).  A unit
// of more than three cells inside one round is solved as on shorter lines:
// every cell eliminates from the unit's end down to itself, takes its Z_k
// into the scan and checks its own row; the first cell's thread finishes a
// unit whose check failed with the active-set iteration.  The unit rows live in
// a ring of two rounds (RingBuf).  A cell's new value is written as soon as
// it is final (cells of a unit that ends in the next round: one round
// later).  LDS holds the previous own line (the fresh upstream neighbour,
// prev) and the recomputed neighbour line (red), each cell at its visit
// position, read and written only by the thread that owns the position.  A
// split sweep (written in its own layout) recomputes no line and reads the
// previous own line from the plane it was written to (A.fresh; visible after
// the barrier that opens the next line), so its LDS is the masks and the
// ring alone.
// The transposed output of a full band goes out as float2 pairs of lines
// (0, 1) and (2, 3), written when the pair's second line is done.  The
// rounds are a loop, not unrolled: one copy of the round's code, and no
// per-round addresses held across rounds.
template <int NT, bool REV, bool CF>
__device__ __forceinline__ void long_band(const LineArgs &A, int b, float *ring, float *prev, float *red,
                                          uint64_t *msk, Ramp *wtot, unsigned *wlast, unsigned *wfail)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nl = A.nl, ml = A.ml, nw = (ml + 63) >> 6;
    const RingBuf<2 * NT> B{ring};
    const float area = A.area ? (float)(*A.area) : 0.0f;
    auto cell = [&](int p) { return REV ? ml - 1 - p : p; };
    const int K = (ml + NT - 1) / NT;
    const int r0 = 4 * b;
    const bool pack = A.tout != nullptr && r0 + 3 < nl;
    const bool gfresh = A.split != 0;      // no line in LDS: prev and red are not there
#pragma nounroll
    for (int st = 0; st < 5; st++) {
        int r; bool redundant, up_fresh, dn_fresh;
        band_step<REV>(r0, nl, st, r, redundant, up_fresh, dn_fresh);
        if (r < 0 || r >= nl) continue;
        // a split sweep: the first three lines, or the fourth with both neighbours final in memory
        if ((A.split == 1 && st >= 3) || (A.split == 2 && st != 4)) continue;
        if (A.split == 2) { up_fresh = false; dn_fresh = false; }
        const bool has_up = REV ? r + 1 < nl : r > 0, has_dn = REV ? r > 0 : r + 1 < nl;
        // a split sweep reads the fresh upstream line from memory with the cell's other inputs
        const bool upg = gfresh && up_fresh;
        LineRows R = line_rows<REV>(A, r, up_fresh && !upg, dn_fresh);
        if (upg) R.vu = A.fresh + (long long)(REV ? r + 1 : r - 1) * A.pitch;
        // steps 1 and 4 end a pair of own lines (forward: 0,1 and 2,3; reverse: 3,2 and 1,0)
        const bool pair_w = pack && (st == 1 || st == 4);
        const bool single_w = !redundant && !pack;
        const int rp = r0 + ((r - r0) & 2);
        // the final value v of position p: write it, keep it (a split sweep writes its own
        // layout, never pairs)
        auto fin = [&](int p, float v) {
            const long long q = cell(p);
            if (single_w) {
                if (A.tout) A.tout[q * A.tpitch + r] = v;
                else A.phi_new[(long long)r * A.pitch + q] = v;
            } else if (pair_w) {
                const float o = prev[p];
                *reinterpret_cast<float2 *>(A.tout + q * A.tpitch + rp) = REV ? make_float2(v, o) : make_float2(o, v);
            }
            if (!gfresh) {
                if (redundant) red[p] = v;
                else prev[p] = v;
            }
        };
        // starred masks of the whole line
#pragma nounroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            const bool s0 = p < ml && starred(A, R.lab[cell(p)]);
            const unsigned long long bm = __ballot(s0);
            if (lane == 0 && k * NT + wave * 64 < ml) msk[((k * NT) >> 6) + wave] = bm;
        }
        __syncthreads();
        float carry = 0.0f;
        bool pend = false;                       // the last round's cell waits for a unit ending in this one
        // the next round's inputs are read at the start of a round (round 0: here),
        // so that their latency overlaps the round's computation
        CellIn cn;
        if (t < ml) cell_load<REV, CF>(R, ml, t, cn);
#pragma nounroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            const bool in = p < ml;
            const CellIn c = cn;
            if (p + NT < ml) cell_load<REV, CF>(R, ml, p + NT, cn);
            CellRow w;
            w.ok = false; w.x = 0.0f;
            bool inu = false, last = false;
            int ps = p, L = 1;
            if (in) {
                const float vu = has_up ? (up_fresh && !upg ? prev[p] : c.vu) : 0.0f;
                const float vd = has_dn ? (dn_fresh ? red[p] : c.vd) : 0.0f;
                w = cell_row<REV, CF>(A, c, r, cell(p), vu, vd, area);
                if (mask_bit(msk, p)) {
                    unit_of(msk, nw, ml, p, run_cut(A) > 0 && run_cut(A) < NT ? run_cut(A) : NT, ps, L);
                    inu = true;
                } else if (p >= 1 && mask_bit(msk, p - 1) && (p < 2 || !mask_bit(msk, p - 2))) {
                    ps = p - 1; L = 2;               // the cell after a single starred cell
                    inu = true;
                }
                last = inu && ps + L - 1 == p;
                if (inu) {
                    row_store(B, p, w);
                    B.at(RG_S, p) = c.sig;
                }
            }
            // a unit of more than three cells inside this round: every cell eliminates from the
            // unit's last cell down to itself and takes its Z_k into the scan (as on shorter lines)
            const bool inr = inu && L > 3 && ps >= k * NT && ps + L - 1 < (k + 1) * NT;
            // rows of the round visible; uk: a unit of the block ends in this round
            const unsigned long long lm = __ballot(last);
            if (lane == 0) wlast[wave] = lm != 0ull ? 1u : 0u;
            __syncthreads();
            const bool uk = __ballot(lane < NT / 64 && wlast[lane] != 0u) != 0ull;
            Ramp u = ramp_id();
            if (in && !inu) u = cell_ramp(w);
            float lP1 = 0.0f, lQ1 = 0.0f;
            if (inr) {
                const int lp = ps + L - 1;
                float P, Q;
                long_elim(B, p, lp, B.sig_after(lp, ml), P, Q, lP1, lQ1);
                u = Ramp{P, Q, w.lo, w.hi};
                if (p == ps) B.at(RF_P, ps) = 0.0f;      // the unit's failed-check flag
            } else if (last) {
                if (L <= 2) {
                    PairRows Q;
                    pair_load(B, ps, L, ml, Q);
                    u = pair_ramp(Q, L);
                } else if (L == 3) {
                    TriRows T3;
                    tri_load(B, ps, ml, T3);
                    u = tri_ramp(T3);
                } else {
                    u = long_ramp(B, ps, L, ml);
                }
            }
            Ramp tot;
            const Ramp ex = block_scan_excl<NT>(u, wtot, k & 1, tot, t);
            const float x = ramp_eval(ex, carry);
            float v = 0.0f;
            if (in && (!inu || inr)) v = ramp_eval(u, x);
            carry = ramp_eval(tot, carry);
            // the row check of an in-round unit's cell at its predecessor's value x and its
            // successor's Z_{k+1}(v)
            bool bad = false;
            if (inr) {
                const int lp = ps + L - 1;
                const float yn = p == lp ? lQ1 : mg_clip(fmaf(lP1, v, lQ1), B.at(RF_LO, p + 1), B.at(RF_HI, p + 1));
                const float ta = w.a * x, tc = w.c * yn;
                bad = w.ok && !long_row_ok(v, (ta + tc) - w.rr, fabsf(ta) + fabsf(tc) + fabsf(w.rr), w.lo, w.hi);
                B.y(p) = v;
                if (bad) B.at(RF_P, ps) = 1.0f;
            }
            if (uk) {
                const unsigned long long fb = __ballot(bad);
                if (lane == 0) wfail[wave] = fb != 0ull ? 1u : 0u;
                if (last && !inr) {
                    if (L <= 2) {
                        PairRows Q;
                        pair_load(B, ps, L, ml, Q);
                        float y0, y1;
                        pair_solve(Q, L, x, y0, y1);
                        B.y(ps) = y0;
                        if (L == 2) B.y(ps + 1) = y1;
                    } else if (L > 3) {
                        long_solve(B, ps, L, ml, x);
                    } else {
                        TriRows T3;
                        tri_load(B, ps, ml, T3);
                        float y0, y1, y2;
                        tri_solve(T3, x, y0, y1, y2);
                        B.y(ps) = y0;
                        B.y(ps + 1) = y1;
                        B.y(ps + 2) = y2;
                    }
                }
                __syncthreads();
                // an in-round unit whose check failed: its first cell's thread finishes it with the
                // active-set iteration from the scan's values
                if (__ballot(lane < NT / 64 && wfail[lane] != 0u) != 0ull) {
                    if (inr && p == ps && B.at(RF_P, ps) != 0.0f) long_active_set(B, ps, L, ml, x);
                    __syncthreads();
                }
                if (inu && ps + L - 1 < (k + 1) * NT) v = B.y(p);
                if (k > 0 && pend) fin(p - NT, B.y(p - NT));
            }
            pend = inu && ps + L - 1 >= (k + 1) * NT;
            if (in && !pend) fin(p, v);
        }
    }
}

// Workgroup of the long-line kernel: 1024 threads; rounds of 1024 cells, so
// units of up to 1024 cells fit the ring of two rounds.  A split sweep keeps
// no line in LDS (masks and ring: about 73 KB at 8192 cells), so two
// workgroups share a CU.
constexpr int LONG_NT = 1024;
// dynamic LDS of the long-line kernel: [starred masks][RING_FIELDS fields x 2 NT
// ring][prev: ml floats][red: ml floats]; lines = false (a split sweep): no prev, no red
template <int NT>
__host__ __device__ inline size_t long_lds_bytes(int ml, bool lines = true)
{
    return (size_t)sweep_mask_words(ml) * 8 +
           ((size_t)RING_FIELDS * 2 * NT + (lines ? 2 * (size_t)ml : 0)) * sizeof(float);
}
// Eight waves per SIMD (two 1024-thread workgroups per CU): at most 64
// registers per lane; the few values the compiler then keeps in scratch cost
// less than the second workgroup gains, which runs its rounds while the other
// waits at a barrier behind a long unit's serial solve.
template <int NT, bool REV, bool CF>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(8 * NT / 1024))) k_sweep_long(LineArgs A)
{
    if (A.skip && *A.skip) return;
    extern __shared__ uint64_t smem64[];
    __shared__ Ramp wtot[2 * (NT / 64)];
    __shared__ unsigned wlast[NT / 64], wfail[NT / 64];
    uint64_t *msk = smem64;
    float *ring = reinterpret_cast<float *>(smem64 + sweep_mask_words(A.ml));
    float *prev = ring + RING_FIELDS * 2 * NT;
    // (a split sweep touches neither prev nor red; its launch leaves out their room)
    long_band<NT, REV, CF>(A, blockIdx.x, ring, prev, prev + A.ml, msk, wtot, wlast, wfail);
}

// dynamic LDS: [starred masks, 8 B per 64 cells][2 x RB_FIELDS * ml floats of rows]
__host__ __device__ inline size_t sweep_lds_bytes(int ml)
{
    return (size_t)sweep_mask_words(ml) * 8 + 2 * (size_t)RB_FIELDS * ml * sizeof(float);
}

// dynamic LDS of the two-half sweep: [masks of each half][2 x RB_FIELDS * ml
// floats of rows of each half][ml floats of the recomputed line]
__host__ __device__ inline size_t sweep2_lds_bytes(int ml)
{
    return 2 * sweep_lds_bytes(ml) + (size_t)ml * sizeof(float);
}

template <int NT, bool REV, bool CF, bool WH = false>
__global__ void __launch_bounds__(2 * NT) k_sweep2(LineArgs A)
{
    if (A.skip && *A.skip) return;
    extern __shared__ uint64_t smem64[];
    __shared__ Ramp wtot[2][2 * (NT / 64)];
    __shared__ unsigned wbad[2 * (NT / 64)];
    __shared__ Elim etot[2][NT / 64];
    const int nw = sweep_mask_words(A.ml);
    RunBuf B0, B1;
    B0.fs = A.ml;
    B0.p = reinterpret_cast<float *>(smem64 + 2 * nw);
    B1.fs = A.ml;
    B1.p = B0.p + 2 * RB_FIELDS * A.ml;
    float *redl = B1.p + 2 * RB_FIELDS * A.ml;
    // read-ahead of the next line where the registers allow it (1024 threads: only with the stored
    // coefficients, and not beside the whole-line elimination)
    sweep_band2<NT, REV, (NT <= 256 || (CF && !WH)), CF, WH>(A, blockIdx.x, B0, B1, smem64, smem64 + nw, wtot[0], wtot[1], redl,
                                                wbad, etot[0], etot[1]);
}

template <int NT, bool REV, bool CF, bool WH = false>
__global__ void __launch_bounds__(NT) k_sweep(LineArgs A)
{
    if (A.skip && *A.skip) return;
    extern __shared__ uint64_t smem64[];
    __shared__ Ramp wtot[2 * (NT / 64 > 0 ? NT / 64 : 1)];
    __shared__ unsigned wbad[NT / 64 > 0 ? NT / 64 : 1];
    __shared__ Elim etot[NT / 64 > 0 ? NT / 64 : 1];
    uint64_t *msk = smem64;
    RunBuf B;
    B.fs = A.ml;
    B.p = reinterpret_cast<float *>(smem64 + sweep_mask_words(A.ml));
    // read-ahead of the next line where the registers allow it (at 1024 threads, 128 registers per
    // lane: only with the stored coefficients)
    int lpar = 0;
    sweep_band<NT, REV, (NT <= 512 || CF) && !WH, CF, false, WH>(A, blockIdx.x, B, msk, wtot, wbad, etot, lpar);
}
