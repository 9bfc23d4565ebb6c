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
__device__ __forceinline__ float mg_clip(float x, float lo, float hi)
{
    return fminf(fmaxf(x, lo), hi);
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
    float *tout;                        // non-null: new values written transposed,
    int tpitch;                         //   cell q of line r at tout[q * tpitch + r]
    float *scr;                         // unit-row scratch of lines longer than RB_LDS_MAX
    const double *area;                 // Rada-Chen area term (null: 0)
    int pitch, lpitch, nl, ml;
    float kap, e2, M, eps;
    int bit, scaled;
};

// --------------------------------------------------------------------------
// Collective units of Hybrid Smoother 2 (Sec. 4.3, Fig. 3).  A maximal run
// of starred cells along the line is solved as one box-constrained
// tridiagonal system; a single starred cell takes the next cell of the line
// into its unit (a single starred cell at the line end stays alone).  Runs
// longer than RUN_MAX are cut into ceil(len / RUN_MAX) pieces of near-equal
// length (the longer pieces first), each solved as its own unit, so that
// every unit fits in registers.
#define RUN_MAX 4
// A held cell is released only when its residual points inward by more than
// FP32 rounding, so that the hold / release iteration cannot alternate on a
// cell whose free value equals its bound.
#define RUN_TOL 1e-6f

// Row buffer of the line being swept, indexed by visit position p:
//   a y_{p-1} - y_p + c y_{p+1} = r  (a = NaN marks S = 0), box [lo, hi],
// x = old value, y = new value of a unit cell.  LDS for lines up to
// RB_LDS_MAX cells, else a global scratch plane of the band.
enum { RF_A = 0, RF_C, RF_R, RF_LO, RF_HI, RF_X, RF_Y, RF_COUNT };
#define RB_LDS_MAX 2048

struct RunBuf {
    float *p;
    int fs;            // elements between fields (>= line length)
    __device__ __forceinline__ float &at(int f, int q) const { return p[f * fs + q]; }
};

struct RunRegs {
    float a[RUN_MAX], c[RUN_MAX], r[RUN_MAX], lo[RUN_MAX], hi[RUN_MAX];
    float sig;         // old value of the cell after the unit (0 at the line end)
    int L;
    unsigned hh, hl;   // bit k: the old value of cell k sits at its upper / lower bound
    bool ok;           // false: an S = 0 cell, the unit keeps its values
};

__device__ __forceinline__ void run_load(const RunBuf &B, int ps, int L, int ml, RunRegs &R)
{
    R.L = L;
    R.ok = true;
    R.hh = 0u; R.hl = 0u;
#pragma unroll
    for (int k = 0; k < RUN_MAX; k++) {
        if (k < L) {
            R.a[k] = B.at(RF_A, ps + k); R.c[k] = B.at(RF_C, ps + k); R.r[k] = B.at(RF_R, ps + k);
            R.lo[k] = B.at(RF_LO, ps + k); R.hi[k] = B.at(RF_HI, ps + k);
            const float x = B.at(RF_X, ps + k);
            if (x >= R.hi[k]) R.hh |= 1u << k;
            else if (x <= R.lo[k]) R.hl |= 1u << k;
            if (isnan(R.a[k])) R.ok = false;
        } else {
            R.a[k] = 0.0f; R.c[k] = 0.0f; R.r[k] = 0.0f; R.lo[k] = 0.0f; R.hi[k] = 0.0f;
        }
    }
    R.sig = ps + L < ml ? B.at(RF_X, ps + L) : 0.0f;
}

// Thomas pass with held rows (bit k of hh / hl) as identity rows y_k = bound
__device__ __forceinline__ bool run_thomas_regs(const RunRegs &R, unsigned hh, unsigned hl, float x,
                                                float (&y)[RUN_MAX])
{
    float qq[RUN_MAX];
    float pprev = x, qprev = 0.0f;
#pragma unroll
    for (int k = 0; k < RUN_MAX; k++) {
        if (k >= R.L) { y[k] = 0.0f; qq[k] = 0.0f; continue; }
        if ((hh >> k) & 1u) { y[k] = R.hi[k]; qq[k] = 0.0f; }
        else if ((hl >> k) & 1u) { y[k] = R.lo[k]; qq[k] = 0.0f; }
        else {
            const float a = R.a[k];
            const float den = (k == 0) ? 1.0f : 1.0f - a * qprev;
            if (!(den > 0.0f)) return false;
            const float inv = __builtin_amdgcn_rcpf(den);
            y[k] = (a * pprev - R.r[k]) * inv;
            if (k == R.L - 1) { y[k] = y[k] + R.c[k] * inv * R.sig; qq[k] = 0.0f; }
            else qq[k] = R.c[k] * inv;
        }
        pprev = y[k]; qprev = qq[k];
    }
#pragma unroll
    for (int k = RUN_MAX - 2; k >= 0; k--)
        if (k + 1 < R.L) y[k] = fmaf(qq[k], y[k + 1], y[k]);
    return true;
}

// The unit's variational inequality: y in [lo, hi], y_k at a bound only
// where its row pushes outward.  Active-set iteration: free cells solved
// exactly with held cells as known values, free cells outside the box held,
// held cells whose residual turns inward released, until stable (at most
// 2 L + 4 passes), starting from the cells whose old value sits at a bound.
// pin = -1 / +1 holds cell 0 at its lower / upper bound (the limit of an
// incoming value -> -inf / +inf); pin = 0 uses x.
__device__ __forceinline__ bool run_vi_regs(const RunRegs &R, float x, int pin, float (&y)[RUN_MAX])
{
    if (!R.ok) return false;
    unsigned hh = R.hh, hl = R.hl;
    if (pin > 0) { hh |= 1u; hl &= ~1u; }
    else if (pin < 0) { hl |= 1u; hh &= ~1u; }
    for (int it = 0; it < 2 * R.L + 4; it++) {
        if (!run_thomas_regs(R, hh, hl, x, y)) return false;
        unsigned nh = hh, nl = hl;
#pragma unroll
        for (int k = 0; k < RUN_MAX; k++) {
            if (k >= R.L) continue;
            const unsigned bit = 1u << k;
            if (!((hh | hl) & bit)) {
                if (y[k] > R.hi[k]) nh |= bit;
                else if (y[k] < R.lo[k]) nl |= bit;
            } else if (!(k == 0 && pin != 0)) {
                const float yp = (k == 0) ? x : y[k > 0 ? k - 1 : 0];
                const float yn = (k == R.L - 1) ? R.sig : y[k + 1 < RUN_MAX ? k + 1 : k];
                const float v = R.a[k] * yp + R.c[k] * yn - R.r[k] - y[k];
                const float tau = RUN_TOL * (fabsf(R.a[k] * yp) + fabsf(R.c[k] * yn) + fabsf(R.r[k]) + fabsf(y[k]));
                if ((hh & bit) && v < -tau) nh &= ~bit;
                if ((hl & bit) && v > tau) nl &= ~bit;
            }
        }
        if (nh == hh && nl == hl) break;
        hh = nh; hl = nl;
    }
#pragma unroll
    for (int k = 0; k < RUN_MAX; k++)
        if (k < R.L) y[k] = mg_clip(y[k], R.lo[k], R.hi[k]);
    return true;
}

// unconstrained affine solution of the last cell: y_L = u_L + v_L x
__device__ __forceinline__ bool run_affine_regs(const RunRegs &R, float &uL, float &vL)
{
    if (!R.ok) return false;
    float pu = 0.0f, pv = 0.0f, q = 0.0f;
#pragma unroll
    for (int k = 0; k < RUN_MAX; k++) {
        if (k >= R.L) continue;
        const float a = R.a[k];
        const float den = (k == 0) ? 1.0f : 1.0f - a * q;
        if (!(den > 0.0f)) return false;
        const float inv = __builtin_amdgcn_rcpf(den);
        const float npu = (k == 0) ? -R.r[k] * inv : (a * pu - R.r[k]) * inv;
        const float npv = (k == 0) ? a * inv : a * pv * inv;
        pu = npu; pv = npv;
        if (k == R.L - 1) { pu = pu + R.c[k] * inv * R.sig; q = 0.0f; }
        else q = R.c[k] * inv;
    }
    uL = pu; vL = pv;
    return true;
}

__device__ __forceinline__ float last_of(const float (&y)[RUN_MAX], int L)
{
    float v = y[0];
#pragma unroll
    for (int k = 1; k < RUN_MAX; k++)
        if (k == L - 1) v = y[k];
    return v;
}

// The map from the value entering the unit to the value of its last cell is
// the clipped ramp clip(u_L + v_L x, y-, y+): y_L is the unconstrained
// affine solution while every cell is free, and constant (y- / y+, the
// solutions with cell 0 held at its bounds) once a cell holds.  yold: the
// old value of the last cell (kept by a unit with an S = 0 cell).
__device__ __forceinline__ Ramp unit_ramp(const RunRegs &R, float yold)
{
    float uL = 0.0f, vL = 0.0f, ylo = 0.0f, yhi = 0.0f, y[RUN_MAX];
    bool ok = run_affine_regs(R, uL, vL);
    const bool coupled = R.a[0] > 0.0f;
#pragma nounroll
    for (int s = 0; s < 2 && ok; s++) {
        ok = run_vi_regs(R, 0.0f, coupled ? (s == 0 ? -1 : 1) : 0, y);
        const float v = last_of(y, R.L);
        if (s == 0) ylo = v;
        else yhi = v;
        if (!coupled) { yhi = ylo; vL = 0.0f; uL = ylo; break; }
    }
    if (!ok) return Ramp{0.0f, yold, yold, yold};
    return Ramp{vL, uL, fminf(ylo, yhi), fmaxf(ylo, yhi)};
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
// unit of the starred position p: first position ps and length L
__device__ __forceinline__ void unit_of(const uint64_t *msk, int nw, int ml, int p, int &ps, int &L)
{
    const int t0 = run_first(msk, p), e = run_last(msk, nw, p);
    const int rl = e - t0 + 1;
    if (rl == 1) { ps = p; L = p + 1 < ml ? 2 : 1; return; }
    if (rl <= RUN_MAX) { ps = t0; L = rl; return; }
    const int np = (rl + RUN_MAX - 1) / RUN_MAX, base = rl / np, extra = rl % np;
    const int o = p - t0, big = extra * (base + 1);
    if (o < big) { ps = t0 + (o / (base + 1)) * (base + 1); L = base + 1; }
    else { ps = t0 + big + ((o - big) / base) * base; L = base; }
}

// --------------------------------------------------------------------------
// Block-wide exclusive scan of ramps in thread order: wave-level shuffles,
// then the wave totals through LDS.  Also returns the block total.
__device__ __forceinline__ Ramp shfl_ramp(const Ramp &r, int src_lane)
{
    return Ramp{__shfl(r.a, src_lane), __shfl(r.b, src_lane), __shfl(r.lo, src_lane), __shfl(r.hi, src_lane)};
}

template <int NT>
__device__ __forceinline__ Ramp block_scan_excl(Ramp mine, Ramp *wtot, Ramp &total)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    constexpr int NW = NT / 64;
    Ramp inc = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        Ramp o = shfl_ramp(inc, (lane - off) & 63);
        if (lane >= off) inc = ramp_comp(inc, o);
    }
    Ramp ex = shfl_ramp(inc, (lane - 1) & 63);
    if (lane == 0) ex = ramp_id();
    if (NW > 1) {
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        Ramp pre = ramp_id();
        for (int w = 0; w < wave; w++) pre = ramp_comp(wtot[w], pre);
        ex = ramp_comp(ex, pre);
        Ramp tot = ramp_id();
        for (int w = 0; w < NW; w++) tot = ramp_comp(wtot[w], tot);
        total = tot;
        __syncthreads();
    } else {
        total = shfl_ramp(inc, 63);
    }
    return ex;
}

// --------------------------------------------------------------------------
// One line of one directional sweep.  Cells are taken in visit order
// (REV: q = ml-1 down to 0); thread t handles visit positions p = k*NT + t
// for rounds k = 0..K-1, so that every load is coalesced.  REV takes the
// upstream line at r+1.  up_fresh / dn_fresh: the cross-line neighbour
// values are the caller's registers (same thread, same round = same cell)
// instead of phi_old.  On return val[] holds the new values of the
// thread's cells.  Every point and every unit is a clipped ramp of the value
// entering it, so the line is one block scan; a unit's ramp sits at its first
// position and its other cells take the identity.
template <int NT, int K, bool REV>
__device__ __forceinline__ void sweep_line(const LineArgs &A, int r, const RunBuf &B, uint64_t *msk, bool write,
                                           const float (&upv)[K], bool up_fresh, const float (&dnv)[K],
                                           bool dn_fresh, float (&val)[K], Ramp *wtot)
{
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nl = A.nl, ml = A.ml, P = A.pitch, nw = (ml + 63) >> 6;
    const int ru = REV ? r + 1 : r - 1;      // upstream line
    const int rd = REV ? r - 1 : r + 1;      // downstream line
    const int rm1 = mg_mirror(r - 1, nl), rp1 = mg_mirror(r + 1, nl);
    const long long ro = (long long)r * P;
    const float *ps0 = A.psi + ro, *psm = A.psi + (long long)rm1 * P, *psp = A.psi + (long long)rp1 * P;
    const float *w0 = A.w + ro, *wm = A.w + (long long)rm1 * P, *wp = A.w + (long long)rp1 * P;
    const float *old = A.phi_old + ro;
    const uint8_t *lrow = A.lab + (long long)r * A.lpitch;
    const float e2 = A.e2;
    const float area = A.area ? (float)(*A.area) : 0.0f;
    const bool has_up = ru >= 0 && ru < nl, has_dn = rd >= 0 && rd < nl;
    auto cell = [&](int p) { return REV ? ml - 1 - p : p; };

    // phase 1: frozen coefficients (eq. abcdrc), point ramps, unit rows,
    // starred masks
    float pa[K], pb[K], plo[K], phv[K];
    unsigned sm = 0;
    bool any_star = false;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int p = k * NT + t;
        pa[k] = 0.0f; pb[k] = 0.0f; plo[k] = 0.0f; phv[k] = 0.0f;
        bool s0 = false;
        if (p < ml) {
            const int q = cell(p);
            s0 = ((lrow[q] >> A.bit) & 1) != 0;
            const bool has_next = p + 1 < ml;
            const int qm = mg_mirror(q - 1, ml), qp = mg_mirror(q + 1, ml);
            const float p0 = ps0[q];
            const float w00 = w0[q];
            float xp = 0.0f, xm = 0.0f, lp = 0.0f, lm = 0.0f;
            if (r + 1 < nl)
                xp = mg_face(p0, psp[q], ps0[qp], psp[qp], ps0[qm], psp[qm], w00, wp[q], e2);
            if (r > 0)
                xm = mg_face(psm[q], p0, psm[qp], ps0[qp], psm[qm], ps0[qm], wm[q], w00, e2);
            if (q + 1 < ml)
                lp = mg_face(p0, ps0[q + 1], psp[q], psp[q + 1], psm[q], psm[q + 1], w00, w0[q + 1], e2);
            if (q > 0)
                lm = mg_face(ps0[q - 1], p0, psp[q - 1], psp[q], psm[q - 1], psm[q], w0[q - 1], w00, e2);
            const float dl = A.scaled ? 1.0f : mg_delta(p0, A.eps);
            const float sc = A.kap * dl;
            xp *= sc; xm *= sc; lp *= sc; lm *= sc;
            const float S = xp + xm + lp + lm;
            const float f = A.fit ? dl * (A.fit[ro + q] + area) : 0.0f;   // null fit: f is part of F
            const float Fv = A.F ? A.F[ro + q] : 0.0f;
            const float Xu = REV ? xp : xm, Xd = REV ? xm : xp;
            const float Lp = REV ? lp : lm, Ls = REV ? lm : lp;
            float vu = 0.0f, vd = 0.0f;
            if (has_up) vu = up_fresh ? upv[k] : A.phi_old[(long long)ru * P + q];
            if (has_dn) vd = dn_fresh ? dnv[k] : A.phi_old[(long long)rd * P + q];
            const float rhs = f + Fv - Xu * vu - Xd * vd;
            const float sig = has_next ? old[cell(p + 1)] : 0.0f;
            const float lo = A.lo ? A.lo[ro + q] : -A.M;
            const float hi = A.lo ? A.hi[ro + q] : A.M;
            const float pold = old[q];
            const bool ok = S > 0.0f;
            const float inv = ok ? __builtin_amdgcn_rcpf(S) : 0.0f;
            if (ok) {
                pa[k] = Lp * inv;
                pb[k] = (Ls * sig - rhs) * inv;
                plo[k] = lo;
                phv[k] = hi;
            } else {                          // S == 0: the cell keeps its value
                pa[k] = 0.0f; pb[k] = pold; plo[k] = pold; phv[k] = pold;
            }
            B.at(RF_A, p) = ok ? Lp * inv : __builtin_nanf("");
            B.at(RF_C, p) = ok ? Ls * inv : 0.0f;
            B.at(RF_R, p) = ok ? rhs * inv : 0.0f;
            B.at(RF_LO, p) = lo;
            B.at(RF_HI, p) = hi;
            B.at(RF_X, p) = pold;
        }
        const unsigned long long bm = __ballot(s0);
        if (lane == 0 && k * NT + wave * 64 < ml) msk[((k * NT) >> 6) + wave] = bm;
        if (s0) { sm |= 1u << k; any_star = true; }
    }
    any_star = __syncthreads_or(any_star);

    // phase 2: unit membership; units starting here get their chain ramp
    unsigned inunit = 0, ustart = 0;
    int uL[K];
    Ramp um[K];
#pragma unroll
    for (int k = 0; k < K; k++) { uL[k] = 0; um[k] = ramp_id(); }
    if (any_star) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            if (p >= ml) continue;
            if ((sm >> k) & 1) {
                inunit |= 1u << k;
                int ps, L;
                unit_of(msk, nw, ml, p, ps, L);
                if (ps == p) {
                    ustart |= 1u << k;
                    uL[k] = L;
                    RunRegs R;
                    run_load(B, p, L, ml, R);
                    um[k] = unit_ramp(R, B.at(RF_X, p + L - 1));
                }
            } else if (p >= 1 && mask_bit(msk, p - 1) && (p < 2 || !mask_bit(msk, p - 2))) {
                inunit |= 1u << k;         // the cell after a single starred cell
            }
        }
    }

    // phase 3: scan round by round in visit order; carry = value leaving the round
    float carry = 0.0f;
    float xin[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int p = k * NT + t;
        xin[k] = 0.0f;
        Ramp u = ramp_id();
        if (p < ml) {
            if (!((inunit >> k) & 1)) u = Ramp{pa[k], pb[k], plo[k], phv[k]};
            else if ((ustart >> k) & 1) u = um[k];
        }
        Ramp tot;
        const Ramp ex = block_scan_excl<NT>(u, wtot, tot);
        const float x = ramp_eval(ex, carry);
        if (p < ml) {
            if ((ustart >> k) & 1) xin[k] = x;
            if (!((inunit >> k) & 1)) val[k] = ramp_eval(u, x);
        }
        carry = ramp_eval(tot, carry);
    }

    // phase 4: units at their actual entering value
    if (any_star) {
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!((ustart >> k) & 1)) continue;
            const int p = k * NT + t;
            RunRegs R;
            run_load(B, p, uL[k], ml, R);
            float y[RUN_MAX];
            if (!run_vi_regs(R, xin[k], 0, y)) {
#pragma unroll
                for (int c = 0; c < RUN_MAX; c++) y[c] = c < uL[k] ? B.at(RF_X, p + c) : 0.0f;
            }
#pragma unroll
            for (int c = 0; c < RUN_MAX; c++)
                if (c < uL[k]) B.at(RF_Y, p + c) = y[c];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            if (p < ml && ((inunit >> k) & 1)) val[k] = B.at(RF_Y, p);
        }
    }
    if (write) {
        if (A.tout) {
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int p = k * NT + t;
                if (p < ml) A.tout[(long long)cell(p) * A.tpitch + r] = val[k];
            }
        } else {
            float *orow = A.phi_new + ro;
#pragma unroll
            for (int k = 0; k < K; k++) {
                const int p = k * NT + t;
                if (p < ml) orow[cell(p)] = val[k];
            }
        }
    }
    __syncthreads();
}

// One band of four lines (one per class r mod 4) of a directional sweep,
// processed in the class order 0,1,2,3 (forward) or 3,2,1,0 (reverse); the
// neighbouring band's first-processed line is recomputed (not written) where
// a line of this band needs it fresh.
template <int NT, int K, bool REV>
__device__ __forceinline__ void sweep_band(const LineArgs &A, int b, const RunBuf &B, uint64_t *msk, Ramp *wtot)
{
    // Five line steps (the band's four lines plus the recomputed one), one call
    // site.  Forward order: r0, r0+1, r0+2, [r0+4 recomputed], r0+3.
    // Reverse order: r0+3, r0+2, r0+1, [r0-1 recomputed], r0.
    float prev[K], red[K], cur[K];
#pragma unroll
    for (int k = 0; k < K; k++) { prev[k] = 0.0f; red[k] = 0.0f; cur[k] = 0.0f; }
    const int nl = A.nl;
    const int r0 = 4 * b;
    bool have_prev = false;      // prev holds the previously processed own line
#pragma nounroll
    for (int st = 0; st < 5; st++) {
        int r;
        bool redundant = (st == 3);
        if (!REV) r = (st < 3) ? r0 + st : (st == 3 ? r0 + 4 : r0 + 3);
        else r = (st < 3) ? r0 + 3 - st : (st == 3 ? r0 - 1 : r0);
        if (r < 0 || r >= nl) continue;
        bool up_fresh, dn_fresh;
        if (redundant) { up_fresh = false; dn_fresh = false; }
        else if (st < 3) { up_fresh = have_prev; dn_fresh = false; }
        else {
            // the last own line: upstream = the line processed just before it,
            // downstream = the recomputed neighbour line (if it exists)
            up_fresh = have_prev;
            int rn = REV ? r0 - 1 : r0 + 4;
            dn_fresh = rn >= 0 && rn < nl;
        }
        sweep_line<NT, K, REV>(A, r, B, msk, !redundant, prev, up_fresh, red, dn_fresh, cur, wtot);
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (redundant) red[k] = cur[k];
            else prev[k] = cur[k];
        }
        if (!redundant) have_prev = true;
    }
}

// dynamic LDS: [starred masks, 8 B per 64 cells][RF_COUNT * ml floats unit rows
// when ml <= RB_LDS_MAX, else a global scratch plane per band]
__host__ __device__ inline int sweep_mask_words(int ml) { return (ml + 63) / 64; }
__host__ __device__ inline size_t sweep_lds_bytes(int ml)
{
    size_t mb = (size_t)sweep_mask_words(ml) * 8;
    return ml <= RB_LDS_MAX ? mb + (size_t)RF_COUNT * ml * sizeof(float) : mb;
}

template <int NT, int K, bool REV>
__global__ void __launch_bounds__(NT) k_sweep(LineArgs A)
{
    extern __shared__ uint64_t smem64[];
    __shared__ Ramp wtot[NT / 64 > 0 ? NT / 64 : 1];
    uint64_t *msk = smem64;
    RunBuf B;
    B.fs = A.ml;
    if (A.ml <= RB_LDS_MAX) B.p = reinterpret_cast<float *>(smem64 + sweep_mask_words(A.ml));
    else B.p = A.scr + (long long)blockIdx.x * RF_COUNT * A.ml;
    sweep_band<NT, K, REV>(A, blockIdx.x, B, msk, wtot);
}
