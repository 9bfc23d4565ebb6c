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
    return wf / sqrtf(dn * dn + dt * dt + e2);
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
    float *scr;                         // run scratch
    const double *area;                 // Rada-Chen area term (null: 0)
    long long scr_field;                // elements per scratch field (>= nl*ml)
    int pitch, lpitch, nl, ml;
    float kap, e2, M, eps;
    int bit, scaled;
};

// Run buffer: per-cell fields of the starred runs of the line being swept.
// For lines up to RB_LDS_MAX cells it lives in LDS (field stride = line
// length); longer lines use a global scratch plane (stride = scr_field).
enum {
    SF_A = 0, SF_C, SF_R, SF_LO, SF_HI, SF_Y, SF_PU, SF_Q, SF_HELD, SF_MA, SF_MB, SF_MLO, SF_MHI, SF_XIN,
    SF_COUNT
};
#define RB_LDS_MAX 1024
// A held run cell is released only when its residual points inward by more
// than FP32 rounding, so that the hold / release iteration cannot alternate on
// a cell whose free value equals its bound.
#define RUN_TOL 1e-6f

struct RunBuf {
    float *p;
    long long fs;      // elements between fields
    long long base;    // offset of cell 0 of the line
    __device__ __forceinline__ float &at(int f, int q) const { return p[(long long)f * fs + base + q]; }
};

// Thomas elimination of one chain of free cells k = s..e of a run, in the
// normalised rows  a_k y_{k-1} - y_k + c_k y_{k+1} = r_k.  yl is the value
// left of the chain (its coefficient a_s) and yr the value right of it (its
// coefficient c_e).  Cells are at q0 + k*step.  Returns false on a
// non-positive pivot.
__device__ __noinline__ bool run_chain_solve(RunBuf B, int q0, int step, int s, int e, float yl, float yr)
{
    float pu = 0.0f, q = 0.0f;
    for (int k = s; k <= e; k++) {
        int id = q0 + k * step;
        float a = B.at(SF_A, id), c = B.at(SF_C, id), r = B.at(SF_R, id);
        float pprev = (k == s) ? yl : pu;
        float qprev = (k == s) ? 0.0f : q;
        float den = 1.0f - a * qprev;
        if (!(den > 0.0f)) return false;
        float inv = 1.0f / den;
        pu = (a * pprev - r) * inv;
        q = (k == e) ? 0.0f : c * inv;
        if (k == e) pu = pu + c * inv * yr;
        B.at(SF_PU, id) = pu;
        B.at(SF_Q, id) = q;
    }
    float y = 0.0f;
    for (int k = e; k >= s; k--) {
        int id = q0 + k * step;
        y = (k == e) ? B.at(SF_PU, id) : fmaf(B.at(SF_Q, id), y, B.at(SF_PU, id));
        B.at(SF_Y, id) = y;
    }
    return true;
}

// Box-constrained solve of a run (cells k = 0..L-1 along the visit order):
// the variational inequality y in [lo, hi], y_k at a bound only where the
// row residual pushes outward.  Active-set iteration: free cells are solved
// exactly with held cells as boundary values; free cells outside the box are
// held, held cells whose residual turned inward are released; until stable
// (at most 2 L + 4 passes).
// pin = -1 / +1 pins cell 0 at its lower / upper bound for good (the limit of
// an incoming value -> -inf / +inf); pin = 0 uses the incoming value x.
// Result in SF_Y; returns false on a zero pivot or an S == 0 cell.
__device__ __noinline__ bool run_vi_solve(RunBuf B, int q0, int step, int L, float x, float sig, int pin)
{
    for (int k = 0; k < L; k++) {
        int id = q0 + k * step;
        if (isnan(B.at(SF_A, id))) return false;
        B.at(SF_HELD, id) = (k == 0) ? (float)pin : 0.0f;
    }
    for (int it = 0; it < 2 * L + 4; it++) {
        int k = 0;
        while (k < L) {
            int id = q0 + k * step;
            float hk = B.at(SF_HELD, id);
            if (hk != 0.0f) {
                B.at(SF_Y, id) = hk > 0.0f ? B.at(SF_HI, id) : B.at(SF_LO, id);
                k++;
                continue;
            }
            int e = k;
            while (e + 1 < L && B.at(SF_HELD, q0 + (e + 1) * step) == 0.0f) e++;
            float yl = (k == 0) ? x : B.at(SF_Y, q0 + (k - 1) * step);
            float yr;
            if (e == L - 1) yr = sig;
            else {
                int idn = q0 + (e + 1) * step;
                yr = B.at(SF_HELD, idn) > 0.0f ? B.at(SF_HI, idn) : B.at(SF_LO, idn);
            }
            if (!run_chain_solve(B, q0, step, k, e, yl, yr)) return false;
            k = e + 1;
        }
        bool changed = false;
        for (int t = 0; t < L; t++) {
            int id = q0 + t * step;
            float y = B.at(SF_Y, id);
            float h = B.at(SF_HELD, id);
            if (h == 0.0f) {
                if (y > B.at(SF_HI, id)) { B.at(SF_HELD, id) = 1.0f; changed = true; }
                else if (y < B.at(SF_LO, id)) { B.at(SF_HELD, id) = -1.0f; changed = true; }
            } else if (!(t == 0 && pin != 0)) {
                float yp = (t == 0) ? x : B.at(SF_Y, q0 + (t - 1) * step);
                float yn = (t == L - 1) ? sig : B.at(SF_Y, q0 + (t + 1) * step);
                float v = B.at(SF_A, id) * yp + B.at(SF_C, id) * yn - B.at(SF_R, id) - y;
                float tau = RUN_TOL * (fabsf(B.at(SF_A, id) * yp) + fabsf(B.at(SF_C, id) * yn) +
                                       fabsf(B.at(SF_R, id)) + fabsf(y));
                if ((h > 0.0f && v < -tau) || (h < 0.0f && v > tau)) {
                    B.at(SF_HELD, id) = 0.0f;
                    changed = true;
                }
            }
        }
        if (!changed) break;
    }
    for (int k = 0; k < L; k++) {
        int id = q0 + k * step;
        B.at(SF_Y, id) = mg_clip(B.at(SF_Y, id), B.at(SF_LO, id), B.at(SF_HI, id));
    }
    return true;
}

// Unconstrained affine solution y_k = u_k + v_k x of a run (all cells
// free): (v_L, u_L) of the last cell.
__device__ __noinline__ bool run_affine_last(RunBuf B, int q0, int step, int L, float sig, float *uL, float *vL)
{
    float pu = 0.0f, pv = 0.0f, q = 0.0f;
    for (int k = 0; k < L; k++) {
        int id = q0 + k * step;
        float a = B.at(SF_A, id), c = B.at(SF_C, id), r = B.at(SF_R, id);
        if (isnan(a)) return false;
        float den = (k == 0) ? 1.0f : 1.0f - a * q;
        if (!(den > 0.0f)) return false;
        float inv = 1.0f / den;
        float npu = (k == 0) ? -r * inv : (a * pu - r) * inv;
        float npv = (k == 0) ? a * inv : a * pv * inv;
        pu = npu; pv = npv;
        if (k == L - 1) { pu = pu + c * inv * sig; q = 0.0f; }
        else q = c * inv;
    }
    *uL = pu;
    *vL = pv;
    return true;
}

// --------------------------------------------------------------------------
// Register-resident run solves for short runs (L <= RUN_REG).  A held cell
// becomes the identity row y_k = bound, so a single Thomas pass over the run
// solves every chain of free cells with the held cells as known values.
#define RUN_REG 4

struct RunRegs {
    float a[RUN_REG], c[RUN_REG], r[RUN_REG], lo[RUN_REG], hi[RUN_REG];
    float sig;
    int L;
    bool ok;
};

__device__ __forceinline__ void run_load(const RunBuf &B, int p, int L, RunRegs &R)
{
    R.L = L;
    R.ok = true;
#pragma unroll
    for (int k = 0; k < RUN_REG; k++) {
        if (k < L) {
            R.a[k] = B.at(SF_A, p + k); R.c[k] = B.at(SF_C, p + k); R.r[k] = B.at(SF_R, p + k);
            R.lo[k] = B.at(SF_LO, p + k); R.hi[k] = B.at(SF_HI, p + k);
            if (isnan(R.a[k])) R.ok = false;
        } else {
            R.a[k] = 0.0f; R.c[k] = 0.0f; R.r[k] = 0.0f; R.lo[k] = 0.0f; R.hi[k] = 0.0f;
        }
    }
    R.sig = B.at(SF_MB, p + L - 1);
}

// Thomas pass with held rows as identity rows; held[k] in {-1, 0, +1}
__device__ __forceinline__ bool run_thomas_regs(const RunRegs &R, const int (&held)[RUN_REG], float x,
                                                float (&y)[RUN_REG])
{
    float pu[RUN_REG], qq[RUN_REG];
    float pprev = x, qprev = 0.0f;
#pragma unroll
    for (int k = 0; k < RUN_REG; k++) {
        if (k >= R.L) { pu[k] = 0.0f; qq[k] = 0.0f; continue; }
        if (held[k] != 0) {
            pu[k] = held[k] > 0 ? R.hi[k] : R.lo[k];
            qq[k] = 0.0f;
        } else {
            const float a = R.a[k];
            const float den = (k == 0) ? 1.0f : 1.0f - a * qprev;
            if (!(den > 0.0f)) return false;
            const float inv = 1.0f / den;
            pu[k] = (a * pprev - R.r[k]) * inv;
            if (k == R.L - 1) { pu[k] = pu[k] + R.c[k] * inv * R.sig; qq[k] = 0.0f; }
            else qq[k] = R.c[k] * inv;
        }
        pprev = pu[k]; qprev = qq[k];
    }
    float yn = 0.0f;
#pragma unroll
    for (int kk = RUN_REG - 1; kk >= 0; kk--) {
        if (kk >= R.L) { y[kk] = 0.0f; continue; }
        yn = (kk == R.L - 1) ? pu[kk] : fmaf(qq[kk], yn, pu[kk]);
        y[kk] = yn;
    }
    return true;
}

// the box-constrained run problem (see run_vi_solve) in registers
__device__ __forceinline__ bool run_vi_regs(const RunRegs &R, float x, int pin, float (&y)[RUN_REG])
{
    if (!R.ok) return false;
    int held[RUN_REG];
#pragma unroll
    for (int k = 0; k < RUN_REG; k++) held[k] = (k == 0) ? pin : 0;
    for (int it = 0; it < 2 * R.L + 4; it++) {
        if (!run_thomas_regs(R, held, x, y)) return false;
        bool changed = false;
#pragma unroll
        for (int k = 0; k < RUN_REG; k++) {
            if (k >= R.L) continue;
            if (held[k] == 0) {
                if (y[k] > R.hi[k]) { held[k] = 1; changed = true; }
                else if (y[k] < R.lo[k]) { held[k] = -1; changed = true; }
            } else if (!(k == 0 && pin != 0)) {
                const float yp = (k == 0) ? x : y[k > 0 ? k - 1 : 0];
                const float yn = (k == R.L - 1) ? R.sig : y[k + 1 < RUN_REG ? k + 1 : k];
                const float v = R.a[k] * yp + R.c[k] * yn - R.r[k] - y[k];
                const float tau = RUN_TOL * (fabsf(R.a[k] * yp) + fabsf(R.c[k] * yn) + fabsf(R.r[k]) + fabsf(y[k]));
                if ((held[k] > 0 && v < -tau) || (held[k] < 0 && v > tau)) { held[k] = 0; changed = true; }
            }
        }
        if (!changed) break;
    }
#pragma unroll
    for (int k = 0; k < RUN_REG; k++)
        if (k < R.L) y[k] = mg_clip(y[k], R.lo[k], R.hi[k]);
    return true;
}

// unconstrained affine solution of the last cell: y_L = u_L + v_L x
__device__ __forceinline__ bool run_affine_regs(const RunRegs &R, float &uL, float &vL)
{
    if (!R.ok) return false;
    float pu = 0.0f, pv = 0.0f, q = 0.0f;
#pragma unroll
    for (int k = 0; k < RUN_REG; k++) {
        if (k >= R.L) continue;
        const float a = R.a[k];
        const float den = (k == 0) ? 1.0f : 1.0f - a * q;
        if (!(den > 0.0f)) return false;
        const float inv = 1.0f / den;
        const float npu = (k == 0) ? -R.r[k] * inv : (a * pu - R.r[k]) * inv;
        const float npv = (k == 0) ? a * inv : a * pv * inv;
        pu = npu; pv = npv;
        if (k == R.L - 1) { pu = pu + R.c[k] * inv * R.sig; q = 0.0f; }
        else q = R.c[k] * inv;
    }
    uL = pu; vL = pv;
    return true;
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
// thread's cells.  Run buffers are indexed by visit position.
template <int NT, int K, bool REV>
__device__ __forceinline__ void sweep_line(const LineArgs &A, int r, const RunBuf &B, bool write,
                                           const float (&upv)[K], bool up_fresh, const float (&dnv)[K],
                                           bool dn_fresh, float (&val)[K], Ramp *wtot, uint8_t *sst)
{
    const int t = threadIdx.x;
    const int nl = A.nl, ml = A.ml, P = A.pitch;
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

    float pa[K], pb[K], plo[K], phv[K];
    unsigned inrun = 0, runlast = 0, runstart = 0;
    auto cell = [&](int p) { return REV ? ml - 1 - p : p; };
    auto starred = [&](int p) -> bool {
        return (p >= 0 && p < ml) ? ((lrow[cell(p)] >> A.bit) & 1) != 0 : false;
    };

    bool any_run = false;
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int p = k * NT + t;
        pa[k] = 0.0f; pb[k] = 0.0f; plo[k] = 0.0f; phv[k] = 0.0f;
        if (p >= ml) continue;
        const int q = cell(p);
        // run structure in visit order
        const bool s0 = starred(p), sp = starred(p - 1), sn = starred(p + 1), spp = starred(p - 2);
        const bool has_prev = p > 0, has_next = p + 1 < ml;
        const bool start = s0 && !sp;
        const bool single = start && !sn;
        const bool ext = !s0 && has_prev && sp && !spp;
        const bool last = ext || (s0 && !sn && !(single && has_next));
        if (s0 || ext) inrun |= 1u << k;
        if ((s0 || ext) && last) runlast |= 1u << k;
        if (start) runstart |= 1u << k;

        // frozen coefficients at psi (eq. abcdrc)
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
        if (S > 0.0f) {
            const float inv = 1.0f / S;
            pa[k] = Lp * inv;
            pb[k] = (Ls * sig - rhs) * inv;
            plo[k] = lo;
            phv[k] = hi;
        } else {                          // S == 0: the cell keeps its value
            pa[k] = 0.0f; pb[k] = pold; plo[k] = pold; phv[k] = pold;
        }
        if (s0 || ext) {
            const bool ok = S > 0.0f;
            B.at(SF_A, p) = ok ? Lp / S : __builtin_nanf("");
            B.at(SF_C, p) = ok ? Ls / S : 0.0f;
            B.at(SF_R, p) = ok ? rhs / S : 0.0f;
            B.at(SF_LO, p) = lo;
            B.at(SF_HI, p) = hi;
            B.at(SF_Y, p) = pold;
            B.at(SF_MB, p) = sig;       // successor value (used at the run's last cell)
            B.at(SF_XIN, p) = pold;     // old value (a degenerate run keeps it)
            any_run = true;
        }
        sst[p] = s0 ? 1 : 0;
    }
    any_run = __syncthreads_or(any_run);

    if (any_run) {
        // runs owned by this thread: chain map of the run's last cell
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!((runstart >> k) & 1)) continue;
            const int p = k * NT + t;
            int L = 1;
            if (p + 1 < ml && sst[p + 1]) {
                int pp = p + 1;
                while (pp < ml && sst[pp]) { L++; pp++; }
            } else if (p + 1 < ml) {
                L = 2;
            }
            const int pl = p + L - 1;
            const float sig = B.at(SF_MB, pl);
            float uL = 0.0f, vL = 0.0f, ylo = 0.0f, yhi = 0.0f;
            bool ok;
            if (L <= RUN_REG) {
                RunRegs R;
                run_load(B, p, L, R);
                float y[RUN_REG];
                ok = run_affine_regs(R, uL, vL);
                if (ok) {
                    if (R.a[0] > 0.0f) {
                        ok = run_vi_regs(R, 0.0f, -1, y);
                        ylo = y[0];
#pragma unroll
                        for (int c = 0; c < RUN_REG; c++) if (c == L - 1) ylo = y[c];
                        ok = ok && run_vi_regs(R, 0.0f, +1, y);
                        yhi = y[0];
#pragma unroll
                        for (int c = 0; c < RUN_REG; c++) if (c == L - 1) yhi = y[c];
                    } else {
                        ok = run_vi_regs(R, 0.0f, 0, y);
                        ylo = y[0];
#pragma unroll
                        for (int c = 0; c < RUN_REG; c++) if (c == L - 1) ylo = y[c];
                        yhi = ylo;
                        vL = 0.0f; uL = ylo;
                    }
                }
            } else {
                ok = run_affine_last(B, p, 1, L, sig, &uL, &vL);
                if (ok) {
                    if (B.at(SF_A, p) > 0.0f) {
                        ok = run_vi_solve(B, p, 1, L, 0.0f, sig, -1);
                        ylo = B.at(SF_Y, pl);
                        ok = ok && run_vi_solve(B, p, 1, L, 0.0f, sig, +1);
                        yhi = B.at(SF_Y, pl);
                    } else {
                        ok = run_vi_solve(B, p, 1, L, 0.0f, sig, 0);
                        ylo = yhi = B.at(SF_Y, pl);
                        vL = 0.0f; uL = ylo;
                    }
                }
            }
            if (!ok) {        // degenerate run: every cell keeps its value
                const float yold = B.at(SF_XIN, pl);
                vL = 0.0f; uL = yold; ylo = yold; yhi = yold;
            }
            B.at(SF_HELD, p) = ok ? 0.0f : 2.0f;
            B.at(SF_MA, pl) = vL;
            B.at(SF_MLO, pl) = fminf(ylo, yhi);
            B.at(SF_MHI, pl) = fmaxf(ylo, yhi);
            B.at(SF_PU, pl) = uL;            // b of the chain map
            B.at(SF_Q, p) = (float)L;        // run length at the start cell
        }
        __syncthreads();
    }

    // scan round by round in visit order; carry = value leaving the round
    float carry = 0.0f;
    float xin[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const int p = k * NT + t;
        xin[k] = 0.0f;
        Ramp u = ramp_id();
        if (p < ml) {
            if (!((inrun >> k) & 1)) u = Ramp{pa[k], pb[k], plo[k], phv[k]};
            else if ((runlast >> k) & 1) u = Ramp{B.at(SF_MA, p), B.at(SF_PU, p), B.at(SF_MLO, p), B.at(SF_MHI, p)};
        }
        Ramp tot;
        const Ramp ex = block_scan_excl<NT>(u, wtot, tot);
        const float x = ramp_eval(ex, carry);
        if (p < ml) {
            if ((runstart >> k) & 1) xin[k] = x;
            if (!((inrun >> k) & 1) || ((runlast >> k) & 1)) val[k] = ramp_eval(u, x);
        }
        carry = ramp_eval(tot, carry);
    }

    if (any_run) {
        // run owners: the run at its actual incoming value
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (!((runstart >> k) & 1)) continue;
            const int p = k * NT + t;
            const int L = (int)B.at(SF_Q, p);
            const int pl = p + L - 1;
            bool ok = B.at(SF_HELD, p) == 0.0f;
            if (ok) {
                if (L <= RUN_REG) {
                    RunRegs R;
                    run_load(B, p, L, R);
                    float y[RUN_REG];
                    ok = run_vi_regs(R, xin[k], 0, y);
#pragma unroll
                    for (int c = 0; c < RUN_REG; c++)
                        if (ok && c < L) B.at(SF_Y, p + c) = y[c];
                } else {
                    ok = run_vi_solve(B, p, 1, L, xin[k], B.at(SF_MB, pl), 0);
                }
            }
            if (!ok) {
                for (int c = 0; c < L; c++) B.at(SF_Y, p + c) = B.at(SF_XIN, p + c);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            if (p < ml && ((inrun >> k) & 1) && !((runlast >> k) & 1)) val[k] = B.at(SF_Y, p);
        }
    }
    if (write) {
        float *orow = A.phi_new + ro;
#pragma unroll
        for (int k = 0; k < K; k++) {
            const int p = k * NT + t;
            if (p < ml) orow[cell(p)] = val[k];
        }
    }
    __syncthreads();
}

// One band of four lines (one per class r mod 4) of a directional sweep,
// processed in the class order 0,1,2,3 (forward) or 3,2,1,0 (reverse); the
// neighbouring band's first-processed line is recomputed (not written) where
// a line of this band needs it fresh.  B0 / B1: run buffers for the band's
// own lines and for the recomputed line.
template <int NT, int K, bool REV>
__device__ __forceinline__ void sweep_band(const LineArgs &A, int b, const RunBuf &B0, const RunBuf &B1,
                                           Ramp *wtot, uint8_t *sst, bool lds_runs)
{
    // Five line steps (the band's four lines plus the recomputed one), one call
    // site.  Forward order: r0, r0+1, r0+2, [r0+4 recomputed], r0+3.
    // Reverse order: r0+3, r0+2, r0+1, [r0-1 recomputed], r0.
    float prev[K], red[K], cur[K];
#pragma unroll
    for (int k = 0; k < K; k++) { prev[k] = 0.0f; red[k] = 0.0f; cur[k] = 0.0f; }
    const int nl = A.nl, ml = A.ml;
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
        RunBuf Bx = redundant ? B1 : B0;
        if (!lds_runs) Bx.base = (long long)r * ml;
        sweep_line<NT, K, REV>(A, r, Bx, !redundant, prev, up_fresh, red, dn_fresh, cur, wtot, sst);
#pragma unroll
        for (int k = 0; k < K; k++) {
            if (redundant) red[k] = cur[k];
            else prev[k] = cur[k];
        }
        if (!redundant) have_prev = true;
    }
}

// dynamic LDS: [SF_COUNT * ml floats run buffer][ml bytes starred flags]
template <int NT, int K, bool REV>
__global__ void __launch_bounds__(NT) k_sweep(LineArgs A)
{
    extern __shared__ float smem[];
    __shared__ Ramp wtot[NT / 64 > 0 ? NT / 64 : 1];
    const bool lds_runs = A.ml <= RB_LDS_MAX;
    RunBuf B0, B1;
    uint8_t *sst;
    if (lds_runs) {
        B0.p = smem; B0.fs = A.ml; B0.base = 0;
        B1 = B0;
        sst = reinterpret_cast<uint8_t *>(smem + (long long)SF_COUNT * A.ml);
    } else {
        B0.p = A.scr; B0.fs = A.scr_field; B0.base = 0;
        B1.p = A.scr + (long long)SF_COUNT * A.scr_field; B1.fs = A.scr_field; B1.base = 0;
        sst = reinterpret_cast<uint8_t *>(smem);
    }
    sweep_band<NT, K, REV>(A, blockIdx.x, B0, B1, wtot, sst, lds_runs);
}

// LDS bytes of one k_sweep launch
__host__ __device__ inline size_t sweep_lds_bytes(int ml)
{
    return ml <= RB_LDS_MAX ? (size_t)SF_COUNT * ml * sizeof(float) + (size_t)ml : (size_t)ml;
}
