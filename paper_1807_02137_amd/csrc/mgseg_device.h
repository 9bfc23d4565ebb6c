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

// scratch fields (per cell, in the cell's line-layout index r*ml + q)
enum {
    SF_A = 0, SF_C, SF_R, SF_LO, SF_HI, SF_SIG, SF_MA, SF_MB, SF_MLO, SF_MHI,
    SF_XIN, SF_Y, SF_HELD, SF_PU, SF_PV, SF_Q, SF_COUNT
};

__device__ __forceinline__ float &scr_at(const LineArgs &A, int plane, int f, long long idx)
{
    return A.scr[((long long)plane * SF_COUNT + f) * A.scr_field + idx];
}

// Thomas elimination of one chain of free cells k = s..e of a run, in the
// normalised rows  a_k y_{k-1} - y_k + c_k y_{k+1} = r_k.  yl is the value
// left of the chain (its coefficient a_s) and yr the value right of it (its
// coefficient c_e).  Returns false on a non-positive pivot.
__device__ bool run_chain_solve(const LineArgs &A, int plane, long long base, int step, int s, int e,
                                float yl, float yr)
{
    float pu = 0.0f, q = 0.0f;
    for (int k = s; k <= e; k++) {
        long long id = base + (long long)k * step;
        float a = scr_at(A, plane, SF_A, id), c = scr_at(A, plane, SF_C, id), r = scr_at(A, plane, SF_R, id);
        float pprev = (k == s) ? yl : pu;
        float qprev = (k == s) ? 0.0f : q;
        float den = 1.0f - a * qprev;
        if (!(den > 0.0f)) return false;
        float inv = 1.0f / den;
        pu = (a * pprev - r) * inv;
        q = (k == e) ? 0.0f : c * inv;
        if (k == e) pu = pu + c * inv * yr;
        scr_at(A, plane, SF_PU, id) = pu;
        scr_at(A, plane, SF_Q, id) = q;
    }
    float y = 0.0f;
    for (int k = e; k >= s; k--) {
        long long id = base + (long long)k * step;
        y = (k == e) ? scr_at(A, plane, SF_PU, id)
                     : fmaf(scr_at(A, plane, SF_Q, id), y, scr_at(A, plane, SF_PU, id));
        scr_at(A, plane, SF_Y, id) = y;
    }
    return true;
}

// Box-constrained solve of a run (cells k = 0..L-1 along the visit order,
// scratch index base + k*step): the variational inequality
//   y in [lo, hi],  y_k = lo_k or hi_k only where the row residual pushes
//   outward.  Active-set iteration: free cells are solved exactly with held
//   cells as boundary values; free cells outside the box are held, held
//   cells whose residual turned inward are released; until stable.
// pin = -1 / +1 pins cell 0 at its lower / upper bound for good (the limit of
// an incoming value -> -inf / +inf); pin = 0 uses the incoming value x.
// Result in SF_Y; returns false on a zero pivot or an S == 0 cell.
__device__ bool run_vi_solve(const LineArgs &A, int plane, long long base, int step, int L, float x,
                             float sig, int pin)
{
    for (int k = 0; k < L; k++) {
        long long id = base + (long long)k * step;
        if (isnan(scr_at(A, plane, SF_A, id))) return false;
        scr_at(A, plane, SF_HELD, id) = (k == 0) ? (float)pin : 0.0f;
    }
    for (int it = 0; it < 4 * L + 8; it++) {
        // solve every chain of free cells
        int k = 0;
        while (k < L) {
            long long id = base + (long long)k * step;
            float hk = scr_at(A, plane, SF_HELD, id);
            if (hk != 0.0f) {
                scr_at(A, plane, SF_Y, id) = hk > 0.0f ? scr_at(A, plane, SF_HI, id) : scr_at(A, plane, SF_LO, id);
                k++;
                continue;
            }
            int e = k;
            while (e + 1 < L && scr_at(A, plane, SF_HELD, base + (long long)(e + 1) * step) == 0.0f) e++;
            float yl = (k == 0) ? x : scr_at(A, plane, SF_Y, base + (long long)(k - 1) * step);
            float yr;
            if (e == L - 1) yr = sig;
            else {
                long long idn = base + (long long)(e + 1) * step;
                yr = scr_at(A, plane, SF_HELD, idn) > 0.0f ? scr_at(A, plane, SF_HI, idn) : scr_at(A, plane, SF_LO, idn);
            }
            if (!run_chain_solve(A, plane, base, step, k, e, yl, yr)) return false;
            k = e + 1;
        }
        bool changed = false;
        for (int t = 0; t < L; t++) {
            long long id = base + (long long)t * step;
            float y = scr_at(A, plane, SF_Y, id);
            float lo = scr_at(A, plane, SF_LO, id), hi = scr_at(A, plane, SF_HI, id);
            float h = scr_at(A, plane, SF_HELD, id);
            if (h == 0.0f) {
                if (y > hi) { scr_at(A, plane, SF_HELD, id) = 1.0f; changed = true; }
                else if (y < lo) { scr_at(A, plane, SF_HELD, id) = -1.0f; changed = true; }
            } else if (!(t == 0 && pin != 0)) {
                float yp = (t == 0) ? x : scr_at(A, plane, SF_Y, base + (long long)(t - 1) * step);
                float yn = (t == L - 1) ? sig : scr_at(A, plane, SF_Y, base + (long long)(t + 1) * step);
                float v = scr_at(A, plane, SF_A, id) * yp + scr_at(A, plane, SF_C, id) * yn
                        - scr_at(A, plane, SF_R, id) - y;
                if ((h > 0.0f && v < 0.0f) || (h < 0.0f && v > 0.0f)) {
                    scr_at(A, plane, SF_HELD, id) = 0.0f;
                    changed = true;
                }
            }
        }
        if (!changed) break;
    }
    for (int k = 0; k < L; k++) {
        long long id = base + (long long)k * step;
        scr_at(A, plane, SF_Y, id) = mg_clip(scr_at(A, plane, SF_Y, id), scr_at(A, plane, SF_LO, id),
                                             scr_at(A, plane, SF_HI, id));
    }
    return true;
}

// Unconstrained affine solution y_k = u_k + v_k x of a run (all cells free):
// returns (v_L, u_L) of the last cell.
__device__ bool run_affine_last(const LineArgs &A, int plane, long long base, int step, int L, float sig,
                                float *uL, float *vL)
{
    float pu = 0.0f, pv = 0.0f, q = 0.0f;
    for (int k = 0; k < L; k++) {
        long long id = base + (long long)k * step;
        float a = scr_at(A, plane, SF_A, id), c = scr_at(A, plane, SF_C, id), r = scr_at(A, plane, SF_R, id);
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
// Block-wide exclusive scan of ramps in the order ord (0..NT-1).
template <int NT>
__device__ Ramp block_scan_excl(Ramp mine, int ord, Ramp *sh)
{
    sh[ord] = mine;
    __syncthreads();
    for (int off = 1; off < NT; off <<= 1) {
        Ramp cur = sh[ord];
        Ramp prev = (ord >= off) ? sh[ord - off] : ramp_id();
        __syncthreads();
        if (ord >= off) sh[ord] = ramp_comp(cur, prev);
        __syncthreads();
    }
    Ramp ex = (ord > 0) ? sh[ord - 1] : ramp_id();
    __syncthreads();
    return ex;
}

// --------------------------------------------------------------------------
// One line of one directional sweep.  Thread t owns the cells q in
// [t*K, t*K + K) of the line (memory order).  REV visits the line from
// q = ml-1 down to 0 and takes the upstream line at r+1.
//   up_fresh / dn_fresh: the cross-line neighbour values are the caller's
//   registers (freshly updated) instead of phi_old.
// On return val[] holds the new values of the thread's cells.
template <int NT, int K, bool REV>
__device__ void sweep_line(const LineArgs &A, int r, int plane, bool write,
                           const float *upv, bool up_fresh, const float *dnv, bool dn_fresh,
                           float *val, Ramp *sh)
{
    const int t = threadIdx.x;
    const int q0 = t * K;
    const int nl = A.nl, ml = A.ml, P = A.pitch;
    const int ru = REV ? r + 1 : r - 1;      // upstream line
    const int rd = REV ? r - 1 : r + 1;      // downstream line
    const int rm1 = mg_mirror(r - 1, nl), rp1 = mg_mirror(r + 1, nl);
    const float *ps0 = A.psi + (long long)r * P, *psm = A.psi + (long long)rm1 * P, *psp = A.psi + (long long)rp1 * P;
    const float *w0 = A.w + (long long)r * P, *wm = A.w + (long long)rm1 * P, *wp = A.w + (long long)rp1 * P;
    const float e2 = A.e2;
    float area = 0.0f;
    if (A.area) area = (float)(*A.area);
    const long long rbase = (long long)r * ml;

    float pa[K], pb[K], plo[K], phi_[K];
    bool inrun[K], runlast[K], runstart[K], starred[K];

    // --- run structure from the labels (visit order)
    auto st = [&](int q) -> bool {
        return (q >= 0 && q < ml) ? ((A.lab[(long long)r * A.lpitch + q] >> A.bit) & 1) != 0 : false;
    };
    auto prevq = [&](int q) { return REV ? q + 1 : q - 1; };
    auto nextq = [&](int q) { return REV ? q - 1 : q + 1; };
    auto exists = [&](int q) { return q >= 0 && q < ml; };

#pragma unroll
    for (int k = 0; k < K; k++) {
        int q = q0 + k;
        inrun[k] = runlast[k] = runstart[k] = starred[k] = false;
        pa[k] = 0.0f; pb[k] = 0.0f; plo[k] = 0.0f; phi_[k] = 0.0f;
        if (q >= ml) continue;
        bool s0 = st(q), sp = st(prevq(q)), sn = st(nextq(q)), spp = st(prevq(prevq(q)));
        bool start = s0 && !sp;
        bool single = start && !sn;
        bool ext = !s0 && exists(prevq(q)) && sp && !spp;   // prev is a singleton start
        starred[k] = s0;
        inrun[k] = s0 || ext;
        runstart[k] = start;
        runlast[k] = ext || (s0 && !sn && !(single && exists(nextq(q))));

        // --- frozen coefficients at psi (eq. abcdrc)
        int qm = mg_mirror(q - 1, ml), qp = mg_mirror(q + 1, ml);
        float p0 = ps0[q];
        float xp = 0.0f, xm = 0.0f, lp = 0.0f, lm = 0.0f;
        if (r + 1 < nl)
            xp = mg_face(p0, psp[q], ps0[qp], psp[qp], ps0[qm], psp[qm], w0[q], wp[q], e2);
        if (r > 0)
            xm = mg_face(psm[q], p0, psm[qp], ps0[qp], psm[qm], ps0[qm], wm[q], w0[q], e2);
        if (q + 1 < ml)
            lp = mg_face(p0, ps0[q + 1], psp[q], psp[q + 1], psm[q], psm[q + 1], w0[q], w0[q + 1], e2);
        if (q > 0)
            lm = mg_face(ps0[q - 1], p0, psp[q - 1], psp[q], psm[q - 1], psm[q], w0[q - 1], w0[q], e2);
        float dl = A.scaled ? 1.0f : mg_delta(p0, A.eps);
        float s = A.kap * dl;
        xp *= s; xm *= s; lp *= s; lm *= s;
        float S = xp + xm + lp + lm;
        float f = dl * (A.fit[(long long)r * P + q] + area);
        float Fv = A.F ? A.F[(long long)r * P + q] : 0.0f;
        float Xu = REV ? xp : xm, Xd = REV ? xm : xp;
        float Lp = REV ? lp : lm, Ls = REV ? lm : lp;
        float vu = 0.0f, vd = 0.0f;
        if (ru >= 0 && ru < nl) vu = up_fresh ? upv[k] : A.phi_old[(long long)ru * P + q];
        if (rd >= 0 && rd < nl) vd = dn_fresh ? dnv[k] : A.phi_old[(long long)rd * P + q];
        float rhs = f + Fv - Xu * vu - Xd * vd;
        int qs = nextq(q);
        float sig = exists(qs) ? A.phi_old[(long long)r * P + qs] : 0.0f;
        float lo = A.lo ? A.lo[(long long)r * P + q] : -A.M;
        float hi = A.hi ? A.hi[(long long)r * P + q] : A.M;
        float pold = A.phi_old[(long long)r * P + q];
        if (S > 0.0f) {
            float inv = 1.0f / S;
            pa[k] = Lp * inv;
            pb[k] = (Ls * sig - rhs) * inv;
            plo[k] = lo;
            phi_[k] = hi;
        } else {                          // S == 0: the cell keeps its value
            pa[k] = 0.0f; pb[k] = pold; plo[k] = pold; phi_[k] = pold;
        }
        if (inrun[k]) {
            long long id = rbase + q;
            bool ok = S > 0.0f;
            scr_at(A, plane, SF_A, id) = ok ? Lp / S : __builtin_nanf("");
            scr_at(A, plane, SF_C, id) = ok ? Ls / S : 0.0f;
            scr_at(A, plane, SF_R, id) = ok ? rhs / S : 0.0f;
            scr_at(A, plane, SF_LO, id) = lo;
            scr_at(A, plane, SF_HI, id) = hi;
            scr_at(A, plane, SF_SIG, id) = sig;
            scr_at(A, plane, SF_Y, id) = pold;
        }
    }
    __syncthreads();

    // --- runs owned by this thread: chain map of the run's last cell
    const int step = REV ? -1 : 1;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (!runstart[k]) continue;
        int q = q0 + k;
        // extent of the run in visit order
        int L = 1;
        bool s1 = st(nextq(q));
        if (s1) {
            int qq = nextq(q);
            while (exists(qq) && st(qq)) { L++; qq = nextq(qq); }
        } else if (exists(nextq(q))) {
            L = 2;
        }
        long long base = rbase + q;
        long long idl = base + (long long)(L - 1) * step;
        float sig = scr_at(A, plane, SF_SIG, idl);
        float uL, vL;
        bool ok = run_affine_last(A, plane, base, step, L, sig, &uL, &vL);
        float ylo, yhi;
        if (ok) {
            if (scr_at(A, plane, SF_A, base) > 0.0f) {
                ok = run_vi_solve(A, plane, base, step, L, 0.0f, sig, -1);
                ylo = scr_at(A, plane, SF_Y, idl);
                ok = ok && run_vi_solve(A, plane, base, step, L, 0.0f, sig, +1);
                yhi = scr_at(A, plane, SF_Y, idl);
            } else {
                ok = run_vi_solve(A, plane, base, step, L, 0.0f, sig, 0);
                ylo = yhi = scr_at(A, plane, SF_Y, idl);
                vL = 0.0f; uL = ylo;
            }
        }
        if (!ok) {        // degenerate run: every cell keeps its value
            float yold = A.phi_old[(long long)r * P + (q + (L - 1) * step)];
            vL = 0.0f; uL = yold; ylo = yold; yhi = yold;
            scr_at(A, plane, SF_XIN, base) = __builtin_nanf("");
        } else {
            scr_at(A, plane, SF_XIN, base) = 0.0f;
        }
        scr_at(A, plane, SF_MA, idl) = vL;
        scr_at(A, plane, SF_MB, idl) = uL;
        scr_at(A, plane, SF_MLO, idl) = fminf(ylo, yhi);
        scr_at(A, plane, SF_MHI, idl) = fmaxf(ylo, yhi);
    }
    __syncthreads();

    // --- compose this thread's cells in visit order
    Ramp mine = ramp_id();
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
        int k = REV ? K - 1 - kk : kk;
        int q = q0 + k;
        if (q >= ml) continue;
        Ramp u;
        if (!inrun[k]) u = Ramp{pa[k], pb[k], plo[k], phi_[k]};
        else if (runlast[k]) {
            long long id = rbase + q;
            u = Ramp{scr_at(A, plane, SF_MA, id), scr_at(A, plane, SF_MB, id),
                     scr_at(A, plane, SF_MLO, id), scr_at(A, plane, SF_MHI, id)};
        } else continue;
        mine = ramp_comp(u, mine);
    }
    const int ord = REV ? NT - 1 - t : t;
    Ramp ex = block_scan_excl<NT>(mine, ord, sh);
    float x = ramp_eval(ex, 0.0f);

    // --- apply: point values and the value entering every run
#pragma unroll
    for (int kk = 0; kk < K; kk++) {
        int k = REV ? K - 1 - kk : kk;
        int q = q0 + k;
        if (q >= ml) continue;
        if (!inrun[k]) {
            x = mg_clip(fmaf(pa[k], x, pb[k]), plo[k], phi_[k]);
            val[k] = x;
            continue;
        }
        long long id = rbase + q;
        if (runstart[k]) {
            float flag = scr_at(A, plane, SF_XIN, id);
            scr_at(A, plane, SF_XIN, id) = isnan(flag) ? flag : x;
        }
        if (runlast[k]) {
            x = mg_clip(fmaf(scr_at(A, plane, SF_MA, id), x, scr_at(A, plane, SF_MB, id)),
                        scr_at(A, plane, SF_MLO, id), scr_at(A, plane, SF_MHI, id));
            val[k] = x;
        }
    }
    __syncthreads();

    // --- run owners: the run at its actual incoming value
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (!runstart[k]) continue;
        int q = q0 + k;
        int L = 1;
        if (st(nextq(q))) {
            int qq = nextq(q);
            while (exists(qq) && st(qq)) { L++; qq = nextq(qq); }
        } else if (exists(nextq(q))) {
            L = 2;
        }
        long long base = rbase + q;
        float xin = scr_at(A, plane, SF_XIN, base);
        long long idl = base + (long long)(L - 1) * step;
        bool ok = !isnan(xin);
        if (ok) ok = run_vi_solve(A, plane, base, step, L, xin, scr_at(A, plane, SF_SIG, idl), 0);
        if (!ok) {
            for (int c = 0; c < L; c++) {
                long long id = base + (long long)c * step;
                scr_at(A, plane, SF_Y, id) = A.phi_old[(long long)r * P + (q + c * step)];
            }
        }
    }
    __syncthreads();

    // --- results
#pragma unroll
    for (int k = 0; k < K; k++) {
        int q = q0 + k;
        if (q >= ml) continue;
        if (inrun[k] && !runlast[k]) val[k] = scr_at(A, plane, SF_Y, rbase + q);
        if (write) A.phi_new[(long long)r * P + q] = val[k];
    }
    __syncthreads();
}

// One band of four lines (one per class r mod 4) of a directional sweep,
// processed in the class order 0,1,2,3 (forward) or 3,2,1,0 (reverse); the
// neighbouring band's first-processed line is recomputed (not written) where
// a line of this band needs it fresh.
template <int NT, int K, bool REV>
__device__ void sweep_band(const LineArgs &A, int b, Ramp *sh)
{
    float prev[K], red[K], cur[K];
#pragma unroll
    for (int k = 0; k < K; k++) { prev[k] = 0.0f; red[k] = 0.0f; cur[k] = 0.0f; }
    const int nl = A.nl;
    const int r0 = 4 * b;
    if (!REV) {
        // classes 0,1,2 in order; class 3 needs the next band's class-0 line
        for (int c = 0; c < 3; c++) {
            int r = r0 + c;
            if (r >= nl) return;
            sweep_line<NT, K, false>(A, r, 0, true, prev, c > 0, nullptr, false, cur, sh);
#pragma unroll
            for (int k = 0; k < K; k++) prev[k] = cur[k];
        }
        int r3 = r0 + 3;
        if (r3 >= nl) return;
        bool have_red = (r0 + 4 < nl);
        if (have_red) sweep_line<NT, K, false>(A, r0 + 4, 1, false, nullptr, false, nullptr, false, red, sh);
        sweep_line<NT, K, false>(A, r3, 0, true, prev, true, red, have_red, cur, sh);
    } else {
        // classes 3,2,1 in order; class 0 needs the previous band's class-3 line
        bool first = true;
        for (int c = 3; c >= 1; c--) {
            int r = r0 + c;
            if (r >= nl) continue;
            sweep_line<NT, K, true>(A, r, 0, true, prev, !first, nullptr, false, cur, sh);
            first = false;
#pragma unroll
            for (int k = 0; k < K; k++) prev[k] = cur[k];
        }
        bool have_red = (r0 - 1 >= 0);
        if (have_red) sweep_line<NT, K, true>(A, r0 - 1, 1, false, nullptr, false, nullptr, false, red, sh);
        bool up_fresh = (r0 + 1 < nl);
        sweep_line<NT, K, true>(A, r0, 0, true, prev, up_fresh, red, have_red, cur, sh);
    }
}

template <int NT, int K, bool REV>
__global__ void __launch_bounds__(NT) k_sweep(LineArgs A)
{
    __shared__ Ramp sh[NT];
    sweep_band<NT, K, REV>(A, blockIdx.x, sh);
}
