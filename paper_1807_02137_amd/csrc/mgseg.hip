// mgseg.hip -- libmgseg host driver and C ABI (see include/mgseg.h).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/mgseg.h"
#include "mgseg_kernels.h"
#include "mgseg_aos.h"
#include "mgseg_lfa.h"
#include "mgseg_local.h"

#define MAXLEV 16

namespace {

// device scalar slots (doubles)
enum {
    DS_C1 = 0, DS_C2 = 1,
    DS_AREA_FRZ = 2,          // area term of the current freeze
    DS_AREA_EVAL = 3,         // area term for operator evaluations
    DS_AREA64 = 4,            // area term at the FP64 finest phi
    DS_RES = 5,               // last residual norm of the paper's rows (the stopping measure)
    DS_ETA = 6,               // last relative change of phi (right after DS_RES)
    DS_RESR = 7,              // last residual norm of the smoother's rows (right after DS_ETA)
    DS_AREAB0 = 8,            // deviation form: area term at the base of level l is slot DS_AREAB0 + l
    DS_CO = 8 + MAXLEV,       // coarsest-solve changes (2 slots)
    DS_ENERGY = 8 + MAXLEV + 2,   // the model's energy (mgseg_get_stats)
    DS_COUNT = 8 + MAXLEV + 3
};

struct Level {
    int n = 0, m = 0, prm = 0, pcm = 0;
    double h = 0.0;
    float *z = nullptr, *d = nullptr, *w = nullptr, *fit = nullptr, *F = nullptr;
    float *P[3] = {nullptr, nullptr, nullptr};
    float *psi = nullptr, *phic = nullptr, *r = nullptr, *lo = nullptr, *hi = nullptr;
    float *G = nullptr;       // deviation form: the level's residual part of F (row-major)
    float *w_cm = nullptr, *fit_cm = nullptr, *F_cm = nullptr, *lo_cm = nullptr, *hi_cm = nullptr;
    float *T[3] = {nullptr, nullptr, nullptr};
    float *psi_cm = nullptr;
    float4 *cf = nullptr, *cf_cm = nullptr;   // deviation form: the sweeps' frozen face coefficients
    uint8_t *lab = nullptr, *lab_cm = nullptr;
    bool has_F = false;
};

}  // namespace

struct mgseg_ctx {
    mgseg_params p;
    hipStream_t s = nullptr;
    int L = 0, n = 0, m = 0;
    double h0 = 0.0, A1 = 0.0, res0 = 0.0, res = 0.0, eta = 0.0, rel = 0.0;
    double res0_rows = 0.0, res_rows = 0.0;   // the same for the rows as the smoother holds them
    int cycles = 0;
    Level lev[MAXLEV];
    double *phi64 = nullptr, *w64 = nullptr, *d64 = nullptr, *g64 = nullptr, *prev64 = nullptr;
    double *phi0m = nullptr;        // the marker-based initial level set of setup
    double *dsc = nullptr;          // device scalars
    double *part = nullptr;         // reduction partials
    int part_n = 0;
    float *co_prev = nullptr, *co_entry = nullptr;   // multi-kernel coarsest solve
    int *flags = nullptr;           // device flags: [0] coarsest solve finished, [1] markers inside phi0
    double *hres = nullptr;         // host copy of DS_RES, DS_ETA, DS_RESR (pinned, or hres_local)
    double hres_local[3] = {0.0, 0.0, 0.0};
    bool arena_owned = true;        // false: the arena is the library's static scratch
    bool noalloc = false;           // a context that may not allocate (no graph, no pinned memory)
    const int *sweep_skip = nullptr;
    double *hull_d = nullptr, *mk_d = nullptr;
    int hv = 0, k = 0;
    char *arena = nullptr;          // every device array of the context (dalloc)
    size_t arena_size = 0, arena_used = 0;
    float *pred = nullptr;          // network input and output of mgseg_predict_phi0 (first call)
    double *aos = nullptr;          // six n x m FP64 planes of the AOS solver (first call)
    double *lfa = nullptr;          // partials of mgseg_smoothing_rates (first call)
    mgseg_schedule sched{64, 0, 1, 1}; // launch schedule (mgseg_set_schedule, mgseg_tune)
    hipError_t err = hipSuccess;
    bool oom = false;
    // one V-cycle captured as a HIP graph (replayed on s); cap: private capture stream
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap = nullptr;
    bool graph_failed = false;
    // event timing of the finest-grid sweep launches
    bool prof_on = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
    size_t ev_next = 0;
};

namespace {

const int RED_BLOCKS = 1024;

// A context's device arrays are pieces (256-byte aligned) of one allocation,
// the arena: setup runs its allocation sequence once to size the arena
// (arena null: dalloc only counts) and once to hand out the pieces, so that
// setup makes one allocation and one zero fill and destroy one free.
template <typename T>
T *dalloc(mgseg_ctx *c, size_t count)
{
    if (count == 0) count = 1;
    const size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
    const size_t off = c->arena_used;
    c->arena_used += bytes;
    if (!c->arena) return nullptr;
    if (c->arena_used > c->arena_size) { c->oom = true; return nullptr; }
    return reinterpret_cast<T *>(c->arena + off);
}

inline int pad64(int x) { return (x + 63) / 64 * 64; }

inline void chk(mgseg_ctx *c)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && c->err == hipSuccess) c->err = e;
}

inline dim3 grid2(int n, int m, int bx = 256) { return dim3((m + bx - 1) / bx, n); }

// ---- host convex hull of the markers by gift wrapping (Jarvis march): from the
// lowest (row, col) point, each next vertex is the point that leaves every other
// point on one side of the edge (the farthest of collinear candidates, so no
// collinear vertex is kept); fixed arrays, no allocation.  pts: k <= 64 (row,
// col) pairs; hull: room for 2 k values; returns the vertex count (one for a
// single distinct point, two for collinear points)
int host_hull(const double *pts, int k, double *hull)
{
    double U[64][2];
    int nu = 0;
    for (int t = 0; t < k && t < 64; t++) {
        bool dup = false;
        for (int v = 0; v < nu && !dup; v++) dup = U[v][0] == pts[2 * t] && U[v][1] == pts[2 * t + 1];
        if (!dup) { U[nu][0] = pts[2 * t]; U[nu][1] = pts[2 * t + 1]; nu++; }
    }
    if (nu == 0) return 0;
    int start = 0;
    for (int v = 1; v < nu; v++)
        if (U[v][0] < U[start][0] || (U[v][0] == U[start][0] && U[v][1] < U[start][1])) start = v;
    int hv = 0, cur = start;
    do {
        hull[2 * hv] = U[cur][0]; hull[2 * hv + 1] = U[cur][1]; hv++;
        int nxt = cur == 0 ? 1 % nu : 0;
        for (int v = 0; v < nu; v++) {
            if (v == cur) continue;
            const double ar = U[nxt][0] - U[cur][0], ac = U[nxt][1] - U[cur][1];
            const double br = U[v][0] - U[cur][0], bc = U[v][1] - U[cur][1];
            const double side = ar * bc - ac * br;
            if (side < 0.0 || (side == 0.0 && br * br + bc * bc > ar * ar + ac * ac)) nxt = v;
        }
        cur = nxt;
    } while (cur != start && hv < nu);
    return hv;
}

// the hull as device edges (start, unit direction, length, outward normal and
// its offset) followed by its vertices: edges[8 ne] then vertices[2 hv];
// ne = hv for a polygon, 1 for a segment, 0 for a point; returns the count of
// values written (out: room for 10 hv)
int hull_geometry(const double *hull, int hv, double *out, int &ne, int &closed)
{
    closed = hv >= 3;
    ne = hv >= 3 ? hv : (hv == 2 ? 1 : 0);
    double cr = 0.0, cc = 0.0;
    for (int v = 0; v < hv; v++) { cr += hull[2 * v] / hv; cc += hull[2 * v + 1] / hv; }
    int o = 0;
    for (int e = 0; e < ne; e++) {
        const int f = (e + 1) % hv;
        const double ar = hull[2 * e], ac = hull[2 * e + 1];
        const double dr = hull[2 * f] - ar, dc = hull[2 * f + 1] - ac, len = std::hypot(dr, dc);
        const double ur = dr / len, uc = dc / len;
        double nr = uc, nc = -ur;
        // outward: away from the vertices' centroid (a polygon), either side (a segment)
        if (closed && nr * (cr - ar) + nc * (cc - ac) > 0.0) { nr = -nr; nc = -nc; }
        const double e8[8] = {ar, ac, ur, uc, len, nr, nc, nr * ar + nc * ac};
        for (int t = 0; t < 8; t++) out[o++] = e8[t];
    }
    for (int t = 0; t < 2 * hv; t++) out[o++] = hull[t];
    return o;
}

double host_area(const double *h, int hv)
{
    if (hv < 3) return 0.0;
    double s = 0.0;
    for (int t = 0; t < hv; t++) {
        int u = (t + 1) % hv;
        s += h[2 * t] * h[2 * u + 1] - h[2 * u] * h[2 * t + 1];
    }
    return 0.5 * std::fabs(s);
}

// mixed-precision mode: every level holds an FP32 deviation from a base
inline bool devm(const mgseg_ctx *c) { return c->p.mixed_precision != 0; }

float lev_e2(const mgseg_ctx *c, int l)
{
    double e = c->p.eps_tv_px * (double)(1 << l);
    return (float)(e * e);
}

// --------------------------------------------------------------------------
void transpose_f(mgseg_ctx *c, const float *in, int pin, float *out, int pout, int n, int m)
{
    dim3 g((m + TILE - 1) / TILE, (n + TILE - 1) / TILE), b(TILE, 8);
    hipLaunchKernelGGL(k_transpose<float>, g, b, 0, c->s, in, pin, out, pout, n, m);
}
void transpose_u8(mgseg_ctx *c, const uint8_t *in, int pin, uint8_t *out, int pout, int n, int m)
{
    dim3 g((m + TILE - 1) / TILE, (n + TILE - 1) / TILE), b(TILE, 8);
    hipLaunchKernelGGL(k_transpose<uint8_t>, g, b, 0, c->s, in, pin, out, pout, n, m);
}

// area term 2 nu (h^2 sum H(phi) - A1) of level l at phi (row-major) -> slot
void area_term(mgseg_ctx *c, int l, const float *phi, int pp, int slot)
{
    Level &L = c->lev[l];
    int nb = std::min(RED_BLOCKS, std::max(1, (L.n * L.m + 255) / 256));
    hipLaunchKernelGGL(k_sums<float>, dim3(nb), dim3(256), 0, c->s, phi, pp, (const float *)nullptr, 0, L.n, L.m,
                       c->p.eps, c->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, nb, 0, (double)L.n * L.m, L.h * L.h, c->A1,
                       c->p.nu, c->dsc + slot);
}

void update_fit(mgseg_ctx *c)
{
    FitLevels F;
    F.L = c->L;
    F.trow0[0] = 0;
    for (int l = 0; l < c->L; l++) {
        const Level &L = c->lev[l];
        // the mixed mode's column sweeps take the fit term inside T: no column-major copy
        F.z[l] = L.z; F.d[l] = L.d; F.fit[l] = L.fit; F.fit_cm[l] = devm(c) ? nullptr : L.fit_cm;
        F.p[l] = L.prm; F.pc[l] = L.pcm; F.n[l] = L.n; F.m[l] = L.m;
        F.trow0[l + 1] = F.trow0[l] + (L.n + TILE - 1) / TILE;
    }
    const dim3 g((c->m + TILE - 1) / TILE, F.trow0[c->L]);
    const dim3 tb(TILE, tile_rows((long long)g.x * g.y));
    hipLaunchKernelGGL(k_fit, g, tb, 0, c->s, F, c->dsc + DS_C1, (float)c->p.lambda1, (float)c->p.lambda2,
                       (float)c->p.theta, c->p.model);
}

// c1, c2 (eq. c1c2) from the FP64 finest phi; sums_done: the partial sums are
// already in c->part (k_finish0_sums)
void update_c(mgseg_ctx *c, bool sums_done = false)
{
    Level &L = c->lev[0];
    int nb = std::min(RED_BLOCKS, std::max(1, (c->n * c->m + 255) / 256));
    if (!sums_done)
        hipLaunchKernelGGL(k_sums<double>, dim3(nb), dim3(256), 0, c->s, c->phi64, c->m, L.z, L.prm, c->n, c->m,
                           c->p.eps, c->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, nb, 1, (double)c->n * c->m, 0.0, 0.0, 0.0,
                       c->dsc + DS_C1);
    update_fit(c);
}

// FP64 finest residual: norm into DS_RES; FP32 mode: phi32 <- fl32(phi64);
// deviation form: G of the finest grid <- fl32(r64)
void res64(mgseg_ctx *c)
{
    Level &L = c->lev[0];
    if (c->p.model == 1) {
        int nb = std::min(RED_BLOCKS, std::max(1, (c->n * c->m + 255) / 256));
        hipLaunchKernelGGL(k_sums<double>, dim3(nb), dim3(256), 0, c->s, c->phi64, c->m, (const float *)nullptr, 0,
                           c->n, c->m, c->p.eps, c->part);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, nb, 0, (double)c->n * c->m,
                           L.h * L.h, c->A1, c->p.nu, c->dsc + DS_AREA64);
    }
    Res64Args A;
    A.phi64 = c->phi64; A.w64 = c->w64; A.d64 = c->d64;
    A.z32 = L.z; A.w32 = L.w; A.fit32 = L.fit; A.p32 = L.prm;
    A.c12 = c->dsc + DS_C1; A.area = c->p.model == 1 ? c->dsc + DS_AREA64 : nullptr;
    A.kap = c->p.mu / L.h; A.e2 = lev_e2(c, 0); A.eps = c->p.eps;
    A.l1 = c->p.lambda1; A.l2 = c->p.lambda2; A.theta = c->p.theta; A.M = c->p.M;
    A.model = c->p.model; A.scaled = c->p.scaled; A.n = c->n; A.m = c->m;
    A.phi32 = devm(c) ? nullptr : L.P[0];
    A.G = devm(c) ? L.G : nullptr;
    A.partial = c->part;
    const dim3 g((c->m + TILE - 1) / TILE, std::min((c->n + TILE - 1) / TILE, 32));
    hipLaunchKernelGGL(k_res64, g, dim3(TILE, R64_ROWS), 0, c->s, A);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, (int)(g.x * g.y), 4, 0.0, 0.0, 0.0, 0.0,
                       c->dsc + DS_RES);
}

// --------------------------------------------------------------------------
// one directional sweep on level l: s = 0 (A), 1 (B) row-major, 2 (C), 3 (D)
// column-major; phi_old -> phi_new in the layout of the sweep
// bit: the label bit of the starred cells (default: the sweep's own; a bit no
// label carries makes every cell a point)
// scratch (reverse sweeps): a free plane in the sweep's line layout, which lets a long-line
// sweep run split, written there in its own layout and then transposed to tout
void launch_sweep(mgseg_ctx *c, int l, int s, const float *phi_old, float *phi_new, float *tout = nullptr,
                  int tpitch = 0, int bit = -1, const float *qd = nullptr, float *scratch = nullptr)
{
    Level &L = c->lev[l];
    bool cm = s >= 2;
    LineArgs A;
    A.phi_old = phi_old; A.phi_new = phi_new; A.tout = tout; A.tpitch = tpitch; A.skip = c->sweep_skip;
    A.psi = cm ? L.psi_cm : L.psi;
    A.w = cm ? L.w_cm : L.w;
    A.fit = devm(c) ? nullptr : (cm ? L.fit_cm : L.fit);
    A.F = L.has_F ? (cm ? L.F_cm : L.F) : nullptr;
    A.lab = cm ? L.lab_cm : L.lab;
    const bool bnd = l > 0 || devm(c);
    A.lo = bnd ? (cm ? L.lo_cm : L.lo) : nullptr;
    A.hi = bnd ? (cm ? L.hi_cm : L.hi) : nullptr;
    A.area = c->p.model == 1 ? c->dsc + DS_AREA_FRZ : nullptr;
    // deviation form: the freeze stored the scaled face coefficients (and the fit term is in T)
    const bool cfm = devm(c) && L.cf != nullptr;
    A.cf = cfm ? (cm ? L.cf_cm : L.cf) : nullptr;
    A.qd = qd;
    A.split = 0; A.nb_old = nullptr;
    A.pitch = cm ? L.pcm : L.prm;
    A.lpitch = A.pitch;
    A.nl = cm ? L.m : L.n;
    A.ml = cm ? L.n : L.m;
    A.kap = (float)(c->p.mu / L.h); A.e2 = lev_e2(c, l); A.M = (float)c->p.M; A.eps = (float)c->p.eps;
    A.bit = bit < 0 ? s : bit; A.scaled = c->p.scaled; A.run_max = c->p.run_max;
    bool rev = (s == 1 || s == 3);
    int bands = (A.nl + 3) / 4;
    int ml = A.ml;
    if (ml > 8192) {   // setup accepts sides up to 8192
        if (c->err == hipSuccess) c->err = hipErrorInvalidValue;
        return;
    }
    // whole-line systems (every cell starred) exist for the forward sweep on the stored coefficients
    const bool whl = A.bit == LAB_ALL && ml <= 1024;
    if (whl && (rev || !cfm)) {
        if (c->err == hipSuccess) c->err = hipErrorInvalidValue;
        return;
    }
    const size_t lds = sweep_lds_bytes(ml), llds = long_lds_bytes<LONG_NT>(ml), lds2 = sweep2_lds_bytes(ml);
    const size_t llds_s = long_lds_bytes<LONG_NT>(ml, false);   // a split long sweep: no line in LDS
    // a forward sweep written in its own layout may run as two launches (the bands' first three
    // lines, then their fourth lines reading the final neighbours), with no recomputed line
    const bool split = c->sched.split_long && !rev && !tout && phi_new;
#define MG_SWEEP_CF(NT, CF)                                                                       \
    do {                                                                                              \
        if (rev) hipLaunchKernelGGL((k_sweep<NT, true, CF>), dim3(bands), dim3(NT), lds, c->s, A); \
        else if (split) {                                                                             \
            LineArgs A1 = A, A2 = A;                                                                  \
            A1.split = 1;                                                                             \
            A2.split = 2; A2.nb_old = phi_new;                                                        \
            hipLaunchKernelGGL((k_sweep<NT, false, CF>), dim3(bands), dim3(NT), lds, c->s, A1);      \
            hipLaunchKernelGGL((k_sweep<NT, false, CF>), dim3(bands), dim3(NT), lds, c->s, A2);      \
        } else hipLaunchKernelGGL((k_sweep<NT, false, CF>), dim3(bands), dim3(NT), lds, c->s, A);    \
    } while (0)
#define MG_SWEEP(NT)                   \
    do {                               \
        if (cfm) MG_SWEEP_CF(NT, true);    \
        else MG_SWEEP_CF(NT, false);   \
    } while (0)
#define MG_SWEEP2_CF(NT, CF)                                                                              \
    do {                                                                                                  \
        if (rev) hipLaunchKernelGGL((k_sweep2<NT, true, CF>), dim3(bands), dim3(2 * NT), lds2, c->s, A); \
        else hipLaunchKernelGGL((k_sweep2<NT, false, CF>), dim3(bands), dim3(2 * NT), lds2, c->s, A);    \
    } while (0)
#define MG_SWEEP2(NT)                  \
    do {                               \
        if (cfm) MG_SWEEP2_CF(NT, true);   \
        else MG_SWEEP2_CF(NT, false);  \
    } while (0)
    // a reverse sweep with a transposed output and a free plane runs split as the forward sweep
    // does, written in its own layout to the free plane, which one tiled transpose then copies
    // to the output (coalesced on both sides, where the sweep's own transposed stores hit a new
    // page every few cells)
    const bool split_rev = c->sched.split_long && rev && tout && scratch;
#define MG_SWEEP_LONG_CF(CF)                                                                                    \
    do {                                                                                                        \
        if (rev && split_rev) {                                                                                 \
            LineArgs A1 = A, A2 = A;                                                                            \
            A1.tout = A2.tout = nullptr; A1.phi_new = A2.phi_new = scratch;                                     \
            A1.split = 1; A1.fresh = scratch;                                                                   \
            A2.split = 2; A2.nb_old = scratch; A2.fresh = scratch;                                              \
            hipLaunchKernelGGL((k_sweep_long<LONG_NT, true, CF>), dim3(bands), dim3(LONG_NT), llds_s, c->s, A1);       \
            hipLaunchKernelGGL((k_sweep_long<LONG_NT, true, CF>), dim3(bands), dim3(LONG_NT), llds_s, c->s, A2);       \
            transpose_f(c, scratch, A.pitch, tout, tpitch, A.nl, A.ml);                                       \
        } else if (rev) hipLaunchKernelGGL((k_sweep_long<LONG_NT, true, CF>), dim3(bands), dim3(LONG_NT), llds, c->s, A);  \
        else if (split) {                                                                                       \
            LineArgs A1 = A, A2 = A;                                                                            \
            A1.split = 1; A1.fresh = phi_new;                                                                   \
            A2.split = 2; A2.nb_old = phi_new; A2.fresh = phi_new;                                              \
            hipLaunchKernelGGL((k_sweep_long<LONG_NT, false, CF>), dim3(bands), dim3(LONG_NT), llds_s, c->s, A1);      \
            hipLaunchKernelGGL((k_sweep_long<LONG_NT, false, CF>), dim3(bands), dim3(LONG_NT), llds_s, c->s, A2);      \
        } else hipLaunchKernelGGL((k_sweep_long<LONG_NT, false, CF>), dim3(bands), dim3(LONG_NT), llds, c->s, A);    \
    } while (0)
#define MG_SWEEP_LONG()                \
    do {                               \
        if (cfm) MG_SWEEP_LONG_CF(true);   \
        else MG_SWEEP_LONG_CF(false);  \
    } while (0)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool timed = c->prof_on && l == 0;
    if (timed) {
        while (c->ev_pool.size() < c->ev_next + 2) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) { timed = false; break; }
            c->ev_pool.push_back(e);
        }
    }
    if (timed) {
        e0 = c->ev_pool[c->ev_next]; e1 = c->ev_pool[c->ev_next + 1];
        c->ev_next += 2;
        (void)hipEventRecord(e0, c->s);
    }
    // one thread per cell up to 1024-cell lines; longer lines take rounds.  Up
    // to 512 cells the workgroup has a second half that computes the
    // recomputed neighbour line beside the band's first line.
    // A whole-line system (every cell starred: the line relaxation of Hybrid
    // Smoother 1, forward, on the stored coefficients) has kernels of its own
    // that eliminate the line by a scan.
    // the schedule's line_threads = 1 gives each line the next wider group (lines of at most 512 cells)
    const int mls = c->sched.line_threads && ml <= 512 ? 2 * ml : ml;
    if (whl) {
        if (mls <= 64) hipLaunchKernelGGL((k_sweep2<64, false, true, true>), dim3(bands), dim3(128), lds2, c->s, A);
        else if (mls <= 128) hipLaunchKernelGGL((k_sweep2<128, false, true, true>), dim3(bands), dim3(256), lds2, c->s, A);
        else if (mls <= 256) hipLaunchKernelGGL((k_sweep2<256, false, true, true>), dim3(bands), dim3(512), lds2, c->s, A);
        else if (mls <= 512) hipLaunchKernelGGL((k_sweep2<512, false, true, true>), dim3(bands), dim3(1024), lds2, c->s, A);
        else hipLaunchKernelGGL((k_sweep<1024, false, true, true>), dim3(bands), dim3(1024), lds, c->s, A);
    } else if (mls <= 64) MG_SWEEP2(64);
    else if (mls <= 128) MG_SWEEP2(128);
    else if (mls <= 256) MG_SWEEP2(256);
    else if (mls <= 512) MG_SWEEP2(512);
    else if (mls <= 1024) MG_SWEEP(1024);
    else MG_SWEEP_LONG();
#undef MG_SWEEP
#undef MG_SWEEP_CF
#undef MG_SWEEP2
#undef MG_SWEEP2_CF
#undef MG_SWEEP_LONG
#undef MG_SWEEP_LONG_CF
    if (timed) {
        (void)hipEventRecord(e1, c->s);
        c->ev_used.push_back({e0, e1});
    }
    chk(c);
}

int area_b_slot(int l) { return l == 0 ? DS_AREA64 : DS_AREAB0 + l; }

// deviation-form arguments of level l; fn is called with DevArgs<double> on the
// finest grid (base = the FP64 iterate) and DevArgs<float> below (base = phic)
template <typename BT>
DevArgs<BT> dev_args(mgseg_ctx *c, int l, const BT *b, int pb)
{
    Level &L = c->lev[l];
    DevArgs<BT> A;
    A.b = b; A.pb = pb;
    A.e = L.P[0]; A.G = L.G; A.w = L.w; A.fit = L.fit; A.lo = L.lo; A.hi = L.hi;
    A.psi = L.psi; A.T = L.F; A.r = L.r; A.lab = L.lab;
    A.psi_cm = nullptr; A.T_cm = nullptr; A.lab_cm = nullptr; A.pc = L.pcm;
    A.cf = nullptr; A.cf_cm = nullptr;
    A.area_b = c->p.model == 1 ? c->dsc + area_b_slot(l) : nullptr;
    A.area_u = nullptr;
    A.p = L.prm; A.n = L.n; A.m = L.m; A.scaled = c->p.scaled;
    A.kap = (float)(c->p.mu / L.h); A.e2 = lev_e2(c, l); A.eps = (float)c->p.eps; A.Sigma = (float)c->p.Sigma;
    return A;
}
template <class Fn>
void with_dev(mgseg_ctx *c, int l, Fn fn)
{
    if (l == 0) fn(dev_args<double>(c, 0, c->phi64, c->m));
    else fn(dev_args<float>(c, l, c->lev[l].phic, c->lev[l].prm));
}

// area term at b + e of level l (deviation form) -> slot
void dev_area(mgseg_ctx *c, int l, int slot)
{
    Level &L = c->lev[l];
    int nb = std::min(RED_BLOCKS, std::max(1, (L.n * L.m + 255) / 256));
    if (l == 0)
        hipLaunchKernelGGL(k_sums_dev<double>, dim3(nb), dim3(256), 0, c->s, c->phi64, c->m, L.P[0], L.prm, L.n, L.m,
                           c->p.eps, c->part);
    else
        hipLaunchKernelGGL(k_sums_dev<float>, dim3(nb), dim3(256), 0, c->s, L.phic, L.prm, L.P[0], L.prm, L.n, L.m,
                           c->p.eps, c->part);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, nb, 0, (double)L.n * L.m, L.h * L.h, c->A1,
                       c->p.nu, c->dsc + slot);
}

// freeze at the current state: psi, labels, area term; deviation form also
// the frozen right-hand side T (in F)
void freeze(mgseg_ctx *c, int l)
{
    Level &L = c->lev[l];
    if (devm(c)) {
        const bool rc = c->p.model == 1;
        if (rc) dev_area(c, l, DS_AREA_FRZ);
        with_dev(c, l, [&](auto A) {
            using BT = std::remove_const_t<std::remove_pointer_t<decltype(A.b)>>;
            A.area_u = rc ? c->dsc + DS_AREA_FRZ : nullptr;
            // with stored coefficients no sweep reads psi
            A.psi = L.cf ? nullptr : L.psi;
            A.psi_cm = L.cf ? nullptr : L.psi_cm; A.T_cm = L.F_cm; A.lab_cm = L.lab_cm;
            A.cf = L.cf; A.cf_cm = L.cf_cm;
            dim3 gt((L.m + TILE - 1) / TILE, (L.n + TILE - 1) / TILE);
            hipLaunchKernelGGL(k_freeze_dev<BT>, gt, dim3(TILE, tile_rows((long long)gt.x * gt.y)), 0, c->s, A);
        });
        L.has_F = true;
        chk(c);
        return;
    }
    hipLaunchKernelGGL(k_freeze32, grid2(L.n, L.m), dim3(256), 0, c->s, L.P[0], L.w, L.prm, L.n, L.m, lev_e2(c, l),
                       (float)c->p.Sigma, L.psi, L.psi_cm, L.lab, L.lab_cm, L.pcm);
    if (c->p.model == 1) area_term(c, l, L.psi, L.prm, DS_AREA_FRZ);
    chk(c);
}

// one pass of a local ("-II") smoother (Sec. 3.2): 5 GSLEX-II, 6 GSLINE-II, 7 NEWT-II
// (Spencer-Chen rows: the same as GSLEX-II); the rows of each class, or its columns,
// at once, the coefficients refreshed from the current iterate where they are used
void outer_local(mgseg_ctx *c, int l)
{
    Level &L = c->lev[l];
    with_dev(c, l, [&](auto A) {
        using BT = std::remove_const_t<std::remove_pointer_t<decltype(A.b)>>;
        if (c->p.smoother != 6) {
            for (int cls = 0; cls < 4; cls++) {
                const int rows = (L.n - cls + 3) / 4;
                if (rows > 0)
                    hipLaunchKernelGGL(k_gslex_local<BT>, dim3((rows + 63) / 64), dim3(64), 0, c->s, A, cls,
                                       c->sweep_skip);
            }
            return;
        }
        LineArgs S;
        std::memset(&S, 0, sizeof(S));
        S.tout = L.P[0]; S.tpitch = L.prm; S.pitch = L.pcm; S.lpitch = L.pcm; S.skip = c->sweep_skip;
        S.nl = L.m; S.ml = L.n; S.kap = (float)(c->p.mu / L.h); S.e2 = lev_e2(c, l); S.M = (float)c->p.M;
        S.eps = (float)c->p.eps; S.bit = LAB_ALL; S.scaled = c->p.scaled; S.run_max = c->p.run_max;
        const size_t lds = gsline_local_lds(L.n);
        for (int cls = 0; cls < 4; cls++) {
            const int cols = (L.m - cls + 3) / 4;
            if (cols <= 0) continue;
            if (L.n <= 64) hipLaunchKernelGGL((k_gsline_local<64, BT>), dim3(cols), dim3(64), lds, c->s, A, S, cls);
            else if (L.n <= 128) hipLaunchKernelGGL((k_gsline_local<128, BT>), dim3(cols), dim3(128), lds, c->s, A, S, cls);
            else if (L.n <= 256) hipLaunchKernelGGL((k_gsline_local<256, BT>), dim3(cols), dim3(256), lds, c->s, A, S, cls);
            else if (L.n <= 512) hipLaunchKernelGGL((k_gsline_local<512, BT>), dim3(cols), dim3(512), lds, c->s, A, S, cls);
            else hipLaunchKernelGGL((k_gsline_local<1024, BT>), dim3(cols), dim3(1024), lds, c->s, A, S, cls);
        }
    });
    chk(c);
}

// one outer iteration of Hybrid Smoother 2: freeze, sweeps A, B, C, D
void outer(mgseg_ctx *c, int l)
{
    Level &L = c->lev[l];
    if (c->p.smoother >= 5) {
        outer_local(c, l);
        return;
    }
    freeze(c, l);
    if (c->p.smoother == 1 || c->p.smoother == 4) {
        // GSLEX-I: one pass of point updates in the order of sweep A (no cell starred).
        // NEWT-I (eq. newtrc) is the same pass with the derivative Q' of the Rada-Chen
        // area term added to every diagonal (Spencer-Chen: Q = 0, and NEWT is GSLEX)
        const float *qd = nullptr;
        if (c->p.smoother == 4 && c->p.model == 1) {
            const double h2nu2 = 2.0 * c->p.nu * L.h * L.h;
            if (devm(c)) {
                if (l == 0)
                    hipLaunchKernelGGL(k_newton_diag<double>, grid2(L.n, L.m), dim3(256), 0, c->s, c->phi64, c->m,
                                       L.P[0], L.prm, L.n, L.m, h2nu2, c->p.eps, c->p.scaled,
                                       c->dsc + DS_AREA_FRZ, L.r);
                else
                    hipLaunchKernelGGL(k_newton_diag<float>, grid2(L.n, L.m), dim3(256), 0, c->s, L.phic, L.prm,
                                       L.P[0], L.prm, L.n, L.m, h2nu2, c->p.eps, c->p.scaled,
                                       c->dsc + DS_AREA_FRZ, L.r);
            } else {
                hipLaunchKernelGGL(k_newton_diag<float>, grid2(L.n, L.m), dim3(256), 0, c->s, (const float *)nullptr,
                                   0, L.psi, L.prm, L.n, L.m, h2nu2, c->p.eps, c->p.scaled, c->dsc + DS_AREA_FRZ,
                                   L.r);
            }
            qd = L.r;       // the residual plane is free while the level smooths
        }
        launch_sweep(c, l, 0, L.P[0], L.P[1], nullptr, 0, LAB_NONE, qd);
        (void)hipMemcpyAsync(L.P[0], L.P[1], sizeof(float) * (size_t)L.n * L.prm, hipMemcpyDeviceToDevice, c->s);
        chk(c);
        return;
    }
    if (c->p.smoother == 2 || c->p.smoother == 3) {
        // GSLINE-I (eq. system): every column one line system, in sweep C's order and
        // layout, every cell starred, the result written row-major.  Hybrid Smoother 1
        // (Algorithm 2) follows it with the blocks at the jump-set cells in eight classes.
        transpose_f(c, L.P[0], L.prm, L.T[1], L.pcm, L.n, L.m);
        launch_sweep(c, l, 2, L.T[1], nullptr, L.P[0], L.prm, LAB_ALL);
        if (c->p.smoother == 3) {
            chk(c);
            return;
        }
        BlockArgs B;
        B.e = L.P[0]; B.cf = L.cf; B.T = L.F; B.lo = L.lo; B.hi = L.hi; B.lab = L.lab; B.skip = c->sweep_skip;
        B.p = L.prm; B.n = L.n; B.m = L.m;
        for (int cls = 0; cls < 8; cls++) {
            B.cls = cls;
            hipLaunchKernelGGL(k_hs1_blocks, grid2(L.n, L.m), dim3(256), 0, c->s, B);
        }
        chk(c);
        return;
    }
    launch_sweep(c, l, 0, L.P[0], L.P[1]);
    launch_sweep(c, l, 1, L.P[1], nullptr, L.T[1], L.pcm, -1, nullptr, L.P[0]);   // written column-major
    launch_sweep(c, l, 2, L.T[1], L.T[2]);
    launch_sweep(c, l, 3, L.T[2], nullptr, L.P[0], L.prm, -1, nullptr, L.T[1]);   // written row-major
    chk(c);
}

// arguments of the one-workgroup smoother on level l (a coarse grid)
CoarseArgs coarse_args(mgseg_ctx *c, int l, int iters, double rtol)
{
    Level &L = c->lev[l];
    const bool dev = devm(c);
    CoarseArgs C;
    C.P0 = L.P[0]; C.w = L.w; C.fit = L.fit; C.lo = L.lo; C.hi = L.hi;
    C.F = (!dev && L.has_F) ? L.F : nullptr;
    C.base = dev ? L.phic : nullptr; C.G = dev ? L.G : nullptr;
    C.area_b = dev && c->p.model == 1 ? c->dsc + area_b_slot(l) : nullptr;
    C.area = c->p.model == 1 ? c->dsc + DS_AREA_FRZ : nullptr;
    C.h2 = L.h * L.h; C.A1 = c->A1; C.nu = c->p.nu; C.eps = c->p.eps;
    C.n = L.n; C.m = L.m; C.prm = L.prm; C.iters = iters; C.scaled = c->p.scaled;
    C.kap = (float)(c->p.mu / L.h); C.e2 = lev_e2(c, l); C.M = (float)c->p.M; C.Sigma = (float)c->p.Sigma;
    C.rtol = (float)rtol;
    C.smoother = c->p.smoother;
    C.run_max = c->p.run_max;
    return C;
}
// a coarse grid the one-workgroup smoother holds in LDS
bool lds_level(mgseg_ctx *c, int l)
{
    const Level &L = c->lev[l];
    const int side = std::min(64, c->sched.lds_side);
    return l > 0 && L.n <= side && L.m <= side && L.n * L.m <= CO_MAX_CELLS;
}

void smooth(mgseg_ctx *c, int l, int iters)
{
    // grids of at most 8 bands each way: all outer iterations in one workgroup, one band per wave
    if (iters > 0 && lds_level(c, l) && c->lev[l].n <= 32 && c->lev[l].m <= 32 && c->p.smoother <= 1) {
        hipLaunchKernelGGL((k_coarse_smooth<512>), dim3(1), dim3(512), coarse_lds_bytes(c->lev[l].n, c->lev[l].m),
                           c->s, coarse_args(c, l, iters, 0.0));
        chk(c);
        return;
    }
    for (int it = 0; it < iters; it++) outer(c, l);
}

void coarsest(mgseg_ctx *c, int l)
{
    Level &L = c->lev[l];
    const bool dev = devm(c);
    // a grid of one cell has no interior face, so the curvature operator (and the
    // smooth error a coarse grid corrects) vanishes there: it returns the state it
    // received, a zero coarse correction
    if (L.n * L.m == 1) return;
    if (lds_level(c, l) && c->p.smoother <= 1) {
        // one wave for a grid of one band, else one band per wave of 512 threads
        const CoarseArgs C = coarse_args(c, l, c->p.coarse_iters, c->p.coarse_rtol);
        if (L.n <= 4 && L.m <= 4)
            hipLaunchKernelGGL((k_coarse_smooth<64>), dim3(1), dim3(64), coarse_lds_bytes(L.n, L.m), c->s, C);
        else
            hipLaunchKernelGGL((k_coarse_smooth<512>), dim3(1), dim3(512), coarse_lds_bytes(L.n, L.m), c->s, C);
        chk(c);
        return;
    }
    // multi-kernel path: all coarse_iters outer iterations are enqueued; the
    // stopping test sets a device flag after which the sweeps return at once
    // (the freezes of the remaining iterations recompute the same state)
    const size_t bytes = sizeof(float) * (size_t)L.n * L.prm;
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, c->s, c->flags, 0);
    (void)hipMemcpyAsync(c->co_entry, L.P[0], bytes, hipMemcpyDeviceToDevice, c->s);
    c->sweep_skip = c->flags;
    for (int it = 0; it < c->p.coarse_iters; it++) {
        (void)hipMemcpyAsync(c->co_prev, L.P[0], bytes, hipMemcpyDeviceToDevice, c->s);
        outer(c, l);
        hipLaunchKernelGGL(k_coarse_delta, dim3(1), dim3(256), 0, c->s, L.P[0], c->co_prev, c->co_entry, L.prm, L.n,
                           L.m, c->p.coarse_rtol, c->flags);
    }
    c->sweep_skip = nullptr;
    chk(c);
}

void residual(mgseg_ctx *c, int l, float *r, double *partial)
{
    Level &L = c->lev[l];
    if (devm(c)) {
        const bool rc = c->p.model == 1;
        if (rc) dev_area(c, l, DS_AREA_EVAL);
        with_dev(c, l, [&](auto A) {
            using BT = std::remove_const_t<std::remove_pointer_t<decltype(A.b)>>;
            A.area_u = rc ? c->dsc + DS_AREA_EVAL : nullptr;
            A.r = r;
            const dim3 gt((L.m + TILE - 1) / TILE, (L.n + TILE - 1) / TILE);
            hipLaunchKernelGGL(k_res_dev<BT>, gt, dim3(TILE, tile_rows((long long)gt.x * gt.y)), 0, c->s, A);
        });
        chk(c);
        return;
    }
    if (c->p.model == 1) area_term(c, l, L.P[0], L.prm, DS_AREA_EVAL);
    hipLaunchKernelGGL(k_residual, grid2(L.n, L.m), dim3(256), 0, c->s, L.P[0], L.w, L.fit,
                       L.has_F ? L.F : nullptr, l > 0 ? L.lo : nullptr, l > 0 ? L.hi : nullptr, L.prm, L.n, L.m,
                       (float)(c->p.mu / L.h), lev_e2(c, l), (float)c->p.eps,
                       c->p.model == 1 ? c->dsc + DS_AREA_EVAL : nullptr, c->p.scaled, (float)c->p.M, r, partial);
    chk(c);
}

// FAS V-cycle (Algorithm-1 box, gamma = 1) from level l0 down and back.
// Deviation form: the coarse base is the restricted state, the coarse
// deviation starts at zero and G is the restricted residual; the FP32 mode
// keeps full values with F_c = N_c(phic) + R r.
void vcycle_from(mgseg_ctx *c, int l0)
{
    const bool dev = devm(c);
    for (int l = l0; l < c->L - 1; l++) {
        Level &L = c->lev[l], &Lc = c->lev[l + 1];
        smooth(c, l, c->p.nu1);
        dim3 gc = grid2(Lc.n, Lc.m);
        if (dev) {
            // the fine residual and its restriction (to G) and the state (base, deviation,
            // bounds) in one launch; the fine residual stays in LDS
            const bool rc = c->p.model == 1;
            if (rc) dev_area(c, l, DS_AREA_EVAL);
            with_dev(c, l, [&](auto A) {
                using BT = std::remove_const_t<std::remove_pointer_t<decltype(A.b)>>;
                A.area_u = rc ? c->dsc + DS_AREA_EVAL : nullptr;
                A.r = nullptr;
                const dim3 g((Lc.m + RR_CT - 1) / RR_CT, (Lc.n + RR_CT - 1) / RR_CT);
                hipLaunchKernelGGL(k_res_restrict_dev<BT>, g, dim3(RR_CT, RR_CT), 0, c->s, A, Lc.phic, Lc.P[0],
                                   Lc.lo, Lc.hi, Lc.prm, Lc.n, Lc.m, Lc.lo_cm, Lc.hi_cm, Lc.pcm, Lc.G);
            });
            if (rc) area_term(c, l + 1, Lc.phic, Lc.prm, DS_AREAB0 + l + 1);
        } else {
            residual(c, l, L.r, nullptr);
            hipLaunchKernelGGL(k_restrict, gc, dim3(256), 0, c->s, L.r, L.prm, Lc.r, Lc.prm, Lc.n, Lc.m);
            hipLaunchKernelGGL(k_restrict, gc, dim3(256), 0, c->s, L.P[0], L.prm, Lc.phic, Lc.prm, Lc.n, Lc.m);
            hipLaunchKernelGGL(k_coarse_bounds, gc, dim3(256), 0, c->s, L.P[0], l > 0 ? L.lo : nullptr,
                               l > 0 ? L.hi : nullptr, L.prm, L.n, L.m, Lc.phic, Lc.lo, Lc.hi, Lc.prm, Lc.n, Lc.m,
                               (float)c->p.M);
            if (c->p.model == 1) area_term(c, l + 1, Lc.phic, Lc.prm, DS_AREA_EVAL);
            hipLaunchKernelGGL(k_coarse_rhs, gc, dim3(256), 0, c->s, Lc.phic, Lc.w, Lc.fit, Lc.r, Lc.prm, Lc.n, Lc.m,
                               (float)(c->p.mu / Lc.h), lev_e2(c, l + 1), (float)c->p.eps,
                               c->p.model == 1 ? c->dsc + DS_AREA_EVAL : nullptr, c->p.scaled, Lc.F, Lc.P[0]);
            transpose_f(c, Lc.F, Lc.prm, Lc.F_cm, Lc.pcm, Lc.n, Lc.m);
            transpose_f(c, Lc.lo, Lc.prm, Lc.lo_cm, Lc.pcm, Lc.n, Lc.m);
            transpose_f(c, Lc.hi, Lc.prm, Lc.hi_cm, Lc.pcm, Lc.n, Lc.m);
            Lc.has_F = true;
        }
        chk(c);
    }
    coarsest(c, c->L - 1);
    for (int l = c->L - 2; l >= l0; l--) {
        Level &L = c->lev[l], &Lc = c->lev[l + 1];
        const bool bnd = l > 0 || dev;
        hipLaunchKernelGGL(k_prolong_correct, grid2(L.n, L.m), dim3(256), 0, c->s, L.P[0], bnd ? L.lo : nullptr,
                           bnd ? L.hi : nullptr, L.prm, L.n, L.m, Lc.P[0], dev ? nullptr : Lc.phic, Lc.prm,
                           (float)c->p.M);
        smooth(c, l, c->p.nu2);
        chk(c);
    }
}

mgseg_status sync_status(mgseg_ctx *c)
{
    hipError_t e = hipStreamSynchronize(c->s);
    if (e != hipSuccess && c->err == hipSuccess) c->err = e;
    if (c->err != hipSuccess) return MGSEG_E_HIP;
    return MGSEG_OK;
}

double read_scalar(mgseg_ctx *c, int slot)
{
    double v = 0.0;
    (void)hipMemcpyAsync(&v, c->dsc + slot, sizeof(double), hipMemcpyDeviceToHost, c->s);
    (void)hipStreamSynchronize(c->s);
    return v;
}

// refresh c1, c2, then the FP64 residual (norm, phi32, F~)
mgseg_status refresh_and_residual(mgseg_ctx *c)
{
    update_c(c);
    res64(c);
    c->lev[0].has_F = false;
    return MGSEG_OK;
}

// the device work of one cycle (V-cycle, finest update, c refresh, FP64
// residual, eta partials), all on c->s and without host synchronisation
// unless the coarsest grid needs the multi-kernel path
void enqueue_cycle(mgseg_ctx *c)
{
    Level &L0 = c->lev[0];
    size_t N = (size_t)c->n * c->m;
    const int nb = std::min(RED_BLOCKS, std::max(1, (int)((N + 255) / 256)));
    dim3 g = grid2(c->n, c->m);
    if (c->p.mixed_precision) {
        // the base phi64 stays fixed through the V-cycle, so the cycle's end takes the
        // change and the c1, c2 sums in the pass that updates it
        const dim3 gt((c->m + TILE - 1) / TILE, (c->n + TILE - 1) / TILE);
        const dim3 tb(TILE, tile_rows((long long)gt.x * gt.y));
        hipLaunchKernelGGL(k_start0, gt, tb, 0, c->s, c->phi64, c->n, c->m, c->p.M, L0.P[0], L0.lo, L0.hi, L0.prm,
                           L0.lo_cm, L0.hi_cm, L0.pcm);
        vcycle_from(c, 0);
        hipLaunchKernelGGL(k_finish0_sums, dim3(nb), dim3(256), 0, c->s, c->phi64, L0.P[0], L0.lo, L0.hi, L0.prm,
                           L0.z, L0.prm, c->n, c->m, c->p.M, c->p.eps, c->part, c->part + 4 * RED_BLOCKS);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part + 4 * RED_BLOCKS, nb, 3, 0.0, 0.0, 0.0,
                           0.0, c->dsc + DS_ETA);
        update_c(c, true);
        res64(c);
        c->lev[0].has_F = false;
        chk(c);
        return;
    }
    (void)hipMemcpyAsync(c->prev64, c->phi64, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s);
    vcycle_from(c, 0);
    hipLaunchKernelGGL(k_copy32to64, g, dim3(256), 0, c->s, L0.P[0], L0.prm, c->phi64, c->n, c->m);
    refresh_and_residual(c);
    hipLaunchKernelGGL(k_eta, dim3(nb), dim3(256), 0, c->s, c->phi64, c->prev64, (long long)N, c->part + 4 * RED_BLOCKS);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part + 4 * RED_BLOCKS, nb, 3, 0.0, 0.0, 0.0, 0.0,
                       c->dsc + DS_ETA);
    chk(c);
}

// Every step of a cycle runs without host synchronisation, so the whole
// cycle can be captured.  Event timing and MGSEG_GRAPH=0 in the environment
// keep the eager launches.
bool graph_usable(const mgseg_ctx *c)
{
    if (c->prof_on || c->graph_failed || c->noalloc || !c->sched.graph) return false;
    const char *env = std::getenv("MGSEG_GRAPH");
    if (env && env[0] == '0') return false;
    return true;
}

// capture enqueue_cycle on a private stream, instantiate once
bool build_graph(mgseg_ctx *c)
{
    if (!c->cap && hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    hipStream_t user = c->s;
    c->s = c->cap;
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
        enqueue_cycle(c);
        ok = hipStreamEndCapture(c->cap, &g) == hipSuccess && g != nullptr && c->err == hipSuccess;
    }
    c->s = user;
    if (ok) ok = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    if (!ok) {
        c->gexec = nullptr;
        (void)hipGetLastError();
        c->err = hipSuccess;
    }
    return ok;
}

// enqueue one cycle and the copy of its residual norm and eta to pinned host
// memory; cycle_end reads them after the stream has been synchronised
void cycle_begin(mgseg_ctx *c)
{
    bool launched = false;
    if (graph_usable(c)) {
        if (!c->gexec && !build_graph(c)) c->graph_failed = true;
        if (c->gexec) {
            if (hipGraphLaunch(c->gexec, c->s) == hipSuccess) launched = true;
            else { (void)hipGetLastError(); c->graph_failed = true; }
        }
    }
    if (!launched) enqueue_cycle(c);
    (void)hipMemcpyAsync(c->hres, c->dsc + DS_RES, 3 * sizeof(double), hipMemcpyDeviceToHost, c->s);
    chk(c);
}

mgseg_status cycle_end(mgseg_ctx *c, double *rel_out)
{
    if (c->err != hipSuccess) return MGSEG_E_HIP;
    const double res = c->hres[0];
    c->eta = c->hres[1];
    c->res = res;
    c->res_rows = c->hres[2];
    c->cycles++;
    c->rel = c->res0 > 0.0 ? res / c->res0 : 0.0;
    if (rel_out) *rel_out = c->rel;
    if (!std::isfinite(res)) return MGSEG_E_NONFINITE;
    return MGSEG_OK;
}

mgseg_status one_cycle(mgseg_ctx *c, double *rel_out)
{
    cycle_begin(c);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    return cycle_end(c, rel_out);
}

}  // namespace

namespace {

// frees what a context owns (not the context itself)
void release_ctx(mgseg_ctx *c)
{
    if (c->s) (void)hipStreamSynchronize(c->s);
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->hres && c->hres != c->hres_local) (void)hipHostFree(c->hres);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->arena && c->arena_owned) (void)hipFree(c->arena);
    if (c->pred) (void)hipFree(c->pred);
    if (c->aos) (void)hipFree(c->aos);
    if (c->lfa) (void)hipFree(c->lfa);
}

// argument checks of a setup and the kernels' LDS attributes; Lv: the grid count
mgseg_status setup_check(const float *image_dev, int n, int m, int pitch, const float *markers_host, int k,
                         const mgseg_params *p, int &Lv)
{
    if (!image_dev || !markers_host || !p || k < 1 || k > 64 || n < 2 || m < 2 || pitch < m) return MGSEG_E_ARG;
    if (p->struct_size != sizeof(mgseg_params)) return MGSEG_E_ARG;
    if (p->model == MGSEG_RADA_CHEN && k < 3) return MGSEG_E_ARG;   // the marker polygon needs an area (A1 > 0)
    if (p->nu1 < 0 || p->nu2 < 0 || p->coarse_iters < 0 || !(p->coarse_rtol >= 0.0) || !(p->M > 0.0) || !(p->eps > 0.0) || p->levels < 0 ||
        p->levels > MAXLEV || p->smoother < 0 || p->smoother > 7 || (p->smoother >= 2 && p->smoother != 4 && !p->mixed_precision) ||
        (p->smoother >= 5 && p->model != MGSEG_SPENCER_CHEN) ||
        ((p->smoother == 2 || p->smoother == 3 || p->smoother == 6) && n > 1024) ||   // one workgroup per column system
        p->run_max < 0 ||
        !(p->sigma_g >= 0.0 && p->sigma_g <= 16.0))
        return MGSEG_E_ARG;
    for (int t = 0; t < 2 * k; t++)
        if (!std::isfinite(markers_host[t])) return MGSEG_E_ARG;
    for (int t = 0; t < k; t++)
        if (!(markers_host[2 * t] >= 0.0f && markers_host[2 * t] < (float)n && markers_host[2 * t + 1] >= 0.0f &&
              markers_host[2 * t + 1] < (float)m))
            return MGSEG_E_ARG;
    Lv = p->levels;
    if (Lv == 0) {
        Lv = 1;
        while (Lv < MAXLEV && n % (1 << Lv) == 0 && m % (1 << Lv) == 0 && std::min(n, m) >> Lv >= 4) Lv++;
    }
    int div = 1 << (Lv - 1);
    if (n % div || m % div) return MGSEG_E_SHAPE;
    if (n > 8192 || m > 8192) return MGSEG_E_SHAPE;
    // lines longer than one workgroup keep the band's previous and recomputed
    // lines in LDS: the device must allow that much per workgroup
    if (std::max(n, m) > 1024) {
        const size_t need = long_lds_bytes<LONG_NT>(std::max(n, m));   // dynamic; the wave totals are static
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            return MGSEG_E_HIP;
        if (need + 2 * (LONG_NT / 64) * sizeof(Ramp) > (size_t)lds_max) return MGSEG_E_SHAPE;
        const void *fns[4] = {reinterpret_cast<const void *>(&k_sweep_long<LONG_NT, false, false>),
                              reinterpret_cast<const void *>(&k_sweep_long<LONG_NT, true, false>),
                              reinterpret_cast<const void *>(&k_sweep_long<LONG_NT, false, true>),
                              reinterpret_cast<const void *>(&k_sweep_long<LONG_NT, true, true>)};
        for (const void *fn : fns)
            if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need) != hipSuccess)
                return MGSEG_E_HIP;
    }

    // the one-workgroup smoother (coarsest solve, small grids) stages its level in LDS (up to
    // CO_MAX_CELLS cells)
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_coarse_smooth<64>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)coarse_lds_bytes(CO_MAX_CELLS, 1)) !=
            hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void *>(&k_coarse_smooth<512>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)coarse_lds_bytes(CO_MAX_CELLS, 1)) !=
            hipSuccess)
        return MGSEG_E_HIP;
    return MGSEG_OK;
}

// builds the context c (constructed by the caller) for one image: the arena is
// allocated, or (ext non-null) the caller's memory of ext_cap bytes
mgseg_status setup_into(mgseg_ctx *c, const float *image_dev, int n, int m, int pitch, const float *markers_host,
                        int k, const mgseg_params *p, void *stream, int Lv, char *ext, size_t ext_cap)
{
    c->p = *p; c->p.levels = Lv;
    c->s = (hipStream_t)stream;
    c->L = Lv; c->n = n; c->m = m;
    c->h0 = 1.0 / std::sqrt((double)n * (double)m);
    size_t N = (size_t)n * m;
    // Gaussian kernel of the image smoothing
    int R = (int)std::ceil(4.0 * p->sigma_g);
    double ker[2 * 64 + 1];
    double ks = 0.0;
    for (int t = -R; t <= R; t++) {
        double v = p->sigma_g > 0 ? std::exp(-(double)(t * t) / (2.0 * p->sigma_g * p->sigma_g)) : (t == 0);
        ker[t + R] = v; ks += v;
    }
    for (int t = 0; t <= 2 * R; t++) ker[t] /= ks;
    double *zb = nullptr, *t64 = nullptr, *ker_d = nullptr;
    // the allocation sequence: sizing pass, then the pieces of the arena
    auto carve = [&]() {
        c->arena_used = 0;
        for (int l = 0; l < Lv; l++) {
            Level &L = c->lev[l];
            L.n = n >> l; L.m = m >> l; L.h = c->h0 * (double)(1 << l);
            L.prm = pad64(L.m); L.pcm = pad64(L.n);
            size_t Nr = (size_t)L.n * L.prm, Nc = (size_t)L.m * L.pcm;
            L.z = dalloc<float>(c, Nr); L.d = dalloc<float>(c, Nr); L.w = dalloc<float>(c, Nr);
            L.fit = dalloc<float>(c, Nr); L.F = dalloc<float>(c, Nr);
            for (int t = 0; t < 3; t++) { L.P[t] = dalloc<float>(c, Nr); L.T[t] = dalloc<float>(c, Nc); }
            L.psi = dalloc<float>(c, Nr); L.psi_cm = dalloc<float>(c, Nc);
            L.phic = dalloc<float>(c, Nr); L.r = dalloc<float>(c, Nr); L.G = dalloc<float>(c, Nr);
            L.lo = dalloc<float>(c, Nr); L.hi = dalloc<float>(c, Nr);
            L.w_cm = dalloc<float>(c, Nc); L.fit_cm = dalloc<float>(c, Nc); L.F_cm = dalloc<float>(c, Nc);
            L.lo_cm = dalloc<float>(c, Nc); L.hi_cm = dalloc<float>(c, Nc);
            L.lab = dalloc<uint8_t>(c, Nr); L.lab_cm = dalloc<uint8_t>(c, Nc);
            if (p->mixed_precision) { L.cf = dalloc<float4>(c, Nr); L.cf_cm = dalloc<float4>(c, Nc); }
        }
        c->phi64 = dalloc<double>(c, N); c->w64 = dalloc<double>(c, N); c->d64 = dalloc<double>(c, N);
        c->g64 = dalloc<double>(c, N); c->prev64 = dalloc<double>(c, N); c->phi0m = dalloc<double>(c, N);
        c->dsc = dalloc<double>(c, DS_COUNT);
        c->part_n = 8 * RED_BLOCKS + 2 * (int)((N + 255) / 256) + n + 16;
        c->part = dalloc<double>(c, (size_t)c->part_n);
        {
            const Level &Lc = c->lev[Lv - 1];
            c->co_prev = dalloc<float>(c, (size_t)Lc.n * Lc.prm);
            c->co_entry = dalloc<float>(c, (size_t)Lc.n * Lc.prm);
        }
        c->flags = dalloc<int>(c, 4);
        zb = dalloc<double>(c, N); t64 = dalloc<double>(c, N);
        c->mk_d = dalloc<double>(c, 2 * (size_t)k);
        c->hull_d = dalloc<double>(c, 10 * (size_t)k + 10);
        ker_d = dalloc<double>(c, 2 * (size_t)R + 1);
    };
    carve();
    c->arena_size = c->arena_used;
    if (ext) {
        // the caller's memory (the static scratch): no allocation
        if (c->arena_size > ext_cap) return MGSEG_E_SCRATCH;
        c->arena = ext;
        c->arena_owned = false;
        c->noalloc = true;
        c->hres = c->hres_local;
    } else {
        if (hipMalloc((void **)&c->arena, c->arena_size) != hipSuccess) {
            (void)hipGetLastError();
            c->arena = nullptr;
            return MGSEG_E_NOMEM;
        }
        if (hipHostMalloc((void **)&c->hres, 3 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->hres = nullptr;
            c->oom = true;
        }
    }
    carve();
    (void)hipMemsetAsync(c->arena, 0, c->arena_size, c->s);
    if (c->oom) return MGSEG_E_NOMEM;

    // markers and their convex hull (host arrays live until the stream is synchronised below)
    double mk[128], hull[128], geo[640];
    for (int t = 0; t < 2 * k; t++) mk[t] = markers_host[t];
    c->k = k;
    c->hv = host_hull(mk, k, hull);
    c->A1 = host_area(hull, c->hv) * c->h0 * c->h0;
    int ne = 0, closed = 0;
    const int ng = hull_geometry(hull, c->hv, geo, ne, closed);
    (void)hipMemcpyAsync(c->mk_d, mk, sizeof(double) * 2 * k, hipMemcpyHostToDevice, c->s);
    if (ng > 0) (void)hipMemcpyAsync(c->hull_d, geo, sizeof(double) * ng, hipMemcpyHostToDevice, c->s);
    (void)hipMemcpyAsync(ker_d, ker, sizeof(double) * (2 * R + 1), hipMemcpyHostToDevice, c->s);

    Level &L0 = c->lev[0];
    dim3 g = grid2(n, m);
    hipLaunchKernelGGL(k_blur_rows, g, dim3(256), 0, c->s, image_dev, pitch, t64, n, m, ker_d, R);
    hipLaunchKernelGGL(k_blur_cols, g, dim3(256), 0, c->s, t64, zb, n, m, ker_d, R);
    const dim3 gt((m + TILE - 1) / TILE, (n + TILE - 1) / TILE);
    hipLaunchKernelGGL(k_edge_detector, gt, dim3(256), 0, c->s, zb, n, m, p->beta, c->g64);
    MarkerArgs S;
    S.mk = c->mk_d; S.k = k;
    S.edge = reinterpret_cast<const HullEdge *>(c->hull_d); S.ne = ne;
    S.vtx = c->hull_d + 8 * (size_t)ne; S.nv = c->hv; S.closed = closed;
    S.h0 = c->h0; S.sigma_d = p->sigma_d; S.M = p->M; S.model = p->model; S.n = n; S.m = m;
    S.g64 = c->g64; S.z = image_dev; S.pz = pitch;
    S.d64 = c->d64; S.w64 = c->w64; S.phi64 = c->phi64;
    S.w32 = L0.w; S.d32 = L0.d; S.z32 = L0.z; S.phi32 = L0.P[0]; S.p32 = L0.prm;
    hipLaunchKernelGGL(k_marker_maps, g, dim3(256), 0, c->s, S);
    for (int l = 1; l < Lv; l++) {
        Level &Lf = c->lev[l - 1], &Lc = c->lev[l];
        dim3 gc = grid2(Lc.n, Lc.m);
        hipLaunchKernelGGL(k_restrict, gc, dim3(256), 0, c->s, Lf.z, Lf.prm, Lc.z, Lc.prm, Lc.n, Lc.m);
        hipLaunchKernelGGL(k_restrict, gc, dim3(256), 0, c->s, Lf.d, Lf.prm, Lc.d, Lc.prm, Lc.n, Lc.m);
        hipLaunchKernelGGL(k_restrict, gc, dim3(256), 0, c->s, Lf.w, Lf.prm, Lc.w, Lc.prm, Lc.n, Lc.m);
    }
    for (int l = 0; l < Lv; l++) {
        Level &L = c->lev[l];
        transpose_f(c, L.w, L.prm, L.w_cm, L.pcm, L.n, L.m);
    }
    (void)hipMemcpyAsync(c->phi0m, c->phi64, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s);
    chk(c);
    refresh_and_residual(c);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->res0 = read_scalar(c, DS_RES);
    c->res0_rows = read_scalar(c, DS_RESR);
    c->res_rows = c->res0_rows;
    c->res = c->res0;
    c->rel = 1.0;
    return MGSEG_OK;
}


}  // namespace

// ==========================================================================
extern "C" {

void mgseg_params_default(mgseg_params *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(mgseg_params);
    p->model = MGSEG_SPENCER_CHEN;
    p->mu = 0.5; p->lambda1 = 6.5025; p->lambda2 = 6.5025; p->theta = 4.0; p->nu = 1.0;
    p->eps = 1.0; p->eps_tv_px = 1.0; p->beta = 16384.0; p->sigma_g = 1.0; p->sigma_d = 0.1;
    p->Sigma = 2.0; p->M = 4.0; p->nu1 = 2; p->nu2 = 2; p->levels = 0; p->coarse_iters = 10;
    p->mixed_precision = 1; p->scaled = 1; p->coarse_rtol = 1e-4; p->smoother = 0; p->run_max = 0;
}

const char *mgseg_strerror(mgseg_status s)
{
    switch (s) {
    case MGSEG_OK: return "ok";
    case MGSEG_E_SCRATCH: return "image too large for the no-allocation scratch (MGSEG_NOALLOC_BYTES)";
    case MGSEG_E_ARG: return "invalid argument";
    case MGSEG_E_SHAPE: return "image shape not divisible by 2^(levels-1)";
    case MGSEG_E_NOMEM: return "device allocation failed";
    case MGSEG_E_HIP: return "HIP runtime error";
    case MGSEG_E_NONFINITE: return "non-finite residual";
    case MGSEG_E_NOT_CONVERGED: return "not converged within max_cycles";
    case MGSEG_E_STATE: return "invalid state";
    }
    return "unknown status";
}

void mgseg_destroy(mgseg_ctx *c)
{
    if (!c) return;
    release_ctx(c);
    delete c;
}

mgseg_status mgseg_setup(const float *image_dev, int n, int m, int pitch, const float *markers_host, int k,
                         const mgseg_params *p, void *stream, mgseg_ctx **out)
{
    if (!out) return MGSEG_E_ARG;
    *out = nullptr;
    int Lv = 0;
    const mgseg_status ck = setup_check(image_dev, n, m, pitch, markers_host, k, p, Lv);
    if (ck != MGSEG_OK) return ck;
    mgseg_ctx *c = new (std::nothrow) mgseg_ctx();
    if (!c) return MGSEG_E_NOMEM;
    const mgseg_status st = setup_into(c, image_dev, n, m, pitch, markers_host, k, p, stream, Lv, nullptr, 0);
    if (st != MGSEG_OK) { mgseg_destroy(c); return st; }
    *out = c;
    return MGSEG_OK;
}

}  // extern "C"

// --------------------------------------------------------------------------
// The no-allocation entry point's scratch: every device array of one solve
// (the context's arena), MGSEG_NOALLOC_BYTES on each device the library runs
// on, held until the process ends.  Host code reaches it only through the
// address hipGetSymbolAddress gives on that device (the array's name is a
// host-side stand-in).
static __device__ __align__(256) char scratch[MGSEG_NOALLOC_BYTES];

namespace {
std::mutex g_scratch_mu;
char *g_scratch_dev[64] = {};

// the current device's copy of the scratch (looked up once per device)
mgseg_status scratch_address(char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MGSEG_E_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return MGSEG_E_HIP;
        }
        g_scratch_dev[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_dev[dev];
    return MGSEG_OK;
}
}  // namespace

extern "C" {

mgseg_status mgseg_solve_noalloc(const float *image_dev, int n, int m, int pitch, const float *markers_host, int k,
                                 const mgseg_params *p, void *stream, double tol, int max_cycles, double *phi_dev,
                                 int phi_pitch, int *cycles_out, double *rel_res_out)
{
    if (!phi_dev || phi_pitch < m || !(tol > 0.0) || max_cycles < 1) return MGSEG_E_ARG;
    int Lv = 0;
    mgseg_status st = setup_check(image_dev, n, m, pitch, markers_host, k, p, Lv);
    if (st != MGSEG_OK) return st;
    char *buf = nullptr;
    st = scratch_address(&buf);
    if (st != MGSEG_OK) return st;
    mgseg_ctx c;
    st = setup_into(&c, image_dev, n, m, pitch, markers_host, k, p, stream, Lv, buf, MGSEG_NOALLOC_BYTES);
    if (st == MGSEG_OK) {
        st = mgseg_solve(&c, tol, max_cycles, cycles_out, rel_res_out);
        if (st == MGSEG_OK || st == MGSEG_E_NOT_CONVERGED) {
            const mgseg_status sg = mgseg_get_phi(&c, phi_dev, phi_pitch);
            if (sg != MGSEG_OK) st = sg;
        }
    }
    release_ctx(&c);
    return st;
}

mgseg_status mgseg_set_phi0(mgseg_ctx *c, const float *phi_dev, int pitch)
{
    if (!c || !phi_dev || pitch < c->m) return MGSEG_E_ARG;
    Level &L0 = c->lev[0];
    hipLaunchKernelGGL(k_set_phi0, grid2(c->n, c->m), dim3(256), 0, c->s, phi_dev, pitch, c->p.M, c->phi64,
                       L0.P[0], L0.prm, c->n, c->m);
    refresh_and_residual(c);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->res0 = read_scalar(c, DS_RES);
    c->res0_rows = read_scalar(c, DS_RESR);
    c->res_rows = c->res0_rows;
    c->res = c->res0; c->rel = 1.0; c->cycles = 0;
    return MGSEG_OK;
}

mgseg_status mgseg_vcycle(mgseg_ctx *c, double *rel_res_out)
{
    if (!c) return MGSEG_E_ARG;
    return one_cycle(c, rel_res_out);
}

mgseg_status mgseg_solve(mgseg_ctx *c, double tol, int max_cycles, int *cycles_out, double *rel_res_out)
{
    if (!c || !(tol > 0.0) || max_cycles < 0) return MGSEG_E_ARG;
    int done = 0;
    double rel = c->rel;
    mgseg_status st = MGSEG_OK;
    while (done < max_cycles && !(rel <= tol)) {
        st = one_cycle(c, &rel);
        done++;
        if (st != MGSEG_OK) break;
    }
    if (cycles_out) *cycles_out = done;
    if (rel_res_out) *rel_res_out = rel;
    if (st != MGSEG_OK) return st;
    return rel <= tol ? MGSEG_OK : MGSEG_E_NOT_CONVERGED;
}

mgseg_status mgseg_get_phi(mgseg_ctx *c, double *phi_dev, int pitch)
{
    if (!c || !phi_dev || pitch < c->m) return MGSEG_E_ARG;
    hipLaunchKernelGGL(k_out_phi, grid2(c->n, c->m), dim3(256), 0, c->s, c->phi64, c->n, c->m, phi_dev, pitch);
    chk(c);
    return sync_status(c);
}

mgseg_status mgseg_get_mask(mgseg_ctx *c, uint8_t *mask_dev, int pitch)
{
    if (!c || !mask_dev || pitch < c->m) return MGSEG_E_ARG;
    hipLaunchKernelGGL(k_out_mask, grid2(c->n, c->m), dim3(256), 0, c->s, c->phi64, c->n, c->m, mask_dev, pitch);
    chk(c);
    return sync_status(c);
}

namespace {

// one AOS step of the finest FP64 phi (time step tau_hat h / mu), then c1, c2
// and the relative change of phi (DS_ETA)
void aos_step(mgseg_ctx *c, double tau_hat)
{
    Level &L = c->lev[0];
    const long long N = (long long)c->n * c->m;
    double *uA = c->aos, *uB = uA + N, *uC = uB + N, *uD = uC + N, *r = uD + N, *y1 = r + N;
    (void)hipMemcpyAsync(c->prev64, c->phi64, sizeof(double) * N, hipMemcpyDeviceToDevice, c->s);
    const int nb = std::min(RED_BLOCKS, std::max(1, (int)((N + 255) / 256)));
    if (c->p.model == 1) {
        hipLaunchKernelGGL(k_sums<double>, dim3(nb), dim3(256), 0, c->s, c->phi64, c->m, (const float *)nullptr, 0,
                           c->n, c->m, c->p.eps, c->part);
        hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part, nb, 0, (double)N, L.h * L.h, c->A1,
                           c->p.nu, c->dsc + DS_AREA64);
    }
    AosArgs A;
    A.phi64 = c->phi64; A.w64 = c->w64; A.d64 = c->d64; A.z32 = L.z; A.p32 = L.prm;
    A.c12 = c->dsc + DS_C1; A.area = c->p.model == 1 ? c->dsc + DS_AREA64 : nullptr;
    A.kap = c->p.mu / L.h; A.e2 = lev_e2(c, 0); A.eps = c->p.eps;
    A.l1 = c->p.lambda1; A.l2 = c->p.lambda2; A.theta = c->p.theta; A.tau = tau_hat * L.h / c->p.mu;
    A.model = c->p.model; A.scaled = c->p.scaled; A.n = c->n; A.m = c->m;
    A.uA = uA; A.uB = uB; A.uC = uC; A.uD = uD; A.r = r;
    hipLaunchKernelGGL(k_aos_coef, grid2(c->n, c->m), dim3(256), 0, c->s, A);
    // columns: m lines of n cells (stride m), y_1 to its own plane; rows: n lines of m cells
    // (contiguous), y_2 over uA (free once the columns are done)
    hipLaunchKernelGGL(k_aos_lines<8>, dim3((c->m + 3) / 4), dim3(256), 0, c->s, uA, uB, r, y1, c->m, c->n, 1LL,
                       (long long)c->m);
    hipLaunchKernelGGL(k_aos_lines<8>, dim3((c->n + 3) / 4), dim3(256), 0, c->s, uC, uD, r, uA, c->n, c->m,
                       (long long)c->m, 1LL);
    hipLaunchKernelGGL(k_aos_combine, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, c->s, c->phi64, y1, uA, N,
                       c->p.M);
    update_c(c);
    hipLaunchKernelGGL(k_eta, dim3(nb), dim3(256), 0, c->s, c->phi64, c->prev64, N, c->part + 4 * RED_BLOCKS);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_NT), 0, c->s, c->part + 4 * RED_BLOCKS, nb, 3, 0.0, 0.0, 0.0, 0.0,
                       c->dsc + DS_ETA);
    chk(c);
}

}  // namespace

mgseg_status mgseg_aos(mgseg_ctx *c, double tau, double eta_tol, int max_iters, int *iters_out, double *eta_out,
                       double *rel_res_out)
{
    if (!c || !(tau > 0.0) || !(eta_tol >= 0.0) || max_iters < 0) return MGSEG_E_ARG;
    if (c->noalloc) return MGSEG_E_ARG;
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    const size_t N = (size_t)c->n * c->m;
    if (!c->aos && hipMalloc(&c->aos, 6 * N * sizeof(double)) != hipSuccess) {
        c->aos = nullptr;
        (void)hipGetLastError();
        return MGSEG_E_NOMEM;
    }
    int done = 0;
    double eta = 0.0;
    while (done < max_iters) {
        aos_step(c, tau);
        (void)hipMemcpyAsync(c->hres, c->dsc + DS_RES, 3 * sizeof(double), hipMemcpyDeviceToHost, c->s);
        st = sync_status(c);
        if (st != MGSEG_OK) return st;
        eta = c->hres[1];
        done++;
        if (!std::isfinite(eta)) return MGSEG_E_NONFINITE;
        if (eta < eta_tol) break;
    }
    // the paper's residual at the result, and the FP32 / deviation-form state of the multigrid
    refresh_and_residual(c);
    (void)hipMemcpyAsync(c->hres, c->dsc + DS_RES, 3 * sizeof(double), hipMemcpyDeviceToHost, c->s);
    st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->res = c->hres[0];
    c->res_rows = c->hres[2];
    c->eta = eta;
    c->rel = c->res0 > 0.0 ? c->res / c->res0 : 0.0;
    if (iters_out) *iters_out = done;
    if (eta_out) *eta_out = eta;
    if (rel_res_out) *rel_res_out = c->rel;
    if (!std::isfinite(c->res)) return MGSEG_E_NONFINITE;
    return done > 0 && eta < eta_tol ? MGSEG_OK : MGSEG_E_NOT_CONVERGED;
}

mgseg_status mgseg_smoothing_rates(mgseg_ctx *c, int smoother, double *out5, float *mu_dev, int mu_pitch)
{
    if (!c || !out5 || (smoother != 0 && smoother != 1 && smoother != 3 && smoother != 4)) return MGSEG_E_ARG;
    if (mu_dev && mu_pitch < c->m) return MGSEG_E_ARG;
    if (c->noalloc) return MGSEG_E_ARG;
    Level &L0 = c->lev[0];
    if (!devm(c) || !L0.cf) return MGSEG_E_STATE;
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    const long long N = (long long)c->n * c->m;
    const int nb = (int)((N + LFA_NB - 1) / LFA_NB);
    if (!c->lfa && hipMalloc(&c->lfa, (5 * (size_t)nb + 5) * sizeof(double)) != hipSuccess) {
        c->lfa = nullptr;
        (void)hipGetLastError();
        return MGSEG_E_NOMEM;
    }
    // the frozen couplings at the current finest phi (the deviation restarted from it)
    const dim3 gt((c->m + TILE - 1) / TILE, (c->n + TILE - 1) / TILE);
    const dim3 tb(TILE, tile_rows((long long)gt.x * gt.y));
    hipLaunchKernelGGL(k_start0, gt, tb, 0, c->s, c->phi64, c->n, c->m, c->p.M, L0.P[0], L0.lo, L0.hi, L0.prm,
                       L0.lo_cm, L0.hi_cm, L0.pcm);
    freeze(c, 0);
    const float *qd = nullptr;
    if (smoother == 4 && c->p.model == 1) {
        hipLaunchKernelGGL(k_newton_diag<double>, grid2(L0.n, L0.m), dim3(256), 0, c->s, c->phi64, c->m, L0.P[0],
                           L0.prm, L0.n, L0.m, 2.0 * c->p.nu * L0.h * L0.h, c->p.eps, c->p.scaled,
                           c->dsc + DS_AREA_FRZ, L0.r);
        qd = L0.r;
    }
    LfaArgs A;
    A.cf = L0.cf; A.qd = qd; A.lab = L0.lab; A.p = L0.prm; A.n = c->n; A.m = c->m;
    A.mode = smoother == 0 ? 2 : (smoother == 3 ? 1 : 0);
    A.mu = mu_dev; A.mp = mu_pitch; A.partial = c->lfa;
    hipLaunchKernelGGL(k_lfa_rates, dim3(nb), dim3(LFA_NB), 0, c->s, A);
    hipLaunchKernelGGL(k_lfa_final, dim3(1), dim3(64), 0, c->s, c->lfa, nb, c->lfa + 5 * (size_t)nb);
    double r[5];
    (void)hipMemcpyAsync(r, c->lfa + 5 * (size_t)nb, sizeof(r), hipMemcpyDeviceToHost, c->s);
    st = sync_status(c);
    if (st != MGSEG_OK) return st;
    out5[0] = r[0];
    out5[1] = r[1] / (double)N;
    out5[2] = r[2];
    out5[3] = r[4] > 0.0 ? r[3] / r[4] : 0.0;
    out5[4] = r[4] / (double)N;
    return MGSEG_OK;
}

mgseg_status mgseg_get_stats(mgseg_ctx *c, mgseg_stats *s)
{
    if (!c || !s) return MGSEG_E_ARG;
    Level &L0 = c->lev[0];
    const size_t N = (size_t)c->n * c->m;
    const int nb = std::min(RED_BLOCKS, std::max(1, (int)((N + 255) / 256)));
    EnergyArgs E;
    E.phi = c->phi64; E.g = c->g64; E.d = c->d64; E.dsc = c->dsc + DS_C1; E.z = L0.z; E.pz = L0.prm;
    E.n = c->n; E.m = c->m; E.model = c->p.model; E.h = c->h0; E.mu = c->p.mu; E.lambda1 = c->p.lambda1;
    E.lambda2 = c->p.lambda2; E.theta = c->p.theta; E.eps = c->p.eps; E.partial = c->part;
    const dim3 ge((c->m + TILE - 1) / TILE, (c->n + TILE - 1) / TILE);
    const int nbe = (int)(ge.x * ge.y);
    hipLaunchKernelGGL(k_energy, ge, dim3(256), 0, c->s, E);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, c->s, c->part, nbe, c->h0 * c->h0, (double)N, c->p.model,
                       c->p.nu, c->A1, c->dsc + DS_ENERGY);
    hipLaunchKernelGGL(k_count_labels, dim3(nb), dim3(256), 0, c->s, L0.lab, L0.prm, c->n, c->m, c->part + 2 * RED_BLOCKS);
    chk(c);
    double c12[2] = {0, 0}, en = 0.0;
    std::vector<double> cnt(nb);
    (void)hipMemcpyAsync(c12, c->dsc + DS_C1, sizeof(c12), hipMemcpyDeviceToHost, c->s);
    (void)hipMemcpyAsync(&en, c->dsc + DS_ENERGY, sizeof(double), hipMemcpyDeviceToHost, c->s);
    (void)hipMemcpyAsync(cnt.data(), c->part + 2 * RED_BLOCKS, sizeof(double) * nb, hipMemcpyDeviceToHost, c->s);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    std::vector<double> ph(N);
    (void)hipMemcpy(ph.data(), c->phi64, sizeof(double) * ph.size(), hipMemcpyDeviceToHost);
    size_t fg = 0;
    for (double v : ph) fg += v > 0.0;
    double nd = 0.0;
    for (double v : cnt) nd += v;
    s->c1 = c12[0]; s->c2 = c12[1]; s->rel_res = c->rel; s->res = c->res; s->res0 = c->res0;
    s->res_rows = c->res_rows; s->res0_rows = c->res0_rows;
    s->rel_res_rows = c->res0_rows > 0.0 ? c->res_rows / c->res0_rows : 0.0;
    s->eta = c->eta; s->cycles = c->cycles; s->levels = c->L;
    s->frac_fg = ph.empty() ? 0.0 : (double)fg / (double)ph.size();
    s->energy = en;
    s->frac_D = N ? nd / (double)N : 0.0;
    return MGSEG_OK;
}

namespace {
struct StateHeader {
    uint64_t magic;
    int32_t n, m, levels, cycles;
    double res0, res, rel, eta;
    double res0_rows;
};
static_assert(sizeof(StateHeader) == 64, "state header is 64 bytes");
constexpr uint64_t STATE_MAGIC = 0x3254535347534d47ull;   // "GMSGSST2"
}  // namespace

mgseg_status mgseg_get_state(mgseg_ctx *c, void *blob, size_t *bytes)
{
    if (!c || !bytes) return MGSEG_E_ARG;
    const size_t N = (size_t)c->n * c->m, need = sizeof(StateHeader) + sizeof(double) * N;
    if (!blob) { *bytes = need; return MGSEG_OK; }
    if (*bytes < need) { *bytes = need; return MGSEG_E_ARG; }
    StateHeader h{STATE_MAGIC, c->n, c->m, c->L, c->cycles, c->res0, c->res, c->rel, c->eta, c->res0_rows};
    std::memcpy(blob, &h, sizeof(h));
    (void)hipMemcpyAsync(static_cast<char *>(blob) + sizeof(h), c->phi64, sizeof(double) * N, hipMemcpyDeviceToHost,
                         c->s);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    *bytes = need;
    return MGSEG_OK;
}

mgseg_status mgseg_set_state(mgseg_ctx *c, const void *blob, size_t bytes)
{
    if (!c || !blob || bytes < sizeof(StateHeader)) return MGSEG_E_ARG;
    StateHeader h;
    std::memcpy(&h, blob, sizeof(h));
    if (h.magic != STATE_MAGIC) return MGSEG_E_ARG;
    if (h.n != c->n || h.m != c->m || h.levels != c->L) return MGSEG_E_SHAPE;
    const size_t N = (size_t)c->n * c->m;
    if (bytes < sizeof(h) + sizeof(double) * N || h.cycles < 0) return MGSEG_E_ARG;
    Level &L0 = c->lev[0];
    (void)hipMemcpyAsync(c->phi64, static_cast<const char *>(blob) + sizeof(h), sizeof(double) * N,
                         hipMemcpyHostToDevice, c->s);
    hipLaunchKernelGGL(k_copy64to32, grid2(c->n, c->m), dim3(256), 0, c->s, c->phi64, c->n, c->m, L0.P[0], L0.prm);
    refresh_and_residual(c);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->res0 = h.res0; c->res = h.res; c->rel = h.rel; c->eta = h.eta; c->cycles = h.cycles;
    c->res0_rows = h.res0_rows; c->res_rows = read_scalar(c, DS_RESR);
    return MGSEG_OK;
}

mgseg_status mgseg_get_schedule(mgseg_ctx *c, mgseg_schedule *out)
{
    if (!c || !out) return MGSEG_E_ARG;
    *out = c->sched;
    return MGSEG_OK;
}

mgseg_status mgseg_set_schedule(mgseg_ctx *c, const mgseg_schedule *sc)
{
    if (!c || !sc || sc->lds_side < 0 || sc->line_threads < 0 || sc->line_threads > 1 || sc->graph < 0 ||
        sc->graph > 1 || sc->split_long < 0 || sc->split_long > 1)
        return MGSEG_E_ARG;
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    const bool relaunch = sc->lds_side != c->sched.lds_side || sc->line_threads != c->sched.line_threads ||
                          sc->split_long != c->sched.split_long;
    c->sched = *sc;
    // a captured cycle holds the old launches
    if (relaunch && c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    return MGSEG_OK;
}

mgseg_status mgseg_tune(mgseg_ctx *c, int trial_cycles, mgseg_schedule *best_out, double *ms_per_cycle_out)
{
    if (!c || trial_cycles < 1) return MGSEG_E_ARG;
    size_t bytes = 0;
    mgseg_status st = mgseg_get_state(c, nullptr, &bytes);
    if (st != MGSEG_OK) return st;
    std::vector<char> saved(bytes);
    st = mgseg_get_state(c, saved.data(), &bytes);
    if (st != MGSEG_OK) return st;
    const mgseg_schedule start = c->sched;
    mgseg_schedule best = start;
    double best_ms = 1e300;
    const int sides[] = {0, 16, 32, 64};
    const bool has_long = c->n > 512 || c->m > 512;
    std::vector<mgseg_schedule> cands;
    for (int side : sides)
        for (int lt = 0; lt <= 1; lt++)
            for (int g = 0; g <= 1; g++)
                for (int sp = 0; sp <= (has_long ? 1 : 0); sp++) cands.push_back(mgseg_schedule{side, lt, g, sp});
    for (const mgseg_schedule &cand : cands) {
        st = mgseg_set_schedule(c, &cand);
        if (st == MGSEG_OK) st = mgseg_set_state(c, saved.data(), bytes);
        double rel = 0.0;
        if (st == MGSEG_OK) st = one_cycle(c, &rel);    // untimed: the capture of a graph
        if (st != MGSEG_OK && st != MGSEG_E_NONFINITE) break;
        auto t0 = std::chrono::steady_clock::now();
        for (int k = 0; k < trial_cycles && st == MGSEG_OK; k++) st = one_cycle(c, &rel);
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / trial_cycles;
        if (st == MGSEG_OK && ms < best_ms) { best_ms = ms; best = cand; }
        if (st != MGSEG_OK && st != MGSEG_E_NONFINITE) break;
    }
    // the solve continues from where it stood, with the fastest schedule
    mgseg_status st2 = mgseg_set_schedule(c, best_ms < 1e300 ? &best : &start);
    if (st2 == MGSEG_OK) st2 = mgseg_set_state(c, saved.data(), bytes);
    if (best_out) *best_out = c->sched;
    if (ms_per_cycle_out) *ms_per_cycle_out = best_ms;
    if (st != MGSEG_OK && st != MGSEG_E_NONFINITE) return st;
    return st2;
}

mgseg_status mgseg_level_shape(mgseg_ctx *c, int level, int *n, int *m, double *h)
{
    if (!c || level < 0 || level >= c->L) return MGSEG_E_ARG;
    if (n) *n = c->lev[level].n;
    if (m) *m = c->lev[level].m;
    if (h) *h = c->lev[level].h;
    return MGSEG_OK;
}

static float *field_ptr(mgseg_ctx *c, int l, int field)
{
    Level &L = c->lev[l];
    switch (field) {
    case 0: return L.z; case 1: return L.d; case 2: return L.w; case 3: return L.fit;
    case 4: return L.P[0]; case 5: return L.F; case 6: return L.lo; case 7: return L.hi;
    case 11: return L.r;
    default: return nullptr;
    }
}

mgseg_status mgseg_debug_get(mgseg_ctx *c, int l, int field, void *host)
{
    if (!c || !host || l < 0 || l >= c->L) return MGSEG_E_ARG;
    Level &L = c->lev[l];
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    hipError_t e = hipSuccess;
    if (field == 8 || field == 9) {
        if (l != 0) return MGSEG_E_ARG;
        e = hipMemcpy(host, field == 8 ? c->g64 : c->phi64, sizeof(double) * (size_t)c->n * c->m,
                      hipMemcpyDeviceToHost);
    } else if (field == 10) {
        e = hipMemcpy2D(host, L.m, L.lab, L.prm, L.m, L.n, hipMemcpyDeviceToHost);
    } else {
        float *f = field_ptr(c, l, field);
        if (!f) return MGSEG_E_ARG;
        e = hipMemcpy2D(host, sizeof(float) * L.m, f, sizeof(float) * L.prm, sizeof(float) * L.m, L.n,
                        hipMemcpyDeviceToHost);
    }
    return e == hipSuccess ? MGSEG_OK : MGSEG_E_HIP;
}

mgseg_status mgseg_debug_set(mgseg_ctx *c, int l, int field, const void *host)
{
    if (!c || !host || l < 0 || l >= c->L) return MGSEG_E_ARG;
    Level &L = c->lev[l];
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    hipError_t e = hipSuccess;
    if (field == 9) {
        if (l != 0) return MGSEG_E_ARG;
        e = hipMemcpy(c->phi64, host, sizeof(double) * (size_t)c->n * c->m, hipMemcpyHostToDevice);
    } else if (field == 10) {
        e = hipMemcpy2D(L.lab, L.prm, host, L.m, L.m, L.n, hipMemcpyHostToDevice);
        transpose_u8(c, L.lab, L.prm, L.lab_cm, L.pcm, L.n, L.m);
    } else {
        float *f = field_ptr(c, l, field);
        if (!f || field == 8 || field == 11) return MGSEG_E_ARG;
        e = hipMemcpy2D(f, sizeof(float) * L.prm, host, sizeof(float) * L.m, sizeof(float) * L.m, L.n,
                        hipMemcpyHostToDevice);
        if (field == 2) transpose_f(c, L.w, L.prm, L.w_cm, L.pcm, L.n, L.m);
        if (field == 3) transpose_f(c, L.fit, L.prm, L.fit_cm, L.pcm, L.n, L.m);
        if (field == 5) { transpose_f(c, L.F, L.prm, L.F_cm, L.pcm, L.n, L.m); L.has_F = true; }
        if (field == 6) transpose_f(c, L.lo, L.prm, L.lo_cm, L.pcm, L.n, L.m);
        if (field == 7) transpose_f(c, L.hi, L.prm, L.hi_cm, L.pcm, L.n, L.m);
    }
    if (e != hipSuccess) return MGSEG_E_HIP;
    chk(c);
    return sync_status(c);
}

mgseg_status mgseg_debug_scalars(mgseg_ctx *c, double *out5)
{
    if (!c || !out5) return MGSEG_E_ARG;
    double c12[2];
    (void)hipMemcpyAsync(c12, c->dsc + DS_C1, sizeof(c12), hipMemcpyDeviceToHost, c->s);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    out5[0] = c12[0]; out5[1] = c12[1]; out5[2] = c->A1; out5[3] = c->res0; out5[4] = c->h0;
    return MGSEG_OK;
}

mgseg_status mgseg_debug_set_c(mgseg_ctx *c, double c1, double c2)
{
    if (!c) return MGSEG_E_ARG;
    double c12[2] = {c1, c2};
    (void)hipMemcpyAsync(c->dsc + DS_C1, c12, sizeof(c12), hipMemcpyHostToDevice, c->s);
    update_fit(c);
    chk(c);
    return sync_status(c);
}

mgseg_status mgseg_debug_op(mgseg_ctx *c, int l, int op, int arg)
{
    if (!c || l < 0 || l >= c->L) return MGSEG_E_ARG;
    Level &L = c->lev[l];
    switch (op) {
    case 0: freeze(c, l); break;
    case 1: case 2:
        launch_sweep(c, l, op - 1, L.P[0], L.P[1]);
        (void)hipMemcpyAsync(L.P[0], L.P[1], sizeof(float) * (size_t)L.n * L.prm, hipMemcpyDeviceToDevice, c->s);
        break;
    case 3: case 4:
        transpose_f(c, L.P[0], L.prm, L.T[1], L.pcm, L.n, L.m);
        launch_sweep(c, l, op - 1, L.T[1], L.T[2]);
        transpose_f(c, L.T[2], L.pcm, L.P[0], L.prm, L.m, L.n);
        break;
    case 5: smooth(c, l, arg); break;
    case 6:
        if (l != c->L - 1) return MGSEG_E_ARG;
        coarsest(c, l);
        break;
    case 7: vcycle_from(c, l); break;
    case 8: residual(c, l, L.r, nullptr); break;
    case 9: update_c(c); break;
    default: return MGSEG_E_ARG;
    }
    chk(c);
    return sync_status(c);
}

mgseg_status mgseg_profile(mgseg_ctx *c, int kernel, int enable)
{
    if (!c || kernel != 0) return MGSEG_E_ARG;
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->prof_on = enable != 0;
    if (enable) { c->ev_used.clear(); c->ev_next = 0; }
    return MGSEG_OK;
}

mgseg_status mgseg_profile_read(mgseg_ctx *c, int kernel, double *total_ms, int *count, double *bytes_per_launch)
{
    if (!c || kernel != 0) return MGSEG_E_ARG;
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    double tot = 0.0;
    for (auto &pr : c->ev_used) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return MGSEG_E_HIP;
        tot += ms;
    }
    if (total_ms) *total_ms = tot;
    if (count) *count = (int)c->ev_used.size();
    // compulsory bytes of one finest-grid sweep per cell.  Mixed mode: read
    // phi (4 B), the four stored face coefficients (16 B), the label byte, T
    // (4 B) and the bounds of the deviation (8 B); write phi (4 B): 37 B.
    // FP32 mode: read phi, psi, w (4 B each), the label byte, fit and F (4 B
    // each, F only where set); write phi (4 B).
    if (bytes_per_launch) {
        const double per = devm(c) ? 4.0 + 16.0 + 1.0 + 4.0 + 8.0 + 4.0
                                    : 4.0 * 3 + 1.0 + 4.0 + (c->lev[0].has_F ? 4.0 : 0.0) + 4.0;
        *bytes_per_launch = (double)c->n * c->m * per;
    }
    return MGSEG_OK;
}


}  // extern "C"

// --------------------------------------------------------------------------
// batches
struct mgseg_batch {
    std::vector<mgseg_ctx *> ctx;
    std::vector<int> order;                 // images by decreasing size (LPT)
    std::vector<hipStream_t> streams;       // internal streams (default priority)
    std::vector<hipEvent_t> done;           // one per internal stream
    hipEvent_t entry = nullptr;
    hipStream_t user = nullptr;
    int nstreams = 4;
};

namespace {

// longest-processing-time assignment of images to the first S streams
void batch_assign(mgseg_batch *b, int S)
{
    std::vector<double> load(S, 0.0);
    for (int i : b->order) {
        int best = 0;
        for (int s = 1; s < S; s++)
            if (load[s] < load[best]) best = s;
        load[best] += (double)b->ctx[i]->n * b->ctx[i]->m;
        b->ctx[i]->s = b->streams[best];
    }
    b->nstreams = S;
}

// one cycle on every listed image, then one wait per stream
mgseg_status batch_round(mgseg_batch *b, const std::vector<int> &imgs, std::vector<double> &rel)
{
    for (int i : imgs) cycle_begin(b->ctx[i]);
    mgseg_status st = MGSEG_OK;
    for (int s = 0; s < b->nstreams; s++)
        if (hipStreamSynchronize(b->streams[s]) != hipSuccess) st = MGSEG_E_HIP;
    if (st != MGSEG_OK) return st;
    for (int i : imgs) {
        mgseg_status e = cycle_end(b->ctx[i], &rel[i]);
        if (e != MGSEG_OK) st = e;
    }
    return st;
}

void batch_enter(mgseg_batch *b)
{
    (void)hipEventRecord(b->entry, b->user);
    for (int s = 0; s < (int)b->streams.size(); s++) (void)hipStreamWaitEvent(b->streams[s], b->entry, 0);
}

void batch_leave(mgseg_batch *b)
{
    for (int s = 0; s < (int)b->streams.size(); s++) {
        (void)hipEventRecord(b->done[s], b->streams[s]);
        (void)hipStreamWaitEvent(b->user, b->done[s], 0);
    }
}

}  // namespace

extern "C" {

void mgseg_destroy_batch(mgseg_batch *b)
{
    if (!b) return;
    for (auto s : b->streams) (void)hipStreamSynchronize(s);
    for (auto c : b->ctx) {
        c->s = b->user;           // contexts release their buffers on the caller's stream
        mgseg_destroy(c);
    }
    for (auto e : b->done) (void)hipEventDestroy(e);
    if (b->entry) (void)hipEventDestroy(b->entry);
    for (auto s : b->streams) (void)hipStreamDestroy(s);
    delete b;
}

mgseg_status mgseg_setup_batch(int count, const float *const *images_dev, const int *n, const int *m,
                               const int *pitch, const float *const *markers_host, const int *k,
                               const mgseg_params *p, void *stream, mgseg_batch **out)
{
    if (!out) return MGSEG_E_ARG;
    *out = nullptr;
    if (count < 1 || !images_dev || !n || !m || !pitch || !markers_host || !k || !p) return MGSEG_E_ARG;
    mgseg_batch *b = new (std::nothrow) mgseg_batch();
    if (!b) return MGSEG_E_NOMEM;
    b->user = (hipStream_t)stream;
    for (int s = 0; s < 8; s++) {
        hipStream_t h = nullptr;
        hipEvent_t e = nullptr;
        if (hipStreamCreateWithFlags(&h, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (h) (void)hipStreamDestroy(h);
            mgseg_destroy_batch(b);
            return MGSEG_E_HIP;
        }
        b->streams.push_back(h);
        b->done.push_back(e);
    }
    if (hipEventCreateWithFlags(&b->entry, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        mgseg_destroy_batch(b);
        return MGSEG_E_HIP;
    }
    for (int i = 0; i < count; i++) {
        mgseg_ctx *c = nullptr;
        mgseg_status st = mgseg_setup(images_dev[i], n[i], m[i], pitch[i], markers_host[i], k[i], p, stream, &c);
        if (st != MGSEG_OK) { mgseg_destroy_batch(b); return st; }
        b->ctx.push_back(c);
    }
    b->order.resize(count);
    for (int i = 0; i < count; i++) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) {
        return (double)b->ctx[x]->n * b->ctx[x]->m > (double)b->ctx[y]->n * b->ctx[y]->m;
    });
    batch_assign(b, std::min(4, count));
    *out = b;
    return MGSEG_OK;
}

mgseg_status mgseg_batch_set_streams(mgseg_batch *b, int nstreams)
{
    if (!b || nstreams < 1 || nstreams > (int)b->streams.size()) return MGSEG_E_ARG;
    for (auto s : b->streams) (void)hipStreamSynchronize(s);
    batch_assign(b, nstreams);
    return MGSEG_OK;
}

mgseg_status mgseg_batch_tune(mgseg_batch *b, int trial_rounds, int *nstreams_out, double *ms_per_round_out)
{
    if (!b || trial_rounds < 1) return MGSEG_E_ARG;
    const int count = (int)b->ctx.size();
    std::vector<int> all(count);
    for (int i = 0; i < count; i++) all[i] = i;
    std::vector<double> rel(count, 0.0);
    batch_enter(b);
    mgseg_status st = batch_round(b, all, rel);      // untimed: first use captures each cycle
    int best = b->nstreams;
    double best_ms = 1e300;
    for (int S = 1; S <= 8 && st == MGSEG_OK; S *= 2) {
        if (S > count) break;
        batch_assign(b, S);
        auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < trial_rounds && st == MGSEG_OK; r++) st = batch_round(b, all, rel);
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / trial_rounds;
        if (ms < best_ms) { best_ms = ms; best = S; }
    }
    batch_assign(b, best);
    batch_leave(b);
    if (nstreams_out) *nstreams_out = best;
    if (ms_per_round_out) *ms_per_round_out = best_ms;
    return st;
}

mgseg_status mgseg_solve_batch(mgseg_batch *b, double tol, int max_cycles, int *cycles_out, double *rel_out)
{
    if (!b || !(tol > 0.0) || max_cycles < 0) return MGSEG_E_ARG;
    const int count = (int)b->ctx.size();
    std::vector<double> rel(count, 0.0);
    for (int i = 0; i < count; i++) rel[i] = b->ctx[i]->rel;
    batch_enter(b);
    mgseg_status st = MGSEG_OK;
    for (;;) {
        std::vector<int> act;
        for (int i : b->order)
            if (rel[i] > tol && b->ctx[i]->cycles < max_cycles) act.push_back(i);
        if (act.empty()) break;
        st = batch_round(b, act, rel);
        if (st != MGSEG_OK && st != MGSEG_E_NONFINITE) break;
        if (st == MGSEG_E_NONFINITE) break;
    }
    batch_leave(b);
    bool all_ok = true;
    for (int i = 0; i < count; i++) {
        if (cycles_out) cycles_out[i] = b->ctx[i]->cycles;
        if (rel_out) rel_out[i] = b->ctx[i]->rel;
        if (!(b->ctx[i]->rel <= tol)) all_ok = false;
    }
    if (st != MGSEG_OK) return st;
    return all_ok ? MGSEG_OK : MGSEG_E_NOT_CONVERGED;
}

mgseg_status mgseg_batch_ctx(mgseg_batch *b, int index, mgseg_ctx **view)
{
    if (!b || !view || index < 0 || index >= (int)b->ctx.size()) return MGSEG_E_ARG;
    *view = b->ctx[index];
    return MGSEG_OK;
}


// ---- learned warm start on a context
mgseg_status mgseg_ctx_features(mgseg_ctx *c, float *out_dev)
{
    if (!c || !out_dev) return MGSEG_E_ARG;
    Level &L = c->lev[0];
    hipLaunchKernelGGL(k_features, grid2(c->n, c->m), dim3(256), 0, c->s, L.z, L.d, L.prm, c->n, c->m, c->mk_d, c->k,
                       out_dev);
    chk(c);
    return sync_status(c);
}

mgseg_status mgseg_reset_phi0(mgseg_ctx *c)
{
    if (!c) return MGSEG_E_ARG;
    Level &L0 = c->lev[0];
    (void)hipMemcpyAsync(c->phi64, c->phi0m, sizeof(double) * (size_t)c->n * c->m, hipMemcpyDeviceToDevice, c->s);
    hipLaunchKernelGGL(k_copy64to32, grid2(c->n, c->m), dim3(256), 0, c->s, c->phi64, c->n, c->m, L0.P[0], L0.prm);
    refresh_and_residual(c);
    mgseg_status st = sync_status(c);
    if (st != MGSEG_OK) return st;
    c->res0 = read_scalar(c, DS_RES);
    c->res0_rows = read_scalar(c, DS_RESR);
    c->res_rows = c->res0_rows;
    c->res = c->res0; c->rel = 1.0; c->cycles = 0;
    return MGSEG_OK;
}

mgseg_status mgseg_predict_phi0(mgseg_ctx *c, mgseg_net *net, double scale, int *accepted_out)
{
    if (!c || !net || !(scale > 0.0 && scale <= 1.0)) return MGSEG_E_ARG;
    const size_t N = (size_t)c->n * c->m;
    if (!c->pred && hipMalloc((void **)&c->pred, sizeof(float) * 4 * N) != hipSuccess) {
        (void)hipGetLastError();
        c->pred = nullptr;
        return MGSEG_E_NOMEM;
    }
    float *feat = c->pred, *phi = c->pred + 3 * N;
    mgseg_status st = mgseg_ctx_features(c, feat);
    if (st == MGSEG_OK) st = mgseg_net_forward(net, feat, 1, c->n, c->m, scale * c->p.M, phi, c->s);
    int inside = 0;
    if (st == MGSEG_OK) {
        hipLaunchKernelGGL(k_markers_inside, dim3(1), dim3(256), 0, c->s, phi, c->n, c->m, c->mk_d, c->k, c->flags + 1);
        (void)hipMemcpyAsync(&inside, c->flags + 1, sizeof(int), hipMemcpyDeviceToHost, c->s);
        chk(c);
        st = sync_status(c);
    }
    if (st == MGSEG_OK) st = inside ? mgseg_set_phi0(c, phi, c->m) : mgseg_reset_phi0(c);
    if (accepted_out) *accepted_out = st == MGSEG_OK ? inside : 0;
    return st;
}

}  // extern "C"
