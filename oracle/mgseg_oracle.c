/*
 * mgseg_oracle.c -- plain, slow FP64 CPU oracle for the FAS multigrid with
 * the jump-aware Hybrid Smoother 2 (Roberts, Chen & Irion, arXiv 1807.02137).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can check the GPU library against an
 * independent implementation written straight from the paper.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Every routine is a direct transcription of the paper's definitions, with
 * plain loops in double precision and no blocking, fusion or reordering.
 * Where the paper is silent or ambiguous the chosen reading is named in the
 * comment (the same readings are listed in the design notes of the project).
 *
 * Grid convention: level l is an n x m cell-centred grid stored row-major;
 * i = row (first index, 0..n-1), j = column (0..m-1).  The finest spacing is
 * h0 = 1/sqrt(n m) so that the image domain has unit area (Sec. 2: the
 * paper writes A2 = 1 - A1, i.e. |Omega| = 1), and h_l = 2^l h0.
 * The level-set function phi is measured in finest-pixel units, so that the
 * smoothed Heaviside with eps = 1 (Sec. 2) has a one-pixel-wide transition.
 */
#define _DEFAULT_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXLEV 16

typedef struct {
    int model;          /* 0 = Spencer-Chen (eq. scfunc), 1 = Rada-Chen (eq. rcfunc) */
    double mu, lambda1, lambda2, theta, nu;
    double eps;         /* smoothed-Heaviside width (Sec. 2, eps = 1)              */
    double eps_tv_px;   /* |grad phi| regularisation, in phi units per pixel       */
    double beta;        /* edge detector g(s) = 1/(1 + beta s), s per pixel (Sec. 2.2) */
    double sigma_g;     /* Gaussian pre-blur of z for g, in pixels                 */
    double sigma_d;     /* marker distance function width, domain units (Sec. 2.2) */
    double Sigma;       /* jump threshold: max/min coefficient ratio (Sec. 5.2)    */
    double M;           /* box bound |phi| <= M (projection)                       */
    int nu1, nu2;       /* pre / post smoothing: Hybrid-2 outer iterations         */
    int levels;         /* number of grids including the finest                    */
    int coarse_iters;   /* most outer iterations of the coarsest-grid solve        */
    double coarse_rtol; /* coarsest solve stops once an outer iteration moves no   */
                        /* value by more than coarse_rtol times the largest total  */
                        /* change since the solve began                            */
    int order;          /* 0 = paper lexicographic line order, 1 = 4-colour line order */
    int smoother;       /* 0 = Hybrid Smoother 2, 1 = GSLEX-I, 2 = Hybrid Smoother 1 */
    int obstacle;       /* 1 = coarse corrections bounded by the fine slack        */
    int scaled;         /* 1 = each row divided by its factor delta_eps(psi_ij)    */
    int run_max;        /* 0 = maximal runs; else longer runs are cut into pieces  */
} or_params;

typedef struct {
    int n, m;
    double h;
    double *z, *d, *w, *fit;   /* static maps (fit refreshed with c1, c2) */
    double *phi, *F, *phic, *tmp, *tmp2;
    double *lo, *hi;           /* per-pixel bounds of phi on this level */
    /* frozen quantities of the current outer iteration */
    double *A, *B, *C, *D, *S, *f;
    uint8_t *lab;
} or_level;

typedef struct {
    or_params p;
    int L;
    double h0, A1, c1, c2;
    double res0;        /* |r~_0| of the paper's rows (eq. abcdrc, each row with its delta factor) */
    double res0_rows;   /* |r~_0| of the rows as the smoother holds them (divided by delta if scaled) */
    double rel_rows;    /* the last cycle's relative residual of the latter */
    or_level lev[OR_MAXLEV];
    double *g0, *phi_prev;
} or_ctx;

/* ------------------------------------------------------------------------ */
/* smoothed Heaviside and delta (Sec. 2, H_eps = 1/2 + atan(phi/eps)/pi)    */
static double Heps(double phi, double eps) { return 0.5 + atan(phi / eps) / M_PI; }
static double deps(double phi, double eps) { return eps / (M_PI * (eps * eps + phi * phi)); }
static double clampM(double x, double M) { return x < -M ? -M : (x > M ? M : x); }
static double clampB(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

/* half-sample mirror index for the cell-centred Neumann boundary */
static int mirror(int t, int n)
{
    if (n == 1) return 0;
    for (;;) {
        if (t < 0) t = -t - 1;
        else if (t >= n) t = 2 * n - t - 1;
        else return t;
    }
}

static double *dalloc(size_t k) { return (double *)calloc(k ? k : 1, sizeof(double)); }

/* ------------------------------------------------------------------------ */
/* Inter-grid transfers (Sec. 3.1).                                           */
/* Full weighting: the paper's 9-point stencil 1/16[1 2 1; 2 4 2; 1 2 1]      */
/* with coarse (1-based) i taking fine rows 2i-1, 2i, 2i+1, and the boundary */
/* rule 1/2[fine n-1 + fine n] at the last coarse index.  In 0-based indices */
/* coarse I takes fine 2I, 2I+1, 2I+2 with weights 1/4, 1/2, 1/4, and the    */
/* last coarse index takes fine 2I, 2I+1 with 1/2, 1/2; 2-D is the tensor     */
/* product of the 1-D rule.                                                  */
static void fw1d_weights(int I, int nc, int nf, int idx[3], double wt[3], int *cnt)
{
    (void)nf;
    if (I < nc - 1) {
        idx[0] = 2 * I; idx[1] = 2 * I + 1; idx[2] = 2 * I + 2;
        wt[0] = 0.25; wt[1] = 0.5; wt[2] = 0.25; *cnt = 3;
    } else {
        idx[0] = 2 * I; idx[1] = 2 * I + 1;
        wt[0] = 0.5; wt[1] = 0.5; *cnt = 2;
    }
}

void or_restrict(const double *fine, int n, int m, double *coarse)
{
    int nc = n / 2, mc = m / 2;
    for (int I = 0; I < nc; I++) {
        int ri[3], rc; double rw[3];
        fw1d_weights(I, nc, n, ri, rw, &rc);
        for (int J = 0; J < mc; J++) {
            int ci[3], cc; double cw[3];
            fw1d_weights(J, mc, m, ci, cw, &cc);
            double s = 0.0;
            for (int a = 0; a < rc; a++)
                for (int b = 0; b < cc; b++)
                    s += rw[a] * cw[b] * fine[(size_t)ri[a] * m + ci[b]];
            coarse[(size_t)I * mc + J] = s;
        }
    }
}

/* Bilinear interpolation (Sec. 3.1): fine (1-based) 2i <- coarse i and     */
/* fine 2i+1 <- (coarse i + coarse i+1)/2.  In 0-based indices fine 2I+1    */
/* takes coarse I, fine 2I (I >= 1) takes the mean of coarse I-1 and I, and */
/* fine 0 mirrors coarse 0 (the paper gives no rule there).  2-D = tensor.  */
static void pl1d(int f, int nc, int idx[2], double wt[2], int *cnt)
{
    if (f & 1) { idx[0] = f / 2; wt[0] = 1.0; *cnt = 1; }
    else if (f == 0) { idx[0] = 0; wt[0] = 1.0; *cnt = 1; }
    else { idx[0] = f / 2 - 1; idx[1] = f / 2; wt[0] = 0.5; wt[1] = 0.5; *cnt = 2; }
    (void)nc;
}

void or_prolong(const double *coarse, int nc, int mc, double *fine)
{
    int n = 2 * nc, m = 2 * mc;
    for (int i = 0; i < n; i++) {
        int ri[2], rc; double rw[2];
        pl1d(i, nc, ri, rw, &rc);
        for (int j = 0; j < m; j++) {
            int ci[2], cc; double cw[2];
            pl1d(j, mc, ci, cw, &cc);
            double s = 0.0;
            for (int a = 0; a < rc; a++)
                for (int b = 0; b < cc; b++)
                    s += rw[a] * cw[b] * coarse[(size_t)ri[a] * mc + ci[b]];
            fine[(size_t)i * m + j] = s;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Setup maps (Sec. 2.2 and Sec. 5).                                          */

/* convex hull of the marker points (Andrew's monotone chain), CCW, no      */
/* collinear points; returns the number of vertices                          */
static double cross3(const double *o, const double *a, const double *b)
{
    return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0]);
}
static int cmp_pt(const void *x, const void *y)
{
    const double *a = (const double *)x, *b = (const double *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}
int or_hull(const double *pts, int k, double *hull)
{
    double P[64][2], H[130][2];
    if (k > 64) k = 64;
    for (int t = 0; t < k; t++) { P[t][0] = pts[2 * t]; P[t][1] = pts[2 * t + 1]; }
    qsort(P, (size_t)k, sizeof(P[0]), cmp_pt);
    int u = 0;
    for (int t = 0; t < k; t++) {                 /* drop duplicates */
        if (u > 0 && P[t][0] == P[u - 1][0] && P[t][1] == P[u - 1][1]) continue;
        P[u][0] = P[t][0]; P[u][1] = P[t][1]; u++;
    }
    k = u;
    if (k <= 2) {
        for (int t = 0; t < k; t++) { hull[2 * t] = P[t][0]; hull[2 * t + 1] = P[t][1]; }
        return k;
    }
    int c = 0;
    for (int t = 0; t < k; t++) {
        while (c >= 2 && cross3(H[c - 2], H[c - 1], P[t]) <= 0) c--;
        H[c][0] = P[t][0]; H[c][1] = P[t][1]; c++;
    }
    for (int t = k - 2, lo = c + 1; t >= 0; t--) {
        while (c >= lo && cross3(H[c - 2], H[c - 1], P[t]) <= 0) c--;
        H[c][0] = P[t][0]; H[c][1] = P[t][1]; c++;
    }
    c--;
    for (int t = 0; t < c; t++) { hull[2 * t] = H[t][0]; hull[2 * t + 1] = H[t][1]; }
    return c;
}

static double seg_dist(double px, double py, double ax, double ay, double bx, double by)
{
    double vx = bx - ax, vy = by - ay, wx = px - ax, wy = py - ay;
    double L2 = vx * vx + vy * vy;
    double t = L2 > 0.0 ? (wx * vx + wy * vy) / L2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double dx = px - (ax + t * vx), dy = py - (ay + t * vy);
    return sqrt(dx * dx + dy * dy);
}

/* signed distance (pixels) from the point (pr, pc) to the boundary of the   */
/* hull polygon, positive inside.  The paper initialises the contour as the  */
/* boundary of the polygon formed by the markers (Sec. 5); the convex hull   */
/* removes any dependence on the order in which markers are given.           */
static double hull_sdist(const double *hull, int hv, double pr, double pc)
{
    if (hv == 0) return -1e30;
    if (hv == 1) return -sqrt((pr - hull[0]) * (pr - hull[0]) + (pc - hull[1]) * (pc - hull[1]));
    double dmin = 1e300;
    int inside = (hv >= 3);
    for (int t = 0; t < hv; t++) {
        const double *a = hull + 2 * t, *b = hull + 2 * ((t + 1) % hv);
        double dd = seg_dist(pr, pc, a[0], a[1], b[0], b[1]);
        if (dd < dmin) dmin = dd;
        double cr = (b[0] - a[0]) * (pc - a[1]) - (b[1] - a[1]) * (pr - a[0]);
        if (cr < 0.0) inside = 0;
        if (hv == 2) break;
    }
    return inside ? dmin : -dmin;
}

static double hull_area(const double *hull, int hv)
{
    if (hv < 3) return 0.0;
    double s = 0.0;
    for (int t = 0; t < hv; t++) {
        const double *a = hull + 2 * t, *b = hull + 2 * ((t + 1) % hv);
        s += a[0] * b[1] - b[0] * a[1];
    }
    return 0.5 * fabs(s);
}

/* Static maps of the finest grid.
 *  g  : edge detector g = 1/(1 + beta |grad(G_sigma * z)|^2) (Sec. 2.2, with
 *       the Gaussian pre-blur of the image; gradient by central differences per
 *       pixel, mirror boundary, so that beta does not depend on the resolution);
 *  d  : marker distance function, the product over markers of
 *       1 - exp(-((x_k - x)^2 + (y_k - y)^2)/(2 sigma^2)) (Sec. 2.2);
 *  w  : weight inside the curvature term: g for Spencer-Chen (eq. scel),
 *       d g for Rada-Chen (eq. rcel);
 *  phi0: clamp(signed distance to the marker polygon boundary, [-M, M]);
 *  A1 : area of the marker polygon in domain units (Sec. 2.2, eq. rcfunc).
 */
void or_setup_maps(const double *z, int n, int m, const double *markers, int k,
                   const or_params *p, double *g, double *d, double *w,
                   double *phi0, double *A1)
{
    double h0 = 1.0 / sqrt((double)n * (double)m);
    int R = (int)ceil(4.0 * p->sigma_g);
    double *ker = dalloc((size_t)(2 * R + 1));
    double ks = 0.0;
    for (int t = -R; t <= R; t++) {
        double v = p->sigma_g > 0 ? exp(-(double)(t * t) / (2.0 * p->sigma_g * p->sigma_g)) : (t == 0);
        ker[t + R] = v; ks += v;
    }
    for (int t = 0; t <= 2 * R; t++) ker[t] /= ks;
    double *t1 = dalloc((size_t)n * m), *zb = dalloc((size_t)n * m);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double s = 0.0;
            for (int t = -R; t <= R; t++) s += ker[t + R] * z[(size_t)i * m + mirror(j + t, m)];
            t1[(size_t)i * m + j] = s;
        }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double s = 0.0;
            for (int t = -R; t <= R; t++) s += ker[t + R] * t1[(size_t)mirror(i + t, n) * m + j];
            zb[(size_t)i * m + j] = s;
        }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double gx = (zb[(size_t)i * m + mirror(j + 1, m)] - zb[(size_t)i * m + mirror(j - 1, m)]) / 2.0;
            double gy = (zb[(size_t)mirror(i + 1, n) * m + j] - zb[(size_t)mirror(i - 1, n) * m + j]) / 2.0;
            g[(size_t)i * m + j] = 1.0 / (1.0 + p->beta * (gx * gx + gy * gy));
        }
    double hull[128];
    int hv = or_hull(markers, k, hull);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double prod = 1.0;
            for (int t = 0; t < k; t++) {
                double dy = (markers[2 * t] - (i + 0.5)) * h0;
                double dx = (markers[2 * t + 1] - (j + 0.5)) * h0;
                prod *= 1.0 - exp(-(dx * dx + dy * dy) / (2.0 * p->sigma_d * p->sigma_d));
            }
            d[(size_t)i * m + j] = prod;
            double gg = g[(size_t)i * m + j];
            w[(size_t)i * m + j] = (p->model == 1) ? prod * gg : gg;
            phi0[(size_t)i * m + j] = clampM(hull_sdist(hull, hv, i + 0.5, j + 0.5), p->M);
        }
    *A1 = hull_area(hull, hv) * h0 * h0;
    free(ker); free(t1); free(zb);
}

/* ------------------------------------------------------------------------ */
/* The discrete operator (eq. rcabcd / abcdrc, eq. abcd).                     */
/* Face coefficient on the face between cells P and Q:                       */
/*   Ghat = w_face / sqrt(dn^2 + dt^2 + e^2),                                */
/* dn = psi_Q - psi_P (normal difference), dt = the tangential difference    */
/* averaged over both cells (central, /4), w_face = (w_P + w_Q)/2, e the      */
/* gradient regularisation in pixel units on this level; faces on the        */
/* domain boundary carry 0 (Neumann condition, eq. rcel).  The paper defines */
/* G only at cell centres; this face form is the conservative reading.       */
/* Stencil coefficient = (mu/h) delta_eps(psi_ij) Ghat = mu delta G / h^2.   */
static double face_h(const double *psi, const double *w, int m, int i, int j, double e2)
{   /* face between (i,j) and (i+1,j) */
    double dn = psi[(size_t)(i + 1) * m + j] - psi[(size_t)i * m + j];
    int jp = mirror(j + 1, m), jm = mirror(j - 1, m);
    double dt = (psi[(size_t)i * m + jp] + psi[(size_t)(i + 1) * m + jp]
               - psi[(size_t)i * m + jm] - psi[(size_t)(i + 1) * m + jm]) / 4.0;
    double wf = 0.5 * (w[(size_t)i * m + j] + w[(size_t)(i + 1) * m + j]);
    return wf / sqrt(dn * dn + dt * dt + e2);
}
static double face_v(const double *psi, const double *w, int n, int m, int i, int j, double e2)
{   /* face between (i,j) and (i,j+1) */
    double dn = psi[(size_t)i * m + j + 1] - psi[(size_t)i * m + j];
    int ip = mirror(i + 1, n), im = mirror(i - 1, n);
    double dt = (psi[(size_t)ip * m + j] + psi[(size_t)ip * m + j + 1]
               - psi[(size_t)im * m + j] - psi[(size_t)im * m + j + 1]) / 4.0;
    double wf = 0.5 * (w[(size_t)i * m + j] + w[(size_t)i * m + j + 1]);
    return wf / sqrt(dn * dn + dt * dt + e2);
}

/* the four face values of cell (i,j): index 0 = A (i+1/2), 1 = B (i-1/2),  */
/* 2 = C (j+1/2), 3 = D (j-1/2); interior[k] = 0 on boundary faces           */
static void cell_faces(const double *psi, const double *w, int n, int m, int i, int j, double e2,
                       double G[4], int interior[4])
{
    interior[0] = i < n - 1; interior[1] = i > 0; interior[2] = j < m - 1; interior[3] = j > 0;
    G[0] = interior[0] ? face_h(psi, w, m, i, j, e2) : 0.0;
    G[1] = interior[1] ? face_h(psi, w, m, i - 1, j, e2) : 0.0;
    G[2] = interior[2] ? face_v(psi, w, n, m, i, j, e2) : 0.0;
    G[3] = interior[3] ? face_v(psi, w, n, m, i, j - 1, e2) : 0.0;
}

double or_sumH(const double *phi, int n, int m, double eps)
{
    double s = 0.0;
    for (size_t t = 0; t < (size_t)n * m; t++) s += Heps(phi[t], eps);
    return s;
}

/* selection / area term inside f (eq. rcabcd and the f of eq. gslexrc):    */
/* Rada-Chen: 2 nu (h^2 sum_kl H(phi_kl) - A1), taken with the + sign that  */
/* the Euler-Lagrange equation (eq. rcel) and the f of eq. gslexrc carry;   */
/* Spencer-Chen: theta d sits inside the fit map (eq. scel).                 */
static double area_term(const or_ctx *c, int l, const double *psi)
{
    const or_level *L = &c->lev[l];
    if (c->p.model != 1) return 0.0;
    return 2.0 * c->p.nu * (L->h * L->h * or_sumH(psi, L->n, L->m, c->p.eps) - c->A1);
}

static double lev_e2(const or_ctx *c, int l)
{
    double e = c->p.eps_tv_px * (double)(1 << l);
    return e * e;
}

/* A..D, S, f at psi on level l (eq. abcdrc); these are the "frozen"         */
/* coefficients of the -I smoothers (Sec. 3.2: refreshed globally once per  */
/* outer iteration).                                                         */
static void coeffs_at(or_ctx *c, int l, const double *psi, double *A, double *B, double *C,
                      double *D, double *S, double *f)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    double kap = c->p.mu / L->h, e2 = lev_e2(c, l);
    double s = area_term(c, l, psi);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double G[4]; int in[4];
            cell_faces(psi, L->w, n, m, i, j, e2, G, in);
            size_t q = (size_t)i * m + j;
            double dl = c->p.scaled ? 1.0 : deps(psi[q], c->p.eps);
            A[q] = kap * dl * G[0]; B[q] = kap * dl * G[1];
            C[q] = kap * dl * G[2]; D[q] = kap * dl * G[3];
            S[q] = A[q] + B[q] + C[q] + D[q];
            f[q] = dl * (L->fit[q] + s);
        }
}

/* N(phi) (eq. abcd): A phi_{i+1,j} + B phi_{i-1,j} + C phi_{i,j+1}         */
/* + D phi_{i,j-1} - S phi_ij - f, all coefficients evaluated at phi.        */
static void apply_N(or_ctx *c, int l, const double *phi, double *out)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    size_t N = (size_t)n * m;
    double *A = dalloc(N), *B = dalloc(N), *C = dalloc(N), *D = dalloc(N), *S = dalloc(N), *f = dalloc(N);
    coeffs_at(c, l, phi, A, B, C, D, S, f);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            size_t q = (size_t)i * m + j;
            double v = -S[q] * phi[q] - f[q];
            if (i < n - 1) v += A[q] * phi[q + m];
            if (i > 0) v += B[q] * phi[q - m];
            if (j < m - 1) v += C[q] * phi[q + 1];
            if (j > 0) v += D[q] * phi[q - 1];
            out[q] = v;
        }
    free(A); free(B); free(C); free(D); free(S); free(f);
}

/* residual r = F - N(phi); projected residual (box reading): zero where    */
/* the Gauss-Seidel correction -r/S would leave [-M, M].                     */
static void residual(or_ctx *c, int l, const double *phi, const double *F, double *r, int project)
{
    or_level *L = &c->lev[l];
    size_t N = (size_t)L->n * L->m;
    apply_N(c, l, phi, r);
    for (size_t q = 0; q < N; q++) {
        double v = (F ? F[q] : 0.0) - r[q];
        if (project && ((phi[q] >= L->hi[q] && v < 0.0) || (phi[q] <= L->lo[q] && v > 0.0))) v = 0.0;
        r[q] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Jump set and lagging labels (Sec. 4.1 Definition, Sec. 4.1 "lag only the  */
/* smallest", Sec. 5.2 Definition of Sigma).  A pixel is in the jump set     */
/* when the largest of its interior coefficients exceeds Sigma times the     */
/* smallest (a zero interior coefficient counts as an infinite ratio); its   */
/* label is the coefficient that is smallest (first of A, B, C, D on ties).  */
/* The common factor mu delta/h^2 cancels in both tests, so they are taken   */
/* on the face values.  Label byte: bit s set <=> starred in sweep s.        */
static void labels_at(or_ctx *c, int l, const double *psi, uint8_t *lab)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    double e2 = lev_e2(c, l);
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            double G[4]; int in[4];
            cell_faces(psi, L->w, n, m, i, j, e2, G, in);
            int cnt = 0, amin = -1;
            double gmin = 0.0, gmax = 0.0;
            for (int s = 0; s < 4; s++) {
                if (!in[s]) continue;
                if (cnt == 0 || G[s] < gmin) { gmin = G[s]; amin = s; }
                if (cnt == 0 || G[s] > gmax) gmax = G[s];
                cnt++;
            }
            uint8_t b = 0;
            if (cnt >= 2 && gmax > c->p.Sigma * gmin) b = (uint8_t)(1u << amin);
            lab[(size_t)i * m + j] = b;
        }
}

/* ------------------------------------------------------------------------ */
/* Hybrid Smoother 2 (Sec. 4.3, Fig. 3, Fig. 4).                              */
/* Sweep s in {A, B, C, D}: lines and in-line visit order of Fig. 4:         */
/*  A rows top->bottom, left->right;  B rows bottom->top, right->left;       */
/*  C columns left->right, top->bottom;  D columns right->left, bottom->top. */
/* Starred pixels (jump set, smallest coefficient = s) form maximal runs     */
/* along the line; a single starred pixel is grouped with the next pixel in  */
/* the visit order (Sec. 4.3; a singleton that is the last pixel of its line */
/* has no next pixel and is updated alone).  Non-starred pixels get the      */
/* GSLEX-I point update (eq. gslexrc) with the frozen coefficients; a run is */
/* solved collectively (partial line solve) with everything outside the run  */
/* at its current value, then clamped to the box.  Each pixel is updated     */
/* exactly once per sweep.                                                   */
/* Line order: order = 0 is the paper's (lines in visit order); order = 1 is */
/* the parallel ordering: the lines of a sweep are split into four classes   */
/* by index mod 4, processed 0,1,2,3 for A and C and 3,2,1,0 for B and D.    */

typedef struct { int nl, len; } lineinfo;

/* pixel index of position t on line r for direction s */
static size_t line_px(int s, int n, int m, int r, int t)
{
    switch (s) {
    case 0: return (size_t)r * m + t;                       /* A: row r, left->right  */
    case 1: return (size_t)r * m + (m - 1 - t);             /* B: row r, right->left  */
    case 2: return (size_t)t * m + r;                       /* C: col r, top->bottom  */
    default: return (size_t)(n - 1 - t) * m + r;            /* D: col r, bottom->top  */
    }
}

static void lines_of(int s, int n, int m, int *nl, int *len)
{
    if (s < 2) { *nl = n; *len = m; } else { *nl = m; *len = n; }
}

/* point update at pixel q (i,j) with the frozen coefficients of level L */
static void point_update(or_ctx *c, or_level *L, size_t q)
{
    (void)c;
    int m = L->m, n = L->n;
    int i = (int)(q / m), j = (int)(q % m);
    if (L->S[q] == 0.0) return;
    double v = -L->f[q] - L->F[q];
    if (i < n - 1) v += L->A[q] * L->phi[q + m];
    if (i > 0) v += L->B[q] * L->phi[q - m];
    if (j < m - 1) v += L->C[q] * L->phi[q + 1];
    if (j > 0) v += L->D[q] * L->phi[q - 1];
    L->phi[q] = clampB(v / L->S[q], L->lo[q], L->hi[q]);
}

/* coefficient of the frozen stencil at q pointing to neighbour q2 */
static double coef_to(or_level *L, size_t q, size_t q2)
{
    int m = L->m;
    if (q2 == q + (size_t)m) return L->A[q];
    if (q2 + (size_t)m == q) return L->B[q];
    if (q2 == q + 1) return L->C[q];
    return L->D[q];
}

/* neighbour contribution sum excluding the given set of pixels */
static double outside_sum(or_level *L, size_t q, const size_t *ex, int nex)
{
    int m = L->m, n = L->n;
    int i = (int)(q / m), j = (int)(q % m);
    size_t nb[4]; double cf[4]; int k = 0;
    if (i < n - 1) { nb[k] = q + m; cf[k++] = L->A[q]; }
    if (i > 0) { nb[k] = q - m; cf[k++] = L->B[q]; }
    if (j < m - 1) { nb[k] = q + 1; cf[k++] = L->C[q]; }
    if (j > 0) { nb[k] = q - 1; cf[k++] = L->D[q]; }
    double s = 0.0;
    for (int t = 0; t < k; t++) {
        int skip = 0;
        for (int e = 0; e < nex; e++) if (ex[e] == nb[t]) skip = 1;
        if (!skip) s += cf[t] * L->phi[nb[t]];
    }
    return s;
}

/* plain Gaussian elimination (no pivoting) of a tridiagonal system;      */
/* returns 0 on a zero pivot                                                  */
static int tridiag(int len, const double *lo0, const double *di0, const double *up0,
                   const double *rh0, double *x)
{
    double *di = dalloc(len), *rh = dalloc(len);
    memcpy(di, di0, sizeof(double) * len); memcpy(rh, rh0, sizeof(double) * len);
    int ok = 1;
    for (int k = 1; k < len; k++) {
        if (di[k - 1] == 0.0) { ok = 0; break; }
        double fac = lo0[k] / di[k - 1];
        di[k] -= fac * up0[k - 1];
        rh[k] -= fac * rh[k - 1];
    }
    if (ok && di[len - 1] == 0.0) ok = 0;
    if (ok) {
        x[len - 1] = rh[len - 1] / di[len - 1];
        for (int k = len - 2; k >= 0; k--) x[k] = (rh[k] - up0[k] * x[k + 1]) / di[k];
    }
    free(di); free(rh);
    return ok;
}

/* Box-constrained tridiagonal system (the variational inequality of one run):
 * rows k = 0..len-1:  lo_k x_{k-1} + di_k x_k + up_k x_{k+1} = rh_k,  with
 * bl_k <= x_k <= bh_k; a row may hold x_k at a bound only where its residual
 * pushes outward.  Active-set iteration: free cells solved exactly with held
 * cells as known values; free cells outside the box are held, held cells whose
 * residual turns inward (beyond rounding) are released; until the held set is
 * stable (at most 2 len + 4 passes).
 * Returns 0 on a zero pivot.  lo_0 and up_{len-1} are ignored. */
int or_box_tridiag(int len, const double *lo, const double *di, const double *up, const double *rh,
                   const double *bl, const double *bh, double *x)
{
    double *l2 = dalloc(len), *d2 = dalloc(len), *u2 = dalloc(len), *r2 = dalloc(len), *y = dalloc(len);
    int *held = (int *)calloc((size_t)len, sizeof(int)), *map = (int *)malloc(sizeof(int) * (size_t)(len + 1));
    int ok = 1;
    for (int it = 0; ok && it < 2 * len + 4; it++) {
        int nf = 0;
        for (int k = 0; k < len; k++) {
            if (held[k]) { x[k] = held[k] > 0 ? bh[k] : bl[k]; continue; }
            map[nf] = k;
            double r = rh[k];
            if (k > 0 && held[k - 1]) r -= lo[k] * x[k - 1];
            if (k < len - 1 && held[k + 1]) r -= up[k] * (held[k + 1] > 0 ? bh[k + 1] : bl[k + 1]);
            l2[nf] = (k > 0 && !held[k - 1]) ? lo[k] : 0.0;
            u2[nf] = (k < len - 1 && !held[k + 1]) ? up[k] : 0.0;
            d2[nf] = di[k]; r2[nf] = r; nf++;
        }
        int s0 = 0;
        while (ok && s0 < nf) {          /* chains of free cells between held ones */
            int e0 = s0;
            while (e0 + 1 < nf && map[e0 + 1] == map[e0] + 1) e0++;
            l2[s0] = 0.0; u2[e0] = 0.0;
            if (!tridiag(e0 - s0 + 1, l2 + s0, d2 + s0, u2 + s0, r2 + s0, y + s0)) ok = 0;
            for (int t = s0; t <= e0; t++) x[map[t]] = y[t];
            s0 = e0 + 1;
        }
        if (!ok) break;
        int changed = 0;
        for (int k = 0; k < len; k++) {
            if (!held[k]) {
                if (x[k] > bh[k]) { held[k] = 1; changed = 1; }
                else if (x[k] < bl[k]) { held[k] = -1; changed = 1; }
            } else {
                double v = di[k] * x[k] - rh[k];
                double mag = fabs(di[k] * x[k]) + fabs(rh[k]);
                if (k > 0) { v += lo[k] * x[k - 1]; mag += fabs(lo[k] * x[k - 1]); }
                if (k < len - 1) { v += up[k] * x[k + 1]; mag += fabs(up[k] * x[k + 1]); }
                /* v = row value minus rhs; the point update moves x_k by -v / di_k.
                 * A held cell is released only when its residual points inward
                 * by more than rounding, so that the hold / release iteration
                 * cannot alternate on a cell whose free value is the bound. */
                double tau = 1e-12 * mag;
                if ((held[k] == 1 && v < -tau) || (held[k] == -1 && v > tau)) { held[k] = 0; changed = 1; }
            }
        }
        if (!changed) break;
    }
    for (int k = 0; ok && k < len; k++) x[k] = clampB(x[k], bl[k], bh[k]);
    free(l2); free(d2); free(u2); free(r2); free(y); free(held); free(map);
    return ok;
}

/* collective solve of the run of pixels px[0..len-1] (consecutive along a   */
/* line): for each k, coef(prev) phi_prev + coef(next) phi_next - S phi_k   */
/* = f_k + F_k - (contributions of pixels outside the run).  The system is  */
/* tridiagonal and diagonally dominant (Sec. 3.2).  With the box reading   */
/* the run is solved as the box-constrained problem above; a zero pivot or  */
/* a cell with S = 0 leaves the run unchanged.                              */
static void run_update(or_ctx *c, or_level *L, const size_t *px, int len)
{
    (void)c;
    double *lo = dalloc(len), *di = dalloc(len), *up = dalloc(len), *rh = dalloc(len), *x = dalloc(len);
    double *bl = dalloc(len), *bh = dalloc(len);
    int ok = 1;
    for (int k = 0; k < len; k++) {
        size_t q = px[k];
        bl[k] = L->lo[q]; bh[k] = L->hi[q];
        if (L->S[q] == 0.0) ok = 0;
        di[k] = -L->S[q];
        lo[k] = k > 0 ? coef_to(L, q, px[k - 1]) : 0.0;
        up[k] = k < len - 1 ? coef_to(L, q, px[k + 1]) : 0.0;
        rh[k] = L->f[q] + L->F[q] - outside_sum(L, q, px, len);
    }
    if (ok && or_box_tridiag(len, lo, di, up, rh, bl, bh, x))
        for (int k = 0; k < len; k++) L->phi[px[k]] = x[k];
    free(lo); free(di); free(up); free(rh); free(x); free(bl); free(bh);
}

/* units of one line in visit order: a starred pixel starts a run of the     */
/* maximal consecutive starred pixels; a single starred pixel takes the next */
/* pixel in the visit order into its run (Sec. 4.3, Fig. 3 step V); every    */
/* other pixel is a point unit.  Returns the last position of the unit       */
/* starting at t (t itself for a point unit).                                */
static int unit_end_max(const uint8_t *lab_line, int len, int t, uint8_t bit, int run_max)
{
    if (!(lab_line[t] & bit)) return t;
    int t0 = t, e = t;
    while (t0 > 0 && (lab_line[t0 - 1] & bit)) t0--;
    while (e + 1 < len && (lab_line[e + 1] & bit)) e++;
    if (e == t && t0 == t && t + 1 < len) return t + 1;
    int rl = e - t0 + 1;
    if (run_max <= 0 || rl <= run_max) return e;
    /* cut into P = ceil(rl / run_max) pieces of near-equal length, longer first */
    int P = (rl + run_max - 1) / run_max, base = rl / P, extra = rl % P, s = t0;
    for (int k = 0; k < P; k++) {
        int pl = base + (k < extra ? 1 : 0);
        if (t < s + pl) return s + pl - 1;
        s += pl;
    }
    return e;
}

/* test hook: unit structure of a line of labels: writes for every position */
/* the index of the first position of its unit (run_max 0: maximal runs)    */
void or_line_units(const uint8_t *lab_line, int len, int bit, int run_max, int *unit_start)
{
    int t = 0;
    while (t < len) {
        int e = unit_end_max(lab_line, len, t, (uint8_t)(1u << bit), run_max);
        for (int u = t; u <= e; u++) unit_start[u] = t;
        t = e + 1;
    }
}

/* one pass over a single line in visit order */
static void sweep_line(or_ctx *c, or_level *L, int s, int r)
{
    int nl, len;
    lines_of(s, L->n, L->m, &nl, &len);
    size_t *px = (size_t *)malloc(sizeof(size_t) * (size_t)(len + 1));
    uint8_t *ll = (uint8_t *)malloc((size_t)len + 1);
    for (int t = 0; t < len; t++) ll[t] = L->lab[line_px(s, L->n, L->m, r, t)];
    int t = 0;
    while (t < len) {
        int e = unit_end_max(ll, len, t, (uint8_t)(1u << s), c->p.run_max);
        if (e == t && !(ll[t] & (1u << s))) { point_update(c, L, line_px(s, L->n, L->m, r, t)); t++; continue; }
        int k = 0;
        for (int u = t; u <= e; u++) px[k++] = line_px(s, L->n, L->m, r, u);
        run_update(c, L, px, k);
        t = e + 1;
    }
    free(px); free(ll);
}

/* test hook: the pixels of the n x m grid in the order sweep s visits them  */
/* (order = 0 paper order, 1 four-class order)                               */
void or_visit_order(int s, int n, int m, int order, long *out)
{
    int nl, len, k = 0;
    lines_of(s, n, m, &nl, &len);
    if (order == 0) {
        for (int r = 0; r < nl; r++) {
            int line = (s == 1 || s == 3) ? nl - 1 - r : r;
            for (int t = 0; t < len; t++) out[k++] = (long)line_px(s, n, m, line, t);
        }
    } else {
        for (int cl = 0; cl < 4; cl++) {
            int col = (s == 1 || s == 3) ? 3 - cl : cl;
            for (int r = col; r < nl; r += 4)
                for (int t = 0; t < len; t++) out[k++] = (long)line_px(s, n, m, r, t);
        }
    }
}

static void hs2_sweep(or_ctx *c, int l, int s)
{
    or_level *L = &c->lev[l];
    int nl, len;
    lines_of(s, L->n, L->m, &nl, &len);
    if (c->p.order == 0) {
        for (int r = 0; r < nl; r++) {
            int line = (s == 1 || s == 3) ? nl - 1 - r : r;
            sweep_line(c, L, s, line);
        }
    } else {
        for (int k = 0; k < 4; k++) {
            int col = (s == 1 || s == 3) ? 3 - k : k;
            for (int r = col; r < nl; r += 4) sweep_line(c, L, s, r);
        }
    }
}

/* freeze: coefficients, f and labels at psi = phi (start of every outer    */
/* iteration, -I variant of Sec. 3.2)                                        */
static void freeze(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    memcpy(L->tmp, L->phi, sizeof(double) * (size_t)L->n * L->m);
    coeffs_at(c, l, L->tmp, L->A, L->B, L->C, L->D, L->S, L->f);
    labels_at(c, l, L->tmp, L->lab);
}

/* GSLEX-I: lexicographic point Gauss-Seidel with frozen coefficients        */
/* (Sec. 3.2), every pixel a point update in the order of sweep A: rows top  */
/* to bottom, each left to right (order = 0), or the rows in the four        */
/* classes of the parallel line order, each row left to right (order = 1).   */
static void gslex_sweep(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    const int n = L->n, m = L->m;
    for (int k = 0; k < (c->p.order == 0 ? 1 : 4); k++)
        for (int i = (c->p.order == 0 ? 0 : k); i < n; i += (c->p.order == 0 ? 1 : 4))
            for (int j = 0; j < m; j++) point_update(c, L, (size_t)i * m + j);
}

/* ------------------------------------------------------------------------ */
/* Hybrid Smoother 1 (Sec. 4.2, "Implementing Hybrid Smoother 1"): step I,   */
/* GSLINE-I on every column (each column one line system, the paper's       */
/* column-by-column line Gauss-Seidel); step II, at every pixel of the jump  */
/* set the collective update of the pixel and its three neighbours other     */
/* than the one behind its smallest coefficient, which is lagged             */
/* (eqs. caseAlagged .. caseDlagged).  Each neighbour's row is its own       */
/* discrete equation (eq. abcd), its coupling to the centre being its own    */
/* coefficient towards the centre (with delta-scaled rows this is the        */
/* centre's coefficient towards it, as the paper's arrow matrices write it); */
/* all other pixels enter at their current values.  With the box reading the */
/* block is solved as its box-constrained system.                            */
/* Order: 0 = the paper's (columns left to right; jump pixels row by row);   */
/* 1 = the parallel one (columns in four classes as sweep C; jump pixels in  */
/* eight classes (i + 3 j) mod 8, row by row within a class: two pixels of    */
/* one class are at least four cells apart, so their blocks neither share    */
/* nor read each other's pixels).                                            */

/* Box-constrained small dense system M x = b (M diagonally dominant with a   */
/* negative diagonal), bl <= x <= bh: active-set iteration (free unknowns    */
/* solved by Gaussian elimination with the held ones at their bounds; free   */
/* unknowns outside the box are held, held unknowns whose row residual turns */
/* inward are released).  Returns 0 on a zero pivot.                         */
int or_box_dense(int k, const double *M, const double *b, const double *bl, const double *bh, double *x)
{
    int held[8] = {0}, idx[8];
    double A[64], r[8], y[8];
    if (k > 8) return 0;
    for (int it = 0; it < 2 * k + 4; it++) {
        int nf = 0;
        for (int a = 0; a < k; a++) {
            if (held[a]) x[a] = held[a] > 0 ? bh[a] : bl[a];
            else idx[nf++] = a;
        }
        for (int a = 0; a < nf; a++) {
            double v = b[idx[a]];
            for (int t = 0; t < k; t++)
                if (held[t]) v -= M[idx[a] * k + t] * x[t];
            r[a] = v;
            for (int c2 = 0; c2 < nf; c2++) A[a * nf + c2] = M[idx[a] * k + idx[c2]];
        }
        for (int p2 = 0; p2 < nf; p2++) {         /* elimination without pivoting */
            if (A[p2 * nf + p2] == 0.0) return 0;
            for (int q2 = p2 + 1; q2 < nf; q2++) {
                double fct = A[q2 * nf + p2] / A[p2 * nf + p2];
                for (int c2 = p2; c2 < nf; c2++) A[q2 * nf + c2] -= fct * A[p2 * nf + c2];
                r[q2] -= fct * r[p2];
            }
        }
        for (int p2 = nf - 1; p2 >= 0; p2--) {
            double v = r[p2];
            for (int c2 = p2 + 1; c2 < nf; c2++) v -= A[p2 * nf + c2] * y[c2];
            y[p2] = v / A[p2 * nf + p2];
        }
        for (int a = 0; a < nf; a++) x[idx[a]] = y[a];
        int changed = 0;
        for (int a = 0; a < k; a++) {
            if (!held[a]) {
                if (x[a] > bh[a]) { held[a] = 1; changed = 1; }
                else if (x[a] < bl[a]) { held[a] = -1; changed = 1; }
            } else {
                double v = -b[a], mag = fabs(b[a]);
                for (int t = 0; t < k; t++) { v += M[a * k + t] * x[t]; mag += fabs(M[a * k + t] * x[t]); }
                /* the row's update moves x_a by -v / M_aa = v / |M_aa|: a unknown held at its upper  */
                /* bound is released where that move is downward (v < 0), at its lower bound where   */
                /* it is upward, beyond rounding                                                       */
                if ((held[a] == 1 && v < -1e-12 * mag) || (held[a] == -1 && v > 1e-12 * mag)) { held[a] = 0; changed = 1; }
            }
        }
        if (!changed) break;
    }
    for (int a = 0; a < k; a++) x[a] = clampB(x[a], bl[a], bh[a]);
    return 1;
}

/* neighbour of (i, j) behind coefficient s (0 A: i+1, 1 B: i-1, 2 C: j+1, 3 D: j-1), -1 outside */
static long nb_of(const or_level *L, int i, int j, int s)
{
    int ii = i + (s == 0) - (s == 1), jj = j + (s == 2) - (s == 3);
    if (ii < 0 || ii >= L->n || jj < 0 || jj >= L->m) return -1;
    return (long)ii * L->m + jj;
}
static double coef_s(const or_level *L, size_t q, int s)
{
    return s == 0 ? L->A[q] : (s == 1 ? L->B[q] : (s == 2 ? L->C[q] : L->D[q]));
}

/* the collective update at jump pixel (i, j) lagging its coefficient lag */
static void hs1_block(or_ctx *c, or_level *L, int i, int j, int lag)
{
    (void)c;
    size_t q0 = (size_t)i * L->m + j;
    long cell[4];
    int k = 0;
    cell[k++] = (long)q0;
    for (int s = 0; s < 4; s++) {
        if (s == lag) continue;
        long nq = nb_of(L, i, j, s);
        if (nq >= 0) cell[k++] = nq;
    }
    double M[16] = {0}, b[4], bl[4], bh[4], x[4];
    for (int a = 0; a < k; a++) {
        size_t q = (size_t)cell[a];
        if (L->S[q] == 0.0) return;
        int qi = (int)(q / L->m), qj = (int)(q % L->m);
        M[a * k + a] = -L->S[q];
        double rhs = L->f[q] + L->F[q];
        for (int s = 0; s < 4; s++) {
            long nq = nb_of(L, qi, qj, s);
            if (nq < 0) continue;
            int inblock = -1;
            for (int t = 0; t < k; t++) if (cell[t] == nq) inblock = t;
            /* the leaves couple only to the centre (the arrow): a leaf's other block */
            /* neighbours, and the centre's lagged one, enter at their current values */
            if (inblock >= 0 && (a == 0 || inblock == 0)) M[a * k + inblock] += coef_s(L, q, s);
            else rhs -= coef_s(L, q, s) * L->phi[nq];
        }
        b[a] = rhs; bl[a] = L->lo[q]; bh[a] = L->hi[q];
    }
    if (or_box_dense(k, M, b, bl, bh, x))
        for (int a = 0; a < k; a++) L->phi[cell[a]] = x[a];
}

/* GSLINE-I (Sec. 3.2, Smoothers 3-4, eq. system): every column one         */
/* tridiagonal line system with the frozen coefficients, columns left to    */
/* right (order = 0) or in the four classes of sweep C (order = 1).          */
static void gsline_sweep(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    size_t *px = (size_t *)malloc(sizeof(size_t) * (size_t)(n + 1));
    for (int k = 0; k < (c->p.order == 0 ? 1 : 4); k++)
        for (int j = (c->p.order == 0 ? 0 : k); j < m; j += (c->p.order == 0 ? 1 : 4)) {
            for (int i = 0; i < n; i++) px[i] = (size_t)i * m + j;
            run_update(c, L, px, n);
        }
    free(px);
}

static void hs1_outer(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    /* step I: GSLINE-I, every column one line system (the order of sweep C) */
    gsline_sweep(c, l);
    /* step II: the blocks at the jump pixels */
    for (int cls = 0; cls < (c->p.order == 0 ? 1 : 8); cls++)
        for (int i = 0; i < n; i++)
            for (int j = 0; j < m; j++) {
                if (c->p.order != 0 && ((i + 3 * j) % 8) != cls) continue;
                uint8_t b = L->lab[(size_t)i * m + j];
                if (!b) continue;
                int lag = b & 1 ? 0 : (b & 2 ? 1 : (b & 4 ? 2 : 3));
                hs1_block(c, L, i, j, lag);
            }
}

/* ------------------------------------------------------------------------ */
/* The other standard smoothers of Sec. 3.2.                                 */
/*                                                                            */
/* NEWT (Smoothers 5-6, eq. newtrc): a point Newton step on the pixel's own  */
/* equation, whose only nonlinearity in phi_ij beyond the frozen stencil is  */
/* the Rada-Chen area term Q (eq. rcabcd).  With the rows as the solver      */
/* holds them: scaled (divided by delta_eps), the row carries Q = 2 nu       */
/* (h^2 sum H - A1) with dQ/dphi_ij = 2 nu h^2 delta_eps(phi_ij); unscaled,  */
/* Q = delta_eps(phi_ij) 2 nu (h^2 sum H - A1) with derivative               */
/* 2 nu delta_eps^2 h^2 + delta_eps' 2 nu (h^2 sum H - A1).  The update is   */
/*   phi_ij <- (P - Q + Q' phi_ij) / (S + Q'),                                */
/* P the neighbour sum minus the fit part of f; for Spencer-Chen Q = 0 and   */
/* NEWT is GSLEX.  NEWT-I takes Q' at the frozen state.                      */
static double newton_qprime(const or_ctx *c, const or_level *L, double phi, double area)
{
    if (c->p.model != 1) return 0.0;
    double d = deps(phi, c->p.eps);
    double a = 2.0 * c->p.nu * L->h * L->h * d;
    if (c->p.scaled) return a;
    double dd = -2.0 * phi * d * d * M_PI / c->p.eps;     /* delta_eps'(phi) */
    return a * d + dd * area;
}

static void newt_sweep(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    const int n = L->n, m = L->m;
    double area = area_term(c, l, L->tmp);                /* at the frozen state */
    for (int k = 0; k < (c->p.order == 0 ? 1 : 4); k++)
        for (int i = (c->p.order == 0 ? 0 : k); i < n; i += (c->p.order == 0 ? 1 : 4))
            for (int j = 0; j < m; j++) {
                size_t q = (size_t)i * m + j;
                if (L->S[q] == 0.0) continue;
                double qp = newton_qprime(c, L, L->tmp[q], area);
                double v = -L->f[q] - L->F[q] + qp * L->phi[q];
                if (i < n - 1) v += L->A[q] * L->phi[q + m];
                if (i > 0) v += L->B[q] * L->phi[q - m];
                if (j < m - 1) v += L->C[q] * L->phi[q + 1];
                if (j > 0) v += L->D[q] * L->phi[q - 1];
                L->phi[q] = clampB(v / (L->S[q] + qp), L->lo[q], L->hi[q]);
            }
}

/* The local ("-II") variants refresh a pixel's coefficients from the       */
/* current phi right before they are used (Sec. 3.2: GSLEX-II, GSLINE-II,   */
/* NEWT-II), the area term's sum of H included (kept current after every    */
/* update).  coeffs_cell: A..D, S, f of eq. abcdrc at pixel q from phi.      */
static void coeffs_cell(or_ctx *c, int l, const double *phi, size_t q, double area)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m, i = (int)(q / m), j = (int)(q % m);
    double G[4]; int in[4];
    cell_faces(phi, L->w, n, m, i, j, lev_e2(c, l), G, in);
    double kap = c->p.mu / L->h;
    double dl = c->p.scaled ? 1.0 : deps(phi[q], c->p.eps);
    L->A[q] = kap * dl * G[0]; L->B[q] = kap * dl * G[1];
    L->C[q] = kap * dl * G[2]; L->D[q] = kap * dl * G[3];
    L->S[q] = L->A[q] + L->B[q] + L->C[q] + L->D[q];
    L->f[q] = dl * (L->fit[q] + area);
}

static double area_delta(const or_ctx *c, const or_level *L, double before, double after)
{
    if (c->p.model != 1) return 0.0;
    return 2.0 * c->p.nu * L->h * L->h * (Heps(after, c->p.eps) - Heps(before, c->p.eps));
}

/* GSLEX-II (newton = 0) and NEWT-II (newton = 1): lexicographic point      */
/* updates, each with its pixel's coefficients (and Q') at the current phi. */
static void point_local_sweep(or_ctx *c, int l, int newton)
{
    or_level *L = &c->lev[l];
    const int n = L->n, m = L->m;
    double area = area_term(c, l, L->phi);
    for (int k = 0; k < (c->p.order == 0 ? 1 : 4); k++)
        for (int i = (c->p.order == 0 ? 0 : k); i < n; i += (c->p.order == 0 ? 1 : 4))
            for (int j = 0; j < m; j++) {
                size_t q = (size_t)i * m + j;
                coeffs_cell(c, l, L->phi, q, area);
                if (L->S[q] == 0.0) continue;
                double qp = newton ? newton_qprime(c, L, L->phi[q], area) : 0.0;
                double old = L->phi[q];
                double v = -L->f[q] - L->F[q] + qp * old;
                if (i < n - 1) v += L->A[q] * L->phi[q + m];
                if (i > 0) v += L->B[q] * L->phi[q - m];
                if (j < m - 1) v += L->C[q] * L->phi[q + 1];
                if (j > 0) v += L->D[q] * L->phi[q - 1];
                L->phi[q] = clampB(v / (L->S[q] + qp), L->lo[q], L->hi[q]);
                area += area_delta(c, L, old, L->phi[q]);
            }
}

/* GSLINE-II: column line solves, each with its column's coefficients at   */
/* the current phi.                                                          */
static void gsline_local_sweep(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    size_t *px = (size_t *)malloc(sizeof(size_t) * (size_t)(n + 1));
    double *old = dalloc((size_t)n);
    double area = area_term(c, l, L->phi);
    for (int k = 0; k < (c->p.order == 0 ? 1 : 4); k++)
        for (int j = (c->p.order == 0 ? 0 : k); j < m; j += (c->p.order == 0 ? 1 : 4)) {
            for (int i = 0; i < n; i++) {
                px[i] = (size_t)i * m + j;
                coeffs_cell(c, l, L->phi, px[i], area);
                old[i] = L->phi[px[i]];
            }
            run_update(c, L, px, n);
            for (int i = 0; i < n; i++) area += area_delta(c, L, old[i], L->phi[px[i]]);
        }
    free(px); free(old);
}

/* smoother: 0 Hybrid Smoother 2, 1 GSLEX-I, 2 Hybrid Smoother 1, 3 GSLINE-I, */
/* 4 NEWT-I, 5 GSLEX-II, 6 GSLINE-II, 7 NEWT-II                              */
static void smooth(or_ctx *c, int l, int iters)
{
    for (int it = 0; it < iters; it++) {
        freeze(c, l);
        switch (c->p.smoother) {
        case 1: gslex_sweep(c, l); break;
        case 2: hs1_outer(c, l); break;
        case 3: gsline_sweep(c, l); break;
        case 4: newt_sweep(c, l); break;
        case 5: point_local_sweep(c, l, 0); break;
        case 6: gsline_local_sweep(c, l); break;
        case 7: point_local_sweep(c, l, 1); break;
        default:
            for (int s = 0; s < 4; s++) hs2_sweep(c, l, s);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Coarsest grid.  The paper solves it "exactly" with 100 AOS iterations    */
/* (Sec. 5); here the smoother itself is iterated coarse_iters times, with   */
/* a relative stop.  A grid of one cell has no interior face: the discrete  */
/* curvature operator (eq. abcdrc) vanishes there, and with it the smooth    */
/* error components that a coarse grid exists to correct (Sec. 3.1); its    */
/* scalar equation carries only the fit term, which with rows scaled by     */
/* delta_eps is a constant and has no solution in general.  Such a grid     */
/* therefore returns the state it received: a zero coarse correction.       */
static void coarsest(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    if (L->n * L->m == 1) return;                 /* no interior face: zero correction */
    size_t N = (size_t)L->n * L->m;
    double *x0 = dalloc(N), *prev = dalloc(N);
    memcpy(x0, L->phi, sizeof(double) * N);
    for (int it = 0; it < c->p.coarse_iters; it++) {
        memcpy(prev, L->phi, sizeof(double) * N);
        smooth(c, l, 1);
        double dmax = 0.0, tot = 0.0;
        for (size_t q = 0; q < N; q++) {
            dmax = fmax(dmax, fabs(L->phi[q] - prev[q]));
            tot = fmax(tot, fabs(L->phi[q] - x0[q]));
        }
        if (dmax <= c->p.coarse_rtol * tot) break;
    }
    free(x0); free(prev);
}

static double l2(const double *v, size_t N)
{
    double s = 0.0;
    for (size_t q = 0; q < N; q++) s += v[q] * v[q];
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* FAS V-cycle (Algorithm 1 box, gamma = 1): pre-smoothing, residual,       */
/* restriction of the (projected) residual and of phi, coarse right-hand    */
/* side N(R phi) + R r, recursion (or the coarsest solve), correction with  */
/* the interpolated coarse error, post-smoothing.  The coarse-grid operator */
/* is the rediscretisation on the coarse grid with restricted static maps.  */
/* Box reading on coarse grids: the coarse unknown may only move as far as  */
/* every fine pixel that its interpolated correction touches can follow     */
/* inside that pixel's own bounds (coarse bounds = phi_c + [max(lo_f -      */
/* phi_f), min(hi_f - phi_f)] over the interpolation support), so the      */
/* correction never has to be cut back on the fine grid.                    */
static void coarse_bounds(or_ctx *c, int l)
{
    or_level *L = &c->lev[l], *Lc = &c->lev[l + 1];
    int nc = Lc->n, mc = Lc->m, n = L->n, m = L->m;
    for (int I = 0; I < nc; I++)
        for (int J = 0; J < mc; J++) {
            size_t qc = (size_t)I * mc + J;
            if (!c->p.obstacle) { Lc->lo[qc] = -c->p.M; Lc->hi[qc] = c->p.M; continue; }
            double dl = -1e300, dh = 1e300;
            for (int i = 2 * I; i <= 2 * I + 2; i++) {
                if (i >= n) continue;
                for (int j = 2 * J; j <= 2 * J + 2; j++) {
                    if (j >= m) continue;
                    /* interpolation weight of coarse (I, J) at fine (i, j) is nonzero */
                    size_t q = (size_t)i * m + j;
                    double a = L->lo[q] - L->phi[q], b = L->hi[q] - L->phi[q];
                    if (a > dl) dl = a;
                    if (b < dh) dh = b;
                }
            }
            Lc->lo[qc] = Lc->phic[qc] + dl;
            Lc->hi[qc] = Lc->phic[qc] + dh;
        }
}

/* the coarse problem of level l + 1 from the state of level l: projected    */
/* residual, restriction of phi and of the residual, coarse bounds, coarse    */
/* right-hand side N(R phi) + R r (FAS)                                       */
static void to_coarse(or_ctx *c, int l)
{
    or_level *L = &c->lev[l], *Lc = &c->lev[l + 1];
    size_t Nc = (size_t)Lc->n * Lc->m;
    residual(c, l, L->phi, L->F, L->tmp, 1);
    or_restrict(L->phi, L->n, L->m, Lc->phic);
    or_restrict(L->tmp, L->n, L->m, Lc->tmp2);
    coarse_bounds(c, l);
    memcpy(Lc->phi, Lc->phic, sizeof(double) * Nc);
    apply_N(c, l + 1, Lc->phic, Lc->F);
    for (size_t q = 0; q < Nc; q++) Lc->F[q] += Lc->tmp2[q];
}

static void vcycle_level(or_ctx *c, int l)
{
    or_level *L = &c->lev[l];
    if (l == c->L - 1) { coarsest(c, l); return; }
    smooth(c, l, c->p.nu1);
    or_level *Lc = &c->lev[l + 1];
    size_t Nc = (size_t)Lc->n * Lc->m, N = (size_t)L->n * L->m;
    to_coarse(c, l);
    vcycle_level(c, l + 1);
    for (size_t q = 0; q < Nc; q++) Lc->tmp2[q] = Lc->phi[q] - Lc->phic[q];
    or_prolong(Lc->tmp2, Lc->n, Lc->m, L->tmp);
    for (size_t q = 0; q < N; q++) L->phi[q] = clampB(L->phi[q] + L->tmp[q], L->lo[q], L->hi[q]);
    smooth(c, l, c->p.nu2);
}

/* ------------------------------------------------------------------------ */
/* c1, c2 (eq. c1c2) from level-0 phi; fit maps on every level              */
static void update_c(or_ctx *c)
{
    or_level *L = &c->lev[0];
    size_t N = (size_t)L->n * L->m;
    double sH = 0.0, sHz = 0.0, sz = 0.0;
    for (size_t q = 0; q < N; q++) {
        double H = Heps(L->phi[q], c->p.eps);
        sH += H; sHz += H * L->z[q]; sz += L->z[q];
    }
    c->c1 = sH > 0.0 ? sHz / sH : 0.0;
    c->c2 = ((double)N - sH) > 0.0 ? (sz - sHz) / ((double)N - sH) : 0.0;
}

static void update_fit(or_ctx *c)
{
    for (int l = 0; l < c->L; l++) {
        or_level *L = &c->lev[l];
        for (size_t q = 0; q < (size_t)L->n * L->m; q++) {
            double a = L->z[q] - c->c1, b = L->z[q] - c->c2;
            double v = c->p.lambda1 * a * a - c->p.lambda2 * b * b;
            if (c->p.model == 0) v += c->p.theta * L->d[q];
            L->fit[q] = v;
        }
    }
}


/* projected residual norms on level 0: of the paper's discrete equations    */
/* (eq. abcdrc: every row carries its factor delta_eps(phi_ij)), and of the  */
/* rows as the smoother holds them (divided by delta_eps(phi_ij) when the    */
/* rows are scaled; the same rows otherwise)                                 */
static void res_norms(or_ctx *c, double *paper, double *rows)
{
    or_level *L = &c->lev[0];
    size_t N = (size_t)L->n * L->m;
    residual(c, 0, L->phi, NULL, L->tmp, 1);
    double sp = 0.0, sr = 0.0;
    for (size_t q = 0; q < N; q++) {
        double v = L->tmp[q];
        double vp = c->p.scaled ? deps(L->phi[q], c->p.eps) * v : v;
        sr += v * v; sp += vp * vp;
    }
    *paper = sqrt(sp);
    *rows = sqrt(sr);
}

double or_res_norm(or_ctx *c)
{
    double p, r;
    res_norms(c, &p, &r);
    return p;
}

double or_res_norm_rows(or_ctx *c)
{
    double p, r;
    res_norms(c, &p, &r);
    return r;
}

/* ------------------------------------------------------------------------ */
/* context                                                                   */
void or_params_default(or_params *p)
{
    p->model = 0; p->mu = 0.5; p->lambda1 = 6.5025; p->lambda2 = 6.5025;
    p->theta = 4.0; p->nu = 1.0; p->eps = 1.0; p->eps_tv_px = 1.0; p->beta = 16384.0;
    p->sigma_g = 1.0; p->sigma_d = 0.1; p->Sigma = 2.0; p->M = 4.0;
    p->nu1 = 2; p->nu2 = 2; p->levels = 1; p->coarse_iters = 10; p->coarse_rtol = 1e-4; p->order = 1; p->smoother = 0; p->obstacle = 1; p->scaled = 1; p->run_max = 0;
}

or_ctx *or_create(const double *z, int n, int m, const double *markers, int k, const or_params *p)
{
    if (p->levels < 1 || p->levels > OR_MAXLEV) return NULL;
    int div = 1 << (p->levels - 1);
    if (n % div || m % div) return NULL;
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->p = *p; c->L = p->levels;
    c->h0 = 1.0 / sqrt((double)n * (double)m);
    for (int l = 0; l < c->L; l++) {
        or_level *L = &c->lev[l];
        L->n = n >> l; L->m = m >> l; L->h = c->h0 * (double)(1 << l);
        size_t N = (size_t)L->n * L->m;
        L->z = dalloc(N); L->d = dalloc(N); L->w = dalloc(N); L->fit = dalloc(N);
        L->phi = dalloc(N); L->F = dalloc(N); L->phic = dalloc(N); L->tmp = dalloc(N); L->tmp2 = dalloc(N);
        L->A = dalloc(N); L->B = dalloc(N); L->C = dalloc(N); L->D = dalloc(N); L->S = dalloc(N); L->f = dalloc(N);
        L->lab = (uint8_t *)calloc(N, 1);
        L->lo = dalloc(N); L->hi = dalloc(N);
        for (size_t q = 0; q < N; q++) { L->lo[q] = -p->M; L->hi[q] = p->M; }
    }
    or_level *L0 = &c->lev[0];
    size_t N0 = (size_t)n * m;
    c->g0 = dalloc(N0); c->phi_prev = dalloc(N0);
    memcpy(L0->z, z, sizeof(double) * N0);
    or_setup_maps(z, n, m, markers, k, p, c->g0, L0->d, L0->w, L0->phi, &c->A1);
    for (int l = 1; l < c->L; l++) {
        or_level *Lf = &c->lev[l - 1], *Lc = &c->lev[l];
        or_restrict(Lf->w, Lf->n, Lf->m, Lc->w);
        or_restrict(Lf->z, Lf->n, Lf->m, Lc->z);
        or_restrict(Lf->d, Lf->n, Lf->m, Lc->d);
    }
    update_c(c);
    update_fit(c);
    res_norms(c, &c->res0, &c->res0_rows);
    c->rel_rows = 1.0;
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    for (int l = 0; l < c->L; l++) {
        or_level *L = &c->lev[l];
        free(L->z); free(L->d); free(L->w); free(L->fit); free(L->phi); free(L->F); free(L->phic);
        free(L->tmp); free(L->tmp2); free(L->A); free(L->B); free(L->C); free(L->D); free(L->S);
        free(L->f); free(L->lab); free(L->lo); free(L->hi);
    }
    free(c->g0); free(c->phi_prev); free(c);
}

/* one cycle followed by the c1, c2 refresh (Sec. 5: updated at the end of  */
/* each multigrid iteration); returns |r~|/|r~_0| of the paper's rows on     */
/* level 0 (the stopping measure), keeps that of the smoother's rows, and    */
/* gives the paper's relative change eta = |phi_new - phi_old| / |phi_old|   */
/* (Sec. 5.1)                                                                */
double or_vcycle(or_ctx *c, double *eta)
{
    or_level *L = &c->lev[0];
    size_t N = (size_t)L->n * L->m;
    memcpy(c->phi_prev, L->phi, sizeof(double) * N);
    memset(L->F, 0, sizeof(double) * N);
    vcycle_level(c, 0);
    update_c(c);
    update_fit(c);
    if (eta) {
        double dn = 0.0, pn = 0.0;
        for (size_t q = 0; q < N; q++) {
            double dd = L->phi[q] - c->phi_prev[q];
            dn += dd * dd; pn += c->phi_prev[q] * c->phi_prev[q];
        }
        *eta = pn > 0.0 ? sqrt(dn / pn) : 0.0;
    }
    double rp, rr;
    res_norms(c, &rp, &rr);
    c->rel_rows = c->res0_rows > 0.0 ? rr / c->res0_rows : 0.0;
    return c->res0 > 0.0 ? rp / c->res0 : 0.0;
}
double or_rel_rows(or_ctx *c) { return c->rel_rows; }

int or_solve(or_ctx *c, double tol, int max_cycles, double *hist)
{
    int k;
    for (k = 0; k < max_cycles; k++) {
        double rel = or_vcycle(c, NULL);
        if (hist) hist[k] = rel;
        if (rel <= tol) return k + 1;
    }
    return -k;
}

/* ------------------------------------------------------------------------ */
/* Energy (eq. scfunc / eq. rcfunc) as a Riemann sum with cell area h0^2;   */
/* |grad H(phi)| = delta(phi) |grad phi| with central differences.           */
double or_energy(or_ctx *c)
{
    or_level *L = &c->lev[0];
    int n = L->n, m = L->m;
    double h = L->h, E = 0.0, sH = 0.0;
    for (int i = 0; i < n; i++)
        for (int j = 0; j < m; j++) {
            size_t q = (size_t)i * m + j;
            double ph = L->phi[q];
            double gx = (L->phi[(size_t)i * m + mirror(j + 1, m)] - L->phi[(size_t)i * m + mirror(j - 1, m)]) / (2.0 * h);
            double gy = (L->phi[(size_t)mirror(i + 1, n) * m + j] - L->phi[(size_t)mirror(i - 1, n) * m + j]) / (2.0 * h);
            double H = Heps(ph, c->p.eps);
            double a = L->z[q] - c->c1, b = L->z[q] - c->c2;
            double wgt = (c->p.model == 1) ? c->g0[q] * L->d[q] : c->g0[q];
            double e = c->p.mu * wgt * deps(ph, c->p.eps) * sqrt(gx * gx + gy * gy)
                     + c->p.lambda1 * a * a * H + c->p.lambda2 * b * b * (1.0 - H);
            if (c->p.model == 0) e += c->p.theta * L->d[q] * H;
            E += e * h * h;
            sH += H;
        }
    if (c->p.model == 1) {
        double a1 = h * h * sH - c->A1, a2 = h * h * ((double)n * m - sH) - (1.0 - c->A1);
        E += c->p.nu * (a1 * a1 + a2 * a2);
    }
    return E;
}

/* ------------------------------------------------------------------------ */
/* Projected explicit time-marching of phi_t = N(phi) (the "time-marching"  */
/* solver the Algorithm-1 box names for the coarse grid), on level 0 with   */
/* F = 0: phi <- clamp(phi + tau N(phi)), tau = cfl / max S(phi); c1, c2     */
/* refreshed every crefresh steps.  Returns the final relative projected     */
/* residual.                                                                  */
double or_timemarch(or_ctx *c, long steps, double cfl, int crefresh, double tol)
{
    or_level *L = &c->lev[0];
    size_t N = (size_t)L->n * L->m;
    double *Nv = dalloc(N);
    double *A = dalloc(N), *B = dalloc(N), *C = dalloc(N), *D = dalloc(N), *S = dalloc(N), *f = dalloc(N);
    double rel = 1.0;
    for (long it = 0; it < steps; it++) {
        coeffs_at(c, 0, L->phi, A, B, C, D, S, f);
        double smax = 0.0;
        for (size_t q = 0; q < N; q++) if (S[q] > smax) smax = S[q];
        apply_N(c, 0, L->phi, Nv);
        double tau = smax > 0.0 ? cfl / smax : cfl;
        for (size_t q = 0; q < N; q++) L->phi[q] = clampB(L->phi[q] + tau * Nv[q], L->lo[q], L->hi[q]);
        if (crefresh > 0 && (it + 1) % crefresh == 0) {
            update_c(c); update_fit(c);
            rel = or_res_norm(c) / c->res0;
            if (rel <= tol) break;
        }
    }
    free(Nv); free(A); free(B); free(C); free(D); free(S); free(f);
    return rel;
}

/* ------------------------------------------------------------------------ */
/* AOS: additive operator splitting, the semi-implicit time stepper of the  */
/* comparison in Sec. 5 (Table 4) and one of the "exact" solvers Algorithm 1 */
/* names for the coarsest grid.  The paper gives no formula of its own; this */
/* is the standard scheme (Weickert, ter Haar Romeny & Viergever 1998) for   */
/* phi_t = N(phi) - F on level l with the coefficients of eq. abcdrc frozen  */
/* at phi^k:                                                                  */
/*   y_1 = (I - 2 tau A_1)^{-1} (phi^k - tau (f + F))   (A_1: the couplings  */
/*         A, B to i+1, i-1, one tridiagonal system per column),              */
/*   y_2 = (I - 2 tau A_2)^{-1} (phi^k - tau (f + F))   (A_2: C, D to j+-1,  */
/*         one system per row),                                               */
/*   phi^{k+1} = clamp((y_1 + y_2) / 2, lo, hi).                              */
/* A_1 and A_2 have zero row sums, so each factor keeps constants.  tau_hat  */
/* is the step in units of h / mu, so that 2 tau A = 2 tau_hat G with G the  */
/* face values.                                                               */

/* Thomas algorithm for lo_k x_{k-1} + di_k x_k + up_k x_{k+1} = x_k (the    */
/* right-hand side in x, the solution returned there); the rows are strictly */
/* diagonally dominant, so no pivoting is needed.  cp: n doubles of scratch. */
static void tridiag_solve(int n, const double *lo, const double *di, const double *up, double *x, double *cp)
{
    double den = di[0];
    cp[0] = up[0] / den;
    x[0] = x[0] / den;
    for (int k = 1; k < n; k++) {
        den = di[k] - lo[k] * cp[k - 1];
        cp[k] = up[k] / den;
        x[k] = (x[k] - lo[k] * x[k - 1]) / den;
    }
    for (int k = n - 2; k >= 0; k--) x[k] -= cp[k] * x[k + 1];
}
void or_tridiag_solve(int n, const double *lo, const double *di, const double *up, double *x)
{
    double *cp = dalloc((size_t)n);
    tridiag_solve(n, lo, di, up, x, cp);
    free(cp);
}

/* one AOS step on level l; returns |phi^{k+1} - phi^k| / |phi^k| */
static double aos_step(or_ctx *c, int l, double tau_hat)
{
    or_level *L = &c->lev[l];
    int n = L->n, m = L->m;
    size_t N = (size_t)n * m;
    double tau = tau_hat * L->h / c->p.mu;
    double *A = dalloc(N), *B = dalloc(N), *C = dalloc(N), *D = dalloc(N), *S = dalloc(N), *f = dalloc(N);
    double *rhs = dalloc(N), *y1 = dalloc(N), *y2 = dalloc(N);
    int K = n > m ? n : m;
    double *lo = dalloc((size_t)K), *di = dalloc((size_t)K), *up = dalloc((size_t)K), *x = dalloc((size_t)K),
           *cp = dalloc((size_t)K);
    coeffs_at(c, l, L->phi, A, B, C, D, S, f);
    for (size_t q = 0; q < N; q++) rhs[q] = L->phi[q] - tau * (f[q] + L->F[q]);
    for (int j = 0; j < m; j++) {          /* columns: i varies */
        for (int i = 0; i < n; i++) {
            size_t q = (size_t)i * m + j;
            lo[i] = -2.0 * tau * B[q];
            up[i] = -2.0 * tau * A[q];
            di[i] = 1.0 + 2.0 * tau * (A[q] + B[q]);
            x[i] = rhs[q];
        }
        tridiag_solve(n, lo, di, up, x, cp);
        for (int i = 0; i < n; i++) y1[(size_t)i * m + j] = x[i];
    }
    for (int i = 0; i < n; i++) {          /* rows: j varies */
        for (int j = 0; j < m; j++) {
            size_t q = (size_t)i * m + j;
            lo[j] = -2.0 * tau * D[q];
            up[j] = -2.0 * tau * C[q];
            di[j] = 1.0 + 2.0 * tau * (C[q] + D[q]);
            x[j] = rhs[q];
        }
        tridiag_solve(m, lo, di, up, x, cp);
        for (int j = 0; j < m; j++) y2[(size_t)i * m + j] = x[j];
    }
    double dn = 0.0, pn = 0.0;
    for (size_t q = 0; q < N; q++) {
        double v = clampB(0.5 * (y1[q] + y2[q]), L->lo[q], L->hi[q]);
        dn += (v - L->phi[q]) * (v - L->phi[q]);
        pn += L->phi[q] * L->phi[q];
        L->phi[q] = v;
    }
    free(A); free(B); free(C); free(D); free(S); free(f);
    free(rhs); free(y1); free(y2); free(lo); free(di); free(up); free(x); free(cp);
    return pn > 0.0 ? sqrt(dn / pn) : 0.0;
}

/* one AOS step of the finest grid (F = 0), then c1, c2 refreshed */
double or_aos_step(or_ctx *c, double tau_hat)
{
    or_level *L = &c->lev[0];
    memset(L->F, 0, sizeof(double) * (size_t)L->n * L->m);
    double eta = aos_step(c, 0, tau_hat);
    update_c(c);
    update_fit(c);
    return eta;
}

/* AOS solve of the finest grid: steps until the relative change falls     */
/* below eta_tol (the stopping rule of the comparison in Sec. 5); returns   */
/* the number of steps (negative: not reached), the changes in hist.        */
int or_aos(or_ctx *c, double tau_hat, double eta_tol, int max_iters, double *hist)
{
    int k;
    for (k = 0; k < max_iters; k++) {
        double eta = or_aos_step(c, tau_hat);
        if (hist) hist[k] = eta;
        if (eta < eta_tol) return k + 1;
    }
    return -k;
}

/* ------------------------------------------------------------------------ */
/* accessors and single-step entry points for the tests                     */
int or_levels(or_ctx *c) { return c->L; }
void or_level_shape(or_ctx *c, int l, int *n, int *m, double *h) { *n = c->lev[l].n; *m = c->lev[l].m; *h = c->lev[l].h; }
void or_scalars(or_ctx *c, double *out)
{
    out[0] = c->c1; out[1] = c->c2; out[2] = c->A1; out[3] = c->res0; out[4] = c->h0;
}
void or_set_c(or_ctx *c, double c1, double c2) { c->c1 = c1; c->c2 = c2; update_fit(c); }
void or_set_res0(or_ctx *c, double r0) { c->res0 = r0; }
void or_set_res0_rows(or_ctx *c, double r0) { c->res0_rows = r0; }

/* field ids: 0 z, 1 d, 2 w, 3 fit, 4 phi, 5 F, 6 A, 7 B, 8 C, 9 D, 10 S, 11 f, 12 g (level 0 only), */
/* 13 lo, 14 hi, 15 phic (the restricted state of the last coarse problem) */
static double *field(or_ctx *c, int l, int id)
{
    or_level *L = &c->lev[l];
    switch (id) {
    case 0: return L->z; case 1: return L->d; case 2: return L->w; case 3: return L->fit;
    case 4: return L->phi; case 5: return L->F; case 6: return L->A; case 7: return L->B;
    case 8: return L->C; case 9: return L->D; case 10: return L->S; case 11: return L->f;
    case 12: return l == 0 ? c->g0 : NULL;
    case 13: return L->lo; case 14: return L->hi; case 15: return L->phic;
    default: return NULL;
    }
}
int or_get(or_ctx *c, int l, int id, double *out)
{
    double *f = field(c, l, id);
    if (!f) return -1;
    memcpy(out, f, sizeof(double) * (size_t)c->lev[l].n * c->lev[l].m);
    return 0;
}
int or_set(or_ctx *c, int l, int id, const double *in)
{
    double *f = field(c, l, id);
    if (!f) return -1;
    memcpy(f, in, sizeof(double) * (size_t)c->lev[l].n * c->lev[l].m);
    return 0;
}
void or_get_labels(or_ctx *c, int l, uint8_t *out) { memcpy(out, c->lev[l].lab, (size_t)c->lev[l].n * c->lev[l].m); }
void or_set_labels(or_ctx *c, int l, const uint8_t *in) { memcpy(c->lev[l].lab, in, (size_t)c->lev[l].n * c->lev[l].m); }

/* single steps on level l */
void or_step_freeze(or_ctx *c, int l) { freeze(c, l); }
/* s: 0-3 the sweeps of Hybrid Smoother 2, 4 GSLEX-I, 5 Hybrid Smoother 1, 6 GSLINE-I, 7 NEWT-I, */
/* 8 GSLEX-II, 9 GSLINE-II, 10 NEWT-II (after a freeze)                                         */
void or_step_sweep(or_ctx *c, int l, int s)
{
    switch (s) {
    case 4: gslex_sweep(c, l); break;
    case 5: hs1_outer(c, l); break;
    case 6: gsline_sweep(c, l); break;
    case 7: newt_sweep(c, l); break;
    case 8: point_local_sweep(c, l, 0); break;
    case 9: gsline_local_sweep(c, l); break;
    case 10: point_local_sweep(c, l, 1); break;
    default: hs2_sweep(c, l, s);
    }
}
void or_step_smooth(or_ctx *c, int l, int iters) { smooth(c, l, iters); }
/* NEWT's diagonal term Q' of every cell of level l at its current phi */
void or_newton_qprime(or_ctx *c, int l, double *out)
{
    or_level *L = &c->lev[l];
    double area = area_term(c, l, L->phi);
    for (size_t q = 0; q < (size_t)L->n * L->m; q++) out[q] = newton_qprime(c, L, L->phi[q], area);
}
void or_step_coarsest(or_ctx *c, int l) { coarsest(c, l); }
void or_step_vcycle_level(or_ctx *c, int l) { vcycle_level(c, l); }
void or_step_to_coarse(or_ctx *c, int l) { if (l + 1 < c->L) to_coarse(c, l); }
void or_step_residual(or_ctx *c, int l, double *r, int project) { residual(c, l, c->lev[l].phi, c->lev[l].F, r, project); }
void or_step_operator(or_ctx *c, int l, double *out) { apply_N(c, l, c->lev[l].phi, out); }
void or_step_update_c(or_ctx *c) { update_c(c); update_fit(c); }
double or_step_area_term(or_ctx *c, int l) { return area_term(c, l, c->lev[l].phi); }
