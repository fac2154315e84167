/*
 * nopcs_oracle.c -- plain FP64 CPU oracle for the NOHAP/OUCS3 compressible
 * Navier-Stokes hot path of "Ultrasound Triggering of Rayleigh-Taylor
 * Instability: Solution of Compressible Navier-Stokes Equation by a
 * Non-Overlapping Parallel Compact Scheme" (Sundaram, Sengupta, Sengupta).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU library: it has its own constants, its own tridiagonal solver,
 * its own equivalent-explicit rows and its own physics.
 *
 * Everything is FP64, non-dimensional (Section 2, eqs. ge14-ge15), written
 * for readability: plain loops over lines, OpenMP only across independent
 * lines.  Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared.
 *
 * Readings of the paper used here (each also listed in the design notes):
 *  - OUCS3 (eta = 0) interior rows with antisymmetric B (Section 3, the
 *    A/B entries printed after Eq. CS:AfpBf; the signs are not printed, the
 *    consistency 1 + 2 alpha = 2 b1 + 4 b2 and the Appendix fix them).
 *  - Physical-boundary closures are cited but not given (Section 3): rows 0
 *    and n-1 use the second-order one-sided difference, rows 1 and n-2 the
 *    second-order central difference.
 *  - The plain definition of the derivative is the sequential global solve
 *    [A]{f'} = [B]{f} on each full line (Section 3: the NOHAP closure is
 *    "equivalent to treating the full domain as a single domain").  The
 *    segmented NOHAP evaluation is implemented separately to pin that claim.
 *  - Segment-end rows use the row of the global C = A^-1 B (Eq. CS:fpCf),
 *    truncated to |j - e| <= n_b = 48 (Eq. CS:fpCf_i), also near walls.
 *  - Energy is carried as E' = rho e_t - E_ref with E_ref = Rh/(gamma-1),
 *    Rh = R* T_s / (g L) (the equation of state after ge20); this is an
 *    exact constant shift of the fifth conserved variable.
 *  - Viscous fluxes and "other gradients" use second-order explicit
 *    differences (Section 4, first paragraph), central inside and one-sided
 *    at walls, for the inner gradients and the outer divergence alike.
 *  - Classical four-stage RK4 (Section 4); wall conditions applied after each
 *    stage: zero momentum, adiabatic wall temperature from the one-sided
 *    second-order normal derivative set to zero, density from continuity.
 *  - The implicit filter of Section 4 (cited, not printed) is read as the
 *    fourth-order tridiagonal compact filter with the printed coefficient
 *    0.135, wall rows unfiltered, applied along x, y, z in turn.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* OUCS3 with eta = 0: A_{i,i+-1} = alpha, A_{i,i} = 1,                      */
/* B_{i,i+-1} = +-b1/h, B_{i,i+-2} = +-b2/h  (Section 3, after Eq. CS:AfpBf) */
/* ------------------------------------------------------------------------ */
static const double ORA_ALPHA = 0.3793894912;
static const double ORA_B1 = 0.7877868952;
static const double ORA_B2 = 0.045801298;
enum { ORA_NB = 48 }; /* semi-bandwidth n_b (Section 3, after Eq. CS:fpCf_i) */

double ora_alpha(void) { return ORA_ALPHA; }
double ora_b1(void) { return ORA_B1; }
double ora_b2(void) { return ORA_B2; }
int ora_nb(void) { return ORA_NB; }

/* ------------------------------------------------------------------------ */
/* General tridiagonal solve (Thomas algorithm, Section 3).                  */
/* sub[i] x[i-1] + dia[i] x[i] + sup[i] x[i+1] = rhs[i], i = 0..m-1.         */
/* work: m doubles.  x may alias rhs.                                        */
/* ------------------------------------------------------------------------ */
void ora_thomas(int m, const double *sub, const double *dia, const double *sup,
                const double *rhs, double *x, double *work)
{
    double *cp = work;
    double dp_prev = 0.0, cp_prev = 0.0;
    for (int i = 0; i < m; ++i) {
        double s = (i > 0) ? sub[i] : 0.0;
        double den = dia[i] - s * cp_prev;
        double dp = (rhs[i] - s * dp_prev) / den;
        cp[i] = (i < m - 1) ? sup[i] / den : 0.0;
        x[i] = dp;
        dp_prev = dp;
        cp_prev = cp[i];
    }
    for (int i = m - 2; i >= 0; --i)
        x[i] = x[i] - cp[i] * x[i + 1];
}

/* ------------------------------------------------------------------------ */
/* Global line operator.  Rows 0, 1, n-2, n-1: explicit second order (the    */
/* physical-boundary closure reading).  Rows 2..n-3: OUCS3 compact.          */
/* All derivative values carry the factor ih = 1/h.                          */
/* ------------------------------------------------------------------------ */
static double wall_left0(const double *f, ptrdiff_t s, double ih)
{   /* (-3 f0 + 4 f1 - f2) / 2h */
    return 0.5 * ih * (4.0 * (f[s] - f[0]) - (f[2 * s] - f[0]));
}
static double wall_left1(const double *f, ptrdiff_t s, double ih)
{   /* (f2 - f0) / 2h at row 1 */
    return 0.5 * ih * (f[2 * s] - f[0]);
}
static double wall_right1(const double *f, ptrdiff_t s, int n, double ih)
{   /* (f_{n-1} - f_{n-3}) / 2h at row n-2 */
    return 0.5 * ih * (f[(ptrdiff_t)(n - 1) * s] - f[(ptrdiff_t)(n - 3) * s]);
}
static double wall_right0(const double *f, ptrdiff_t s, int n, double ih)
{   /* (3 f_{n-1} - 4 f_{n-2} + f_{n-3}) / 2h */
    double fl = f[(ptrdiff_t)(n - 1) * s];
    return -0.5 * ih * (4.0 * (f[(ptrdiff_t)(n - 2) * s] - fl) - (f[(ptrdiff_t)(n - 3) * s] - fl));
}
static double compact_rhs(const double *f, ptrdiff_t s, int i, double ih)
{   /* (B f)_i = [b1 (f_{i+1} - f_{i-1}) + b2 (f_{i+2} - f_{i-2})] / h */
    const double *c = f + (ptrdiff_t)i * s;
    return ih * (ORA_B1 * (c[s] - c[-s]) + ORA_B2 * (c[2 * s] - c[-2 * s]));
}

static int is_wall_row(int i, int n) { return i <= 1 || i >= n - 2; }

static double wall_row_value(const double *f, ptrdiff_t s, int n, int i, double ih)
{
    if (i == 0) return wall_left0(f, s, ih);
    if (i == 1) return wall_left1(f, s, ih);
    if (i == n - 2) return wall_right1(f, s, n, ih);
    return wall_right0(f, s, n, ih);
}

/* Solve the compact rows strictly between two known rows lo < hi of a line:
 * alpha x_{i-1} + x_i + alpha x_{i+1} = d_i for lo < i < hi, x_lo and x_hi
 * known (already in x).  d holds (B f)_i. */
static void solve_run(int lo, int hi, const double *d, double *x, double *work)
{
    int m = hi - lo - 1;
    if (m <= 0) return;
    double *sub = work, *dia = work + m, *sup = work + 2 * m, *rhs = work + 3 * m, *w = work + 4 * m;
    for (int k = 0; k < m; ++k) {
        int i = lo + 1 + k;
        sub[k] = ORA_ALPHA;
        dia[k] = 1.0;
        sup[k] = ORA_ALPHA;
        double r = d[i];
        if (k == 0) r = r - ORA_ALPHA * x[lo];
        if (k == m - 1) r = r - ORA_ALPHA * x[hi];
        rhs[k] = r;
    }
    ora_thomas(m, sub, dia, sup, rhs, x + lo + 1, w);
}

/* Sequential (one-segment) first derivative of one line: the plain
 * definition [A]{f'} = [B]{f} of Eq. CS:AfpBf.  f has stride sf, result df
 * stride sd.  work: 8n doubles.  n >= 5. */
void ora_d1_line(int n, double ih, const double *f, ptrdiff_t sf, double *df, ptrdiff_t sd, double *work)
{
    double *x = work, *d = work + n, *w = work + 2 * n;
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    x[0] = wall_row_value(f, sf, n, 0, ih);
    x[1] = wall_row_value(f, sf, n, 1, ih);
    x[n - 2] = wall_row_value(f, sf, n, n - 2, ih);
    x[n - 1] = wall_row_value(f, sf, n, n - 1, ih);
    for (int i = 2; i <= n - 3; ++i) d[i] = compact_rhs(f, sf, i, ih);
    solve_run(1, n - 2, d, x, w);
    for (int i = 0; i < n; ++i) df[(ptrdiff_t)i * sd] = x[i];
}

/* ------------------------------------------------------------------------ */
/* Row e of the equivalent explicit operator C = A^-1 B of the global line   */
/* (Eq. CS:fpCf), with h = 1.  row: n doubles.  Method: solve A^T y = e_e    */
/* and set row_j = sum_i y_i B_ij.  work: 8n doubles.                        */
/* ------------------------------------------------------------------------ */
void ora_equiv_row(int n, int e, double *row, double *work)
{
    double *sub = work, *dia = work + n, *sup = work + 2 * n, *rhs = work + 3 * n,
           *y = work + 4 * n, *w = work + 5 * n;
    /* A: rows 0, 1, n-2, n-1 identity; rows 2..n-3: alpha, 1, alpha. */
    /* (A^T)_{j,j-1} = A_{j-1,j}, (A^T)_{j,j+1} = A_{j+1,j}.          */
    for (int j = 0; j < n; ++j) {
        double a_jm1_j = (j - 1 >= 2 && j - 1 <= n - 3) ? ORA_ALPHA : 0.0; /* A_{j-1,j} */
        double a_jp1_j = (j + 1 >= 2 && j + 1 <= n - 3) ? ORA_ALPHA : 0.0; /* A_{j+1,j} */
        sub[j] = (j > 0) ? a_jm1_j : 0.0;
        sup[j] = (j < n - 1) ? a_jp1_j : 0.0;
        dia[j] = 1.0;
        rhs[j] = (j == e) ? 1.0 : 0.0;
    }
    ora_thomas(n, sub, dia, sup, rhs, y, w);
    for (int j = 0; j < n; ++j) row[j] = 0.0;
    for (int i = 0; i < n; ++i) {
        double yi = y[i];
        if (yi == 0.0) continue;
        if (i == 0) {
            row[0] += yi * -1.5; row[1] += yi * 2.0; row[2] += yi * -0.5;
        } else if (i == 1) {
            row[0] += yi * -0.5; row[2] += yi * 0.5;
        } else if (i == n - 2) {
            row[n - 3] += yi * -0.5; row[n - 1] += yi * 0.5;
        } else if (i == n - 1) {
            row[n - 3] += yi * 0.5; row[n - 2] += yi * -2.0; row[n - 1] += yi * 1.5;
        } else {
            row[i - 2] += yi * -ORA_B2; row[i - 1] += yi * -ORA_B1;
            row[i + 1] += yi * ORA_B1;  row[i + 2] += yi * ORA_B2;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Segmented NOHAP first derivative of one line (Section 3, Fig. 2).         */
/* Segments s = 0..nseg-1 start at seg_lo[s] (seg_lo[0] = 0, increasing) and */
/* end at seg_lo[s+1]-1 (last ends at n-1).  The first and last point of each */
/* segment that is not a domain boundary row is a segment end: its          */
/* derivative is the truncated equivalent explicit sum (Eq. CS:fpCf_i) with */
/* the row of the global C.  The remaining rows of each segment are solved  */
/* independently by the Thomas algorithm.  work: 16n doubles.               */
/* ------------------------------------------------------------------------ */
void ora_d1_line_seg(int n, double ih, int nseg, const int *seg_lo, const double *f,
                     ptrdiff_t sf, double *df, ptrdiff_t sd, double *work)
{
    double *x = work, *d = work + n, *row = work + 2 * n, *w = work + 3 * n;
    char *known = (char *)(work + 13 * n);
    memset(known, 0, (size_t)n);
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    for (int i = 0; i < n; ++i)
        if (is_wall_row(i, n)) { x[i] = wall_row_value(f, sf, n, i, ih); known[i] = 1; }
    for (int s = 0; s < nseg; ++s) {
        int lo = seg_lo[s], hi = (s + 1 < nseg) ? seg_lo[s + 1] - 1 : n - 1;
        int ends[2] = {lo, hi};
        for (int q = 0; q < 2; ++q) {
            int e = ends[q];
            if ((q == 0 && s == 0) || (q == 1 && s == nseg - 1)) continue;
            if (is_wall_row(e, n)) continue;
            ora_equiv_row(n, e, row, w);
            int j0 = e - ORA_NB < 0 ? 0 : e - ORA_NB;
            int j1 = e + ORA_NB > n - 1 ? n - 1 : e + ORA_NB;
            double acc = 0.0;
            for (int j = j0; j <= j1; ++j) acc += row[j] * f[(ptrdiff_t)j * sf];
            x[e] = ih * acc;
            known[e] = 1;
        }
    }
    for (int i = 2; i <= n - 3; ++i)
        if (!known[i]) d[i] = compact_rhs(f, sf, i, ih);
    /* every maximal run of unknown rows lies between two known rows */
    int lo = 1;
    for (int i = 2; i <= n - 2; ++i) {
        if (known[i]) { solve_run(lo, i, d, x, w); lo = i; }
    }
    for (int i = 0; i < n; ++i) df[(ptrdiff_t)i * sd] = x[i];
}

/* ------------------------------------------------------------------------ */
/* 3D helpers: field f[k][j][i], i (x) fastest.                             */
/* ------------------------------------------------------------------------ */
static void line_geometry(const int n[3], int dir, ptrdiff_t *stride, long *nlines)
{
    ptrdiff_t s[3] = {1, n[0], (ptrdiff_t)n[0] * n[1]};
    *stride = s[dir];
    *nlines = (long)n[0] * n[1] * n[2] / n[dir];
}
static ptrdiff_t line_base(const int n[3], int dir, long l)
{
    int a = (dir == 0) ? 1 : 0, b = (dir == 2) ? 1 : 2;   /* the two cross directions */
    ptrdiff_t s[3] = {1, n[0], (ptrdiff_t)n[0] * n[1]};
    long ia = l % n[a], ib = l / n[a];
    return ia * s[a] + ib * s[b];
}

/* First derivative along dir of a 3D field by global line solves.  len is   */
/* the non-dimensional box edge (h = len/(n-1)).                             */
void ora_d1_3d(const int n[3], const double len[3], int dir, const double *f, double *df)
{
    ptrdiff_t st; long nl;
    line_geometry(n, dir, &st, &nl);
    int nd = n[dir];
    double ih = (double)(nd - 1) / len[dir];
    #pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 8 * (size_t)nd);
        #pragma omp for schedule(static)
        for (long l = 0; l < nl; ++l) {
            ptrdiff_t b = line_base(n, dir, l);
            ora_d1_line(nd, ih, f + b, st, df + b, st, work);
        }
        free(work);
    }
}

/* Segmented (NOHAP) first derivative along dir with nseg near-equal segments. */
void ora_d1_3d_seg(const int n[3], const double len[3], int dir, int nseg, const int *seg_lo,
                   const double *f, double *df)
{
    ptrdiff_t st; long nl;
    line_geometry(n, dir, &st, &nl);
    int nd = n[dir];
    double ih = (double)(nd - 1) / len[dir];
    #pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 16 * (size_t)nd);
        #pragma omp for schedule(static)
        for (long l = 0; l < nl; ++l) {
            ptrdiff_t b = line_base(n, dir, l);
            ora_d1_line_seg(nd, ih, nseg, seg_lo, f + b, st, df + b, st, work);
        }
        free(work);
    }
}

/* Second derivative as the first-derivative operator applied twice. */
void ora_d2_3d(const int n[3], const double len[3], int dir, const double *f, double *d2f)
{
    size_t N = (size_t)n[0] * n[1] * n[2];
    double *tmp = (double *)malloc(sizeof(double) * N);
    ora_d1_3d(n, len, dir, f, tmp);
    ora_d1_3d(n, len, dir, tmp, d2f);
    free(tmp);
}

/* ------------------------------------------------------------------------ */
/* Physics (Section 2).  SI parameters in, non-dimensional constants out.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double gamma, R_gas, g, L, T_s, rho_s, Pr, mu_ref, T_ref, S_suth, mub_a, mub_b;
    int32_t viscous, gravity;
} ora_params;

typedef struct {
    double gamma, Rh, Re, M2, Pr, St, mu_s, kappa, Eref, H, ghat, iRe, mub_a, mub_b, T_s;
    int viscous;
} ora_nd;

static double sutherland_dim(const ora_params *p, double Tdim)
{   /* mu(T) = mu_ref (T/T_ref)^{3/2} (T_ref + S)/(T + S) */
    double r = Tdim / p->T_ref;
    return p->mu_ref * r * sqrt(r) * (p->T_ref + p->S_suth) / (Tdim + p->S_suth);
}

/* Scales of Section 2: U_s = sqrt(g L), t_s = sqrt(L/g); Re = rho_s U_s L / mu_s,
 * M = U_s / sqrt(gamma R T_s); R = R* T_s / U_s^2 (equation of state after ge20). */
void ora_nondim(const ora_params *p, ora_nd *o)
{
    double Us = sqrt(p->g * p->L);
    o->gamma = p->gamma;
    o->Rh = p->R_gas * p->T_s / (p->g * p->L);
    o->M2 = (p->g * p->L) / (p->gamma * p->R_gas * p->T_s);
    o->mu_s = sutherland_dim(p, p->T_s);
    o->Re = p->rho_s * Us * p->L / o->mu_s;
    o->iRe = 1.0 / o->Re;
    o->Pr = p->Pr;
    o->St = p->S_suth / p->T_s;
    o->kappa = 1.0 / ((p->gamma - 1.0) * p->Pr * o->Re * o->M2);   /* ge20 */
    o->Eref = o->Rh / (p->gamma - 1.0);
    o->H = o->Eref + o->Rh;
    o->ghat = p->gravity ? 1.0 : 0.0;   /* g L / U_s^2 = 1 */
    o->mub_a = p->mub_a;
    o->mub_b = p->mub_b;
    o->T_s = p->T_s;
    o->viscous = p->viscous;
}

/* Non-dimensional scales exposed for tests: out = {Us, ts, Rh, M, Re, mu_s} */
void ora_scales(const ora_params *p, double *out)
{
    ora_nd o;
    ora_nondim(p, &o);
    out[0] = sqrt(p->g * p->L);
    out[1] = sqrt(p->L / p->g);
    out[2] = o.Rh;
    out[3] = sqrt(o.M2);
    out[4] = o.Re;
    out[5] = o.mu_s;
}

typedef struct { double rho, u, v, w, pp, T, mu, beta; } ora_prim;

/* Primitive recovery from Q = [rho, rho u, rho v, rho w, E'] (ge2, ge12, ge13). */
static ora_prim prim_at(const ora_nd *o, const double *Q, size_t N, size_t c)
{
    ora_prim q;
    double rho = Q[c], mx = Q[N + c], my = Q[2 * N + c], mz = Q[3 * N + c], Ep = Q[4 * N + c];
    double ri = 1.0 / rho;
    q.rho = rho;
    q.u = mx * ri; q.v = my * ri; q.w = mz * ri;
    double ke = 0.5 * (mx * q.u + my * q.v + mz * q.w);
    q.pp = (o->gamma - 1.0) * (Ep - ke);                 /* p - p_ref */
    q.T = (q.pp + o->Rh) / (rho * o->Rh);                /* p = rho R T */
    q.mu = q.T * sqrt(q.T) * (1.0 + o->St) / (q.T + o->St);   /* Sutherland, mu/mu_s */
    q.beta = (o->mub_a * (q.T * o->T_s) - o->mub_b) / o->mu_s; /* eq. reg, mu_b/mu_s */
    return q;
}

/* second-order explicit derivative along one axis at index i of a line of n */
static double d2nd(const double *f, ptrdiff_t s, int i, int n, double ih)
{
    const double *c = f + (ptrdiff_t)i * s;
    if (i == 0) return 0.5 * ih * (4.0 * (c[s] - c[0]) - (c[2 * s] - c[0]));
    if (i == n - 1) return -0.5 * ih * (4.0 * (c[-s] - c[0]) - (c[-2 * s] - c[0]));
    return 0.5 * ih * (c[s] - c[-s]);
}

static void idx3(const int n[3], size_t c, int *i, int *j, int *k)
{
    *i = (int)(c % (size_t)n[0]);
    *j = (int)((c / (size_t)n[0]) % (size_t)n[1]);
    *k = (int)(c / ((size_t)n[0] * n[1]));
}

/* Right-hand side of ge17:
 *   R = dEv/dx + dFv/dy + dGv/dz + S - dE/dx - dF/dy - dG/dz
 * accumulated in that order.  Convective terms use the OUCS3 global solve,
 * viscous terms the explicit second-order differences (Section 4).
 * Q, R: 5 fields of n0*n1*n2 each, field-major. */
static void rhs_impl(const ora_params *p, const int n[3], const double len[3], const double *Q, double *R,
                     int compact_visc)
{
    ora_nd o;
    ora_nondim(p, &o);
    size_t N = (size_t)n[0] * n[1] * n[2];
    ptrdiff_t st[3] = {1, n[0], (ptrdiff_t)n[0] * n[1]};
    double ih[3];
    for (int d = 0; d < 3; ++d) ih[d] = (double)(n[d] - 1) / len[d];

    double *u = malloc(sizeof(double) * N), *v = malloc(sizeof(double) * N),
           *w = malloc(sizeof(double) * N), *T = malloc(sizeof(double) * N),
           *pp = malloc(sizeof(double) * N), *mu = malloc(sizeof(double) * N),
           *be = malloc(sizeof(double) * N);
    #pragma omp parallel for schedule(static)
    for (size_t c = 0; c < N; ++c) {
        ora_prim q = prim_at(&o, Q, N, c);
        u[c] = q.u; v[c] = q.v; w[c] = q.w; T[c] = q.T; pp[c] = q.pp; mu[c] = q.mu; be[c] = q.beta;
    }
    for (size_t c = 0; c < 5 * N; ++c) R[c] = 0.0;

    /* ---- viscous fluxes (ge6-ge8, ge19, ge20, bv1-bv3) and their divergence ---- */
    if (o.viscous) {
        double *Fv = malloc(sizeof(double) * 12 * N);   /* [dir][comp 1..4][N] */
        /* compact variant: the twelve gradients of (u, v, w, T) by the compact
         * first derivative (global line solves), [a][d][N] */
        double *Gc = NULL;
        if (compact_visc) {
            const double *fa[4] = {u, v, w, T};
            Gc = malloc(sizeof(double) * 12 * N);
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d) ora_d1_3d(n, len, d, fa[a], Gc + (size_t)(a * 3 + d) * N);
        }
        #pragma omp parallel for schedule(static)
        for (size_t c = 0; c < N; ++c) {
            int i, j, k;
            idx3(n, c, &i, &j, &k);
            int ijk[3] = {i, j, k};
            double g[4][3];   /* d(u,v,w,T)/d(x,y,z) */
            const double *fld[4] = {u, v, w, T};
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d) {
                    size_t base = c - (size_t)ijk[d] * (size_t)st[d];
                    g[a][d] = compact_visc ? Gc[(size_t)(a * 3 + d) * N + c]
                                           : d2nd(fld[a] + base, st[d], ijk[d], n[d], ih[d]);
                }
            double m = mu[c], b = be[c];
            double A = (4.0 / 3.0) * m + b, B = b - (2.0 / 3.0) * m;
            double txx = (A * g[0][0] + B * (g[1][1] + g[2][2])) * o.iRe;
            double tyy = (A * g[1][1] + B * (g[0][0] + g[2][2])) * o.iRe;
            double tzz = (A * g[2][2] + B * (g[0][0] + g[1][1])) * o.iRe;
            double txy = m * (g[0][1] + g[1][0]) * o.iRe;
            double txz = m * (g[0][2] + g[2][0]) * o.iRe;
            double tyz = m * (g[1][2] + g[2][1]) * o.iRe;
            double qx = -o.kappa * m * g[3][0], qy = -o.kappa * m * g[3][1], qz = -o.kappa * m * g[3][2];
            double uu = u[c], vv = v[c], ww = w[c];
            double t[3][3] = {{txx, txy, txz}, {txy, tyy, tyz}, {txz, tyz, tzz}};
            double q3[3] = {qx, qy, qz};
            for (int d = 0; d < 3; ++d) {
                Fv[(size_t)(d * 4 + 0) * N + c] = t[d][0];
                Fv[(size_t)(d * 4 + 1) * N + c] = t[d][1];
                Fv[(size_t)(d * 4 + 2) * N + c] = t[d][2];
                Fv[(size_t)(d * 4 + 3) * N + c] = uu * t[d][0] + vv * t[d][1] + ww * t[d][2] - q3[d];
            }
        }
        /* compact variant: each flux component differentiated along its own
         * direction by the compact first derivative, [d][comp][N] */
        if (compact_visc)
            for (int d = 0; d < 3; ++d)
                for (int q = 0; q < 4; ++q)
                    ora_d1_3d(n, len, d, Fv + (size_t)(d * 4 + q) * N, Gc + (size_t)(d * 4 + q) * N);
        #pragma omp parallel for schedule(static)
        for (size_t c = 0; c < N; ++c) {
            int i, j, k;
            idx3(n, c, &i, &j, &k);
            int ijk[3] = {i, j, k};
            for (int comp = 1; comp < 5; ++comp) {
                double acc = 0.0;
                for (int d = 0; d < 3; ++d) {
                    size_t base = c - (size_t)ijk[d] * (size_t)st[d];
                    acc += compact_visc ? Gc[(size_t)(d * 4 + comp - 1) * N + c]
                                        : d2nd(Fv + (size_t)(d * 4 + comp - 1) * N + base, st[d], ijk[d], n[d], ih[d]);
                }
                R[(size_t)comp * N + c] = acc;
            }
        }
        free(Fv);
        free(Gc);
    }

    /* ---- gravity source (ge8a): S = [0, 0, -rho g, 0, -rho v g] ---- */
    #pragma omp parallel for schedule(static)
    for (size_t c = 0; c < N; ++c) {
        R[2 * N + c] = R[2 * N + c] - o.ghat * Q[c];
        R[4 * N + c] = R[4 * N + c] - o.ghat * Q[2 * N + c];
    }

    /* ---- convective fluxes (ge3-ge5) by the compact first derivative ---- */
    double *F = malloc(sizeof(double) * N), *DF = malloc(sizeof(double) * N);
    const double *vel[3] = {u, v, w};
    for (int d = 0; d < 3; ++d) {
        for (int comp = 0; comp < 5; ++comp) {
            const double *ud = vel[d];
            #pragma omp parallel for schedule(static)
            for (size_t c = 0; c < N; ++c) {
                double val;
                if (comp == 0) val = Q[(size_t)(1 + d) * N + c];
                else if (comp <= 3) {
                    val = Q[(size_t)comp * N + c] * ud[c];
                    if (comp - 1 == d) val = val + pp[c];
                } else val = ((Q[4 * N + c] + pp[c]) + o.H) * ud[c];
                F[c] = val;
            }
            ora_d1_3d(n, len, d, F, DF);
            #pragma omp parallel for schedule(static)
            for (size_t c = 0; c < N; ++c)
                R[(size_t)comp * N + c] = R[(size_t)comp * N + c] - DF[c];
        }
    }
    free(F); free(DF);
    free(u); free(v); free(w); free(T); free(pp); free(mu); free(be);
}

/* Right-hand side of ge17 with the viscous terms by the explicit second-order
 * differences of Section 4 (the paper's scheme for the viscous fluxes). */
void ora_rhs(const ora_params *p, const int n[3], const double len[3], const double *Q, double *R)
{
    rhs_impl(p, n, len, Q, R, 0);
}

/* The same right-hand side with every derivative of the viscous terms (the
 * gradients of u, v, w, T inside Ev, Fv, Gv and their divergence) taken by the
 * compact first derivative instead: the D1-based viscous variant.  Operation
 * order otherwise as ora_rhs. */
void ora_rhs_compact_visc(const ora_params *p, const int n[3], const double len[3], const double *Q, double *R)
{
    rhs_impl(p, n, len, Q, R, 1);
}

/* ------------------------------------------------------------------------ */
/* Wall conditions (Section 2: isolated, adiabatically insulated box).       */
/* At every wall node: momentum = 0; T_w from the one-sided second-order     */
/* normal derivative set to zero, T_w = T_1 + (T_1 - T_2)/3; density kept    */
/* (it evolves by continuity); E' from the equation of state with zero       */
/* kinetic energy.  Faces in the order x, y, z.                              */
/* ------------------------------------------------------------------------ */
static double temp_at(const ora_nd *o, const double *Q, size_t N, size_t c)
{
    return prim_at(o, Q, N, c).T;
}

void ora_apply_bc(const ora_params *p, const int n[3], double *Q)
{
    ora_nd o;
    ora_nondim(p, &o);
    size_t N = (size_t)n[0] * n[1] * n[2];
    ptrdiff_t st[3] = {1, n[0], (ptrdiff_t)n[0] * n[1]};
    for (int d = 0; d < 3; ++d) {
        int a = (d == 0) ? 1 : 0, b = (d == 2) ? 1 : 2;
        for (int side = 0; side < 2; ++side) {
            int iw = side ? n[d] - 1 : 0;
            ptrdiff_t inward = side ? -st[d] : st[d];
            #pragma omp parallel for schedule(static)
            for (long l = 0; l < (long)n[a] * n[b]; ++l) {
                long ia = l % n[a], ib = l / n[a];
                size_t c = (size_t)(ia * st[a] + ib * st[b] + (ptrdiff_t)iw * st[d]);
                double T1 = temp_at(&o, Q, N, (size_t)((ptrdiff_t)c + inward));
                double T2 = temp_at(&o, Q, N, (size_t)((ptrdiff_t)c + 2 * inward));
                double Tw = T1 + (T1 - T2) / 3.0;
                double rho = Q[c];
                Q[N + c] = 0.0; Q[2 * N + c] = 0.0; Q[3 * N + c] = 0.0;
                Q[4 * N + c] = (rho * o.Rh * Tw - o.Rh) / (o.gamma - 1.0);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Classical four-stage fourth-order Runge-Kutta (Section 4).                */
/*   k1 = R(q); k2 = R(q + dt/2 k1); k3 = R(q + dt/2 k2); k4 = R(q + dt k3)   */
/*   q  <- q + dt/6 ((((k1) + 2 k2) + 2 k3) + k4)                            */
/* bc (optional) is applied to every stage state and to the new state.      */
/* ------------------------------------------------------------------------ */
typedef void (*ora_rhs_fn)(void *ctx, const double *q, double *r);
typedef void (*ora_bc_fn)(void *ctx, double *q);

void ora_rk4_generic(size_t m, double *q, double dt, int nsteps, ora_rhs_fn rhs, ora_bc_fn bc, void *ctx)
{
    double *qs = malloc(sizeof(double) * m), *k = malloc(sizeof(double) * m),
           *acc = malloc(sizeof(double) * m);
    const double half = 0.5 * dt, sixth = dt / 6.0;
    for (int step = 0; step < nsteps; ++step) {
        rhs(ctx, q, k);                                     /* k1 */
        for (size_t c = 0; c < m; ++c) { acc[c] = k[c]; qs[c] = q[c] + half * k[c]; }
        if (bc) bc(ctx, qs);
        rhs(ctx, qs, k);                                    /* k2 */
        for (size_t c = 0; c < m; ++c) { acc[c] = acc[c] + 2.0 * k[c]; qs[c] = q[c] + half * k[c]; }
        if (bc) bc(ctx, qs);
        rhs(ctx, qs, k);                                    /* k3 */
        for (size_t c = 0; c < m; ++c) { acc[c] = acc[c] + 2.0 * k[c]; qs[c] = q[c] + dt * k[c]; }
        if (bc) bc(ctx, qs);
        rhs(ctx, qs, k);                                    /* k4 */
        for (size_t c = 0; c < m; ++c) q[c] = q[c] + sixth * (acc[c] + k[c]);
        if (bc) bc(ctx, q);
    }
    free(qs); free(k); free(acc);
}

typedef struct { const ora_params *p; const int *n; const double *len; } nse_ctx;
static void nse_rhs_cb(void *ctx, const double *q, double *r)
{
    nse_ctx *c = (nse_ctx *)ctx;
    ora_rhs(c->p, c->n, c->len, q, r);
}
static void nse_bc_cb(void *ctx, double *q)
{
    nse_ctx *c = (nse_ctx *)ctx;
    ora_apply_bc(c->p, c->n, q);
}

/* Advance the NSE state Q (5 fields, field-major, non-dimensional) nsteps. */
void ora_rk4(const ora_params *p, const int n[3], const double len[3], double *Q, double dt, int nsteps)
{
    nse_ctx c = {p, n, len};
    ora_rk4_generic((size_t)5 * n[0] * n[1] * n[2], Q, dt, nsteps, nse_rhs_cb, nse_bc_cb, &c);
}

static void nse_rhs_cv_cb(void *ctx, const double *q, double *r)
{
    nse_ctx *c = (nse_ctx *)ctx;
    ora_rhs_compact_visc(c->p, c->n, c->len, q, r);
}

/* The same stepping with the D1-based viscous variant of the right-hand side. */
void ora_rk4_compact_visc(const ora_params *p, const int n[3], const double len[3], double *Q, double dt, int nsteps)
{
    nse_ctx c = {p, n, len};
    ora_rk4_generic((size_t)5 * n[0] * n[1] * n[2], Q, dt, nsteps, nse_rhs_cv_cb, nse_bc_cb, &c);
}

/* RK4 on the scalar linear test problem dq/dt = lambda q (real lambda),
 * using the same stage driver; used to pin the stage combination. */
typedef struct { double lam; } lin_ctx;
static void lin_rhs(void *ctx, const double *q, double *r)
{
    lin_ctx *c = (lin_ctx *)ctx;
    r[0] = c->lam * q[0];
}
double ora_rk4_linear(double q0, double lam, double dt, int nsteps)
{
    lin_ctx c = {lam};
    double q = q0;
    ora_rk4_generic(1, &q, dt, nsteps, lin_rhs, NULL, &c);
    return q;
}

/* ------------------------------------------------------------------------ */
/* RHS at selected points only (for sampled parity at large sizes): the     */
/* compact derivatives need only the three lines through each point, the    */
/* explicit viscous terms a radius-two neighbourhood.  out: 5 x npts.        */
/* ------------------------------------------------------------------------ */
static double prim_comp(const ora_prim *q, int a)
{
    return a == 0 ? q->u : a == 1 ? q->v : a == 2 ? q->w : q->T;
}

/* derivative of primitive a (u, v, w, T) along axis e at node c */
static double grad_at(const ora_nd *o, const double *Q, const int n[3], const ptrdiff_t st[3],
                      const double ih[3], size_t c, int ie, int a, int e)
{
    size_t N = (size_t)n[0] * n[1] * n[2];
    double f[3];
    int lo = (ie == 0) ? 0 : (ie == n[e] - 1 ? ie - 2 : ie - 1);
    for (int s = 0; s < 3; ++s) {
        ora_prim ps = prim_at(o, Q, N, (size_t)((ptrdiff_t)c + (ptrdiff_t)(lo + s - ie) * st[e]));
        f[s] = prim_comp(&ps, a);
    }
    return d2nd(f, 1, ie - lo, 3, ih[e]);
}

/* viscous flux (E_v, F_v or G_v for d = 0, 1, 2), component comp = 1..4, at c */
static double visc_flux_at(const ora_nd *o, const double *Q, const int n[3], const ptrdiff_t st[3],
                           const double ih[3], size_t c, int d, int comp)
{
    size_t N = (size_t)n[0] * n[1] * n[2];
    int ijk[3];
    idx3(n, c, &ijk[0], &ijk[1], &ijk[2]);
    double g[4][3];
    for (int a = 0; a < 4; ++a)
        for (int e = 0; e < 3; ++e) g[a][e] = grad_at(o, Q, n, st, ih, c, ijk[e], a, e);
    ora_prim pc = prim_at(o, Q, N, c);
    double m = pc.mu, b = pc.beta;
    double A = (4.0 / 3.0) * m + b, B = b - (2.0 / 3.0) * m;
    double txx = (A * g[0][0] + B * (g[1][1] + g[2][2])) * o->iRe;
    double tyy = (A * g[1][1] + B * (g[0][0] + g[2][2])) * o->iRe;
    double tzz = (A * g[2][2] + B * (g[0][0] + g[1][1])) * o->iRe;
    double txy = m * (g[0][1] + g[1][0]) * o->iRe;
    double txz = m * (g[0][2] + g[2][0]) * o->iRe;
    double tyz = m * (g[1][2] + g[2][1]) * o->iRe;
    double t[3][3] = {{txx, txy, txz}, {txy, tyy, tyz}, {txz, tyz, tzz}};
    if (comp < 4) return t[d][comp - 1];
    double qd = -o->kappa * m * g[3][d];
    return pc.u * t[d][0] + pc.v * t[d][1] + pc.w * t[d][2] - qd;
}

void ora_rhs_points(const ora_params *p, const int n[3], const double len[3], const double *Q,
                    int npts, const int *pts /* 3*npts: i,j,k */, double *out)
{
    ora_nd o;
    ora_nondim(p, &o);
    size_t N = (size_t)n[0] * n[1] * n[2];
    ptrdiff_t st[3] = {1, n[0], (ptrdiff_t)n[0] * n[1]};
    double ih[3];
    for (int d = 0; d < 3; ++d) ih[d] = (double)(n[d] - 1) / len[d];
    int nmax = n[0] > n[1] ? n[0] : n[1];
    if (n[2] > nmax) nmax = n[2];

    #pragma omp parallel
    {
        double *F = malloc(sizeof(double) * (size_t)nmax), *DF = malloc(sizeof(double) * (size_t)nmax),
               *work = malloc(sizeof(double) * 8 * (size_t)nmax);
        #pragma omp for schedule(dynamic)
        for (int q = 0; q < npts; ++q) {
            int ijk[3] = {pts[3 * q], pts[3 * q + 1], pts[3 * q + 2]};
            size_t c0 = (size_t)ijk[0] + (size_t)n[0] * ((size_t)ijk[1] + (size_t)n[1] * ijk[2]);
            double r[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (o.viscous) {
                for (int comp = 1; comp < 5; ++comp) {
                    double acc = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        int id = ijk[d];
                        double fv[3];
                        int lo = (id == 0) ? 0 : (id == n[d] - 1 ? id - 2 : id - 1);
                        for (int s = 0; s < 3; ++s) {
                            size_t c = (size_t)((ptrdiff_t)c0 + (ptrdiff_t)(lo + s - id) * st[d]);
                            fv[s] = (id > 0 && id < n[d] - 1 && s == 1) ? 0.0
                                                                        : visc_flux_at(&o, Q, n, st, ih, c, d, comp);
                        }
                        acc += d2nd(fv, 1, id - lo, 3, ih[d]);
                    }
                    r[comp] = acc;
                }
            }
            r[2] = r[2] - o.ghat * Q[c0];
            r[4] = r[4] - o.ghat * Q[2 * N + c0];
            for (int d = 0; d < 3; ++d) {
                size_t base = c0 - (size_t)ijk[d] * (size_t)st[d];
                for (int comp = 0; comp < 5; ++comp) {
                    for (int t = 0; t < n[d]; ++t) {
                        size_t c = base + (size_t)t * (size_t)st[d];
                        ora_prim pc = prim_at(&o, Q, N, c);
                        double ud = d == 0 ? pc.u : d == 1 ? pc.v : pc.w;
                        double val;
                        if (comp == 0) val = Q[(size_t)(1 + d) * N + c];
                        else if (comp <= 3) {
                            val = Q[(size_t)comp * N + c] * ud;
                            if (comp - 1 == d) val = val + pc.pp;
                        } else val = ((Q[4 * N + c] + pc.pp) + o.H) * ud;
                        F[t] = val;
                    }
                    ora_d1_line(n[d], ih[d], F, 1, DF, 1, work);
                    r[comp] = r[comp] - DF[ijk[d]];
                }
            }
            for (int comp = 0; comp < 5; ++comp) out[(size_t)comp * npts + q] = r[comp];
        }
        free(F); free(DF); free(work);
    }
}

/* ------------------------------------------------------------------------ */
/* Implicit low-pass filter, applied every 50 steps with coefficient 0.135  */
/* (Section 4; the paper cites the filter without printing it).  Reading:   */
/* the fourth-order member of the one-parameter family of tridiagonal       */
/* compact filters,                                                         */
/*   af fh_{i-1} + fh_i + af fh_{i+1}                                       */
/*       = a0 f_i + (a1/2)(f_{i+1} + f_{i-1}) + (a2/2)(f_{i+2} + f_{i-2}),  */
/*   a0 = 5/8 + 3af/4,  a1 = 1/2 + af,  a2 = -1/8 + af/4,                   */
/* on rows 2..n-3 of a line; rows 0, 1, n-2, n-1 are left unfiltered.  The  */
/* 3D filter applies it along x, then y, then z.  Its transfer function is  */
/* (a0 + a1 cos t + a2 cos 2t)/(1 + 2 af cos t): 1 at t = 0, 0 at t = pi.   */
/* ------------------------------------------------------------------------ */
static void filter_coefs(double af, double *a0, double *a1, double *a2)
{
    *a0 = 5.0 / 8.0 + 0.75 * af;
    *a1 = 0.5 + af;
    *a2 = -1.0 / 8.0 + 0.25 * af;
}

static double filter_rhs(const double *f, ptrdiff_t s, int i, double af)
{
    double a0, a1, a2;
    filter_coefs(af, &a0, &a1, &a2);
    const double *c = f + (ptrdiff_t)i * s;
    return a0 * c[0] + 0.5 * a1 * (c[s] + c[-s]) + 0.5 * a2 * (c[2 * s] + c[-2 * s]);
}

/* Rows lo+1..hi-1 of a filtered line between two known rows (Thomas).      */
static void filter_run(int lo, int hi, double af, const double *d, double *x, double *work)
{
    int m = hi - lo - 1;
    if (m <= 0) return;
    double *sub = work, *dia = work + m, *sup = work + 2 * m, *rhs = work + 3 * m, *w = work + 4 * m;
    for (int k = 0; k < m; ++k) {
        int i = lo + 1 + k;
        sub[k] = af;
        dia[k] = 1.0;
        sup[k] = af;
        double r = d[i];
        if (k == 0) r = r - af * x[lo];
        if (k == m - 1) r = r - af * x[hi];
        rhs[k] = r;
    }
    ora_thomas(m, sub, dia, sup, rhs, x + lo + 1, w);
}

/* Filter one line: the global (one-segment) solve.  work: 8n doubles. */
void ora_filter_line(int n, double af, const double *f, ptrdiff_t sf, double *fh, ptrdiff_t sh, double *work)
{
    double *x = work, *d = work + n, *w = work + 2 * n;
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    for (int i = 0; i < n; ++i)
        if (is_wall_row(i, n)) x[i] = f[(ptrdiff_t)i * sf];
    for (int i = 2; i <= n - 3; ++i) d[i] = filter_rhs(f, sf, i, af);
    filter_run(1, n - 2, af, d, x, w);
    for (int i = 0; i < n; ++i) fh[(ptrdiff_t)i * sh] = x[i];
}

/* Row e of the filter's equivalent explicit operator C_f = A_f^-1 B_f of the */
/* global line (as ora_equiv_row for the derivative).  work: 8n doubles.     */
void ora_filter_equiv_row(int n, double af, int e, double *row, double *work)
{
    double a0, a1, a2;
    filter_coefs(af, &a0, &a1, &a2);
    double *sub = work, *dia = work + n, *sup = work + 2 * n, *rhs = work + 3 * n,
           *y = work + 4 * n, *w = work + 5 * n;
    for (int j = 0; j < n; ++j) {
        double a_jm1_j = (j - 1 >= 2 && j - 1 <= n - 3) ? af : 0.0;
        double a_jp1_j = (j + 1 >= 2 && j + 1 <= n - 3) ? af : 0.0;
        sub[j] = (j > 0) ? a_jm1_j : 0.0;
        sup[j] = (j < n - 1) ? a_jp1_j : 0.0;
        dia[j] = 1.0;
        rhs[j] = (j == e) ? 1.0 : 0.0;
    }
    ora_thomas(n, sub, dia, sup, rhs, y, w);
    for (int j = 0; j < n; ++j) row[j] = 0.0;
    for (int i = 0; i < n; ++i) {
        double yi = y[i];
        if (yi == 0.0) continue;
        if (is_wall_row(i, n)) {
            row[i] += yi;
        } else {
            row[i - 2] += yi * 0.5 * a2; row[i - 1] += yi * 0.5 * a1; row[i] += yi * a0;
            row[i + 1] += yi * 0.5 * a1; row[i + 2] += yi * 0.5 * a2;
        }
    }
}

/* Segmented NOHAP filter of one line: segment ends take the truncated sum    */
/* with the row of the global C_f (|j - e| <= 48), the other rows of each    */
/* segment are solved on their own.  work: 16n doubles.                      */
void ora_filter_line_seg(int n, double af, int nseg, const int *seg_lo, const double *f, ptrdiff_t sf,
                         double *fh, ptrdiff_t sh, double *work)
{
    double *x = work, *d = work + n, *row = work + 2 * n, *w = work + 3 * n;
    char *known = (char *)(work + 13 * n);
    memset(known, 0, (size_t)n);
    for (int i = 0; i < n; ++i) d[i] = 0.0;
    for (int i = 0; i < n; ++i)
        if (is_wall_row(i, n)) { x[i] = f[(ptrdiff_t)i * sf]; known[i] = 1; }
    for (int s = 0; s < nseg; ++s) {
        int lo = seg_lo[s], hi = (s + 1 < nseg) ? seg_lo[s + 1] - 1 : n - 1;
        int ends[2] = {lo, hi};
        for (int q = 0; q < 2; ++q) {
            int e = ends[q];
            if ((q == 0 && s == 0) || (q == 1 && s == nseg - 1)) continue;
            if (is_wall_row(e, n)) continue;
            ora_filter_equiv_row(n, af, e, row, w);
            int j0 = e - ORA_NB < 0 ? 0 : e - ORA_NB;
            int j1 = e + ORA_NB > n - 1 ? n - 1 : e + ORA_NB;
            double acc = 0.0;
            for (int j = j0; j <= j1; ++j) acc += row[j] * f[(ptrdiff_t)j * sf];
            x[e] = acc;
            known[e] = 1;
        }
    }
    for (int i = 2; i <= n - 3; ++i)
        if (!known[i]) d[i] = filter_rhs(f, sf, i, af);
    int lo = 1;
    for (int i = 2; i <= n - 2; ++i) {
        if (known[i]) { filter_run(lo, i, af, d, x, w); lo = i; }
    }
    for (int i = 0; i < n; ++i) fh[(ptrdiff_t)i * sh] = x[i];
}

/* Filter along dir of a 3D field (global line solves); out may equal f.     */
void ora_filter_dir(const int n[3], int dir, double af, const double *f, double *out)
{
    ptrdiff_t st; long nl;
    line_geometry(n, dir, &st, &nl);
    int nd = n[dir];
    #pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 9 * (size_t)nd);
        double *tmp = work + 8 * nd;
        #pragma omp for schedule(static)
        for (long l = 0; l < nl; ++l) {
            ptrdiff_t b = line_base(n, dir, l);
            ora_filter_line(nd, af, f + b, st, tmp, 1, work);
            for (int i = 0; i < nd; ++i) out[b + (ptrdiff_t)i * st] = tmp[i];
        }
        free(work);
    }
}

/* Segmented filter along dir (NOHAP); out may equal f. */
void ora_filter_dir_seg(const int n[3], int dir, double af, int nseg, const int *seg_lo, const double *f,
                        double *out)
{
    ptrdiff_t st; long nl;
    line_geometry(n, dir, &st, &nl);
    int nd = n[dir];
    #pragma omp parallel
    {
        double *work = (double *)malloc(sizeof(double) * 17 * (size_t)nd);
        double *tmp = work + 16 * nd;
        #pragma omp for schedule(static)
        for (long l = 0; l < nl; ++l) {
            ptrdiff_t b = line_base(n, dir, l);
            ora_filter_line_seg(nd, af, nseg, seg_lo, f + b, st, tmp, 1, work);
            for (int i = 0; i < nd; ++i) out[b + (ptrdiff_t)i * st] = tmp[i];
        }
        free(work);
    }
}

/* The 3D filter of a state: every conserved field along x, then y, then z,  */
/* then the wall conditions (the filtered near-wall values set the adiabatic */
/* wall temperature).  Q in/out. */
void ora_filter_state(const ora_params *p, const int n[3], double af, double *Q)
{
    size_t N = (size_t)n[0] * n[1] * n[2];
    for (int c = 0; c < 5; ++c)
        for (int d = 0; d < 3; ++d) ora_filter_dir(n, d, af, Q + c * N, Q + c * N);
    ora_apply_bc(p, n, Q);
}

/* RK4 stepping with the 3D filter after every `every`-th step (Section 4:   */
/* every 50 steps).  every <= 0: never. */
void ora_rk4_filtered(const ora_params *p, const int n[3], const double len[3], double *Q, double dt, int nsteps,
                      double af, int every)
{
    for (int s = 1; s <= nsteps; ++s) {
        ora_rk4(p, n, len, Q, dt, 1);
        if (every > 0 && s % every == 0) ora_filter_state(p, n, af, Q);
    }
}

/* Number of OpenMP threads a parallel region of the oracle uses. */
#include <omp.h>
int ora_num_threads(void) { return omp_get_max_threads(); }
