/*
 * Plain FP64 C oracle for D3 with Becke-Johnson damping.
 *
 * TEST INFRASTRUCTURE ONLY: called by the test suite and by the benchmark's
 * CPU-baseline leg, never by the product path, with which it shares no code.
 *
 * It computes the same quantities as the NumPy oracle, by the same plain
 * definitions (Ying & Fan, Sec. II A):
 *   entries   all (i, j, T) with (j,T) != (i,0) and |r_j + T - r_i|^2 < R^2,
 *             by brute force over every atom j and every lattice translation
 *             T that can reach R, or (cell-list mode, for large cells) from
 *             the bins within R of the atom's bin, each bin offset taken
 *             once with its own image translation;
 *   n_i       Eq. 4 over entries with r < R_cn;
 *   C6        Eq. 3 per entry, the double sum over reference pairs with all
 *             exponents shifted by their maximum (the shift cancels);
 *   U_i, E    Eqs. 2 and 1 with C8 = C6 R0^2, R0^2 = 3 r2r4_i r2r4_j; or,
 *             with zero damping, -s_n C_n f_n / r^n, f_n = 1 / (1 + 6 (r /
 *             (s_r,n R0))^-alpha_n), alpha 14 and 16, and optionally the
 *             three-body (Axilrod-Teller-Muto) term, both as defined by the
 *             D3 reference the paper cites (Grimme et al. 2010) for the
 *             variants the paper sets aside;
 *   F_i       exact -dE/dr_i: a direct term at fixed C6 plus the chain term
 *             through dE/dn (C6 depends on the coordination numbers);
 *   W         -dE/d(strain) = Eq. 7 summed over atoms;
 *   W_i       Eq. 7 per atom: the terms of W from the entries of atom i
 *             (each pair's term split half and half between its atoms).
 * Per-atom partial virials are summed in atom order at the end, so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXREF 5
static const double HARTREE_EV = 27.211386245988;
static const double BOHR_ANG = 0.529177210903;

typedef struct {
    int n, cap;
    int *j;
    double *d; /* 3 per entry */
} elist;

static void push(elist *l, int j, double dx, double dy, double dz)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 64;
        l->j = (int *)realloc(l->j, sizeof(int) * l->cap);
        l->d = (double *)realloc(l->d, sizeof(double) * 3 * l->cap);
    }
    l->j[l->n] = j;
    l->d[3 * l->n + 0] = dx;
    l->d[3 * l->n + 1] = dy;
    l->d[3 * l->n + 2] = dz;
    l->n++;
}

static void inv3(const double *m, double *o)
{
    double det = m[0] * (m[4] * m[8] - m[5] * m[7]) -
                 m[1] * (m[3] * m[8] - m[5] * m[6]) +
                 m[2] * (m[3] * m[7] - m[4] * m[6]);
    o[0] = (m[4] * m[8] - m[5] * m[7]) / det;
    o[1] = (m[2] * m[7] - m[1] * m[8]) / det;
    o[2] = (m[1] * m[5] - m[2] * m[4]) / det;
    o[3] = (m[5] * m[6] - m[3] * m[8]) / det;
    o[4] = (m[0] * m[8] - m[2] * m[6]) / det;
    o[5] = (m[2] * m[3] - m[0] * m[5]) / det;
    o[6] = (m[3] * m[7] - m[4] * m[6]) / det;
    o[7] = (m[1] * m[6] - m[0] * m[7]) / det;
    o[8] = (m[0] * m[4] - m[1] * m[3]) / det;
}

/* translations reaching rmax: |n_k| <= ceil(rmax/h_k + spread_k) */
static int make_translations(int n, const double *pos, const double *cell,
                             const int *pbc, double rmax, double **tv)
{
    double inv[9], spread[3] = {0, 0, 0}, lo[3], hi[3];
    int reach[3], k;
    inv3(cell, inv);
    for (k = 0; k < 3; k++) { lo[k] = 1e300; hi[k] = -1e300; }
    for (int i = 0; i < n; i++)
        for (k = 0; k < 3; k++) {
            double s = pos[3 * i] * inv[k] + pos[3 * i + 1] * inv[3 + k] +
                       pos[3 * i + 2] * inv[6 + k];
            if (s < lo[k]) lo[k] = s;
            if (s > hi[k]) hi[k] = s;
        }
    for (k = 0; k < 3; k++) spread[k] = n ? hi[k] - lo[k] : 1.0;
    double vol = fabs(cell[0] * (cell[4] * cell[8] - cell[5] * cell[7]) -
                      cell[1] * (cell[3] * cell[8] - cell[5] * cell[6]) +
                      cell[2] * (cell[3] * cell[7] - cell[4] * cell[6]));
    for (k = 0; k < 3; k++) {
        if (!pbc[k]) { reach[k] = 0; continue; }
        const double *u = cell + 3 * ((k + 1) % 3), *v = cell + 3 * ((k + 2) % 3);
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
               cz = u[0] * v[1] - u[1] * v[0];
        double h = vol / sqrt(cx * cx + cy * cy + cz * cz);
        reach[k] = (int)ceil(rmax / h + spread[k]);
    }
    int nt = (2 * reach[0] + 1) * (2 * reach[1] + 1) * (2 * reach[2] + 1);
    double *t = (double *)malloc(sizeof(double) * 4 * nt);
    int c = 0;
    for (int a = -reach[0]; a <= reach[0]; a++)
        for (int b = -reach[1]; b <= reach[1]; b++)
            for (int q = -reach[2]; q <= reach[2]; q++) {
                for (k = 0; k < 3; k++)
                    t[4 * c + k] = a * cell[k] + b * cell[3 + k] + q * cell[6 + k];
                t[4 * c + 3] = (a == 0 && b == 0 && q == 0) ? 1.0 : 0.0;
                c++;
            }
    *tv = t;
    return nt;
}

/* Eq. 3 with derivative wrt the first CN; refs of element zi and zj */
static double c6_eq3(int ki, const double *ri, int kj, const double *rj,
                     const double *cref /* [MAXREF][MAXREF] of (zi,zj) */,
                     double ni, double nj, double *dc6_dni)
{
    double x[MAXREF][MAXREF], xmax = -1e300;
    for (int a = 0; a < ki; a++)
        for (int b = 0; b < kj; b++) {
            double da = ni - ri[a], db = nj - rj[b];
            x[a][b] = -4.0 * (da * da + db * db);
            if (x[a][b] > xmax) xmax = x[a][b];
        }
    double Z = 0, S = 0, Zd = 0, Sd = 0;
    for (int a = 0; a < ki; a++)
        for (int b = 0; b < kj; b++) {
            double L = exp(x[a][b] - xmax);
            double dx = -8.0 * (ni - ri[a]);
            double c = cref[a * MAXREF + b];
            Z += L;
            S += c * L;
            Zd += L * dx;
            Sd += c * L * dx;
        }
    double c6 = S / Z;
    *dc6_dni = (Sd - c6 * Zd) / Z;
    return c6;
}

/* OpenMP threads of the process at the first call (OMP_NUM_THREADS or the
 * host's cores): the count an evaluation with n_threads = 0 uses */
static int default_threads(void)
{
#ifdef _OPENMP
    static int t = 0;
    if (t == 0) t = omp_get_max_threads();
    return t;
#else
    return 1;
#endif
}

/* threads an evaluation with n_threads uses (0: the default) */
int d3ref_threads_for(int n_threads)
{
#ifdef _OPENMP
    return n_threads > 0 ? n_threads : default_threads();
#else
    (void)n_threads;
    return 1;
#endif
}

int d3ref_threads(void) { return d3ref_threads_for(0); }

/* ------------------------------------------------------------------
 * Cell-list enumeration of the same entries.  Positions are wrapped into
 * the cell on periodic axes; the displacement set {r_j + T - r_i} over all
 * lattice translations T does not change under wrapping.  Along a periodic
 * axis k the cell is cut into nb_k bins at least rc (1 + 1e-9) wide, or
 * one bin when it is thinner; an atom's neighbours within rc then lie in
 * the bins whose index differs by at most reach_k = ceil(rc nb_k / h_k)
 * (h_k the distance between lattice planes), every such offset taken once
 * with its own image translation, so short cells are visited several
 * times with different images.  Open axes hold one bin and no image.
 * ------------------------------------------------------------------ */
typedef struct {
    int nb[3], reach[3];
    int *start; /* nb0*nb1*nb2 + 1 offsets into order */
    int *order; /* atom indices sorted by bin, by index inside a bin */
    const double *xw; /* wrapped positions (n,3) */
    const double *cell;
    int pbc[3];
} cgrid;

static void grid_build(cgrid *g, int n, const double *xw, const double *sfrac,
                       const double *cell, const int *pbc, double rc)
{
    double vol = fabs(cell[0] * (cell[4] * cell[8] - cell[5] * cell[7]) -
                      cell[1] * (cell[3] * cell[8] - cell[5] * cell[6]) +
                      cell[2] * (cell[3] * cell[7] - cell[4] * cell[6]));
    g->xw = xw;
    g->cell = cell;
    for (int k = 0; k < 3; k++) {
        g->pbc[k] = pbc[k] ? 1 : 0;
        if (!pbc[k]) { g->nb[k] = 1; g->reach[k] = 0; continue; }
        const double *u = cell + 3 * ((k + 1) % 3), *v = cell + 3 * ((k + 2) % 3);
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2],
               cz = u[0] * v[1] - u[1] * v[0];
        double h = vol / sqrt(cx * cx + cy * cy + cz * cz);
        long nb = (long)floor(h / (rc * (1.0 + 1e-9)));
        if (nb < 1) nb = 1;
        if (nb > 512) nb = 512;
        g->nb[k] = (int)nb;
        g->reach[k] = (int)ceil(rc * (double)nb / h * (1.0 + 1e-9));
    }
    size_t nbins = (size_t)g->nb[0] * g->nb[1] * g->nb[2];
    int *bin = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    g->start = (int *)calloc(nbins + 1, sizeof(int));
    g->order = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int i = 0; i < n; i++) {
        int b[3];
        for (int k = 0; k < 3; k++) {
            int q = g->pbc[k] ? (int)floor(sfrac[3 * i + k] * g->nb[k]) : 0;
            b[k] = q < 0 ? 0 : (q >= g->nb[k] ? g->nb[k] - 1 : q);
        }
        bin[i] = (b[2] * g->nb[1] + b[1]) * g->nb[0] + b[0];
        g->start[bin[i] + 1]++;
    }
    for (size_t b = 0; b < nbins; b++) g->start[b + 1] += g->start[b];
    int *fill = (int *)calloc(nbins, sizeof(int));
    for (int i = 0; i < n; i++) g->order[g->start[bin[i]] + fill[bin[i]]++] = i;
    free(fill);
    free(bin);
}

static void grid_free(cgrid *g)
{
    free(g->start);
    free(g->order);
}

static int floordiv_i(int a, int b)
{
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

/* entries of atom i within rc from the grid, appended to l (cleared) */
static void grid_gather(const cgrid *g, int i, double rc, const double *sfrac, elist *l)
{
    const double rc2 = rc * rc;
    const double *x = g->xw;
    int b[3];
    l->n = 0;
    for (int k = 0; k < 3; k++) {
        int q = g->pbc[k] ? (int)floor(sfrac[3 * i + k] * g->nb[k]) : 0;
        b[k] = q < 0 ? 0 : (q >= g->nb[k] ? g->nb[k] - 1 : q);
    }
    for (int d2 = -g->reach[2]; d2 <= g->reach[2]; d2++)
        for (int d1 = -g->reach[1]; d1 <= g->reach[1]; d1++)
            for (int d0 = -g->reach[0]; d0 <= g->reach[0]; d0++) {
                int u[3] = {b[0] + d0, b[1] + d1, b[2] + d2}, t[3], w[3];
                for (int k = 0; k < 3; k++) {
                    t[k] = floordiv_i(u[k], g->nb[k]);
                    w[k] = u[k] - t[k] * g->nb[k];
                }
                double T[3];
                for (int m = 0; m < 3; m++)
                    T[m] = t[0] * g->cell[m] + t[1] * g->cell[3 + m] + t[2] * g->cell[6 + m];
                const int self_img = t[0] == 0 && t[1] == 0 && t[2] == 0;
                int bb = (w[2] * g->nb[1] + w[1]) * g->nb[0] + w[0];
                for (int q = g->start[bb]; q < g->start[bb + 1]; q++) {
                    int j = g->order[q];
                    if (j == i && self_img) continue;
                    double dx = x[3 * j] + T[0] - x[3 * i];
                    double dy = x[3 * j + 1] + T[1] - x[3 * i + 1];
                    double dz = x[3 * j + 2] + T[2] - x[3 * i + 2];
                    if (dx * dx + dy * dy + dz * dz < rc2) push(l, j, dx, dy, dz);
                }
            }
}

/* ------------------------------------------------------------------
 * Per-atom physics, shared by both enumerations.  Each takes atom i's
 * entries (j, d = r_j + T - r_i) within at least the cutoff it needs and
 * applies the hard cutoff itself.
 * ------------------------------------------------------------------ */
typedef struct {
    int ne;
    const int *types, *n_ref;
    const double *cn_ref, *rcov, *c6, *r0sq;
    double s6, a1, s8, a2, rp2, rc2;
    int zero;          /* 0: Becke-Johnson damping (Eq. 2); 1: zero damping */
    double rs6, rs8;   /* zero damping: s_r,6, s_r,8 */
    double s9, ra2;    /* three-body scale and cutoff squared */
} phys;

/* zero damping of -s C / r^n: f = 1 / (1 + 6 (r / (sr R0))^-alpha); returns
 * the term's value, sets *de_r to its r-derivative over r and *g to f/r^n */
static double zero_term(double r2, double c, double s, double sr, double r0, int n,
                        double alpha, double *de_r, double *g)
{
    double r = sqrt(r2);
    double q = pow(r / (sr * r0), -alpha);
    double f = 1.0 / (1.0 + 6.0 * q);
    double rn = pow(r2, 0.5 * n);
    *de_r = -s * c * (6.0 * alpha * q * f * f - n * f) / (rn * r2);
    *g = f / rn;
    return -s * c * f / rn;
}

/* ATM geometry and damping of one triangle with squared sides a = AB^2,
 * b = BC^2, c = CA^2 and pair radii r0ab, r0bc, r0ca:
 * g = (1 + 3 cosA cosB cosC) / (r_AB r_BC r_CA)^3 f3 with the cosine
 * product (a + c - b)(a + b - c)(b + c - a) / (8abc), f3 = 1 / (1 + 6
 * (rbar / (4/3 R0bar))^-16) (geometric means); derivatives in ga, gb, gc */
static double atm_g(double a, double b, double c, double r0ab, double r0bc, double r0ca,
                    double *ga, double *gb, double *gc)
{
    const double alpha = 16.0, sr3 = 4.0 / 3.0;
    double u = a * b * c;
    double x = a + c - b, y = a + b - c, z = b + c - a;
    double P = x * y * z;
    double dP[3] = {y * z + x * z - x * y, x * z - y * z + x * y, y * z - x * z + x * y};
    double du[3] = {b * c, a * c, a * b};
    double ang = 1.0 + 3.0 * P / (8.0 * u);
    double k0 = pow(sr3 * sr3 * sr3 * r0ab * r0bc * r0ca, alpha / 3.0);
    double q = k0 * pow(u, -alpha / 6.0);
    double f3 = 1.0 / (1.0 + 6.0 * q);
    double u15 = pow(u, -1.5);
    double *out[3] = {ga, gb, gc};
    for (int k = 0; k < 3; k++) {
        double dang = 3.0 / 8.0 * (dP[k] * u - P * du[k]) / (u * u);
        double du15 = -1.5 * u15 / u * du[k];
        double df3 = 6.0 * f3 * f3 * q * (alpha / 6.0) * du[k] / u;
        *out[k] = dang * u15 * f3 + ang * du15 * f3 + ang * u15 * df3;
    }
    return ang * u15 * f3;
}

/* Eq. 4 */
static double cn_atom(const phys *P, int i, const elist *l)
{
    double s = 0;
    for (int e = 0; e < l->n; e++) {
        const double *d = l->d + 3 * e;
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < P->rc2)) continue;
        double r = sqrt(r2), rs = P->rcov[P->types[i]] + P->rcov[P->types[l->j[e]]];
        s += 1.0 / (1.0 + exp(-16.0 * (rs / r - 1.0)));
    }
    return s;
}

/* Eqs. 2-3: site energy, direct force at fixed C6, dE/dn_i, the direct
 * part of the atom's virial; returns the number of entries within R_pot */
static long disp_atom(const phys *P, int i, const elist *l, const double *cn, double *u_out,
                      double *g_out, double *f_out, double *w_out)
{
    int zi = P->types[i], ne = P->ne;
    double u = 0, gi = 0, fx = 0, fy = 0, fz = 0, w[6] = {0, 0, 0, 0, 0, 0};
    long total = 0;
    for (int e = 0; e < l->n; e++) {
        const double *d = l->d + 3 * e;
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < P->rp2)) continue;
        total++;
        int j = l->j[e], zj = P->types[j];
        double dci;
        double c = c6_eq3(P->n_ref[zi], P->cn_ref + MAXREF * zi, P->n_ref[zj],
                          P->cn_ref + MAXREF * zj,
                          P->c6 + ((size_t)zi * ne + zj) * MAXREF * MAXREF, cn[i], cn[j], &dci);
        double q = P->r0sq[zi * ne + zj];
        double phi, dphi_r, dphi_dc6;
        if (P->zero) {
            double d6, d8, g6, g8, r0 = sqrt(q);
            phi = zero_term(r2, c, P->s6, P->rs6, r0, 6, 14.0, &d6, &g6) +
                  zero_term(r2, c * q, P->s8, P->rs8, r0, 8, 16.0, &d8, &g8);
            dphi_r = d6 + d8;
            dphi_dc6 = -(P->s6 * g6 + P->s8 * q * g8);
        } else {
            double rd = P->a1 * sqrt(q) + P->a2;
            double rd2 = rd * rd, rd6 = rd2 * rd2 * rd2, rd8 = rd6 * rd2;
            double r6 = r2 * r2 * r2, r8 = r6 * r2;
            double t6 = 1.0 / (r6 + rd6), t8 = 1.0 / (r8 + rd8);
            phi = -(P->s6 * c * t6 + P->s8 * c * q * t8);
            dphi_r = P->s6 * c * 6.0 * r2 * r2 * t6 * t6 + P->s8 * c * q * 8.0 * r6 * t8 * t8;
            dphi_dc6 = -(P->s6 * t6 + P->s8 * q * t8);
        }
        u += 0.5 * phi;
        gi += dphi_dc6 * dci;
        fx += dphi_r * d[0];
        fy += dphi_r * d[1];
        fz += dphi_r * d[2];
        w[0] -= 0.5 * dphi_r * d[0] * d[0];
        w[1] -= 0.5 * dphi_r * d[0] * d[1];
        w[2] -= 0.5 * dphi_r * d[0] * d[2];
        w[3] -= 0.5 * dphi_r * d[1] * d[1];
        w[4] -= 0.5 * dphi_r * d[1] * d[2];
        w[5] -= 0.5 * dphi_r * d[2] * d[2];
    }
    *u_out = u;
    *g_out = gi;
    f_out[0] = fx;
    f_out[1] = fy;
    f_out[2] = fz;
    for (int k = 0; k < 6; k++) w_out[k] = w[k];
    return total;
}

/* three-body (ATM) term of atom i: every pair of its entries within
 * r_atm whose third side is also within r_atm is a triangle it belongs to;
 * adds a third of each triangle's energy and virial, the triangle's force
 * on i and its dE/dn_i */
static void atm_atom(const phys *P, int i, const elist *l, const double *cn, double *u_out,
                     double *g_out, double *f, double *w)
{
    int ne = P->ne, zi = P->types[i];
    double u = 0, gi = 0;
    for (int e1 = 0; e1 < l->n; e1++) {
        const double *d1 = l->d + 3 * e1;
        double a = d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2];
        if (!(a < P->ra2)) continue;
        int jb = l->j[e1], zb = P->types[jb];
        double dab, cab = c6_eq3(P->n_ref[zi], P->cn_ref + MAXREF * zi, P->n_ref[zb],
                                 P->cn_ref + MAXREF * zb,
                                 P->c6 + ((size_t)zi * ne + zb) * MAXREF * MAXREF, cn[i], cn[jb],
                                 &dab);
        for (int e2 = e1 + 1; e2 < l->n; e2++) {
            const double *d2 = l->d + 3 * e2;
            double c = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
            if (!(c < P->ra2)) continue;
            double bx = d2[0] - d1[0], by = d2[1] - d1[1], bz = d2[2] - d1[2];
            double b = bx * bx + by * by + bz * bz;
            if (!(b < P->ra2)) continue;
            int jc = l->j[e2], zc = P->types[jc];
            double dac, dummy;
            double cac = c6_eq3(P->n_ref[zi], P->cn_ref + MAXREF * zi, P->n_ref[zc],
                                P->cn_ref + MAXREF * zc,
                                P->c6 + ((size_t)zi * ne + zc) * MAXREF * MAXREF, cn[i], cn[jc],
                                &dac);
            double cbc = c6_eq3(P->n_ref[zb], P->cn_ref + MAXREF * zb, P->n_ref[zc],
                                P->cn_ref + MAXREF * zc,
                                P->c6 + ((size_t)zb * ne + zc) * MAXREF * MAXREF, cn[jb], cn[jc],
                                &dummy);
            double ga, gb, gc;
            double g = atm_g(a, b, c, sqrt(P->r0sq[zi * ne + zb]), sqrt(P->r0sq[zb * ne + zc]),
                             sqrt(P->r0sq[zc * ne + zi]), &ga, &gb, &gc);
            double cc = P->s9 * sqrt(cab * cbc * cac);
            double E = cc * g;
            u += E / 3.0;
            gi += 0.5 * E * (dab / cab + dac / cac);
            f[0] += 2.0 * cc * (ga * d1[0] + gc * d2[0]);
            f[1] += 2.0 * cc * (ga * d1[1] + gc * d2[1]);
            f[2] += 2.0 * cc * (ga * d1[2] + gc * d2[2]);
            double ha = -2.0 * cc * ga / 3.0, hb = -2.0 * cc * gb / 3.0, hc = -2.0 * cc * gc / 3.0;
            w[0] += ha * d1[0] * d1[0] + hb * bx * bx + hc * d2[0] * d2[0];
            w[1] += ha * d1[0] * d1[1] + hb * bx * by + hc * d2[0] * d2[1];
            w[2] += ha * d1[0] * d1[2] + hb * bx * bz + hc * d2[0] * d2[2];
            w[3] += ha * d1[1] * d1[1] + hb * by * by + hc * d2[1] * d2[1];
            w[4] += ha * d1[1] * d1[2] + hb * by * bz + hc * d2[1] * d2[2];
            w[5] += ha * d1[2] * d1[2] + hb * bz * bz + hc * d2[2] * d2[2];
        }
    }
    *u_out += u;
    *g_out += gi;
}

/* chain term through the coordination numbers, added to f and w */
static void chain_atom(const phys *P, int i, const elist *l, const double *g, double *f,
                       double *w)
{
    for (int e = 0; e < l->n; e++) {
        const double *d = l->d + 3 * e;
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (!(r2 < P->rc2)) continue;
        int j = l->j[e];
        double r = sqrt(r2), rs = P->rcov[P->types[i]] + P->rcov[P->types[j]];
        double ex = exp(-16.0 * (rs / r - 1.0));
        double df = -16.0 * rs * ex / (r2 * (1.0 + ex) * (1.0 + ex));
        double coef = (g[i] + g[j]) * df / r;
        f[0] += coef * d[0];
        f[1] += coef * d[1];
        f[2] += coef * d[2];
        w[0] -= 0.5 * coef * d[0] * d[0];
        w[1] -= 0.5 * coef * d[0] * d[1];
        w[2] -= 0.5 * coef * d[0] * d[2];
        w[3] -= 0.5 * coef * d[1] * d[1];
        w[4] -= 0.5 * coef * d[1] * d[2];
        w[5] -= 0.5 * coef * d[2] * d[2];
    }
}

/*
 * Full evaluation.  Table arrays: n_ref[ne], cn_ref[ne][5],
 * c6_au[ne][ne][5][5] (Hartree bohr^6), rcov[ne] (A), r2r4[ne] (bohr).
 * use_cells: 0 = entries by brute force over every atom and translation,
 * kept for all atoms; 1 = entries from cell lists, found again in each
 * pass (memory O(n); the mode for large cells).  n_eval < n (cell-list
 * mode only, for timing a sample of a large cell): each pass runs for
 * atoms 0..n_eval-1 only, so the work is that of n_eval atoms of the cell
 * but the results are not those of the cell.  Outputs (any may be NULL
 * except energy): forces[n][3], virial[9], atom_energy[n], cn[n],
 * dedn[n], atom_virial[n][9].  Returns the number of entries within
 * R_pot (>= 0).
 */
long d3ref_evaluate_mode(int n, const double *pos, const int *types,
                         const double *cell, const int *pbc, int ne,
                         const int *n_ref, const double *cn_ref,
                         const double *c6_au, const double *rcov,
                         const double *r2r4, double s6, double a1, double s8,
                         double a2, double r_pot, double r_cn, int damping, double rs6,
                         double rs8, double s9, double r_atm, int n_threads,
                         int use_cells, int n_eval, double *energy, double *forces,
                         double *virial, double *atom_energy, double *cn_out,
                         double *dedn_out, double *atom_virial)
{
    double idcell[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    int nopbc[3] = {0, 0, 0};
    if (!cell) { cell = idcell; pbc = nopbc; }
#ifdef _OPENMP
    omp_set_num_threads(d3ref_threads_for(n_threads));
#endif
    const int atm = s9 != 0.0;
    double rmax = r_pot > r_cn ? r_pot : r_cn;
    if (atm && r_atm > rmax) rmax = r_atm;
    double *c6 = (double *)malloc(sizeof(double) * ne * ne * MAXREF * MAXREF);
    double *r0sq = (double *)malloc(sizeof(double) * ne * ne);
    const double conv = HARTREE_EV * pow(BOHR_ANG, 6);
    for (int q = 0; q < ne * ne * MAXREF * MAXREF; q++) c6[q] = c6_au[q] * conv;
    for (int e = 0; e < ne; e++)
        for (int f = 0; f < ne; f++)
            r0sq[e * ne + f] = 3.0 * r2r4[e] * r2r4[f] * BOHR_ANG * BOHR_ANG;
    phys P = {ne, types, n_ref, cn_ref, rcov, c6, r0sq, s6, a1, s8, a2,
              r_pot * r_pot, r_cn * r_cn, damping, rs6, rs8, s9, r_atm * r_atm};

    double *cn = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *g = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *ue = (double *)calloc(n > 0 ? n : 1, sizeof(double));
    double *fo = (double *)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
    double *wv = (double *)calloc(6 * (size_t)(n > 0 ? n : 1), sizeof(double));
    long total = 0;

    if (!use_cells) {
        double *tv = NULL;
        int nt = make_translations(n, pos, cell, pbc, rmax, &tv);
        const double rm2 = rmax * rmax;
        elist *L = (elist *)calloc(n > 0 ? n : 1, sizeof(elist));
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; i++) {
            const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
            for (int j = 0; j < n; j++)
                for (int t = 0; t < nt; t++) {
                    if (j == i && tv[4 * t + 3] != 0.0) continue;
                    double dx = pos[3 * j] + tv[4 * t] - xi;
                    double dy = pos[3 * j + 1] + tv[4 * t + 1] - yi;
                    double dz = pos[3 * j + 2] + tv[4 * t + 2] - zi;
                    if (dx * dx + dy * dy + dz * dz < rm2) push(&L[i], j, dx, dy, dz);
                }
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; i++) cn[i] = cn_atom(&P, i, &L[i]);
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
        for (int i = 0; i < n; i++)
            total += disp_atom(&P, i, &L[i], cn, &ue[i], &g[i], fo + 3 * (size_t)i,
                               wv + 6 * (size_t)i);
        if (atm) {
#pragma omp parallel for schedule(dynamic, 16)
            for (int i = 0; i < n; i++)
                atm_atom(&P, i, &L[i], cn, &ue[i], &g[i], fo + 3 * (size_t)i, wv + 6 * (size_t)i);
        }
#pragma omp parallel for schedule(dynamic, 64)
        for (int i = 0; i < n; i++) chain_atom(&P, i, &L[i], g, fo + 3 * (size_t)i, wv + 6 * (size_t)i);
        for (int i = 0; i < n; i++) { free(L[i].j); free(L[i].d); }
        free(L);
        free(tv);
    } else {
        /* wrapped positions and their fractional coordinates */
        double inv[9];
        inv3(cell, inv);
        double *xw = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        double *sf = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
        for (int i = 0; i < n; i++) {
            double s[3], fl[3];
            for (int k = 0; k < 3; k++) {
                s[k] = pos[3 * i] * inv[k] + pos[3 * i + 1] * inv[3 + k] + pos[3 * i + 2] * inv[6 + k];
                fl[k] = pbc[k] ? floor(s[k]) : 0.0;
                sf[3 * i + k] = s[k] - fl[k];
            }
            for (int m = 0; m < 3; m++)
                xw[3 * i + m] = pos[3 * i + m] - fl[0] * cell[m] - fl[1] * cell[3 + m] -
                                fl[2] * cell[6 + m];
        }
        const int ne_atoms = (n_eval >= 0 && n_eval < n) ? n_eval : n;
        cgrid gp, gc, ga;
        grid_build(&gp, n, xw, sf, cell, pbc, r_pot);
        grid_build(&gc, n, xw, sf, cell, pbc, r_cn);
        grid_build(&ga, n, xw, sf, cell, pbc, atm ? r_atm : r_cn);
#pragma omp parallel
        {
            elist l = {0, 0, NULL, NULL};
#pragma omp for schedule(dynamic, 64)
            for (int i = 0; i < ne_atoms; i++) {
                grid_gather(&gc, i, r_cn, sf, &l);
                cn[i] = cn_atom(&P, i, &l);
            }
#pragma omp for schedule(dynamic, 64) reduction(+ : total)
            for (int i = 0; i < ne_atoms; i++) {
                grid_gather(&gp, i, r_pot, sf, &l);
                total += disp_atom(&P, i, &l, cn, &ue[i], &g[i], fo + 3 * (size_t)i,
                                   wv + 6 * (size_t)i);
            }
            if (atm) {
#pragma omp for schedule(dynamic, 16)
                for (int i = 0; i < ne_atoms; i++) {
                    grid_gather(&ga, i, r_atm, sf, &l);
                    atm_atom(&P, i, &l, cn, &ue[i], &g[i], fo + 3 * (size_t)i, wv + 6 * (size_t)i);
                }
            }
#pragma omp for schedule(dynamic, 64)
            for (int i = 0; i < ne_atoms; i++) {
                grid_gather(&gc, i, r_cn, sf, &l);
                chain_atom(&P, i, &l, g, fo + 3 * (size_t)i, wv + 6 * (size_t)i);
            }
            free(l.j);
            free(l.d);
        }
        grid_free(&gp);
        grid_free(&gc);
        grid_free(&ga);
        free(xw);
        free(sf);
    }

    double esum = 0, ws[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < n; i++) {
        esum += ue[i];
        for (int k = 0; k < 6; k++) ws[k] += wv[6 * i + k];
    }
    *energy = esum;
    if (virial) {
        virial[0] = ws[0]; virial[1] = ws[1]; virial[2] = ws[2];
        virial[3] = ws[1]; virial[4] = ws[3]; virial[5] = ws[4];
        virial[6] = ws[2]; virial[7] = ws[4]; virial[8] = ws[5];
    }
    if (forces) memcpy(forces, fo, sizeof(double) * 3 * (size_t)n);
    if (atom_energy) memcpy(atom_energy, ue, sizeof(double) * n);
    if (cn_out) memcpy(cn_out, cn, sizeof(double) * n);
    if (dedn_out) memcpy(dedn_out, g, sizeof(double) * n);
    if (atom_virial)
        for (int i = 0; i < n; i++) {
            const double *w = wv + 6 * (size_t)i;
            double *o = atom_virial + 9 * (size_t)i;
            o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
            o[3] = w[1]; o[4] = w[3]; o[5] = w[4];
            o[6] = w[2]; o[7] = w[4]; o[8] = w[5];
        }
    free(cn); free(g); free(ue); free(fo); free(wv);
    free(c6); free(r0sq);
    return total;
}

/* brute-force evaluation (d3ref_evaluate_mode with use_cells = 0) */
long d3ref_evaluate(int n, const double *pos, const int *types,
                    const double *cell, const int *pbc, int ne,
                    const int *n_ref, const double *cn_ref,
                    const double *c6_au, const double *rcov,
                    const double *r2r4, double s6, double a1, double s8,
                    double a2, double r_pot, double r_cn, int n_threads,
                    double *energy, double *forces, double *virial,
                    double *atom_energy, double *cn_out, double *dedn_out,
                    double *atom_virial)
{
    return d3ref_evaluate_mode(n, pos, types, cell, pbc, ne, n_ref, cn_ref, c6_au, rcov, r2r4,
                               s6, a1, s8, a2, r_pot, r_cn, 0, 1.217, 1.0, 0.0, r_cn, n_threads,
                               0, n, energy, forces,
                               virial, atom_energy, cn_out, dedn_out, atom_virial);
}
