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
 *             T that can reach R;
 *   n_i       Eq. 4 over entries with r < R_cn;
 *   C6        Eq. 3 per entry, the double sum over reference pairs with all
 *             exponents shifted by their maximum (the shift cancels);
 *   U_i, E    Eqs. 2 and 1 with C8 = C6 R0^2, R0^2 = 3 r2r4_i r2r4_j;
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

int d3ref_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Full evaluation.  Table arrays: n_ref[ne], cn_ref[ne][5],
 * c6_au[ne][ne][5][5] (Hartree bohr^6), rcov[ne] (A), r2r4[ne] (bohr).
 * Outputs (any may be NULL except energy): forces[n][3], virial[9],
 * atom_energy[n], cn[n], dedn[n], atom_virial[n][9].  Returns the number of entries within
 * R_pot (>= 0) or -1 on allocation failure.
 */
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
    double idcell[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    int nopbc[3] = {0, 0, 0};
    if (!cell) { cell = idcell; pbc = nopbc; }
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
    double rmax = r_pot > r_cn ? r_pot : r_cn;
    double *tv = NULL;
    int nt = make_translations(n, pos, cell, pbc, rmax, &tv);
    double *c6 = (double *)malloc(sizeof(double) * ne * ne * MAXREF * MAXREF);
    double *r0sq = (double *)malloc(sizeof(double) * ne * ne);
    const double conv = HARTREE_EV * pow(BOHR_ANG, 6);
    for (int q = 0; q < ne * ne * MAXREF * MAXREF; q++) c6[q] = c6_au[q] * conv;
    for (int e = 0; e < ne; e++)
        for (int f = 0; f < ne; f++)
            r0sq[e * ne + f] = 3.0 * r2r4[e] * r2r4[f] * BOHR_ANG * BOHR_ANG;

    elist *L = (elist *)calloc(n, sizeof(elist));
    double *cn = (double *)calloc(n, sizeof(double));
    double *g = (double *)calloc(n, sizeof(double));
    double *ue = (double *)calloc(n, sizeof(double));
    double *fo = (double *)calloc(3 * (size_t)n, sizeof(double));
    double *wv = (double *)calloc(6 * (size_t)n, sizeof(double));
    const double rm2 = rmax * rmax, rp2 = r_pot * r_pot, rc2 = r_cn * r_cn;

    /* entries, by brute force */
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
    /* Eq. 4 */
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        double s = 0;
        for (int e = 0; e < L[i].n; e++) {
            const double *d = L[i].d + 3 * e;
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            double r = sqrt(r2), rs = rcov[types[i]] + rcov[types[L[i].j[e]]];
            s += 1.0 / (1.0 + exp(-16.0 * (rs / r - 1.0)));
        }
        cn[i] = s;
    }
    /* Eqs. 2-3: energy, direct force, dE/dn */
    long total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int i = 0; i < n; i++) {
        int zi = types[i];
        double u = 0, gi = 0, fx = 0, fy = 0, fz = 0, w[6] = {0, 0, 0, 0, 0, 0};
        for (int e = 0; e < L[i].n; e++) {
            const double *d = L[i].d + 3 * e;
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rp2)) continue;
            total++;
            int j = L[i].j[e], zj = types[j];
            double dci;
            double c = c6_eq3(n_ref[zi], cn_ref + MAXREF * zi, n_ref[zj],
                              cn_ref + MAXREF * zj,
                              c6 + ((size_t)zi * ne + zj) * MAXREF * MAXREF,
                              cn[i], cn[j], &dci);
            double q = r0sq[zi * ne + zj];
            double rd = a1 * sqrt(q) + a2;
            double rd2 = rd * rd, rd6 = rd2 * rd2 * rd2, rd8 = rd6 * rd2;
            double r6 = r2 * r2 * r2, r8 = r6 * r2;
            double t6 = 1.0 / (r6 + rd6), t8 = 1.0 / (r8 + rd8);
            double phi = -(s6 * c * t6 + s8 * c * q * t8);
            double dphi_r = s6 * c * 6.0 * r2 * r2 * t6 * t6 +
                            s8 * c * q * 8.0 * r6 * t8 * t8;
            u += 0.5 * phi;
            gi += -(s6 * t6 + s8 * q * t8) * dci;
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
        ue[i] = u;
        g[i] = gi;
        fo[3 * i] = fx;
        fo[3 * i + 1] = fy;
        fo[3 * i + 2] = fz;
        for (int k = 0; k < 6; k++) wv[6 * i + k] = w[k];
    }
    /* chain term through the coordination numbers */
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; i++) {
        for (int e = 0; e < L[i].n; e++) {
            const double *d = L[i].d + 3 * e;
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < rc2)) continue;
            int j = L[i].j[e];
            double r = sqrt(r2), rs = rcov[types[i]] + rcov[types[j]];
            double ex = exp(-16.0 * (rs / r - 1.0));
            double df = -16.0 * rs * ex / (r2 * (1.0 + ex) * (1.0 + ex));
            double coef = (g[i] + g[j]) * df / r;
            fo[3 * i] += coef * d[0];
            fo[3 * i + 1] += coef * d[1];
            fo[3 * i + 2] += coef * d[2];
            wv[6 * i + 0] -= 0.5 * coef * d[0] * d[0];
            wv[6 * i + 1] -= 0.5 * coef * d[0] * d[1];
            wv[6 * i + 2] -= 0.5 * coef * d[0] * d[2];
            wv[6 * i + 3] -= 0.5 * coef * d[1] * d[1];
            wv[6 * i + 4] -= 0.5 * coef * d[1] * d[2];
            wv[6 * i + 5] -= 0.5 * coef * d[2] * d[2];
        }
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
    for (int i = 0; i < n; i++) { free(L[i].j); free(L[i].d); }
    free(L); free(cn); free(g); free(ue); free(fo); free(wv);
    free(c6); free(r0sq); free(tv);
    return total;
}
