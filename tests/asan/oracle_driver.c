/*
 * Host AddressSanitizer / UBSan run of the CPU oracle (test infrastructure):
 * the oracle's source is compiled into this driver with -fsanitize=address,
 * undefined and every entry point the tests use is exercised once on a small
 * Kuhn-split mesh (a hard-magnetic 3 x 2 x 2-cell grain in an air box).
 * Exit status 0 means the calls completed; the sanitizers abort on any
 * invalid access, leak or undefined behaviour.
 */
#include "../../oracle/oracle.c"

#include <stdio.h>

/* Kuhn split of an nx x ny x nz box of cubic cells of edge h; cells inside
   [m0, m1) per axis are magnetic (region 1) */
static void kuhn_box(int nx, int ny, int nz, double h, const int m0[3], const int m1[3], double **xyz, long *nn,
                     int **tets, long *nt, int **region) {
    long np = (long)(nx + 1) * (ny + 1) * (nz + 1);
    *xyz = (double *)malloc(sizeof(double) * 3 * np);
    for (int k = 0; k <= nz; k++)
        for (int j = 0; j <= ny; j++)
            for (int i = 0; i <= nx; i++) {
                long v = i + (long)(nx + 1) * (j + (long)(ny + 1) * k);
                (*xyz)[3 * v] = i * h;
                (*xyz)[3 * v + 1] = j * h;
                (*xyz)[3 * v + 2] = k * h;
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    long nc = (long)nx * ny * nz;
    *tets = (int *)malloc(sizeof(int) * 4 * 6 * nc);
    *region = (int *)malloc(sizeof(int) * 6 * nc);
    long t = 0;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int mag = i >= m0[0] && i < m1[0] && j >= m0[1] && j < m1[1] && k >= m0[2] && k < m1[2];
                for (int p = 0; p < 6; p++) {
                    int c[3] = {i, j, k};
                    for (int q = 0; q < 4; q++) {
                        if (q > 0) c[perm[p][q - 1]]++;
                        (*tets)[4 * t + q] = (int)(c[0] + (long)(nx + 1) * (c[1] + (long)(ny + 1) * c[2]));
                    }
                    (*region)[t] = mag;
                    t++;
                }
            }
    *nn = np;
    *nt = t;
}

int main(void) {
    double *xyz;
    int *tets, *region;
    long nn, nt;
    const int m0[3] = {3, 2, 2}, m1[3] = {6, 4, 4};
    kuhn_box(9, 6, 6, 4.0, m0, m1, &xyz, &nn, &tets, &nt, &region);
    double *Ms = (double *)malloc(sizeof(double) * nt), *A = (double *)malloc(sizeof(double) * nt);
    double *K1 = (double *)malloc(sizeof(double) * nt), *ax = (double *)malloc(sizeof(double) * 3 * nt);
    for (long e = 0; e < nt; e++) {
        Ms[e] = 1.61 / OR_MU0;
        A[e] = 7.7e-12;
        K1[e] = 4.3e6;
        ax[3 * e] = 0.1;
        ax[3 * e + 1] = 0.0;
        ax[3 * e + 2] = 0.995;
    }
    or_ctx *c = or_create(xyz, nn, tets, nt, region, Ms, A, K1, ax);
    if (!c) return 2;
    long nm = or_n_mag(c), np = or_n_pot(c);
    double *m = (double *)malloc(sizeof(double) * 3 * nm);
    for (long a = 0; a < nm; a++) {
        double th = 0.1 * ((a * 7919) % 101) / 101.0, ph = 6.283185307179586 * ((a * 104729) % 97) / 97.0;
        m[3 * a] = sin(th) * cos(ph);
        m[3 * a + 1] = sin(th) * sin(ph);
        m[3 * a + 2] = cos(th);
    }
    double E[5], tmax, hT[3] = {0.0, 0.0, -2.0}, h[3];
    double *G = (double *)malloc(sizeof(double) * 3 * nm), *g = (double *)malloc(sizeof(double) * 3 * nm);
    double *lam = (double *)malloc(sizeof(double) * nm), *y = (double *)malloc(sizeof(double) * 3 * nm);
    double *q = (double *)malloc(sizeof(double) * 3 * nm), *b = (double *)malloc(sizeof(double) * np);
    double *u = (double *)calloc(np, sizeof(double));
    or_reduce_field(c, hT, h);
    if (or_eval(c, m, h, 15, E, G, g, lam, &tmax) < 0) return 3;
    or_precond_pub(c, m, lam, g, 10, NULL, y, 3, 0);
    or_apply_P(c, m, lam, g, y, q, 3, 1);
    or_bmul(c, m, b);
    if (or_poisson(c, b, u, 1e-10, 10000) < 0) return 4;
    or_btmul(c, u, q);
    double ac;
    or_cubic_min_pub(1.0, -0.5, -2.0, 1.0, &ac);
    int fb;
    double *dn = (double *)malloc(sizeof(double) * 3 * nm);
    or_direction_pub(0, 3 * nm, g, G, y, q, 1.0, dn, &fb);
    or_opts o = {4, 1e-6, 0, 1e-10, 0.2, 0.01, 1e-4, 0.1, 2000, 15, 20, 0, 0};
    or_stats st;
    int rc = or_minimize(c, m, h, &o, &st, E);
    double fields[9] = {0.0, 0.0, -1.0, 0.0, 0.0, -2.0, 0.0, 0.0, -3.0}, mavg[9], Et[3];
    or_stats sts[3];
    double *hist = (double *)malloc(sizeof(double) * 3 * 3 * nm);
    int rc2 = or_curve(c, m, fields, 3, &o, mavg, Et, sts, hist);
    printf("oracle under sanitizers: n_mag %ld n_pot %ld minimize rc %d nli %ld curve rc %d\n", nm, np, rc, st.nli,
           rc2);
    or_destroy(c);
    free(xyz); free(tets); free(region); free(Ms); free(A); free(K1); free(ax);
    free(m); free(G); free(g); free(lam); free(y); free(q); free(b); free(u); free(dn); free(hist);
    return (rc == 0 && rc2 == 0) ? 0 : 5;
}
