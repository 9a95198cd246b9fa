/*
 * CPU FP64 oracle for the preconditioned projected nonlinear conjugate
 * gradient (PNCG) minimizer of the P1 finite-element micromagnetic energy
 * (Exl, Fischbacher, Kovacs, Oezelt, Gusenbauer, Schrefl, "Preconditioned
 * nonlinear conjugate gradient method for micromagnetic energy minimization").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the HIP library.
 *
 * Style: element loops written out from the definitions, FP64 everywhere,
 * Neumaier-compensated global sums, single-threaded, no reordering beyond what
 * the definitions state.
 *
 * What it computes (paper sections / equations in brackets):
 *   - the energy F(m) = 1/2 m^T C m - 1/2 h_d^T M m - h_ext^T M m with
 *     C = C_A + C_K (exchange + anisotropy)                        [Sec. 2.2, eq. (energy)]
 *   - the Lagrange multiplier lambda_i = m_i . grad F_i and the projected
 *     gradient Pi_{m-perp}(grad F)                       [eqs. (nablaLF), (proj), (optcond)]
 *   - the preconditioner action: eq. (precond) without its last term    [Sec. 2.2]
 *     (the paper's choice), and for comparison the other candidates the
 *     equation offers: all of it, or only its projected local part
 *   - preconditioned linear CG (Alg. 1) with the exits (li1)-(li3), Jacobi
 *     preconditioner = diagonal of the exchange matrix                  [Alg. 1, Sec. 3.1]
 *   - Alg. 4 with beta*ZA (restarted Hestenes-Stiefel), the descent
 *     safeguard, normalization after each update, and a line search
 *     that caps the rotation per step                                   [Alg. 4, Sec. 2.2]
 *   - field stepping for demagnetization curves, stopping rules
 *     (t1)-(t3) or a max-torque rule                                    [Sec. 3.1]
 *
 * Readings where the paper is silent (discretization details, line search,
 * index-garbled safeguard) are stated next to the code that implements them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MU0 (4.0e-7 * 3.14159265358979323846)

enum { T_EXCH = 1, T_ANIS = 2, T_ZEE = 4, T_DEMAG = 8 };

/* ------------------------------------------------------------------ */
/* compensated summation (Neumaier)                                    */
/* ------------------------------------------------------------------ */
typedef struct { double s, c; } ksum;
static void ks_add(ksum *k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double ks_val(const ksum *k) { return k->s + k->c; }

static double dot_n(const double *a, const double *b, long n) {
    ksum k = {0, 0};
    for (long i = 0; i < n; i++) ks_add(&k, a[i] * b[i]);
    return ks_val(&k);
}

/* ------------------------------------------------------------------ */
/* context                                                             */
/* ------------------------------------------------------------------ */
typedef struct {
    long nn, nt;
    double *xyz;
    int *tet;
    int *region;
    /* reduced per-tet material (reading S1: length unit 1 nm, magnetization
       unit Ms_ref = max Ms, energy unit mu0 Ms_ref^2 nm^3) */
    double Ms_ref;
    double *ms, *a, *k, *u; /* u: 3 per tet */
    /* geometry */
    double *vol;  /* V_e */
    double *grad; /* 12 per tet: grad phi_0..3 */
    /* magnet nodes */
    long nm;
    int *mag_of_node;   /* -1 if not magnet */
    int *node_of_mag;
    double *L;          /* Ms-weighted lumped nodal volume (matrix M) */
    double *Dex;        /* Jacobi diagonal: exchange matrix diagonal */
    /* potential unknowns (free nodes) */
    long np;
    int *free_of_node;  /* -1 on the outer boundary (Dirichlet u = 0) */
    long *Kp; int *Kj; double *Kv; double *Kd;
    double *u_pot;      /* warm start: the previous evaluation's potential */
    double poisson_rtol;
    long poisson_maxit;
    /* counters */
    long evals, mi, li;
} or_ctx;

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    return p;
}

/* 3x3 inverse by cofactors; returns the determinant */
static double inv3(const double J[3][3], double Ji[3][3]) {
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    return det;
}

/* faces for boundary detection */
typedef struct { int v[3]; } face3;
static int cmp_face(const void *pa, const void *pb) {
    const face3 *a = (const face3 *)pa, *b = (const face3 *)pb;
    for (int i = 0; i < 3; i++) {
        if (a->v[i] < b->v[i]) return -1;
        if (a->v[i] > b->v[i]) return 1;
    }
    return 0;
}
static void sort3(int *v) {
    int t;
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
    if (v[1] > v[2]) { t = v[1]; v[1] = v[2]; v[2] = t; }
    if (v[0] > v[1]) { t = v[0]; v[0] = v[1]; v[1] = t; }
}

typedef struct { long r; int c; double v; } trip;
static int cmp_trip(const void *pa, const void *pb) {
    const trip *a = (const trip *)pa, *b = (const trip *)pb;
    if (a->r != b->r) return a->r < b->r ? -1 : 1;
    if (a->c != b->c) return a->c < b->c ? -1 : 1;
    return 0;
}

void or_destroy(or_ctx *c) {
    if (!c) return;
    free(c->xyz); free(c->tet); free(c->region);
    free(c->ms); free(c->a); free(c->k); free(c->u);
    free(c->vol); free(c->grad);
    free(c->mag_of_node); free(c->node_of_mag); free(c->L); free(c->Dex);
    free(c->free_of_node); free(c->Kp); free(c->Kj); free(c->Kv); free(c->Kd);
    free(c->u_pot);
    free(c);
}

/*
 * Build the discretization. xyz in nm, tets 0-based (4 per tet), region 0 =
 * air, > 0 = magnetic material; SI material constants per tet.
 * Returns NULL on a degenerate tet or bad input.
 */
or_ctx *or_create(const double *xyz, long nn, const int *tets, long nt, const int *region,
                  const double *Ms, const double *A, const double *K1, const double *axis) {
    or_ctx *c = (or_ctx *)xcalloc(1, sizeof(or_ctx));
    c->nn = nn; c->nt = nt;
    c->xyz = (double *)xcalloc(3 * nn, sizeof(double));
    memcpy(c->xyz, xyz, sizeof(double) * 3 * nn);
    c->tet = (int *)xcalloc(4 * nt, sizeof(int));
    memcpy(c->tet, tets, sizeof(int) * 4 * nt);
    c->region = (int *)xcalloc(nt, sizeof(int));
    memcpy(c->region, region, sizeof(int) * nt);
    c->poisson_rtol = 1e-10;
    c->poisson_maxit = 100000;

    /* reduced units (reading S1) */
    double Ms_ref = 0.0;
    for (long e = 0; e < nt; e++)
        if (region[e] > 0 && Ms[e] > Ms_ref) Ms_ref = Ms[e];
    if (!(Ms_ref > 0.0)) { or_destroy(c); return NULL; }
    c->Ms_ref = Ms_ref;
    double Kd = OR_MU0 * Ms_ref * Ms_ref;   /* J/m^3 */
    c->ms = (double *)xcalloc(nt, sizeof(double));
    c->a = (double *)xcalloc(nt, sizeof(double));
    c->k = (double *)xcalloc(nt, sizeof(double));
    c->u = (double *)xcalloc(3 * nt, sizeof(double));
    for (long e = 0; e < nt; e++) {
        if (region[e] <= 0) continue;
        c->ms[e] = Ms[e] / Ms_ref;
        c->a[e] = A[e] / (Kd * 1e-18);      /* nm^2 */
        c->k[e] = K1[e] / Kd;
        if (axis) {
            double ax = axis[3 * e], ay = axis[3 * e + 1], az = axis[3 * e + 2];
            double n = sqrt(ax * ax + ay * ay + az * az);
            if (n > 0) { c->u[3 * e] = ax / n; c->u[3 * e + 1] = ay / n; c->u[3 * e + 2] = az / n; }
        }
    }

    /* geometry: V_e = |det J|/6, grad phi_1..3 = rows of J^-1, grad phi_0 = -sum */
    c->vol = (double *)xcalloc(nt, sizeof(double));
    c->grad = (double *)xcalloc(12 * nt, sizeof(double));
    for (long e = 0; e < nt; e++) {
        const int *t = tets + 4 * e;
        double J[3][3], Ji[3][3];
        for (int col = 0; col < 3; col++)
            for (int row = 0; row < 3; row++)
                J[row][col] = xyz[3 * t[col + 1] + row] - xyz[3 * t[0] + row];
        double det = inv3(J, Ji);
        if (!(fabs(det) > 0.0) || !isfinite(det)) { or_destroy(c); return NULL; }
        c->vol[e] = fabs(det) / 6.0;
        double *gr = c->grad + 12 * e;
        for (int i = 0; i < 3; i++) {
            gr[3 * (i + 1) + 0] = Ji[i][0];
            gr[3 * (i + 1) + 1] = Ji[i][1];
            gr[3 * (i + 1) + 2] = Ji[i][2];
        }
        for (int d = 0; d < 3; d++) gr[d] = -(gr[3 + d] + gr[6 + d] + gr[9 + d]);
    }

    /* magnet nodes: touched by a magnetic tet, ascending node order */
    c->mag_of_node = (int *)xcalloc(nn, sizeof(int));
    for (long i = 0; i < nn; i++) c->mag_of_node[i] = -1;
    for (long e = 0; e < nt; e++)
        if (region[e] > 0)
            for (int j = 0; j < 4; j++) c->mag_of_node[tets[4 * e + j]] = 1;
    long nm = 0;
    for (long i = 0; i < nn; i++)
        if (c->mag_of_node[i] == 1) c->mag_of_node[i] = (int)nm++;
    c->nm = nm;
    c->node_of_mag = (int *)xcalloc(nm, sizeof(int));
    for (long i = 0; i < nn; i++)
        if (c->mag_of_node[i] >= 0) c->node_of_mag[c->mag_of_node[i]] = (int)i;

    /* M = diag(L) (x) I3, L_a = sum_{e ni a, magnet} ms_e V_e / 4 (reading S4);
       Jacobi diagonal = exchange matrix diagonal 2 sum_e a_e V_e |grad phi_a|^2 */
    c->L = (double *)xcalloc(nm, sizeof(double));
    c->Dex = (double *)xcalloc(nm, sizeof(double));
    for (long e = 0; e < nt; e++) {
        if (region[e] <= 0) continue;
        const double *gr = c->grad + 12 * e;
        for (int j = 0; j < 4; j++) {
            int ia = c->mag_of_node[tets[4 * e + j]];
            c->L[ia] += c->ms[e] * c->vol[e] / 4.0;
            double g2 = gr[3 * j] * gr[3 * j] + gr[3 * j + 1] * gr[3 * j + 1] + gr[3 * j + 2] * gr[3 * j + 2];
            c->Dex[ia] += 2.0 * c->a[e] * c->vol[e] * g2;
        }
    }

    /* Dirichlet set: nodes on faces that belong to exactly one tet */
    face3 *F = (face3 *)xcalloc(4 * nt, sizeof(face3));
    static const int fl[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    for (long e = 0; e < nt; e++)
        for (int f = 0; f < 4; f++) {
            for (int j = 0; j < 3; j++) F[4 * e + f].v[j] = tets[4 * e + fl[f][j]];
            sort3(F[4 * e + f].v);
        }
    qsort(F, 4 * nt, sizeof(face3), cmp_face);
    char *onb = (char *)xcalloc(nn, 1);
    for (long i = 0; i < 4 * nt;) {
        long j = i + 1;
        while (j < 4 * nt && cmp_face(&F[i], &F[j]) == 0) j++;
        if (j - i == 1)
            for (int q = 0; q < 3; q++) onb[F[i].v[q]] = 1;
        i = j;
    }
    free(F);
    c->free_of_node = (int *)xcalloc(nn, sizeof(int));
    long np = 0;
    for (long i = 0; i < nn; i++) c->free_of_node[i] = onb[i] ? -1 : (int)np++;
    free(onb);
    c->np = np;

    /* Poisson matrix K_jk = sum_e V_e grad phi_j . grad phi_k over all tets,
       Dirichlet rows/columns removed (reading S5). Triplets, sort, sum. */
    long ntr = 0;
    trip *T = (trip *)xcalloc(16 * nt, sizeof(trip));
    for (long e = 0; e < nt; e++) {
        const double *gr = c->grad + 12 * e;
        for (int i = 0; i < 4; i++) {
            int fi = c->free_of_node[tets[4 * e + i]];
            if (fi < 0) continue;
            for (int j = 0; j < 4; j++) {
                int fj = c->free_of_node[tets[4 * e + j]];
                if (fj < 0) continue;
                double v = c->vol[e] * (gr[3 * i] * gr[3 * j] + gr[3 * i + 1] * gr[3 * j + 1] +
                                        gr[3 * i + 2] * gr[3 * j + 2]);
                T[ntr].r = fi; T[ntr].c = fj; T[ntr].v = v; ntr++;
            }
        }
    }
    qsort(T, ntr, sizeof(trip), cmp_trip);
    c->Kp = (long *)xcalloc(np + 1, sizeof(long));
    c->Kj = (int *)xcalloc(ntr, sizeof(int));
    c->Kv = (double *)xcalloc(ntr, sizeof(double));
    c->Kd = (double *)xcalloc(np, sizeof(double));
    long nz = 0;
    for (long i = 0; i < ntr;) {
        long j = i;
        ksum s = {0, 0};
        while (j < ntr && T[j].r == T[i].r && T[j].c == T[i].c) { ks_add(&s, T[j].v); j++; }
        c->Kj[nz] = T[i].c;
        c->Kv[nz] = ks_val(&s);
        c->Kp[T[i].r + 1] = nz + 1;
        if (T[i].r == T[i].c) c->Kd[T[i].r] = c->Kv[nz];
        nz++;
        i = j;
    }
    for (long r = 0; r < np; r++)
        if (c->Kp[r + 1] < c->Kp[r]) c->Kp[r + 1] = c->Kp[r];
    free(T);
    c->u_pot = (double *)xcalloc(np, sizeof(double));
    return c;
}

long or_n_mag(const or_ctx *c) { return c->nm; }
long or_n_pot(const or_ctx *c) { return c->np; }
double or_ms_ref(const or_ctx *c) { return c->Ms_ref; }
void or_mag_nodes(const or_ctx *c, int *ids) { memcpy(ids, c->node_of_mag, sizeof(int) * c->nm); }
void or_free_nodes(const or_ctx *c, int *free_of_node) { memcpy(free_of_node, c->free_of_node, sizeof(int) * c->nn); }
void or_lumped(const or_ctx *c, double *L) { memcpy(L, c->L, sizeof(double) * c->nm); }
void or_jacobi_diag(const or_ctx *c, double *D) { memcpy(D, c->Dex, sizeof(double) * c->nm); }
void or_set_poisson(or_ctx *c, double rtol, long maxit) { c->poisson_rtol = rtol; c->poisson_maxit = maxit; }
void or_reset_warm(or_ctx *c) { memset(c->u_pot, 0, sizeof(double) * c->np); }
void or_get_potential(const or_ctx *c, double *u) { memcpy(u, c->u_pot, sizeof(double) * c->np); }
void or_set_potential(or_ctx *c, const double *u) { memcpy(c->u_pot, u, sizeof(double) * c->np); }
void or_counters(const or_ctx *c, long *out3) { out3[0] = c->evals; out3[1] = c->mi; out3[2] = c->li; }
/* K in CSR (free-node numbering) for tests */
long or_K_nnz(const or_ctx *c) { return c->Kp[c->np]; }
void or_K_csr(const or_ctx *c, long *p, int *j, double *v) {
    memcpy(p, c->Kp, sizeof(long) * (c->np + 1));
    memcpy(j, c->Kj, sizeof(int) * c->Kp[c->np]);
    memcpy(v, c->Kv, sizeof(double) * c->Kp[c->np]);
}
/* reduced field from Tesla: h = B / (mu0 Ms_ref) */
void or_reduce_field(const or_ctx *c, const double *BT, double *h) {
    for (int d = 0; d < 3; d++) h[d] = BT[d] / (OR_MU0 * c->Ms_ref);
}

/* ------------------------------------------------------------------ */
/* local operator C v = (C_A + C_K) v by element loops                 */
/* exchange  E_ex = sum_e a_e V_e sum_ab (grad phi_a . grad phi_b)(m_a.m_b)
 * anisotropy E_an = -sum_e k_e sum_ab M^e_ab (u.m_a)(u.m_b),
 *            M^e_ab = V_e (1 + delta_ab) / 20 (consistent mass, reading S3) */
/* ------------------------------------------------------------------ */
static void apply_local(const or_ctx *c, const double *v, double *out, int terms) {
    memset(out, 0, sizeof(double) * 3 * c->nm);
    for (long e = 0; e < c->nt; e++) {
        if (c->region[e] <= 0) continue;
        const int *t = c->tet + 4 * e;
        const double *gr = c->grad + 12 * e;
        const double *u = c->u + 3 * e;
        int ia[4];
        for (int j = 0; j < 4; j++) ia[j] = c->mag_of_node[t[j]];
        for (int p = 0; p < 4; p++) {
            for (int q = 0; q < 4; q++) {
                const double *vq = v + 3 * ia[q];
                if (terms & T_EXCH) {
                    double s = c->a[e] * c->vol[e] *
                               (gr[3 * p] * gr[3 * q] + gr[3 * p + 1] * gr[3 * q + 1] + gr[3 * p + 2] * gr[3 * q + 2]);
                    for (int d = 0; d < 3; d++) out[3 * ia[p] + d] += 2.0 * s * vq[d];
                }
                if ((terms & T_ANIS) && c->k[e] != 0.0) {
                    double w = c->k[e] * c->vol[e] * (p == q ? 2.0 : 1.0) / 20.0;
                    double uv = u[0] * vq[0] + u[1] * vq[1] + u[2] * vq[2];
                    for (int d = 0; d < 3; d++) out[3 * ia[p] + d] -= 2.0 * w * uv * u[d];
                }
            }
        }
    }
}

void or_apply_C(const or_ctx *c, const double *v, double *out, int terms) { apply_local(c, v, out, terms); }

/* divergence right-hand side b_j = sum_{e ni j, magnet} ms_e V_e mbar_e . grad phi_j (free j) */
void or_bmul(const or_ctx *c, const double *m, double *b) {
    memset(b, 0, sizeof(double) * c->np);
    for (long e = 0; e < c->nt; e++) {
        if (c->region[e] <= 0) continue;
        const int *t = c->tet + 4 * e;
        const double *gr = c->grad + 12 * e;
        double mb[3] = {0, 0, 0};
        for (int j = 0; j < 4; j++) {
            const double *mj = m + 3 * c->mag_of_node[t[j]];
            for (int d = 0; d < 3; d++) mb[d] += 0.25 * mj[d];
        }
        for (int j = 0; j < 4; j++) {
            int fj = c->free_of_node[t[j]];
            if (fj < 0) continue;
            b[fj] += c->ms[e] * c->vol[e] * (mb[0] * gr[3 * j] + mb[1] * gr[3 * j + 1] + mb[2] * gr[3 * j + 2]);
        }
    }
}

/* demag gradient dE_d/dm_a = sum_{e ni a, magnet} ms_e (V_e/4) grad u_e */
void or_btmul(const or_ctx *c, const double *u, double *Gd) {
    memset(Gd, 0, sizeof(double) * 3 * c->nm);
    for (long e = 0; e < c->nt; e++) {
        if (c->region[e] <= 0) continue;
        const int *t = c->tet + 4 * e;
        const double *gr = c->grad + 12 * e;
        double gu[3] = {0, 0, 0};
        for (int j = 0; j < 4; j++) {
            int fj = c->free_of_node[t[j]];
            double uj = fj >= 0 ? u[fj] : 0.0;
            for (int d = 0; d < 3; d++) gu[d] += uj * gr[3 * j + d];
        }
        double w = c->ms[e] * c->vol[e] / 4.0;
        for (int j = 0; j < 4; j++) {
            int ia = c->mag_of_node[t[j]];
            for (int d = 0; d < 3; d++) Gd[3 * ia + d] += w * gu[d];
        }
    }
}

static void kmul(const or_ctx *c, const double *x, double *y) {
    for (long r = 0; r < c->np; r++) {
        double s = 0.0;
        for (long q = c->Kp[r]; q < c->Kp[r + 1]; q++) s += c->Kv[q] * x[c->Kj[q]];
        y[r] = s;
    }
}
void or_kmul(const or_ctx *c, const double *x, double *y) { kmul(c, x, y); }

/*
 * Jacobi-preconditioned CG for K u = b (the scalar-potential problem; the
 * paper uses CG with an AMG preconditioner, this oracle uses the diagonal,
 * reading S5). Warm start from u on entry; stops when ||r||_2 <= rtol ||b||_2.
 * Returns the iteration count (-1 if maxit was reached).
 */
long or_poisson(const or_ctx *c, const double *b, double *u, double rtol, long maxit) {
    long n = c->np;
    double bn = sqrt(dot_n(b, b, n));
    if (bn == 0.0) { memset(u, 0, sizeof(double) * n); return 0; }
    double *r = (double *)xcalloc(n, sizeof(double));
    double *z = (double *)xcalloc(n, sizeof(double));
    double *p = (double *)xcalloc(n, sizeof(double));
    double *q = (double *)xcalloc(n, sizeof(double));
    kmul(c, u, q);
    for (long i = 0; i < n; i++) r[i] = b[i] - q[i];
    for (long i = 0; i < n; i++) { z[i] = r[i] / c->Kd[i]; p[i] = z[i]; }
    double rz = dot_n(r, z, n);
    double rn = sqrt(dot_n(r, r, n));
    long it = 0;
    while (rn > rtol * bn) {
        if (it >= maxit) { it = -1; break; }
        kmul(c, p, q);
        double alpha = rz / dot_n(p, q, n);
        for (long i = 0; i < n; i++) { u[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        it++;
        rn = sqrt(dot_n(r, r, n));
        if (rn <= rtol * bn) break;
        for (long i = 0; i < n; i++) z[i] = r[i] / c->Kd[i];
        double rz1 = dot_n(r, z, n);
        double beta = rz1 / rz;
        rz = rz1;
        for (long i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
    }
    free(r); free(z); free(p); free(q);
    return it;
}

/*
 * Energy and gradient [eq. (energy)], multiplier and projected gradient
 * [eqs. (nablaLF), (proj)], torque |m x h_eff| = |g_a| / L_a.
 * E[0..4] = exchange, anisotropy, Zeeman, demag, total. h is the reduced field.
 * The potential solve is warm-started from the previous evaluation's u.
 * Any output pointer may be NULL. Returns Poisson iterations (-1 on failure).
 */
long or_eval(or_ctx *c, const double *m, const double *h, int terms, double *E, double *G,
             double *g, double *lam, double *tmax) {
    long nm = c->nm;
    double *Gl = (double *)xcalloc(3 * nm, sizeof(double));
    double *Ge = (double *)xcalloc(3 * nm, sizeof(double));
    double *Ga = (double *)xcalloc(3 * nm, sizeof(double));
    double *Gd = (double *)xcalloc(3 * nm, sizeof(double));
    apply_local(c, m, Ge, terms & T_EXCH);
    apply_local(c, m, Ga, terms & T_ANIS);
    ksum eex = {0, 0}, ean = {0, 0}, ez = {0, 0}, ed = {0, 0};
    for (long i = 0; i < 3 * nm; i++) { ks_add(&eex, 0.5 * m[i] * Ge[i]); ks_add(&ean, 0.5 * m[i] * Ga[i]); }
    long it = 0;
    if (terms & T_DEMAG) {
        double *b = (double *)xcalloc(c->np, sizeof(double));
        or_bmul(c, m, b);
        it = or_poisson(c, b, c->u_pot, c->poisson_rtol, c->poisson_maxit);
        or_btmul(c, c->u_pot, Gd);
        for (long i = 0; i < c->np; i++) ks_add(&ed, 0.5 * b[i] * c->u_pot[i]);
        free(b);
        if (it > 0) c->mi += it;
    }
    double tm = 0.0;
    for (long a = 0; a < nm; a++) {
        double Gt[3];
        for (int d = 0; d < 3; d++) {
            double gz = (terms & T_ZEE) ? -c->L[a] * h[d] : 0.0;
            Gt[d] = Ge[3 * a + d] + Ga[3 * a + d] + Gd[3 * a + d] + gz;
            if (terms & T_ZEE) ks_add(&ez, -c->L[a] * h[d] * m[3 * a + d]);
        }
        const double *ma = m + 3 * a;
        double l = ma[0] * Gt[0] + ma[1] * Gt[1] + ma[2] * Gt[2];
        double gp[3] = {Gt[0] - l * ma[0], Gt[1] - l * ma[1], Gt[2] - l * ma[2]};
        double t = sqrt(gp[0] * gp[0] + gp[1] * gp[1] + gp[2] * gp[2]) / c->L[a];
        if (t > tm || t != t) tm = t;   /* a NaN torque stays NaN */
        if (G) for (int d = 0; d < 3; d++) G[3 * a + d] = Gt[d];
        if (g) for (int d = 0; d < 3; d++) g[3 * a + d] = gp[d];
        if (lam) lam[a] = l;
    }
    if (E) {
        E[0] = ks_val(&eex); E[1] = ks_val(&ean); E[2] = ks_val(&ez); E[3] = ks_val(&ed);
        ksum tot = {0, 0};
        for (int q = 0; q < 4; q++) ks_add(&tot, E[q]);
        E[4] = ks_val(&tot);
    }
    if (tmax) *tmax = tm;
    c->evals++;
    free(Gl); free(Ge); free(Ga); free(Gd);
    return it;
}

/*
 * Preconditioner action, eq. (precond) with C = exchange + anisotropy only
 * and lambda_a = m_a . grad F_a from the full gradient:
 *   form 0 (the paper's choice, without the last term):
 *     (P v)_a = (C v)_a - (m_a . (C v)_a) m_a - lambda_a v_a
 *   form 1 (all four terms): form 0 - (v_a . grad F_a) m_a, where
 *     grad F_a = g_a + lambda_a m_a (g the projected gradient)
 *   form 2 (the projected local part only): (C v)_a - (m_a . (C v)_a) m_a
 */
void or_apply_P(const or_ctx *c, const double *m, const double *lam, const double *g, const double *v,
                double *out, int terms, int form) {
    apply_local(c, v, out, terms & (T_EXCH | T_ANIS));
    for (long a = 0; a < c->nm; a++) {
        const double *ma = m + 3 * a, *va = v + 3 * a;
        double *o = out + 3 * a;
        double mc = ma[0] * o[0] + ma[1] * o[1] + ma[2] * o[2];
        double shift = form == 2 ? 0.0 : lam[a];
        double vG = 0.0;
        if (form == 1) {
            const double *ga = g + 3 * a;
            for (int d = 0; d < 3; d++) vG += va[d] * (ga[d] + lam[a] * ma[d]);
        }
        for (int d = 0; d < 3; d++) o[d] = o[d] - mc * ma[d] - shift * va[d] - vG * ma[d];
    }
}

/*
 * Solve P y = g approximately with Alg. 1 (standard-sign form: residual
 * r = g - P y), y_0 = 0, Jacobi preconditioner D = exchange diagonal (scaled
 * by dscale when given), exits:
 *   (li1) at most jmax iterations (reading S8: jmax = 0 gives y = g)
 *   (li2) non-positive curvature p.Pp <= 0: y = g if no step was taken yet,
 *         else the current y (reading S9)
 *   (li3) ||r|| < min(0.5, sqrt(||g||)) ||g|| (reading S10: b = g)
 * Returns the number of inner iterations taken.
 */
long or_precond(or_ctx *c, const double *m, const double *lam, const double *g, int jmax,
                const double *dscale, double *y, int terms, int form) {
    long n3 = 3 * c->nm;
    memset(y, 0, sizeof(double) * n3);
    if (jmax <= 0) { memcpy(y, g, sizeof(double) * n3); return 0; }
    double *r = (double *)xcalloc(n3, sizeof(double));
    double *z = (double *)xcalloc(n3, sizeof(double));
    double *p = (double *)xcalloc(n3, sizeof(double));
    double *q = (double *)xcalloc(n3, sizeof(double));
    double gn = sqrt(dot_n(g, g, n3));
    double eta = sqrt(gn) < 0.5 ? sqrt(gn) : 0.5;
    memcpy(r, g, sizeof(double) * n3);
    for (long a = 0; a < c->nm; a++) {
        double D = c->Dex[a] * (dscale ? dscale[a] : 1.0);
        for (int d = 0; d < 3; d++) { z[3 * a + d] = r[3 * a + d] / D; p[3 * a + d] = z[3 * a + d]; }
    }
    double rz = dot_n(r, z, n3);
    long it = 0;
    for (int j = 0; j < jmax; j++) {
        or_apply_P(c, m, lam, g, p, q, terms, form);
        double pq = dot_n(p, q, n3);
        if (!(pq > 0.0)) {
            if (j == 0) memcpy(y, g, sizeof(double) * n3);
            break;
        }
        double alpha = rz / pq;
        for (long i = 0; i < n3; i++) { y[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        it++;
        double rn = sqrt(dot_n(r, r, n3));
        if (rn < eta * gn) break;
        for (long a = 0; a < c->nm; a++) {
            double D = c->Dex[a] * (dscale ? dscale[a] : 1.0);
            for (int d = 0; d < 3; d++) z[3 * a + d] = r[3 * a + d] / D;
        }
        double rz1 = dot_n(r, z, n3);
        double beta = rz1 / rz;
        rz = rz1;
        for (long i = 0; i < n3; i++) p[i] = z[i] + beta * p[i];
    }
    c->li += it;
    free(r); free(z); free(p); free(q);
    return it;
}
long or_precond_pub(or_ctx *c, const double *m, const double *lam, const double *g, int jmax,
                    const double *dscale, double *y, int terms, int form) {
    return or_precond(c, m, lam, g, jmax, dscale, y, terms, form);
}

/* ------------------------------------------------------------------ */
/* Alg. 4 with the line search (reading S6)                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int jmax;
    double tol_torque;
    int stop_mode;      /* 0: max torque < tol; 1: (t1)-(t3) with tau_F */
    double tau_F;
    double theta_max, theta_init, c1, c2;
    long max_nli;
    int terms;
    int ls_max_halvings;
    int beta;           /* 0: beta*ZA (Alg. 4), 1: beta*FR, 2: beta*PRP, 3: beta*HS (Sec. 2.1) */
    int pform;          /* preconditioner form of or_apply_P (0: the paper's) */
    int theta_adapt;    /* 1: the rotation cap follows the accepted steps (reading S6's cap) */
    double theta_hi;    /* its upper bound (rad) */
} or_opts;

typedef struct {
    long evals, nli, li, mi, restarts, fallbacks, ls_fail;
    double F;
    double tmax;
    long status;        /* 0 ok, 1 not converged, 2 stalled, 3 non-finite energy or gradient */
    double max_trap_err; /* max |(F+ - F) - dF_trapezoid| over accepted steps */
    long n_rise;        /* accepted steps whose energy total F+ exceeds F */
    double max_rise;    /* largest F+ - F over accepted steps (<= 0 when every step decreased F) */
} or_stats;

typedef struct {
    double *x, *G, *g, *lam;
    double E[5];
    double tmax;
} or_state;

static void st_alloc(or_state *s, long nm) {
    s->x = (double *)xcalloc(3 * nm, sizeof(double));
    s->G = (double *)xcalloc(3 * nm, sizeof(double));
    s->g = (double *)xcalloc(3 * nm, sizeof(double));
    s->lam = (double *)xcalloc(nm, sizeof(double));
}
static void st_free(or_state *s) { free(s->x); free(s->G); free(s->g); free(s->lam); }
static void st_copy(or_state *dst, const or_state *src, long nm) {
    memcpy(dst->x, src->x, sizeof(double) * 3 * nm);
    memcpy(dst->G, src->G, sizeof(double) * 3 * nm);
    memcpy(dst->g, src->g, sizeof(double) * 3 * nm);
    memcpy(dst->lam, src->lam, sizeof(double) * nm);
    memcpy(dst->E, src->E, sizeof(dst->E));
    dst->tmax = src->tmax;
}

/* evaluate at x(alpha) = N(x + alpha d); returns dF (trapezoid) and phi'(alpha) */
static void ls_eval(or_ctx *c, const or_state *s0, const double *d, double alpha, const double *h,
                    int terms, or_state *st, double *dF, double *dphi, or_stats *stats) {
    long nm = c->nm;
    for (long a = 0; a < nm; a++) {
        double w[3];
        for (int k = 0; k < 3; k++) w[k] = s0->x[3 * a + k] + alpha * d[3 * a + k];
        double n = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        for (int k = 0; k < 3; k++) st->x[3 * a + k] = w[k] / n;
    }
    or_eval(c, st->x, h, terms, st->E, st->G, st->g, st->lam, &st->tmax);
    stats->evals++;
    /* Exact energy difference of the quadratic F between unit vectors (reading
       S26 written in tangential form): with G = g + lambda x and |x| = |x+| = 1,
       F(x+) - F(x) = 1/2 sum_a [ dx.(g + g+) + 1/2 (lambda+ - lambda) |dx|^2 ],
       dx = x+ - x. It equals 1/2 dx.(G + G+) in exact arithmetic, and it keeps
       the large radial part of G (|lambda| >> |g| near a minimum) out of the sum. */
    ksum t = {0, 0}, p = {0, 0};
    for (long a = 0; a < nm; a++) {
        double w[3], dx[3];
        for (int k = 0; k < 3; k++) w[k] = s0->x[3 * a + k] + alpha * d[3 * a + k];
        double n = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        double dx2 = 0.0, dg = 0.0;
        for (int k = 0; k < 3; k++) {
            dx[k] = st->x[3 * a + k] - s0->x[3 * a + k];
            dx2 += dx[k] * dx[k];
            dg += dx[k] * (st->g[3 * a + k] + s0->g[3 * a + k]);
            ks_add(&p, st->g[3 * a + k] * d[3 * a + k] / n);
        }
        ks_add(&t, 0.5 * (dg + 0.5 * (st->lam[a] - s0->lam[a]) * dx2));
    }
    *dF = ks_val(&t);
    *dphi = ks_val(&p);
}

/* cubic Hermite minimizer through (0, 0, dp0) and (at, dFt, dpt)
   (Nocedal & Wright, interpolation step of the line search); returns 0 if none */
int or_cubic_min_pub(double at, double dFt, double dp0, double dpt, double *ac);
static int cubic_min(double at, double dFt, double dp0, double dpt, double *ac) {
    double d1 = dp0 + dpt - 3.0 * dFt / at;
    double disc = d1 * d1 - dp0 * dpt;
    if (!(disc >= 0.0) || !isfinite(disc)) return 0;
    double d2 = sqrt(disc);
    double den = dpt - dp0 + 2.0 * d2;
    if (!(den != 0.0) || !isfinite(den)) return 0;
    double a = at - at * (dpt + d2 - d1) / den;
    if (!isfinite(a)) return 0;
    *ac = a;
    return 1;
}

/*
 * Line search on phi(alpha) = F(N(x + alpha d)) (reading S6, "LS-2P").
 * alpha_max caps the largest nodal rotation at theta (theta_max, or the
 * adapted cap). On success st1 holds the accepted state and the function
 * returns 1; *alpha the step and *amax_out the alpha_max it used.
 */
static int line_search(or_ctx *c, const or_opts *o, double theta, const double *h, const or_state *s0,
                       const double *d, double dp0, double a0, or_state *st1, or_state *tmp,
                       double *alpha, double *dF_acc, or_stats *stats, double *amax_out) {
    long nm = c->nm;
    double dmax = 0.0;
    for (long a = 0; a < nm; a++) {
        double n = sqrt(d[3 * a] * d[3 * a] + d[3 * a + 1] * d[3 * a + 1] + d[3 * a + 2] * d[3 * a + 2]);
        if (n > dmax) dmax = n;
    }
    if (!(dmax > 0.0)) return 0;
    double amax = theta / dmax;
    *amax_out = amax;
    double at = a0 < amax ? a0 : amax;
    double dFt, dpt;
    ls_eval(c, s0, d, at, h, o->terms, st1, &dFt, &dpt, stats);
    int arm_t = dFt <= o->c1 * at * dp0;
    if (arm_t && fabs(dpt) <= o->c2 * fabs(dp0)) { *alpha = at; *dF_acc = dFt; return 1; }
    int over = !arm_t || dpt > 0.0;
    if (!over && at >= amax) { *alpha = at; *dF_acc = dFt; return 1; }
    double ac;
    if (!cubic_min(at, dFt, dp0, dpt, &ac)) ac = over ? 0.5 * at : (2.0 * at < amax ? 2.0 * at : amax);
    if (over) {
        if (ac < 0.1 * at) ac = 0.1 * at;
        if (ac > 0.9 * at) ac = 0.9 * at;
    } else {
        double hi = 4.0 * at < amax ? 4.0 * at : amax;
        if (ac > hi) ac = hi;
        if (ac < 1.1 * at) ac = 1.1 * at;
        if (ac > hi) { *alpha = at; *dF_acc = dFt; return 1; }
    }
    double dFc, dpc;
    ls_eval(c, s0, d, ac, h, o->terms, tmp, &dFc, &dpc, stats);
    if (dFc <= o->c1 * ac * dp0) { st_copy(st1, tmp, nm); *alpha = ac; *dF_acc = dFc; return 1; }
    if (arm_t) { *alpha = at; *dF_acc = dFt; return 1; }
    double a = at < ac ? at : ac;
    for (int k = 0; k < o->ls_max_halvings; k++) {
        a *= 0.5;
        double dFa, dpa;
        ls_eval(c, s0, d, a, h, o->terms, st1, &dFa, &dpa, stats);
        if (dFa <= o->c1 * a * dp0) { *alpha = a; *dF_acc = dFa; return 1; }
    }
    return 0;
}

/*
 * The adapted rotation cap (reading S6): a step the cap stopped doubles it,
 * up to theta_hi; a step shorter than a quarter of the cap halves it, down
 * to theta_max; any other step leaves it. Each field starts at theta_max.
 */
static double adapt_cap(const or_opts *o, double theta, double alpha, double amax) {
    if (alpha >= amax * (1.0 - 1e-12)) return 2.0 * theta < o->theta_hi ? 2.0 * theta : o->theta_hi;
    if (alpha < 0.25 * amax) return 0.5 * theta > o->theta_max ? 0.5 * theta : o->theta_max;
    return theta;
}

int or_cubic_min_pub(double at, double dFt, double dp0, double dpt, double *ac) {
    return cubic_min(at, dFt, dp0, dpt, ac);
}

static double max_norm3(const double *v, long nm) {
    double mx = 0;
    for (long a = 0; a < nm; a++) {
        double n = sqrt(v[3 * a] * v[3 * a] + v[3 * a + 1] * v[3 * a + 1] + v[3 * a + 2] * v[3 * a + 2]);
        if (n > mx) mx = n;
    }
    return mx;
}
static double inf_norm(const double *v, long n) {
    double mx = 0;
    for (long i = 0; i < n; i++) if (fabs(v[i]) > mx) mx = fabs(v[i]);
    return mx;
}

/*
 * beta* of the preconditioned NCG (Sec. 2.1, eqs. FR*, PRP*, HS*, and Alg. 4's
 * ZA, the HS form restarted when y_{j+1}.g_{j+1} <= y_{j+1}.g_j), from
 * num = <g_{j+1} - g_j, y_{j+1}>, den = <g_{j+1} - g_j, d_j>,
 * gy1 = <g_{j+1}, y_{j+1}> and gy0 = <g_j, y_j> of the previous direction.
 * A non-positive denominator gives 0 (reading S12).
 */
static double beta_star(int kind, double num, double den, double gy1, double gy0) {
    switch (kind) {
        case 1: return gy0 > 0.0 ? gy1 / gy0 : 0.0;
        case 2: return gy0 > 0.0 ? num / gy0 : 0.0;
        case 3: return den > 0.0 ? num / den : 0.0;
        default: return (num > 0.0 && den > 0.0) ? num / den : 0.0;
    }
}

/*
 * The next direction of Alg. 4 from the gradients g1 (new iterate) and g0
 * (previous), the preconditioned gradient y at g1 and the previous direction
 * d: dn = -y + beta* d. With the descent safeguard (reading S7): if dn is
 * not a descent direction, y is replaced by g1 and beta* recomputed, and if
 * that fails too, dn = -g1. gy_prev is <g, y> of the previous step. Returns
 * the <g, y> the next step divides by; *dpn = <g1, dn>; *fallback = 1 when
 * the safeguard acted.
 */
static double direction(int kind, long n3, const double *g1, const double *g0, const double *y,
                        const double *d, double gy_prev, double *dn, double *dpn, int *fallback) {
    ksum kn = {0, 0}, kd = {0, 0}, ky = {0, 0};
    for (long i = 0; i < n3; i++) {
        double dg = g1[i] - g0[i];
        ks_add(&kn, dg * y[i]);
        ks_add(&kd, dg * d[i]);
        ks_add(&ky, g1[i] * y[i]);
    }
    double num = ks_val(&kn), den = ks_val(&kd), gy1 = ks_val(&ky);
    double beta = beta_star(kind, num, den, gy1, gy_prev);
    for (long i = 0; i < n3; i++) dn[i] = -y[i] + beta * d[i];
    double dp = dot_n(g1, dn, n3);
    double gy_next = gy1;
    *fallback = 0;
    if (!(dp < 0.0)) {
        *fallback = 1;
        ksum k2 = {0, 0}, kg = {0, 0};
        for (long i = 0; i < n3; i++) {
            ks_add(&k2, (g1[i] - g0[i]) * g1[i]);
            ks_add(&kg, g1[i] * g1[i]);
        }
        double num2 = ks_val(&k2);
        gy_next = ks_val(&kg);
        beta = beta_star(kind, num2, den, gy_next, gy_prev);
        for (long i = 0; i < n3; i++) dn[i] = -g1[i] + beta * d[i];
        dp = dot_n(g1, dn, n3);
        if (!(dp < 0.0)) {
            for (long i = 0; i < n3; i++) dn[i] = -g1[i];
            dp = dot_n(g1, dn, n3);
        }
    }
    *dpn = dp;
    return gy_next;
}

/* the same, for tests */
double or_direction_pub(int kind, long n3, const double *g1, const double *g0, const double *y, const double *d,
                        double gy_prev, double *dn, int *fallback) {
    double dp;
    return direction(kind, n3, g1, g0, y, d, gy_prev, dn, &dp, fallback);
}

/*
 * Alg. 4 for one reduced field h, starting from m (unit vectors), m updated in place.
 * Direction update: beta*ZA = <g+ - g, y+> / <g+ - g, d> if y+.g+ > y+.g else 0
 * (zero also when the denominator is not positive, reading S12), or the
 * beta* variant o->beta selects (beta_star); <g, y> of the direction taken is
 * kept for the FR* and PRP* denominators (<g, g> when g stood in for y).
 * Descent safeguard (reading S7): if <g+, d+> >= 0 use y+ = g+ and recompute;
 * if still not descent, d+ = -g+.
 */
int or_minimize(or_ctx *c, double *m, const double *h, const or_opts *o, or_stats *stats, double *E_out) {
    long nm = c->nm, n3 = 3 * nm;
    or_state s0, s1, tmp;
    st_alloc(&s0, nm); st_alloc(&s1, nm); st_alloc(&tmp, nm);
    double *y = (double *)xcalloc(n3, sizeof(double));
    double *d = (double *)xcalloc(n3, sizeof(double));
    double *dn = (double *)xcalloc(n3, sizeof(double));
    memcpy(s0.x, m, sizeof(double) * n3);
    long mi0 = c->mi, li0 = c->li;
    memset(stats, 0, sizeof(*stats));
    or_eval(c, s0.x, h, o->terms, s0.E, s0.G, s0.g, s0.lam, &s0.tmax);
    stats->evals++;
    stats->max_rise = -INFINITY;
    int status = 1;
    /* a NaN or infinite energy or torque is reported, never taken for convergence */
    if (!isfinite(s0.E[4]) || !isfinite(s0.tmax)) { status = 3; goto done; }
    if (o->stop_mode == 0 && s0.tmax < o->tol_torque) { status = 0; goto done; }
    or_precond(c, s0.x, s0.lam, s0.g, o->jmax, NULL, y, o->terms, o->pform);
    for (long i = 0; i < n3; i++) d[i] = -y[i];
    double dp0 = dot_n(s0.g, d, n3);
    double gy_prev = -dp0;  /* <g, y> of the direction taken */
    if (!(dp0 < 0.0)) {
        for (long i = 0; i < n3; i++) d[i] = -s0.g[i];
        dp0 = dot_n(s0.g, d, n3);
        gy_prev = -dp0;
        stats->fallbacks++;
    }
    int first = 1;
    double a_prev = 0.0, dp_prev = 0.0;
    double theta = o->theta_max, amax_used = 0.0;
    for (long it = 0; it < o->max_nli; it++) {
        /* after the safeguard d = -g gives dp0 = -|g|^2: zero only at a zero
           projected gradient; anything else that is not negative is NaN */
        if (!(dp0 < 0.0)) { status = dp0 == 0.0 ? 0 : 3; break; }
        double dmax = max_norm3(d, nm);
        double a0;
        if (first) a0 = o->jmax > 0 ? 1.0 : o->theta_init / dmax;
        else a0 = a_prev * dp_prev / dp0;
        double alpha, dFacc;
        int ok = line_search(c, o, theta, h, &s0, d, dp0, a0, &s1, &tmp, &alpha, &dFacc, stats, &amax_used);
        if (!ok) {
            /* restart along the steepest descent direction */
            stats->restarts++;
            for (long i = 0; i < n3; i++) d[i] = -s0.g[i];
            dp0 = dot_n(s0.g, d, n3);
            gy_prev = -dp0;
            dmax = max_norm3(d, nm);
            if (!(dp0 < 0.0) || !(dmax > 0.0)) { status = 2; break; }
            ok = line_search(c, o, theta, h, &s0, d, dp0, o->theta_init / dmax, &s1, &tmp, &alpha, &dFacc, stats,
                             &amax_used);
            if (!ok) { stats->ls_fail++; status = 2; break; }
        }
        if (o->theta_adapt) theta = adapt_cap(o, theta, alpha, amax_used);
        if (!isfinite(s1.E[4]) || !isfinite(s1.tmax)) { status = 3; break; }
        double rise = s1.E[4] - s0.E[4];
        double terr = fabs(rise - dFacc);
        if (terr > stats->max_trap_err) stats->max_trap_err = terr;
        if (rise > 0.0) stats->n_rise++;
        if (rise > stats->max_rise) stats->max_rise = rise;
        stats->nli++;
        /* convergence */
        int conv;
        if (o->stop_mode == 0) {
            conv = s1.tmax < o->tol_torque;
        } else {
            double tau = o->tau_F;
            double dx = 0.0;
            for (long i = 0; i < n3; i++) if (fabs(s0.x[i] - s1.x[i]) > dx) dx = fabs(s0.x[i] - s1.x[i]);
            int t1 = (s0.E[4] - s1.E[4]) < tau * (1.0 + fabs(s1.E[4]));
            int t2 = dx < sqrt(tau) * (1.0 + inf_norm(s1.x, n3));
            int t3 = inf_norm(s1.g, n3) < cbrt(tau) * (1.0 + fabs(s1.E[4]));
            conv = t1 && t2 && t3;
        }
        if (conv) { st_copy(&s0, &s1, nm); status = 0; break; }
        /* precondition at the new iterate */
        or_precond(c, s1.x, s1.lam, s1.g, o->jmax, NULL, y, o->terms, o->pform);
        int fallback;
        double dpn;
        double gy_next = direction(o->beta, n3, s1.g, s0.g, y, d, gy_prev, dn, &dpn, &fallback);
        if (fallback) stats->fallbacks++;
        gy_prev = gy_next;
        a_prev = alpha;
        dp_prev = dp0;
        first = 0;
        st_copy(&s0, &s1, nm);
        memcpy(d, dn, sizeof(double) * n3);
        dp0 = dpn;
    }
done:
    memcpy(m, s0.x, sizeof(double) * n3);
    if (E_out) memcpy(E_out, s0.E, sizeof(double) * 5);
    stats->F = s0.E[4];
    stats->tmax = s0.tmax;
    stats->status = status;
    stats->mi = c->mi - mi0;
    stats->li = c->li - li0;
    st_free(&s0); st_free(&s1); st_free(&tmp);
    free(y); free(d); free(dn);
    return status;
}

/*
 * Demagnetization curve: for each field (Tesla) in order, minimize starting
 * from the previous minimizer [Sec. 3.1]. Records the volume-weighted mean
 * magnetization sum L_a m_a / sum L_a, the total energy and per-step stats.
 */
int or_curve(or_ctx *c, double *m, const double *fields_T, long nf, const or_opts *o,
             double *m_avg, double *E_tot, or_stats *st, double *m_hist) {
    long nm = c->nm;
    int worst = 0;
    double Lsum = 0.0;
    for (long a = 0; a < nm; a++) Lsum += c->L[a];
    for (long k = 0; k < nf; k++) {
        double h[3];
        or_reduce_field(c, fields_T + 3 * k, h);
        or_stats s;
        double E[5];
        int rc = or_minimize(c, m, h, o, &s, E);
        if (rc > worst) worst = rc;
        ksum av[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (long a = 0; a < nm; a++)
            for (int q = 0; q < 3; q++) ks_add(&av[q], c->L[a] * m[3 * a + q]);
        if (m_avg) for (int q = 0; q < 3; q++) m_avg[3 * k + q] = ks_val(&av[q]) / Lsum;
        if (E_tot) E_tot[k] = E[4];
        if (st) st[k] = s;
        if (m_hist) memcpy(m_hist + 3 * nm * k, m, sizeof(double) * 3 * nm);
    }
    return worst;
}

/* struct sizes so the Python side can check its ctypes layouts */
long or_sizeof_opts(void) { return (long)sizeof(or_opts); }
long or_sizeof_stats(void) { return (long)sizeof(or_stats); }
