/* pbref.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE, see pbref.h).
 *
 * Written for readability against the paper, not for speed: matrix-free FEM
 * element loops, row-by-row Galerkin BEM, textbook restarted GMRES with
 * modified Gram-Schmidt, and the Newton / relaxation-factor iteration in the
 * order the paper states it.  Only OpenMP over independent rows is used.
 *
 * Units (the paper gives none): potentials are u = e phi / (k_B T); a charge
 * z_k (in e) enters as Q_k = 4 pi l_B z_k with the vacuum Bjerrum length l_B in
 * Angstrom, so -div(eps grad u) = sum Q_k delta_k and the Coulomb potential in
 * the solute is sum l_B z_k / (eps_m |x - x_k|).  Energies are in kcal/mol.
 */
#include "pbref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* physical constants, SI 2019 exact values + CODATA 2018 vacuum permittivity */
/* ------------------------------------------------------------------------- */
static const double E_CHARGE = 1.602176634e-19;
static const double EPS0 = 8.8541878128e-12;
static const double K_BOLTZ = 1.380649e-23;
static const double N_AVO = 6.02214076e23;
static const double CAL = 4.184;

/* ------------------------------------------------------------------------- */
/* quadrature                                                                  */
/* ------------------------------------------------------------------------- */

/* Gauss-Legendre on [0,1]: roots of P_n by Newton on the three-term recurrence. */
int pbref_rule_gauss01(int n, double *x, double *w)
{
    if (n < 1) return -1;
    for (int i = 0; i < n; ++i) {
        double t = cos(PI * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = t; p0 = 1.0; }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        /* recompute derivative at the converged root */
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = t; p0 = 1.0; }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        x[n - 1 - i] = 0.5 * (t + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - t * t) * dp * dp); /* 2/((1-t^2)P'^2) scaled by 1/2 */
    }
    return 0;
}

/* Gauss rule on [0,1] for the weight (1-x)^alpha with 3 nodes (alpha integer
 * >= 0).  Nodes: roots of the cubic orthogonal polynomial, found from the
 * moments mu_k = int_0^1 x^k (1-x)^alpha dx = k! alpha! / (k+alpha+1)! by
 * solving the Hankel system for its monic coefficients and then Newton on the
 * cubic; weights from the 3x3 Vandermonde moment system. */
static double beta_moment(int k, int alpha)
{
    double v = 1.0; /* k! alpha! / (k+alpha+1)! */
    for (int i = 1; i <= k; ++i) v *= i;
    for (int i = 1; i <= alpha; ++i) v *= i;
    for (int i = 1; i <= k + alpha + 1; ++i) v /= i;
    return v;
}

static void solve3(double M[3][3], double r[3], double out[3])
{
    /* Gaussian elimination with partial pivoting on a 3x3 system */
    double A[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) A[i][j] = M[i][j];
        A[i][3] = r[i];
    }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int i = c + 1; i < 3; ++i)
            if (fabs(A[i][c]) > fabs(A[p][c])) p = i;
        for (int j = 0; j < 4; ++j) {
            double t = A[c][j];
            A[c][j] = A[p][j];
            A[p][j] = t;
        }
        for (int i = c + 1; i < 3; ++i) {
            double f = A[i][c] / A[c][c];
            for (int j = c; j < 4; ++j) A[i][j] -= f * A[c][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = A[i][3];
        for (int j = i + 1; j < 3; ++j) s -= A[i][j] * out[j];
        out[i] = s / A[i][i];
    }
}

static void gauss_jacobi3(int alpha, double x[3], double w[3])
{
    /* monic p(x) = x^3 + c2 x^2 + c1 x + c0 orthogonal to 1, x, x^2 */
    double H[3][3], r[3], c[3];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) H[i][j] = beta_moment(i + j, alpha);
        r[i] = -beta_moment(i + 3, alpha);
    }
    solve3(H, r, c); /* c[0]=c0, c[1]=c1, c[2]=c2 */
    double guess[3] = {0.1, 0.45, 0.85};
    for (int i = 0; i < 3; ++i) {
        double t = guess[i];
        for (int it = 0; it < 200; ++it) {
            /* deflate already-found roots */
            double p = ((t + c[2]) * t + c[1]) * t + c[0];
            double dp = (3.0 * t + 2.0 * c[2]) * t + c[1];
            double s = 0.0;
            for (int k = 0; k < i; ++k) s += 1.0 / (t - x[k]);
            double dt = p / (dp - p * s);
            t -= dt;
            if (fabs(dt) < 1e-17) break;
        }
        x[i] = t;
    }
    /* sort */
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (x[j] < x[i]) {
                double t = x[i];
                x[i] = x[j];
                x[j] = t;
            }
    double V[3][3], m[3];
    for (int k = 0; k < 3; ++k) {
        for (int j = 0; j < 3; ++j) V[k][j] = pow(x[j], k);
        m[k] = beta_moment(k, alpha);
    }
    solve3(V, m, w);
}

/* Symmetric 6-point degree-4 triangle rule (two S21 orbits, Strang-Fix /
 * Dunavant).  Solved here from its moment equations by Newton, starting from
 * the published 12-digit values, so every digit is the rule's own. */
int pbref_rule_tri6(double *bary, double *w)
{
    double a[2] = {0.445948490915965, 0.091576213509771};
    double ww[2] = {0.223381589678011, 0.109951743655322};
    /* unknowns z = (a0, w0, a1, w1); equations k = 0,2,3,4:
       sum_o w_o (2 a_o^k + (1-2a_o)^k) = 2 / ((k+1)(k+2)), the mean of
       lambda_1^k over the triangle (three points per orbit) */
    const int ks[4] = {0, 2, 3, 4};
    for (int it = 0; it < 50; ++it) {
        double F[4], J[4][4];
        for (int e = 0; e < 4; ++e) {
            int k = ks[e];
            double target = 2.0 / ((k + 1.0) * (k + 2.0));
            F[e] = -target;
            for (int o = 0; o < 2; ++o) {
                double b = 1.0 - 2.0 * a[o];
                double val = 2.0 * pow(a[o], k) + pow(b, k);
                double dval = (k == 0) ? 0.0 : 2.0 * k * pow(a[o], k - 1) - 2.0 * k * pow(b, k - 1);
                F[e] += ww[o] * val;
                J[e][2 * o] = ww[o] * dval;
                J[e][2 * o + 1] = val;
            }
        }
        /* solve J dz = -F (4x4, Gaussian elimination) */
        double A[4][5];
        for (int i = 0; i < 4; ++i) {
            for (int j = 0; j < 4; ++j) A[i][j] = J[i][j];
            A[i][4] = -F[i];
        }
        for (int cidx = 0; cidx < 4; ++cidx) {
            int p = cidx;
            for (int i = cidx + 1; i < 4; ++i)
                if (fabs(A[i][cidx]) > fabs(A[p][cidx])) p = i;
            for (int j = 0; j < 5; ++j) {
                double t = A[cidx][j];
                A[cidx][j] = A[p][j];
                A[p][j] = t;
            }
            for (int i = cidx + 1; i < 4; ++i) {
                double f = A[i][cidx] / A[cidx][cidx];
                for (int j = cidx; j < 5; ++j) A[i][j] -= f * A[cidx][j];
            }
        }
        double dz[4];
        for (int i = 3; i >= 0; --i) {
            double s = A[i][4];
            for (int j = i + 1; j < 4; ++j) s -= A[i][j] * dz[j];
            dz[i] = s / A[i][i];
        }
        a[0] += dz[0];
        ww[0] += dz[1];
        a[1] += dz[2];
        ww[1] += dz[3];
        if (fabs(dz[0]) + fabs(dz[1]) + fabs(dz[2]) + fabs(dz[3]) < 1e-17) break;
    }
    int q = 0;
    for (int o = 0; o < 2; ++o) {
        double b = 1.0 - 2.0 * a[o];
        double pts[3][3] = {{b, a[o], a[o]}, {a[o], b, a[o]}, {a[o], a[o], b}};
        for (int p = 0; p < 3; ++p, ++q) {
            for (int d = 0; d < 3; ++d) bary[3 * q + d] = pts[p][d];
            w[q] = ww[o];
        }
    }
    return 6;
}

/* m x m collapsed (Duffy) Gauss rule on the triangle, exact to degree 2m-2. */
int pbref_rule_tri_collapsed(int m, double *bary, double *w)
{
    double *x = malloc(sizeof(double) * m), *wx = malloc(sizeof(double) * m);
    pbref_rule_gauss01(m, x, wx);
    int q = 0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j, ++q) {
            double s = x[i], t = x[j];
            /* (xi1, xi2) = (s, s t) in {0 <= xi2 <= xi1 <= 1}; barycentrics of
               P0 + xi1 (P1-P0) + xi2 (P2-P1) are (1-xi1, xi1-xi2, xi2) */
            bary[3 * q + 0] = 1.0 - s;
            bary[3 * q + 1] = s - s * t;
            bary[3 * q + 2] = s * t;
            w[q] = 2.0 * wx[i] * wx[j] * s; /* area of reference cell = 1/2 */
        }
    free(x);
    free(wx);
    return m * m;
}

/* Stroud conical-product rule on the tetrahedron: 3 Gauss-Jacobi points for
 * the weights (1-x)^2 and (1-x)^1 and 3 Gauss-Legendre points; 27 points,
 * positive weights, exact to total degree 5. */
int pbref_rule_tet27(double *bary, double *w)
{
    double x2[3], w2[3], x1[3], w1[3], x0[3], w0[3];
    gauss_jacobi3(2, x2, w2);
    gauss_jacobi3(1, x1, w1);
    gauss_jacobi3(0, x0, w0);
    int q = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k, ++q) {
                double X = x2[i];
                double Y = x1[j] * (1.0 - X);
                double Z = x0[k] * (1.0 - X) * (1.0 - x1[j]);
                bary[4 * q + 0] = 1.0 - X - Y - Z;
                bary[4 * q + 1] = X;
                bary[4 * q + 2] = Y;
                bary[4 * q + 3] = Z;
                w[q] = 6.0 * w2[i] * w1[j] * w0[k]; /* reference volume = 1/6 */
            }
    return 27;
}

/* ------------------------------------------------------------------------- */
/* problem state                                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t nv, nt;
    int32_t *g;       /* local vertex -> FEM node (a surface given over FEM nodes) */
    double *xv;       /* own vertex coordinates (a surface given independently), else NULL */
    int32_t *itet;    /* independent surface: the tet holding each vertex ... */
    double *iw;       /* ... and the vertex's 4 barycentric coordinates in it */
    int32_t *tri;     /* triangles in local vertex ids, 3*nt */
    int32_t *v2t_ptr; /* vertex -> triangles adjacency */
    int32_t *v2t;
    double *area, *nrm; /* nt, 3*nt */
    double kappa;
    double *V, *K;      /* dense nv x nv, lazily */
} surface;

struct pbref {
    int64_t nn, nt, nq;
    double *x;
    int32_t *tet;
    double *qx, *qz;
    double eps_m, eps_s, kappa, temp, lB, kT;
    surface s[3];    /* Gamma_m, Gamma_s; s[2]: the independent Gamma_m mesh of the two-field form */
    int32_t *loc[2]; /* FEM node -> local surface vertex or -1 */
    int reg_order, n_ss;
    int nrq;
    double *rq_b, *rq_w; /* regular triangle rule */
    double tq_b[27 * 4], tq_w[27];
    double *ss_x, *ss_w;
    int32_t *n2t_ptr, *n2t; /* FEM node -> tets */
    double *tgrad, *tvol;   /* per-tet barycentric gradients (4x3) and volume */
    double *rhs_extra;      /* optional vector added to b (manufactured-solution tests) */
    /* two-field form (Sec. 2.3, eq. fembem_matrix): the tets from nt_i on fill
     * the solute, where the permittivity is eps_m and there is no reaction
     * term; otherwise nt_i = nt and every tet is in the shell */
    int64_t nt_i;
    int two_field;
    /* two-field form with a Gamma_m surface mesh independent of the volume
     * mesh (s[2]): the reaction potential and lam_m live on it, and its
     * trace of u is the P1 interpolant of u at its vertices (Sec. 2.3.1) */
    int has_r;
};

/* permittivity and reaction coefficient eps kappa^2 of tet t */
static double tet_eps(const pbref *p, int64_t t) { return t < p->nt_i ? p->eps_s : p->eps_m; }
static double tet_react(const pbref *p, int64_t t) { return t < p->nt_i ? p->eps_s * p->kappa * p->kappa : 0.0; }

static int64_t nunk(const pbref *p) { return p->nn + p->s[0].nv + p->s[1].nv; }
static void compute_tet_geom(const pbref *p, int64_t t, double grad[4][3], double *vol);

static void vsub(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}
static double vdot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void vcross(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static int build_surface(pbref *p, int which, int64_t nt, const int32_t *tri, double kappa)
{
    surface *S = &p->s[which];
    S->nt = nt;
    S->kappa = kappa;
    int32_t *loc = malloc(sizeof(int32_t) * p->nn);
    for (int64_t i = 0; i < p->nn; ++i) loc[i] = -1;
    for (int64_t t = 0; t < 3 * nt; ++t) {
        if (tri[t] < 0 || tri[t] >= p->nn) {
            free(loc);
            return -1;
        }
        loc[tri[t]] = 0;
    }
    int64_t nv = 0;
    for (int64_t i = 0; i < p->nn; ++i)
        if (loc[i] == 0) loc[i] = (int32_t)nv++;
    S->nv = nv;
    S->g = malloc(sizeof(int32_t) * nv);
    for (int64_t i = 0; i < p->nn; ++i)
        if (loc[i] >= 0) S->g[loc[i]] = (int32_t)i;
    S->tri = malloc(sizeof(int32_t) * 3 * nt);
    for (int64_t t = 0; t < 3 * nt; ++t) S->tri[t] = loc[tri[t]];
    S->area = malloc(sizeof(double) * nt);
    S->nrm = malloc(sizeof(double) * 3 * nt);
    for (int64_t t = 0; t < nt; ++t) {
        const double *a = p->x + 3 * tri[3 * t], *b = p->x + 3 * tri[3 * t + 1], *c = p->x + 3 * tri[3 * t + 2];
        double e1[3], e2[3], n[3];
        vsub(b, a, e1);
        vsub(c, a, e2);
        vcross(e1, e2, n);
        double len = sqrt(vdot(n, n));
        S->area[t] = 0.5 * len;
        for (int d = 0; d < 3; ++d) S->nrm[3 * t + d] = n[d] / len;
    }
    S->v2t_ptr = calloc(nv + 1, sizeof(int32_t));
    for (int64_t t = 0; t < 3 * nt; ++t) S->v2t_ptr[S->tri[t] + 1]++;
    for (int64_t i = 0; i < nv; ++i) S->v2t_ptr[i + 1] += S->v2t_ptr[i];
    S->v2t = malloc(sizeof(int32_t) * 3 * nt);
    int32_t *fill = calloc(nv, sizeof(int32_t));
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t v = S->tri[3 * t + k];
            S->v2t[S->v2t_ptr[v] + fill[v]++] = (int32_t)t;
        }
    free(fill);
    p->loc[which] = loc;
    S->V = S->K = NULL;
    return 0;
}

pbref *pbref_create(int64_t n_nodes, const double *nodes, int64_t n_tets, const int32_t *tets,
                    int64_t n_tri_m, const int32_t *tri_m, int64_t n_tri_s, const int32_t *tri_s,
                    int64_t n_q, const double *q_xyz, const double *q_z, double eps_in, double eps_out,
                    double kappa, double temperature, int reg_order, int n_ss)
{
    pbref *p = calloc(1, sizeof(pbref));
    p->nn = n_nodes;
    p->nt = n_tets;
    p->nt_i = n_tets;
    p->nq = n_q;
    p->x = malloc(sizeof(double) * 3 * n_nodes);
    memcpy(p->x, nodes, sizeof(double) * 3 * n_nodes);
    p->tet = malloc(sizeof(int32_t) * 4 * n_tets);
    memcpy(p->tet, tets, sizeof(int32_t) * 4 * n_tets);
    p->qx = malloc(sizeof(double) * 3 * (n_q > 0 ? n_q : 1));
    p->qz = malloc(sizeof(double) * (n_q > 0 ? n_q : 1));
    if (n_q) {
        memcpy(p->qx, q_xyz, sizeof(double) * 3 * n_q);
        memcpy(p->qz, q_z, sizeof(double) * n_q);
    }
    p->eps_m = eps_in;
    p->eps_s = eps_out;
    p->kappa = kappa;
    p->temp = temperature;
    p->lB = E_CHARGE * E_CHARGE / (4.0 * PI * EPS0 * K_BOLTZ * temperature) * 1e10;
    p->kT = K_BOLTZ * temperature * N_AVO / (1000.0 * CAL);
    p->reg_order = reg_order;
    p->n_ss = n_ss;
    if (build_surface(p, 0, n_tri_m, tri_m, 0.0) || build_surface(p, 1, n_tri_s, tri_s, kappa)) {
        pbref_destroy(p);
        return NULL;
    }
    if (reg_order <= 0) {
        p->nrq = 6;
        p->rq_b = malloc(sizeof(double) * 18);
        p->rq_w = malloc(sizeof(double) * 6);
        pbref_rule_tri6(p->rq_b, p->rq_w);
    } else {
        p->nrq = reg_order * reg_order;
        p->rq_b = malloc(sizeof(double) * 3 * p->nrq);
        p->rq_w = malloc(sizeof(double) * p->nrq);
        pbref_rule_tri_collapsed(reg_order, p->rq_b, p->rq_w);
    }
    pbref_rule_tet27(p->tq_b, p->tq_w);
    p->ss_x = malloc(sizeof(double) * n_ss);
    p->ss_w = malloc(sizeof(double) * n_ss);
    pbref_rule_gauss01(n_ss, p->ss_x, p->ss_w);
    /* node -> tet adjacency (used by the row-sampled products) */
    p->n2t_ptr = calloc(n_nodes + 1, sizeof(int32_t));
    for (int64_t i = 0; i < 4 * n_tets; ++i) p->n2t_ptr[tets[i] + 1]++;
    for (int64_t i = 0; i < n_nodes; ++i) p->n2t_ptr[i + 1] += p->n2t_ptr[i];
    p->n2t = malloc(sizeof(int32_t) * 4 * n_tets);
    int32_t *fill = calloc(n_nodes, sizeof(int32_t));
    for (int64_t t = 0; t < n_tets; ++t)
        for (int k = 0; k < 4; ++k) {
            int32_t v = tets[4 * t + k];
            p->n2t[p->n2t_ptr[v] + fill[v]++] = (int32_t)t;
        }
    free(fill);
    p->tgrad = malloc(sizeof(double) * 12 * (n_tets > 0 ? n_tets : 1));
    p->tvol = malloc(sizeof(double) * (n_tets > 0 ? n_tets : 1));
    for (int64_t t = 0; t < n_tets; ++t) {
        double G[4][3];
        compute_tet_geom(p, t, G, &p->tvol[t]);
        memcpy(p->tgrad + 12 * t, G, sizeof G);
    }
    return p;
}

static void free_surface(surface *S)
{
    free(S->g);
    free(S->xv);
    free(S->itet);
    free(S->iw);
    free(S->tri);
    free(S->v2t_ptr);
    free(S->v2t);
    free(S->area);
    free(S->nrm);
    free(S->V);
    free(S->K);
    memset(S, 0, sizeof *S);
}

void pbref_destroy(pbref *p)
{
    if (!p) return;
    free(p->rhs_extra);
    for (int w = 0; w < 3; ++w) free_surface(&p->s[w]);
    for (int w = 0; w < 2; ++w) free(p->loc[w]);
    free(p->x);
    free(p->tet);
    free(p->qx);
    free(p->qz);
    free(p->rq_b);
    free(p->rq_w);
    free(p->ss_x);
    free(p->ss_w);
    free(p->n2t_ptr);
    free(p->n2t);
    free(p->tgrad);
    free(p->tvol);
    free(p);
}

void pbref_sizes(const pbref *p, int64_t out[4])
{
    out[0] = p->nn;
    out[1] = p->s[0].nv;
    out[2] = p->s[1].nv;
    out[3] = nunk(p);
}

void pbref_constants(const pbref *p, double out[2])
{
    out[0] = p->lB;
    out[1] = p->kT;
}

void pbref_surface_nodes(const pbref *p, int surf, int32_t *out)
{
    memcpy(out, p->s[surf].g, sizeof(int32_t) * p->s[surf].nv);
}

/* ------------------------------------------------------------------------- */
/* boundary operators                                                         */
/* ------------------------------------------------------------------------- */

/* Fundamental solution g = exp(-kappa r)/(4 pi r) (kappa = 0: Laplace) and its
 * normal derivative in the source point y: d g / d n_y = (x-y).n_y (1 + kappa
 * r) exp(-kappa r) / (4 pi r^3). */
static void kernel_eval(double kappa, const double *x, const double *y, const double *ny, double *g,
                        double *dg)
{
    double d[3];
    vsub(x, y, d);
    double r = sqrt(vdot(d, d));
    double e = exp(-kappa * r);
    *g = e / (4.0 * PI * r);
    *dg = vdot(d, ny) * (1.0 + kappa * r) * e / (4.0 * PI * r * r * r);
}

static const double *vx(const pbref *p, const surface *S, int32_t lv)
{
    return S->xv ? S->xv + 3 * lv : p->x + 3 * S->g[lv];
}

/* Regular (non-touching) pair: tensor product of the triangle rule. */
static void pair_regular(const pbref *p, const surface *S, int64_t ta, int64_t sb, double V[3][3],
                         double K[3][3])
{
    const int32_t *A = S->tri + 3 * ta, *B = S->tri + 3 * sb;
    const double *ny = S->nrm + 3 * sb;
    double fa = S->area[ta], fb = S->area[sb];
    for (int i = 0; i < p->nrq; ++i) {
        const double *li = p->rq_b + 3 * i;
        double x[3] = {0, 0, 0};
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) x[d] += li[k] * vx(p, S, A[k])[d];
        for (int j = 0; j < p->nrq; ++j) {
            const double *lj = p->rq_b + 3 * j;
            double y[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) y[d] += lj[k] * vx(p, S, B[k])[d];
            double g, dg;
            kernel_eval(S->kappa, x, y, ny, &g, &dg);
            double w = fa * p->rq_w[i] * fb * p->rq_w[j];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    V[a][b] += w * li[a] * lj[b] * g;
                    K[a][b] += w * li[a] * lj[b] * dg;
                }
        }
    }
}

/* Sauter-Schwab rules on the reference triangle {0 <= xi2 <= xi1 <= 1} with
 * chi(xi) = P0 + xi1 (P1 - P0) + xi2 (P2 - P1) and P1 shape functions
 * (1 - xi1, xi1 - xi2, xi2) (Sauter & Schwab, Boundary Element Methods, 5.2).
 * The 4-D integrand is written in the variables (xi, eta1, eta2, eta3) of
 * [0,1]^4; each case is a sum of Duffy-type maps with the Jacobian shown. */
typedef struct {
    double x1, x2, y1, y2;
} ref_pair;

static int ss_maps(int kind, double xi, double e1, double e2, double e3, ref_pair *m, double *jac)
{
    if (kind == 3) { /* identical panels: six maps, Jacobian xi^3 eta1^2 eta2 */
        double J = xi * xi * xi * e1 * e1 * e2;
        ref_pair t[6] = {
            {xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1)},
            {xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2)},
            {xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2)},
            {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3)},
            {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2)},
            {xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)},
        };
        for (int i = 0; i < 6; ++i) {
            m[i] = t[i];
            jac[i] = J;
        }
        return 6;
    }
    if (kind == 2) { /* common edge P0-P1 of both: five maps */
        double J1 = xi * xi * xi * e1 * e1;
        double J = J1 * e2;
        ref_pair t[5] = {
            {xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2)},
            {xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)},
            {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3},
            {xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1},
            {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2},
        };
        for (int i = 0; i < 5; ++i) {
            m[i] = t[i];
            jac[i] = (i == 0) ? J1 : J;
        }
        return 5;
    }
    /* common vertex P0 of both: two maps, Jacobian xi^3 eta2 */
    double J = xi * xi * xi * e2;
    m[0] = (ref_pair){xi, xi * e1, xi * e2, xi * e2 * e3};
    m[1] = (ref_pair){xi * e2, xi * e2 * e3, xi, xi * e1};
    jac[0] = jac[1] = J;
    return 2;
}

static void pair_singular(const pbref *p, const surface *S, int64_t ta, int64_t sb, int kind,
                          const int pa[3], const int pb[3], double V[3][3], double K[3][3])
{
    const int32_t *A = S->tri + 3 * ta, *B = S->tri + 3 * sb;
    const double *P[3], *Q[3];
    for (int k = 0; k < 3; ++k) {
        P[k] = vx(p, S, A[pa[k]]);
        Q[k] = vx(p, S, B[pb[k]]);
    }
    const double *ny = S->nrm + 3 * sb;
    double scale = 4.0 * S->area[ta] * S->area[sb]; /* |det chi_tau| |det chi_sig| */
    int n = p->n_ss;
    for (int i0 = 0; i0 < n; ++i0)
        for (int i1 = 0; i1 < n; ++i1)
            for (int i2 = 0; i2 < n; ++i2)
                for (int i3 = 0; i3 < n; ++i3) {
                    double w4 = p->ss_w[i0] * p->ss_w[i1] * p->ss_w[i2] * p->ss_w[i3];
                    ref_pair m[6];
                    double jac[6];
                    int nm = ss_maps(kind, p->ss_x[i0], p->ss_x[i1], p->ss_x[i2], p->ss_x[i3], m, jac);
                    for (int r = 0; r < nm; ++r) {
                        double x[3], y[3];
                        for (int d = 0; d < 3; ++d) {
                            x[d] = P[0][d] + m[r].x1 * (P[1][d] - P[0][d]) + m[r].x2 * (P[2][d] - P[1][d]);
                            y[d] = Q[0][d] + m[r].y1 * (Q[1][d] - Q[0][d]) + m[r].y2 * (Q[2][d] - Q[1][d]);
                        }
                        double fx[3] = {1.0 - m[r].x1, m[r].x1 - m[r].x2, m[r].x2};
                        double fy[3] = {1.0 - m[r].y1, m[r].y1 - m[r].y2, m[r].y2};
                        double g, dg;
                        kernel_eval(S->kappa, x, y, ny, &g, &dg);
                        if (kind == 3) dg = 0.0; /* (x-y).n_y vanishes on a flat panel */
                        double w = scale * w4 * jac[r];
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) {
                                V[pa[a]][pb[b]] += w * fx[a] * fy[b] * g;
                                K[pa[a]][pb[b]] += w * fx[a] * fy[b] * dg;
                            }
                    }
                }
}

/* Local 3x3 blocks V[a][b] = int_tau int_sig phi_a(x) phi_b(y) g and K likewise
 * with dg/dn_y, indexed by the triangles' own vertex order. */
static void pair_integral(const pbref *p, const surface *S, int64_t ta, int64_t sb, double V[3][3],
                          double K[3][3])
{
    memset(V, 0, sizeof(double) * 9);
    memset(K, 0, sizeof(double) * 9);
    const int32_t *A = S->tri + 3 * ta, *B = S->tri + 3 * sb;
    int shared = 0, ia[3], ib[3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (A[a] == B[b]) {
                ia[shared] = a;
                ib[shared] = b;
                shared++;
            }
    if (shared == 0) {
        pair_regular(p, S, ta, sb, V, K);
        return;
    }
    int pa[3], pb[3];
    if (shared == 3) {
        for (int k = 0; k < 3; ++k) pa[k] = pb[k] = k;
    } else if (shared == 2) {
        pa[0] = ia[0];
        pa[1] = ia[1];
        pa[2] = 3 - ia[0] - ia[1];
        pb[0] = ib[0];
        pb[1] = ib[1];
        pb[2] = 3 - ib[0] - ib[1];
    } else {
        pa[0] = ia[0];
        pa[1] = (ia[0] + 1) % 3;
        pa[2] = (ia[0] + 2) % 3;
        pb[0] = ib[0];
        pb[1] = (ib[0] + 1) % 3;
        pb[2] = (ib[0] + 2) % 3;
    }
    pair_singular(p, S, ta, sb, shared, pa, pb, V, K);
}

int pbref_pair_integral(pbref *p, int surf, int64_t tau, int64_t sig, double *V9, double *K9)
{
    double V[3][3], K[3][3];
    pair_integral(p, &p->s[surf], tau, sig, V, K);
    memcpy(V9, V, sizeof V);
    memcpy(K9, K, sizeof K);
    return 0;
}

/* One Galerkin row: V_ij = sum_{tau ∋ i} sum_{sig} int int phi_i phi_j g. */
static void bem_row(const pbref *p, const surface *S, int64_t i, double *Vr, double *Kr)
{
    memset(Vr, 0, sizeof(double) * S->nv);
    memset(Kr, 0, sizeof(double) * S->nv);
    for (int32_t e = S->v2t_ptr[i]; e < S->v2t_ptr[i + 1]; ++e) {
        int64_t ta = S->v2t[e];
        int a = 0;
        while (S->tri[3 * ta + a] != i) ++a;
        for (int64_t sb = 0; sb < S->nt; ++sb) {
            double V[3][3], K[3][3];
            pair_integral(p, S, ta, sb, V, K);
            for (int b = 0; b < 3; ++b) {
                int32_t j = S->tri[3 * sb + b];
                Vr[j] += V[a][b];
                Kr[j] += K[a][b];
            }
        }
    }
}

int pbref_bem_dense(pbref *p, int surf)
{
    surface *S = &p->s[surf];
    if (S->V) return 0;
    int64_t n = S->nv;
    S->V = malloc(sizeof(double) * n * n);
    S->K = malloc(sizeof(double) * n * n);
    if (!S->V || !S->K) return -4;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) bem_row(p, S, i, S->V + i * n, S->K + i * n);
    return 0;
}

int pbref_bem_get(const pbref *p, int surf, double *V, double *K)
{
    const surface *S = &p->s[surf];
    if (!S->V) return -8;
    memcpy(V, S->V, sizeof(double) * S->nv * S->nv);
    memcpy(K, S->K, sizeof(double) * S->nv * S->nv);
    return 0;
}

int pbref_bem_rows(pbref *p, int surf, int64_t nrows, const int64_t *rows, double *V, double *K)
{
    surface *S = &p->s[surf];
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) bem_row(p, S, rows[r], V + r * S->nv, K + r * S->nv);
    return 0;
}

/* Exact P1 Gram matrix on each triangle: |tau| (1 + delta_ab) / 12. */
void pbref_surface_mass_apply(const pbref *p, int surf, const double *x, double *y)
{
    const surface *S = &p->s[surf];
    memset(y, 0, sizeof(double) * S->nv);
    for (int64_t t = 0; t < S->nt; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                int32_t i = S->tri[3 * t + a], j = S->tri[3 * t + b];
                y[i] += S->area[t] * (a == b ? 2.0 : 1.0) / 12.0 * x[j];
            }
}

static double coulomb(const pbref *p, const double *x)
{
    double s = 0.0;
    for (int64_t k = 0; k < p->nq; ++k) {
        double d[3];
        vsub(x, p->qx + 3 * k, d);
        s += p->lB * p->qz[k] / (p->eps_m * sqrt(vdot(d, d)));
    }
    return s;
}

/* f_i = int_{Gamma_m} phi_i phi_coul, with the regular triangle rule. */
static void coulomb_load_on(const pbref *p, const surface *S, double *f)
{
    memset(f, 0, sizeof(double) * S->nv);
    for (int64_t t = 0; t < S->nt; ++t)
        for (int q = 0; q < p->nrq; ++q) {
            const double *l = p->rq_b + 3 * q;
            double x[3] = {0, 0, 0};
            for (int k = 0; k < 3; ++k)
                for (int d = 0; d < 3; ++d) x[d] += l[k] * vx(p, S, S->tri[3 * t + k])[d];
            double c = S->area[t] * p->rq_w[q] * coulomb(p, x);
            for (int a = 0; a < 3; ++a) f[S->tri[3 * t + a]] += c * l[a];
        }
}

void pbref_coulomb_load(const pbref *p, double *f) { coulomb_load_on(p, &p->s[0], f); }

/* ------------------------------------------------------------------------- */
/* FEM on the shell                                                           */
/* ------------------------------------------------------------------------- */
static void compute_tet_geom(const pbref *p, int64_t t, double grad[4][3], double *vol)
{
    const int32_t *T = p->tet + 4 * t;
    const double *x0 = p->x + 3 * T[0];
    double B[3][3]; /* columns x_k - x_0 */
    for (int k = 1; k <= 3; ++k)
        for (int d = 0; d < 3; ++d) B[d][k - 1] = p->x[3 * T[k] + d] - x0[d];
    double det = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                 B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                 B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    *vol = fabs(det) / 6.0;
    /* rows of B^{-1} are the gradients of the barycentrics 1..3 */
    double inv[3][3];
    inv[0][0] = (B[1][1] * B[2][2] - B[1][2] * B[2][1]) / det;
    inv[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) / det;
    inv[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) / det;
    inv[1][0] = (B[1][2] * B[2][0] - B[1][0] * B[2][2]) / det;
    inv[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) / det;
    inv[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) / det;
    inv[2][0] = (B[1][0] * B[2][1] - B[1][1] * B[2][0]) / det;
    inv[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) / det;
    inv[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) / det;
    for (int d = 0; d < 3; ++d) {
        grad[1][d] = inv[0][d];
        grad[2][d] = inv[1][d];
        grad[3][d] = inv[2][d];
        grad[0][d] = -inv[0][d] - inv[1][d] - inv[2][d];
    }
}

/* cached copy of compute_tet_geom (filled once at creation) */
static void tet_geom(const pbref *p, int64_t t, double grad[4][3], double *vol)
{
    memcpy(grad, p->tgrad + 12 * t, sizeof(double) * 12);
    *vol = p->tvol[t];
}

/* Scheme functions: N, N', N'' for LIN (t), the Taylor schemes T3 / T5 / T7
 * (sinh t = sum over odd j of t^j / j!, cut after j = 3, 5, 7), HS (sinh t);
 * NONE has no reaction term. */
static int taylor_order(int s)
{
    return s == PBREF_T3 ? 3 : s == PBREF_T5 ? 5 : s == PBREF_T7 ? 7 : 0;
}
/* sum of t^j / j! over j <= m with j of the parity of m */
static double series(int m, double t)
{
    double sum = 0.0, term = (m % 2) ? t : 1.0;
    for (int j = m % 2; j <= m; j += 2) {
        sum += term;
        term *= t * t / ((j + 1.0) * (j + 2.0));
    }
    return sum;
}
static double sch_f(int s, double t)
{
    if (s == PBREF_NONE) return 0.0;
    if (s == PBREF_LIN) return t;
    if (s == PBREF_HS) return sinh(t);
    return series(taylor_order(s), t);
}
static double sch_d1(int s, double t)
{
    if (s == PBREF_NONE) return 0.0;
    if (s == PBREF_LIN) return 1.0;
    if (s == PBREF_HS) return cosh(t);
    return series(taylor_order(s) - 1, t);
}
static double sch_d2(int s, double t)
{
    if (s == PBREF_NONE || s == PBREF_LIN) return 0.0;
    if (s == PBREF_HS) return sinh(t);
    return series(taylor_order(s) - 2, t);
}

void pbref_stiffness_entries(const pbref *p, int32_t *rows, int32_t *cols, double *vals)
{
    for (int64_t t = 0; t < p->nt; ++t) {
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                int64_t e = 16 * t + 4 * a + b;
                rows[e] = p->tet[4 * t + a];
                cols[e] = p->tet[4 * t + b];
                vals[e] = tet_eps(p, t) * vol * vdot(G[a], G[b]);
            }
    }
}

/* Consistent mass with the tet rule (exact for P1 x P1). */
void pbref_mass_entries(const pbref *p, int32_t *rows, int32_t *cols, double *vals)
{
    for (int64_t t = 0; t < p->nt; ++t) {
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int q = 0; q < 27; ++q) s += p->tq_w[q] * p->tq_b[4 * q + a] * p->tq_b[4 * q + b];
                int64_t e = 16 * t + 4 * a + b;
                rows[e] = p->tet[4 * t + a];
                cols[e] = p->tet[4 * t + b];
                vals[e] = vol * s;
            }
    }
}

/* Element contribution of the reaction term on tet t:
 *   mode 0: out_a += c int N(u_h) phi_a
 *   mode 1: out_a += c int N'(u_h) v_h phi_a
 *   mode 2: out_a += c int N''(u_h) v_h^2 phi_a
 * with c = eps_s kappa^2 (0 in a solute tet of the two-field form) and the
 * 27-point tet rule. */
static void tet_reaction(const pbref *p, int64_t t, int scheme, int mode, const double *u, const double *v,
                         double out[4])
{
    double G[4][3], vol;
    tet_geom(p, t, G, &vol);
    const int32_t *T = p->tet + 4 * t;
    double c = tet_react(p, t);
    for (int a = 0; a < 4; ++a) out[a] = 0.0;
    /* a solute tet has no reaction term; its N(u) is never evaluated (the
     * potential at a point charge's node is far outside sinh's range) */
    if (c == 0.0) return;
    for (int q = 0; q < 27; ++q) {
        const double *l = p->tq_b + 4 * q;
        double uh = 0.0, vh = 0.0;
        for (int k = 0; k < 4; ++k) {
            uh += l[k] * u[T[k]];
            if (v) vh += l[k] * v[T[k]];
        }
        double f = mode == 0 ? sch_f(scheme, uh) : mode == 1 ? sch_d1(scheme, uh) * vh : sch_d2(scheme, uh) * vh * vh;
        for (int a = 0; a < 4; ++a) out[a] += c * vol * p->tq_w[q] * f * l[a];
    }
}

static void fem_reaction(const pbref *p, int scheme, int mode, const double *u, const double *v, double *out)
{
    memset(out, 0, sizeof(double) * p->nn);
    for (int64_t t = 0; t < p->nt; ++t) {
        double e[4];
        tet_reaction(p, t, scheme, mode, u, v, e);
        for (int a = 0; a < 4; ++a) out[p->tet[4 * t + a]] += e[a];
    }
}

void pbref_fem_nonlinear(const pbref *p, int scheme, const double *u, double *out)
{
    fem_reaction(p, scheme, 0, u, NULL, out);
}
void pbref_fem_jacobian(const pbref *p, int scheme, const double *u, const double *v, double *out)
{
    fem_reaction(p, scheme, 1, u, v, out);
}
void pbref_fem_hessian(const pbref *p, int scheme, const double *u, const double *v, double *out)
{
    fem_reaction(p, scheme, 2, u, v, out);
}

static void stiffness_apply(const pbref *p, const double *v, double *y)
{
    memset(y, 0, sizeof(double) * p->nn);
    for (int64_t t = 0; t < p->nt; ++t) {
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                y[p->tet[4 * t + a]] += tet_eps(p, t) * vol * vdot(G[a], G[b]) * v[p->tet[4 * t + b]];
    }
}

/* diag(A + J_scheme(u)) */
static void fem_diag(const pbref *p, int scheme, const double *u, double *dg)
{
    memset(dg, 0, sizeof(double) * p->nn);
    for (int64_t t = 0; t < p->nt; ++t) {
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        const int32_t *T = p->tet + 4 * t;
        const double c = tet_react(p, t);
        for (int a = 0; a < 4; ++a) {
            double s = tet_eps(p, t) * vol * vdot(G[a], G[a]);
            for (int q = 0; q < 27 && c != 0.0; ++q) {
                const double *l = p->tq_b + 4 * q;
                double uh = 0.0;
                for (int k = 0; k < 4; ++k) uh += l[k] * u[T[k]];
                s += c * vol * p->tq_w[q] * sch_d1(scheme, uh) * l[a] * l[a];
            }
            dg[T[a]] += s;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* coupled operator                                                            */
/* ------------------------------------------------------------------------- */
static int need_dense(pbref *p)
{
    int r = pbref_bem_dense(p, 0);
    if (r) return r;
    return pbref_bem_dense(p, 1);
}

/* y = A_coupled phi (the linear operator of the 3x3 block system) */
int pbref_apply_A(pbref *p, const double *phi, double *y)
{
    int r = need_dense(p);
    if (r) return r;
    int64_t nn = p->nn, nm = p->s[0].nv, ns = p->s[1].nv;
    const double *u = phi, *lm = phi + nn, *ls = phi + nn + nm;
    double *yu = y, *ym = y + nn, *ys = y + nn + nm;
    /* FEM row: A u + eps_m T_m^T M_m lam_m - eps_s T_s^T M_s lam_s; in the
     * two-field form Gamma_m is inside the FEM domain: no lam_m term */
    stiffness_apply(p, u, yu);
    double *tmp = malloc(sizeof(double) * (nm > ns ? nm : ns));
    pbref_surface_mass_apply(p, 0, lm, tmp);
    if (!p->two_field)
        for (int64_t i = 0; i < nm; ++i) yu[p->s[0].g[i]] += p->eps_m * tmp[i];
    pbref_surface_mass_apply(p, 1, ls, tmp);
    for (int64_t i = 0; i < ns; ++i) yu[p->s[1].g[i]] -= p->eps_s * tmp[i];
    /* Gamma_m row: (1/2 M_m + K0_m) u_m - V0_m lam_m; in the two-field form
     * lam_m is not an unknown of the solve (it is recovered afterwards) and
     * its row is the identity, so it stays zero */
    double *um = malloc(sizeof(double) * nm), *us = malloc(sizeof(double) * ns);
    for (int64_t i = 0; i < nm; ++i) um[i] = u[p->s[0].g[i]];
    for (int64_t i = 0; i < ns; ++i) us[i] = u[p->s[1].g[i]];
    pbref_surface_mass_apply(p, 0, um, tmp);
#pragma omp parallel for
    for (int64_t i = 0; i < nm; ++i) {
        double s = 0.5 * tmp[i];
        for (int64_t j = 0; j < nm; ++j) s += p->s[0].K[i * nm + j] * um[j] - p->s[0].V[i * nm + j] * lm[j];
        ym[i] = p->two_field ? lm[i] : s;
    }
    /* Gamma_s row: (1/2 M_s - Kk_s) u_s + Vk_s lam_s */
    pbref_surface_mass_apply(p, 1, us, tmp);
#pragma omp parallel for
    for (int64_t i = 0; i < ns; ++i) {
        double s = 0.5 * tmp[i];
        for (int64_t j = 0; j < ns; ++j) s += -p->s[1].K[i * ns + j] * us[j] + p->s[1].V[i * ns + j] * ls[j];
        ys[i] = s;
    }
    free(tmp);
    free(um);
    free(us);
    return 0;
}

/* Point-charge load of the two-field form (Sec. 2.3: rho_c = sum_k Q_k delta_k
 * tested with the P1 basis): b_a = sum_k Q_k phi_a(x_k), Q_k = 4 pi l_B z_k,
 * with phi_a(x_k) the barycentric coordinates of x_k in the solute tet that
 * holds it (the one whose smallest coordinate is largest). */
static int point_load(const pbref *p, double *b)
{
    memset(b, 0, sizeof(double) * p->nn);
    for (int64_t k = 0; k < p->nq; ++k) {
        const double *xk = p->qx + 3 * k;
        int64_t best = -1;
        double bmin = -1e300, bb[4] = {0, 0, 0, 0};
        for (int64_t t = p->nt_i; t < p->nt; ++t) {
            double G[4][3], vol, l[4], d[3], lo = 1e300;
            tet_geom(p, t, G, &vol);
            vsub(xk, p->x + 3 * p->tet[4 * t], d);
            for (int a = 0; a < 4; ++a) {
                l[a] = (a == 0 ? 1.0 : 0.0) + vdot(G[a], d);
                if (l[a] < lo) lo = l[a];
            }
            if (lo > bmin) {
                bmin = lo;
                best = t;
                memcpy(bb, l, sizeof bb);
            }
        }
        if (best < 0 || bmin < -1e-10) return -3;
        for (int a = 0; a < 4; ++a) b[p->tet[4 * best + a]] += 4.0 * PI * p->lB * p->qz[k] * bb[a];
    }
    return 0;
}

int pbref_set_two_field(pbref *p, int64_t n_tets_m)
{
    if (n_tets_m <= 0 || n_tets_m >= p->nt) return -1;
    p->nt_i = p->nt - n_tets_m;
    p->two_field = 1;
    return 0;
}

/* The tet of the FEM mesh that holds x: the one whose smallest barycentric
 * coordinate of x is largest (ties: the lowest tet id), and those
 * coordinates.  -1 if x lies outside every tet (by more than rounding). */
static int64_t locate_point(const pbref *p, const double *x, double l_out[4])
{
    int64_t best = -1;
    double bmin = -1e300;
    for (int64_t t = 0; t < p->nt; ++t) {
        double G[4][3], vol, l[4], d[3], lo = 1e300;
        tet_geom(p, t, G, &vol);
        vsub(x, p->x + 3 * p->tet[4 * t], d);
        for (int a = 0; a < 4; ++a) {
            l[a] = (a == 0 ? 1.0 : 0.0) + vdot(G[a], d);
            if (l[a] < lo) lo = l[a];
        }
        if (lo > bmin) {
            bmin = lo;
            best = t;
            memcpy(l_out, l, sizeof(double) * 4);
        }
    }
    return (best >= 0 && bmin >= -1e-10) ? best : -1;
}

/* Two-field form: a Gamma_m surface mesh given independently of the volume
 * mesh (its own vertices verts[3 nv] and triangles tri[3 nt], oriented like
 * the interface).  Sec. 2.3.1 takes the trace of the volume solution on it
 * by interpolation between the two meshes: here the P1 interpolant, i.e.
 * at each vertex the value of u in the tet that holds the vertex.  nv = 0
 * removes it.  Returns -1 for bad sizes or ids, -3 if a vertex lies outside
 * the FEM mesh. */
int pbref_set_reaction_surface(pbref *p, int64_t nv, const double *verts, int64_t nt, const int32_t *tri)
{
    surface *S = &p->s[2];
    free_surface(S);
    p->has_r = 0;
    if (nv == 0) return 0;
    if (nv < 3 || nt < 1) return -1;
    for (int64_t k = 0; k < 3 * nt; ++k)
        if (tri[k] < 0 || tri[k] >= nv) return -1;
    S->nv = nv;
    S->nt = nt;
    S->kappa = 0.0;
    S->xv = malloc(sizeof(double) * 3 * nv);
    memcpy(S->xv, verts, sizeof(double) * 3 * nv);
    S->g = malloc(sizeof(int32_t) * nv);
    for (int64_t i = 0; i < nv; ++i) S->g[i] = -1; /* no FEM node */
    S->tri = malloc(sizeof(int32_t) * 3 * nt);
    memcpy(S->tri, tri, sizeof(int32_t) * 3 * nt);
    S->area = malloc(sizeof(double) * nt);
    S->nrm = malloc(sizeof(double) * 3 * nt);
    for (int64_t t = 0; t < nt; ++t) {
        const double *a = vx(p, S, tri[3 * t]), *b = vx(p, S, tri[3 * t + 1]), *c = vx(p, S, tri[3 * t + 2]);
        double e1[3], e2[3], n[3];
        vsub(b, a, e1);
        vsub(c, a, e2);
        vcross(e1, e2, n);
        double len = sqrt(vdot(n, n));
        S->area[t] = 0.5 * len;
        for (int d = 0; d < 3; ++d) S->nrm[3 * t + d] = n[d] / len;
    }
    S->v2t_ptr = calloc(nv + 1, sizeof(int32_t));
    for (int64_t t = 0; t < 3 * nt; ++t) S->v2t_ptr[S->tri[t] + 1]++;
    for (int64_t i = 0; i < nv; ++i) S->v2t_ptr[i + 1] += S->v2t_ptr[i];
    S->v2t = malloc(sizeof(int32_t) * 3 * nt);
    int32_t *fill = calloc(nv, sizeof(int32_t));
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int32_t v = S->tri[3 * t + k];
            S->v2t[S->v2t_ptr[v] + fill[v]++] = (int32_t)t;
        }
    free(fill);
    S->itet = malloc(sizeof(int32_t) * nv);
    S->iw = malloc(sizeof(double) * 4 * nv);
    int bad = 0;
#pragma omp parallel for reduction(| : bad)
    for (int64_t i = 0; i < nv; ++i) {
        int64_t t = locate_point(p, S->xv + 3 * i, S->iw + 4 * i);
        S->itet[i] = (int32_t)t;
        if (t < 0) bad = 1;
    }
    if (bad) {
        free_surface(S);
        return -3;
    }
    p->has_r = 1;
    return 0;
}

/* Values of u on the vertices of S: node selection for a surface given
 * over FEM nodes, the P1 interpolant for an independent one. */
static void surface_trace(const pbref *p, const surface *S, const double *u, double *out)
{
    for (int64_t i = 0; i < S->nv; ++i) {
        if (S->itet) {
            const int32_t *T = p->tet + 4 * (int64_t)S->itet[i];
            const double *l = S->iw + 4 * i;
            out[i] = l[0] * u[T[0]] + l[1] * u[T[1]] + l[2] * u[T[2]] + l[3] * u[T[3]];
        } else {
            out[i] = u[S->g[i]];
        }
    }
}

/* the surface that carries lam_m and the reaction potential */
static int gamma_m_index(const pbref *p) { return (p->two_field && p->has_r) ? 2 : 0; }

int64_t pbref_gamma_m_vertices(const pbref *p) { return p->s[gamma_m_index(p)].nv; }

int pbref_gamma_m_trace(const pbref *p, const double *u, double *out)
{
    surface_trace(p, &p->s[gamma_m_index(p)], u, out);
    return 0;
}

int pbref_rhs(pbref *p, double *b)
{
    memset(b, 0, sizeof(double) * nunk(p));
    if (p->two_field) {
        int r = point_load(p, b);
        if (r) return r;
    } else {
        pbref_coulomb_load(p, b + p->nn);
    }
    if (p->rhs_extra)
        for (int64_t i = 0; i < nunk(p); ++i) b[i] += p->rhs_extra[i];
    return 0;
}

void pbref_set_rhs_extra(pbref *p, const double *e)
{
    free(p->rhs_extra);
    p->rhs_extra = NULL;
    if (!e) return;
    p->rhs_extra = malloc(sizeof(double) * nunk(p));
    memcpy(p->rhs_extra, e, sizeof(double) * nunk(p));
}

/* The Gamma rows of apply_A on a sample of rows, given those rows of the
 * dense operators (same loop as apply_A; used to time the oracle). */
int pbref_dense_rows_apply(const pbref *p, int surf, int64_t nrows, const double *V, const double *K,
                           const double *x, double *out)
{
    int64_t nv = p->s[surf].nv;
    const double *lam = x + p->nn + (surf == 0 ? 0 : p->s[0].nv);
#pragma omp parallel for
    for (int64_t r = 0; r < nrows; ++r) {
        double s = 0.0;
        for (int64_t j = 0; j < nv; ++j) {
            double uj = x[p->s[surf].g[j]];
            if (surf == 0)
                s += K[r * nv + j] * uj - V[r * nv + j] * lam[j];
            else
                s += -K[r * nv + j] * uj + V[r * nv + j] * lam[j];
        }
        out[r] = s;
    }
    return 0;
}

int pbref_residual(pbref *p, int scheme, const double *phi, double *F)
{
    int64_t n = nunk(p);
    int r = pbref_apply_A(p, phi, F);
    if (r) return r;
    double *Nu = malloc(sizeof(double) * p->nn), *b = malloc(sizeof(double) * n);
    pbref_fem_nonlinear(p, scheme, phi, Nu);
    pbref_rhs(p, b);
    for (int64_t i = 0; i < p->nn; ++i) F[i] += Nu[i];
    for (int64_t i = 0; i < n; ++i) F[i] -= b[i];
    free(Nu);
    free(b);
    return 0;
}

int pbref_apply_jacobian(pbref *p, int scheme, const double *phi, const double *v, double *Jv)
{
    int r = pbref_apply_A(p, v, Jv);
    if (r) return r;
    double *t = malloc(sizeof(double) * p->nn);
    pbref_fem_jacobian(p, scheme, phi, v, t);
    for (int64_t i = 0; i < p->nn; ++i) Jv[i] += t[i];
    free(t);
    return 0;
}

/* Row-sampled version: mode 0 -> rows of F(phi) (v ignored), mode 1 -> rows of J(phi) v. */
static int coupled_rows(pbref *p, int scheme, int mode, const double *phi, const double *v, int64_t nrows,
                        const int64_t *rows, double *out)
{
    int64_t nn = p->nn, nm = p->s[0].nv, ns = p->s[1].nv;
    const double *x = mode == 0 ? phi : v;
    double *fm = NULL, *bu = NULL;
    if (mode == 0) {
        fm = malloc(sizeof(double) * nm);
        pbref_coulomb_load(p, fm);
        if (p->two_field) {
            bu = malloc(sizeof(double) * nn);
            if (point_load(p, bu)) {
                free(fm);
                free(bu);
                return -3;
            }
        }
    }
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t row = rows[r];
        double s = 0.0;
        if (row < nn) {
            /* stiffness and reaction from the tets around this node */
            for (int32_t e = p->n2t_ptr[row]; e < p->n2t_ptr[row + 1]; ++e) {
                int64_t t = p->n2t[e];
                double G[4][3], vol;
                tet_geom(p, t, G, &vol);
                int a = 0;
                while (p->tet[4 * t + a] != row) ++a;
                for (int b = 0; b < 4; ++b) s += tet_eps(p, t) * vol * vdot(G[a], G[b]) * x[p->tet[4 * t + b]];
                double loc[4];
                tet_reaction(p, t, scheme, mode == 0 ? 0 : 1, phi, mode == 0 ? NULL : v, loc);
                s += loc[a];
            }
            if (bu) s -= bu[row];
            /* surface mass couplings */
            for (int w = p->two_field ? 1 : 0; w < 2; ++w) {
                const surface *S = &p->s[w];
                int32_t i = p->loc[w][row];
                if (i < 0) continue;
                const double *lam = x + nn + (w == 0 ? 0 : nm);
                double c = w == 0 ? p->eps_m : -p->eps_s;
                for (int32_t e = S->v2t_ptr[i]; e < S->v2t_ptr[i + 1]; ++e) {
                    int64_t t = S->v2t[e];
                    for (int b = 0; b < 3; ++b) {
                        int32_t j = S->tri[3 * t + b];
                        s += c * S->area[t] * (j == i ? 2.0 : 1.0) / 12.0 * lam[j];
                    }
                }
            }
        } else if (p->two_field && row < nn + nm) {
            s = x[row]; /* identity row of lam_m */
        } else if (row < nn + nm + ns) {
            int w = row < nn + nm ? 0 : 1;
            const surface *S = &p->s[w];
            int64_t i = row - nn - (w == 0 ? 0 : nm);
            double *Vr = malloc(sizeof(double) * S->nv), *Kr = malloc(sizeof(double) * S->nv);
            bem_row(p, S, i, Vr, Kr);
            const double *lam = x + nn + (w == 0 ? 0 : nm);
            double mass = 0.0;
            for (int32_t e = S->v2t_ptr[i]; e < S->v2t_ptr[i + 1]; ++e) {
                int64_t t = S->v2t[e];
                for (int b = 0; b < 3; ++b) {
                    int32_t j = S->tri[3 * t + b];
                    mass += S->area[t] * (j == i ? 2.0 : 1.0) / 12.0 * x[S->g[j]];
                }
            }
            s = 0.5 * mass;
            for (int64_t j = 0; j < S->nv; ++j) {
                double uj = x[S->g[j]];
                if (w == 0)
                    s += Kr[j] * uj - Vr[j] * lam[j];
                else
                    s += -Kr[j] * uj + Vr[j] * lam[j];
            }
            if (mode == 0 && w == 0) s -= fm[i];
            free(Vr);
            free(Kr);
        } else {
            err = -1;
        }
        out[r] = s;
    }
    free(fm);
    free(bu);
    return err;
}

int pbref_residual_rows(pbref *p, int scheme, const double *phi, int64_t nrows, const int64_t *rows, double *out)
{
    return coupled_rows(p, scheme, 0, phi, NULL, nrows, rows, out);
}

int pbref_jacobian_rows(pbref *p, int scheme, const double *phi, const double *v, int64_t nrows,
                        const int64_t *rows, double *out)
{
    return coupled_rows(p, scheme, 1, phi, v, nrows, rows, out);
}

/* ------------------------------------------------------------------------- */
/* GMRES (restarted, right-preconditioned by the block-diagonal of J)          */
/* ------------------------------------------------------------------------- */
static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void precond_diag(pbref *p, int scheme, const double *phi, double *dinv)
{
    int64_t nn = p->nn, nm = p->s[0].nv, ns = p->s[1].nv;
    fem_diag(p, scheme, phi, dinv);
    for (int64_t i = 0; i < nn; ++i) dinv[i] = 1.0 / dinv[i];
    for (int64_t i = 0; i < nm; ++i) dinv[nn + i] = 1.0 / (-p->s[0].V[i * nm + i]);
    for (int64_t i = 0; i < ns; ++i) dinv[nn + nm + i] = 1.0 / (p->s[1].V[i * ns + i]);
}

/* The paper leaves the GMRES preconditioner open.  Two right preconditioners:
 *
 * PBREF_PC_DIAG: the inverse of the diagonal of J.
 *
 * PBREF_PC_CHEB_SPAI: block diagonal.
 *   FEM block F = A + J_scheme(u): k terms of the Chebyshev iteration for
 *   F z = r started from z = 0 with Jacobi scaling D = diag(F) (Saad,
 *   Iterative Methods for Sparse Linear Systems, Chebyshev acceleration), on
 *   the interval [lmax / ratio, lmax] with lmax the Gershgorin bound
 *   max_i sum_j |F_ij| / F_ii of D^-1 F.  The k terms form a fixed polynomial
 *   in D^-1 F, so the preconditioner is one linear operator.
 *   Boundary blocks B (the single-layer blocks of the operator: -V0 on
 *   Gamma_m, +Vk on Gamma_s): a sparse approximate inverse M whose row i is
 *   supported on the vertex i and its triangle neighbours and minimises
 *   || m^T B - e_i^T ||_2 (normal equations, Cholesky). */

/* row i of the 1-ring pattern: i and every vertex sharing a triangle with it, ascending */
int64_t pbref_surface_ring(const pbref *p, int surf, int32_t *ptr, int32_t *col)
{
    const surface *S = &p->s[surf];
    int64_t nnz = 0;
    for (int64_t i = 0; i < S->nv; ++i) {
        int32_t lst[256];
        int m = 0;
        lst[m++] = (int32_t)i;
        for (int32_t e = S->v2t_ptr[i]; e < S->v2t_ptr[i + 1]; ++e) {
            int64_t t = S->v2t[e];
            for (int b = 0; b < 3; ++b) {
                int32_t j = S->tri[3 * t + b];
                int seen = 0;
                for (int k = 0; k < m; ++k) seen |= lst[k] == j;
                if (!seen && m < 256) lst[m++] = j;
            }
        }
        for (int a = 1; a < m; ++a) /* insertion sort */
            for (int b = a; b > 0 && lst[b - 1] > lst[b]; --b) {
                int32_t t = lst[b];
                lst[b] = lst[b - 1];
                lst[b - 1] = t;
            }
        if (ptr) ptr[i] = (int32_t)nnz;
        if (col) memcpy(col + nnz, lst, sizeof(int32_t) * m);
        nnz += m;
    }
    if (ptr) ptr[S->nv] = (int32_t)nnz;
    return nnz;
}

/* rows of the sparse approximate inverse of a dense n x n matrix B on the
 * given pattern; returns 0, or -1 if a Gram matrix is not positive definite */
int pbref_spai_rows(int64_t n, const double *B, const int32_t *ptr, const int32_t *col, double *val)
{
    int err = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : err)
    for (int64_t i = 0; i < n; ++i) {
        const int32_t *P = col + ptr[i];
        int m = ptr[i + 1] - ptr[i];
        double G[64][64], r[64];
        if (m > 64) {
            err |= 1;
            continue;
        }
        for (int a = 0; a < m; ++a) {
            r[a] = B[(int64_t)P[a] * n + i];
            for (int b = 0; b <= a; ++b) {
                double s = 0.0;
                for (int64_t c = 0; c < n; ++c) s += B[(int64_t)P[a] * n + c] * B[(int64_t)P[b] * n + c];
                G[a][b] = G[b][a] = s;
            }
        }
        /* Cholesky G = L L^T in place (lower triangle), then two triangular solves */
        for (int a = 0; a < m; ++a) {
            double d = G[a][a];
            for (int k = 0; k < a; ++k) d -= G[a][k] * G[a][k];
            if (!(d > 0.0)) {
                err |= 1;
                break;
            }
            G[a][a] = sqrt(d);
            for (int b = a + 1; b < m; ++b) {
                double s = G[b][a];
                for (int k = 0; k < a; ++k) s -= G[b][k] * G[a][k];
                G[b][a] = s / G[a][a];
            }
        }
        for (int a = 0; a < m; ++a) {
            double s = r[a];
            for (int k = 0; k < a; ++k) s -= G[a][k] * r[k];
            r[a] = s / G[a][a];
        }
        for (int a = m - 1; a >= 0; --a) {
            double s = r[a];
            for (int k = a + 1; k < m; ++k) s -= G[k][a] * r[k];
            r[a] = s / G[a][a];
        }
        for (int a = 0; a < m; ++a) val[ptr[i] + a] = r[a];
    }
    return err ? -1 : 0;
}

/* entries of row i of F = A + J_scheme(u), assembled from the tets at i */
/* distinct neighbours of node i (itself included) are at most 3 per tet + 1 */
static int64_t row_cap(const pbref *p, int64_t i) { return 3 * (int64_t)(p->n2t_ptr[i + 1] - p->n2t_ptr[i]) + 1; }

static int fem_row(const pbref *p, int scheme, const double *u, int64_t i, int32_t *cols, double *vals)
{
    const int64_t cap = row_cap(p, i);
    int m = 0;
    for (int32_t e = p->n2t_ptr[i]; e < p->n2t_ptr[i + 1]; ++e) {
        int64_t t = p->n2t[e];
        const int32_t *T = p->tet + 4 * t;
        int a = 0;
        while (T[a] != i) ++a;
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        const double c = tet_react(p, t);
        for (int b = 0; b < 4; ++b) {
            double s = tet_eps(p, t) * vol * vdot(G[a], G[b]);
            for (int q = 0; q < 27 && c != 0.0; ++q) {
                const double *l = p->tq_b + 4 * q;
                double uh = 0.0;
                for (int k = 0; k < 4; ++k) uh += l[k] * u[T[k]];
                s += c * vol * p->tq_w[q] * sch_d1(scheme, uh) * l[a] * l[b];
            }
            int k = 0;
            while (k < m && cols[k] != T[b]) ++k;
            if (k == m) {
                if (m == cap) return -1;
                cols[m] = T[b];
                vals[m++] = 0.0;
            }
            vals[k] += s;
        }
    }
    return m;
}

double pbref_fem_gershgorin(const pbref *p, int scheme, const double *u)
{
    double best = 0.0;
    int64_t mx = 1;
    for (int64_t i = 0; i < p->nn; ++i)
        if (row_cap(p, i) > mx) mx = row_cap(p, i);
    int32_t *cols = malloc(sizeof(int32_t) * mx);
    double *vals = malloc(sizeof(double) * mx);
    for (int64_t i = 0; i < p->nn; ++i) {
        double sum = 0.0, dg = 0.0;
        int m = fem_row(p, scheme, u, i, cols, vals);
        if (m < 0) {
            best = NAN;
            break;
        }
        for (int k = 0; k < m; ++k) {
            sum += fabs(vals[k]);
            if (cols[k] == i) dg = vals[k];
        }
        best = fmax(best, sum / dg);
    }
    free(cols);
    free(vals);
    return best;
}

typedef void (*lin_apply)(const void *ctx, const double *in, double *out);

/* k terms of the Jacobi-scaled Chebyshev iteration for F z = r, z0 = 0 */
static void cheb_terms(int64_t n, lin_apply F, const void *ctx, const double *dinv, double lmax, double ratio, int k,
                       const double *r, double *z)
{
    double lo = lmax / ratio, theta = 0.5 * (lmax + lo), delta = 0.5 * (lmax - lo);
    double sigma = theta / delta, rho = 1.0 / sigma;
    double *d = malloc(sizeof(double) * n), *res = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) {
        d[i] = dinv[i] * r[i] / theta;
        z[i] = 0.0;
    }
    for (int s = 0; s < k; ++s) {
        for (int64_t i = 0; i < n; ++i) z[i] += d[i];
        if (s == k - 1) break;
        F(ctx, z, res);
        double rho1 = 1.0 / (2.0 * sigma - rho);
        for (int64_t i = 0; i < n; ++i) d[i] = rho1 * rho * d[i] + 2.0 * rho1 / delta * dinv[i] * (r[i] - res[i]);
        rho = rho1;
    }
    free(d);
    free(res);
}

typedef struct {
    int64_t n;
    const double *f;
} diag_ctx;
static void diag_apply(const void *ctx, const double *in, double *out)
{
    const diag_ctx *c = ctx;
    for (int64_t i = 0; i < c->n; ++i) out[i] = c->f[i] * in[i];
}

/* the Chebyshev terms for a diagonal F (test hook: the residual polynomial
 * has a closed form there) */
void pbref_cheb_diag(int64_t n, const double *fdiag, const double *dinv, double lmax, double ratio, int k,
                     const double *r, double *z)
{
    diag_ctx c = {n, fdiag};
    cheb_terms(n, diag_apply, &c, dinv, lmax, ratio, k, r, z);
}

/* the FEM block F = A + J_scheme(u) as rows (assembled once per GMRES call) */
typedef struct {
    int64_t n;
    int32_t *ptr, *col;
    double *val;
} csr;
static int fem_block_csr(const pbref *p, int scheme, const double *u, csr *F)
{
    F->n = p->nn;
    F->ptr = malloc(sizeof(int32_t) * (p->nn + 1));
    F->col = malloc(sizeof(int32_t) * (12 * p->nt + p->nn));
    F->val = malloc(sizeof(double) * (12 * p->nt + p->nn));
    F->ptr[0] = 0;
    for (int64_t i = 0; i < p->nn; ++i) {
        int m = fem_row(p, scheme, u, i, F->col + F->ptr[i], F->val + F->ptr[i]);
        if (m < 0) return -1;
        F->ptr[i + 1] = F->ptr[i] + m;
    }
    return 0;
}
static void csr_apply(const void *ctx, const double *in, double *out)
{
    const csr *F = ctx;
    for (int64_t i = 0; i < F->n; ++i) {
        double s = 0.0;
        for (int32_t e = F->ptr[i]; e < F->ptr[i + 1]; ++e) s += F->val[e] * in[F->col[e]];
        out[i] = s;
    }
}

typedef struct {
    int mode, k;
    double ratio, lmax;
    double *dinv;
    csr F;
    int32_t *sp_ptr[2], *sp_col[2];
    double *sp_val[2];
} precond;

static int precond_build(pbref *p, int scheme, const double *phi, int mode, int k, double ratio, precond *P)
{
    memset(P, 0, sizeof *P);
    int64_t n = nunk(p);
    P->mode = mode;
    P->k = k;
    P->ratio = ratio;
    P->dinv = malloc(sizeof(double) * n);
    precond_diag(p, scheme, phi, P->dinv);
    if (mode == PBREF_PC_DIAG) return 0;
    P->lmax = pbref_fem_gershgorin(p, scheme, phi);
    if (!isfinite(P->lmax)) return -1;
    if (fem_block_csr(p, scheme, phi, &P->F)) return -1;
    for (int w = 0; w < 2; ++w) {
        const surface *S = &p->s[w];
        int64_t nnz = pbref_surface_ring(p, w, NULL, NULL);
        P->sp_ptr[w] = malloc(sizeof(int32_t) * (S->nv + 1));
        P->sp_col[w] = malloc(sizeof(int32_t) * nnz);
        P->sp_val[w] = malloc(sizeof(double) * nnz);
        pbref_surface_ring(p, w, P->sp_ptr[w], P->sp_col[w]);
        if (pbref_spai_rows(S->nv, S->V, P->sp_ptr[w], P->sp_col[w], P->sp_val[w])) return -1;
        if (w == 0) /* the Gamma_m block is -V0 */
            for (int64_t e = 0; e < nnz; ++e) P->sp_val[w][e] = -P->sp_val[w][e];
    }
    return 0;
}

static void precond_free(precond *P)
{
    free(P->dinv);
    free(P->F.ptr);
    free(P->F.col);
    free(P->F.val);
    for (int w = 0; w < 2; ++w) {
        free(P->sp_ptr[w]);
        free(P->sp_col[w]);
        free(P->sp_val[w]);
    }
}

/* z = P^-1 v */
static void precond_apply(pbref *p, const precond *P, const double *v, double *z)
{
    int64_t n = nunk(p), nn = p->nn;
    if (P->mode == PBREF_PC_DIAG) {
        for (int64_t i = 0; i < n; ++i) z[i] = P->dinv[i] * v[i];
        return;
    }
    cheb_terms(nn, csr_apply, &P->F, P->dinv, P->lmax, P->ratio, P->k, v, z);
    int64_t off = nn;
    for (int w = 0; w < 2; ++w) {
        const surface *S = &p->s[w];
        for (int64_t i = 0; i < S->nv; ++i) {
            double s = 0.0;
            for (int32_t e = P->sp_ptr[w][i]; e < P->sp_ptr[w][i + 1]; ++e) s += P->sp_val[w][e] * v[off + P->sp_col[w][e]];
            z[off + i] = s;
        }
        off += S->nv;
    }
}

/* Solve J_scheme(phi) x = b to ||b - J x|| <= tol ||b||, x0 = 0, right preconditioned. */
int pbref_gmres_pc(pbref *p, int scheme, const double *phi, const double *b, double *x, double tol, int restart,
                   int maxit, int pc, int cheb_degree, double cheb_ratio, int *iters)
{
    int r = need_dense(p);
    if (r) return r;
    int64_t n = nunk(p);
    int m = restart;
    precond P;
    if (precond_build(p, scheme, phi, pc, cheb_degree, cheb_ratio, &P)) {
        precond_free(&P);
        return -7;
    }
    double *Vb = malloc(sizeof(double) * n * (m + 1));
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m), *g = malloc(sizeof(double) * (m + 1));
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n), *res = malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    double bnorm = sqrt(dot(n, b, b));
    int total = 0, status = 0;
    *iters = 0;
    if (bnorm == 0.0) goto done;
    double target = tol * bnorm;
    for (;;) {
        /* true residual */
        pbref_apply_jacobian(p, scheme, phi, x, res);
        for (int64_t i = 0; i < n; ++i) res[i] = b[i] - res[i];
        double beta = sqrt(dot(n, res, res));
        if (!(beta == beta)) {
            status = -7;
            break;
        }
        if (beta <= target) break;
        if (total >= maxit) {
            status = -6;
            break;
        }
        for (int64_t i = 0; i < n; ++i) Vb[i] = res[i] / beta;
        memset(g, 0, sizeof(double) * (m + 1));
        g[0] = beta;
        int j = 0;
        for (; j < m && total < maxit;) {
            double *vj = Vb + (size_t)j * n, *vn = Vb + (size_t)(j + 1) * n;
            precond_apply(p, &P, vj, z);
            pbref_apply_jacobian(p, scheme, phi, z, w);
            ++total;
            for (int i = 0; i <= j; ++i) { /* modified Gram-Schmidt */
                double h = dot(n, w, Vb + (size_t)i * n);
                H[(size_t)i * m + j] = h;
                for (int64_t k = 0; k < n; ++k) w[k] -= h * Vb[(size_t)i * n + k];
            }
            double hn = sqrt(dot(n, w, w));
            H[(size_t)(j + 1) * m + j] = hn;
            for (int64_t k = 0; k < n; ++k) vn[k] = hn > 0 ? w[k] / hn : 0.0;
            for (int i = 0; i < j; ++i) { /* previous Givens rotations */
                double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
            double den = hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (fabs(g[j]) <= target || hn == 0.0) break;
        }
        /* back substitution, update x += P^{-1} V y */
        double *y = malloc(sizeof(double) * j);
        for (int i = j - 1; i >= 0; --i) {
            double s = g[i];
            for (int k = i + 1; k < j; ++k) s -= H[(size_t)i * m + k] * y[k];
            y[i] = s / H[(size_t)i * m + i];
        }
        memset(res, 0, sizeof(double) * n);
        for (int i = 0; i < j; ++i)
            for (int64_t k = 0; k < n; ++k) res[k] += y[i] * Vb[(size_t)i * n + k];
        precond_apply(p, &P, res, z);
        for (int64_t k = 0; k < n; ++k) x[k] += z[k];
        free(y);
    }
done:
    *iters = total;
    precond_free(&P);
    free(Vb);
    free(H);
    free(cs);
    free(sn);
    free(g);
    free(w);
    free(z);
    free(res);
    return status;
}

/* ------------------------------------------------------------------------- */
/* energy                                                                      */
/* ------------------------------------------------------------------------- */

/* u_r(x) = int_{Gamma_m} [g0(x,y) lam_m(y) - dg0/dn_y(x,y) u(y)] dy, the
 * reaction potential of the interior representation formula (eq.
 * Potential_in_Omega_m), with the regular triangle rule. */
int pbref_gmres(pbref *p, int scheme, const double *phi, const double *b, double *x, double tol, int restart,
                int maxit, int *iters)
{
    return pbref_gmres_pc(p, scheme, phi, b, x, tol, restart, maxit, PBREF_PC_DIAG, 1, 1.0, iters);
}

/* u_r(x) = (V lam)(x) - (K um)(x) over the surface S (eq.
 * Potential_in_Omega_m), with lam and um its per-vertex lam_m and trace */
static void reaction_potential_on(const pbref *p, const surface *S, const double *lam, const double *um,
                                  int64_t np, const double *pts, double *out)
{
#pragma omp parallel for
    for (int64_t k = 0; k < np; ++k) {
        double s = 0.0;
        for (int64_t t = 0; t < S->nt; ++t) {
            const int32_t *T = S->tri + 3 * t;
            for (int q = 0; q < p->nrq; ++q) {
                const double *l = p->rq_b + 3 * q;
                double y[3] = {0, 0, 0}, lh = 0.0, uh = 0.0;
                for (int a = 0; a < 3; ++a) {
                    for (int d = 0; d < 3; ++d) y[d] += l[a] * vx(p, S, T[a])[d];
                    lh += l[a] * lam[T[a]];
                    uh += l[a] * um[T[a]];
                }
                double g, dg;
                kernel_eval(0.0, pts + 3 * k, y, S->nrm + 3 * t, &g, &dg);
                s += S->area[t] * p->rq_w[q] * (g * lh - dg * uh);
            }
        }
        out[k] = s;
    }
}

int pbref_reaction_potential(const pbref *p, const double *phi, int64_t np, const double *pts, double *out)
{
    const surface *S = &p->s[0];
    double *um = malloc(sizeof(double) * (S->nv > 0 ? S->nv : 1));
    surface_trace(p, S, phi, um);
    reaction_potential_on(p, S, phi + p->nn, um, np, pts, out);
    free(um);
    return 0;
}

/* Solve A x = r for a dense n x n A (row-major, overwritten) by Gaussian
 * elimination with partial pivoting; r is overwritten by x. */
static int dense_solve(int64_t n, double *A, double *r)
{
    for (int64_t k = 0; k < n; ++k) {
        int64_t piv = k;
        for (int64_t i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > fabs(A[piv * n + k])) piv = i;
        if (A[piv * n + k] == 0.0) return -1;
        if (piv != k) {
            for (int64_t j = 0; j < n; ++j) {
                double t = A[k * n + j];
                A[k * n + j] = A[piv * n + j];
                A[piv * n + j] = t;
            }
            double t = r[k];
            r[k] = r[piv];
            r[piv] = t;
        }
#pragma omp parallel for
        for (int64_t i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            for (int64_t j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            r[i] -= f * r[k];
        }
    }
    for (int64_t k = n - 1; k >= 0; --k) {
        double s = r[k];
        for (int64_t j = k + 1; j < n; ++j) s -= A[k * n + j] * r[j];
        r[k] = s / A[k * n + k];
    }
    return 0;
}

/* Normal derivative on Gamma_m from the trace of u (Sec. 2.3.1, the limit
 * of the representation formula on Gamma_m): V0 lam_m = (1/2 M_m + K0_m) u_m
 * - f_m, with f_m the Coulomb load when with_load is set (the linear part
 * Phi_L carries the charges; the correction Phi_NL does not). */
int pbref_lambda_m(pbref *p, const double *u, int with_load, double *lam)
{
    const int w = gamma_m_index(p);
    int r = pbref_bem_dense(p, w);
    if (r) return r;
    const surface *S = &p->s[w];
    int64_t nm = S->nv;
    double *um = malloc(sizeof(double) * nm), *fm = malloc(sizeof(double) * nm);
    double *A = malloc(sizeof(double) * nm * nm);
    surface_trace(p, S, u, um);
    pbref_surface_mass_apply(p, w, um, lam);
    if (with_load) coulomb_load_on(p, S, fm);
    for (int64_t i = 0; i < nm; ++i) {
        double s = 0.5 * lam[i];
        for (int64_t j = 0; j < nm; ++j) s += S->K[i * nm + j] * um[j];
        lam[i] = s - (with_load ? fm[i] : 0.0);
    }
    for (int64_t i = 0; i < nm * nm; ++i) A[i] = S->V[i];
    r = dense_solve(nm, A, lam);
    free(um);
    free(fm);
    free(A);
    return r;
}

/* out = {Total, LC, NC, dG_Omega_i} in kcal/mol (eqs. Esolv, Esolv_Lineal):
 * LC, NC = 1/2 kT sum_k z_k u_r[Phi_L or Phi_NL](x_k);
 * dG = kT/(4 pi l_B) * 1/2 eps_s kappa^2 int (u sinh u - 2 cosh u + 2). */
int pbref_energy(pbref *p, const double *phi_lin, const double *phi_nl, double out[4])
{
    /* the reaction potential from lam_m and the trace of u on Gamma_m; in the
     * two-field form lam_m is recovered from the trace for each part first
     * (Sec. 2.3.1), on the independent Gamma_m mesh when one is set */
    const int w = p->two_field ? gamma_m_index(p) : 0;
    const surface *S = &p->s[w];
    const int64_t nm = S->nv > 0 ? S->nv : 1;
    double *lam = malloc(sizeof(double) * nm), *um = malloc(sizeof(double) * nm);
    double *ur = malloc(sizeof(double) * (p->nq > 0 ? p->nq : 1));
    double lc = 0.0, nc = 0.0;
    for (int part = 0; part < 2; ++part) {
        const double *phi = part == 0 ? phi_lin : phi_nl;
        if (!phi) continue;
        if (p->two_field) {
            int r = pbref_lambda_m(p, phi, part == 0, lam);
            if (r) {
                free(lam);
                free(um);
                free(ur);
                return r;
            }
        } else {
            memcpy(lam, phi + p->nn, sizeof(double) * S->nv);
        }
        surface_trace(p, S, phi, um);
        reaction_potential_on(p, S, lam, um, p->nq, p->qx, ur);
        double e = 0.0;
        for (int64_t k = 0; k < p->nq; ++k) e += 0.5 * p->kT * p->qz[k] * ur[k];
        if (part == 0) lc = e;
        else nc = e;
    }
    double integral = 0.0;
    for (int64_t t = 0; t < p->nt_i; ++t) { /* Omega_i only */
        double G[4][3], vol;
        tet_geom(p, t, G, &vol);
        const int32_t *T = p->tet + 4 * t;
        for (int q = 0; q < 27; ++q) {
            const double *l = p->tq_b + 4 * q;
            double uh = 0.0;
            for (int a = 0; a < 4; ++a) uh += l[a] * (phi_lin[T[a]] + (phi_nl ? phi_nl[T[a]] : 0.0));
            integral += vol * p->tq_w[q] * (uh * sinh(uh) - 2.0 * cosh(uh) + 2.0);
        }
    }
    double dg = phi_nl ? p->kT / (4.0 * PI * p->lB) * 0.5 * p->eps_s * p->kappa * p->kappa * integral : 0.0;
    out[0] = lc + nc + dg;
    out[1] = lc;
    out[2] = nc;
    out[3] = dg;
    free(ur);
    free(lam);
    free(um);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Newton-Raphson with self-adjusted relaxation (Sec. 2.4-2.5, App. A, App. B) */
/* ------------------------------------------------------------------------- */
void pbref_opts_default(pbref_opts *o)
{
    o->scheme_first = PBREF_T3;
    o->omega_auto = 1;
    o->omega_fixed = 1.0;
    o->tol_nl = 1e-3;
    o->tol_gr = 1e-6;
    o->tol_gr0 = 1e-3;
    o->tol_omega = 0.1;
    o->l_e = 0.35;
    o->omega0_first = 2.0;
    o->omega0_next = 1.0;
    o->omega_min = 0.0;
    o->omega_max = 4.0;
    o->max_newton = 50;
    o->max_omega_it = 50;
    o->gmres_restart = 200;
    o->max_gmres = 2000;
    o->precond = PBREF_PC_CHEB_SPAI;
    o->cheb_degree = 24;
    o->cheb_ratio = 200.0;
    o->omega_method = PBREF_OMEGA_NEWTON;
    o->nonlinear_method = PBREF_NEWTON;
    o->r_e = 1.4;
    o->n_schedule = 0;
    for (int k = 0; k < 8; ++k) o->schedule[k] = PBREF_HS;
}

static int all_finite(int64_t n, const double *x)
{
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* f_d and its derivative (eq. fd=0 and App. A) for the Newton step Delta at
 * Phi, with c = b - A Phi and p = -A Delta:
 *   r(w)  = c - [N(u + w Delta_u); 0; 0]
 *   r'(w) = -[J(u + w Delta_u) Delta_u; 0; 0]
 *   r''(w)= -[H(u + w Delta_u)[Delta_u]; 0; 0]
 *   f_d   = -((p + r').r) / ((p + r').p) - w
 *   f_d'  = -((p + r').r' + r.r'') / beta + ((p + r').r)(p.r'') / beta^2 - 1
 * Returns 1 when the denominator beta vanishes. */
static int fd_eval(const pbref *p, int s, const double *phi, const double *c, const double *D, const double *pv,
                   double omega, double *fd, double *dfd, double *work)
{
    int64_t n = nunk(p), nn = p->nn;
    double *uw = work, *tmp = work + nn, *rv = work + 2 * nn, *r1 = rv + n, *r2 = r1 + n;
    for (int64_t i = 0; i < nn; ++i) uw[i] = phi[i] + omega * D[i];
    memcpy(rv, c, sizeof(double) * n);
    memset(r1, 0, sizeof(double) * n);
    memset(r2, 0, sizeof(double) * n);
    pbref_fem_nonlinear(p, s, uw, tmp);
    for (int64_t i = 0; i < nn; ++i) rv[i] -= tmp[i];
    pbref_fem_jacobian(p, s, uw, D, tmp);
    for (int64_t i = 0; i < nn; ++i) r1[i] = -tmp[i];
    pbref_fem_hessian(p, s, uw, D, tmp);
    for (int64_t i = 0; i < nn; ++i) r2[i] = -tmp[i];
    double pr = dot(n, pv, rv), r1r = dot(n, r1, rv), pp = dot(n, pv, pv), r1p = dot(n, r1, pv);
    double r1r1 = dot(n, r1, r1), rr2 = dot(n, rv, r2), pr2 = dot(n, pv, r2);
    double a = pr + r1r, beta = pp + r1p;
    if (beta == 0.0) return 1;
    *fd = -a / beta - omega;
    *dfd = -(r1p + r1r1 + rr2) / beta + a * pr2 / (beta * beta) - 1.0;
    return 0;
}

/* ---- one-dimensional root finders of f_d -------------------------------- */
static double clamp_omega(double w, const pbref_opts *o)
{
    if (w < o->omega_min) w = o->omega_min;
    if (w > o->omega_max) w = o->omega_max;
    return w;
}

/* Newton-Raphson on f_d from w (iterates clamped); stops at |f_d| < tol */
static double root_newton(pbref_fd_fn f, void *ctx, double w, const pbref_opts *o, int *ev, int *fb)
{
    for (int j = 0; *ev < o->max_omega_it; ++j) {
        double fd, dfd;
        ++*ev;
        if (f(ctx, w, &fd, &dfd)) {
            *fb = 1;
            return 1.0;
        }
        if (fabs(fd) < o->tol_omega) return w;
        if (dfd == 0.0 || !isfinite(dfd)) {
            *fb = 1;
            return 1.0;
        }
        w = clamp_omega(w - fd / dfd, o);
    }
    return w;
}

/* secant on f_d from the pair (w0, w1); stops at |f_d| < tol */
static double root_secant(pbref_fd_fn f, void *ctx, double w0, double w1, const pbref_opts *o, int *ev, int *fb)
{
    double f0, f1, d;
    ++*ev;
    if (f(ctx, w0, &f0, &d)) {
        *fb = 1;
        return 1.0;
    }
    if (fabs(f0) < o->tol_omega) return w0;
    ++*ev;
    if (f(ctx, w1, &f1, &d)) {
        *fb = 1;
        return 1.0;
    }
    while (fabs(f1) >= o->tol_omega && *ev < o->max_omega_it) {
        const double den = f0 - f1;
        if (den == 0.0 || !isfinite(den)) {
            *fb = 1;
            return 1.0;
        }
        const double w2 = clamp_omega(w0 - (w0 - w1) * f0 / den, o);
        w0 = w1;
        f0 = f1;
        w1 = w2;
        ++*ev;
        if (f(ctx, w1, &f1, &d)) {
            *fb = 1;
            return 1.0;
        }
    }
    return w1;
}

/* bisection of [lo, hi]; without a sign change of f_d over it the search
 * continues with Newton from w_start */
static double root_bisect(pbref_fd_fn f, void *ctx, double lo, double hi, double w_start, const pbref_opts *o,
                          int *ev, int *fb)
{
    double flo, fhi, fm, d;
    ++*ev;
    if (f(ctx, lo, &flo, &d)) {
        *fb = 1;
        return 1.0;
    }
    if (fabs(flo) < o->tol_omega) return lo;
    ++*ev;
    if (f(ctx, hi, &fhi, &d)) {
        *fb = 1;
        return 1.0;
    }
    if (fabs(fhi) < o->tol_omega) return hi;
    if ((flo > 0.0) == (fhi > 0.0)) return root_newton(f, ctx, w_start, o, ev, fb);
    double mid = 0.5 * (lo + hi);
    while (*ev < o->max_omega_it) {
        mid = 0.5 * (lo + hi);
        ++*ev;
        if (f(ctx, mid, &fm, &d)) {
            *fb = 1;
            return 1.0;
        }
        if (fabs(fm) < o->tol_omega) return mid;
        if ((fm > 0.0) == (flo > 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return mid;
}

/* start value of the first-iteration Newton search: three bisection
 * midpoints of [2, 3] (f_d decreases through its root: a positive value
 * moves the search up), then secant steps from the last two until two
 * successive iterates differ by less than 0.05 */
static double guess_bisect_secant(pbref_fd_fn f, void *ctx, const pbref_opts *o, int *ev, int *fb)
{
    double lo = 2.0, hi = 3.0, w[3], fv[3], d;
    for (int i = 0; i < 3; ++i) {
        w[i] = 0.5 * (lo + hi);
        ++*ev;
        if (f(ctx, w[i], &fv[i], &d)) {
            *fb = 1;
            return 1.0;
        }
        if (fv[i] > 0.0) lo = w[i];
        else hi = w[i];
    }
    double w0 = w[1], f0 = fv[1], w1 = w[2], f1 = fv[2];
    while (*ev < o->max_omega_it) {
        const double den = f0 - f1;
        if (den == 0.0 || !isfinite(den)) break;
        const double w2 = clamp_omega(w0 - (w0 - w1) * f0 / den, o);
        if (fabs(w2 - w1) < 0.05) return w2;
        w0 = w1;
        f0 = f1;
        w1 = w2;
        ++*ev;
        if (f(ctx, w1, &f1, &d)) {
            *fb = 1;
            return 1.0;
        }
    }
    return w1;
}

double pbref_root_find(int method, int k, double omega0, pbref_fd_fn f, void *ctx, const pbref_opts *o,
                       int *evals, int *fallback)
{
    *evals = 0;
    *fallback = 0;
    switch (method) {
    case PBREF_OMEGA_BISECT: return root_bisect(f, ctx, o->omega_min, o->omega_max, omega0, o, evals, fallback);
    case PBREF_OMEGA_SECANT: return root_secant(f, ctx, omega0, omega0 + 0.125, o, evals, fallback);
    case PBREF_OMEGA_BSEC:
        if (k == 1) return root_bisect(f, ctx, o->omega_min, o->omega_max, omega0, o, evals, fallback);
        return root_secant(f, ctx, omega0, omega0 + 0.125, o, evals, fallback);
    case PBREF_OMEGA_NEWTON_BS:
        if (k == 1) {
            const double w = guess_bisect_secant(f, ctx, o, evals, fallback);
            if (*fallback) return w;
            return root_newton(f, ctx, w, o, evals, fallback);
        }
        return root_newton(f, ctx, omega0, o, evals, fallback);
    case PBREF_OMEGA_BSEC_DF:
        if (k == 1) return root_bisect(f, ctx, o->omega_min, o->omega_max, omega0, o, evals, fallback);
        {
            const double w0 = 0.125;
            double f0, d;
            ++*evals;
            if (f(ctx, w0, &f0, &d) || f0 == 1.0 || !isfinite(f0)) {
                *fallback = 1;
                return 1.0;
            }
            return clamp_omega(w0 / (1.0 - f0), o);
        }
    default: return root_newton(f, ctx, omega0, o, evals, fallback);
    }
}

struct fd_ctx {
    pbref *p;
    int s;
    const double *phi, *c, *D, *pv;
    double *work;
};

static int fd_cb(void *vc, double w, double *fd, double *dfd)
{
    struct fd_ctx *x = vc;
    return fd_eval(x->p, x->s, x->phi, x->c, x->D, x->pv, w, fd, dfd, x->work);
}

/* root of f_d for the step D at phi with the method of o, from *omega_io;
 * *iters = f_d evaluations after the first (the Newton updates, for NEWTON) */
static void omega_search(pbref *p, int s, int k, const double *phi, const double *c, const double *D,
                         const pbref_opts *o, double *omega_io, int *iters, int *fallback)
{
    int64_t n = nunk(p), nn = p->nn;
    double *pv = malloc(sizeof(double) * n);
    double *work = malloc(sizeof(double) * (2 * nn + 3 * n));
    pbref_apply_A(p, D, pv);
    for (int64_t i = 0; i < n; ++i) pv[i] = -pv[i];
    struct fd_ctx x = {p, s, phi, c, D, pv, work};
    int ev = 0;
    *omega_io = pbref_root_find(o->omega_method, k, *omega_io, fd_cb, &x, o, &ev, fallback);
    *iters = ev > 0 ? ev - 1 : 0;
    free(pv);
    free(work);
}

int pbref_fd(pbref *p, int scheme, const double *phi, const double *D, double omega, double out[2])
{
    int r = need_dense(p);
    if (r) return r;
    int64_t n = nunk(p), nn = p->nn;
    double *b = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n), *pv = malloc(sizeof(double) * n);
    double *work = malloc(sizeof(double) * (2 * nn + 3 * n));
    pbref_rhs(p, b);
    pbref_apply_A(p, phi, c);
    for (int64_t i = 0; i < n; ++i) c[i] = b[i] - c[i];
    pbref_apply_A(p, D, pv);
    for (int64_t i = 0; i < n; ++i) pv[i] = -pv[i];
    int st = fd_eval(p, scheme, phi, c, D, pv, omega, &out[0], &out[1], work);
    free(b);
    free(c);
    free(pv);
    free(work);
    return st;
}

int pbref_omega_search(pbref *p, int scheme, const double *phi, const double *D, const pbref_opts *o,
                       double *omega, int *iters)
{
    int r = need_dense(p);
    if (r) return r;
    int64_t n = nunk(p);
    double *b = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    pbref_rhs(p, b);
    pbref_apply_A(p, phi, c);
    for (int64_t i = 0; i < n; ++i) c[i] = b[i] - c[i];
    int fb = 0;
    omega_search(p, scheme, 1, phi, c, D, o, omega, iters, &fb);
    free(b);
    free(c);
    return fb;
}

int pbref_solve(pbref *p, const pbref_opts *o, pbref_result *res, double *phi_lin, double *phi_nl)
{
    memset(res, 0, sizeof *res);
    int r = need_dense(p);
    if (r) return r;
    int64_t n = nunk(p), nn = p->nn;
    double *b = malloc(sizeof(double) * n), *phi = malloc(sizeof(double) * n), *c = malloc(sizeof(double) * n);
    double *d = malloc(sizeof(double) * n), *D = malloc(sizeof(double) * n);
    double *tmp = malloc(sizeof(double) * nn);
    pbref_rhs(p, b);
    /* 1. linear component: (A + eps_s kappa^2 M) Phi_L = b */
    double tol = o->tol_gr0;
    int it;
    int st = pbref_gmres_pc(p, PBREF_LIN, b /*u: unused for LIN*/, b, phi_lin, tol, o->gmres_restart, o->max_gmres,
                            o->precond, o->cheb_degree, o->cheb_ratio, &it);
    res->gmres_lin = it;
    res->gmres_iters_total = it;
    memset(phi_nl, 0, sizeof(double) * n);
    int frozen = 0, status = st;
    double omega_last = 1.0, e_km1 = 0.0, e_km2 = 0.0; /* e of the two previous steps */
    int k;
    for (k = 1; k <= o->max_newton && status == 0; ++k) {
        int s;
        if (o->n_schedule > 0) s = k <= o->n_schedule ? o->schedule[k - 1] : PBREF_HS;
        else s = (k == 1 && o->scheme_first == PBREF_T3) ? PBREF_T3 : PBREF_HS;
        for (int64_t i = 0; i < n; ++i) phi[i] = phi_lin[i] + phi_nl[i];
        /* c = b - A Phi ; d = c - N_s(u) */
        pbref_apply_A(p, phi, c);
        for (int64_t i = 0; i < n; ++i) c[i] = b[i] - c[i];
        pbref_fem_nonlinear(p, s, phi, tmp);
        memcpy(d, c, sizeof(double) * n);
        for (int64_t i = 0; i < nn; ++i) d[i] -= tmp[i];
        if (!all_finite(n, d)) {
            status = -7;
            break;
        }
        /* Newton: J_s(Phi) Delta = d (eq. NR_main); Picard: A Delta = d, Delta =
         * the intermediate estimate minus Phi_NL (eq. Ec_NL_Previo2) */
        const int lin = o->nonlinear_method == PBREF_PICARD ? PBREF_NONE : s;
        st = pbref_gmres_pc(p, lin, phi, d, D, tol, o->gmres_restart, o->max_gmres, o->precond, o->cheb_degree,
                            o->cheb_ratio, &it);
        int idx = k - 1 < 64 ? k - 1 : 63;
        res->gmres_iters[idx] = it;
        res->gmres_iters_total += it;
        if (st) {
            status = st;
            break;
        }
        double omega;
        int oit = 0;
        if (!o->omega_auto) {
            omega = o->omega_fixed;
        } else if (frozen) {
            omega = omega_last;
        } else if (o->nonlinear_method == PBREF_PICARD && o->r_e > 0 && k >= 3 && e_km2 >= o->r_e * e_km1) {
            omega = omega_last; /* e_{k-2} / e_{k-1} >= R_e: converging fast enough, reuse */
        } else {
            omega = (s == PBREF_T3) ? o->omega0_first : o->omega0_next;
            int fb = 0;
            omega_search(p, s, k, phi, c, D, o, &omega, &oit, &fb);
            res->omega_fallback += fb;
            omega_last = omega;
        }
        for (int64_t i = 0; i < n; ++i) phi_nl[i] += omega * D[i];
        double ek = omega * sqrt(dot(n, D, D));
        res->omega[idx] = omega;
        res->e_k[idx] = ek;
        res->omega_iters[idx] = oit;
        e_km2 = e_km1;
        e_km1 = ek;
        if (!isfinite(ek)) {
            status = -7;
            break;
        }
        if (o->l_e > 0 && ek < o->l_e) frozen = 1;
        if (o->tol_gr0 > o->tol_gr && ek < 1250.0 * tol) tol = fmax(o->tol_gr, 0.1 * tol);
        if (ek < o->tol_nl && s == PBREF_HS) { /* a Taylor step solves another equation */
            ++k;
            break;
        }
        if (k == o->max_newton) status = -6;
    }
    res->newton_iters = k - 1;
    res->status = status;
    double en[4];
    pbref_energy(p, phi_lin, phi_nl, en);
    res->total = en[0];
    res->lc = en[1];
    res->nc = en[2];
    res->dg_omega_i = en[3];
    free(b);
    free(phi);
    free(c);
    free(d);
    free(D);
    free(tmp);
    return status;
}
