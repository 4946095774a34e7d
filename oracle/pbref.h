/* pbref -- plain FP64 CPU oracle for the three-region FEM-BEM nonlinear
 * Poisson-Boltzmann problem (and its two-field form, pbref_set_two_field).  TEST INFRASTRUCTURE ONLY: it exists to check the
 * HIP library, it is slow on purpose, and no product code may link or call it.
 *
 * Unknowns: Phi = [u (FEM nodes) | lambda_m (Gamma_m vertices) | lambda_s
 * (Gamma_s vertices)], surface vertices numbered by ascending FEM node id.
 *
 * Coupled system (Sec. 2, eq. fembem_matrix, rewritten for FEM in the shell
 * only, with the interior Laplace BIE of Sec. 2.3 as the Gamma_m row):
 *   A u + N(u) + eps_m T_m^T M_m lam_m - eps_s T_s^T M_s lam_s = 0
 *   (1/2 M_m + K0_m) T_m u - V0_m lam_m                        = f_m
 *   (1/2 M_s - Kk_s) T_s u + Vk_s lam_s                        = 0
 */
#ifndef PBREF_H
#define PBREF_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbref pbref;

/* reaction term N(t): LIN t, T3 / T5 / T7 the sinh series through t^3/3!,
 * t^5/5!, t^7/7! (the schemes of Sec. 3.3.1), HS sinh t */
enum { PBREF_LIN = 0, PBREF_T3 = 1, PBREF_HS = 2, PBREF_T5 = 3, PBREF_T7 = 4 };
/* no reaction term (N = J = H = 0): the linear operator A of the Picard step */
enum { PBREF_NONE = 7 };

/* quadrature rules (weights normalised to sum 1 over the reference cell) */
int pbref_rule_tri6(double *bary /*6x3*/, double *w /*6*/);
int pbref_rule_tet27(double *bary /*27x4*/, double *w /*27*/);
int pbref_rule_gauss01(int n, double *x, double *w);
int pbref_rule_tri_collapsed(int m, double *bary /*m*m x 3*/, double *w);

/* reg_order: 0 = 6-point degree-4 triangle rule, m>0 = m x m collapsed Gauss
 * rule; n_ss: Gauss points per direction of the Sauter-Schwab rules. */
pbref *pbref_create(int64_t n_nodes, const double *nodes, int64_t n_tets, const int32_t *tets,
                    int64_t n_tri_m, const int32_t *tri_m, int64_t n_tri_s, const int32_t *tri_s,
                    int64_t n_q, const double *q_xyz, const double *q_z,
                    double eps_in, double eps_out, double kappa, double temperature,
                    int reg_order, int n_ss);
void pbref_destroy(pbref *);
void pbref_sizes(const pbref *, int64_t out[4]); /* n_nodes, n_m, n_s, n_unknowns */
void pbref_constants(const pbref *, double out[2]); /* Bjerrum length (A), kT (kcal/mol) */
void pbref_surface_nodes(const pbref *, int surf, int32_t *out);

/* surface operators; surf 0 = Gamma_m (Laplace), 1 = Gamma_s (Yukawa) */
int pbref_bem_dense(pbref *, int surf);                           /* assemble and keep */
int pbref_bem_get(const pbref *, int surf, double *V, double *K);  /* copy dense N x N */
int pbref_bem_rows(pbref *, int surf, int64_t nrows, const int64_t *rows, double *V, double *K);
int pbref_pair_integral(pbref *, int surf, int64_t tau, int64_t sig, double *V9, double *K9);
void pbref_surface_mass_apply(const pbref *, int surf, const double *x, double *y);
void pbref_coulomb_load(const pbref *, double *f);

/* FEM pieces: element entries (16 per tet) and matrix-free products on u */
void pbref_stiffness_entries(const pbref *, int32_t *rows, int32_t *cols, double *vals);
void pbref_mass_entries(const pbref *, int32_t *rows, int32_t *cols, double *vals);
void pbref_fem_nonlinear(const pbref *, int scheme, const double *u, double *out);
void pbref_fem_jacobian(const pbref *, int scheme, const double *u, const double *v, double *out);
void pbref_fem_hessian(const pbref *, int scheme, const double *u, const double *v, double *out);

/* coupled operator (needs the dense surface operators of both surfaces) */
int pbref_apply_A(pbref *, const double *phi, double *y);
int pbref_dense_rows_apply(const pbref *, int surf, int64_t nrows, const double *V, const double *K,
                           const double *x, double *out);
int pbref_rhs(pbref *, double *b);
/* Two-field form (Sec. 2.3, eq. fembem_matrix): the last n_tets_m tets fill
 * the solute (eps_m, no reaction term), the load is the point charges in the
 * FEM rows, the FEM rows lose their lam_m term and the lam_m rows become the
 * identity (lam_m is recovered after the solve by pbref_lambda_m, and
 * pbref_energy does so itself).  Returns -1 unless 0 < n_tets_m < n_tets. */
int pbref_set_two_field(pbref *, int64_t n_tets_m);
/* Two-field form: a Gamma_m surface mesh independent of the volume mesh
 * (own vertices verts[3 nv], triangles tri[3 nt] oriented like the
 * interface).  lam_m and the reaction potential then live on it, and the
 * trace of u on it is the P1 interpolant of u at its vertices, each vertex
 * in the tet holding it (Sec. 2.3.1: the trace by interpolation between the
 * volume and surface meshes).  nv = 0 removes it.  -1 for bad sizes or ids,
 * -3 if a vertex lies outside the FEM mesh. */
int pbref_set_reaction_surface(pbref *, int64_t nv, const double *verts, int64_t nt, const int32_t *tri);
/* vertices of the surface that carries lam_m and the reaction potential
 * (the independent mesh in the two-field form when set, else Gamma_m) */
int64_t pbref_gamma_m_vertices(const pbref *);
/* the trace of the FEM field u on that surface (pbref_gamma_m_vertices values) */
int pbref_gamma_m_trace(const pbref *, const double *u, double *out);
/* lam = V0^-1 ((1/2 M_m + K0_m) u|Gamma_m - [with_load] f_m) (Sec. 2.3.1), on
 * that surface (pbref_gamma_m_vertices values) */
int pbref_lambda_m(pbref *, const double *u, int with_load, double *lam);
/* add a fixed vector to b in pbref_rhs, pbref_residual and pbref_solve (NULL clears);
 * used to impose the volume source and interface jumps of manufactured solutions */
void pbref_set_rhs_extra(pbref *, const double *e);
int pbref_residual(pbref *, int scheme, const double *phi, double *F);
int pbref_apply_jacobian(pbref *, int scheme, const double *phi, const double *v, double *Jv);
/* selected rows of F or J v without dense assembly; rows are global unknown ids */
int pbref_residual_rows(pbref *, int scheme, const double *phi, int64_t nrows, const int64_t *rows, double *out);
int pbref_jacobian_rows(pbref *, int scheme, const double *phi, const double *v, int64_t nrows,
                        const int64_t *rows, double *out);

typedef struct {
    int scheme_first, omega_auto;
    double omega_fixed, tol_nl, tol_gr, tol_gr0, tol_omega, l_e, omega0_first, omega0_next,
        omega_min, omega_max;
    int max_newton, max_omega_it, gmres_restart, max_gmres;
    int precond, cheb_degree; /* PBREF_PC_*, Chebyshev terms of the FEM block */
    double cheb_ratio;        /* lmax / lower end of the Chebyshev interval */
    int omega_method;         /* PBREF_OMEGA_*: root finder of f_d */
    int nonlinear_method;     /* PBREF_NEWTON or PBREF_PICARD (Sec. 2.4.2) */
    double r_e;               /* Picard: the relaxation factor is searched again only when
                               * e_{k-2} / e_{k-1} < r_e (0: at every step) */
    int n_schedule;           /* > 0: iteration k <= n_schedule uses schedule[k-1], later ones HS
                               * (T3-T5-HS and the like, Sec. 3.3.1); 0: the scheme_first rule */
    int schedule[8];
} pbref_opts;

enum { PBREF_NEWTON = 0, PBREF_PICARD = 1 };

/* Root finders of f_d(omega) = 0 (Sec. 2.5 and the appendix on one-dimensional
 * root finding; the comparison of Sec. 4 and the first-iteration guess of the
 * appendix on other optimisations):
 *   NEWTON   Newton-Raphson from omega0 (omega0_first in a T3 iteration, else omega0_next)
 *   BISECT   bisection of [omega_min, omega_max]
 *   SECANT   secant from omega0 and omega0 + 1/8
 *   BSEC     bisection in the first nonlinear iteration, secant afterwards
 *   NEWTON_BS  Newton whose first-iteration start comes from three bisection
 *            midpoints in [2, 3] followed by secant steps until two iterates
 *            differ by less than 0.05
 *   BSEC_DF  bisection in the first nonlinear iteration, afterwards the
 *            direct secant formula from omega = 0 (where f_d = 1 in a Picard
 *            step) and omega = 1/8: omega0 / (1 - f_d(omega0)), one evaluation */
enum { PBREF_OMEGA_NEWTON = 0, PBREF_OMEGA_BISECT = 1, PBREF_OMEGA_SECANT = 2, PBREF_OMEGA_BSEC = 3,
       PBREF_OMEGA_NEWTON_BS = 4, PBREF_OMEGA_BSEC_DF = 5 };
/* f(ctx, omega, &f_d, &f_d') returns nonzero when f_d is undefined (beta = 0) */
typedef int (*pbref_fd_fn)(void *ctx, double omega, double *fd, double *dfd);
/* One root search with a caller-supplied f_d: method, nonlinear iteration k
 * (1-based) and the start value omega0; returns omega; *evals = number of f_d
 * evaluations; *fallback = 1 when the search fell back to omega = 1. */
double pbref_root_find(int method, int k, double omega0, pbref_fd_fn f, void *ctx, const pbref_opts *o,
                       int *evals, int *fallback);

enum { PBREF_PC_DIAG = 0, PBREF_PC_CHEB_SPAI = 1 };

typedef struct {
    int status; /* 0 ok, -6 not converged, -7 non-finite */
    double total, lc, nc, dg_omega_i;
    int newton_iters, gmres_iters_total, gmres_lin;
    int gmres_iters[64];
    double omega[64], e_k[64];
    int omega_iters[64];
    int omega_fallback;
} pbref_result;

void pbref_opts_default(pbref_opts *);
int pbref_gmres(pbref *, int scheme, const double *phi, const double *b, double *x, double tol,
                int restart, int maxit, int *iters);
int pbref_gmres_pc(pbref *, int scheme, const double *phi, const double *b, double *x, double tol,
                   int restart, int maxit, int pc, int cheb_degree, double cheb_ratio, int *iters);
/* preconditioner pieces: 1-ring pattern (returns nnz; ptr/col may be NULL),
 * sparse approximate inverse rows of a dense n x n matrix on a pattern,
 * Gershgorin bound of diag(F)^-1 F for the FEM block, and the Chebyshev
 * terms for a diagonal F */
int64_t pbref_surface_ring(const pbref *, int surf, int32_t *ptr, int32_t *col);
int pbref_spai_rows(int64_t n, const double *B, const int32_t *ptr, const int32_t *col, double *val);
double pbref_fem_gershgorin(const pbref *, int scheme, const double *u);
void pbref_cheb_diag(int64_t n, const double *fdiag, const double *dinv, double lmax, double ratio, int k,
                     const double *r, double *z);
int pbref_solve(pbref *, const pbref_opts *, pbref_result *, double *phi_lin, double *phi_nl);
/* f_d(omega) and f_d'(omega) for the step D at phi (out[0], out[1]) */
int pbref_fd(pbref *, int scheme, const double *phi, const double *D, double omega, double out[2]);
/* Newton search for the root of f_d starting at *omega; returns 1 on fallback */
int pbref_omega_search(pbref *, int scheme, const double *phi, const double *D, const pbref_opts *o,
                       double *omega, int *iters);
/* energy pieces from given Phi_L and Phi_NL (kcal/mol) */
int pbref_energy(pbref *, const double *phi_lin, const double *phi_nl, double out[4]);
/* reaction potential u_r at arbitrary points from a given Phi (units of kT/e) */
int pbref_reaction_potential(const pbref *, const double *phi, int64_t np, const double *pts, double *out);

#ifdef __cplusplus
}
#endif
#endif
