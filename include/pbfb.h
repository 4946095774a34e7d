/* pbfb.h -- C ABI of the MI355X FEM-BEM nonlinear Poisson-Boltzmann library.
 *
 * Problem (paper Sec. 2.1, eqs. EcGeneral_PBE, Variables_2Superficie, pbe_vp):
 * three regions -- solute Omega_m (eps_in, point charges), shell Omega_i
 * (eps_out, screening kappa, nonlinear sinh term) and far solvent Omega_s
 * (eps_out, kappa, linear) -- separated by the triangulated interfaces
 * Gamma_m and Gamma_s.  The shell is discretised with P1 tetrahedra; the
 * interior uses the Laplace boundary integral equation of Sec. 2.3 and the
 * exterior the Yukawa boundary integral equation of Sec. 2.2, both as dense
 * Galerkin P1 operators.  Unknowns Phi = [u | lambda_m | lambda_s] (FEM nodal
 * potential in units of kT/e, normal derivatives on Gamma_m and Gamma_s):
 *
 *   A u + N(u) + eps_in T_m^T M_m lambda_m - eps_out T_s^T M_s lambda_s = 0
 *   (1/2 M_m + K_m) T_m u - V_m lambda_m                                = f_m
 *   (1/2 M_s - K_s) T_s u + V_s lambda_s                                = 0
 *
 * (the 2x2 block system of eq. fembem_matrix, extended by the interior
 * Laplace equation as a third block row), with N(u) = eps_out kappa^2
 * int sinh(u_h) v.  Newton-Raphson with a cubic first step and a
 * self-adjusted relaxation factor solves it (Sec. 2.4-2.5, App. A, App. B).
 *
 * Conventions for every entry point:
 *  - return value: pbfb_status, 0 = success, negative = error; the message of
 *    the last failing call on this thread is returned by pbfb_last_error();
 *  - array arguments are borrowed for the duration of the call and copied;
 *    the caller keeps ownership; outputs are written into caller buffers;
 *  - `mem` says where vector arguments live: PBFB_MEM_HOST (pageable host
 *    memory) or PBFB_MEM_DEVICE (device memory of the context's GPU);
 *  - `hip_stream` is a hipStream_t (NULL = the library's own stream); device
 *    outputs are complete when the stream reaches the end of the call; host
 *    outputs are complete when the call returns;
 *  - a pbfb_problem is not thread-safe: serialise calls per handle.
 */
#ifndef PBFB_H
#define PBFB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pbfb_ctx pbfb_ctx;
typedef struct pbfb_problem pbfb_problem;

typedef enum {
    PBFB_OK = 0,
    PBFB_EINVAL = -1,   /* bad argument (null pointer, eps <= 0, kappa < 0, size) */
    PBFB_EMESH = -2,    /* degenerate tet, open, non-manifold or inward-oriented surface */
    PBFB_ECHARGE = -3,  /* charge outside Gamma_m or closer than 1 A to it */
    PBFB_ENOMEM = -4,   /* device allocation failed */
    PBFB_EDEVICE = -5,  /* HIP runtime error */
    PBFB_ENOTCONV = -6, /* Newton or GMRES iteration limit reached (results hold the last iterate) */
    PBFB_ENAN = -7,     /* non-finite residual */
    PBFB_ESTATE = -8    /* call order violated (mesh/charges/params missing) */
} pbfb_status;

typedef enum { PBFB_FP64 = 0, PBFB_MIXED = 1 } pbfb_precision;
/* nonlinearity of the shell reaction term: N(u) = u, u + u^3/6, sinh(u) */
/* Reaction term of the FEM rows (Sec. 2.4.2; the schemes of Sec. 3.3.1 that raise
 * the Taylor order of sinh as the iterations advance): LIN t, T3 t + t^3/3!,
 * T5 through t^5/5!, T7 through t^7/7!, HS sinh t */
typedef enum { PBFB_LIN = 0, PBFB_T3 = 1, PBFB_HS = 2, PBFB_T5 = 3, PBFB_T7 = 4 } pbfb_scheme;
enum { PBFB_MEM_HOST = 0, PBFB_MEM_DEVICE = 1 };

/* ---- context ------------------------------------------------------------ */
pbfb_status pbfb_ctx_create(int device, pbfb_ctx **out);
/* Problems of the context should be destroyed first.  Any that are still
 * alive are detached: every later call on them returns PBFB_ESTATE except
 * pbfb_problem_destroy, which still releases their device memory. */
void pbfb_ctx_destroy(pbfb_ctx *ctx);
const char *pbfb_last_error(void);

/* ---- problem ------------------------------------------------------------ */
/* precision PBFB_FP64: every operator evaluated, stored and applied in FP64.
 * PBFB_MIXED: the regular (non-touching) boundary-element quadrature is
 * evaluated in FP32 (point offsets from FP64 triangle centroids, FP32 kernel
 * values and per-pair sums over the 36 quadrature pairs), folded onto the
 * vertices in FP64; dense
 * boundary operators and FEM matrix values are stored in FP32 (rounded once
 * from their FP64 sums) and every product is accumulated in FP64.  Krylov
 * vectors (unless krylov_fp32), Newton update, relaxation search,
 * orthogonalisation and touching-panel integrals stay FP64. */
pbfb_status pbfb_problem_create(pbfb_ctx *ctx, int precision, pbfb_problem **out);
void pbfb_problem_destroy(pbfb_problem *p);

/* Shell mesh in Angstrom (Sec. 2.1 three-region model).  nodes[3*n_nodes];
 * tets[4*n_tets] 0-based FEM node ids, any orientation with nonzero volume;
 * tri_m[3*n_tri_m] / tri_s[3*n_tri_s]: Gamma_m / Gamma_s triangles over FEM
 * node ids, oriented so that the right-hand normal points away from the
 * solute.  The surface unknowns are numbered by ascending FEM node id.
 * Errors: EINVAL (sizes / ids out of range), EMESH (surface not closed or
 * not consistently oriented here; at setup, where the geometry is computed on
 * the device: degenerate tet, zero-area triangle, or a surface whose
 * right-hand normals enclose a negative volume, i.e. oriented towards the
 * solute; the double layer's sign depends on the orientation). */
pbfb_status pbfb_set_mesh(pbfb_problem *p, int64_t n_nodes, const double *nodes, int64_t n_tets,
                          const int32_t *tets, int64_t n_tri_m, const int32_t *tri_m, int64_t n_tri_s,
                          const int32_t *tri_s);
/* Point charges (Sec. 2.1, rho_c): positions xyz[3*n] in Angstrom and
 * valences z[n] in units of e.  ECHARGE if a charge is outside Gamma_m or
 * within 1 A of it (the surface integrals of the Coulomb load assume it). */
pbfb_status pbfb_set_charges(pbfb_problem *p, int64_t n, const double *xyz, const double *z);
/* eps_in = eps_m, eps_out = eps_s (relative permittivities, > 0), kappa in
 * 1/Angstrom (>= 0), temperature in K (> 0; potentials are in kT/e). */
pbfb_status pbfb_set_params(pbfb_problem *p, double eps_in, double eps_out, double kappa, double temperature_K);
/* sizes: FEM nodes, Gamma_m vertices, Gamma_s vertices, unknowns, device bytes held */
pbfb_status pbfb_get_sizes(const pbfb_problem *p, int64_t *n_nodes, int64_t *n_m, int64_t *n_s,
                           int64_t *n_unknowns, int64_t *hbm_bytes);
/* Device setup: geometry, sparse pattern, stiffness, surface masses, Coulomb
 * load, dense boundary operators with touching-panel corrections.  Done
 * lazily by the first call that needs it. */
pbfb_status pbfb_setup(pbfb_problem *p, void *hip_stream);

/* Mark every device-computed operator (geometry, FEM values, Coulomb load,
 * dense boundary operators) stale, so that the next call recomputes them from
 * the device-resident mesh; the uploaded mesh, its topology and all device
 * allocations are kept.  Used to time a whole solve from resident inputs. */
pbfb_status pbfb_reset_operators(pbfb_problem *p);

/* ---- operator evaluations (vectors of length n_unknowns, FP64) ---------- */
/* F = A Phi + [N_scheme(u); 0; 0] - b (eq. general_nonlinear) */
pbfb_status pbfb_residual(pbfb_problem *p, int scheme, const double *phi, double *F, int mem, void *hip_stream);
/* Jv = (A + [J_scheme(u) 0 0; 0 0 0; 0 0 0]) v, the Newton matrix of eq. NR_main */
pbfb_status pbfb_apply_jacobian(pbfb_problem *p, int scheme, const double *phi, const double *v, double *Jv,
                                int mem, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of pbfb_residual (same kernels, same result) with every work
 * buffer taken from a fixed per-device work array of 256 MiB that the
 * library holds from its first context on that device until the process
 * ends; the call itself allocates and frees nothing.  phi and F are device
 * memory of the context's GPU (length n_unknowns); the problem must already
 * be set up (pbfb_setup or any earlier call), with dense boundary operators.
 * Errors: ESTATE (not set up), EINVAL (host pointers, matrix-free mode, or a
 * problem whose work memory -- 8 bytes per FEM node, 32 per tet, and per
 * interface of n vertices about 8 n^2 / 16 + 16 n -- exceeds 256 MiB, about
 * 15k vertices per interface).  Every call on one GPU shares the work array:
 * calls that overlap in time on one GPU (other streams, other host threads)
 * race and must be serialised by the caller.  F is complete when the stream
 * reaches the end of the call. */
pbfb_status pbfb_residual_noalloc(pbfb_problem *p, int scheme, const double *phi, double *F, void *hip_stream);

/* ---- Newton solve (Sec. 2.4.2, 2.5, App. A, App. B) --------------------- */
typedef struct {
    int scheme_first;    /* PBFB_T3 (cubic start, default) or PBFB_HS; ignored when n_schedule > 0 */
    int omega_auto;      /* 1: relaxation factor from the root of f_d; 0: omega_fixed */
    double omega_fixed;  /* constant relaxation factor when omega_auto == 0 */
    double tol_nl;       /* stop when omega ||Delta||_2 < tol_nl (1e-3) after a PBFB_HS step */
    double tol_gr;       /* final GMRES relative tolerance (1e-6) */
    double tol_gr0;      /* initial GMRES tolerance (1e-3); == tol_gr disables adaptivity */
    double tol_omega;    /* |f_d| tolerance of the omega search (0.1) */
    double l_e;          /* freeze omega once omega ||Delta|| < l_e (0.35; 0 disables) */
    double omega0_first; /* omega search start in the cubic step (2) */
    double omega0_next;  /* omega search start afterwards (1) */
    double omega_min, omega_max; /* clamp of the search (0, 4) */
    int max_newton;      /* 50 */
    int max_omega_it;    /* 50 */
    int gmres_restart;   /* 200 */
    int max_gmres;       /* iterations per linear solve (2000) */
    int krylov_fp32;     /* PBFB_MIXED only: 1 stores the GMRES basis in FP32, so every restart cycle
                          * is an FP32-basis inner solve inside FP64 iterative refinement (half the
                          * basis memory); 0 (default) keeps the basis FP64 */
    int precond;         /* right preconditioner of GMRES (the paper leaves it open):
                          * PBFB_PC_CHEB_SPAI (default): block diagonal; FEM block F = A + J_N(u):
                          *   cheb_degree terms of the Jacobi-scaled Chebyshev iteration for F z = r
                          *   from z = 0 on [lmax / cheb_ratio, lmax], lmax = max_i sum_j |F_ij| / F_ii;
                          *   single-layer blocks: sparse approximate inverse on each vertex 1-ring
                          *   (row i minimises || m^T V' - e_i^T ||_2);
                          * PBFB_PC_DIAG: inverse of the diagonal of J */
    int cheb_degree;     /* 24 (1..64) */
    double cheb_ratio;   /* 200 (> 1) */
    int hip_graph;       /* 1 (default): each Krylov step of a batch is captured once as a HIP graph and replayed;
                          * 0: kernels launched one by one (also the case while kernel timing is enabled or on
                          * a stream that cannot be captured).  Results are the same bit for bit */
    int omega_method;    /* root finder of f_d (Sec. 2.5, the appendix on one-dimensional root finding):
                          * PBFB_OMEGA_NEWTON (default): Newton-Raphson from omega0_first / omega0_next;
                          * PBFB_OMEGA_BISECT: bisection of [omega_min, omega_max] (Newton from the
                          *   start value when f_d keeps its sign over it);
                          * PBFB_OMEGA_SECANT: secant from omega0 and omega0 + 1/8;
                          * PBFB_OMEGA_BSEC: bisection in the first nonlinear iteration, secant after;
                          * PBFB_OMEGA_NEWTON_BS: Newton, the first iteration starting from three
                          *   bisection midpoints of [2, 3] and secant steps until two iterates differ
                          *   by < 0.05 (the first-iteration start of the appendix on other
                          *   optimisations);
                          * PBFB_OMEGA_BSEC_DF: bisection in the first nonlinear iteration, afterwards
                          *   the direct secant formula omega = w0 / (1 - f_d(w0)), w0 = 1/8 (f_d(0) = 1
                          *   in a Picard step).  pbfb_result.omega_iters counts f_d evaluations after
                          *   the first */
    int nonlinear_method; /* PBFB_NEWTON (default): (A + J_N) Delta = d (eq. NR_main);
                          * PBFB_PICARD: A Delta = d, Delta = intermediate estimate - Phi_NL
                          *   (eqs. Ec_NL_Previo2, Ec_NL_Previo3); the paper searches omega in [0, 1]
                          *   for Picard: set omega_max = 1 */
    double r_e;          /* Picard: the relaxation factor is searched again only when e_{k-2}/e_{k-1} < r_e
                          * (the norm-ratio rule of the section on reducing omega searches; 1.4; 0: every
                          * step) */
    int n_schedule;      /* 0 (default): the scheme_first rule.  1..8: nonlinear iteration k <= n_schedule
                          * uses schedule[k-1] (PBFB_T3, PBFB_T5, PBFB_T7 or PBFB_HS), later ones PBFB_HS:
                          * the T3-T5-HS and T3-T5-T7-T7-HS sequences of Sec. 3.3.1.  The omega search
                          * starts from omega0_first in a T3 iteration, from omega0_next otherwise */
    int schedule[8];
} pbfb_solve_opts;
enum { PBFB_PC_DIAG = 0, PBFB_PC_CHEB_SPAI = 1 };
enum { PBFB_OMEGA_NEWTON = 0, PBFB_OMEGA_BISECT = 1, PBFB_OMEGA_SECANT = 2, PBFB_OMEGA_BSEC = 3,
       PBFB_OMEGA_NEWTON_BS = 4, PBFB_OMEGA_BSEC_DF = 5 };
enum { PBFB_NEWTON = 0, PBFB_PICARD = 1 };
void pbfb_solve_opts_default(pbfb_solve_opts *o);

typedef struct {
    pbfb_status status;
    double total, lc, nc, dg_omega_i; /* kcal/mol: Total = LC + NC + dG_Omega_i (eq. Esolv) */
    int newton_iters, gmres_iters_total, gmres_lin;
    int gmres_iters[64];
    double omega[64], e_k[64];
    int omega_iters[64];
    double t_setup_s; /* from the start of the call (batch: of the batch; server: admission) to the end of setup */
    double t_solve_s; /* from the end of setup to the result */
    int applies;      /* coupled-operator applications performed (Krylov steps, restart residuals, Newton residuals
                       * and relaxation-search products) */
    double t_wait_s;  /* server: from submission to admission (waiting for a slot or for HBM budget); 0 otherwise */
} pbfb_result;

/* Full solve: linear component Phi_L, Newton on Phi_NL, energy.  phi_out
 * (nullable, length 2*n_unknowns) receives [Phi_L | Phi_NL]. */
pbfb_status pbfb_solve(pbfb_problem *p, const pbfb_solve_opts *o, pbfb_result *res, double *phi_out, int mem,
                       void *hip_stream);
/* Batched solve (Sec. 2.4-2.5 for each instance): n independent problems
 * of one context, any mix of sizes and parameters, advanced together.  Each
 * round runs every instance to its next linear solve and then one batched
 * GMRES over all of them (one launch per Krylov step for the whole batch,
 * no host synchronisation between steps).  res[n] receives each instance's
 * result; the per-instance arithmetic does not depend on the batch, so each
 * result equals the one pbfb_solve gives alone.  Returns PBFB_OK when every
 * instance succeeded, otherwise the first failing status. */
pbfb_status pbfb_solve_batch(pbfb_ctx *ctx, int n, pbfb_problem *const *probs, const pbfb_solve_opts *o,
                             pbfb_result *res, void *hip_stream);

/* ---- serving: continuous batching -------------------------------------- */
/* A server owns two streams and two host threads.  Submitted problems wait
 * until a slot (at most max_slots concurrent requests) is free and their
 * estimated device footprint fits in hbm_budget_bytes; they are then set up
 * on a side stream while the running requests keep iterating, join the
 * running set at the next Newton-step boundary and leave it when done.  The
 * problem is borrowed from submit until poll reports done (the caller must
 * not touch it meanwhile and destroys it afterwards); the budget counts a
 * request from admission to completion, plus the context's assembly
 * workspace (shared by the context's problems, grown to the largest
 * assembly it has served and kept).  A completed request's device memory is
 * released (the problem keeps its mesh, charges and parameters; a later call
 * on it sets it up again), so a finished request holds no budget.  ENOMEM at
 * submit: the request alone exceeds the budget; otherwise a request that does
 * not fit waits until running ones complete. */
typedef struct pbfb_server pbfb_server;
pbfb_status pbfb_server_create(pbfb_ctx *ctx, size_t hbm_budget_bytes, int max_slots, pbfb_server **out);
pbfb_status pbfb_server_submit(pbfb_server *s, pbfb_problem *p, const pbfb_solve_opts *o, uint64_t *ticket);
/* The device bytes the server charges for a request: steady (held from
 * admission to completion) and setup (the context's assembly workspace the
 * request's setup needs; charged once per context, see above).  A budget of
 * at least steady + setup admits the request. */
pbfb_status pbfb_request_footprint(const pbfb_problem *p, const pbfb_solve_opts *o, size_t *steady_bytes,
                                   size_t *setup_bytes);
/* done = 1 once the request finished; res (nullable) then receives its result */
pbfb_status pbfb_server_poll(pbfb_server *s, uint64_t ticket, int *done, pbfb_result *res);
/* drains every submitted request, then stops the threads and frees the server;
 * a server must be destroyed before its context */
pbfb_status pbfb_server_destroy(pbfb_server *s);

/* Energy split {Total, LC, NC, dG_Omega_i} (kcal/mol) of given Phi_L, Phi_NL
 * (eqs. Esolv, Esolv_Lineal, Potential_in_Omega_m); phi_nl may be NULL. */
pbfb_status pbfb_energy(pbfb_problem *p, const double *phi_lin, const double *phi_nl, double out[4], int mem,
                        void *hip_stream);

/* ---- regular-assembly tile shape ---------------------------------------- */
/* The non-touching triangle pairs of each interface are integrated in tiles
 * of ta target x tb source triangles (Morton-ordered), one pair per GPU
 * thread.  By default (ta = tb = 0) the shape is chosen by the library's
 * autotuner: the first assembly of a (precision, kernel, size class) in a
 * context times every candidate shape on a sample of that surface and keeps
 * the fastest for the context's lifetime.  Candidates: 16x32, 8x32, 8x64,
 * 16x16, 8x16.  pbfb_set_tile_shape pins one candidate for this problem
 * (PBFB_EINVAL for any other pair) and marks its operators stale.  The shape
 * changes only the order of floating-point sums, never the integrals. */
pbfb_status pbfb_set_tile_shape(pbfb_problem *p, int ta, int tb);
/* Shape used by the last assembly of surface `surf` (0 = Gamma_m, 1 =
 * Gamma_s); 0, 0 before the first assembly. */
pbfb_status pbfb_get_tile_shape(const pbfb_problem *p, int surf, int *ta, int *tb);

/* ---- boundary operator storage ------------------------------------------ */
/* PBFB_BEM_DENSE (default): the four Galerkin blocks are assembled once per
 * setup and stored (n x 2n per interface, FP64 or FP32), every apply is a
 * dense GEMV.  PBFB_BEM_MATRIX_FREE: nothing dense is stored; every apply
 * evaluates the regular quadrature-point pairs on the fly (about 36 N_t^2
 * kernel evaluations per interface) and adds the touching-pair blocks and
 * 1/2 M kept from setup: for instances whose dense blocks would not fit
 * (the paper switches to a fast multipole method above 90k vertices for the
 * same reason).  The 1-ring approximate inverse of the single layers (the
 * GMRES preconditioner) is then built from the near field of V' (for each
 * row, the columns within three rings of its vertex) instead of full rows,
 * so Krylov iteration counts differ a little from dense mode.  Results equal
 * the dense mode's to rounding.  With PBFB_MIXED the FP32 evaluation rounds each apply's source
 * strengths, so the apply is linear to ~1e-7 only and GMRES tolerances below
 * that are not reached.  Marks the operators stale. */
enum { PBFB_BEM_DENSE = 0, PBFB_BEM_MATRIX_FREE = 1 };
pbfb_status pbfb_set_bem_mode(pbfb_problem *p, int mode);

/* The two-field form of Sec. 2.3 (eq. fembem_matrix): the FEM domain is the
 * solute and the shell, and the last n_tets_m tets of the mesh fill the
 * solute (Gamma_m is then an interface inside the FEM mesh; the solute's
 * nodes may be numbered anywhere).  There the permittivity is eps_in and
 * there is no reaction term; the charges load the FEM rows as point sources
 * (b_a = sum_k 4 pi l_B z_k phi_a(x_k), each charge in the solute tet that
 * holds it, else PBFB_ECHARGE at setup); the FEM rows have no lambda_m term
 * and the lambda_m rows are the identity, so lambda_m stays zero through
 * the Newton solve and Phi = [u | 0 | lambda_s].  The energy (pbfb_energy,
 * pbfb_solve's result) recovers lambda_m first from the trace of u with the
 * Laplace operators of Gamma_m (Sec. 2.3.1: V0 lambda_m = (1/2 M_m + K0_m)
 * u - f_m, by conjugate gradients to 1e-13, PBFB_ENOTCONV otherwise).
 * n_tets_m = 0 returns to the shell-only form above.  Needs dense boundary
 * operators (PBFB_EINVAL in matrix-free mode, and set_bem_mode refuses
 * matrix-free while it is on); PBFB_ESTATE before set_mesh, PBFB_EINVAL
 * unless 0 <= n_tets_m < n_tets.  set_mesh resets it to 0. */
pbfb_status pbfb_set_two_field(pbfb_problem *p, int64_t n_tets_m);

/* Two-field form: a surface mesh of Gamma_m given independently of the
 * volume mesh (Sec. 2.3.1, where the trace of the volume solution on Gamma_m
 * is taken by interpolating between the volume and the surface meshes):
 * verts[3*n_verts] in Angstrom, tri[3*n_tri] 0-based vertex ids, oriented
 * like the interface (right-hand normals away from the solute).  lambda_m is
 * then recovered on this mesh, with its own Laplace operators and Coulomb
 * load, from the trace of u at its vertices -- the P1 interpolant of u in the
 * FEM tet that holds each vertex (the one whose smallest barycentric
 * coordinate is largest, ties to the lower tet id) -- and the reaction
 * potential and energy are taken on it.  The interface faces of the volume
 * mesh (tri_m of set_mesh) still separate the permittivities.  Used only in
 * the two-field form; n_verts = 0 removes it; set_mesh removes it.  The
 * arrays are copied.  Errors: PBFB_ESTATE before set_mesh; PBFB_EINVAL (sizes,
 * ids out of range, non-finite coordinates); PBFB_EMESH (not closed, not
 * consistently oriented; at setup: zero-area triangle, oriented inward, or a
 * vertex outside every FEM tet). */
pbfb_status pbfb_set_reaction_surface(pbfb_problem *p, int64_t n_verts, const double *verts, int64_t n_tri,
                                      const int32_t *tri);

/* ---- inspection --------------------------------------------------------- */
/* Copy the two dense blocks stored for surface `surf` (0 = Gamma_m, Laplace;
 * 1 = Gamma_s, Yukawa) as row-major n x n host arrays (either may be NULL):
 *   Gamma_m: Kp = 1/2 M_m + K0_m,  Vp = -V0_m
 *   Gamma_s: Kp = 1/2 M_s - Kk_s,  Vp = +Vk_s
 * i.e. the Galerkin blocks of the second and third block rows above, with
 * M the P1 surface mass, V/K the single/double layer (Sec. 2.2, eq. KV).
 * In mixed precision the FP32 stored values are widened.  PBFB_ESTATE in
 * matrix-free mode (nothing is stored). */
pbfb_status pbfb_export_bem(pbfb_problem *p, int surf, double *Vp, double *Kp);
/* The same blocks for the listed rows only: rows[n_rows] (0-based surface
 * vertex ids, any order, repeats allowed) and row-major n_rows x n host
 * arrays Vp, Kp (either may be NULL), row r of each holding row rows[r] of
 * the block.  For large surfaces, where the full blocks would not fit on the
 * host.  EINVAL for a row out of range; ESTATE in matrix-free mode. */
pbfb_status pbfb_export_bem_rows(pbfb_problem *p, int surf, int64_t n_rows, const int64_t *rows, double *Vp,
                                 double *Kp);
/* Right-hand side b = [0 | f_m | 0] (host array of length n_unknowns); in
 * the two-field form b = [point-charge load | 0 | 0]. */
pbfb_status pbfb_export_rhs(pbfb_problem *p, double *b);
/* Kernel timing with HIP events recorded on the stream each kernel runs on.
 * While enabled, every launch of the timed kernel classes is bracketed by an
 * event pair; pbfb_timing returns the average duration (ms) and the number
 * of launches since the last reset for: which = 0 coupled apply (dense GEMV +
 * FEM SpMV), 1 dense GEMV, 2 FEM SpMV, 3 regular BEM assembly, 4 touching-
 * panel integrals, 5 GMRES preconditioner.  Batched GMRES launches its
 * kernels for every iteration of the batch, so an instance that is between
 * cycles or already converged is counted with a launch that returns at once;
 * pbfb_result.applies counts the applications that did work.
 * pbfb_timing synchronises the problem's last stream. */
pbfb_status pbfb_timing_enable(pbfb_problem *p, int on);
pbfb_status pbfb_timing(pbfb_problem *p, int which, double *avg_ms, int64_t *count, int reset);

#ifdef __cplusplus
}
#endif
#endif /* PBFB_H */
