// Newton driver (Sec. 2.4.2, 2.5, App. A, App. B) as a per-instance state
// machine, and the scheduler that advances any number of instances together:
// every instance runs until it needs a linear solve, then one batched GMRES
// (gmres_batched.hip) serves all of them.  A single solve is a batch of one.
//
// Newton: Phi = Phi_L + Phi_NL, c = b - A Phi, d = c - N(u); solve
// (A + J) Delta = d; Phi_NL += omega Delta; stop when omega ||Delta||_2 <
// Tol_NL.  The first step uses the cubic Taylor scheme (T3), later steps
// sinh (HS), unless a schedule of Taylor orders is given (T3-T5-HS and the
// like of Sec. 3.3.1).  omega is the root of f_d (eq. fd=0) found by Newton's method
// with the derivative of App. A (second derivative r'' = -H[Delta], the
// minus sign the printed formula drops), started at 2 in the T3 step and 1
// afterwards, each iterate clamped to [omega_min, omega_max]; it is frozen
// once e_k < L_e, and the GMRES tolerance is tightened tenfold per step once
// e_k < 1250 tol (App. B).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <thread>

#include "pbfb_internal.hpp"

namespace pbfb {

static inline unsigned nbk(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

__global__ void k_precond(int64_t nn, int64_t nm, int64_t ns, const double *__restrict__ val,
                          const int32_t *__restrict__ diag, const double *__restrict__ vdm,
                          const double *__restrict__ vds, double *__restrict__ dinv)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < nn) dinv[i] = 1.0 / val[diag[i]];
    else if (i < nn + nm) dinv[i] = 1.0 / vdm[i - nn];
    else if (i < nn + nm + ns) dinv[i] = 1.0 / vds[i - nn - nm];
}

__global__ void k_sub_fem(int64_t nn, const double *__restrict__ c, const double *__restrict__ f,
                          double *__restrict__ out)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < nn) out[i] = c[i] - f[i];
}

// block diagonal of the Newton matrix: diag(A + J) on the FEM rows, the
// diagonals of the signed single layers on the surface rows
void build_precond(Problem &p, double *dinv, hipStream_t s)
{
    hipLaunchKernelGGL(k_precond, dim3(nbk(p.n(), 256)), dim3(256), 0, s, p.nn, p.surf[0].nv, p.surf[1].nv, p.d_val,
                       p.d_diag, p.surf[0].vdiag, p.surf[1].vdiag, dinv);
}

// Gershgorin bound of diag(F)^-1 F for the FEM block F = A + J_N (the upper
// end of the Chebyshev interval): per-block maxima, then one block.  A
// maximum does not depend on the order, so the bound is exact and
// reproducible.
__global__ void __launch_bounds__(256) k_gershgorin(int64_t nn, const int32_t *__restrict__ sptr,
                                                    const int32_t *__restrict__ col, const double *__restrict__ val,
                                                    const int32_t *__restrict__ diag, double *__restrict__ part)
{
    __shared__ double red[256];
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    double v = 0.0;
    if (i < nn) {
        const int64_t q = i / SLICE;
        double sum = 0.0; // slice padding adds zeros
        for (int32_t e = sptr[q] + int32_t(i - q * SLICE); e < sptr[q + 1]; e += SLICE)
            if (col[e] < nn) sum += fabs(val[e]);
        v = sum / val[diag[i]];
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_max_final(int64_t nb, const double *__restrict__ part,
                                                   double *__restrict__ out)
{
    __shared__ double red[256];
    double v = 0.0;
    for (int64_t b = threadIdx.x; b < nb; b += 256) v = fmax(v, part[b]);
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// lmax_dev[0] = bound; lmax_dev[1 ..] partial maxima (1 + ceil(nn / 256) doubles)
void fem_gershgorin(Problem &p, double *lmax_dev, hipStream_t s)
{
    const unsigned nb = nbk(p.nn, 256);
    hipLaunchKernelGGL(k_gershgorin, dim3(nb), dim3(256), 0, s, p.nn, p.d_sptr, p.d_col, p.d_val, p.d_diag,
                       lmax_dev + 1);
    hipLaunchKernelGGL(k_max_final, dim3(1), dim3(256), 0, s, int64_t(nb), lmax_dev + 1, lmax_dev);
    PB_HIP(hipGetLastError());
}

enum RunPhase { PH_START = 0, PH_LINEAR = 1, PH_NEWTON = 2, PH_DONE = 3, PH_POST = 4 };
// PH_POST: back from a Newton linear solve, omega of the step set up (searched with the batch's)

// the linear-solve request of the current Newton matrix (its FEM values,
// diagonal and Chebyshev bound are computed here)
static GmresJob make_job(NewtonRun &r, const double *b, double *x, hipStream_t s)
{
    Problem &p = *r.p;
    build_precond(p, r.dinv, s);
    if (r.o.precond == PBFB_PC_CHEB_SPAI) fem_gershgorin(p, r.lmax, s);
    GmresJob J{&p, b, x, r.dinv, r.tol, r.o.gmres_restart, r.o.max_gmres, 0, 0, r.o.krylov_fp32};
    J.pc = r.o.precond;
    J.cheb_k = r.o.cheb_degree;
    J.cheb_ratio = r.o.cheb_ratio;
    J.lmax = r.lmax;
    J.applies = 0;
    J.graph = r.o.hip_graph;
    return J;
}

NewtonRun::NewtonRun(Problem *p_, const pbfb_solve_opts &o_, pbfb_result *res_, double *out)
    : p(p_), o(o_), res(res_), phi_out_dev(out)
{
    *res = pbfb_result{};
    t0 = std::chrono::steady_clock::now(); // batch start / admission time
}

static void finish(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n();
    double en[4] = {0, 0, 0, 0};
    if (r.phil) {
        energy(p, r.phil, r.phinl, en, s);
        if (r.phi_out_dev) {
            PB_HIP(hipMemcpyAsync(r.phi_out_dev, r.phil, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            PB_HIP(hipMemcpyAsync(r.phi_out_dev + n, r.phinl, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        }
    }
    PB_HIP(hipStreamSynchronize(s));
    auto t2 = std::chrono::steady_clock::now();
    r.res->total = en[0];
    r.res->lc = en[1];
    r.res->nc = en[2];
    r.res->dg_omega_i = en[3];
    r.res->newton_iters = r.k;
    r.res->status = pbfb_status(r.status);
    r.res->t_setup_s = std::chrono::duration<double>(r.t1 - r.t0).count();
    r.res->t_solve_s = std::chrono::duration<double>(t2 - r.t1).count();
    r.phase = PH_DONE;
}

// Newton pre-step: residual, Jacobian values, preconditioner, linear solve request
static bool newton_pre(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n(), nn = p.nn;
    if (r.o.n_schedule > 0) r.sch = r.k <= r.o.n_schedule ? r.o.schedule[r.k - 1] : PBFB_HS;
    else r.sch = (r.k == 1 && r.o.scheme_first == PBFB_T3) ? PBFB_T3 : PBFB_HS;
    vec_add(n, r.phil, r.phinl, r.phi, s);
    if (!r.c_ready) { // else c was carried over from the last step's omega search
        coupled_apply_linear(p, r.phi, r.c, s);
        vec_axpby(n, 1.0, p.d_b, -1.0, r.c, s);
        r.res->applies += 1; // c = b - A Phi
    }
    r.c_ready = false;
    fem_nonlinear(p, r.sch, r.phi, r.rN, s);
    PB_HIP(hipMemcpyAsync(r.d, r.c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_sub_fem, dim3(nbk(nn, 256)), dim3(256), 0, s, nn, r.c, r.rN, r.d);
    const double dd = dot(p, r.d, r.d, n, s);
    if (!std::isfinite(dd)) {
        r.status = PBFB_ENAN;
        return false;
    }
    // Newton: (A + J_N) Delta = d; Picard: A Delta = d
    if (r.o.nonlinear_method == PBFB_PICARD) fem_assemble_linear(p, s);
    else fem_assemble_jacobian(p, r.sch, r.phi, s);
    r.job = make_job(r, r.d, r.D, s);
    return true;
}

// ---------------------------------------------------------------------------
// root of f_d (Sec. 2.5; the appendix on one-dimensional root finding and
// the first-iteration start of the appendix on other optimisations), on the
// device.  Every method stops at |f_d| < tol_omega or after max_omega_it
// evaluations; iterates are clamped to [omega_min, omega_max]; an undefined
// f_d (beta = 0) or a vanishing derivative / secant slope gives omega = 1.
//
// The search of one instance is a small state machine in device memory
// (OmegaSearch).  One evaluation round is: the f_d terms at S.w (the element
// kernel reads omega from S.w), their six dot products into S.v, then
// k_omega_step, one thread that forms f_d and f_d' and moves the state to
// the next point to evaluate or to its result.  Once S.done is set the
// round's kernels return at once.  The host enqueues rounds for every
// searching instance of the batch and reads the done flags back only every
// few rounds, one copy and one synchronisation for all of them.
// ---------------------------------------------------------------------------
enum OmPhase {
    OM_NEWTON = 0, // evaluating w of the Newton iteration
    OM_SEC_A,      // secant: the first point w0
    OM_SEC_B,      // secant: the second point / each new point w1
    OM_BIS_LO,     // bisection: the lower end
    OM_BIS_HI,     // bisection: the upper end
    OM_BIS_MID,    // bisection: a midpoint
    OM_BS_START,   // first-iteration start: the three midpoints of [2, 3]
    OM_BS_SEC,     // first-iteration start: its secant steps
    OM_DF          // direct secant through (0, 1): the point 1/8
};

struct OmegaSearch {
    // setup
    int method, k, max_it;
    double tol, wmin, wmax, omega0;
    double pp; // p.p of this step
    // state
    int phase, ev, done, fb, si;
    double w; // the point of the next evaluation (the element kernel reads it)
    double lo, hi, flo, wstart;
    double w0, f0, w1, f1;
    double blo, bhi, bw[3], bf[3];
    double result;
    double v[6]; // (p . r) over all unknowns, then (rJ.r, rJ.p, rJ.rJ, r.rH, p.rH) over the FEM rows
};

__device__ inline double om_clamp(const OmegaSearch &S, double w) { return fmin(S.wmax, fmax(S.wmin, w)); }
__device__ inline void om_finish(OmegaSearch &S, double w, bool fallback)
{
    S.result = w;
    S.fb = fallback ? 1 : S.fb;
    S.done = 1;
}
// Newton from w (the while condition of the iteration is checked first)
__device__ inline void om_newton_start(OmegaSearch &S, double w)
{
    if (S.ev >= S.max_it) return om_finish(S, w, false);
    S.phase = OM_NEWTON;
    S.w = w;
}
__device__ inline void om_bisect_start(OmegaSearch &S, double lo, double hi, double wstart)
{
    S.lo = lo;
    S.hi = hi;
    S.wstart = wstart;
    S.phase = OM_BIS_LO;
    S.w = lo;
}
__device__ inline void om_secant_start(OmegaSearch &S, double w0, double w1)
{
    S.w0 = w0;
    S.w1 = w1;
    S.phase = OM_SEC_A;
    S.w = w0;
}
// the secant loop of the first-iteration start, from (w0, f0), (w1, f1)
__device__ inline void om_bs_loop(OmegaSearch &S)
{
    if (S.ev >= S.max_it) return om_newton_start(S, S.w1);
    const double slope = S.f0 - S.f1;
    if (slope == 0.0 || !isfinite(slope)) return om_newton_start(S, S.w1);
    const double w2 = om_clamp(S, S.w0 - (S.w0 - S.w1) * S.f0 / slope);
    if (fabs(w2 - S.w1) < 0.05) return om_newton_start(S, w2);
    S.w0 = S.w1;
    S.f0 = S.f1;
    S.w1 = w2;
    S.phase = OM_BS_SEC;
    S.w = w2;
}

__global__ void k_omega_init(OmegaSearch *__restrict__ S_, int method, int k, int max_it, double tol, double wmin,
                             double wmax, double omega0)
{
    if (threadIdx.x != 0) return;
    OmegaSearch S{};
    S.method = method;
    S.k = k;
    S.max_it = max_it;
    S.tol = tol;
    S.wmin = wmin;
    S.wmax = wmax;
    S.omega0 = omega0;
    switch (method) {
    case PBFB_OMEGA_BISECT: om_bisect_start(S, wmin, wmax, omega0); break;
    case PBFB_OMEGA_SECANT: om_secant_start(S, omega0, omega0 + 0.125); break;
    case PBFB_OMEGA_BSEC:
        if (k == 1) om_bisect_start(S, wmin, wmax, omega0);
        else om_secant_start(S, omega0, omega0 + 0.125);
        break;
    case PBFB_OMEGA_NEWTON_BS:
        if (k == 1) {
            S.blo = 2.0;
            S.bhi = 3.0;
            S.si = 0;
            S.phase = OM_BS_START;
            S.w = 2.5;
        } else {
            om_newton_start(S, omega0);
        }
        break;
    case PBFB_OMEGA_BSEC_DF:
        if (k == 1) {
            om_bisect_start(S, wmin, wmax, omega0);
        } else {
            S.phase = OM_DF;
            S.w = 0.125;
        }
        break;
    default: om_newton_start(S, omega0); break;
    }
    *S_ = S;
}

// f_d and f_d' at S.w from the dot products (eq. fd=0 and its derivative,
// r' = -[rJ; 0; 0], r'' = -[rH; 0; 0]), then the next state
__global__ void k_omega_step(OmegaSearch *__restrict__ S_)
{
    if (threadIdx.x != 0) return;
    OmegaSearch S = *S_;
    if (S.done) return;
    const double w = S.w;
    const double a = S.v[0] - S.v[1];     // (p + r').r
    const double beta = S.pp - S.v[2];    // (p + r').p
    const bool ok = beta != 0.0;
    double fd = 0.0, dfd = 0.0;
    if (ok) {
        fd = -a / beta - w;
        dfd = -(-S.v[2] + S.v[3] - S.v[4]) / beta + a * (-S.v[5]) / (beta * beta) - 1.0;
    }
    ++S.ev;
    if (!ok) {
        om_finish(S, 1.0, true);
        *S_ = S;
        return;
    }
    switch (S.phase) {
    case OM_NEWTON:
        if (fabs(fd) < S.tol) om_finish(S, w, false);
        else if (dfd == 0.0 || !isfinite(dfd)) om_finish(S, 1.0, true);
        else {
            const double wn = om_clamp(S, w - fd / dfd);
            if (S.ev >= S.max_it) om_finish(S, wn, false);
            else S.w = wn;
        }
        break;
    case OM_SEC_A:
        if (fabs(fd) < S.tol) {
            om_finish(S, w, false);
        } else {
            S.f0 = fd;
            S.phase = OM_SEC_B;
            S.w = S.w1;
        }
        break;
    case OM_SEC_B:
        S.f1 = fd;
        if (fabs(S.f1) >= S.tol && S.ev < S.max_it) {
            const double slope = S.f0 - S.f1;
            if (slope == 0.0 || !isfinite(slope)) {
                om_finish(S, 1.0, true);
            } else {
                const double w2 = om_clamp(S, S.w0 - (S.w0 - S.w1) * S.f0 / slope);
                S.w0 = S.w1;
                S.f0 = S.f1;
                S.w1 = w2;
                S.w = w2;
            }
        } else {
            om_finish(S, S.w1, false);
        }
        break;
    case OM_BIS_LO:
        if (fabs(fd) < S.tol) {
            om_finish(S, S.lo, false);
        } else {
            S.flo = fd;
            S.phase = OM_BIS_HI;
            S.w = S.hi;
        }
        break;
    case OM_BIS_HI:
        if (fabs(fd) < S.tol) om_finish(S, S.hi, false);
        else if ((S.flo > 0.0) == (fd > 0.0)) om_newton_start(S, S.wstart); // no sign change over the interval
        else if (S.ev >= S.max_it) om_finish(S, 0.5 * (S.lo + S.hi), false);
        else {
            S.phase = OM_BIS_MID;
            S.w = 0.5 * (S.lo + S.hi);
        }
        break;
    case OM_BIS_MID:
        if (fabs(fd) < S.tol) {
            om_finish(S, w, false);
        } else {
            if ((fd > 0.0) == (S.flo > 0.0)) {
                S.lo = w;
                S.flo = fd;
            } else {
                S.hi = w;
            }
            if (S.ev < S.max_it) S.w = 0.5 * (S.lo + S.hi);
            else om_finish(S, w, false);
        }
        break;
    case OM_BS_START:
        S.bw[S.si] = w;
        S.bf[S.si] = fd;
        if (fd > 0.0) S.blo = w;
        else S.bhi = w;
        ++S.si;
        if (S.si < 3) {
            S.w = 0.5 * (S.blo + S.bhi);
        } else {
            S.w0 = S.bw[1];
            S.f0 = S.bf[1];
            S.w1 = S.bw[2];
            S.f1 = S.bf[2];
            om_bs_loop(S);
        }
        break;
    case OM_BS_SEC:
        S.f1 = fd;
        om_bs_loop(S);
        break;
    case OM_DF:
        if (fd == 1.0 || !isfinite(fd)) om_finish(S, 1.0, true);
        else om_finish(S, om_clamp(S, 0.125 / (1.0 - fd)), false);
        break;
    default: om_finish(S, 1.0, true); break;
    }
    *S_ = S;
}

__global__ void k_omega_read(const OmegaSearch *__restrict__ S, double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    out[0] = S->done;
    out[1] = S->result;
    out[2] = S->ev;
    out[3] = S->fb;
}

__global__ void k_sub_fem_skip(int64_t nn, const double *__restrict__ c, const double *__restrict__ f,
                               double *__restrict__ out, const int *__restrict__ skip)
{
    if (*skip) return;
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < nn) out[i] = c[i] - f[i];
}

static OmegaSearch *om_state(NewtonRun &r) { return static_cast<OmegaSearch *>(r.om_dev); }

// one evaluation round of a search: f_d terms at S.w, the dot products, the step
static void omega_round(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n(), nn = p.nn;
    OmegaSearch *S = om_state(r);
    const int *skip = &S->done;
    fem_omega_terms_dev(p, r.sch, r.phi, r.D, &S->w, skip, r.rN, r.rJ, r.rH, s);
    hipLaunchKernelGGL(k_sub_fem_skip, dim3(nbk(nn, 256)), dim3(256), 0, s, nn, r.c, r.rN, r.rv, skip);
    const double *pa = r.pv, *pb = r.rv;
    dots_dev(p, 1, &pa, &pb, n, S->v, skip, s);
    const double *A5[5] = {r.rJ, r.rJ, r.rJ, r.rv, r.pv};
    const double *B5[5] = {r.rv, r.pv, r.rJ, r.rH, r.rH};
    dots_dev(p, 5, A5, B5, nn, S->v + 1, skip, s);
    hipLaunchKernelGGL(k_omega_step, dim3(1), dim3(64), 0, s, S);
}

// the searches of all runs in `srch` together: rounds for every run whose
// search is not known to be done, the done flags read back every few rounds
static void omega_search_all(std::vector<NewtonRun *> &srch, hipStream_t s)
{
    constexpr int ROUNDS = 2; // evaluation rounds between two host checks
    std::vector<NewtonRun *> act = srch;
    while (!act.empty()) {
        for (int q = 0; q < ROUNDS; ++q)
            for (NewtonRun *r : act) omega_round(*r, s);
        for (NewtonRun *r : act) {
            double *h = scratch<double>(*r->p, SCR_OMEGA, sizeof(OmegaSearch) / 8 + 8) + sizeof(OmegaSearch) / 8 + 2;
            hipLaunchKernelGGL(k_omega_read, dim3(1), dim3(64), 0, s, om_state(*r), h);
            PB_HIP(hipMemcpyAsync(r->om_host, h, sizeof(r->om_host), hipMemcpyDeviceToHost, s));
        }
        PB_HIP(hipStreamSynchronize(s));
        std::vector<NewtonRun *> next;
        for (NewtonRun *r : act) {
            if (r->om_host[0] != 0.0) {
                r->omega = r->om_host[1];
                r->searching = false;
            } else {
                next.push_back(r);
            }
        }
        act.swap(next);
    }
}

// omega of this step: fixed, frozen, reused (Picard) or searched.  A search
// is set up here (p = -A Delta, p.p into the device state) and run later
// together with the other instances' (omega_search_all).
static void newton_post_begin(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n();
    const pbfb_solve_opts &o = r.o;
    r.searching = r.searched = false;
    if (!o.omega_auto) {
        r.omega = o.omega_fixed;
    } else if (r.frozen) {
        r.omega = r.omega_last;
    } else if (o.nonlinear_method == PBFB_PICARD && o.r_e > 0 && r.k >= 3 && r.e_km2 >= o.r_e * r.e_km1) {
        r.omega = r.omega_last; // e_{k-2} / e_{k-1} >= R_e: converging fast enough, reuse
    } else {
        const double omega0 = r.sch == PBFB_T3 ? o.omega0_first : o.omega0_next;
        // p = -A Delta
        coupled_apply_linear(p, r.D, r.pv, s);
        r.res->applies += 1;
        r.searched = r.searching = true;
        vec_axpby(n, -1.0, r.pv, 0.0, r.pv, s);
        PB_HIP(hipMemcpyAsync(r.rv, r.c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        r.om_dev = scratch<double>(p, SCR_OMEGA, sizeof(OmegaSearch) / 8 + 8);
        OmegaSearch *S = om_state(r);
        hipLaunchKernelGGL(k_omega_init, dim3(1), dim3(64), 0, s, S, o.omega_method, r.k, o.max_omega_it, o.tol_omega,
                           o.omega_min, o.omega_max, omega0);
        const double *pa = r.pv;
        dots_dev(p, 1, &pa, &pa, n, &S->pp, nullptr, s);
    }
}

// update and stop test after the search (or without one); true when converged
static bool newton_post_end(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n();
    const pbfb_solve_opts &o = r.o;
    const int idx = std::min(r.k - 1, 63);
    const double omega = r.omega;
    int oit = 0;
    if (r.searched) {
        const int evals = int(r.om_host[2]);
        oit = evals > 0 ? evals - 1 : 0;
        r.omega_last = omega;
    }
    vec_axpby(n, omega, r.D, 1.0, r.phinl, s);
    if (r.searched) {
        // A (Phi + omega Delta) = A Phi - omega p: the next c = b - A Phi without an apply
        vec_axpby(n, omega, r.pv, 1.0, r.c, s);
        r.c_ready = true;
    }
    const double ek = omega * std::sqrt(dot(p, r.D, r.D, n, s));
    r.res->omega[idx] = omega;
    r.res->e_k[idx] = ek;
    r.res->omega_iters[idx] = oit;
    r.e_km2 = r.e_km1;
    r.e_km1 = ek;
    if (!std::isfinite(ek)) {
        r.status = PBFB_ENAN;
        return true;
    }
    if (o.l_e > 0 && ek < o.l_e) r.frozen = true;
    if (o.tol_gr0 > o.tol_gr && ek < 1250.0 * r.tol) r.tol = std::max(o.tol_gr, 0.1 * r.tol);
    // only a sinh step ends the iteration: a Taylor step solves another equation
    if (ek < o.tol_nl && r.sch == PBFB_HS) return true;
    if (r.k >= o.max_newton) {
        r.status = PBFB_ENOTCONV;
        return true;
    }
    return false;
}

// Advance one instance until it needs a linear solve (returns true) or is done.
static bool advance_impl(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n(), nn = p.nn;
    if (r.phase == PH_START) {
        ensure_all(p, s);
        PB_HIP(hipStreamSynchronize(s));
        r.t1 = std::chrono::steady_clock::now();
        r.phil = scratch<double>(p, SCR_G3, n);
        r.phinl = scratch<double>(p, SCR_G4, n);
        r.phi = scratch<double>(p, SCR_G5, n);
        r.c = scratch<double>(p, SCR_G6, n);
        r.d = scratch<double>(p, SCR_G7, n);
        r.D = scratch<double>(p, SCR_G8, n);
        r.pv = scratch<double>(p, SCR_G9, n);
        r.rv = scratch<double>(p, SCR_G10, n);
        double *t3 = scratch<double>(p, SCR_G11, 3 * nn);
        r.rN = t3;
        r.rJ = t3 + nn;
        r.rH = t3 + 2 * nn;
        r.dinv = scratch<double>(p, SCR_G2, n);
        r.tol = r.o.tol_gr0;
        PB_HIP(hipMemsetAsync(r.phinl, 0, sizeof(double) * n, s));
        // linear component: (A + eps_s kappa^2 M) Phi_L = b
        r.lmax = scratch<double>(p, SCR_LMAX, 1 + nbk(nn, 256));
        fem_assemble_jacobian(p, PBFB_LIN, r.phinl, s);
        r.job = make_job(r, p.d_b, r.phil, s);
        r.phase = PH_LINEAR;
        return true;
    }
    if (r.phase == PH_LINEAR) {
        r.res->gmres_lin = r.job.iters;
        r.res->gmres_iters_total = r.job.iters;
        r.res->applies += r.job.applies;
        if (r.job.status) {
            r.status = r.job.status;
            finish(r, s);
            return false;
        }
        r.k = 1;
        r.phase = PH_NEWTON;
        if (!newton_pre(r, s)) {
            finish(r, s);
            return false;
        }
        return true;
    }
    if (r.phase == PH_NEWTON) {
        const int idx = std::min(r.k - 1, 63);
        r.res->gmres_iters[idx] = r.job.iters;
        r.res->gmres_iters_total += r.job.iters;
        r.res->applies += r.job.applies;
        if (r.job.status) {
            r.status = r.job.status;
            finish(r, s);
            return false;
        }
        newton_post_begin(r, s);
        r.phase = PH_POST; // the search (if any) runs with the other instances'
        return false;
    }
    if (r.phase == PH_POST) {
        if (newton_post_end(r, s)) {
            finish(r, s);
            return false;
        }
        ++r.k;
        r.phase = PH_NEWTON;
        if (!newton_pre(r, s)) {
            finish(r, s);
            return false;
        }
        return true;
    }
    return false;
}

bool advance(NewtonRun &r, hipStream_t s)
{
    try {
        return advance_impl(r, s);
    } catch (const Error &e) {
        r.status = e.code;
        r.message = e.msg;
        r.res->status = e.code;
        r.phase = PH_DONE;
        return false;
    }
}

// Device setup (geometry, load, operators) of the runs that have not
// started, on up to N_ASM_WS host threads with a stream of the context each:
// the assembly kernels of a small instance leave most of the GPU idle, and
// several instances at once fill it.  Each run's state machine then finds its
// operators ready.  An error ends that run with its code.
static void parallel_setup(std::vector<NewtonRun *> &fresh, hipStream_t s)
{
    Ctx *C = fresh[0]->p->ctx;
    for (NewtonRun *r : fresh)
        if (r->p->ctx != C) return; // the streams and workspaces are the context's
    const int nt = int(std::min<size_t>(N_ASM_WS, fresh.size()));
    PB_HIP(hipStreamSynchronize(s)); // work the caller enqueued before the solve is complete
    {
        std::lock_guard<std::mutex> lk(C->setup_mu);
        for (int t = 0; t < nt; ++t)
            if (!C->setup_stream[t]) PB_HIP(hipStreamCreateWithFlags(&C->setup_stream[t], hipStreamNonBlocking));
    }
    std::atomic<size_t> next{0};
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            const bool dev_ok = hipSetDevice(C->device) == hipSuccess;
            for (size_t i; (i = next++) < fresh.size();) {
                NewtonRun &r = *fresh[i];
                try {
                    PB_CHECK(dev_ok, PBFB_EDEVICE, "hipSetDevice failed in the setup thread");
                    ensure_all(*r.p, C->setup_stream[t]);
                    PB_HIP(hipStreamSynchronize(C->setup_stream[t]));
                } catch (const Error &e) {
                    r.status = e.code;
                    r.message = e.msg;
                    r.res->status = e.code;
                    r.phase = PH_DONE;
                }
            }
        });
    for (std::thread &x : th) x.join();
}

void advance_all(std::vector<NewtonRun *> &runs, std::vector<GmresJob *> &jobs, std::vector<NewtonRun *> *finished,
                 hipStream_t s)
{
    std::vector<NewtonRun *> fresh;
    for (NewtonRun *r : runs)
        if (r->phase == PH_START) fresh.push_back(r);
    if (fresh.size() > 1) parallel_setup(fresh, s);
    for (NewtonRun *r : fresh)
        if (r->phase == PH_DONE && finished) finished->push_back(r);
    auto step = [&](NewtonRun *r) {
        if (advance(*r, s)) jobs.push_back(&r->job);
        else if (r->phase == PH_DONE && finished) finished->push_back(r);
    };
    for (NewtonRun *r : runs)
        if (r->phase != PH_DONE && r->phase != PH_POST) step(r);
    // relaxation searches of every instance between two linear solves, together
    std::vector<NewtonRun *> srch;
    for (NewtonRun *r : runs)
        if (r->phase == PH_POST && r->searching) srch.push_back(r);
    if (!srch.empty()) {
        try {
            omega_search_all(srch, s);
        } catch (const Error &e) {
            for (NewtonRun *r : srch) {
                r->status = e.code;
                r->message = e.msg;
                r->res->status = e.code;
                r->phase = PH_DONE;
                if (finished) finished->push_back(r);
            }
        }
    }
    for (NewtonRun *r : runs)
        if (r->phase == PH_POST) step(r);
}

void run_newton(std::vector<NewtonRun *> &runs, hipStream_t s)
{
    std::vector<GmresJob *> jobs;
    for (;;) {
        jobs.clear();
        advance_all(runs, jobs, nullptr, s);
        if (jobs.empty()) break;
        try {
            batched_gmres(jobs, s);
        } catch (const Error &e) {
            // a device error ends every instance of the batch with its code
            for (NewtonRun *r : runs)
                if (r->phase != PH_DONE) {
                    r->job.status = e.code;
                    r->message = e.msg;
                }
        }
    }
}

pbfb_status solve(Problem &p, const pbfb_solve_opts &o, pbfb_result &res, double *phi_out_dev, hipStream_t s)
{
    NewtonRun r(&p, o, &res, phi_out_dev);
    std::vector<NewtonRun *> runs{&r};
    run_newton(runs, s);
    if (!r.message.empty()) set_error(r.message);
    return res.status;
}

} // namespace pbfb
