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
#include <chrono>
#include <cmath>

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

enum RunPhase { PH_START = 0, PH_LINEAR = 1, PH_NEWTON = 2, PH_DONE = 3 };

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
// the first-iteration start of the appendix on other optimisations).
// Every method stops at |f_d| < tol_omega or after max_omega_it
// evaluations; iterates are clamped to [omega_min, omega_max]; an undefined
// f_d (beta = 0) or a vanishing derivative / secant slope gives omega = 1.
// ---------------------------------------------------------------------------
static double clampw(double w, const pbfb_solve_opts &o) { return std::min(o.omega_max, std::max(o.omega_min, w)); }

template <class F>
static double omega_newton(const pbfb_solve_opts &o, F &f, double w, int &ev, bool &fb)
{
    while (ev < o.max_omega_it) {
        double fd = 0.0, dfd = 0.0;
        ++ev;
        if (!f(w, fd, dfd)) {
            fb = true;
            return 1.0;
        }
        if (std::fabs(fd) < o.tol_omega) return w;
        if (dfd == 0.0 || !std::isfinite(dfd)) {
            fb = true;
            return 1.0;
        }
        w = clampw(w - fd / dfd, o);
    }
    return w;
}

// secant from the pair (w0, w1)
template <class F>
static double omega_secant(const pbfb_solve_opts &o, F &f, double w0, double w1, int &ev, bool &fb)
{
    double f0 = 0.0, f1 = 0.0, d = 0.0;
    ++ev;
    if (!f(w0, f0, d)) {
        fb = true;
        return 1.0;
    }
    if (std::fabs(f0) < o.tol_omega) return w0;
    ++ev;
    if (!f(w1, f1, d)) {
        fb = true;
        return 1.0;
    }
    while (std::fabs(f1) >= o.tol_omega && ev < o.max_omega_it) {
        const double slope = f0 - f1;
        if (slope == 0.0 || !std::isfinite(slope)) {
            fb = true;
            return 1.0;
        }
        const double w2 = clampw(w0 - (w0 - w1) * f0 / slope, o);
        w0 = w1;
        f0 = f1;
        w1 = w2;
        ++ev;
        if (!f(w1, f1, d)) {
            fb = true;
            return 1.0;
        }
    }
    return w1;
}

// bisection of [lo, hi]; Newton from w_start when f_d keeps its sign over it
template <class F>
static double omega_bisect(const pbfb_solve_opts &o, F &f, double lo, double hi, double w_start, int &ev, bool &fb)
{
    double flo = 0.0, fhi = 0.0, d = 0.0;
    ++ev;
    if (!f(lo, flo, d)) {
        fb = true;
        return 1.0;
    }
    if (std::fabs(flo) < o.tol_omega) return lo;
    ++ev;
    if (!f(hi, fhi, d)) {
        fb = true;
        return 1.0;
    }
    if (std::fabs(fhi) < o.tol_omega) return hi;
    if ((flo > 0.0) == (fhi > 0.0)) return omega_newton(o, f, w_start, ev, fb);
    double mid = 0.5 * (lo + hi);
    while (ev < o.max_omega_it) {
        mid = 0.5 * (lo + hi);
        double fm = 0.0;
        ++ev;
        if (!f(mid, fm, d)) {
            fb = true;
            return 1.0;
        }
        if (std::fabs(fm) < o.tol_omega) return mid;
        if ((fm > 0.0) == (flo > 0.0)) {
            lo = mid;
            flo = fm;
        } else {
            hi = mid;
        }
    }
    return mid;
}

// first-iteration start: three bisection midpoints of [2, 3] (a positive
// f_d moves up: f_d decreases through its root), then secant steps from the
// last two until successive iterates differ by less than 0.05
template <class F> static double omega_start_bs(const pbfb_solve_opts &o, F &f, int &ev, bool &fb)
{
    double lo = 2.0, hi = 3.0, w[3], fv[3], d = 0.0;
    for (int i = 0; i < 3; ++i) {
        w[i] = 0.5 * (lo + hi);
        ++ev;
        if (!f(w[i], fv[i], d)) {
            fb = true;
            return 1.0;
        }
        if (fv[i] > 0.0) lo = w[i];
        else hi = w[i];
    }
    double w0 = w[1], f0 = fv[1], w1 = w[2], f1 = fv[2];
    while (ev < o.max_omega_it) {
        const double slope = f0 - f1;
        if (slope == 0.0 || !std::isfinite(slope)) break;
        const double w2 = clampw(w0 - (w0 - w1) * f0 / slope, o);
        if (std::fabs(w2 - w1) < 0.05) return w2;
        w0 = w1;
        f0 = f1;
        w1 = w2;
        ++ev;
        if (!f(w1, f1, d)) {
            fb = true;
            return 1.0;
        }
    }
    return w1;
}

// the root finder of opts.omega_method at nonlinear iteration k (1-based)
template <class F>
static double omega_root(const pbfb_solve_opts &o, int k, double omega0, F &f, int &ev, bool &fb)
{
    switch (o.omega_method) {
    case PBFB_OMEGA_BISECT: return omega_bisect(o, f, o.omega_min, o.omega_max, omega0, ev, fb);
    case PBFB_OMEGA_SECANT: return omega_secant(o, f, omega0, omega0 + 0.125, ev, fb);
    case PBFB_OMEGA_BSEC:
        if (k == 1) return omega_bisect(o, f, o.omega_min, o.omega_max, omega0, ev, fb);
        return omega_secant(o, f, omega0, omega0 + 0.125, ev, fb);
    case PBFB_OMEGA_NEWTON_BS:
        if (k == 1) {
            const double w = omega_start_bs(o, f, ev, fb);
            if (fb) return w;
            return omega_newton(o, f, w, ev, fb);
        }
        return omega_newton(o, f, omega0, ev, fb);
    case PBFB_OMEGA_BSEC_DF:
        if (k == 1) return omega_bisect(o, f, o.omega_min, o.omega_max, omega0, ev, fb);
        {
            // the secant through (0, 1) and (w0, f_d(w0)): f_d(0) = 1 in a Picard step
            const double w0 = 0.125;
            double f0 = 0.0, d = 0.0;
            ++ev;
            if (!f(w0, f0, d) || f0 == 1.0 || !std::isfinite(f0)) {
                fb = true;
                return 1.0;
            }
            return clampw(w0 / (1.0 - f0), o);
        }
    default: return omega_newton(o, f, omega0, ev, fb);
    }
}

// omega search and update after the Newton linear solve; true when converged
static bool newton_post(NewtonRun &r, hipStream_t s)
{
    Problem &p = *r.p;
    const int64_t n = p.n(), nn = p.nn;
    const pbfb_solve_opts &o = r.o;
    const int idx = std::min(r.k - 1, 63);
    double omega;
    int oit = 0;
    bool searched = false; // r.pv = -A Delta was formed
    if (!o.omega_auto) {
        omega = o.omega_fixed;
    } else if (r.frozen) {
        omega = r.omega_last;
    } else if (o.nonlinear_method == PBFB_PICARD && o.r_e > 0 && r.k >= 3 && r.e_km2 >= o.r_e * r.e_km1) {
        omega = r.omega_last; // e_{k-2} / e_{k-1} >= R_e: converging fast enough, reuse
    } else {
        const double omega0 = r.sch == PBFB_T3 ? o.omega0_first : o.omega0_next;
        // p = -A Delta
        coupled_apply_linear(p, r.D, r.pv, s);
        r.res->applies += 1;
        searched = true;
        vec_axpby(n, -1.0, r.pv, 0.0, r.pv, s);
        const double pp = dot(p, r.pv, r.pv, n, s);
        PB_HIP(hipMemcpyAsync(r.rv, r.c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        // f_d(omega) and f_d'(omega) (eq. fd=0 and its derivative); false when beta = 0
        auto fd_at = [&](double w, double &fd, double &dfd) {
            fem_omega_terms(p, r.sch, r.phi, r.D, w, r.rN, r.rJ, r.rH, s);
            hipLaunchKernelGGL(k_sub_fem, dim3(nbk(nn, 256)), dim3(256), 0, s, nn, r.c, r.rN, r.rv);
            const double pr = dot(p, r.pv, r.rv, n, s);
            const double *A5[5] = {r.rJ, r.rJ, r.rJ, r.rv, r.pv};
            const double *B5[5] = {r.rv, r.pv, r.rJ, r.rH, r.rH};
            double v5[5];
            dots(p, 5, A5, B5, nn, v5, s);
            // r' = -[rJ; 0; 0], r'' = -[rH; 0; 0]
            const double a = pr - v5[0];    // (p + r').r
            const double beta = pp - v5[1]; // (p + r').p
            if (beta == 0.0) return false;
            fd = -a / beta - w;
            dfd = -(-v5[1] + v5[2] - v5[3]) / beta + a * (-v5[4]) / (beta * beta) - 1.0;
            return true;
        };
        int evals = 0;
        bool fallback = false;
        omega = omega_root(o, r.k, omega0, fd_at, evals, fallback);
        oit = evals > 0 ? evals - 1 : 0;
        r.omega_last = omega;
    }
    vec_axpby(n, omega, r.D, 1.0, r.phinl, s);
    if (searched) {
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
        if (newton_post(r, s)) {
            finish(r, s);
            return false;
        }
        ++r.k;
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

void run_newton(std::vector<NewtonRun *> &runs, hipStream_t s)
{
    std::vector<GmresJob *> jobs;
    for (;;) {
        jobs.clear();
        for (NewtonRun *r : runs)
            if (r->phase != PH_DONE && advance(*r, s)) jobs.push_back(&r->job);
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
