// Krylov and Newton drivers (host control, device data).
//
// GMRES: restarted, right preconditioned by the block diagonal of the Newton
// matrix (diag(A + J), diag(-V0_m), diag(Vk_s)), x0 = 0, classical
// Gram-Schmidt applied twice in FP64, Givens rotations on the host; stops
// when the recurrence residual reaches tol * ||b|| and confirms it with the
// true residual at every restart (the reading of the paper's unstated GMRES
// settings).
//
// Newton (Sec. 2.4.2): Phi = Phi_L + Phi_NL, d = b - A Phi - N(u), solve
// (A + J) Delta = d, Phi_NL += omega Delta, e_k = omega ||Delta||_2 < Tol_NL.
// The first step uses the cubic Taylor scheme T3, later steps sinh (T3-HS).
// omega is the root of f_d (eq. fd=0) found by Newton's method with the
// derivative of App. A (second derivative r'' = -H[Delta], the minus sign the
// printed formula drops), started at 2 in the T3 step and 1 afterwards,
// clamped to [omega_min, omega_max]; it is frozen once e_k < L_e and the GMRES
// tolerance is tightened tenfold per step once e_k < 1250 tol (App. B).
#include <algorithm>
#include <chrono>
#include <cmath>

#include "pbfb_internal.hpp"

namespace pbfb {

void vec_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void vec_mul(int64_t n, const double *a, const double *x, double *y, hipStream_t s);
void vec_add(int64_t n, const double *a, const double *b, double *y, hipStream_t s);
void vec_scale_dev(int64_t n, const double *num, const double *x, double *y, hipStream_t s);
void basis_dots(int64_t n, int k, const double *Vb, int64_t ldv, const double *w, double *part, int kmax, double *h,
                hipStream_t s);
void basis_sub(int64_t n, int k, const double *Vb, int64_t ldv, const double *h, double *w, hipStream_t s);
void basis_update(int64_t n, int k, const double *Vb, int64_t ldv, const double *y, const double *dinv, double *x,
                  hipStream_t s);
void sq_norm_dev(Problem &p, int64_t n, const double *x, double *out_dev, hipStream_t s);

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

static void build_precond(Problem &p, double *dinv, hipStream_t s)
{
    hipLaunchKernelGGL(k_precond, dim3(nbk(p.n(), 256)), dim3(256), 0, s, p.nn, p.surf[0].nv, p.surf[1].nv, p.d_val,
                       p.d_diag, p.surf[0].vdiag, p.surf[1].vdiag, dinv);
}

// Solve J x = b with the current CSR values (d_val) and preconditioner dinv.
static int gmres_core(Problem &p, const double *dinv, const double *b, double *x, double tol, int m, int maxit,
                      int *iters, hipStream_t s)
{
    const int64_t n = p.n();
    double *Vb = scratch<double>(p, SCR_BASIS, size_t(m + 1) * n);
    double *w = scratch<double>(p, SCR_G0, n);
    double *z = scratch<double>(p, SCR_G1, n);
    double *hv = scratch<double>(p, SCR_HVEC, 2 * (m + 1) + 2 + m);
    double *part = scratch<double>(p, SCR_HPART, size_t(128) * (m + 1));
    double *h1 = hv, *h2 = hv + (m + 1), *nrm2 = hv + 2 * (m + 1), *ydev = hv + 2 * (m + 1) + 2;
    std::vector<double> H(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), hh(2 * (m + 1) + 1), y(m);
    PB_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    const double bnorm = std::sqrt(dot(p, b, b, n, s));
    *iters = 0;
    if (!(bnorm == bnorm)) return PBFB_ENAN;
    if (bnorm == 0.0) return 0;
    const double target = tol * bnorm;
    int total = 0;
    bool fresh = true;
    for (;;) {
        // true residual into the first basis slot
        if (fresh) {
            PB_HIP(hipMemcpyAsync(Vb, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        } else {
            coupled_apply(p, x, w, s);
            PB_HIP(hipMemcpyAsync(Vb, b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            vec_axpby(n, -1.0, w, 1.0, Vb, s);
        }
        fresh = false;
        const double beta = std::sqrt(dot(p, Vb, Vb, n, s));
        if (!(beta == beta)) return PBFB_ENAN;
        if (beta <= target) break;
        if (total >= maxit) {
            *iters = total;
            return PBFB_ENOTCONV;
        }
        vec_axpby(n, 1.0 / beta, Vb, 0.0, Vb, s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int j = 0;
        while (j < m && total < maxit) {
            double *vj = Vb + size_t(j) * n, *vn = Vb + size_t(j + 1) * n;
            vec_mul(n, dinv, vj, z, s);
            coupled_apply(p, z, w, s);
            ++total;
            basis_dots(n, j + 1, Vb, n, w, part, m + 1, h1, s);
            basis_sub(n, j + 1, Vb, n, h1, w, s);
            basis_dots(n, j + 1, Vb, n, w, part, m + 1, h2, s);
            basis_sub(n, j + 1, Vb, n, h2, w, s);
            sq_norm_dev(p, n, w, nrm2, s);
            vec_scale_dev(n, nrm2, w, vn, s);
            PB_HIP(hipMemcpyAsync(hh.data(), hv, sizeof(double) * (2 * (m + 1) + 1), hipMemcpyDeviceToHost, s));
            PB_HIP(hipStreamSynchronize(s));
            for (int i = 0; i <= j; ++i) H[size_t(i) * m + j] = hh[i] + hh[m + 1 + i];
            const double hn = std::sqrt(hh[2 * (m + 1)]);
            H[size_t(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {
                const double a = H[size_t(i) * m + j], c = H[size_t(i + 1) * m + j];
                H[size_t(i) * m + j] = cs[i] * a + sn[i] * c;
                H[size_t(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[size_t(j) * m + j], c = H[size_t(j + 1) * m + j];
            const double den = std::hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[size_t(j) * m + j] = den;
            H[size_t(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++j;
            if (!(g[j] == g[j])) return PBFB_ENAN;
            if (std::fabs(g[j]) <= target || hn == 0.0) break;
        }
        for (int i = j - 1; i >= 0; --i) {
            double sacc = g[i];
            for (int k = i + 1; k < j; ++k) sacc -= H[size_t(i) * m + k] * y[k];
            y[i] = sacc / H[size_t(i) * m + i];
        }
        PB_HIP(hipMemcpyAsync(ydev, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
        basis_update(n, j, Vb, n, ydev, dinv, x, s);
    }
    *iters = total;
    return 0;
}

int gmres(Problem &p, int scheme, const double *u, const double *b, double *x, double tol, int restart, int maxit,
          int *iters, hipStream_t s)
{
    fem_assemble_jacobian(p, scheme, u, s);
    double *dinv = scratch<double>(p, SCR_G2, p.n());
    build_precond(p, dinv, s);
    return gmres_core(p, dinv, b, x, tol, restart, maxit, iters, s);
}

pbfb_status solve(Problem &p, const pbfb_solve_opts &o, pbfb_result &res, double *phi_out_dev, hipStream_t s)
{
    using clk = std::chrono::steady_clock;
    auto t0 = clk::now();
    ensure_all(p, s);
    PB_HIP(hipStreamSynchronize(s));
    auto t1 = clk::now();
    res = pbfb_result{};
    const int64_t n = p.n(), nn = p.nn;
    double *phil = scratch<double>(p, SCR_G3, n);
    double *phinl = scratch<double>(p, SCR_G4, n);
    double *phi = scratch<double>(p, SCR_G5, n);
    double *c = scratch<double>(p, SCR_G6, n);
    double *d = scratch<double>(p, SCR_G7, n);
    double *D = scratch<double>(p, SCR_G8, n);
    double *pv = scratch<double>(p, SCR_G9, n);
    double *rv = scratch<double>(p, SCR_G10, n);
    double *t3 = scratch<double>(p, SCR_G11, 3 * nn);
    double *rN = t3, *rJ = t3 + nn, *rH = t3 + 2 * nn;
    const double *b = p.d_b;

    // 1. linear component: (A + eps_s kappa^2 M) Phi_L = b
    double tol = o.tol_gr0;
    int it = 0;
    PB_HIP(hipMemsetAsync(phinl, 0, sizeof(double) * n, s));
    int st = gmres(p, PBFB_LIN, phinl, b, phil, tol, o.gmres_restart, o.max_gmres, &it, s);
    res.gmres_lin = it;
    res.gmres_iters_total = it;
    int status = st;
    bool frozen = false;
    double omega_last = 1.0;
    int k;
    for (k = 1; k <= o.max_newton && status == 0; ++k) {
        const int sch = (k == 1 && o.scheme_first == PBFB_T3) ? PBFB_T3 : PBFB_HS;
        const int idx = std::min(k - 1, 63);
        vec_add(n, phil, phinl, phi, s);
        // c = b - A Phi ; d = c - [N(u); 0; 0]
        coupled_apply_linear(p, phi, c, s);
        vec_axpby(n, 1.0, b, -1.0, c, s);
        fem_nonlinear(p, sch, phi, rN, s);
        PB_HIP(hipMemcpyAsync(d, c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL(k_sub_fem, dim3(nbk(nn, 256)), dim3(256), 0, s, nn, c, rN, d);
        const double dd = dot(p, d, d, n, s);
        if (!std::isfinite(dd)) {
            status = PBFB_ENAN;
            break;
        }
        st = gmres(p, sch, phi, d, D, tol, o.gmres_restart, o.max_gmres, &it, s);
        res.gmres_iters[idx] = it;
        res.gmres_iters_total += it;
        if (st) {
            status = st;
            break;
        }
        double omega;
        int oit = 0;
        if (!o.omega_auto) {
            omega = o.omega_fixed;
        } else if (frozen) {
            omega = omega_last;
        } else {
            omega = sch == PBFB_T3 ? o.omega0_first : o.omega0_next;
            coupled_apply_linear(p, D, pv, s);
            vec_axpby(n, -1.0, pv, 0.0, pv, s);
            const double pp = dot(p, pv, pv, n, s);
            PB_HIP(hipMemcpyAsync(rv, c, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            for (oit = 0; oit < o.max_omega_it; ++oit) {
                fem_omega_terms(p, sch, phi, D, omega, rN, rJ, rH, s);
                hipLaunchKernelGGL(k_sub_fem, dim3(nbk(nn, 256)), dim3(256), 0, s, nn, c, rN, rv);
                const double pr = dot(p, pv, rv, n, s);
                const double *A5[5] = {rJ, rJ, rJ, rv, pv};
                const double *B5[5] = {rv, pv, rJ, rH, rH};
                double v5[5];
                dots(p, 5, A5, B5, nn, v5, s);
                // r' = -[rJ;0;0], r'' = -[rH;0;0]
                const double a = pr - v5[0];
                const double beta = pp - v5[1];
                if (beta == 0.0) {
                    omega = 1.0;
                    break;
                }
                const double fd = -a / beta - omega;
                if (std::fabs(fd) < o.tol_omega) break;
                const double dfd = -(-v5[1] + v5[2] - v5[3]) / beta + a * (-v5[4]) / (beta * beta) - 1.0;
                if (dfd == 0.0 || !std::isfinite(dfd)) {
                    omega = 1.0;
                    break;
                }
                omega -= fd / dfd;
                omega = std::min(o.omega_max, std::max(o.omega_min, omega));
            }
            omega_last = omega;
        }
        vec_axpby(n, omega, D, 1.0, phinl, s);
        const double ek = omega * std::sqrt(dot(p, D, D, n, s));
        res.omega[idx] = omega;
        res.e_k[idx] = ek;
        res.omega_iters[idx] = oit;
        if (!std::isfinite(ek)) {
            status = PBFB_ENAN;
            break;
        }
        if (o.l_e > 0 && ek < o.l_e) frozen = true;
        if (o.tol_gr0 > o.tol_gr && ek < 1250.0 * tol) tol = std::max(o.tol_gr, 0.1 * tol);
        if (ek < o.tol_nl) {
            ++k;
            break;
        }
        if (k == o.max_newton) status = PBFB_ENOTCONV;
    }
    res.newton_iters = k - 1;
    double en[4];
    energy(p, phil, phinl, en, s);
    res.total = en[0];
    res.lc = en[1];
    res.nc = en[2];
    res.dg_omega_i = en[3];
    if (phi_out_dev) {
        PB_HIP(hipMemcpyAsync(phi_out_dev, phil, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        PB_HIP(hipMemcpyAsync(phi_out_dev + n, phinl, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    PB_HIP(hipStreamSynchronize(s));
    auto t2 = clk::now();
    res.t_setup_s = std::chrono::duration<double>(t1 - t0).count();
    res.t_solve_s = std::chrono::duration<double>(t2 - t1).count();
    res.status = pbfb_status(status);
    return res.status;
}

} // namespace pbfb
