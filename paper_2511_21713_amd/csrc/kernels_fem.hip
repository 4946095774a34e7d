// Geometry, shell FEM (stiffness, reaction terms by row gather), surface mass
// coupling, Coulomb load, charge validation and the solvation energy pieces.
//
// Every FEM kernel is "row owned": one thread per FEM node visits the tets
// around that node and adds the node's own row/entry, so no two threads ever
// write the same value (deterministic, no atomics).  Each tet is therefore
// evaluated once per corner; the reaction terms are cheap beside the coupled
// apply, so the 4x redundancy is a good trade for determinism.
#include <cmath>

#include "pbfb_internal.hpp"

namespace pbfb {

struct TetRuleArg {
    double b[27][4];
    double w[27];
};
struct TriRuleArg {
    double b[6][3];
    double w[6];
};

static TetRuleArg tet_rule_arg()
{
    TetRuleArg r;
    const Rules &R = rules();
    for (int q = 0; q < 27; ++q) {
        for (int k = 0; k < 4; ++k) r.b[q][k] = R.tet_bary[q][k];
        r.w[q] = R.tet_w[q];
    }
    return r;
}
static TriRuleArg tri_rule_arg()
{
    TriRuleArg r;
    const Rules &R = rules();
    for (int q = 0; q < 6; ++q) {
        for (int k = 0; k < 3; ++k) r.b[q][k] = R.tri_bary[q][k];
        r.w[q] = R.tri_w[q];
    }
    return r;
}

static inline unsigned nblocks(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
// Per tet: gradients of the four barycentric functions (rows of B^{-1} for
// B = [x1-x0, x2-x0, x3-x0], the first one minus their sum) and |T|.
__global__ void k_tet_geom(int64_t nt, const double *__restrict__ x, const int32_t *__restrict__ tet,
                           double *__restrict__ tg, int *__restrict__ bad)
{
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    const int32_t *T = tet + 4 * t;
    double B[3][3];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) B[d][k] = x[3 * T[k + 1] + d] - x[3 * T[0] + d];
    double c00 = B[1][1] * B[2][2] - B[1][2] * B[2][1];
    double c01 = B[1][2] * B[2][0] - B[1][0] * B[2][2];
    double c02 = B[1][0] * B[2][1] - B[1][1] * B[2][0];
    double det = B[0][0] * c00 + B[0][1] * c01 + B[0][2] * c02;
    double *o = tg + 16 * t;
    double scale = fabs(B[0][0]) + fabs(B[1][1]) + fabs(B[2][2]) + fabs(B[0][1]) + fabs(B[1][0]);
    if (!(fabs(det) > 1e-12 * scale * scale * scale)) atomicOr(bad, 1);
    double id = 1.0 / det;
    double inv[3][3];
    inv[0][0] = c00 * id;
    inv[0][1] = (B[0][2] * B[2][1] - B[0][1] * B[2][2]) * id;
    inv[0][2] = (B[0][1] * B[1][2] - B[0][2] * B[1][1]) * id;
    inv[1][0] = c01 * id;
    inv[1][1] = (B[0][0] * B[2][2] - B[0][2] * B[2][0]) * id;
    inv[1][2] = (B[0][2] * B[1][0] - B[0][0] * B[1][2]) * id;
    inv[2][0] = c02 * id;
    inv[2][1] = (B[0][1] * B[2][0] - B[0][0] * B[2][1]) * id;
    inv[2][2] = (B[0][0] * B[1][1] - B[0][1] * B[1][0]) * id;
    for (int d = 0; d < 3; ++d) {
        o[3 + d] = inv[0][d];
        o[6 + d] = inv[1][d];
        o[9 + d] = inv[2][d];
        o[d] = -inv[0][d] - inv[1][d] - inv[2][d];
    }
    o[12] = fabs(det) / 6.0;
    o[13] = o[14] = o[15] = 0.0;
}

// Per surface triangle: area, unit normal (right-hand rule of the given
// orientation) and the six quadrature points of the degree-4 rule.
__global__ void k_tri_geom(int64_t nt, const double *__restrict__ x, const int32_t *__restrict__ g,
                           const int32_t *__restrict__ tri, TriRuleArg R, double *__restrict__ qp,
                           double *__restrict__ nrm, double *__restrict__ area, int *__restrict__ bad)
{
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    double P[3][3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) P[a][d] = x[3 * g[tri[3 * t + a]] + d];
    double e1[3], e2[3], n[3];
    for (int d = 0; d < 3; ++d) {
        e1[d] = P[1][d] - P[0][d];
        e2[d] = P[2][d] - P[0][d];
    }
    n[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n[2] = e1[0] * e2[1] - e1[1] * e2[0];
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    double l1 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    if (!(len > 1e-12 * l1)) atomicOr(bad, 2);
    area[t] = 0.5 * len;
    for (int d = 0; d < 3; ++d) nrm[3 * t + d] = n[d] / len;
    for (int q = 0; q < 6; ++q)
        for (int d = 0; d < 3; ++d)
            qp[18 * t + 3 * q + d] = R.b[q][0] * P[0][d] + R.b[q][1] * P[1][d] + R.b[q][2] * P[2][d];
}

// Signed volume enclosed by a closed surface, (1/3) sum_t |t| n_t . c_t (the
// divergence theorem for the field x / 3; c_t the centroid): positive when
// every right-hand normal points away from the enclosed region.  One
// workgroup, strided partial sums added in a fixed tree.
__global__ void __launch_bounds__(256) k_enclosed_volume(int64_t nt, const double *__restrict__ x,
                                                         const int32_t *__restrict__ g, const int32_t *__restrict__ tri,
                                                         const double *__restrict__ nrm, const double *__restrict__ area,
                                                         double *__restrict__ vol)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < nt; t += 256) {
        double c[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) c[d] += x[3 * g[tri[3 * t + a]] + d];
        s += area[t] * (nrm[3 * t] * c[0] + nrm[3 * t + 1] * c[1] + nrm[3 * t + 2] * c[2]) / 9.0;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *vol = red[0];
}

// ---------------------------------------------------------------------------
// stiffness and coupling values (row gather)
// ---------------------------------------------------------------------------
__global__ void k_stiffness(int64_t nn, const int32_t *__restrict__ n2t_ptr, const int32_t *__restrict__ n2t,
                            const int32_t *__restrict__ slot4, const double *__restrict__ tg, double eps_s,
                            int64_t nt_i, double eps_m, double *__restrict__ val0)
{
    int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (a >= nn) return;
    for (int32_t e = n2t_ptr[a]; e < n2t_ptr[a + 1]; ++e) {
        int32_t t = n2t[e] >> 2, la = n2t[e] & 3;
        const double *G = tg + 16 * int64_t(t);
        const double vol = G[12], eps = t < nt_i ? eps_s : eps_m; // tets from nt_i on: solute
        for (int b = 0; b < 4; ++b) {
            double gg = G[3 * la] * G[3 * b] + G[3 * la + 1] * G[3 * b + 1] + G[3 * la + 2] * G[3 * b + 2];
            val0[slot4[4 * int64_t(e) + b]] += eps * vol * gg;
        }
    }
}

// Surface mass coupling of the FEM rows: coef * |tau| (1 + delta_ab) / 12,
// coef = eps_m on Gamma_m and -eps_s on Gamma_s (normal flux terms of the
// shell weak form).
__global__ void k_surface_coupling(int64_t nv, const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                                   const double *__restrict__ area, const int32_t *__restrict__ cslot, double coef,
                                   double *__restrict__ val0)
{
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    for (int32_t e = v2t_ptr[i]; e < v2t_ptr[i + 1]; ++e) {
        int32_t t = v2t[e] / 3, a = v2t[e] % 3;
        for (int b = 0; b < 3; ++b) val0[cslot[3 * int64_t(e) + b]] += coef * area[t] * (a == b ? 2.0 : 1.0) / 12.0;
    }
}

// ---------------------------------------------------------------------------
// reaction terms: calN, calN', calN'' for LIN / T3 / T5 / T7 / HS
// ---------------------------------------------------------------------------
// sinh and cosh together: below 1/2 in magnitude from their Taylor series
// (terms through t^15 and t^16, remainder below 1e-19 relative), above from
// one exponential (cancellation in e - 1/e costs at most a factor 2.2 there)
__device__ inline void sinh_cosh(double t, double &sh, double &ch)
{
    const double a = fabs(t);
    if (a < 0.5) {
        const double t2 = t * t;
        sh = t * (1.0 + t2 * (1.0 / 6.0) *
                            (1.0 + t2 * (1.0 / 20.0) *
                                       (1.0 + t2 * (1.0 / 42.0) *
                                                  (1.0 + t2 * (1.0 / 72.0) *
                                                             (1.0 + t2 * (1.0 / 110.0) *
                                                                        (1.0 + t2 * (1.0 / 156.0) *
                                                                                   (1.0 + t2 * (1.0 / 210.0))))))));
        ch = 1.0 + t2 * 0.5 *
                       (1.0 + t2 * (1.0 / 12.0) *
                                  (1.0 + t2 * (1.0 / 30.0) *
                                             (1.0 + t2 * (1.0 / 56.0) *
                                                        (1.0 + t2 * (1.0 / 90.0) *
                                                                   (1.0 + t2 * (1.0 / 132.0) *
                                                                              (1.0 + t2 * (1.0 / 182.0) *
                                                                                         (1.0 + t2 * (1.0 / 240.0))))))));
    } else {
        const double e = exp(a), ei = 1.0 / e;
        ch = 0.5 * (e + ei);
        sh = copysign(0.5 * (e - ei), t);
    }
}

__device__ inline void scheme_eval(int s, double t, double &f0, double &f1, double &f2)
{
    if (s == PBFB_LIN) {
        f0 = t;
        f1 = 1.0;
        f2 = 0.0;
    } else if (s == PBFB_T3 || s == PBFB_T5 || s == PBFB_T7) {
        // truncated sinh series: f0 through t^o / o!, f1 = f0' through
        // t^(o-1) / (o-1)!, f2 = f0'' through t^(o-2) / (o-2)!  (o = 3, 5, 7)
        const bool o5 = s != PBFB_T3, o7 = s == PBFB_T7;
        const double t2 = t * t;
        const double a5 = o5 ? t2 * (1.0 / 20.0) * (1.0 + (o7 ? t2 * (1.0 / 42.0) : 0.0)) : 0.0;
        f0 = t * (1.0 + t2 * (1.0 / 6.0) * (1.0 + a5));
        const double a4 = o5 ? t2 * (1.0 / 12.0) * (1.0 + (o7 ? t2 * (1.0 / 30.0) : 0.0)) : 0.0;
        f1 = 1.0 + t2 * 0.5 * (1.0 + a4);
        f2 = t * (1.0 + (o5 ? t2 * (1.0 / 6.0) * (1.0 + (o7 ? t2 * (1.0 / 20.0) : 0.0)) : 0.0));
    } else {
        sinh_cosh(t, f0, f1);
        f2 = f0;
    }
}

// Element pass of the reaction terms: each tet evaluates the 27-point rule
// once and leaves its contributions to its four nodes (row gathers below add
// them up in a fixed order, so no atomics are needed).
//   MODE_N: N_a           = c sum_q w_q |T| calN(u_h)  phi_a                 (4 per tet)
//   MODE_W: N_a, J_a, H_a at u + omega D: calN, calN' D_h, calN'' D_h^2        (12 per tet)
//   MODE_J: J_ab          = c sum_q w_q |T| calN'(u_h) phi_a phi_b           (16 per tet)
enum { MODE_N = 0, MODE_W = 1, MODE_J = 2 };
template <int MODE>
__global__ void __launch_bounds__(128)
    k_tet_reaction(int64_t ntet, const double *__restrict__ tg, const int32_t *__restrict__ tet,
                   const double *__restrict__ u, const double *__restrict__ D, double omega, int scheme, double c,
                   TetRuleArg R, int64_t nt_i, double *__restrict__ out, const double *__restrict__ wdev,
                   const int *__restrict__ skip)
{
    // MODE_W: omega from wdev when given (a search on the device); skip: optional flag, nonzero = nothing to do
    if (skip && *skip) return;
    if (MODE == MODE_W && wdev) omega = *wdev;
    const int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= ntet) return;
    constexpr int NZ = MODE == MODE_N ? 4 : MODE == MODE_W ? 12 : 16;
    if (t >= nt_i) { // solute tet: no reaction term, and calN is never evaluated there
#pragma unroll
        for (int k = 0; k < NZ; ++k) out[NZ * t + k] = 0.0;
        return;
    }
    const int32_t *T = tet + 4 * t;
    double uk[4], dk[4] = {0, 0, 0, 0};
    for (int k = 0; k < 4; ++k) {
        if (MODE == MODE_W) dk[k] = D[T[k]];
        uk[k] = u[T[k]] + (MODE == MODE_W ? omega * dk[k] : 0.0);
    }
    const double cv = c * tg[16 * t + 12];
    constexpr int NO = MODE == MODE_N ? 4 : MODE == MODE_W ? 12 : 16;
    double acc[NO];
#pragma unroll
    for (int k = 0; k < NO; ++k) acc[k] = 0.0;
    for (int q = 0; q < 27; ++q) {
        const double uh = R.b[q][0] * uk[0] + R.b[q][1] * uk[1] + R.b[q][2] * uk[2] + R.b[q][3] * uk[3];
        double f0, f1, f2;
        scheme_eval(scheme, uh, f0, f1, f2);
        if (MODE == MODE_N) {
#pragma unroll
            for (int a = 0; a < 4; ++a) acc[a] += cv * R.w[q] * f0 * R.b[q][a];
        } else if (MODE == MODE_W) {
            const double dh = R.b[q][0] * dk[0] + R.b[q][1] * dk[1] + R.b[q][2] * dk[2] + R.b[q][3] * dk[3];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double w = cv * R.w[q] * R.b[q][a];
                acc[a] += w * f0;
                acc[4 + a] += w * f1 * dh;
                acc[8 + a] += w * f2 * dh * dh;
            }
        } else {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double wq = cv * R.w[q] * f1 * R.b[q][a];
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[4 * a + b] += wq * R.b[q][b];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NO; ++k) out[NO * t + k] = acc[k];
}

// d_val = d_val0 + J_scheme(u) on the u columns of each FEM row, from the
// element blocks (16 per tet), row by row (Jt null: d_val = d_val0, the
// operator without reaction term); the copy covers the slice padding (zero
// in d_val0) and is coalesced across the rows of a slice
__global__ void k_jacobian(int64_t nn, const int32_t *__restrict__ sptr, const double *__restrict__ val0,
                           double *__restrict__ val, float *__restrict__ val32, const int32_t *__restrict__ n2t_ptr,
                           const int32_t *__restrict__ n2t, const int32_t *__restrict__ slot4,
                           const double *__restrict__ Jt)
{
    int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (a >= nn) return;
    const int64_t q = a / SLICE;
    const int32_t b0 = sptr[q] + int32_t(a - q * SLICE), b1 = sptr[q + 1];
    for (int32_t s = b0; s < b1; s += SLICE) val[s] = val0[s];
    if (Jt)
        for (int32_t e = n2t_ptr[a]; e < n2t_ptr[a + 1]; ++e) {
            const int64_t t = n2t[e] >> 2;
            const int la = n2t[e] & 3;
            for (int b = 0; b < 4; ++b) val[slot4[4 * int64_t(e) + b]] += Jt[16 * t + 4 * la + b];
        }
    if (val32)
        for (int32_t s = b0; s < b1; s += SLICE) val32[s] = float(val[s]);
}

// out_k[a] = sum over the tets at node a of their contribution k to a (K per tet and node)
template <int K>
__global__ void k_node_gather(int64_t nn, const int32_t *__restrict__ n2t_ptr, const int32_t *__restrict__ n2t,
                              const double *__restrict__ per_tet, double *__restrict__ o0, double *__restrict__ o1,
                              double *__restrict__ o2, const int *__restrict__ skip)
{
    if (skip && *skip) return;
    int64_t a = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (a >= nn) return;
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = 0.0;
    for (int32_t e = n2t_ptr[a]; e < n2t_ptr[a + 1]; ++e) {
        const int64_t t = n2t[e] >> 2;
        const int la = n2t[e] & 3;
#pragma unroll
        for (int k = 0; k < K; ++k) s[k] += per_tet[4 * K * t + 4 * k + la];
    }
    o0[a] = s[0];
    if (K > 1) o1[a] = s[1];
    if (K > 2) o2[a] = s[2];
}

// per-tet integral of u sinh u - 2 cosh u + 2 for u = u_lin + u_nl (block partial sums)
__global__ void k_energy_integral(int64_t nt, const double *__restrict__ tg, const int32_t *__restrict__ tet,
                                  const double *__restrict__ ul, const double *__restrict__ unl, TetRuleArg R,
                                  double *__restrict__ partial)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < nt; t += int64_t(gridDim.x) * blockDim.x) {
        const int32_t *T = tet + 4 * t;
        double uk[4];
        for (int k = 0; k < 4; ++k) uk[k] = ul[T[k]] + (unl ? unl[T[k]] : 0.0);
        double vol = tg[16 * t + 12];
        for (int q = 0; q < 27; ++q) {
            double uh = R.b[q][0] * uk[0] + R.b[q][1] * uk[1] + R.b[q][2] * uk[2] + R.b[q][3] * uk[3];
            double f;
            if (fabs(uh) < 0.5) {
                // sum_k u^{2k} (2k-2)/(2k)!, k = 2..8, where the closed form cancels
                double u2 = uh * uh;
                f = u2 * u2 *
                    (1.0 / 12.0 +
                     u2 * (1.0 / 180.0 +
                           u2 * (1.0 / 6720.0 +
                                 u2 * (1.0 / 453600.0 +
                                       u2 * (1.0 / 47900160.0 +
                                             u2 * (1.0 / 7264857600.0 + u2 * (1.0 / 1494484992000.0)))))));
            } else {
                f = uh * sinh(uh) - 2.0 * cosh(uh) + 2.0;
            }
            s += vol * R.w[q] * f;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// Point-charge load of the two-field form (Sec. 2.3): b_a = sum_k Q_k phi_a(x_k),
// Q_k = 4 pi l_B z_k.  One workgroup per charge finds the solute tet whose
// smallest barycentric coordinate of x_k is largest (ties: the lower tet id);
// one thread then adds the charges in order, so the sum is deterministic.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_point_locate(int64_t nt0, int64_t nt, const double *__restrict__ x,
                                                      const int32_t *__restrict__ tet, const double *__restrict__ tg,
                                                      const double *__restrict__ q, double *__restrict__ loc)
{
    __shared__ double sv[256];
    __shared__ int64_t st[256];
    const int64_t k = blockIdx.x;
    const double xk[3] = {q[4 * k], q[4 * k + 1], q[4 * k + 2]};
    double best = -1e300;
    int64_t bt = -1;
    for (int64_t t = nt0 + threadIdx.x; t < nt; t += 256) {
        const double *G = tg + 16 * t, *x0 = x + 3 * int64_t(tet[4 * t]);
        const double d[3] = {xk[0] - x0[0], xk[1] - x0[1], xk[2] - x0[2]};
        double lo = 1e300;
        for (int a = 0; a < 4; ++a)
            lo = fmin(lo, (a == 0 ? 1.0 : 0.0) + G[3 * a] * d[0] + G[3 * a + 1] * d[1] + G[3 * a + 2] * d[2]);
        if (lo > best) { best = lo; bt = t; }
    }
    sv[threadIdx.x] = best;
    st[threadIdx.x] = bt;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double o = sv[threadIdx.x + w];
            const int64_t ot = st[threadIdx.x + w];
            if (o > sv[threadIdx.x] || (o == sv[threadIdx.x] && ot >= 0 && (st[threadIdx.x] < 0 || ot < st[threadIdx.x]))) {
                sv[threadIdx.x] = o;
                st[threadIdx.x] = ot;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t t = st[0];
        loc[6 * k] = double(t);
        loc[6 * k + 1] = sv[0];
        if (t >= 0) {
            const double *G = tg + 16 * t, *x0 = x + 3 * int64_t(tet[4 * t]);
            const double d[3] = {xk[0] - x0[0], xk[1] - x0[1], xk[2] - x0[2]};
            for (int a = 0; a < 4; ++a)
                loc[6 * k + 2 + a] = (a == 0 ? 1.0 : 0.0) + G[3 * a] * d[0] + G[3 * a + 1] * d[1] + G[3 * a + 2] * d[2];
        }
    }
}

// the vertices of a surface as points for k_point_locate (x, y, z, 0)
__global__ void k_surface_points(int64_t nv, const double *__restrict__ x, const int32_t *__restrict__ g,
                                 double *__restrict__ pts)
{
    const int64_t v = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (v >= nv) return;
    for (int d = 0; d < 3; ++d) pts[4 * v + d] = x[3 * int64_t(g[v]) + d];
    pts[4 * v + 3] = 0.0;
}

__global__ void k_point_scatter(int64_t nq, const int32_t *__restrict__ tet, const double *__restrict__ q,
                                const double *__restrict__ loc, double qscale, double *__restrict__ b)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int64_t k = 0; k < nq; ++k) {
        const int64_t t = int64_t(loc[6 * k]);
        for (int a = 0; a < 4; ++a) b[tet[4 * t + a]] += qscale * q[4 * k + 3] * loc[6 * k + 2 + a];
    }
}

// ---------------------------------------------------------------------------
// Coulomb load f_i = int_{Gamma_m} phi_i sum_k l_B z_k / (eps_m |x - x_k|)
// ---------------------------------------------------------------------------
__global__ void k_coulomb_tri(int64_t nt, const double *__restrict__ qp, const double *__restrict__ area,
                              const double *__restrict__ q, int64_t nq, double scale, TriRuleArg R,
                              double *__restrict__ trif)
{
    int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (t >= nt) return;
    double acc[3] = {0, 0, 0};
    for (int p = 0; p < 6; ++p) {
        const double *y = qp + 18 * t + 3 * p;
        double s = 0.0;
        for (int64_t k = 0; k < nq; ++k) {
            double dx = y[0] - q[4 * k], dy = y[1] - q[4 * k + 1], dz = y[2] - q[4 * k + 2];
            s += q[4 * k + 3] * rsqrt(dx * dx + dy * dy + dz * dz);
        }
        double w = area[t] * R.w[p] * scale * s;
        for (int a = 0; a < 3; ++a) acc[a] += w * R.b[p][a];
    }
    for (int a = 0; a < 3; ++a) trif[3 * t + a] = acc[a];
}

__global__ void k_gather_vertex(int64_t nv, const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                                const double *__restrict__ trif, double *__restrict__ f)
{
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    double s = 0.0;
    for (int32_t e = v2t_ptr[i]; e < v2t_ptr[i + 1]; ++e) s += trif[v2t[e]];
    f[i] = s;
}

// ---------------------------------------------------------------------------
// reaction potential at the charges (eq. Potential_in_Omega_m):
// u_r(x) = int [g0(x,y) lambda_m(y) - dg0/dn_y(x,y) u(y)] dy over Gamma_m
// one block per charge; two densities (Phi_L and Phi_NL) at once
// ---------------------------------------------------------------------------
// u_r(x_k) = (V lam)(x_k) - (K u)(x_k) over Gamma_m (eq. Potential_in_Omega_m) for
// two fields at once (Phi_L, Phi_NL); lam0 / lam1: lambda_m per surface
// vertex; the trace of u0 / u1 at vertex v is u[g[v]], or on an independent
// Gamma_m mesh (loc non-null: tet and barycentric coordinates per vertex,
// 6 doubles) the P1 interpolant.
__device__ inline double surface_trace(const double *__restrict__ u, int32_t v, const int32_t *__restrict__ g,
                                       const double *__restrict__ loc, const int32_t *__restrict__ tet)
{
    if (!loc) return u[g[v]];
    const double *l = loc + 6 * int64_t(v);
    const int32_t *T = tet + 4 * int64_t(l[0]);
    return l[2] * u[T[0]] + l[3] * u[T[1]] + l[4] * u[T[2]] + l[5] * u[T[3]];
}

__global__ void k_reaction_potential(int64_t nt, const double *__restrict__ qp, const double *__restrict__ nrm,
                                     const double *__restrict__ area, const int32_t *__restrict__ tri,
                                     const int32_t *__restrict__ g, const double *__restrict__ loc,
                                     const int32_t *__restrict__ tet, const double *__restrict__ q,
                                     const double *__restrict__ phi0, const double *__restrict__ lam0,
                                     const double *__restrict__ phi1, const double *__restrict__ lam1, TriRuleArg R,
                                     double *__restrict__ out)
{
    __shared__ double r0[256], r1[256];
    int64_t k = blockIdx.x;
    double xk[3] = {q[4 * k], q[4 * k + 1], q[4 * k + 2]};
    double s0 = 0.0, s1 = 0.0;
    const double inv4pi = 0.07957747154594767;
    for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) {
        int32_t v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        double l0[3], u0[3], l1[3], u1[3];
        for (int a = 0; a < 3; ++a) {
            l0[a] = lam0[v[a]];
            u0[a] = surface_trace(phi0, v[a], g, loc, tet);
            l1[a] = phi1 ? lam1[v[a]] : 0.0;
            u1[a] = phi1 ? surface_trace(phi1, v[a], g, loc, tet) : 0.0;
        }
        const double *n = nrm + 3 * t;
        for (int p = 0; p < 6; ++p) {
            const double *y = qp + 18 * t + 3 * p;
            double d[3] = {xk[0] - y[0], xk[1] - y[1], xk[2] - y[2]};
            double rinv = rsqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double gk = inv4pi * rinv;
            double dg = inv4pi * (d[0] * n[0] + d[1] * n[1] + d[2] * n[2]) * rinv * rinv * rinv;
            double w = area[t] * R.w[p];
            double lh0 = R.b[p][0] * l0[0] + R.b[p][1] * l0[1] + R.b[p][2] * l0[2];
            double uh0 = R.b[p][0] * u0[0] + R.b[p][1] * u0[1] + R.b[p][2] * u0[2];
            double lh1 = R.b[p][0] * l1[0] + R.b[p][1] * l1[1] + R.b[p][2] * l1[2];
            double uh1 = R.b[p][0] * u1[0] + R.b[p][1] * u1[1] + R.b[p][2] * u1[2];
            s0 += w * (gk * lh0 - dg * uh0);
            s1 += w * (gk * lh1 - dg * uh1);
        }
    }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            r0[threadIdx.x] += r0[threadIdx.x + w];
            r1[threadIdx.x] += r1[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * k] = r0[0];
        out[2 * k + 1] = r1[0];
    }
}

// charge validation: distance to Gamma_m and solid angle (inside: 4 pi)
__global__ void k_charge_check(int64_t nt, const double *__restrict__ x, const int32_t *__restrict__ g,
                               const int32_t *__restrict__ tri, const double *__restrict__ q, double *__restrict__ out)
{
    __shared__ double dmin[256], sang[256];
    int64_t k = blockIdx.x;
    double p[3] = {q[4 * k], q[4 * k + 1], q[4 * k + 2]};
    double dm = 1e300, sa = 0.0;
    for (int64_t t = threadIdx.x; t < nt; t += blockDim.x) {
        double A[3], B[3], C[3];
        for (int d = 0; d < 3; ++d) {
            A[d] = x[3 * g[tri[3 * t]] + d] - p[d];
            B[d] = x[3 * g[tri[3 * t + 1]] + d] - p[d];
            C[d] = x[3 * g[tri[3 * t + 2]] + d] - p[d];
        }
        // solid angle (Van Oosterom & Strackee)
        double la = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        double lb = sqrt(B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        double lc = sqrt(C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
        double trip = A[0] * (B[1] * C[2] - B[2] * C[1]) - A[1] * (B[0] * C[2] - B[2] * C[0]) +
                      A[2] * (B[0] * C[1] - B[1] * C[0]);
        double den = la * lb * lc + (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]) * lc +
                     (A[0] * C[0] + A[1] * C[1] + A[2] * C[2]) * lb + (B[0] * C[0] + B[1] * C[1] + B[2] * C[2]) * la;
        sa += 2.0 * atan2(trip, den);
        // point-triangle distance: closest point by barycentric clamping (origin = charge)
        double ab[3], ac[3];
        for (int d = 0; d < 3; ++d) {
            ab[d] = B[d] - A[d];
            ac[d] = C[d] - A[d];
        }
        double best = fmin(la, fmin(lb, lc));
        // interior projection
        double nrm[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
        double nn2 = nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2];
        double h = -(A[0] * nrm[0] + A[1] * nrm[1] + A[2] * nrm[2]) / nn2;
        double P0[3] = {h * nrm[0], h * nrm[1], h * nrm[2]}; // projection of the origin on the plane
        double v0[3] = {P0[0] - A[0], P0[1] - A[1], P0[2] - A[2]};
        double d00 = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2], d01 = ab[0] * ac[0] + ab[1] * ac[1] + ab[2] * ac[2];
        double d11 = ac[0] * ac[0] + ac[1] * ac[1] + ac[2] * ac[2];
        double d20 = v0[0] * ab[0] + v0[1] * ab[1] + v0[2] * ab[2], d21 = v0[0] * ac[0] + v0[1] * ac[1] + v0[2] * ac[2];
        double den2 = d00 * d11 - d01 * d01;
        double bv = (d11 * d20 - d01 * d21) / den2, bw = (d00 * d21 - d01 * d20) / den2;
        if (bv >= 0 && bw >= 0 && bv + bw <= 1) best = fmin(best, fabs(h) * sqrt(nn2));
        // edges
        const double *E0[3] = {A, B, C}, *E1[3] = {B, C, A};
        for (int e = 0; e < 3; ++e) {
            double dd[3] = {E1[e][0] - E0[e][0], E1[e][1] - E0[e][1], E1[e][2] - E0[e][2]};
            double L = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
            double s = -(E0[e][0] * dd[0] + E0[e][1] * dd[1] + E0[e][2] * dd[2]) / L;
            if (s > 0 && s < 1) {
                double c[3] = {E0[e][0] + s * dd[0], E0[e][1] + s * dd[1], E0[e][2] + s * dd[2]};
                best = fmin(best, sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]));
            }
        }
        dm = fmin(dm, best);
    }
    dmin[threadIdx.x] = dm;
    sang[threadIdx.x] = sa;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            dmin[threadIdx.x] = fmin(dmin[threadIdx.x], dmin[threadIdx.x + w]);
            sang[threadIdx.x] += sang[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * k] = dmin[0];
        out[2 * k + 1] = sang[0];
    }
}

// ===========================================================================
// host wrappers
// ===========================================================================
// One-time per mesh: upload of the mesh and its integer topology.
void ensure_topology(Problem &p, hipStream_t s)
{
    if (p.topo_ready) return;
    PB_CHECK(p.have_mesh, PBFB_ESTATE, "set_mesh must precede setup");
    Arena &A = p.mesh_arena;
    A.release();
    p.d_x = A.upload(p.x, s);
    p.d_tet = A.upload(p.tet, s);
    std::vector<int32_t> sptr, col, n2t_ptr, n2t, slot4, diag, cslot[2];
    build_fem_topology(p, sptr, col, n2t_ptr, n2t, slot4, diag, cslot);
    p.nnz = int64_t(col.size());
    p.d_sptr = A.upload(sptr, s);
    p.d_col = A.upload(col, s);
    p.d_n2t_ptr = A.upload(n2t_ptr, s);
    p.d_n2t = A.upload(n2t, s);
    p.d_slot4 = A.upload(slot4, s);
    p.d_diag = A.upload(diag, s);
    p.d_tgeo = A.alloc<double>(16 * p.ntet);
    p.d_val0 = A.alloc<double>(p.nnz);
    p.d_val = A.alloc<double>(p.nnz);
    p.d_val32 = p.precision == PBFB_MIXED ? A.alloc<float>(p.nnz) : nullptr;
    p.d_bad = A.alloc<int>(1);
    for (int w = 0; w < NSURF; ++w) {
        SurfaceTopo &T = p.topo[w];
        SurfaceDev &S = p.surf[w];
        S.nv = T.nv;
        S.nt = T.nt;
        S.itet = nullptr;
        S.iw = nullptr;
        if (w == 2 && !p.has_rs()) {
            S.x = nullptr;
            continue;
        }
        // coordinates indexed through g: the FEM nodes, or the independent mesh's own vertices
        S.x = w == 2 ? A.upload(p.rs_x, s) : p.d_x;
        S.g = A.upload(T.g, s);
        S.mvert = A.upload(T.mvert, s);
        S.minv = A.upload(T.minv, s);
        S.gmv = A.upload(T.gmv, s);
        S.tri = A.upload(T.tri, s);
        S.v2t_ptr = A.upload(T.v2t_ptr, s);
        S.v2t = A.upload(T.v2t, s);
        S.qp = A.alloc<double>(18 * T.nt);
        S.nrm = A.alloc<double>(3 * T.nt);
        S.area = A.alloc<double>(T.nt);
        S.cslot = w < 2 ? A.upload(cslot[w], s) : nullptr;
        if (w == 2) S.iw = A.alloc<double>(6 * T.nv);
    }
    PB_HIP(hipStreamSynchronize(s));
    p.topo_ready = true;
}

// Geometry of the tets and surface triangles from the device-resident mesh.
void ensure_geometry(Problem &p, hipStream_t s)
{
    if (p.geom_ready) return;
    PB_CHECK(p.have_mesh && p.have_params, PBFB_ESTATE, "set_mesh and set_params must precede setup");
    ensure_topology(p, s);
    PB_HIP(hipMemsetAsync(p.d_bad, 0, sizeof(int), s));
    hipLaunchKernelGGL(k_tet_geom, dim3(nblocks(p.ntet, 256)), dim3(256), 0, s, p.ntet, p.d_x, p.d_tet, p.d_tgeo,
                       p.d_bad);
    TriRuleArg TR = tri_rule_arg();
    double *d_vol = scratch<double>(p, SCR_VOL, NSURF);
    const int nsurf = p.has_rs() ? 3 : 2;
    for (int w = 0; w < nsurf; ++w) {
        SurfaceDev &S = p.surf[w];
        hipLaunchKernelGGL(k_tri_geom, dim3(nblocks(S.nt, 256)), dim3(256), 0, s, S.nt, S.x, S.g, S.tri, TR, S.qp,
                           S.nrm, S.area, p.d_bad);
        hipLaunchKernelGGL(k_enclosed_volume, dim3(1), dim3(256), 0, s, S.nt, S.x, S.g, S.tri, S.nrm, S.area,
                           d_vol + w);
    }
    if (p.has_rs()) {
        // the tet of the FEM mesh that holds each vertex of the independent
        // Gamma_m mesh, and the vertex's barycentric coordinates there: the
        // trace of u on it is the P1 interpolant (Sec. 2.3.1)
        SurfaceDev &R = p.surf[2];
        double *pts = scratch<double>(p, SCR_RLOC, 4 * R.nv);
        hipLaunchKernelGGL(k_surface_points, dim3(nblocks(R.nv, 256)), dim3(256), 0, s, R.nv, R.x, R.g, pts);
        hipLaunchKernelGGL(k_point_locate, dim3(unsigned(R.nv)), dim3(256), 0, s, int64_t(0), p.ntet, p.d_x, p.d_tet,
                           p.d_tgeo, pts, R.iw);
    }
    int bad = 0;
    double vol[NSURF] = {0.0, 0.0, 0.0};
    PB_HIP(hipMemcpyAsync(&bad, p.d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    PB_HIP(hipMemcpyAsync(vol, d_vol, sizeof(vol), hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    PB_CHECK(!(bad & 1), PBFB_EMESH, "degenerate (zero-volume) tetrahedron");
    PB_CHECK(!(bad & 2), PBFB_EMESH, "degenerate (zero-area) surface triangle");
    // the formulation's normals point away from the solute on both interfaces
    // (the sign of the double layer depends on it): the right-hand normals must
    // enclose a positive volume
    PB_CHECK(vol[0] > 0.0, PBFB_EMESH, "Gamma_m is oriented inward (its right-hand normals enclose a negative volume)");
    PB_CHECK(vol[1] > 0.0, PBFB_EMESH, "Gamma_s is oriented inward (its right-hand normals enclose a negative volume)");
    if (p.has_rs()) {
        PB_CHECK(vol[2] > 0.0, PBFB_EMESH,
                 "the Gamma_m surface mesh is oriented inward (its right-hand normals enclose a negative volume)");
        std::vector<double> loc(6 * p.surf[2].nv);
        PB_HIP(hipMemcpyAsync(loc.data(), p.surf[2].iw, sizeof(double) * loc.size(), hipMemcpyDeviceToHost, s));
        PB_HIP(hipStreamSynchronize(s));
        for (int64_t v = 0; v < p.surf[2].nv; ++v)
            PB_CHECK(loc[6 * v] >= 0 && loc[6 * v + 1] >= -1e-10, PBFB_EMESH,
                     "vertex " + std::to_string(v) + " of the Gamma_m surface mesh lies outside the FEM mesh");
    }
    p.geom_ready = true;
}

// Stiffness and surface-coupling values of the FEM rows (they carry the
// permittivities; the boundary operators do not).
void ensure_values(Problem &p, hipStream_t s)
{
    if (p.val_ready) return;
    ensure_geometry(p, s);
    PB_HIP(hipMemsetAsync(p.d_val0, 0, sizeof(double) * p.nnz, s));
    hipLaunchKernelGGL(k_stiffness, dim3(nblocks(p.nn, 256)), dim3(256), 0, s, p.nn, p.d_n2t_ptr, p.d_n2t,
                       p.d_slot4, p.d_tgeo, p.eps_s, p.ntet_i(), p.eps_m, p.d_val0);
    // the two-field form has Gamma_m inside the FEM domain: no lambda_m columns
    for (int w = p.two_field() ? 1 : 0; w < 2; ++w) {
        SurfaceDev &S = p.surf[w];
        double coef = w == 0 ? p.eps_m : -p.eps_s;
        hipLaunchKernelGGL(k_surface_coupling, dim3(nblocks(S.nv, 256)), dim3(256), 0, s, S.nv, S.v2t_ptr, S.v2t,
                           S.area, S.cslot, coef, p.d_val0);
    }
    PB_HIP(hipGetLastError());
    p.val_ready = true;
}

void ensure_rhs(Problem &p, hipStream_t s)
{
    if (p.fm_ready) return;
    ensure_geometry(p, s);
    PB_CHECK(p.have_charges, PBFB_ESTATE, "set_charges must precede the solve");
    p.d_b = scratch<double>(p, SCR_B, p.n());
    PB_HIP(hipMemsetAsync(p.d_b, 0, sizeof(double) * p.n(), s));
    if (p.nq > 0) {
        p.d_q = scratch<double>(p, SCR_Q, 4 * p.nq);
        PB_HIP(hipMemcpyAsync(p.d_q, p.q.data(), sizeof(double) * 4 * p.nq, hipMemcpyHostToDevice, s));
        SurfaceDev &S = p.surf[0];
        // validation: inside Gamma_m (solid angle 4 pi) and at least 1 A away
        double *d_chk = scratch<double>(p, SCR_CHK, 2 * p.nq);
        hipLaunchKernelGGL(k_charge_check, dim3(unsigned(p.nq)), dim3(256), 0, s, S.nt, p.d_x, S.g, S.tri, p.d_q,
                           d_chk);
        std::vector<double> chk(2 * p.nq);
        PB_HIP(hipMemcpyAsync(chk.data(), d_chk, sizeof(double) * 2 * p.nq, hipMemcpyDeviceToHost, s));
        PB_HIP(hipStreamSynchronize(s));
        for (int64_t k = 0; k < p.nq; ++k) {
            PB_CHECK(chk[2 * k + 1] > 2.0 * M_PI, PBFB_ECHARGE, "charge " + std::to_string(k) + " lies outside Gamma_m");
            PB_CHECK(chk[2 * k] >= 1.0, PBFB_ECHARGE,
                     "charge " + std::to_string(k) + " is closer than 1 A to Gamma_m");
        }
        // the Coulomb load f_m: the Gamma_m rows of b, or (two-field form) kept
        // for the recovery of lambda_m while the point charges load the FEM
        // rows, on the surface that carries lambda_m
        const SurfaceDev &F = p.surf[p.gm()];
        double *trif = scratch<double>(p, SCR_TRIF, 3 * F.nt);
        double *fm = p.two_field() ? scratch<double>(p, SCR_FM, F.nv) : p.d_b + p.nn;
        hipLaunchKernelGGL(k_coulomb_tri, dim3(nblocks(F.nt, 128)), dim3(128), 0, s, F.nt, F.qp, F.area, p.d_q, p.nq,
                           p.lB / p.eps_m, tri_rule_arg(), trif);
        hipLaunchKernelGGL(k_gather_vertex, dim3(nblocks(F.nv, 256)), dim3(256), 0, s, F.nv, F.v2t_ptr, F.v2t, trif,
                           fm);
        if (p.two_field()) {
            double *loc = scratch<double>(p, SCR_PLOC, 6 * p.nq);
            hipLaunchKernelGGL(k_point_locate, dim3(unsigned(p.nq)), dim3(256), 0, s, p.ntet_i(), p.ntet, p.d_x,
                               p.d_tet, p.d_tgeo, p.d_q, loc);
            std::vector<double> h(6 * p.nq);
            PB_HIP(hipMemcpyAsync(h.data(), loc, sizeof(double) * 6 * p.nq, hipMemcpyDeviceToHost, s));
            PB_HIP(hipStreamSynchronize(s));
            for (int64_t k = 0; k < p.nq; ++k)
                PB_CHECK(h[6 * k] >= 0 && h[6 * k + 1] >= -1e-10, PBFB_ECHARGE,
                         "charge " + std::to_string(k) + " lies in no solute tet");
            hipLaunchKernelGGL(k_point_scatter, dim3(1), dim3(64), 0, s, p.nq, p.d_tet, p.d_q, loc,
                               4.0 * M_PI * p.lB, p.d_b);
        }
        PB_HIP(hipGetLastError());
    }
    p.fm_ready = true;
}

void fem_assemble_jacobian(Problem &p, int scheme, const double *u, hipStream_t s)
{
    const double c = p.eps_s * p.kappa * p.kappa;
    double *Jt = scratch<double>(p, SCR_TETR, 16 * size_t(p.ntet));
    hipLaunchKernelGGL(k_tet_reaction<MODE_J>, dim3(nblocks(p.ntet, 128)), dim3(128), 0, s, p.ntet, p.d_tgeo, p.d_tet,
                       u, (const double *)nullptr, 0.0, scheme, c, tet_rule_arg(), p.ntet_i(), Jt,
                       (const double *)nullptr, (const int *)nullptr);
    hipLaunchKernelGGL(k_jacobian, dim3(nblocks(p.nn, 128)), dim3(128), 0, s, p.nn, p.d_sptr, p.d_val0, p.d_val,
                       p.d_val32, p.d_n2t_ptr, p.d_n2t, p.d_slot4, Jt);
    PB_HIP(hipGetLastError());
}

// FEM values of the coupled operator without reaction term (the Picard step)
void fem_assemble_linear(Problem &p, hipStream_t s)
{
    hipLaunchKernelGGL(k_jacobian, dim3(nblocks(p.nn, 128)), dim3(128), 0, s, p.nn, p.d_sptr, p.d_val0, p.d_val,
                       p.d_val32, p.d_n2t_ptr, p.d_n2t, p.d_slot4, (const double *)nullptr);
    PB_HIP(hipGetLastError());
}

void fem_nonlinear(Problem &p, int scheme, const double *u, double *out, hipStream_t s)
{
    fem_nonlinear_buf(p, scheme, u, out, scratch<double>(p, SCR_TETR, 16 * size_t(p.ntet)), s);
}

void fem_nonlinear_buf(Problem &p, int scheme, const double *u, double *out, double *Nt, hipStream_t s)
{
    const double c = p.eps_s * p.kappa * p.kappa;
    hipLaunchKernelGGL(k_tet_reaction<MODE_N>, dim3(nblocks(p.ntet, 128)), dim3(128), 0, s, p.ntet, p.d_tgeo, p.d_tet,
                       u, (const double *)nullptr, 0.0, scheme, c, tet_rule_arg(), p.ntet_i(), Nt,
                       (const double *)nullptr, (const int *)nullptr);
    hipLaunchKernelGGL(k_node_gather<1>, dim3(nblocks(p.nn, 128)), dim3(128), 0, s, p.nn, p.d_n2t_ptr, p.d_n2t, Nt,
                       out, (double *)nullptr, (double *)nullptr, (const int *)nullptr);
    PB_HIP(hipGetLastError());
}

void fem_omega_terms_dev(Problem &p, int scheme, const double *u, const double *D, const double *wdev,
                         const int *skip, double *rN, double *rJ, double *rH, hipStream_t s)
{
    const double c = p.eps_s * p.kappa * p.kappa;
    double *Wt = scratch<double>(p, SCR_TETR, 16 * size_t(p.ntet));
    hipLaunchKernelGGL(k_tet_reaction<MODE_W>, dim3(nblocks(p.ntet, 128)), dim3(128), 0, s, p.ntet, p.d_tgeo, p.d_tet,
                       u, D, 0.0, scheme, c, tet_rule_arg(), p.ntet_i(), Wt, wdev, skip);
    hipLaunchKernelGGL(k_node_gather<3>, dim3(nblocks(p.nn, 128)), dim3(128), 0, s, p.nn, p.d_n2t_ptr, p.d_n2t, Wt,
                       rN, rJ, rH, skip);
    PB_HIP(hipGetLastError());
}

double fem_energy_integral(Problem &p, const double *ul, const double *unl, hipStream_t s)
{
    const int nb = 512;
    double *part = scratch<double>(p, SCR_EPART, nb);
    hipLaunchKernelGGL(k_energy_integral, dim3(nb), dim3(256), 0, s, p.ntet_i(), p.d_tgeo, p.d_tet, ul, unl,
                       tet_rule_arg(), part); // Omega_i: the shell tets come first
    std::vector<double> h(nb);
    PB_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double v : h) sum += v;
    return sum;
}

void energy(Problem &p, const double *phi_lin, const double *phi_nl, double out[4], hipStream_t s)
{
    ensure_rhs(p, s);
    // lambda_m per vertex of the surface that carries it: part of Phi in the
    // three-field form; in the two-field form recovered from the trace of u,
    // with the Coulomb load for the linear part only (Sec. 2.3.1), on the
    // independent Gamma_m mesh when one is set
    const SurfaceDev &S = p.surf[p.gm()];
    const double *lam_l = phi_lin + p.nn, *lam_n = phi_nl ? phi_nl + p.nn : nullptr;
    if (p.two_field()) {
        double *ll = scratch<double>(p, SCR_PL, S.nv);
        lambda_m_recover(p, phi_lin, true, ll, s);
        lam_l = ll;
        if (phi_nl) {
            double *ln = scratch<double>(p, SCR_PN, S.nv);
            lambda_m_recover(p, phi_nl, false, ln, s);
            lam_n = ln;
        }
    }
    double lc = 0.0, nc = 0.0;
    if (p.nq > 0) {
        double *d_ur = scratch<double>(p, SCR_UR, 2 * p.nq);
        hipLaunchKernelGGL(k_reaction_potential, dim3(unsigned(p.nq)), dim3(256), 0, s, S.nt, S.qp, S.nrm, S.area,
                           S.tri, S.g, S.iw, p.d_tet, p.d_q, phi_lin, lam_l, phi_nl, lam_n, tri_rule_arg(), d_ur);
        std::vector<double> ur(2 * p.nq);
        PB_HIP(hipMemcpyAsync(ur.data(), d_ur, sizeof(double) * 2 * p.nq, hipMemcpyDeviceToHost, s));
        PB_HIP(hipStreamSynchronize(s));
        for (int64_t k = 0; k < p.nq; ++k) {
            lc += 0.5 * p.kT * p.q[4 * k + 3] * ur[2 * k];
            nc += 0.5 * p.kT * p.q[4 * k + 3] * ur[2 * k + 1];
        }
    }
    double dg = 0.0;
    if (phi_nl) {
        double integral = fem_energy_integral(p, phi_lin, phi_nl, s);
        dg = p.kT / (4.0 * M_PI * p.lB) * 0.5 * p.eps_s * p.kappa * p.kappa * integral;
    }
    out[0] = lc + nc + dg;
    out[1] = lc;
    out[2] = phi_nl ? nc : 0.0;
    out[3] = dg;
}

} // namespace pbfb
