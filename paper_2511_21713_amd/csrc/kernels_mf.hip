// Matrix-free boundary-element apply, for instances whose dense Galerkin
// operators would not fit the device: every apply evaluates the regular
// (non-touching) part of [K' | V'] x as a quadrature-point N-body sum and
// adds the touching-pair blocks and 1/2 M from small resident tables
// (Sec. 2.2, eq. KV; the paper switches to a fast multipole method above
// 90k vertices for the same reason).
//
//   1. k_mf_src: per source triangle sigma and rule point y_q the strengths
//      w_q |sigma| lambda_h(y_q) and w_q |sigma| u_h(y_q);
//   2. k_mf_pot: per target triangle tau, for each of its 6 rule points x_p,
//      the single- and double-layer potentials of all non-touching source
//      triangles, then the corner values |tau| / (4 pi) sum_p w_p b_p[a]
//      (s_V P_V(x_p) + s_K P_K(x_p)).  One workgroup owns 16 target
//      triangles and sweeps all source triangles in blocks of 32 staged in
//      LDS; thread (target, source) accumulates in FP64 across source blocks
//      (6-term sums in the evaluation precision, as in the dense assembly),
//      and the 32 source lanes of a target are added by a fixed xor-shuffle
//      tree, so the result is bitwise reproducible;
//   3. k_mf_gather: per vertex, the corner values of its triangles, the
//      touching-pair blocks (Sauter-Schwab, FP64, computed once at setup)
//      and the P1 mass, in a fixed order.
//
// The same integrals as the dense operator, summed in another order.
#include <cmath>

#include "bem_quad.hpp"
#include "pbfb_internal.hpp"

namespace pbfb {

constexpr int MF_TA = 16, MF_TB = 32, MF_NT = MF_TA * MF_TB;

static inline unsigned nbk_(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// batched use: only an instance in its Arnoldi or restart-residual phase applies
__device__ inline bool mf_active(const int *st) { return !st || *st == G_ARN || *st == G_RES; }

__global__ void k_mf_src(int64_t nt, int64_t nv, const int32_t *__restrict__ m_tri, const double *__restrict__ m_area,
                         const double *__restrict__ x, QRule6 R, const int *__restrict__ st, double *__restrict__ sl,
                         double *__restrict__ su)
{
    if (!mf_active(st)) return;
    const int64_t m = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (m >= nt) return;
    const int32_t v0 = m_tri[3 * m], v1 = m_tri[3 * m + 1], v2 = m_tri[3 * m + 2];
    const double u0 = x[v0], u1 = x[v1], u2 = x[v2];
    const double l0 = x[nv + v0], l1 = x[nv + v1], l2 = x[nv + v2];
    const double ar = m_area[m];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double wq = R.w[q] * ar;
        sl[6 * m + q] = wq * (R.b[q][0] * l0 + R.b[q][1] * l1 + R.b[q][2] * l2);
        su[6 * m + q] = wq * (R.b[q][0] * u0 + R.b[q][1] * u1 + R.b[q][2] * u2);
    }
}

// RT = double: FP64 positions (xq, nq: Morton-ordered points and normals)
// RT = float : FP32 offsets from FP64 centroids (cen)
template <bool YUK, typename RT>
__global__ void __launch_bounds__(MF_NT, 2)
    k_mf_pot(int64_t nt, const int32_t *__restrict__ m_tri, const RT *__restrict__ xq, const RT *__restrict__ nq,
             const double *__restrict__ cen, const double *__restrict__ m_area, const double *__restrict__ sl,
             const double *__restrict__ su, double kappa, double sV, double sK, QRule6 R,
             const int *__restrict__ st, double *__restrict__ Yc)
{
    if (!mf_active(st)) return;
    constexpr bool F32 = sizeof(RT) == 4;
    __shared__ RT sX[MF_TA][18];
    __shared__ double sCa[F32 ? MF_TA : 1][3];
    __shared__ int sVa[MF_TA][3];
    __shared__ RT sY[MF_TB][18], sN[MF_TB][3], sL[MF_TB][6], sU[MF_TB][6];
    __shared__ double sCb[F32 ? MF_TB : 1][3];
    __shared__ int sVb[MF_TB][3];

    const int tid = threadIdx.x, tl = tid / MF_TB, sli = tid % MF_TB;
    const int64_t mA = int64_t(blockIdx.x) * MF_TA + tl;
    for (int k = tid; k < MF_TA * 18; k += MF_NT) {
        const int t = k / 18, c = k % 18;
        const int64_t m = int64_t(blockIdx.x) * MF_TA + t;
        sX[t][c] = m < nt ? xq[18 * m + c] : RT(0);
    }
    if (tid < MF_TA * 3) {
        const int t = tid / 3, c = tid % 3;
        const int64_t m = int64_t(blockIdx.x) * MF_TA + t;
        sVa[t][c] = m < nt ? m_tri[3 * m + c] : -2;
        if constexpr (F32) sCa[t][c] = m < nt ? cen[3 * m + c] : 0.0;
    }
    const RT kap = RT(kappa);
    double PV[6], PK[6];
#pragma unroll
    for (int p = 0; p < 6; ++p) PV[p] = PK[p] = 0.0;
    const int64_t nbB = (nt + MF_TB - 1) / MF_TB;
    for (int64_t bB = 0; bB < nbB; ++bB) {
        __syncthreads();
        for (int k = tid; k < MF_TB * 18; k += MF_NT) {
            const int t = k / 18, c = k % 18;
            const int64_t m = bB * MF_TB + t;
            sY[t][c] = m < nt ? xq[18 * m + c] : RT(0);
        }
        for (int k = tid; k < MF_TB * 6; k += MF_NT) {
            const int t = k / 6, q = k % 6;
            const int64_t m = bB * MF_TB + t;
            sL[t][q] = m < nt ? RT(sl[6 * m + q]) : RT(0);
            sU[t][q] = m < nt ? RT(su[6 * m + q]) : RT(0);
        }
        if (tid < MF_TB * 3) {
            const int t = tid / 3, c = tid % 3;
            const int64_t m = bB * MF_TB + t;
            sN[t][c] = m < nt ? nq[3 * m + c] : RT(0);
            sVb[t][c] = m < nt ? m_tri[3 * m + c] : -1;
            if constexpr (F32) sCb[t][c] = m < nt ? cen[3 * m + c] : 0.0;
        }
        __syncthreads();
        const int64_t mB = bB * MF_TB + sli;
        if (mA >= nt || mB >= nt) continue;
        bool touch = false;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) touch |= (sVa[tl][a] == sVb[sli][b]);
        if (touch) continue;
        RT c0 = 0, c1 = 0, c2 = 0; // FP32: target frame relative to the source centroid
        if constexpr (F32) {
            c0 = float(sCa[tl][0] - sCb[sli][0]);
            c1 = float(sCa[tl][1] - sCb[sli][1]);
            c2 = float(sCa[tl][2] - sCb[sli][2]);
        }
        const RT n0 = sN[sli][0], n1 = sN[sli][1], n2 = sN[sli][2];
#pragma unroll 1
        for (int p = 0; p < 6; ++p) {
            const RT x0 = sX[tl][3 * p] + c0, x1 = sX[tl][3 * p + 1] + c1, x2 = sX[tl][3 * p + 2] + c2;
            // (x - y_q).n is the same for the 6 coplanar source points
            const RT dn = (x0 - sY[sli][0]) * n0 + (x1 - sY[sli][1]) * n1 + (x2 - sY[sli][2]) * n2;
            RT av = 0, ak = 0;
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const RT d0 = x0 - sY[sli][3 * q], d1 = x1 - sY[sli][3 * q + 1], d2 = x2 - sY[sli][3 * q + 2];
                const RT r2 = d0 * d0 + d1 * d1 + d2 * d2;
                const RT ri = rsqrt_pos(r2);
                RT gv, hk;
                if constexpr (YUK) {
                    const RT r = r2 * ri;
                    RT e;
                    if constexpr (F32) e = __builtin_amdgcn_exp2f(-1.44269504088896341f * kap * r);
                    else e = exp_neg(kap * r);
                    gv = e * ri;
                    hk = gv * ri * (ri + kap); // e (1 + kappa r) / r^3
                } else {
                    gv = ri;
                    hk = ri * ri * ri;
                }
                av += gv * sL[sli][q];
                ak += hk * sU[sli][q];
            }
            PV[p] += double(av);
            PK[p] += double(ak * dn);
        }
    }
    // the 32 source lanes of each target triangle, in a fixed order
#pragma unroll
    for (int p = 0; p < 6; ++p)
        for (int off = MF_TB / 2; off > 0; off >>= 1) {
            PV[p] += __shfl_xor(PV[p], off);
            PK[p] += __shfl_xor(PK[p], off);
        }
    if (sli != 0 || mA >= nt) return;
    const double sc = m_area[mA] * INV4PI;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double y = 0.0;
#pragma unroll
        for (int p = 0; p < 6; ++p) y += R.w[p] * R.b[p][a] * (sV * PV[p] + sK * PK[p]);
        Yc[3 * mA + a] = sc * y;
    }
}

// y_i = corner values of the triangles at i + touching-pair blocks + 1/2 M
__global__ void k_mf_gather(int64_t nv, const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                            const int32_t *__restrict__ tri, const int32_t *__restrict__ mpos,
                            const int32_t *__restrict__ tp_ptr, const int32_t *__restrict__ tp_sig,
                            const double *__restrict__ tpv, const double *__restrict__ area,
                            const double *__restrict__ Yc, const double *__restrict__ x, double sV, double sK,
                            const int *__restrict__ st, double *__restrict__ y)
{
    if (!mf_active(st)) return;
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    double acc = 0.0;
    for (int32_t e = v2t_ptr[i]; e < v2t_ptr[i + 1]; ++e) {
        const int32_t ta = v2t[e] / 3, a = v2t[e] % 3;
        acc += Yc[3 * int64_t(mpos[ta]) + a];
        for (int32_t pp = tp_ptr[ta]; pp < tp_ptr[ta + 1]; ++pp) {
            const int32_t sb = tp_sig[pp];
            const double *blk = tpv + 18 * int64_t(pp);
            for (int b = 0; b < 3; ++b) {
                const int32_t j = tri[3 * sb + b];
                acc += sV * blk[3 * a + b] * x[nv + j] + sK * blk[9 + 3 * a + b] * x[j];
            }
        }
        for (int b = 0; b < 3; ++b) acc += 0.5 * area[ta] * (a == b ? 2.0 : 1.0) / 12.0 * x[tri[3 * ta + b]];
    }
    y[i] = acc;
}

void mf_apply(Problem &p, int w, const double *x, double *y, const int *st, hipStream_t s)
{
    const SurfaceDev &S = p.surf[w];
    const int64_t nt = S.nt, nv = S.nv;
    const bool yuk = (w == 1) && p.kappa > 0.0;
    const double kappa = (w == 1) ? p.kappa : 0.0;
    const double sV = (w == 0) ? -1.0 : 1.0, sK = (w == 0) ? 1.0 : -1.0;
    const int base = w == 0 ? SCR_MF0 : SCR_MF1;
    double *sl = scratch<double>(p, base, 15 * size_t(nt));
    double *su = sl + 6 * nt, *Yc = su + 6 * nt;
    const QRule6 R = q6arg();
    hipLaunchKernelGGL(k_mf_src, dim3(nbk_(nt, 256)), dim3(256), 0, s, nt, nv, S.m_tri, S.m_area, x, R, st, sl, su);
    const dim3 grid(nbk_(nt, MF_TA));
    if (p.precision == PBFB_MIXED) {
        if (yuk)
            hipLaunchKernelGGL((k_mf_pot<true, float>), grid, dim3(MF_NT), 0, s, nt, S.m_tri, S.m_qf, S.m_nf, S.m_cen,
                               S.m_area, sl, su, kappa, sV, sK, R, st, Yc);
        else
            hipLaunchKernelGGL((k_mf_pot<false, float>), grid, dim3(MF_NT), 0, s, nt, S.m_tri, S.m_qf, S.m_nf,
                               S.m_cen, S.m_area, sl, su, kappa, sV, sK, R, st, Yc);
    } else {
        if (yuk)
            hipLaunchKernelGGL((k_mf_pot<true, double>), grid, dim3(MF_NT), 0, s, nt, S.m_tri, S.m_qp, S.m_nrm,
                               (const double *)nullptr, S.m_area, sl, su, kappa, sV, sK, R, st, Yc);
        else
            hipLaunchKernelGGL((k_mf_pot<false, double>), grid, dim3(MF_NT), 0, s, nt, S.m_tri, S.m_qp, S.m_nrm,
                               (const double *)nullptr, S.m_area, sl, su, kappa, sV, sK, R, st, Yc);
    }
    hipLaunchKernelGGL(k_mf_gather, dim3(nbk_(nv, 256)), dim3(256), 0, s, nv, S.v2t_ptr, S.v2t, S.tri, S.mpos,
                       S.tp_ptr, S.tp_sig, S.tpv, S.area, Yc, x, sV, sK, st, y);
    PB_HIP(hipGetLastError());
}

} // namespace pbfb

namespace pbfb {

// diagonal of the signed single layer V': only touching pairs (every pair of
// triangles at a vertex shares it) reach the diagonal
__global__ void k_mf_vdiag(int64_t nv, const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                           const int32_t *__restrict__ tri, const int32_t *__restrict__ tp_ptr,
                           const int32_t *__restrict__ tp_sig, const double *__restrict__ tpv, double sV,
                           double *__restrict__ vdiag)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    double acc = 0.0;
    for (int32_t e = v2t_ptr[i]; e < v2t_ptr[i + 1]; ++e) {
        const int32_t ta = v2t[e] / 3, a = v2t[e] % 3;
        for (int32_t pp = tp_ptr[ta]; pp < tp_ptr[ta + 1]; ++pp) {
            const int32_t sb = tp_sig[pp];
            for (int b = 0; b < 3; ++b)
                if (tri[3 * sb + b] == i) acc += tpv[18 * int64_t(pp) + 3 * a + b];
        }
    }
    vdiag[i] = sV * acc;
}

void mf_vdiag(Problem &p, int w, hipStream_t s)
{
    const SurfaceDev &S = p.surf[w];
    hipLaunchKernelGGL(k_mf_vdiag, dim3(nbk_(S.nv, 256)), dim3(256), 0, s, S.nv, S.v2t_ptr, S.v2t, S.tri, S.tp_ptr,
                       S.tp_sig, S.tpv, (w == 0) ? -1.0 : 1.0, S.vdiag);
    PB_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// preconditioner of the single layers without stored rows: the 1-ring
// sparse approximate inverse (row i minimises || m^T V' - e_i^T ||_2 over m
// on the 1-ring P(i)) built from the near field of V' instead of its full
// rows.  The near field keeps, for every row a, the columns within three
// rings of a, each entry the same Galerkin integral as the dense operator
// (touching pairs from the resident blocks, the others by the 6 x 6 rule).
// ---------------------------------------------------------------------------
// entry e = (a, c): sum over triangles tau at a and sigma at c (one thread per entry)
template <bool YUK>
__global__ void k_mf_near(int64_t nnz, const int32_t *__restrict__ nf_row, const int32_t *__restrict__ nf_col,
                          const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                          const int32_t *__restrict__ tp_ptr, const int32_t *__restrict__ tp_sig,
                          const double *__restrict__ tpv, const double *__restrict__ qp,
                          const double *__restrict__ area, double kappa, double sV, QRule6 R,
                          double *__restrict__ nf_val)
{
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= nnz) return;
    const int32_t a = nf_row[e], c = nf_col[e];
    double acc = 0.0;
    for (int32_t ea = v2t_ptr[a]; ea < v2t_ptr[a + 1]; ++ea) {
        const int32_t ta = v2t[ea] / 3, la = v2t[ea] % 3;
        for (int32_t ec = v2t_ptr[c]; ec < v2t_ptr[c + 1]; ++ec) {
            const int32_t sc = v2t[ec] / 3, lc = v2t[ec] % 3;
            int32_t pp = -1;
            for (int32_t k = tp_ptr[ta]; k < tp_ptr[ta + 1]; ++k)
                if (tp_sig[k] == sc) {
                    pp = k;
                    break;
                }
            if (pp >= 0) { // touching pair: the resident V block
                acc += tpv[18 * int64_t(pp) + 3 * la + lc];
                continue;
            }
            const double *X = qp + 18 * int64_t(ta), *Y = qp + 18 * int64_t(sc);
            double sum = 0.0;
            for (int p = 0; p < 6; ++p) {
                double sp = 0.0;
                for (int q = 0; q < 6; ++q) {
                    const double d0 = X[3 * p] - Y[3 * q], d1 = X[3 * p + 1] - Y[3 * q + 1],
                                 d2 = X[3 * p + 2] - Y[3 * q + 2];
                    const double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    const double g = YUK ? exp(-kappa * r) / r : 1.0 / r;
                    sp += R.w[q] * R.b[q][lc] * g;
                }
                sum += R.w[p] * R.b[p][la] * sp;
            }
            acc += area[ta] * area[sc] * INV4PI * sum;
        }
    }
    nf_val[e] = sV * acc;
}

// one 64-thread workgroup per row i: lanes take the (a, b) pairs of the Gram
// matrix of the near-field rows P(i), each a merge of two ascending sparse
// rows; lane 0 solves the normal equations by Cholesky
__global__ void __launch_bounds__(64)
    k_mf_spai(int64_t nv, const int32_t *__restrict__ ring_ptr, const int32_t *__restrict__ ring,
              const int32_t *__restrict__ nf_ptr, const int32_t *__restrict__ nf_col,
              const double *__restrict__ nf_val, double *__restrict__ val, int *__restrict__ bad)
{
    __shared__ double G[MAXRING][MAXRING + 1];
    __shared__ double rhs[MAXRING];
    const int lane = threadIdx.x;
    const int64_t i = blockIdx.x;
    if (i >= nv) return;
    const int p0 = ring_ptr[i], m = ring_ptr[i + 1] - p0;
    const int npair = m * (m + 1) / 2;
    for (int pr = lane; pr < npair; pr += 64) {
        int a = int((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
        while (a * (a + 1) / 2 > pr) --a;
        while ((a + 1) * (a + 2) / 2 <= pr) ++a;
        const int b = pr - a * (a + 1) / 2;
        const int32_t ra = ring[p0 + a], rb = ring[p0 + b];
        int32_t ka = nf_ptr[ra], kb = nf_ptr[rb];
        const int32_t ea = nf_ptr[ra + 1], eb = nf_ptr[rb + 1];
        double sum = 0.0;
        while (ka < ea && kb < eb) {
            const int32_t ca = nf_col[ka], cb = nf_col[kb];
            if (ca == cb) sum = fma(nf_val[ka++], nf_val[kb++], sum);
            else if (ca < cb) ++ka;
            else ++kb;
        }
        G[a][b] = G[b][a] = sum;
    }
    for (int a = lane; a < m; a += 64) {
        const int32_t ra = ring[p0 + a];
        double v = 0.0; // V'(P_a, i): i is in the 1-ring of P_a, hence in its pattern
        for (int32_t k = nf_ptr[ra]; k < nf_ptr[ra + 1]; ++k)
            if (nf_col[k] == int32_t(i)) v = nf_val[k];
        rhs[a] = v;
    }
    __syncthreads();
    if (lane != 0) return;
    bool ok = true;
    for (int a = 0; a < m && ok; ++a) {
        double d = G[a][a];
        for (int k = 0; k < a; ++k) d -= G[a][k] * G[a][k];
        if (!(d > 0.0)) {
            ok = false;
            break;
        }
        G[a][a] = sqrt(d);
        for (int b = a + 1; b < m; ++b) {
            double t = G[b][a];
            for (int k = 0; k < a; ++k) t -= G[b][k] * G[a][k];
            G[b][a] = t / G[a][a];
        }
    }
    if (!ok) {
        atomicOr(bad, 4);
        for (int a = 0; a < m; ++a) val[p0 + a] = 0.0;
        return;
    }
    for (int a = 0; a < m; ++a) {
        double t = rhs[a];
        for (int k = 0; k < a; ++k) t -= G[a][k] * rhs[k];
        rhs[a] = t / G[a][a];
    }
    for (int a = m - 1; a >= 0; --a) {
        double t = rhs[a];
        for (int k = a + 1; k < m; ++k) t -= G[k][a] * rhs[k];
        rhs[a] = t / G[a][a];
    }
    for (int a = 0; a < m; ++a) val[p0 + a] = rhs[a];
}

void mf_spai(Problem &p, int w, hipStream_t s)
{
    const SurfaceDev &S = p.surf[w];
    const bool yuk = (w == 1) && p.kappa > 0.0;
    const double kappa = (w == 1) ? p.kappa : 0.0, sV = (w == 0) ? -1.0 : 1.0;
    const QRule6 R = q6arg();
    const dim3 g(nbk_(S.nf_nnz, 256));
    if (yuk)
        hipLaunchKernelGGL(k_mf_near<true>, g, dim3(256), 0, s, S.nf_nnz, S.nf_row, S.nf_col, S.v2t_ptr, S.v2t,
                           S.tp_ptr, S.tp_sig, S.tpv, S.qp, S.area, kappa, sV, R, S.nf_val);
    else
        hipLaunchKernelGGL(k_mf_near<false>, g, dim3(256), 0, s, S.nf_nnz, S.nf_row, S.nf_col, S.v2t_ptr, S.v2t,
                           S.tp_ptr, S.tp_sig, S.tpv, S.qp, S.area, kappa, sV, R, S.nf_val);
    hipLaunchKernelGGL(k_mf_spai, dim3(unsigned(S.nv)), dim3(64), 0, s, S.nv, S.ring_ptr, S.ring, S.nf_ptr, S.nf_col,
                       S.nf_val, S.spai, p.d_bad);
    PB_HIP(hipGetLastError());
}

} // namespace pbfb
