// Batched restarted GMRES with device-resident control.
//
// Every instance of a batch solves its own system J x = b (right
// preconditioned by the block diagonal, x0 = 0, classical Gram-Schmidt
// applied twice, Givens rotations), and all of them advance together: each
// kernel below takes a packed work list that covers every instance, so one
// launch per step serves the whole batch whatever the mesh sizes.  The Krylov
// scalars (Hessenberg column, rotations, residual estimate, restart and
// convergence decisions, triangular solve) live on the device in one thread
// per instance, so the host only enqueues iterations and polls a completion
// counter asynchronously; nothing waits on the host between iterations.
//
// Per-instance state machine (P^-1 the right preconditioner):
//   INIT  -> w = b, V_0 = b/|b|, target = tol |b|              -> ARN (or DONE if b = 0)
//   ARN   -> z = P^-1 V_j, w = J z, CGS2, V_{j+1}, Givens       -> UPD at convergence/restart/limit
//   UPD   -> y = H^{-1} g, t = V y                               -> RES
//   RES   -> x += P^-1 t, w = b - J x, beta = |w|: beta <= target -> DONE, else V_0 = w/beta -> ARN
// which is the restarted GMRES of the oracle (true residual at every restart).
// P^-1 is either the inverse diagonal of J or the block preconditioner:
// Jacobi-scaled Chebyshev terms on the FEM block (one SpMV launch per term
// after the first) and a sparse approximate inverse on each single-layer
// block.
//
// Mixed precision may store the basis in FP32 (products, projections, norms,
// Hessenberg, rotations, w and x stay FP64).  A restart cycle is then an
// FP32-basis inner solve for the correction of the current iterate, and the
// FP64 true residual b - J x that starts the next cycle is the outer
// iterative refinement: the tolerance is always decided on that residual.
#include <algorithm>
#include <cmath>

#include "gemv_rows.hpp"
#include "pbfb_internal.hpp"
#include "sell_slice.hpp"

namespace pbfb {


struct GDesc {
    const void *Bm, *Bs;
    int64_t ldm, lds, nm, ns;
    int f32;  // operator values in FP32
    int vf32; // Krylov basis stored in FP32
    int mf;   // boundary operators applied matrix-free (no dense GEMV)
    int two_field; // lambda_m is not an unknown (two-field form): identity row, no Gamma_m GEMV
    // symmetric use of the stored single layer, per surface: column partials, Delta rows
    int symm[2];
    void *symP[2]; // FP64 column partials
    const int32_t *dl_ptr[2], *dl_col[2];
    const double *dl_val[2];
    // packing maps: operator index -> FEM node, and -> surface vertex (Morton
    // vertex order of the stored operators; matrix-free: ascending, mv null)
    const int32_t *gm, *gs, *mvm, *mvs;
    const int32_t *sptr, *col; // FEM rows, sliced ELL
    const void *val;
    int64_t nn, n;
    const double *dinv;
    void *V; // (m + 1) x n basis, FP64 or FP32 (vf32)
    double *w, *xm, *xs, *x;
    const double *b;
    double *H, *cs, *sn, *g, *y, *h1, *h2, *part, *npart, *nrm;
    int *cnt; // completion counter of the x update (index 257)
    int64_t nch, nchb;
    double tol;
    int m, maxit;
    // preconditioner
    int pc, cheb_k;
    double cheb_ratio;
    const double *lmax;
    const int32_t *sp_ptr[2], *sp_col[2];
    const double *sp_val[2];
    double *z, *zb, *dk, *t; // P^-1 input (full), Chebyshev ping-pong buffer and direction, V y
    double *coef;            // Chebyshev coefficients: [0] = theta, [2s], [2s+1] = rho_s rho_{s-1}, 2 rho_s/delta
};

struct GState {
    int st, j, total, code, napply, fin; // fin: the cycle ended on the residual estimate
    double beta, target, hn;
};

struct WItem {
    int inst, a;
    int64_t b;
};

constexpr int CH = 256;      // rows per chunk: one per thread of a workgroup
constexpr int GROWS = GSYM; // GEMV rows per workgroup


__device__ inline bool applies(int st) { return st == G_ARN || st == G_RES; }

// basis entry V_i[k], widened to FP64
__device__ inline double vget(const GDesc &d, int64_t i, int64_t k)
{
    return d.vf32 ? double(static_cast<const float *>(d.V)[i * d.n + k]) : static_cast<const double *>(d.V)[i * d.n + k];
}
template <typename VT> __device__ inline const VT *vcol(const GDesc &d, int64_t i)
{
    return static_cast<const VT *>(d.V) + i * d.n;
}

// ---------------------------------------------------------------------------
// apply: pack, dense GEMV, sliced-ELL SpMV on the current input of each instance
// (ARN: D^{-1} V_j, RES: x)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bpack(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (!applies(s.st)) return;
    const GDesc &d = D[it.inst];
    const double *in0 = s.st == G_ARN ? d.z : d.x; // ARN: P^-1 V_j, RES: x
    auto in = [&](int64_t r) { return in0[r]; };
    for (int64_t k = it.b + threadIdx.x; k < it.b + CH; k += 256) {
        if (d.two_field) {
            if (k < d.nm) d.w[d.nn + k] = in(d.nn + k); // identity row of lambda_m
        } else if (k < d.ldm) {
            double v = 0.0;
            if (k < d.nm) v = in(d.gm[k]);
            else if (k < 2 * d.nm) v = in(d.nn + (d.mvm ? d.mvm[k - d.nm] : k - d.nm));
            d.xm[k] = v;
        }
        if (k < d.lds) {
            double v = 0.0;
            if (k < d.ns) v = in(d.gs[k]);
            else if (k < 2 * d.ns) v = in(d.nn + d.nm + (d.mvs ? d.mvs[k - d.ns] : k - d.ns));
            d.xs[k] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// preconditioner stage: z = P^-1 src with src = V_j (ARN) or t = V y (RES,
// which also adds the result to x).  Chebyshev term s (0-based) of the FEM
// block is written to z when k - 1 - s is even and to zb otherwise, so the
// last term always lands in z.
// ---------------------------------------------------------------------------
// the Chebyshev coefficients of every instance, from its bound lmax (one
// thread per instance, once per batched solve)
__global__ void k_cheb_coef(const GDesc *__restrict__ D, int nb)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nb) return;
    const GDesc &d = D[q];
    if (d.pc != PBFB_PC_CHEB_SPAI) return;
    const double hi = *d.lmax, lo = hi / d.cheb_ratio;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    d.coef[0] = theta;
    d.coef[1] = 0.0;
    for (int s = 1; s < d.cheb_k; ++s) {
        const double rho1 = 1.0 / (2.0 * sigma - rho);
        d.coef[2 * s] = rho1 * rho;
        d.coef[2 * s + 1] = 2.0 * rho1 / delta;
        rho = rho1;
    }
}

__device__ inline double pc_src(const GDesc &d, const GState &s, int64_t r)
{
    return (s.st == G_RES || s.st == G_FIN) ? d.t[r] : vget(d, s.j, r);
}

// first term (FEM rows), the approximate inverse (surface rows) or the diagonal
__global__ void __launch_bounds__(256) k_bprec0(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                                const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (s.st != G_ARN && s.st != G_RES && s.st != G_FIN) return;
    const GDesc &d = D[it.inst];
    const int64_t k = it.b + threadIdx.x;
    if (k >= d.n) return;
    double zv;
    bool last = true;
    if (d.pc == PBFB_PC_DIAG) {
        zv = d.dinv[k] * pc_src(d, s, k);
        d.z[k] = zv;
    } else if (k < d.nn) {
        zv = d.dinv[k] * pc_src(d, s, k) / d.coef[0];
        d.dk[k] = zv;
        ((d.cheb_k - 1) % 2 == 0 ? d.z : d.zb)[k] = zv;
        last = d.cheb_k == 1;
    } else {
        const int w = k < d.nn + d.nm ? 0 : 1;
        const int64_t off = d.nn + (w == 0 ? 0 : d.nm), i = k - off;
        double acc = 0.0;
        for (int32_t e = d.sp_ptr[w][i]; e < d.sp_ptr[w][i + 1]; ++e)
            acc = fma(d.sp_val[w][e], pc_src(d, s, off + d.sp_col[w][e]), acc);
        zv = acc;
        d.z[k] = zv;
    }
    if (last && (s.st == G_RES || s.st == G_FIN)) d.x[k] += zv;
}

// Chebyshev term `step` >= 1 of the FEM block: one workgroup per 64-row
// slice (work item: inst, b = first row of the slice)
__global__ void __launch_bounds__(256) k_bcheb(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S, int step)
{
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (s.st != G_ARN && s.st != G_RES && s.st != G_FIN) return;
    const GDesc &d = D[it.inst];
    if (d.pc != PBFB_PC_CHEB_SPAI || step >= d.cheb_k) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = it.b / SLICE, row = it.b + lane;
    const double *zp = ((d.cheb_k - step) % 2 == 0) ? d.z : d.zb; // term step - 1
    double *zn = ((d.cheb_k - 1 - step) % 2 == 0) ? d.z : d.zb;
    const double part = d.f32 ? sell_part<float, true>(d.sptr, d.col, static_cast<const float *>(d.val), zp, q,
                                                       lane, wv, d.nn)
                              : sell_part<double, true>(d.sptr, d.col, static_cast<const double *>(d.val), zp, q,
                                                        lane, wv, d.nn);
    const double acc = sell_reduce(part, lane, wv);
    if (wv != 0 || row >= d.nn) return;
    const double dv = d.coef[2 * step] * d.dk[row] + d.coef[2 * step + 1] * d.dinv[row] * (pc_src(d, s, row) - acc);
    d.dk[row] = dv;
    const double zv = zp[row] + dv;
    zn[row] = zv;
    if (step == d.cheb_k - 1 && (s.st == G_RES || s.st == G_FIN)) d.x[row] += zv;
}

// work item: inst, a = interface (0/1), b = first row of the workgroup.  One
// instantiation per storage type, each skipping the instances of the other:
// a kernel holding both row routines would be register-allocated for their
// union and run at half the occupancy of either.
template <typename MT>
__global__ void __launch_bounds__(GEMV_THREADS, gemv_occupancy<MT>()) k_bgemv(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    if (!applies(S[it.inst].st)) return;
    const GDesc &d = D[it.inst];
    if (d.mf || d.f32 != (sizeof(MT) == 4)) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int a = it.a & 1; // surface; it.a & 2: K item of the symmetric use
    const int64_t n = a == 0 ? d.nm : d.ns;
    const int64_t ld = a == 0 ? d.ldm : d.lds;
    const double *x = a == 0 ? d.xm : d.xs;
    double *y = d.w + d.nn + (a == 0 ? 0 : d.nm);
    const MT *B = static_cast<const MT *>(a == 0 ? d.Bm : d.Bs);
    if (!d.symm[a]) {
        const int64_t r0 = it.b + wv * GEMV_RW;
        if (r0 < n) gemv_rows<MT>(B, x, y, a == 0 ? d.mvm : d.mvs, n, ld, r0, lane);
    } else if (it.a & 2) {
        gemv_rows_symK<MT>(B, x, y, a == 0 ? d.mvm : d.mvs, n, ld, it.b, threadIdx.x);
    } else {
        gemv_rows_symV<MT>(B, x, static_cast<sym_part_t<MT> *>(d.symP[a]), n, ld, it.b, threadIdx.x);
    }
}

// second stage of the symmetric use (work item: inst, a = surface, b = first of GFIN_ROWS rows)
__global__ void __launch_bounds__(256) k_bgemv_fin(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                                   const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    if (!applies(S[it.inst].st)) return;
    const GDesc &d = D[it.inst];
    if (d.mf || !d.symm[it.a]) return;
    const int64_t n = it.a == 0 ? d.nm : d.ns;
    const double *x = it.a == 0 ? d.xm : d.xs;
    double *y = d.w + d.nn + (it.a == 0 ? 0 : d.nm);
    gemv_sym_finish(n, static_cast<const double *>(d.symP[it.a]), d.dl_ptr[it.a], d.dl_col[it.a], d.dl_val[it.a], x, y,
                    it.a == 0 ? d.mvm : d.mvs,
                    it.b, threadIdx.x);
}

__global__ void __launch_bounds__(256) k_bspmv(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (!applies(s.st)) return;
    const GDesc &d = D[it.inst];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = it.b / SLICE, row = it.b + lane;
    const double *in = s.st == G_ARN ? d.z : d.x;
    const double part = d.f32 ? sell_part<float, false>(d.sptr, d.col, static_cast<const float *>(d.val), in, q,
                                                        lane, wv, d.nn)
                              : sell_part<double, false>(d.sptr, d.col, static_cast<const double *>(d.val), in, q,
                                                         lane, wv, d.nn);
    const double acc = sell_reduce(part, lane, wv);
    if (wv == 0 && row < d.nn) d.w[row] = acc;
}

// ---------------------------------------------------------------------------
// classical Gram-Schmidt pass: partial dot products V_i . w over 2048-row
// chunks (work item: inst, a = chunk, b = first row; blockIdx.y = group of 8
// coefficients), then one workgroup per (instance, group) sums the chunk
// partials in chunk order, so every coefficient is deterministic.  Kernel
// boundaries order the passes (no device-scope fences).
// ---------------------------------------------------------------------------
constexpr int CHB = 2048; // rows per dot-product chunk (8 per thread)

__global__ void __launch_bounds__(256) k_bmdot(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S)
{
    __shared__ double red[8][256];
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (s.st != G_ARN) return;
    const int i0 = blockIdx.y * 8;
    if (i0 > s.j) return;
    const GDesc &d = D[it.inst];
    const int kk = min(8, s.j + 1 - i0);
    double acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.0;
    auto body = [&](auto *V0) {
        for (int64_t k = it.b + threadIdx.x; k < it.b + CHB && k < d.n; k += 256) {
            const double wk = d.w[k];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < kk) acc[q] = fma(double(V0[int64_t(q) * d.n + k]), wk, acc[q]);
        }
    };
    if (d.vf32) body(vcol<float>(d, i0));
    else body(vcol<double>(d, i0));
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int wd = 128; wd > 0; wd >>= 1) {
        if (threadIdx.x < wd)
#pragma unroll
            for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x < kk) d.part[int64_t(it.a) * (d.m + 1) + i0 + threadIdx.x] = red[threadIdx.x][0];
}

// h[i] = sum over chunks of part[c][i]; grid (instances, groups of 8)
__global__ void __launch_bounds__(256) k_breduce(const GDesc *__restrict__ D, const GState *__restrict__ S, int pass)
{
    const int q = blockIdx.x;
    const GState s = S[q];
    if (s.st != G_ARN) return;
    const int i0 = blockIdx.y * 8;
    if (i0 > s.j) return;
    const GDesc &d = D[q];
    const int kk = min(8, s.j + 1 - i0);
    const int g = threadIdx.x >> 5, lane = threadIdx.x & 31;
    if (g >= kk) return;
    double t = 0.0;
    for (int64_t c = lane; c < d.nchb; c += 32) t += d.part[c * (d.m + 1) + i0 + g];
    for (int off = 16; off > 0; off >>= 1) t += __shfl_xor(t, off, 32);
    if (lane == 0) (pass == 0 ? d.h1 : d.h2)[i0 + g] = t;
}

// First pass (second = 0): w -= sum_i h1_i V_i for ARN.
// Second pass (second = 1): ARN: w -= sum_i h2_i V_i;  RES: w = b - w;
// INIT: w = b; then |w|^2 per 256-row chunk into npart.
__global__ void __launch_bounds__(256) k_bmsub(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               const GState *__restrict__ S, int second)
{
    __shared__ double hs[1024];
    __shared__ double red[256];
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    const GDesc &d = D[it.inst];
    const bool arn = s.st == G_ARN;
    if (!arn && !(second && (s.st == G_RES || s.st == G_INIT))) return;
    const int jj = arn ? s.j + 1 : 0;
    const double *h = second ? d.h2 : d.h1;
    for (int i = threadIdx.x; i < jj; i += 256) hs[i] = h[i];
    __syncthreads();
    const int64_t k = it.b + threadIdx.x;
    double v = 0.0;
    if (k < d.n) {
        if (s.st == G_INIT) v = d.b[k];
        else if (s.st == G_RES) v = d.b[k] - d.w[k];
        else {
            v = d.w[k];
            if (d.vf32) {
                const float *V0 = vcol<float>(d, 0);
                for (int i = 0; i < jj; ++i) v = fma(-hs[i], double(V0[int64_t(i) * d.n + k]), v);
            } else {
                const double *V0 = vcol<double>(d, 0);
                for (int i = 0; i < jj; ++i) v = fma(-hs[i], V0[int64_t(i) * d.n + k], v);
            }
        }
        d.w[k] = v;
    }
    if (!second) return;
    red[threadIdx.x] = v * v;
    __syncthreads();
    for (int wd = 128; wd > 0; wd >>= 1) {
        if (threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x == 0) d.npart[it.a] = red[0];
}

// |w|^2 = sum of the chunk partials, one workgroup per instance
__global__ void __launch_bounds__(256) k_bnorm(const GDesc *__restrict__ D, const GState *__restrict__ S)
{
    __shared__ double red[256];
    const int q = blockIdx.x;
    const int st = S[q].st;
    if (st != G_ARN && st != G_RES && st != G_INIT) return;
    const GDesc &d = D[q];
    double t = 0.0;
    for (int64_t c = threadIdx.x; c < d.nch; c += 256) t += d.npart[c];
    red[threadIdx.x] = t;
    __syncthreads();
    for (int wd = 128; wd > 0; wd >>= 1) {
        if (threadIdx.x < wd) red[threadIdx.x] += red[threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x == 0) *d.nrm = red[0];
}

// ARN: V_{j+1} = w / |w|;  INIT/RES: V_0 = w / |w|
__global__ void __launch_bounds__(256) k_bscale(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                                const GState *__restrict__ S)
{
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (s.st != G_ARN && s.st != G_RES && s.st != G_INIT) return;
    const GDesc &d = D[it.inst];
    const double nr = sqrt(*d.nrm);
    const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
    const int64_t off = (s.st == G_ARN ? int64_t(s.j + 1) * d.n : 0);
    const int64_t k = it.b + threadIdx.x;
    if (k < d.n) {
        if (d.vf32) static_cast<float *>(d.V)[off + k] = float(d.w[k] * inv);
        else static_cast<double *>(d.V)[off + k] = d.w[k] * inv;
    }
}

// ---------------------------------------------------------------------------
// control: one wavefront per instance.  ARN: Hessenberg column, Givens chain
// (in LDS, one lane), residual estimate, cycle end; at the end of a cycle the
// triangular solve H y = g (column sweep across the lanes).  INIT/RES: true
// residual test and cycle start.  Transitions to DONE/FAIL bump ndone.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_bcontrol(const GDesc *__restrict__ D, GState *__restrict__ S,
                                                 int *__restrict__ ndone)
{
    __shared__ double hc[1024], cs[1024], sn[1024], gl[1024];
    __shared__ GState ss;
    const int q = blockIdx.x, lane = threadIdx.x;
    const GDesc &d = D[q];
    if (lane == 0) ss = S[q];
    __syncthreads();
    const int st0 = ss.st;
    if (st0 == G_FIN) {
        if (lane == 0) {
            S[q].st = G_DONE;
            atomicAdd(ndone, 1);
        }
        return;
    }
    if (st0 != G_ARN && st0 != G_RES && st0 != G_INIT) return;
    const int m = d.m;
    const double nr = sqrt(*d.nrm);
    if (st0 == G_ARN) {
        const int j = ss.j;
        for (int i = lane; i <= j; i += 64) {
            hc[i] = d.h1[i] + d.h2[i];
            if (i < j) {
                cs[i] = d.cs[i];
                sn[i] = d.sn[i];
            }
        }
        __syncthreads();
        if (lane == 0) {
            double t = hc[0];
            for (int i = 0; i < j; ++i) {
                const double c2 = hc[i + 1];
                hc[i] = cs[i] * t + sn[i] * c2;
                t = -sn[i] * t + cs[i] * c2;
            }
            const double den = hypot(t, nr);
            const double cj = t / den, sj = nr / den;
            d.cs[j] = cj;
            d.sn[j] = sj;
            hc[j] = den;
            const double gj = d.g[j];
            d.g[j + 1] = -sj * gj;
            d.g[j] = cj * gj;
            ss.j = j + 1;
            ss.total += 1;
            ss.napply += 1;
            ss.hn = nr;
            const double res = fabs(d.g[j + 1]);
            if (!(res == res)) {
                ss.st = G_FAIL;
                ss.code = PBFB_ENAN;
                atomicAdd(ndone, 1);
            } else if (res <= ss.target || nr == 0.0 || ss.j == m || ss.total >= d.maxit) {
                ss.st = G_UPD;
                // converged on the estimate: no true-residual check, except with an
                // FP32 basis, whose restarts are refinement steps that need it
                ss.fin = (res <= ss.target || nr == 0.0) && !d.vf32;
            }
        }
        __syncthreads();
        double *Hj = d.H + int64_t(j) * (m + 1);
        for (int i = lane; i <= j; i += 64) Hj[i] = hc[i];
        if (lane == 0) Hj[j + 1] = 0.0;
        if (ss.st == G_UPD) {
            // back substitution by columns: y_i = g_i / H_ii, then g_k -= H_ki y_i for k < i
            const int jc = ss.j;
            __threadfence_block();
            for (int i = lane; i < jc; i += 64) gl[i] = d.g[i];
            __syncthreads();
            for (int i = jc - 1; i >= 0; --i) {
                // column j (this step's) is taken from LDS, older columns from global memory
                const double yi = gl[i] / (i == j ? hc[j] : d.H[int64_t(i) * (m + 1) + i]);
                for (int k = lane; k < i; k += 64) gl[k] -= (i == j ? hc[k] : d.H[int64_t(i) * (m + 1) + k]) * yi;
                if (lane == 0) d.y[i] = yi;
                __syncthreads();
            }
        }
    } else if (lane == 0) {
        if (st0 == G_INIT) ss.target = d.tol * nr;
        else ss.napply += 1; // RES: the true residual took one application
        ss.beta = nr;
        if (!(nr == nr)) {
            ss.st = G_FAIL;
            ss.code = PBFB_ENAN;
            atomicAdd(ndone, 1);
        } else if (nr <= ss.target) {
            ss.st = G_DONE;
            atomicAdd(ndone, 1);
        } else if (ss.total >= d.maxit) {
            ss.st = G_FAIL;
            ss.code = PBFB_ENOTCONV;
            atomicAdd(ndone, 1);
        } else {
            for (int i = 0; i <= m; ++i) d.g[i] = 0.0;
            d.g[0] = nr;
            ss.j = 0;
            ss.st = G_ARN;
        }
    }
    __syncthreads();
    if (lane == 0) S[q] = ss;
}

// UPD: t = V y; the last workgroup of the instance moves it to RES
__global__ void __launch_bounds__(256) k_bupdx(const WItem *__restrict__ wl, const GDesc *__restrict__ D,
                                               GState *__restrict__ S)
{
    __shared__ double ys[1024];
    __shared__ int last;
    const WItem it = wl[blockIdx.x];
    const GState s = S[it.inst];
    if (s.st != G_UPD) return;
    const GDesc &d = D[it.inst];
    for (int i = threadIdx.x; i < s.j; i += 256) ys[i] = d.y[i];
    __syncthreads();
    const int64_t k = it.b + threadIdx.x;
    if (k < d.n) {
        double v = 0.0;
        if (d.vf32) {
            const float *V0 = vcol<float>(d, 0);
            for (int i = 0; i < s.j; ++i) v = fma(ys[i], double(V0[int64_t(i) * d.n + k]), v);
        } else {
            const double *V0 = vcol<double>(d, 0);
            for (int i = 0; i < s.j; ++i) v = fma(ys[i], V0[int64_t(i) * d.n + k], v);
        }
        d.t[k] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int *cnt = d.cnt + 257;
        last = atomicAdd(cnt, 1) == int(d.nch) - 1;
        if (last) {
            *cnt = 0;
            S[it.inst].st = s.fin ? G_FIN : G_RES;
        }
    }
}

// ===========================================================================
// host driver
// ===========================================================================
// a captured Krylov step is valid for the same device buffer and launch shapes
struct GraphKey {
    void *dev = nullptr;
    unsigned nvec = 0, ngemv = 0, nspmv = 0, npack = 0, ndot = 0, ngroups = 0, nb = 0, nfin = 0;
    int kmax = 0, types = 0; // types: bit 0 FP64 operators present, bit 1 FP32
    bool operator==(const GraphKey &o) const
    {
        return dev == o.dev && nvec == o.nvec && ngemv == o.ngemv && nspmv == o.nspmv && npack == o.npack &&
               ndot == o.ndot && ngroups == o.ngroups && nb == o.nb && nfin == o.nfin && kmax == o.kmax &&
               types == o.types;
    }
};

struct BatchBuffers {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    int *pinned = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipGraphExec_t step = nullptr; // the captured Krylov step (left to process exit)
    GraphKey key;
    ~BatchBuffers()
    {
        if (dev) (void)hipFree(dev);
        if (pinned) (void)hipHostFree(pinned);
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

static BatchBuffers &batch_buffers()
{
    static thread_local BatchBuffers B;
    if (!B.pinned) {
        PB_HIP(hipHostMalloc(reinterpret_cast<void **>(&B.pinned), 64 * sizeof(int), hipHostMallocDefault));
        for (auto &e : B.ev) PB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    return B;
}

void batched_gmres(std::vector<GmresJob *> &jobs, hipStream_t s)
{
    const int nb = int(jobs.size());
    if (nb == 0) return;
    std::vector<GDesc> desc(nb);
    std::vector<GState> st(nb);
    std::vector<WItem> wl_vec, wl_gemv, wl_spmv, wl_pack, wl_dot, wl_fin;
    // GEMV items in the order of gemv_item, over the batch: the heavy V items
    // of every instance, then the K and full-row items, then the other V items
    std::vector<WItem> wl_gemv_k, wl_gemv_v;
    int maxiter_host = 0, kmax = 1;
    for (int q = 0; q < nb; ++q) {
        GmresJob &J = *jobs[q];
        Problem &p = *J.p;
        const int m = J.restart;
        const int64_t n = p.n();
        GDesc &d = desc[q];
        d.Bm = p.surf[0].B;
        d.Bs = p.surf[1].B;
        d.nm = p.surf[0].nv;
        d.ns = p.surf[1].nv;
        d.ldm = bem_ld(d.nm);
        d.lds = bem_ld(d.ns);
        d.f32 = p.precision == PBFB_MIXED;
        d.mf = p.bem_mf ? 1 : 0;
        d.two_field = p.two_field() ? 1 : 0;
        d.gm = p.bem_mf ? p.surf[0].g : p.surf[0].gmv;
        d.gs = p.bem_mf ? p.surf[1].g : p.surf[1].gmv;
        d.mvm = p.bem_mf ? nullptr : p.surf[0].mvert;
        d.mvs = p.bem_mf ? nullptr : p.surf[1].mvert;
        d.sptr = p.d_sptr;
        d.col = p.d_col;
        d.val = d.f32 ? static_cast<const void *>(p.d_val32) : static_cast<const void *>(p.d_val);
        d.nn = p.nn;
        d.n = n;
        d.dinv = J.dinv;
        d.pc = J.pc;
        d.cheb_k = J.cheb_k;
        d.cheb_ratio = J.cheb_ratio;
        d.lmax = J.lmax;
        for (int w = 0; w < 2; ++w) {
            d.sp_ptr[w] = p.surf[w].ring_ptr;
            d.sp_col[w] = p.surf[w].ring;
            d.sp_val[w] = p.surf[w].spai;
            const SurfaceDev &SD = p.surf[w];
            d.symm[w] = (!p.bem_mf && SD.sym) ? 1 : 0;
            d.symP[w] = d.symm[w] ? scratch<double>(p, w == 0 ? SCR_SYMP0 : SCR_SYMP1,
                                                    size_t(sym_partials_doubles(SD.nv)))
                                  : nullptr;
            d.dl_ptr[w] = SD.d_ptr;
            d.dl_col[w] = SD.d_col;
            d.dl_val[w] = SD.d_val;
        }
        d.z = scratch<double>(p, SCR_PZ, n);
        d.t = scratch<double>(p, SCR_PT, n);
        d.zb = scratch<double>(p, SCR_PZB, p.nn);
        d.dk = scratch<double>(p, SCR_PDK, p.nn);
        d.coef = scratch<double>(p, SCR_PCOEF, 2 * 64 + 2);
        if (J.pc == PBFB_PC_CHEB_SPAI) kmax = std::max(kmax, J.cheb_k);
        d.vf32 = J.basis32 && p.precision == PBFB_MIXED;
        if (d.vf32) d.V = scratch<float>(p, SCR_BASIS32, size_t(m + 1) * n);
        else d.V = scratch<double>(p, SCR_BASIS, size_t(m + 1) * n);
        d.w = scratch<double>(p, SCR_G0, n);
        d.xm = scratch<double>(p, SCR_XM, d.ldm);
        d.xs = scratch<double>(p, SCR_XS, d.lds);
        d.x = J.x;
        d.b = J.b;
        d.nch = (n + CH - 1) / CH;
        double *kry = scratch<double>(p, SCR_HVEC, size_t(m) * (m + 1) + 3 * m + 3 * (m + 1) + 8);
        d.H = kry;
        d.cs = d.H + size_t(m) * (m + 1);
        d.sn = d.cs + m;
        d.y = d.sn + m;
        d.g = d.y + m;
        d.h1 = d.g + (m + 1);
        d.h2 = d.h1 + (m + 1);
        d.nchb = (n + CHB - 1) / CHB;
        d.part = scratch<double>(p, SCR_HPART, size_t(d.nchb) * (m + 1));
        d.npart = scratch<double>(p, SCR_NRM, d.nch + 1);
        d.nrm = d.npart + d.nch;
        d.cnt = scratch<int>(p, SCR_CNT, 258);
        PB_HIP(hipMemsetAsync(d.cnt, 0, sizeof(int) * 258, s));
        d.tol = J.tol;
        d.m = m;
        d.maxit = J.maxit;
        st[q] = GState{G_INIT, 0, 0, 0, 0, 0, 0.0, 0.0, 0.0};
        PB_HIP(hipMemsetAsync(J.x, 0, sizeof(double) * n, s));
        for (int64_t c = 0; c < d.nch; ++c) wl_vec.push_back(WItem{q, int(c), c * CH});
        for (int64_t c = 0; c < d.nchb; ++c) wl_dot.push_back(WItem{q, int(c), c * CHB});
        static_assert(GROWS == GSYM, "GEMV work items are the symmetric routine's row blocks");
        {
            // per surface: K (or full-row) items in row order, V items last
            // row block first (the last rows read the most); the first
            // gemv_heavy of the V items go before every K item; the two
            // surfaces alternate inside each stretch
            std::vector<WItem> kit[2], vit[2];
            for (int a = d.two_field ? 1 : 0; a < 2; ++a) {
                const int64_t nv = a == 0 ? d.nm : d.ns;
                for (int64_t r = 0; r < nv; r += GROWS) kit[a].push_back(WItem{q, a | (d.symm[a] ? 2 : 0), r});
                if (d.symm[a]) {
                    for (int64_t r = (nv - 1) / GROWS * GROWS; r >= 0; r -= GROWS) vit[a].push_back(WItem{q, a, r});
                    for (int64_t r = 0; r < nv; r += GFIN_ROWS) wl_fin.push_back(WItem{q, a, r});
                }
            }
            auto alternate = [](const std::vector<WItem> &u, size_t u0, size_t u1, const std::vector<WItem> &v,
                                size_t v0, size_t v1, std::vector<WItem> &out) {
                for (size_t i = u0, j = v0; i < u1 || j < v1;) {
                    if (i < u1) out.push_back(u[i++]);
                    if (j < v1) out.push_back(v[j++]);
                }
            };
            const size_t h0 = size_t(gemv_heavy(d.f32 != 0, int64_t(vit[0].size())));
            const size_t h1 = size_t(gemv_heavy(d.f32 != 0, int64_t(vit[1].size())));
            alternate(vit[0], 0, h0, vit[1], 0, h1, wl_gemv);
            alternate(kit[0], 0, kit[0].size(), kit[1], 0, kit[1].size(), wl_gemv_k);
            alternate(vit[0], h0, vit[0].size(), vit[1], h1, vit[1].size(), wl_gemv_v);
        }
        for (int64_t r = 0; r < p.nn; r += SLICE) wl_spmv.push_back(WItem{q, 0, r});
        for (int64_t k = 0; k < std::max(d.ldm, d.lds); k += CH) wl_pack.push_back(WItem{q, 0, k});
        maxiter_host = std::max(maxiter_host, J.maxit + J.maxit / std::max(m, 1) + 4);
    }
    wl_gemv.insert(wl_gemv.end(), wl_gemv_k.begin(), wl_gemv_k.end());
    wl_gemv.insert(wl_gemv.end(), wl_gemv_v.begin(), wl_gemv_v.end());
    int maxm = 0;
    for (auto *J : jobs) maxm = std::max(maxm, J->restart);
    // device copies of descriptors, states and work lists
    BatchBuffers &BB = batch_buffers();
    const size_t bytes = sizeof(GDesc) * nb + sizeof(GState) * nb +
                         sizeof(WItem) * (wl_vec.size() + wl_gemv.size() + wl_spmv.size() + wl_pack.size() +
                                          wl_dot.size() + wl_fin.size()) + 512;
    if (BB.dev_bytes < bytes) {
        if (BB.step) PB_HIP(hipGraphExecDestroy(BB.step));
        BB.step = nullptr;
        if (BB.dev) PB_HIP(hipFree(BB.dev));
        BB.dev = nullptr;
        PB_HIP(hipMalloc(&BB.dev, bytes));
        BB.dev_bytes = bytes;
    }
    char *cur = static_cast<char *>(BB.dev);
    auto put = [&](const void *src, size_t b) {
        char *d = cur;
        PB_HIP(hipMemcpyAsync(d, src, b, hipMemcpyHostToDevice, s));
        cur += (b + 15) / 16 * 16;
        return static_cast<void *>(d);
    };
    GDesc *dD = static_cast<GDesc *>(put(desc.data(), sizeof(GDesc) * nb));
    GState *dS = static_cast<GState *>(put(st.data(), sizeof(GState) * nb));
    WItem *dvec = static_cast<WItem *>(put(wl_vec.data(), sizeof(WItem) * wl_vec.size()));
    WItem *dgemv = static_cast<WItem *>(put(wl_gemv.data(), sizeof(WItem) * wl_gemv.size()));
    WItem *dspmv = static_cast<WItem *>(put(wl_spmv.data(), sizeof(WItem) * wl_spmv.size()));
    WItem *dpack = static_cast<WItem *>(put(wl_pack.data(), sizeof(WItem) * wl_pack.size()));
    WItem *ddot = static_cast<WItem *>(put(wl_dot.data(), sizeof(WItem) * wl_dot.size()));
    WItem *dfin = static_cast<WItem *>(put(wl_fin.data(), sizeof(WItem) * wl_fin.size()));
    int *dcount = reinterpret_cast<int *>(cur);
    PB_HIP(hipMemsetAsync(dcount, 0, sizeof(int), s));
    const unsigned nvec = unsigned(wl_vec.size()), ngemv = unsigned(wl_gemv.size()),
                   nspmv = unsigned(wl_spmv.size()), npack = unsigned(wl_pack.size()),
                   ndot = unsigned(wl_dot.size()), nfin = unsigned(wl_fin.size());
    const unsigned ngroups = unsigned((maxm + 1 + 7) / 8);

    EventTimer *tm = nullptr;
    for (auto *J : jobs)
        if (J->p->timing) {
            tm = &J->p->timer;
            break;
        }
    // Enqueue iterations; poll a completion counter copied to pinned memory
    // every POLL iterations, blocking only on the copy of the previous poll:
    // the device keeps 2 to 4 iterations queued, and at most that many launch
    // rounds return at once after the last instance has finished.
    const int POLL = 2;
    int polls = 0;
    bool finished = false;
    hipLaunchKernelGGL(k_cheb_coef, dim3(unsigned((nb + 63) / 64)), dim3(64), 0, s, dD, nb);
    int types = 0;
    bool any_mf = false;
    for (auto *J : jobs) {
        if (J->p->bem_mf) any_mf = true;
        else types |= J->p->precision == PBFB_MIXED ? 2 : 1;
    }
    // one Krylov step of the whole batch
    auto enqueue_step = [&]() {
        if (tm) tm->begin(T_PREC, s);
        hipLaunchKernelGGL(k_bprec0, dim3(nvec), dim3(256), 0, s, dvec, dD, dS);
        for (int step = 1; step < kmax; ++step)
            hipLaunchKernelGGL(k_bcheb, dim3(nspmv), dim3(256), 0, s, dspmv, dD, dS, step);
        if (tm) tm->end(s);
        if (tm) tm->begin(T_APPLY, s);
        hipLaunchKernelGGL(k_bpack, dim3(npack), dim3(256), 0, s, dpack, dD, dS);
        if (tm) tm->begin(T_GEMV, s);
        if (types & 1) hipLaunchKernelGGL(k_bgemv<double>, dim3(ngemv), dim3(GEMV_THREADS), 0, s, dgemv, dD, dS);
        if (types & 2) hipLaunchKernelGGL(k_bgemv<float>, dim3(ngemv), dim3(GEMV_THREADS), 0, s, dgemv, dD, dS);
        if (nfin) hipLaunchKernelGGL(k_bgemv_fin, dim3(nfin), dim3(256), 0, s, dfin, dD, dS);
        // matrix-free instances: their own launches, gated by their state word
        for (size_t q = 0; q < jobs.size() && any_mf; ++q) {
            Problem &pq = *jobs[q]->p;
            if (!pq.bem_mf) continue;
            const int *stq = reinterpret_cast<const int *>(dS + q);
            mf_apply(pq, 0, desc[q].xm, desc[q].w + pq.nn, stq, s);
            mf_apply(pq, 1, desc[q].xs, desc[q].w + pq.nn + pq.surf[0].nv, stq, s);
        }
        if (tm) {
            tm->end(s);
            tm->begin(T_SPMV, s);
        }
        hipLaunchKernelGGL(k_bspmv, dim3(nspmv), dim3(256), 0, s, dspmv, dD, dS);
        if (tm) {
            tm->end(s);
            tm->end(s);
        }
        hipLaunchKernelGGL(k_bmdot, dim3(ndot, ngroups), dim3(256), 0, s, ddot, dD, dS);
        hipLaunchKernelGGL(k_breduce, dim3(unsigned(nb), ngroups), dim3(256), 0, s, dD, dS, 0);
        hipLaunchKernelGGL(k_bmsub, dim3(nvec), dim3(256), 0, s, dvec, dD, dS, 0);
        hipLaunchKernelGGL(k_bmdot, dim3(ndot, ngroups), dim3(256), 0, s, ddot, dD, dS);
        hipLaunchKernelGGL(k_breduce, dim3(unsigned(nb), ngroups), dim3(256), 0, s, dD, dS, 1);
        hipLaunchKernelGGL(k_bmsub, dim3(nvec), dim3(256), 0, s, dvec, dD, dS, 1);
        hipLaunchKernelGGL(k_bnorm, dim3(unsigned(nb)), dim3(256), 0, s, dD, dS);
        hipLaunchKernelGGL(k_bscale, dim3(nvec), dim3(256), 0, s, dvec, dD, dS);
        hipLaunchKernelGGL(k_bcontrol, dim3(unsigned(nb)), dim3(64), 0, s, dD, dS, dcount);
        hipLaunchKernelGGL(k_bupdx, dim3(nvec), dim3(256), 0, s, dvec, dD, dS);
    };
    // Without timers the step is captured once as a HIP graph (kernel nodes
    // only) and replayed; the capture is reused while the buffer and launch
    // shapes stay the same (the Newton steps of a solve, repeated solves).
    bool graph = !tm && !any_mf; // matrix-free launches carry per-instance pointers: not captured
    for (auto *J : jobs) graph = graph && J->graph;
    if (graph) {
        const GraphKey key{BB.dev, nvec, ngemv, nspmv, npack, ndot, ngroups, unsigned(nb), nfin, kmax, types};
        if (!(BB.step && BB.key == key)) {
            if (BB.step) PB_HIP(hipGraphExecDestroy(BB.step));
            BB.step = nullptr;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
                enqueue_step();
                hipGraph_t g = nullptr;
                PB_HIP(hipStreamEndCapture(s, &g));
                PB_HIP(hipGraphInstantiate(&BB.step, g, nullptr, nullptr, 0));
                PB_HIP(hipGraphDestroy(g));
                BB.key = key;
            } else {
                (void)hipGetLastError(); // a stream that cannot be captured: launch one by one
                graph = false;
            }
        }
    }
    for (int it = 0; it < maxiter_host && !finished; ++it) {
        if (graph) PB_HIP(hipGraphLaunch(BB.step, s));
        else enqueue_step();
        PB_HIP(hipGetLastError());
        if ((it + 1) % POLL == 0) {
            const int slot = polls % 3;
            PB_HIP(hipMemcpyAsync(BB.pinned + slot, dcount, sizeof(int), hipMemcpyDeviceToHost, s));
            PB_HIP(hipEventRecord(BB.ev[slot], s));
            ++polls;
            if (polls >= 2) {
                const int old = (polls - 2) % 3; // the copy of the previous poll
                PB_HIP(hipEventSynchronize(BB.ev[old]));
                if (BB.pinned[old] >= nb) finished = true;
            }
            // a newer copy may already be complete.  A query of a pending
            // event returns hipErrorNotReady and HIP also records that as the
            // thread's last error, which the launch checks of the next
            // iteration would report; it is cleared here (launch errors of
            // this iteration were checked above).
            for (int k = 1; k <= 1 && !finished && polls - k >= 0; ++k) {
                const int sl = (polls - k) % 3;
                const hipError_t q = hipEventQuery(BB.ev[sl]);
                if (q == hipErrorNotReady) {
                    (void)hipGetLastError();
                    break;
                }
                PB_HIP(q);
                if (BB.pinned[sl] >= nb) finished = true;
            }
        }
    }
    PB_HIP(hipMemcpyAsync(st.data(), dS, sizeof(GState) * nb, hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < nb; ++q) {
        GmresJob &J = *jobs[q];
        J.iters = st[q].total;
        J.applies = st[q].napply;
        if (st[q].st == G_DONE) J.status = 0;
        else if (st[q].st == G_FAIL) J.status = st[q].code;
        else J.status = PBFB_ENOTCONV;
    }
}

} // namespace pbfb
