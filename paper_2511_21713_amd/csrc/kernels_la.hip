// Linear algebra of the coupled operator outside GMRES (residuals, the
// omega search, the C-ABI apply): surface packing, the dense Galerkin GEMV,
// the FEM sliced-ELL SpMV and small vector kernels.  Reductions use a fixed grid
// and a fixed tree, so every result is bitwise reproducible run to run.
#include <cmath>

#include "gemv_rows.hpp"
#include "pbfb_internal.hpp"
#include "sell_slice.hpp"

namespace pbfb {

static inline unsigned nb_(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

// ---------------------------------------------------------------------------
// packing: x_w = [u(g_w) | lambda_w | 0 pad] for both surfaces, in the
// Morton vertex order of the stored operators (gmv: FEM node, mv: surface
// vertex of each operator index; matrix-free: g and mv null, ascending order)
// ---------------------------------------------------------------------------
__global__ void k_pack(int64_t nn, int64_t nm, int64_t ns, int64_t ldm, int64_t lds, const int32_t *__restrict__ gmm,
                       const int32_t *__restrict__ mvm, const int32_t *__restrict__ gms,
                       const int32_t *__restrict__ mvs, const double *__restrict__ x, double *__restrict__ xm,
                       double *__restrict__ xs)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k < ldm) {
        double v = 0.0;
        if (k < nm) v = x[gmm[k]];
        else if (k < 2 * nm) v = x[nn + (mvm ? mvm[k - nm] : k - nm)];
        xm[k] = v;
    }
    if (k < lds) {
        double v = 0.0;
        if (k < ns) v = x[gms[k]];
        else if (k < 2 * ns) v = x[nn + nm + (mvs ? mvs[k - ns] : k - ns)];
        xs[k] = v;
    }
}

// ---------------------------------------------------------------------------
// dense GEMV over both surfaces in one launch (rows: gemv_rows.hpp)
// ---------------------------------------------------------------------------
// one surface's operator as the GEMV sees it
struct GemvSurf {
    const void *B;
    const double *x;
    double *y;
    const int32_t *oidx; // output position of each operator row (its vertex)
    void *P; // FP64 column partials of the symmetric use
    int64_t n, ld;
    int sym, f32;
    const int32_t *dptr, *dcol;
    const double *dval;
};

// work items in gemv_item order: K and V items of the symmetric use, full-row
// items of a surface that is not used symmetrically
struct GemvGrid {
    int64_t nk0, nk1, nv0, nv1, h0, h1;
};
template <typename MT>
__global__ void __launch_bounds__(GEMV_THREADS, gemv_occupancy<MT>()) k_gemv(GemvSurf S0, GemvSurf S1, GemvGrid W)
{
    const GemvItem it = gemv_item(blockIdx.x, W.nk0, W.nk1, W.nv0, W.nv1, W.h0, W.h1);
    const GemvSurf &S = it.s ? S1 : S0;
    const int64_t r0 = it.b * int64_t(GSYM);
    const MT *B = static_cast<const MT *>(S.B);
    if (!it.k) {
        gemv_rows_symV<MT>(B, S.x, static_cast<sym_part_t<MT> *>(S.P), S.n, S.ld, r0, threadIdx.x);
    } else if (S.sym) {
        gemv_rows_symK<MT>(B, S.x, S.y, S.oidx, S.n, S.ld, r0, threadIdx.x);
    } else {
        const int64_t rw = r0 + (threadIdx.x >> 6) * GEMV_RW;
        if (rw < S.n) gemv_rows<MT>(B, S.x, S.y, S.oidx, S.n, S.ld, rw, threadIdx.x & 63);
    }
}
// the grid of surfaces 0 / 1 (n0 = 0: surface 0 left out)
static GemvGrid gemv_grid(const GemvSurf &S0, int64_t n0, const GemvSurf &S1, int64_t n1)
{
    GemvGrid W;
    W.nk0 = (n0 + GSYM - 1) / GSYM;
    W.nk1 = (n1 + GSYM - 1) / GSYM;
    W.nv0 = S0.sym ? W.nk0 : 0;
    W.nv1 = S1.sym ? W.nk1 : 0;
    W.h0 = gemv_heavy(S0.f32 != 0, W.nv0);
    W.h1 = gemv_heavy(S1.f32 != 0, W.nv1);
    return W;
}
static unsigned gemv_items(const GemvGrid &W) { return unsigned(W.nk0 + W.nk1 + W.nv0 + W.nv1); }

// second stage of the symmetric use: transposed column partials and Delta
__global__ void __launch_bounds__(256) k_gemv_fin(GemvSurf S0, GemvSurf S1, int64_t nb0)
{
    const bool s1 = blockIdx.x >= nb0;
    const GemvSurf &S = s1 ? S1 : S0;
    if (!S.sym) return;
    const int64_t i0 = (s1 ? blockIdx.x - nb0 : blockIdx.x) * int64_t(GFIN_ROWS);
    gemv_sym_finish(S.n, static_cast<const double *>(S.P), S.dptr, S.dcol, S.dval, S.x, S.y, S.oidx, i0, threadIdx.x);
}

// ---------------------------------------------------------------------------
// FEM SpMV over the shell rows (sliced ELL): one workgroup per 64-row slice
// ---------------------------------------------------------------------------
template <typename VT>
__global__ void __launch_bounds__(256)
    k_spmv(int64_t nrows, const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
           const VT *__restrict__ val, const double *__restrict__ x, double *__restrict__ y)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = blockIdx.x;
    const double part = sell_part<VT, false>(sptr, col, val, x, q, lane, wv, nrows);
    const double s = sell_reduce(part, lane, wv);
    const int64_t row = q * SLICE + lane;
    if (wv == 0 && row < nrows) y[row] = s;
}

// ---------------------------------------------------------------------------
// vector kernels
// ---------------------------------------------------------------------------
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = a * x[i] + b * y[i];
}
__global__ void k_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = a[i] * x[i];
}

constexpr int RED_BLOCKS = 256;

struct PtrTab {
    const double *a[8];
    const double *b[8];
};

// partial dot products of k <= 8 vector pairs; partial[b * k + j] (skip:
// optional device flag, nonzero = nothing to do)
__global__ void __launch_bounds__(256) k_dots_partial(int64_t n, int k, PtrTab T, double *__restrict__ partial,
                                                      const int *__restrict__ skip)
{
    if (skip && *skip) return;
    const double *const *A = T.a;
    const double *const *Bv = T.b;
    __shared__ double red[8][256];
    double s[8];
    for (int j = 0; j < 8; ++j) s[j] = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        for (int j = 0; j < k; ++j) s[j] = fma(A[j][i], Bv[j][i], s[j]);
    for (int j = 0; j < k; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int j = 0; j < k; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < k) partial[blockIdx.x * k + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_reduce_partial(int nb, int k, const double *__restrict__ partial, double *__restrict__ out,
                                 const int *__restrict__ skip)
{
    if (skip && *skip) return;
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += partial[b * k + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

__global__ void k_add_vec(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = a[i] + b[i];
}

// ===========================================================================
// host wrappers
// ===========================================================================
// column partials of the symmetric use: ((nv + GSYM - 1) / GSYM) x nv FP64
int64_t sym_partials_doubles(int64_t nv) { return ((nv + GSYM - 1) / GSYM) * nv + nv; }

static GemvSurf gemv_surf(Problem &p, int w, const double *x, double *y, double *P)
{
    const SurfaceDev &D = p.surf[w];
    GemvSurf G{};
    G.B = D.B;
    G.x = x;
    G.y = y;
    G.oidx = D.mvert;
    G.n = D.nv;
    G.ld = bem_ld(D.nv);
    G.sym = D.sym ? 1 : 0;
    G.f32 = p.precision == PBFB_MIXED ? 1 : 0;
    G.P = D.sym ? P : nullptr;
    G.dptr = D.d_ptr;
    G.dcol = D.d_col;
    G.dval = D.d_val;
    return G;
}

// both surfaces' rows in one launch; skip_m leaves out Gamma_m (two-field form)
static void gemv_launch(Problem &p, const ApplyBufs &bf, double *y, hipStream_t s, bool skip_m, bool timed)
{
    const SurfaceDev &M = p.surf[0], &S = p.surf[1];
    const GemvSurf G0 = gemv_surf(p, 0, bf.xm, y + p.nn, bf.P[0]), G1 = gemv_surf(p, 1, bf.xs, y + p.nn + M.nv, bf.P[1]);
    const GemvGrid W = gemv_grid(G0, skip_m ? 0 : M.nv, G1, S.nv);
    if (timed) p.timer.begin(T_GEMV, s);
    if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_gemv<float>, dim3(gemv_items(W)), dim3(GEMV_THREADS), 0, s, G0, G1, W);
    else
        hipLaunchKernelGGL(k_gemv<double>, dim3(gemv_items(W)), dim3(GEMV_THREADS), 0, s, G0, G1, W);
    if (G0.sym || G1.sym) {
        const int64_t f0 = skip_m ? 0 : (M.nv + GFIN_ROWS - 1) / GFIN_ROWS, f1 = (S.nv + GFIN_ROWS - 1) / GFIN_ROWS;
        hipLaunchKernelGGL(k_gemv_fin, dim3(unsigned(f0 + f1)), dim3(256), 0, s, G0, G1, f0);
    }
    if (timed) p.timer.end(s);
}

// bufs: caller-provided work buffers (no allocation, no timing), else the
// problem's scratch
static void apply_impl(Problem &p, const double *x, double *y, bool with_jac, hipStream_t s,
                       const ApplyBufs *bufs = nullptr)
{
    const SurfaceDev &M = p.surf[0], &S = p.surf[1];
    const int64_t ldm = bem_ld(M.nv), lds = bem_ld(S.nv);
    ApplyBufs bf;
    if (bufs) {
        bf = *bufs;
    } else {
        bf.xm = scratch<double>(p, SCR_XM, ldm);
        bf.xs = scratch<double>(p, SCR_XS, lds);
        for (int w = 0; w < 2; ++w)
            bf.P[w] = p.surf[w].sym ? scratch<double>(p, w == 0 ? SCR_SYMP0 : SCR_SYMP1,
                                                      sym_partials_doubles(p.surf[w].nv))
                                    : nullptr;
    }
    const bool timed = p.timing && !bufs;
    if (timed) p.timer.begin(T_APPLY, s);
    hipLaunchKernelGGL(k_pack, dim3(nb_(std::max(ldm, lds), 256)), dim3(256), 0, s, p.nn, M.nv, S.nv, ldm, lds,
                       p.bem_mf ? M.g : M.gmv, p.bem_mf ? nullptr : M.mvert, p.bem_mf ? S.g : S.gmv,
                       p.bem_mf ? nullptr : S.mvert, x, bf.xm, bf.xs);
    if (p.bem_mf) {
        PB_CHECK(!bufs, PBFB_EINVAL, "matrix-free boundary operators need the problem's own work buffers");
        if (timed) p.timer.begin(T_GEMV, s);
        mf_apply(p, 0, bf.xm, y + p.nn, nullptr, s);
        mf_apply(p, 1, bf.xs, y + p.nn + p.surf[0].nv, nullptr, s);
        if (timed) p.timer.end(s);
    } else {
        gemv_launch(p, bf, y, s, p.two_field(), timed);
    }
    // two-field form: lambda_m is not an unknown of the solve; its row is the identity
    if (p.two_field())
        PB_HIP(hipMemcpyAsync(y + p.nn, x + p.nn, sizeof(double) * M.nv, hipMemcpyDeviceToDevice, s));
    if (timed) p.timer.begin(T_SPMV, s);
    const unsigned g = nb_(p.nn, SLICE);
    if (!with_jac)
        hipLaunchKernelGGL(k_spmv<double>, dim3(g), dim3(256), 0, s, p.nn, p.d_sptr, p.d_col, p.d_val0, x, y);
    else if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_spmv<float>, dim3(g), dim3(256), 0, s, p.nn, p.d_sptr, p.d_col, p.d_val32, x, y);
    else
        hipLaunchKernelGGL(k_spmv<double>, dim3(g), dim3(256), 0, s, p.nn, p.d_sptr, p.d_col, p.d_val, x, y);
    if (timed) {
        p.timer.end(s); // spmv
        p.timer.end(s); // apply
    }
    PB_HIP(hipGetLastError());
}

void coupled_apply(Problem &p, const double *x, double *y, hipStream_t s) { apply_impl(p, x, y, true, s); }
void coupled_apply_linear_bufs(Problem &p, const double *x, double *y, hipStream_t s, const ApplyBufs &bufs)
{
    apply_impl(p, x, y, false, s, &bufs);
}

// ---------------------------------------------------------------------------
// lambda_m from the trace of u (two-field form, Sec. 2.3.1):
// V0 lam = (1/2 M_m + K0_m) u_m - [with_load] f_m, with the stored Gamma_m
// rows [K' | V'] = [1/2 M_m + K0_m | -V0]: the right-hand side is the row
// product with [u_m | 0], and V0 p = -(row product with [0 | p]).  V0 is
// symmetric positive definite, so conjugate gradients with its diagonal as
// preconditioner.
// ---------------------------------------------------------------------------
// packed Gamma_m input in the operator's Morton vertex order (gmv: FEM node,
// mv: surface vertex of each operator index)
__global__ void k_pack_m(int64_t nm, int64_t ldm, const int32_t *__restrict__ gmv, const int32_t *__restrict__ mv,
                         const double *__restrict__ u, const double *__restrict__ lam, double *__restrict__ xm)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k >= ldm) return;
    double v = 0.0;
    if (k < nm) v = u ? u[gmv[k]] : 0.0;
    else if (k < 2 * nm) v = lam ? lam[mv[k - nm]] : 0.0;
    xm[k] = v;
}

// packed Gamma_m input [trace of u | 0] of an independent Gamma_m mesh: at
// Morton position k the P1 interpolant of u at vertex mv[k] (loc: its tet and
// barycentric coordinates, 6 doubles per vertex)
__global__ void k_pack_trace(int64_t nm, int64_t ldm, const int32_t *__restrict__ mv, const double *__restrict__ loc,
                             const int32_t *__restrict__ tet, const double *__restrict__ u, double *__restrict__ xm)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k >= ldm) return;
    double v = 0.0;
    if (k < nm) {
        const double *l = loc + 6 * int64_t(mv[k]);
        const int32_t *T = tet + 4 * int64_t(l[0]);
        v = l[2] * u[T[0]] + l[3] * u[T[1]] + l[4] * u[T[2]] + l[5] * u[T[3]];
    }
    xm[k] = v;
}

template <typename MT>
__global__ void k_vdiag_inv(int64_t nm, int64_t ld, const int32_t *__restrict__ mv, const MT *__restrict__ B,
                            double *__restrict__ dinv)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k < nm) dinv[mv[k]] = -1.0 / double(B[k * ld + nm + k]);
}

// rows of one Gamma_m operator (w = 0, or 2: an independent Gamma_m mesh)
static void gemv_m(Problem &p, int w, const double *xm, double *y, hipStream_t s)
{
    const GemvSurf G = gemv_surf(p, w, xm, y,
                                 p.surf[w].sym ? scratch<double>(p, w == 0 ? SCR_SYMP0 : SCR_SYMP2,
                                                                 sym_partials_doubles(p.surf[w].nv))
                                               : nullptr);
    const int64_t f0 = (G.n + GFIN_ROWS - 1) / GFIN_ROWS;
    const GemvGrid W = gemv_grid(G, G.n, G, 0);
    if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_gemv<float>, dim3(gemv_items(W)), dim3(GEMV_THREADS), 0, s, G, G, W);
    else
        hipLaunchKernelGGL(k_gemv<double>, dim3(gemv_items(W)), dim3(GEMV_THREADS), 0, s, G, G, W);
    if (G.sym) hipLaunchKernelGGL(k_gemv_fin, dim3(unsigned(f0)), dim3(256), 0, s, G, G, f0);
}

// CG scalars kept on the device (sc[0] = r.z, sc[1] = alpha, sc[2] = beta,
// sc[3] = r.r): no host round trip per step
__global__ void k_cg_alpha(const double *__restrict__ pq, double *__restrict__ sc)
{
    if (threadIdx.x == 0) sc[1] = pq[0] != 0.0 ? -sc[0] / pq[0] : 0.0; // q = -V0 d
}
__global__ void k_cg_beta(const double *__restrict__ red, double *__restrict__ sc)
{
    if (threadIdx.x == 0) {
        sc[2] = sc[0] != 0.0 ? red[0] / sc[0] : 0.0;
        sc[0] = red[0];
        sc[3] = red[1];
    }
}
__global__ void k_cg_dir(int64_t n, const double *__restrict__ sc, const double *__restrict__ z, double *__restrict__ d)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) d[i] = z[i] + sc[2] * d[i];
}

// z = -1/2 (S + S^T) r with S the 1-ring approximate inverse of V' = -V0 (the
// GMRES preconditioner's block; the 1-ring pattern is symmetric, tslot[e] is
// the slot of the transposed entry): a symmetric approximation of V0^-1
__global__ void k_cg_spai(int64_t n, const int32_t *__restrict__ ptr, const int32_t *__restrict__ col,
                          const double *__restrict__ val, const int32_t *__restrict__ tslot,
                          const double *__restrict__ r, double *__restrict__ z)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) acc += (val[e] + val[tslot[e]]) * r[col[e]];
    z[i] = -0.5 * acc;
}
__global__ void k_cg_update_spai(int64_t n, const double *__restrict__ sc, const double *__restrict__ d,
                                 const double *__restrict__ q, double *__restrict__ lam, double *__restrict__ r)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    const double a = sc[1];
    lam[i] += a * d[i];
    r[i] += a * q[i];
}

void lambda_m_recover(Problem &p, const double *phi, bool with_load, double *lam, hipStream_t s)
{
    PB_CHECK(!p.bem_mf, PBFB_ESTATE, "the two-field form needs the dense Gamma_m operator");
    ensure_rhs(p, s);
    // the surface that carries lambda_m: Gamma_m, or the independent Gamma_m
    // mesh (whose trace of u is the P1 interpolant at its vertices)
    const int w = p.gm();
    ensure_bem(p, w, s);
    const SurfaceDev &M = p.surf[w];
    const SurfaceTopo &TM = p.topo[w];
    const int64_t nm = M.nv, ldm = bem_ld(nm);
    double *xm = scratch<double>(p, SCR_CGX, ldm);
    double *wv = scratch<double>(p, SCR_CGV, 6 * nm + 8);
    double *b = wv, *r = wv + nm, *z = wv + 2 * nm, *d = wv + 3 * nm, *q = wv + 4 * nm, *dinv = wv + 5 * nm,
           *sc = wv + 6 * nm;
    double *part = scratch<double>(p, SCR_DOT, RED_BLOCKS * 8 + 8), *red = part + RED_BLOCKS * 8;
    const unsigned g = nb_(ldm, 256), gn = nb_(nm, 256);
    auto dev_dots = [&](int k, const double *a0, const double *b0, const double *a1, const double *b1) {
        PtrTab T{};
        T.a[0] = a0;
        T.b[0] = b0;
        T.a[1] = a1;
        T.b[1] = b1;
        hipLaunchKernelGGL(k_dots_partial, dim3(RED_BLOCKS), dim3(256), 0, s, nm, k, T, part, (const int *)nullptr);
        hipLaunchKernelGGL(k_reduce_partial, dim3(k), dim3(256), 0, s, RED_BLOCKS, k, part, red,
                           (const int *)nullptr);
    };
    if (M.iw)
        hipLaunchKernelGGL(k_pack_trace, dim3(g), dim3(256), 0, s, nm, ldm, M.mvert, M.iw, p.d_tet, phi, xm);
    else
        hipLaunchKernelGGL(k_pack_m, dim3(g), dim3(256), 0, s, nm, ldm, M.gmv, M.mvert, phi, (const double *)nullptr,
                           xm);
    gemv_m(p, w, xm, b, s);
    if (with_load && p.nq > 0) vec_axpby(nm, -1.0, scratch<double>(p, SCR_FM, nm), 1.0, b, s);
    if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_vdiag_inv<float>, dim3(gn), dim3(256), 0, s, nm, ldm, M.mvert,
                           static_cast<const float *>(M.B), dinv);
    else
        hipLaunchKernelGGL(k_vdiag_inv<double>, dim3(gn), dim3(256), 0, s, nm, ldm, M.mvert,
                           static_cast<const double *>(M.B), dinv);
    // transposed slots of the approximate inverse's 1-ring pattern (host, from the topology)
    int32_t *tslot = nullptr;
    if (M.spai && !TM.ring_ptr.empty()) {
        std::vector<int32_t> ts(TM.ring.size(), -1);
        bool ok = true;
        for (int64_t i = 0; i < nm && ok; ++i)
            for (int32_t e = TM.ring_ptr[i]; e < TM.ring_ptr[i + 1] && ok; ++e) {
                const int32_t j = TM.ring[e];
                for (int32_t f = TM.ring_ptr[j]; f < TM.ring_ptr[j + 1]; ++f)
                    if (TM.ring[f] == i) ts[e] = f;
                ok = ts[e] >= 0;
            }
        if (ok) {
            tslot = scratch<int32_t>(p, SCR_TSLOT, ts.size());
            PB_HIP(hipMemcpyAsync(tslot, ts.data(), sizeof(int32_t) * ts.size(), hipMemcpyHostToDevice, s));
        }
    }
    auto precond = [&](const double *rr, double *zz) {
        if (tslot)
            hipLaunchKernelGGL(k_cg_spai, dim3(gn), dim3(256), 0, s, nm, M.ring_ptr, M.ring, M.spai, tslot, rr, zz);
        else
            vec_mul(nm, dinv, rr, zz, s);
    };
    double h[4];
    dev_dots(1, b, b, nullptr, nullptr);
    PB_HIP(hipMemcpyAsync(h, red, sizeof(double), hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    const double b0 = std::sqrt(h[0]), tol = 1e-13 * b0;
    PB_HIP(hipMemsetAsync(lam, 0, sizeof(double) * nm, s));
    if (b0 == 0.0) return;
    // one CG run from lam = 0; false if the preconditioner lost definiteness or
    // the step budget ran out.  Convergence is read back every CHECK steps.
    auto run = [&](int maxit) -> bool {
        PB_HIP(hipMemsetAsync(lam, 0, sizeof(double) * nm, s));
        PB_HIP(hipMemcpyAsync(r, b, sizeof(double) * nm, hipMemcpyDeviceToDevice, s));
        precond(r, z);
        PB_HIP(hipMemcpyAsync(d, z, sizeof(double) * nm, hipMemcpyDeviceToDevice, s));
        dev_dots(2, r, z, r, r);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, s, red, sc); // sc[0] = r.z, sc[3] = r.r
        PB_HIP(hipMemcpyAsync(h, sc, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
        PB_HIP(hipStreamSynchronize(s));
        if (!(h[0] > 0.0)) return false;
        constexpr int CHECK = 8;
        for (int it = 0; it < maxit;) {
            for (int k = 0; k < CHECK; ++k, ++it) {
                hipLaunchKernelGGL(k_pack_m, dim3(g), dim3(256), 0, s, nm, ldm, M.gmv, M.mvert, (const double *)nullptr, d,
                                   xm);
                gemv_m(p, w, xm, q, s); // q = V' d = -V0 d
                dev_dots(1, d, q, nullptr, nullptr);
                hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, s, red, sc);
                hipLaunchKernelGGL(k_cg_update_spai, dim3(gn), dim3(256), 0, s, nm, sc, d, q, lam, r);
                precond(r, z);
                dev_dots(2, r, z, r, r);
                hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, s, red, sc);
                hipLaunchKernelGGL(k_cg_dir, dim3(gn), dim3(256), 0, s, nm, sc, z, d);
            }
            PB_HIP(hipMemcpyAsync(h, sc, sizeof(double) * 4, hipMemcpyDeviceToHost, s));
            PB_HIP(hipStreamSynchronize(s));
            if (!std::isfinite(h[0]) || !std::isfinite(h[3]) || !(h[0] > 0.0)) return std::sqrt(h[3]) <= tol;
            if (std::sqrt(h[3]) <= tol) return true;
        }
        return false;
    };
    const int maxit = int(std::min<int64_t>(20 * nm + 100, 20000));
    if (tslot && run(std::min(maxit, 2000))) return;
    tslot = nullptr; // the diagonal of V0 instead
    PB_CHECK(run(maxit), PBFB_ENOTCONV, "lambda_m recovery did not converge");
}
void coupled_apply_linear(Problem &p, const double *x, double *y, hipStream_t s) { apply_impl(p, x, y, false, s); }

void dots_dev(Problem &p, int k, const double *const *a, const double *const *b, int64_t n, double *out,
              const int *skip, hipStream_t s)
{
    // k <= 8 pairs; fixed-order partial sums over RED_BLOCKS blocks, then one block each
    double *part = scratch<double>(p, SCR_DOT, RED_BLOCKS * 8 + 8);
    PtrTab T{};
    for (int j = 0; j < k; ++j) {
        T.a[j] = a[j];
        T.b[j] = b[j];
    }
    hipLaunchKernelGGL(k_dots_partial, dim3(RED_BLOCKS), dim3(256), 0, s, n, k, T, part, skip);
    hipLaunchKernelGGL(k_reduce_partial, dim3(k), dim3(256), 0, s, RED_BLOCKS, k, part, out, skip);
}

void dots(Problem &p, int k, const double *const *a, const double *const *b, int64_t n, double *out, hipStream_t s)
{
    double *res = scratch<double>(p, SCR_DOT, RED_BLOCKS * 8 + 8) + RED_BLOCKS * 8;
    dots_dev(p, k, a, b, n, res, nullptr, s);
    PB_HIP(hipMemcpyAsync(out, res, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
}

double dot(Problem &p, const double *a, const double *b, int64_t n, hipStream_t s)
{
    double r;
    dots(p, 1, &a, &b, n, &r, s);
    return r;
}

// ---- kernels used by the solver (exported through small wrappers) ----------
void vec_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(nb_(n, 256)), dim3(256), 0, s, n, a, x, b, y);
}
void vec_mul(int64_t n, const double *a, const double *x, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_mul, dim3(nb_(n, 256)), dim3(256), 0, s, n, a, x, y);
}
void vec_add(int64_t n, const double *a, const double *b, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_add_vec, dim3(nb_(n, 256)), dim3(256), 0, s, n, a, b, y);
}

} // namespace pbfb
