// Linear algebra of the coupled operator: surface packing, the dense
// Galerkin GEMV (the bandwidth-bound hot kernel), the FEM CSR SpMV and the
// vector kernels of GMRES.  Reductions use a fixed grid and a fixed tree, so
// every result is bitwise reproducible run to run.
#include <cmath>

#include "pbfb_internal.hpp"

namespace pbfb {

static inline unsigned nb_(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// packing: x_w = [u(g_w) | lambda_w | 0 pad] for both surfaces
// ---------------------------------------------------------------------------
__global__ void k_pack(int64_t nn, int64_t nm, int64_t ns, int64_t ldm, int64_t lds, const int32_t *__restrict__ gm,
                       const int32_t *__restrict__ gs, const double *__restrict__ x, double *__restrict__ xm,
                       double *__restrict__ xs)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k < ldm) {
        double v = 0.0;
        if (k < nm) v = x[gm[k]];
        else if (k < 2 * nm) v = x[nn + (k - nm)];
        xm[k] = v;
    }
    if (k < lds) {
        double v = 0.0;
        if (k < ns) v = x[gs[k]];
        else if (k < 2 * ns) v = x[nn + nm + (k - ns)];
        xs[k] = v;
    }
}

// ---------------------------------------------------------------------------
// dense GEMV over both surfaces in one launch.  A wavefront owns RW rows and
// streams them with 16-byte loads; the packed input chunk is loaded once per
// wavefront and reused for its RW rows.  Row sums are reduced across the
// wavefront with xor shuffles.  Rows are padded to ld (multiple of 256).
// ---------------------------------------------------------------------------
template <int RW>
__global__ void __launch_bounds__(256)
    k_gemv_f64(const double *__restrict__ B0, const double *__restrict__ x0, double *__restrict__ y0, int64_t n0,
               int64_t ld0, int64_t nblk0, const double *__restrict__ B1, const double *__restrict__ x1,
               double *__restrict__ y1, int64_t n1, int64_t ld1)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool s1 = blockIdx.x >= nblk0;
    const double *B = s1 ? B1 : B0;
    const double *x = s1 ? x1 : x0;
    double *y = s1 ? y1 : y0;
    const int64_t n = s1 ? n1 : n0, ld = s1 ? ld1 : ld0;
    const int64_t r0 = ((s1 ? blockIdx.x - nblk0 : blockIdx.x) * 4 + wv) * RW;
    if (r0 >= n) return;
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    const dvec2 *xv = reinterpret_cast<const dvec2 *>(x);
    const int64_t nchunk = ld / 128; // 64 lanes x 2 doubles
    const dvec2 *rows[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int64_t rr = r0 + r < n ? r0 + r : n - 1;
        rows[r] = reinterpret_cast<const dvec2 *>(B + rr * ld);
    }
#pragma unroll 2
    for (int64_t c = 0; c < nchunk; ++c) {
        const dvec2 xx = xv[c * 64 + lane];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const dvec2 b = __builtin_nontemporal_load(rows[r] + c * 64 + lane);
            acc[r] = fma(b.x, xx.x, acc[r]);
            acc[r] = fma(b.y, xx.y, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
    if (lane < RW && r0 + lane < n) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < RW; ++r)
            if (lane == r) v = acc[r];
        y[r0 + lane] = v;
    }
}

// FP32 storage, FP64 accumulation (mixed precision)
template <int RW>
__global__ void __launch_bounds__(256)
    k_gemv_f32(const float *__restrict__ B0, const double *__restrict__ x0, double *__restrict__ y0, int64_t n0,
               int64_t ld0, int64_t nblk0, const float *__restrict__ B1, const double *__restrict__ x1,
               double *__restrict__ y1, int64_t n1, int64_t ld1)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const bool s1 = blockIdx.x >= nblk0;
    const float *B = s1 ? B1 : B0;
    const double *x = s1 ? x1 : x0;
    double *y = s1 ? y1 : y0;
    const int64_t n = s1 ? n1 : n0, ld = s1 ? ld1 : ld0;
    const int64_t r0 = ((s1 ? blockIdx.x - nblk0 : blockIdx.x) * 4 + wv) * RW;
    if (r0 >= n) return;
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    const int64_t nchunk = ld / 256; // 64 lanes x 4 floats
    const fvec4 *rows[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int64_t rr = r0 + r < n ? r0 + r : n - 1;
        rows[r] = reinterpret_cast<const fvec4 *>(B + rr * ld);
    }
    const dvec2 *xv = reinterpret_cast<const dvec2 *>(x);
#pragma unroll 2
    for (int64_t c = 0; c < nchunk; ++c) {
        const dvec2 xa = xv[(c * 64 + lane) * 2], xb = xv[(c * 64 + lane) * 2 + 1];
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            const fvec4 b = __builtin_nontemporal_load(rows[r] + c * 64 + lane);
            acc[r] = fma(double(b.x), xa.x, acc[r]);
            acc[r] = fma(double(b.y), xa.y, acc[r]);
            acc[r] = fma(double(b.z), xb.x, acc[r]);
            acc[r] = fma(double(b.w), xb.y, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
    if (lane < RW && r0 + lane < n) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < RW; ++r)
            if (lane == r) v = acc[r];
        y[r0 + lane] = v;
    }
}

// ---------------------------------------------------------------------------
// FEM CSR SpMV over the shell rows, 8 lanes per row
// ---------------------------------------------------------------------------
template <typename VT>
__global__ void __launch_bounds__(256)
    k_spmv(int64_t nrows, const int32_t *__restrict__ rowptr, const int32_t *__restrict__ col,
           const VT *__restrict__ val, const double *__restrict__ x, double *__restrict__ y)
{
    const int64_t row = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) >> 3;
    const int sub = threadIdx.x & 7;
    double s = 0.0;
    if (row < nrows) {
        const int32_t e = rowptr[row + 1];
        for (int32_t j = rowptr[row] + sub; j < e; j += 8) s = fma(double(val[j]), x[col[j]], s);
    }
    s += __shfl_xor(s, 4);
    s += __shfl_xor(s, 2);
    s += __shfl_xor(s, 1);
    if (sub == 0 && row < nrows) y[row] = s;
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
__global__ void k_scale_dev(int64_t n, const double *__restrict__ num, const double *__restrict__ x,
                            double *__restrict__ y)
{
    // y = x / sqrt(num[0]) (normalisation with a device-resident squared norm)
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const double d = sqrt(num[0]);
    if (i < n) y[i] = d > 0 ? x[i] / d : 0.0;
}

constexpr int RED_BLOCKS = 256;

struct PtrTab {
    const double *a[8];
    const double *b[8];
};

// partial dot products of k <= 8 vector pairs; partial[b * k + j]
__global__ void __launch_bounds__(256) k_dots_partial(int64_t n, int k, PtrTab T, double *__restrict__ partial)
{
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

__global__ void k_reduce_partial(int nb, int k, const double *__restrict__ partial, double *__restrict__ out)
{
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

// h[j] = V_j . w for j < k (basis stored with stride ldv); partials per block
// of rows: partial[b * kmax + j]
__global__ void __launch_bounds__(256)
    k_mdot_partial(int64_t n, int k, const double *__restrict__ Vb, int64_t ldv, const double *__restrict__ w,
                   double *__restrict__ partial, int kmax)
{
    __shared__ double red[8][256];
    const int j0 = blockIdx.y * 8;
    const int kk = min(8, k - j0);
    double s[8];
    for (int j = 0; j < 8; ++j) s[j] = 0.0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j < kk) s[j] = fma(Vb[(j0 + j) * ldv + i], wi, s[j]);
    }
    for (int j = 0; j < 8; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int wd = 128; wd > 0; wd >>= 1) {
        if (threadIdx.x < wd)
            for (int j = 0; j < 8; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + wd];
        __syncthreads();
    }
    if (threadIdx.x < kk) partial[blockIdx.x * kmax + j0 + threadIdx.x] = red[threadIdx.x][0];
}

// w -= sum_j h[j] V_j ; hacc[j] += h[j] (thread 0 of block 0)
__global__ void k_msub(int64_t n, int k, const double *__restrict__ Vb, int64_t ldv, const double *__restrict__ h,
                       double *__restrict__ w)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = w[i];
    for (int j = 0; j < k; ++j) s = fma(-h[j], Vb[j * ldv + i], s);
    w[i] = s;
}

// x += dinv .* (sum_j y_j V_j)
__global__ void k_update(int64_t n, int k, const double *__restrict__ Vb, int64_t ldv, const double *__restrict__ y,
                         const double *__restrict__ dinv, double *__restrict__ x)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s = fma(y[j], Vb[j * ldv + i], s);
    x[i] += dinv[i] * s;
}

__global__ void k_add_vec(int64_t n, const double *__restrict__ a, const double *__restrict__ b, double *__restrict__ y)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i < n) y[i] = a[i] + b[i];
}

// ===========================================================================
// host wrappers
// ===========================================================================
static void gemv_launch(Problem &p, const double *xm, const double *xs, double *y, hipStream_t s)
{
    constexpr int RW = 4;
    const SurfaceDev &M = p.surf[0], &S = p.surf[1];
    const int64_t ldm = bem_ld(M.nv), lds = bem_ld(S.nv);
    const int64_t nb0 = (M.nv + 4 * RW - 1) / (4 * RW), nb1 = (S.nv + 4 * RW - 1) / (4 * RW);
    double *ym = y + p.nn, *ys = y + p.nn + M.nv;
    if (p.timing) p.timer.begin(T_GEMV, s);
    if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_gemv_f32<RW>, dim3(unsigned(nb0 + nb1)), dim3(256), 0, s, (const float *)M.B, xm, ym,
                           M.nv, ldm, nb0, (const float *)S.B, xs, ys, S.nv, lds);
    else
        hipLaunchKernelGGL(k_gemv_f64<RW>, dim3(unsigned(nb0 + nb1)), dim3(256), 0, s, (const double *)M.B, xm, ym,
                           M.nv, ldm, nb0, (const double *)S.B, xs, ys, S.nv, lds);
    if (p.timing) p.timer.end(s);
}

static void apply_impl(Problem &p, const double *x, double *y, bool with_jac, hipStream_t s)
{
    const SurfaceDev &M = p.surf[0], &S = p.surf[1];
    const int64_t ldm = bem_ld(M.nv), lds = bem_ld(S.nv);
    double *xm = scratch<double>(p, SCR_XM, ldm);
    double *xs = scratch<double>(p, SCR_XS, lds);
    if (p.timing) p.timer.begin(T_APPLY, s);
    hipLaunchKernelGGL(k_pack, dim3(nb_(std::max(ldm, lds), 256)), dim3(256), 0, s, p.nn, M.nv, S.nv, ldm, lds, M.g,
                       S.g, x, xm, xs);
    gemv_launch(p, xm, xs, y, s);
    if (p.timing) p.timer.begin(T_SPMV, s);
    const unsigned g = nb_(p.nn * 8, 256);
    if (!with_jac)
        hipLaunchKernelGGL(k_spmv<double>, dim3(g), dim3(256), 0, s, p.nn, p.d_rowptr, p.d_col, p.d_val0, x, y);
    else if (p.precision == PBFB_MIXED)
        hipLaunchKernelGGL(k_spmv<float>, dim3(g), dim3(256), 0, s, p.nn, p.d_rowptr, p.d_col, p.d_val32, x, y);
    else
        hipLaunchKernelGGL(k_spmv<double>, dim3(g), dim3(256), 0, s, p.nn, p.d_rowptr, p.d_col, p.d_val, x, y);
    if (p.timing) {
        p.timer.end(s); // spmv
        p.timer.end(s); // apply
    }
    PB_HIP(hipGetLastError());
}

void coupled_apply(Problem &p, const double *x, double *y, hipStream_t s) { apply_impl(p, x, y, true, s); }
void coupled_apply_linear(Problem &p, const double *x, double *y, hipStream_t s) { apply_impl(p, x, y, false, s); }

void dots(Problem &p, int k, const double *const *a, const double *const *b, int64_t n, double *out, hipStream_t s)
{
    // k <= 8 pairs
    double *part = scratch<double>(p, SCR_DOT, RED_BLOCKS * 8 + 8);
    double *res = part + RED_BLOCKS * 8;
    PtrTab T{};
    for (int j = 0; j < k; ++j) {
        T.a[j] = a[j];
        T.b[j] = b[j];
    }
    hipLaunchKernelGGL(k_dots_partial, dim3(RED_BLOCKS), dim3(256), 0, s, n, k, T, part);
    hipLaunchKernelGGL(k_reduce_partial, dim3(k), dim3(256), 0, s, RED_BLOCKS, k, part, res);
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
void vec_scale_dev(int64_t n, const double *num, const double *x, double *y, hipStream_t s)
{
    hipLaunchKernelGGL(k_scale_dev, dim3(nb_(n, 256)), dim3(256), 0, s, n, num, x, y);
}
// h[0..k) = V^T w into device array h (partials in part, size RED_BLOCKS * kmax)
void basis_dots(int64_t n, int k, const double *Vb, int64_t ldv, const double *w, double *part, int kmax, double *h,
                hipStream_t s)
{
    const int nbx = 128;
    hipLaunchKernelGGL(k_mdot_partial, dim3(nbx, (k + 7) / 8), dim3(256), 0, s, n, k, Vb, ldv, w, part, kmax);
    hipLaunchKernelGGL(k_reduce_partial, dim3(k), dim3(256), 0, s, nbx, kmax, part, h);
}
void basis_sub(int64_t n, int k, const double *Vb, int64_t ldv, const double *h, double *w, hipStream_t s)
{
    hipLaunchKernelGGL(k_msub, dim3(nb_(n, 256)), dim3(256), 0, s, n, k, Vb, ldv, h, w);
}
void basis_update(int64_t n, int k, const double *Vb, int64_t ldv, const double *y, const double *dinv, double *x,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_update, dim3(nb_(n, 256)), dim3(256), 0, s, n, k, Vb, ldv, y, dinv, x);
}
void sq_norm_dev(Problem &p, int64_t n, const double *x, double *out_dev, hipStream_t s)
{
    double *part = scratch<double>(p, SCR_NRM, RED_BLOCKS);
    PtrTab T{};
    T.a[0] = x;
    T.b[0] = x;
    hipLaunchKernelGGL(k_dots_partial, dim3(RED_BLOCKS), dim3(256), 0, s, n, 1, T, part);
    hipLaunchKernelGGL(k_reduce_partial, dim3(1), dim3(256), 0, s, RED_BLOCKS, 1, part, out_dev);
}

} // namespace pbfb
