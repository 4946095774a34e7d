// Dense Galerkin GEMV rows: y[oidx[r]] = sum_c B[r][c] x[c] for the rows owned
// by one wavefront (oidx: the output position of operator row r).  B is a surface operator [K' | V'] stored row-major with a
// padded row length ld (a multiple of 256 entries, zero past 2n); x is the
// packed FP64 input of the same length.  A wavefront owns RW consecutive
// rows and streams them with 16-byte non-temporal loads (the operator is
// read once per apply and must not evict the vectors from L2); the input
// chunk is loaded once and reused for the RW rows; the row sums are reduced
// across the 64 lanes with xor shuffles in a fixed order, so the result is
// bitwise reproducible.  FP32 storage is widened and accumulated in FP64.
//
// This is the bandwidth-bound kernel of every coupled apply: it reads
// n * ld * sizeof(MT) bytes of operator per interface.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

namespace pbfb {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

constexpr int GEMV_RW = 4; // rows per wavefront

template <typename MT>
__device__ inline void gemv_rows(const MT *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                 const int32_t *__restrict__ oidx, int64_t n, int64_t ld, int64_t r0, int lane)
{
    constexpr int RW = GEMV_RW;
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) acc[r] = 0.0;
    if constexpr (sizeof(MT) == 8) {
        const dvec2 *xv = reinterpret_cast<const dvec2 *>(x);
        const dvec2 *rows[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) rows[r] = reinterpret_cast<const dvec2 *>(B + (r0 + r < n ? r0 + r : n - 1) * ld);
        const int64_t nc = ld / 128; // 64 lanes x 2 doubles
#pragma unroll 2
        for (int64_t c = 0; c < nc; ++c) {
            const dvec2 xx = xv[c * 64 + lane];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const dvec2 bb = __builtin_nontemporal_load(rows[r] + c * 64 + lane);
                acc[r] = fma(bb.x, xx.x, acc[r]);
                acc[r] = fma(bb.y, xx.y, acc[r]);
            }
        }
    } else {
        const dvec2 *xv = reinterpret_cast<const dvec2 *>(x);
        const fvec4 *rows[RW];
#pragma unroll
        for (int r = 0; r < RW; ++r) rows[r] = reinterpret_cast<const fvec4 *>(B + (r0 + r < n ? r0 + r : n - 1) * ld);
        const int64_t nc = ld / 256; // 64 lanes x 4 floats
#pragma unroll 2
        for (int64_t c = 0; c < nc; ++c) {
            const dvec2 xa = xv[(c * 64 + lane) * 2], xb = xv[(c * 64 + lane) * 2 + 1];
#pragma unroll
            for (int r = 0; r < RW; ++r) {
                const fvec4 bb = __builtin_nontemporal_load(rows[r] + c * 64 + lane);
                acc[r] = fma(double(bb.x), xa.x, acc[r]);
                acc[r] = fma(double(bb.y), xa.y, acc[r]);
                acc[r] = fma(double(bb.z), xb.x, acc[r]);
                acc[r] = fma(double(bb.w), xb.y, acc[r]);
            }
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
        y[oidx[r0 + lane]] = v;
    }
}

// Symmetric single layer.  The regular part of V' is stored bitwise
// symmetric; the touching-pair blocks make V' differ from its transpose on
// a sparse pattern only, kept as Delta = upper(V') - lower(V')^T.  A workgroup
// of 4 wavefronts owns GSYM = 16 rows r0.. (r0 a multiple of 16) and reads
// K' in full but V' only up to its diagonal block:
//   y_i = sum_j K'_ij u_j + sum_{j <= i} V'_ij l_j                  (here)
//       + sum_{j > i} V'_ji l_j + sum_{j > i} Delta_ij l_j      (gemv_sym_finish)
// For the third sum the workgroup forms the column sums
// P[blk][j] = sum_{r in its rows, r > j} V'_rj l_r over the V' columns it
// reads (the four wavefronts' partials added in LDS in wavefront order, in
// groups of gsym_g chunks of the row stream), blk = r0 / 16.  Rows past n
// contribute nothing.  Reads n + r0 + 16 entries of each row instead of 2 n.
constexpr int GSYM = 4 * GEMV_RW;
// chunks per LDS exchange (FP64 storage: 16, 64 KB of column partials per
// workgroup, two workgroups per CU: measured 4 % faster than 8 at the
// 80k-triangle size; FP32: 4, 32 KB).  The partials are FP64 for both
// storage precisions: with FP32 partials the apply is linear only to FP32
// rounding of the partial sums, which left strongly charged instances short
// of the Newton tolerance in mixed mode.
template <typename MT> constexpr int gsym_g() { return sizeof(MT) == 8 ? 16 : 4; }
// occupancy of the dense-apply kernels: the FP64 symmetric form's LDS allows two workgroups per CU
template <typename MT> constexpr int gemv_occupancy() { return sizeof(MT) == 8 ? 2 : 4; }
template <typename MT> using sym_part_t = double;

template <typename MT>
__device__ inline void gemv_rows_sym(const MT *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                     const int32_t *__restrict__ oidx, sym_part_t<MT> *__restrict__ P, int64_t n,
                                     int64_t ld, int64_t r0, int tid)
{
    using PT = sym_part_t<MT>;
    constexpr int RW = GEMV_RW;
    constexpr int EL = sizeof(MT) == 8 ? 2 : 4; // entries per lane per chunk
    constexpr int CW = 64 * EL;                 // columns per chunk
    constexpr int GSYM_G = gsym_g<MT>();
    __shared__ PT part[4][GSYM_G * CW];
    const int lane = tid & 63, wv = tid >> 6;
    const int64_t rw = r0 + RW * wv; // this wavefront's first row
    const int64_t blk = r0 / GSYM;
    double acc[RW], lam[RW];
    const MT *rows[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        acc[r] = 0.0;
        const bool in = rw + r < n;
        lam[r] = in ? x[n + rw + r] : 0.0;
        rows[r] = B + (in ? rw + r : n - 1) * ld;
    }
    const int64_t cend = n + r0 + GSYM;                            // columns [0, cend) are used
    const int64_t kch = n / CW;                                    // chunks entirely in K'
    const int64_t nch = std::min((cend + CW - 1) / CW, ld / CW);   // chunks read (ld: multiple of 256)
    // K' only: row sums
    for (int64_t c = 0; c < kch; ++c) {
        const int64_t c0 = c * CW + lane * EL;
#pragma unroll
        for (int r = 0; r < RW; ++r) {
            if constexpr (EL == 2) {
                const dvec2 bb = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(rows[r] + c0));
                acc[r] = fma(bb.x, x[c0], acc[r]);
                acc[r] = fma(bb.y, x[c0 + 1], acc[r]);
            } else {
                const fvec4 bb = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(rows[r] + c0));
                acc[r] = fma(double(bb.x), x[c0], acc[r]);
                acc[r] = fma(double(bb.y), x[c0 + 1], acc[r]);
                acc[r] = fma(double(bb.z), x[c0 + 2], acc[r]);
                acc[r] = fma(double(bb.w), x[c0 + 3], acc[r]);
            }
        }
    }
    // chunks that reach V': row sums of the entries j <= row, column partials of j < row
    for (int64_t g0 = kch; g0 < nch; g0 += GSYM_G) {
#pragma unroll
        for (int g = 0; g < GSYM_G; ++g) {
            const int64_t c = g0 + g;
            double t[EL];
#pragma unroll
            for (int e = 0; e < EL; ++e) t[e] = 0.0;
            // a chunk strictly inside [n, n + r0) has j < every row: no masks
            const bool clean = c * CW >= n && (c + 1) * CW <= n + r0;
            if (clean) {
                const int64_t c0 = c * CW + lane * EL;
                double xv[EL];
#pragma unroll
                for (int e = 0; e < EL; ++e) xv[e] = x[c0 + e];
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    double bv[EL];
                    if constexpr (EL == 2) {
                        const dvec2 bb = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(rows[r] + c0));
                        bv[0] = bb.x;
                        bv[1] = bb.y;
                    } else {
                        const fvec4 bb = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(rows[r] + c0));
                        bv[0] = bb.x;
                        bv[1] = bb.y;
                        bv[2] = bb.z;
                        bv[3] = bb.w;
                    }
#pragma unroll
                    for (int e = 0; e < EL; ++e) {
                        acc[r] = fma(bv[e], xv[e], acc[r]);
                        t[e] = fma(bv[e], lam[r], t[e]);
                    }
                }
            } else if (c < nch) {
                const int64_t c0 = c * CW + lane * EL;
                double xv[EL];
#pragma unroll
                for (int e = 0; e < EL; ++e) xv[e] = c0 + e < cend ? x[c0 + e] : 0.0;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
                    double bv[EL];
                    if constexpr (EL == 2) {
                        const dvec2 bb = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(rows[r] + c0));
                        bv[0] = bb.x;
                        bv[1] = bb.y;
                    } else {
                        const fvec4 bb = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(rows[r] + c0));
                        bv[0] = bb.x;
                        bv[1] = bb.y;
                        bv[2] = bb.z;
                        bv[3] = bb.w;
                    }
                    const int64_t row = rw + r;
#pragma unroll
                    for (int e = 0; e < EL; ++e) {
                        const int64_t col = c0 + e, j = col - n; // j < 0: a K' column
                        if (j <= row && col < cend) acc[r] = fma(bv[e], xv[e], acc[r]);
                        if (j >= 0 && j < row) t[e] = fma(bv[e], lam[r], t[e]);
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < EL; ++e) part[wv][g * CW + lane * EL + e] = PT(t[e]);
        }
        __syncthreads();
        for (int k = tid; k < GSYM_G * CW; k += 256) {
            const int64_t col = g0 * CW + k, j = col - n;
            if (j >= 0 && j < n && col < cend)
                P[blk * n + j] = PT((double(part[0][k]) + double(part[1][k])) + (double(part[2][k]) + double(part[3][k])));
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
    if (lane < RW && rw + lane < n) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < RW; ++r)
            if (lane == r) v = acc[r];
        y[oidx[rw + lane]] = v;
    }
}

// y_i += sum over blocks blk >= i / 16 of P[blk][i] + sum_j Delta_ij l_j.  A
// workgroup of 256 threads takes GFIN_ROWS rows i0..: thread (ty, tx) adds
// the blocks ty, ty + GFIN_NY, ... for row i0 + tx, and the GFIN_NY partial
// sums are then added in ty order (fixed, so the result is reproducible).
constexpr int GFIN_ROWS = 32, GFIN_NY = 256 / GFIN_ROWS;
template <typename PT>
__device__ inline void gemv_sym_finish(int64_t n, const PT *__restrict__ P, const int32_t *__restrict__ dptr,
                                       const int32_t *__restrict__ dcol, const double *__restrict__ dval,
                                       const double *__restrict__ x, double *__restrict__ y,
                                       const int32_t *__restrict__ oidx, int64_t i0, int tid)
{
    __shared__ double red[GFIN_NY][GFIN_ROWS];
    const int tx = tid % GFIN_ROWS, ty = tid / GFIN_ROWS;
    const int64_t i = i0 + tx;
    const int64_t nblk = (n + GSYM - 1) / GSYM;
    double s = 0.0;
    if (i < n) {
#pragma unroll 4
        for (int64_t b = i / GSYM + ty; b < nblk; b += GFIN_NY) s += double(P[b * n + i]);
    }
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && i < n) {
        double t = red[0][tx];
#pragma unroll
        for (int k = 1; k < GFIN_NY; ++k) t += red[k][tx];
        for (int32_t e = dptr[i]; e < dptr[i + 1]; ++e) t = fma(dval[e], x[n + dcol[e]], t);
        y[oidx[i]] += t;
    }
}

} // namespace pbfb
