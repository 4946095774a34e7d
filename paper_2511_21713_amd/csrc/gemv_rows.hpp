// Dense Galerkin GEMV rows: y[r] = sum_c B[r][c] x[c] for the rows owned by
// one wavefront.  B is a surface operator [K' | V'] stored row-major with a
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

#include <cstdint>

namespace pbfb {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

constexpr int GEMV_RW = 4; // rows per wavefront

template <typename MT>
__device__ inline void gemv_rows(const MT *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                 int64_t n, int64_t ld, int64_t r0, int lane)
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
        y[r0 + lane] = v;
    }
}

} // namespace pbfb
