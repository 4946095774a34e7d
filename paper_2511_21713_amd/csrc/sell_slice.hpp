// FEM rows of the coupled operator in sliced ELL: a slice is 64 consecutive
// rows (one wavefront wide); entry k of row 64 q + l is stored at
// sptr[q] + 64 k + l for k below the slice width w_q = (sptr[q+1] - sptr[q]) / 64,
// columns ascending, padding entries column = row and value 0.  Row lengths
// of the layered shell mesh are nearly uniform, so the padding is about 1 %
// of the entries and every value and column load of a wavefront is one
// contiguous 512- or 256-byte segment, with no row-pointer load in front of
// it.
//
// A workgroup of four wavefronts owns one slice: wavefront v takes the
// entries k = v, v + 4, v + 8, ... of its 64 rows, issuing SELL_U value and
// column loads and then SELL_U gathers of the input before it waits, so a
// slice of width 16 is read by one round of loads.  The four partial sums of
// a row are added in wavefront order through LDS (bitwise reproducible).
// FP32 values are widened; products and sums are FP64.
//
// This is the bandwidth-bound sparse kernel of every coupled apply and of
// every Chebyshev term of the FEM-block preconditioner.  Its loads are plain
// (cached): the Chebyshev terms read the same slices many times in a row.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pbfb {

constexpr int SELL_W = 4; // wavefronts per slice (one workgroup of 256 threads)
constexpr int SELL_U = 4; // entries per lane in flight

// Partial sum of row 64 q + lane over the entries k = wv, wv + 4, ... of
// slice q.  FEM_ONLY skips the coupling columns (index >= nn).
template <typename VT, bool FEM_ONLY>
__device__ inline double sell_part(const int32_t *__restrict__ sptr, const int32_t *__restrict__ col,
                                   const VT *__restrict__ val, const double *__restrict__ x, int64_t q, int lane,
                                   int wv, int64_t nn)
{
    const int32_t b0 = sptr[q], w = (sptr[q + 1] - b0) / 64;
    double acc = 0.0;
    for (int k0 = wv; k0 < w; k0 += SELL_W * SELL_U) {
        int32_t c[SELL_U];
        VT v[SELL_U];
#pragma unroll
        for (int j = 0; j < SELL_U; ++j) {
            // a clamped index keeps the load in bounds; its term is dropped below
            const int k = min(k0 + SELL_W * j, w - 1);
            const int64_t at = b0 + int64_t(k) * 64 + lane;
            c[j] = col[at];
            v[j] = val[at];
        }
        double xv[SELL_U];
#pragma unroll
        for (int j = 0; j < SELL_U; ++j) xv[j] = (FEM_ONLY && c[j] >= nn) ? 0.0 : x[c[j]];
#pragma unroll
        for (int j = 0; j < SELL_U; ++j)
            if (k0 + SELL_W * j < w) acc = fma(double(v[j]), xv[j], acc);
    }
    return acc;
}

// Sum of the four wavefront partials of each row of the slice, in order;
// valid in wavefront 0 (every thread of the workgroup must call it).
__device__ inline double sell_reduce(double part, int lane, int wv)
{
    __shared__ double red[SELL_W][64];
    red[wv][lane] = part;
    __syncthreads();
    double s = 0.0;
    if (wv == 0) {
        s = red[0][lane];
#pragma unroll
        for (int v = 1; v < SELL_W; ++v) s += red[v][lane];
    }
    return s;
}

} // namespace pbfb
