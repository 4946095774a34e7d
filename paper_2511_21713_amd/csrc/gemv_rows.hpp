// Dense Galerkin GEMV rows: y[oidx[r]] = sum_c B[r][c] x[c] for the rows owned
// by one workgroup (oidx: the output position of operator row r).  B is a
// surface operator [K' | V'] stored row-major with a padded row length ld (a
// multiple of 256 entries, zero past 2n); x is the packed FP64 input of the
// same length.  A workgroup is GEMV_WAVES wavefronts; each wavefront owns
// GEMV_RW consecutive rows and streams them in chunks of 64 lanes x 16 bytes
// with non-temporal loads (the operator is read once per apply and must not
// evict the vectors from L2); the input chunk is loaded once and reused for
// the GEMV_RW rows; the row sums are reduced across the 64 lanes with xor
// shuffles in a fixed order, so the result is bitwise reproducible.  FP32
// storage is widened and accumulated in FP64.  Pointers are taken in the
// global address space so that the loads are global (not flat) loads and the
// waits count vector memory only.
//
// This is the bandwidth-bound kernel of every coupled apply: it reads
// n * ld * sizeof(MT) bytes of operator per interface (about n * (n + n / 2)
// with the symmetric use below).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

namespace pbfb {

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <typename T> using gptr = const __attribute__((address_space(1))) T *;
template <typename MT> struct GemvLoad { using T = dvec2; };
template <> struct GemvLoad<float> { using T = fvec4; };

constexpr int GEMV_WAVES = 8;                    // wavefronts per workgroup
constexpr int GEMV_THREADS = 64 * GEMV_WAVES;    // threads per workgroup
constexpr int GEMV_RW = 8;                       // rows per wavefront
constexpr int GSYM = GEMV_WAVES * GEMV_RW;       // rows per workgroup (both forms)
// minimum wavefronts per SIMD of the dense-apply kernels (register budget):
// FP64 storage asks for four (at most 128 VGPRs, two 512-thread workgroups per
// CU), which the FP64 routines fit without spills; at 200 VGPRs (one
// workgroup per CU) the same FP64 apply ran at 0.61 of HBM instead of 0.80.
// The FP32 routines need more registers (one workgroup per CU either way).
template <typename MT> constexpr int gemv_occupancy() { return sizeof(MT) == 8 ? 4 : 2; }

// one chunk of GEMV_RW rows (EL entries per lane) and the matching input entries
template <typename MT> struct GemvChunk {
    static constexpr int EL = sizeof(MT) == 8 ? 2 : 4;
    static constexpr int CW = 64 * EL; // columns per chunk
    typename GemvLoad<MT>::T b[GEMV_RW];
    dvec2 x[EL / 2];
    __device__ inline void load(const gptr<typename GemvLoad<MT>::T> (&rows)[GEMV_RW], gptr<dvec2> xg, int64_t c,
                                int lane)
    {
        const uint32_t o = uint32_t(c) * 64u + uint32_t(lane);
#pragma unroll
        for (int h = 0; h < EL / 2; ++h) x[h] = xg[o * (EL / 2) + h];
#pragma unroll
        for (int r = 0; r < GEMV_RW; ++r) b[r] = __builtin_nontemporal_load(rows[r] + o);
    }
    __device__ inline double bv(int r, int e) const { return double(b[r][e]); }
    __device__ inline double xv(int e) const { return x[e / 2][e % 2]; }
};

template <typename MT>
__device__ inline void gemv_rows(const MT *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                 const int32_t *__restrict__ oidx, int64_t n, int64_t ld, int64_t r0, int lane)
{
    constexpr int RW = GEMV_RW;
    using C = GemvChunk<MT>;
    gptr<typename GemvLoad<MT>::T> rows[RW];
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        acc[r] = 0.0;
        rows[r] = (gptr<typename GemvLoad<MT>::T>)(B + (r0 + r < n ? r0 + r : n - 1) * ld);
    }
    const gptr<dvec2> xg = (gptr<dvec2>)(x);
    const int64_t nc = ld / C::CW;
    for (int64_t c = 0; c < nc; ++c) {
        C ch;
        ch.load(rows, xg, c, lane);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
#pragma unroll
            for (int e = 0; e < C::EL; ++e) acc[r] = fma(ch.bv(r, e), ch.xv(e), acc[r]);
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

__device__ inline void gemv_lds_barrier()
{
    // orders LDS only: loads of the operator stay in flight across it
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Symmetric single layer.  The regular part of V' is stored bitwise
// symmetric; the touching-pair blocks make V' differ from its transpose on
// a sparse pattern only, kept as Delta = upper(V') - lower(V')^T.  A row
// block of GSYM = 64 rows r0.. (r0 a multiple of 64) is two work items of
// one launch: its K item reads the chunks entirely inside K' (full rows of
// uniform length), its V item the remaining chunks up to the block's
// diagonal (the few K' columns of the chunk that straddles column n and the
// lower triangle of V'):
//   y_i = sum_{j < kch CW} K'_ij u_j                                 (K item)
//       + sum_{kch CW <= j' , j <= i} [K' | V']_ij' x_j'               (V item)
//       + sum_{j > i} V'_ji l_j + sum_{j > i} Delta_ij l_j      (gemv_sym_finish)
// For the third sum the V item forms the column sums
// P[blk][j] = sum_{r in its rows, r > j} V'_rj l_r over the V' columns it
// reads (the eight wavefronts' partials added in LDS in a fixed tree order,
// gsym_g chunks of the row stream at a time), blk = r0 / 64; its row sums go
// to P[nblk * n + row] and the finish adds them.  Rows past n contribute
// nothing.  Together the items read n + r0 + 64 entries of each row instead
// of 2 n; the partials are 1/64 of the V' bytes read (written once, read
// once).  Splitting the row block lets the launch order the items for the
// memory system (gemv_item): the uniform K items and the triangle's V items
// of decreasing length overlap instead of every workgroup streaming both.
// chunks per LDS exchange: FP32 storage 8 (128 KB of partials; its kernel runs
// one workgroup per CU either way; 0.769 -> 0.772 of HBM against 4, 2 slower),
// FP64 storage 4 (32 KB, two workgroups per CU)
template <typename MT> constexpr int gsym_g() { return sizeof(MT) == 4 ? 8 : 4; }
// The partials are FP64 for both storage precisions: with FP32 partials the
// apply is linear only to FP32 rounding of the partial sums, which left
// strongly charged instances short of the Newton tolerance in mixed mode.
template <typename MT> using sym_part_t = double;

// K item: row sums over the chunks entirely inside K', written to y
template <typename MT>
__device__ inline void gemv_rows_symK(const MT *__restrict__ B, const double *__restrict__ x, double *__restrict__ y,
                                      const int32_t *__restrict__ oidx, int64_t n, int64_t ld, int64_t r0, int tid)
{
    constexpr int RW = GEMV_RW;
    using C = GemvChunk<MT>;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t rw = r0 + RW * wv; // this wavefront's first row
    gptr<typename GemvLoad<MT>::T> rows[RW];
    double acc[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        acc[r] = 0.0;
        rows[r] = (gptr<typename GemvLoad<MT>::T>)(B + (rw + r < n ? rw + r : n - 1) * ld);
    }
    const gptr<dvec2> xg = (gptr<dvec2>)(x);
    const int64_t kch = n / C::CW; // chunks entirely in K'
    for (int64_t c = 0; c < kch; ++c) {
        C ch;
        ch.load(rows, xg, c, lane);
#pragma unroll
        for (int r = 0; r < RW; ++r) {
#pragma unroll
            for (int e = 0; e < C::EL; ++e) acc[r] = fma(ch.bv(r, e), ch.xv(e), acc[r]);
        }
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

// V item: row sums of the entries j <= row from chunk kch on, column
// partials of j < row; P holds nblk * n partials, then the n row sums
template <typename MT>
__device__ inline void gemv_rows_symV(const MT *__restrict__ B, const double *__restrict__ x,
                                      double *__restrict__ P, int64_t n, int64_t ld, int64_t r0, int tid)
{
    constexpr int RW = GEMV_RW, WV = GEMV_WAVES, G = gsym_g<MT>();
    static_assert(WV == 8, "the partials are added in an eight-term tree");
    using C = GemvChunk<MT>;
    constexpr int EL = C::EL, CW = C::CW;
    __shared__ double part[WV][G * CW];
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t rw = r0 + RW * wv; // this wavefront's first row
    const int64_t blk = r0 / GSYM, nblk = (n + GSYM - 1) / GSYM;
    gptr<typename GemvLoad<MT>::T> rows[RW];
    double acc[RW], lam[RW];
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        acc[r] = 0.0;
        const bool in = rw + r < n;
        lam[r] = in ? ((gptr<double>)(x))[n + rw + r] : 0.0;
        rows[r] = (gptr<typename GemvLoad<MT>::T>)(B + (in ? rw + r : n - 1) * ld);
    }
    const gptr<dvec2> xg = (gptr<dvec2>)(x);
    const int64_t cend = n + r0 + GSYM;                          // columns [0, cend) are used
    const int64_t kch = n / CW;                                  // chunks of the K item
    const int64_t nch = std::min((cend + CW - 1) / CW, ld / CW); // chunks read (ld: multiple of 256)
    for (int64_t g0 = kch; g0 < nch; g0 += G) {
        // every column of the group is a V' column left of every row of the workgroup
        const bool clean = g0 * CW >= n && (g0 + G) * CW <= n + r0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t c = g0 + g;
            double t[EL];
#pragma unroll
            for (int e = 0; e < EL; ++e) t[e] = 0.0;
            if (clean) {
                C ch;
                ch.load(rows, xg, c, lane);
#pragma unroll
                for (int r = 0; r < RW; ++r) {
#pragma unroll
                    for (int e = 0; e < EL; ++e) {
                        acc[r] = fma(ch.bv(r, e), ch.xv(e), acc[r]);
                        t[e] = fma(ch.bv(r, e), lam[r], t[e]);
                    }
                }
            } else if (c < nch) {
                C ch;
                ch.load(rows, xg, c, lane);
                // column - n - (this wavefront's first row); |.| < 2^31
                const int jb = int(c * CW - n - rw) + lane * EL;
#pragma unroll
                for (int r = 0; r < RW; ++r) {
#pragma unroll
                    for (int e = 0; e < EL; ++e) {
                        const int d = jb + e - r;                        // j - row (j < 0: a K' column)
                        if (d <= 0) acc[r] = fma(ch.bv(r, e), ch.xv(e), acc[r]);
                        if (d < 0 && jb + e + int(rw) >= 0) t[e] = fma(ch.bv(r, e), lam[r], t[e]);
                    }
                }
            }
#pragma unroll
            for (int e = 0; e < EL; ++e) part[wv][g * CW + lane * EL + e] = t[e];
        }
        gemv_lds_barrier();
        for (int k = tid; k < G * CW; k += GEMV_THREADS) {
            const int64_t col = g0 * CW + k, j = col - n;
            if (j >= 0 && j < n && col < cend) {
                const double v = ((part[0][k] + part[1][k]) + (part[2][k] + part[3][k])) +
                                 ((part[4][k] + part[5][k]) + (part[6][k] + part[7][k]));
                // FP32 storage: cached stores (merged in L2 before they reach
                // HBM: 0.762 -> 0.767 of HBM); FP64 storage: non-temporal
                // (cached stores cost it 0.797 -> 0.781)
                if constexpr (sizeof(MT) == 4) P[blk * n + j] = v;
                else __builtin_nontemporal_store(v, P + blk * n + j);
            }
        }
        gemv_lds_barrier();
    }
#pragma unroll
    for (int r = 0; r < RW; ++r)
        for (int off = 32; off > 0; off >>= 1) acc[r] += __shfl_xor(acc[r], off);
    if (lane < RW && rw + lane < n) {
        double v = acc[0];
#pragma unroll
        for (int r = 1; r < RW; ++r)
            if (lane == r) v = acc[r];
        P[nblk * n + rw + lane] = v;
    }
}

// Order of the work items of a launch over two surfaces: surface s has
// nk_s K items (its row blocks; full-row items when it is not used
// symmetrically) and nv_s V items (nb or 0).  The h0 / h1 heaviest V items
// (last row blocks first) come first, then every K item, then the remaining
// V items, heaviest first; inside each stretch the two surfaces alternate.
// Measured on the 80k-triangle operators: FP64 storage is fastest with a
// quarter of the V items first (h = nb / 4), FP32 storage with every K item
// first (h = 0).
struct GemvItem {
    int s;     // surface
    bool k;    // K item (else V item)
    int64_t b; // row block
};
__device__ inline void gemv_alternate(int64_t k, int64_t c0, int64_t c1, int &s, int64_t &i)
{
    const int64_t m = c0 < c1 ? c0 : c1;
    if (k < 2 * m) {
        s = int(k & 1);
        i = k >> 1;
    } else {
        s = c0 > c1 ? 0 : 1;
        i = m + (k - 2 * m);
    }
}
__device__ inline GemvItem gemv_item(int64_t bi, int64_t nk0, int64_t nk1, int64_t nv0, int64_t nv1, int64_t h0,
                                     int64_t h1)
{
    GemvItem it;
    int64_t i;
    if (bi < h0 + h1) {
        gemv_alternate(bi, h0, h1, it.s, i);
        it.k = false;
        it.b = (it.s ? nv1 : nv0) - 1 - i;
        return it;
    }
    bi -= h0 + h1;
    if (bi < nk0 + nk1) {
        gemv_alternate(bi, nk0, nk1, it.s, i);
        it.k = true;
        it.b = i;
        return it;
    }
    bi -= nk0 + nk1;
    gemv_alternate(bi, nv0 - h0, nv1 - h1, it.s, i);
    it.k = false;
    it.b = (it.s ? nv1 - h1 : nv0 - h0) - 1 - i;
    return it;
}
// V items dispatched before the K items (see gemv_item), of nv
inline int64_t gemv_heavy(bool f32, int64_t nv) { return f32 ? 0 : (nv + 3) / 4; }

// y_i += (V item's row sum) + sum over blocks blk >= i / 64 of P[blk][i] +
// sum_j Delta_ij l_j.  A workgroup of 256 threads takes GFIN_ROWS rows
// i0..: thread (ty, tx) adds the blocks ty, ty + GFIN_NY, ... for row
// i0 + tx, and the GFIN_NY partial sums are then added in ty order (fixed,
// so the result is reproducible).
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
        double t = double(P[nblk * n + i]);
#pragma unroll
        for (int k = 0; k < GFIN_NY; ++k) t += red[k][tx];
        for (int32_t e = dptr[i]; e < dptr[i + 1]; ++e) t = fma(dval[e], x[n + dcol[e]], t);
        y[oidx[i]] += t;
    }
}

} // namespace pbfb
