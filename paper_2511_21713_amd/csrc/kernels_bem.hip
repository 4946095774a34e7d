// Dense Galerkin P1 boundary operators on one surface:
//   V_ij = int int zeta_i(x) g(x,y) zeta_j(y),   K_ij = int int zeta_i(x) dg/dn_y zeta_j(y),
//   g = exp(-kappa r) / (4 pi r)   (Sec. 2.2 Yukawa kernel; kappa = 0: Sec. 2.3 Laplace kernel)
// stored as one row-major matrix per surface, row i = [K'_i | V'_i] with
//   Gamma_m: K' = 1/2 M + K0,  V' = -V0   (interior Laplace equation)
//   Gamma_s: K' = 1/2 M - Kk,  V' = +Vk   (exterior Yukawa equation)
// so the Galerkin rows of the coupled operator are one dense GEMV each.
//
// Rows and columns follow the Morton vertex order (first appearance along
// the Morton-ordered triangles; SurfaceTopo::mvert), so the vertices of a
// block of consecutive triangles are nearby rows and columns.
//
// Assembly, deterministic and free of atomics, straight into that storage:
//  1. regular tiles: a workgroup takes TA target x TB source Morton-ordered
//     triangles (shape chosen by an autotuner), evaluates the 6 x 6 product
//     rule for every non-touching pair, reduces the 3x3 pair blocks to the
//     blocks' vertices in LDS and adds the result into the stored operator.
//     The triangle blocks are coloured so that blocks of one colour share no
//     vertex; one launch per colour pair then has tiles that touch disjoint
//     entries, and the launches run one after the other, so every entry
//     receives its contributions in a fixed order.  Square shapes evaluate
//     each unordered pair once and also add the double layer of the
//     mirrored pair to an nv x nv matrix T (the only workspace);
//  2. square shapes: a transpose pass completes V' = U + U^T and K' += T^T
//     (the regular part of V' bitwise symmetric);
//  3. touching pairs (identical, common edge, common vertex) are integrated
//     with the Sauter-Schwab rules (one wavefront per pair) and added, with
//     the 1/2 M term, by a row-owned scatter.
//
// In mixed precision the regular tiles evaluate the kernels in FP32: each
// quadrature point is held as an FP32 offset from its triangle's centroid,
// the centroid difference of a pair is formed in FP64 and rounded once, so
// x - y never cancels large coordinates in FP32.  A pair's 3x3 V and K
// blocks are summed over its 36 quadrature pairs in FP32, and so are the
// fold's corner sums onto a tile's vertices (at most MS terms each); each
// tile's sum is added to the FP32 stored entry in FP64 and rounded once (an
// entry receives one tile's sum for each pair of blocks holding its two
// vertices).  The touching pairs stay FP64 throughout.
#include <chrono>
#include <cmath>
#include <thread>
#include <type_traits>

#include "bem_quad.hpp"
#include "pbfb_internal.hpp"

namespace pbfb {

struct GL4 {
    double x[4];
    double w[4];
};

static GL4 gl4arg()
{
    GL4 r;
    for (int i = 0; i < 4; ++i) {
        r.x[i] = rules().gl_x[i];
        r.w[i] = rules().gl_w[i];
    }
    return r;
}

static inline unsigned nblk(int64_t n, int bs) { return unsigned((n + bs - 1) / bs); }



// Morton-ordered copies of the triangle data used by the regular assembly.
// FP64 evaluation reads m_qp/m_nrm; FP32 evaluation reads m_cen/m_qf/m_nf
// (whichever pointers are non-null are written).
__global__ void k_tri_morton(int64_t nt, const int32_t *__restrict__ morton, const int32_t *__restrict__ tri,
                             const double *__restrict__ qp, const double *__restrict__ nrm,
                             const double *__restrict__ area, const int32_t *__restrict__ g,
                             const double *__restrict__ x, int32_t *__restrict__ m_tri, double *__restrict__ m_qp,
                             double *__restrict__ m_nrm, double *__restrict__ m_area, double *__restrict__ m_cen,
                             float *__restrict__ m_qf, float *__restrict__ m_nf)
{
    int64_t m = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (m >= nt) return;
    int32_t t = morton[m];
    for (int k = 0; k < 3; ++k) m_tri[3 * m + k] = tri[3 * t + k];
    m_area[m] = area[t];
    if (m_qp) {
        for (int k = 0; k < 3; ++k) m_nrm[3 * m + k] = nrm[3 * t + k];
        for (int k = 0; k < 18; ++k) m_qp[18 * m + k] = qp[18 * t + k];
    }
    if (m_cen) {
        double c[3];
        for (int d = 0; d < 3; ++d)
            c[d] = (x[3 * g[tri[3 * t]] + d] + x[3 * g[tri[3 * t + 1]] + d] + x[3 * g[tri[3 * t + 2]] + d]) / 3.0;
        for (int d = 0; d < 3; ++d) {
            m_cen[3 * m + d] = c[d];
            m_nf[3 * m + d] = float(nrm[3 * t + d]);
        }
        for (int q = 0; q < 6; ++q)
            for (int d = 0; d < 3; ++d) m_qf[18 * m + 3 * q + d] = float(qp[18 * t + 3 * q + d] - c[d]);
    }
}

// ---------------------------------------------------------------------------
// 1. regular tiles
// ---------------------------------------------------------------------------


// Read-modify-write of one folded operator entry into the stored operator
// (FP64 or FP32 storage; the sum is formed in FP64 and rounded once).  No
// other thread of the launch touches the same entry (the launch's tiles have
// vertex-disjoint target blocks and vertex-disjoint source blocks).
template <typename MT> __device__ inline void add_entry(MT *__restrict__ U, int64_t at, double v)
{
    U[at] = MT(double(U[at]) + v);
}

// Rows of the fold's last stage whose operator entries a thread reads ahead
// (the rest are read when they are added to): FP32 tiles one, before the
// quadrature (342 -> 325 ms per 80k-triangle assembly; two cost registers and
// gained nothing more); FP64 tiles one, after the quadrature, whose registers
// are free by then, so that the reads overlap the fold's LDS passes (before
// it they spill; 572 -> 565 ms).  The two reads are written out in place:
// the FP32 kernels' register allocation (six wavefronts per SIMD) did not
// survive moving them into a shared function.
constexpr int FOLD_PF32 = 1, FOLD_PF64 = 1;
template <typename MT> constexpr int fold_pf() { return sizeof(MT) == 4 ? FOLD_PF32 : FOLD_PF64; }

// A thread's part of the fold of a tile, the same for every operator
// folded: source vertex jb, first row r0 and row step of its strided rows, and
// the tile columns of jb's corners (absent corners: the zero column CMAX)
template <int MS> struct FoldMap {
    int jb, r0, rstep;
    int cb[MS];
};
template <int NT, int MS>
__device__ inline FoldMap<MS> fold_map(int tid, int nB, const int (*sSb)[MS], int cmax)
{
    FoldMap<MS> fm;
    fm.jb = tid % nB;
    fm.r0 = tid / nB;
    fm.rstep = NT / nB;
#pragma unroll
    for (int l = 0; l < MS; ++l) {
        const int c = sSb[fm.jb][l];
        fm.cb[l] = c < 0 ? cmax : c;
    }
    return fm;
}

// Fold of a tile's pair blocks onto the blocks' vertices through the shared
// tile, one operator at a time (FP64 evaluation: V, K and the mirrored K in
// turn through one FP64 plane, which keeps the LDS of a workgroup small
// enough for four per CU): first
// the source corners of each source vertex (in place, row by row), then the
// target corners of each target vertex, added into U at row vA[ia], column
// off + vB[jb] with factor sc.  A thread owns one source vertex jb and a
// strided set of rows; the corner lists are read once into registers and
// every tile read is independent (an absent corner reads the zero row /
// column), so the reads pipeline.  MS >= the largest number of corners of
// any vertex of either block: the lists past it hold only absent corners,
// whose +0 terms are skipped.
template <int TA, int TB, int MS, int SLOT, typename MT, typename ST, typename XT>
__device__ inline void fold_tile_one(int tid, int tl, int sl, int nA, const FoldMap<MS> &fm, const int (*sSa)[MS],
                                     ST (*acc)[TB * 3 + 1], const XT *Xl, const int *vA,
                                     const int *vB, MT *__restrict__ U, int64_t ld, int64_t off, double sc,
                                     const MT (*pre)[3])
{
    constexpr int NT = TA * TB;
    const int jb = fm.jb, r0 = fm.r0, rstep = fm.rstep;
    const bool colthread = r0 < rstep; // NT - rstep * nB threads stay idle
    const int (&cb)[MS] = fm.cb;
    for (int k = tid; k < TB * 3 + 1; k += NT) acc[TA * 3][k] = 0.0;
    if (tid < TA * 3) acc[tid][TB * 3] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) acc[3 * tl + a][3 * sl + b] = ST(Xl[3 * a + b]);
    __syncthreads();
    constexpr int RMAX = TA * 3;
    constexpr int RPT = (RMAX + NT / (TB * 3) - 1) / (NT / (TB * 3)); // rows per thread, nB <= TB * 3
    double colsum[RPT];
    int nrow = 0;
    if (colthread) {
#pragma unroll
        for (int r = 0; r < RPT; ++r) {
            const int sa = r0 + r * rstep;
            double t = 0.0;
            if (sa < RMAX) {
                double v[MS];
#pragma unroll
                for (int l = 0; l < MS; ++l) v[l] = double(acc[sa][cb[l]]);
#pragma unroll
                for (int l = 0; l < MS; ++l) t += v[l];
                nrow = r + 1;
            }
            colsum[r] = t;
        }
    }
    __syncthreads();
    if (colthread)
#pragma unroll
        for (int r = 0; r < RPT; ++r)
            if (r < nrow) acc[r0 + r * rstep][jb] = ST(colsum[r]);
    __syncthreads();
    if (colthread) {
        const int64_t col = off + vB[jb];
        auto rowsum = [&](int ia) {
            double v[MS];
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const int ra = sSa[ia][k];
                v[k] = double(acc[ra < 0 ? TA * 3 : ra][jb]);
            }
            double t = 0.0;
#pragma unroll
            for (int k = 0; k < MS; ++k) t += v[k];
            return t;
        };
        // the first fold_pf rows add to the entries read before the quadrature
#pragma unroll
        for (int k = 0; k < fold_pf<MT>(); ++k) {
            const int ia = r0 + k * rstep;
            if (ia < nA) U[int64_t(vA[ia]) * ld + col] = MT(double(pre[k][SLOT]) + sc * rowsum(ia));
        }
        for (int ia = r0 + fold_pf<MT>() * rstep; ia < nA; ia += rstep) add_entry(U, int64_t(vA[ia]) * ld + col, sc * rowsum(ia));
    }
    __syncthreads();
}

// Fold of an FP32 tile's pair blocks (corner sums in FP32, the evaluation
// precision), V and K in two FP32 planes of the shared tile read at the same
// index (TOT = false: V to column off + vB[jb]
// with factor s0, K to column vB[jb] with factor s1 of row vA[ia] of U), or
// the mirrored K of a square tile in one plane (TOT = true: to column vB[jb]
// of row vA[ia] of U = T with factor s0); otherwise as fold_tile_one.
template <int TA, int TB, int MS, bool TOT, typename MT>
__device__ inline void fold_tile_f32(int tid, int tl, int sl, int nA, const FoldMap<MS> &fm, const int (*sSa)[MS],
                                     float (*acc)[TA * 3 + 1][TB * 3 + 1],
                                     const float (*blk)[9], const int *vA, const int *vB, MT *__restrict__ U,
                                     int64_t ld, int64_t off, double s0, double s1, const MT (*pre)[3])
{
    constexpr int NT = TA * TB, RMAX = TA * 3, CMAX = TB * 3, RC = 4, NPL = TOT ? 1 : 2;
    const int jb = fm.jb, r0 = fm.r0, rstep = fm.rstep;
    const bool colthread = r0 < rstep; // NT - rstep * nB threads stay idle
    const int (&cb)[MS] = fm.cb;
    for (int k = tid; k < CMAX + 1; k += NT)
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) acc[pl][RMAX][k] = 0.0f;
    if (tid < RMAX)
#pragma unroll
        for (int pl = 0; pl < NPL; ++pl) acc[pl][tid][CMAX] = 0.0f;
#pragma unroll
    for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) acc[pl][3 * tl + a][3 * sl + b] = blk[pl][3 * a + b];
    __syncthreads();
    const int rows_pt = (RMAX + rstep - 1) / rstep; // uniform
    for (int rb = 0; rb < rows_pt; rb += RC) {
        float colsum[RC][NPL];
        int nrow = 0;
        if (colthread) {
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                const int sa = r0 + (rb + r) * rstep;
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl) colsum[r][pl] = 0.0f;
                if (sa < RMAX) {
#pragma unroll
                    for (int l = 0; l < MS; ++l)
#pragma unroll
                        for (int pl = 0; pl < NPL; ++pl) colsum[r][pl] += acc[pl][sa][cb[l]];
                    nrow = r + 1;
                }
            }
        }
        __syncthreads();
        if (colthread)
#pragma unroll
            for (int r = 0; r < RC; ++r)
                if (r < nrow)
#pragma unroll
                    for (int pl = 0; pl < NPL; ++pl) acc[pl][r0 + (rb + r) * rstep][jb] = colsum[r][pl];
        __syncthreads();
    }
    if (colthread) {
        const int64_t col = vB[jb];
        auto rowsum = [&](int ia, double (&t)[NPL]) {
            float f[NPL];
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) f[pl] = 0.0f;
#pragma unroll
            for (int k = 0; k < MS; ++k) {
                const int ra = sSa[ia][k] < 0 ? RMAX : sSa[ia][k];
#pragma unroll
                for (int pl = 0; pl < NPL; ++pl) f[pl] += acc[pl][ra][jb];
            }
#pragma unroll
            for (int pl = 0; pl < NPL; ++pl) t[pl] = double(f[pl]);
        };
        // the first fold_pf rows add to the entries read before the quadrature
#pragma unroll
        for (int k = 0; k < fold_pf<MT>(); ++k) {
            const int ia = r0 + k * rstep;
            if (ia < nA) {
                double t[NPL];
                rowsum(ia, t);
                const int64_t row = int64_t(vA[ia]) * ld;
                if constexpr (TOT) {
                    U[row + col] = MT(double(pre[k][2]) + s0 * t[0]);
                } else {
                    U[row + off + col] = MT(double(pre[k][0]) + s0 * t[0]);
                    U[row + col] = MT(double(pre[k][1]) + s1 * t[1]);
                }
            }
        }
        for (int ia = r0 + fold_pf<MT>() * rstep; ia < nA; ia += rstep) {
            double t[NPL];
            rowsum(ia, t);
            const int64_t row = int64_t(vA[ia]) * ld;
            if constexpr (TOT) {
                add_entry(U, row + col, s0 * t[0]);
            } else {
                add_entry(U, row + off + col, s0 * t[0]);
                add_entry(U, row + col, s1 * t[1]);
            }
        }
    }
}

// occupancy asked of the compiler: FP32 tiles fit in 80 VGPRs (six
// wavefronts per SIMD by registers and LDS), FP64 tiles in 128 (four)
constexpr int TILE_F32_WAVES = 5;
constexpr int TILE_F64_WAVES = 4;

// RT = double: positions and normals in FP64 (xq, nq: m_qp, m_nrm; cen unused)
// RT = float : FP32 offsets from FP64 centroids (xq, nq: m_qf, m_nf; cen: m_cen)
// MT: storage of the operator (double, or float in mixed precision)
// TA x TB: target x source triangles of the tile, one pair per thread; MS:
// bound on the corners of one vertex in one block (6, 12 or MAXS).  The
// tile of workgroup (x, y) is target block listA[y] x source block listB[x]
// (skip_lower: tiles whose source block precedes the target block return).
// The tile's V and K blocks are folded onto its vertices and added into the
// stored operator U (rows: [K' | V'] in the Morton vertex order, sK K and sV
// V) -- the launch's tiles touch disjoint entries, see BlockSide.
// SYM (square tiles): each unordered pair is evaluated once (the launches
// cover each unordered block pair once, in either orientation, and a
// diagonal tile only its pairs with the source after the target).  Besides
// V and K of (tau, sigma) a pair also yields K of (sigma, tau): the kernel
// values are shared, only the normal distance changes ((y_q - x).n_tau, the
// same for the six target points, which lie in the plane of tau).  It is
// added, transposed, to T (nv x nv: T[i][j] collects sK K(j, i)); V of
// (sigma, tau) is the transpose of V of (tau, sigma).  k_bem_symm then
// completes the operator: V' = U_V + U_V^T, K' = U_K + T^T.
//
// Every lane runs the quadrature: a pair that is not evaluated (padding
// triangle, shared vertex, or the mirror of a diagonal-tile pair) has its
// target moved 1e4 away and a zero factor, so its terms are exact zeros.
template <bool YUK, typename RT, typename MT, int TA, int TB, int MS, bool SYM>
__global__ void __launch_bounds__(TA * TB) __attribute__((amdgpu_waves_per_eu(sizeof(RT) == 4 ? TILE_F32_WAVES : TILE_F64_WAVES)))
    k_bem_regular(int64_t nt, const int32_t *__restrict__ m_tri, const RT *__restrict__ xq,
                  const RT *__restrict__ nq, const double *__restrict__ cen, const double *__restrict__ m_area,
                  const int32_t *__restrict__ A_pref, const int32_t *__restrict__ A_nv,
                  const int32_t *__restrict__ A_slots, const int32_t *__restrict__ A_vid,
                  const int32_t *__restrict__ B_pref, const int32_t *__restrict__ B_nv,
                  const int32_t *__restrict__ B_slots, const int32_t *__restrict__ B_vid,
                  const int32_t *__restrict__ listA, const int32_t *__restrict__ listB, int skip_lower,
                  MT *__restrict__ U, MT *__restrict__ T, int64_t ld, int64_t nv, double sV, double sK,
                  double kappa, QRule6 R, QRule6F RF)
{
    static_assert(!SYM || TA == TB, "symmetric evaluation needs square tiles");
    constexpr bool F32 = sizeof(RT) == 4;
    constexpr int NT = TA * TB;
    const int64_t bA = listA[blockIdx.y], bB = listB[blockIdx.x];
    if (SYM && skip_lower && bB < bA) return; // evaluated as (bB, bA)
    __shared__ RT sX[TA * 18]; // quadrature points, 18 values per triangle
    __shared__ RT sY[TB * 18];
    __shared__ RT sN[TB][3];
    __shared__ RT sNa[SYM ? TA : 1][3];
    __shared__ double sCa[F32 ? TA : 1][3], sCb[F32 ? TB : 1][3];
    __shared__ double sAa[TA], sAb[TB];
    __shared__ int sVa[TA][3], sVb[TB][3];
    __shared__ int sSa[TA * 3][MS], sSb[TB * 3][MS];
    __shared__ int sIa[TA * 3], sIb[TB * 3]; // operator index of each block vertex
    // the tile of pair blocks in the evaluation precision, + a zero row and a
    // zero column: FP32 one plane each for V and K, then the mirrored K of a
    // square tile in the first; FP64 one plane, one operator at a time
    constexpr int NPL = F32 ? 2 : 1;
    __shared__ std::conditional_t<F32, float, double> acc[NPL][TA * 3 + 1][TB * 3 + 1];

    const int tid = threadIdx.x;
    const int nA = A_nv[bA], nB = B_nv[bB];
    const int64_t pA = A_pref[bA], pB = B_pref[bB];

    {
        // a block's quadrature points are contiguous
        const int64_t xa = 18 * bA * TA, xb = 18 * bB * TB, xe = 18 * nt;
        for (int k = tid; k < TA * 18; k += NT) sX[k] = xa + k < xe ? xq[xa + k] : RT(0);
        for (int k = tid; k < TB * 18; k += NT) sY[k] = xb + k < xe ? xq[xb + k] : RT(0);
    }
    if (tid < TB * 3) {
        int sl = tid / 3, c = tid % 3;
        int64_t m = bB * TB + sl;
        sN[sl][c] = m < nt ? nq[3 * m + c] : RT(0);
        sVb[sl][c] = m < nt ? m_tri[3 * m + c] : -1;
        if constexpr (F32) sCb[sl][c] = m < nt ? cen[3 * m + c] : 0.0;
        sIb[tid] = tid < nB ? B_vid[pB + tid] : 0;
    }
    if (tid < TA * 3) {
        int tl = tid / 3, c = tid % 3;
        int64_t m = bA * TA + tl;
        sVa[tl][c] = m < nt ? m_tri[3 * m + c] : -2;
        if constexpr (F32) sCa[tl][c] = m < nt ? cen[3 * m + c] : 0.0;
        if constexpr (SYM) sNa[tl][c] = m < nt ? nq[3 * m + c] : RT(0);
        sIa[tid] = tid < nA ? A_vid[pA + tid] : 0;
    }
    if (tid < TA) sAa[tid] = (bA * TA + tid) < nt ? m_area[bA * TA + tid] : 0.0;
    if (tid < TB) sAb[tid] = (bB * TB + tid) < nt ? m_area[bB * TB + tid] : 0.0;
    for (int k = tid; k < TA * 3 * MS; k += NT) {
        int r = k / MS, c = k % MS;
        sSa[r][c] = r < nA ? A_slots[(pA + r) * MAXS + c] : -1;
    }
    for (int k = tid; k < TB * 3 * MS; k += NT) {
        int r = k / MS, c = k % MS;
        sSb[r][c] = r < nB ? B_slots[(pB + r) * MAXS + c] : -1;
    }
    __syncthreads();

    // this thread's pair (target tl, source sl)
    const int tl = tid / TB, sl = tid % TB;
    bool live = sVa[tl][0] >= 0 && sVb[sl][0] >= 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) live = live && sVa[tl][a] != sVb[sl][b];
    if (SYM && bA == bB && sl <= tl) live = false; // the mirror pair carries it
    RT c0 = RT(0), c1 = RT(0), c2 = RT(0); // FP32: target frame relative to the source centroid
    if constexpr (F32) {
        c0 = float(sCa[tl][0] - sCb[sl][0]);
        c1 = float(sCa[tl][1] - sCb[sl][1]);
        c2 = float(sCa[tl][2] - sCb[sl][2]);
    }
    if (!live) c0 += RT(1.0e4);
    const RT sc = live ? RT(sAa[tl] * sAb[sl] * INV4PI) : RT(0);
    const RT *xt = sX + 18 * tl, *ys = sY + 18 * sl;
    const RT n0 = sN[sl][0], n1 = sN[sl][1], n2 = sN[sl][2];
    RT y0n = RT(0); // FP32: y_0.n (offsets from the source centroid are small)
    if constexpr (F32) y0n = ys[0] * n0 + ys[1] * n1 + ys[2] * n2;
    RT dm[SYM ? 6 : 1]; // (y_q - x).n_tau, the same for every target point x
    if constexpr (SYM) {
        const RT m0 = sNa[tl][0], m1 = sNa[tl][1], m2 = sNa[tl][2];
        const RT xa0 = xt[0] + c0, xa1 = xt[1] + c1, xa2 = xt[2] + c2;
#pragma unroll
        for (int q = 0; q < 6; ++q)
            dm[q] = (ys[3 * q] - xa0) * m0 + (ys[3 * q + 1] - xa1) * m1 + (ys[3 * q + 2] - xa2) * m2;
    }
    RT oA0, oA1, oD0, oD1;
    if constexpr (F32) {
        oA0 = RF.oA[0], oA1 = RF.oA[1], oD0 = RF.oD[0], oD1 = RF.oD[1];
    } else {
        oA0 = R.oA[0], oA1 = R.oA[1], oD0 = R.oD[0], oD1 = R.oD[1];
    }
    const RT kap = RT(kappa);
    const RT kl2 = RT(-1.44269504088896341 * kappa); // FP32: e^{-kappa r} = 2^{kl2 r}

    // Target point p: the kernels at its 6 source points and their sums with
    // the source rule's orbits.  The source points lie in the plane of the
    // source triangle, so the normal distance (x - y_q).n is the same for all
    // six: it is taken once per target point and factored out of the
    // double-layer sums.  s: single layer, t: double layer / (x - y).n, u:
    // mirrored double layer (SYM).
    auto point = [&](int p, RT (&s)[3], RT (&t)[3], RT (&u)[3], RT &dn) {
        const RT x0 = xt[3 * p] + c0;
        RT x1 = xt[3 * p + 1], x2 = xt[3 * p + 2];
        if constexpr (F32) {
            x1 += c1;
            x2 += c2;
            dn = x0 * n0 + x1 * n1 + x2 * n2 - y0n;
        } else {
            dn = (x0 - ys[0]) * n0 + (x1 - ys[1]) * n1 + (x2 - ys[2]) * n2;
        }
        RT gv[6], hk[6]; // single-layer kernel, double-layer kernel / (x - y).n
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const RT d0 = x0 - ys[3 * q], d1 = x1 - ys[3 * q + 1], d2 = x2 - ys[3 * q + 2];
            const RT r2 = d0 * d0 + d1 * d1 + d2 * d2;
            const RT ri = rsqrt_pos(r2);
            if constexpr (YUK) {
                const RT r = r2 * ri;
                RT e;
                if constexpr (F32) e = __builtin_amdgcn_exp2f(kl2 * r);
                else e = exp_neg(kap * r);
                gv[q] = e * ri;
                hk[q] = gv[q] * ri * (ri + kap); // e (1 + kappa r) / r^3
            } else {
                gv[q] = ri;
                hk[q] = ri * ri * ri;
            }
        }
        auto orb = [&](const RT (&g)[6], RT (&o)[3]) {
            const RT c = oA0 * (g[0] + g[1] + g[2]) + oA1 * (g[3] + g[4] + g[5]);
            o[0] = c + oD0 * g[0] + oD1 * g[3];
            o[1] = c + oD0 * g[1] + oD1 * g[4];
            o[2] = c + oD0 * g[2] + oD1 * g[5];
        };
        orb(gv, s);
        orb(hk, t);
        if constexpr (SYM) {
            RT hm[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) hm[q] = hk[q] * dm[q];
            orb(hm, u);
        }
    };

    // FP32: the stored entries this thread adds to in the fold's last stage
    // (row vA[ia], column vB[jb] of V', K' and, square tiles, T; the fold's
    // thread map), read now so that their latency hides behind the
    // quadrature.  No other workgroup of the launch touches them.
    MT pre[fold_pf<MT>() > 0 ? fold_pf<MT>() : 1][3];
    if constexpr (F32) {
        const int jb = tid % nB, r0 = tid / nB, rstep = NT / nB;
        if (r0 < rstep) {
            const int64_t col = sIb[jb];
#pragma unroll
            for (int k = 0; k < fold_pf<MT>(); ++k) {
                const int ia = r0 + k * rstep;
                if (ia < nA) {
                    const int64_t row = sIa[ia];
                    pre[k][0] = U[row * ld + nv + col];
                    pre[k][1] = U[row * ld + col];
                    if constexpr (SYM) pre[k][2] = T[row * nv + col];
                }
            }
        }
    }

    // the pair's 3x3 blocks, summed over its 36 quadrature pairs; the first
    // target point assigns them
    RT Vl[9] = {}, Kl[9] = {}, Ktl[SYM ? 9 : 1] = {};
    auto accumulate = [&](auto first, int p) {
        // the source points are read from LDS at every target point rather
        // than held in registers (a compiler-only fence): fewer registers,
        // more wavefronts per SIMD
        asm volatile("" ::: "memory");
        RT s[3], t[3], u[3], dn;
        point(p, s, t, u, dn);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            RT wa;
            if constexpr (F32) wa = sc * RF.wb[p][a];
            else wa = sc * R.wb[p][a];
            const RT wk = wa * dn;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                Vl[3 * a + b] = decltype(first)::value ? wa * s[b] : fma(wa, s[b], Vl[3 * a + b]);
                Kl[3 * a + b] = decltype(first)::value ? wk * t[b] : fma(wk, t[b], Kl[3 * a + b]);
                if constexpr (SYM)
                    Ktl[3 * a + b] = decltype(first)::value ? wa * u[b] : fma(wa, u[b], Ktl[3 * a + b]);
            }
        }
    };
    accumulate(std::true_type{}, 0);
    // not unrolled: the 6 source points of one target point are the unit of ILP
#pragma unroll 1
    for (int p = 1; p < 6; ++p) accumulate(std::false_type{}, p);

    if constexpr (F32) {
        float blk[2][9], bmt[1][9];
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            blk[0][k] = Vl[k];
            blk[1][k] = Kl[k];
            bmt[0][k] = Ktl[SYM ? k : 0];
        }
        const FoldMap<MS> fm = fold_map<NT, MS>(tid, nB, sSb, TB * 3);
        fold_tile_f32<TA, TB, MS, false>(tid, tl, sl, nA, fm, sSa, acc, blk, sIa, sIb, U, ld, nv, sV, sK, pre);
        if constexpr (SYM) {
            __syncthreads();
            fold_tile_f32<TA, TB, MS, true>(tid, tl, sl, nA, fm, sSa, acc, bmt, sIa, sIb, T, nv, 0, sK, 0.0, pre);
        }
    } else {
        // FP64: the stored entries are read after the quadrature, whose registers are free by now
        const int jb = tid % nB, r0 = tid / nB, rstep = NT / nB;
        if (r0 < rstep) {
            const int64_t col = sIb[jb];
#pragma unroll
            for (int k = 0; k < fold_pf<MT>(); ++k) {
                const int ia = r0 + k * rstep;
                if (ia < nA) {
                    const int64_t row = sIa[ia];
                    pre[k][0] = U[row * ld + nv + col];
                    pre[k][1] = U[row * ld + col];
                    if constexpr (SYM) pre[k][2] = T[row * nv + col];
                }
            }
        }
        const FoldMap<MS> fm = fold_map<NT, MS>(tid, nB, sSb, TB * 3);
        fold_tile_one<TA, TB, MS, 0>(tid, tl, sl, nA, fm, sSa, acc[0], Vl, sIa, sIb, U, ld, nv, sV, pre);
        fold_tile_one<TA, TB, MS, 1>(tid, tl, sl, nA, fm, sSa, acc[0], Kl, sIa, sIb, U, ld, 0, sK, pre);
        if constexpr (SYM)
            fold_tile_one<TA, TB, MS, 2>(tid, tl, sl, nA, fm, sSa, acc[0], Ktl, sIa, sIb, T, nv, 0, sK, pre);
    }
}

// ---------------------------------------------------------------------------
// 2. completion of a symmetric evaluation
// ---------------------------------------------------------------------------
// On 32 x 32 tiles (I <= J, both mirror tiles handled by one workgroup):
// V'(i, j) = U_V(i, j) + U_V(j, i) and K'(i, j) = U_K(i, j) + T(j, i), where
// B holds [U_K | U_V] per row (signed; the regular part of V' comes out
// bitwise symmetric).
constexpr int SYMT = 32;
template <typename MT>
__global__ void __launch_bounds__(256) k_bem_symm(int64_t nv, int64_t ld, MT *__restrict__ B, const MT *__restrict__ T)
{
    const int64_t I = blockIdx.y, J = blockIdx.x;
    if (J < I) return;
    __shared__ double a[SYMT][SYMT + 1], b[SYMT][SYMT + 1], t1[SYMT][SYMT + 1], t2[SYMT][SYMT + 1];
    const int tx = threadIdx.x % SYMT, ty = threadIdx.x / SYMT;
    for (int r = ty; r < SYMT; r += 256 / SYMT) {
        const int64_t i = I * SYMT + r, j = J * SYMT + tx;   // tile (I, J)
        const int64_t i2 = J * SYMT + r, j2 = I * SYMT + tx; // tile (J, I)
        const bool in1 = i < nv && j < nv, in2 = i2 < nv && j2 < nv;
        a[r][tx] = in1 ? double(B[i * ld + nv + j]) : 0.0;
        t2[r][tx] = in1 ? double(T[i * nv + j]) : 0.0;
        b[r][tx] = in2 ? double(B[i2 * ld + nv + j2]) : 0.0;
        t1[r][tx] = in2 ? double(T[i2 * nv + j2]) : 0.0;
    }
    __syncthreads();
    for (int r = ty; r < SYMT; r += 256 / SYMT) {
        const int64_t i = I * SYMT + r, j = J * SYMT + tx;
        if (i < nv && j < nv) {
            B[i * ld + nv + j] = MT(a[r][tx] + b[tx][r]);
            add_entry(B, i * ld + j, t1[tx][r]);
        }
        const int64_t i2 = J * SYMT + r, j2 = I * SYMT + tx;
        if (I != J && i2 < nv && j2 < nv) {
            B[i2 * ld + nv + j2] = MT(b[r][tx] + a[tx][r]);
            add_entry(B, i2 * ld + j2, t2[tx][r]);
        }
    }
}

// The same completion for an even nv (every row offset of B and T is then
// even, so each thread moves aligned pairs of entries), launched over the
// tile pairs I <= J only (block k = J (J + 1) / 2 + I), with the stored K'
// entries read together with the other inputs, before the exchange.  The
// sums are those of k_bem_symm, so the results are identical.
template <typename MT>
__global__ void __launch_bounds__(256) k_bem_symm2(int64_t nv, int64_t ld, MT *__restrict__ B,
                                                   const MT *__restrict__ T)
{
    typedef MT pair_t __attribute__((ext_vector_type(2)));
    const int64_t k = blockIdx.x;
    int64_t J = int64_t((sqrt(8.0 * double(k) + 1.0) - 1.0) * 0.5);
    while (J * (J + 1) / 2 > k) --J;
    while ((J + 1) * (J + 2) / 2 <= k) ++J;
    const int64_t I = k - J * (J + 1) / 2;
    __shared__ double a[SYMT][SYMT + 1], b[SYMT][SYMT + 1], t1[SYMT][SYMT + 1], t2[SYMT][SYMT + 1];
    constexpr int TXN = SYMT / 2, RP = 256 / TXN; // threads per tile row, rows per pass
    const int tx = threadIdx.x % TXN, ty = threadIdx.x / TXN, c = 2 * tx;
    pair_t k1[SYMT / RP], k2[SYMT / RP]; // stored K' of tile (I, J) and of tile (J, I)
#pragma unroll
    for (int h = 0; h < SYMT / RP; ++h) {
        const int r = ty + h * RP;
        const int64_t i = I * SYMT + r, j = J * SYMT + c;   // tile (I, J)
        const int64_t i2 = J * SYMT + r, j2 = I * SYMT + c; // tile (J, I)
        // nv even and c even: the pair (j, j + 1) lies entirely inside or outside
        const bool in1 = i < nv && j < nv, in2 = i2 < nv && j2 < nv;
        const pair_t z = {MT(0), MT(0)};
        const pair_t va = in1 ? *reinterpret_cast<const pair_t *>(B + i * ld + nv + j) : z;
        const pair_t vt2 = in1 ? *reinterpret_cast<const pair_t *>(T + i * nv + j) : z;
        const pair_t vb = in2 ? *reinterpret_cast<const pair_t *>(B + i2 * ld + nv + j2) : z;
        const pair_t vt1 = in2 ? *reinterpret_cast<const pair_t *>(T + i2 * nv + j2) : z;
        k1[h] = in1 ? *reinterpret_cast<const pair_t *>(B + i * ld + j) : z;
        k2[h] = in2 && I != J ? *reinterpret_cast<const pair_t *>(B + i2 * ld + j2) : z;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            a[r][c + e] = double(va[e]);
            t2[r][c + e] = double(vt2[e]);
            b[r][c + e] = double(vb[e]);
            t1[r][c + e] = double(vt1[e]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < SYMT / RP; ++h) {
        const int r = ty + h * RP;
        const int64_t i = I * SYMT + r, j = J * SYMT + c;
        if (i < nv && j < nv) {
            pair_t v, w;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                v[e] = MT(a[r][c + e] + b[c + e][r]);
                w[e] = MT(double(k1[h][e]) + t1[c + e][r]);
            }
            *reinterpret_cast<pair_t *>(B + i * ld + nv + j) = v;
            *reinterpret_cast<pair_t *>(B + i * ld + j) = w;
        }
        const int64_t i2 = J * SYMT + r, j2 = I * SYMT + c;
        if (I != J && i2 < nv && j2 < nv) {
            pair_t v, w;
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                v[e] = MT(b[r][c + e] + a[c + e][r]);
                w[e] = MT(double(k2[h][e]) + t2[c + e][r]);
            }
            *reinterpret_cast<pair_t *>(B + i2 * ld + nv + j2) = v;
            *reinterpret_cast<pair_t *>(B + i2 * ld + j2) = w;
        }
    }
}

// ---------------------------------------------------------------------------
// 3. touching pairs: Sauter-Schwab (Sauter & Schwab, Boundary Element
//    Methods, Sec. 5.2) on the reference triangle {0 <= xi2 <= xi1 <= 1},
//    chi(xi) = P0 + xi1 (P1 - P0) + xi2 (P2 - P1), shape functions
//    (1 - xi1, xi1 - xi2, xi2); vertices reordered so that the shared
//    vertex is P0 (common vertex) or the shared edge is P0 P1 (common edge).
// ---------------------------------------------------------------------------
struct RefPair {
    double x1, x2, y1, y2;
};

__device__ inline int ss_region(int kind, int r, double xi, double e1, double e2, double e3, RefPair &m)
{
    // returns via m the r-th region map; the Jacobian is applied by the caller
    if (kind == 3) {
        switch (r) {
        case 0: m = {xi, xi * (1 - e1 + e1 * e2), xi * (1 - e1 * e2 * e3), xi * (1 - e1)}; break;
        case 1: m = {xi * (1 - e1 * e2 * e3), xi * (1 - e1), xi, xi * (1 - e1 + e1 * e2)}; break;
        case 2: m = {xi, xi * e1 * (1 - e2 + e2 * e3), xi * (1 - e1 * e2), xi * e1 * (1 - e2)}; break;
        case 3: m = {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * (1 - e2 + e2 * e3)}; break;
        case 4: m = {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * (1 - e2)}; break;
        default: m = {xi, xi * e1 * (1 - e2), xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3)}; break;
        }
        return 0;
    }
    if (kind == 2) {
        switch (r) {
        case 0: m = {xi, xi * e1 * e3, xi * (1 - e1 * e2), xi * e1 * (1 - e2)}; break;
        case 1: m = {xi, xi * e1, xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3)}; break;
        case 2: m = {xi * (1 - e1 * e2), xi * e1 * (1 - e2), xi, xi * e1 * e2 * e3}; break;
        case 3: m = {xi * (1 - e1 * e2 * e3), xi * e1 * e2 * (1 - e3), xi, xi * e1}; break;
        default: m = {xi * (1 - e1 * e2 * e3), xi * e1 * (1 - e2 * e3), xi, xi * e1 * e2}; break;
        }
        return 0;
    }
    if (r == 0)
        m = {xi, xi * e1, xi * e2, xi * e2 * e3};
    else
        m = {xi * e2, xi * e2 * e3, xi, xi * e1};
    return 0;
}

__device__ inline double ss_jac(int kind, int r, double xi, double e1, double e2)
{
    const double x3 = xi * xi * xi;
    if (kind == 3) return x3 * e1 * e1 * e2;
    if (kind == 2) return r == 0 ? x3 * e1 * e1 : x3 * e1 * e1 * e2;
    return x3 * e2;
}

// One wavefront per touching ordered pair (tau, sigma); lanes split the
// regions x n^4 Gauss points; the 3x3 V and K blocks (in the triangles' own
// vertex order) go to out[18 * pair].
template <bool YUK>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    k_bem_singular(int64_t ntp, const int32_t *__restrict__ tp_tau, const int32_t *__restrict__ tp_sig,
                   const int32_t *__restrict__ tri, const double *__restrict__ vx, const double *__restrict__ nrm,
                   const double *__restrict__ area, double kappa, GL4 G, double *__restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int64_t pair = (blockIdx.x * int64_t(blockDim.x) + threadIdx.x) >> 6;
    if (pair >= ntp) return;
    const int32_t ta = tp_tau[pair], sb = tp_sig[pair];
    int A[3], B[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = tri[3 * ta + k];
        B[k] = tri[3 * sb + k];
    }
    int shared = 0, ia[3] = {0, 0, 0}, ib[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (A[a] == B[b]) {
                ia[shared] = a;
                ib[shared] = b;
                ++shared;
            }
    int pa[3], pb[3];
    if (shared == 3) {
        pa[0] = pb[0] = 0;
        pa[1] = pb[1] = 1;
        pa[2] = pb[2] = 2;
    } else if (shared == 2) {
        pa[0] = ia[0];
        pa[1] = ia[1];
        pa[2] = 3 - ia[0] - ia[1];
        pb[0] = ib[0];
        pb[1] = ib[1];
        pb[2] = 3 - ib[0] - ib[1];
    } else {
        pa[0] = ia[0];
        pa[1] = (ia[0] + 1) % 3;
        pa[2] = (ia[0] + 2) % 3;
        pb[0] = ib[0];
        pb[1] = (ib[0] + 1) % 3;
        pb[2] = (ib[0] + 2) % 3;
    }
    double P[3][3], Q[3][3];
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
            P[k][d] = vx[3 * A[pa[k]] + d];
            Q[k][d] = vx[3 * B[pb[k]] + d];
        }
    const double ny0 = nrm[3 * sb], ny1 = nrm[3 * sb + 1], ny2 = nrm[3 * sb + 2];
    const int nreg = shared == 3 ? 6 : shared == 2 ? 5 : 2;
    double V[9], K[9];
    for (int k = 0; k < 9; ++k) V[k] = K[k] = 0.0;
    const int npt = nreg * 256;
    for (int idx = lane; idx < npt; idx += 64) {
        const int r = idx >> 8, pt = idx & 255;
        const int i0 = pt >> 6, i1 = (pt >> 4) & 3, i2 = (pt >> 2) & 3, i3 = pt & 3;
        const double xi = G.x[i0], e1 = G.x[i1], e2 = G.x[i2], e3 = G.x[i3];
        RefPair m;
        ss_region(shared, r, xi, e1, e2, e3, m);
        const double w = G.w[i0] * G.w[i1] * G.w[i2] * G.w[i3] * ss_jac(shared, r, xi, e1, e2);
        double x[3], y[3];
        for (int d = 0; d < 3; ++d) {
            x[d] = P[0][d] + m.x1 * (P[1][d] - P[0][d]) + m.x2 * (P[2][d] - P[1][d]);
            y[d] = Q[0][d] + m.y1 * (Q[1][d] - Q[0][d]) + m.y2 * (Q[2][d] - Q[1][d]);
        }
        const double d0 = x[0] - y[0], d1 = x[1] - y[1], d2 = x[2] - y[2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        const double ri = rsqrt(r2);
        double gv, gk;
        if (YUK) {
            const double rr = r2 * ri;
            const double e = exp(-kappa * rr);
            gv = e * ri;
            gk = (d0 * ny0 + d1 * ny1 + d2 * ny2) * (1.0 + kappa * rr) * e * ri * ri * ri;
        } else {
            gv = ri;
            gk = (d0 * ny0 + d1 * ny1 + d2 * ny2) * ri * ri * ri;
        }
        if (shared == 3) gk = 0.0; // (x - y).n_y vanishes on a flat panel
        const double fx[3] = {1.0 - m.x1, m.x1 - m.x2, m.x2};
        const double fy[3] = {1.0 - m.y1, m.y1 - m.y2, m.y2};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double ww = w * fx[a] * fy[b];
                V[3 * a + b] += ww * gv;
                K[3 * a + b] += ww * gk;
            }
    }
    for (int k = 0; k < 9; ++k)
        for (int off = 32; off > 0; off >>= 1) {
            V[k] += __shfl_xor(V[k], off);
            K[k] += __shfl_xor(K[k], off);
        }
    if (lane == 0) {
        const double sc = 4.0 * area[ta] * area[sb] * INV4PI;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                out[18 * pair + 3 * pa[a] + pb[b]] = sc * V[3 * a + b];
                out[18 * pair + 9 + 3 * pa[a] + pb[b]] = sc * K[3 * a + b];
            }
    }
}

// Row-owned scatter of the touching-pair blocks and of the 1/2 M term into
// the stored operator (Morton vertex order: vertex i is row minv[i]).
template <typename MT>
__global__ void k_bem_scatter(int64_t nv, int64_t ld, const int32_t *__restrict__ minv,
                              const int32_t *__restrict__ v2t_ptr, const int32_t *__restrict__ v2t,
                              const int32_t *__restrict__ tri, const int32_t *__restrict__ tp_ptr,
                              const int32_t *__restrict__ tp_sig, const double *__restrict__ tpv,
                              const double *__restrict__ area, double sV, double sK, MT *__restrict__ Bo)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    MT *row = Bo + int64_t(minv[i]) * ld;
    for (int32_t e = v2t_ptr[i]; e < v2t_ptr[i + 1]; ++e) {
        const int32_t ta = v2t[e] / 3, a = v2t[e] % 3;
        for (int32_t pp = tp_ptr[ta]; pp < tp_ptr[ta + 1]; ++pp) {
            const int32_t sb = tp_sig[pp];
            const double *blk = tpv + 18 * int64_t(pp);
            for (int b = 0; b < 3; ++b) {
                const int64_t j = minv[tri[3 * sb + b]];
                add_entry(row, nv + j, sV * blk[3 * a + b]);
                add_entry(row, j, sK * blk[9 + 3 * a + b]);
            }
        }
        for (int b = 0; b < 3; ++b)
            add_entry(row, minv[tri[3 * ta + b]], 0.5 * area[ta] * (a == b ? 2.0 : 1.0) / 12.0);
    }
}

__global__ void k_gather_coords(int64_t nv, const int32_t *__restrict__ g, const double *__restrict__ x,
                                double *__restrict__ vx)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    for (int d = 0; d < 3; ++d) vx[3 * i + d] = x[3 * g[i] + d];
}

// diagonal of V' in the ascending vertex order
template <typename MT>
__global__ void k_vdiag(int64_t nv, int64_t ld, const int32_t *__restrict__ mvert, const MT *__restrict__ B,
                        double *__restrict__ vdiag)
{
    const int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (k < nv) vdiag[mvert[k]] = double(B[k * ld + nv + k]);
}

// ---------------------------------------------------------------------------
// sparse approximate inverse of the single-layer block (GMRES preconditioner)
// ---------------------------------------------------------------------------
constexpr int SPAI_SMALL = 8; // largest 1-ring of the one-wavefront path
// Row i minimises || m^T V' - e_i^T ||_2 over m supported on the 1-ring P(i)
// of vertex i, V' = columns [nv, 2nv) of the stored rows (the signed
// single-layer block of the operator; vertex v is row / column minv[v]).  Normal equations
// (V'_P V'_P^T) m = V'_P e_i, solved by Cholesky.  One workgroup per row;
// the Gram matrix accumulates over 64-column tiles of the rows P staged in
// LDS, one thread per (a, b) pair, in a fixed order.
template <typename MT>
__global__ void __launch_bounds__(256)
    k_spai(int64_t nv, const MT *__restrict__ B, int64_t ld, const int32_t *__restrict__ minv,
           const int32_t *__restrict__ ring_ptr, const int32_t *__restrict__ ring, double *__restrict__ val,
           int *__restrict__ bad)
{
    __shared__ double T[MAXRING][65];
    __shared__ double G[MAXRING][MAXRING + 1];
    __shared__ double rhs[MAXRING];
    __shared__ int P[MAXRING];
    const int tid = threadIdx.x;
    const int64_t i = blockIdx.x;
    const int p0 = ring_ptr[i], m = ring_ptr[i + 1] - p0;
    if (m <= SPAI_SMALL) return; // handled by k_spai_small
    for (int a = tid; a < m; a += 256) P[a] = minv[ring[p0 + a]];
    __syncthreads();
    const int npair = m * (m + 1) / 2;
    constexpr int PPT = (MAXRING * (MAXRING + 1) / 2 + 255) / 256; // pairs per thread
    double acc[PPT];
    int pa[PPT], pb[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        acc[q] = 0.0;
        const int pr = tid + 256 * q;
        int a = int((sqrt(8.0 * pr + 1.0) - 1.0) * 0.5);
        while (a * (a + 1) / 2 > pr) --a;
        while ((a + 1) * (a + 2) / 2 <= pr) ++a;
        pa[q] = a;
        pb[q] = pr - a * (a + 1) / 2;
    }
    for (int64_t c0 = 0; c0 < nv; c0 += 64) {
        for (int k = tid; k < m * 64; k += 256) {
            const int a = k >> 6, c = k & 63;
            T[a][c] = c0 + c < nv ? double(B[int64_t(P[a]) * ld + nv + c0 + c]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (tid + 256 * q < npair) {
                const int a = pa[q], b = pb[q];
                double s = 0.0;
                for (int c = 0; c < 64; ++c) s = fma(T[a][c], T[b][c], s);
                acc[q] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PPT; ++q)
        if (tid + 256 * q < npair) G[pa[q]][pb[q]] = G[pb[q]][pa[q]] = acc[q];
    for (int a = tid; a < m; a += 256) rhs[a] = double(B[int64_t(P[a]) * ld + nv + minv[i]]);
    __syncthreads();
    if (tid == 0) {
        // Cholesky G = L L^T (lower triangle), then L y = rhs, L^T m = y
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
                double s = G[b][a];
                for (int k = 0; k < a; ++k) s -= G[b][k] * G[a][k];
                G[b][a] = s / G[a][a];
            }
        }
        if (!ok) {
            atomicOr(bad, 4);
            for (int a = 0; a < m; ++a) val[p0 + a] = 0.0;
        } else {
            for (int a = 0; a < m; ++a) {
                double s = rhs[a];
                for (int k = 0; k < a; ++k) s -= G[a][k] * rhs[k];
                rhs[a] = s / G[a][a];
            }
            for (int a = m - 1; a >= 0; --a) {
                double s = rhs[a];
                for (int k = a + 1; k < m; ++k) s -= G[k][a] * rhs[k];
                rhs[a] = s / G[a][a];
            }
            for (int a = 0; a < m; ++a) val[p0 + a] = rhs[a];
        }
    }
}

// Rows whose 1-ring has at most SPAI_SMALL vertices (every vertex of the
// usual surface meshes): one wavefront per row, each lane streams W
// consecutive columns at a time (one 16-byte load per row: W = 4 for FP32,
// 2 for FP64) of the m rows and keeps the m (m + 1) / 2 Gram partial sums in
// registers; a fixed xor-shuffle tree then sums them across the lanes.  The
// V' columns start at column nv of rows of ld (a multiple of 256) entries,
// so the first head = (-nv) mod W columns are taken one per lane and the
// W-wide loads start at an aligned column.
template <typename MT, int W> struct alignas(W * sizeof(MT)) SpaiVec {
    MT v[W];
};
template <typename MT, int W>
__global__ void __launch_bounds__(256)
    k_spai_small(int64_t nv, const MT *__restrict__ B, int64_t ld, const int32_t *__restrict__ minv,
                 const int32_t *__restrict__ ring_ptr, const int32_t *__restrict__ ring, double *__restrict__ val,
                 int *__restrict__ bad)
{
    constexpr int NP = SPAI_SMALL * (SPAI_SMALL + 1) / 2;
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * int64_t(4) + (threadIdx.x >> 6);
    if (i >= nv) return;
    const int p0 = ring_ptr[i], m = ring_ptr[i + 1] - p0;
    if (m > SPAI_SMALL) return; // handled by k_spai
    const MT *rows[SPAI_SMALL];
#pragma unroll
    for (int a = 0; a < SPAI_SMALL; ++a) rows[a] = B + int64_t(minv[ring[p0 + (a < m ? a : 0)]]) * ld + nv;
    double g[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) g[k] = 0.0;
    const int head = int((W - nv % W) % W);
    if (lane < head) {
        double x[SPAI_SMALL];
#pragma unroll
        for (int a = 0; a < SPAI_SMALL; ++a) x[a] = a < m ? double(rows[a][lane]) : 0.0;
        int k = 0;
#pragma unroll
        for (int a = 0; a < SPAI_SMALL; ++a)
#pragma unroll
            for (int b = 0; b <= a; ++b, ++k) g[k] = fma(x[a], x[b], g[k]);
    }
    for (int64_t c = head + int64_t(W) * lane; c < nv; c += 64 * W) {
        if constexpr (sizeof(MT) == 4) {
            // FP32 storage: the loaded values stay FP32 and each column is
            // widened when its products are formed (162 instead of 181 VGPRs,
            // three wavefronts per SIMD instead of two: 11.2 -> 4.7 ms per
            // 80k-triangle interface)
            SpaiVec<MT, W> t[SPAI_SMALL];
            if (c + W <= nv) {
#pragma unroll
                for (int a = 0; a < SPAI_SMALL; ++a) t[a] = *reinterpret_cast<const SpaiVec<MT, W> *>(rows[a] + c);
            } else {
#pragma unroll
                for (int a = 0; a < SPAI_SMALL; ++a)
#pragma unroll
                    for (int w = 0; w < W; ++w) t[a].v[w] = c + w < nv ? rows[a][c + w] : MT(0);
            }
#pragma unroll
            for (int w = 0; w < W; ++w) {
                double x[SPAI_SMALL];
#pragma unroll
                for (int a = 0; a < SPAI_SMALL; ++a) x[a] = a < m ? double(t[a].v[w]) : 0.0;
                int k = 0;
#pragma unroll
                for (int a = 0; a < SPAI_SMALL; ++a)
#pragma unroll
                    for (int b = 0; b <= a; ++b, ++k) g[k] = fma(x[a], x[b], g[k]);
            }
            continue;
        }
        double x[SPAI_SMALL][W];
        if (c + W <= nv) {
#pragma unroll
            for (int a = 0; a < SPAI_SMALL; ++a) {
                const SpaiVec<MT, W> t = *reinterpret_cast<const SpaiVec<MT, W> *>(rows[a] + c);
#pragma unroll
                for (int w = 0; w < W; ++w) x[a][w] = a < m ? double(t.v[w]) : 0.0;
            }
        } else {
#pragma unroll
            for (int a = 0; a < SPAI_SMALL; ++a)
#pragma unroll
                for (int w = 0; w < W; ++w) x[a][w] = a < m && c + w < nv ? double(rows[a][c + w]) : 0.0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            int k = 0;
#pragma unroll
            for (int a = 0; a < SPAI_SMALL; ++a)
#pragma unroll
                for (int b = 0; b <= a; ++b, ++k) g[k] = fma(x[a][w], x[b][w], g[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k)
        for (int off = 32; off > 0; off >>= 1) g[k] += __shfl_xor(g[k], off);
    if (lane != 0) return;
    // Cholesky in place on the packed lower triangle g[a (a + 1) / 2 + b]
#define GP(a, b) g[(a) * ((a) + 1) / 2 + (b)]
    double r[SPAI_SMALL];
    const int64_t ci = minv[i];
#pragma unroll
    for (int a = 0; a < SPAI_SMALL; ++a) r[a] = a < m ? double(rows[a][ci]) : 0.0;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < SPAI_SMALL; ++a) {
        if (a < m) {
            double d = GP(a, a);
#pragma unroll
            for (int k = 0; k < a; ++k) d -= GP(a, k) * GP(a, k);
            ok = ok && d > 0.0;
            GP(a, a) = sqrt(d);
#pragma unroll
            for (int b = a + 1; b < SPAI_SMALL; ++b) {
                if (b < m) {
                    double t = GP(b, a);
#pragma unroll
                    for (int k = 0; k < a; ++k) t -= GP(b, k) * GP(a, k);
                    GP(b, a) = t / GP(a, a);
                }
            }
        }
    }
    if (!ok) {
        atomicOr(bad, 4);
        for (int a = 0; a < m; ++a) val[p0 + a] = 0.0;
        return;
    }
#pragma unroll
    for (int a = 0; a < SPAI_SMALL; ++a) {
        if (a < m) {
            double t = r[a];
#pragma unroll
            for (int k = 0; k < a; ++k) t -= GP(a, k) * r[k];
            r[a] = t / GP(a, a);
        }
    }
#pragma unroll
    for (int a = SPAI_SMALL - 1; a >= 0; --a) {
        if (a < m) {
            double t = r[a];
#pragma unroll
            for (int k = a + 1; k < SPAI_SMALL; ++k)
                if (k < m) t -= GP(k, a) * r[k];
            r[a] = t / GP(a, a);
        }
    }
#undef GP
#pragma unroll
    for (int a = 0; a < SPAI_SMALL; ++a)
        if (a < m) val[p0 + a] = r[a];
}

// Delta_kl = V'_kl - V'_lk on the upper two-ring pattern of the Morton vertex
// order, from the stored operator (one thread per row)
template <typename MT>
__global__ void k_sym_delta(int64_t nv, int64_t ld, const MT *__restrict__ B, const int32_t *__restrict__ dptr,
                            const int32_t *__restrict__ dcol, double *__restrict__ dval)
{
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= nv) return;
    for (int32_t e = dptr[i]; e < dptr[i + 1]; ++e) {
        const int64_t j = dcol[e];
        dval[e] = double(B[i * ld + nv + j]) - double(B[j * ld + nv + i]);
    }
}

// ===========================================================================
// host orchestration
// ===========================================================================
int64_t bem_ld(int64_t nv) { return ((2 * nv + 255) / 256) * 256; }

// device copy of the block tables of block size bs (in the surface's arena)
static const BlockSideDev &device_side(Problem &p, int w, int bs, hipStream_t s)
{
    SurfaceDev &S = p.surf[w];
    auto it = S.sides.find(bs);
    if (it != S.sides.end()) return it->second;
    const BlockSide &H = block_side(p.topo[w], bs);
    Arena &A = p.bem_arena[w];
    BlockSideDev D;
    D.bs = bs;
    D.nb = H.nb;
    D.S = H.S;
    D.pref = A.upload(H.pref, s);
    D.nvb = A.upload(H.nvb, s);
    D.slots = A.upload(H.slots, s);
    D.vid = A.upload(H.vid, s);
    // the blocks of each colour, then every block in order (the tuner's lists)
    std::vector<int32_t> lists(H.col_blk);
    for (int64_t b = 0; b < H.nb; ++b) lists.push_back(int32_t(b));
    D.col_blk = A.upload(lists, s);
    return S.sides.emplace(bs, D).first->second;
}

struct RegArgs {
    int64_t nt = 0;
    const int32_t *m_tri = nullptr;
    const void *xq = nullptr, *nq = nullptr;
    const double *cen = nullptr, *m_area = nullptr;
    BlockSideDev A, B;
    const int32_t *listA = nullptr, *listB = nullptr; // device block lists of the launch
    int64_t nA = 0, nB = 0;                            // their lengths
    int skip_lower = 0;
    void *U = nullptr, *T = nullptr; // operator rows [K' | V'] and the mirrored double layer (square shapes)
    int64_t ld = 0, nv = 0;
    double sV = 0.0, sK = 0.0;
    double kappa = 0.0;
    int ms = MAXS; // largest corner count of a vertex in a block, both sides
    QRule6 R;
    QRule6F RF;
};

// square shapes evaluate each unordered pair once (SYM)
template <int TA, int TB> constexpr bool shape_sym() { return TA == TB; }
template <int TA, int TB, int MS> static void launch_regular_ms(bool yuk, bool f32, const RegArgs &a, hipStream_t s)
{
    if (a.nA == 0 || a.nB == 0) return;
    const dim3 grid(unsigned(a.nB), unsigned(a.nA));
    constexpr bool SYM = shape_sym<TA, TB>();
#define PB_REG(Y, RT)                                                                                              \
    hipLaunchKernelGGL((k_bem_regular<Y, RT, RT, TA, TB, MS, SYM>), grid, dim3(TA * TB), 0, s, a.nt, a.m_tri,      \
                       static_cast<const RT *>(a.xq), static_cast<const RT *>(a.nq), a.cen, a.m_area, a.A.pref,     \
                       a.A.nvb, a.A.slots, a.A.vid, a.B.pref, a.B.nvb, a.B.slots, a.B.vid, a.listA, a.listB,        \
                       a.skip_lower, static_cast<RT *>(a.U), static_cast<RT *>(a.T), a.ld, a.nv, a.sV, a.sK,        \
                       a.kappa, a.R, a.RF)
    if (f32) {
        if (yuk) PB_REG(true, float);
        else PB_REG(false, float);
    } else {
        if (yuk) PB_REG(true, double);
        else PB_REG(false, double);
    }
#undef PB_REG
}
template <int TA, int TB> static void launch_regular_t(bool yuk, bool f32, const RegArgs &a, hipStream_t s)
{
    if (a.ms <= 6) launch_regular_ms<TA, TB, 6>(yuk, f32, a, s);
    else if (a.ms <= 12) launch_regular_ms<TA, TB, 12>(yuk, f32, a, s);
    else launch_regular_ms<TA, TB, MAXS>(yuk, f32, a, s);
}

static_assert(N_TILE_SHAPES == 5, "one launch case per candidate tile shape");
static void launch_regular(int shape, bool yuk, bool f32, const RegArgs &a, hipStream_t s)
{
    switch (shape) {
    case 0: launch_regular_t<TILE_SHAPES[0].ta, TILE_SHAPES[0].tb>(yuk, f32, a, s); break;
    case 1: launch_regular_t<TILE_SHAPES[1].ta, TILE_SHAPES[1].tb>(yuk, f32, a, s); break;
    case 2: launch_regular_t<TILE_SHAPES[2].ta, TILE_SHAPES[2].tb>(yuk, f32, a, s); break;
    case 3: launch_regular_t<TILE_SHAPES[3].ta, TILE_SHAPES[3].tb>(yuk, f32, a, s); break;
    case 4: launch_regular_t<TILE_SHAPES[4].ta, TILE_SHAPES[4].tb>(yuk, f32, a, s); break;
    default: PB_CHECK(false, PBFB_EINVAL, "unknown tile shape");
    }
}

// Every tile of the assembly, one launch per pair of colours so that no two
// tiles of a launch touch the same operator entry; launches follow each other
// on the stream, so every entry receives its contributions in a fixed order.
// Square shapes: launch (c1, c2), c1 < c2, takes every target block of colour
// c1 against every source block of colour c2 (one orientation per unordered
// block pair); launch (c, c) the pairs with source block >= target block.
// Rectangular shapes (target and source blocks coloured separately): every
// colour pair, every tile.
static void launch_all_tiles(int shape, bool yuk, bool f32, RegArgs a, const BlockSide &HA, const BlockSide &HB,
                             hipStream_t s)
{
    const bool sym = TILE_SHAPES[shape].ta == TILE_SHAPES[shape].tb;
    for (int c1 = 0; c1 < HA.ncolor; ++c1)
        for (int c2 = sym ? c1 : 0; c2 < HB.ncolor; ++c2) {
            a.listA = a.A.col_blk + HA.col_ptr[c1];
            a.nA = HA.col_ptr[c1 + 1] - HA.col_ptr[c1];
            a.listB = a.B.col_blk + HB.col_ptr[c2];
            a.nB = HB.col_ptr[c2 + 1] - HB.col_ptr[c2];
            a.skip_lower = sym && c1 == c2 ? 1 : 0;
            launch_regular(shape, yuk, f32, a, s);
        }
}

// cache key of the tuned shape: precision, kernel and size class (floor log2 of the triangle count)
static int tile_key(int precision, bool yuk, int64_t nt)
{
    int c = 0;
    while (c < 62 && (int64_t(2) << c) <= nt) ++c;
    return (precision * 2 + (yuk ? 1 : 0)) * 64 + c;
}

// Autotuner: times the regular tile kernel of every candidate shape on the
// same sample of this surface (min(nt, 512) Morton-ordered target triangles
// from the middle of the order against all source triangles, so that a
// symmetric shape, which skips the source blocks below the target block,
// does the average share of its work; one warm-up launch, then the fastest
// of three timed launches) and returns the shape with the shortest time per
// target triangle.  Runs with the context workspace held.
static void tune_range(const BlockSide &HA, int64_t nsample, int64_t &b0, int64_t &b1)
{
    const int64_t nbs = std::min<int64_t>((nsample + HA.bs - 1) / HA.bs, HA.nb);
    b0 = (HA.nb - nbs) / 2;
    b1 = b0 + nbs;
}
static int tile_tune(Problem &p, int w, RegArgs a, bool yuk, bool f32, hipStream_t s)
{
    // the timed launches add into the operator and T (a.U, a.T), which are
    // cleared before the assembly proper; their tiles are not coloured (the
    // values are discarded, so unordered additions do not matter here)
    SurfaceTopo &T = p.topo[w];
    const int64_t nsample = std::min<int64_t>(T.nt, 512);
    hipEvent_t e0, e1;
    PB_HIP(hipEventCreate(&e0));
    PB_HIP(hipEventCreate(&e1));
    int best = 0;
    double best_t = 1e300;
    for (int k = 0; k < N_TILE_SHAPES; ++k) {
        const BlockSide &HA = block_side(T, TILE_SHAPES[k].ta), &HB = block_side(T, TILE_SHAPES[k].tb);
        a.A = device_side(p, w, HA.bs, s);
        a.B = device_side(p, w, HB.bs, s);
        a.ms = std::max(HA.ms_max, HB.ms_max);
        int64_t b0, b1;
        tune_range(HA, nsample, b0, b1);
        a.listA = a.A.col_blk + HA.nb + b0; // blocks b0 .. b1 - 1 of the in-order list
        a.nA = b1 - b0;
        a.listB = a.B.col_blk + HB.nb;
        a.nB = HB.nb;
        a.skip_lower = TILE_SHAPES[k].ta == TILE_SHAPES[k].tb ? 1 : 0;
        const int64_t tris = std::min<int64_t>(b1 * HA.bs, T.nt) - b0 * HA.bs;
        launch_regular(k, yuk, f32, a, s);
        float ms = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            PB_HIP(hipEventRecord(e0, s));
            launch_regular(k, yuk, f32, a, s);
            PB_HIP(hipEventRecord(e1, s));
            PB_HIP(hipEventSynchronize(e1));
            float t = 0.0f;
            PB_HIP(hipEventElapsedTime(&t, e0, e1));
            ms = std::min(ms, t);
        }
        PB_HIP(hipGetLastError());
        const double per = double(ms) / double(tris);
        if (per < best_t) {
            best_t = per;
            best = k;
        }
    }
    PB_HIP(hipEventDestroy(e0));
    PB_HIP(hipEventDestroy(e1));
    return best;
}

void ensure_bem(Problem &p, int w, hipStream_t s)
{
    if (p.bem_ready[w]) return;
    ensure_geometry(p, s);
    SurfaceTopo &T = p.topo[w];
    SurfaceDev &S = p.surf[w];
    Arena &A = p.bem_arena[w];
    const bool yuk = (w == 1) && p.kappa > 0.0;
    const bool f32 = p.precision == PBFB_MIXED;
    const double kappa = (w == 1) ? p.kappa : 0.0;
    if (!p.bem_topo_ready[w]) {
        // Morton order and triangle data: once per mesh (block tables are
        // uploaded per block size when a tile shape needs them)
        A.release();
        S.sides.clear();
        S.tile = -1;
        S.B = nullptr;
        S.m_tri = A.alloc<int32_t>(3 * T.nt);
        S.m_area = A.alloc<double>(T.nt);
        S.m_qp = S.m_nrm = S.m_cen = nullptr;
        S.m_qf = S.m_nf = nullptr;
        if (f32) {
            S.m_cen = A.alloc<double>(3 * T.nt);
            S.m_qf = A.alloc<float>(18 * T.nt);
            S.m_nf = A.alloc<float>(3 * T.nt);
        } else {
            S.m_qp = A.alloc<double>(18 * T.nt);
            S.m_nrm = A.alloc<double>(3 * T.nt);
        }
        S.morton = A.upload(T.morton, s);
        S.tp_ptr = A.upload(T.tp_ptr, s);
        S.tp_sig = A.upload(T.tp_sig, s);
        S.ntp = int64_t(T.tp_sig.size());
        std::vector<int32_t> tp_tau(S.ntp);
        for (int64_t t = 0; t < T.nt; ++t)
            for (int32_t k = T.tp_ptr[t]; k < T.tp_ptr[t + 1]; ++k) tp_tau[k] = int32_t(t);
        S.tp_tau = A.upload(tp_tau, s);
        S.vdiag = A.alloc<double>(T.nv);
        S.tpv = nullptr;
        S.mpos = nullptr;
        S.nf_ptr = S.nf_col = S.nf_row = nullptr;
        S.nf_val = nullptr;
        S.nf_nnz = 0;
        S.d_ptr = S.d_col = nullptr;
        S.d_val = nullptr;
        S.sym = false;
        S.ring_ptr = A.upload(T.ring_ptr, s);
        S.ring = A.upload(T.ring, s);
        S.spai = A.alloc<double>(T.ring.size());
        if (p.bem_mf) {
            // matrix-free: resident touching-pair blocks, the Morton position of
            // each triangle and the near-field rows of the preconditioner
            S.tpv = A.alloc<double>(18 * S.ntp);
            std::vector<int32_t> mpos(T.nt);
            for (int64_t m = 0; m < T.nt; ++m) mpos[T.morton[m]] = int32_t(m);
            S.mpos = A.upload(mpos, s);
            near_pattern(T);
            S.nf_nnz = int64_t(T.nf_col.size());
            std::vector<int32_t> nf_row(S.nf_nnz);
            for (int64_t i = 0; i < T.nv; ++i)
                for (int32_t k = T.nf_ptr[i]; k < T.nf_ptr[i + 1]; ++k) nf_row[k] = int32_t(i);
            S.nf_ptr = A.upload(T.nf_ptr, s);
            S.nf_col = A.upload(T.nf_col, s);
            S.nf_row = A.upload(nf_row, s);
            S.nf_val = A.alloc<double>(S.nf_nnz);
        } else {
            const int64_t ldt = bem_ld(T.nv);
            if (f32) S.B = A.alloc<float>(T.nv * ldt);
            else S.B = A.alloc<double>(T.nv * ldt);
            delta_pattern(T);
            S.d_ptr = A.upload(T.d2_ptr, s);
            S.d_col = A.upload(T.d2_col, s);
            S.d_val = A.alloc<double>(std::max<size_t>(T.d2_col.size(), 1));
        }
        PB_HIP(hipStreamSynchronize(s));
        p.bem_topo_ready[w] = true;
    }
    int32_t *d_tptau = S.tp_tau;
    hipLaunchKernelGGL(k_tri_morton, dim3(nblk(T.nt, 256)), dim3(256), 0, s, T.nt, S.morton, S.tri, S.qp, S.nrm,
                       S.area, S.g, S.x, S.m_tri, S.m_qp, S.m_nrm, S.m_area, S.m_cen, S.m_qf, S.m_nf);

    // one of the context's assembly workspaces (see below), used by one assembly at a time
    Workspace *wsp = nullptr;
    std::unique_lock<std::mutex> ws_lock;
    while (!wsp) {
        for (Workspace &W : p.ctx->asm_ws) {
            std::unique_lock<std::mutex> l(W.mu, std::try_to_lock);
            if (l.owns_lock()) {
                wsp = &W;
                ws_lock = std::move(l);
                break;
            }
        }
        if (!wsp) std::this_thread::sleep_for(std::chrono::microseconds(100));
    }
    struct Drain { // on every exit the stream drains before the workspace is released
        hipStream_t s;
        ~Drain() { (void)hipStreamSynchronize(s); }
    } drain{s};
    if (p.bem_mf) {
        // matrix-free: only the touching-pair blocks (kept) and the diagonal of V'
        double *vxm = wsp->doubles(3 * T.nv);
        hipLaunchKernelGGL(k_gather_coords, dim3(nblk(T.nv, 256)), dim3(256), 0, s, T.nv, S.g, S.x, vxm);
        GL4 G = gl4arg();
        if (p.timing) p.timer.begin(T_SING, s);
        if (yuk)
            hipLaunchKernelGGL(k_bem_singular<true>, dim3(nblk(S.ntp * 64, 256)), dim3(256), 0, s, S.ntp, d_tptau,
                               S.tp_sig, S.tri, vxm, S.nrm, S.area, kappa, G, S.tpv);
        else
            hipLaunchKernelGGL(k_bem_singular<false>, dim3(nblk(S.ntp * 64, 256)), dim3(256), 0, s, S.ntp, d_tptau,
                               S.tp_sig, S.tri, vxm, S.nrm, S.area, kappa, G, S.tpv);
        if (p.timing) p.timer.end(s);
        PB_HIP(hipGetLastError());
        mf_vdiag(p, w, s);
        mf_spai(p, w, s);
        PB_HIP(hipStreamSynchronize(s));
        S.tile = -1;
        p.bem_ready[w] = true;
        return;
    }
    const int64_t nv = T.nv, ld = bem_ld(nv);
    const size_t elem = f32 ? sizeof(float) : sizeof(double);
    // Gamma_m (and an independent Gamma_m mesh): V' = -V0, K' = 1/2 M + K0;
    // Gamma_s: V' = +Vk, K' = 1/2 M - Kk
    const double sV = (w != 1) ? -1.0 : 1.0, sK = (w != 1) ? 1.0 : -1.0;
    RegArgs ra;
    ra.nt = T.nt;
    ra.m_tri = S.m_tri;
    ra.xq = f32 ? static_cast<const void *>(S.m_qf) : static_cast<const void *>(S.m_qp);
    ra.nq = f32 ? static_cast<const void *>(S.m_nf) : static_cast<const void *>(S.m_nrm);
    ra.cen = S.m_cen;
    ra.m_area = S.m_area;
    ra.kappa = kappa;
    ra.R = q6arg();
    ra.RF = q6farg();
    ra.U = S.B;
    ra.ld = ld;
    ra.nv = nv;
    ra.sV = sV;
    ra.sK = sK;
    // the context's assembly workspace: the mirrored double layer T of a
    // square-tile assembly (nv x nv in the storage precision), vertex
    // coordinates and the touching-pair blocks
    const size_t tbytes = (size_t(nv) * nv * elem + 255) / 256 * 256;
    double *ws = wsp->doubles((tbytes + 8 * (3 * size_t(nv) + 18 * size_t(S.ntp))) / 8 + 1);
    void *Tm = ws;
    double *vx = reinterpret_cast<double *>(static_cast<char *>(Tm) + tbytes), *tpv = vx + 3 * nv;
    ra.T = Tm;
    // tile shape: forced, or tuned once per (precision, kernel, size class) and context
    int shape = p.tile_fixed;
    if (shape < 0) {
        const int key = tile_key(p.precision, yuk, T.nt);
        std::lock_guard<std::mutex> tl(p.ctx->tune_mu);
        auto it = p.ctx->tile_choice.find(key);
        if (it != p.ctx->tile_choice.end()) {
            shape = it->second;
        } else {
            shape = tile_tune(p, w, ra, yuk, f32, s);
            p.ctx->tile_choice[key] = shape;
        }
    }
    S.tile = shape;
    const BlockSide &HA = block_side(T, TILE_SHAPES[shape].ta), &HB = block_side(T, TILE_SHAPES[shape].tb);
    ra.A = device_side(p, w, TILE_SHAPES[shape].ta, s);
    ra.B = device_side(p, w, TILE_SHAPES[shape].tb, s);
    ra.ms = std::max(HA.ms_max, HB.ms_max);
    const bool sym = TILE_SHAPES[shape].ta == TILE_SHAPES[shape].tb;
    // every tile adds into the operator: start from zero (the row padding
    // past 2 nv, read by the dense apply against zero inputs, stays zero)
    PB_HIP(hipMemsetAsync(S.B, 0, size_t(nv) * ld * elem, s));
    if (sym) PB_HIP(hipMemsetAsync(Tm, 0, size_t(nv) * nv * elem, s));
    if (p.timing) p.timer.begin(T_ASM, s);
    launch_all_tiles(shape, yuk, f32, ra, HA, HB, s);
    if (p.timing) p.timer.end(s);
    PB_HIP(hipGetLastError());
    if (sym) {
        const unsigned nbt = unsigned((nv + SYMT - 1) / SYMT);
        // FP32 storage with an even nv: pairs of entries, upper tile pairs only
        // (11.3 -> 7.7 ms per 80k-triangle interface); the same form ran FP64
        // storage slower (14.5 -> 19.9 ms), which keeps the one-entry kernel
        const int64_t npair = int64_t(nbt) * (nbt + 1) / 2; // one-dimensional grid: npair * 256 < 2^32
        if (f32 && nv % 2 == 0 && ld % 2 == 0 && npair * 256 < (int64_t(1) << 32))
            hipLaunchKernelGGL(k_bem_symm2<float>, dim3(unsigned(npair)), dim3(256), 0, s, nv, ld,
                               static_cast<float *>(S.B), static_cast<const float *>(Tm));
        else if (f32)
            hipLaunchKernelGGL(k_bem_symm<float>, dim3(nbt, nbt), dim3(256), 0, s, nv, ld, static_cast<float *>(S.B),
                               static_cast<const float *>(Tm));
        else
            hipLaunchKernelGGL(k_bem_symm<double>, dim3(nbt, nbt), dim3(256), 0, s, nv, ld,
                               static_cast<double *>(S.B), static_cast<const double *>(Tm));
        PB_HIP(hipGetLastError());
    }
    // touching pairs
    hipLaunchKernelGGL(k_gather_coords, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, S.g, S.x, vx);
    GL4 G = gl4arg();
    if (p.timing) p.timer.begin(T_SING, s);
    if (yuk)
        hipLaunchKernelGGL(k_bem_singular<true>, dim3(nblk(S.ntp * 64, 256)), dim3(256), 0, s, S.ntp, d_tptau,
                           S.tp_sig, S.tri, vx, S.nrm, S.area, kappa, G, tpv);
    else
        hipLaunchKernelGGL(k_bem_singular<false>, dim3(nblk(S.ntp * 64, 256)), dim3(256), 0, s, S.ntp, d_tptau,
                           S.tp_sig, S.tri, vx, S.nrm, S.area, kappa, G, tpv);
    if (p.timing) p.timer.end(s);
    PB_HIP(hipGetLastError());
    if (f32)
        hipLaunchKernelGGL(k_bem_scatter<float>, dim3(nblk(nv, 64)), dim3(64), 0, s, nv, ld, S.minv, S.v2t_ptr, S.v2t,
                           S.tri, S.tp_ptr, S.tp_sig, tpv, S.area, sV, sK, static_cast<float *>(S.B));
    else
        hipLaunchKernelGGL(k_bem_scatter<double>, dim3(nblk(nv, 64)), dim3(64), 0, s, nv, ld, S.minv, S.v2t_ptr,
                           S.v2t, S.tri, S.tp_ptr, S.tp_sig, tpv, S.area, sV, sK, static_cast<double *>(S.B));
    PB_HIP(hipGetLastError());
    // diagonal of V', symmetric storage use (Delta from the stored values),
    // approximate inverse of the single-layer block (from the stored values)
    // symmetric use: the apply reads K' and the lower triangle of V' (square
    // tiles leave the regular part of V' bitwise symmetric)
    S.sym = sym;
    PB_HIP(hipMemsetAsync(p.d_bad, 0, sizeof(int), s));
    if (f32) {
        const float *Bf = static_cast<const float *>(S.B);
        hipLaunchKernelGGL(k_vdiag<float>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, ld, S.mvert, Bf, S.vdiag);
        if (sym)
            hipLaunchKernelGGL(k_sym_delta<float>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, ld, Bf, S.d_ptr, S.d_col,
                               S.d_val);
        hipLaunchKernelGGL((k_spai_small<float, 4>), dim3(nblk(nv, 4)), dim3(256), 0, s, nv, Bf, ld, S.minv,
                           S.ring_ptr, S.ring, S.spai, p.d_bad);
        if (T.max_ring > SPAI_SMALL)
            hipLaunchKernelGGL(k_spai<float>, dim3(unsigned(nv)), dim3(256), 0, s, nv, Bf, ld, S.minv, S.ring_ptr,
                               S.ring, S.spai, p.d_bad);
    } else {
        const double *Bd = static_cast<const double *>(S.B);
        hipLaunchKernelGGL(k_vdiag<double>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, ld, S.mvert, Bd, S.vdiag);
        if (sym)
            hipLaunchKernelGGL(k_sym_delta<double>, dim3(nblk(nv, 256)), dim3(256), 0, s, nv, ld, Bd, S.d_ptr,
                               S.d_col, S.d_val);
        hipLaunchKernelGGL((k_spai_small<double, 2>), dim3(nblk(nv, 4)), dim3(256), 0, s, nv, Bd, ld, S.minv,
                           S.ring_ptr, S.ring, S.spai, p.d_bad);
        if (T.max_ring > SPAI_SMALL)
            hipLaunchKernelGGL(k_spai<double>, dim3(unsigned(nv)), dim3(256), 0, s, nv, Bd, ld, S.minv, S.ring_ptr,
                               S.ring, S.spai, p.d_bad);
    }
    PB_HIP(hipGetLastError());
    int bad = 0;
    PB_HIP(hipMemcpyAsync(&bad, p.d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    PB_CHECK(!(bad & 4), PBFB_EMESH, "single-layer block not positive definite on a vertex 1-ring");
    p.bem_ready[w] = true;
}

void ensure_all(Problem &p, hipStream_t s)
{
    ensure_geometry(p, s);
    ensure_values(p, s);
    ensure_rhs(p, s);
    ensure_bem(p, 0, s);
    ensure_bem(p, 1, s);
    if (p.gm() == 2) ensure_bem(p, 2, s); // lambda_m and u_r on the independent Gamma_m mesh
}

} // namespace pbfb
