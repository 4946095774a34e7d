// Quadrature pieces shared by the regular boundary-element kernels (dense
// assembly and the matrix-free apply): the 6-point triangle rule in the form
// the kernels use, and the positive reciprocal square root.
#pragma once

#include <hip/hip_runtime.h>

#include "pbfb_internal.hpp"

namespace pbfb {

constexpr double INV4PI = 0.079577471545947667884441881686257181;

// The 6-point rule is two orbits of 3 points: point k of orbit o has
// barycentric coordinate beta_o at index k and alpha_o at the other two.  A
// sum s_j = sum_q w_q b_q[j] g_q is then A_0 G_0 + A_1 G_1 + D_0 g_{0,j} +
// D_1 g_{1,j} with G_o the orbit's sum of g, A_o = w_o alpha_o and D_o =
// w_o (beta_o - alpha_o) (12 operations for the three j instead of 18).
struct QRule6 {
    double b[6][3];
    double w[6];
    double oA[2], oD[2];
    double wb[6][3]; // w_q b_q[a]
};
inline QRule6 q6arg()
{
    QRule6 r;
    const Rules &R = rules();
    for (int q = 0; q < 6; ++q) {
        for (int k = 0; k < 3; ++k) r.b[q][k] = R.tri_bary[q][k];
        r.w[q] = R.tri_w[q];
        for (int k = 0; k < 3; ++k) r.wb[q][k] = R.tri_w[q] * R.tri_bary[q][k];
    }
    for (int o = 0; o < 2; ++o) {
        // the orbit structure the regular kernel relies on
        const double al = R.tri_bary[3 * o][1], be = R.tri_bary[3 * o][0];
        for (int k = 0; k < 3; ++k)
            for (int j = 0; j < 3; ++j)
                PB_CHECK(R.tri_bary[3 * o + k][j] == (j == k ? be : al) && R.tri_w[3 * o + k] == R.tri_w[3 * o],
                         PBFB_EDEVICE, "triangle rule is not two 3-point orbits");
        r.oA[o] = R.tri_w[3 * o] * al;
        r.oD[o] = R.tri_w[3 * o] * (be - al);
    }
    return r;
}
// the orbit factors of the 6-point rule and the products w_q b_q[a] in FP32
struct QRule6F {
    float oA[2], oD[2];
    float wb[6][3];
};
inline QRule6F q6farg()
{
    const QRule6 R = q6arg();
    QRule6F r;
    for (int o = 0; o < 2; ++o) {
        r.oA[o] = float(R.oA[o]);
        r.oD[o] = float(R.oD[o]);
    }
    for (int q = 0; q < 6; ++q)
        for (int a = 0; a < 3; ++a) r.wb[q][a] = float(R.wb[q][a]);
    return r;
}

// 1/sqrt(x) for finite x > 0 (quadrature points of non-touching panels are
// never coincident): the hardware estimate refined by one third-order step
// y (1 + e/2 + 3e^2/8), e = 1 - x y^2.
__device__ inline double rsqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ inline float rsqrt_pos(float x) { return __builtin_amdgcn_rsqf(x); }

// e^{-a} for finite a >= 0 (the FP64 Yukawa kernel): -a = k ln 2 + f with
// |f| <= ln(2)/2 (Cody-Waite reduction: ln 2 split into a head of 21
// significant bits, so that k times it is exact, and a tail), e^f by its
// Taylor polynomial of degree 13 in Horner form (truncation below 5e-18
// relative), scaled by 2^k.  a is clamped at 800, where e^{-a} has
// underflowed to 0, which keeps k within int range.
__device__ inline double exp_neg(double a)
{
    a = fmin(a, 800.0);
    const double k = rint(a * -1.4426950408889634);
    const double f = fma(-k, 4.7493250390316726e-07, fma(-k, 0.6931467056274414, -a));
    double p = 1.0 / 6227020800.0;
    p = fma(p, f, 1.0 / 479001600.0);
    p = fma(p, f, 1.0 / 39916800.0);
    p = fma(p, f, 1.0 / 3628800.0);
    p = fma(p, f, 1.0 / 362880.0);
    p = fma(p, f, 1.0 / 40320.0);
    p = fma(p, f, 1.0 / 5040.0);
    p = fma(p, f, 1.0 / 720.0);
    p = fma(p, f, 1.0 / 120.0);
    p = fma(p, f, 1.0 / 24.0);
    p = fma(p, f, 1.0 / 6.0);
    p = fma(p, f, 0.5);
    p = fma(p, f, 1.0);
    p = fma(p, f, 1.0);
    return ldexp(p, int(k));
}

} // namespace pbfb
