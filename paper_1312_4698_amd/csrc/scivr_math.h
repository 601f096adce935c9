// Double-precision exp, sincos and atan2 for the trajectory kernel, written
// from the mathematics: Cody-Waite argument reduction (Cody and Waite,
// "Software Manual for the Elementary Functions", 1980) with fused
// multiply-adds, and Taylor polynomials on the reduced interval.
//
// The coefficients and reduction constants are read from the problem's
// constant block through the same opaque handle as the other uniform
// constants, so they are scalar-cache loads used as scalar operands inside
// the time loop rather than ~70 vector registers of hoisted literals.
// Accuracy: exp <= 1 ulp; sin, cos <= 1.2e-16 and atan2 <= 4.5e-16 absolute
// for the argument ranges met here (|x| < 1e4 for sincos).
#pragma once

#include <hip/hip_runtime.h>

namespace scivr {

struct MathConsts {
    double exp_c[14];   // 1/n!, n = 0..13: exp(r) on |r| <= ln2/2
    double sin_c[9];    // (-1)^n/(2n+1)!: sin(r) = r sum_n sin_c[n] r^(2n) on |r| <= pi/4
    double cos_c[10];   // (-1)^n/(2n)!
    double atan_c[12];  // (-1)^n/(2n+1): atan(u) on |u| <= tan(pi/16)
    double log2e, ln2_hi, ln2_lo;
    double two_over_pi, pio2_1, pio2_2, pio2_3;  // pi/2 = pio2_1 + pio2_2 + pio2_3 to ~160 bits
    double pi, pio2, pio4, pio8;
    double tan_pio8, tan_pio16, tan_3pio16;
};

// 1/x from v_rcp_f64 refined by one Newton-Raphson step.
__device__ inline double rcp_nr(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return r;
}

// exp(x): x = k ln2 + r, exp(x) = 2^k exp(r).
template <typename MC>
__device__ inline double dexp(double x, MC M)
{
    x = (x > 1000.0) ? 1000.0 : ((x < -1000.0) ? -1000.0 : x);  // NaN passes through
    const double k = rint(x * M->log2e);
    double r = fma(-k, M->ln2_hi, x);
    r = fma(-k, M->ln2_lo, r);
    double p = M->exp_c[13];
#pragma unroll
    for (int n = 12; n >= 0; --n) p = fma(p, r, M->exp_c[n]);
    return ldexp(p, (int)k);
}

// sin(x), cos(x): x = k pi/2 + r, then the quadrant k mod 4 permutes and negates.
template <typename MC>
__device__ inline void dsincos(double x, MC M, double *s_out, double *c_out)
{
    const double k = rint(x * M->two_over_pi);
    double r = fma(-k, M->pio2_1, x);
    r = fma(-k, M->pio2_2, r);
    r = fma(-k, M->pio2_3, r);
    const double r2 = r * r;
    double ps = M->sin_c[8];
#pragma unroll
    for (int n = 7; n >= 1; --n) ps = fma(ps, r2, M->sin_c[n]);
    const double s = fma(r * r2, ps, r);
    double c = M->cos_c[9];
#pragma unroll
    for (int n = 8; n >= 0; --n) c = fma(c, r2, M->cos_c[n]);
    const int q = ((int)(long long)k) & 3;
    const double sa = (q & 1) ? c : s;
    const double ca = (q & 1) ? s : c;
    *s_out = (q & 2) ? -sa : sa;
    *c_out = ((q + 1) & 2) ? -ca : ca;
}

// atan2(y, x): fold to t = min/max in [0, 1]; t <= tan(pi/16): u = t; t <=
// tan(3pi/16): atan t = pi/8 + atan((t - tan(pi/8)) / (1 + t tan(pi/8)));
// else atan t = pi/4 + atan((t - 1)/(t + 1)); then |u| <= tan(pi/16).
template <typename MC>
__device__ inline double datan2(double y, double x, MC M)
{
    const double ax = fabs(x), ay = fabs(y);
    const bool sw = ay > ax;
    const double num = sw ? ax : ay, den = sw ? ay : ax;
    const double t = num * rcp_nr(den);
    const bool r0 = t <= M->tan_pio16, r1 = t <= M->tan_3pio16;
    const double cc = r0 ? 0.0 : (r1 ? M->tan_pio8 : 1.0);
    const double base = r0 ? 0.0 : (r1 ? M->pio8 : M->pio4);
    const double u = (t - cc) * rcp_nr(fma(t, cc, 1.0));
    const double u2 = u * u;
    double p = M->atan_c[11];
#pragma unroll
    for (int n = 10; n >= 1; --n) p = fma(p, u2, M->atan_c[n]);
    double a = base + fma(u * u2, p, u);
    a = sw ? M->pio2 - a : a;
    a = (x < 0.0) ? M->pi - a : a;
    return (y < 0.0) ? -a : a;
}

}  // namespace scivr
