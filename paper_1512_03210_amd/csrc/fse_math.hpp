// Device sine and cosine (own implementations: no library call, no branch
// for huge arguments), used by the phase factors and the time-dependent
// coefficients.
#pragma once
#include <hip/hip_runtime.h>

namespace fse {

// ---------------------------------------------------------------------------
// Sine and cosine.
// FP64: Cody-Waite reduction x = k pi/2 + r with pi/2 split into three doubles
// (the first two with 33 significant bits, so k*P1 and k*P2 are exact for
// |k| < 2^20; beyond that the reduction error stays within a few ulp of x, the
// rounding the argument itself carries), then the Taylor series of sin and
// cos on |r| <= pi/4 to degree 19 and 20 (truncation below 1e-22) and the
// quadrant k mod 4.
// FP32: the same steps in single precision.  pi/2 = P1 + P2 + P3 (floats,
// exact to 1e-23); each FMA forms x - k*Pi exactly before its one rounding,
// so r is accurate to about an ulp while k*P3 stays far below it (|k| < 2^22;
// larger arguments carry 0.25 rad of rounding themselves).  Taylor series to
// degree 11 and 10 (truncation below 1.1e-10 on |r| <= pi/4, far under the
// float rounding).  Error at most 1.2 ulp of 1 (7e-8);
// the float rounding of 1/6 and 1/24 biases s^2 + c^2 by -1e-8 r^4 (below
// 4e-9, and 2e-11 for the phase angles of a time step, |r| < 0.2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fsincos(double x, double* s, double* c) {
    const double k = rint(x * 0.6366197723675814);  // 2/pi
    double r = fma(-k, 1.5707963267341256, x);
    r = fma(-k, 6.077100506303966e-11, r);
    r = fma(-k, 2.0222662487959506e-21, r);
    const double r2 = r * r;
    double ps = -8.22063524662433e-18;  // -1/19!
    ps = fma(ps, r2, 2.8114572543455206e-15);
    ps = fma(ps, r2, -7.647163731819816e-13);
    ps = fma(ps, r2, 1.6059043836821613e-10);
    ps = fma(ps, r2, -2.505210838544172e-08);
    ps = fma(ps, r2, 2.7557319223985893e-06);
    ps = fma(ps, r2, -0.0001984126984126984);
    ps = fma(ps, r2, 0.008333333333333333);
    ps = fma(ps, r2, -0.16666666666666666);
    const double sn = fma(r * r2, ps, r);
    double pc = 4.110317623312165e-19;  // 1/20!
    pc = fma(pc, r2, -1.5619206968586225e-16);
    pc = fma(pc, r2, 4.779477332387385e-14);
    pc = fma(pc, r2, -1.1470745597729725e-11);
    pc = fma(pc, r2, 2.08767569878681e-09);
    pc = fma(pc, r2, -2.755731922398589e-07);
    pc = fma(pc, r2, 2.48015873015873e-05);
    pc = fma(pc, r2, -0.001388888888888889);
    pc = fma(pc, r2, 0.041666666666666664);
    pc = fma(pc, r2, -0.5);
    const double cs = fma(r2, pc, 1.0);
    const int q = (int)(k - 4.0 * floor(0.25 * k));  // k mod 4, exact for any integral k
    *s = (q == 0) ? sn : (q == 1) ? cs : (q == 2) ? -sn : -cs;
    *c = (q == 0) ? cs : (q == 1) ? -sn : (q == 2) ? -cs : sn;
}

__device__ __forceinline__ void fsincos(float x, float* s, float* c) {
    const float k = rintf(x * 0.63661975f);  // 2/pi
    float r = fmaf(-k, 1.57079637f, x);
    r = fmaf(-k, -4.37113883e-08f, r);
    r = fmaf(-k, -1.71512451e-15f, r);
    const float r2 = r * r;
    float ps = -2.50521079e-08f;  // -1/11!
    ps = fmaf(ps, r2, 2.75573188e-06f);
    ps = fmaf(ps, r2, -1.98412701e-04f);
    ps = fmaf(ps, r2, 8.33333377e-03f);
    ps = fmaf(ps, r2, -1.66666672e-01f);
    const float sn = fmaf(r * r2, ps, r);
    float pc = 2.75573200e-07f;  // 1/10!
    pc = fmaf(pc, r2, -2.48015876e-05f);
    pc = fmaf(pc, r2, 1.38888892e-03f);
    pc = fmaf(pc, r2, -4.16666679e-02f);
    pc = fmaf(pc, r2, 0.5f);
    const float cs = fmaf(-r2, pc, 1.0f);
    const int q = ((int)k) & 3;  // k mod 4 (two's complement)
    *s = (q == 0) ? sn : (q == 1) ? cs : (q == 2) ? -sn : -cs;
    *c = (q == 0) ? cs : (q == 1) ? -sn : (q == 2) ? -cs : sn;
}

}  // namespace fse
