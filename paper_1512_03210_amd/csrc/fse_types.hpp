// Plain argument structs shared by the kernels and the host plan, and the
// time-dependent coefficients that both evaluate.
//
// Time lives in device memory (one double per plan): a coefficient that
// depends on the time t of the state is evaluated on the device from
// *tp + toff, where toff is the offset of the sub-step inside the call, so a
// launch recorded into a graph replays at the time the plan has then.  Where
// a coefficient does not depend on t (no rotation, or an isotropic trap), the
// host evaluates it once and tp is null.
#pragma once
#include <hip/hip_runtime.h>

#include "fse_math.hpp"

namespace fse {

// The rotating part of the trap integral P(x~; t, t+tau) (eq. int_poten) for
// the harmonic trap: with gd = (gx^2 - gy^2)/4,
//   cc = gd int_t^{t+tau} cos(2 Omega s) ds,  cs = gd int_t^{t+tau} sin(2 Omega s) ds,
// in the closed form cos/sin(Omega (2t + tau)) sin(Omega tau)/Omega (tau gd
// and 0 without rotation).
__host__ __device__ inline void trap_rotating(double t, double tau, double Om, double gd, double* cc, double* cs) {
    if (Om == 0.0) {
        *cc = gd * tau;
        *cs = 0.0;
        return;
    }
    const double f = sin(Om * tau) / Om;
    *cc = gd * (cos(Om * (2.0 * t + tau)) * f);
    *cs = gd * (sin(Om * (2.0 * t + tau)) * f);
}

// The same on the device with the time-independent factor sf = sin(Om tau)/Om
// (tau without rotation) taken from the host: one sine/cosine pair per thread.
__device__ inline void trap_rotating_dev(double t, double tau, double Om, double gd, double sf, double* cc,
                                         double* cs) {
    double s, c;
    fsincos(Om * (2.0 * t + tau), &s, &c);
    *cc = gd * (c * sf);
    *cs = gd * (s * sf);
}

// Row of the multiplier table for a contiguous line: i0 = line / D1,
// i1 = line % D1, each folded to min(i, F - i) when F > 0,
// row = (k0 * T1 + k1) * T2.
// X0, X1 (0 or 1): visit the lines in mirror order along axis 0 / 1 (F0 / F1
// even and > 0), so that the lines i and F - i that share a row are handled
// by the same block and the row is read once.  With both set, D1 == F1 and
// consecutive groups of four lines are {i0, F0 - i0} x {i1, F1 - i1}.
struct LineIdx {
    int D1, F0, F1, T1, T2;
    int X0 = 0, X1 = 0;
};

// Grid and coefficients of the fused nonlinear sub-step.
struct PhaseArgs {
    double x0, hx, y0, hy, z0, hz;  // grid origin and spacing per axis
    int N2;                          // 3D: length of axis 2 (columns = N1*N2); 2D: 0
    double ca;                       // coefficient of (x~^2 + y~^2) in P
    double cz;                       // coefficient of z~^2
    double cc;                       // coefficient of (x~^2 - y~^2)
    double cs;                       // coefficient of 2 x~ y~
    double bdt;                      // beta * dt
    double ldt;                      // lambda * dt
    const void* U;                   // optional real potential on the grid (plan precision) or null
    double udt;                      // dt, the factor of U in the phase
    // time-dependent cc, cs: with tp set they are trap_rotating(*tp + toff, tau, Om, gd);
    // sf = sin(Om tau)/Om
    const double* tp = nullptr;
    double toff = 0.0, tau = 0.0, Om = 0.0, gd = 0.0, sf = 0.0;
};

// cc, cs of the phase arguments at the device time (or as given when tp is null).
__device__ inline void phase_time(const PhaseArgs& pa, double* cc, double* cs) {
    if (pa.tp) {
        trap_rotating_dev(*pa.tp + pa.toff, pa.tau, pa.Om, pa.gd, pa.sf, cc, cs);
    } else {
        *cc = pa.cc;
        *cs = pa.cs;
    }
}

// Dipolar multiplier as a quadratic form (an axis with products n_i n_j, or
// one that turns in the rotating frame):
//   K(kappa) = c0 + Kc(kappa) * sum_ij m_ij kappa_i kappa_j,
// Kc the Coulomb-part symbol held in the multiplier table (which carries the
// FFT scale; c0 carries it too).  kappa_j = k_j dk_j with signed indices;
// index 0 is the row's axis-0 frequency (0..n0), index 1 the row's axis-1
// frequency (3D, padded length 2 n1), index 2 the line's frequency.  The odd
// products (i != j) take kappa = 0 at Nyquist indices (k0 = n0, k1 = n1, and
// the middle of the line), which keeps K even on the grid.
struct QForm {
    double c0, m00, m11, m22, m01, m02, m12;
    double dk0, dk1, dk2;
    int n0, n1;
    // the axis, from which the m_ij follow (qform_fill): n = (r cos phi0, r sin phi0, n2);
    // d3: the 3D multiplier -1 + 3 Kc kappa^T M kappa (c0 = -kscale), else the 2D one
    double r = 0.0, phi0 = 0.0, n2 = 0.0, Om = 0.0, kscale = 0.0;
    int d3 = 0;
    // with tp set, the m_ij are the average over [t, t+tau], t = *tp + toff, taken on the device
    const double* tp = nullptr;
    double toff = 0.0, tau = 0.0;
};

// The dipolar quadratic form over [t, t+tau] (tau = 0: at the instant t) in
// the rotating Lagrangian coordinates: the axis m(s) = A(s)^{-1} n is n_perp
// turned by +Omega s, and the time average of m m^T has, for each harmonic
// cos/sin(a + b s), its midpoint value times sinc(b tau / 2) (eq. Kernel_Rot).
__host__ __device__ inline void qform_fill(QForm& q, double t, double tau) {
    const double r = q.r, W = q.Om;
    const double a1 = q.phi0 + W * (t + 0.5 * tau), x1 = 0.5 * W * tau, x2 = W * tau;
    const double s1 = (x1 == 0.0) ? 1.0 : sin(x1) / x1, s2 = (x2 == 0.0) ? 1.0 : sin(x2) / x2;
    const double mc1 = cos(a1) * s1, ms1 = sin(a1) * s1, mc2 = cos(2.0 * a1) * s2, ms2 = sin(2.0 * a1) * s2;
    const double M00 = r * r * (0.5 + 0.5 * mc2), M11 = r * r * (0.5 - 0.5 * mc2);
    const double M01 = r * r * 0.5 * ms2, M02 = q.n2 * r * mc1, M12 = q.n2 * r * ms1;
    const double M22 = q.n2 * q.n2;
    if (q.d3) {
        // -1 + 3 Khat_C kappa^T M kappa; the line axis is axis 2
        q.c0 = -q.kscale;
        q.m00 = 3.0 * M00;
        q.m11 = 3.0 * M11;
        q.m22 = 3.0 * M22;
        q.m01 = 3.0 * M01;
        q.m02 = 3.0 * M02;
        q.m12 = 3.0 * M12;
    } else {
        // (3/2) Khat_C (kappa^T M_perp kappa - M22 |kappa|^2); the line axis is axis 1
        q.c0 = 0.0;
        q.m00 = 1.5 * (M00 - M22);
        q.m11 = 0.0;
        q.m22 = 1.5 * (M11 - M22);
        q.m01 = 0.0;
        q.m02 = 1.5 * M01;
        q.m12 = 0.0;
    }
}

// Optical lattice V_L = sum_j v_j sin^2(k_j x_j), defined in the frame of
// eq. SFSE, evaluated along the rotating frame: out = sum_q w_q V_L(A_q x~)
// + uf U, A_q turning (x, y) by the angle with cosine c[q] and sine s[q] (z is
// not turned).  One node with w = 1 gives V_L at one instant; Gauss-Legendre
// nodes over [t, t+tau] (weights times tau/2) give its time integral.
struct LatArgs {
    double v[3], k[3];
    double c[8], s[8], w[8];
    int nq;
    double uf;
    // with tp set, c, s and w follow on the device from the nodes (lat_fill)
    const double* tp = nullptr;
    double toff = 0.0, tau = 0.0, Om = 0.0;
    double gx[8], gw[8];  // Gauss-Legendre nodes and weights on [-1, 1] (nq of them; tau = 0: one node, w = 1)
};

// Quadrature nodes of the lattice over [t, t+tau]: frame angles Omega s_q,
// s_q = t + tau (x_q + 1)/2, weights tau w_q / 2 (tau = 0: the instant t).
__host__ __device__ inline void lat_fill(LatArgs& la, double t) {
    for (int q = 0; q < la.nq; ++q) {
        const double sq = (la.tau == 0.0) ? t : t + 0.5 * la.tau * (la.gx[q] + 1.0);
        la.c[q] = cos(la.Om * sq);
        la.s[q] = sin(la.Om * sq);
        la.w[q] = (la.tau == 0.0) ? 1.0 : 0.5 * la.tau * la.gw[q];
    }
}

// Grid geometry for the elementwise kernels and reductions.
struct GridGeom {
    int d, N0, N1, N2;
    double x0, hx, y0, hy, z0, hz;
};

// One instance of a batched 2D sweep (device memory).  The state lives at
// psi_base + psi_off (elements) of the packed buffer passed to each launch;
// *t is the instance's time at the start of the call.
struct BInst {
    long psi_off;
    void* X1;            // axis-0 real-to-complex workspace, (N0+1) x N1
    const void* khat;    // GauSum multiplier (carries 1/(4 N0 N1)), or null
    const void* kin0;    // kinetic table for dt/2 (carries 1/(N0 N1))
    const void* kin1;    // kinetic table for dt
    double* t;
    double dt, Omega;
    double ca;           // dt (gx^2 + gy^2)/4
    double gdiff;        // (gx^2 - gy^2)/4
    double sf;           // sin(Omega dt)/Omega (dt without rotation)
    double bdt, ldt;     // beta dt, lambda dt
    double x0, hx, y0, hy;
    double* rn;          // FP64 mass renormalisation {mass at the call's start, factor, mass before the exit pass}
};

}  // namespace fse
