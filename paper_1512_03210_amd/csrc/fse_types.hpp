// Plain argument structs shared by the kernels and the host plan.
#pragma once

namespace fse {

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
};

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
};

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
};

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
    double bdt, ldt;     // beta dt, lambda dt
    double x0, hx, y0, hy;
};

}  // namespace fse
