// Plain argument structs shared by the kernels and the host plan.
#pragma once

namespace fse {

// Row of the multiplier table for a contiguous line: i0 = line / D1,
// i1 = line % D1, each folded to min(i, F - i) when F > 0,
// row = (k0 * T1 + k1) * T2.
struct LineIdx {
    int D1, F0, F1, T1, T2;
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
};

// Grid geometry for the elementwise kernels and reductions.
struct GridGeom {
    int d, N0, N1, N2;
    double x0, hx, y0, hy, z0, hz;
};

}  // namespace fse
