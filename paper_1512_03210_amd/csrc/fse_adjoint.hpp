// Pointwise kernels of the adjoint (reverse-mode derivative) of the split
// step.  The paper gives no adjoint; these are the pieces of the hand-derived
// reverse of one TS2-GauSum step (eqs. tssp1-tssp3):
//   forward   psi1 = K psi,  theta = dt beta |psi1|^2 + lam dt Phi[|psi1|^2]
//                                   + P(x~; t, t+dt) + dt U,
//             psi2 = psi1 exp(-i theta),  psi' = K psi2;
//   reverse   g2 = K^H g',  q = Im(conj(g2) psi2),
//             g1 = g2 exp(+i theta) + 2 (dt beta q + lam dt Phi[q]) psi1,
//             g = K^H g1,  dL/dU += dt q,
// with g = dL/dRe(psi) + i dL/dIm(psi) for a real loss L.  K and K^H are the
// kinetic passes with +tau and -tau; Phi is the GauSum convolution, which is
// self-adjoint (real, even multiplier).  Pointwise work is done in FP64 (the
// library's own sine/cosine, fsincos) and stored in the plan's precision.
#pragma once
#include "fse_kernels.hpp"

namespace fse {

namespace adj {
template <typename T> __device__ __forceinline__ double2 up(T v) { return double2{(double)v.x, (double)v.y}; }
}  // namespace adj

// theta and, when psi2 is not null, psi2 = psi1 exp(-i theta).  P is the trap
// integral of the phase arguments (the same quadratic form as the fused
// nonlinear pass).
template <typename R>
__global__ void k_adj_theta(const typename CT<R>::T* __restrict__ psi1, const R* __restrict__ Phi,
                            const R* __restrict__ U, R* __restrict__ theta, typename CT<R>::T* __restrict__ psi2,
                            long n, GridGeom g, PhaseArgs pa) {
    double pcc, pcs;
    phase_time(pa, &pcc, &pcs);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const double P = pa.cz * z * z + (pa.ca - pcc) * y * y + (pa.ca + pcc) * x * x + pcs * 2.0 * x * y;
        const double2 v = adj::up(psi1[i]);
        double th = pa.bdt * (v.x * v.x + v.y * v.y) + P;
        if (Phi) th += pa.ldt * (double)Phi[i];
        if (U) th += pa.udt * (double)U[i];
        theta[i] = R(th);
        if (psi2) {
            double sn, cs;
            fsincos(th, &sn, &cs);
            psi2[i] = typename CT<R>::T{R(v.x * cs + v.y * sn), R(v.y * cs - v.x * sn)};
        }
    }
}

// q = Im(conj(g2) psi2) with psi2 = psi1 exp(-i theta); gU += udt q when gU is not null.
template <typename R>
__global__ void k_adj_q(const typename CT<R>::T* __restrict__ g2, const typename CT<R>::T* __restrict__ psi1,
                        const R* __restrict__ theta, R* __restrict__ q, R* __restrict__ gU, long n, double udt) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double2 v = adj::up(psi1[i]), a = adj::up(g2[i]);
        double sn, cs;
        fsincos((double)theta[i], &sn, &cs);
        const double px = v.x * cs + v.y * sn, py = v.y * cs - v.x * sn;  // psi2
        const double qi = a.x * py - a.y * px;                          // Im(conj(a) psi2)
        q[i] = R(qi);
        if (gU) gU[i] = R((double)gU[i] + udt * qi);
    }
}

// g <- g exp(+i theta) + 2 (bdt q + ldt Phiq) psi1 (Phiq may be null).
template <typename R>
__global__ void k_adj_g1(typename CT<R>::T* __restrict__ g, const typename CT<R>::T* __restrict__ psi1,
                         const R* __restrict__ theta, const R* __restrict__ q, const R* __restrict__ Phiq, long n,
                         double bdt, double ldt) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double2 v = adj::up(psi1[i]), a = adj::up(g[i]);
        double sn, cs;
        fsincos((double)theta[i], &sn, &cs);
        double r = bdt * (double)q[i];
        if (Phiq) r += ldt * (double)Phiq[i];
        g[i] = typename CT<R>::T{R(a.x * cs - a.y * sn + 2.0 * r * v.x), R(a.y * cs + a.x * sn + 2.0 * r * v.y)};
    }
}

}  // namespace fse
