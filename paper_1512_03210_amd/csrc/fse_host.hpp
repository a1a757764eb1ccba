// Host-side internals: GauSum precompute (fse_gausum.cpp).
#pragma once
#include <vector>

namespace fse {

// Weights and exponents of the sinc-quadrature Gaussian sum for c/r^mu.
void sinc_gaussian_sum(double mu, double c, int d, double Lmax, double delta, double ht, std::vector<double>& w,
                       std::vector<double>& tau);

// G[q*K + k] = 2 int_0^D exp(-tau_q^2 y^2) cos(pi k y / D) dy, k < K.
void gauss_factor_table(const std::vector<double>& tau, double D, int K, std::vector<double>& G);

// Near-field constants C0, C2 (multiplier C0 - C2 |kappa|^2).
void near_field(int d, double mu, double c, double delta, const std::vector<double>& w, const std::vector<double>& tau,
                double& C0, double& C2);

// Gauss-Legendre nodes and weights on [-1, 1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Multiplier on the non-negative octant, (N_j + 1) values per axis, row-major.
// kind: 1 Coulomb c/|x|^mu, 2 3D dipole, 3 2D dipole, along the unit axis n
// (kinds 2 and 3; the multiplier must be even in every frequency, so n has no
// two nonzero components among those that enter it).  delta, ht <= 0 select
// defaults.
std::vector<double> gausum_symbol(int d, const int* N, const double* L, int kind, double mu, double c, double delta,
                                  double ht, const double* n);

}  // namespace fse
