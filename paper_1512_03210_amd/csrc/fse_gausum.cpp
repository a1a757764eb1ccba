// Host FP64 construction of the GauSum multiplier (Section 2 of the paper).
//
// Khat(kappa) = sum_q w_q prod_j G(tau_q, kappa_j, D_j) + C0 - C2 |kappa|^2
//   * (w_q, tau_q): trapezoidal (sinc) quadrature of the integral
//     representation r^{-mu} = (2/Gamma(mu/2)) int exp(-r^2 e^{2t} + mu t) dt
//     (the Gaussian sum of eq. GS-Gene), step ht, nodes from
//     t_lo = ln(1e-17)/mu - ln(2 sqrt(d) L) - 1 to t_hi = ln(9/delta), so the
//     sum is accurate on [delta, 2 sqrt(d) L];
//   * G(tau, kappa, D) = 2 int_0^D exp(-tau^2 y^2) cos(kappa y) dy, the 1D
//     factors of the separable tensor (eq. tensor) on the kernel box
//     [-2L, 2L] (D = 2L, padding factor 2);
//   * C0, C2: the near-field correction of eq. taylor, integrating
//     U - U_GS over the ball |y| < delta against the constant and the
//     Laplacian terms of the Taylor polynomial;
//   * the 3D dipole multiplier -1 + 3 (n.kappa)^2 Khat_C, Khat_C for the
//     kernel 1/(4 pi |x|), and the 2D dipole multiplier
//     (3/2)[(n_perp.kappa)^2 - n3^2 |kappa|^2] Khat_C, Khat_C for
//     1/(2 pi |x|) (both eq. Kernel); n has at most one nonzero component
//     among those that multiply a frequency, so (n.kappa)^2 = sum n_j^2 kappa_j^2.
// kappa_j = pi k / D_j for k = 0..N_j: the non-negative frequencies of the
// 2N_j-point padded grid; Khat is even in every kappa_j.
//
// How the 1D integrals are evaluated here: where tau*D >= 6.5 the Gaussian
// has decayed inside the box (tail below 1e-19 relative) and G is the
// full-line transform sqrt(pi)/tau exp(-kappa^2/(4 tau^2)); below, composite
// Gauss-Legendre on [0, D] with one panel per half period of the highest
// frequency, evaluated for all (tau, kappa) pairs as one matrix product.
#include <algorithm>
#include <cmath>
#include <thread>
#include <vector>

#include "fse_host.hpp"

namespace fse {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;


// Series for the lower incomplete gamma function scaled as
// gamma(a, x) / x^a = e^{-x} sum_k x^k / (a (a+1) ... (a+k)).
double lower_gamma_over_xa(double a, double x) {
    double term = 1.0 / a, sum = term;
    for (int k = 1; k < 2000; ++k) {
        term *= x / (a + k);
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return std::exp(-x) * sum;
}

// Integral of exp(-tau^2 |y|^2) |y|^{2a-d} over the ball |y| < delta in R^d:
// S_d gamma(a, tau^2 delta^2) / (2 tau^{2a}).
double ball_gauss(int d, double a, double tau, double delta) {
    const double Sd = (d == 2) ? 2.0 * kPi : 4.0 * kPi;
    const double x = tau * tau * delta * delta;
    if (x > 700.0) return Sd * std::tgamma(a) / (2.0 * std::pow(tau, 2.0 * a));
    return Sd * std::pow(delta, 2.0 * a) * lower_gamma_over_xa(a, x) / 2.0;
}

template <typename F> void parallel_for(int n, F f) {
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 2 || nt == 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t)
        th.emplace_back([&, t]() {
            for (int i = (int)t; i < n; i += (int)nt) f(i);
        });
    for (auto& x : th) x.join();
}

}  // namespace

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            // p1 = P_n(z), p0 = P_{n-1}(z)
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

void sinc_gaussian_sum(double mu, double c, int d, double Lmax, double delta, double ht, std::vector<double>& w,
                       std::vector<double>& tau) {
    const double t_lo = std::log(1e-17) / mu - std::log(2.0 * std::sqrt((double)d) * Lmax) - 1.0;
    const double t_hi = std::log(9.0 / delta);
    const int Q = (int)std::ceil((t_hi - t_lo) / ht);
    w.resize(Q + 1);
    tau.resize(Q + 1);
    const double g = std::tgamma(mu / 2.0);
    for (int q = 0; q <= Q; ++q) {
        const double t = t_lo + ht * q;
        tau[q] = std::exp(t);
        w[q] = c * 2.0 * ht * std::exp(mu * t) / g;
    }
}

// G[q*K + k] for kappa_k = pi k / D, k < K.
void gauss_factor_table(const std::vector<double>& tau, double D, int K, std::vector<double>& G) {
    const int Q = (int)tau.size();
    G.assign((size_t)Q * K, 0.0);
    std::vector<int> small;
    for (int q = 0; q < Q; ++q) {
        if (tau[q] * D >= 6.5) {
            const double pre = std::sqrt(kPi) / tau[q];
            for (int k = 0; k < K; ++k) {
                const double kap = kPi * k / D;
                const double a = kap / (2.0 * tau[q]);
                G[(size_t)q * K + k] = pre * std::exp(-a * a);
            }
        } else {
            small.push_back(q);
        }
    }
    if (small.empty()) return;
    const int npan = std::max(8, K + 2);
    const int ng = 12;
    std::vector<double> gx, gw;
    gauss_legendre(ng, gx, gw);
    const int nn = npan * ng;
    std::vector<double> y(nn), wy(nn);
    for (int p = 0; p < npan; ++p) {
        const double a = D * p / npan, b = D * (p + 1) / npan;
        for (int i = 0; i < ng; ++i) {
            y[p * ng + i] = a + 0.5 * (b - a) * (gx[i] + 1.0);
            wy[p * ng + i] = 0.5 * (b - a) * gw[i];
        }
    }
    // cosm[k][n] = 2 w_n cos(kappa_k y_n)
    std::vector<double> cosm((size_t)K * nn);
    parallel_for(K, [&](int k) {
        const double kap = kPi * k / D;
        for (int n = 0; n < nn; ++n) cosm[(size_t)k * nn + n] = 2.0 * wy[n] * std::cos(kap * y[n]);
    });
    parallel_for((int)small.size(), [&](int si) {
        const int q = small[si];
        std::vector<double> g(nn);
        for (int n = 0; n < nn; ++n) {
            const double a = tau[q] * y[n];
            g[n] = std::exp(-a * a);
        }
        for (int k = 0; k < K; ++k) {
            const double* c = &cosm[(size_t)k * nn];
            double s = 0.0;
            for (int n = 0; n < nn; ++n) s += c[n] * g[n];
            G[(size_t)q * K + k] = s;
        }
    });
}

void near_field(int d, double mu, double c, double delta, const std::vector<double>& w, const std::vector<double>& tau,
                double& C0, double& C2) {
    const double Sd = (d == 2) ? 2.0 * kPi : 4.0 * kPi;
    double s0 = 0.0, s2 = 0.0;
    for (size_t q = 0; q < tau.size(); ++q) {
        s0 += w[q] * ball_gauss(d, d / 2.0, tau[q], delta);
        s2 += w[q] * ball_gauss(d, d / 2.0 + 1.0, tau[q], delta);
    }
    C0 = c * Sd * std::pow(delta, d - mu) / (d - mu) - s0;
    C2 = (c * Sd * std::pow(delta, d + 2 - mu) / (d + 2 - mu) - s2) / (2.0 * d);
}

std::vector<double> gausum_symbol(int d, const int* N, const double* L, int kind, double mu, double c, double delta,
                                  double ht, const double* n) {
    double Lmax = 0.0;
    for (int j = 0; j < d; ++j) Lmax = std::max(Lmax, L[j]);
    if (delta <= 0.0) delta = 1e-4 * Lmax;
    if (ht <= 0.0) ht = 0.14;
    // dipoles: Coulomb part 1/(4 pi |x|) in 3D, 1/(2 pi |x|) in 2D
    if (kind == 2 || kind == 3) {
        mu = 1.0;
        c = (kind == 2) ? 1.0 / (4.0 * kPi) : 1.0 / (2.0 * kPi);
    }
    // derivative factor sum_j a_j kappa_j^2 applied to Khat_C
    double a[3] = {0.0, 0.0, 0.0};
    if (kind == 2) {
        for (int j = 0; j < 3; ++j) a[j] = 3.0 * n[j] * n[j];
    } else if (kind == 3) {
        a[0] = 1.5 * (n[0] * n[0] - n[2] * n[2]);
        a[1] = 1.5 * (n[1] * n[1] - n[2] * n[2]);
    }
    std::vector<double> w, tau;
    sinc_gaussian_sum(mu, c, d, Lmax, delta, ht, w, tau);
    const int Q = (int)tau.size();
    int K[3] = {1, 1, 1};
    double D[3] = {1.0, 1.0, 1.0};
    std::vector<double> G[3];
    for (int j = 0; j < d; ++j) {
        K[j] = N[j] + 1;
        D[j] = 2.0 * L[j];
        bool reused = false;
        for (int i = 0; i < j; ++i) {
            if (K[i] == K[j] && D[i] == D[j]) {
                G[j] = G[i];
                reused = true;
                break;
            }
        }
        if (!reused) gauss_factor_table(tau, D[j], K[j], G[j]);
    }
    double C0, C2;
    near_field(d, mu, c, delta, w, tau, C0, C2);
    const int K0 = K[0], K1 = K[1], K2 = (d == 3) ? K[2] : 1;
    std::vector<double> out((size_t)K0 * K1 * K2);
    parallel_for(K0, [&](int k0) {
        std::vector<double> wg(Q), row(K2);
        const double kap0 = kPi * k0 / D[0];
        for (int k1 = 0; k1 < K1; ++k1) {
            for (int q = 0; q < Q; ++q) wg[q] = w[q] * G[0][(size_t)q * K0 + k0] * G[1][(size_t)q * K1 + k1];
            const double kap1 = kPi * k1 / D[1];
            if (d == 2) {
                double s = 0.0;
                for (int q = 0; q < Q; ++q) s += wg[q];
                const double kc = s + C0 - C2 * (kap0 * kap0 + kap1 * kap1);
                out[(size_t)k0 * K1 + k1] = (kind == 3) ? (a[0] * kap0 * kap0 + a[1] * kap1 * kap1) * kc : kc;
                continue;
            }
            std::fill(row.begin(), row.end(), 0.0);
            for (int q = 0; q < Q; ++q) {
                const double aq = wg[q];
                const double* g2 = &G[2][(size_t)q * K2];
                for (int k2 = 0; k2 < K2; ++k2) row[k2] += aq * g2[k2];
            }
            double* o = &out[((size_t)k0 * K1 + k1) * K2];
            for (int k2 = 0; k2 < K2; ++k2) {
                const double kap2 = kPi * k2 / D[2];
                const double kc = row[k2] + C0 - C2 * (kap0 * kap0 + kap1 * kap1 + kap2 * kap2);
                o[k2] = (kind == 2) ? -1.0 + (a[0] * kap0 * kap0 + a[1] * kap1 * kap1 + a[2] * kap2 * kap2) * kc : kc;
            }
        }
    });
    return out;
}

}  // namespace fse
