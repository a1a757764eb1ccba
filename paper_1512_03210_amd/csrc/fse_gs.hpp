// Kernels of the ground-state step: the semi-implicit backward-Euler
// discretisation of the gradient flow with discrete normalisation (Section
// 3.2, eqs. gf-eq2 to gffg33), solved through the first preconditioned system
// of eq. precond_type1,
//     (I + P_Delta A_TF) phi1 = P_Delta phi^n / dt,
//     P_Delta = [I/dt + (1/2)(-Lap+m^2)^s]^{-1},  A_TF = W^n - Omega Lz,
//     W^n = V + beta |phi^n|^2 + lam Phi^n   (frozen over the step),
// by BiCGStab.  Vectors are in the plan's precision; every scalar of the
// Krylov recurrence and every inner product is FP64.
#pragma once
#include "fse_kernels.hpp"

namespace fse {

namespace gsd {
template <typename T> __device__ __forceinline__ double2 up(T v) { return double2{(double)v.x, (double)v.y}; }
template <typename R> __device__ __forceinline__ typename CT<R>::T down(double2 v) {
    return typename CT<R>::T{R(v.x), R(v.y)};
}
__device__ __forceinline__ double2 cm(double2 a, double2 b) {
    return double2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
}  // namespace gsd

// W = V(x) + beta |psi|^2 + lam Phi (+ U, an optional potential on the grid),
// with the trap V unrotated (the frame in which the energy carries -Omega Lz).
template <typename R>
__global__ void k_gs_frozen(const typename CT<R>::T* __restrict__ psi, const R* __restrict__ Phi,
                            const R* __restrict__ U, R* __restrict__ W, long n, GridGeom g, double beta, double lam,
                            double g0, double g1, double g2) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const double2 v = gsd::up(psi[i]);
        const double V = 0.5 * (g0 * g0 * x * x + g1 * g1 * y * y + g2 * g2 * z * z);
        W[i] = R(V + beta * (v.x * v.x + v.y * v.y) + (Phi ? lam * (double)Phi[i] : 0.0) + (U ? (double)U[i] : 0.0));
    }
}

// The first and last passes of the preconditioned operator on the strided
// axis 0, with the pointwise work folded in (one HBM sweep each instead of two):
//   OP 1 (forward): A = FFT_0[W v + i Omega (x Dy - y Dx)] (Dx, Dy null when
//        Omega = 0; W v - Omega Lz v with Lz = -i (x D_y - y D_x)), the value
//        built in FP64 and rounded to the plan's precision;
//   OP 2 (inverse): out = v + IFFT_0[A], the sum in FP64 as k_gs_axpy forms it.
// Column tiles as in the plain column pass; C columns, x from the row index,
// y from the column (c / N2 in 3D, c in 2D).
template <typename R, int N, int OP>
__global__ __launch_bounds__((ColCfg<R, N>::NTH))
FSE_COL_OCC(R, N, ColCfg<R, N>::W * pitch_cols<N>(N) * csz<R>(), ColCfg<R, N>::NTH)
void k_gs_cols(
    const typename CT<R>::T* __restrict__ v, const typename CT<R>::T* __restrict__ Dx,
    const typename CT<R>::T* __restrict__ Dy, const R* __restrict__ W, const typename CT<R>::T* A,
    typename CT<R>::T* out, int C, GridGeom g, double Omega, const typename CT<R>::T* __restrict__ twN) {
    using T = typename CT<R>::T;
    using Cf = ColCfg<R, N>;
    constexpr int Wt = Cf::W, TPL = Cf::TPL;
    constexpr int P = pitch_cols<N>(N);
    using F = Fft<T, N, OP == 2, TPL, ColPlan<N>>;
    __shared__ T lds[Wt * P];
    const int l = threadIdx.x % Wt, jt = threadIdx.x / Wt;
    const int c = blockIdx.x * Wt + l;
    const bool lv = c < C;
    T* line = lds + l * P;
    typename F::In in;
    typename F::Out u;
    if constexpr (OP == 1) {
        const double y = g.y0 + ((g.d == 3) ? (c / g.N2) : c) * g.hy;
        for_pos<N, TPL, F::R0>(jt, [&](int b, int r, int e) {
            T a{0, 0};
            if (lv) {
                const long i = (long)e * C + c;
                const double2 vv = gsd::up(v[i]);
                const double w = (double)W[i];
                double2 o{w * vv.x, w * vv.y};
                if (Dx) {
                    const double x = g.x0 + e * g.hx;
                    const double2 dx = gsd::up(Dx[i]), dy = gsd::up(Dy[i]);
                    o.x -= Omega * (x * dy.y - y * dx.y);
                    o.y += Omega * (x * dy.x - y * dx.x);
                }
                a = gsd::down<R>(o);
            }
            in[b][r] = a;
        });
    } else {
        for_pos<N, TPL, F::R0>(jt, [&](int b, int r, int e) { in[b][r] = lv ? A[(long)e * C + c] : T{0, 0}; });
    }
    F::run(in, u, line, jt, twN);
    for_pos<N, TPL, F::RK>(jt, [&](int b, int r, int e) {
        if (!lv) return;
        const long i = (long)e * C + c;
        if constexpr (OP == 1) {
            out[i] = u[b][r];
        } else {
            const double2 a = gsd::up(v[i]), q = gsd::up(u[b][r]);
            out[i] = gsd::down<R>(double2{a.x + q.x, a.y + q.y});
        }
    });
}

// out = a + c b (c complex, FP64); out may be a.
template <typename R>
__global__ void k_gs_axpy(const typename CT<R>::T* a, const typename CT<R>::T* __restrict__ b,
                          typename CT<R>::T* out, long n, double cr, double ci) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double2 x = gsd::up(a[i]), y = gsd::cm(double2{cr, ci}, gsd::up(b[i]));
        out[i] = gsd::down<R>(double2{x.x + y.x, x.y + y.y});
    }
}

// x += alpha p + omega s;  r = s - omega t.
template <typename R>
__global__ void k_gs_update_xr(typename CT<R>::T* __restrict__ x, typename CT<R>::T* __restrict__ r,
                               const typename CT<R>::T* __restrict__ p, const typename CT<R>::T* __restrict__ s,
                               const typename CT<R>::T* __restrict__ t, long n, double ar, double ai, double wr,
                               double wi) {
    const double2 al{ar, ai}, om{wr, wi};
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double2 sv = gsd::up(s[i]);
        const double2 ap = gsd::cm(al, gsd::up(p[i])), os = gsd::cm(om, sv), ot = gsd::cm(om, gsd::up(t[i]));
        const double2 xv = gsd::up(x[i]);
        x[i] = gsd::down<R>(double2{xv.x + ap.x + os.x, xv.y + ap.y + os.y});
        r[i] = gsd::down<R>(double2{sv.x - ot.x, sv.y - ot.y});
    }
}

// p = r + beta (p - omega v).
template <typename R>
__global__ void k_gs_update_p(typename CT<R>::T* __restrict__ p, const typename CT<R>::T* __restrict__ r,
                              const typename CT<R>::T* __restrict__ v, long n, double br, double bi, double wr,
                              double wi) {
    const double2 be{br, bi}, om{wr, wi};
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const double2 ov = gsd::cm(om, gsd::up(v[i])), pv = gsd::up(p[i]);
        const double2 q = gsd::cm(be, double2{pv.x - ov.x, pv.y - ov.y});
        const double2 rv = gsd::up(r[i]);
        p[i] = gsd::down<R>(double2{rv.x + q.x, rv.y + q.y});
    }
}

// Inner products sum conj(a_k) b_k of up to three pairs, FP64 partial sums
// per block into slots 2k (real) and 2k+1 (imaginary).
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_gs_dots(const typename CT<R>::T* __restrict__ a0,
                                                         const typename CT<R>::T* __restrict__ b0,
                                                         const typename CT<R>::T* __restrict__ a1,
                                                         const typename CT<R>::T* __restrict__ b1,
                                                         const typename CT<R>::T* __restrict__ a2,
                                                         const typename CT<R>::T* __restrict__ b2, int npair, long n,
                                                         double* partials) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        const typename CT<R>::T* as[3] = {a0, a1, a2};
        const typename CT<R>::T* bs[3] = {b0, b1, b2};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k < npair) {
                const double2 a = gsd::up(as[k][i]), b = gsd::up(bs[k][i]);
                acc[2 * k] += a.x * b.x + a.y * b.y;
                acc[2 * k + 1] += a.x * b.y - a.y * b.x;
            }
        }
    }
    block_reduce_store<6>(acc, partials, 0, gridDim.x);
}

// psi <- scale x; per-block partial maxima of |scale x - psi_old| into slot 0.
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_gs_finish(const typename CT<R>::T* __restrict__ x,
                                                           typename CT<R>::T* __restrict__ psi, long n, double scale,
                                                           double* partials) {
    double m = 0.0;
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        const double2 a = gsd::up(x[i]), b = gsd::up(psi[i]);
        const double2 y{scale * a.x, scale * a.y};
        const typename CT<R>::T yr = gsd::down<R>(y);
        const double dx = (double)yr.x - b.x, dy = (double)yr.y - b.y;
        m = fmax(m, sqrt(dx * dx + dy * dy));
        psi[i] = yr;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    __shared__ double red[RED_THREADS / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) s = fmax(s, red[w]);
        partials[blockIdx.x] = s;
    }
}

// out[k] = sum (op 0) or max (op 1) of partials[k * nblk + b] over b; one block per slot.
static __global__ __launch_bounds__(RED_THREADS) void k_gs_slots(const double* __restrict__ partials, int nblk,
                                                                 int op, double* __restrict__ out) {
    const int k = blockIdx.x;
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RED_THREADS) {
        const double v = partials[(long)k * nblk + b];
        a = op ? fmax(a, v) : a + v;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(a, off, 64);
        a = op ? fmax(a, o) : a + o;
    }
    __shared__ double red[RED_THREADS / 64];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) r = op ? fmax(r, red[w]) : r + red[w];
        out[k] = r;
    }
}

}  // namespace fse
