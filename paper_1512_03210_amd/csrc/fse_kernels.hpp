// HIP kernels of the split step (templates; instantiated per precision in
// fse_launch_f64.hip / fse_launch_f32.hip).
//
// Data layout: psi is C-contiguous [N0][N1]([N2]); axis 0 is the slowest.
// Every pass is one HBM sweep over one axis:
//   * strided passes transform axis 0 (and axis 1 in 3D): a workgroup owns W
//     adjacent columns (W*sizeof(complex) = 128 B per row) and all rows;
//   * line passes transform the contiguous axis: a workgroup owns LPB whole
//     lines.
// Fused passes of one TS2-GauSum step (rotating coordinates):
//   k_r2c         inverse FFT of axis 0 (completing the pending inverse of the
//                 previous linear step), density rho = |psi|^2, zero padding
//                 to 2N0 and the real-to-complex FFT of that padded line
//                 computed as a length-N0 complex FFT of (rho_2m + i rho_2m+1).
//   k_strided     padded forward / cropped inverse FFTs of axis 1 (3D).
//   k_line<conv>  forward FFT of the contiguous axis on 2N points, the real
//                 GauSum multiplier, inverse FFT, crop to N.
//   k_c2r_phase   complex-to-real inverse of axis 0 (Phi), the pending
//                 inverse FFT of axis 0 of the state, the nonlinear phase
//                 exp(-i[dt beta rho + lam dt Phi + P(x~)]), forward FFT of
//                 axis 0.
//   k_line<kin>   forward FFT, kinetic phase exp(-i tau omega/2)/n from a
//                 table folded by |p|, inverse FFT (contiguous axis).
#pragma once
#include "fse_fft.hpp"
#include "fse_types.hpp"

namespace fse {

constexpr int NT = 256;  // threads of the strided kernels

template <typename R> struct StridedCfg {
    static constexpr int W = (sizeof(R) == 8) ? 8 : 16;  // columns per tile: 128 B rows
    static constexpr int TPL = NT / W;                    // threads per line
};

template <typename L> struct Head;
template <int R0, int... Rs> struct Head<RList<R0, Rs...>> { static constexpr int value = R0; };

constexpr int floor_pow2(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

template <typename R, int M> struct LineCfg {
    using T = typename CT<R>::T;
    static constexpr int P = line_pitch<R>(M);
    static constexpr int TPL0 = M / Head<typename Radix<M>::L>::value;
    static constexpr int TPL = TPL0 < 4 ? 4 : (TPL0 > 64 ? 64 : TPL0);
    static constexpr int LB = 40960 / (P * (int)sizeof(T));
    static constexpr int LPB0 = floor_pow2(LB < 1 ? 1 : LB);
    static constexpr int LPB = (LPB0 * TPL > 256) ? (256 / TPL) : LPB0;
    static constexpr int THREADS = LPB * TPL;
};

// ---------------------------------------------------------------------------
// Tile movement helpers (strided tiles, column-fastest thread order so that
// each wavefront reads whole 128 B row segments).
// ---------------------------------------------------------------------------
template <typename R, int ROWS, int W, int P>
__device__ __forceinline__ void load_cols(typename CT<R>::T* lds, const typename CT<R>::T* g, long rstride, int cv) {
    using T = typename CT<R>::T;
    constexpr int TOT = ROWS * W;
    constexpr int NQ = (TOT + NT - 1) / NT;
    T v[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = threadIdx.x + q * NT;
        if ((TOT % NT) == 0 || i < TOT) {
            const int e = i / W, l = i % W;
            v[q] = (l < cv) ? g[(long)e * rstride + l] : T{0, 0};
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = threadIdx.x + q * NT;
        if ((TOT % NT) == 0 || i < TOT) {
            const int e = i / W, l = i % W;
            lds[l * P + padx<R>(e)] = v[q];
        }
    }
}

template <typename R, int ROWS, int W, int P>
__device__ __forceinline__ void store_cols(typename CT<R>::T* g, long rstride, const typename CT<R>::T* lds, int cv) {
    constexpr int TOT = ROWS * W;
    constexpr int NQ = (TOT + NT - 1) / NT;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = threadIdx.x + q * NT;
        if ((TOT % NT) == 0 || i < TOT) {
            const int e = i / W, l = i % W;
            if (l < cv) g[(long)e * rstride + l] = lds[l * P + padx<R>(e)];
        }
    }
}

template <typename R, int E0, int E1, int W, int P>
__device__ __forceinline__ void zero_rows(typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    constexpr int TOT = (E1 - E0) * W;
    for (int i = threadIdx.x; i < TOT; i += NT) {
        const int e = E0 + i / W, l = i % W;
        lds[l * P + padx<R>(e)] = T{0, 0};
    }
}

// ---------------------------------------------------------------------------
// Strided complex FFT of one axis.  Array viewed as [B0][rows][B2]; tile =
// W columns of B2 at one b0 (blockIdx.y).  MODE 0: M rows in, M rows out.
// MODE 1: M/2 rows in (zero padded to M), M rows out (padded forward).
// MODE 2: M rows in, first M/2 rows out (cropped inverse).
// ---------------------------------------------------------------------------
template <typename R, int M, bool INV, int MODE>
__global__ __launch_bounds__(NT) void k_strided(const typename CT<R>::T* in, typename CT<R>::T* out, int B2,
                                                const typename CT<R>::T* __restrict__ tw) {
    using T = typename CT<R>::T;
    constexpr int W = StridedCfg<R>::W, TPL = StridedCfg<R>::TPL;
    constexpr int RIN = (MODE == 1) ? M / 2 : M;
    constexpr int ROUT = (MODE == 2) ? M / 2 : M;
    constexpr int P = line_pitch<R>(M);
    __shared__ T lds[W * P];
    const int col0 = blockIdx.x * W;
    const int cv = min(W, B2 - col0);
    const T* gin = in + (long)blockIdx.y * RIN * B2 + col0;
    T* gout = out + (long)blockIdx.y * ROUT * B2 + col0;
    load_cols<R, RIN, W, P>(lds, gin, B2, cv);
    if (MODE == 1) zero_rows<R, RIN, M, W, P>(lds);
    const int line = threadIdx.x / TPL, jt = threadIdx.x % TPL;
    fft_line<R, M, INV, TPL>(lds + line * P, jt, tw);
    __syncthreads();
    store_cols<R, ROUT, W, P>(gout, B2, lds, cv);
}

// ---------------------------------------------------------------------------
// Contiguous-axis line kernel.
//   MODE 0 (conv): lines of N = M/2 points, zero padded to M, forward FFT,
//                  times the real multiplier K[row(line)][min(p, M-p)],
//                  inverse FFT, first N points stored.
//   MODE 1 (kin):  lines of N = M points, forward FFT, times the complex
//                  table Q[row(line)][min(p, M-p)], inverse FFT.
//   MODE 2 / 3:    plain forward / inverse FFT.
// row(line): i0 = line / D1, i1 = line % D1, folded by F0/F1 (0: no fold),
// row = (k0*T1 + k1)*T2.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int fold(int i, int F) { return (F == 0) ? i : min(i, F - i); }

template <typename R, int M, int MODE>
__global__ __launch_bounds__(256) void k_line(typename CT<R>::T* data, int nlines, const void* __restrict__ mult,
                                              LineIdx li, const typename CT<R>::T* __restrict__ tw) {
    using T = typename CT<R>::T;
    using Cfg = LineCfg<R, M>;
    constexpr int P = Cfg::P, TPL = Cfg::TPL, LPB = Cfg::LPB, NTH = Cfg::THREADS;
    constexpr int N = (MODE == 0) ? M / 2 : M;
    __shared__ T lds[LPB * P];
    const int line0 = blockIdx.x * LPB;
    const int lv = min(LPB, nlines - line0);
    T* g = data + (long)line0 * N;
    {
        constexpr int TOT = LPB * N;
        constexpr int NQ = (TOT + NTH - 1) / NTH;
        T v[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NTH;
            if ((TOT % NTH) == 0 || i < TOT) {
                const int l = i / N;
                v[q] = (l < lv) ? g[i] : T{0, 0};
            }
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NTH;
            if ((TOT % NTH) == 0 || i < TOT) {
                const int l = i / N, e = i % N;
                lds[l * P + padx<R>(e)] = v[q];
            }
        }
        if (MODE == 0) {
            for (int i = threadIdx.x; i < LPB * (M - N); i += NTH) {
                const int l = i / (M - N), e = N + i % (M - N);
                lds[l * P + padx<R>(e)] = T{0, 0};
            }
        }
    }
    const int line = threadIdx.x / TPL, jt = threadIdx.x % TPL;
    if (MODE != 3) fft_line<R, M, false, TPL>(lds + line * P, jt, tw);
    if (MODE == 0 || MODE == 1) {
        __syncthreads();
        for (int i = threadIdx.x; i < LPB * M; i += NTH) {
            const int l = i / M, p = i % M;
            if (l < lv) {
                const int gl = line0 + l;
                const int k0 = fold(gl / li.D1, li.F0), k1 = fold(gl % li.D1, li.F1);
                const long idx = (long)(k0 * li.T1 + k1) * li.T2 + min(p, M - p);
                T x = lds[l * P + padx<R>(p)];
                if (MODE == 0) {
                    const R k = static_cast<const R*>(mult)[idx];
                    x = T{x.x * k, x.y * k};
                } else {
                    x = cmul(x, static_cast<const T*>(mult)[idx]);
                }
                lds[l * P + padx<R>(p)] = x;
            }
        }
    }
    if (MODE != 2) fft_line<R, M, true, TPL>(lds + line * P, jt, tw);
    __syncthreads();
    {
        constexpr int TOT = LPB * N;
        for (int i = threadIdx.x; i < TOT; i += NTH) {
            const int l = i / N, e = i % N;
            if (l < lv) g[i] = lds[l * P + padx<R>(e)];
        }
    }
}

// ---------------------------------------------------------------------------
// Axis-0 density + padded real-to-complex FFT.
//   SRC 0: input is the state with the axis-0 inverse FFT pending;
//   SRC 1: input is psi in physical space;
//   SRC 2: input is a real density array.
// Output X1[k][c], k = 0..N0: the length-2N0 DFT of (rho_0..rho_{N0-1}, 0..0)
// at non-negative frequencies, from Z = FFT_N0(rho_2m + i rho_2m+1):
//   X_k = (Z_k + conj Z_{N0-k})/2 + exp(-i pi k/N0) (Z_k - conj Z_{N0-k})/(2i).
// ---------------------------------------------------------------------------
template <typename R, int N0, int SRC>
__global__ __launch_bounds__(NT) void k_r2c(const void* src, typename CT<R>::T* __restrict__ X1, int C,
                                            const typename CT<R>::T* __restrict__ twN,
                                            const typename CT<R>::T* __restrict__ tw2N) {
    using T = typename CT<R>::T;
    constexpr int W = StridedCfg<R>::W, TPL = StridedCfg<R>::TPL;
    constexpr int P = line_pitch<R>(N0 + 1);
    __shared__ T lds[W * P];
    const int col0 = blockIdx.x * W;
    const int cv = min(W, C - col0);
    const int line = threadIdx.x / TPL, jt = threadIdx.x % TPL;
    if (SRC == 2) {
        const R* g = static_cast<const R*>(src) + col0;
        for (int i = threadIdx.x; i < N0 * W; i += NT) {
            const int e = i / W, l = i % W;
            const R r = (l < cv) ? g[(long)e * C + l] : R(0);
            lds[l * P + padx<R>(e)] = T{r, R(0)};
        }
    } else {
        load_cols<R, N0, W, P>(lds, static_cast<const T*>(src) + col0, C, cv);
        if (SRC == 0) fft_line<R, N0, true, TPL>(lds + line * P, jt, twN);
    }
    __syncthreads();
    // z_m = rho_{2m} + i rho_{2m+1} for m < N0/2, zero above.
    {
        constexpr int TOT = (N0 / 2) * W;
        constexpr int NQ = (TOT + NT - 1) / NT;
        T z[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int m = i / W, l = i % W;
                const T a = lds[l * P + padx<R>(2 * m)];
                const T b = lds[l * P + padx<R>(2 * m + 1)];
                z[q] = (SRC == 2) ? T{a.x, b.x} : T{a.x * a.x + a.y * a.y, b.x * b.x + b.y * b.y};
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int m = i / W, l = i % W;
                lds[l * P + padx<R>(m)] = z[q];
            }
        }
        zero_rows<R, N0 / 2, N0, W, P>(lds);
    }
    fft_line<R, N0, false, TPL>(lds + line * P, jt, twN);
    __syncthreads();
    T* g = X1 + col0;
    for (int i = threadIdx.x; i < (N0 + 1) * W; i += NT) {
        const int k = i / W, l = i % W;
        if (l < cv) {
            const T zk = lds[l * P + padx<R>(k == N0 ? 0 : k)];
            const T zc = cconj(lds[l * P + padx<R>(k == 0 ? 0 : N0 - k)]);
            const T ev = T{R(0.5) * (zk.x + zc.x), R(0.5) * (zk.y + zc.y)};
            const T dv = csub(zk, zc);
            const T ov = T{R(0.5) * dv.y, -R(0.5) * dv.x};  // (zk - zc)/(2i)
            g[(long)k * C + l] = cadd(ev, cmul(tw2N[k], ov));
        }
    }
}

// ---------------------------------------------------------------------------
// Axis-0 complex-to-real inverse (nonlocal potential) fused with the
// nonlinear sub-step.
//   MODE 0: Phi from X1; state S (axis-0 inverse pending) -> psi -> phase
//           -> forward FFT of axis 0 -> S.
//   MODE 1: no nonlocal term: psi -> phase -> forward FFT of axis 0.
//   MODE 2: Phi only, written to Phi_out[e][c] (real).
// Inverse real transform of the Hermitian half X_0..X_N0 (length 2N0):
//   Z'_k = (X_k + conj X_{N0-k}) + i exp(+i pi k/N0) (X_k - conj X_{N0-k}),
//   y = IFFT_N0(Z') unnormalised, Phi_{2m} = Re y_m, Phi_{2m+1} = Im y_m.
// The GauSum multiplier already carries 1/prod(2 N_j).
// ---------------------------------------------------------------------------

template <typename R, int N0, int MODE>
__global__ __launch_bounds__(NT) void k_c2r_phase(const typename CT<R>::T* __restrict__ X1, typename CT<R>::T* S,
                                                  R* __restrict__ Phi_out, int C, PhaseArgs pa,
                                                  const typename CT<R>::T* __restrict__ twN,
                                                  const typename CT<R>::T* __restrict__ tw2N) {
    using T = typename CT<R>::T;
    constexpr int W = StridedCfg<R>::W, TPL = StridedCfg<R>::TPL;
    constexpr int P = line_pitch<R>(N0 + 1);
    constexpr int TOT = N0 * W;
    constexpr int NQ = (TOT + NT - 1) / NT;
    __shared__ T lds[W * P];
    const int col0 = blockIdx.x * W;
    const int cv = min(W, C - col0);
    const int line = threadIdx.x / TPL, jt = threadIdx.x % TPL;
    T sv[NQ];
    R phi[NQ];
    if (MODE != 2) {
        const T* g = S + col0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int e = i / W, l = i % W;
                sv[q] = (l < cv) ? g[(long)e * C + l] : T{0, 0};
            }
        }
    }
    if (MODE != 1) {
        load_cols<R, N0 + 1, W, P>(lds, X1 + col0, C, cv);
        __syncthreads();
        T zr[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int k = i / W, l = i % W;
                const T xk = lds[l * P + padx<R>(k)];
                const T xc = cconj(lds[l * P + padx<R>(N0 - k)]);
                const T a = cadd(xk, xc);
                const T b = cmulc(csub(xk, xc), tw2N[k]);  // exp(+i pi k/N0) (xk - xc)
                zr[q] = T{a.x - b.y, a.y + b.x};           // a + i b
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int k = i / W, l = i % W;
                lds[l * P + padx<R>(k)] = zr[q];
            }
        }
        fft_line<R, N0, true, TPL>(lds + line * P, jt, twN);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int i = threadIdx.x + q * NT;
            if ((TOT % NT) == 0 || i < TOT) {
                const int e = i / W, l = i % W;
                const T y = lds[l * P + padx<R>(e >> 1)];
                phi[q] = (e & 1) ? y.y : y.x;
            }
        }
        if (MODE == 2) {
            R* g = Phi_out + col0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int i = threadIdx.x + q * NT;
                if ((TOT % NT) == 0 || i < TOT) {
                    const int e = i / W, l = i % W;
                    if (l < cv) g[(long)e * C + l] = phi[q];
                }
            }
            return;
        }
        __syncthreads();
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) phi[q] = R(0);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = threadIdx.x + q * NT;
        if ((TOT % NT) == 0 || i < TOT) {
            const int e = i / W, l = i % W;
            lds[l * P + padx<R>(e)] = sv[q];
        }
    }
    fft_line<R, N0, true, TPL>(lds + line * P, jt, twN);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int i = threadIdx.x + q * NT;
        if ((TOT % NT) == 0 || i < TOT) {
            const int e = i / W, l = i % W;
            const int c = col0 + l;
            const R x = R(pa.x0 + e * pa.hx);
            R y, z;
            if (pa.N2 > 0) {
                y = R(pa.y0 + (c / pa.N2) * pa.hy);
                z = R(pa.z0 + (c % pa.N2) * pa.hz);
            } else {
                y = R(pa.y0 + c * pa.hy);
                z = R(0);
            }
            const R x2 = x * x, y2 = y * y;
            const R Pv = R(pa.ca) * (x2 + y2) + R(pa.cz) * (z * z) + R(pa.cc) * (x2 - y2) + R(pa.cs) * (R(2) * x * y);
            T v = lds[l * P + padx<R>(e)];
            const R rho = v.x * v.x + v.y * v.y;
            const R th = R(pa.bdt) * rho + R(pa.ldt) * phi[q] + Pv;
            R sn, cs;
            if constexpr (sizeof(R) == 4) {
                sincosf(th, &sn, &cs);
            } else {
                sincos(th, &sn, &cs);
            }
            lds[l * P + padx<R>(e)] = T{v.x * cs + v.y * sn, v.y * cs - v.x * sn};  // v * exp(-i th)
        }
    }
    fft_line<R, N0, false, TPL>(lds + line * P, jt, twN);
    __syncthreads();
    store_cols<R, N0, W, P>(S + col0, C, lds, cv);
}

// ---------------------------------------------------------------------------
// Kinetic phase table Q[k0][k1][k2] = scale * exp(-i tau omega/2),
// omega = (|mu|^2 + m^2)^s, mu_j = k_j * dmu_j, k_j = 0..N_j/2 (the table is
// even in each frequency index).  FP64 arithmetic, rounded to the path type.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_build_kin(typename CT<R>::T* __restrict__ Q, int T0, int T1, int T2, double dmu0, double dmu1,
                            double dmu2, double s, double m2, double tau, double scale) {
    using T = typename CT<R>::T;
    const long n = (long)T0 * T1 * T2;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const int k2 = (int)(i % T2);
        const long r = i / T2;
        const int k1 = (int)(r % T1);
        const int k0 = (int)(r / T1);
        const double a = k0 * dmu0, b = k1 * dmu1, c = k2 * dmu2;
        const double q = a * a + b * b + c * c + m2;
        const double om = (q > 0.0) ? pow(q, s) : 0.0;
        double sn, cs;
        sincos(-0.5 * tau * om, &sn, &cs);
        Q[i] = T{R(scale * cs), R(scale * sn)};
    }
}

// ---------------------------------------------------------------------------
// FP64 reductions.  Each kernel accumulates per-thread partial sums in FP64,
// reduces them across the block (wave shuffles, then LDS) and writes one
// value per block and slot to partials[slot * nblk + block].
// ---------------------------------------------------------------------------
constexpr int RED_THREADS = 256;

template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NV], double* partials, int slot0, int nblk) {
    __shared__ double red[NV][RED_THREADS / 64];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double x = acc[v];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((threadIdx.x & 63) == 0) red[v][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < RED_THREADS / 64; ++w) s += red[threadIdx.x][w];
        partials[(long)(slot0 + threadIdx.x) * nblk + blockIdx.x] = s;
    }
}


__device__ __forceinline__ void decode(long i, const GridGeom& g, int& i0, int& i1, int& i2) {
    if (g.d == 3) {
        i2 = (int)(i % g.N2);
        const long r = i / g.N2;
        i1 = (int)(r % g.N1);
        i0 = (int)(r / g.N1);
    } else {
        i2 = 0;
        i1 = (int)(i % g.N1);
        i0 = (int)(i / g.N1);
    }
}

// slots: 0 sum rho, 1 sum W rho, 2 sum rho^2, 3 sum Phi rho.
// W = wa (x^2+y^2) + wz z^2 + wc (x^2-y^2) + ws 2xy.
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_red_local(const typename CT<R>::T* __restrict__ psi,
                                                           const R* __restrict__ Phi, long n, GridGeom g, double wa,
                                                           double wz, double wc, double ws, double* partials,
                                                           int slot0) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const auto v = psi[i];
        const double rho = (double)v.x * v.x + (double)v.y * v.y;
        const double Wv = wa * (x * x + y * y) + wz * z * z + wc * (x * x - y * y) + ws * 2.0 * x * y;
        acc[0] += rho;
        acc[1] += Wv * rho;
        acc[2] += rho * rho;
        if (Phi) acc[3] += (double)Phi[i] * rho;
    }
    block_reduce_store<4>(acc, partials, slot0, gridDim.x);
}

// sum omega(k) |psihat_k|^2, omega = (|mu|^2 + m^2)^s, mu in DFT order.
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_red_kin(const typename CT<R>::T* __restrict__ ph, long n, GridGeom g,
                                                         double dmu0, double dmu1, double dmu2, double s, double m2,
                                                         double* partials, int slot0) {
    double acc[1] = {0.0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const int p0 = (i0 < g.N0 / 2) ? i0 : i0 - g.N0;
        const int p1 = (i1 < g.N1 / 2) ? i1 : i1 - g.N1;
        const int p2 = (g.d == 3) ? ((i2 < g.N2 / 2) ? i2 : i2 - g.N2) : 0;
        const double a = p0 * dmu0, b = p1 * dmu1, c = p2 * dmu2;
        const double q = a * a + b * b + c * c + m2;
        const double om = (q > 0.0) ? pow(q, s) : 0.0;
        const auto v = ph[i];
        acc[0] += om * ((double)v.x * v.x + (double)v.y * v.y);
    }
    block_reduce_store<1>(acc, partials, slot0, gridDim.x);
}

// sum coord * Im(conj(psi) * D), coord = x (axis 0) or y (axis 1).
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_red_lz(const typename CT<R>::T* __restrict__ psi,
                                                        const typename CT<R>::T* __restrict__ D, long n, GridGeom g,
                                                        int coord_axis, double* partials, int slot0) {
    double acc[1] = {0.0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double c = (coord_axis == 0) ? g.x0 + i0 * g.hx : g.y0 + i1 * g.hy;
        const auto a = psi[i];
        const auto b = D[i];
        acc[0] += c * ((double)a.x * b.y - (double)a.y * b.x);
    }
    block_reduce_store<1>(acc, partials, slot0, gridDim.x);
}

// Final combination (one block).  tot[s] = sum over blocks of slot s.
//   KIND 0 (mass):   out[0] = vol * tot[0]
//   KIND 1 (energy): out = {kin, pot, int, non, rot, total} from
//                    tot[0..3] local, tot[4] kinetic, tot[5], tot[6] Lz parts
//   KIND 2 (Lz):     out[0] = vol * (tot[5] - tot[6])
static __global__ __launch_bounds__(RED_THREADS) void k_red_final(const double* __restrict__ partials, int nblk, int nslot,
                                                           int kind, double vol, double n, double beta, double lam,
                                                           double Omega, double* out) {
    __shared__ double tot[8];
    __shared__ double red[RED_THREADS / 64];
    for (int s = 0; s < nslot; ++s) {
        double x = 0.0;
        for (int b = threadIdx.x; b < nblk; b += RED_THREADS) x += partials[(long)s * nblk + b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
            tot[s] = t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (kind == 0) {
            out[0] = vol * tot[0];
        } else if (kind == 1) {
            const double ekin = 0.5 * vol / n * tot[4];
            const double epot = vol * tot[1];
            const double eint = 0.5 * beta * vol * tot[2];
            const double enon = 0.5 * lam * vol * tot[3];
            const double lz = vol * (tot[5] - tot[6]);
            const double erot = -Omega * lz;
            out[0] = ekin;
            out[1] = epot;
            out[2] = eint;
            out[3] = enon;
            out[4] = erot;
            out[5] = ekin + epot + eint + enon + erot;
        } else {
            out[0] = vol * (tot[5] - tot[6]);
        }
    }
}

// ---------------------------------------------------------------------------
// Elementwise helpers for the diagnostics and H*psi.
// ---------------------------------------------------------------------------
// out = in * f(k) * scale; f = i mu_axis (WHAT 0) or omega/2 (WHAT 1).
template <typename R>
__global__ void k_fourier_mult(const typename CT<R>::T* __restrict__ in, typename CT<R>::T* __restrict__ out, long n,
                               GridGeom g, int what, int axis, double dmu0, double dmu1, double dmu2, double s,
                               double m2, double scale) {
    using T = typename CT<R>::T;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const int p0 = (i0 < g.N0 / 2) ? i0 : i0 - g.N0;
        const int p1 = (i1 < g.N1 / 2) ? i1 : i1 - g.N1;
        const int p2 = (g.d == 3) ? ((i2 < g.N2 / 2) ? i2 : i2 - g.N2) : 0;
        const T v = in[i];
        if (what == 0) {
            const double mu = (axis == 0) ? p0 * dmu0 : (axis == 1 ? p1 * dmu1 : p2 * dmu2);
            const double f = mu * scale;
            out[i] = T{R(-v.y * f), R(v.x * f)};
        } else {
            const double a = p0 * dmu0, b = p1 * dmu1, c = p2 * dmu2;
            const double q = a * a + b * b + c * c + m2;
            const double f = 0.5 * ((q > 0.0) ? pow(q, s) : 0.0) * scale;
            out[i] = T{R(v.x * f), R(v.y * f)};
        }
    }
}

// H psi accumulation:
//   WHAT 0: H += i Omega x D  (D = D_y psi)
//   WHAT 1: H += -i Omega y D (D = D_x psi)
//   WHAT 2: H += (V + beta rho + lam Phi) psi, rho = |psi|^2 or rho_in.
template <typename R>
__global__ void k_H_accum(typename CT<R>::T* __restrict__ H, const typename CT<R>::T* __restrict__ D,
                          const typename CT<R>::T* __restrict__ psi, const R* __restrict__ rho_in,
                          const R* __restrict__ Phi, long n, GridGeom g, int what, double Omega, double beta,
                          double lam, double g0, double g1, double g2) {
    using T = typename CT<R>::T;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        T h = H[i];
        if (what == 0 || what == 1) {
            const T dv = D[i];
            const double f = (what == 0) ? Omega * x : -Omega * y;
            h = T{R(h.x - f * dv.y), R(h.y + f * dv.x)};
        } else {
            const T v = psi[i];
            const double rho = rho_in ? (double)rho_in[i] : (double)v.x * v.x + (double)v.y * v.y;
            const double V = 0.5 * (g0 * g0 * x * x + g1 * g1 * y * y + g2 * g2 * z * z);
            const double f = V + beta * rho + (Phi ? lam * (double)Phi[i] : 0.0);
            h = T{R(h.x + f * v.x), R(h.y + f * v.y)};
        }
        H[i] = h;
    }
}

}  // namespace fse
