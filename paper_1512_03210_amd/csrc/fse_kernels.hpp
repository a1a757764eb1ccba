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
#include <type_traits>

#include "fse_fft.hpp"
#include "fse_types.hpp"

namespace fse {

// ---------------------------------------------------------------------------
// Tile configurations.
//   Column tiles (axes 0 and 1 of the strided passes): W adjacent columns
//   (128 B of every row), lanes ordered column-fastest so that each load and
//   store instruction touches whole 128 B row segments; TPL threads per
//   column.
//   Line tiles (contiguous axis): LPB whole lines, lanes ordered
//   position-fastest.
// ---------------------------------------------------------------------------
// Radix plan of the column (strided-axis) transforms: CV = 0 the plain plan,
// CV = 1 an alternative where the length has one (256 as 8.8.4 beside 16.16:
// twice the threads per column, 8 points each, one more LDS exchange; the
// autotuner picks per plan).
template <int N, int CV = 0> struct ColPlanOf {
    static constexpr bool has_alt = false;
    using L = FwdPlan<N>;
};
template <> struct ColPlanOf<256, 1> {
    static constexpr bool has_alt = true;
    using L = RList<8, 8, 4>;
};
template <> struct ColPlanOf<256, 0> {
    static constexpr bool has_alt = true;
    using L = FwdPlan<256>;
};
template <int N, int CV = 0> using ColPlan = typename ColPlanOf<N, CV>::L;

template <int N, typename PL> struct PlanOf { using L = PL; };
template <int N> struct PlanOf<N, void> { using L = ColPlan<N>; };

// Column tile: W columns of 128 B, TPL threads per column (the plan's first
// radix sets the points per thread); PL = void selects the plain plan.  A
// 512-point complex64 tile (64 KB of LDS: two workgroups per CU) takes 1024
// threads, so that the two workgroups bring 32 waves to the CU, not 16.
template <typename R, int N, typename PL = void> struct ColCfg {
    static constexpr int W = (sizeof(R) == 8) ? 8 : 16;
    static constexpr int TPL0 = N / Head<typename PlanOf<N, PL>::L>::value;
    static constexpr int CAP = (sizeof(R) == 4 && N == 512) ? 1024 : 512;  // threads per workgroup
    static constexpr int TPL = TPL0 < 4 ? 4 : (TPL0 * W > CAP ? CAP / W : TPL0);
    static constexpr int NTH = W * TPL;
};

// Radix plan of the fused complex-to-real + nonlinear phase kernel: in FP64
// it keeps three arrays per thread live, so where the plain plan gives a
// thread 16 points this one gives it 8 (one more LDS exchange per transform,
// half the registers per array: occupancy 4 instead of 2).  FV = 1 is the
// other of the two 256-point plans (16.16 in FP64, 8.8.4 in FP32; the
// autotuner times both).
template <typename R, int N, int FV = 0> struct FusedPlan {
    static constexpr bool has_alt = false;
    using L = FwdPlan<N>;
};
template <> struct FusedPlan<double, 256, 0> {
    static constexpr bool has_alt = true;
    using L = RList<8, 8, 4>;
};
template <> struct FusedPlan<double, 256, 1> {
    static constexpr bool has_alt = true;
    using L = FwdPlan<256>;
};
template <> struct FusedPlan<float, 256, 0> {
    static constexpr bool has_alt = true;
    using L = FwdPlan<256>;
};
template <> struct FusedPlan<float, 256, 1> {
    static constexpr bool has_alt = true;
    using L = RList<8, 8, 4>;
};
template <typename R, int N, int FV = 0> using FusedCfg = ColCfg<R, N, typename FusedPlan<R, N, FV>::L>;

// Waves per SIMD that the LDS of one workgroup allows (160 KB per CU, four
// SIMDs).  Column kernels hold 37-78 KB of LDS, so the LDS caps them at 2-4
// waves per SIMD.  For FP64 up to length 256 their register budget is set to
// that same occupancy (FSE_COL_OCC): left to itself the compiler spends spare
// registers on scheduling and can end one wave below it (the FP64 phase
// kernel: 130 VGPRs and 3 waves, where 128 give 4 with no spills).  The
// complex64 phase kernel needs 161 and would spill at 128, and the 512-point
// tiles spill too, so those keep the compiler's choice.
constexpr int lds_waves(int lds_bytes, int nth) {
    const int wg = (160 * 1024) / lds_bytes;
    const int w = (wg < 1 ? 1 : wg) * (nth / 64) / 4;
    return w < 1 ? 1 : (w > 8 ? 8 : w);
}
template <typename R, int N> constexpr int col_occ(int lds_bytes, int nth) {
    return (sizeof(R) == 8 && N <= 256) ? lds_waves(lds_bytes, nth) : 1;
}
#define FSE_COL_OCC(R, N, ...) __attribute__((amdgpu_waves_per_eu(col_occ<R, N>(__VA_ARGS__), 8)))
template <typename R> constexpr int csz() { return (int)sizeof(typename CT<R>::T); }

constexpr int floor_pow2(int x) {
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}

// Radix schedules of the line transforms: V = 0 the plain one (Radix<M>),
// V = 1 an alternative for the lengths where one is worth timing (fewer,
// fuller threads per line, or the reverse); the plan's autotuner picks one
// per pass.  Lengths without an alternative use the plain schedule for both.
template <int M> struct AltRadix {
    static constexpr bool has = false;
    using L = void;
};
template <> struct AltRadix<256> {
    static constexpr bool has = true;
    using L = RList<8, 8, 4>;
};
template <> struct AltRadix<512> {
    static constexpr bool has = true;
    using L = RList<16, 8, 4>;
};
template <int M, int V> struct LineFwdOf { using L = FwdPlan<M>; };
template <int M> struct LineFwdOf<M, 1> { using L = typename AltRadix<M>::L; };
template <int M, int V> using LineFwd = typename LineFwdOf<M, V>::L;
template <int M, int V> using LineInv = typename Rev<LineFwd<M, V>>::L;

template <typename R, int N, bool CONV, int V = 0> struct LineCfg {
    using T = typename CT<R>::T;
    static constexpr int P = (sizeof(R) == 8) ? (N + (N >> PadShift<N>::value)) : pitch_lines<N>(N);
    static constexpr int TPL0 = N / Head<LineFwd<N, V>>::value;
    static constexpr int TPL = TPL0 < 4 ? 4 : (TPL0 > 64 ? 64 : TPL0);
    static constexpr int SUB = CONV ? 2 : 1;  // LDS sub-lines (and thread groups) per data line
    // LDS per workgroup aimed at: small workgroups (down to one wavefront)
    // strand less of the 160 KB per CU than a few large ones (FP64 256^3:
    // convolution 16 -> 17 lines per CU, kinetic pass 8 -> 9; both ~2.5 %
    // faster than with a 40 KB budget)
    static constexpr int BUDGET = 10240 / (P * (int)sizeof(T) * SUB);
    static constexpr int LPB0 = floor_pow2(BUDGET < 1 ? 1 : BUDGET);
    static constexpr int LPB1 = (LPB0 * TPL * SUB > 256) ? 256 / (TPL * SUB) : LPB0;
    static constexpr int LPBW = (TPL * SUB >= 64) ? 1 : 64 / (TPL * SUB);  // at least one full wavefront
    static constexpr int LPB = LPB1 < LPBW ? LPBW : LPB1;
    static constexpr int NTH = LPB * TPL * SUB;
    // FP64 512-point lines of the padded convolution (default radix plan)
    // exchange one component at a time (xchg_split): half the LDS per line, so
    // the LDS no longer caps a CU at 17 lines
    static constexpr bool XS = !CONV && sizeof(R) == 8 && N == 512 && V == 0;
    static constexpr int LDS = XS ? (LPB * P + 1) / 2 : LPB * P;  // complex elements per workgroup
    // waves per SIMD asked of the register allocator with split exchanges: the
    // LDS would allow 8, but 7 and 8 spill (6: 74 VGPRs, no spill)
    static constexpr int OCC = lds_waves(LDS * (int)sizeof(T), NTH) < 6 ? lds_waves(LDS * (int)sizeof(T), NTH) : 6;
};

// Calls f(b, r, e) for every position e = j + r*N/RAD the thread owns.
template <int N, int TPL, int RAD, typename F> __device__ __forceinline__ void for_pos(int jt, F f) {
    using S = Shape<N, TPL, RAD>;
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) f(b, r, j + r * S::NB);
        }
    }
}

// Calls f(i, k) for the rows k = jt + i*TPL <= N that the thread owns (N + 1
// rows), unrolled so that the loads in f issue together.
template <int N, int TPL, typename F> __device__ __forceinline__ void for_rows_incl(int jt, F f) {
#pragma unroll
    for (int i = 0; i < (N + TPL) / TPL; ++i) {
        const int k = jt + i * TPL;
        if (k <= N) f(i, k);
    }
}

// Tile order of a column-tile launch.  Workgroup w (linear over the grid) is
// dispatched to XCD w mod 8.  With XR, w -> (w mod 8)(nw/8) + w/8 gives each
// XCD one contiguous range of tiles, so the tiles that run side by side on one
// XCD cover whole rows of the array rather than every eighth 128 B segment of
// them: that pattern alone streams ~10 % faster (5.5 against 5.0 TB/s).  In the
// step it also changes what the next pass finds in the last-level cache, so it
// is used where the step as a whole is faster (256^3, both precisions): the
// forward column transform, the cropped inverse, and in FP64 the padded
// forward.  Workgroups past the last multiple of 8 keep their tile; the map is
// a bijection on the grid.
template <bool XR> __device__ __forceinline__ void col_tile(int& bx, int& by) {
    if constexpr (!XR) {
        bx = (int)blockIdx.x;
        by = (int)blockIdx.y;
    } else {
        const int gx = (int)gridDim.x, nw = gx * (int)gridDim.y;
        const int w = (int)blockIdx.x + (int)blockIdx.y * gx;
        const int full = nw & ~7;
        const int t = (w < full) ? (w & 7) * (full >> 3) + (w >> 3) : w;
        bx = t % gx;
        by = t / gx;
    }
}

// ---------------------------------------------------------------------------
// Column-tile complex FFT of one strided axis, array [B0][N][B2], tile = W
// columns of B2 at b0 = blockIdx.y, forward or inverse, in place allowed.
// twN: exp(-2 pi i m/N), m < N.
// ---------------------------------------------------------------------------
// Multiply by f = 1 + d, d = *scale - 1 (a factor within rounding distance of 1): in FP32 as v + v d with the
// product inside the FMA, so that the tiny d is not lost to the rounding of f itself.
template <typename R> __device__ __forceinline__ typename CT<R>::T scale_near_one(typename CT<R>::T v, double f) {
    if constexpr (sizeof(R) == 4) {
        const float dd = float(f - 1.0);
        return typename CT<R>::T{fmaf(v.x, dd, v.x), fmaf(v.y, dd, v.y)};
    } else {
        return typename CT<R>::T{v.x * f, v.y * f};
    }
}

template <typename R, int N, bool INV, int CV = 0>
__device__ __forceinline__ void cols_body(const typename CT<R>::T* in, typename CT<R>::T* out,
                                                            int B2, const typename CT<R>::T* twN, int bx, int by, typename CT<R>::T* lds,
                                                            const double* scale = nullptr) {
    using T = typename CT<R>::T;
    using C = ColCfg<R, N, ColPlan<N, CV>>;
    constexpr int W = C::W, TPL = C::TPL;
    constexpr int P = pitch_cols<N>(N);
    using F = Fft<T, N, INV, TPL, ColPlan<N, CV>>;
    const int l = threadIdx.x % W, jt = threadIdx.x / W;
    const int col0 = bx * W;
    const bool lv = (col0 + l) < B2;
    T* line = lds + l * P;
    const T* g = in + (long)by * N * B2 + col0 + l;
    T* o = out + (long)by * N * B2 + col0 + l;
    {
        typename F::In v;
        typename F::Out u;
        for_pos<N, TPL, F::R0>(jt, [&](int b, int r, int e) { v[b][r] = lv ? g[(long)e * B2] : T{0, 0}; });
        F::run(v, u, line, jt, twN);
        if (scale) {
            const double f = *scale;
            for_pos<N, TPL, F::RK>(jt, [&](int b, int r, int) { u[b][r] = scale_near_one<R>(u[b][r], f); });
        }
        for_pos<N, TPL, F::RK>(jt, [&](int b, int r, int e) {
            if (lv) o[(long)e * B2] = u[b][r];
        });
    }
}

// scale: null, or a device factor applied to the output (the complex64 mass renormalisation).
template <typename R, int N, bool INV, int CV = 0>
__global__ __launch_bounds__((ColCfg<R, N, ColPlan<N, CV>>::NTH))
FSE_COL_OCC(R, N, ColCfg<R, N>::W * pitch_cols<N>(N) * csz<R>(), ColCfg<R, N, ColPlan<N, CV>>::NTH)
void k_cols(const typename CT<R>::T* in, typename CT<R>::T* out,
                                                            int B2, const typename CT<R>::T* twN,
                                                            const double* scale) {
    __shared__ typename CT<R>::T lds[ColCfg<R, N>::W * pitch_cols<N>(N)];
    int bx, by;
    col_tile<!INV>(bx, by);
    cols_body<R, N, INV, CV>(in, out, B2, twN, bx, by, lds, scale);
}

// ---------------------------------------------------------------------------
// Fourier derivative along a strided axis in one pass: forward FFT of the
// column, times i mu_p * scale (mu_p = p * dmu, p = e for e < N/2, else
// e - N, the Nyquist index kept as -N/2), inverse FFT with the reversed plan
// (no LDS traffic between the two), out of place allowed.
// ---------------------------------------------------------------------------
template <typename R, int N>
__device__ __forceinline__ void cols_deriv_body(const typename CT<R>::T* in, typename CT<R>::T* out, int B2,
                                                const typename CT<R>::T* twN, double dmu, double scale, int bx,
                                                int by, typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    using C = ColCfg<R, N>;
    constexpr int W = C::W, TPL = C::TPL;
    constexpr int P = pitch_cols<N>(N);
    using FF = Fft<T, N, false, TPL, ColPlan<N>>;
    using FI = Fft<T, N, true, TPL, typename Rev<ColPlan<N>>::L>;
    const int l = threadIdx.x % W, jt = threadIdx.x / W;
    const int col0 = bx * W;
    const bool lv = (col0 + l) < B2;
    T* line = lds + l * P;
    const T* g = in + (long)by * N * B2 + col0 + l;
    T* o = out + (long)by * N * B2 + col0 + l;
    typename FF::In v;
    typename FF::Out u;
    for_pos<N, TPL, FF::R0>(jt, [&](int b, int r, int e) { v[b][r] = lv ? g[(long)e * B2] : T{0, 0}; });
    FF::run(v, u, line, jt, twN);
    for_pos<N, TPL, FF::RK>(jt, [&](int b, int r, int e) {
        const R f = R(((e < N / 2) ? e : e - N) * dmu * scale);
        u[b][r] = T{-u[b][r].y * f, u[b][r].x * f};
    });
    typename FI::Out w;
    __syncthreads();
    FI::run(u, w, line, jt, twN);
    for_pos<N, TPL, FI::RK>(jt, [&](int b, int r, int e) {
        if (lv) o[(long)e * B2] = w[b][r];
    });
}

template <typename R, int N>
__global__ __launch_bounds__((ColCfg<R, N>::NTH))
FSE_COL_OCC(R, N, ColCfg<R, N>::W * pitch_cols<N>(N) * csz<R>(), ColCfg<R, N>::NTH)
void k_cols_deriv(const typename CT<R>::T* in,
                                                                     typename CT<R>::T* out, int B2,
                                                                     const typename CT<R>::T* twN, double dmu,
                                                                     double scale) {
    __shared__ typename CT<R>::T lds[ColCfg<R, N>::W * pitch_cols<N>(N)];
    cols_deriv_body<R, N>(in, out, B2, twN, dmu, scale, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Zero-padded transforms of a strided axis as one length-M = 2N transform
// per column: PAD = 1, forward, N rows in (the first stage skips the zero
// half) and 2N rows out; PAD = 2, inverse, 2N rows in and only the first N
// rows stored.
// ---------------------------------------------------------------------------
template <typename R, int M, int PAD>
__device__ __forceinline__ void cols_full_body(const typename CT<R>::T* in,
                                                                   typename CT<R>::T* out, int B2,
                                                                   const typename CT<R>::T* twM, int bx, int by, typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    using C = ColCfg<R, M>;
    constexpr int W = C::W, TPL = C::TPL;
    constexpr int P = pitch_cols<M>(M);
    constexpr bool INV = (PAD == 2);
    using F = Fft<T, M, INV, TPL, ColPlan<M>>;
    const int l = threadIdx.x % W, jt = threadIdx.x / W;
    const int col0 = bx * W;
    const bool lv = (col0 + l) < B2;
    T* line = lds + l * P;
    constexpr int RIN = (PAD == 1) ? M / 2 : M;
    constexpr int ROUT = (PAD == 2) ? M / 2 : M;
    const T* g = in + (long)by * RIN * B2 + col0 + l;
    T* o = out + (long)by * ROUT * B2 + col0 + l;
    typename F::In v;
    typename F::Out u;
    for_pos<M, TPL, F::R0>(jt, [&](int b, int r, int e) { v[b][r] = (lv && e < RIN) ? g[(long)e * B2] : T{0, 0}; });
    F::run(v, u, line, jt, twM);
    for_pos<M, TPL, F::RK>(jt, [&](int b, int r, int e) {
        if (lv && e < ROUT) o[(long)e * B2] = u[b][r];
    });
}

template <typename R, int M, int PAD>
__global__ __launch_bounds__((ColCfg<R, M>::NTH))
FSE_COL_OCC(R, M, ColCfg<R, M>::W * pitch_cols<M>(M) * csz<R>(), ColCfg<R, M>::NTH)
void k_cols_full(const typename CT<R>::T* in,
                                                                   typename CT<R>::T* out, int B2,
                                                                   const typename CT<R>::T* twM) {
    __shared__ typename CT<R>::T lds[ColCfg<R, M>::W * pitch_cols<M>(M)];
    int bx, by;
    col_tile<PAD == 2 || sizeof(R) == 8>(bx, by);
    cols_full_body<R, M, PAD>(in, out, B2, twM, bx, by, lds);
}

// ---------------------------------------------------------------------------
// Contiguous-axis line kernel, lines of N points.
//   MODE 0 (conv, used where 2N exceeds the longest compiled transform):
//          zero-padded length-2N convolution by a real multiplier, computed
//          as two length-N halves: sub-line h = 0 transforms x,
//          h = 1 transforms x_n w^n (w = exp(-i pi/N)); their spectra are the
//          even (p = 2k) and odd (p = 2k+1) frequencies of the padded line,
//          multiplied by K[row(line)][min(p, 2N-p)]; after the inverse
//          halves the line is y_n = ya_n + w^{-n} yb_n.
//   MODE 1 (kin): forward FFT, times Q[row(line)][min(p, N-p)] (complex),
//          inverse FFT.
//   MODE 2 / 3: plain forward / inverse FFT.
// row(line): i0 = line / D1, i1 = line % D1, folded by F0/F1 (0: no fold),
// row = (k0*T1 + k1)*T2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int fold(int i, int F) { return (F == 0) ? i : min(i, F - i); }

// Position q of the mirror order over [0, F) -> index: q = 2m -> m,
// q = 2m + 1 -> F - m (m >= 1) or F/2 (m = 0).
__device__ __forceinline__ int mirror_order(int q, int F) {
    const int m = q >> 1;
    return (q & 1) == 0 ? m : (m == 0 ? F / 2 : F - m);
}

// Line handled at visit position gl (identity unless X0 or X1 is set).
__device__ __forceinline__ int line_at(int gl, const LineIdx& li) {
    if (li.X0 && li.X1) {
        const int G = gl >> 2, h1 = li.F1 >> 1;
        const int q0 = 2 * (G / h1) + ((gl >> 1) & 1), q1 = 2 * (G % h1) + (gl & 1);
        return mirror_order(q0, li.F0) * li.D1 + mirror_order(q1, li.F1);
    }
    if (li.X1) return (gl / li.D1) * li.D1 + mirror_order(gl % li.D1, li.F1);
    if (li.X0) return mirror_order(gl, li.F0);
    return gl;
}

// Workgroups are dispatched to the eight XCDs round-robin (w mod 8), each XCD
// with its own L2.  Visit position pairs (2j, 2j+1), which share a multiplier
// row in mirror order, go to workgroups w and w + 8: the same XCD, one after
// the other (a bijection on every group of 16; the identity when the grid is
// not a multiple of 16).
__device__ __forceinline__ int xcd_pairs(int w, int nw) {
    if (nw & 15) return w;
    const int s = w >> 3;  // dispatch slot on the XCD
    return ((s >> 1) << 4) + ((w & 7) << 1) + (s & 1);
}

__device__ __forceinline__ long mult_row(int gl, const LineIdx& li) {
    const int k0 = fold(gl / li.D1, li.F0), k1 = fold(gl % li.D1, li.F1);
    return (long)(k0 * li.T1 + k1) * li.T2;
}

template <typename R, int N, int MODE, int V = 0>
__device__ __forceinline__ void lines_body(
    typename CT<R>::T* data, int nlines, const void* mult, LineIdx li,
    const typename CT<R>::T* twN, const typename CT<R>::T* tw2, int bx, int by, typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    using C = LineCfg<R, N, MODE == 0, V>;
    constexpr int P = C::P, TPL = C::TPL, LPB = C::LPB, SUB = C::SUB;
    constexpr bool WS = (64 % (TPL * SUB)) == 0;  // a data line's threads share one wavefront
    using FF = Fft<T, N, false, TPL, LineFwd<N, V>, WS, 2>;
    using FI = Fft<T, N, true, TPL, LineInv<N, V>, WS, 2>;
    const int jt = threadIdx.x % TPL;
    const int sl = threadIdx.x / TPL;  // sub-line
    const int dl = sl / SUB, h = sl % SUB;
    const int gv = bx * LPB + dl;
    const bool valid = gv < nlines;
    const int gl = valid ? line_at(gv, li) : 0;
    T* line = lds + sl * P;
    T* g = data + (long)gl * N;
    if constexpr (MODE == 3) {
        using FP = Fft<T, N, true, TPL, LineFwd<N, V>, WS, 2>;
        typename FP::In v;
        typename FP::Out u;
        for_pos<N, TPL, FP::R0>(jt, [&](int b, int r, int e) { v[b][r] = g[e]; });
        FP::run(v, u, line, jt, twN);
        for_pos<N, TPL, FP::RK>(jt, [&](int b, int r, int e) {
            if (valid) g[e] = u[b][r];
        });
    } else {
        typename FF::In v;
        typename FF::Out u;
        // (a line past the end reads line 0 and stores nothing)
        for_pos<N, TPL, FF::R0>(jt, [&](int b, int r, int e) {
            T x = g[e];
            if (MODE == 0 && h == 1) x = cmul(x, tw2[e]);
            v[b][r] = x;
        });
        // FP32 kinetic pass with a palindromic plan: the inverse takes the
        // forward's twiddles from registers
        constexpr bool KEEP = MODE == 1 && sizeof(R) == 4 && std::is_same<LineFwd<N, V>, LineInv<N, V>>::value;
        typename FF::Keep keep;
        if constexpr (KEEP) FF::template run_tw<TW_KEEP>(v, u, line, jt, twN, keep);
        else FF::run(v, u, line, jt, twN);
        if constexpr (MODE == 2) {
            for_pos<N, TPL, FF::RK>(jt, [&](int b, int r, int e) {
                if (valid) g[e] = u[b][r];
            });
        } else {
            const long row = mult_row(gl, li);
            for_pos<N, TPL, FF::RK>(jt, [&](int b, int r, int e) {
                if (MODE == 0) {
                    const int p = 2 * e + h;
                    const R k = static_cast<const R*>(mult)[row + min(p, 2 * N - p)];
                    u[b][r] = T{u[b][r].x * k, u[b][r].y * k};
                } else {
                    const T q = static_cast<const T*>(mult)[row + min(e, N - e)];
                    u[b][r] = cmul(u[b][r], q);
                }
            });
            typename FI::Out w;
            lds_sync<WS>();
            if constexpr (KEEP) FI::template run_tw<TW_REUSE>(u, w, line, jt, twN, keep);
            else FI::run(u, w, line, jt, twN);
            if constexpr (MODE == 1) {
                for_pos<N, TPL, FI::RK>(jt, [&](int b, int r, int e) {
                    if (valid) g[e] = w[b][r];
                });
            } else {
                // combine the halves: y = ya + w^{-n} yb (the odd half goes through LDS)
                lds_sync<WS>();
                if (h == 1) {
                    for_pos<N, TPL, FI::RK>(jt, [&](int b, int r, int e) { line[padx<N>(e)] = cmulc(w[b][r], tw2[e]); });
                }
                lds_sync<WS>();
                if (h == 0) {
                    const T* other = line + P;
                    for_pos<N, TPL, FI::RK>(jt, [&](int b, int r, int e) {
                        if (valid) g[e] = cadd(w[b][r], other[padx<N>(e)]);
                    });
                }
            }
        }
    }
}

template <typename R, int N, int MODE, int V = 0>
__global__ __launch_bounds__((LineCfg<R, N, MODE == 0, V>::NTH)) void k_lines(
    typename CT<R>::T* data, int nlines, const void* mult, LineIdx li,
    const typename CT<R>::T* twN, const typename CT<R>::T* tw2) {
    using C = LineCfg<R, N, MODE == 0, V>;
    __shared__ typename CT<R>::T lds[C::LPB * C::SUB * C::P];
    lines_body<R, N, MODE, V>(data, nlines, mult, li, twN, tw2, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Fourier derivative along the contiguous axis in one pass (as
// cols_deriv_body, whole lines), out of place allowed.
// ---------------------------------------------------------------------------
template <typename R, int N>
__global__ __launch_bounds__((LineCfg<R, N, false>::NTH)) void k_lines_deriv(const typename CT<R>::T* in,
                                                                              typename CT<R>::T* out, int nlines,
                                                                              const typename CT<R>::T* twN,
                                                                              double dmu, double scale) {
    using T = typename CT<R>::T;
    using C = LineCfg<R, N, false>;
    constexpr int P = C::P, TPL = C::TPL, LPB = C::LPB;
    constexpr bool WS = (64 % TPL) == 0;  // a line's threads share one wavefront
    using FF = Fft<T, N, false, TPL, FwdPlan<N>, WS, 2>;
    using FI = Fft<T, N, true, TPL, InvPlan<N>, WS, 2>;
    __shared__ T lds[LPB * P];
    const int jt = threadIdx.x % TPL;
    const int dl = threadIdx.x / TPL;
    const int gl = blockIdx.x * LPB + dl;
    const bool valid = gl < nlines;
    T* line = lds + dl * P;
    const T* g = in + (long)(valid ? gl : 0) * N;  // a line past the end reads line 0 and stores nothing
    T* o = out + (long)gl * N;
    typename FF::In v;
    typename FF::Out u;
    for_pos<N, TPL, FF::R0>(jt, [&](int b, int r, int e) { v[b][r] = g[e]; });
    FF::run(v, u, line, jt, twN);
    for_pos<N, TPL, FF::RK>(jt, [&](int b, int r, int e) {
        const R f = R(((e < N / 2) ? e : e - N) * dmu * scale);
        u[b][r] = T{-u[b][r].y * f, u[b][r].x * f};
    });
    typename FI::Out w;
    lds_sync<WS>();
    FI::run(u, w, line, jt, twN);
    for_pos<N, TPL, FI::RK>(jt, [&](int b, int r, int e) {
        if (valid) o[e] = w[b][r];
    });
}

// ---------------------------------------------------------------------------
// The padded convolution along the contiguous axis as one length-M = 2N
// transform per line (2N <= 512): the first stage skips the zero half, the multiplier is applied in
// registers between the forward and the inverse, and only the first N points
// are stored.
// ---------------------------------------------------------------------------
// The multiplier of one convolution line at the positions of the forward
// transform's last stage: the stored row, or with QF the dipolar quadratic form
// evaluated from it.
template <typename R, int M, int TPL, int RK, int BK, bool QF>
__device__ __forceinline__ void conv_mult(R (&kq)[BK][RK], const R* mult, long row, int gl, const LineIdx& li,
                                          const QForm* qf, int jt) {
    if constexpr (QF) {
        QForm qd = *qf;
        if (qd.tp) qform_fill(qd, *qd.tp + qd.toff, qd.tau);
        const QForm* q = &qd;
        // row frequencies (signed; odd products vanish at Nyquist indices)
        const int k0 = gl / li.D1, k1r = gl % li.D1;
        const int k1 = (k1r <= q->n1) ? k1r : k1r - li.D1;
        const double a0 = k0 * q->dk0, a1 = k1 * q->dk1;
        const double x0 = (k0 == q->n0) ? 0.0 : a0, x1 = (k1r == q->n1) ? 0.0 : a1;
        const double base = q->m00 * a0 * a0 + q->m11 * a1 * a1 + 2.0 * q->m01 * x0 * x1;
        const double lin = 2.0 * (q->m02 * x0 + q->m12 * x1);
        for_pos<M, TPL, RK>(jt, [&](int b, int r, int p) {
            const int k2 = (p <= M / 2) ? p : p - M;
            const double a2 = k2 * q->dk2, x2 = (p == M / 2) ? 0.0 : a2;
            const double Q = base + q->m22 * a2 * a2 + lin * x2;
            kq[b][r] = R(q->c0 + (double)mult[row + min(p, M - p)] * Q);
        });
    } else {
        for_pos<M, TPL, RK>(jt, [&](int b, int r, int p) { kq[b][r] = mult[row + min(p, M - p)]; });
    }
}

template <typename R, int M, int V = 0, bool QF = false>
__device__ __forceinline__ void conv_full_body(
    typename CT<R>::T* data, int nlines, const R* mult, LineIdx li,
    const typename CT<R>::T* twM, int bx, int by, typename CT<R>::T* lds, const QForm* qf = nullptr) {
    using T = typename CT<R>::T;
    using C = LineCfg<R, M, false, V>;
    constexpr int P = C::P, TPL = C::TPL, LPB = C::LPB;
    constexpr int N = M / 2;
    constexpr bool WS = (64 % TPL) == 0;  // a line's threads share one wavefront
    constexpr bool XS = C::XS && !QF;  // (the quadratic form needs the registers more than the waves)
    using FF = Fft<T, M, false, TPL, LineFwd<M, V>, WS, 2, XS>;
    using FI = Fft<T, M, true, TPL, LineInv<M, V>, WS, 2, XS>;
    const int jt = threadIdx.x % TPL;
    // one line per wavefront (TPL = 64): the line index is uniform, so the
    // line and multiplier-row arithmetic stays in scalar registers and the
    // loads take a scalar base with 32-bit lane offsets
    const int dl = (TPL == 64) ? __builtin_amdgcn_readfirstlane(threadIdx.x / TPL) : threadIdx.x / TPL;
    const int gv = ((LPB == 1) ? xcd_pairs(bx, gridDim.x) : bx) * LPB + dl;
    const bool valid = gv < nlines;
    const int gl = valid ? line_at(gv, li) : 0;
    // (with split exchanges a line is P scalars)
    T* line = XS ? reinterpret_cast<T*>(reinterpret_cast<R*>(lds) + dl * P) : lds + dl * P;
    T* g = data + (long)gl * N;
    typename FF::In v;
    typename FF::Out u;
    // (a line past the end reads line 0 and stores nothing)
    for_pos<M, TPL, FF::R0>(jt, [&](int b, int r, int e) { v[b][r] = (e < N) ? g[e] : T{0, 0}; });
    const long row = mult_row(gl, li);
    R kq[FF::BK][FF::RK];
    // the multiplier row is read while the forward transform runs, except with
    // split exchanges, which need those registers to fit the occupancy their
    // LDS allows
    if constexpr (!XS) conv_mult<R, M, TPL, FF::RK, FF::BK, QF>(kq, mult, row, gl, li, qf, jt);
    // FP32 (bound by VALU issue) with a palindromic plan: the inverse takes the
    // forward's twiddles from registers
    constexpr bool KEEP = sizeof(R) == 4 && std::is_same<LineFwd<M, V>, LineInv<M, V>>::value;
    typename FF::Keep keep;
    if constexpr (KEEP) FF::template run_tw<TW_KEEP>(v, u, line, jt, twM, keep);
    else FF::run(v, u, line, jt, twM);
    if constexpr (XS) conv_mult<R, M, TPL, FF::RK, FF::BK, QF>(kq, mult, row, gl, li, qf, jt);
    for_pos<M, TPL, FF::RK>(jt, [&](int b, int r, int) {
        u[b][r] = T{u[b][r].x * kq[b][r], u[b][r].y * kq[b][r]};
    });
    typename FI::Out w;
    lds_sync<WS>();
    if constexpr (KEEP) FI::template run_tw<TW_REUSE>(u, w, line, jt, twM, keep);
    else FI::run(u, w, line, jt, twM);
    for_pos<M, TPL, FI::RK>(jt, [&](int b, int r, int e) {
        if (valid && e < N) g[e] = w[b][r];
    });
}

// The padded convolution with the quadratic-form dipolar multiplier (QForm).
template <typename R, int M>
__global__ __launch_bounds__((LineCfg<R, M, false>::NTH)) void k_conv_qf(
    typename CT<R>::T* data, int nlines, const R* mult, LineIdx li,
    const typename CT<R>::T* twM, QForm q) {
    __shared__ typename CT<R>::T lds[LineCfg<R, M, false>::LPB * LineCfg<R, M, false>::P];
    conv_full_body<R, M, 0, true>(data, nlines, mult, li, twM, blockIdx.x, blockIdx.y, lds, &q);
}

template <typename R, int M, int V = 0>
__global__ __launch_bounds__((LineCfg<R, M, false, V>::NTH)) void k_conv_full(
    typename CT<R>::T* data, int nlines, const R* mult, LineIdx li,
    const typename CT<R>::T* twM) {
    __shared__ typename CT<R>::T lds[LineCfg<R, M, false, V>::LDS];
    conv_full_body<R, M, V>(data, nlines, mult, li, twM, blockIdx.x, blockIdx.y, lds);
}

// The same with split exchanges (LineCfg::XS), at the occupancy their LDS
// allows within the registers (a kernel of its own: the occupancy request
// changes the register allocation of every kernel it is attached to).
template <typename R, int M>
__global__ __launch_bounds__((LineCfg<R, M, false>::NTH))
__attribute__((amdgpu_waves_per_eu(LineCfg<R, M, false>::OCC, 8))) void k_conv_xs(
    typename CT<R>::T* data, int nlines, const R* mult, LineIdx li,
    const typename CT<R>::T* twM) {
    static_assert(LineCfg<R, M, false>::XS, "split-exchange configuration only");
    __shared__ typename CT<R>::T lds[LineCfg<R, M, false>::LDS];
    conv_full_body<R, M, 0>(data, nlines, mult, li, twM, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Axis-0 density + padded real-to-complex FFT (column tiles over the C =
// n/N0 columns).
//   SRC 0: input is the state with the axis-0 inverse FFT pending;
//   SRC 1: input is psi in physical space;
//   SRC 2: input is a real density array.
// Output X1[k][c], k = 0..N0: the length-2N0 DFT of (rho_0..rho_{N0-1}, 0..0)
// at non-negative frequencies, from Z = FFT_N0(rho_2m + i rho_2m+1) (zero for
// m >= N0/2):
//   X_k = (Z_k + conj Z_{N0-k})/2 + exp(-i pi k/N0) (Z_k - conj Z_{N0-k})/(2i).
// ---------------------------------------------------------------------------
template <typename R, int N0, int SRC, int CV = 0>
__device__ __forceinline__ void r2c_body(const void* src, typename CT<R>::T* X1,
                                                            int C, const typename CT<R>::T* twN,
                                                            const typename CT<R>::T* tw2N, int bx, int by, typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    using Cf = ColCfg<R, N0, ColPlan<N0, CV>>;
    constexpr int W = Cf::W, TPL = Cf::TPL;
    constexpr int P = pitch_cols<N0>(N0 + 1);
    using FI = Fft<T, N0, true, TPL, ColPlan<N0, CV>>;
    using FF = Fft<T, N0, false, TPL, ColPlan<N0, CV>>;
    const int l = threadIdx.x % W, jt = threadIdx.x / W;
    const int col0 = bx * W;
    const bool lv = (col0 + l) < C;
    T* line = lds + l * P;
    // FP32: the forward transform of the packed density has the stages of the
    // state's inverse and takes its twiddles from registers
    constexpr bool KEEP = SRC == 0 && sizeof(R) == 4;
    typename FI::Keep keep;
    // density at the thread's positions, then into LDS (real part)
    if constexpr (SRC == 0) {
        const T* g = static_cast<const T*>(src) + col0 + l;
        typename FI::In v;
        typename FI::Out u;
        for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int e) { v[b][r] = lv ? g[(long)e * C] : T{0, 0}; });
        if constexpr (KEEP) FI::template run_tw<TW_KEEP>(v, u, line, jt, twN, keep);
        else FI::run(v, u, line, jt, twN);
        __syncthreads();
        for_pos<N0, TPL, FI::RK>(jt, [&](int b, int r, int e) {
            line[padx<N0>(e)].x = u[b][r].x * u[b][r].x + u[b][r].y * u[b][r].y;
        });
    } else if constexpr (SRC == 1) {
        const T* g = static_cast<const T*>(src) + col0 + l;
        for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int e) {
            const T x = lv ? g[(long)e * C] : T{0, 0};
            line[padx<N0>(e)].x = x.x * x.x + x.y * x.y;
        });
    } else {
        const R* g = static_cast<const R*>(src) + col0 + l;
        for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int e) { line[padx<N0>(e)].x = lv ? g[(long)e * C] : R(0); });
    }
    __syncthreads();
    typename FF::In z;
    typename FF::Out Z;
    for_pos<N0, TPL, FF::R0>(jt, [&](int b, int r, int m) {
        z[b][r] = (m < N0 / 2) ? T{line[padx<N0>(2 * m)].x, line[padx<N0>(2 * m + 1)].x} : T{0, 0};
    });
    __syncthreads();
    if constexpr (KEEP) FF::template run_tw<TW_REUSE>(z, Z, line, jt, twN, keep);
    else FF::run(z, Z, line, jt, twN);
    __syncthreads();
    for_pos<N0, TPL, FF::RK>(jt, [&](int b, int r, int k) { line[padx<N0>(k)] = Z[b][r]; });
    __syncthreads();
    T* gout = X1 + col0 + l;
    // exp(-i pi k/N0) for k = jt + i*TPL as tw2N[jt] * tw2N[i*TPL]: one table
    // read per thread, the second factor is the same for every lane
    const T wj = tw2N[jt];
    for_rows_incl<N0, TPL>(jt, [&](int i, int k) {
        const T zk = line[padx<N0>(k == N0 ? 0 : k)];
        const T zc = cconj(line[padx<N0>(k == 0 ? 0 : N0 - k)]);
        const T ev = T{R(0.5) * (zk.x + zc.x), R(0.5) * (zk.y + zc.y)};
        const T dv = csub(zk, zc);
        const T ov = T{R(0.5) * dv.y, -R(0.5) * dv.x};  // (zk - zc)/(2i)
        if (lv) gout[(long)k * C] = cadd(ev, cmul(cmul(wj, tw2N[i * TPL]), ov));
    });
}

template <typename R, int N0, int SRC, int CV = 0>
__global__ __launch_bounds__((ColCfg<R, N0, ColPlan<N0, CV>>::NTH))
FSE_COL_OCC(R, N0, ColCfg<R, N0>::W * pitch_cols<N0>(N0 + 1) * csz<R>(), ColCfg<R, N0, ColPlan<N0, CV>>::NTH)
void k_r2c(const void* src, typename CT<R>::T* X1,
                                                            int C, const typename CT<R>::T* __restrict__ twN,
                                                            const typename CT<R>::T* __restrict__ tw2N) {
    __shared__ typename CT<R>::T lds[ColCfg<R, N0>::W * pitch_cols<N0>(N0 + 1)];
    r2c_body<R, N0, SRC, CV>(src, X1, C, twN, tw2N, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Axis-0 complex-to-real inverse (nonlocal potential) fused with the
// nonlinear sub-step (column tiles).
//   MODE 0: Phi from X1; state S (axis-0 inverse pending) -> psi -> phase
//           -> forward FFT of axis 0 -> S.
//   MODE 1: no nonlocal term: psi -> phase -> forward FFT of axis 0.
//   MODE 2: Phi only, written to Phi_out[e][c] (real).
// Inverse real transform of the Hermitian half X_0..X_N0 (length 2N0):
//   Z'_k = (X_k + conj X_{N0-k}) + i exp(+i pi k/N0) (X_k - conj X_{N0-k}),
//   y = IFFT_N0(Z') unnormalised, Phi_{2m} = Re y_m, Phi_{2m+1} = Im y_m.
// The GauSum multiplier already carries 1/prod(2 N_j).
// ---------------------------------------------------------------------------
template <typename R, int N0, int MODE, int FV = 0>
__device__ __forceinline__ void c2r_phase_body(const typename CT<R>::T* X1,
                                                                  typename CT<R>::T* S, R* Phi_out,
                                                                  int C, PhaseArgs pa,
                                                                  const typename CT<R>::T* twN,
                                                                  const typename CT<R>::T* tw2N, int bx, int by, typename CT<R>::T* lds) {
    using T = typename CT<R>::T;
    using PL = typename PlanOf<N0, typename FusedPlan<R, N0, FV>::L>::L;
    using Cf = FusedCfg<R, N0, FV>;
    constexpr int W = Cf::W, TPL = Cf::TPL;
    constexpr int P = pitch_cols<N0>(N0 + 1);
    using FI = Fft<T, N0, true, TPL, PL>;                    // inverse transforms, outputs at radix-RK positions
    using FF = Fft<T, N0, false, TPL, typename Rev<PL>::L>;  // forward after the phase, inputs at radix-RK positions
    const int l = threadIdx.x % W, jt = threadIdx.x / W;
    const int col0 = bx * W;
    const bool lv = (col0 + l) < C;
    T* line = lds + l * P;
    R phi[FI::BK][FI::RK];
    if constexpr (MODE != 1) {
        const T* gx = X1 + col0 + l;
        {
            T xr[(N0 + TPL) / TPL];
            for_rows_incl<N0, TPL>(jt, [&](int i, int k) { xr[i] = lv ? gx[(long)k * C] : T{0, 0}; });
            for_rows_incl<N0, TPL>(jt, [&](int i, int k) { line[padx<N0>(k)] = xr[i]; });
        }
        __syncthreads();
        typename FI::In zc;
        typename FI::Out y;
        // exp(-i pi k/N0) for k = j + r*N0/R0 as tw2N[j] * tw2N[r*N0/R0] (the
        // second factor is the same for every lane)
        T wj[FI::B0];
        for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int k) {
            if (r == 0) wj[b] = tw2N[k];
        });
        for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int k) {
            const T xk = line[padx<N0>(k)];
            const T xc = cconj(line[padx<N0>(N0 - k)]);
            const T a = cadd(xk, xc);
            const T w = (r == 0) ? wj[b] : cmul(wj[b], tw2N[r * (N0 / FI::R0)]);
            const T bb = cmulc(csub(xk, xc), w);  // exp(+i pi k/N0) (xk - xc)
            zc[b][r] = T{a.x - bb.y, a.y + bb.x};       // a + i bb
        });
        __syncthreads();
        FI::run(zc, y, line, jt, twN);
        __syncthreads();
        // only y_m with m < N0/2 carry the physical samples Phi_0..Phi_{N0-1}
        for_pos<N0, TPL, FI::RK>(jt, [&](int b, int r, int m) {
            if (m < N0 / 2) {
                line[padx<N0>(2 * m)].x = y[b][r].x;
                line[padx<N0>(2 * m + 1)].x = y[b][r].y;
            }
        });
        __syncthreads();
        if constexpr (MODE == 2) {
            R* go = Phi_out + col0 + l;
            for_rows_incl<N0 - 1, TPL>(jt, [&](int, int e) {
                if (lv) go[(long)e * C] = line[padx<N0>(e)].x;
            });
            return;
        }
        for_pos<N0, TPL, FI::RK>(jt, [&](int b, int r, int e) { phi[b][r] = line[padx<N0>(e)].x; });
        __syncthreads();
    } else {
#pragma unroll
        for (int b = 0; b < FI::BK; ++b)
#pragma unroll
            for (int r = 0; r < FI::RK; ++r) phi[b][r] = R(0);
    }
    if constexpr (MODE != 2) {
        typename FI::Out psi;
        typename FI::In vs;
        {
            const T* g = S + col0 + l;
            for_pos<N0, TPL, FI::R0>(jt, [&](int b, int r, int e) { vs[b][r] = lv ? g[(long)e * C] : T{0, 0}; });
        }
        FI::run(vs, psi, line, jt, twN);
        const int c = col0 + l;
        R yv, zv;
        if (pa.N2 > 0) {
            yv = R(pa.y0 + (c / pa.N2) * pa.hy);
            zv = R(pa.z0 + (c % pa.N2) * pa.hz);
        } else {
            yv = R(pa.y0 + c * pa.hy);
            zv = R(0);
        }
        double pcc, pcs;
        phase_time(pa, &pcc, &pcs);
        const R y2 = yv * yv;
        const R base = R(pa.cz) * (zv * zv) + R(pa.ca - pcc) * y2;
        const R* Ux = static_cast<const R*>(pa.U);
        for_pos<N0, TPL, FI::RK>(jt, [&](int b, int r, int e) {
            const R x = R(pa.x0 + e * pa.hx);
            const R Pv = base + R(pa.ca + pcc) * (x * x) + R(pcs) * (R(2) * x * yv);
            const T v = psi[b][r];
            const R rho = v.x * v.x + v.y * v.y;
            R th = R(pa.bdt) * rho + R(pa.ldt) * phi[b][r] + Pv;
            if (Ux && lv) th += R(pa.udt) * Ux[(long)e * C + c];
            R sn, cs;
            fsincos(th, &sn, &cs);
            psi[b][r] = T{v.x * cs + v.y * sn, v.y * cs - v.x * sn};  // v * exp(-i th)
        });
        typename FF::Out out;
        __syncthreads();
        FF::run(psi, out, line, jt, twN);
        T* go = S + col0 + l;
        for_pos<N0, TPL, FF::RK>(jt, [&](int b, int r, int e) {
            if (lv) go[(long)e * C] = out[b][r];
        });
    }
}

template <typename R, int N0, int MODE, int FV = 0>
__global__ __launch_bounds__((FusedCfg<R, N0, FV>::NTH))
FSE_COL_OCC(R, N0, FusedCfg<R, N0, FV>::W * pitch_cols<N0>(N0 + 1) * csz<R>(), FusedCfg<R, N0, FV>::NTH)
void k_c2r_phase(const typename CT<R>::T* X1,
                                                                  typename CT<R>::T* S, R* Phi_out,
                                                                  int C, PhaseArgs pa,
                                                                  const typename CT<R>::T* __restrict__ twN,
                                                                  const typename CT<R>::T* __restrict__ tw2N) {
    __shared__ typename CT<R>::T lds[FusedCfg<R, N0, FV>::W * pitch_cols<N0>(N0 + 1)];
    c2r_phase_body<R, N0, MODE, FV>(X1, S, Phi_out, C, pa, twN, tw2N, blockIdx.x, blockIdx.y, lds);
}

// ---------------------------------------------------------------------------
// Batched 2D passes: blockIdx.y selects the instance of a group of equal-size
// instances; the tile index is blockIdx.x as in the single-instance kernels.
//   KIND 0 / 1: forward / inverse FFT of axis 0 (column tiles over N1)
//   KIND 2:     kinetic line pass (which = 0: dt/2 table, 1: dt table)
//   KIND 3:     density + padded real-to-complex FFT of axis 0
//   KIND 4:     padded convolution along axis 1
//   KIND 5 / 6: complex-to-real + nonlinear phase (with / without nonlocal
//               term) at t_n = *t + which * dt
// ---------------------------------------------------------------------------
__device__ __forceinline__ PhaseArgs batch_phase(const BInst& b, int kstep) {
    const double tn = *b.t + kstep * b.dt;
    PhaseArgs pa;
    pa.x0 = b.x0;
    pa.hx = b.hx;
    pa.y0 = b.y0;
    pa.hy = b.hy;
    pa.z0 = 0.0;
    pa.hz = 0.0;
    pa.N2 = 0;
    pa.ca = b.ca;
    pa.cz = 0.0;
    trap_rotating_dev(tn, b.dt, b.Omega, b.gdiff, b.sf, &pa.cc, &pa.cs);
    pa.bdt = b.bdt;
    pa.ldt = b.ldt;
    pa.U = nullptr;
    pa.udt = 0.0;
    return pa;
}

template <typename R, int N0, bool INV>
__global__ __launch_bounds__((ColCfg<R, N0>::NTH))
FSE_COL_OCC(R, N0, ColCfg<R, N0>::W * pitch_cols<N0>(N0) * csz<R>(), ColCfg<R, N0>::NTH)
void k_b_cols(void* psi, const BInst* bi, int N1,
                                                                const typename CT<R>::T* twN0, int scaled) {
    using T = typename CT<R>::T;
    T* x = static_cast<T*>(psi) + bi[blockIdx.y].psi_off;
    __shared__ typename CT<R>::T lds[ColCfg<R, N0>::W * pitch_cols<N0>(N0)];
    // scaled: the exit pass applies the instance's mass renormalisation factor
    cols_body<R, N0, INV>(x, x, N1, twN0, blockIdx.x, 0, lds, scaled ? bi[blockIdx.y].rn + 1 : nullptr);
}

template <typename R, int N1>
__global__ __launch_bounds__((LineCfg<R, N1, false>::NTH)) void k_b_kin(void* psi, const BInst* bi,
                                                                       int N0, int which, LineIdx li,
                                                                       const typename CT<R>::T* twN1) {
    using T = typename CT<R>::T;
    const BInst& b = bi[blockIdx.y];
    __shared__ typename CT<R>::T lds[LineCfg<R, N1, (1) == 0>::LPB * LineCfg<R, N1, (1) == 0>::SUB * LineCfg<R, N1, (1) == 0>::P];
    lines_body<R, N1, 1>(static_cast<T*>(psi) + b.psi_off, N0, which ? b.kin1 : b.kin0, li, twN1, nullptr, blockIdx.x,
                         0, lds);
}

template <typename R, int N0>
__global__ __launch_bounds__((ColCfg<R, N0>::NTH))
FSE_COL_OCC(R, N0, ColCfg<R, N0>::W * pitch_cols<N0>(N0 + 1) * csz<R>(), ColCfg<R, N0>::NTH)
void k_b_r2c(void* psi, const BInst* bi, int N1,
                                                               const typename CT<R>::T* __restrict__ twN0,
                                                               const typename CT<R>::T* __restrict__ tw2N0) {
    using T = typename CT<R>::T;
    const BInst& b = bi[blockIdx.y];
    __shared__ typename CT<R>::T lds[ColCfg<R, N0>::W * pitch_cols<N0>(N0 + 1)];
    r2c_body<R, N0, 0>(static_cast<const T*>(psi) + b.psi_off, static_cast<T*>(b.X1), N1, twN0, tw2N0, blockIdx.x, 0, lds);
}

template <typename R, int M>
__global__ __launch_bounds__((LineCfg<R, M, false>::NTH)) void k_b_conv_full(const BInst* bi, int nlines,
                                                                            LineIdx li,
                                                                            const typename CT<R>::T* twM) {
    using T = typename CT<R>::T;
    const BInst& b = bi[blockIdx.y];
    __shared__ typename CT<R>::T lds[LineCfg<R, M, false>::LDS];
    conv_full_body<R, M>(static_cast<T*>(b.X1), nlines, static_cast<const R*>(b.khat), li, twM, blockIdx.x, 0, lds);
}

template <typename R, int N1>
__global__ __launch_bounds__((LineCfg<R, N1, true>::NTH)) void k_b_conv_halves(
    const BInst* bi, int nlines, LineIdx li, const typename CT<R>::T* twN1,
    const typename CT<R>::T* tw2N1) {
    using T = typename CT<R>::T;
    const BInst& b = bi[blockIdx.y];
    __shared__ typename CT<R>::T lds[LineCfg<R, N1, (0) == 0>::LPB * LineCfg<R, N1, (0) == 0>::SUB * LineCfg<R, N1, (0) == 0>::P];
    lines_body<R, N1, 0>(static_cast<T*>(b.X1), nlines, b.khat, li, twN1, tw2N1, blockIdx.x, 0, lds);
}

template <typename R, int N0, int MODE>
__global__ __launch_bounds__((FusedCfg<R, N0>::NTH))
FSE_COL_OCC(R, N0, FusedCfg<R, N0>::W * pitch_cols<N0>(N0 + 1) * csz<R>(), FusedCfg<R, N0>::NTH)
void k_b_c2r_phase(void* psi, const BInst* bi,
                                                                     int N1, int kstep,
                                                                     const typename CT<R>::T* __restrict__ twN0,
                                                                     const typename CT<R>::T* __restrict__ tw2N0) {
    using T = typename CT<R>::T;
    const BInst& b = bi[blockIdx.y];
    const PhaseArgs pa = batch_phase(b, kstep);
    __shared__ typename CT<R>::T lds[FusedCfg<R, N0>::W * pitch_cols<N0>(N0 + 1)];
    c2r_phase_body<R, N0, MODE>(static_cast<const T*>(b.X1), static_cast<T*>(psi) + b.psi_off, nullptr, N1, pa, twN0,
                                tw2N0, blockIdx.x, 0, lds);
}

// Advances every instance's time by nsteps * dt (one thread per instance).
static __global__ void k_b_time(const BInst* __restrict__ bi, int count, int nsteps) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) *bi[i].t += nsteps * bi[i].dt;
}

// Advances a plan's device time by dtot (one thread).
static __global__ void k_time_add(double* t, double dtot) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *t += dtot;
}

// ---------------------------------------------------------------------------
// Kinetic phase table Q[k0][k1][k2] = scale * exp(-i tau omega/2),
// omega = (|mu|^2 + m^2)^s, mu_j = k_j * dmu_j, k_j = 0..N_j/2 (the table is
// even in each frequency index).  FP64 arithmetic, rounded to the path type.
// kind 1: the real resolvent scale / (c0 + omega/2) instead; kind 2: the real
// symbol scale * omega/2.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_build_kin(typename CT<R>::T* __restrict__ Q, int T0, int T1, int T2, double dmu0, double dmu1,
                            double dmu2, double s, double m2, int kind, double tau, double c0, double scale) {
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
        if (kind == 1) {  // resolvent [c0 + omega/2]^{-1} (the P_Delta preconditioner, c0 = 1/dt)
            Q[i] = T{R(scale / (c0 + 0.5 * om)), R(0)};
            continue;
        }
        if (kind == 2) {  // the kinetic symbol omega/2 itself
            Q[i] = T{R(scale * 0.5 * om), R(0)};
            continue;
        }
        double sn, cs;
        sincos(-0.5 * tau * om, &sn, &cs);
        if constexpr (sizeof(R) == 4) {
            // The same entry multiplies the same mode every step, so a bias in
            // its magnitude accumulates in the mass: of the four FP32 pairs that
            // bracket (cx, cy), take the one whose squared modulus is closest.
            const double cx = scale * cs, cy = scale * sn, tgt = cx * cx + cy * cy;
            const float x0 = (float)cx, y0 = (float)cy;
            const float xs[2] = {x0, ((double)x0 < cx) ? nextafterf(x0, 2.0f) : nextafterf(x0, -2.0f)};
            const float ys[2] = {y0, ((double)y0 < cy) ? nextafterf(y0, 2.0f) : nextafterf(y0, -2.0f)};
            float bx = x0, by = y0;
            double best = fabs((double)x0 * x0 + (double)y0 * y0 - tgt);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const double e = fabs((double)xs[a] * xs[a] + (double)ys[b] * ys[b] - tgt);
                    if (e < best) {
                        best = e;
                        bx = xs[a];
                        by = ys[b];
                    }
                }
            Q[i] = T{bx, by};
        } else {
            Q[i] = T{R(scale * cs), R(scale * sn)};
        }
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
// W = wa (x^2+y^2) + wz z^2 + wc (x^2-y^2) + ws 2xy, plus U when given.
// With tp set, wc = gd cos(2 Omega t) and ws = gd sin(2 Omega t) at the device time t = *tp.
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_red_local(const typename CT<R>::T* __restrict__ psi,
                                                           const R* __restrict__ Phi, const R* __restrict__ U, long n,
                                                           GridGeom g, double wa, double wz, double wc, double ws,
                                                           const double* tp, double Om, double gd,
                                                           double* partials, int slot0) {
    if (tp) {
        double s2, c2;
        fsincos(2.0 * Om * *tp, &s2, &c2);
        wc = gd * c2;
        ws = gd * s2;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const auto v = psi[i];
        const double rho = (double)v.x * v.x + (double)v.y * v.y;
        double Wv = wa * (x * x + y * y) + wz * z * z + wc * (x * x - y * y) + ws * 2.0 * x * y;
        if (U) Wv += (double)U[i];
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

// Moments of rho = |psi|^2 on the rotating-frame grid: slots 0 sum rho,
// 1..3 sum x~_j rho, 4..6 sum x~_j^2 rho, 7 sum x~ y~ rho (z terms 0 in 2D).
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_red_moments(const typename CT<R>::T* __restrict__ psi, long n,
                                                             GridGeom g, double* partials) {
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const auto v = psi[i];
        const double rho = (double)v.x * v.x + (double)v.y * v.y;
        const double xr = x * rho, yr = y * rho, zr = z * rho;
        acc[0] += rho;
        acc[1] += xr;
        acc[2] += yr;
        acc[3] += zr;
        acc[4] += x * xr;
        acc[5] += y * yr;
        acc[6] += z * zr;
        acc[7] += x * yr;
    }
    block_reduce_store<8>(acc, partials, 0, gridDim.x);
}

// Lab-frame mass, centre of mass and widths (eqs. mass, CoM, ConWidth) from
// the eight moment slots, with x = A x~, A = [[c, s], [-s, c]] on (x, y):
//   out = {N, x_c, y_c, z_c, delta_x, delta_y, delta_z}.  One block.
static __global__ __launch_bounds__(RED_THREADS) void k_moments_final(const double* __restrict__ partials, int nblk,
                                                               double vol, double c, double s, const double* tp,
                                                               double Om, double* out) {
    if (tp) {  // frame angle Omega t at the device time
        c = cos(Om * *tp);
        s = sin(Om * *tp);
    }
    __shared__ double tot[8];
    __shared__ double red[RED_THREADS / 64];
    for (int k = 0; k < 8; ++k) {
        double x = 0.0;
        for (int b = threadIdx.x; b < nblk; b += RED_THREADS) x += partials[(long)k * nblk + b];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
            tot[k] = vol * t;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mx = tot[1], my = tot[2], sxx = tot[4], syy = tot[5], sxy = tot[7];
        out[0] = tot[0];
        out[1] = c * mx + s * my;
        out[2] = -s * mx + c * my;
        out[3] = tot[3];
        out[4] = c * c * sxx + 2.0 * c * s * sxy + s * s * syy;
        out[5] = s * s * sxx - 2.0 * c * s * sxy + c * c * syy;
        out[6] = tot[6];
    }
}

// Mass renormalisation factor: r = {M_ref, f, M}; f = sqrt(M_ref / (mscale * M)) with M the FP64 sum
// of the nblk partials times vol, or 1 if that is zero or not finite (one block).
static __global__ __launch_bounds__(RED_THREADS) void k_renorm_factor(const double* __restrict__ partials, int nblk,
                                                                      double vol, double mscale, double* r) {
    __shared__ double red[RED_THREADS / 64];
    double x = 0.0;
    for (int b = threadIdx.x; b < nblk; b += RED_THREADS) x += partials[b];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
        const double M = mscale * vol * t;
        const double f = sqrt(r[0] / M);
        r[2] = M;
        r[1] = (M > 0.0 && isfinite(f)) ? f : 1.0;
    }
}

// Batched FP64 mass of the instances of a group (grid.y = instance within the
// group, n points each): per-block partial sums of |psi|^2 into
// partials[instance * gridDim.x + block].
template <typename R>
__global__ __launch_bounds__(RED_THREADS) void k_b_mass_part(const void* psi, const BInst* __restrict__ bi, long n,
                                                             double* __restrict__ partials) {
    using T = typename CT<R>::T;
    __shared__ double red[RED_THREADS / 64];
    const T* x = static_cast<const T*>(psi) + bi[blockIdx.y].psi_off;
    double acc = 0.0;
    for (long i = blockIdx.x * (long)RED_THREADS + threadIdx.x; i < n; i += (long)gridDim.x * RED_THREADS) {
        const T v = x[i];
        acc += (double)v.x * (double)v.x + (double)v.y * (double)v.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
        partials[(long)blockIdx.y * gridDim.x + blockIdx.x] = t;
    }
}

// One block per instance of the group: M = mscale * hx * hy * (sum of its
// partials).  slot 0: rn[0] = M (the mass at the call's start); slot 1:
// rn[2] = M and rn[1] = sqrt(rn[0] / M), the factor the exit pass applies (1
// when M is zero or the factor is not finite).
static __global__ __launch_bounds__(RED_THREADS) void k_b_mass_final(const double* __restrict__ partials, int nblk,
                                                                     const BInst* __restrict__ bi, double mscale,
                                                                     int slot) {
    __shared__ double red[RED_THREADS / 64];
    const BInst& b = bi[blockIdx.x];
    double x = 0.0;
    for (int k = threadIdx.x; k < nblk; k += RED_THREADS) x += partials[(long)blockIdx.x * nblk + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RED_THREADS / 64; ++w) t += red[w];
        const double M = mscale * b.hx * b.hy * t;
        if (slot == 0) {
            b.rn[0] = M;
        } else {
            const double f = sqrt(b.rn[0] / M);
            b.rn[2] = M;
            b.rn[1] = (M > 0.0 && isfinite(f)) ? f : 1.0;
        }
    }
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
// Elementwise helper for H*psi.
// ---------------------------------------------------------------------------
// H psi accumulation:
//   WHAT 0: H += i Omega x D  (D = D_y psi)
//   WHAT 1: H += -i Omega y D (D = D_x psi)
//   WHAT 2: H += (V + beta rho + lam Phi) psi, rho = |psi|^2 or rho_in.
// For WHAT 0 and 1, Omega is multiplied by *wscale when wscale is not null.
template <typename R>
__global__ void k_H_accum(typename CT<R>::T* __restrict__ H, const typename CT<R>::T* __restrict__ D,
                          const typename CT<R>::T* __restrict__ psi, const R* __restrict__ rho_in,
                          const R* __restrict__ Phi, const R* __restrict__ U, long n, GridGeom g, int what,
                          double Omega, double beta, double lam, double g0, double g1, double g2,
                          const double* __restrict__ wscale) {
    using T = typename CT<R>::T;
    if (wscale) Omega *= *wscale;
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
            const double f = V + beta * rho + (Phi ? lam * (double)Phi[i] : 0.0) + (U ? (double)U[i] : 0.0);
            h = T{R(h.x + f * v.x), R(h.y + f * v.y)};
        }
        H[i] = h;
    }
}

// Lattice potential or its time integral (LatArgs), plus uf U when U is given; FP64 inside.
template <typename R>
__global__ void k_lattice(R* __restrict__ out, const R* __restrict__ U, long n, GridGeom g, LatArgs la) {
    if (la.tp) lat_fill(la, *la.tp + la.toff);
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        int i0, i1, i2;
        decode(i, g, i0, i1, i2);
        const double x = g.x0 + i0 * g.hx, y = g.y0 + i1 * g.hy, z = (g.d == 3) ? g.z0 + i2 * g.hz : 0.0;
        const double sz = (la.v[2] != 0.0) ? sin(la.k[2] * z) : 0.0;
        double acc = 0.0;
        for (int q = 0; q < la.nq; ++q) {
            const double xr = la.c[q] * x + la.s[q] * y, yr = -la.s[q] * x + la.c[q] * y;
            const double sx = sin(la.k[0] * xr), sy = sin(la.k[1] * yr);
            acc += la.w[q] * (la.v[0] * sx * sx + la.v[1] * sy * sy + la.v[2] * sz * sz);
        }
        if (U) acc += la.uf * (double)U[i];
        out[i] = R(acc);
    }
}

// Plain streaming copy (HBM bandwidth calibration): 16-byte vectors, each
// thread loads four elements 256 apart, then stores them; one pass, no loop.
// NT: non-temporal loads and stores (the data is not kept in the caches).
template <bool NT>
__global__ __launch_bounds__(256) void k_copy16(double2* dst, const double2* src, long n) {
    const long base = (long)blockIdx.x * 1024L + threadIdx.x;
    double2 v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const long i = base + 256L * u;
        if (i < n) {
            if constexpr (NT) {
                v[u].x = __builtin_nontemporal_load(&src[i].x);
                v[u].y = __builtin_nontemporal_load(&src[i].y);
            } else {
                // (component accesses: a whole-struct copy here made the compiler
                // move v into LDS)
                v[u].x = src[i].x;
                v[u].y = src[i].y;
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const long i = base + 256L * u;
        if (i < n) {
            if constexpr (NT) {
                __builtin_nontemporal_store(v[u].x, &dst[i].x);
                __builtin_nontemporal_store(v[u].y, &dst[i].y);
            } else {
                dst[i].x = v[u].x;
                dst[i].y = v[u].y;
            }
        }
    }
}

}  // namespace fse
