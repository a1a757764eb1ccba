// Device-side FFT building blocks for gfx950 (CDNA4, wave64).
//
// A line of length M is transformed by a mixed-radix Stockham autosort FFT
// with radices 2, 3, 4, 8, 16.  In stage s (radix R, Ns = product of the
// earlier radices) the thread owning butterfly j takes the R inputs at
// j + r*M/R, multiplies them by the twiddles W_{Ns R}^{(j mod Ns) r}, does a
// radix-R DFT in registers and produces outputs for positions
// (j/Ns)*Ns*R + j%Ns + r*Ns.
//
// Register-resident ends: the first stage takes its inputs from registers
// (loaded straight from HBM by the caller) and the last stage leaves its
// outputs in registers at positions j + r*M/R_last, which is also the input
// pattern of a first stage of radix R_last.  A forward transform with radix
// order (R0..Rk) followed by an inverse with the reversed order (Rk..R0)
// therefore needs no LDS traffic between them: a pointwise multiplier is
// applied in registers.  Only the exchanges between consecutive stages go
// through LDS.
//
// All transforms are unnormalised; forward uses exp(-2 pi i nk/M).
#pragma once
#include <hip/hip_runtime.h>

#include "fse_math.hpp"

namespace fse {

template <typename R> struct CT;
template <> struct CT<double> { using T = double2; };
template <> struct CT<float> { using T = float2; };

template <typename T> struct RealOf;
template <> struct RealOf<double2> { using R = double; };
template <> struct RealOf<float2> { using R = float; };

template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }
template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
    return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ T cmulc(T a, T b) {
    return T{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T> __device__ __forceinline__ T cconj(T a) { return T{a.x, -a.y}; }
template <typename T, typename S> __device__ __forceinline__ T cscale(T a, S s) { return T{a.x * s, a.y * s}; }
// Multiply by -i (forward) or +i (inverse).
template <bool INV, typename T> __device__ __forceinline__ T mul_ni(T a) {
    return INV ? T{-a.y, a.x} : T{a.y, -a.x};
}
// Twiddle multiply: w = exp(-2 pi i m/M) from the table; the inverse uses conj(w).
template <bool INV, typename T> __device__ __forceinline__ T twmul(T a, T w) {
    return INV ? cmulc(a, w) : cmul(a, w);
}

// ---------------------------------------------------------------------------
// Products with the butterflies' irrational constants (sqrt(1/2), cos and sin
// of pi/8, sqrt(3)/2).  In FP32 every such constant rounds below its exact
// value, so a product with it shrinks |z| by 1e-8 to 3e-8 relative, the same
// way in every transform: the mass of a complex64 state then decays by about
// 1e-7 per step.  The FP32 path therefore carries each constant as hi + lo
// (lo = the rounding residual) and adds the lo product inside the FMA of the
// hi product, whose product is exact there: the result is the correctly
// rounded product up to one unbiased rounding, and the decay goes away.  FP64
// keeps the plain product (its residual bias is ~1e-17).
// ---------------------------------------------------------------------------
template <typename R> struct KConst {
    R hi, lo;
    constexpr KConst(double c) : hi(R(c)), lo(sizeof(R) == 4 ? R(c - double(R(c))) : R(0)) {}
};

// x * c
template <typename R> __device__ __forceinline__ R kmul(R x, KConst<R> c) {
    if constexpr (sizeof(R) == 4) return fmaf(x, c.hi, x * c.lo);
    else return x * c.hi;
}

// a * (cr + i ci) for a constant rotation
template <typename T, typename R> __device__ __forceinline__ T krot(T a, KConst<R> cr, KConst<R> ci) {
    if constexpr (sizeof(R) == 4) {
        const R tr = a.x * cr.lo - a.y * ci.lo;
        const R ti = a.x * ci.lo + a.y * cr.lo;
        return T{fmaf(a.x, cr.hi, fmaf(-a.y, ci.hi, tr)), fmaf(a.x, ci.hi, fmaf(a.y, cr.hi, ti))};
    } else {
        return T{a.x * cr.hi - a.y * ci.hi, a.x * ci.hi + a.y * cr.hi};
    }
}

// ---------------------------------------------------------------------------
// Radix-R DFTs in registers.
// ---------------------------------------------------------------------------
template <int R, bool INV> struct DFT;

template <bool INV> struct DFT<2, INV> {
    template <typename T> __device__ __forceinline__ static void run(T* v) {
        T a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <bool INV> struct DFT<3, INV> {
    template <typename T> __device__ __forceinline__ static void run(T* v) {
        using R = typename RealOf<T>::R;
        constexpr KConst<R> s3(0.86602540378443864676372317075294);  // sqrt(3)/2
        T s = cadd(v[1], v[2]);
        T dd = mul_ni<INV>(csub(v[1], v[2]));
        T a = T{v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y};
        T b = T{kmul(dd.x, s3), kmul(dd.y, s3)};  // -i sqrt(3)/2 (v1 - v2) forward
        v[0] = cadd(v[0], s);
        v[1] = cadd(a, b);
        v[2] = csub(a, b);
    }
};

template <bool INV> struct DFT<4, INV> {
    template <typename T> __device__ __forceinline__ static void run(T* v) {
        T t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
        T t2 = cadd(v[1], v[3]), t3 = mul_ni<INV>(csub(v[1], v[3]));
        v[0] = cadd(t0, t2);
        v[2] = csub(t0, t2);
        v[1] = cadd(t1, t3);
        v[3] = csub(t1, t3);
    }
};

template <bool INV> struct DFT<8, INV> {
    template <typename T> __device__ __forceinline__ static void run(T* v) {
        using R = typename RealOf<T>::R;
        constexpr KConst<R> c(0.70710678118654752440084436210485);  // sqrt(1/2)
        T e[4] = {v[0], v[2], v[4], v[6]};
        T o[4] = {v[1], v[3], v[5], v[7]};
        DFT<4, INV>::run(e);
        DFT<4, INV>::run(o);
        // o[k] *= W8^k, W8 = exp(-+ i pi/4)
        T o1 = INV ? T{kmul(o[1].x - o[1].y, c), kmul(o[1].x + o[1].y, c)}
                   : T{kmul(o[1].x + o[1].y, c), kmul(o[1].y - o[1].x, c)};
        T o2 = mul_ni<INV>(o[2]);
        T o3 = INV ? T{-kmul(o[3].x + o[3].y, c), kmul(o[3].x - o[3].y, c)}
                   : T{kmul(o[3].y - o[3].x, c), -kmul(o[3].x + o[3].y, c)};
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[5] = csub(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[6] = csub(e[2], o2);
        v[3] = cadd(e[3], o3);
        v[7] = csub(e[3], o3);
    }
};

template <bool INV> struct DFT<16, INV> {
    template <typename T> __device__ __forceinline__ static void run(T* v) {
        using R = typename RealOf<T>::R;
        // cos(pi m / 8) and sin(pi m / 8), m = 0..9
        constexpr double C1 = 0.92387953251128675612818318939679;
        constexpr double S1 = 0.38268343236508977172845998403040;
        constexpr double C2 = 0.70710678118654752440084436210485;
        // Y[n2][k1] = DFT4 over n1 of v[4 n1 + n2]
        T y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
            T t[4] = {v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]};
            DFT<4, INV>::run(t);
#pragma unroll
            for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = t[k1];
        }
        // twiddles W16^{n2 k1}
        constexpr double cs[10] = {1.0, C1, C2, S1, 0.0, -S1, -C2, -C1, -1.0, -C1};
        constexpr double sn[10] = {0.0, S1, C2, C1, 1.0, C1, C2, S1, 0.0, -S1};
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                const int m = n2 * k1;
                if (m == 4) {
                    y[n2][k1] = mul_ni<INV>(y[n2][k1]);  // W16^4 = -+i
                } else {
                    y[n2][k1] = krot<T, R>(y[n2][k1], KConst<R>(cs[m]), KConst<R>(INV ? sn[m] : -sn[m]));
                }
            }
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            T t[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            DFT<4, INV>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
        }
    }
};

// ---------------------------------------------------------------------------
// Radix schedules (products equal M) and type-level helpers.
// ---------------------------------------------------------------------------
template <int... Rs> struct RList {};
template <int M> struct Radix;
template <> struct Radix<16> { using L = RList<16>; };
template <> struct Radix<24> { using L = RList<8, 3>; };
template <> struct Radix<32> { using L = RList<8, 4>; };
template <> struct Radix<48> { using L = RList<16, 3>; };
template <> struct Radix<64> { using L = RList<8, 8>; };
template <> struct Radix<96> { using L = RList<8, 4, 3>; };
template <> struct Radix<128> { using L = RList<16, 8>; };
template <> struct Radix<192> { using L = RList<16, 4, 3>; };
template <> struct Radix<256> { using L = RList<16, 16>; };
template <> struct Radix<384> { using L = RList<16, 8, 3>; };
template <> struct Radix<512> { using L = RList<8, 8, 8>; };

template <typename L> struct Head;
template <int R0, int... Rs> struct Head<RList<R0, Rs...>> { static constexpr int value = R0; };

template <typename L> struct Last;
template <int R0> struct Last<RList<R0>> { static constexpr int value = R0; };
template <int R0, int R1, int... Rs> struct Last<RList<R0, R1, Rs...>> {
    static constexpr int value = Last<RList<R1, Rs...>>::value;
};

template <typename L> struct Len;
template <int... Rs> struct Len<RList<Rs...>> { static constexpr int value = sizeof...(Rs); };

template <typename A, typename B> struct Cat;
template <int... As, int... Bs> struct Cat<RList<As...>, RList<Bs...>> { using L = RList<As..., Bs...>; };

template <typename L> struct Rev;
template <> struct Rev<RList<>> { using L = RList<>; };
template <int R0, int... Rs> struct Rev<RList<R0, Rs...>> {
    using L = typename Cat<typename Rev<RList<Rs...>>::L, RList<R0>>::L;
};

template <typename L> struct Tail;
template <int R0, int... Rs> struct Tail<RList<R0, Rs...>> { using L = RList<Rs...>; };

// Radices strictly between the first and the last.
template <typename L> struct Mid;
template <int R0> struct Mid<RList<R0>> { using L = RList<>; };
template <int R0, int R1> struct Mid<RList<R0, R1>> { using L = RList<>; };
template <int R0, int R1, int R2, int... Rs> struct Mid<RList<R0, R1, R2, Rs...>> {
    using L = typename Cat<RList<R1>, typename Mid<RList<R1, R2, Rs...>>::L>::L;
};

// ---------------------------------------------------------------------------
// LDS layout: one pad element every 16 elements (8 for length 512); the line
// pitch is chosen by the kernel for its lane order.
// ---------------------------------------------------------------------------
// Pad granularity per transform length: one pad element every 2^value
// elements (every 8 for the 512-point plan: about 1% faster there, neutral
// elsewhere).
template <int M> struct PadShift {
    static constexpr int value = (M == 512) ? 3 : 4;
};
template <int M> __device__ __forceinline__ int padx(int e) { return e + (e >> PadShift<M>::value); }

constexpr int round_up(int x, int m) { return ((x + m - 1) / m) * m; }
// Lanes that differ in the line index first (column tiles): pitch = 2 mod 32.
template <int M> constexpr int pitch_cols(int E) { return round_up(E + (E >> PadShift<M>::value) + 1, 32) + 2; }
// Lanes that differ in the position first (whole lines): pitch = 16 mod 32.
template <int M> constexpr int pitch_lines(int E) { return round_up(E + (E >> PadShift<M>::value), 32) + 16; }

// ---------------------------------------------------------------------------
// Stage primitives.  A thread owns butterflies j = jt + b*TPL (b < B) of its
// line; stages with fewer butterflies than TPL*B leave the extra lanes idle.
// ---------------------------------------------------------------------------
template <int M, int TPL, int RAD> struct Shape {
    static constexpr int NB = M / RAD;
    static constexpr int B = (NB + TPL - 1) / TPL;
    __device__ __forceinline__ static bool active(int j) { return (NB % TPL) == 0 || j < NB; }
};

// Twiddle W^r for r < RAD from the loaded powers W, W^2, W^4, W^8 (binary
// decomposition of r: at most three roundings per twiddle, and only four
// table reads per butterfly).
template <bool INV, typename T, int RAD>
__device__ __forceinline__ T twpow(const T (&p)[4], int r) {
    T w{};
    bool have = false;
#pragma unroll
    for (int bit = 0; bit < 4; ++bit) {
        if ((r >> bit) & 1) {
            w = have ? cmul(w, p[bit]) : p[bit];
            have = true;
        }
    }
    return w;
}

// Twiddle powers W^(k 2^bit), 2^bit < RAD, k = j mod NS, of the thread's
// butterflies in a stage with NS > 1.  Loaded ahead of the stage's LDS
// exchange so that their latency overlaps it.  The first TWL powers are read
// from the table and the rest are squares of the previous one: line kernels,
// whose lanes all need different twiddles, trade table reads (which bound
// them) for a few multiplies; column kernels, whose lanes share them, read
// all.
template <typename T, int M, int TPL, int NS, int RAD, int TWL> struct TwP {
    static constexpr int B = Shape<M, TPL, RAD>::B;
    static constexpr int NP = 1 + (RAD > 2) + (RAD > 4) + (RAD > 8);
    T p[B][NP];
    __device__ __forceinline__ void load(int jt, const T* __restrict__ tw) {
        if constexpr (NS > 1) {
            constexpr int TWS = M / (NS * RAD);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = jt + b * TPL;
                if (Shape<M, TPL, RAD>::active(j)) {
                    const int k = j % NS;
#pragma unroll
                    for (int bit = 0; bit < NP; ++bit) {
                        if (bit < TWL) {
                            p[b][bit] = tw[(k << bit) * TWS];
                        } else {
                            const T q = p[b][bit - 1];
                            p[b][bit] = T{(q.x - q.y) * (q.x + q.y), 2 * q.x * q.y};
                        }
                    }
                }
            }
        }
    }
};

// Twiddles (stage with NS > 1, from preloaded powers) and the radix-RAD DFT,
// in registers.
template <typename T, int M, bool INV, int TPL, int NS, int RAD, int B, int TWL>
__device__ __forceinline__ void bfly(T (&v)[B][RAD], int jt, const TwP<T, M, TPL, NS, RAD, TWL>& tp) {
    using S = Shape<M, TPL, RAD>;
    static_assert(B == S::B, "register array shape");
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
            if constexpr (NS > 1) {
                T p[4];
#pragma unroll
                for (int bit = 0; bit < 4; ++bit)
                    if (bit < TwP<T, M, TPL, NS, RAD, TWL>::NP) p[bit] = tp.p[b][bit];
#pragma unroll
                for (int r = 1; r < RAD; ++r) v[b][r] = twmul<INV>(v[b][r], twpow<INV, T, RAD>(p, r));
            }
            DFT<RAD, INV>::run(v[b]);
        }
    }
}

// Twiddle sources of a transform's stages after the first: the table (TW_TABLE),
// the table with the twiddles kept in registers (TW_KEEP), or the registers kept
// by an earlier transform with the same stages (TW_REUSE: no table reads and no
// products; an inverse takes the conjugates of the same values, so its results
// are the same as from the table).
enum : int { TW_TABLE = 0, TW_KEEP = 1, TW_REUSE = 2 };

// Kept twiddles W^r (r >= 1) of the butterflies of each stage of the list L,
// whose first stage has NS = NS0.
template <typename T, int M, int TPL, int NS0, typename L> struct TwKeep {
    static constexpr int LEN = 0;
};
template <typename T, int M, int TPL, int NS0, int R0, int... Rs>
struct TwKeep<T, M, TPL, NS0, RList<R0, Rs...>> {
    static constexpr int LEN = 1 + sizeof...(Rs);
    T w[Shape<M, TPL, R0>::B][R0];
    TwKeep<T, M, TPL, NS0 * R0, RList<Rs...>> next;
};
template <typename K> __device__ __forceinline__ auto& tw_last(K& k) {
    if constexpr (K::LEN == 1) return k.w;
    else return tw_last(k.next);
}

// bfly with a twiddle source (TW_KEEP stores into w, TW_REUSE reads from it).
template <int MODE, typename T, int M, bool INV, int TPL, int NS, int RAD, int B, int TWL>
__device__ __forceinline__ void bfly_tw(T (&v)[B][RAD], int jt, const TwP<T, M, TPL, NS, RAD, TWL>& tp,
                                        T (&w)[B][RAD]) {
    using S = Shape<M, TPL, RAD>;
    static_assert(B == S::B, "register array shape");
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
            if constexpr (NS > 1) {
                T p[4];
                if constexpr (MODE != TW_REUSE) {
#pragma unroll
                    for (int bit = 0; bit < 4; ++bit)
                        if (bit < TwP<T, M, TPL, NS, RAD, TWL>::NP) p[bit] = tp.p[b][bit];
                }
#pragma unroll
                for (int r = 1; r < RAD; ++r) {
                    T t;
                    if constexpr (MODE == TW_REUSE) {
                        t = w[b][r];
                    } else {
                        t = twpow<INV, T, RAD>(p, r);
                        if constexpr (MODE == TW_KEEP) w[b][r] = t;
                    }
                    v[b][r] = twmul<INV>(v[b][r], t);
                }
            }
            DFT<RAD, INV>::run(v[b]);
        }
    }
}

template <typename T, int M, bool INV, int TPL, int NS, int RAD, int B>
__device__ __forceinline__ void bfly(T (&v)[B][RAD], int jt, const T* __restrict__ tw) {
    TwP<T, M, TPL, NS, RAD, 4> tp;
    tp.load(jt, tw);
    bfly<T, M, INV, TPL, NS, RAD>(v, jt, tp);
}

// Write the stage outputs to their Stockham positions in LDS.
template <typename T, int M, int TPL, int NS, int RAD, int B>
__device__ __forceinline__ void put(const T (&v)[B][RAD], T* line, int jt) {
    using S = Shape<M, TPL, RAD>;
    static_assert(B == S::B, "register array shape");
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
            const int base = (j / NS) * NS * RAD + j % NS;
#pragma unroll
            for (int r = 0; r < RAD; ++r) line[padx<M>(base + r * NS)] = v[b][r];
        }
    }
}

// Read a stage's inputs (positions j + r*M/RAD) from LDS.
template <typename T, int M, int TPL, int RAD, int B>
__device__ __forceinline__ void get(T (&v)[B][RAD], const T* line, int jt) {
    using S = Shape<M, TPL, RAD>;
    static_assert(B == S::B, "register array shape");
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[b][r] = line[padx<M>(j + r * S::NB)];
        }
    }
}

// Ordering point between the LDS writes and reads of an exchange.  WS: every
// thread that touches the LDS region is a lane of one wavefront, whose LDS
// accesses execute in program order, so only the compiler has to be kept
// from moving accesses across it; otherwise a workgroup barrier.
template <bool WS> __device__ __forceinline__ void lds_sync() {
    if constexpr (WS) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// Middle stages entirely in LDS (each: barrier, read, barrier, compute, write).
template <typename T, int M, bool INV, int TPL, int NS, typename L, bool WS, int TWL> struct MidStages;
template <typename T, int M, bool INV, int TPL, int NS, bool WS, int TWL>
struct MidStages<T, M, INV, TPL, NS, RList<>, WS, TWL> {
    __device__ __forceinline__ static void run(T*, int, const T*) {}
};
template <typename T, int M, bool INV, int TPL, int NS, int R0, int... Rs, bool WS, int TWL>
struct MidStages<T, M, INV, TPL, NS, RList<R0, Rs...>, WS, TWL> {
    __device__ __forceinline__ static void run(T* line, int jt, const T* __restrict__ tw) {
        T v[Shape<M, TPL, R0>::B][R0];
        TwP<T, M, TPL, NS, R0, TWL> tp;
        tp.load(jt, tw);
        lds_sync<WS>();
        get<T, M, TPL, R0>(v, line, jt);
        lds_sync<WS>();
        bfly<T, M, INV, TPL, NS, R0>(v, jt, tp);
        put<T, M, TPL, NS, R0>(v, line, jt);
        MidStages<T, M, INV, TPL, NS * R0, RList<Rs...>, WS, TWL>::run(line, jt, tw);
    }
};

// Middle stages with a twiddle source (see TW_TABLE); K holds this stage's
// kept twiddles and those of the stages after it.
template <typename T, int M, bool INV, int TPL, int NS, typename L, bool WS, int TWL, int MODE> struct MidStagesTw;
template <typename T, int M, bool INV, int TPL, int NS, bool WS, int TWL, int MODE>
struct MidStagesTw<T, M, INV, TPL, NS, RList<>, WS, TWL, MODE> {
    template <typename K> __device__ __forceinline__ static void run(T*, int, const T*, K&) {}
};
template <typename T, int M, bool INV, int TPL, int NS, int R0, int... Rs, bool WS, int TWL, int MODE>
struct MidStagesTw<T, M, INV, TPL, NS, RList<R0, Rs...>, WS, TWL, MODE> {
    template <typename K>
    __device__ __forceinline__ static void run(T* line, int jt, const T* __restrict__ tw, K& keep) {
        T v[Shape<M, TPL, R0>::B][R0];
        TwP<T, M, TPL, NS, R0, TWL> tp;
        if constexpr (MODE != TW_REUSE) tp.load(jt, tw);
        lds_sync<WS>();
        get<T, M, TPL, R0>(v, line, jt);
        lds_sync<WS>();
        bfly_tw<MODE, T, M, INV, TPL, NS, R0>(v, jt, tp, keep.w);
        put<T, M, TPL, NS, R0>(v, line, jt);
        MidStagesTw<T, M, INV, TPL, NS * R0, RList<Rs...>, WS, TWL, MODE>::run(line, jt, tw, keep.next);
    }
};

// One component (C = 0: real, 1: imaginary) of a stage's values to / from a
// line of scalars, at the positions of put and get.
template <int C, typename T, int M, int TPL, int NS, int RAD, int B>
__device__ __forceinline__ void put_c(const T (&v)[B][RAD], typename RealOf<T>::R* line, int jt) {
    using S = Shape<M, TPL, RAD>;
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
            const int base = (j / NS) * NS * RAD + j % NS;
#pragma unroll
            for (int r = 0; r < RAD; ++r) line[padx<M>(base + r * NS)] = (C == 0) ? v[b][r].x : v[b][r].y;
        }
    }
}

template <int C, typename T, int M, int TPL, int RAD, int B>
__device__ __forceinline__ void get_c(T (&v)[B][RAD], const typename RealOf<T>::R* line, int jt) {
    using S = Shape<M, TPL, RAD>;
#pragma unroll
    for (int b = 0; b < S::B; ++b) {
        const int j = jt + b * TPL;
        if (S::active(j)) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) {
                if constexpr (C == 0) v[b][r].x = line[padx<M>(j + r * S::NB)];
                else v[b][r].y = line[padx<M>(j + r * S::NB)];
            }
        }
    }
}

// Stage-to-stage exchange through a line of scalars, one component at a time:
// half the LDS of a complex line, so more lines fit on a CU; four ordering
// points instead of two.  a: the outputs of a stage of radix RP at stride NSP;
// b: the inputs of the next stage (radix RN).
template <typename T, int M, int TPL, int NSP, int RP, int RN, bool WS, int BP, int BN>
__device__ __forceinline__ void xchg_split(const T (&a)[BP][RP], T (&b)[BN][RN], typename RealOf<T>::R* line, int jt) {
    lds_sync<WS>();
    put_c<0, T, M, TPL, NSP, RP>(a, line, jt);
    lds_sync<WS>();
    get_c<0, T, M, TPL, RN>(b, line, jt);
    lds_sync<WS>();
    put_c<1, T, M, TPL, NSP, RP>(a, line, jt);
    lds_sync<WS>();
    get_c<1, T, M, TPL, RN>(b, line, jt);
}

// The stages after the first with split exchanges.  vp holds the outputs of
// the previous stage (radix RP at stride NSP); L lists the middle radices
// left; the last stage (radix RK) writes u.
template <typename T, int M, bool INV, int TPL, int NSP, int RP, typename L, int RK, bool WS, int TWL> struct SplitStages;
template <typename T, int M, bool INV, int TPL, int NSP, int RP, int RK, bool WS, int TWL>
struct SplitStages<T, M, INV, TPL, NSP, RP, RList<>, RK, WS, TWL> {
    template <int BP, int BK>
    __device__ __forceinline__ static void run(T (&vp)[BP][RP], T (&u)[BK][RK], typename RealOf<T>::R* line, int jt,
                                               const T* __restrict__ tw) {
        TwP<T, M, TPL, M / RK, RK, TWL> tp;
        tp.load(jt, tw);
        xchg_split<T, M, TPL, NSP, RP, RK, WS>(vp, u, line, jt);
        bfly<T, M, INV, TPL, M / RK, RK>(u, jt, tp);
    }
};
template <typename T, int M, bool INV, int TPL, int NSP, int RP, int R0, int... Rs, int RK, bool WS, int TWL>
struct SplitStages<T, M, INV, TPL, NSP, RP, RList<R0, Rs...>, RK, WS, TWL> {
    static constexpr int NS = NSP * RP;
    template <int BP, int BK>
    __device__ __forceinline__ static void run(T (&vp)[BP][RP], T (&u)[BK][RK], typename RealOf<T>::R* line, int jt,
                                               const T* __restrict__ tw) {
        T v[Shape<M, TPL, R0>::B][R0];
        TwP<T, M, TPL, NS, R0, TWL> tp;
        tp.load(jt, tw);
        xchg_split<T, M, TPL, NSP, RP, R0, WS>(vp, v, line, jt);
        bfly<T, M, INV, TPL, NS, R0>(v, jt, tp);
        SplitStages<T, M, INV, TPL, NS, R0, RList<Rs...>, RK, WS, TWL>::run(v, u, line, jt, tw);
    }
};

// Whole transform with register-resident ends.
//   in:  v = inputs at positions j + r*M/R0 (first radix R0 of the plan L)
//   out: u = outputs at positions j + r*M/Rk (last radix Rk)
// The caller guarantees that no thread still reads the line's LDS when this
// starts; on return other threads may still be reading it (barrier before
// reuse).  Single-stage plans use no LDS.  WS: the threads of a line are
// lanes of one wavefront (see lds_sync).  TWL: twiddle powers read per
// butterfly (see TwP).
// XS: split exchanges (xchg_split); `line` then holds M padded scalars.
template <typename T, int M, bool INV, int TPL, typename L, bool WS = false, int TWL = 4, bool XS = false> struct Fft {
    static constexpr int R0 = Head<L>::value;
    static constexpr int RK = Last<L>::value;
    static constexpr int B0 = Shape<M, TPL, R0>::B;
    static constexpr int BK = Shape<M, TPL, RK>::B;
    static constexpr int NSTAGE = Len<L>::value;
    using In = T[B0][R0];
    using Out = T[BK][RK];

    __device__ __forceinline__ static void run(T (&v)[B0][R0], T (&u)[BK][RK], T* line, int jt,
                                               const T* __restrict__ tw) {
        if constexpr (NSTAGE == 1) {
#pragma unroll
            for (int b = 0; b < B0; ++b)
#pragma unroll
                for (int r = 0; r < R0; ++r) u[b][r] = v[b][r];
            bfly<T, M, INV, TPL, 1, R0>(u, jt, tw);
        } else if constexpr (XS) {
            bfly<T, M, INV, TPL, 1, R0>(v, jt, tw);
            SplitStages<T, M, INV, TPL, 1, R0, typename Mid<L>::L, RK, WS, TWL>::run(
                v, u, reinterpret_cast<typename RealOf<T>::R*>(line), jt, tw);
        } else {
            bfly<T, M, INV, TPL, 1, R0>(v, jt, tw);
            put<T, M, TPL, 1, R0>(v, line, jt);
            MidStages<T, M, INV, TPL, R0, typename Mid<L>::L, WS, TWL>::run(line, jt, tw);
            TwP<T, M, TPL, M / RK, RK, TWL> tp;
            tp.load(jt, tw);
            lds_sync<WS>();
            get<T, M, TPL, RK>(u, line, jt);
            bfly<T, M, INV, TPL, M / RK, RK>(u, jt, tp);
        }
    }

    // Twiddles of the stages after the first kept in registers: a transform
    // run with TW_KEEP fills `keep`, a later one with the same stages (the same
    // plan, or the inverse of a palindromic one) runs with TW_REUSE from it.
    using Keep = TwKeep<T, M, TPL, R0, typename Tail<L>::L>;
    template <int MODE>
    __device__ __forceinline__ static void run_tw(T (&v)[B0][R0], T (&u)[BK][RK], T* line, int jt,
                                                  const T* __restrict__ tw, Keep& keep) {
        static_assert(!XS, "split exchanges take the twiddles from the table");
        if constexpr (NSTAGE == 1) {
            run(v, u, line, jt, tw);
        } else {
            bfly<T, M, INV, TPL, 1, R0>(v, jt, tw);
            put<T, M, TPL, 1, R0>(v, line, jt);
            MidStagesTw<T, M, INV, TPL, R0, typename Mid<L>::L, WS, TWL, MODE>::run(line, jt, tw, keep);
            TwP<T, M, TPL, M / RK, RK, TWL> tp;
            if constexpr (MODE != TW_REUSE) tp.load(jt, tw);
            lds_sync<WS>();
            get<T, M, TPL, RK>(u, line, jt);
            bfly_tw<MODE, T, M, INV, TPL, M / RK, RK>(u, jt, tp, tw_last(keep));
        }
    }
};

// Forward plan and its reversal for the inverse.
template <int M> using FwdPlan = typename Radix<M>::L;
template <int M> using InvPlan = typename Rev<typename Radix<M>::L>::L;

}  // namespace fse
