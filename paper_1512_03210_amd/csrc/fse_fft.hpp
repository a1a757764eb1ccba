// Device-side FFT building blocks for gfx950 (CDNA4, wave64).
//
// A workgroup owns a tile of LPB lines of one axis, resident in LDS.  Each
// line is transformed by a mixed-radix Stockham autosort FFT (radices
// 2, 3, 4, 8, 16): in every stage a thread reads R elements strided by M/R,
// applies the twiddles W_{Ns R}^{k r}, does a radix-R DFT in registers and
// writes the results to positions (j/Ns)*Ns*R + j%Ns + r*Ns.  The LDS
// layout inserts one pad element every 16 (complex double) or 32 (complex
// float) elements and gives each line an odd pitch, so the strided Stockham
// writes and the column-wise tile loads spread over the 64 LDS banks.
//
// All transforms are unnormalised; forward uses exp(-2 pi i nk/M).
#pragma once
#include <hip/hip_runtime.h>

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
        const R s3 = R(0.86602540378443864676372317075294);  // sqrt(3)/2
        T s = cadd(v[1], v[2]);
        T dd = csub(v[1], v[2]);
        T a = T{v[0].x - R(0.5) * s.x, v[0].y - R(0.5) * s.y};
        T b = cscale(mul_ni<INV>(dd), s3);  // -i sqrt(3)/2 (v1 - v2) forward
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
        const R c = R(0.70710678118654752440084436210485);  // sqrt(1/2)
        T e[4] = {v[0], v[2], v[4], v[6]};
        T o[4] = {v[1], v[3], v[5], v[7]};
        DFT<4, INV>::run(e);
        DFT<4, INV>::run(o);
        // o[k] *= W8^k, W8 = exp(-+ i pi/4)
        T o1 = INV ? T{c * (o[1].x - o[1].y), c * (o[1].x + o[1].y)}
                   : T{c * (o[1].x + o[1].y), c * (o[1].y - o[1].x)};
        T o2 = mul_ni<INV>(o[2]);
        T o3 = INV ? T{-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y)}
                   : T{c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y)};
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
        const R C1 = R(0.92387953251128675612818318939679);
        const R S1 = R(0.38268343236508977172845998403040);
        const R C2 = R(0.70710678118654752440084436210485);
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
        const R cs[10] = {R(1), C1, C2, S1, R(0), -S1, -C2, -C1, R(-1), -C1};
        const R sn[10] = {R(0), S1, C2, C1, R(1), C1, C2, S1, R(0), -S1};
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2) {
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                const int m = n2 * k1;
                const T w = T{cs[m], INV ? sn[m] : -sn[m]};
                y[n2][k1] = cmul(y[n2][k1], w);
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
// Radix schedules (products equal M).
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
template <> struct Radix<768> { using L = RList<16, 16, 3>; };
template <> struct Radix<1024> { using L = RList<16, 16, 4>; };

// ---------------------------------------------------------------------------
// LDS layout.
// ---------------------------------------------------------------------------
template <typename R> struct LdsPad;
template <> struct LdsPad<double> { static constexpr int SHIFT = 4; };
template <> struct LdsPad<float> { static constexpr int SHIFT = 5; };

template <typename R> __device__ __forceinline__ int padx(int e) { return e + (e >> LdsPad<R>::SHIFT); }

// Line pitch (in elements) for lines holding up to E elements: padded length, made odd.
template <typename R> constexpr int line_pitch(int E) {
    return ((E + (E >> LdsPad<R>::SHIFT) + 1) | 1);
}

// ---------------------------------------------------------------------------
// One Stockham stage on every line of the tile.  Thread (line, jt) handles
// butterflies j = jt, jt + TPL, ...; callers pass the line's LDS base.
// The stage begins with a barrier (previous writes visible) and has one
// between its reads and writes (in-place buffer).
// ---------------------------------------------------------------------------
template <typename R, int M, bool INV, int TPL, int NS, int RAD>
__device__ __forceinline__ void fft_stage(typename CT<R>::T* line, int jt,
                                          const typename CT<R>::T* __restrict__ tw) {
    using T = typename CT<R>::T;
    constexpr int NB = M / RAD;
    constexpr int B = (NB + TPL - 1) / TPL;
    constexpr int TWS = M / (NS * RAD);
    T v[B][RAD];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = jt + b * TPL;
        if ((NB % TPL) == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[b][r] = line[padx<R>(j + r * NB)];
            if (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < RAD; ++r) v[b][r] = twmul<INV>(v[b][r], tw[k * r * TWS]);
            }
            DFT<RAD, INV>::run(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int j = jt + b * TPL;
        if ((NB % TPL) == 0 || j < NB) {
            const int k = j % NS;
            const int base = (j / NS) * NS * RAD + k;
#pragma unroll
            for (int r = 0; r < RAD; ++r) line[padx<R>(base + r * NS)] = v[b][r];
        }
    }
}

template <typename R, int M, bool INV, int TPL, int NS, typename L> struct Stages;
template <typename R, int M, bool INV, int TPL, int NS> struct Stages<R, M, INV, TPL, NS, RList<>> {
    __device__ __forceinline__ static void run(typename CT<R>::T*, int, const typename CT<R>::T*) {}
};
template <typename R, int M, bool INV, int TPL, int NS, int R0, int... Rs>
struct Stages<R, M, INV, TPL, NS, RList<R0, Rs...>> {
    __device__ __forceinline__ static void run(typename CT<R>::T* line, int jt,
                                               const typename CT<R>::T* __restrict__ tw) {
        fft_stage<R, M, INV, TPL, NS, R0>(line, jt, tw);
        Stages<R, M, INV, TPL, NS * R0, RList<Rs...>>::run(line, jt, tw);
    }
};

// Full length-M transform of the calling thread's line (all threads of the
// block must call it).  Ends after the last stage's writes, without a barrier.
template <typename R, int M, bool INV, int TPL>
__device__ __forceinline__ void fft_line(typename CT<R>::T* line, int jt, const typename CT<R>::T* __restrict__ tw) {
    Stages<R, M, INV, TPL, 1, typename Radix<M>::L>::run(line, jt, tw);
}

}  // namespace fse
