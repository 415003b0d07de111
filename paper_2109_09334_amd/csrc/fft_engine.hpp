// Line FFT engine for gfx950: a mixed-radix (2, 3, 4, 8, 16) Stockham
// autosort transform of one line held in LDS, computed in place. Each pass
// stages the thread's butterfly inputs in registers, synchronises, applies
// the inter-pass twiddles and the radix-R DFT, and writes the results back
// at their Stockham positions:
//   inputs   v[r] = x[j + r N/R]                 (j = butterfly, r < R)
//   twiddle  v[r] *= W_N^(r k N/(Ns R)),  k = j mod Ns, W_N = e^(S 2 pi i / N)
//   outputs  y[(j / Ns) Ns R + k + r Ns] = DFT_R(v)[r]
// with Ns the product of the radices already applied. After the last pass
// the line holds its transform in natural order. S = -1 is the forward
// (e^-) transform, S = +1 the unnormalised inverse.
#pragma once
#include "common.hpp"

namespace sfft {

// cos / sin of 2 pi k / 16, k = 0..15 (exact decimal expansions of the
// algebraic values, rounded by the compiler to the target precision).
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// x * e^(S 2 pi i k / R) for compile-time R | 16, with the trivial factors
// (1, +-i, (1 +- i)/sqrt 2) written out.
template <int R, int S, int K, typename T>
__device__ __forceinline__ cx<T> rot(cx<T> x) {
    constexpr int q = (K * 16 / R) & 15;   // angle in units of 2 pi / 16
    if constexpr (q == 0) {
        return x;
    } else if constexpr (q == 4) {
        return S > 0 ? cx<T>{-x.im, x.re} : cx<T>{x.im, -x.re};
    } else if constexpr (q == 8) {
        return cx<T>{-x.re, -x.im};
    } else if constexpr (q == 12) {
        return S > 0 ? cx<T>{x.im, -x.re} : cx<T>{-x.im, x.re};
    } else if constexpr (q == 2 || q == 6 || q == 10 || q == 14) {
        // |cos| = |sin| = 1/sqrt 2: two add/sub and two multiplies
        constexpr int sc = (q == 2 || q == 14) ? 1 : -1;
        constexpr int ss0 = (q == 2 || q == 6) ? 1 : -1;
        constexpr int ss = S > 0 ? ss0 : -ss0;
        const T h = T(0.70710678118654752440);
        const T re = (sc > 0 ? x.re : -x.re) - (ss > 0 ? x.im : -x.im);
        const T im = (ss > 0 ? x.re : -x.re) + (sc > 0 ? x.im : -x.im);
        return cx<T>{h * re, h * im};
    } else {
        const T c = T(kCos16[q]);
        const T s = S > 0 ? T(kSin16[q]) : -T(kSin16[q]);
        return cx<T>{x.re * c - x.im * s, x.re * s + x.im * c};
    }
}

// In-place DFT of R points in registers, output in natural order.
template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<2, S, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    }
};

template <int S, typename T>
struct Dft<3, S, T> {
    static __device__ __forceinline__ void run(cx<T>* v) {
        const T c = T(-0.5);
        const T s = T(S) * T(0.86602540378443864676);   // S sin(2 pi / 3)
        cx<T> a = v[0], t = v[1] + v[2], u = v[1] - v[2];
        cx<T> m = {a.re + c * t.re, a.im + c * t.im};
        v[0] = a + t;
        // X1 = m + i s u, X2 = m - i s u
        v[1] = {m.re - s * u.im, m.im + s * u.re};
        v[2] = {m.re + s * u.im, m.im - s * u.re};
    }
};

// Power-of-two sizes: split into even and odd halves (decimation in time).
template <int R, int S, typename T>
struct Dft {
    static_assert(R == 4 || R == 8 || R == 16, "unsupported radix");
    template <int K>
    static __device__ __forceinline__ void combine(cx<T>* v, const cx<T>* e, const cx<T>* o) {
        if constexpr (K < R / 2) {
            cx<T> t = rot<R, S, K, T>(o[K]);
            v[K] = e[K] + t;
            v[K + R / 2] = e[K] - t;
            combine<K + 1>(v, e, o);
        }
    }
    static __device__ __forceinline__ void run(cx<T>* v) {
        cx<T> e[R / 2], o[R / 2];
#pragma unroll
        for (int k = 0; k < R / 2; ++k) {
            e[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        Dft<R / 2, S, T>::run(e);
        Dft<R / 2, S, T>::run(o);
        combine<0>(v, e, o);
    }
};

// One Stockham pass of radix R over a line of n points at buf.
// lt = thread index within the line, tl = threads per line.
// tw = table of W_n^t = e^(-2 pi i t / n), t < n (conjugated for S > 0).
template <int R, int S, typename T>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int n, int ns, int lt, int tl,
                                              const cx<T>* __restrict__ tw) {
    constexpr int NB = (kElemsPerThread + R - 1) / R;
    const int nbf = n / R;
    const int step = n / (ns * R);
    cx<T> v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = lt + b * tl;
        if (j < nbf) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[j + r * nbf];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = lt + b * tl;
        if (j < nbf) {
            const int k = j % ns;
            const int tstep = k * step;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> w = tw[r * tstep];
                if (S > 0) w.im = -w.im;
                v[b][r] = cmul(v[b][r], w);
            }
            Dft<R, S, T>::run(v[b]);
            const int o = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[o + r * ns] = v[b][r];
        }
    }
    __syncthreads();
}

// Full transform of the line at buf (all threads of the workgroup call it).
template <int S, typename T>
__device__ __forceinline__ void line_fft(cx<T>* buf, const LinePlan& lp, int lt,
                                         const cx<T>* __restrict__ tw) {
    int ns = 1;
    for (int p = 0; p < lp.npass; ++p) {
        const int R = lp.radix[p];
        switch (R) {
            case 16: stockham_pass<16, S, T>(buf, lp.n, ns, lt, lp.tl, tw); break;
            case 8: stockham_pass<8, S, T>(buf, lp.n, ns, lt, lp.tl, tw); break;
            case 4: stockham_pass<4, S, T>(buf, lp.n, ns, lt, lp.tl, tw); break;
            case 3: stockham_pass<3, S, T>(buf, lp.n, ns, lt, lp.tl, tw); break;
            default: stockham_pass<2, S, T>(buf, lp.n, ns, lt, lp.tl, tw); break;
        }
        ns *= R;
    }
}

}  // namespace sfft
