// Line FFT engine for gfx950: a mixed-radix (2, 3, 4, 8, 16) Stockham
// autosort transform of one line, 16 elements per thread. The first and (for
// a radix-16 tail) last passes run on registers; the passes between stage the
// thread's butterfly inputs from a padded LDS line, synchronise, apply the
// inter-pass twiddles (per-pass tables) and the radix-R DFT, and write the
// results back at their Stockham positions:
//   inputs   v[r] = x[j + r N/R]                 (j = butterfly, r < R)
//   twiddle  v[r] *= W_N^(r k N/(Ns R)),  k = j mod Ns, W_N = e^(S 2 pi i / N)
//   outputs  y[(j / Ns) Ns R + k + r Ns] = DFT_R(v)[r]
// with Ns the product of the radices already applied. After the last pass
// the line holds its transform in natural order. S = -1 is the forward
// (e^-) transform, S = +1 the unnormalised inverse.
#pragma once
#include <type_traits>

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

// LDS index with one padding slot per 16 elements. The first pass writes
// each thread's 16 outputs contiguously (a stride of 16 elements across the
// lanes), which without padding maps every lane to the same few banks.
__host__ __device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int line_lds_elems(int n) { return n + (n >> 4); }

// w[1..R-1] = row[1..R-1] (a twiddle row of the pass tables, 16 entries,
// 16-entry aligned), conjugated for the inverse transform.
template <int R, int S>
__device__ __forceinline__ void load_twiddles(cx<float>* w, const cx<float>* __restrict__ row) {
    const float4* q = reinterpret_cast<const float4*>(row);
#pragma unroll
    for (int h = 0; h < (R + 1) / 2; ++h) {
        const float4 t = q[h];
        w[2 * h] = cx<float>{t.x, S > 0 ? -t.y : t.y};
        if (2 * h + 1 < R) w[2 * h + 1] = cx<float>{t.z, S > 0 ? -t.w : t.w};
    }
}
template <int R, int S>
__device__ __forceinline__ void load_twiddles(cx<double>* w, const cx<double>* __restrict__ row) {
    const double2* q = reinterpret_cast<const double2*>(row);
#pragma unroll
    for (int r = 1; r < R; ++r) {
        const double2 t = q[r];
        w[r] = cx<double>{t.x, S > 0 ? -t.y : t.y};
    }
}

// One Stockham pass of radix R (> the first) through the padded LDS line.
// twt: the pass table, row k = W_(ns R)^(r k), r < 16.
template <int R, int S, typename T>
__device__ __forceinline__ void pass_lds(cx<T>* buf, int n, int ns, int lt, int tl,
                                         const cx<T>* __restrict__ twt) {
    constexpr int NB = (kElemsPerThread + R - 1) / R;
    const int nbf = n / R;
    cx<T> v[NB][R], w[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = lt + b * tl;
        if (j < nbf) {
            const int k = j % ns;
            load_twiddles<R, S>(w[b], twt + (size_t)k * 16);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[lpad(j + r * nbf)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = lt + b * tl;
        if (j < nbf) {
            const int k = j % ns;
#pragma unroll
            for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[b][r]);
            Dft<R, S, T>::run(v[b]);
            const int o = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[lpad(o + r * ns)] = v[b][r];
        }
    }
    __syncthreads();
}

// Transform of one line whose data stays in registers at both ends: on entry
// v[e] = x[lt + e tl], on exit v[e] = X[lt + e tl] (natural order), e < 16.
// The plan starts with radix 16, so the first pass runs on the registers as
// loaded (Ns = 1, no twiddles); when it also ends with radix 16, the last
// pass (Ns = n/16 = tl, butterfly j = lt) leaves its outputs in natural order
// in the registers. The passes between go through the padded LDS line buf.
// All threads of the workgroup call it (it synchronises); the caller must
// not touch buf between a call and the next barrier.
template <int S, typename T>
__device__ __forceinline__ void line_fft_regs(cx<T>* v, cx<T>* buf, const LinePlan& lp, int lt,
                                              const cx<T>* __restrict__ twt) {
    Dft<16, S, T>::run(v);
    if (lp.npass == 1) return;
    const int n = lp.n, tl = lp.tl;
    __syncthreads();   // buf may still be read by a previous transform
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[lpad(16 * lt + r)] = v[r];
    __syncthreads();
    int ns = 16;
    const int last = lp.npass - 1;
    const bool tail16 = lp.radix[last] == 16;
    const int pend = tail16 ? last : lp.npass;
    for (int p = 1; p < pend; ++p) {
        const cx<T>* tp = twt + lp.twoff[p];
        switch (lp.radix[p]) {
            case 16: pass_lds<16, S, T>(buf, n, ns, lt, tl, tp); break;
            case 8: pass_lds<8, S, T>(buf, n, ns, lt, tl, tp); break;
            case 4: pass_lds<4, S, T>(buf, n, ns, lt, tl, tp); break;
            case 3: pass_lds<3, S, T>(buf, n, ns, lt, tl, tp); break;
            default: pass_lds<2, S, T>(buf, n, ns, lt, tl, tp); break;
        }
        ns *= lp.radix[p];
    }
    if (tail16) {
        cx<T> w[16];
        load_twiddles<16, S>(w, twt + lp.twoff[last] + (size_t)lt * 16);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[lpad(lt + r * tl)];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[r]);
        Dft<16, S, T>::run(v);
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = buf[lpad(lt + e * tl)];
    }
}

// ---- compile-time plans for the common line lengths ----------------------
// The same passes as line_fft_regs with the radix sequence (and so every ns)
// known at compile time: no radix switch (whose union of code paths holds
// ~60 more VGPRs) and no runtime modulo. The sequences equal the runtime
// plans' order, so the same pass twiddle tables serve both.
template <int... R>
struct RadixSeq {};
struct DynPlan {};

template <int... R>
struct SeqProd;
template <>
struct SeqProd<> {
    static constexpr int value = 1;
};
template <int R, int... Rest>
struct SeqProd<R, Rest...> {
    static constexpr int value = R * SeqProd<Rest...>::value;
};

// Passes after the first, starting with radix R at stride NS; twoff is the
// offset of this pass's twiddle table.
template <int S, typename T, int N, int NS, int R, int... Rest>
__device__ __forceinline__ void passes_static(cx<T>* v, cx<T>* buf, int lt,
                                              const cx<T>* __restrict__ twt, int twoff) {
    constexpr int TL = N / kElemsPerThread;
    if constexpr (sizeof...(Rest) == 0 && R == 16) {
        cx<T> w[16];
        load_twiddles<16, S>(w, twt + twoff + (size_t)lt * 16);
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = buf[lpad(lt + r * TL)];
#pragma unroll
        for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], w[r]);
        Dft<16, S, T>::run(v);
    } else {
        pass_lds<R, S, T>(buf, N, NS, lt, TL, twt + twoff);
        if constexpr (sizeof...(Rest) > 0) {
            passes_static<S, T, N, NS * R, Rest...>(v, buf, lt, twt, twoff + NS * 16);
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) v[e] = buf[lpad(lt + e * TL)];
        }
    }
}

template <int S, typename T, int... Rs>
__device__ __forceinline__ void line_fft_static(cx<T>* v, cx<T>* buf, int lt,
                                                const cx<T>* __restrict__ twt, RadixSeq<16, Rs...>) {
    Dft<16, S, T>::run(v);
    if constexpr (sizeof...(Rs) > 0) {
        constexpr int N = 16 * SeqProd<Rs...>::value;
        __syncthreads();   // buf may still be read by a previous transform
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[lpad(16 * lt + r)] = v[r];
        __syncthreads();
        passes_static<S, T, N, 16, Rs...>(v, buf, lt, twt, 0);
    }
}

// Line transform with the plan PL: RadixSeq<...> (compile time) or DynPlan
// (lp at run time). Same contract as line_fft_regs.
template <int S, typename T, typename PL>
__device__ __forceinline__ void line_fft(cx<T>* v, cx<T>* buf, const LinePlan& lp, int lt,
                                         const cx<T>* __restrict__ twt) {
    if constexpr (std::is_same<PL, DynPlan>::value) {
        line_fft_regs<S, T>(v, buf, lp, lt, twt);
    } else {
        line_fft_static<S, T>(v, buf, lt, twt, PL{});
    }
}

// Plan tag of a Bluestein line: the chirp form below around transforms of
// length lp.n with the plan P. Lines of other plans have no padding (lp.nl =
// lp.n), and kernels compile their padding clamps and masks only for this
// tag (pad_index, in_line).
template <typename P>
struct Chirp {
    using plan = P;
};
template <typename PL>
struct IsChirp : std::false_type {};
template <typename P>
struct IsChirp<Chirp<P>> : std::true_type {};

// Index t of a line's element, clamped into its n true points (a padded
// line's loads past n read a valid element, masked after).
template <typename PL>
__device__ __forceinline__ int pad_index(int t, int n) {
    if constexpr (IsChirp<PL>::value) return t < n ? t : n - 1;
    else return t;
}
// Whether index t is one of the line's n true points.
template <typename PL>
__device__ __forceinline__ bool in_line(int t, int n) {
    if constexpr (IsChirp<PL>::value) return t < n;
    else return true;
}

// The DFT of a line of lp.nl points, in the layout of line_fft (element t in
// register t / TL of thread t mod TL; entries t >= nl are ignored on input
// and zero on output). For plans other than Chirp this is line_fft; for
// Chirp<P> the Bluestein form of the forward DFT,
//   X_k = conj(c_k) sum_t (x_t conj(c_t)) c_(k-t),  c_t = e^(+i pi t^2 / nl),
// the sum a circular convolution of length n >= 2 nl - 1 evaluated as
// IDFT_n(DFT_n(a) DFT_n(b)) / n (the 1/n is in bhat); the inverse (S = +1)
// is conj(forward(conj(x))).
template <int S, typename T, typename PL>
__device__ __forceinline__ void line_dft(cx<T>* v, cx<T>* buf, const LinePlan& lp, int lt,
                                         const cx<T>* __restrict__ twt) {
    if constexpr (!IsChirp<PL>::value) {
        line_fft<S, T, PL>(v, buf, lp, lt, twt);
    } else {
        using P = typename PL::plan;
        // the tables are FP64 and every product is formed in FP64 and rounded
        // once to T (FP64 and FP32 vector rates are equal on this hardware)
        const cx<double>* __restrict__ ch = static_cast<const cx<double>*>(lp.chirp);
        const cx<double>* __restrict__ bh = static_cast<const cx<double>*>(lp.bhat);
        auto wide = [](cx<T> a) { return mk((double)a.re, (double)a.im); };
        auto narrow = [](cx<double> a) { return mk(T(a.re), T(a.im)); };
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int t = lt + e * lp.tl;
            const bool in = t < lp.nl;
            const cx<double> c = ch[in ? t : 0];
            const cx<T> x = S > 0 ? cconj(v[e]) : v[e];
            v[e] = in ? narrow(cmulc(c, wide(x))) : mk(T(0), T(0));
        }
        line_fft<-1, T, P>(v, buf, lp, lt, twt);
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) v[e] = narrow(cmul(wide(v[e]), bh[lt + e * lp.tl]));
        line_fft<1, T, P>(v, buf, lp, lt, twt);
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int t = lt + e * lp.tl;
            const bool in = t < lp.nl;
            const cx<T> y = narrow(cmulc(ch[in ? t : 0], wide(v[e])));
            v[e] = in ? (S > 0 ? cconj(y) : y) : mk(T(0), T(0));
        }
    }
}

// Calls f(PL{}) with the plan of lp: the compile-time plan of its length or
// DynPlan, wrapped in Chirp for a Bluestein line (compile-time plans for the
// transform lengths of 2046 and 4094 points, the DECam CCD sides).
template <typename F>
inline hipError_t with_line_plan(const LinePlan& lp, F&& f) {
    if (lp.chirp) {
        switch (lp.n) {
            case 4096: return f(Chirp<RadixSeq<16, 16, 16>>{});
            case 8192: return f(Chirp<RadixSeq<16, 2, 16, 16>>{});
            default: return f(Chirp<DynPlan>{});
        }
    }
    switch (lp.n) {
        case 4096: return f(RadixSeq<16, 16, 16>{});
        case 2048: return f(RadixSeq<16, 8, 16>{});
        case 1024: return f(RadixSeq<16, 4, 16>{});
        case 8192: return f(RadixSeq<16, 2, 16, 16>{});
        case 6144: return f(RadixSeq<16, 8, 3, 16>{});
        default: return f(DynPlan{});
    }
}

}  // namespace sfft
