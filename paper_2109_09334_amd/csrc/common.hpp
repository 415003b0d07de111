// Shared types for the SFFT gfx950 library: geometry of one problem, FFT
// line plans, complex arithmetic, launch helpers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sfft {

// Complex number in a given real type, stored as (re, im) and aligned so a
// single 64-bit (float) or 128-bit (double) access moves it.
template <typename T>
struct alignas(2 * sizeof(T)) cx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__host__ __device__ __forceinline__ cx<T> cconj(cx<T> a) { return {a.re, -a.im}; }

// Maximum number of radix passes of one line transform.
// Zero, hidden from the optimiser. Inside a loop, p + opaque_zero() keeps
// the addresses derived from p from being formed once before the loop and
// held in registers across every iteration (p keeps its address space).
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+v"(z));
    return z;
}

// Batched launches: one launch serves a batch of pairs of one geometry,
// blockIdx.z selecting the pair. The pairs' workspaces are laid out zs bytes
// apart, so a workspace buffer of pair z is the argument (pair 0's) plus
// z * zs; outside a batch z = 0. Twiddle tables are shared and never offset.
template <typename T>
__device__ __forceinline__ T* zoff(T* p, long long zs) {
    return p ? reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) +
                                    (uintptr_t)((long long)blockIdx.z * zs))
             : p;
}

// Address of a caller-owned buffer as a kernel sees it: the argument p, or,
// when tab is set, entry `slot` of a device table that is written before
// each launch (a captured graph fixes its kernel arguments, the table keeps
// the caller's buffers free to change between replays). In a batch each
// pair has its own table in its workspace, and a plain pointer is a
// workspace buffer: both are offset by z * zs.
template <typename T>
struct IoRef {
    T* p = nullptr;
    void* const* tab = nullptr;
    int slot = 0;
    IoRef() = default;
    __host__ __device__ IoRef(T* ptr) : p(ptr) {}
    __host__ __device__ IoRef(void* const* t, int s) : tab(t), slot(s) {}
    __device__ __forceinline__ T* get(long long zs) const {
        return tab ? static_cast<T*>(zoff(tab, zs)[slot]) : zoff(p, zs);
    }
};

// Slots of a request's caller buffers in the I/O table.
constexpr int kIoRfit = 0, kIoSfit = 1, kIoR = 2, kIoS = 3, kIoCoef = 4, kIoD = 5, kIoSlots = 8;

// A wave-uniform value moved to a scalar register (lane 0's copy).
__device__ __forceinline__ float uniform(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}

// a * b + c with one rounding, in the operands' precision.
__host__ __device__ __forceinline__ float fmat(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmat(double a, double b, double c) { return fma(a, b, c); }

// f(std::integral_constant<int, I>{}) for I = B .. E - 1, in order.
template <int B, int E, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

constexpr int kMaxPass = 8;
constexpr int kMaxDegree = 4;   // largest DK and DB
// Elements of one line held by one thread during a transform.
constexpr int kElemsPerThread = 16;

// Plan of one line of nl points: the transform length n (nl itself when
// nl = 2^a 3^b is a multiple of 16; otherwise the Bluestein length, the
// power of two >= 2 nl - 1), its radix sequence and the thread layout (TL
// threads per line, LPW lines per workgroup). Element t of the line sits in
// register e of thread lt = t mod TL, e = t / TL; t >= nl is padding.
struct LinePlan {
    int n;
    int npass;
    int radix[kMaxPass];
    int twoff[kMaxPass];   // offset of pass p's twiddle table (pass tables)
    int tl;     // threads per line = n / kElemsPerThread
    int lpw;    // lines per workgroup
    int nl;     // points of the line
    // Bluestein (chirp-z) lines, null otherwise: chirp[t] = e^(+i pi t^2 / nl)
    // (t < nl) and bhat = DFT_n(b) / n with b_t = b_(n-t) = chirp[t], both
    // cx<double>.
    const void* chirp;
    const void* bhat;
    // Bluestein lines: e^(-2 pi i t / n), t < n, in the compute type (the
    // transform length's twiddles; null otherwise)
    const void* twm;
};

// Geometry of one subtraction problem (Eq. 1-6): image N0 x N1 (x = axis 0),
// kernel half widths w0, w1, polynomial degrees DK (kernel) and DB
// (background), ConstPhotRatio flag, and every derived count.
struct Geom {
    int n0, n1;
    int h;        // N1/2 + 1: columns of a half spectrum along axis 1
    int hp;       // padded row pitch (complex elements) of half-spectrum arrays
    int w0, w1, dk, db, cp;
    int P, Q;     // kernel / background polynomial term counts
    int L0, L1;   // 2w+1
    int nk, nu;   // kernel unknowns, all unknowns
    int npair;    // P(P+1)/2 kernel-kernel correlation pairs
    int nprod;    // npair + P spectral products per frequency
    int nr;       // real rows fed to the row transform: DK+1 weighted R, and S
    int D0, D1;   // 4w+1: lag range of the kernel-kernel tables
    int nb;       // pairs per launch (gridDim.z), 1 outside a batch
    long long zs; // bytes between the workspaces of consecutive pairs
};

// Monomial index t -> exponents (i, j), i ascending then j ascending.
__host__ __device__ __forceinline__ void term_ij(int deg, int t, int& i, int& j) {
    int c = t;
    for (int a = 0; a <= deg; ++a) {
        int len = deg - a + 1;
        if (c < len) { i = a; j = c; return; }
        c -= len;
    }
    i = j = 0;
}
// (i, j) -> monomial index.
__host__ __device__ __forceinline__ int term_index(int deg, int i, int j) {
    int t = 0;
    for (int a = 0; a < i; ++a) t += deg - a + 1;
    return t + j;
}

// Centred, normalised coordinate c(x) = (2x - (N-1)) / (N-1).
template <typename T>
__host__ __device__ __forceinline__ T coord(int x, int n) {
    return (T(2) * T(x) - T(n - 1)) / T(n - 1);
}

template <typename T>
__host__ __device__ __forceinline__ T ipow(T b, int e) {
    T r = T(1);
    for (int k = 0; k < e; ++k) r *= b;
    return r;
}

// b^e for 0 <= e <= MaxE as a fixed chain of MaxE selected products: the same
// products in the same order as ipow, without a loop on a runtime count.
template <int MaxE, typename T>
__host__ __device__ __forceinline__ T ipow_upto(T b, int e) {
    T r = T(1);
#pragma unroll
    for (int k = 0; k < MaxE; ++k) r = k < e ? r * b : r;
    return r;
}

// Binomial coefficient C(n, k) as a double (small n).
__host__ __device__ __forceinline__ double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
    return r;
}

__host__ __device__ __forceinline__ int imod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

// Kernel unknown u -> (k, a, b) in solver order (k, then a, then b, with the
// (k>0, 0, 0) entries skipped under ConstPhotRatio).
__host__ __device__ __forceinline__ void decode_unknown(const Geom& g, int u, int& k, int& a, int& b) {
    int L = g.L0 * g.L1;
    int rem;
    if (!g.cp || u < L) {
        k = u / L;
        rem = u - k * L;
    } else {
        int up = u - L;
        k = 1 + up / (L - 1);
        rem = up - (k - 1) * (L - 1);
        int centre = g.w0 * g.L1 + g.w1;
        if (rem >= centre) rem += 1;
    }
    a = rem / g.L1 - g.w0;
    b = rem % g.L1 - g.w1;
}

}  // namespace sfft
