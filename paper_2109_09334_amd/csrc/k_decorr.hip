// Noise decorrelation of the difference image (App. C, Eq. C21-C24).
//
// For co-adds of M science images S_j and N reference images R_i with white
// noise sigma_Sj, sigma_Ri, matched by the kernels G_j, H_i (unit kernels for
// single images) and the fitted kernel K, the difference image
//   D = sum_j S_j (x) G_j - [sum_i R_i (x) H_i] (x) K                (Eq. C21)
// has the noise power spectrum
//   den(p) = sum_j sigma_Sj^2 |G^_j(p)|^2 + |K^(p)|^2 sum_i sigma_Ri^2 |H^_i(p)|^2,
// and D (x) Q with Q^(p) = sqrt(den(0) / den(p)) (Eq. C24, scaled to unit
// kernel sum: Q^(0) = 1) has white noise. K is the fitted kernel field at one
// position (its spatial variation is ignored, App. C).
//
// On the device: the stamps (K from the coefficients, G_j, H_i) and their
// row DFTs k_a(m) = sum_b st(a, b) W_N1^(m b) are formed once; the image is
// transformed along axis 1 (rowfwd), then one kernel per column m transforms
// along axis 0, multiplies by Q^(l, m) -- evaluated in place from the row
// DFTs, Kh(l, m) = sum_a W_N0^(l a) k_a(m) -- and transforms back; the row
// inverse (rowinv) ends the convolution.
#include "fft_engine.hpp"
#include "kernels.hpp"

namespace sfft {

// Stamps [nst][L0][L1]: slot 0 the kernel K at (u0, u1) = sum_k kappa_k
// u0^i u1^j (Eq. 5-6 at one point); slots 1..M the G_j; M+1..M+N the H_i (a
// unit stamp where the caller passes none). wts[1..M] = sigma_Sj^2,
// wts[M+1..M+N] = sigma_Ri^2, wts[0] = den(0) from the stamp sums.
__global__ void __launch_bounds__(256) decorr_stamps_kernel(Geom g, const double* __restrict__ kap,
                                                             double u0, double u1, int M,
                                                             const double* __restrict__ sig_s,
                                                             const double* __restrict__ gst, int N,
                                                             const double* __restrict__ sig_r,
                                                             const double* __restrict__ hst,
                                                             double* __restrict__ st,
                                                             double* __restrict__ wts) {
    __shared__ double sums[1 + 2 * kMaxCoadd];
    const int L = g.L0 * g.L1, centre = g.w0 * g.L1 + g.w1;
    const int nst = 1 + M + N;
    for (int t = threadIdx.x; t < nst * L; t += blockDim.x) {
        const int s = t / L, e = t - s * L;
        double v;
        if (s == 0) {
            v = 0.0;
            for (int k = 0; k < g.P; ++k) {
                int i, j;
                term_ij(g.dk, k, i, j);
                v += kap[(size_t)k * L + e] * ipow(u0, i) * ipow(u1, j);
            }
        } else if (s <= M) {
            v = gst ? gst[(size_t)(s - 1) * L + e] : (e == centre ? 1.0 : 0.0);
        } else {
            v = hst ? hst[(size_t)(s - 1 - M) * L + e] : (e == centre ? 1.0 : 0.0);
        }
        st[t] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nst) {
        const int s = threadIdx.x;
        double a = 0.0;
        for (int e = 0; e < L; ++e) a += st[(size_t)s * L + e];
        sums[s] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double gs = 0.0, hs = 0.0;
        for (int j = 0; j < M; ++j) {
            const double v2 = sig_s[j] * sig_s[j];
            wts[1 + j] = v2;
            gs += v2 * sums[1 + j] * sums[1 + j];
        }
        for (int i = 0; i < N; ++i) {
            const double v2 = sig_r[i] * sig_r[i];
            wts[1 + M + i] = v2;
            hs += v2 * sums[1 + M + i] * sums[1 + M + i];
        }
        wts[0] = gs + sums[0] * sums[0] * hs;
    }
}

// One column m of the half spectrum per line: forward transform along axis
// 0, times Q^(l, m) / N0, inverse transform, in place in Z ([N0][hp]).
// kr: row DFTs of the stamps, [nst][L0][hp]; tw: W_N0^t (compute type).
template <typename T, typename PL>
__global__ void __launch_bounds__(512) colconv_kernel(Geom g, LinePlan lp, cx<T>* __restrict__ Z,
                                                       const cx<T>* __restrict__ kr,
                                                       const double* __restrict__ wts, int M, int N,
                                                       const cx<T>* __restrict__ tw,
                                                       const cx<T>* __restrict__ twt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    // groups of 16 adjacent column blocks on one XCD (workgroups are dealt
    // to the 8 XCDs round robin): their strided row reads share L2 lines
    const int ncb = (g.h + lp.lpw - 1) / lp.lpw;
    const int per_xcd = (ncb + 127) / 128 * 16;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int r = slot % per_xcd;
    const int cb = 16 * (8 * (r >> 4) + xcd) + (r & 15);
    const int m = cb * lp.lpw + line;
    const bool act = m < g.h;
    const int n0 = g.n0, w0 = g.w0;
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    cx<T>* zc = Z + m;
    cx<T> v[kElemsPerThread];
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e)   // rows >= n0: a Bluestein line's padding
        v[e] = act && in_line<PL>(lt + e * lp.tl, n0) ? zc[(size_t)(lt + e * lp.tl) * g.hp]
                                                      : mk(T(0), T(0));
    line_dft<-1, T, PL>(v, buf, lp, lt, twt);
    // the column's stamp row DFTs k_(s,a)(m) staged in the line's LDS buffer,
    // free between the two transforms (read from HBM where a short line's
    // buffer cannot hold them)
    const int nst = 1 + M + N, nk = nst * g.L0;
    const bool staged = nk <= line_lds_elems(lp.n);
    __syncthreads();
    if (act && staged)
        for (int i = lt; i < nk; i += lp.tl) buf[i] = kr[(size_t)i * g.hp + m];
    __syncthreads();
    const cx<T>* kb = staged ? buf : kr + m;
    const size_t kst = staged ? 1 : (size_t)g.hp;
    if (act) {
        const T den0 = T(wts[0]);
        const T inv_n0 = T(1) / T(n0);
        // unrolled: v stays in registers (a run-time index would put it in
        // scratch memory)
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int l = lt + e * lp.tl;
            if (!in_line<PL>(l, n0)) continue;
            const cx<T> t1 = tw[l];   // W^l; W^(l a) by the recurrence t <- t W^l
            T gsum = T(0), hsum = T(0), kk = T(0);
#pragma unroll 1
            for (int s = 0; s < nst; ++s) {
                // stamp spectrum at (l, m): k_0 + sum_a W^(l a) k_a + conj(W^(l a)) k_-a
                const cx<T>* ka = kb + (size_t)(s * g.L0 + w0) * kst;
                cx<T> acc = ka[0], t = t1;
#pragma unroll 4
                for (int a = 1; a <= w0; ++a) {
                    acc = acc + cmul(t, ka[(size_t)a * kst]) + cmul(cconj(t), ka[-(ptrdiff_t)a * (ptrdiff_t)kst]);
                    t = cmul(t, t1);
                }
                const T p2 = acc.re * acc.re + acc.im * acc.im;
                if (s == 0)
                    kk = p2;
                else if (s <= M)
                    gsum += T(wts[s]) * p2;
                else
                    hsum += T(wts[s]) * p2;
            }
            const T den = gsum + kk * hsum;
            const T q = sqrt(den0 / den) * inv_n0;
            v[e] = cscale(v[e], q);
        }
    }
    line_dft<1, T, PL>(v, buf, lp, lt, twt);
    if (act) {
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e)
            if (in_line<PL>(lt + e * lp.tl, n0)) zc[(size_t)(lt + e * lp.tl) * g.hp] = v[e];
    }
}

hipError_t launch_decorr_stamps(const Geom& g, const double* kap, double u0, double u1, int M,
                                const double* sig_s, const double* gst, int N, const double* sig_r,
                                const double* hst, double* st, double* wts, hipStream_t st_) {
    if (M < 1 || N < 1 || M > kMaxCoadd || N > kMaxCoadd) return hipErrorInvalidValue;
    hipLaunchKernelGGL(decorr_stamps_kernel, dim3(1), dim3(256), 0, st_, g, kap, u0, u1, M, sig_s,
                       gst, N, sig_r, hst, st, wts);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_colconv(const Geom& g, const LinePlan& lp, cx<T>* Z, const cx<T>* kr,
                          const double* wts, int M, int N, const cx<T>* tw, const cx<T>* twt,
                          hipStream_t st) {
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    const int ncb = (g.h + lp.lpw - 1) / lp.lpw;
    dim3 grid((ncb + 127) / 128 * 128);
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        auto k = colconv_kernel<T, decltype(pl)>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, Z, kr, wts, M, N, tw, twt);
        return hipGetLastError();
    });
}

template hipError_t launch_colconv<float>(const Geom&, const LinePlan&, cx<float>*, const cx<float>*,
                                          const double*, int, int, const cx<float>*,
                                          const cx<float>*, hipStream_t);
template hipError_t launch_colconv<double>(const Geom&, const LinePlan&, cx<double>*,
                                           const cx<double>*, const double*, int, int,
                                           const cx<double>*, const cx<double>*, hipStream_t);

}  // namespace sfft
