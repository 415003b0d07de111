// Correlation-lag tables of App. B from the weighted spectra.
//
// For spectra A = DFT[a], B = DFT[b] of real images (forward, e^-),
//   sum_x a(x - d) b(x) = (1/n) Re sum_l conj(A(l)) B(l) e^(+2 pi i l.d / N),
// which gives Omega_{kb k}(d) (Eq. B6, a = R^kb, b = R^k) and
// Theta_kb(d) (Eq. B14, a = R^kb, b = S) in pixel units. Only |d| <= 2w
// (Omega) or |d| <= w (Theta) is needed.
//
// lagcol: per column m of the half spectrum, the product line is inverse
// transformed along axis 0 and the needed lag rows are kept.
// lagrow: the kept rows are inverse transformed along axis 1 over the half
// spectrum (m = 0 and m = N1/2 weight 1, the others weight 2 by Hermitian
// symmetry), accumulated in FP64.
#include "fft_engine.hpp"
#include "kernels.hpp"

namespace sfft {

template <typename T>
__device__ __forceinline__ cx<T>* lds_base_l() {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    return reinterpret_cast<cx<T>*>(smem_raw);
}

__host__ __device__ __forceinline__ void decode_pair(int P, int pr, int& kb, int& k) {
    kb = 0;
    int c = pr;
    while (c >= P - kb) {
        c -= P - kb;
        ++kb;
    }
    k = kb + c;
}

template <typename T>
__global__ void __launch_bounds__(512) lagcol_kernel(Geom g, LinePlan lp, int p0, int sslot,
                                                      const cx<T>* __restrict__ X,
                                                      cx<T>* __restrict__ Cl,
                                                      const cx<T>* __restrict__ tw) {
    cx<T>* lds = lds_base_l<T>();
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    const int m = blockIdx.x * lp.lpw + line;
    const bool act = m < g.h;
    const int p = p0 + blockIdx.y;
    const int n0 = g.n0;
    int kb, k;
    if (p < g.npair) decode_pair(g.P, p, kb, k);
    else { kb = p - g.npair; k = sslot; }
    const int K = p < g.npair ? 2 * g.w0 : g.w0;
    cx<T>* buf = lds + line * lp.n;
    if (act) {
        const cx<T>* A = X + ((size_t)kb * g.h + m) * n0;
        const cx<T>* B = X + ((size_t)k * g.h + m) * n0;
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int l = lt + e * lp.tl;
            buf[l] = cmulc(A[l], B[l]);
        }
    }
    __syncthreads();
    line_fft<1, T>(buf, lp, lt, tw);
    if (act) {
        for (int t = lt; t <= 2 * K; t += lp.tl) {
            const int d0 = t - K;
            Cl[((size_t)p * g.D0 + d0 + 2 * g.w0) * g.hp + m] = buf[imod(d0, n0)];
        }
    }
}

// Block-wide sum of NV doubles per thread; result valid in lane 0 of wave 0
// written to red[0..NV).
template <int NV>
__device__ __forceinline__ void block_sum(double* v, double* red) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double x = v[i];
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[i] = x;
    }
    __syncthreads();
    if (lane == 0)
        for (int i = 0; i < NV; ++i) red[wv * NV + i] = v[i];
    __syncthreads();
    if (threadIdx.x < NV) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += red[w * NV + threadIdx.x];
        red[threadIdx.x] = s;   // each thread reads only its own column above
    }
    __syncthreads();
}

constexpr int kLagChunk = 16;

template <typename T>
__global__ void __launch_bounds__(256) lagrow_kernel(Geom g, int p0, const cx<T>* __restrict__ Cl,
                                                      const double* __restrict__ twp,
                                                      double* __restrict__ omega,
                                                      double* __restrict__ theta) {
    __shared__ double red[4 * kLagChunk + kLagChunk];
    const int p = p0 + blockIdx.y;
    const int r = blockIdx.x;            // row index: d0 = r - 2 w0
    const bool om = p < g.npair;
    const int K0 = om ? 2 * g.w0 : g.w0, K1 = om ? 2 * g.w1 : g.w1;
    const int d0 = r - 2 * g.w0;
    if (d0 < -K0 || d0 > K0) return;     // uniform over the block
    const int n1 = g.n1;
    const double inv_n = 1.0 / ((double)g.n0 * (double)n1);
    const cx<T>* row = Cl + ((size_t)p * g.D0 + r) * g.hp;
    for (int base = -K1; base <= K1; base += kLagChunk) {
        double acc[kLagChunk];
#pragma unroll
        for (int t = 0; t < kLagChunk; ++t) acc[t] = 0.0;
        for (int m = threadIdx.x; m < g.h; m += blockDim.x) {
            const cx<T> c = row[m];
            const double wm = (m == 0 || 2 * m == n1) ? 1.0 : 2.0;
            const double cr = wm * (double)c.re, ci = wm * (double)c.im;
#pragma unroll
            for (int t = 0; t < kLagChunk; ++t) {
                const int d1 = base + t;
                if (d1 <= K1) {
                    const int idx = imod(m * d1, n1);
                    acc[t] += cr * twp[2 * idx] - ci * twp[2 * idx + 1];
                }
            }
        }
        block_sum<kLagChunk>(acc, red);
        if (threadIdx.x < kLagChunk) {
            const int d1 = base + threadIdx.x;
            if (d1 <= K1) {
                const double v = red[threadIdx.x] * inv_n;
                if (om)
                    omega[((size_t)p * g.D0 + r) * g.D1 + d1 + 2 * g.w1] = v;
                else
                    theta[((size_t)(p - g.npair) * g.L0 + d0 + g.w0) * g.L1 + d1 + g.w1] = v;
            }
        }
        __syncthreads();
    }
}

template <typename T>
hipError_t launch_lagcol(const Geom& g, const LinePlan& lp, int p0, int p1, int sslot,
                         const cx<T>* X, cx<T>* Cl, const cx<T>* tw, hipStream_t st) {
    if (p1 <= p0) return hipSuccess;
    const size_t lds = (size_t)lp.lpw * lp.n * sizeof(cx<T>);
    auto k = lagcol_kernel<T>;
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    dim3 grid((g.h + lp.lpw - 1) / lp.lpw, p1 - p0);
    hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, p0, sslot, X, Cl, tw);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lagrow(const Geom& g, int p0, int p1, const cx<T>* Cl, const double* twp,
                         double* omega, double* theta, hipStream_t st) {
    if (p1 <= p0) return hipSuccess;
    dim3 grid(g.D0, p1 - p0);
    hipLaunchKernelGGL(lagrow_kernel<T>, grid, dim3(256), 0, st, g, p0, Cl, twp, omega, theta);
    return hipGetLastError();
}

template hipError_t launch_lagcol<float>(const Geom&, const LinePlan&, int, int, int,
                                         const cx<float>*, cx<float>*, const cx<float>*, hipStream_t);
template hipError_t launch_lagcol<double>(const Geom&, const LinePlan&, int, int, int,
                                          const cx<double>*, cx<double>*, const cx<double>*,
                                          hipStream_t);
template hipError_t launch_lagrow<float>(const Geom&, int, int, const cx<float>*, const double*,
                                         double*, double*, hipStream_t);
template hipError_t launch_lagrow<double>(const Geom&, int, int, const cx<double>*, const double*,
                                          double*, double*, hipStream_t);

}  // namespace sfft
