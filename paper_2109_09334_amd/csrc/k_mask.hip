// Crowded-flavour preprocessing of the fit pair (Sec. 3.1).
//
// Pixels affected by saturated sources are masked in both images and
// replaced by the neighbouring background, giving the fit pair
// (R-breve, S-breve); the unmasked images stay the apply pair. The paper
// fixes no details; the reading implemented here:
//  * saturated: not (R < u_R and S < u_S) -- a non-finite pixel included;
//  * affected: a saturated pixel within the kernel footprint, at x + (a, b)
//    with |a| <= g0, |b| <= g1, offsets circular as in Eq. 12;
//  * background: per tile of t0 x t1 pixels (the last tiles ragged), the
//    lower median -- element (m - 1) / 2 of the m unmasked values in
//    ascending order; a tile with none takes the lower median of the other
//    tiles' backgrounds (0 if every pixel is masked);
//  * masked pixels take their tile's background, the others keep theirs.
// Every step is a comparison or a selection, so the result is exact (the
// same bits as any correct evaluation in the image's precision).
#include <algorithm>

#include "kernels.hpp"

namespace sfft {

template <typename Tin>
__global__ void __launch_bounds__(256) sat_kernel(long long n, const Tin* __restrict__ r,
                                                   const Tin* __restrict__ s, Tin ur, Tin us,
                                                   unsigned char* __restrict__ sat) {
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        sat[i] = (r[i] < ur && s[i] < us) ? 0 : 1;
}

// out(x0, x1) = OR of in over the circular window of half width g along one
// axis (axis 1: contiguous, axis 0: strided by n1).
template <int AXIS>
__global__ void __launch_bounds__(256) dilate_kernel(int n0, int n1, int g,
                                                      const unsigned char* __restrict__ in,
                                                      unsigned char* __restrict__ out) {
    const long long n = (long long)n0 * n1;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int x0 = (int)(i / n1), x1 = (int)(i - (long long)x0 * n1);
        unsigned char v = 0;
        for (int a = -g; a <= g; ++a) {
            if (AXIS == 1) {
                int y = x1 + a;
                y += y < 0 ? n1 : 0;
                y -= y >= n1 ? n1 : 0;
                v |= in[(long long)x0 * n1 + y];
            } else {
                int y = x0 + a;
                y += y < 0 ? n0 : 0;
                y -= y >= n0 ? n0 : 0;
                v |= in[(long long)y * n1 + x1];
            }
        }
        out[i] = v;
    }
}

// In-place ascending bitonic sort of p2 (a power of two) values in LDS.
template <typename T>
__device__ void bitonic_sort(T* v, int p2) {
    for (int k = 2; k <= p2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < p2; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const T a = v[i], b = v[l];
                    if ((a > b) == up) {
                        v[i] = b;
                        v[l] = a;
                    }
                }
            }
        }
    }
    __syncthreads();
}

__device__ __forceinline__ float pad_max(float) { return __builtin_inff(); }
__device__ __forceinline__ double pad_max(double) { return __builtin_inf(); }

// One workgroup per (tile, image): the lower median of the tile's unmasked
// pixels, or an empty flag. blockIdx.y: 0 = R, 1 = S.
template <typename Tin>
__global__ void __launch_bounds__(256) tile_median_kernel(int n0, int n1, int t0, int t1, int p2,
                                                           const Tin* __restrict__ r,
                                                           const Tin* __restrict__ s,
                                                           const unsigned char* __restrict__ mask,
                                                           Tin* __restrict__ bg,
                                                           unsigned char* __restrict__ empty) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Tin* v = reinterpret_cast<Tin*>(smem_raw);
    __shared__ int cnt;
    const int nt1 = (n1 + t1 - 1) / t1, ntiles = ((n0 + t0 - 1) / t0) * nt1;
    const int tile = blockIdx.x, ti = tile / nt1, tj = tile - ti * nt1;
    const Tin* img = blockIdx.y ? s : r;
    const int r0 = ti * t0, c0 = tj * t1;
    const int h0 = min(t0, n0 - r0), h1 = min(t1, n1 - c0);
    if (threadIdx.x == 0) cnt = 0;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) v[i] = pad_max(Tin(0));
    __syncthreads();
    // unmasked values in any order (the sort below orders them)
    for (int e = threadIdx.x; e < h0 * h1; e += blockDim.x) {
        const long long px = (long long)(r0 + e / h1) * n1 + c0 + e % h1;
        if (!mask[px]) v[atomicAdd(&cnt, 1)] = img[px];
    }
    __syncthreads();
    const int m = cnt;
    bitonic_sort(v, p2);
    if (threadIdx.x == 0) {
        const size_t o = (size_t)blockIdx.y * ntiles + tile;
        bg[o] = m ? v[(m - 1) / 2] : Tin(0);
        empty[o] = m ? 0 : 1;
    }
}

// One workgroup per image: the lower median of the non-empty tiles'
// backgrounds written into the empty tiles (0 when all are empty).
template <typename Tin>
__global__ void __launch_bounds__(256) tile_fallback_kernel(int ntiles, int p2, Tin* __restrict__ bg,
                                                             const unsigned char* __restrict__ empty) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Tin* v = reinterpret_cast<Tin*>(smem_raw);
    __shared__ int cnt;
    Tin* b = bg + (size_t)blockIdx.x * ntiles;
    const unsigned char* em = empty + (size_t)blockIdx.x * ntiles;
    if (threadIdx.x == 0) cnt = 0;
    for (int i = threadIdx.x; i < p2; i += blockDim.x) v[i] = pad_max(Tin(0));
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        if (!em[t]) v[atomicAdd(&cnt, 1)] = b[t];
    __syncthreads();
    const int m = cnt;
    if (m == ntiles) return;   // uniform: no empty tile
    bitonic_sort(v, p2);
    const Tin fb = m ? v[(m - 1) / 2] : Tin(0);
    for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
        if (em[t]) b[t] = fb;
}

// (ro, so may be r, s: each element is read, then written, by one thread.)
template <typename Tin>
__global__ void __launch_bounds__(256) fill_kernel(int n0, int n1, int t0, int t1, const Tin* r,
                                                    const Tin* s,
                                                    const unsigned char* __restrict__ mask,
                                                    const Tin* __restrict__ bg, Tin* ro, Tin* so,
                                                    unsigned char* __restrict__ mask_out) {
    const long long n = (long long)n0 * n1;
    const int nt1 = (n1 + t1 - 1) / t1, ntiles = ((n0 + t0 - 1) / t0) * nt1;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const int x0 = (int)(i / n1), x1 = (int)(i - (long long)x0 * n1);
        const int t = (x0 / t0) * nt1 + x1 / t1;
        const bool m = mask[i] != 0;
        ro[i] = m ? bg[t] : r[i];
        so[i] = m ? bg[ntiles + t] : s[i];
        if (mask_out) mask_out[i] = m ? 1 : 0;
    }
}

static int pow2_at_least(int n) {
    int p = 1;
    while (p < n) p <<= 1;
    return p;
}

template <typename Tin>
hipError_t launch_crowded_mask(int n0, int n1, const Tin* r, const Tin* s, double ur, double us,
                               int g0, int g1, int t0, int t1, unsigned char* sat,
                               unsigned char* tmp, Tin* bg, unsigned char* empty, Tin* ro, Tin* so,
                               unsigned char* mask_out, hipStream_t st) {
    const long long n = (long long)n0 * n1;
    const int grid = (int)std::min<long long>((n + 255) / 256, 8192);
    const int nt0 = (n0 + t0 - 1) / t0, nt1 = (n1 + t1 - 1) / t1, ntiles = nt0 * nt1;
    hipLaunchKernelGGL(sat_kernel<Tin>, dim3(grid), dim3(256), 0, st, n, r, s, Tin(ur), Tin(us), sat);
    hipLaunchKernelGGL(dilate_kernel<1>, dim3(grid), dim3(256), 0, st, n0, n1, g1, sat, tmp);
    hipLaunchKernelGGL(dilate_kernel<0>, dim3(grid), dim3(256), 0, st, n0, n1, g0, tmp, sat);
    const int p2 = pow2_at_least(t0 * t1);
    hipLaunchKernelGGL(tile_median_kernel<Tin>, dim3(ntiles, 2), dim3(256), p2 * sizeof(Tin), st, n0,
                       n1, t0, t1, p2, r, s, sat, bg, empty);
    const int q2 = pow2_at_least(ntiles);
    const size_t lds = (size_t)q2 * sizeof(Tin);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(tile_fallback_kernel<Tin>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(tile_fallback_kernel<Tin>, dim3(2), dim3(256), lds, st, ntiles, q2, bg, empty);
    hipLaunchKernelGGL(fill_kernel<Tin>, dim3(grid), dim3(256), 0, st, n0, n1, t0, t1, r, s, sat, bg,
                       ro, so, mask_out);
    return hipGetLastError();
}

template hipError_t launch_crowded_mask<float>(int, int, const float*, const float*, double, double,
                                               int, int, int, int, unsigned char*, unsigned char*,
                                               float*, unsigned char*, float*, float*,
                                               unsigned char*, hipStream_t);
template hipError_t launch_crowded_mask<double>(int, int, const double*, const double*, double,
                                                double, int, int, int, int, unsigned char*,
                                                unsigned char*, double*, unsigned char*, double*,
                                                double*, unsigned char*, hipStream_t);

}  // namespace sfft
