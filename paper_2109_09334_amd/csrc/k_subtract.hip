// Difference image D = S - sum_k R^k o kappa_k - B (Eq. 12-13).
//
// Stamps: kappa_k(a) = c_(k,a) for a != 0 and kappa_k(0) = c_(k,0) minus the
// off-centre sum (delta basis of Eq. 3-4). The convolution runs spectrally
// along axis 1 and directly along axis 0: with the row spectra
// Z_j(x0, m) = DFT_row[c1^j R](x0, m), the shift by a1 is the factor
// W_N1^(m a1) of Eq. 14, so
//   Dt(x0, m) = Z_S(x0, m) - sum_j sum_a0 Z_j(x0 - a0, m)
//               sum_i Kt_(i,j)(a0, m) c0(x0 - a0)^i,
//   Kt_k(a0, m) = sum_a1 kappa_k(a0, a1) W_N1^(m a1),
// a (2 w0 + 1)-tap stencil along x0 per column m; the row inverse (k_fft)
// then gives D and subtracts the smooth FP64 part tabulated by sky_kernel
// (the background polynomial and, when the transforms ran on the pedestal-
// free pair R - c_R, S - c_S, the pedestal terms c_R (1 o K) - c_S).
#include "kernels.hpp"

namespace sfft {

// Coefficient index of kernel unknown (k, a, b), or -1 when it is fixed
// (ConstPhotRatio centre entries of k > 0).
__device__ __forceinline__ int coef_index(const Geom& g, int k, int a, int b) {
    const int L = g.L0 * g.L1;
    int rem = (a + g.w0) * g.L1 + (b + g.w1);
    if (!g.cp) return k * L + rem;
    if (k == 0) return rem;
    const int centre = g.w0 * g.L1 + g.w1;
    if (rem == centre) return -1;
    if (rem > centre) rem -= 1;
    return L + (k - 1) * (L - 1) + rem;
}

__global__ void __launch_bounds__(256) stamps_kernel(Geom g, const double* __restrict__ coef,
                                                      double* __restrict__ kap) {
    __shared__ double red[4];
    coef = zoff(coef, g.zs);
    kap = zoff(kap, g.zs);
    const int k = blockIdx.x;
    const int L = g.L0 * g.L1;
    double off = 0.0;
    for (int t = threadIdx.x; t < L; t += blockDim.x) {
        const int a = t / g.L1 - g.w0, b = t % g.L1 - g.w1;
        const int ci = coef_index(g, k, a, b);
        const double c = ci >= 0 ? coef[ci] : 0.0;
        kap[(size_t)k * L + t] = c;
        if (a || b) off += c;
    }
    for (int o = 32; o > 0; o >>= 1) off += __shfl_down(off, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = off;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        const int ci = coef_index(g, k, 0, 0);
        kap[(size_t)k * L + g.w0 * g.L1 + g.w1] = (ci >= 0 ? coef[ci] : 0.0) - s;
    }
}

template <typename T>
__global__ void __launch_bounds__(256) stamp_spectra_kernel(Geom g, const double* __restrict__ kap,
                                                             const double* __restrict__ twp,
                                                             cx<T>* __restrict__ Kt) {
    kap = zoff(kap, g.zs);
    Kt = zoff(Kt, g.zs);
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    const int row = blockIdx.y;   // k * L0 + a0 index
    if (m >= g.h) return;
    const double* kr = kap + (size_t)row * g.L1;
    double re = 0.0, im = 0.0;
    for (int b = -g.w1; b <= g.w1; ++b) {
        const int idx = imod(m * b, g.n1);
        // W^(m b) = e^(-2 pi i m b / N1) = conj(twp[idx])
        re += kr[b + g.w1] * twp[2 * idx];
        im -= kr[b + g.w1] * twp[2 * idx + 1];
    }
    Kt[(size_t)row * g.hp + m] = mk(T(re), T(im));
}

// Smooth part of the difference image, in FP64:
//   sky(x) = B(x) + c_R V(x) - c_S,
//   V(x) = sum_k sum_a kappa_k(a) T^k((x - a) mod N)   (V = 1 o K, Eq. 12),
// so that D = IDFT[Dt] - sky with Dt from the pedestal-free spectra (c_R =
// c_S = 0 when the transforms ran on R and S themselves: sky = B). Rows
// w0 <= x0 < N0 - w0 see no wrap along axis 0, where c0(x0 - a0) =
// c0(x0) + s_a0 with s_a0 = -2 a0 / (N0 - 1); there
//   sky(x0, x1) = sum_r c0(x0)^r Y_r(x1),
// and the 2 w0 edge rows (0..w0-1, N0-w0..N0-1) are tabulated as they are.
// Every table row rho is a 1-D correlation along axis 1,
//   c_R sum_k sum_a1 kappa'_(rho,k)(a1) c1((x1 - a1) mod N1)^(j_k) + (B, c_S terms),
//   kappa'_(rho,k)(a1) = sum_a0 omega_rho(a0, i_k) kappa_k(a0, a1),
// omega_r(a0, i) = C(i, r) s_a0^(i-r) (r <= i) for Y_r, and
// omega_e(a0, i) = c0((x0_e - a0) mod N0)^i for edge row e.
// Table: sky[r][x1] for r <= max(DK, DB), then edge row e at
// sky[max(DK, DB) + 1 + e][x1].
__global__ void __launch_bounds__(256) sky_stamps_kernel(Geom g, const double* __restrict__ kap,
                                                          double* __restrict__ kap1) {
    kap = zoff(kap, g.zs);
    kap1 = zoff(kap1, g.zs);
    const int rho = blockIdx.x;
    const int R = max(g.dk, g.db);
    const int L = g.L0 * g.L1;
    for (int t = threadIdx.x; t < g.P * g.L1; t += blockDim.x) {
        const int k = t / g.L1, b = t % g.L1;
        int i, j;
        term_ij(g.dk, k, i, j);
        double v = 0.0;
        for (int a0 = -g.w0; a0 <= g.w0; ++a0) {
            double om;
            if (rho <= R) {
                om = rho <= i ? binom(i, rho) * ipow(-2.0 * (double)a0 / (double)(g.n0 - 1), i - rho)
                              : 0.0;
            } else {
                const int e = rho - R - 1;
                const int x0 = e < g.w0 ? e : g.n0 - 2 * g.w0 + e;
                om = ipow(coord<double>(imod(x0 - a0, g.n0), g.n0), i);
            }
            v += om * kap[(size_t)k * L + (a0 + g.w0) * g.L1 + b];
        }
        kap1[((size_t)rho * g.P + k) * g.L1 + b] = v;
    }
}

constexpr int kSkyThreads = 64;
constexpr int kMaxHalfWidth = 16;                                      // largest w0, w1

__global__ void __launch_bounds__(kSkyThreads) sky_kernel(Geom g, const double* __restrict__ kap1,
                                                          const double* __restrict__ bcoef,
                                                          const double* __restrict__ ped,
                                                          double* __restrict__ sky) {
    // this rho's 1-D stamps summed over the kernel terms of equal axis-1
    // degree j, kj[j][b] (j <= DK, |b| <= w1), staged once per block
    __shared__ double kj[(kMaxDegree + 1) * (2 * kMaxHalfWidth + 1)];
    kap1 = zoff(kap1, g.zs);
    bcoef = zoff(bcoef, g.zs);
    ped = zoff(ped, g.zs);
    sky = zoff(sky, g.zs);
    const int x1 = blockIdx.x * kSkyThreads + threadIdx.x;
    const int rho = blockIdx.y;
    const int n1 = g.n1, w1 = g.w1, L1 = g.L1;
    const int R = max(g.dk, g.db);
    const double cR = ped ? ped[0] : 0.0, cS = ped ? ped[1] : 0.0;
    if (cR != 0.0) {
        const double* src = kap1 + (size_t)rho * g.P * L1;
        for (int t = threadIdx.x; t < (g.dk + 1) * L1; t += blockDim.x) {
            const int jj = t / L1, b = t - jj * L1;
            double s = 0.0;
            for (int k = 0; k < g.P; ++k) {
                int i, j;
                term_ij(g.dk, k, i, j);
                if (j == jj) s += src[(size_t)k * L1 + b];
            }
            kj[t] = s;
        }
        __syncthreads();
    }
    if (x1 >= g.n1) return;
    double v = 0.0;
    if (cR != 0.0) {
        // sum over the taps b of (Horner over j in c1 of the source column
        // x1 - b), four taps at a time in separate partial sums
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int b0 = -w1; b0 <= w1; b0 += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int b = b0 + u;
                if (b > w1) break;
                int xs = x1 - b;   // |b| < N1: one wrap at most
                xs += xs < 0 ? n1 : 0;
                xs -= xs >= n1 ? n1 : 0;
                const double c = coord<double>(xs, n1);
                double p = kj[g.dk * L1 + b + w1];
                for (int jj = g.dk - 1; jj >= 0; --jj) p = p * c + kj[jj * L1 + b + w1];
                acc[u] += p;
            }
        }
        v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) * cR;
    }
    const double c1 = coord<double>(x1, n1);
    const bool edge = rho > R;
    const int e = rho - R - 1;
    const double c0 = edge ? coord<double>(e < g.w0 ? e : g.n0 - 2 * g.w0 + e, g.n0) : 0.0;
    for (int m = 0; m < g.Q; ++m) {
        int p, q;
        term_ij(g.db, m, p, q);
        const double t = bcoef[m] * ipow(c1, q);
        if (edge) v += t * ipow(c0, p);
        else if (p == rho) v += t;
    }
    if (edge || rho == 0) v -= cS;
    sky[(size_t)rho * n1 + x1] = v;
}

// Tile: 64 columns x kStTile rows per block of 256 threads (4 row groups of
// kStRows rows per thread). The (kStTile + 2 w0) source rows of one row
// spectrum Z_j are staged in LDS at a time, so each Z element is read from
// HBM once per tile instead of 2 w0 + 1 times; the stamp spectra of the
// thread's column are loaded once per tap.
constexpr int kStCols = 64;
constexpr int kStRows = 8;
constexpr int kStTile = 4 * kStRows;

template <typename T>
__global__ void __launch_bounds__(256) stencil_kernel(Geom g, const cx<T>* __restrict__ Z, int zs,
                                                       const cx<T>* __restrict__ Kt,
                                                       cx<T>* __restrict__ Dt) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Z = zoff(Z, g.zs);
    Kt = zoff(Kt, g.zs);
    Dt = zoff(Dt, g.zs);
    const int nsrc = kStTile + 2 * g.w0;
    cx<T>* zt = reinterpret_cast<cx<T>*>(smem_raw);            // [nsrc][kStCols]
    T* ct = reinterpret_cast<T*>(zt + (size_t)nsrc * kStCols);  // [nsrc] source coordinates
    const int mc = threadIdx.x & 63, rg = threadIdx.x >> 6;
    const int m = blockIdx.x * kStCols + mc;
    const int x0b = blockIdx.y * kStTile;
    const int n0 = g.n0;
    const bool mok = m < g.h;
    const size_t plane = (size_t)n0 * g.hp;
    for (int r = threadIdx.x; r < nsrc; r += blockDim.x)
        ct[r] = coord<T>(imod(x0b - g.w0 + r, n0), n0);
    cx<T> acc[kStRows];
#pragma unroll
    for (int o = 0; o < kStRows; ++o) {
        const int x0 = x0b + rg * kStRows + o;
        acc[o] = mk(T(0), T(0));
        if (mok && x0 < n0) acc[o] = Z[(size_t)zs * plane + (size_t)x0 * g.hp + m];
    }
    for (int j = 0; j <= g.dk; ++j) {
        __syncthreads();
        const cx<T>* Zj = Z + (size_t)j * plane;
        for (int r = rg; r < nsrc; r += 4) {
            const int xs = imod(x0b - g.w0 + r, n0);
            zt[r * kStCols + mc] = mok ? Zj[(size_t)xs * g.hp + m] : mk(T(0), T(0));
        }
        __syncthreads();
        const int ni = g.dk - j;   // polynomial degree in c0 for this j
        for (int a0 = -g.w0; a0 <= g.w0; ++a0) {
            cx<T> kt[5];
#pragma unroll
            for (int i = 0; i < 5; ++i)
                kt[i] = (i <= ni && mok)
                            ? Kt[((size_t)term_index(g.dk, i, j) * g.L0 + a0 + g.w0) * g.hp + m]
                            : mk(T(0), T(0));
#pragma unroll
            for (int o = 0; o < kStRows; ++o) {
                const int r = rg * kStRows + o + g.w0 - a0;   // source row in the tile
                const cx<T> z = zt[r * kStCols + mc];
                const T c = ct[r];
                // sum_i kt[i] c^i, i <= ni (ni is uniform over the block)
                cx<T> poly = kt[0];
                T cp = c;
#pragma unroll
                for (int i = 1; i < 5; ++i) {
                    if (i <= ni) {
                        poly.re += kt[i].re * cp;
                        poly.im += kt[i].im * cp;
                        cp *= c;
                    }
                }
                acc[o] = acc[o] - cmul(poly, z);
            }
        }
    }
#pragma unroll
    for (int o = 0; o < kStRows; ++o) {
        const int x0 = x0b + rg * kStRows + o;
        if (mok && x0 < n0) Dt[(size_t)x0 * g.hp + m] = acc[o];
    }
}

// Register-resident stencil for compile-time (DK, W0): each thread owns NO
// consecutive output rows of one column m and holds the NO + 2 W0 source rows
// of each row spectrum Z_j in registers (read straight from HBM; neighbouring
// threads of the same column share them through the caches), so every tap
// is FMAs on registers:
//   Dt(x0, m) = Z_S(x0, m) - sum_j sum_a0 Z_j(x0 - a0, m) poly_j(a0, m, x0 - a0),
//   poly_j = sum_(i <= DK - j) Kt_(i,j)(a0, m) c0(x0 - a0)^i (Horner).
// The block's stamp spectra (P x (2 W0 + 1) x 64 columns) are staged in LDS
// once; a scheduling barrier between taps keeps the compiler from hoisting
// every tap's stamp values into registers at once.
// 64 columns x 4 row groups per 256-thread block.
template <typename T, int DK, int W0, int NO>
__global__ void __launch_bounds__(256) stencil_reg_kernel(Geom g, const cx<T>* __restrict__ Z,
                                                           int zs, const cx<T>* __restrict__ Kt,
                                                           cx<T>* __restrict__ Dt) {
    constexpr int NS = NO + 2 * W0;
    constexpr int L0 = 2 * W0 + 1;
    constexpr int P = (DK + 1) * (DK + 2) / 2;
    __shared__ cx<T> ktl[P * L0][64];
    Z = zoff(Z, g.zs);
    Kt = zoff(Kt, g.zs);
    Dt = zoff(Dt, g.zs);
    const int mc = threadIdx.x & 63;
    const int m = blockIdx.x * 64 + mc;
    // one wave per row group: x0b, the source rows and their coordinates are
    // wave-uniform and kept in scalar registers
    const int x0b = __builtin_amdgcn_readfirstlane((blockIdx.y * 4 + (threadIdx.x >> 6)) * NO);
    const int n0 = g.n0;
    const bool mok = m < g.h;
    for (int t = threadIdx.x >> 6; t < P * L0; t += 4)
        ktl[t][mc] = mok ? Kt[(size_t)t * g.hp + m] : mk(T(0), T(0));
    __syncthreads();
    if (!mok || x0b >= n0) return;   // no barriers below
    const size_t plane = (size_t)n0 * g.hp;
    int xs[NS];
    T cs[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        xs[s] = imod(x0b - W0 + s, n0);
        cs[s] = uniform(coord<T>(xs[s], n0));
    }
    cx<T> acc[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o)
        acc[o] = x0b + o < n0 ? Z[(size_t)zs * plane + (size_t)(x0b + o) * g.hp + m] : mk(T(0), T(0));
    // Horner over degree DK - j in c0 of the source row. The j loop stays a
    // runtime loop (one set of source rows live at a time); its body is
    // compiled once per degree and picked by a switch.
#pragma unroll 1
    for (int j = 0; j <= DK; ++j) {
        const cx<T>* Zj = Z + (size_t)j * plane + m;
        // row offsets formed per j (an opaque zero keeps them out of the
        // registers held across the loop)
        const int oz = opaque_zero();
        cx<T> z[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) z[s] = Zj[(size_t)(xs[s] + oz) * g.hp];
        auto taps = [&](auto ni_c) {
            constexpr int NI = decltype(ni_c)::value;
#pragma unroll
            for (int a = 0; a < L0; ++a) {   // tap a0 = a - W0
                cx<T> kt[NI + 1];
#pragma unroll
                for (int i = 0; i <= NI; ++i) kt[i] = ktl[term_index(DK, i, DK - NI) * L0 + a][mc];
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    const int s = o + 2 * W0 - a;   // source row x0 - a0
                    const T c = cs[s];
                    cx<T> poly = kt[NI];
#pragma unroll
                    for (int i = NI - 1; i >= 0; --i)
                        poly = mk(fmat(poly.re, c, kt[i].re), fmat(poly.im, c, kt[i].im));
                    // two FMAs per component into the accumulator: two
                    // roundings per tap at its magnitude (|Z_S|, far above
                    // the result) against one for forming the tap's term
                    // first, for 4 instead of 6 instructions per tap
                    acc[o].re = fmat(-poly.re, z[s].re, fmat(poly.im, z[s].im, acc[o].re));
                    acc[o].im = fmat(-poly.re, z[s].im, fmat(-poly.im, z[s].re, acc[o].im));
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        static_for<0, DK + 1>([&](auto ni_c) {
            if (DK - j == decltype(ni_c)::value) taps(ni_c);
        });
    }
#pragma unroll
    for (int o = 0; o < NO; ++o)
        if (x0b + o < n0) Dt[(size_t)(x0b + o) * g.hp + m] = acc[o];
}

template <typename T, int DK, int W0>
static hipError_t launch_stencil_reg(const Geom& g, const cx<T>* Z, int zs, const cx<T>* Kt,
                                     cx<T>* Dt, hipStream_t st) {
    constexpr int NO = 16;
    dim3 grid((g.h + 63) / 64, (g.n0 + 4 * NO - 1) / (4 * NO), g.nb);
    hipLaunchKernelGGL((stencil_reg_kernel<T, DK, W0, NO>), grid, dim3(256), 0, st, g, Z, zs, Kt, Dt);
    return hipGetLastError();
}

// Specialised (DK, w0) pairs; false when the generic kernel must run.
template <typename T, int DK>
static bool stencil_reg_w(const Geom& g, const cx<T>* Z, int zs, const cx<T>* Kt, cx<T>* Dt,
                          hipStream_t st, hipError_t* e) {
    switch (g.w0) {
        case 2: *e = launch_stencil_reg<T, DK, 2>(g, Z, zs, Kt, Dt, st); return true;
        case 3: *e = launch_stencil_reg<T, DK, 3>(g, Z, zs, Kt, Dt, st); return true;
        case 4: *e = launch_stencil_reg<T, DK, 4>(g, Z, zs, Kt, Dt, st); return true;
        case 5: *e = launch_stencil_reg<T, DK, 5>(g, Z, zs, Kt, Dt, st); return true;
        case 7: *e = launch_stencil_reg<T, DK, 7>(g, Z, zs, Kt, Dt, st); return true;
        default: return false;
    }
}

hipError_t launch_stamps(const Geom& g, const double* coef, double* kap, hipStream_t st) {
    hipLaunchKernelGGL(stamps_kernel, dim3(g.P, 1, g.nb), dim3(256), 0, st, g, coef, kap);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stamp_spectra(const Geom& g, const double* kap, const double* twp, cx<T>* Kt,
                                hipStream_t st) {
    hipLaunchKernelGGL(stamp_spectra_kernel<T>, dim3((g.h + 255) / 256, g.P * g.L0, g.nb), dim3(256), 0,
                       st, g, kap, twp, Kt);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_stencil(const Geom& g, const cx<T>* Z, int zs_index, const cx<T>* Kt, cx<T>* Dt,
                          hipStream_t st) {
    hipError_t e = hipSuccess;
    bool done = false;
    // the register form for the FP32 transforms (in FP64 its register
    // footprint spills for the larger kernels)
    if constexpr (sizeof(T) == 4) {
        switch (g.dk) {
            case 0: done = stencil_reg_w<T, 0>(g, Z, zs_index, Kt, Dt, st, &e); break;
            case 1: done = stencil_reg_w<T, 1>(g, Z, zs_index, Kt, Dt, st, &e); break;
            case 2: done = stencil_reg_w<T, 2>(g, Z, zs_index, Kt, Dt, st, &e); break;
            default: break;
        }
    }
    if (done) return e;
    const size_t nsrc = kStTile + 2 * g.w0;
    const size_t lds = nsrc * kStCols * sizeof(cx<T>) + nsrc * sizeof(T);
    if (lds > 65536) {
        e = hipFuncSetAttribute(reinterpret_cast<const void*>(stencil_kernel<T>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(stencil_kernel<T>, dim3((g.h + kStCols - 1) / kStCols, (g.n0 + kStTile - 1) / kStTile, g.nb),
                       dim3(256), lds, st, g, Z, zs_index, Kt, Dt);
    return hipGetLastError();
}

hipError_t launch_sky(const Geom& g, const double* kap, const double* bcoef, const double* ped,
                      double* kap1, double* sky, hipStream_t st) {
    if (g.dk > kMaxDegree || g.db > kMaxDegree || g.w1 > kMaxHalfWidth) return hipErrorInvalidValue;
    const int nrho = max(g.dk, g.db) + 1 + 2 * g.w0;
    if (ped) hipLaunchKernelGGL(sky_stamps_kernel, dim3(nrho, 1, g.nb), dim3(256), 0, st, g, kap, kap1);
    hipLaunchKernelGGL(sky_kernel, dim3((g.n1 + kSkyThreads - 1) / kSkyThreads, nrho, g.nb),
                       dim3(kSkyThreads), 0, st, g, kap1, bcoef, ped, sky);
    return hipGetLastError();
}

template hipError_t launch_stamp_spectra<float>(const Geom&, const double*, const double*,
                                                cx<float>*, hipStream_t);
template hipError_t launch_stamp_spectra<double>(const Geom&, const double*, const double*,
                                                 cx<double>*, hipStream_t);
template hipError_t launch_stencil<float>(const Geom&, const cx<float>*, int, const cx<float>*,
                                          cx<float>*, hipStream_t);
template hipError_t launch_stencil<double>(const Geom&, const cx<double>*, int, const cx<double>*,
                                           cx<double>*, hipStream_t);

}  // namespace sfft
