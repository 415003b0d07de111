// Normal-matrix gather (Eq. 18 elements through the App. B case rules).
//
// Row u = (kb, ab) and column v = (k, a) of the kernel-kernel block
// (Eq. B5), with Omega_{k kb}(d) = Omega_{kb k}(-d):
//   Omega(ab - a) - [a != 0] Omega(ab) - [ab != 0] Omega(-a) + [both] Omega(0)
// kernel-background (Eq. B7 / B9): Lambda_{kb m}(ab) - [ab != 0] Lambda(0);
// background-background (Eq. B11): C; right-hand side (Eq. B13, B15):
// Theta_kb(ab) - [ab != 0] Theta_kb(0) and E_m.
// Each element is evaluated once for (max(u,v), min(u,v)), so G is exactly
// symmetric, and written row-major with coalesced stores.
#include "kernels.hpp"

namespace sfft {

__device__ __forceinline__ double omega_at(const Geom& g, const double* __restrict__ om, int kb,
                                           int k, int d0, int d1) {
    if (kb > k) {
        const int t = kb;
        kb = k;
        k = t;
        d0 = -d0;
        d1 = -d1;
    }
    const int pr = kb * g.P - kb * (kb - 1) / 2 + (k - kb);
    return om[((size_t)pr * g.D0 + d0 + 2 * g.w0) * g.D1 + d1 + 2 * g.w1];
}

__device__ double g_value(const Geom& g, const double* __restrict__ om,
                          const double* __restrict__ la, const double* __restrict__ cm, int u,
                          int v) {
    // u >= v
    if (u < g.nk) {
        int kb, ab, bb, k, a, b;
        decode_unknown(g, u, kb, ab, bb);
        decode_unknown(g, v, k, a, b);
        const bool zb = (ab == 0 && bb == 0), z = (a == 0 && b == 0);
        if (!zb && !z)
            return omega_at(g, om, kb, k, ab - a, bb - b) - omega_at(g, om, kb, k, ab, bb) -
                   omega_at(g, om, kb, k, -a, -b) + omega_at(g, om, kb, k, 0, 0);
        if (zb && !z) return omega_at(g, om, kb, k, -a, -b) - omega_at(g, om, kb, k, 0, 0);
        if (!zb && z) return omega_at(g, om, kb, k, ab, bb) - omega_at(g, om, kb, k, 0, 0);
        return omega_at(g, om, kb, k, 0, 0);
    }
    const int m = u - g.nk;
    if (v >= g.nk) return cm[m * g.Q + (v - g.nk)];
    int k, a, b;
    decode_unknown(g, v, k, a, b);
    const double* L = la + ((size_t)k * g.Q + m) * g.L0 * g.L1;
    double val = L[(a + g.w0) * g.L1 + b + g.w1];
    if (a || b) val -= L[g.w0 * g.L1 + g.w1];
    return val;
}

__global__ void __launch_bounds__(256) gather_kernel(Geom g, const double* __restrict__ om,
                                                      const double* __restrict__ th,
                                                      const double* __restrict__ la,
                                                      const double* __restrict__ cm,
                                                      const double* __restrict__ ev,
                                                      double* __restrict__ G,
                                                      double* __restrict__ h, int rhs_only) {
    om = zoff(om, g.zs);
    th = zoff(th, g.zs);
    la = zoff(la, g.zs);
    cm = zoff(cm, g.zs);
    ev = zoff(ev, g.zs);
    G = zoff(G, g.zs);
    h = zoff(h, g.zs);
    const int v = blockIdx.x * 64 + (threadIdx.x & 63);
    const int u = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (u >= g.nu) return;
    if (!rhs_only && v < g.nu) G[(size_t)u * g.nu + v] = g_value(g, om, la, cm, max(u, v), min(u, v));
    if (blockIdx.x == 0 && (threadIdx.x & 63) == 0) {
        double val;
        if (u < g.nk) {
            int k, a, b;
            decode_unknown(g, u, k, a, b);
            const double* T = th + (size_t)k * g.L0 * g.L1;
            val = T[(a + g.w0) * g.L1 + b + g.w1];
            if (a || b) val -= T[g.w0 * g.L1 + g.w1];
        } else {
            val = ev[u - g.nk];
        }
        h[u] = val;
    }
}

hipError_t launch_gather(const Geom& g, const double* om, const double* th, const double* la,
                         const double* cm, const double* ev, double* G, double* h, int rhs_only,
                         hipStream_t st) {
    dim3 grid(rhs_only ? 1 : (g.nu + 63) / 64, (g.nu + 3) / 4, g.nb);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, st, g, om, th, la, cm, ev, G, h, rhs_only);
    return hipGetLastError();
}


// The I/O tables of the pairs of a batch: pair z's table lies zs bytes
// after pair z-1's; entry (z, slot) per thread.
__global__ void set_io_kernel(void** io, long long zs, IoBatch b) {
    const int t = threadIdx.x;
    if (t >= b.n * kIoUsed) return;
    const int z = t / kIoUsed, slot = t - z * kIoUsed;
    void** tab = reinterpret_cast<void**>(reinterpret_cast<char*>(io) + (long long)z * zs);
    tab[slot] = const_cast<void*>(b.p[z][slot]);
}

__global__ void __launch_bounds__(256) copy_f64_kernel(IoRef<double> dstr,
                                                       const double* __restrict__ src, int n,
                                                       long long zs) {
    double* __restrict__ dst = dstr.get(zs);
    src = zoff(src, zs);
    if (!dst) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_set_io(void** io, long long zs, const IoBatch& b, hipStream_t st) {
    if (b.n < 1 || b.n > kMaxBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(set_io_kernel, dim3(1), dim3(kMaxBatch * kIoUsed), 0, st, io, zs, b);
    return hipGetLastError();
}

hipError_t launch_copy_f64(const Geom& g, IoRef<double> dst, const double* src, int n,
                           hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_f64_kernel, dim3((n + 255) / 256, 1, g.nb), dim3(256), 0, st, dst, src,
                       n, g.zs);
    return hipGetLastError();
}

}  // namespace sfft
