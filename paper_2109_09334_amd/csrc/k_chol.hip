// FP64 solve of the normal equations G c = h (the solution of Eq. 18).
//
// Jacobi scaling d = diag(G)^-1/2 keeps the factor well scaled; the scaled
// matrix D G D is factorised by a blocked right-looking Cholesky (64-wide
// panels: the diagonal block is factorised in LDS, the panel below it solved
// against that factor, the trailing lower triangle updated by 64x64 FP64
// tiles), then L y = D b and L^T z = y are solved with 64-row blocks and
// c = D z. A non-positive or non-finite pivot sets a device flag instead of
// stopping; the host reports it and the coefficients are set to NaN.
#include "kernels.hpp"

namespace sfft {

constexpr int NBK = 64;
constexpr int kFlagNotSpd = 1;
constexpr int kFlagNonFinite = 2;

__global__ void clear_flag_kernel(int* flag) { *flag = 0; }

__global__ void __launch_bounds__(256) diag_kernel(int n, const double* __restrict__ G,
                                                    double* __restrict__ dsc, int* flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gii = G[(size_t)i * n + i];
    if (!isfinite(gii)) {
        atomicOr(flag, kFlagNonFinite);
        dsc[i] = 0.0;
    } else if (!(gii > 0.0)) {
        atomicOr(flag, kFlagNotSpd);
        dsc[i] = 0.0;
    } else {
        dsc[i] = 1.0 / sqrt(gii);
    }
}

__global__ void __launch_bounds__(256) scale_kernel(int n, const double* __restrict__ G,
                                                     const double* __restrict__ dsc,
                                                     double* __restrict__ L, int* flag) {
    const int i = blockIdx.x;
    const double di = dsc[i];
    bool bad = false;
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
        const double gij = G[(size_t)i * n + j];
        bad |= !isfinite(gij);
        L[(size_t)i * n + j] = di * gij * dsc[j];
    }
    if (bad) atomicOr(flag, kFlagNonFinite);
}

// Factorise the nb x nb diagonal block at (kb, kb) in LDS (lower, in place).
__device__ void potrf_lds(double (*A)[NBK + 1], int nb, int* flag) {
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            double s = A[j][j];
            if (!(s > 0.0) || !isfinite(s)) {
                atomicOr(flag, isfinite(s) ? kFlagNotSpd : kFlagNonFinite);
                s = 1.0;
            }
            A[j][j] = sqrt(s);
        }
        __syncthreads();
        const double inv = 1.0 / A[j][j];
        for (int i = j + 1 + threadIdx.x; i < nb; i += blockDim.x) A[i][j] *= inv;
        __syncthreads();
        const int m = nb - j - 1;   // trailing size
        for (int t = threadIdx.x; t < m * m; t += blockDim.x) {
            const int i = j + 1 + t / m, c = j + 1 + t % m;
            if (c <= i) A[i][c] -= A[i][j] * A[c][j];
        }
        __syncthreads();
    }
}

// Every block factorises the panel's diagonal block from L in LDS (L is not
// written there during the launch, so all blocks see the same input); block 0
// stores the factor in dfac (copied into L after the last panel), block
// b >= 1 solves row block b of the panel, X L_d^T = A (forward substitution,
// one row per thread).
__global__ void __launch_bounds__(256) panel_kernel(int n, double* __restrict__ L, int kb,
                                                     double* __restrict__ dfac, int* flag) {
    __shared__ double D[NBK][NBK + 1];
    __shared__ double A[NBK][NBK + 1];
    const int nb = min(NBK, n - kb);
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t / nb, j = t % nb;
        D[i][j] = j <= i ? L[(size_t)(kb + i) * n + kb + j] : 0.0;
    }
    __syncthreads();
    potrf_lds(D, nb, flag);
    if (blockIdx.x == 0) {
        double* out = dfac + (size_t)(kb / NBK) * NBK * NBK;
        for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
            const int i = t / nb, j = t % nb;
            out[i * NBK + j] = j <= i ? D[i][j] : 0.0;
        }
        return;
    }
    const int r0 = kb + blockIdx.x * NBK;
    const int nr = min(NBK, n - r0);
    for (int t = threadIdx.x; t < nr * nb; t += blockDim.x) {
        const int i = t / nb, j = t % nb;
        A[i][j] = L[(size_t)(r0 + i) * n + kb + j];
    }
    __syncthreads();
    if (threadIdx.x < nr) {
        const int i = threadIdx.x;
        for (int j = 0; j < nb; ++j) {
            double s = A[i][j];
            for (int c = 0; c < j; ++c) s -= A[i][c] * D[j][c];
            A[i][j] = s / D[j][j];
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nr * nb; t += blockDim.x) {
        const int i = t / nb, j = t % nb;
        L[(size_t)(r0 + i) * n + kb + j] = A[i][j];
    }
}

// Diagonal factors of every panel into L (after the last panel).
__global__ void __launch_bounds__(256) diag_copy_kernel(int n, double* __restrict__ L,
                                                         const double* __restrict__ dfac) {
    const int kb = blockIdx.x * NBK;
    const int nb = min(NBK, n - kb);
    const double* in = dfac + (size_t)blockIdx.x * NBK * NBK;
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t / nb, j = t % nb;
        if (j <= i) L[(size_t)(kb + i) * n + kb + j] = in[i * NBK + j];
    }
}

// Trailing update of the lower triangle: tile (I, J), I >= J, of the rows
// and columns after the panel: A_IJ -= L_I,panel L_J,panel^T.
__global__ void __launch_bounds__(256) syrk_kernel(int n, double* __restrict__ L, int kb) {
    __shared__ double PI[NBK][NBK + 1];
    __shared__ double PJ[NBK][NBK + 1];
    const int nb = min(NBK, n - kb);
    const int t0 = kb + nb;
    // triangular tile index -> (I, J)
    int I = 0, rem = blockIdx.x;
    while (rem > I) { rem -= I + 1; ++I; }
    const int J = rem;
    const int i0 = t0 + I * NBK, j0 = t0 + J * NBK;
    const int ni = min(NBK, n - i0), nj = min(NBK, n - j0);
    for (int t = threadIdx.x; t < NBK * nb; t += blockDim.x) {
        const int i = t / nb, c = t % nb;
        PI[i][c] = i < ni ? L[(size_t)(i0 + i) * n + kb + c] : 0.0;
        PJ[i][c] = i < nj ? L[(size_t)(j0 + i) * n + kb + c] : 0.0;
    }
    __syncthreads();
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;   // 16 x 16 threads, 4x4 each
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int c = 0; c < nb; ++c) {
        double x[4], y[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            x[a] = PI[ty + 16 * a][c];
            y[a] = PJ[tx + 16 * a][c];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += x[a] * y[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int i = ty + 16 * a;
        if (i >= ni) continue;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int j = tx + 16 * b;
            if (j >= nj || (I == J && j > i)) continue;
            L[(size_t)(i0 + i) * n + j0 + j] -= acc[a][b];
        }
    }
}

// Solve (D G D) z = D b with the factor L, then coef (+)= D z. One
// workgroup of 1024 threads; 64-row blocks solved by wave 0 with lane
// shuffles, the rest of the vector updated by all threads.
__global__ void __launch_bounds__(1024) trsv_kernel(int n, const double* __restrict__ L,
                                                     const double* __restrict__ dsc,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ y,
                                                     double* __restrict__ coef, int accumulate,
                                                     const int* __restrict__ flag) {
    __shared__ double yb[NBK];
    for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = dsc[i] * b[i];
    __syncthreads();
    const int nblk = (n + NBK - 1) / NBK;
    const int lane = threadIdx.x & 63;
    // forward: L y = D b
    for (int B = 0; B < nblk; ++B) {
        const int r0 = B * NBK, nb = min(NBK, n - r0);
        if (threadIdx.x < 64) {
            double v = lane < nb ? y[r0 + lane] : 0.0;
            for (int j = 0; j < nb; ++j) {
                const double yj = __shfl(v, j, 64) / L[(size_t)(r0 + j) * n + r0 + j];
                if (lane == j) v = yj;
                else if (lane > j && lane < nb) v -= L[(size_t)(r0 + lane) * n + r0 + j] * yj;
            }
            if (lane < nb) {
                y[r0 + lane] = v;
                yb[lane] = v;
            }
        }
        __syncthreads();
        for (int i = r0 + nb + threadIdx.x; i < n; i += blockDim.x) {
            const double* Li = L + (size_t)i * n + r0;
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += Li[j] * yb[j];
            y[i] -= s;
        }
        __syncthreads();
    }
    // backward: L^T z = y
    for (int B = nblk - 1; B >= 0; --B) {
        const int r0 = B * NBK, nb = min(NBK, n - r0);
        if (threadIdx.x < 64) {
            double v = lane < nb ? y[r0 + lane] : 0.0;
            for (int j = nb - 1; j >= 0; --j) {
                const double zj = __shfl(v, j, 64) / L[(size_t)(r0 + j) * n + r0 + j];
                if (lane == j) v = zj;
                else if (lane < j) v -= L[(size_t)(r0 + j) * n + r0 + lane] * zj;
            }
            if (lane < nb) {
                y[r0 + lane] = v;
                yb[lane] = v;
            }
        }
        __syncthreads();
        for (int i = threadIdx.x; i < r0; i += blockDim.x) {
            double s = 0.0;
            for (int j = 0; j < nb; ++j) s += L[(size_t)(r0 + j) * n + i] * yb[j];
            y[i] -= s;
        }
        __syncthreads();
    }
    const bool bad = *flag != 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double z = bad ? __builtin_nan("") : dsc[i] * y[i];
        coef[i] = accumulate ? coef[i] + z : z;
    }
}

hipError_t launch_clear_flag(int* flag, hipStream_t st) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, st, flag);
    return hipGetLastError();
}

hipError_t launch_jacobi(int n, const double* G, const double* h, double* L, double* dsc,
                         double* rhs, int* flag, hipStream_t st) {
    (void)h;
    (void)rhs;
    hipLaunchKernelGGL(diag_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, G, dsc, flag);
    hipLaunchKernelGGL(scale_kernel, dim3(n), dim3(256), 0, st, n, G, dsc, L, flag);
    return hipGetLastError();
}

hipError_t launch_cholesky(int n, double* L, double* dfac, int* flag, hipStream_t st) {
    for (int kb = 0; kb < n; kb += NBK) {
        const int nblk = (n - kb + NBK - 1) / NBK;
        hipLaunchKernelGGL(panel_kernel, dim3(nblk), dim3(256), 0, st, n, L, kb, dfac, flag);
        const int nb = min(NBK, n - kb);
        const int rest = n - kb - nb;
        if (rest > 0) {
            const int T = (rest + NBK - 1) / NBK;
            hipLaunchKernelGGL(syrk_kernel, dim3(T * (T + 1) / 2), dim3(256), 0, st, n, L, kb);
        }
    }
    hipLaunchKernelGGL(diag_copy_kernel, dim3((n + NBK - 1) / NBK), dim3(256), 0, st, n, L, dfac);
    return hipGetLastError();
}

hipError_t launch_chol_solve(int n, const double* L, const double* dsc, double* rhs, double* coef,
                             int accumulate, const int* flag, hipStream_t st) {
    // rhs holds b on entry and is used as the work vector y
    hipLaunchKernelGGL(trsv_kernel, dim3(1), dim3(1024), 0, st, n, L, dsc, rhs, rhs, coef,
                       accumulate, flag);
    return hipGetLastError();
}

}  // namespace sfft
