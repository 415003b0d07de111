// FP64 solve of the normal equations G c = h (the solution of Eq. 18).
//
// Jacobi scaling d = diag(G)^-1/2 keeps the factor well scaled; the scaled
// matrix D G D is factorised by a blocked right-looking Cholesky (64-wide
// panels: the diagonal block is factorised and the panel below it solved
// against that factor in one register-tiled pass, the trailing lower
// triangle updated by 64x64 FP64 tiles), then L y = D b and L^T z = y are solved with 64-row blocks and
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

// One launch per 64-wide panel at column kb. Every workgroup factorises the
// panel's diagonal block D (L is not written there during the launch, so all
// workgroups see the same input and compute the same factor); workgroup 0
// stores it in dfac (copied into L after the last panel), workgroup b >= 1
// also solves row block b of the panel, X L_D^T = A. Both run as one
// right-looking pass over the 64 columns: 256 threads own 4x4 register tiles
// (rows ty + 16 a, columns tx + 16 b) of D and of A; the raw column j is
// published through LDS (double buffered, so one barrier per column) and
// every thread scales it by the pivot itself before its rank-1 update.
__global__ void __launch_bounds__(256) panel_kernel(int n, double* __restrict__ L, int kb,
                                                     double* __restrict__ dfac, int* flag) {
    __shared__ double colD[2][NBK];
    __shared__ double colA[2][NBK];
    const int nb = min(NBK, n - kb);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int r0 = kb + blockIdx.x * NBK;
    const int nr = blockIdx.x == 0 ? 0 : min(NBK, n - r0);
    double d[4][4], x[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            d[a][b] = (i < nb && c <= i) ? L[(size_t)(kb + i) * n + kb + c] : 0.0;
            x[a][b] = (i < nr && c < nb) ? L[(size_t)(r0 + i) * n + kb + c] : 0.0;
        }
    for (int j = 0; j < nb; ++j) {
        const int buf = j & 1, bj = j >> 4;
        const bool owner = tx == (j & 15);
        if (owner) {
            // static register indexing (a runtime index would move the tiles
            // to scratch memory)
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double vd = d[a][0], vx = x[a][0];
#pragma unroll
                for (int b = 1; b < 4; ++b)
                    if (b == bj) {
                        vd = d[a][b];
                        vx = x[a][b];
                    }
                colD[buf][ty + 16 * a] = vd;
                colA[buf][ty + 16 * a] = vx;
            }
        }
        __syncthreads();
        // all LDS reads first (unconditional, so they issue together), then
        // selects
        double cd[4], cx[4], cc[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            cd[a] = colD[buf][ty + 16 * a];
            cx[a] = colA[buf][ty + 16 * a];
            cc[a] = colD[buf][tx + 16 * a];
        }
        double piv = colD[buf][j];
        if (!(piv > 0.0) || !isfinite(piv)) {
            if (threadIdx.x == 0) atomicOr(flag, isfinite(piv) ? kFlagNotSpd : kFlagNonFinite);
            piv = 1.0;
        }
        const double ljj = sqrt(piv), inv = 1.0 / ljj;
        double li[4], xi[4], lc[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            li[a] = ty + 16 * a > j ? cd[a] * inv : 0.0;
            xi[a] = cx[a] * inv;
            lc[a] = tx + 16 * a > j ? cc[a] * inv : 0.0;
        }
        if (owner) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int i = ty + 16 * a;
                const double nd = i == j ? ljj : (i > j ? li[a] : 0.0);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    if (b == bj) {
                        d[a][b] = nd;
                        x[a][b] = xi[a];
                    }
            }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                d[a][b] -= li[a] * lc[b];
                x[a][b] -= xi[a] * lc[b];
            }
    }
    if (blockIdx.x == 0) {
        double* out = dfac + (size_t)(kb / NBK) * NBK * NBK;
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int i = ty + 16 * a, c = tx + 16 * b;
                if (i < nb && c < nb) out[i * NBK + c] = c <= i ? d[a][b] : 0.0;
            }
        return;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            if (i < nr && c < nb) L[(size_t)(r0 + i) * n + kb + c] = x[a][b];
        }
}

// After the last panel, per diagonal block B: the factor held in dfac goes
// into L (lower part, with its transpose in the upper part of the tile), and
// W_B = L_BB^-1 and W_B^T are stored in dinv[B][0] and dinv[B][1] (64 x 64
// row-major, zero outside the triangle) for the triangular solves. One wave
// per block; lane c computes column c of W by forward substitution.
__global__ void __launch_bounds__(64) diag_finish_kernel(int n, double* __restrict__ L,
                                                          const double* __restrict__ dfac,
                                                          double* __restrict__ dinv) {
    __shared__ double Lb[NBK][NBK + 1];
    __shared__ double Wb[NBK][NBK + 1];
    __shared__ double rd[NBK];
    const int B = blockIdx.x, kb = B * NBK, nb = min(NBK, n - kb);
    const double* in = dfac + (size_t)B * NBK * NBK;
    const int c = threadIdx.x;
    for (int i = 0; i < NBK; ++i) Lb[i][c] = (i < nb && c <= i) ? in[i * NBK + c] : 0.0;
    __syncthreads();
    if (c < nb)
        for (int i = 0; i < nb; ++i)
            L[(size_t)(kb + i) * n + kb + c] = c <= i ? Lb[i][c] : Lb[c][i];
    rd[c] = c < nb ? 1.0 / Lb[c][c] : 0.0;
    __syncthreads();
    for (int i = 0; i < NBK; ++i) {
        double w = 0.0;
        if (c < nb && i < nb && i >= c) {
            if (i == c) {
                w = rd[c];
            } else {
                double s = 0.0;
                for (int j = c; j < i; ++j) s += Lb[i][j] * Wb[j][c];
                w = -s * rd[i];
            }
        }
        Wb[i][c] = w;   // lane c reads back only its own column
    }
    __syncthreads();
    double* out = dinv + (size_t)B * 2 * NBK * NBK;
    for (int i = 0; i < NBK; ++i) {
        out[i * NBK + c] = Wb[i][c];
        out[NBK * NBK + i * NBK + c] = Wb[c][i];
    }
}

// Upper triangle of L := L^T for the strictly lower 64 x 64 tiles (I > J),
// so that the backward solve reads rows (coalesced) instead of columns.
__global__ void __launch_bounds__(256) mirror_kernel(int n, double* __restrict__ L) {
    __shared__ double t[NBK][NBK + 1];
    int I = 1, rem = blockIdx.x;
    while (rem >= I) {
        rem -= I;
        ++I;
    }
    const int J = rem;
    const int i0 = I * NBK, j0 = J * NBK;   // J < I: the tile has 64 full columns
    const int ni = min(NBK, n - i0);
    for (int k = threadIdx.x; k < NBK * NBK; k += blockDim.x) {
        const int r = k >> 6, col = k & 63;
        if (r < ni) t[r][col] = L[(size_t)(i0 + r) * n + j0 + col];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NBK * NBK; k += blockDim.x) {
        const int col = k >> 6, r = k & 63;
        if (r < ni) L[(size_t)(j0 + col) * n + i0 + r] = t[r][col];
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

// y[i] -= sum_(q < nb) M[i n + col0 + q] yb[q] for row_lo <= i < row_hi.
// 8 lanes per row, 8 contiguous doubles per lane; each lane keeps 4 rows'
// loads in flight before reducing (FULL: nb = 64, no column guard).
template <bool FULL>
__device__ __forceinline__ void update_rows(const double* __restrict__ M, int n, int row_lo,
                                            int row_hi, int col0, int nb,
                                            const double* __restrict__ yb, double* y) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const int sub = lane >> 3, part = lane & 7;
    double yq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) yq[q] = (FULL || part * 8 + q < nb) ? yb[part * 8 + q] : 0.0;
    const int stride = nwv * 8;
    for (int base = row_lo + wv * 8 + sub; base < row_hi; base += 4 * stride) {
        double s[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * stride;
            s[u] = 0.0;
            if (i < row_hi) {
                const double* Mi = M + (size_t)i * n + col0 + part * 8;
                if (FULL) {
                    double v[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) v[q] = Mi[q];
#pragma unroll
                    for (int q = 0; q < 8; ++q) s[u] += v[q] * yq[q];
                } else {
                    for (int q = 0; q < 8 && part * 8 + q < nb; ++q) s[u] += Mi[q] * yq[q];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            double v = s[u];
            v += __shfl_xor(v, 1, 64);
            v += __shfl_xor(v, 2, 64);
            v += __shfl_xor(v, 4, 64);
            const int i = base + u * stride;
            if (part == 0 && i < row_hi) y[i] -= v;
        }
    }
}

// y_B := W y_B for the 64 x 64 block W (row-major): 16 threads per row, 4
// columns each.
__device__ __forceinline__ void block_matvec(const double* __restrict__ W, int r0, int nb,
                                             double* y, double* yb) {
    const int i = threadIdx.x >> 4, part = threadIdx.x & 15;
    double s = 0.0;
    if (i < NBK) {
        const double* Wi = W + i * NBK + part * 4;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int c = part * 4 + q;
            const double yc = c < nb ? y[r0 + c] : 0.0;
            s += Wi[q] * yc;
        }
    }
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 4, 64);
    s += __shfl_xor(s, 8, 64);
    __syncthreads();   // every read of y_B precedes the writes
    if (part == 0 && i < nb) {
        y[r0 + i] = s;
        yb[i] = s;
    }
    __syncthreads();
}

// Solve (D G D) z = D b with the factor L (lower part; the upper part holds
// L^T), then coef (+)= D z. One workgroup of 1024 threads, 64-row blocks:
// forward, y_B = W_B y_B then the rows below are updated; backward,
// z_B = W_B^T y_B then the rows above are updated from the rows of L^T.
__global__ void __launch_bounds__(1024) trsv_kernel(int n, const double* __restrict__ L,
                                                     const double* __restrict__ dinv,
                                                     const double* __restrict__ dsc,
                                                     const double* b, double* y,
                                                     double* __restrict__ coef, int accumulate,
                                                     const int* __restrict__ flag) {
    __shared__ double yb[NBK];
    for (int i = threadIdx.x; i < n; i += blockDim.x) y[i] = dsc[i] * b[i];
    __syncthreads();
    const int nblk = (n + NBK - 1) / NBK;
    for (int B = 0; B < nblk; ++B) {
        const int r0 = B * NBK, nb = min(NBK, n - r0);
        block_matvec(dinv + (size_t)B * 2 * NBK * NBK, r0, nb, y, yb);
        if (nb == NBK) update_rows<true>(L, n, r0 + nb, n, r0, nb, yb, y);
        else update_rows<false>(L, n, r0 + nb, n, r0, nb, yb, y);
        __syncthreads();
    }
    for (int B = nblk - 1; B >= 0; --B) {
        const int r0 = B * NBK, nb = min(NBK, n - r0);
        block_matvec(dinv + (size_t)B * 2 * NBK * NBK + NBK * NBK, r0, nb, y, yb);
        if (nb == NBK) update_rows<true>(L, n, 0, r0, r0, nb, yb, y);
        else update_rows<false>(L, n, 0, r0, r0, nb, yb, y);
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

hipError_t launch_cholesky(int n, double* L, double* dfac, double* dinv, int* flag, hipStream_t st) {
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
    const int T = (n + NBK - 1) / NBK;
    hipLaunchKernelGGL(diag_finish_kernel, dim3(T), dim3(64), 0, st, n, L, dfac, dinv);
    if (T > 1) hipLaunchKernelGGL(mirror_kernel, dim3(T * (T - 1) / 2), dim3(256), 0, st, n, L);
    return hipGetLastError();
}

hipError_t launch_chol_solve(int n, const double* L, const double* dinv, const double* dsc,
                             double* rhs, double* coef, int accumulate, const int* flag,
                             hipStream_t st) {
    // rhs holds b on entry and is used as the work vector y
    hipLaunchKernelGGL(trsv_kernel, dim3(1), dim3(1024), 0, st, n, L, dinv, dsc, rhs, rhs, coef,
                       accumulate, flag);
    return hipGetLastError();
}

}  // namespace sfft
