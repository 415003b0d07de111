// FP64 solve of the normal equations G c = h (the solution of Eq. 18).
//
// Jacobi scaling d = diag(G)^-1/2 keeps the factor well scaled; the scaled
// matrix D G D is factorised by a blocked right-looking Cholesky (64-wide
// panels: the diagonal block is factorised and the panel below it solved
// against that factor in one register-tiled pass; each panel's update of the
// trailing lower triangle, in 64x64 FP64 tiles on the matrix cores, runs in
// the next panel's launch), then L y = D b and L^T z = y are solved as a
// dataflow of 64-row blocks across workgroups and c = D z. A non-positive or
// non-finite pivot sets a device flag instead of stopping; the host reports
// it and the coefficients are set to NaN.
#include "kernels.hpp"

namespace sfft {

constexpr int NBK = 64;
constexpr int kFlagNotSpd = 1;
constexpr int kFlagNonFinite = 2;
constexpr int kFlagStall = 4;          // a bounded wait ran out (never expected)
constexpr int kSolveSpin = 1 << 22;    // bound of every poll loop
constexpr int kStallTestSpin = 64;     // the bound under the give-up test
// An empty entry of the triangular solves' result buffers: a signalling NaN,
// which no arithmetic result equals (results are never signalling NaNs)
constexpr unsigned long long kTsvEmpty = 0x7FF4000000005EEDull;

// The result buffer (2 n entries: forward, then backward) of the solve of
// generation gen: two buffers alternate.
__host__ __device__ __forceinline__ unsigned long long* tsv_buffer(double* tsv, int n, int gen) {
    return reinterpret_cast<unsigned long long*>(tsv) + (size_t)(gen & 1) * 2 * n;
}

// A request's start: status flag cleared, and the result buffer of its first
// solve (generation 1) emptied.
__global__ void clear_flag_kernel(int* flag, double* tsv, int n, long long zs) {
    flag = zoff(flag, zs);
    tsv = zoff(tsv, zs);
    if (threadIdx.x == 0) *flag = 0;
    unsigned long long* b = tsv_buffer(tsv, n, 1);
    for (int i = threadIdx.x; i < 2 * n; i += blockDim.x) b[i] = kTsvEmpty;
}

// Jacobi scaling, one block per row i: L_ij = d_i G_ij d_j (j <= i) with
// d_j = 1/sqrt(G_jj) formed where it is used (0 for a bad diagonal, which
// row j's own block reports).
__device__ __forceinline__ double jacobi_d(double gjj) {
    return (isfinite(gjj) && gjj > 0.0) ? 1.0 / sqrt(gjj) : 0.0;
}

__global__ void __launch_bounds__(256) jacobi_kernel(int n, const double* __restrict__ G,
                                                      double* __restrict__ dsc,
                                                      double* __restrict__ L, int* flag,
                                                      long long zs) {
    G = zoff(G, zs);
    dsc = zoff(dsc, zs);
    L = zoff(L, zs);
    flag = zoff(flag, zs);
    const int i = blockIdx.x;
    const double gii = G[(size_t)i * n + i];
    const double di = jacobi_d(gii);
    if (threadIdx.x == 0) {
        dsc[i] = di;
        if (!isfinite(gii)) atomicOr(flag, kFlagNonFinite);
        else if (!(gii > 0.0)) atomicOr(flag, kFlagNotSpd);
    }
    bool bad = false;
    for (int j = threadIdx.x; j <= i; j += blockDim.x) {
        const double gij = G[(size_t)i * n + j];
        bad |= !isfinite(gij);
        L[(size_t)i * n + j] = di * gij * jacobi_d(G[(size_t)j * n + j]);
    }
    if (bad) atomicOr(flag, kFlagNonFinite);
}

// FP64 matrix-core product of two 64-row panels staged in LDS:
//   acc[I] = sum_c P[16 I + r][c] Q[16 wv + s][c]   (r, s < 16)
// for the 16-column strip wv of the 64 x 64 result and its four row blocks
// I (v_mfma_f64_16x16x4: lane l holds A[l%16][l/16], B[l/16][l%16], and
// result row l/16 + 4 q, column l%16 in register q).
typedef double dbl4 __attribute__((ext_vector_type(4)));
constexpr int kStepThreads = 512;   // threads per panel / tile workgroup
// The 4 x 4 blocks (16 x 16) of a 64 x 64 matrix-core product over the
// waves: with eight waves, column strip w % 4 and row blocks 2 (w / 4) + {0,
// 1}; with four, strip w and all row blocks; with two, strips 2w, 2w + 1.
constexpr int kStepWaves = kStepThreads / 64;
constexpr int kBlocksPerStrip = kStepWaves >= 4 ? 16 / kStepWaves : 4;
constexpr int kStripsPerWave = kStepWaves >= 4 ? 1 : 4 / kStepWaves;
__device__ __forceinline__ int strip_of(int wv, int t) {
    return kStepWaves >= 4 ? (wv & 3) : kStripsPerWave * wv + t;
}
__device__ __forceinline__ int rowblock0_of(int wv) {
    return kStepWaves >= 4 ? kBlocksPerStrip * (wv >> 2) : 0;
}

// Row blocks I0 .. I0+NI-1 of the strip s:
//   acc[I] = sum_c P[16 (I0 + I) + r][c] Q[16 s + t][c]   (r, t < 16).
template <int NI>
__device__ __forceinline__ void panel_mfma(const double (*P)[NBK + 1], const double (*Q)[NBK + 1],
                                           int I0, int s, int lane, dbl4* acc) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int I = 0; I < NI; ++I) acc[I] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int kk = 0; kk < NBK / 4; ++kk) {
        const int cc = 4 * kk + lk;
        const double b = Q[16 * s + lr][cc];
#pragma unroll
        for (int I = 0; I < NI; ++I)
            acc[I] = __builtin_amdgcn_mfma_f64_16x16x4f64(P[16 * (I0 + I) + lr][cc], b, acc[I], 0, 0,
                                                          0);
    }
}

// PI = L_(i0 .. i0+ni, kp .. kp+63), PJ = L_(j0 .. j0+nj, kp .. kp+63), rows
// past ni / nj zero: each thread issues all its loads before the LDS writes
// (one memory latency instead of one per element), then a barrier.
__device__ __forceinline__ void stage_panels(const double* __restrict__ L, int n, int kp, int i0,
                                             int ni, int j0, int nj, double (*PI)[NBK + 1],
                                             double (*PJ)[NBK + 1]) {
    constexpr int kRows = kStepThreads / 64, kPer = NBK / kRows;
    double vi[kPer], vj[kPer];
    const int c = threadIdx.x & 63, r = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int i = r + kRows * q;
        vi[q] = i < ni ? L[(size_t)(i0 + i) * n + kp + c] : 0.0;
        vj[q] = i < nj ? L[(size_t)(j0 + i) * n + kp + c] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        PI[r + kRows * q][c] = vi[q];
        PJ[r + kRows * q][c] = vj[q];
    }
    __syncthreads();
}

// A_(i0.., j0..) -= L_(i0.., kp..kp+63) L_(j0.., kp..kp+63)^T on one 64 x 64
// tile of the lower triangle (diag: i0 == j0, only c <= i is stored).
__device__ __forceinline__ void tile_update(int n, double* __restrict__ L, int kp, int i0, int j0,
                                            double (*PI)[NBK + 1], double (*PJ)[NBK + 1]) {
    const int ni = min(NBK, n - i0), nj = min(NBK, n - j0);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // the tile's current values, loaded first and unconditionally (indices
    // clamped into the matrix) so that they are all in flight together and
    // behind the staging and the products (a load under a per-lane condition
    // is a branch with its own wait)
    double old[kStripsPerWave][kBlocksPerStrip][4];
#pragma unroll
    for (int t = 0; t < kStripsPerWave; ++t) {
        const int jc = min(16 * strip_of(wv, t) + (lane & 15), nj - 1);
#pragma unroll
        for (int I = 0; I < kBlocksPerStrip; ++I)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * (rowblock0_of(wv) + I) + (lane >> 4) + 4 * q;
                old[t][I][q] = L[(size_t)(i0 + min(i, ni - 1)) * n + j0 + jc];
            }
    }
    stage_panels(L, n, kp, i0, ni, j0, nj, PI, PJ);
#pragma unroll
    for (int t = 0; t < kStripsPerWave; ++t) {
        const int sc = strip_of(wv, t), I0 = rowblock0_of(wv);
        dbl4 acc[kBlocksPerStrip];
        panel_mfma<kBlocksPerStrip>(PI, PJ, I0, sc, lane, acc);
        const int jc = 16 * sc + (lane & 15);
#pragma unroll
        for (int I = 0; I < kBlocksPerStrip; ++I)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = 16 * (I0 + I) + (lane >> 4) + 4 * q;
                if (i < ni && jc < nj && !(i0 == j0 && jc > i))
                    L[(size_t)(i0 + i) * n + j0 + jc] = old[t][I][q] - acc[I][q];
            }
    }
}

// Broadcast of lane `src`'s value to the wave.
__device__ __forceinline__ double bcast(double v, int src) {
    const long long u = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffff), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// 16 x 16 block of P Q^T over the 16 columns c0..c0+15 on the matrix cores:
//   acc[q] = sum_k P[pr + lane/16 + 4 q][c0 + k] Q[qr + lane%16][c0 + k].
__device__ __forceinline__ dbl4 mfma16(const double (*P)[NBK + 1], int pr,
                                       const double (*Q)[NBK + 1], int qr, int c0, int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int cc = c0 + 4 * kk + lk;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(P[pr + lr][cc], Q[qr + lr][cc], acc, 0, 0, 0);
    }
    return acc;
}

// Cholesky factor of the 64 x 64 block D (lower part, identity padding) and
// the solve of the na rows of A against it (A := A L_D^-T), in place in LDS,
// by 16-column blocks jb:
//  (1) wave 0 factorises D_jj = L_jj L_jj^T in registers (lane i holds row
//      i; the pivot and the column below it are broadcast by readlane): the
//      16 dependent steps need no barrier;
//  (2) every row below the block in D and every row of A is solved against
//      L_jj, one row per thread (y_j = (a_j - sum_(k<j) y_k L_jk) / L_jj,
//      the terms subtracted as each y_k is formed);
//  (3) the 16 x 16 blocks right of the column block take the rank-16 update
//      (D_IJ -= L_Ij L_Jj^T for J <= I, A_IJ -= Y_I L_Jj^T) on the FP64
//      matrix cores, one block per wave at a time.
// A pivot that is not positive and finite sets the flag and is taken as 1.
// Every thread of the workgroup calls it (it synchronises).
__device__ __forceinline__ void factor_panel(double (*D)[NBK + 1], double (*A)[NBK + 1], int na,
                                             int* flag) {
    __shared__ double rdiag[16];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll 1
    for (int jb = 0; jb < 4; ++jb) {
        const int c0 = 16 * jb;
        if (wv == 0) {   // (1)
            const int li = lane & 15;
            double r[16];
#pragma unroll
            for (int c = 0; c < 16; ++c) r[c] = D[c0 + li][c0 + c];
            bool bad = false, nonfin = false;
            // dn: in lane j, the pivot of step j once the steps before it are
            // applied. Lane j + 1 forms it from its own scaled entry, so the
            // dependent chain from pivot to pivot is one broadcast, the
            // reciprocal square root, the scale and one FMA; the broadcasts
            // of the column for the other updates run beside it.
            double dn = r[0];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const double pv = bcast(dn, j);
                const bool ok = pv > 0.0 && isfinite(pv);   // uniform
                if (!ok) {
                    bad = true;
                    nonfin |= !isfinite(pv);
                }
                // hardware estimate and one Newton step with the cubic term,
                // y (1 + e/2 + 3e^2/8), e = 1 - x y^2 (a positive finite
                // pivot needs no special cases); a bad pivot is taken as 1
                const double y0 = __builtin_amdgcn_rsq(pv);
                const double e = fma(-(pv * y0), y0, 1.0);
                const double inv = ok ? fma(y0 * e, fma(e, 0.375, 0.5), y0) : 1.0;
                const double lj = r[j] * inv;
                if (j < 15) dn = fma(-lj, lj, r[j + 1]);
                r[j] = li > j ? lj : (li == j ? (ok ? pv : 1.0) * inv : 0.0);
#pragma unroll
                for (int kc = j + 1; kc < 16; ++kc) r[kc] = fma(-r[j], bcast(r[j], kc), r[kc]);
            }
            if (lane < 16) {
#pragma unroll
                for (int c = 0; c < 16; ++c) D[c0 + lane][c0 + c] = c <= lane ? r[c] : 0.0;
                rdiag[lane] = 1.0 / r[lane];
            }
            if (bad && lane == 0) atomicOr(flag, nonfin ? kFlagNonFinite : kFlagNotSpd);
        }
        __syncthreads();
        // (2): rows c0+16 .. 63 of D, then the na rows of A
        const int nd = NBK - c0 - 16;
        for (int t = threadIdx.x; t < nd + na; t += kStepThreads) {
            double* row = t < nd ? D[c0 + 16 + t] : A[t - nd];
            double y[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) y[j] = row[c0 + j];
            // right-looking: y_j is final once scaled, then leaves its term
            // in every later entry, so the dependent chain is one product
            // and one FMA per column
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                y[j] *= rdiag[j];
#pragma unroll
                for (int kc = j + 1; kc < 16; ++kc) y[kc] = fma(-y[j], D[c0 + kc][c0 + j], y[kc]);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) row[c0 + j] = y[j];
        }
        __syncthreads();
        if (jb == 3) break;
        // (3): D blocks (I, J), jb < J <= I < 4, then A blocks (I, J), I < 4, J > jb
        const int nj = 3 - jb, ndb = nj * (nj + 1) / 2, nab = 4 * nj;
        for (int bi = wv; bi < ndb + nab; bi += kStepWaves) {
            int I, J;
            const bool isd = bi < ndb;
            if (isd) {
                int rem = bi;
                I = 0;
                while (rem > I) {
                    rem -= I + 1;
                    ++I;
                }
                J = rem + jb + 1;
                I += jb + 1;
            } else {
                I = (bi - ndb) / nj;
                J = jb + 1 + (bi - ndb) % nj;
            }
            const dbl4 acc = isd ? mfma16(D, 16 * I, D, 16 * J, c0, lane)
                                 : mfma16(A, 16 * I, D, 16 * J, c0, lane);
            double (*T)[NBK + 1] = isd ? D : A;
            const int jc = 16 * J + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) T[16 * I + (lane >> 4) + 4 * q][jc] -= acc[q];
        }
        __syncthreads();
    }
}

// Step k of the right-looking factorisation, with the trailing update of
// step k - 1 folded in: one launch per 64-column panel (kb = 64 k).
//  * Workgroups b < T - k (T = number of 64-blocks) work on panel k, row
//    block k + b. For k > 0 they first apply panel k-1's update to their own
//    tile of column block k and to the diagonal tile (every panel workgroup
//    forms the updated diagonal tile itself, nothing is written there during
//    the launch): the panel rows are staged in LDS and multiplied on the
//    FP64 matrix cores. Then every one factorises the diagonal block D;
//    workgroup 0 stores it in dfac (copied into L after the last step),
//    workgroup b >= 1 also solves its row block X L_D^T = A.
//    Factor and solve run on D and A in LDS, 16 columns at a time
//    (factor_panel): one wave factorises the 16 x 16 diagonal block in
//    registers, the rows below it and the rows of A are solved against it
//    one row per thread, and the trailing 16 x 16 blocks take the rank-16
//    update on the matrix cores; three barriers per 16 columns.
//  * The other workgroups give the tiles (I, J), I >= J > k, of the trailing
//    matrix panel k-1's update.
// After the launch column block k is final and every tile right of it has
// the updates of panels 0 .. k-1.
__global__ void __launch_bounds__(kStepThreads) chol_step_kernel(int n, double* __restrict__ L,
                                                                  int k, double* __restrict__ dfac,
                                                                  int* flag, long long zs) {
    L = zoff(L, zs);
    dfac = zoff(dfac, zs);
    flag = zoff(flag, zs);
    constexpr int RY = kStepThreads / 16;   // row groups: thread rows ty + RY a
    constexpr int RA = NBK / RY;            // rows per thread
    __shared__ double PI[NBK][NBK + 1];
    __shared__ double PJ[NBK][NBK + 1];
    const int T = (n + NBK - 1) / NBK;
    const int kb = k * NBK;
    const int npan = T - k;
    if ((int)blockIdx.x >= npan) {
        int I = 0, rem = blockIdx.x - npan;
        while (rem > I) {
            rem -= I + 1;
            ++I;
        }
        tile_update(n, L, kb - NBK, (k + 1 + I) * NBK, (k + 1 + rem) * NBK, PI, PJ);
        return;
    }
    const int nb = min(NBK, n - kb);
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int r0 = kb + blockIdx.x * NBK;
    const int nr = blockIdx.x == 0 ? 0 : min(NBK, n - r0);
    double d[RA][4], x[RA][4];
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + RY * a, c = tx + 16 * b;
            d[a][b] = (i < nb && c <= i) ? L[(size_t)(kb + i) * n + kb + c] : 0.0;
            x[a][b] = (i < nr && c < nb) ? L[(size_t)(r0 + i) * n + kb + c] : 0.0;
        }
    if (k > 0) {
        // panel k-1 (64 full columns at kp) onto D and onto this row block
        const int kp = kb - NBK;
        stage_panels(L, n, kp, r0, nr, kb, nb, PI, PJ);
        // the update on the matrix cores (blocks over the waves as in
        // strip_of / rowblock0_of); the strips go through LDS into the
        // factor's register tiles
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        dbl4 ud[kStripsPerWave][kBlocksPerStrip], ux[kStripsPerWave][kBlocksPerStrip];
#pragma unroll
        for (int t = 0; t < kStripsPerWave; ++t) {
            panel_mfma<kBlocksPerStrip>(PJ, PJ, rowblock0_of(wv), strip_of(wv, t), lane, ud[t]);
            panel_mfma<kBlocksPerStrip>(PI, PJ, rowblock0_of(wv), strip_of(wv, t), lane, ux[t]);
        }
        __syncthreads();   // every wave is done reading the panels
#pragma unroll
        for (int t = 0; t < kStripsPerWave; ++t) {
            const int jc = 16 * strip_of(wv, t) + (lane & 15);
#pragma unroll
            for (int I = 0; I < kBlocksPerStrip; ++I)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = 16 * (rowblock0_of(wv) + I) + (lane >> 4) + 4 * q;
                    PJ[i][jc] = ud[t][I][q];
                    PI[i][jc] = ux[t][I][q];
                }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < RA; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                d[a][b] -= PJ[ty + RY * a][tx + 16 * b];
                x[a][b] -= PI[ty + RY * a][tx + 16 * b];
            }
    }
    // D (lower part; identity past nb) and A into LDS for the blocked pass
#pragma unroll
    for (int a = 0; a < RA; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + RY * a, c = tx + 16 * b;
            PJ[i][c] = (i < nb && c < nb) ? d[a][b] : (i == c ? 1.0 : 0.0);
            PI[i][c] = x[a][b];
        }
    __syncthreads();
    factor_panel(PJ, PI, blockIdx.x == 0 ? 0 : nr, flag);
    if (blockIdx.x == 0) {
        double* out = dfac + (size_t)k * NBK * NBK;
        for (int t = threadIdx.x; t < NBK * NBK; t += kStepThreads) {
            const int i = t >> 6, c = t & 63;
            if (i < nb && c < nb) out[i * NBK + c] = c <= i ? PJ[i][c] : 0.0;
        }
        return;
    }
    for (int t = threadIdx.x; t < NBK * NBK; t += kStepThreads) {
        const int i = t >> 6, c = t & 63;
        if (i < nr && c < nb) L[(size_t)(r0 + i) * n + kb + c] = PI[i][c];
    }
}

// After the last panel, per diagonal block B: the factor held in dfac goes
// into L (lower part, with its transpose in the upper part of the tile), and
// W_B = L_BB^-1 and W_B^T are stored in dinv[B][0] and dinv[B][1] (64 x 64
// row-major, zero outside the triangle) for the triangular solves. W comes
// from L W = I by a right-looking sweep over the rows: row j of W is the
// current row j of the right-hand side divided by L_jj, then every row i > j
// loses L_ij times it. 256 threads own 4x4 tiles (rows ty + 16 a, columns
// tx + 16 b) of the right-hand side; row j is published through LDS (double
// buffered, one barrier per row).
__global__ void __launch_bounds__(256) diag_finish_kernel(int n, double* __restrict__ L,
                                                           const double* __restrict__ dfac,
                                                           double* __restrict__ dinv,
                                                           long long zs) {
    L = zoff(L, zs);
    dfac = zoff(dfac, zs);
    dinv = zoff(dinv, zs);
    __shared__ double Lb[NBK][NBK + 1];
    __shared__ double wrow[2][NBK];
    const int B = blockIdx.x, kb = B * NBK, nb = min(NBK, n - kb);
    const double* in = dfac + (size_t)B * NBK * NBK;
    // the whole 64 x 64 block of dfac (always allocated) loaded at once,
    // then masked: no load waits under a per-lane condition
    constexpr int kPer = NBK * NBK / 256;   // launched with 256 threads
    double v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) v[q] = in[threadIdx.x + 256 * q];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int t = threadIdx.x + 256 * q, i = t >> 6, c = t & 63;
        Lb[i][c] = (i < nb && c <= i && c < nb) ? v[q] : (i == c ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb * nb; t += blockDim.x) {
        const int i = t / nb, c = t % nb;
        L[(size_t)(kb + i) * n + kb + c] = c <= i ? Lb[i][c] : Lb[c][i];
    }
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double w[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) w[a][b] = (ty + 16 * a == tx + 16 * b) ? 1.0 : 0.0;
#pragma unroll
    for (int aj = 0; aj < 4; ++aj) {
#pragma unroll 1
        for (int jj = 0; jj < 16; ++jj) {
            const int j = 16 * aj + jj;
            const int buf = j & 1;
            const double rd = 1.0 / Lb[j][j];
            if (ty == jj) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    w[aj][b] *= rd;
                    wrow[buf][tx + 16 * b] = w[aj][b];
                }
            }
            __syncthreads();
            double wc[4], li[4];
#pragma unroll
            for (int b = 0; b < 4; ++b) wc[b] = wrow[buf][tx + 16 * b];
#pragma unroll
            for (int a = 0; a < 4; ++a) li[a] = ty + 16 * a > j ? Lb[ty + 16 * a][j] : 0.0;
#pragma unroll
            for (int a = aj; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) w[a][b] -= li[a] * wc[b];
        }
    }
    double* out = dinv + (size_t)B * 2 * NBK * NBK;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int i = ty + 16 * a, c = tx + 16 * b;
            const double v = (i < nb && c < nb) ? w[a][b] : 0.0;
            out[i * NBK + c] = v;
            out[NBK * NBK + c * NBK + i] = v;
        }
}

// Upper triangle of L := L^T for the strictly lower 64 x 64 tiles (I > J),
// so that the backward solve reads rows (coalesced) instead of columns.
__global__ void __launch_bounds__(256) mirror_kernel(int n, double* __restrict__ L, long long zs) {
    __shared__ double t[NBK][NBK + 1];
    L = zoff(L, zs);
    int I = 1, rem = blockIdx.x;
    while (rem >= I) {
        rem -= I;
        ++I;
    }
    const int J = rem;
    const int i0 = I * NBK, j0 = J * NBK;   // J < I: the tile has 64 full columns
    const int ni = min(NBK, n - i0);
    // every load issued before any is used (rows clamped into the matrix)
    constexpr int kPer = NBK * NBK / 256;   // launched with 256 threads
    double v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = threadIdx.x + 256 * q, r = k >> 6, col = k & 63;
        v[q] = L[(size_t)(i0 + min(r, ni - 1)) * n + j0 + col];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = threadIdx.x + 256 * q, r = k >> 6, col = k & 63;
        if (r < ni) t[r][col] = v[q];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < NBK * NBK; k += blockDim.x) {
        const int col = k >> 6, r = k & 63;
        if (r < ni) L[(size_t)(j0 + col) * n + i0 + r] = t[r][col];
    }
}

// Triangular solves as a dataflow over 64-row blocks, one workgroup per
// block and direction (T = ceil(n/64) blocks, 2 T workgroups per pair):
//   forward  y_B = W_B (D b_B - sum_(C < B) L_BC y_C),        workgroup B
//   backward z_B = W_B^T (y_B - sum_(C > B) (L^T)_BC z_C),     workgroup 2T-1-B
// then coef_B (+)= D z_B, with W_B, W_B^T the inverted diagonal blocks and
// (L^T)_BC read from the mirrored upper triangle (rows, coalesced). Each
// workgroup takes its dependency blocks in a fixed order (forward C = 0, 1,
// ..., backward y_B first, then C = T-1, T-2, ...), so the sums do not depend
// on timing; while it waits for block C it already holds that tile's row
// slices and its W in registers.
// Hand-off. The results are the flags: every entry of the solve's result
// buffer starts empty (kTsvEmpty), the producing thread stores its value
// with a relaxed device-scope atomic, and each reading thread polls its own
// entries with relaxed device-scope atomic loads until they are not empty.
// Each entry is published and read on its own, so per-location coherence is
// all the hand-off needs: no fences (an agent-scope release or acquire
// writes back or invalidates the whole L2 of an XCD). The buffers of
// generations gen and gen + 1 alternate; a solve empties the next
// generation's buffer (its own blocks' entries) while it runs, and
// clear_flag_kernel empties generation 1's at the request's start.
// Placement. A pair's 2T tasks x (forward block x for x < T, then backward
// block 2T-1-x) each wait only for earlier tasks. Workgroups are dealt to
// the 8 XCDs round robin and each XCD starts its own in order; workgroup i
// is XCD i mod 8, place j = i / 8 there. Batches: every task of a pair on
// one XCD (pair (i mod 8) + 8 (j / 2T), task x = j mod 2T), its flags in one
// L2. One pair: its tasks in 8 contiguous chunks of cs = ceil(2T / 8), chunk
// c on XCD c (task x = c cs + j), which spreads the hand-offs' cache
// maintenance over the XCDs. Either way every task a workgroup waits for is
// earlier on the same XCD (already started) or on a lower XCD, whose tasks
// wait only on earlier or lower ones: whatever else runs on the GPU, no wait
// can be on a workgroup that cannot start. Each poll is bounded: past the
// bound the block sets kFlagStall and goes on (its result is then NaN).
// The value of result entry v once it is published (at most `spin` polls;
// past that kFlagStall and NaN).
__device__ __forceinline__ double wait_value(const unsigned long long* v, int spin, int* flag) {
    unsigned long long u = __hip_atomic_load(v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (u == kTsvEmpty) {
        __builtin_amdgcn_s_sleep(2);
        if (++spins >= spin) {
            atomicOr(flag, kFlagStall);
            break;
        }
        u = __hip_atomic_load(v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    return __builtin_bit_cast(double, u);
}

__global__ void __launch_bounds__(256) trsv_flow_kernel(int n, const double* __restrict__ L,
                                                         const double* __restrict__ dinv,
                                                         const double* __restrict__ dsc,
                                                         const double* __restrict__ b,
                                                         double* __restrict__ coef, int accumulate,
                                                         int* flag, double* tsv, int gen,
                                                         int publish, int spin, int npairs,
                                                         long long zstride) {
    __shared__ double vsh[NBK];
    const int T = (n + NBK - 1) / NBK;
    const int xcd = blockIdx.x & 7, j = blockIdx.x >> 3;
    int pair, x;
    if (npairs == 1) {
        const int cs = (2 * T + 7) / 8;
        pair = 0;
        x = xcd * cs + j;
        if (j >= cs || x >= 2 * T) return;   // uniform over the workgroup, before any barrier
    } else {
        pair = xcd + 8 * (j / (2 * T));
        x = j % (2 * T);
        if (pair >= npairs) return;
    }
    const long long zo = (long long)pair * zstride;
    auto at = [zo](auto* p) {
        return reinterpret_cast<decltype(p)>(reinterpret_cast<uintptr_t>(p) + (uintptr_t)zo);
    };
    L = at(L);
    dinv = at(dinv);
    dsc = at(dsc);
    b = at(b);
    coef = at(coef);
    flag = at(flag);
    tsv = at(tsv);
    const bool fwd = x < T;
    const int B = fwd ? x : 2 * T - 1 - x;
    const int r0 = B * NBK, nb = min(NBK, n - r0);
    const int i = threadIdx.x >> 2, p = threadIdx.x & 3;   // row, quarter of the columns
    unsigned long long* res = tsv_buffer(tsv, n, gen);      // y: [0, n), z: [n, 2n)
    // this block's entries of the next generation's buffer emptied
    if (p == 0 && i < nb) tsv_buffer(tsv, n, gen + 1)[(fwd ? 0 : n) + r0 + i] = kTsvEmpty;
    // this block's inverse (row i, columns 16 p ..), loaded while waiting
    const double* W = dinv + (size_t)B * 2 * NBK * NBK + (fwd ? 0 : NBK * NBK);
    double w[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = W[i * NBK + 16 * p + q];
    double acc = 0.0;
    const int nd = fwd ? B : T - 1 - B;
    for (int t = 0; t < nd; ++t) {
        const int C = fwd ? t : T - 1 - t;
        const int c0 = C * NBK + 16 * p;
        double m[16];
        const double* row = L + (size_t)(r0 + min(i, nb - 1)) * n;
#pragma unroll
        for (int q = 0; q < 16; ++q) m[q] = (i < nb && c0 + q < n) ? row[c0 + q] : 0.0;
        if (threadIdx.x < NBK) {
            const int cc = C * NBK + threadIdx.x;
            vsh[threadIdx.x] = cc < n ? wait_value(res + (fwd ? 0 : n) + cc, spin, flag) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += m[q] * vsh[16 * p + q];
        __syncthreads();   // vsh is rewritten next
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (p == 0) {
        const double rhs = i < nb ? (fwd ? dsc[r0 + i] * b[r0 + i] : wait_value(res + r0 + i, spin, flag))
                                  : 0.0;
        vsh[i] = i < nb ? rhs - acc : 0.0;
    }
    __syncthreads();
    double y = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) y += w[q] * vsh[16 * p + q];
    y += __shfl_xor(y, 1, 64);
    y += __shfl_xor(y, 2, 64);
    if (p == 0 && i < nb) {
        if (publish)
            __hip_atomic_store(res + (fwd ? 0 : n) + r0 + i, __builtin_bit_cast(unsigned long long, y),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!fwd) {
            const bool bad = *flag != 0;
            const double z = bad ? __builtin_nan("") : dsc[r0 + i] * y;
            coef[r0 + i] = accumulate ? coef[r0 + i] + z : z;
        }
    }
}

hipError_t launch_clear_flag(const Geom& g, int* flag, double* tsv, hipStream_t st) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1, 1, g.nb), dim3(256), 0, st, flag, tsv, g.nu, g.zs);
    return hipGetLastError();
}

hipError_t launch_jacobi(const Geom& g, int n, const double* G, const double* h, double* L,
                         double* dsc, double* rhs, int* flag, hipStream_t st) {
    (void)h;
    (void)rhs;
    hipLaunchKernelGGL(jacobi_kernel, dim3(n, 1, g.nb), dim3(256), 0, st, n, G, dsc, L, flag, g.zs);
    return hipGetLastError();
}

hipError_t launch_cholesky(const Geom& g, int n, double* L, double* dfac, double* dinv, int* flag,
                           hipStream_t st) {
    const int T = (n + NBK - 1) / NBK;
    for (int k = 0; k < T; ++k) {
        const int npan = T - k;
        const int ntrail = k > 0 ? (T - k - 1) * (T - k) / 2 : 0;
        hipLaunchKernelGGL(chol_step_kernel, dim3(npan + ntrail, 1, g.nb), dim3(kStepThreads), 0, st,
                           n, L, k, dfac, flag, g.zs);
    }
    hipLaunchKernelGGL(diag_finish_kernel, dim3(T, 1, g.nb), dim3(256), 0, st, n, L, dfac, dinv, g.zs);
    if (T > 1)
        hipLaunchKernelGGL(mirror_kernel, dim3(T * (T - 1) / 2, 1, g.nb), dim3(256), 0, st, n, L, g.zs);
    return hipGetLastError();
}

hipError_t launch_chol_solve(const Geom& g, int n, const double* L, const double* dinv,
                             const double* dsc,
                             const double* rhs, double* coef, int accumulate, int* flag,
                             double* tsv, int gen, int stall_test, hipStream_t st) {
    const int T = (n + NBK - 1) / NBK;
    // under the give-up test no block publishes its result, and the bound is
    // short: each wait gives up, every block exits
    const int spin = stall_test ? kStallTestSpin : kSolveSpin;
    // placement: see the kernel
    const int wgs = g.nb == 1 ? 8 * ((2 * T + 7) / 8) : 8 * 2 * T * ((g.nb + 7) / 8);
    hipLaunchKernelGGL(trsv_flow_kernel, dim3(wgs), dim3(256), 0, st, n, L, dinv, dsc,
                       rhs, coef, accumulate, flag, tsv, gen, stall_test ? 0 : 1, spin, g.nb, g.zs);
    return hipGetLastError();
}

}  // namespace sfft
