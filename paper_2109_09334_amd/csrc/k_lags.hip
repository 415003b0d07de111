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

#include <algorithm>
#include <cstdlib>
#include <type_traits>

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

template <typename T, typename PL>
__global__ void __launch_bounds__(512) lagcol_kernel(Geom g, LinePlan lp, int p0, int np, int sslot,
                                                      const cx<T>* __restrict__ X,
                                                      cx<T>* __restrict__ Cl,
                                                      const cx<T>* __restrict__ twt) {
    cx<T>* lds = lds_base_l<T>();
    X = zoff(X, g.zs);
    Cl = zoff(Cl, g.zs);
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    // Block -> (column block, product): the products of one column block run
    // back to back on one XCD (workgroups are dealt to the 8 XCDs round
    // robin), so the column's spectra are read from HBM once and reused in L2.
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int jx = slot / np;
    const int p = p0 + (slot - jx * np);
    const int cb = 8 * jx + xcd;
    const int m = cb * lp.lpw + line;
    const bool act = m < g.h;
    const int n0 = g.n0;
    int kb, k;
    if (p < g.npair) decode_pair(g.P, p, kb, k);
    else { kb = p - g.npair; k = sslot; }
    const int K = p < g.npair ? 2 * g.w0 : g.w0;
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    cx<T> v[kElemsPerThread];
    if (act) {
        const cx<T>* A = X + ((size_t)kb * g.h + m) * n0;
        const cx<T>* B = X + ((size_t)k * g.h + m) * n0;
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int l = lt + e * lp.tl;   // >= n0: a Bluestein line's padding
            const int lc = pad_index<PL>(l, n0);
            v[e] = in_line<PL>(l, n0) ? cmulc(A[lc], B[lc]) : mk(T(0), T(0));
        }
    } else {
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) v[e] = mk(T(0), T(0));
    }
    line_dft<1, T, PL>(v, buf, lp, lt, twt);
    if (act) {
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int l = lt + e * lp.tl;   // lag d0 = l or l - N0
            const int d0 = l <= K ? l : l - n0;
            if (in_line<PL>(l, n0) && d0 >= -K && d0 <= K)
                Cl[((size_t)p * g.D0 + d0 + 2 * g.w0) * g.hp + m] = v[e];
        }
    }
}

// Pruned inverse along axis 0 by decimation. Thread j of a line holds the
// 16 strided product values P(j + M q), q < 16 (M = N0/16 threads per line),
// and applies the radix-16 inverse DFT in registers:
//   Y_j(r) = sum_q P(j + M q) e^(+2 pi i q r / 16).
// Each kept lag d0 is then the M-term sum
//   C(d0) = sum_j e^(+2 pi i j d0 / N0) Y_j(d0 mod 16),
// formed 16 lags at a time (one per residue r) and summed over the lanes of
// each wave by a transpose-reduce (every step halves the values a lane
// carries and doubles the lanes each value is summed over), then across
// waves through LDS. One block covers one column and one kernel term kb and
// keeps conj(X_kb) in registers for all of that term's products.
// Lane exchanges of the transpose-reduce (CDNA4 VALU forms, no LDS):
// swap32(a, b): a := [a(0..31) | b(0..31)], b := [a(32..63) | b(32..63)];
// swap16(a, b): the same on 16-lane rows (odd rows of a <-> even rows of b);
// dpp<CTRL>(x): x of lane L ^ 8 (row_ror:8), of lane 8 (L/8) + 7 - L%8
// (row_half_mirror), of L ^ 1, of L ^ 2 (quad permutes).
__device__ __forceinline__ void swap32(float& a, float& b) {
    auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}
__device__ __forceinline__ void swap32(double& a, double& b) {
    float2 x = __builtin_bit_cast(float2, a), y = __builtin_bit_cast(float2, b);
    swap32(x.x, y.x);
    swap32(x.y, y.y);
    a = __builtin_bit_cast(double, x);
    b = __builtin_bit_cast(double, y);
}
__device__ __forceinline__ void swap16(double& a, double& b) {
    float2 x = __builtin_bit_cast(float2, a), y = __builtin_bit_cast(float2, b);
    swap16(x.x, y.x);
    swap16(x.y, y.y);
    a = __builtin_bit_cast(double, x);
    b = __builtin_bit_cast(double, y);
}
constexpr int kDppXor8 = 0x128, kDppHalfMirror = 0x141, kDppXor1 = 0xB1, kDppXor2 = 0x4E;
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double x) {
    float2 v = __builtin_bit_cast(float2, x);
    v.x = dpp<CTRL>(v.x);
    v.y = dpp<CTRL>(v.y);
    return __builtin_bit_cast(double, v);
}
template <int CTRL, typename T>
__device__ __forceinline__ cx<T> dpp(cx<T> x) {
    return mk(dpp<CTRL>(x.re), dpp<CTRL>(x.im));
}

// Wave-wide sums of 16 slots per lane. Every step halves the values a lane
// carries and doubles the lanes each one is summed over: lanes L and L ^ 32,
// then L ^ 16 (register swaps: each lane ends with its half of both), then
// L ^ 8 and the mirror pair within 8 lanes (the lane sends the half it does
// not keep), then the quad. After the call lane L holds in v[0] the sum of
// slot (L >> 2) & 15 over the wave (all 64 lanes must be active).
template <typename T>
__device__ __forceinline__ void wave_transpose_sum16(cx<T>* v, int lane) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        swap32(v[i].re, v[i + 8].re);
        swap32(v[i].im, v[i + 8].im);
        v[i] = v[i] + v[i + 8];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        swap16(v[i].re, v[i + 4].re);
        swap16(v[i].im, v[i + 4].im);
        v[i] = v[i] + v[i + 4];
    }
    const bool h8 = (lane & 8) != 0, h4 = (lane & 4) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const cx<T> send = h8 ? v[i] : v[i + 2];
        const cx<T> keep = h8 ? v[i + 2] : v[i];
        v[i] = keep + dpp<kDppXor8>(send);
    }
    {
        const cx<T> send = h4 ? v[0] : v[1];
        const cx<T> keep = h4 ? v[1] : v[0];
        v[0] = keep + dpp<kDppHalfMirror>(send);
    }
    v[0] = v[0] + dpp<kDppXor1>(v[0]);
    v[0] = v[0] + dpp<kDppXor2>(v[0]);
}

// Table index of the twiddle of slot r in lag block tb, e^(-2 pi i j t / N0)
// with t the lag the slot carries, t = tb + ((r - tb) mod 16); |j t| < 3 N0
// (|t| <= 4 w0 + 15, j < N0/16, 4 w0 < N0).
__device__ __forceinline__ int lag_twiddle_index(int n0, int j, int tb, int r) {
    const int mres = tb & 15;
    const int t = tb - mres + r + (r < mres ? 16 : 0);
    int idx = j * t;
    // a power-of-two N0 reduces the (possibly negative) product with a mask
    if ((n0 & (n0 - 1)) == 0) return idx & (n0 - 1);
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) idx += idx < 0 ? n0 : 0;
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) idx -= idx >= n0 ? n0 : 0;
    return idx;
}

// NB > 0: the Omega lags span NB blocks of 16 and the thread's twiddles are
// formed once and kept in registers: FP32, block 0's 16 twiddles and the
// factor that carries them to block 1; FP64, the 16 NB table indices
// (Theta's lags lie in the same range at the same slot residues, so they
// take the Omega block's twiddle); NB = 0: indices are formed per product
// and block.
template <typename T, int NB>
__global__ void __launch_bounds__(512) lagcol_tail_kernel(Geom g, LinePlan lp, int ir_only,
                                                           int sslot, int pchunk,
                                                           const cx<T>* __restrict__ X,
                                                           cx<T>* __restrict__ Cl,
                                                           const cx<T>* __restrict__ tw) {
    // red[product in chunk][lag block][wave of the workgroup][16]: wave sums
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* red = reinterpret_cast<cx<T>*>(smem_raw);
    X = zoff(X, g.zs);
    Cl = zoff(Cl, g.zs);
    const int tl = lp.tl;                       // M: threads per line, multiple of 64
    const int line = threadIdx.x / tl, j = threadIdx.x - line * tl;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const int nwl = tl >> 6;                    // waves per line
    // ir_only: one block per column block holds the spectrum in slot sslot
    // and forms conj(X_k) X_sslot for every kernel term k (Theta products
    // only). Otherwise a block holds X_kb and forms its Omega products with
    // k >= kb and its Theta product. With the twiddles in registers (FP32) a
    // block takes kb and P - 1 - kb in turn (P + 2 products, the same for
    // every block), so its twiddles serve twice as many products; the
    // column's ceil(P/2) blocks are adjacent on one XCD and run together,
    // sharing the spectra's columns through L2. FP64: one block per kb.
    constexpr bool kTwReg = NB > 0 && sizeof(T) == 4;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int nkbb = ir_only ? 1 : (kTwReg ? (g.P + 1) / 2 : g.P);   // blocks per column block
    const int jx = slot / nkbb, kbb = slot - jx * nkbb;
    const int cb = 8 * jx + xcd;
    const int m = cb * lp.lpw + line;
    const bool act = m < g.h;
    const int n0 = g.n0;
    const int KO = 2 * g.w0, nblk = (2 * KO + 16) / 16;   // lag blocks of Omega (Theta uses fewer)
    // FP32: the conjugated twiddles of Omega block 0 stay in registers. Slot
    // r of block b carries the lag of block 0's slot r plus 16 b, so block
    // 1's twiddles are block 0's times the one factor e^(+2 pi i 16 j / N0)
    // (16 j < N0), which is all that is kept for it. FP64: the NB blocks'
    // table indices stay in registers.
    int twi[(NB > 0 && !kTwReg) ? NB : 1][16];
    cx<T> tw0[16], tstep = mk(T(1), T(0));
    if constexpr (kTwReg) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tw0[r] = cconj(tw[lag_twiddle_index(n0, j, -KO, r)]);
        if constexpr (NB == 2) tstep = cconj(tw[16 * j]);
    } else if constexpr (NB > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) twi[b][r] = lag_twiddle_index(n0, j, -KO + 16 * b, r);
    }
    const int nq = (!ir_only && kTwReg && g.P - 1 - kbb != kbb) ? 2 : 1;
#pragma unroll 1
    for (int half = 0; half < nq; ++half) {
        const int kb = ir_only ? 0 : (half == 0 ? kbb : g.P - 1 - kbb);
        cx<T> a[16];
        if (act) {
            const cx<T>* A = X + ((size_t)(ir_only ? sslot : kb) * g.h + m) * n0 + j;
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = A[(size_t)q * tl];
        }
        const int kbeg = ir_only ? 0 : kb, kend = ir_only ? g.P : g.P + 1;
        for (int k0 = kbeg; k0 < kend; k0 += pchunk) {
            const int k1 = min(kend, k0 + pchunk);
            for (int kk = k0; kk < k1; ++kk) {
                const bool theta = ir_only || kk == g.P;
                const int k = ir_only ? kk : (theta ? sslot : kk);
                const int K = theta ? g.w0 : KO;
                cx<T> v[16];
                if (act) {
                    const cx<T>* B = X + ((size_t)k * g.h + m) * n0 + j;
                    if (ir_only) {
#pragma unroll
                        for (int q = 0; q < 16; ++q) v[q] = cmulc(B[(size_t)q * tl], a[q]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 16; ++q) v[q] = cmulc(a[q], B[(size_t)q * tl]);
                    }
                    Dft<16, 1, T>::run(v);
                } else {
#pragma unroll
                    for (int q = 0; q < 16; ++q) v[q] = mk(T(0), T(0));
                }
                if constexpr (kTwReg) {
                    // NB <= 2 gives Omega NB blocks and Theta (|t| <= w0 < 8)
                    // one, whose slot r lies in Omega block (t + KO) / 16 at
                    // the same residue (uniform over the wave)
                    cx<T> s[16];
#pragma unroll
                    for (int r = 0; r < 16; ++r) s[r] = cmul(v[r], tw0[r]);
                    auto store = [&](cx<T>* x, int blk) {
                        wave_transpose_sum16(x, lane);
                        if ((lane & 3) == 0)
                            red[(((size_t)(kk - k0) * nblk + blk) * nwv + wv) * 16 + ((lane >> 2) & 15)] = x[0];
                    };
                    if constexpr (NB == 2) {
                        if (theta) {
                            const int tb = -K, mres = tb & 15;
#pragma unroll
                            for (int r = 0; r < 16; ++r) {
                                const int t = tb - mres + r + (r < mres ? 16 : 0);
                                if (t + KO >= 16) s[r] = cmul(s[r], tstep);
                            }
                            store(s, 0);
                        } else {
                            cx<T> s1[16];
#pragma unroll
                            for (int r = 0; r < 16; ++r) s1[r] = cmul(s[r], tstep);
                            store(s, 0);
                            store(s1, 1);
                        }
                    } else {
                        store(s, 0);
                    }
                    continue;
                }
                for (int blk = 0; 16 * blk <= 2 * K; ++blk) {
                    const int tb = -K + 16 * blk;
                    cx<T> s[16];
                    if constexpr (NB > 0 && !kTwReg) {
                        // Omega: block blk; Theta: slot r's lag t lies in Omega
                        // block (t + KO) / 16 at the same slot
                        const int mres = tb & 15;
#pragma unroll
                        for (int r = 0; r < 16; ++r) {
                            const int t = tb - mres + r + (r < mres ? 16 : 0);
                            const int ob = theta ? (t + KO) >> 4 : blk;
                            int idx = twi[0][r];
#pragma unroll
                            for (int b = 1; b < NB; ++b)
                                if (b == ob) idx = twi[b][r];
                            s[r] = cmul(v[r], cconj(tw[idx]));   // e^(+2 pi i j t / N0)
                        }
                    } else {
#pragma unroll
                        for (int r = 0; r < 16; ++r)
                            s[r] = cmul(v[r], cconj(tw[lag_twiddle_index(n0, j, tb, r)]));
                    }
                    wave_transpose_sum16(s, lane);
                    if ((lane & 3) == 0)
                        red[(((size_t)(kk - k0) * nblk + blk) * nwv + wv) * 16 + ((lane >> 2) & 15)] = s[0];
                }
            }
            __syncthreads();
            // line sums: one output (product, block, slot) per thread of the line
            const int nout = (k1 - k0) * nblk * 16;
            for (int o = j; o < nout; o += tl) {
                const int r = o & 15, blk = (o >> 4) % nblk, ip = (o >> 4) / nblk;
                const int kk = k0 + ip;
                const bool theta = ir_only || kk == g.P;
                const int K = theta ? g.w0 : KO;
                const int tb = -K + 16 * blk;
                const int t = tb + ((r - tb) & 15);
                if (!act || 16 * blk > 2 * K || t > K) continue;
                cx<T> tot = red[(((size_t)ip * nblk + blk) * nwv + line * nwl) * 16 + r];
                for (int w = 1; w < nwl; ++w)
                    tot = tot + red[(((size_t)ip * nblk + blk) * nwv + line * nwl + w) * 16 + r];
                const int p = theta ? g.npair + (ir_only ? kk : kb)
                                    : kb * g.P - kb * (kb - 1) / 2 + (kk - kb);
                Cl[((size_t)p * g.D0 + t + 2 * g.w0) * g.hp + m] = tot;
            }
            __syncthreads();
        }
    }
}

// Pruned inverse along axis 0 for a Bluestein line (N0 = nl not 16 x its
// threads per line, transform length M = 16 TL): the lags of the inverse
// DFT of length nl, C(d0) = sum_l P(l) e^(+2 pi i l d0 / nl), |d0| <= K, are
// conj of the forward DFT of conj(P) at k = d0 mod nl. In the Bluestein form
// that forward DFT is F(k) = conj(c_k) z(k), z = IDFT_M(DFT_M(a) bhat) with
// a_t = conj(c_t) conj(P(t)): one forward M-point transform per product, and
// z only at k in [0, K] and [nl - K, nl), by the decimation of
// lagcol_tail_kernel (thread j holds DFT_M(a) bhat at j + TL q, q < 16; the
// radix-16 inverse over q; each 16-slot block of k summed over the line
// with twiddles e^(+2 pi i j k / M), the wave transpose-reduce, and the
// waves' sums through LDS). Then C(d0) = c_k conj(z(k)). The chirp products
// are formed in FP64, as in line_dft.
template <typename T, typename PL>
__global__ void __launch_bounds__(512) lagcol_chirp_kernel(Geom g, LinePlan lp, int p0, int np,
                                                            int sslot, const cx<T>* __restrict__ X,
                                                            cx<T>* __restrict__ Cl,
                                                            const cx<T>* __restrict__ twt) {
    using P = typename PL::plan;
    cx<T>* lds = lds_base_l<T>();
    X = zoff(X, g.zs);
    Cl = zoff(Cl, g.zs);
    const int tl = lp.tl;
    const int line = threadIdx.x / tl, lt = threadIdx.x - line * tl;
    const int lane = threadIdx.x & 63, nwl = tl >> 6, wl = (threadIdx.x >> 6) - line * nwl;
    // block -> (column block, product) as in lagcol_kernel
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int jx = slot / np;
    const int p = p0 + (slot - jx * np);
    const int cb = 8 * jx + xcd;
    const int m = cb * lp.lpw + line;
    const bool act = m < g.h;
    const int nl = g.n0, M = lp.n;
    int kb, k;
    if (p < g.npair) decode_pair(g.P, p, kb, k);
    else { kb = p - g.npair; k = sslot; }
    const int K = p < g.npair ? 2 * g.w0 : g.w0;
    cx<T>* buf = lds + line * line_lds_elems(M);
    const cx<double>* __restrict__ ch = static_cast<const cx<double>*>(lp.chirp);
    const cx<double>* __restrict__ bh = static_cast<const cx<double>*>(lp.bhat);
    const cx<T>* __restrict__ twm = static_cast<const cx<T>*>(lp.twm);
    auto wide = [](cx<T> a) { return mk((double)a.re, (double)a.im); };
    auto narrow = [](cx<double> a) { return mk(T(a.re), T(a.im)); };
    cx<T> v[kElemsPerThread];
    const cx<T>* A = X + ((size_t)kb * g.h + (act ? m : 0)) * nl;
    const cx<T>* B = X + ((size_t)k * g.h + (act ? m : 0)) * nl;
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e) {
        const int t = lt + e * tl;
        const bool in = act && t < nl;
        const int tc = t < nl ? t : nl - 1;
        const cx<T> pr = cmulc(A[tc], B[tc]);
        v[e] = in ? narrow(cmulc(ch[tc], wide(cconj(pr)))) : mk(T(0), T(0));
    }
    line_fft<-1, T, P>(v, buf, lp, lt, twt);
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e) v[e] = narrow(cmul(wide(v[e]), bh[lt + e * tl]));
    Dft<16, 1, T>::run(v);
    __syncthreads();   // every thread is past the transform's LDS reads
    // red[blk][wave of the line][16] in the line's buffer
    const int nlo = (K + 16) / 16, nhi = (K + 15) / 16;
#pragma unroll 1
    for (int blk = 0; blk < nlo + nhi; ++blk) {
        const int tb = blk < nlo ? 16 * blk : nl - K + 16 * (blk - nlo);
        cx<T> s[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kk = tb + ((r - tb) & 15);   // the slot's k (k = r mod 16)
            s[r] = cmul(v[r], cconj(twm[(int)(((long long)lt * kk) & (M - 1))]));
        }
        wave_transpose_sum16(s, lane);
        if ((lane & 3) == 0) buf[(blk * nwl + wl) * 16 + ((lane >> 2) & 15)] = s[0];
    }
    __syncthreads();
    for (int o = lt; o < (nlo + nhi) * 16; o += tl) {
        const int blk = o >> 4, r = o & 15;
        const bool lo = blk < nlo;
        const int tb = lo ? 16 * blk : nl - K + 16 * (blk - nlo);
        const int kk = tb + ((r - tb) & 15);
        if (!act || (lo ? kk > K : kk >= nl)) continue;
        cx<T> z = buf[(blk * nwl) * 16 + r];
        for (int w = 1; w < nwl; ++w) z = z + buf[(blk * nwl + w) * 16 + r];
        const int d0 = lo ? kk : kk - nl;
        Cl[((size_t)p * g.D0 + d0 + 2 * g.w0) * g.hp + m] = narrow(cmul(ch[kk], wide(cconj(z))));
    }
}

// The same lags as a dense contraction on the FP32 matrix cores, for the
// FP32 transforms of a Bluestein column (its length has no radix-16 split):
// per column m, C(d0, p) = sum_l E(d0, l) P_p(l), E = e^(+2 pi i l d0 / N0),
// for the products p of the call (conj(X_kb) X_k) and |d0| <= Kmax. As a real
// product: rows 2 di + s (lag di = d0 + Kmax; s = 0 real, 1 imaginary part
// of C), contraction index 2 l + c (c = 0 real, 1 imaginary part of P), so
// the E block of (s, c) is [[Re E, -Im E], [Im E, Re E]]. Wave rb owns row
// block rb (eight lags) and every 16-column block of products. N0 is taken
// in chunks of 32 points: the chunk's column spectra and products are
// staged in LDS (FP32), each lane steps its E(d0, l) through the chunk by
// the FP64 recurrence E(l + 2) = E(l) e^(+2 pi i 2 d0 / N0) from a table
// value, and the chunk's FP32 accumulators are added into FP64 totals (the
// output register q of lane L holds row 4 (L / 16) + q, column L % 16, so a
// lane ends with the real and imaginary parts of two lags).
typedef float flt4 __attribute__((ext_vector_type(4)));
constexpr int kDftChunk = 32;
constexpr int kDftMaxSpec = 16;   // spectra a call reads (P + 2 at DK = 4)
constexpr int kDftMaxProd = 64;   // products of a call (nprod = 35 at DK = 4)

template <int NCB>
__global__ void __launch_bounds__(512) lagcol_dft_kernel(Geom g, int p0, int np, int sslot,
                                                          int nspec, int kmax,
                                                          const cx<float>* __restrict__ X,
                                                          cx<float>* __restrict__ Cl,
                                                          const double* __restrict__ twp) {
    __shared__ cx<float> xs[kDftMaxSpec][kDftChunk];
    __shared__ cx<float> ps[kDftChunk][kDftMaxProd];
    __shared__ unsigned char pkb[kDftMaxProd], pk[kDftMaxProd];
    X = zoff(X, g.zs);
    Cl = zoff(Cl, g.zs);
    const int m = blockIdx.x, n0 = g.n0;
    const int lane = threadIdx.x & 63, rb = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    constexpr int NPP = 16 * NCB;   // products padded to whole 16-column blocks
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
        const int p = p0 + t;
        int kb, k;
        if (p < g.npair) decode_pair(g.P, p, kb, k);
        else { kb = p - g.npair; k = sslot; }
        pkb[t] = (unsigned char)kb;
        pk[t] = (unsigned char)k;
    }
    // this lane's A row: lag d0 = (16 rb + lr) / 2 - kmax, part s = lr % 2;
    // its contraction slots: point 2 j + lk / 2 of step j, part c = lk % 2
    const int d0 = (16 * rb + lr) / 2 - kmax, sa = lr & 1, ca = lk & 1;
    const int step = imod(2 * d0, n0);
    const double sr = twp[2 * step], si = twp[2 * step + 1];   // e^(+2 pi i 2 d0 / N0)
    double tot[NCB][4];
#pragma unroll
    for (int b = 0; b < NCB; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) tot[b][q] = 0.0;
    const cx<float>* xc = X + (size_t)m * n0;
#pragma unroll 1
    for (int l0 = 0; l0 < n0; l0 += kDftChunk) {
        __syncthreads();   // the previous chunk's LDS reads are done
        for (int t = threadIdx.x; t < nspec * kDftChunk; t += blockDim.x) {
            const int sp = t / kDftChunk, l = l0 + t % kDftChunk;
            xs[sp][t % kDftChunk] = l < n0 ? xc[(size_t)sp * g.h * n0 + l] : mk(0.0f, 0.0f);
        }
        __syncthreads();
        for (int t = threadIdx.x; t < NPP * kDftChunk; t += blockDim.x) {
            const int l = t / NPP, pp = t - l * NPP;
            ps[l][pp] = pp < np ? cmulc(xs[pkb[pp]][l], xs[pk[pp]][l]) : mk(0.0f, 0.0f);
        }
        __syncthreads();
        // E at this lane's first point of the chunk, l0 + lk / 2
        // l0 < N0 <= 8192 and |d0| < 64: the product fits 32 bits
        const int e0 = imod((l0 + (lk >> 1)) * d0 % n0, n0);
        double er = twp[2 * e0], ei = twp[2 * e0 + 1];
        // the lane's part (re / im) of P at column 16 b + lr, point 2 j + lk / 2
        const float* pb = reinterpret_cast<const float*>(&ps[lk >> 1][lr]) + ca;
        flt4 acc[NCB];
#pragma unroll
        for (int b = 0; b < NCB; ++b) acc[b] = flt4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < kDftChunk / 2; ++j) {
            // A = [[Re E, -Im E], [Im E, Re E]] at (s, c)
            const float a = (float)(sa == ca ? er : (sa ? ei : -ei));
            float bv[NCB];
#pragma unroll
            for (int b = 0; b < NCB; ++b) bv[b] = pb[2 * (2 * j * kDftMaxProd + 16 * b)];
#pragma unroll
            for (int b = 0; b < NCB; ++b)
                acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv[b], acc[b], 0, 0, 0);
            const double nr = er * sr - ei * si;
            ei = er * si + ei * sr;
            er = nr;
        }
#pragma unroll
        for (int b = 0; b < NCB; ++b) {
            tot[b][0] += (double)acc[b].x;
            tot[b][1] += (double)acc[b].y;
            tot[b][2] += (double)acc[b].z;
            tot[b][3] += (double)acc[b].w;
        }
    }
    // rows 4 lk + q of row block rb: lag 8 rb + 2 lk (q = 0, 1) and + 1 (q = 2, 3)
#pragma unroll
    for (int b = 0; b < NCB; ++b) {
        const int pp = 16 * b + lr;
        if (pp >= np) continue;
        const int p = p0 + pp;
        const int K = p < g.npair ? 2 * g.w0 : g.w0;
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
            const int d = 8 * rb + 2 * lk + h2 - kmax;
            if (d < -K || d > K) continue;
            Cl[((size_t)p * g.D0 + d + 2 * g.w0) * g.hp + m] =
                mk((float)tot[b][2 * h2], (float)tot[b][2 * h2 + 1]);
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
    Cl = zoff(Cl, g.zs);
    omega = zoff(omega, g.zs);
    theta = zoff(theta, g.zs);
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
            double cr = wm * (double)c.re, ci = wm * (double)c.im;
            // (cr + i ci) e^(+2 pi i m d1 / N1) for d1 = base, base+1, ...: one
            // table value for the first lag, then FP64 angle addition
            const int i0 = imod(m * base, n1);
            const double e0r = twp[2 * i0], e0i = twp[2 * i0 + 1];
            const double sr = twp[2 * m], si = twp[2 * m + 1];
            double xr = cr * e0r - ci * e0i, xi = cr * e0i + ci * e0r;
#pragma unroll
            for (int t = 0; t < kLagChunk; ++t) {
                acc[t] += xr;
                const double nr = xr * sr - xi * si;
                xi = xr * si + xi * sr;
                xr = nr;
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
                         const cx<T>* X, cx<T>* Cl, const cx<T>* tw, const cx<T>* twt,
                         const double* twp, hipStream_t st) {
    if (p1 <= p0) return hipSuccess;
    static const bool force_full = getenv("SFFT_LAGCOL_FULL") != nullptr;
    // (the pruned pass needs N0 = 16 x its threads per line: not a Bluestein line)
    if (!force_full && !lp.chirp && lp.tl % 64 == 0 && lp.tl * lp.lpw <= 512 &&
        ((p0 == 0 && p1 == g.nprod) || (p0 == g.npair && p1 == g.nprod))) {
        const int ncb = (g.h + lp.lpw - 1) / lp.lpw;
        const int nwv = lp.tl * lp.lpw / 64;
        const int nblk = (4 * g.w0 + 16) / 16;
        const size_t per = (size_t)nblk * nwv * 16 * sizeof(cx<T>);
        const int pchunk = (int)std::max<size_t>(1, std::min<size_t>(g.P + 1, 32768 / per));
        const bool ir_only = p0 != 0;
        // blocks per column block: ceil(P/2) when the kernel keeps its
        // twiddles in registers (FP32, one or two lag blocks; kb paired with
        // P - 1 - kb), P otherwise, 1 for the Theta-only pass
        const bool tw_reg = sizeof(T) == 4 && (nblk == 1 || nblk == 2);
        const int per_col = ir_only ? 1 : (tw_reg ? (g.P + 1) / 2 : g.P);
        dim3 grid((ncb + 7) / 8 * 8 * per_col, 1, g.nb);
        auto k = nblk == 1 ? lagcol_tail_kernel<T, 1>
                 : nblk == 2 ? lagcol_tail_kernel<T, 2> : lagcol_tail_kernel<T, 0>;
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), pchunk * per, st, g, lp, ir_only ? 1 : 0,
                           sslot, pchunk, X, Cl, tw);
        return hipGetLastError();
    }
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    const int ncb = (g.h + lp.lpw - 1) / lp.lpw;
    dim3 grid((ncb + 7) / 8 * 8 * (p1 - p0), 1, g.nb);
    // Bluestein lines, FP32, the build's products (all of them): the lags as a
    // dense contraction on the matrix cores (row blocks of eight lags, up to
    // 64 products in 16-column blocks); the refinement's few Theta products
    // take the transform path below
    if constexpr (sizeof(T) == 4) {
        const int kmax = p0 == 0 ? 2 * g.w0 : g.w0;
        const int nspec = std::max(g.P + 1, sslot + 1);
        const int rbs = (2 * (2 * kmax + 1) + 15) / 16;
        if (!force_full && p0 == 0 && lp.chirp && twp && rbs * 64 <= 512 &&
            p1 - p0 <= kDftMaxProd && nspec <= kDftMaxSpec) {
            const int ncb = (p1 - p0 + 15) / 16;
            auto k = ncb == 1 ? lagcol_dft_kernel<1>
                     : ncb == 2 ? lagcol_dft_kernel<2>
                     : ncb == 3 ? lagcol_dft_kernel<3> : lagcol_dft_kernel<4>;
            hipLaunchKernelGGL(k, dim3(g.h, 1, g.nb), dim3(64 * rbs), 0, st, g, p0, p1 - p0, sslot,
                               nspec, kmax, X, Cl, twp);
            return hipGetLastError();
        }
    }
    // Bluestein lines: one forward transform per product and the kept lags
    // of the inverse only (needs waves of whole lines and the M-point twiddles)
    if (!force_full && lp.chirp && lp.twm && lp.tl % 64 == 0) {
        return with_line_plan(lp, [&](auto pl) -> hipError_t {
            using PL = decltype(pl);
            if constexpr (IsChirp<PL>::value) {
                auto k = lagcol_chirp_kernel<T, PL>;
                if (lds > 65536) {
                    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)lds);
                    if (e != hipSuccess) return e;
                }
                hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, p0, p1 - p0, sslot,
                                   X, Cl, twt);
                return hipGetLastError();
            } else {
                return hipErrorInvalidValue;   // lp.chirp always gives a Chirp plan
            }
        });
    }
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        auto k = lagcol_kernel<T, decltype(pl)>;
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, p0, p1 - p0, sslot, X, Cl,
                           twt);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_lagrow(const Geom& g, int p0, int p1, const cx<T>* Cl, const double* twp,
                         double* omega, double* theta, hipStream_t st) {
    if (p1 <= p0) return hipSuccess;
    dim3 grid(g.D0, p1 - p0, g.nb);
    hipLaunchKernelGGL(lagrow_kernel<T>, grid, dim3(256), 0, st, g, p0, Cl, twp, omega, theta);
    return hipGetLastError();
}

template hipError_t launch_lagcol<float>(const Geom&, const LinePlan&, int, int, int,
                                         const cx<float>*, cx<float>*, const cx<float>*,
                                         const cx<float>*, const double*, hipStream_t);
template hipError_t launch_lagcol<double>(const Geom&, const LinePlan&, int, int, int,
                                          const cx<double>*, cx<double>*, const cx<double>*,
                                          const cx<double>*, const double*, hipStream_t);
template hipError_t launch_lagrow<float>(const Geom&, int, int, const cx<float>*, const double*,
                                         double*, double*, hipStream_t);
template hipError_t launch_lagrow<double>(const Geom&, int, int, const cx<double>*, const double*,
                                          double*, double*, hipStream_t);

}  // namespace sfft
