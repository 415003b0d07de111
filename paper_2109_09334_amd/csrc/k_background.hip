// FP64 polynomial-correlation tables and the pedestal corrections of the
// spectral lag tables.
//
// Poly-correlation of an image with monomials T^t = c0^i c1^j:
//   Pi_{ta tb}(d) = sum_u img(u) T^ta(u) T^tb((u + d) mod N)
// For img = R, ta = kb, tb = m this is Lambda_{kb m}(d) of Eq. B8; with
// img = S, ta = 0 it holds E_m = Pi_{0 m}(0) (Eq. B15). Because T^tb is
// separable, Pi = sum_u0 c0(u0)^ia c0((u0+d0) mod N0)^ib V_{ja jb}(u0, d1),
//   V_{ja jb}(u0, d1) = sum_u1 img(u0,u1) c1(u1)^ja c1((u1+d1) mod N1)^jb,
// and on the torus c1((u1+d1) mod N1) equals the straight-line value
// c1(u1) + 2 d1/(N1-1) except on the |d1| wrapped columns, so V is a
// binomial combination of the row moments M_e(u0) = sum_u1 img c1^e plus an
// explicit correction over the wrapped columns.
//
// Pedestal: the spectral path transforms R' = R - c_R and S' = S - c_S
// (c = image means, rounded to 8 significant bits) so that FP32 FFT rounding
// scales with the fluctuations and not with the sky level. The exact identities restore the full tables:
//   Omega_{kb k}(d) = Omega'(d) + c_R (Pi^R_{kb k}(d) + Pi^R_{k kb}(-d))
//                     - c_R^2 C_{kb k}(d),  C(d) = sum_x T^kb(x-d) T^k(x)
//   Theta_kb(d)     = Theta'(d) + c_S Pi^R_{kb 0}(0) + c_R Pi^S_{0 kb}(-d)
//                     - c_R c_S sum_x T^kb
// (expand R = R' + c_R, S = S' + c_S in Eq. B6, B14).
#include "kernels.hpp"

namespace sfft {

constexpr int kMaxMom = 2 * kMaxDegree + 1;

template <int NV>
__device__ __forceinline__ void block_sum_bg(double* v, double* red) {
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
        red[threadIdx.x] = s;
    }
    __syncthreads();
}

// One wave per row (four rows per 256-thread block):
// V[u0][ja][jb][d1 + K1], ja <= da, jb <= db, |d1| <= K1. The row moments
// are wave sums (every lane ends with all of them); the wrapped-column
// corrections read the row again (L1).
template <typename Tin, int NE>
__global__ void __launch_bounds__(256) polyrow_kernel(Geom g, IoRef<const Tin> imgr, int da,
                                                      int dbb, int K1, double* __restrict__ vrow) {
    const Tin* __restrict__ img = imgr.get(g.zs);
    vrow = zoff(vrow, g.zs);
    __shared__ double mom[4][kMaxMom];
    __shared__ double esum[4][2][NE][kPolyRowMaxLag + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x0 = blockIdx.x * 4 + wv;
    if (x0 >= g.n0) return;   // wave-level work only below
    const int n1 = g.n1;
    const Tin* row = img + (size_t)x0 * n1;
    // c1(x1) = (2 x1 - (N1 - 1)) / (N1 - 1) with the division as a product
    const double rn = 1.0 / (double)(n1 - 1);
    // edge pixel of this lane: column k of the left end (lane k < 32) or
    // of the right end (lane 32 + k), for k < K1; loaded ahead of the row
    const int ek = lane & 31, eside = lane >> 5;
    const int ex1 = eside ? n1 - 1 - ek : ek;
    const double epx = ek < K1 ? (double)row[min(max(ex1, 0), n1 - 1)] : 0.0;
    double mo[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) mo[e] = 0.0;
    // eight loads of the row in flight per lane, then their moments; the
    // loads past the row's end read its last pixel (clamped index, no
    // branch around the load) and are then dropped
    constexpr int kBatch = 8;
    for (int base = 0; base < n1; base += 64 * kBatch) {
        Tin ld[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) ld[q] = row[min(base + lane + 64 * q, n1 - 1)];
        double px[kBatch];
#pragma unroll
        for (int q = 0; q < kBatch; ++q) px[q] = base + lane + 64 * q < n1 ? (double)ld[q] : 0.0;
#pragma unroll
        for (int q = 0; q < kBatch; ++q) {
            const double c = (double)(2 * (base + lane + 64 * q) - (n1 - 1)) * rn;
            double pw = px[q];
#pragma unroll
            for (int e = 0; e < NE; ++e) {
                mo[e] += pw;
                pw *= c;
            }
        }
    }
    // The wrapped columns of shift d1 are the |d1| columns at one end of
    // the row (the right end for d1 > 0), where c1 of the wrapped column is
    // u - Delta with u = c1(x1) + 2 d1/(N1-1) and Delta = +-2 N1/(N1-1).
    // (u - Delta)^jb - u^jb expands in powers of Delta, u and then of
    // c1(x1), so the correction needs only the edge sums
    //   E_e(side, k) = sum of img c1^e over the k columns nearest that end,
    // formed once per row as prefix sums over the edge lanes.
    {
        const double cc = (double)(2 * ex1 - (n1 - 1)) * rn;
        double pw = epx;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            // inclusive prefix sum over the 32 lanes of this side
            double s = pw;
#pragma unroll
            for (int off = 1; off < 32; off <<= 1) {
                const double t = __shfl_up(s, off, 32);
                if (ek >= off) s += t;
            }
            esum[wv][eside][e][ek + 1] = s;
            if (ek == 0) esum[wv][eside][e][0] = 0.0;
            pw *= cc;
        }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        double x = mo[e];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        if (lane == 0) mom[wv][e] = x;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    // Shift d1 across the lanes, (ja, jb) uniform over the wave: the powers
    // of the shift and of -Delta are formed once per lane by the same
    // repeated products as ipow, and the binomial sums unroll on static
    // bounds (jb <= kMaxDegree).
    const int na = da + 1, nb = dbb + 1, nd = 2 * K1 + 1;
    const double del = 2.0 / (double)(n1 - 1);
    double* out = vrow + (size_t)x0 * na * nb * nd;
    for (int i = lane; i < nd; i += 64) {
        const int d1 = i - K1;
        const int side = d1 > 0 ? 1 : 0, k = d1 > 0 ? d1 : -d1;
        const double sh = del * (double)d1;
        const double mdelta = (d1 > 0 ? -2.0 : 2.0) * (double)n1 * rn;   // -Delta
        double shp[kMaxDegree + 1], mdp[kMaxDegree + 1];
        shp[0] = 1.0;
        mdp[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= kMaxDegree; ++q) {
            shp[q] = shp[q - 1] * sh;
            mdp[q] = mdp[q - 1] * mdelta;
        }
        for (int ja = 0; ja < na; ++ja) {
#pragma unroll
            for (int jb = 0; jb <= kMaxDegree; ++jb) {
                if (jb > dbb) break;
                double v = 0.0;
#pragma unroll
                for (int r = 0; r <= jb; ++r) v += binom(jb, r) * shp[jb - r] * mom[wv][ja + r];
                if (d1 != 0 && jb > 0) {
                    double corr = 0.0;
#pragma unroll
                    for (int t = 1; t <= jb; ++t) {
                        double inner = 0.0;
#pragma unroll
                        for (int q = 0; q <= jb - t; ++q)
                            inner += binom(jb - t, q) * shp[jb - t - q] * esum[wv][side][ja + q][k];
                        corr += binom(jb, t) * mdp[t] * inner;
                    }
                    v += corr;
                }
                out[(ja * nb + jb) * nd + i] = v;
            }
        }
    }
}

// Axis 0 goes the same way as axis 1 in polyrow_kernel: with
// c0((x0+d0) mod N0) = c0(x0) + 2 d0/(N0-1) off the |d0| wrapped rows,
//   Pi_{(ia,ja)(ib,jb)}(d0, d1) = sum_r C(ib,r) s^(ib-r) Mom_{ia+r}(ja, jb, d1)
//                                 + wrapped-row correction,
// with the axis-0 moments Mom_e(item) = sum_x0 c0(x0)^e V(x0, item) and
// item = (ja, jb, d1). The moments are summed per chunk of kPolyRowChunk rows,
// then the chunks in a fixed order (no atomics: the result does not depend
// on scheduling).
__global__ void __launch_bounds__(256) polymom_kernel(Geom g, const double* __restrict__ vrow,
                                                       int nitem, int ne,
                                                       double* __restrict__ part) {
    vrow = zoff(vrow, g.zs);
    part = zoff(part, g.zs);
    const int x0a = blockIdx.x * kPolyRowChunk, x0b = min(g.n0, x0a + kPolyRowChunk);
    const double rn = 1.0 / (double)(g.n0 - 1);
    for (int item = threadIdx.x; item < nitem; item += blockDim.x) {
        double m[kMaxMom];
#pragma unroll
        for (int e = 0; e < kMaxMom; ++e) m[e] = 0.0;
        for (int x0 = x0a; x0 < x0b; ++x0) {
            const double c = (double)(2 * x0 - (g.n0 - 1)) * rn;
            double pw = vrow[(size_t)x0 * nitem + item];
#pragma unroll
            for (int e = 0; e < kMaxMom; ++e) {
                if (e < ne) m[e] += pw;
                pw *= c;
            }
        }
#pragma unroll
        for (int e = 0; e < kMaxMom; ++e)
            if (e < ne) part[((size_t)blockIdx.x * ne + e) * nitem + item] = m[e];
    }
}

// mom[i] = sum over the row chunks (fixed order per lane, then a wave sum).
__global__ void __launch_bounds__(256) momsum_kernel(int nchunk, int nval,
                                                      const double* __restrict__ part,
                                                      double* __restrict__ mom, long long zs) {
    part = zoff(part, zs);
    mom = zoff(mom, zs);
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nval) return;
    double s = 0.0;
    for (int k = lane; k < nchunk; k += 64) s += part[(size_t)k * nval + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) mom[i] = s;
}

// One thread per output Pi[ta][tb][d0 + K0][d1 + K1].
__global__ void __launch_bounds__(256) polycorr_kernel(Geom g, const double* __restrict__ vrow,
                                                        const double* __restrict__ mom, int da,
                                                        int dbb, int K0, int K1,
                                                        double* __restrict__ pi) {
    vrow = zoff(vrow, g.zs);
    mom = zoff(mom, g.zs);
    pi = zoff(pi, g.zs);
    const int n0 = g.n0;
    const int nta = (da + 1) * (da + 2) / 2, ntb = (dbb + 1) * (dbb + 2) / 2;
    const int nd0 = 2 * K0 + 1, nd1 = 2 * K1 + 1;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nta * ntb * nd0 * nd1) return;
    const int d1 = idx % nd1;
    const int d0 = (idx / nd1) % nd0 - K0;
    const int tb = (idx / (nd1 * nd0)) % ntb;
    const int ta = idx / (nd1 * nd0 * ntb);
    int ia, ja, ib, jb;
    term_ij(da, ta, ia, ja);
    term_ij(dbb, tb, ib, jb);
    const int nb = dbb + 1;
    const int nitem = (da + 1) * nb * nd1;
    const int item = (ja * nb + jb) * nd1 + d1;
    const double rn = 1.0 / (double)(n0 - 1);
    const double sh = 2.0 * (double)d0 * rn;
    double v = 0.0;
    for (int r = 0; r <= ib; ++r)
        v += binom(ib, r) * ipow(sh, ib - r) * mom[(size_t)(ia + r) * nitem + item];
    const int lo = d0 > 0 ? n0 - d0 : 0, hi = d0 > 0 ? n0 : -d0;
    for (int x0 = lo; x0 < hi; ++x0) {
        const double c = (double)(2 * x0 - (n0 - 1)) * rn;
        const double tor = (double)(2 * imod(x0 + d0, n0) - (n0 - 1)) * rn;
        v += vrow[(size_t)x0 * nitem + item] * ipow(c, ia) * (ipow(tor, ib) - ipow(c + sh, ib));
    }
    pi[idx] = v;
}

// 1-D sums sig0[ab][a][d0] = sum_x0 c0((x0-d0) mod N0)^ab c0(x0)^a (and the
// same along axis 1), |d| <= 2w, exponents <= DK; pw0[e], pw1[e] = sum c^e
// for e <= 2 max(DK, DB). One block per (axis, ab, a, d) or power.
__global__ void __launch_bounds__(256) polysum_kernel(Geom g, int dmax, double* __restrict__ sig0,
                                                       double* __restrict__ sig1,
                                                       double* __restrict__ pw) {
    __shared__ double red[4];
    sig0 = zoff(sig0, g.zs);
    sig1 = zoff(sig1, g.zs);
    pw = zoff(pw, g.zs);
    const int ne = g.dk + 1;
    const int ns0 = ne * ne * g.D0, ns1 = ne * ne * g.D1;
    int b = blockIdx.x;
    int axis, ab = 0, a = 0, d = 0, e = 0;
    bool power = false;
    if (b < ns0) {
        axis = 0;
        ab = b / (ne * g.D0);
        a = (b / g.D0) % ne;
        d = b % g.D0 - 2 * g.w0;
    } else if (b < ns0 + ns1) {
        b -= ns0;
        axis = 1;
        ab = b / (ne * g.D1);
        a = (b / g.D1) % ne;
        d = b % g.D1 - 2 * g.w1;
    } else {
        b -= ns0 + ns1;
        power = true;
        axis = b / (2 * dmax + 1);
        e = b % (2 * dmax + 1);
    }
    const int n = axis ? g.n1 : g.n0;
    const double rn = 1.0 / (double)(n - 1);
    double acc = 0.0;
    for (int x = threadIdx.x; x < n; x += blockDim.x) {
        const double c = (double)(2 * x - (n - 1)) * rn;
        const double cs = (double)(2 * imod(x - d, n) - (n - 1)) * rn;
        acc += power ? ipow(c, e) : ipow(cs, ab) * ipow(c, a);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
        if (power) pw[axis * (2 * dmax + 1) + e] = s;
        else if (axis == 0) sig0[(ab * ne + a) * g.D0 + d + 2 * g.w0] = s;
        else sig1[(ab * ne + a) * g.D1 + d + 2 * g.w1] = s;
    }
}

// Pedestals: image means from the (0, 0) entries of the poly tables.
// The pedestal is the image mean rounded to 8 significant bits: subtracting
// it from an FP32 pixel of at least its magnitude is then exact, so removing
// it adds no rounding of its own to FP32 images (the identities above hold
// for any constant).
__device__ __forceinline__ double short_pedestal(double c) {
    if (c == 0.0 || !isfinite(c)) return 0.0;
    int e;
    (void)frexp(c, &e);   // |c| = f 2^e, 0.5 <= f < 1
    return ldexp(rint(ldexp(c, 8 - e)), e - 8);
}

__global__ void pedestal_kernel(Geom g, const double* __restrict__ piR, int ntbR, int K0R, int K1R,
                                const double* __restrict__ piS, int ntbS, int K0S, int K1S,
                                double* __restrict__ ped) {
    (void)ntbR;
    (void)ntbS;
    piR = zoff(piR, g.zs);
    piS = zoff(piS, g.zs);
    ped = zoff(ped, g.zs);
    const double n = (double)g.n0 * (double)g.n1;
    ped[0] = short_pedestal(piR[(size_t)K0R * (2 * K1R + 1) + K1R] / n);
    ped[1] = short_pedestal(piS[(size_t)K0S * (2 * K1S + 1) + K1S] / n);
}

// Assemble the FP64 tables used by the gather:
//  mode 0 (build): Omega, Theta += pedestal corrections; Lambda, E, C written.
//  mode 1 (refinement): Theta (of the difference image) += correction; E.
__global__ void __launch_bounds__(256) lagfix_kernel(Geom g, int mode, const double* __restrict__ ped,
                                                      const double* __restrict__ piR,
                                                      const double* __restrict__ piS,
                                                      const double* __restrict__ sig0,
                                                      const double* __restrict__ sig1,
                                                      const double* __restrict__ pw, int dmax,
                                                      double* __restrict__ omega,
                                                      double* __restrict__ theta,
                                                      double* __restrict__ lam,
                                                      double* __restrict__ cmat,
                                                      double* __restrict__ evec) {
    ped = zoff(ped, g.zs);
    piR = zoff(piR, g.zs);
    piS = zoff(piS, g.zs);
    sig0 = zoff(sig0, g.zs);
    sig1 = zoff(sig1, g.zs);
    pw = zoff(pw, g.zs);
    omega = zoff(omega, g.zs);
    theta = zoff(theta, g.zs);
    lam = zoff(lam, g.zs);
    cmat = zoff(cmat, g.zs);
    evec = zoff(evec, g.zs);
    const double cR = ped[0], cS = mode == 0 ? ped[1] : 0.0;
    const int ntb = (dmax + 1) * (dmax + 2) / 2;
    const int ne = g.dk + 1;
    // Pi^R layout [P][ntb][4w0+1][4w1+1]; Pi^S (and Pi^D) layout [ntb][2w0+1][2w1+1]
    auto piR_at = [&](int ta, int tb, int d0, int d1) {
        return piR[(((size_t)ta * ntb + tb) * g.D0 + d0 + 2 * g.w0) * g.D1 + d1 + 2 * g.w1];
    };
    auto piS_at = [&](int tb, int d0, int d1) {
        return piS[((size_t)tb * g.L0 + d0 + g.w0) * g.L1 + d1 + g.w1];
    };
    auto tsum = [&](int i, int j) {   // sum_x T^(i,j)
        return pw[i] * pw[(2 * dmax + 1) + j];
    };
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    const int nth = gridDim.x * blockDim.x;
    // Theta (both modes)
    for (int idx = tid; idx < g.P * g.L0 * g.L1; idx += nth) {
        const int kb = idx / (g.L0 * g.L1);
        const int d0 = (idx / g.L1) % g.L0 - g.w0, d1 = idx % g.L1 - g.w1;
        int ib, jb;
        term_ij(g.dk, kb, ib, jb);
        const int tbk = term_index(dmax, ib, jb);
        double v = cR * piS_at(tbk, -d0, -d1);
        if (mode == 0) v += cS * piR_at(kb, 0, 0, 0) - cR * cS * tsum(ib, jb);
        theta[idx] += v;
    }
    for (int m = tid; m < g.Q; m += nth) {
        int p, q;
        term_ij(g.db, m, p, q);
        evec[m] = piS_at(term_index(dmax, p, q), 0, 0);
    }
    if (mode != 0) return;
    for (int idx = tid; idx < g.npair * g.D0 * g.D1; idx += nth) {
        const int pr = idx / (g.D0 * g.D1);
        const int d0 = (idx / g.D1) % g.D0 - 2 * g.w0, d1 = idx % g.D1 - 2 * g.w1;
        int kb = 0, c = pr;
        while (c >= g.P - kb) { c -= g.P - kb; ++kb; }
        const int k = kb + c;
        int ib, jb, i, j;
        term_ij(g.dk, kb, ib, jb);
        term_ij(g.dk, k, i, j);
        const double Cd = sig0[(ib * ne + i) * g.D0 + d0 + 2 * g.w0] *
                          sig1[(jb * ne + j) * g.D1 + d1 + 2 * g.w1];
        const double v = cR * (piR_at(kb, term_index(dmax, i, j), d0, d1) +
                               piR_at(k, term_index(dmax, ib, jb), -d0, -d1)) -
                         cR * cR * Cd;
        omega[idx] += v;
    }
    for (int idx = tid; idx < g.P * g.Q * g.L0 * g.L1; idx += nth) {
        const int kb = idx / (g.Q * g.L0 * g.L1);
        const int m = (idx / (g.L0 * g.L1)) % g.Q;
        const int d0 = (idx / g.L1) % g.L0 - g.w0, d1 = idx % g.L1 - g.w1;
        int p, q;
        term_ij(g.db, m, p, q);
        lam[idx] = piR_at(kb, term_index(dmax, p, q), d0, d1);
    }
    for (int idx = tid; idx < g.Q * g.Q; idx += nth) {
        int pb, qb, p, q;
        term_ij(g.db, idx / g.Q, pb, qb);
        term_ij(g.db, idx % g.Q, p, q);
        cmat[idx] = pw[pb + p] * pw[(2 * dmax + 1) + qb + q];
    }
}

template <typename Tin>
hipError_t launch_polyrow(const Geom& g, IoRef<const Tin> img, int da, int dbb, int K1,
                          double* vrow, hipStream_t st) {
    if (K1 < 0 || K1 > kPolyRowMaxLag || K1 >= g.n1) return hipErrorInvalidValue;
    if (da < 0 || dbb < 0 || dbb > kMaxDegree || da + dbb + 1 > kMaxMom) return hipErrorInvalidValue;
    const dim3 grid((g.n0 + 3) / 4, 1, g.nb), block(256);
    switch (da + dbb + 1) {
#define SFFT_POLYROW(NE)                                                                        \
    case NE:                                                                                    \
        hipLaunchKernelGGL((polyrow_kernel<Tin, NE>), grid, block, 0, st, g, img, da, dbb, K1, vrow); \
        break;
        SFFT_POLYROW(1)
        SFFT_POLYROW(2)
        SFFT_POLYROW(3)
        SFFT_POLYROW(4)
        SFFT_POLYROW(5)
        SFFT_POLYROW(6)
        SFFT_POLYROW(7)
        SFFT_POLYROW(8)
        SFFT_POLYROW(9)
#undef SFFT_POLYROW
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_polycorr(const Geom& g, const double* vrow, int da, int dbb, int K0, int K1,
                           double* part, double* pi, hipStream_t st) {
    const int nta = (da + 1) * (da + 2) / 2, ntb = (dbb + 1) * (dbb + 2) / 2;
    const int nitem = (da + 1) * (dbb + 1) * (2 * K1 + 1);
    const int ne = da + dbb + 1;
    const int nchunk = (g.n0 + kPolyRowChunk - 1) / kPolyRowChunk;
    // part holds nchunk * ne * nitem partial moments, then ne * nitem sums
    double* mom = part + (size_t)nchunk * ne * nitem;
    hipLaunchKernelGGL(polymom_kernel, dim3(nchunk, 1, g.nb), dim3(256), 0, st, g, vrow, nitem, ne,
                       part);
    const int nval = ne * nitem;
    hipLaunchKernelGGL(momsum_kernel, dim3((nval + 3) / 4, 1, g.nb), dim3(256), 0, st, nchunk, nval,
                       part, mom, g.zs);
    const int nout = nta * ntb * (2 * K0 + 1) * (2 * K1 + 1);
    hipLaunchKernelGGL(polycorr_kernel, dim3((nout + 255) / 256, 1, g.nb), dim3(256), 0, st, g, vrow, mom, da,
                       dbb, K0, K1, pi);
    return hipGetLastError();
}

hipError_t launch_polysum(const Geom& g, int dmax, double* sig0, double* sig1, double* pw,
                          hipStream_t st) {
    const int ne = g.dk + 1;
    const int nb = ne * ne * (g.D0 + g.D1) + 2 * (2 * dmax + 1);
    hipLaunchKernelGGL(polysum_kernel, dim3(nb, 1, g.nb), dim3(256), 0, st, g, dmax, sig0, sig1, pw);
    return hipGetLastError();
}

hipError_t launch_pedestal(const Geom& g, const double* piR, int dmax, const double* piS,
                           double* ped, hipStream_t st) {
    const int ntb = (dmax + 1) * (dmax + 2) / 2;
    hipLaunchKernelGGL(pedestal_kernel, dim3(1, 1, g.nb), dim3(1), 0, st, g, piR, ntb, 2 * g.w0, 2 * g.w1,
                       piS, ntb, g.w0, g.w1, ped);
    return hipGetLastError();
}

hipError_t launch_lagfix(const Geom& g, int mode, const double* ped, const double* piR,
                         const double* piS, const double* sig0, const double* sig1,
                         const double* pw, int dmax, double* omega, double* theta, double* lam,
                         double* cmat, double* evec, hipStream_t st) {
    hipLaunchKernelGGL(lagfix_kernel, dim3(64, 1, g.nb), dim3(256), 0, st, g, mode, ped, piR, piS, sig0, sig1,
                       pw, dmax, omega, theta, lam, cmat, evec);
    return hipGetLastError();
}

template hipError_t launch_polyrow<float>(const Geom&, IoRef<const float>, int, int, int, double*,
                                          hipStream_t);
template hipError_t launch_polyrow<double>(const Geom&, IoRef<const double>, int, int, int,
                                           double*, hipStream_t);

}  // namespace sfft
