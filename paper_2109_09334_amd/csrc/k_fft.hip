// Forward / inverse line-transform passes of the SFFT hot path.
//
// Row pass (axis 1, contiguous): the y-coordinate weights of Eq. 6 and Eq. 2
// vary along the transformed axis, so they are applied on load; two real
// rows are packed as one complex line and separated after the transform
// into half spectra (m = 0 .. N1/2).
// Column pass (axis 0): the x-coordinate weights are per-row scalars of the
// row spectra, applied on load, so DK+2 row transforms feed all (DK+1)(DK+2)/2
// weighted spectra of R plus the spectrum of S (Eq. 13, App. B).
#include "fft_engine.hpp"
#include "kernels.hpp"

namespace sfft {

template <typename T>
__device__ __forceinline__ cx<T>* lds_base() {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    return reinterpret_cast<cx<T>*>(smem_raw);
}

template <typename T, typename Tin, typename PL>
__global__ void __launch_bounds__(512) rowfwd_kernel(Geom g, LinePlan lp, RowSources src,
                                                      IoRef<const Tin> img0r,
                                                      IoRef<const Tin> img1r,
                                                      const double* __restrict__ ped,
                                                      cx<T>* __restrict__ Z,
                                                      const cx<T>* __restrict__ twt) {
    cx<T>* lds = lds_base<T>();
    const Tin* __restrict__ img0 = img0r.get(g.zs);
    const Tin* __restrict__ img1 = img1r.get(g.zs);
    ped = zoff(ped, g.zs);
    Z = zoff(Z, g.zs);
    const int line = threadIdx.x / lp.tl, lt0 = threadIdx.x - line * lp.tl;
    // the line packs two sources of one image row, or (rowpair) one source
    // on the image rows xa = 2 r and xb = 2 r + 1
    const int row = blockIdx.x * lp.lpw + line;
    const int xa = src.rowpair ? 2 * row : row, xb = src.rowpair ? 2 * row + 1 : row;
    const bool act = xb < g.n0;
    const int n1 = g.n1;
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    const int npk = (src.n + 1) / 2;
#pragma unroll 1
    for (int pk = 0; pk < npk; ++pk) {
        const int ia = 2 * pk, ib = src.rowpair ? 0 : 2 * pk + 1;
        const bool hasb = src.rowpair || ib < src.n;
        // the thread index through an opaque zero: addresses are formed per
        // packed pair instead of held in registers across the loop
        const int lt = lt0 + opaque_zero();
        // the pair's rows loaded, then the weights applied (a Bluestein
        // line's padding, t >= n1, loads a valid pixel and is zeroed after);
        // two weights of one image row, or a pair without a second source,
        // load the row once (uniform over the launch)
        const bool one_row = !src.rowpair && (!hasb || src.img[ia] == src.img[ib]);
        const Tin* pa = (src.img[ia] ? img1 : img0) + (size_t)xa * n1;
        const Tin* pb = (hasb && src.img[ib] ? img1 : img0) + (size_t)xb * n1;
        Tin la[kElemsPerThread], lb[kElemsPerThread];
        if (act) {
#pragma unroll
            for (int e = 0; e < kElemsPerThread; ++e) la[e] = pa[pad_index<PL>(lt + e * lp.tl, n1)];
            if (one_row) {
#pragma unroll
                for (int e = 0; e < kElemsPerThread; ++e) lb[e] = la[e];
            } else {
#pragma unroll
                for (int e = 0; e < kElemsPerThread; ++e) lb[e] = pb[pad_index<PL>(lt + e * lp.tl, n1)];
            }
        }
        cx<T> v[kElemsPerThread];
        if (act) {
            const int ea = src.pow[ia], eb = hasb ? src.pow[ib] : 0;
            const double qa = src.ped[ia] >= 0 ? ped[src.ped[ia]] : 0.0;
            const double qb = hasb && src.ped[ib] >= 0 ? ped[src.ped[ib]] : 0.0;
#pragma unroll
            for (int e = 0; e < kElemsPerThread; ++e) {
                const T c = coord<T>(lt + e * lp.tl, n1);
                const T va = ipow_upto<kMaxDegree>(c, ea) * T((double)la[e] - qa);
                const T vb = hasb ? ipow_upto<kMaxDegree>(c, eb) * T((double)lb[e] - qb) : T(0);
                v[e] = in_line<PL>(lt + e * lp.tl, n1) ? mk(va, vb) : mk(T(0), T(0));
            }
        } else {
#pragma unroll
            for (int e = 0; e < kElemsPerThread; ++e) v[e] = mk(T(0), T(0));
        }
        line_dft<-1, T, PL>(v, buf, lp, lt, twt);
        // separate the two real rows: needs X(m) and X(N1 - m) together
        __syncthreads();
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) buf[lpad(lt + e * lp.tl)] = v[e];
        __syncthreads();
        if (act) {
            cx<T>* za = Z + ((size_t)src.out[ia] * g.n0 + xa) * g.hp;
            cx<T>* zb = Z + ((size_t)(hasb ? src.out[ib] : 0) * g.n0 + xb) * g.hp;
            auto half = [&](int m, cx<T>& ra, cx<T>& rb) {
                const cx<T> x = buf[lpad(m)], y = buf[lpad(m == 0 ? 0 : n1 - m)];
                ra = mk((x.re + y.re) * T(0.5), (x.im - y.im) * T(0.5));
                rb = mk((x.im + y.im) * T(0.5), (y.re - x.re) * T(0.5));
            };
            if constexpr (sizeof(T) == 4) {
                // bins m, m + 1 (m even) with one 16-byte store per row; the
                // last pair may write bin h into the row padding (h odd)
#pragma unroll 2
                for (int m = 2 * lt; m < g.h; m += 2 * lp.tl) {
                    cx<T> a0, b0, a1, b1;
                    half(m, a0, b0);
                    half(m + 1, a1, b1);
                    *reinterpret_cast<float4*>(za + m) = make_float4(a0.re, a0.im, a1.re, a1.im);
                    if (hasb) *reinterpret_cast<float4*>(zb + m) = make_float4(b0.re, b0.im, b1.re, b1.im);
                }
            } else {
#pragma unroll 2
                for (int m = lt; m < g.h; m += lp.tl) {
                    cx<T> ra, rb;
                    half(m, ra, rb);
                    za[m] = ra;
                    if (hasb) zb[m] = rb;
                }
            }
        }
        __syncthreads();
    }
}

// Adjacent columns per thread of the column pass: FP32 lines of up to 4096
// points read the two columns m, m + 1 (m even) of a row as one 16-byte
// load, which halves the L1 -> L2 requests of the row-strided column reads.
// FP64, longer and Bluestein lines hold one (two would spill).
template <typename T, typename PL>
struct ColfwdCols {
    static constexpr int value = 1;
};
template <int... R>
struct ColfwdCols<float, RadixSeq<R...>> {
    static constexpr int value = SeqProd<R...>::value <= 4096 ? 2 : 1;
};

template <typename T, typename PL>
__global__ void __launch_bounds__(512) colfwd_kernel(Geom g, LinePlan lp, ColJobs jobs,
                                                      const cx<T>* __restrict__ Z,
                                                      cx<T>* __restrict__ X,
                                                      const cx<T>* __restrict__ twt) {
    constexpr int NC = ColfwdCols<T, PL>::value;
    cx<T>* lds = lds_base<T>();
    Z = zoff(Z, g.zs);
    X = zoff(X, g.zs);
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    // Block -> (column block, job): workgroups are dealt to the 8 XCDs round
    // robin, so groups of 16 adjacent column blocks are kept on one XCD, where
    // their strided row reads share L2 lines.
    const int ncb = (g.h + NC * lp.lpw - 1) / (NC * lp.lpw);
    const int per_xcd = (ncb + 127) / 128 * 16;   // column blocks per XCD per job
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int job = slot / per_xcd, r = slot - job * per_xcd;
    const int cb = 16 * (8 * (r >> 4) + xcd) + (r & 15);
    const int m = (cb * lp.lpw + line) * NC;   // the thread's first column
    const bool act = m < g.h;
    const int n0 = g.n0;
    const int a = jobs.arr[job];
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    // FP32 holds the columns across the weights (z = c0^i Z_a); FP64 reads
    // its column again per weight (from L2 after the first) to stay clear of
    // spills
    constexpr bool kHold = sizeof(T) == 4;
    const cx<T>* zc = Z + (size_t)a * n0 * g.hp + m;
    cx<T> z[NC][kHold ? kElemsPerThread : 1];
    if constexpr (kHold) {
        if (act) {
#pragma unroll
            for (int e = 0; e < kElemsPerThread; ++e) {
                const size_t o = (size_t)pad_index<PL>(lt + e * lp.tl, n0) * g.hp;
                if constexpr (NC == 2) {
                    // columns m, m + 1 < hp (m and hp even: 16-byte aligned)
                    const float4 q = *reinterpret_cast<const float4*>(zc + o);
                    z[0][e] = mk(q.x, q.y);
                    z[1][e] = mk(q.z, q.w);
                } else {
                    z[0][e] = zc[o];
                }
            }
        }
    }
    const int nw = jobs.nw[job];
    T c0[kElemsPerThread];
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e) c0[e] = coord<T>(lt + e * lp.tl, n0);
#pragma unroll 1
    for (int i = 0; i < nw; ++i) {
        // the thread index through an opaque zero: addresses are formed per
        // weight instead of held in registers across the loop
        const int li = lt + opaque_zero();
        if constexpr (kHold) {
            if (i > 0) {
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int e = 0; e < kElemsPerThread; ++e) z[c][e] = cscale(z[c][e], c0[e]);
            }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bool on = act && m + c < g.h;   // every thread takes part in the transform
            cx<T> v[kElemsPerThread];
            if constexpr (kHold) {
#pragma unroll
                for (int e = 0; e < kElemsPerThread; ++e)
                    v[e] = on && in_line<PL>(lt + e * lp.tl, n0) ? z[c][e] : mk(T(0), T(0));
            } else {
#pragma unroll
                for (int e = 0; e < kElemsPerThread; ++e)
                    v[e] = on && in_line<PL>(li + e * lp.tl, n0)
                               ? cscale(zc[(size_t)pad_index<PL>(li + e * lp.tl, n0) * g.hp + c],
                                        ipow(c0[e], i))
                               : mk(T(0), T(0));
            }
            line_dft<-1, T, PL>(v, buf, lp, li, twt);
            if (on) {
                cx<T>* xo = X + ((size_t)jobs.spec[job][i] * g.h + m + c) * n0;
#pragma unroll
                for (int e = 0; e < kElemsPerThread; ++e)
                    if (in_line<PL>(li + e * lp.tl, n0)) xo[li + e * lp.tl] = v[e];
            }
        }
    }
}

// D(x0, .) = (1/N1) IDFT_row[Dt(x0, .)] - sky(x0, .): two rows per packed
// complex line (Hermitian extension of each half spectrum). sky is the FP64
// table of sky_kernel: sum_r c0(x0)^r Y_r(x1) on rows w0 <= x0 < N0 - w0,
// tabulated rows on the 2 w0 edge rows; nullptr: no smooth term.
template <typename T, typename Tout, typename PL>
__global__ void __launch_bounds__(512) rowinv_kernel(Geom g, LinePlan lp,
                                                      const cx<T>* __restrict__ Dt,
                                                      IoRef<Tout> dr,
                                                      const double* __restrict__ sky,
                                                      const cx<T>* __restrict__ twt) {
    Tout* __restrict__ d = dr.get(g.zs);
    Dt = zoff(Dt, g.zs);
    sky = zoff(sky, g.zs);
    cx<T>* lds = lds_base<T>();
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    const int pr = blockIdx.x * lp.lpw + line;
    const int xa = 2 * pr, xb = 2 * pr + 1;
    const bool act = xb < g.n0;
    const int n1 = g.n1;
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    cx<T> v[kElemsPerThread];
    if (act) {
        const cx<T>* A = Dt + (size_t)xa * g.hp;
        const cx<T>* B = Dt + (size_t)xb * g.hp;
        // bins past the half spectrum are the conjugates of their mirrors:
        // every load is issued unconditionally from the folded index
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) {
            const int m = lt + e * lp.tl;   // >= n1: a Bluestein line's padding
            const int mf = m < g.h ? m : (in_line<PL>(m, n1) ? n1 - m : 0);
            cx<T> a = A[mf], b = B[mf];
            if (m >= g.h) { a.im = -a.im; b.im = -b.im; }
            if (m == 0 || 2 * m == n1) { a.im = T(0); b.im = T(0); }
            v[e] = in_line<PL>(m, n1) ? mk(a.re - b.im, a.im + b.re) : mk(T(0), T(0));
        }
    } else {
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) v[e] = mk(T(0), T(0));
    }
    line_dft<1, T, PL>(v, buf, lp, lt, twt);
    // FP32 lines and images of a direct plan (N1 = 16 TL): the inverse goes
    // through LDS so that each thread writes consecutive pixels
    constexpr bool kQuadOut = sizeof(T) == 4 && sizeof(Tout) == 4 && !IsChirp<PL>::value;
    if constexpr (kQuadOut) {
        __syncthreads();   // the transform's last reads of buf
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e) buf[lpad(lt + e * lp.tl)] = v[e];
        __syncthreads();
    }
    if (act) {
        const double inv = 1.0 / (double)n1;
        const int n0 = g.n0, w0 = g.w0, R = max(g.dk, g.db);
        const double ca = coord<double>(xa, n0), cb = coord<double>(xb, n0);
        // edge rows read their own table row; interior rows the c0 powers
        // without a table (sky == nullptr) D is the plain row inverse
        const int nsky = sky ? R + 1 : 0;
        const double* ra = sky && (xa < w0 || xa >= n0 - w0)
                               ? sky + (size_t)(R + 1 + (xa < w0 ? xa : xa - n0 + 2 * w0)) * n1
                               : nullptr;
        const double* rb = sky && (xb < w0 || xb >= n0 - w0)
                               ? sky + (size_t)(R + 1 + (xb < w0 ? xb : xb - n0 + 2 * w0)) * n1
                               : nullptr;
        // four elements at a time, the table rows of each power loaded
        // together (one batch of loads in flight per power)
        constexpr int kChunk = 4;
        static_assert(kElemsPerThread % kChunk == 0, "chunked sky terms");
        if constexpr (kQuadOut) {
            // thread lt owns the four consecutive pixels x1 = 4 (lt + tl k)
            // .. + 3 of both rows, k < 4 (from the line in LDS): 16-byte
            // table loads and, on a 16-byte aligned image, 16-byte stores
            const bool d16 = (reinterpret_cast<uintptr_t>(d) & 15) == 0;
#pragma unroll
            for (int k = 0; k < kElemsPerThread / kChunk; ++k) {
                const int x1 = kChunk * (lt + k * lp.tl);
                double ba[kChunk], bb[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q) ba[q] = bb[q] = 0.0;
                double pa = 1.0, pb = 1.0;
                for (int r = 0; r < nsky; ++r) {
                    const double2* yr = reinterpret_cast<const double2*>(sky + (size_t)r * n1 + x1);
                    const double2 y01 = yr[0], y23 = yr[1];
                    const double y[kChunk] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
                    for (int q = 0; q < kChunk; ++q) {
                        ba[q] += pa * y[q];
                        bb[q] += pb * y[q];
                    }
                    pa *= ca;
                    pb *= cb;
                }
                if (ra) {
                    const double2* e = reinterpret_cast<const double2*>(ra + x1);
                    const double2 e01 = e[0], e23 = e[1];
                    ba[0] = e01.x, ba[1] = e01.y, ba[2] = e23.x, ba[3] = e23.y;
                }
                if (rb) {
                    const double2* e = reinterpret_cast<const double2*>(rb + x1);
                    const double2 e01 = e[0], e23 = e[1];
                    bb[0] = e01.x, bb[1] = e01.y, bb[2] = e23.x, bb[3] = e23.y;
                }
                float oa[kChunk], ob[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q) {
                    const cx<T> u = buf[lpad(x1 + q)];
                    oa[q] = float((double)u.re * inv - ba[q]);
                    ob[q] = float((double)u.im * inv - bb[q]);
                }
                Tout* pa_ = d + (size_t)xa * n1 + x1;
                Tout* pb_ = d + (size_t)xb * n1 + x1;
                if (d16) {
                    *reinterpret_cast<float4*>(pa_) = make_float4(oa[0], oa[1], oa[2], oa[3]);
                    *reinterpret_cast<float4*>(pb_) = make_float4(ob[0], ob[1], ob[2], ob[3]);
                } else {
#pragma unroll
                    for (int q = 0; q < kChunk; ++q) {
                        pa_[q] = oa[q];
                        pb_[q] = ob[q];
                    }
                }
            }
        } else
#pragma unroll
        for (int e0 = 0; e0 < kElemsPerThread; e0 += kChunk) {
            double ba[kChunk], bb[kChunk];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) ba[q] = bb[q] = 0.0;
            double pa = 1.0, pb = 1.0;
            for (int r = 0; r < nsky; ++r) {
                double y[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q)
                    y[q] = sky[(size_t)r * n1 + pad_index<PL>(lt + (e0 + q) * lp.tl, n1)];
#pragma unroll
                for (int q = 0; q < kChunk; ++q) {
                    ba[q] += pa * y[q];
                    bb[q] += pb * y[q];
                }
                pa *= ca;
                pb *= cb;
            }
            if (ra)
#pragma unroll
                for (int q = 0; q < kChunk; ++q) ba[q] = ra[pad_index<PL>(lt + (e0 + q) * lp.tl, n1)];
            if (rb)
#pragma unroll
                for (int q = 0; q < kChunk; ++q) bb[q] = rb[pad_index<PL>(lt + (e0 + q) * lp.tl, n1)];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int x1 = lt + (e0 + q) * lp.tl;
                if (in_line<PL>(x1, n1)) {
                    d[(size_t)xa * n1 + x1] = Tout((double)v[e0 + q].re * inv - ba[q]);
                    d[(size_t)xb * n1 + x1] = Tout((double)v[e0 + q].im * inv - bb[q]);
                }
            }
        }
    }
}

template <typename T, int S, typename PL>
__global__ void __launch_bounds__(512) fft_lines_kernel(LinePlan lp, int nlines,
                                                         const cx<T>* __restrict__ in,
                                                         cx<T>* __restrict__ out,
                                                         const cx<T>* __restrict__ twt) {
    cx<T>* lds = lds_base<T>();
    const int line = threadIdx.x / lp.tl, lt = threadIdx.x - line * lp.tl;
    const int ln = blockIdx.x * lp.lpw + line;
    const bool act = ln < nlines;
    cx<T>* buf = lds + line * line_lds_elems(lp.n);
    const int nl = lp.nl;   // the lines' points (lp.n: the transform length)
    cx<T> v[kElemsPerThread];
#pragma unroll
    for (int e = 0; e < kElemsPerThread; ++e)
        v[e] = act && in_line<PL>(lt + e * lp.tl, nl) ? in[(size_t)ln * nl + lt + e * lp.tl]
                                                     : mk(T(0), T(0));
    line_dft<S, T, PL>(v, buf, lp, lt, twt);
    if (act)
#pragma unroll
        for (int e = 0; e < kElemsPerThread; ++e)
            if (in_line<PL>(lt + e * lp.tl, nl)) out[(size_t)ln * nl + lt + e * lp.tl] = v[e];
}

// ---------------------------------------------------------------- launchers

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
    if (bytes > 65536)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    return hipSuccess;
}

template <typename T, typename Tin>
hipError_t launch_rowfwd(const Geom& g, const LinePlan& lp, const RowSources& src,
                         IoRef<const Tin> img0, IoRef<const Tin> img1, const double* ped, cx<T>* Z,
                         const cx<T>* twt, hipStream_t st) {
    if (src.n < 1 || src.n > kMaxSrc) return hipErrorInvalidValue;
    if (src.rowpair && (src.n != 1 || g.n0 % 2)) return hipErrorInvalidValue;
    for (int s = 0; s < src.n; ++s)
        if (src.pow[s] < 0 || src.pow[s] > kMaxDegree) return hipErrorInvalidValue;
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    const int nlines = src.rowpair ? g.n0 / 2 : g.n0;
    dim3 grid((nlines + lp.lpw - 1) / lp.lpw, 1, g.nb);
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        auto k = rowfwd_kernel<T, Tin, decltype(pl)>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, src, img0, img1, ped, Z,
                           twt);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_colfwd(const Geom& g, const LinePlan& lp, const ColJobs& jobs, const cx<T>* Z,
                         cx<T>* X, const cx<T>* twt, hipStream_t st) {
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        const int cols = ColfwdCols<T, decltype(pl)>::value * lp.lpw;   // columns per workgroup
        const int ncb = (g.h + cols - 1) / cols;
        dim3 grid((ncb + 127) / 128 * 128 * jobs.narr, 1, g.nb);
        auto k = colfwd_kernel<T, decltype(pl)>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, jobs, Z, X, twt);
        return hipGetLastError();
    });
}

template <typename T, typename Tout>
hipError_t launch_rowinv(const Geom& g, const LinePlan& lp, const cx<T>* Dt, IoRef<Tout> d,
                         const double* sky, const cx<T>* twt, hipStream_t st) {
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    dim3 grid((g.n0 / 2 + lp.lpw - 1) / lp.lpw, 1, g.nb);
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        auto k = rowinv_kernel<T, Tout, decltype(pl)>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, g, lp, Dt, d, sky, twt);
        return hipGetLastError();
    });
}

template <typename T>
hipError_t launch_fft_lines(const LinePlan& lp, int nlines, int sign, const cx<T>* in, cx<T>* out,
                            const cx<T>* twt, hipStream_t st) {
    const size_t lds = (size_t)lp.lpw * line_lds_elems(lp.n) * sizeof(cx<T>);
    dim3 grid((nlines + lp.lpw - 1) / lp.lpw);
    return with_line_plan(lp, [&](auto pl) -> hipError_t {
        auto k = sign < 0 ? fft_lines_kernel<T, -1, decltype(pl)> : fft_lines_kernel<T, 1, decltype(pl)>;
        hipError_t e = set_lds(k, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k, grid, dim3(lp.tl * lp.lpw), lds, st, lp, nlines, in, out, twt);
        return hipGetLastError();
    });
}

#define SFFT_INST_T(T)                                                                            \
    template hipError_t launch_colfwd<T>(const Geom&, const LinePlan&, const ColJobs&,            \
                                         const cx<T>*, cx<T>*, const cx<T>*, hipStream_t);         \
    template hipError_t launch_fft_lines<T>(const LinePlan&, int, int, const cx<T>*, cx<T>*,      \
                                            const cx<T>*, hipStream_t);
SFFT_INST_T(float)
SFFT_INST_T(double)
#define SFFT_INST_TT(T, U)                                                                        \
    template hipError_t launch_rowfwd<T, U>(const Geom&, const LinePlan&, const RowSources&,      \
                                            IoRef<const U>, IoRef<const U>, const double*,        \
                                            cx<T>*, const cx<T>*, hipStream_t);                   \
    template hipError_t launch_rowinv<T, U>(const Geom&, const LinePlan&, const cx<T>*, IoRef<U>, \
                                            const double*, const cx<T>*, hipStream_t);
SFFT_INST_TT(float, float)
SFFT_INST_TT(float, double)
SFFT_INST_TT(double, float)
SFFT_INST_TT(double, double)

}  // namespace sfft
