// Host runtime of the SFFT library: parameter validation, per-geometry plans
// (line plans, twiddle tables, device workspaces), the stream-ordered
// pipeline of the hot path, and the C ABI declared in sfft.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "engine.hpp"
#include "runtime.hpp"

namespace sfft {

// ------------------------------------------------------------ parameters

static int nterms(int d) { return (d + 1) * (d + 2) / 2; }

constexpr int kMaxMixedDegree = 3;   // largest DK of the mixed form
constexpr int kMinMixedSide = 48;    // shortest image side of the mixed form

static bool radix23(int n, int* a2, int* a3) {
    int a = 0, b = 0;
    while (n > 1 && n % 2 == 0) { n /= 2; ++a; }
    while (n > 1 && n % 3 == 0) { n /= 3; ++b; }
    *a2 = a;
    *a3 = b;
    return n == 1;
}

// A line length the radix-16/8/4/2/3 passes transform directly.
static bool direct_length(int n) {
    int a, b;
    return n >= 16 && n % 16 == 0 && radix23(n, &a, &b);
}

// Bluestein transform length of a line of n points: the power of two >= 2n - 1.
static int bluestein_length(int n) {
    int m = 16;
    while (m < 2 * n - 1) m *= 2;
    return m;
}

constexpr int kMaxLine = 8192;   // longest transform of the line engine

int check_params(const sfft_params* p) {
    if (!p) return SFFT_E_INVAL;
    if (p->n0 < 16 || p->n1 < 16 || p->w0 < 0 || p->w1 < 0 || p->dk < 0 || p->db < 0)
        return SFFT_E_INVAL;
    if (p->dk > kMaxDegree || p->db > kMaxDegree || p->w0 > 16 || p->w1 > 16) return SFFT_E_UNSUPPORTED;
    if (2 * p->w0 + 1 > p->n0 || 2 * p->w1 + 1 > p->n1) return SFFT_E_INVAL;
    if (p->precision != SFFT_FP64 && p->precision != SFFT_MIXED) return SFFT_E_INVAL;
    if (p->dtype != SFFT_F32 && p->dtype != SFFT_F64) return SFFT_E_INVAL;
    if (p->const_phot_ratio != 0 && p->const_phot_ratio != 1) return SFFT_E_INVAL;
    // The mixed form transforms FP32 data. FP64 images would be rounded to
    // FP32 before the transforms, a perturbation of the problem that the
    // refinement step cannot see (its difference image comes from the same
    // rounded transforms); DK = 4 leaves the FP32 path's fixed point 2-4e-6
    // from the FP64 optimum, and strips narrower than 48 pixels come close to
    // that (the background block, 0.7-3e-6 on 32-34 pixel strips): these run
    // in the FP64 form.
    if (p->precision == SFFT_MIXED &&
        (p->dtype != SFFT_F32 || p->dk > kMaxMixedDegree || p->n0 < kMinMixedSide ||
         p->n1 < kMinMixedSide))
        return SFFT_E_UNSUPPORTED;
    // lengths 2^a 3^b (multiples of 16) are transformed directly, other even
    // lengths by Bluestein's chirp transform of a power-of-two length
    for (int n : {p->n0, p->n1}) {
        if (n % 2) return SFFT_E_UNSUPPORTED;
        if (direct_length(n) ? n > kMaxLine : bluestein_length(n) > kMaxLine) return SFFT_E_UNSUPPORTED;
    }
    // 4w+1 lag rows must stay distinct modulo N (torus wrap of the lag range)
    if (4 * p->w0 + 1 > p->n0 || 4 * p->w1 + 1 > p->n1) return SFFT_E_UNSUPPORTED;
    return SFFT_OK;
}

int64_t num_unknowns(const sfft_params* p) {
    if (!p || p->w0 < 0 || p->w1 < 0 || p->dk < 0 || p->db < 0) return -1;
    const int64_t P = nterms(p->dk), Q = nterms(p->db);
    const int64_t L = (int64_t)(2 * p->w0 + 1) * (2 * p->w1 + 1);
    return P * L - (p->const_phot_ratio ? (P - 1) : 0) + Q;
}

Geom make_geom(const sfft_params* p) {
    Geom g{};
    g.n0 = p->n0;
    g.n1 = p->n1;
    g.h = p->n1 / 2 + 1;
    const int elt = p->precision == SFFT_MIXED ? 8 : 16;   // bytes per complex
    const int line = 256 / elt;                             // complex per 256 B
    g.hp = (g.h + line - 1) / line * line;
    g.w0 = p->w0;
    g.w1 = p->w1;
    g.dk = p->dk;
    g.db = p->db;
    g.cp = p->const_phot_ratio;
    g.P = nterms(p->dk);
    g.Q = nterms(p->db);
    g.L0 = 2 * p->w0 + 1;
    g.L1 = 2 * p->w1 + 1;
    g.nu = (int)num_unknowns(p);
    g.nk = g.nu - g.Q;
    g.npair = g.P * (g.P + 1) / 2;
    g.nprod = g.npair + g.P;
    g.nr = p->dk + 2;
    g.D0 = 4 * p->w0 + 1;
    g.D1 = 4 * p->w1 + 1;
    g.nb = 1;
    g.zs = 0;
    return g;
}

// Radix order: 16 first (the first pass runs on the registers as loaded),
// then the small radices, then the remaining 16s (a radix-16 last pass ends in
// registers in natural order).
LinePlan make_line_plan(int n) {
    if (!direct_length(n)) {   // Bluestein: the plan of its transform length
        LinePlan lp = make_line_plan(bluestein_length(n));
        lp.nl = n;
        return lp;
    }
    LinePlan lp{};
    lp.n = n;
    lp.nl = n;
    int a, b;
    radix23(n, &a, &b);
    int np = 0;
    lp.radix[np++] = 16;
    a -= 4;
    const int n16 = a / 4, rem = a % 4;
    if (rem) lp.radix[np++] = 1 << rem;
    while (b-- > 0) lp.radix[np++] = 3;
    for (int i = 0; i < n16; ++i) lp.radix[np++] = 16;
    lp.npass = np;
    int off = 0, ns = 1;
    for (int p = 0; p < np; ++p) {
        lp.twoff[p] = off;
        if (p > 0) off += ns * 16;
        ns *= lp.radix[p];
    }
    lp.tl = n / kElemsPerThread;
    lp.lpw = lp.tl >= 256 ? 1 : 256 / lp.tl;
    return lp;
}

// Entries of the pass twiddle tables of make_line_plan(n).
int pass_table_len(int n) {
    const LinePlan lp = make_line_plan(n);
    int len = 0, ns = 1;
    for (int p = 0; p < lp.npass; ++p) {
        if (p > 0) len += ns * 16;
        ns *= lp.radix[p];
    }
    return len;
}

size_t workspace_bytes(const sfft_params* p) {
    Geom g = make_geom(p);
    Workspace w;
    const bool mixed = p->precision == SFFT_MIXED;
    return carve(w, g, mixed ? 8 : 16, mixed ? 4 : 8, nullptr);
}

template <typename T>
static hipError_t upload(const std::vector<cx<double>>& v, void** dst) {
    std::vector<cx<T>> h(v.size());
    for (size_t i = 0; i < v.size(); ++i) h[i] = {(T)v[i].re, (T)v[i].im};
    hipError_t e = hipMalloc(dst, h.size() * sizeof(cx<T>));
    if (e) return e;
    return hipMemcpy(*dst, h.data(), h.size() * sizeof(cx<T>), hipMemcpyHostToDevice);
}

// In-place forward DFT (e^-) of a power-of-two length, iterative radix 2,
// in long double (the Bluestein tables).
static void fft_ld(std::vector<std::complex<long double>>& a) {
    const size_t m = a.size();
    for (size_t i = 1, j = 0; i < m; ++i) {
        size_t bit = m >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (size_t len = 2; len <= m; len <<= 1) {
        for (size_t k = 0; k < len / 2; ++k) {
            const long double ang = -two_pi * (long double)k / (long double)len;
            const std::complex<long double> w(cosl(ang), sinl(ang));
            for (size_t i = 0; i < m; i += len) {
                const std::complex<long double> u = a[i + k], v = a[i + k + len / 2] * w;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
        }
    }
}

// Twiddles of length n: the full table W_n^t = e^(-2 pi i t / n), the pass
// tables of the line plan (pass p: row k holds W_(ns R)^(r k), r < R, in 16
// entries, ns = product of the earlier radices), and the FP64 cos / sin
// pairs. Angles in long double, rounded once to the compute type.
static hipError_t make_twiddles(int n, bool mixed, Twiddles& t) {
    const long double two_pi = 6.283185307179586476925286766559005768L;
    auto W = [&](long long num, long long den) {
        const long double ang = two_pi * (long double)(num % den) / (long double)den;
        return cx<double>{(double)cosl(ang), (double)-sinl(ang)};
    };
    std::vector<cx<double>> full(n);
    for (int k = 0; k < n; ++k) full[k] = W(k, n);
    const LinePlan lp = make_line_plan(n);
    std::vector<cx<double>> pass(pass_table_len(n) + 16, cx<double>{0.0, 0.0});
    int ns = 1;
    for (int p = 0; p < lp.npass; ++p) {
        const int R = lp.radix[p];
        if (p > 0)
            for (int k = 0; k < ns; ++k)
                for (int r = 0; r < R; ++r) pass[lp.twoff[p] + (size_t)k * 16 + r] = W((long long)r * k, (long long)ns * R);
        ns *= R;
    }
    hipError_t e = mixed ? upload<float>(full, &t.tw) : upload<double>(full, &t.tw);
    if (e) return e;
    e = mixed ? upload<float>(pass, &t.twt) : upload<double>(pass, &t.twt);
    if (e) return e;
    std::vector<double> vp(2 * n);
    for (int k = 0; k < n; ++k) {
        vp[2 * k] = full[k].re;
        vp[2 * k + 1] = -full[k].im;
    }
    e = hipMalloc(&t.twp, 2 * n * sizeof(double));
    if (e) return e;
    e = hipMemcpy(t.twp, vp.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e || lp.nl == lp.n) return e;
    // Bluestein tables: chirp c_t = e^(+i pi t^2 / n) (the exponent reduced
    // mod 2n), b_t = b_(m-t) = c_t, bhat = DFT_m(b) / m by a radix-2 FFT in
    // long double
    const int m = lp.n;
    std::vector<cx<double>> chirp(n);
    std::vector<std::complex<long double>> b(m, {0.0L, 0.0L});
    for (int k = 0; k < n; ++k) {
        const long long q = ((long long)k * k) % (2LL * n);
        const long double ang = two_pi * 0.5L * (long double)q / (long double)n;
        const std::complex<long double> c(cosl(ang), sinl(ang));
        chirp[k] = {(double)c.real(), (double)c.imag()};
        b[k] = c;
        if (k > 0) b[m - k] = c;
    }
    fft_ld(b);
    std::vector<cx<double>> bh(m);
    for (int k = 0; k < m; ++k) bh[k] = {(double)(b[k].real() / m), (double)(b[k].imag() / m)};
    e = upload<double>(chirp, &t.chirp);   // FP64 in both forms
    if (e) return e;
    e = upload<double>(bh, &t.bhat);
    if (e) return e;
    std::vector<cx<double>> wm(m);
    for (int k = 0; k < m; ++k) wm[k] = W(k, m);
    return mixed ? upload<float>(wm, &t.twm) : upload<double>(wm, &t.twm);
}

static void free_twiddles(Twiddles& t) {
    if (t.chirp) (void)hipFree(t.chirp);
    if (t.bhat) (void)hipFree(t.bhat);
    if (t.twm) (void)hipFree(t.twm);
    t.chirp = t.bhat = t.twm = nullptr;
    if (t.tw) (void)hipFree(t.tw);
    if (t.twt) (void)hipFree(t.twt);
    t.twt = nullptr;
    if (t.twp) (void)hipFree(t.twp);
    t.tw = nullptr;
    t.twp = nullptr;
}

}  // namespace sfft

using namespace sfft;

namespace sfft {

// Status of a HIP result: device memory exhausted (e.g. a graph
// instantiated under memory pressure) is SFFT_E_NOMEM, other failures
// SFFT_E_HIP.
static int hip_status(hipError_t e) {
    if (e == hipSuccess) return SFFT_OK;
    return e == hipErrorOutOfMemory ? SFFT_E_NOMEM : SFFT_E_HIP;
}

// Twiddles are shared by every plan of the context with the same length.
static int get_twiddles(sfft_ctx* ctx, int n, bool mixed, Twiddles* out) {
    auto key = std::make_pair(n, mixed ? 1 : 0);
    auto it = ctx->twid.find(key);
    if (it == ctx->twid.end()) {
        Twiddles t;
        hipError_t e = make_twiddles(n, mixed, t);
        if (e != hipSuccess) {
            free_twiddles(t);
            return SFFT_E_HIP;
        }
        it = ctx->twid.emplace(key, t).first;
    }
    *out = it->second;
    return SFFT_OK;
}

// Bytes between the workspaces of consecutive pairs of a batch.
static size_t pair_stride(const sfft_params* p) { return (workspace_bytes(p) + 255) & ~size_t(255); }

// Allocate a plan (with the workspaces of `cap` pairs) against the context
// budget. Caller holds ctx->mu.
int create_plan(sfft_ctx* ctx, const sfft_params* p, std::unique_ptr<Plan>& out, int cap,
                hipStream_t init_stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (cap < 1 || cap > kMaxBatch) return SFFT_E_INVAL;
    auto pl = std::make_unique<Plan>();
    pl->p = *p;
    pl->g = make_geom(p);
    pl->lp0 = make_line_plan(p->n0);
    pl->lp1 = make_line_plan(p->n1);
    pl->device = ctx->device;
    pl->cap = cap;
    const bool mixed = p->precision == SFFT_MIXED;
    pl->g.zs = (long long)pair_stride(p);
    const size_t bytes = (size_t)pl->g.zs * cap;
    if (ctx->budget && ctx->used + bytes > ctx->budget) return SFFT_E_NOMEM;
    rc = get_twiddles(ctx, p->n0, mixed, &pl->t0);
    if (!rc) rc = get_twiddles(ctx, p->n1, mixed, &pl->t1);
    if (rc) return rc;
    pl->lp0.chirp = pl->t0.chirp;
    pl->lp0.bhat = pl->t0.bhat;
    pl->lp0.twm = pl->t0.twm;
    pl->lp1.chirp = pl->t1.chirp;
    pl->lp1.bhat = pl->t1.bhat;
    pl->lp1.twm = pl->t1.twm;
    char* base = nullptr;
    if (hipMalloc(&base, bytes) != hipSuccess) return SFFT_E_NOMEM;
    carve(pl->ws, pl->g, mixed ? 8 : 16, mixed ? 4 : 8, base);
    // Every pair's status flag starts clear: the allocation may hold a freed
    // workspace's bytes, and the flag is read for every plan at a sync. The
    // 1-D polynomial sums depend on the geometry only: formed once here.
    Geom all = pl->g;
    all.nb = cap;
    // (on init_stream, ahead of the plan's first use there; on the null
    // stream, waited for, when none is given)
    if (launch_clear_flag(all, pl->ws.flag, pl->ws.tsv, init_stream) != hipSuccess ||
        launch_polysum(all, poly_degree(all), pl->ws.sig0, pl->ws.sig1, pl->ws.pw, init_stream) !=
            hipSuccess ||
        (!init_stream && hipStreamSynchronize(nullptr) != hipSuccess)) {
        (void)hipFree(base);
        return SFFT_E_HIP;
    }
    pl->ws.base = base;
    pl->ws.bytes = bytes;
    ctx->used += bytes;
    out = std::move(pl);
    return SFFT_OK;
}

void destroy_plan(sfft_ctx* ctx, std::unique_ptr<Plan>& pl) {
    if (!pl) return;
    for (auto& a : pl->graph)
        for (auto& b : a)
            for (auto& gx : b)
                if (gx) (void)hipGraphExecDestroy(gx);
    if (pl->ws.base) (void)hipFree(pl->ws.base);
    ctx->used -= pl->ws.bytes;
    if (pl->dec) (void)hipFree(pl->dec);
    ctx->used -= pl->dec_bytes;
    pl.reset();
}

// The context's plan of p with room for `pairs` pairs (a plan with less is
// replaced, after the device has finished with it).
static int direct_plan(sfft_ctx* ctx, const sfft_params* p, Plan** out, int pairs = 1) {
    int rc = check_params(p);
    if (rc) return rc;
    auto k = key_of(p);
    auto it = ctx->plans.find(k);
    if (it != ctx->plans.end() && it->second->cap < pairs) {
        if (hipDeviceSynchronize() != hipSuccess) return SFFT_E_HIP;
        destroy_plan(ctx, it->second);
        ctx->plans.erase(it);
        it = ctx->plans.end();
    }
    if (it == ctx->plans.end()) {
        std::unique_ptr<Plan> pl;
        int cap = 1;
        while (cap < pairs) cap *= 2;
        rc = create_plan(ctx, p, pl, cap);
        if (rc) return rc;
        it = ctx->plans.emplace(k, std::move(pl)).first;
    }
    it->second->p.dtype = p->dtype;
    it->second->prof = &ctx->prof;
    it->second->stall_test = ctx->stall_test;
    *out = it->second.get();
    return SFFT_OK;
}

// ------------------------------------------------------------ pipeline

template <typename T>
static cx<T>* cxp(void* p) { return reinterpret_cast<cx<T>*>(p); }

static RowSources pair_sources(const Geom& g, bool pedestal) {
    RowSources src{};
    src.n = g.nr;
    for (int j = 0; j <= g.dk; ++j) {
        src.pow[j] = j;
        src.img[j] = 0;
        src.out[j] = j;
        src.ped[j] = pedestal ? 0 : -1;
    }
    src.pow[g.dk + 1] = 0;
    src.img[g.dk + 1] = 1;
    src.out[g.dk + 1] = g.dk + 1;
    src.ped[g.dk + 1] = pedestal ? 1 : -1;
    return src;
}

// Stage 1 of the build, FP64: polynomial-correlation tables of R (|d| <= 2w)
// and S (|d| <= w), 1-D polynomial sums, and the pedestals (image means).
template <typename Tin>
static hipError_t poly_tables(Plan& pl, IoRef<const Tin> r, IoRef<const Tin> s, hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    const int dm = poly_degree(g);
    StageTimer t_(pl.prof, "background", st);
    hipError_t e = launch_polyrow<Tin>(g, r, g.dk, dm, 2 * g.w1, w.vrow, st);
    if (!e) e = launch_polycorr(g, w.vrow, g.dk, dm, 2 * g.w0, 2 * g.w1, w.vpart, w.piR, st);
    if (!e) e = launch_polyrow<Tin>(g, s, 0, dm, g.w1, w.vrow, st);
    if (!e) e = launch_polycorr(g, w.vrow, 0, dm, g.w0, g.w1, w.vpart, w.piS, st);
    if (!e) e = launch_pedestal(g, w.piR, dm, w.piS, w.ped, st);
    return e;
}

// Row and column transforms of the pedestal-free fit pair: Z[0..nr), X[0..P].
template <typename T, typename Tin>
static hipError_t forward_fit(Plan& pl, IoRef<const Tin> r, IoRef<const Tin> s, hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    hipError_t e;
    {
        StageTimer t_(pl.prof, "rowfwd", st);
        e = launch_rowfwd<T, Tin>(g, pl.lp1, pair_sources(g, true), r, s, w.ped, cxp<T>(w.Z),
                                  cxp<T>(pl.t1.twt), st);
    }
    if (e) return e;
    ColJobs jobs{};
    jobs.narr = g.nr;
    for (int a = 0; a <= g.dk; ++a) {
        jobs.arr[a] = a;
        jobs.nw[a] = g.dk - a + 1;
        for (int i = 0; i < jobs.nw[a]; ++i) jobs.spec[a][i] = term_index(g.dk, i, a);
    }
    jobs.arr[g.dk + 1] = g.dk + 1;
    jobs.nw[g.dk + 1] = 1;
    jobs.spec[g.dk + 1][0] = g.P;
    StageTimer t_(pl.prof, "colfwd", st);
    return launch_colfwd<T>(g, pl.lp0, jobs, cxp<T>(w.Z), cxp<T>(w.X), cxp<T>(pl.t0.twt), st);
}

// Pedestal tables, transforms, products and pruned inverses, then the exact
// FP64 pedestal corrections: Omega, Theta, Lambda, C, E of the fit pair.
template <typename T, typename Tin>
static hipError_t lag_tables(Plan& pl, IoRef<const Tin> r, IoRef<const Tin> s, hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    hipError_t e = poly_tables<Tin>(pl, r, s, st);
    if (!e) e = forward_fit<T, Tin>(pl, r, s, st);
    if (!e) {
        StageTimer t_(pl.prof, "lagcol", st);
        e = launch_lagcol<T>(g, pl.lp0, 0, g.nprod, g.P, cxp<T>(w.X), cxp<T>(w.Cl), cxp<T>(pl.t0.tw), cxp<T>(pl.t0.twt), pl.t0.twp, st);
    }
    if (!e) {
        StageTimer t_(pl.prof, "lagrow", st);
        e = launch_lagrow<T>(g, 0, g.nprod, cxp<T>(w.Cl), pl.t1.twp, w.omega, w.theta, st);
    }
    if (!e) {
        StageTimer t_(pl.prof, "lagfix", st);
        e = launch_lagfix(g, 0, w.ped, w.piR, w.piS, w.sig0, w.sig1, w.pw, poly_degree(g), w.omega,
                          w.theta, w.lam, w.cmat, w.evec, st);
    }
    return e;
}

template <typename T, typename Tin>
static hipError_t build(Plan& pl, IoRef<const Tin> r, IoRef<const Tin> s, double* G, double* h,
                        hipStream_t st) {
    hipError_t e = lag_tables<T, Tin>(pl, r, s, st);
    Workspace& w = pl.ws;
    StageTimer t_(pl.prof, "gather", st);
    if (!e) e = launch_gather(pl.g, w.omega, w.theta, w.lam, w.cmat, w.evec, G, h, 0, st);
    return e;
}

// D from the row spectra in Z (slots 0..DK of R, slot zs of S) and the
// coefficients. With `pedestal` the spectra are those of R - c_R and S - c_S
// (pedestals in w.ped) and the pedestal terms re-enter in FP64 through the
// sky table together with the background.
template <typename T, typename Tout>
static hipError_t difference(Plan& pl, int zs, bool pedestal, const double* coef, IoRef<Tout> d,
                             hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    hipError_t e;
    {
        StageTimer t_(pl.prof, "stencil", st);
        e = launch_stamps(g, coef, w.kap, st);
        if (!e) e = launch_sky(g, w.kap, coef + g.nk, pedestal ? w.ped : nullptr, w.kap1, w.sky, st);
        if (!e) e = launch_stamp_spectra<T>(g, w.kap, pl.t1.twp, cxp<T>(w.Kt), st);
        if (!e) e = launch_stencil<T>(g, cxp<T>(w.Z), zs, cxp<T>(w.Kt), cxp<T>(w.Dt), st);
    }
    if (!e) {
        StageTimer t_(pl.prof, "rowinv", st);
        e = launch_rowinv<T, Tout>(g, pl.lp1, cxp<T>(w.Dt), d, w.sky, cxp<T>(pl.t1.twt), st);
    }
    return e;
}

// Factor G (Jacobi-scaled) and solve into coef.
static hipError_t factor_solve(Plan& pl, const double* G, const double* h, double* coef,
                               hipStream_t st) {
    const int n = pl.g.nu;
    Workspace& w = pl.ws;
    hipError_t e;
    {
        StageTimer t_(pl.prof, "cholesky", st);
        e = launch_jacobi(pl.g, n, G, h, w.L, w.dsc, w.rhs, w.flag, st);
        if (!e) e = launch_cholesky(pl.g, n, w.L, w.dfac, w.dinv, w.flag, st);
    }
    if (!e) {
        StageTimer t_(pl.prof, "trsv", st);
        e = launch_chol_solve(pl.g, n, w.L, w.dinv, w.dsc, h, coef, 0, w.flag, w.tsv, 1,
                              pl.stall_test, st);
    }
    return e;
}

// One refinement step: gradient Phi^T (S_fit - Phi coef) of the current
// difference image of the fit pair (Z, X, ped hold the fit pair's
// transforms), correction solved with the existing factor. Every component
// comes from that one difference image: the rounding of its FP32 evaluation
// then enters the gradient as Phi^T e, whose least-squares image G^-1 Phi^T e
// is the fit of e itself (small); taking some components exactly and the
// others from D breaks that consistency, and G^-1 amplifies the mismatch.
template <typename T>
static hipError_t refine(Plan& pl, double* coef, int gen, hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    T* dfit = reinterpret_cast<T*>(w.dfit);
    StageTimer t_(pl.prof, "refine", st);
    Profiler* saved = pl.prof;
    pl.prof = nullptr;   // inner stages count toward "refine"
    struct Restore {
        Plan& p;
        Profiler* s;
        ~Restore() { p.prof = s; }
    } restore_{pl, saved};
    const int dm = poly_degree(g);
    hipError_t e = difference<T, T>(pl, g.dk + 1, true, coef, dfit, st);
    if (!e) e = launch_polyrow<T>(g, dfit, 0, dm, g.w1, w.vrow, st);
    if (!e) e = launch_polycorr(g, w.vrow, 0, dm, g.w0, g.w1, w.vpart, w.piD, st);
    RowSources src{};
    src.n = 1;
    src.pow[0] = 0;
    src.img[0] = 0;
    src.out[0] = g.nr;
    src.ped[0] = -1;
    src.rowpair = 1;   // D's rows two to a line
    if (!e) e = launch_rowfwd<T, T>(g, pl.lp1, src, dfit, dfit, w.ped, cxp<T>(w.Z), cxp<T>(pl.t1.twt), st);
    ColJobs jobs{};
    jobs.narr = 1;
    jobs.arr[0] = g.nr;
    jobs.nw[0] = 1;
    jobs.spec[0][0] = g.P + 1;
    if (!e) e = launch_colfwd<T>(g, pl.lp0, jobs, cxp<T>(w.Z), cxp<T>(w.X), cxp<T>(pl.t0.twt), st);
    if (!e) e = launch_lagcol<T>(g, pl.lp0, g.npair, g.nprod, g.P + 1, cxp<T>(w.X), cxp<T>(w.Cl), cxp<T>(pl.t0.tw), cxp<T>(pl.t0.twt), pl.t0.twp, st);
    if (!e) e = launch_lagrow<T>(g, g.npair, g.nprod, cxp<T>(w.Cl), pl.t1.twp, w.omega, w.thetaD, st);
    if (!e) e = launch_lagfix(g, 1, w.ped, w.piR, w.piD, w.sig0, w.sig1, w.pw, dm, nullptr,
                              w.thetaD, nullptr, nullptr, w.evecD, st);
    if (!e) e = launch_gather(g, w.omega, w.thetaD, w.lam, w.cmat, w.evecD, nullptr, w.rhs, 1, st);
    if (!e) e = launch_chol_solve(g, g.nu, w.L, w.dinv, w.dsc, w.rhs, coef, 1, w.flag, w.tsv,
                                  gen, pl.stall_test, st);
    return e;
}

// Refinement steps of the mixed form (one by default; SFFT_REFINE_STEPS
// overrides it for diagnostics).
static int refine_steps() {
    static const int n = [] {
        const char* s = getenv("SFFT_REFINE_STEPS");
        return s ? atoi(s) : 1;
    }();
    return n;
}

template <typename T, typename Tin>
static int run_build_t(Plan& pl, const void* r, const void* s, double* G, double* h, hipStream_t st) {
    return hip_status(build<T, Tin>(pl, (const Tin*)r, (const Tin*)s, G, h, st));
}

template <typename T, typename Tin>
static int run_solve_t(Plan& pl, const double* G, const double* h, const void* r, const void* s,
                       double* coef, hipStream_t st) {
    hipError_t e = launch_clear_flag(pl.g, pl.ws.flag, pl.ws.tsv, st);
    if (!e) e = factor_solve(pl, G, h, coef, st);
    if (!e && pl.p.precision == SFFT_MIXED && r && s) {
        e = poly_tables<Tin>(pl, (const Tin*)r, (const Tin*)s, st);
        if (!e) e = forward_fit<T, Tin>(pl, (const Tin*)r, (const Tin*)s, st);
        for (int it = 0; !e && it < refine_steps(); ++it) e = refine<T>(pl, coef, 2 + it, st);
    }
    return hip_status(e);
}

template <typename T, typename Tin>
static hipError_t subtract_path(Plan& pl, IoRef<const Tin> r, IoRef<const Tin> s,
                                const double* coef, IoRef<Tin> d, hipStream_t st) {
    const Geom& g = pl.g;
    hipError_t e;
    {
        StageTimer t_(pl.prof, "rowfwd", st);
        e = launch_rowfwd<T, Tin>(g, pl.lp1, pair_sources(g, false), r, s, nullptr,
                                  cxp<T>(pl.ws.Z), cxp<T>(pl.t1.twt), st);
    }
    if (!e) e = difference<T, Tin>(pl, g.dk + 1, false, coef, d, st);
    return e;
}

template <typename T, typename Tin>
static int run_subtract_t(Plan& pl, const void* r, const void* s, const double* coef, void* d,
                          hipStream_t st) {
    return hip_status(subtract_path<T, Tin>(pl, (const Tin*)r, (const Tin*)s, coef, (Tin*)d, st));
}

// The whole path of one request. same_pair: the apply pair is the fit pair,
// whose pedestal-free transforms are reused for D.
template <typename T, typename Tin>
static hipError_t all_path(Plan& pl, IoRef<const Tin> rf, IoRef<const Tin> sf, IoRef<const Tin> r,
                           IoRef<const Tin> s, IoRef<double> coef, IoRef<Tin> d, bool same_pair,
                           hipStream_t st) {
    Workspace& w = pl.ws;
    hipError_t e = launch_clear_flag(pl.g, w.flag, w.tsv, st);
    if (!e) e = build<T, Tin>(pl, rf, sf, w.G, w.h, st);
    if (!e) e = factor_solve(pl, w.G, w.h, w.coef, st);
    for (int it = 0; !e && pl.p.precision == SFFT_MIXED && it < refine_steps(); ++it)
        e = refine<T>(pl, w.coef, 2 + it, st);
    if (!e) e = launch_copy_f64(pl.g, coef, w.coef, pl.g.nu, st);
    if (e) return e;
    if (same_pair) return difference<T, Tin>(pl, pl.g.dk + 1, true, w.coef, d, st);
    return subtract_path<T, Tin>(pl, r, s, w.coef, d, st);
}

template <typename T, typename Tin>
static int run_all_t(Plan& pl, const void* rf, const void* sf, const void* r, const void* s,
                     double* coef, void* d, hipStream_t st) {
    return hip_status(all_path<T, Tin>(pl, (const Tin*)rf, (const Tin*)sf, (const Tin*)r,
                                       (const Tin*)s, coef, (Tin*)d, r == rf && s == sf, st));
}

// all_path of the pl.g.nb pairs of a batch, every caller buffer read from
// the pair's I/O table (launch arguments stay fixed for graph replays).
template <typename T, typename Tin>
static hipError_t table_path(Plan& pl, bool same_pair, hipStream_t st) {
    void* const* io = pl.ws.io;
    return all_path<T, Tin>(
        pl, IoRef<const Tin>(io, kIoRfit), IoRef<const Tin>(io, kIoSfit), IoRef<const Tin>(io, kIoR),
        IoRef<const Tin>(io, kIoS), IoRef<double>(io, kIoCoef), IoRef<Tin>(io, kIoD), same_pair, st);
}

template <typename T, typename Tin>
static int run_table_t(Plan& pl, bool same_pair, hipStream_t st) {
    return hip_status(table_path<T, Tin>(pl, same_pair, st));
}

// Capture of table_path.
template <typename T, typename Tin>
static int capture_all_t(Plan& pl, bool same_pair, hipStream_t st, hipGraphExec_t* out) {
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
    if (e) return hip_status(e);
    const hipError_t ek = table_path<T, Tin>(pl, same_pair, st);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (ek || e) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_status(ek ? ek : e);
    }
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return hip_status(e);
}

// Noise decorrelation of d into out (App. C, Eq. C21-C24): stamps of the
// kernel at (u0, u1) and of the co-add kernels, their row DFTs, the row
// transform of d, the column convolution with Q, the row inverse.
constexpr int kDecStamps = 1 + 2 * kMaxCoadd;

static size_t decorr_carve(const Geom& g, size_t cxb, char* base, double** stp, double** wts,
                           void** kr) {
    Carver c;
    *stp = c.take<double>(base, (size_t)kDecStamps * g.L0 * g.L1);
    *wts = c.take<double>(base, kDecStamps + 1);
    *kr = c.take<char>(base, cxb * (size_t)kDecStamps * g.L0 * g.hp);
    return c.off + 256;
}

template <typename T, typename Tin>
static hipError_t decorr_path(Plan& pl, const double* coef, double u0, double u1, int M,
                              const double* sig_s, const double* gst, int N, const double* sig_r,
                              const double* hst, const Tin* d, Tin* out, hipStream_t st) {
    const Geom& g = pl.g;
    Workspace& w = pl.ws;
    double *stp, *wts;
    void* kr;
    decorr_carve(g, sizeof(cx<T>), pl.dec, &stp, &wts, &kr);
    StageTimer t_(pl.prof, "decorrelate", st);
    hipError_t e = launch_stamps(g, coef, w.kap, st);
    if (!e) e = launch_decorr_stamps(g, w.kap, u0, u1, M, sig_s, gst, N, sig_r, hst, stp, wts, st);
    Geom gs = g;
    gs.P = 1 + M + N;   // stamp rows of the row DFTs
    if (!e) e = launch_stamp_spectra<T>(gs, stp, pl.t1.twp, cxp<T>(kr), st);
    RowSources src{};
    src.n = 1;
    src.pow[0] = 0;
    src.img[0] = 0;
    src.out[0] = 0;
    src.ped[0] = -1;
    src.rowpair = 1;   // the image's rows two to a line
    if (!e) e = launch_rowfwd<T, Tin>(g, pl.lp1, src, d, d, nullptr, cxp<T>(w.Z), cxp<T>(pl.t1.twt), st);
    if (!e) e = launch_colconv<T>(g, pl.lp0, cxp<T>(w.Z), cxp<T>(kr), wts, M, N, cxp<T>(pl.t0.tw),
                                  cxp<T>(pl.t0.twt), st);
    if (!e) e = launch_rowinv<T, Tin>(g, pl.lp1, cxp<T>(w.Z), out, nullptr, cxp<T>(pl.t1.twt), st);
    return e;
}

template <typename T, typename Tin>
static int run_decorr_t(Plan& pl, const double* coef, double u0, double u1, int M,
                        const double* sig_s, const double* gst, int N, const double* sig_r,
                        const double* hst, const void* d, void* out, hipStream_t st) {
    return hip_status(decorr_path<T, Tin>(pl, coef, u0, u1, M, sig_s, gst, N, sig_r, hst,
                                          (const Tin*)d, (Tin*)out, st));
}

// Dispatch on (compute type, image type).
#define SFFT_DISPATCH(pl, FN, ...)                                                        \
    ((pl).p.precision == SFFT_MIXED                                                       \
         ? ((pl).p.dtype == SFFT_F32 ? FN<float, float>(pl, __VA_ARGS__)                  \
                                     : FN<float, double>(pl, __VA_ARGS__))                \
         : ((pl).p.dtype == SFFT_F32 ? FN<double, float>(pl, __VA_ARGS__)                 \
                                     : FN<double, double>(pl, __VA_ARGS__)))

int plan_run(Plan& pl, const void* rf, const void* sf, const void* r, const void* s, double* coef,
             void* d, hipStream_t st) {
    return SFFT_DISPATCH(pl, run_all_t, rf, sf, r, s, coef, d, st);
}

int plan_run_batch(Plan& pl, const IoBatch& io, bool same_pair, bool graphs, hipStream_t st) {
    const int b = io.n;
    if (b < 1 || b > pl.cap) return SFFT_E_INVAL;
    hipError_t e = launch_set_io(pl.ws.io, pl.g.zs, io, st);
    if (e) return SFFT_E_HIP;
    Profiler* saved = pl.prof;
    if (graphs) pl.prof = nullptr;   // no timing events inside a graph
    int rc = SFFT_OK;
    pl.g.nb = b;
    if (!graphs) {
        rc = SFFT_DISPATCH(pl, run_table_t, same_pair, st);
    } else {
        hipGraphExec_t& gx = pl.graph[same_pair ? 0 : 1][pl.p.dtype == SFFT_F64 ? 1 : 0][b - 1];
        if (!gx) {
            rc = SFFT_DISPATCH(pl, capture_all_t, same_pair, st, &gx);
            if (rc) gx = nullptr;
        }
        if (!rc) rc = hip_status(hipGraphLaunch(gx, st));
    }
    pl.g.nb = 1;
    pl.prof = saved;
    return rc;
}

int plan_read_flag(Plan& pl, hipStream_t st, int* flag) {
    if (hipStreamSynchronize(st) != hipSuccess) return SFFT_E_HIP;
    if (hipMemcpy(flag, pl.ws.flag, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return SFFT_E_HIP;
    return SFFT_OK;
}

int read_pair_flag(const Plan& pl, int z, int* flag) {
    const int* f = reinterpret_cast<const int*>(reinterpret_cast<const char*>(pl.ws.flag) +
                                                (size_t)z * (size_t)pl.g.zs);
    return hipMemcpy(flag, f, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess ? SFFT_OK : SFFT_E_HIP;
}

int flag_status(int f) {
    if (f & 4) return SFFT_E_HIP;   // a solve block waited past its bound
    if (f & 2) return SFFT_E_NONFINITE;
    if (f & 1) return SFFT_E_NOT_SPD;
    return SFFT_OK;
}

}  // namespace sfft

// ------------------------------------------------------------ C ABI

extern "C" {

int sfft_create(sfft_ctx** out, int device, size_t hbm_budget_bytes) {
    if (!out) return SFFT_E_INVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return SFFT_E_INVAL;
    auto* c = new (std::nothrow) sfft_ctx();
    if (!c) return SFFT_E_NOMEM;
    c->device = device;
    c->budget = hbm_budget_bytes;
    // the allocation-free entry point's scratch address on this device
    const int rc = noalloc_init(device);
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return SFFT_OK;
}

void sfft_destroy(sfft_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->engine.reset();
    for (auto& kv : ctx->plans) destroy_plan(ctx, kv.second);
    for (auto& kv : ctx->twid) free_twiddles(kv.second);
    if (ctx->mbuf) (void)hipFree(ctx->mbuf);
    delete ctx;
}

int64_t sfft_num_unknowns(const sfft_params* p) { return num_unknowns(p); }

int sfft_check_params(const sfft_params* p) { return check_params(p); }

int64_t sfft_workspace_bytes(const sfft_params* p) {
    int rc = check_params(p);
    if (rc) return rc;
    return (int64_t)workspace_bytes(p);
}

int sfft_build_system(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                      double* G, double* h, void* stream) {
    if (!ctx || !r_fit || !s_fit || !G || !h) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    return SFFT_DISPATCH(*pl, run_build_t, r_fit, s_fit, G, h, (hipStream_t)stream);
}

int sfft_solve(sfft_ctx* ctx, const sfft_params* p, const double* G, const double* h,
               const void* r_fit, const void* s_fit, double* coef, void* stream) {
    if (!ctx || !G || !h || !coef || ((r_fit == nullptr) != (s_fit == nullptr))) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    rc = SFFT_DISPATCH(*pl, run_solve_t, G, h, r_fit, s_fit, coef, (hipStream_t)stream);
    if (rc || stream) return rc;
    // synchronous mode: the device status of this solve
    int f = 0;
    if (plan_read_flag(*pl, nullptr, &f) != SFFT_OK) return SFFT_E_HIP;
    if (f && hipMemset(pl->ws.flag, 0, sizeof(int)) != hipSuccess) return SFFT_E_HIP;
    return flag_status(f);
}

int sfft_subtract(sfft_ctx* ctx, const sfft_params* p, const void* r, const void* s,
                  const double* coef, void* d, void* stream) {
    if (!ctx || !r || !s || !coef || !d) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    return SFFT_DISPATCH(*pl, run_subtract_t, r, s, coef, d, (hipStream_t)stream);
}

int sfft_run(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
             const void* r, const void* s, double* coef, void* d, void* stream) {
    if (!ctx || !r_fit || !s_fit || !r || !s || !d) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    return plan_run(*pl, r_fit, s_fit, r, s, coef, d, (hipStream_t)stream);
}

int sfft_run_noalloc(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                     const void* r, const void* s, double* coef, void* d, void* stream) {
    if (!ctx || !r_fit || !s_fit || !r || !s || !d) return SFFT_E_INVAL;
    (void)hipSetDevice(ctx->device);
    int rc = noalloc_init(ctx->device);
    if (rc) return rc;
    return run_noalloc(ctx->device, p, r_fit, s_fit, r, s, coef, d, (hipStream_t)stream);
}

int sfft_decorrelate(sfft_ctx* ctx, const sfft_params* p, const double* coef, double u0, double u1,
                     int m_sci, const double* sigma_sci, const double* g_sci, int n_ref,
                     const double* sigma_ref, const double* h_ref, const void* d, void* out,
                     void* stream) {
    if (!ctx || !coef || !sigma_sci || !sigma_ref || !d || !out) return SFFT_E_INVAL;
    if (m_sci < 1 || n_ref < 1) return SFFT_E_INVAL;
    if (m_sci > kMaxCoadd || n_ref > kMaxCoadd) return SFFT_E_UNSUPPORTED;
    if (!std::isfinite(u0) || !std::isfinite(u1)) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    if (!pl->dec) {
        double *stp, *wts;
        void* kr;
        const size_t bytes =
            decorr_carve(pl->g, p->precision == SFFT_MIXED ? 8 : 16, nullptr, &stp, &wts, &kr);
        if (ctx->budget && ctx->used + bytes > ctx->budget) return SFFT_E_NOMEM;
        if (hipMalloc(&pl->dec, bytes) != hipSuccess) {
            pl->dec = nullptr;
            return SFFT_E_NOMEM;
        }
        pl->dec_bytes = bytes;
        ctx->used += bytes;
    }
    return SFFT_DISPATCH(*pl, run_decorr_t, coef, u0, u1, m_sci, sigma_sci, g_sci, n_ref, sigma_ref,
                         h_ref, d, out, (hipStream_t)stream);
}

int sfft_crowded_mask(sfft_ctx* ctx, int n0, int n1, int dtype, const void* r, const void* s,
                      double u_r, double u_s, int g0, int g1, int t0, int t1, void* r_out,
                      void* s_out, unsigned char* mask_out, void* stream) {
    if (!ctx || !r || !s || !r_out || !s_out) return SFFT_E_INVAL;
    if (dtype != SFFT_F32 && dtype != SFFT_F64) return SFFT_E_INVAL;
    if (n0 < 1 || n1 < 1 || g0 < 0 || g1 < 0 || g0 >= n0 || g1 >= n1 || t0 < 1 || t1 < 1)
        return SFFT_E_INVAL;
    if ((long long)t0 * t1 > kMaskTileMax) return SFFT_E_UNSUPPORTED;
    const long long ntiles = (long long)((n0 + t0 - 1) / t0) * ((n1 + t1 - 1) / t1);
    if (ntiles > kMaskTilesMax) return SFFT_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    const size_t n = (size_t)n0 * n1;
    Carver c;
    unsigned char* sat = c.take<unsigned char>(nullptr, n);
    unsigned char* tmp = c.take<unsigned char>(nullptr, n);
    double* bg = c.take<double>(nullptr, 2 * (size_t)ntiles);
    unsigned char* empty = c.take<unsigned char>(nullptr, 2 * (size_t)ntiles);
    const size_t need = c.off + 256;
    if (need > ctx->mbuf_bytes) {
        if (ctx->budget && ctx->used - ctx->mbuf_bytes + need > ctx->budget) return SFFT_E_NOMEM;
        if (ctx->mbuf) {
            if (hipDeviceSynchronize() != hipSuccess) return SFFT_E_HIP;   // earlier calls may use it
            (void)hipFree(ctx->mbuf);
            ctx->used -= ctx->mbuf_bytes;
            ctx->mbuf = nullptr;
            ctx->mbuf_bytes = 0;
        }
        if (hipMalloc(&ctx->mbuf, need) != hipSuccess) {
            ctx->mbuf = nullptr;
            return SFFT_E_NOMEM;
        }
        ctx->mbuf_bytes = need;
        ctx->used += need;
    }
    Carver c2;
    sat = c2.take<unsigned char>(ctx->mbuf, n);
    tmp = c2.take<unsigned char>(ctx->mbuf, n);
    bg = c2.take<double>(ctx->mbuf, 2 * (size_t)ntiles);
    empty = c2.take<unsigned char>(ctx->mbuf, 2 * (size_t)ntiles);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (dtype == SFFT_F32)
        e = launch_crowded_mask<float>(n0, n1, (const float*)r, (const float*)s, u_r, u_s, g0, g1, t0,
                                       t1, sat, tmp, reinterpret_cast<float*>(bg), empty,
                                       (float*)r_out, (float*)s_out, mask_out, st);
    else
        e = launch_crowded_mask<double>(n0, n1, (const double*)r, (const double*)s, u_r, u_s, g0, g1,
                                        t0, t1, sat, tmp, bg, empty, (double*)r_out, (double*)s_out,
                                        mask_out, st);
    return hip_status(e);
}

int sfft_sync(sfft_ctx* ctx, void* stream) {
    if (!ctx) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return SFFT_E_HIP;
    int all = 0;
    for (auto& kv : ctx->plans) {
        for (int z = 0; z < kv.second->cap; ++z) {   // every pair of a batch
            int f = 0;
            if (read_pair_flag(*kv.second, z, &f) != SFFT_OK) return SFFT_E_HIP;
            all |= f;
            char* fz = reinterpret_cast<char*>(kv.second->ws.flag) + (size_t)z * kv.second->g.zs;
            if (f) (void)hipMemset(fz, 0, sizeof(int));
        }
    }
    return flag_status(all);
}

int sfft_run_batch(sfft_ctx* ctx, const sfft_request* reqs, int n, void* stream) {
    if (!ctx || !reqs || n < 1) return SFFT_E_INVAL;
    if (n > kMaxBatch) return SFFT_E_UNSUPPORTED;
    const sfft_params& p0 = reqs[0].p;
    const bool same = reqs[0].r == reqs[0].r_fit && reqs[0].s == reqs[0].s_fit;
    IoBatch io{};
    io.n = n;
    for (int z = 0; z < n; ++z) {
        const sfft_request& q = reqs[z];
        if (!q.r_fit || !q.s_fit || !q.r || !q.s || !q.d) return SFFT_E_INVAL;
        if (std::memcmp(&q.p, &p0, sizeof(sfft_params)) != 0) return SFFT_E_INVAL;
        if ((q.r == q.r_fit && q.s == q.s_fit) != same) return SFFT_E_INVAL;
        const void* ptrs[kIoUsed] = {q.r_fit, q.s_fit, q.r, q.s, q.coef, q.d};
        for (int k = 0; k < kIoUsed; ++k) io.p[z][k] = ptrs[k];
    }
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, &p0, &pl, n);
    if (rc) return rc;
    return plan_run_batch(*pl, io, same, false, (hipStream_t)stream);
}

int sfft_lag_tables(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                    double* omega, double* theta, double* lambda, double* cmat, double* evec,
                    void* stream) {
    if (!ctx || !r_fit || !s_fit) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Plan* pl;
    int rc = direct_plan(ctx, p, &pl);
    if (rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](auto tag_t, auto tag_in) -> hipError_t {
        using T = decltype(tag_t);
        using Tin = decltype(tag_in);
        return lag_tables<T, Tin>(*pl, (const Tin*)r_fit, (const Tin*)s_fit, st);
    };
    hipError_t e;
    if (pl->p.precision == SFFT_MIXED)
        e = pl->p.dtype == SFFT_F32 ? run(float{}, float{}) : run(float{}, double{});
    else
        e = pl->p.dtype == SFFT_F32 ? run(double{}, float{}) : run(double{}, double{});
    if (e) return SFFT_E_HIP;
    const Geom& g = pl->g;
    Workspace& w = pl->ws;
    auto cp = [&](double* dst, const double* src, size_t cnt) -> hipError_t {
        return dst ? hipMemcpyAsync(dst, src, cnt * sizeof(double), hipMemcpyDeviceToDevice, st)
                   : hipSuccess;
    };
    e = cp(omega, w.omega, (size_t)g.npair * g.D0 * g.D1);
    if (!e) e = cp(theta, w.theta, (size_t)g.P * g.L0 * g.L1);
    if (!e) e = cp(lambda, w.lam, (size_t)g.P * g.Q * g.L0 * g.L1);
    if (!e) e = cp(cmat, w.cmat, (size_t)g.Q * g.Q);
    if (!e) e = cp(evec, w.evec, (size_t)g.Q);
    return hip_status(e);
}

int sfft_fft_lines(sfft_ctx* ctx, int n, int lines, int sign, int dtype, const void* in, void* out,
                   void* stream) {
    if (!ctx || !in || !out || lines < 0 || (sign != 1 && sign != -1)) return SFFT_E_INVAL;
    if (n < 2 || (direct_length(n) ? n > kMaxLine : bluestein_length(n) > kMaxLine))
        return SFFT_E_UNSUPPORTED;
    if (dtype != SFFT_F32 && dtype != SFFT_F64) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    Twiddles t;
    int rc = get_twiddles(ctx, n, dtype == SFFT_F32, &t);
    if (rc) return rc;
    LinePlan lp = make_line_plan(n);
    lp.chirp = t.chirp;
    lp.bhat = t.bhat;
    lp.twm = t.twm;
    hipError_t e;
    if (dtype == SFFT_F32)
        e = launch_fft_lines<float>(lp, lines, sign, (const cx<float>*)in, (cx<float>*)out,
                                    (const cx<float>*)t.twt, (hipStream_t)stream);
    else
        e = launch_fft_lines<double>(lp, lines, sign, (const cx<double>*)in, (cx<double>*)out,
                                     (const cx<double>*)t.twt, (hipStream_t)stream);
    return hip_status(e);
}

int sfft_profile(sfft_ctx* ctx, int enable) {
    if (!ctx) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& r : ctx->prof.recs) {
        ctx->prof.pool.push_back(r.a);
        ctx->prof.pool.push_back(r.b);
    }
    ctx->prof.recs.clear();
    ctx->prof.on = enable != 0;
    return SFFT_OK;
}

int sfft_profile_read(sfft_ctx* ctx, int max_stages, char* names, double* total_ms, int* counts) {
    if (!ctx || max_stages < 0 || (max_stages && (!names || !total_ms || !counts))) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    (void)hipSetDevice(ctx->device);
    if (hipDeviceSynchronize() != hipSuccess) return SFFT_E_HIP;
    std::vector<std::string> order;
    std::map<std::string, std::pair<double, int>> acc;
    for (auto& r : ctx->prof.recs) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SFFT_E_HIP;
        auto it = acc.find(r.name);
        if (it == acc.end()) {
            order.push_back(r.name);
            acc[r.name] = {ms, 1};
        } else {
            it->second.first += ms;
            it->second.second += 1;
        }
    }
    const int n = (int)order.size();
    for (int i = 0; i < n && i < max_stages; ++i) {
        std::snprintf(names + 32 * i, 32, "%s", order[i].c_str());
        total_ms[i] = acc[order[i]].first;
        counts[i] = acc[order[i]].second;
    }
    return n;
}

int sfft_debug_solve_stall(sfft_ctx* ctx, int enable) {
    if (!ctx) return SFFT_E_INVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->stall_test = enable ? 1 : 0;
    return SFFT_OK;
}

const char* sfft_strerror(int s) {
    switch (s) {
        case SFFT_OK: return "ok";
        case SFFT_PENDING: return "pending";
        case SFFT_E_INVAL: return "invalid argument";
        case SFFT_E_NOMEM: return "workspace exceeds the HBM budget or device memory";
        case SFFT_E_NOT_SPD: return "normal matrix is not positive definite";
        case SFFT_E_NONFINITE: return "non-finite value in the inputs or normal matrix";
        case SFFT_E_UNSUPPORTED: return "unsupported size or parameter";
        case SFFT_E_HIP: return "HIP runtime error";
        case SFFT_E_NOTFOUND: return "unknown request ticket";
        default: return "unknown status";
    }
}

}  // extern "C"
