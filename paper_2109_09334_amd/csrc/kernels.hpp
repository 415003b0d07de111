// Host-side launchers of the gfx950 kernels. Every launcher enqueues on the
// given stream and returns the hipError_t of the launch.
#pragma once
#include "common.hpp"

namespace sfft {

// Up to kMaxSrc real rows can be fed to one row transform: row source s is
// c1(y)^pow[s] * img[s] (img is R or S of the pair, or an intermediate).
constexpr int kMaxSrc = 10;
struct RowSources {
    int n;                    // number of real sources (output arrays)
    int pow[kMaxSrc];         // exponent of the y-coordinate weight
    int img[kMaxSrc];         // 0 -> first image pointer, 1 -> second
    int out[kMaxSrc];         // output array index in Z
    int ped[kMaxSrc];         // index into the pedestal vector subtracted on load, -1: none
    int rowpair;              // 1: one source (n = 1), rows 2r and 2r+1 packed in line r
};

// Column-transform jobs: input array a of Z produces spectra for x-weight
// exponents i = 0 .. nw[a]-1, written to spectrum index first[a] + i ... as
// given by spec[a][i].
constexpr int kMaxArr = 8;
constexpr int kMaxW = 8;
struct ColJobs {
    int narr;
    int arr[kMaxArr];             // Z array index
    int nw[kMaxArr];              // number of weights
    int spec[kMaxArr][kMaxW];     // output spectrum index for weight i
};

template <typename T, typename Tin>
hipError_t launch_rowfwd(const Geom& g, const LinePlan& lp, const RowSources& src,
                         IoRef<const Tin> img0, IoRef<const Tin> img1, const double* ped, cx<T>* Z,
                         const cx<T>* twt, hipStream_t st);
template <typename T>
hipError_t launch_colfwd(const Geom& g, const LinePlan& lp, const ColJobs& jobs, const cx<T>* Z,
                         cx<T>* X, const cx<T>* twt, hipStream_t st);
template <typename T, typename Tout>
hipError_t launch_rowinv(const Geom& g, const LinePlan& lp, const cx<T>* Dt, IoRef<Tout> d,
                         const double* sky, const cx<T>* twt, hipStream_t st);
template <typename T>
hipError_t launch_fft_lines(const LinePlan& lp, int nlines, int sign, const cx<T>* in, cx<T>* out,
                            const cx<T>* twt, hipStream_t st);

// Products conj(X[kb]) X[k] for products p in [p0, p1): pairs kb <= k of the
// kernel spectra (p < npair) then (kb, S-slot) with the S spectrum at
// index sslot. Pruned inverse along axis 0 kept for |d0| <= lag range.
template <typename T>
// tw: full twiddle table W_N0^t; twt: pass tables of the line plan.
hipError_t launch_lagcol(const Geom& g, const LinePlan& lp, int p0, int p1, int sslot,
                         const cx<T>* X, cx<T>* Cl, const cx<T>* tw, const cx<T>* twt,
                         const double* twp, hipStream_t st);
template <typename T>
hipError_t launch_lagrow(const Geom& g, int p0, int p1, const cx<T>* Cl, const double* twp,
                         double* omega, double* theta, hipStream_t st);

// FP64 polynomial-correlation tables and pedestal corrections (k_background).
// polyrow: row moments for axis-1 shifts |d1| <= K1 (K1 <= kPolyRowMaxLag, < N1).
constexpr int kPolyRowMaxLag = 32;
template <typename Tin>
hipError_t launch_polyrow(const Geom& g, IoRef<const Tin> img, int da, int dbb, int K1,
                          double* vrow, hipStream_t st);
// part: scratch of polycorr_part_len(g, da, dbb, K1) doubles.
hipError_t launch_polycorr(const Geom& g, const double* vrow, int da, int dbb, int K0, int K1,
                           double* part, double* pi, hipStream_t st);
constexpr int kPolyRowChunk = 16;   // rows per partial-moment chunk
inline size_t polycorr_part_len(const Geom& g, int da, int dbb, int K1) {
    const size_t nitem = (size_t)(da + 1) * (dbb + 1) * (2 * K1 + 1);
    const size_t ne = da + dbb + 1;
    return ((size_t)(g.n0 + kPolyRowChunk - 1) / kPolyRowChunk + 1) * ne * nitem;
}
hipError_t launch_polysum(const Geom& g, int dmax, double* sig0, double* sig1, double* pw,
                          hipStream_t st);
hipError_t launch_pedestal(const Geom& g, const double* piR, int dmax, const double* piS,
                           double* ped, hipStream_t st);
hipError_t launch_lagfix(const Geom& g, int mode, const double* ped, const double* piR,
                         const double* piS, const double* sig0, const double* sig1,
                         const double* pw, int dmax, double* omega, double* theta, double* lam,
                         double* cmat, double* evec, hipStream_t st);
hipError_t launch_gather(const Geom& g, const double* om, const double* th, const double* la,
                         const double* cm, const double* ev, double* G, double* h, int rhs_only,
                         hipStream_t st);

// Cholesky of the Jacobi-scaled normal matrix and triangular solves.
// (g: the batch -- nb pairs zs bytes apart -- of the launches below.)
hipError_t launch_jacobi(const Geom& g, int n, const double* G, const double* h, double* L,
                         double* dsc, double* rhs, int* flag, hipStream_t st);
// dfac: scratch of ceil(n/64) * 64 * 64 doubles for the panels' diagonal
// factors; dinv: ceil(n/64) * 2 * 64 * 64 doubles, the inverses of the
// diagonal blocks and their transposes (read by launch_chol_solve). L ends
// with the factor in its lower and its transpose in its upper triangle.
hipError_t launch_cholesky(const Geom& g, int n, double* L, double* dfac, double* dinv, int* flag,
                           hipStream_t st);
// coef (+)= solution of G c = rhs (rhs is read only). tsv: scratch of 4 n
// doubles, the block results of two consecutive solves. flag gains
// kFlagStall if a block of the solve waited past its bound (a broken
// dependency, never expected). gen: this solve's generation within the
// request (1, 2, ...); launch_clear_flag at the request's start prepares
// generation 1, and each solve the next one.
// stall_test: no block publishes its result and every block-to-block wait
// has a short bound (tests the give-up path from the host).
hipError_t launch_chol_solve(const Geom& g, int n, const double* L, const double* dinv,
                             const double* dsc,
                             const double* rhs, double* coef, int accumulate, int* flag,
                             double* tsv, int gen, int stall_test, hipStream_t st);
// A request's start: status flag cleared, the first solve's results emptied
// (n = g.nu).
hipError_t launch_clear_flag(const Geom& g, int* flag, double* tsv, hipStream_t st);
// The caller buffers of the pairs of a batch: p[z] = r_fit, s_fit, r, s,
// coef, d of pair z (slots kIo*).
constexpr int kMaxBatch = 16;
constexpr int kIoUsed = 6;
struct IoBatch {
    const void* p[kMaxBatch][kIoUsed];
    int n;
};
// The I/O table of pair z (at io + z zs) := b.p[z], z < b.n.
hipError_t launch_set_io(void** io, long long zs, const IoBatch& b, hipStream_t st);
// dst[0..n) = src[0..n) (nothing when dst resolves to null).
hipError_t launch_copy_f64(const Geom& g, IoRef<double> dst, const double* src, int n,
                           hipStream_t st);

// Subtraction.
hipError_t launch_stamps(const Geom& g, const double* coef, double* kap, hipStream_t st);
template <typename T>
hipError_t launch_stamp_spectra(const Geom& g, const double* kap, const double* twp, cx<T>* Kt,
                                hipStream_t st);
// Dt = Z_S - sum_k (R^k o kappa_k) in row-spectral form (no background).
template <typename T>
hipError_t launch_stencil(const Geom& g, const cx<T>* Z, int zs_index, const cx<T>* Kt, cx<T>* Dt,
                          hipStream_t st);
// sky[max(DK,DB) + 1 + 2 w0][n1]: smooth FP64 part of D (background and,
// with ped, the pedestal terms c_R (1 o K) - c_S); ped may be null.
// kap1: scratch of (max(DK,DB) + 1 + 2 w0) * P * L1 doubles.
hipError_t launch_sky(const Geom& g, const double* kap, const double* bcoef, const double* ped,
                      double* kap1, double* sky, hipStream_t st);

// Crowded-flavour preprocessing (Sec. 3.1): ro, so = the fit pair with the
// pixels within (g0, g1) of a saturated pixel replaced by their t0 x t1
// tile's lower-median background; mask_out (may be null) = the mask. sat,
// tmp: n0 n1 bytes of scratch; bg: 2 ceil(n0/t0) ceil(n1/t1) values,
// empty: as many bytes. t0 t1 <= kMaskTileMax, tiles <= kMaskTilesMax.
constexpr int kMaskTileMax = 4096;
constexpr int kMaskTilesMax = 16384;
template <typename Tin>
hipError_t launch_crowded_mask(int n0, int n1, const Tin* r, const Tin* s, double ur, double us,
                               int g0, int g1, int t0, int t1, unsigned char* sat,
                               unsigned char* tmp, Tin* bg, unsigned char* empty, Tin* ro, Tin* so,
                               unsigned char* mask_out, hipStream_t st);

// Noise decorrelation (App. C). Up to kMaxCoadd science and reference
// images per co-add.
constexpr int kMaxCoadd = 8;
// st[1 + M + N][L0][L1]: the kernel at (u0, u1) from the stamps kap, then
// the G_j (gst, or unit stamps when null) and H_i (hst, or unit stamps);
// wts[0] = den(0), wts[s] = sigma^2 of stamp s.
hipError_t launch_decorr_stamps(const Geom& g, const double* kap, double u0, double u1, int M,
                                const double* sig_s, const double* gst, int N, const double* sig_r,
                                const double* hst, double* st, double* wts, hipStream_t st_);
// Z ([N0][hp], a row-transformed image) := column transform, times
// Q^(l, m) / N0 from the stamps' row DFTs kr ([1 + M + N][L0][hp]), inverse
// column transform; tw: W_N0^t, twt: pass tables.
template <typename T>
hipError_t launch_colconv(const Geom& g, const LinePlan& lp, cx<T>* Z, const cx<T>* kr,
                          const double* wts, int M, int N, const cx<T>* tw, const cx<T>* twt,
                          hipStream_t st);

}  // namespace sfft
