/*
 * sfft.h -- C ABI of the SFFT image-subtraction library for AMD MI355X (gfx950).
 *
 * The library fits, for a reference image R and a science image S of
 * N0 x N1 pixels, a spatially varying convolution kernel and a polynomial
 * differential background so that R (x) K + B approximates S, then forms the
 * difference image (Hu et al. 2022, "Image Subtraction in Fourier Space",
 * Sec. 2.2):
 *
 *   D(x) = S(x) - sum_{ij ab} a_ijab (R^ij o K_ab)(x) - sum_pq b_pq T^pq(x)   (Eq. 12)
 *
 * with the delta-function basis K_00 = delta, K_ab = delta(. - (a,b)) - delta
 * (Eq. 3-4), kernel variation a_ijab x^i y^j with i + j <= DK (Eq. 5-6),
 * background b_pq x^p y^q with p + q <= DB (Eq. 2), weights applied at the
 * source pixel (Eq. 11, App. A) and circular convolution o (Eq. 12). The
 * least-squares coefficients solve the normal equations of Eq. 18, whose
 * elements are built from correlation-lag tables (App. B, Eq. B5-B16)
 * computed from FFTs of the weighted images, spectral products and pruned
 * inverse FFTs.
 *
 * Conventions (shared by every entry point):
 *  - Images are C row-major arrays of n0 x n1 elements; x (the paper's first
 *    index) is axis 0, y is axis 1.
 *  - Polynomial coordinates are centred and normalised:
 *    c(x) = (2x - (N-1)) / (N-1) in [-1, 1]. This spans the same model as the
 *    raw pixel indices of Eq. 2 and 6 (so D is the same) with a far better
 *    conditioned normal matrix; coefficients refer to these coordinates.
 *  - Kernel offsets a in [-w0, w0], b in [-w1, w1]; K_ab shifts the image by
 *    +(a, b): (R o K_ab)(x) = R(x - (a,b)) - R(x) for (a,b) != 0 (Eq. 14).
 *  - Unknown order: kernel term k over (i, j) with i ascending then j
 *    ascending; inside k the offset (a, b) row-major over the L0 x L1 grid,
 *    skipping (k > 0, a = b = 0) when const_phot_ratio is set; then the
 *    background terms (p, q) in the same order. Coefficients are the
 *    pixel-unit a-ring of Eq. 13 (a = N0 N1 a-ring).
 *  - Supported sizes: even n0, n1 >= 16; lengths 2^a 3^b that are multiples
 *    of 16 up to 8192 are transformed directly, other lengths up to 4096
 *    (e.g. the 2046 x 4094 DECam CCDs of Sec. 5) by Bluestein's chirp-z
 *    transform of a power-of-two length (every result the same DFT);
 *    4 w + 1 <= n; 0 <= DK, DB <= 4; w0, w1 <= 16. SFFT_MIXED takes FP32
 *    images, DK <= 3 and sides of at least 48 pixels (SFFT_E_UNSUPPORTED
 *    otherwise): FP64 images would be rounded to FP32 before its transforms,
 *    a perturbation its refinement step cannot correct, and at DK = 4 or on
 *    narrower strips its coefficients stay 0.7-4e-6 from the FP64 optimum;
 *    those run in SFFT_FP64.
 *
 * Memory and streams: every image, matrix and vector argument is a device
 * pointer owned by the caller (for instance the storage of a PyTorch
 * tensor). The context owns its plans, device workspaces and twiddle tables.
 * Calls are stream-ordered on the HIP stream passed as `stream` (NULL = the
 * null stream) and return without waiting for the GPU; errors found on the
 * host are returned at once. Direct calls that share one context must be
 * ordered on one stream by the caller (they share the context's workspace).
 * The submit/poll engine has its own per-request workspaces and streams.
 *
 * Errors detected on the device (a normal matrix that is not positive
 * definite, non-finite input) are recorded in the context and returned by
 * sfft_sync(); the affected coefficients are set to NaN.
 */
#ifndef SFFT_H
#define SFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfft_ctx sfft_ctx;

/* Status codes. */
enum {
    SFFT_OK = 0,
    SFFT_PENDING = 1,          /* sfft_poll: request not finished yet */
    SFFT_E_INVAL = -1,         /* invalid argument or parameter set */
    SFFT_E_NOMEM = -2,         /* workspace does not fit the HBM budget, or device memory ran out */
    SFFT_E_NOT_SPD = -3,       /* normal matrix not positive definite */
    SFFT_E_NONFINITE = -4,     /* NaN or Inf in the inputs / normal matrix */
    SFFT_E_UNSUPPORTED = -5,   /* odd or too large a size, parameters out of range */
    SFFT_E_HIP = -6,           /* HIP runtime error */
    SFFT_E_NOTFOUND = -7       /* unknown request ticket */
};

/* Arithmetic of the hot path. */
enum {
    SFFT_FP64 = 0,   /* every stage in FP64 */
    SFFT_MIXED = 1   /* FFTs and spectral products in FP32 with FP32 accumulation;
                        lag tables, normal-matrix accumulation, Cholesky solve and
                        one iterative-refinement step in FP64 */
};

/* Element type of the image arrays (inputs and the difference image). */
enum { SFFT_F32 = 0, SFFT_F64 = 1 };

/* Problem parameters (Table A1: -KerPolyOrder = dk, -BGPolyOrder = db,
 * -ConstPhotRatio = const_phot_ratio; the kernel half widths w0, w1 are
 * chosen by the caller, e.g. -KerHWRatio times the seeing FWHM). */
typedef struct {
    int32_t n0, n1;            /* image shape (rows, columns) */
    int32_t w0, w1;            /* kernel half widths: L = 2w + 1 */
    int32_t dk;                /* kernel polynomial degree (Eq. 6) */
    int32_t db;                /* background polynomial degree (Eq. 2) */
    int32_t const_phot_ratio;  /* 1: constant kernel sum across the field */
    int32_t precision;         /* SFFT_FP64 or SFFT_MIXED */
    int32_t dtype;             /* SFFT_F32 or SFFT_F64 */
} sfft_params;

/* Create a context on HIP device `device`. hbm_budget_bytes caps the device
 * memory the context may allocate for workspaces (0 = no cap). Returns
 * SFFT_OK and *out, or an error. */
int sfft_create(sfft_ctx** out, int device, size_t hbm_budget_bytes);

/* Destroy a context: waits for its work, frees every workspace. */
void sfft_destroy(sfft_ctx* ctx);

/* Number of unknowns N_u = P L0 L1 - [const_phot] (P - 1) + Q with
 * P = (DK+1)(DK+2)/2, Q = (DB+1)(DB+2)/2; negative on invalid parameters. */
int64_t sfft_num_unknowns(const sfft_params* p);

/* Validate a parameter set: SFFT_OK, SFFT_E_INVAL or SFFT_E_UNSUPPORTED. */
int sfft_check_params(const sfft_params* p);

/* Device bytes one workspace for `p` occupies (negative on invalid p). */
int64_t sfft_workspace_bytes(const sfft_params* p);

/* Normal equations of the fit pair (the masked images of Sec. 3):
 * G (N_u x N_u, row-major, FP64, exactly symmetric) and h (N_u, FP64) in
 * pixel units, G_uv = sum_x Phi_u Phi_v and h_u = sum_x Phi_u S_fit
 * (Eq. 18-24 through App. B). r_fit, s_fit: n0*n1 elements of `dtype`. */
int sfft_build_system(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                      double* G, double* h, void* stream);

/* Solution of Eq. 18: solve G coef = h (Jacobi-scaled FP64 Cholesky; the
 * paper names no solver). When precision is SFFT_MIXED and r_fit, s_fit are
 * given, one iterative-refinement step follows: the gradient
 * Phi^T (S_fit - Phi coef) of the current difference image (Eq. 16-17) is
 * recomputed from the images and the correction is solved with the same
 * factor. coef: N_u doubles, kernel coefficients then background.
 * G, h: as returned by sfft_build_system (G is read, not modified).
 * With stream == NULL the call is synchronous: it waits for the device and
 * returns SFFT_E_NOT_SPD (a non-positive pivot) or SFFT_E_NONFINITE (a
 * non-finite entry of G) itself, clearing them from the context; on any
 * other stream it returns at once and those errors come from sfft_sync.
 * On either error coef is NaN. */
int sfft_solve(sfft_ctx* ctx, const sfft_params* p, const double* G, const double* h,
               const void* r_fit, const void* s_fit, double* coef, void* stream);

/* Difference image of the apply pair (the unmasked images, Sec. 3):
 * d = s - sum_k (c0^i c1^j r) o kappa_k - B with the stamps kappa_k of
 * `coef` (Eq. 12-13). r, s, d: n0*n1 elements of `dtype`. */
int sfft_subtract(sfft_ctx* ctx, const sfft_params* p, const void* r, const void* s,
                  const double* coef, void* d, void* stream);

/* Whole hot path in one call: build on (r_fit, s_fit), solve (with the
 * refinement step in SFFT_MIXED), subtract on (r, s). Row and column
 * transforms of the fit pair are reused inside the call. coef may be NULL
 * (the context keeps its own copy); G and h are internal. */
int sfft_run(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
             const void* r, const void* s, double* coef, void* d, void* stream);

/* The whole hot path of sfft_run without allocating device memory, for
 * callers that cannot call hipMalloc (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation). Same arguments, results
 * and apply-pair rule as sfft_run; coef may be NULL.
 * Every buffer beyond the caller's inputs and outputs (the workspace of the
 * geometry and the twiddle tables) is carved from one static device array
 * of 128 MiB per GPU, held from the library's load until the process ends;
 * a parameter set whose workspace does not fit returns SFFT_E_NOMEM, and one
 * with a Bluestein length (see the supported sizes) SFFT_E_UNSUPPORTED,
 * before anything is enqueued (e.g. 1024 x 1024 with DK = DB = 2 fits in both
 * precisions, 2048 x 2048 does not). Calls neither hipMalloc, hipFree nor
 * any allocating library routine.
 * Every call on one GPU shares that array, which keeps the last call's
 * contents: calls that overlap on one GPU -- from any context, thread or
 * stream -- race and give undefined results; order them on one stream.
 * With stream == NULL the call waits for the device and returns its status
 * (SFFT_E_NOT_SPD, SFFT_E_NONFINITE); on other streams device-side errors
 * leave the coefficients NaN and are not reported by sfft_sync. */
int sfft_run_noalloc(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                     const void* r, const void* s, double* coef, void* d, void* stream);

/* Noise decorrelation of a difference image (App. C, Eq. C21-C24).
 * The difference of co-adds of m_sci science images (white noise sigma_sci[j],
 * matched by the stamps g_sci[j]) and n_ref reference images (sigma_ref[i],
 * stamps h_ref[i]) convolved with the fitted kernel K,
 *   D = sum_j S_j (x) G_j - [sum_i R_i (x) H_i] (x) K               (Eq. C21),
 * has correlated noise; out = d (x) Q with the real, even kernel
 *   Q^(p) = sqrt(den(0) / den(p)),
 *   den(p) = sum_j sigma_sci[j]^2 |G^_j(p)|^2
 *            + |K^(p)|^2 sum_i sigma_ref[i]^2 |H^_i(p)|^2           (Eq. C24)
 * (unit kernel sum: flux is kept), circular on the n0 x n1 grid, which
 * whitens the noise (Eq. C22-C23). K is the kernel field of `coef` (the
 * solution of a fit with parameters p, N_u doubles) at the normalised
 * position (u0, u1) in [-1, 1]^2 -- its spatial variation is ignored, as in
 * App. C. Stamps: (2 w0 + 1) x (2 w1 + 1) doubles each, row-major with the
 * offset (a, b) at [a + w0][b + w1], placed circularly on the grid;
 * g_sci == NULL (h_ref == NULL) means unit stamps (single images, G = H = delta).
 * 1 <= m_sci, n_ref <= 8. coef, sigma_*, g_sci, h_ref: device arrays of
 * doubles. d, out: n0*n1 elements of p->dtype (out may equal d). The
 * transforms run in the compute type of p->precision (FP32 in SFFT_MIXED,
 * Q^ evaluated in it too; FP64 in SFFT_FP64). Stream-ordered; the first call
 * for a parameter set allocates its stamp buffers (< 40 MB). */
int sfft_decorrelate(sfft_ctx* ctx, const sfft_params* p, const double* coef, double u0, double u1,
                     int m_sci, const double* sigma_sci, const double* g_sci, int n_ref,
                     const double* sigma_ref, const double* h_ref, const void* d, void* out,
                     void* stream);

/* Crowded-flavour preprocessing of the fit pair (Sec. 3.1): the pixels
 * affected by saturated sources are masked and replaced by the neighbouring
 * background, giving the masked pair to fit on (sfft_run's r_fit, s_fit)
 * while the unmasked images stay the apply pair. The paper fixes no details;
 * this library's reading:
 *  - saturated: not (r < u_r and s < u_s), in the images' precision (a
 *    non-finite pixel is saturated); a pixel is masked in both images;
 *  - affected: within the kernel footprint of a saturated pixel, i.e. a
 *    saturated pixel at x + (a, b) for some |a| <= g0, |b| <= g1, offsets
 *    circular as in the convolution of Eq. 12 (g0, g1 = w0, w1 is natural);
 *  - background: per tile of t0 x t1 pixels (the last tiles ragged), the
 *    lower median (element (m - 1) / 2 of the m unmasked values in
 *    ascending order); a tile with no unmasked pixel takes the lower median
 *    of the other tiles' backgrounds, 0 if every pixel is masked;
 *  - r_out, s_out: masked pixels := their tile's background, others copied.
 * r, s, r_out, s_out: n0*n1 elements of dtype (SFFT_F32 / SFFT_F64); the
 * outputs may be the inputs. mask_out: n0*n1 bytes (1 = masked) or NULL.
 * 0 <= g0 < n0, 0 <= g1 < n1; t0 t1 <= 4096 and at most 16384 tiles
 * (SFFT_E_UNSUPPORTED otherwise). Exact: only comparisons and selections.
 * Stream-ordered; the context keeps a scratch of 2 n0 n1 bytes (grown on
 * demand, after waiting for the device). */
int sfft_crowded_mask(sfft_ctx* ctx, int n0, int n1, int dtype, const void* r, const void* s,
                      double u_r, double u_s, int g0, int g1, int t0, int t1, void* r_out,
                      void* s_out, unsigned char* mask_out, void* stream);

/* Wait for `stream` and report device-side errors recorded since the last
 * sfft_sync on this context (SFFT_E_NOT_SPD, SFFT_E_NONFINITE) or SFFT_OK. */
int sfft_sync(sfft_ctx* ctx, void* stream);

/* Lag tables of the fit pair in pixel units, FP64 (diagnostics):
 * omega [P(P+1)/2][4w0+1][4w1+1] for kernel-term pairs kb <= k (Eq. B6),
 * theta [P][2w0+1][2w1+1] (Eq. B14), lambda [P][Q][2w0+1][2w1+1] (Eq. B8),
 * cmat [Q][Q] (Eq. B11), evec [Q] (Eq. B15). Any pointer may be NULL. */
int sfft_lag_tables(sfft_ctx* ctx, const sfft_params* p, const void* r_fit, const void* s_fit,
                    double* omega, double* theta, double* lambda, double* cmat, double* evec,
                    void* stream);

/* Batched complex line transform of the library's FFT engine (diagnostics):
 * `lines` lines of n complex values (interleaved re, im of `dtype`),
 * contiguous; sign -1 forward (e^-), +1 unnormalised inverse. Any n >= 2
 * whose transform length fits 8192 (Bluestein lines for lengths other than
 * multiples of 16 of the form 2^a 3^b). */
int sfft_fft_lines(sfft_ctx* ctx, int n, int lines, int sign, int dtype, const void* in, void* out,
                   void* stream);

/* ---- stage timers (tracing) ------------------------------------------ */

/* Enable (1) or disable (0) per-stage timing of direct calls: each stage of
 * the hot path (row transform, column transform, lag products, lag rows,
 * background blocks, gather, Cholesky, triangular solves, refinement,
 * stencil, row inverse) records HIP events on its stream. Waits for the
 * device and clears previous records. */
int sfft_profile(sfft_ctx* ctx, int enable);

/* Waits for the device and aggregates the recorded stages in first-seen
 * order: names[32*i] (NUL-terminated), total_ms[i] summed over calls,
 * counts[i] calls. Returns the number of distinct stages (may exceed
 * max_stages; only max_stages are written) or a negative error. */
int sfft_profile_read(sfft_ctx* ctx, int max_stages, char* names, double* total_ms, int* counts);

/* Test of the triangular solves' bounded waits (diagnostics). The solves
 * run as a dataflow of 64-row blocks across workgroups, each block waiting
 * -- with a bound -- for the blocks it depends on. With enable = 1, direct
 * calls on this context make every such wait wait for a result that is never
 * published, with a short bound: each wait gives up, every workgroup still
 * runs to its end, the coefficients come out NaN and the next sfft_sync (or
 * a synchronous sfft_solve) returns SFFT_E_HIP. enable = 0 restores normal
 * solves. Plans already created keep the setting they were last used with
 * until their next direct call. */
int sfft_debug_solve_stall(sfft_ctx* ctx, int enable);

/* ---- serving engine: continuous batching of independent pairs ---------- */

/* One request: the fit pair, the apply pair, the outputs, and the caller's
 * HIP stream. All device pointers stay owned by the caller and must stay
 * valid (not freed, not reused) until sfft_poll or sfft_wait has returned
 * the request's final status. coef (N_u doubles) may be NULL.
 * Ordering: the request runs on an engine stream of its own, after the work
 * enqueued on `stream` (NULL = the null stream) before sfft_submit was
 * called -- the work that wrote the inputs or initialised the outputs.
 * Nothing on `stream` waits for the request: read coef and d only after
 * its final status has been returned. */
typedef struct {
    sfft_params p;
    const void* r_fit;
    const void* s_fit;
    const void* r;
    const void* s;
    double* coef;
    void* d;
    void* stream;
} sfft_request;

/* n requests (1 <= n <= 16) of one variant -- identical params, and the
 * apply pair equal to the fit pair in all of them or in none -- as one
 * batch: every stage of sfft_run is one launch for all of them (the pair
 * selected by blockIdx.z), on the context's workspace of that geometry
 * (grown to hold n pairs, after waiting for the device, if it holds fewer).
 * Each pair's result equals sfft_run on it, bit for bit. The requests'
 * own stream fields are ignored: the batch is ordered on `stream`; device
 * errors of any pair are reported by sfft_sync. Stage timers (sfft_profile)
 * time the batch's launches. */
int sfft_run_batch(sfft_ctx* ctx, const sfft_request* reqs, int n, void* stream);

/* Configure the engine: `slots` concurrent batches (each on its own HIP
 * stream with its own workspace), each of up to `max_batch` requests
 * (<= 16) of one variant -- the same parameters and image type, and the
 * apply pair equal to the fit pair or not in all of them -- run as one launch
 * per stage of the hot path (continuous batching: the head of the queue
 * takes the later queued requests of its variant with it). Admission is
 * against the context's HBM budget. Called once before the first submit;
 * 0 slots = 4, max_batch 0 = 4. Slots overlap on the device only if their
 * streams sit on distinct hardware queues: HIP gives a process
 * GPU_MAX_HW_QUEUES of them (4 unless set in the environment before HIP
 * initialises), shared round robin by all streams, so a process serving
 * `slots` batches wants at least slots + 1. */
int sfft_engine_config(sfft_ctx* ctx, int slots, int max_batch);

/* Queue a request. Returns SFFT_OK and a ticket; SFFT_E_NOMEM if the
 * request can never fit the budget; SFFT_E_INVAL/UNSUPPORTED on bad params.
 * Requests are admitted in arrival order as slots and memory free up and
 * run concurrently on the device. */
int sfft_submit(sfft_ctx* ctx, const sfft_request* req, uint64_t* ticket);

/* SFFT_PENDING while the request is queued or running, then its final
 * status (SFFT_OK or an error); SFFT_E_NOTFOUND for an unknown ticket.
 * A finished ticket is forgotten after its status has been returned once. */
int sfft_poll(sfft_ctx* ctx, uint64_t ticket);

/* Block until the request finishes; returns its final status. */
int sfft_wait(sfft_ctx* ctx, uint64_t ticket);

/* Human-readable text of a status code (static string). */
const char* sfft_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* SFFT_H */
