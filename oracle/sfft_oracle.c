/*
 * sfft_oracle.c -- plain FP64 CPU reference for SFFT image subtraction.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg use it. It shares no code, header or table
 * with the GPU library.
 *
 * What it computes (Hu et al. 2022, "Image Subtraction in Fourier Space"):
 *   D(x) = S(x) - sum_{ij ab} a_ijab (R^ij o K_ab)(x) - sum_pq b_pq T^pq(x)
 * (Eq. 12: circular convolution, weights x^i y^j taken at the source pixel,
 * Eq. 10-11 and App. A), with the delta basis of Eq. 3-4, the polynomial
 * kernel variation of Eq. 5-6 and the polynomial background of Eq. 2.
 * The least-squares optimum of sum_x D(x)^2 -- equal to the Fourier-space
 * objective of Eq. 15 by Parseval -- is found from the normal equations of
 * Eq. 18, whose elements are assembled from correlation-lag tables exactly
 * as App. B (Eq. B5-B16) prescribes, except that every lag table is a plain
 * pixel-space sum instead of a DFT of spectral products (same numbers, by
 * the correlation theorem).
 *
 * Readings of the paper adopted here (the GPU library follows the same ones):
 *  - x is axis 0 (rows) of a C row-major N0 x N1 array, y is axis 1.
 *  - Polynomial coordinates are centred and normalised,
 *    c(x) = (2x - (N-1)) / (N-1) in [-1, 1], instead of raw pixel indices.
 *    The affine change spans the same polynomial space, so D is unchanged,
 *    while the normal matrix stays far better conditioned.
 *  - Kernel offsets a in [-w0, w0], b in [-w1, w1] inclusive (odd L).
 *  - K_ab shifts the image by +(a,b): (R o K_ab)(x) = R(x-a) - R(x) for
 *    (a,b) != 0, matching the DFT W^{l a} of Eq. 14.
 *  - Boundary is circular everywhere (Eq. 12), no padding.
 *  - Coefficients are the pixel-unit a-ring (a = N0 N1 a-ring, Eq. 13); the
 *    App. B normalisation factors all cancel in the solution.
 *  - The solver (unspecified in the paper) is FP64 Cholesky of the
 *    Jacobi-scaled normal matrix; a non-positive pivot is an error.
 *  - ConstPhotRatio drops the unknowns a_ij00 for (i,j) != (0,0).
 *
 * Unknown order: kernel term k runs over (i,j) with i ascending then j
 * ascending (i+j <= DK); inside k the offset (a,b) runs row-major over
 * [-w0,w0] x [-w1,w1]; with ConstPhotRatio the (k>0, a=b=0) entries are
 * skipped. The background terms m over (p,q) in the same order follow.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTSPD (-3)

static long imod(long a, long n) { long r = a % n; return r < 0 ? r + n : r; }

/* Centred, normalised coordinate of pixel index x on an axis of length n. */
double orc_coord(long x, long n) {
    return n > 1 ? (2.0 * (double)x - (double)(n - 1)) / (double)(n - 1) : 0.0;
}

/* Number of monomials x^i y^j with i + j <= deg (Eq. 2 and Eq. 6). */
int orc_nterms(int deg) { return deg < 0 ? 0 : (deg + 1) * (deg + 2) / 2; }

/* Exponents of the t-th monomial (i ascending, then j ascending). */
void orc_term(int deg, int t, int* i, int* j) {
    int c = 0;
    for (int a = 0; a <= deg; ++a)
        for (int b = 0; b <= deg - a; ++b) {
            if (c == t) { *i = a; *j = b; return; }
            ++c;
        }
    *i = *j = -1;
}

long orc_num_unknowns(int w0, int w1, int dk, int db, int const_phot) {
    if (w0 < 0 || w1 < 0 || dk < 0 || db < 0) return -1;
    long P = orc_nterms(dk), Q = orc_nterms(db), L = (long)(2 * w0 + 1) * (2 * w1 + 1);
    return P * L - (const_phot ? (P - 1) : 0) + Q;
}

/* Kernel unknown u -> (k, a, b); returns the number of kernel unknowns. */
static long kernel_unknowns(int w0, int w1, int dk, int cp, int* K, int* A, int* B) {
    int P = orc_nterms(dk);
    long u = 0;
    for (int k = 0; k < P; ++k)
        for (int a = -w0; a <= w0; ++a)
            for (int b = -w1; b <= w1; ++b) {
                if (cp && k > 0 && a == 0 && b == 0) continue;
                if (K) { K[u] = k; A[u] = a; B[u] = b; }
                ++u;
            }
    return u;
}

/* R^k(x) = c0(x0)^i c1(x1)^j R(x)  (Eq. 6 weights, abbreviation before Eq. 10). */
void orc_weighted(const double* img, int n0, int n1, int i, int j, double* out) {
    for (long x0 = 0; x0 < n0; ++x0) {
        double w0 = pow(orc_coord(x0, n0), i);
        for (long x1 = 0; x1 < n1; ++x1)
            out[x0 * n1 + x1] = w0 * pow(orc_coord(x1, n1), j) * img[x0 * n1 + x1];
    }
}

/* T^m(x) = c0(x0)^p c1(x1)^q  (Eq. 2). */
static void background_image(int n0, int n1, int p, int q, double* out) {
    for (long x0 = 0; x0 < n0; ++x0) {
        double a = pow(orc_coord(x0, n0), p);
        for (long x1 = 0; x1 < n1; ++x1)
            out[x0 * n1 + x1] = a * pow(orc_coord(x1, n1), q);
    }
}

/* sum_x A((x - d) mod N) B(x), the sum over x split into rows. */
static double lag_sum(const double* A, const double* B, int n0, int n1, int d0, int d1) {
    double acc = 0.0;
    for (long x0 = 0; x0 < n0; ++x0) {
        const double* a = A + imod(x0 - d0, n0) * n1;
        const double* b = B + x0 * n1;
        double row = 0.0;
        for (long x1 = 0; x1 < n1; ++x1) row += a[imod(x1 - d1, n1)] * b[x1];
        acc += row;
    }
    return acc;
}

static double* weighted_stack(const double* r, int n0, int n1, int dk) {
    int P = orc_nterms(dk);
    long n = (long)n0 * n1;
    double* w = (double*)malloc(sizeof(double) * n * P);
    if (!w) return NULL;
    for (int k = 0; k < P; ++k) {
        int i, j;
        orc_term(dk, k, &i, &j);
        orc_weighted(r, n0, n1, i, j, w + k * n);
    }
    return w;
}

/* Omega_{kb k}(d) = sum_x R^kb(x - d) R^k(x) for kb <= k, d in [-2w, 2w]^2
 * (the lag table of Eq. B6, in pixel units). Layout [pair][d0][d1]. */
int orc_omega(const double* r, int n0, int n1, int dk, int w0, int w1, double* out) {
    int P = orc_nterms(dk);
    long n = (long)n0 * n1;
    int D0 = 4 * w0 + 1, D1 = 4 * w1 + 1;
    double* W = weighted_stack(r, n0, n1, dk);
    if (!W) return ORC_ENOMEM;
    int npair = P * (P + 1) / 2;
    long ntask = (long)npair * D0 * D1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < ntask; ++t) {
        int pr = (int)(t / ((long)D0 * D1));
        int d0 = (int)((t / D1) % D0) - 2 * w0, d1 = (int)(t % D1) - 2 * w1;
        int kb = 0, c = pr;
        while (c >= P - kb) { c -= P - kb; ++kb; }
        int k = kb + c;
        out[t] = lag_sum(W + kb * n, W + k * n, n0, n1, d0, d1);
    }
    free(W);
    return ORC_OK;
}

/* Theta_kb(d) = sum_x R^kb(x - d) S(x), d in [-w, w]^2 (Eq. B14). [k][d0][d1] */
int orc_theta(const double* r, const double* s, int n0, int n1, int dk, int w0, int w1,
              double* out) {
    int P = orc_nterms(dk);
    long n = (long)n0 * n1;
    int D0 = 2 * w0 + 1, D1 = 2 * w1 + 1;
    double* W = weighted_stack(r, n0, n1, dk);
    if (!W) return ORC_ENOMEM;
    long ntask = (long)P * D0 * D1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < ntask; ++t) {
        int kb = (int)(t / ((long)D0 * D1));
        int d0 = (int)((t / D1) % D0) - w0, d1 = (int)(t % D1) - w1;
        out[t] = lag_sum(W + kb * n, s, n0, n1, d0, d1);
    }
    free(W);
    return ORC_OK;
}

/* Lambda_{kb m}(d) = sum_x R^kb(x - d) T^m(x), d in [-w, w]^2 (Eq. B8). [k][m][d0][d1] */
int orc_lambda(const double* r, int n0, int n1, int dk, int db, int w0, int w1, double* out) {
    int P = orc_nterms(dk), Q = orc_nterms(db);
    long n = (long)n0 * n1;
    int D0 = 2 * w0 + 1, D1 = 2 * w1 + 1;
    double* W = weighted_stack(r, n0, n1, dk);
    double* T = (double*)malloc(sizeof(double) * n * Q);
    if (!W || !T) { free(W); free(T); return ORC_ENOMEM; }
    for (int m = 0; m < Q; ++m) {
        int p, q;
        orc_term(db, m, &p, &q);
        background_image(n0, n1, p, q, T + m * n);
    }
    long ntask = (long)P * Q * D0 * D1;
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < ntask; ++t) {
        int kb = (int)(t / ((long)Q * D0 * D1));
        int m = (int)((t / ((long)D0 * D1)) % Q);
        int d0 = (int)((t / D1) % D0) - w0, d1 = (int)(t % D1) - w1;
        out[t] = lag_sum(W + kb * n, T + m * n, n0, n1, d0, d1);
    }
    free(W);
    free(T);
    return ORC_OK;
}

/* C_{mb m} = sum_x T^mb T^m (Eq. B11) and E_m = sum_x S T^m (Eq. B15). */
int orc_background_blocks(const double* s, int n0, int n1, int db, double* cmat, double* evec) {
    int Q = orc_nterms(db);
    long n = (long)n0 * n1;
    double* T = (double*)malloc(sizeof(double) * n * Q);
    if (!T) return ORC_ENOMEM;
    for (int m = 0; m < Q; ++m) {
        int p, q;
        orc_term(db, m, &p, &q);
        background_image(n0, n1, p, q, T + m * n);
    }
    for (int a = 0; a < Q; ++a) {
        for (int b = 0; b < Q; ++b) cmat[a * Q + b] = lag_sum(T + a * n, T + b * n, n0, n1, 0, 0);
        evec[a] = lag_sum(T + a * n, s, n0, n1, 0, 0);
    }
    free(T);
    return ORC_OK;
}

/* Omega lookup with the symmetry Omega_{k kb}(d) = Omega_{kb k}(-d). */
static double omega_at(const double* om, int P, int w0, int w1, int kb, int k, int d0, int d1) {
    if (kb > k) { int t = kb; kb = k; k = t; d0 = -d0; d1 = -d1; }
    int pr = kb * P - kb * (kb - 1) / 2 + (k - kb);
    int D0 = 4 * w0 + 1, D1 = 4 * w1 + 1;
    return om[((long)pr * D0 + (d0 + 2 * w0)) * D1 + (d1 + 2 * w1)];
}

/* Assemble the normal matrix G (Eq. 18, blocks A B / B~ C) and right-hand
 * side h (D / E) from the lag tables by the case rules of Eq. B5, B7, B9,
 * B11, B13 and B15. G is N_u x N_u row-major, fully populated. */
int orc_assemble(const double* om, const double* th, const double* la, const double* cmat,
                 const double* evec, int w0, int w1, int dk, int db, int cp, double* G,
                 double* h) {
    int P = orc_nterms(dk), Q = orc_nterms(db);
    long nk = kernel_unknowns(w0, w1, dk, cp, NULL, NULL, NULL);
    long N = nk + Q;
    int* K = (int*)malloc(sizeof(int) * nk * 3);
    if (!K) return ORC_ENOMEM;
    int *A = K + nk, *B = K + 2 * nk;
    kernel_unknowns(w0, w1, dk, cp, K, A, B);
    int T0 = 2 * w0 + 1, T1 = 2 * w1 + 1;
#pragma omp parallel for schedule(dynamic, 8)
    for (long u = 0; u < nk; ++u) {
        int kb = K[u], ab = A[u], bb = B[u];
        int zb = (ab == 0 && bb == 0);
        for (long v = 0; v < nk; ++v) {
            int k = K[v], a = A[v], b = B[v];
            int z = (a == 0 && b == 0);
            double g;
            if (!zb && !z)      /* Eq. B5, first case */
                g = omega_at(om, P, w0, w1, kb, k, ab - a, bb - b) -
                    omega_at(om, P, w0, w1, kb, k, ab, bb) -
                    omega_at(om, P, w0, w1, kb, k, -a, -b) +
                    omega_at(om, P, w0, w1, kb, k, 0, 0);
            else if (zb && !z)  /* second case */
                g = omega_at(om, P, w0, w1, kb, k, -a, -b) - omega_at(om, P, w0, w1, kb, k, 0, 0);
            else if (!zb && z)  /* third case */
                g = omega_at(om, P, w0, w1, kb, k, ab, bb) - omega_at(om, P, w0, w1, kb, k, 0, 0);
            else                /* fourth case */
                g = omega_at(om, P, w0, w1, kb, k, 0, 0);
            G[u * N + v] = g;
        }
        for (int m = 0; m < Q; ++m) {   /* Eq. B7; the transposed block is Eq. B9 */
            const double* L = la + ((long)kb * Q + m) * T0 * T1;
            double g = L[(ab + w0) * T1 + (bb + w1)];
            if (!zb) g -= L[w0 * T1 + w1];
            G[u * N + nk + m] = g;
            G[(nk + m) * N + u] = g;
        }
        const double* Th = th + (long)kb * T0 * T1;   /* Eq. B13 */
        double hv = Th[(ab + w0) * T1 + (bb + w1)];
        if (!zb) hv -= Th[w0 * T1 + w1];
        h[u] = hv;
    }
    for (int a = 0; a < Q; ++a) {   /* Eq. B11 and B15 */
        for (int b = 0; b < Q; ++b) G[(nk + a) * N + nk + b] = cmat[a * Q + b];
        h[nk + a] = evec[a];
    }
    free(K);
    return ORC_OK;
}

/* Full system from the (masked) fit pair: G, h in pixel units. */
int orc_build(const double* r, const double* s, int n0, int n1, int w0, int w1, int dk, int db,
              int cp, double* G, double* h) {
    if (n0 < 2 || n1 < 2 || 2 * w0 + 1 > n0 || 2 * w1 + 1 > n1 || dk < 0 || db < 0)
        return ORC_EINVAL;
    int P = orc_nterms(dk), Q = orc_nterms(db);
    long sz_om = (long)P * (P + 1) / 2 * (4 * w0 + 1) * (4 * w1 + 1);
    long sz_th = (long)P * (2 * w0 + 1) * (2 * w1 + 1);
    long sz_la = (long)P * Q * (2 * w0 + 1) * (2 * w1 + 1);
    double* om = (double*)malloc(sizeof(double) * (sz_om + sz_th + sz_la + Q * Q + Q));
    if (!om) return ORC_ENOMEM;
    double *th = om + sz_om, *la = th + sz_th, *cm = la + sz_la, *ev = cm + Q * Q;
    int rc = orc_omega(r, n0, n1, dk, w0, w1, om);
    if (!rc) rc = orc_theta(r, s, n0, n1, dk, w0, w1, th);
    if (!rc) rc = orc_lambda(r, n0, n1, dk, db, w0, w1, la);
    if (!rc) rc = orc_background_blocks(s, n0, n1, db, cm, ev);
    if (!rc) rc = orc_assemble(om, th, la, cm, ev, w0, w1, dk, db, cp, G, h);
    free(om);
    return rc;
}

/* One element of G straight from the basis-image definition:
 * G_uv = sum_x Phi_u(x) Phi_v(x) with Phi_(k,a) = R^k(x-a) - [a!=0] R^k(x) and
 * Phi_m = T^m (Eq. 12 written as a linear model). u, v are unknown indices. */
double orc_g_entry(const double* r, int n0, int n1, int w0, int w1, int dk, int db, int cp,
                   long u, long v) {
    long nk = kernel_unknowns(w0, w1, dk, cp, NULL, NULL, NULL);
    int ku[2], au[2], bu[2], mu[2];
    long uv[2] = {u, v};
    int* K = (int*)malloc(sizeof(int) * nk * 3);
    kernel_unknowns(w0, w1, dk, cp, K, K + nk, K + 2 * nk);
    for (int t = 0; t < 2; ++t) {
        if (uv[t] < nk) { ku[t] = K[uv[t]]; au[t] = K[nk + uv[t]]; bu[t] = K[2 * nk + uv[t]]; mu[t] = -1; }
        else { ku[t] = -1; mu[t] = (int)(uv[t] - nk); }
    }
    free(K);
    int ik[2], jk[2];
    for (int t = 0; t < 2; ++t) {
        if (ku[t] >= 0) orc_term(dk, ku[t], &ik[t], &jk[t]);
        else orc_term(db, mu[t], &ik[t], &jk[t]);
    }
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (long x0 = 0; x0 < n0; ++x0) {
        double row = 0.0;
        for (long x1 = 0; x1 < n1; ++x1) {
            double f[2];
            for (int t = 0; t < 2; ++t) {
                if (ku[t] >= 0) {
                    long s0 = imod(x0 - au[t], n0), s1 = imod(x1 - bu[t], n1);
                    double shifted = pow(orc_coord(s0, n0), ik[t]) * pow(orc_coord(s1, n1), jk[t]) *
                                     r[s0 * n1 + s1];
                    double here = (au[t] || bu[t]) ? pow(orc_coord(x0, n0), ik[t]) *
                                                         pow(orc_coord(x1, n1), jk[t]) * r[x0 * n1 + x1]
                                                   : 0.0;
                    f[t] = shifted - here;
                } else {
                    f[t] = pow(orc_coord(x0, n0), ik[t]) * pow(orc_coord(x1, n1), jk[t]);
                }
            }
            row += f[0] * f[1];
        }
        acc += row;
    }
    return acc;
}

/* sum_x Phi_u(x) img(x) for one unknown u (one component of Phi^T img):
 * with img = S it is h_u; with img = S - Phi c it is the gradient of the
 * objective at c (Eq. 16-17), zero at the least-squares optimum. */
double orc_phi_dot(const double* r, const double* img, int n0, int n1, int w0, int w1, int dk,
                   int db, int cp, long u) {
    long nk = kernel_unknowns(w0, w1, dk, cp, NULL, NULL, NULL);
    int k = -1, a = 0, b = 0, i, j;
    if (u < nk) {
        int* K = (int*)malloc(sizeof(int) * nk * 3);
        kernel_unknowns(w0, w1, dk, cp, K, K + nk, K + 2 * nk);
        k = K[u];
        a = K[nk + u];
        b = K[2 * nk + u];
        free(K);
        orc_term(dk, k, &i, &j);
    } else {
        orc_term(db, (int)(u - nk), &i, &j);
    }
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (long x0 = 0; x0 < n0; ++x0) {
        double row = 0.0;
        for (long x1 = 0; x1 < n1; ++x1) {
            double f;
            if (k >= 0) {
                long s0 = imod(x0 - a, n0), s1 = imod(x1 - b, n1);
                f = pow(orc_coord(s0, n0), i) * pow(orc_coord(s1, n1), j) * r[s0 * n1 + s1];
                if (a || b) f -= pow(orc_coord(x0, n0), i) * pow(orc_coord(x1, n1), j) * r[x0 * n1 + x1];
            } else {
                f = pow(orc_coord(x0, n0), i) * pow(orc_coord(x1, n1), j);
            }
            row += f * img[x0 * n1 + x1];
        }
        acc += row;
    }
    return acc;
}

/* Solve G c = h: Jacobi scaling d = diag(G)^-1/2, textbook Cholesky of
 * D G D, two triangular solves, c = D y. Returns ORC_ENOTSPD on a
 * non-positive pivot. */
int orc_solve(const double* G, const double* h, long n, double* c) {
    double* L = (double*)malloc(sizeof(double) * n * n);
    double* d = (double*)malloc(sizeof(double) * n);
    double* y = (double*)malloc(sizeof(double) * n);
    if (!L || !d || !y) { free(L); free(d); free(y); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (long i = 0; i < n; ++i) {
        if (!(G[i * n + i] > 0.0)) { rc = ORC_ENOTSPD; goto done; }
        d[i] = 1.0 / sqrt(G[i * n + i]);
    }
    for (long i = 0; i < n; ++i)
        for (long j = 0; j < n; ++j) L[i * n + j] = d[i] * G[i * n + j] * d[j];
    for (long j = 0; j < n; ++j) {
        double s = L[j * n + j];
        for (long k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) { rc = ORC_ENOTSPD; goto done; }
        double ljj = sqrt(s);
        L[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
        for (long i = j + 1; i < n; ++i) {
            double t = L[i * n + j];
            for (long k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / ljj;
        }
    }
    for (long i = 0; i < n; ++i) {          /* L y = D h */
        double s = d[i] * h[i];
        for (long k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (long i = n - 1; i >= 0; --i) {     /* L^T z = y, c = D z */
        double s = y[i];
        for (long k = i + 1; k < n; ++k) s -= L[k * n + i] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (long i = 0; i < n; ++i) c[i] = d[i] * y[i];
done:
    free(L);
    free(d);
    free(y);
    return rc;
}

/* Kernel stamps kappa_k(a) = sum over the delta basis of Eq. 3-4:
 * kappa_k(a) = coef_(k,a) for a != 0 and kappa_k(0) = coef_(k,0) - sum_{a!=0} coef_(k,a).
 * Layout [k][a0 + w0][a1 + w1]. */
void orc_stamps(const double* coef, int w0, int w1, int dk, int cp, double* kap) {
    int P = orc_nterms(dk), L0 = 2 * w0 + 1, L1 = 2 * w1 + 1;
    long u = 0;
    memset(kap, 0, sizeof(double) * P * L0 * L1);
    for (int k = 0; k < P; ++k) {
        double off = 0.0;
        for (int a = -w0; a <= w0; ++a)
            for (int b = -w1; b <= w1; ++b) {
                if (cp && k > 0 && a == 0 && b == 0) continue;
                double cv = coef[u++];
                kap[((long)k * L0 + a + w0) * L1 + b + w1] += cv;
                if (a || b) off += cv;
            }
        kap[((long)k * L0 + w0) * L1 + w1] -= off;
    }
}

/* D(x) = S(x) - sum_k sum_a kappa_k(a) R^k(x - a) - sum_m b_m T^m(x)
 * (Eq. 12 with the solved coefficients; R is the unmasked apply image). */
void orc_subtract(const double* r, const double* s, int n0, int n1, int w0, int w1, int dk,
                  int db, int cp, const double* coef, double* d) {
    int P = orc_nterms(dk), Q = orc_nterms(db), L0 = 2 * w0 + 1, L1 = 2 * w1 + 1;
    long nk = kernel_unknowns(w0, w1, dk, cp, NULL, NULL, NULL);
    long n = (long)n0 * n1;
    double* kap = (double*)malloc(sizeof(double) * P * L0 * L1);
    double* W = weighted_stack(r, n0, n1, dk);
    orc_stamps(coef, w0, w1, dk, cp, kap);
    const double* bcoef = coef + nk;
    int pq[64][2];
    for (int m = 0; m < Q; ++m) orc_term(db, m, &pq[m][0], &pq[m][1]);
#pragma omp parallel for schedule(static)
    for (long x0 = 0; x0 < n0; ++x0) {
        for (long x1 = 0; x1 < n1; ++x1) {
            double conv = 0.0;
            for (int k = 0; k < P; ++k)
                for (int a = -w0; a <= w0; ++a) {
                    const double* row = W + k * n + imod(x0 - a, n0) * n1;
                    const double* kr = kap + ((long)k * L0 + a + w0) * L1 + w1;
                    for (int b = -w1; b <= w1; ++b) conv += kr[b] * row[imod(x1 - b, n1)];
                }
            double bg = 0.0;
            for (int m = 0; m < Q; ++m)
                bg += bcoef[m] * pow(orc_coord(x0, n0), pq[m][0]) * pow(orc_coord(x1, n1), pq[m][1]);
            d[x0 * n1 + x1] = s[x0 * n1 + x1] - conv - bg;
        }
    }
    free(kap);
    free(W);
}

/* D at a list of pixels only (for sampled checks at full image size). */
void orc_subtract_pixels(const double* r, const double* s, int n0, int n1, int w0, int w1,
                         int dk, int db, int cp, const double* coef, const long* pix, long npix,
                         double* out) {
    int P = orc_nterms(dk), Q = orc_nterms(db), L0 = 2 * w0 + 1, L1 = 2 * w1 + 1;
    long nk = kernel_unknowns(w0, w1, dk, cp, NULL, NULL, NULL);
    double* kap = (double*)malloc(sizeof(double) * P * L0 * L1);
    orc_stamps(coef, w0, w1, dk, cp, kap);
    for (long t = 0; t < npix; ++t) {
        long x0 = pix[2 * t], x1 = pix[2 * t + 1];
        double conv = 0.0;
        for (int k = 0; k < P; ++k) {
            int i, j;
            orc_term(dk, k, &i, &j);
            for (int a = -w0; a <= w0; ++a)
                for (int b = -w1; b <= w1; ++b) {
                    long s0 = imod(x0 - a, n0), s1 = imod(x1 - b, n1);
                    conv += kap[((long)k * L0 + a + w0) * L1 + b + w1] *
                            pow(orc_coord(s0, n0), i) * pow(orc_coord(s1, n1), j) * r[s0 * n1 + s1];
                }
        }
        double bg = 0.0;
        for (int m = 0; m < Q; ++m) {
            int p, q;
            orc_term(db, m, &p, &q);
            bg += coef[nk + m] * pow(orc_coord(x0, n0), p) * pow(orc_coord(x1, n1), q);
        }
        out[t] = s[x0 * n1 + x1] - conv - bg;
    }
    free(kap);
}

/* Kernel-sum field sum_k a_(k,00) c0^i c1^j (Eq. 6 at a=b=0: the basis of
 * Eq. 4 sums to zero, so the kernel integral is the 00 coefficient). */
void orc_kernel_sum_field(const double* coef, int n0, int n1, int w0, int w1, int dk, int cp,
                          double* out) {
    int P = orc_nterms(dk), L = (2 * w0 + 1) * (2 * w1 + 1);
    double c00[64];
    long u = 0;
    for (int k = 0; k < P; ++k)
        for (int a = -w0; a <= w0; ++a)
            for (int b = -w1; b <= w1; ++b) {
                if (cp && k > 0 && a == 0 && b == 0) { if (a == 0 && b == 0) c00[k] = 0.0; continue; }
                if (a == 0 && b == 0) c00[k] = coef[u];
                ++u;
            }
    (void)L;
    for (long x0 = 0; x0 < n0; ++x0)
        for (long x1 = 0; x1 < n1; ++x1) {
            double s = 0.0;
            for (int k = 0; k < P; ++k) {
                int i, j;
                orc_term(dk, k, &i, &j);
                s += c00[k] * pow(orc_coord(x0, n0), i) * pow(orc_coord(x1, n1), j);
            }
            out[x0 * n1 + x1] = s;
        }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
