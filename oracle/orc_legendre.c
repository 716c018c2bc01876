/*
 * ORACLE -- test infrastructure only.  Plain, slow, CPU reference for the Legendre part of
 * the exact spherical harmonic transform (Sect. 2.1, Eqs. (1)-(2)).  Nothing in the product
 * path may link or call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.
 *
 * Conventions (Sect. 2.1 names the spherical harmonics the canonical orthonormal basis;
 * the phase is not stated, so the Condon-Shortley phase is used):
 *   Y_lm(theta, phi) = lambda_lm(theta) exp(i m phi),
 *   lambda_lm(theta) = sqrt((2l+1)/(4 pi)) d^l_{m0}(theta),
 *   lambda_{l,-m} = (-1)^m lambda_lm.
 *
 * lambda_lm is produced by the textbook normalised three-term recursion, in long double,
 * with every value carried as (mantissa, binary exponent) so that the deep underflow of
 * lambda_mm = c_m sin^m(theta) near the poles (below 1e-6000 at m = 2047) is represented:
 *   lambda_00       = 1 / sqrt(4 pi)
 *   lambda_mm       = -sqrt((2m+1)/(2m)) sin(theta) lambda_{m-1,m-1}
 *   lambda_{m+1,m}  = sqrt(2m+3) cos(theta) lambda_mm
 *   lambda_lm       = a_lm (cos(theta) lambda_{l-1,m} - b_lm lambda_{l-2,m}),
 *       a_lm = sqrt((4l^2-1)/(l^2-m^2)),  b_lm = sqrt(((l-1)^2-m^2)/(4(l-1)^2-1)).
 *
 * The sampling nodes of the McEwen-Wiaux theorem (Sect. 2.1) are
 *   theta_t = pi (2t+1) / (2k-1),  t = 0..k-1   (theta_{k-1} = pi; the north pole is not sampled).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

typedef long double LD;
typedef struct { LD v; long e; } xld; /* value = v * 2^e */

static const LD PI_L = 3.141592653589793238462643383279502884L;

static xld xnorm(LD v, long e) {
    xld r;
    int ex = 0;
    if (v == 0.0L) { r.v = 0.0L; r.e = 0; return r; }
    r.v = frexpl(v, &ex);
    r.e = e + ex;
    return r;
}

static LD xval(xld x) {
    if (x.v == 0.0L) return 0.0L;
    if (x.e < -20000) return 0.0L;
    return ldexpl(x.v, (int)x.e);
}

static LD node_theta(int k, int t) { return PI_L * (LD)(2 * t + 1) / (LD)(2 * k - 1); }

/* Diagonal values lambda_mm(theta) for m = 0..k-1 as (mantissa, exponent). */
static void diag_values(int k, LD theta, xld* diag) {
    LD s = sinl(theta);
    xld cur = xnorm(1.0L / sqrtl(4.0L * PI_L), 0);
    diag[0] = cur;
    for (int m = 1; m < k; ++m) {
        LD f = -sqrtl((LD)(2 * m + 1) / (LD)(2 * m)) * s;
        cur = xnorm(cur.v * f, cur.e);
        diag[m] = cur;
    }
}

/* Recursion coefficients a_lm, b_lm for one m, l = m..k-1 (entries l < m+2 unused). */
static void column_coefs(int k, int m, LD* a, LD* b) {
    for (int l = m + 2; l < k; ++l) {
        LD ll = (LD)l, mm = (LD)m;
        a[l - m] = sqrtl((4.0L * ll * ll - 1.0L) / (ll * ll - mm * mm));
        b[l - m] = sqrtl(((ll - 1.0L) * (ll - 1.0L) - mm * mm) / (4.0L * (ll - 1.0L) * (ll - 1.0L) - 1.0L));
    }
}

/* Packed coefficient table for every m: column m starts at m*k - m*(m-1)/2. */
static size_t col_offset(int k, int m) { return (size_t)m * k - (size_t)m * (m - 1) / 2; }

static void coef_table(int k, LD** a_out, LD** b_out) {
    size_t tot = (size_t)k * (k + 1) / 2;
    LD* a = (LD*)malloc(sizeof(LD) * tot);
    LD* b = (LD*)malloc(sizeof(LD) * tot);
#pragma omp parallel for schedule(dynamic, 16)
    for (int m = 0; m < k; ++m) column_coefs(k, m, a + col_offset(k, m), b + col_offset(k, m));
    *a_out = a;
    *b_out = b;
}

/* Walk lambda_lm(theta) for l = m..k-1, writing true values (long double, 0 on underflow). */
static void column_values(int k, int m, LD theta, xld dmm, const LD* ca, const LD* cb, LD* out) {
    LD x = cosl(theta);
    LD p2 = dmm.v;                 /* lambda_{l-2} mantissa (common exponent E) */
    long E = dmm.e;
    if (E > -15000) { p2 = ldexpl(p2, (int)E); E = 0; }   /* representable: carry true values */
    out[0] = xval((xld){p2, E});
    if (m + 1 >= k) return;
    LD p1 = sqrtl((LD)(2 * m + 3)) * x * p2;  /* lambda_{m+1,m} */
    out[1] = xval((xld){p1, E});
    for (int l = m + 2; l < k; ++l) {
        LD p = ca[l - m] * (x * p1 - cb[l - m] * p2);
        p2 = p1;
        p1 = p;
        if (E != 0) {
            if (fabsl(p1) > 0x1p100L) {          /* keep the pair inside the long double range */
                p1 = ldexpl(p1, -100);
                p2 = ldexpl(p2, -100);
                E += 100;
                if (E > -15000) { p1 = ldexpl(p1, (int)E); p2 = ldexpl(p2, (int)E); E = 0; }
            }
            out[l - m] = xval((xld){p1, E});
        } else {
            out[l - m] = p1;
        }
    }
}

/* lambda_lm(theta_j) for l = m..k-1 at arbitrary angles: out[j*(k-m) + (l-m)], as double. */
void orc_lambda(int k, int m, const double* theta, int ntheta, double* out) {
    xld* diag = (xld*)malloc(sizeof(xld) * (size_t)k);
    LD* col = (LD*)malloc(sizeof(LD) * (size_t)k);
    LD* ca = (LD*)malloc(sizeof(LD) * (size_t)k);
    LD* cb = (LD*)malloc(sizeof(LD) * (size_t)k);
    column_coefs(k, m, ca, cb);
    for (int j = 0; j < ntheta; ++j) {
        diag_values(k, (LD)theta[j], diag);
        column_values(k, m, (LD)theta[j], diag[m], ca, cb, col);
        for (int l = m; l < k; ++l) out[(size_t)j * (k - m) + (l - m)] = (double)col[l - m];
    }
    free(diag);
    free(col);
    free(ca);
    free(cb);
}

/* log2 |lambda_lm(theta)| for l = m..k-1 (-inf where the value is exactly 0). */
void orc_lambda_log2(int k, int m, double theta, double* out) {
    xld* diag = (xld*)malloc(sizeof(xld) * (size_t)k);
    diag_values(k, (LD)theta, diag);
    LD x = cosl((LD)theta);
    xld d = diag[m];
    LD p2 = d.v, p1;
    long E = d.e;
    out[0] = (p2 == 0.0L) ? -INFINITY : (double)(log2l(fabsl(p2)) + (LD)E);
    if (m + 1 < k) {
        p1 = sqrtl((LD)(2 * m + 3)) * x * p2;
        out[1] = (p1 == 0.0L) ? -INFINITY : (double)(log2l(fabsl(p1)) + (LD)E);
        for (int l = m + 2; l < k; ++l) {
            LD ll = (LD)l, mm = (LD)m;
            LD a = sqrtl((4.0L * ll * ll - 1.0L) / (ll * ll - mm * mm));
            LD b = sqrtl(((ll - 1.0L) * (ll - 1.0L) - mm * mm) / (4.0L * (ll - 1.0L) * (ll - 1.0L) - 1.0L));
            LD p = a * (x * p1 - b * p2);
            p2 = p1;
            p1 = p;
            if (fabsl(p1) > 0x1p100L || (fabsl(p1) < 0x1p-100L && p1 != 0.0L && fabsl(p2) < 0x1p-100L)) {
                int ex;
                frexpl(p1, &ex);
                p1 = ldexpl(p1, -ex);
                p2 = ldexpl(p2, -ex);
                E += ex;
            }
            out[l - m] = (p1 == 0.0L) ? -INFINITY : (double)(log2l(fabsl(p1)) + (LD)E);
        }
    }
    free(diag);
}

/*
 * Inverse Legendre step of Eq. (1) on the MW nodes:
 *   F_m(theta_t) = sum_{l=|m|}^{k-1} f_lm lambda_lm(theta_t),   |m| <= k-1, t = 0..k-1.
 * flm: [ncol][k*k] complex, f_lm at l*l+l+m.   F: [ncol][k][2k-1] complex, m at index m+k-1.
 */
static void legendre_inverse_rings(int k, int ncol, const double complex* flm, int nrings,
                                   const int* rings, double complex* F) {
    const int n = 2 * k - 1;
    LD *ta, *tb;
    coef_table(k, &ta, &tb);
#pragma omp parallel
    {
        xld* diag = (xld*)malloc(sizeof(xld) * (size_t)k);
        LD* col = (LD*)malloc(sizeof(LD) * (size_t)k);
        LD* accp = (LD*)malloc(sizeof(LD) * 2 * (size_t)ncol);
        LD* accn = (LD*)malloc(sizeof(LD) * 2 * (size_t)ncol);
#pragma omp for schedule(dynamic, 1)
        for (int r = 0; r < nrings; ++r) {
            const int t = rings ? rings[r] : r;
            LD theta = node_theta(k, t);
            diag_values(k, theta, diag);
            for (int m = 0; m < k; ++m) {
                column_values(k, m, theta, diag[m], ta + col_offset(k, m), tb + col_offset(k, m), col);
                memset(accp, 0, sizeof(LD) * 2 * (size_t)ncol);
                memset(accn, 0, sizeof(LD) * 2 * (size_t)ncol);
                LD sgn = (m & 1) ? -1.0L : 1.0L;
                for (int c = 0; c < ncol; ++c) {
                    const double complex* f = flm + (size_t)c * k * k;
                    for (int l = m; l < k; ++l) {
                        LD lam = col[l - m];
                        double complex fp = f[l * l + l + m];
                        accp[2 * c] += lam * (LD)creal(fp);
                        accp[2 * c + 1] += lam * (LD)cimag(fp);
                        if (m > 0) {
                            double complex fn = f[l * l + l - m];
                            accn[2 * c] += sgn * lam * (LD)creal(fn);
                            accn[2 * c + 1] += sgn * lam * (LD)cimag(fn);
                        }
                    }
                    double complex* Fc = F + (size_t)c * nrings * n + (size_t)r * n;
                    Fc[k - 1 + m] = (double)accp[2 * c] + I * (double)accp[2 * c + 1];
                    if (m > 0) Fc[k - 1 - m] = (double)accn[2 * c] + I * (double)accn[2 * c + 1];
                }
            }
        }
        free(diag);
        free(col);
        free(accp);
        free(accn);
    }
    free(ta);
    free(tb);
}

void orc_legendre_inverse(int k, int ncol, const double complex* flm, double complex* F) {
    legendre_inverse_rings(k, ncol, flm, k, NULL, F);
}

/* The same sums restricted to the rings listed in rings[0..nrings): F is [ncol][nrings][2k-1]. */
void orc_legendre_inverse_rings(int k, int ncol, const double complex* flm, int nrings,
                                const int* rings, double complex* F) {
    legendre_inverse_rings(k, ncol, flm, nrings, rings, F);
}

/*
 * Forward Legendre step (the last step of the MW quadrature for Eq. (2)):
 *   f_lm = sum_{t=0}^{k-1} lambda_lm(theta_t) H_m(theta_t).
 * H: [ncol][k][2k-1] complex (m at index m+k-1).  flm: [ncol][k*k] complex (output).
 */
void orc_legendre_forward(int k, int ncol, const double complex* H, double complex* flm) {
    const int n = 2 * k - 1;
    xld* diag_all = (xld*)malloc(sizeof(xld) * (size_t)k * (size_t)k);
    LD *ta, *tb;
    coef_table(k, &ta, &tb);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < k; ++t) diag_values(k, node_theta(k, t), diag_all + (size_t)t * k);
    memset(flm, 0, sizeof(double complex) * (size_t)ncol * k * k);
#pragma omp parallel
    {
        LD* col = (LD*)malloc(sizeof(LD) * (size_t)k);
        LD* accp = (LD*)malloc(sizeof(LD) * 2 * (size_t)k * ncol);
        LD* accn = (LD*)malloc(sizeof(LD) * 2 * (size_t)k * ncol);
#pragma omp for schedule(dynamic, 1)
        for (int m = 0; m < k; ++m) {
            int nl = k - m;
            memset(accp, 0, sizeof(LD) * 2 * (size_t)nl * ncol);
            memset(accn, 0, sizeof(LD) * 2 * (size_t)nl * ncol);
            LD sgn = (m & 1) ? -1.0L : 1.0L;
            for (int t = 0; t < k; ++t) {
                LD theta = node_theta(k, t);
                column_values(k, m, theta, diag_all[(size_t)t * k + m], ta + col_offset(k, m), tb + col_offset(k, m), col);
                for (int c = 0; c < ncol; ++c) {
                    const double complex* Hc = H + (size_t)c * k * n + (size_t)t * n;
                    double complex hp = Hc[k - 1 + m];
                    double complex hn = Hc[k - 1 - m];
                    LD* ap = accp + 2 * (size_t)c * nl;
                    LD* an = accn + 2 * (size_t)c * nl;
                    for (int l = m; l < k; ++l) {
                        LD lam = col[l - m];
                        ap[2 * (l - m)] += lam * (LD)creal(hp);
                        ap[2 * (l - m) + 1] += lam * (LD)cimag(hp);
                        if (m > 0) {
                            an[2 * (l - m)] += sgn * lam * (LD)creal(hn);
                            an[2 * (l - m) + 1] += sgn * lam * (LD)cimag(hn);
                        }
                    }
                }
            }
            for (int c = 0; c < ncol; ++c) {
                double complex* f = flm + (size_t)c * k * k;
                LD* ap = accp + 2 * (size_t)c * nl;
                LD* an = accn + 2 * (size_t)c * nl;
                for (int l = m; l < k; ++l) {
                    f[l * l + l + m] = (double)ap[2 * (l - m)] + I * (double)ap[2 * (l - m) + 1];
                    if (m > 0) f[l * l + l - m] = (double)an[2 * (l - m)] + I * (double)an[2 * (l - m) + 1];
                }
            }
        }
        free(col);
        free(accp);
        free(accn);
    }
    free(diag_all);
    free(ta);
    free(tb);
}
