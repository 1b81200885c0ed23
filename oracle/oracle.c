/*
 * oracle.c -- plain, slow, FP64 CPU reference for the batched polynomial
 * root path of "Hardware-Accelerated Algorithm for Complex Function Roots
 * Density Graph Plotting" (Tang & Quan, arXiv 2507.02164).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * code, header, table or helper with the HIP library, and includes none of
 * its files.
 *
 * What it computes:
 *   oracle_solve     -- roots of p(z) = sum_k a_k z^k as eigenvalues of the
 *                       Frobenius companion matrix (Sec. II-B), by
 *                       single-shift QR iteration (Alg. 1) with bottom
 *                       deflation; each step's factorisation A - sI = QR is
 *                       built from the complex Givens rotations of Sec. II-C,
 *                       and the step A <- RQ + sI is formed with dense matrix
 *                       products.
 *   oracle_density   -- roots -> integer pixel counts over a complex window
 *                       (Sec. III, the roots-to-pixels stage).
 *   oracle_backward  -- implicit-function adjoint dr/da_k = -r^k / p'(r).
 *                       The paper has no gradient; this is the textbook
 *                       derivative of a simple root, written out.
 *
 * Storage is a dense row-major d x d matrix; every rotation is formed as a
 * full m x m matrix and applied by a dense matrix product, so there is no
 * band trimming, fusion or in-place shortcut.  Floating point: compiled
 * with -O2 -ffp-contract=off, so
 * every complex operation is a sequence of correctly rounded IEEE double
 * operations (gcc's C99 complex multiply/divide).
 *
 * Readings of the paper taken here (where it is silent):
 *   - companion form: first row -b_{d-1} ... -b_0, ones on the subdiagonal
 *     (the paper names the Frobenius companion matrix without printing it);
 *   - Givens pair: the unique (c, s) = (conj(a), conj(b)) / rho that makes
 *     the Sec. II-C rotation map (a, b) to (rho, 0) with rho = sqrt(|a|^2 +
 *     |b|^2) >= 0; identity when rho == 0;
 *   - the annihilated entry is stored as an exact zero after each row
 *     rotation (the Appendix proves it is zero in exact arithmetic);
 *   - convergence: instead of Alg. 1's fixed iteration count, a level
 *     deflates once cabs1(h[m-1][m-2]) <= eps * (cabs1(h[m-1][m-1]) +
 *     cabs1(h[m-2][m-2])), cabs1(z) = |Re z| + |Im z|, eps = 2^-52;
 *   - exceptional shift at the 10th and 20th iteration of a level:
 *     s = h[m-1][m-1] + cabs1(h[m-1][m-2]) * (0.75 + 0.5i), whichever shift
 *     rule is in force otherwise; cap of 30 iterations per
 *     level, after which the level deflates anyway and NOT_CONVERGED is set;
 *   - a fixed-T mode (flag) reproduces Alg. 2 literally: exactly T QR steps
 *     per level, no test, no exceptional shift;
 *   - an optional shift (flag): instead of Alg. 1's bottom-right entry, the
 *     eigenvalue of the trailing 2 x 2 block nearest that entry (Wilkinson's
 *     shift, the textbook choice for single-shift QR; not in the paper).
 *     It is still one complex shift per QR step; only its value changes.
 *     The fixed-T mode, being Alg. 2 literally, keeps Alg. 1's shift;
 *   - an optional first shift (flag, not in the paper): the very first QR
 *     step of a polynomial is shifted by the root nearest 0 of
 *     b_0 + b_1 z + b_2 z^2, an estimate of the smallest root, which the
 *     first unshifted steps would otherwise isolate slowly (the trailing
 *     block of the companion matrix is [[0, 0], [1, 0]], so both Alg. 1's and
 *     Wilkinson's first shift is 0).  Not in the fixed-T mode either.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <float.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Status bits (values fixed by the library's public contract; restated here
 * so that this file depends on nothing but libc). */
#define OST_BAD_DEGREE 0x1u
#define OST_NONFINITE 0x2u
#define OST_ZERO_LEADING 0x4u
#define OST_NOT_CONVERGED 0x8u
#define OST_SINGULAR_DERIV 0x20u

/* flags for oracle_solve */
#define OFLAG_NO_EXCEPTIONAL_SHIFT 0x1u
#define OFLAG_FIXED_T 0x2u
#define OFLAG_WILKINSON_SHIFT 0x8u
#define OFLAG_QUADRATIC_START 0x10u

#define ODMAX 6

typedef double complex cplx;

static double cabs1(cplx z) { return fabs(creal(z)) + fabs(cimag(z)); }

static int cfinite(cplx z) { return isfinite(creal(z)) && isfinite(cimag(z)); }

/* Sec. II-C equation: the unitary [[c, s], [-conj(s), conj(c)]] maps
 * (a, b) to (sqrt(|a|^2 + |b|^2), 0).  The only such pair is
 * c = conj(a)/rho, s = conj(b)/rho (Cauchy-Schwarz equality).  rho == 0
 * leaves the rows unchanged (identity rotation). */
void oracle_givens(const double *a_ri, const double *b_ri, double *c_ri, double *s_ri)
{
    cplx a = a_ri[0] + I * a_ri[1];
    cplx b = b_ri[0] + I * b_ri[1];
    double rho = hypot(cabs(a), cabs(b));
    cplx c = 1.0, s = 0.0;
    if (rho != 0.0) {
        c = conj(a) / rho;
        s = conj(b) / rho;
    }
    c_ri[0] = creal(c);
    c_ri[1] = cimag(c);
    s_ri[0] = creal(s);
    s_ri[1] = cimag(s);
}

/* Z = X Y for m x m matrices (row-major, leading dimension m): the plain
 * dense product, each entry summed over k = 0..m-1 in order. */
static void matmul(int m, const cplx *X, const cplx *Y, cplx *Z)
{
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            cplx acc = 0.0;
            for (int k = 0; k < m; ++k)
                acc += X[i * m + k] * Y[k * m + j];
            Z[i * m + j] = acc;
        }
}

/* One shifted QR step on the leading m x m block of the dense matrix H
 * (row-major, leading dimension ld), Alg. 1 body: A - sI = QR, then
 * A <- RQ + sI.  The factorisation comes from the Sec. II-C rotations:
 * G_r is the identity except for the 2 x 2 block [[c, s], [-conj(s),
 * conj(c)]] on rows and columns r-1, r, with (c, s) chosen from the matrix
 * G_{r-1}...G_1 (A - sI) reached so far so that its entry (r, r-1) becomes
 * zero.  After r = 1..m-1 the product R = G (A - sI), G = G_{m-1}...G_1,
 * is upper triangular and G is unitary, so A - sI = G^H R: Q = G^H and the
 * new matrix is R G^H + sI.  Every product is a plain dense matrix product
 * (matmul); the entry each rotation annihilates is then stored as an exact
 * zero, which in exact arithmetic it is (Appendix). */
static void qr_step(int m, int ld, cplx *H, cplx shift)
{
    cplx R[ODMAX * ODMAX], G[ODMAX * ODMAX], Gr[ODMAX * ODMAX], T[ODMAX * ODMAX];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            R[i * m + j] = H[i * ld + j];
            G[i * m + j] = i == j ? 1.0 : 0.0;
        }
    for (int i = 0; i < m; ++i)
        R[i * m + i] -= shift;
    for (int r = 1; r < m; ++r) {
        double a[2] = {creal(R[(r - 1) * m + r - 1]), cimag(R[(r - 1) * m + r - 1])};
        double b[2] = {creal(R[r * m + r - 1]), cimag(R[r * m + r - 1])};
        double cc[2], ss[2];
        oracle_givens(a, b, cc, ss);
        cplx c = cc[0] + I * cc[1], s = ss[0] + I * ss[1];
        for (int k = 0; k < m * m; ++k)
            Gr[k] = 0.0;
        for (int i = 0; i < m; ++i)
            Gr[i * m + i] = 1.0;
        Gr[(r - 1) * m + (r - 1)] = c;
        Gr[(r - 1) * m + r] = s;
        Gr[r * m + (r - 1)] = -conj(s);
        Gr[r * m + r] = conj(c);
        matmul(m, Gr, R, T);
        memcpy(R, T, sizeof(cplx) * m * m);
        R[r * m + (r - 1)] = 0.0;
        matmul(m, Gr, G, T);
        memcpy(G, T, sizeof(cplx) * m * m);
    }
    cplx GH[ODMAX * ODMAX];
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            GH[i * m + j] = conj(G[j * m + i]);
    matmul(m, R, GH, T);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j)
            H[i * ld + j] = T[i * m + j];
    for (int i = 0; i < m; ++i)
        H[i * ld + i] += shift;
}

/* Exposed for tests: one QR step with an explicit shift on a dense m x m
 * matrix stored as interleaved (re, im) doubles, row-major. */
void oracle_qr_step(int m, double *H_ri, const double *shift_ri)
{
    cplx H[ODMAX * ODMAX];
    for (int k = 0; k < m * m; ++k)
        H[k] = H_ri[2 * k] + I * H_ri[2 * k + 1];
    qr_step(m, m, H, shift_ri[0] + I * shift_ri[1]);
    for (int k = 0; k < m * m; ++k) {
        H_ri[2 * k] = creal(H[k]);
        H_ri[2 * k + 1] = cimag(H[k]);
    }
}

/* Wilkinson's shift: the eigenvalue of the 2 x 2 block [[a, b], [c, e]]
 * nearest e.  With t = (a - e) / 2 the eigenvalues are e + t + r and
 * e + t - r, r^2 = t^2 + b c.  Of the two square roots r is the one with
 * Re(conj(t) r) >= 0, so that |t + r| >= |t - r| and e + t - r is the nearer
 * eigenvalue; it equals e - b c / (t + r) (multiply by (t + r) / (t + r) and
 * use r^2 - t^2 = b c), which is the form evaluated.  t + r == 0 forces
 * t == r == 0, hence b c == 0 and a double eigenvalue e. */
static cplx wilkinson_shift(cplx a, cplx b, cplx c, cplx e)
{
    cplx t = 0.5 * (a - e);
    cplx bc = b * c;
    cplx r = csqrt(t * t + bc);
    if (creal(t) * creal(r) + cimag(t) * cimag(r) < 0.0)
        r = -r;
    cplx den = t + r;
    if (den == 0.0)
        return e;
    return e - bc / den;
}

/* The root nearest 0 of b0 + b1 z + b2 z^2 (b2 != 0 or b1 != 0): with
 * D = sqrt(b1^2 - 4 b0 b2) the roots are 2 b0 / (-b1 -+ D) (the product of
 * the two roots of the quadratic is b0 / b2, and this form needs no b2 in a
 * denominator); of the two denominators the one of larger modulus gives the
 * smaller root.  Returns 0 (and *ok = 0) where that denominator is zero
 * (b0 == b1 == 0 with b2 == 0, or a double root at 0 -- then 0 is the
 * root) and *ok = 0 where the value is not finite. */
static cplx quadratic_start(cplx b0, cplx b1, cplx b2, int *ok)
{
    cplx d = csqrt(b1 * b1 - 4.0 * b0 * b2);
    cplx den1 = -b1 - d, den2 = -b1 + d;
    cplx den = cabs(den1) >= cabs(den2) ? den1 : den2;
    *ok = 1;
    if (den == 0.0) {
        *ok = b0 == 0.0;
        return 0.0;
    }
    cplx z = 2.0 * b0 / den;
    if (!cfinite(z)) {
        *ok = 0;
        return 0.0;
    }
    return z;
}

/* Exposed for tests: the quadratic start of b0 + b1 z + b2 z^2; returns
 * whether it is defined. */
int oracle_quadratic_start(const double *b0_ri, const double *b1_ri, const double *b2_ri,
                           double *z_ri)
{
    int ok;
    cplx z = quadratic_start(b0_ri[0] + I * b0_ri[1], b1_ri[0] + I * b1_ri[1],
                             b2_ri[0] + I * b2_ri[1], &ok);
    z_ri[0] = creal(z);
    z_ri[1] = cimag(z);
    return ok;
}

/* Exposed for tests: Wilkinson's shift of [[a, b], [c, e]], each complex
 * value as interleaved (re, im) doubles. */
void oracle_wilkinson_shift(const double *a_ri, const double *b_ri, const double *c_ri,
                            const double *e_ri, double *mu_ri)
{
    cplx mu = wilkinson_shift(a_ri[0] + I * a_ri[1], b_ri[0] + I * b_ri[1],
                              c_ri[0] + I * c_ri[1], e_ri[0] + I * e_ri[1]);
    mu_ri[0] = creal(mu);
    mu_ri[1] = cimag(mu);
}

/* Roots of one polynomial of degree d with coefficients a[0..d] (a[d]
 * leading).  eig[0..d-1] receives the eigenvalues in deflation order
 * (eig[d-1] is found first, eig[0] last, as in Alg. 1).  its[m-2] receives
 * the number of QR steps taken at level m (m = 2..d).  Returns status bits.
 */
static unsigned solve_one(int d, const cplx *a, cplx *eig, int *its_out,
                          int cap, unsigned flags, int fixed_t)
{
    unsigned st = 0;
    for (int k = 0; k <= d; ++k)
        if (!cfinite(a[k]))
            st |= OST_NONFINITE;
    if (!st && a[d] == 0.0)
        st |= OST_ZERO_LEADING;
    if (st) {
        for (int k = 0; k < d; ++k)
            eig[k] = NAN + I * NAN;
        return st;
    }

    /* Sec. II-B: the roots of p are those of the monic p / a_d. */
    cplx b[ODMAX + 1];
    for (int k = 0; k < d; ++k)
        b[k] = a[k] / a[d];
    b[d] = 1.0;

    if (d == 1) {
        eig[0] = -b[0];
        return st;
    }

    /* Frobenius companion matrix, first-row form: its characteristic
     * polynomial is z^d + b_{d-1} z^{d-1} + ... + b_0. */
    cplx H[ODMAX * ODMAX];
    for (int k = 0; k < d * d; ++k)
        H[k] = 0.0;
    for (int j = 0; j < d; ++j)
        H[0 * d + j] = -b[d - 1 - j];
    for (int i = 0; i + 1 < d; ++i)
        H[(i + 1) * d + i] = 1.0;

    const double eps = DBL_EPSILON; /* 2^-52 */
    for (int m = d; m >= 2; --m) {
        int its = 0;
        for (;;) {
            cplx hsub = H[(m - 1) * d + (m - 2)];
            if (fixed_t > 0) {
                if (its == fixed_t)
                    break;
            } else {
                double h = cabs1(hsub);
                double t = cabs1(H[(m - 1) * d + (m - 1)]) + cabs1(H[(m - 2) * d + (m - 2)]);
                if (h <= eps * t)
                    break;
                if (its == cap) {
                    st |= OST_NOT_CONVERGED;
                    break;
                }
            }
            /* Alg. 1: the shift is the current bottom-right entry, or, with
             * the flag, Wilkinson's shift of the trailing 2 x 2 block. */
            cplx s = H[(m - 1) * d + (m - 1)];
            if ((flags & OFLAG_WILKINSON_SHIFT) && fixed_t <= 0)
                s = wilkinson_shift(H[(m - 2) * d + (m - 2)], H[(m - 2) * d + (m - 1)], hsub,
                                    H[(m - 1) * d + (m - 1)]);
            if ((flags & OFLAG_QUADRATIC_START) && fixed_t <= 0 && m == d && its == 0) {
                int ok;
                cplx z = quadratic_start(b[0], b[1], d >= 3 ? b[2] : 1.0, &ok);
                if (ok)
                    s = z;
            }
            /* exceptional shift on the 10th and 20th step of a level: the
             * bottom-right entry moved off by cabs1 of the subdiagonal entry,
             * in place of whichever shift the rule would take */
            if (fixed_t <= 0 && !(flags & OFLAG_NO_EXCEPTIONAL_SHIFT) && (its == 10 || its == 20))
                s = H[(m - 1) * d + (m - 1)] + cabs1(hsub) * (0.75 + 0.5 * I);
            qr_step(m, d, H, s);
            ++its;
        }
        if (its_out)
            its_out[m - 2] = its;
        /* Alg. 1: record eig[m-1], then continue on the leading block. */
        eig[m - 1] = H[(m - 1) * d + (m - 1)];
    }
    eig[0] = H[0];
    return st;
}

/* Batched solve.
 *   coeffs  [dmax+1][n] complex128 (interleaved re, im), row k = a_k
 *   degrees [n] int32, or NULL meaning every polynomial has degree dmax
 *   roots   [dmax][n] complex128 out; NaN for rows k >= d_i
 *   status  [n] uint32 out
 *   iters   [dmax-1][n] int32 out or NULL; row m-2 = QR steps at level m
 *   cap     iterations per level before NOT_CONVERGED (<= 0: 30)
 *   fixed_t > 0: Alg. 2 literally, exactly fixed_t steps per level
 *   nthreads <= 0: OpenMP default
 */
void oracle_solve(const double *coeffs, const int32_t *degrees, int64_t n, int dmax,
                  double *roots, uint32_t *status, int32_t *iters, int cap,
                  unsigned flags, int fixed_t, int nthreads)
{
    if (cap <= 0)
        cap = 30;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int d = degrees ? degrees[i] : dmax;
        cplx a[ODMAX + 1], eig[ODMAX];
        int its[ODMAX];
        for (int k = 0; k < ODMAX; ++k) {
            eig[k] = NAN + I * NAN;
            its[k] = 0;
        }
        unsigned st;
        if (d < 1 || d > dmax) {
            st = OST_BAD_DEGREE;
        } else {
            for (int k = 0; k <= d; ++k)
                a[k] = coeffs[2 * (k * n + i)] + I * coeffs[2 * (k * n + i) + 1];
            st = solve_one(d, a, eig, its, cap, flags, fixed_t);
        }
        for (int k = 0; k < dmax; ++k) {
            cplx r = (k < d && d <= dmax) ? eig[k] : NAN + I * NAN;
            roots[2 * (k * n + i)] = creal(r);
            roots[2 * (k * n + i) + 1] = cimag(r);
        }
        if (iters)
            for (int k = 0; k < dmax - 1; ++k)
                iters[k * n + i] = its[k];
        status[i] = st;
    }
}

/* Roots-to-pixels (Sec. III): window [x0, x1) x [y0, y1) split into
 * width x height pixels, row 0 = lowest imaginary part.  For each root
 * u = (re - x0) * sx, v = (im - y0) * sy with sx = width / (x1 - x0) and
 * sy = height / (y1 - y0); the root counts iff 0 <= u < width and
 * 0 <= v < height (a NaN fails every comparison), in pixel
 * (floor(v), floor(u)).  Counts are added to hist (the caller zeroes it).
 * Polynomials with (status & skip_mask) != 0 are skipped; only rows
 * k < degree are read. */
void oracle_density(const double *roots, const int32_t *degrees, const uint32_t *status,
                    uint32_t skip_mask, int64_t n, int dmax, double x0, double x1,
                    double y0, double y1, int width, int height, int32_t *hist)
{
    double sx = (double)width / (x1 - x0);
    double sy = (double)height / (y1 - y0);
    for (int64_t i = 0; i < n; ++i) {
        if (status && (status[i] & skip_mask))
            continue;
        int d = degrees ? degrees[i] : dmax;
        if (d > dmax)
            d = dmax;
        for (int k = 0; k < d; ++k) {
            double re = roots[2 * (k * n + i)];
            double im = roots[2 * (k * n + i) + 1];
            double u = (re - x0) * sx;
            double v = (im - y0) * sy;
            if (u >= 0.0 && u < (double)width && v >= 0.0 && v < (double)height) {
                int iu = (int)u, iv = (int)v;
                hist[(int64_t)iv * width + iu] += 1;
            }
        }
    }
}

/* Roots-to-pixels for roots in local disk coordinates (the approximation
 * front-end, Sec. II-A): root w of polynomial i counts only if
 * |w|^2 < rmax2 (the zero lies in the disk where the polynomial approximates
 * f); it is placed at z = c_i + rho_i w and counted as in oracle_density. */
void oracle_density_local(const double *roots, const int32_t *degrees, const uint32_t *status,
                          uint32_t skip_mask, int64_t n, int dmax, const double *centers,
                          const double *radii, double rmax2, double x0, double x1, double y0,
                          double y1, int width, int height, int32_t *hist)
{
    double sx = (double)width / (x1 - x0);
    double sy = (double)height / (y1 - y0);
    for (int64_t i = 0; i < n; ++i) {
        if (status && (status[i] & skip_mask))
            continue;
        int d = degrees ? degrees[i] : dmax;
        if (d > dmax)
            d = dmax;
        for (int k = 0; k < d; ++k) {
            double wr = roots[2 * (k * n + i)], wi = roots[2 * (k * n + i) + 1];
            if (!(wr * wr + wi * wi < rmax2))
                continue;
            double re = centers[2 * i] + radii[i] * wr;
            double im = centers[2 * i + 1] + radii[i] * wi;
            double u = (re - x0) * sx;
            double v = (im - y0) * sy;
            if (u >= 0.0 && u < (double)width && v >= 0.0 && v < (double)height)
                hist[(int64_t)(int)v * width + (int)u] += 1;
        }
    }
}

/* Implicit-function adjoint.  At a simple root r of p(z) = sum_k a_k z^k,
 * p(r(a); a) = 0 gives dr/da_k = -r^k / p'(r).  For a real loss L with
 * cotangent g_r = dL/dRe r + i dL/dIm r, the cotangent of a_k (same
 * convention) is conj(dr/da_k) * g_r, summed over the roots.
 *   grad_coeffs [dmax+1][n] out, zero for rows k > d_i
 *   status [n] in/out: polynomials with BAD_DEGREE, NONFINITE or
 *   ZERO_LEADING get zero gradient; a root with p'(r) zero or non-finite
 *   contributes nothing and sets SINGULAR_DERIV. */
void oracle_backward(const double *coeffs, const int32_t *degrees, const double *roots,
                     const double *grad_roots, int64_t n, int dmax, double *grad_coeffs,
                     uint32_t *status, int nthreads)
{
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int64_t i = 0; i < n; ++i) {
        int d = degrees ? degrees[i] : dmax;
        cplx g[ODMAX + 1];
        for (int k = 0; k <= ODMAX; ++k)
            g[k] = 0.0;
        unsigned st = status[i];
        if (d >= 1 && d <= dmax && !(st & (OST_BAD_DEGREE | OST_NONFINITE | OST_ZERO_LEADING))) {
            cplx a[ODMAX + 1];
            for (int k = 0; k <= d; ++k)
                a[k] = coeffs[2 * (k * n + i)] + I * coeffs[2 * (k * n + i) + 1];
            for (int j = 0; j < d; ++j) {
                cplx r = roots[2 * (j * n + i)] + I * roots[2 * (j * n + i) + 1];
                cplx gr = grad_roots[2 * (j * n + i)] + I * grad_roots[2 * (j * n + i) + 1];
                /* p'(r) = sum_{k>=1} k a_k r^{k-1}, by Horner */
                cplx dp = d * a[d];
                for (int k = d - 1; k >= 1; --k)
                    dp = dp * r + k * a[k];
                if (!cfinite(dp) || dp == 0.0) {
                    st |= OST_SINGULAR_DERIV;
                    continue;
                }
                cplx rk = 1.0;
                for (int k = 0; k <= d; ++k) {
                    cplx drda = -rk / dp;
                    g[k] += conj(drda) * gr;
                    rk *= r;
                }
            }
        }
        for (int k = 0; k <= dmax; ++k) {
            grad_coeffs[2 * (k * n + i)] = creal(g[k]);
            grad_coeffs[2 * (k * n + i) + 1] = cimag(g[k]);
        }
        status[i] = st;
    }
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
