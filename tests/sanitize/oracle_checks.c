/* The oracle's entry points run under address and undefined-behaviour
 * sanitizers (the CPU test-suite compiles oracle.c with this file and runs
 * it): every code path -- both shift rules, the quadratic start, fixed-T,
 * no exceptional shift, invalid inputs, mixed degrees, density (plain and
 * local), backward and the exposed building blocks -- on inputs whose
 * results are known exactly or in closed form.  Prints "oracle checks ok"
 * and exits 0 when every check holds. */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

void oracle_solve(const double *coeffs, const int32_t *degrees, int64_t n, int dmax,
                  double *roots, uint32_t *status, int32_t *iters, int cap, unsigned flags,
                  int fixed_t, int nthreads);
void oracle_density(const double *roots, const int32_t *degrees, const uint32_t *status,
                    uint32_t skip_mask, int64_t n, int dmax, double x0, double x1, double y0,
                    double y1, int width, int height, int32_t *hist);
void oracle_density_local(const double *roots, const int32_t *degrees, const uint32_t *status,
                          uint32_t skip_mask, int64_t n, int dmax, const double *centers,
                          const double *radii, double rmax2, double x0, double x1, double y0,
                          double y1, int width, int height, int32_t *hist);
void oracle_backward(const double *coeffs, const int32_t *degrees, const double *roots,
                     const double *grad_roots, int64_t n, int dmax, double *grad_coeffs,
                     uint32_t *status, int nthreads);
void oracle_givens(const double *a, const double *b, double *c, double *s);
void oracle_qr_step(int m, double *H, const double *shift);
void oracle_wilkinson_shift(const double *a, const double *b, const double *c, const double *e,
                            double *mu);
int oracle_quadratic_start(const double *b0, const double *b1, const double *b2, double *z);

static int failures = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);               \
            ++failures;                                                       \
        }                                                                     \
    } while (0)

typedef double complex cplx;
enum { N = 8, DM = 6 };

/* Coefficients [DM+1][N] (interleaved) of prod_j (z - r_j) over the first d
 * roots, exact for quarter-integer lattice roots of small modulus. */
static void expand(double *coeffs, int i, int d, const cplx *r)
{
    cplx c[DM + 1] = {1.0};
    for (int j = 0; j < d; ++j) {
        for (int k = j + 1; k >= 1; --k)
            c[k] = c[k - 1] - r[j] * c[k];
        c[0] = -r[j] * c[0];
    }
    for (int k = 0; k <= DM; ++k) {
        cplx v = k <= d ? c[k] : 0.0;
        coeffs[2 * (k * N + i)] = creal(v);
        coeffs[2 * (k * N + i) + 1] = cimag(v);
    }
}

/* Largest distance from each true root to the nearest computed root. */
static double worst(const double *roots, int i, int d, const cplx *r)
{
    double w = 0.0;
    for (int j = 0; j < d; ++j) {
        double best = INFINITY;
        for (int k = 0; k < d; ++k) {
            cplx z = roots[2 * (k * N + i)] + I * roots[2 * (k * N + i) + 1];
            double e = cabs(z - r[j]);
            best = e < best ? e : best;
        }
        w = best > w ? best : w;
    }
    return w;
}

static void solve_paths(void)
{
    static const cplx lattice[N][DM] = {
        {0.25, -0.5, 0.75 + 0.25 * I, -1.0 - 0.5 * I, 0.5 * I, 1.25},
        {1.0, -1.0, 0.5 + 0.5 * I, 0.5 - 0.5 * I, -0.25 * I, 2.0},
        {-1.5, 0.25 + 1.0 * I, 0.0, 1.0 * I, -0.75, 0.5},
        {0.5, 0.75, 1.0, 1.25, -0.5 * I, -1.0 * I},
        {2.0 * I, -2.0 * I, 1.5, -1.5, 0.25, -0.25},
        {0.25 + 0.25 * I, -0.25 + 0.25 * I, 0.25 - 0.25 * I, -0.25 - 0.25 * I, 1.0, -1.0},
        {1.75, -0.25 * I, 0.5 + 1.0 * I, -1.25, 0.75 * I, 0.125},
        {0.5, -0.5, 1.5 * I, -1.5 * I, 1.0 + 1.0 * I, -1.0},
    };
    double coeffs[2 * (DM + 1) * N], roots[2 * DM * N];
    uint32_t st[N];
    int32_t its[(DM - 1) * N], deg[N];
    const unsigned rules[] = {0u, 0x8u, 0x8u | 0x10u};
    for (int i = 0; i < N; ++i) {
        deg[i] = 1 + i % DM;
        expand(coeffs, i, DM, lattice[i]);
    }
    for (int r = 0; r < 3; ++r) {
        oracle_solve(coeffs, NULL, N, DM, roots, st, its, 30, rules[r], 0, 1);
        for (int i = 0; i < N; ++i) {
            CHECK(st[i] == 0);
            CHECK(worst(roots, i, DM, lattice[i]) < 1e-12);
        }
    }
    /* mixed degrees: polynomial i keeps its first deg[i] roots */
    for (int i = 0; i < N; ++i)
        expand(coeffs, i, deg[i], lattice[i]);
    oracle_solve(coeffs, deg, N, DM, roots, st, its, 30, 0x18u, 0, 1);
    for (int i = 0; i < N; ++i) {
        CHECK(st[i] == 0);
        CHECK(worst(roots, i, deg[i], lattice[i]) < 1e-12);
        for (int k = deg[i]; k < DM; ++k)
            CHECK(isnan(roots[2 * (k * N + i)]));
    }
    /* fixed T: exactly T steps per level, no flags */
    for (int i = 0; i < N; ++i)
        expand(coeffs, i, DM, lattice[i]);
    oracle_solve(coeffs, NULL, N, DM, roots, st, its, 30, 0u, 10, 1);
    for (int k = 0; k < (DM - 1) * N; ++k)
        CHECK(its[k] == 10);
    for (int i = 0; i < N; ++i)
        CHECK(st[i] == 0);
    /* z^3 - 1 stalls without the exceptional shift, converges with it */
    double z3[2 * 4] = {-1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0};
    double r3[2 * 3];
    uint32_t s3;
    int32_t i3[2];
    oracle_solve(z3, NULL, 1, 3, r3, &s3, i3, 30, 0x1u, 0, 1);
    CHECK(s3 == 0x8u);
    oracle_solve(z3, NULL, 1, 3, r3, &s3, i3, 30, 0x8u | 0x10u, 0, 1);
    CHECK(s3 == 0);
    for (int k = 0; k < 3; ++k) {
        cplx z = r3[2 * k] + I * r3[2 * k + 1];
        CHECK(cabs(z * z * z - 1.0) < 1e-14);
    }
    /* invalid inputs: a NaN coefficient, a zero leading coefficient, degrees
     * 0 and 7 (dmax 6) */
    for (int i = 0; i < N; ++i)
        expand(coeffs, i, DM, lattice[i]);
    coeffs[2 * (2 * N + 0)] = NAN;
    coeffs[2 * (DM * N + 1)] = 0.0;
    int32_t bad[N] = {6, 6, 0, 7, 6, 6, 6, 6};
    oracle_solve(coeffs, bad, N, DM, roots, st, its, 30, 0u, 0, 1);
    CHECK(st[0] == 0x2u && st[1] == 0x4u && st[2] == 0x1u && st[3] == 0x1u && st[4] == 0);
    for (int k = 0; k < DM; ++k)
        CHECK(isnan(roots[2 * (k * N + 0)]) && isnan(roots[2 * (k * N + 2)]));
}

static void density_paths(void)
{
    /* roots on the window's edges and inside it, a NaN, and a skipped poly */
    double roots[2 * 2 * 3] = {
        /* row 0 */ -1.0, -1.0, 1.0, 0.0, 0.0, 0.0,
        /* row 1 */ NAN, 0.0, 0.999, 0.999, -0.999, 0.5};
    uint32_t st[3] = {0, 0, 0x8u};
    int32_t hist[4 * 4];
    memset(hist, 0, sizeof hist);
    oracle_density(roots, NULL, st, 0x8u, 3, 2, -1.0, 1.0, -1.0, 1.0, 4, 4, hist);
    /* counted: (-1,-1) -> pixel (0,0); (0.999,0.999) -> (3,3); poly 2 skipped;
     * (1, 0) is on the open edge and the NaN never counts */
    int total = 0;
    for (int k = 0; k < 16; ++k)
        total += hist[k];
    CHECK(total == 2 && hist[0] == 1 && hist[15] == 1);
    double centers[2 * 3] = {0.5, 0.5, -0.5, 0.0, 0.0, 0.0};
    double radii[3] = {0.25, 0.25, 1.0};
    memset(hist, 0, sizeof hist);
    oracle_density_local(roots, NULL, NULL, 0u, 3, 2, centers, radii, 1.0, -1.0, 1.0, -1.0, 1.0,
                         4, 4, hist);
    total = 0;
    for (int k = 0; k < 16; ++k)
        total += hist[k];
    /* kept: |w|^2 < 1 -- only (0,0) of poly 2, placed at 0 -> pixel (2,2)
     * and (-0.999, 0.5) of poly 2 (|w|^2 = 1.248... > 1, dropped) */
    CHECK(total == 1 && hist[2 * 4 + 2] == 1);
}

static void backward_paths(void)
{
    /* degree 1: r = -a0/a1, dr/da0 = -1/a1, dr/da1 = a0/a1^2 */
    const cplx a0 = 0.5 - 1.0 * I, a1 = 2.0 + 0.5 * I, g = 1.0 - 0.25 * I;
    double coeffs[4] = {creal(a0), cimag(a0), creal(a1), cimag(a1)};
    cplx r = -a0 / a1;
    double roots[2] = {creal(r), cimag(r)}, grad_r[2] = {creal(g), cimag(g)}, grad[4];
    uint32_t st = 0;
    oracle_backward(coeffs, NULL, roots, grad_r, 1, 1, grad, &st, 1);
    cplx g0 = grad[0] + I * grad[1], g1 = grad[2] + I * grad[3];
    CHECK(st == 0);
    CHECK(cabs(g0 - conj(-1.0 / a1) * g) < 1e-15);
    CHECK(cabs(g1 - conj(a0 / (a1 * a1)) * g) < 1e-15);
    /* a double root: p'(r) = 0 flags SINGULAR_DERIV */
    double c2[6] = {1.0, 0.0, -2.0, 0.0, 1.0, 0.0};
    double r2[4] = {1.0, 0.0, 1.0, 0.0}, gr2[4] = {1.0, 0.0, 1.0, 0.0}, gc2[6];
    st = 0;
    oracle_backward(c2, NULL, r2, gr2, 1, 2, gc2, &st, 1);
    CHECK(st == 0x20u);
}

static void building_blocks(void)
{
    double a[2] = {3.0, 0.0}, b[2] = {0.0, 4.0}, c[2], s[2];
    oracle_givens(a, b, c, s);
    CHECK(fabs(c[0] - 0.6) < 1e-16 && fabs(s[1] + 0.8) < 1e-16);
    double z[2] = {0.0, 0.0};
    oracle_givens(z, z, c, s);
    CHECK(c[0] == 1.0 && c[1] == 0.0 && s[0] == 0.0 && s[1] == 0.0);
    double H[2 * 9] = {1, 0, 2, 0, 3, 0, 1, 0, 4, 0, 5, 0, 0, 0, 1, 0, 6, 0}, sh[2] = {0.5, 0.25};
    double tr0 = H[0] + H[8] + H[16];
    oracle_qr_step(3, H, sh);
    CHECK(H[2 * 6] == 0.0 && H[2 * 6 + 1] == 0.0);          /* below the subdiagonal */
    CHECK(fabs(H[0] + H[8] + H[16] - tr0) < 1e-13);         /* the trace is kept */
    double e[2] = {1.0, 0.0}, zero[2] = {0.0, 0.0}, q[2] = {4.0, 0.0}, one[2] = {1.0, 0.0}, mu[2];
    oracle_wilkinson_shift(zero, q, one, zero, mu);
    CHECK(fabs(fabs(mu[0]) - 2.0) < 1e-15);
    oracle_wilkinson_shift(e, zero, zero, zero, mu);
    CHECK(mu[0] == 0.0 && mu[1] == 0.0);
    double b0[2] = {-6.0, 0.0}, b1[2] = {1.0, 0.0}, b2[2] = {1.0, 0.0}, zz[2];
    CHECK(oracle_quadratic_start(b0, b1, b2, zz) == 1);     /* z^2 + z - 6: roots 2, -3 */
    CHECK(fabs(zz[0] - 2.0) < 1e-15 && zz[1] == 0.0);
}

int main(void)
{
    solve_paths();
    density_paths();
    backward_paths();
    building_blocks();
    if (failures) {
        printf("%d oracle check(s) failed\n", failures);
        return 1;
    }
    printf("oracle checks ok\n");
    return 0;
}
