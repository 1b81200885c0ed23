/*
 * A plain C user of the library: nothing but include/proots.h, libproots.so
 * and the HIP runtime.  It solves polynomials whose roots are known exactly
 * (quarter-integer lattice points, so the expanded coefficients are exact
 * doubles) in both precision forms, checks that pr_solve_bin's image equals
 * pr_density's over the same roots, and checks pr_backward on linear
 * polynomials against the closed form dr/da_0 = -1/a_1, dr/da_1 = -r/a_1.
 * Exit status 0 and a final "ok" line on success.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "proots.h"

#define HIPCHECK(x)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) {                                                            \
            fprintf(stderr, "HIP error %d: %s\n", (int)e_, #x);                            \
            return 2;                                                                      \
        }                                                                                  \
    } while (0)
#define PRCHECK(x)                                                                         \
    do {                                                                                   \
        int rc_ = (x);                                                                     \
        if (rc_ != PR_OK) {                                                                \
            fprintf(stderr, "%s failed: %s\n", #x, pr_strerror(rc_));                      \
            return 3;                                                                      \
        }                                                                                  \
    } while (0)

enum { DMAX = 6 };

static pr_complex cmul(pr_complex a, pr_complex b)
{
    pr_complex c = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return c;
}

/* root k of polynomial i: distinct real parts (k - 2.5) / 4 */
static pr_complex true_root(int64_t i, int k)
{
    pr_complex z = {(k - 2.5) / 4.0, (double)((i * 7 + 3 * k) % 11 - 5) / 4.0};
    return z;
}

int main(void)
{
    const int64_t n = 10007;
    const double win[4] = {-1.0, 1.0, -1.5, 1.5};
    const int32_t W = 64, H = 96;
    pr_complex* coeffs = calloc((size_t)(DMAX + 1) * n, sizeof(pr_complex));
    pr_complex* roots = calloc((size_t)DMAX * n, sizeof(pr_complex));
    uint32_t* status = calloc((size_t)n, sizeof(uint32_t));
    int32_t* h1 = calloc((size_t)W * H, sizeof(int32_t));
    int32_t* h2 = calloc((size_t)W * H, sizeof(int32_t));
    if (!coeffs || !roots || !status || !h1 || !h2)
        return 4;
    for (int64_t i = 0; i < n; ++i) {
        pr_complex p[DMAX + 1];
        memset(p, 0, sizeof p);
        p[0].re = 1.0; /* p(z) = 1, then times (z - z_k) */
        for (int k = 0; k < DMAX; ++k) {
            const pr_complex z = true_root(i, k);
            pr_complex q[DMAX + 1];
            memset(q, 0, sizeof q);
            for (int j = 0; j <= k; ++j) {       /* q = p * z - p * z_k, p in ascending powers */
                pr_complex t = cmul(p[j], z);
                q[j + 1].re += p[j].re;
                q[j + 1].im += p[j].im;
                q[j].re -= t.re;
                q[j].im -= t.im;
            }
            memcpy(p, q, sizeof p);
        }
        for (int k = 0; k <= DMAX; ++k)
            coeffs[(int64_t)k * n + i] = p[k];
    }

    pr_complex *d_coeffs, *d_roots;
    uint32_t* d_status;
    int32_t *d_h1, *d_h2;
    HIPCHECK(hipMalloc((void**)&d_coeffs, sizeof(pr_complex) * (DMAX + 1) * n));
    HIPCHECK(hipMalloc((void**)&d_roots, sizeof(pr_complex) * DMAX * n));
    HIPCHECK(hipMalloc((void**)&d_status, sizeof(uint32_t) * n));
    HIPCHECK(hipMalloc((void**)&d_h1, sizeof(int32_t) * W * H));
    HIPCHECK(hipMalloc((void**)&d_h2, sizeof(int32_t) * W * H));
    HIPCHECK(hipMemcpy(d_coeffs, coeffs, sizeof(pr_complex) * (DMAX + 1) * n,
                       hipMemcpyHostToDevice));

    const int32_t precisions[2] = {PR_FP64, PR_FP32_POLISH};
    for (int pi = 0; pi < 2; ++pi) {
        pr_solve_opts o;
        memset(&o, 0, sizeof o);
        o.precision = precisions[pi];
        PRCHECK(pr_solve(d_coeffs, NULL, n, DMAX, d_roots, d_status, &o, NULL));
        HIPCHECK(hipMemcpy(roots, d_roots, sizeof(pr_complex) * DMAX * n, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(status, d_status, sizeof(uint32_t) * n, hipMemcpyDeviceToHost));
        double worst = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (status[i] != 0) {
                fprintf(stderr, "precision %d: polynomial %lld has status %u\n", precisions[pi],
                        (long long)i, status[i]);
                return 5;
            }
            int used[DMAX] = {0};
            for (int k = 0; k < DMAX; ++k) {   /* nearest true root, each used once */
                const pr_complex r = roots[(int64_t)k * n + i];
                int best = -1;
                double bd = INFINITY;
                for (int j = 0; j < DMAX; ++j) {
                    const pr_complex t = true_root(i, j);
                    const double d = hypot(r.re - t.re, r.im - t.im);
                    if (!used[j] && d < bd) {
                        bd = d;
                        best = j;
                    }
                }
                if (best < 0)
                    return 6;
                used[best] = 1;
                const pr_complex t = true_root(i, best);
                const double rel = bd / hypot(t.re, t.im);
                if (rel > worst)
                    worst = rel;
            }
        }
        if (!(worst <= 1e-12)) {
            fprintf(stderr, "precision %d: worst relative root error %.3e\n", precisions[pi],
                    worst);
            return 7;
        }
        /* one launch (solve + bin) against solve then density */
        HIPCHECK(hipMemset(d_h1, 0, sizeof(int32_t) * W * H));
        HIPCHECK(hipMemset(d_h2, 0, sizeof(int32_t) * W * H));
        PRCHECK(pr_density(d_roots, NULL, d_status, 0, n, DMAX, win[0], win[1], win[2], win[3], W,
                           H, d_h1, NULL));
        PRCHECK(pr_solve_bin(d_coeffs, NULL, n, DMAX, NULL, d_status, &o, 0, win[0], win[1],
                             win[2], win[3], W, H, d_h2, NULL));
        HIPCHECK(hipMemcpy(h1, d_h1, sizeof(int32_t) * W * H, hipMemcpyDeviceToHost));
        HIPCHECK(hipMemcpy(h2, d_h2, sizeof(int32_t) * W * H, hipMemcpyDeviceToHost));
        long total = 0;
        for (int p = 0; p < W * H; ++p) {
            if (h1[p] != h2[p]) {
                fprintf(stderr, "precision %d: images differ at pixel %d\n", precisions[pi], p);
                return 8;
            }
            total += h1[p];
        }
        printf("precision %d: worst root error %.2e, %ld roots binned, images equal\n",
               precisions[pi], worst, total);
    }

    /* backward on p(z) = a0 + a1 z: r = -a0/a1 */
    {
        const int64_t m = 1000;
        pr_complex* a = calloc((size_t)2 * m, sizeof(pr_complex));
        pr_complex* r = calloc((size_t)m, sizeof(pr_complex));
        pr_complex* g = calloc((size_t)m, sizeof(pr_complex));
        pr_complex* ga = calloc((size_t)2 * m, sizeof(pr_complex));
        if (!a || !r || !g || !ga)
            return 4;
        for (int64_t i = 0; i < m; ++i) {
            a[i].re = 0.5 + (double)(i % 13) / 8.0;
            a[i].im = -1.0 + (double)(i % 7) / 4.0;
            a[m + i].re = 1.0 + (double)(i % 5) / 4.0;
            a[m + i].im = 0.25 * (double)(i % 3);
            const pr_complex a1 = a[m + i];
            const double d2 = a1.re * a1.re + a1.im * a1.im;
            const pr_complex inv = {a1.re / d2, -a1.im / d2};    /* 1 / a1 */
            const pr_complex t = cmul(a[i], inv);
            r[i].re = -t.re;
            r[i].im = -t.im;
            g[i].re = 1.0 - (double)(i % 4) / 2.0;
            g[i].im = 0.5;
        }
        pr_complex *d_a, *d_r, *d_g, *d_ga;
        uint32_t* d_st;
        HIPCHECK(hipMalloc((void**)&d_a, sizeof(pr_complex) * 2 * m));
        HIPCHECK(hipMalloc((void**)&d_r, sizeof(pr_complex) * m));
        HIPCHECK(hipMalloc((void**)&d_g, sizeof(pr_complex) * m));
        HIPCHECK(hipMalloc((void**)&d_ga, sizeof(pr_complex) * 2 * m));
        HIPCHECK(hipMalloc((void**)&d_st, sizeof(uint32_t) * m));
        HIPCHECK(hipMemcpy(d_a, a, sizeof(pr_complex) * 2 * m, hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(d_r, r, sizeof(pr_complex) * m, hipMemcpyHostToDevice));
        HIPCHECK(hipMemcpy(d_g, g, sizeof(pr_complex) * m, hipMemcpyHostToDevice));
        HIPCHECK(hipMemset(d_st, 0, sizeof(uint32_t) * m));
        PRCHECK(pr_backward(d_a, NULL, d_r, d_g, m, 1, d_ga, d_st, NULL));
        HIPCHECK(hipMemcpy(ga, d_ga, sizeof(pr_complex) * 2 * m, hipMemcpyDeviceToHost));
        double worst = 0.0;
        for (int64_t i = 0; i < m; ++i) {
            const pr_complex a1 = a[m + i];
            const double d2 = a1.re * a1.re + a1.im * a1.im;
            const pr_complex inv = {a1.re / d2, -a1.im / d2};
            /* grad_a0 = conj(-1/a1) g, grad_a1 = conj(-r/a1) g */
            const pr_complex c0 = {-inv.re, inv.im};
            const pr_complex ra = cmul(r[i], inv);
            const pr_complex c1 = {-ra.re, ra.im};
            const pr_complex w0 = cmul(c0, g[i]), w1 = cmul(c1, g[i]);
            const double e0 = hypot(ga[i].re - w0.re, ga[i].im - w0.im) / hypot(w0.re, w0.im);
            const double e1 =
                hypot(ga[m + i].re - w1.re, ga[m + i].im - w1.im) / hypot(w1.re, w1.im);
            if (e0 > worst)
                worst = e0;
            if (e1 > worst)
                worst = e1;
        }
        if (!(worst <= 1e-13)) {
            fprintf(stderr, "backward: worst relative error %.3e\n", worst);
            return 9;
        }
        printf("backward: worst relative error %.2e\n", worst);
        hipFree(d_a);
        hipFree(d_r);
        hipFree(d_g);
        hipFree(d_ga);
        hipFree(d_st);
        free(a);
        free(r);
        free(g);
        free(ga);
    }
    hipFree(d_coeffs);
    hipFree(d_roots);
    hipFree(d_status);
    hipFree(d_h1);
    hipFree(d_h2);
    free(coeffs);
    free(roots);
    free(status);
    free(h1);
    free(h2);
    printf("ok\n");
    return 0;
}
