/*
 * proots.h -- C ABI of the batched polynomial-root library for AMD MI355X
 * (gfx950).
 *
 * The library computes, for a batch of complex polynomials of degree <= 6,
 * every root as an eigenvalue of the polynomial's Frobenius companion
 * matrix (Tang & Quan, arXiv 2507.02164, Sec. II-B) by single-shift QR
 * iteration (Alg. 1) realised with complex Givens rotations applied in
 * place, two rows then two columns at a time (Sec. II-C, loop shape of
 * Alg. 2), with bottom deflation.  The roots can then be counted into a
 * root-density image (Sec. III, roots converted to pixel coordinates and
 * accumulated in video memory), and root cotangents can be pulled back to
 * coefficient cotangents with the implicit-function adjoint (not in the
 * paper).
 *
 * Conventions shared by every call:
 *   - Every array pointer is a DEVICE pointer (hipMalloc'ed or equivalent),
 *     owned by the caller.  The library never allocates, frees or retains
 *     caller memory.
 *   - Complex numbers are pr_complex: two doubles (re, im), layout-identical
 *     to std::complex<double>, C99 double complex and torch.complex128.
 *   - Batched arrays are structures of arrays: element (k, i) of a [rows][n]
 *     array is at offset k * n + i.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call only
 *     enqueues work on it and returns; nothing synchronises the device.
 *   - With n == 0 nothing is enqueued and the per-polynomial array pointers
 *     may be NULL.  A batch may hold up to (2^31 - 1) * 64 polynomials
 *     (pr_solve, pr_solve_bin), (2^31 - 1) * 128 (pr_backward) or about
 *     (2^31 - 1) * 256 (the other calls); a larger n is an argument error.
 *   - The return value reports argument errors, detected on the host before
 *     anything is enqueued, and kernel-launch failures.  Numerical outcomes
 *     per polynomial are reported only through `status` bits, never as
 *     errors.
 *   - Calls are deterministic for identical inputs and options.
 *   - No call throws across the ABI.
 */
#ifndef PROOTS_H
#define PROOTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One complex double: (re, im). */
typedef struct pr_complex {
    double re;
    double im;
} pr_complex;

/* Return codes. */
enum pr_error {
    PR_OK = 0,
    PR_ERR_INVALID_ARG = -1,  /* a NULL pointer, n < 0, dmax out of range, bad window, ... */
    PR_ERR_UNSUPPORTED = -2,  /* option value the library does not implement */
    PR_ERR_HIP = -3,          /* the HIP runtime refused the launch */
    PR_ERR_NO_MEMORY = -4     /* the caller's workspace is missing or smaller than the call
                                 needs (the library itself never allocates) */
};

/* Per-polynomial status bits (uint32).  0 = every root computed normally. */
enum pr_status_bits {
    PR_ST_BAD_DEGREE = 1u << 0,        /* degree outside [1, dmax]; roots NaN */
    PR_ST_NONFINITE = 1u << 1,         /* some a_k (k <= degree) is Inf or NaN; roots NaN */
    PR_ST_ZERO_LEADING = 1u << 2,      /* a_degree == 0; roots NaN */
    PR_ST_NOT_CONVERGED = 1u << 3,     /* a level hit the iteration cap and was deflated anyway */
    PR_ST_POLISH_UNCONVERGED = 1u << 4,/* FP32 form: a Newton polish did not settle, or two
                                          polished roots coincide */
    PR_ST_SINGULAR_DERIV = 1u << 5,    /* backward: p'(r) zero or non-finite at some root; that
                                          root contributed nothing */
    PR_ST_RESOLVED_FP64 = 1u << 6      /* FP32 form with PR_FLAG_FP64_FALLBACK: the FP32 result
                                          was flagged, the polynomial was solved again in FP64,
                                          and its roots and other bits are the FP64 solve's */
};

/* Arithmetic of the QR sweeps. */
typedef enum pr_precision {
    PR_FP64 = 0,          /* sweeps, deflation test and roots in FP64 */
    PR_FP32_POLISH = 1    /* sweeps in FP32; deflation test in FP64; every root then polished
                             by Newton steps in FP64 on the original polynomial */
} pr_precision;

/* Option flags. */
enum pr_solve_flags {
    PR_FLAG_NO_EXCEPTIONAL_SHIFT = 1u << 0, /* debug: no exceptional shift (a polynomial such
                                               as z^d - c, d >= 3, then stalls to the cap) */
    PR_FLAG_FIXED_STEPS = 1u << 1,          /* Alg. 2 literally: every level takes exactly
                                               max_iter_per_level QR steps shifted by Alg. 1's
                                               bottom-right entry, no convergence test and no
                                               exceptional shift; NOT_CONVERGED is never set */
    PR_FLAG_FP64_FALLBACK = 1u << 2,        /* FP32 form: every polynomial whose FP32 result
                                               ends NOT_CONVERGED or POLISH_UNCONVERGED is
                                               solved again by the FP64 form (a second launch
                                               on the same stream that reads the status array
                                               and solves only those); its roots, status (with
                                               PR_ST_RESOLVED_FP64) and iteration counts are
                                               then the FP64 solve's in lock-step levels
                                               (PR_FLAG_RUN_AHEAD does not apply to this
                                               launch).  No effect on PR_FP64 */
    PR_FLAG_PAIRED_LANES = 1u << 4,         /* FP32 form, index-order launch (no tiles):
                                               each lane solves two polynomials, 64 apart,
                                               stepping both matrices in one level loop;
                                               the same arithmetic per polynomial as the
                                               one-per-lane launch (roots may differ in the
                                               last bits where the compiler fuses products
                                               differently).  Ignored by the FP64 form and
                                               tiled launches */
    PR_FLAG_RUN_AHEAD = 1u << 5,            /* one-per-lane launches (index order, and the
                                               sliced mixed-degree layout, grid_blocks 0):
                                               while a wave still steps level m for some
                                               lanes, the lanes already at level m - 1 take
                                               their level-(m-1) steps inside the same trips
                                               instead of idling (Sec. III's next-task
                                               scheduling, one level deep).  Same tests,
                                               shifts and steps per lane as without it, so
                                               roots, status and step counts agree up to
                                               rounding.  Ignored by the persistent tiled
                                               layout (grid_blocks > 0), by paired lanes
                                               and by the FP64 fallback's second launch */
    PR_FLAG_RAYLEIGH_SHIFT = 1u << 3        /* shift each QR step by Alg. 1's choice, the
                                               bottom-right entry itself.  Default: the
                                               eigenvalue of the trailing 2 x 2 block nearest
                                               that entry (Wilkinson's shift), one complex
                                               shift per step as well, with fewer steps per
                                               level (a 2 x 2 block deflates in one); where
                                               its value is not finite (FP32 entries beyond
                                               about 2^31) a step takes the bottom entry.
                                               The default also shifts each polynomial's
                                               first step by the root nearest 0 of
                                               b_0 + b_1 z + b_2 z^2 (b monic), where both
                                               rules would start from 0 */
};

/* Options of pr_solve.  Zero-initialised = defaults. */
typedef struct pr_solve_opts {
    int32_t precision;            /* pr_precision */
    int32_t max_iter_per_level;   /* QR steps per deflation level before NOT_CONVERGED;
                                     0 = 30; valid 1..1000 */
    int32_t polish_steps;         /* FP32 form: Newton steps per root; 0 = 2; valid 1..8 */
    uint32_t flags;               /* pr_solve_flags */
    double polish_tol;            /* FP32 form: POLISH_UNCONVERGED when the last Newton step
                                     exceeds polish_tol * |r|; 0 = 1e-6; valid (0, 1) */
    int32_t* iter_counts;         /* optional DEVICE array [dmax-1][n] (row m-2 = QR steps
                                     taken at level m), or NULL */
    int32_t tile;                 /* with a degrees array: polynomials are solved in tiles of
                                     this many consecutive indices, each sorted by degree
                                     (highest first) before it is cut into waves of 64, so
                                     that nearly every wave holds one degree (one launch);
                                     0 = library default (2048), -1 = no sorting (index order);
                                     valid -1..4096 */
    int32_t grid_blocks;          /* tiled launch: 0 = one one-wave block per 64 consecutive
                                     polynomials of a sorted tile (only a slice at a degree
                                     boundary mixes degrees); > 0 = that many persistent
                                     one-wave blocks walking the tiles, each degree of a tile
                                     cut into its own slices; valid >= 0 */
} pr_solve_opts;

/*
 * pr_solve -- roots of n polynomials.
 *
 *   coeffs   [dmax+1][n] pr_complex, row k = a_k of p_i(z) = sum_k a_k z^k.
 *            Rows above a polynomial's degree are ignored (they may hold
 *            anything, NaN included; a wave may read them for another lane
 *            whose degree is higher, but never uses them).  Any nonzero
 *            leading coefficient a_d is accepted (the polynomial is divided
 *            by it first, Sec. II-B).
 *   degrees  [n] int32 degree of each polynomial, or NULL (= all dmax).
 *   n        number of polynomials, >= 0 (0 = no work).
 *   dmax     1..6: row count of the arrays (coeffs has dmax+1 rows).
 *   roots    [dmax][n] pr_complex out: the roots in deflation order (the
 *            last diagonal entry found first, Alg. 1), NaN for rows >= the
 *            polynomial's degree.  Must not alias coeffs.
 *   status   [n] uint32 out: pr_status_bits.
 *   opts     NULL = defaults (FP64).
 * Range: a polynomial whose root-modulus bound lies outside [2^-3, 2^10]
 * (FP32 form) or [2^-24, 2^24] (FP64 form) is solved in
 * the variable w = z / 2^s (an exact power-of-two change of variable, s
 * from that bound) and its roots are returned as 2^s w; every other
 * polynomial is solved as given.
 * Errors: PR_ERR_INVALID_ARG for a NULL coeffs/roots/status, n < 0, dmax
 * outside 1..6 or an option out of range; PR_ERR_HIP if a launch fails.
 */
int pr_solve(const pr_complex* coeffs, const int32_t* degrees, int64_t n, int32_t dmax,
             pr_complex* roots, uint32_t* status, const pr_solve_opts* opts, void* stream);

/*
 * pr_density -- count roots into a root-density image (Sec. III: the roots
 * are converted to pixel coordinates and written into video memory).
 *
 * The window [x0, x1) x [y0, y1) of the complex plane is split into
 * width x height pixels; row 0 holds the lowest imaginary parts.  With
 * sx = width / (x1 - x0) and sy = height / (y1 - y0), computed once in FP64
 * on the host, a root z counts iff u = (Re z - x0) * sx and
 * v = (Im z - y0) * sy (each a correctly rounded FP64 subtract then
 * multiply, never fused) satisfy 0 <= u < width and 0 <= v < height; it
 * adds 1 to hist[floor(v)][floor(u)].  NaN roots never count.
 *
 *   roots      [dmax][n] pr_complex (as written by pr_solve).
 *   degrees    [n] int32 or NULL: only rows k < degree are read.
 *   status     [n] uint32 or NULL: polynomials with (status & skip_mask) != 0
 *              are skipped.
 *   hist       [height][width] int32, ACCUMULATED into (the caller zeroes it).
 * Errors: PR_ERR_INVALID_ARG for NULL roots/hist, n < 0, dmax outside 1..6,
 * non-finite window bounds, x1 <= x0, y1 <= y0, width or height <= 0, or an
 * image larger than 2^31 - 1 pixels; PR_ERR_HIP if a launch fails.
 */
int pr_density(const pr_complex* roots, const int32_t* degrees, const uint32_t* status,
               uint32_t skip_mask, int64_t n, int32_t dmax, double x0, double x1, double y0,
               double y1, int32_t width, int32_t height, int32_t* hist, void* stream);

/*
 * pr_density_sorted -- pr_density for roots spread over the image, counted
 * per image tile in on-chip memory (Sec. III: roots converted to pixel
 * coordinates and accumulated in video memory).
 *
 * Same arguments, pixel rule and result as pr_density: the counts added to
 * hist are identical bit for bit (every pixel decision is the same FP64
 * arithmetic and integer addition does not depend on order).  Instead of one
 * device-wide atomic per root, the roots' pixel indices are first grouped by
 * image tile (tiles of 2^14 consecutive row-major pixels) with a counting
 * sort into `workspace` (no atomics: the sorted order is deterministic), each
 * tile is counted in an on-chip histogram, and each pixel of the image is
 * updated once, by one thread.  This pays off
 * when the roots of neighbouring polynomials fall on different pixels (e.g.
 * random coefficients); for smooth families whose neighbours share pixels
 * pr_density, which adds each run of neighbours on one pixel with one
 * atomic, is faster.
 *
 *   workspace        DEVICE memory owned by the caller, 256-byte aligned,
 *                    of at least pr_density_sorted_workspace(n, dmax, width,
 *                    height) bytes; its contents on entry do not matter and
 *                    on return are unspecified.  Calls that share a
 *                    workspace must not overlap in time.
 *   workspace_bytes  its size in bytes.
 * Images of more than 2^24 pixels, and batches with dmax * n >= 2^31, need
 * no workspace (the required size is 0): they are counted as by pr_density.
 * Errors: those of pr_density; PR_ERR_NO_MEMORY when the workspace is NULL
 * or smaller than required, PR_ERR_INVALID_ARG when it is not 256-byte
 * aligned.  The call enqueues five kernels on `stream`.
 */
int pr_density_sorted(const pr_complex* roots, const int32_t* degrees, const uint32_t* status,
                      uint32_t skip_mask, int64_t n, int32_t dmax, double x0, double x1,
                      double y0, double y1, int32_t width, int32_t height, int32_t* hist,
                      void* workspace, int64_t workspace_bytes, void* stream);

/*
 * pr_density_sorted_workspace -- bytes of workspace pr_density_sorted needs
 * for n polynomials of row count dmax and a width x height image: about
 * 6 * dmax * n (a pixel index and a sorted 16-bit offset per root slot),
 * plus 64 KiB per partial tile histogram (at most the tile count plus 512)
 * and at most 512 KiB of per-tile bookkeeping.  0 when no workspace is
 * needed; PR_ERR_INVALID_ARG (negative) for n < 0, dmax outside 1..6, or an
 * empty or over-large image.  A HOST call: nothing is enqueued.
 */
int64_t pr_density_sorted_workspace(int64_t n, int32_t dmax, int32_t width, int32_t height);

/*
 * pr_density_sorted_noalloc -- pr_density_sorted without a workspace
 * argument, for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * Same arguments (less workspace and workspace_bytes), result and errors as
 * pr_density_sorted.  The workspace is instead a static array of 64 MiB
 * (2^26 bytes) in the library, one per GPU, held from the first call on
 * that GPU until the process ends; the call itself allocates nothing.  A
 * batch whose pr_density_sorted_workspace exceeds 2^26 bytes (about 1.2M
 * degree-6 polynomials for a 1920 x 1080 image) is refused with
 * PR_ERR_NO_MEMORY: split it into several calls on the same image.  PR_ERR_HIP if the array's device address cannot be
 * looked up.  Every call on one GPU uses that GPU's array (no state carries
 * from one call to the next: each region is written before it is read), so
 * calls that overlap in time on one GPU -- on different streams or from
 * different host threads -- race and must not be issued.
 */
int pr_density_sorted_noalloc(const pr_complex* roots, const int32_t* degrees,
                              const uint32_t* status, uint32_t skip_mask, int64_t n,
                              int32_t dmax, double x0, double x1, double y0, double y1,
                              int32_t width, int32_t height, int32_t* hist, void* stream);

/*
 * pr_solve_bin -- solve and count in one launch (Sec. III: each eigenvalue
 * goes straight from the solver to its pixel count, the roots need not be
 * kept).
 *
 * The result is that of pr_solve(coeffs, degrees, n, dmax, roots, status,
 * opts) followed by pr_density(roots, degrees, status, skip_mask, n, dmax,
 * x0, x1, y0, y1, width, height, hist) on the same stream: the same roots
 * and status, and the same counts added to hist, bit for bit (integer
 * addition does not depend on order).
 *
 *   coeffs, degrees, n, dmax, status, opts   as for pr_solve.
 *   roots      [dmax][n] pr_complex out as for pr_solve, or NULL: the roots
 *              are counted but not stored.
 *   skip_mask  polynomials whose final status has a bit of skip_mask set are
 *              not counted.
 *   x0..y1, width, height, hist   as for pr_density (hist is accumulated).
 * Errors: those of pr_solve (except that roots may be NULL) and of
 * pr_density; PR_ERR_HIP if a launch fails.
 */
int pr_solve_bin(const pr_complex* coeffs, const int32_t* degrees, int64_t n, int32_t dmax,
                 pr_complex* roots, uint32_t* status, const pr_solve_opts* opts,
                 uint32_t skip_mask, double x0, double x1, double y0, double y1, int32_t width,
                 int32_t height, int32_t* hist, void* stream);

/*
 * pr_backward -- coefficient cotangents from root cotangents.
 *
 * At a simple root r of p, p(r(a); a) = 0 gives dr/da_k = -r^k / p'(r).
 * With root cotangents in PyTorch's convention g_r = dL/dRe r + i dL/dIm r
 * of a real loss L, the coefficient cotangent is
 *     grad_a_k = sum_j conj(-r_j^k / p'(r_j)) * g_{r_j},   k = 0..degree,
 * and 0 for rows k > degree.
 *
 *   coeffs       [dmax+1][n], degrees [n] or NULL, roots [dmax][n] as for
 *                pr_solve (the roots are taken as given).
 *   grad_roots   [dmax][n] pr_complex root cotangents (rows >= degree unread).
 *   grad_coeffs  [dmax+1][n] pr_complex out.
 *   status       [n] uint32 in/out: polynomials with BAD_DEGREE, NONFINITE
 *                or ZERO_LEADING get zero gradient; a root where p'(r) is
 *                zero or non-finite contributes nothing and SINGULAR_DERIV
 *                is or-ed in.
 * Errors: PR_ERR_INVALID_ARG for a NULL array argument (other than degrees),
 * n < 0 or dmax outside 1..6; PR_ERR_HIP if a launch fails.
 */
int pr_backward(const pr_complex* coeffs, const int32_t* degrees, const pr_complex* roots,
                const pr_complex* grad_roots, int64_t n, int32_t dmax, pr_complex* grad_coeffs,
                uint32_t* status, void* stream);

/*
 * The polynomial-approximation front-end (Sec. II-A): a complex function f is
 * approximated on each small disk D_i = {c_i + rho_i w : |w| < 1} by the
 * polynomial g_i(w) = sum_{k<=degree} a_k w^k of least L2 error, with the
 * inner product <g, h> = integral over the unit disk of g(w) conj(h(w)) dA.
 * The normal equations G a = b have G_jk = <w^j, w^k> = pi/(j+1) delta_jk
 * and b_j = <f, w^j>, so a_j = (j+1)/pi * b_j.  b_j is computed by a product
 * quadrature in polar coordinates: nr Gauss-Legendre nodes in the radius
 * (weights carrying the r dr area factor) times nt equally spaced angles.
 * For f a polynomial of degree D the quadrature, and so the fit, is exact
 * when D + degree + 1 <= 2 nr - 1 and D + degree < nt.  Node q = ir * nt + it
 * sits at w_q = r_ir exp(2 pi i it / nt).
 *
 * pr_l2fit_nodes -- HOST call: the nr*nt quadrature nodes w_q (interleaved
 *   re, im: nodes[2q], nodes[2q+1]) and weights (including the r dr factor,
 *   summing to pi) at which the caller samples f(c_i + rho_i w_q).
 *   nodes [2*nr*nt] and weights [nr*nt] are HOST arrays owned by the caller.
 *   Errors: PR_ERR_INVALID_ARG for NULL arrays, nr outside 1..64 or nt
 *   outside 1..256.
 */
int pr_l2fit_nodes(int32_t nr, int32_t nt, double* nodes, double* weights);

/*
 * pr_l2fit -- coefficients of the degree-`degree` L2 approximation on each
 * of n disks, in the disk's local variable w.
 *   samples  [nr*nt][n] pr_complex: row q holds f at node w_q of every disk.
 *   coeffs   [dmax+1][n] pr_complex out (dmax = degree), ready for pr_solve
 *            (whose roots are then local w; pr_density_local maps them back).
 * Errors: PR_ERR_INVALID_ARG for NULL arrays, n < 0, degree outside 1..6,
 * nr outside 1..64 or nt outside 1..256; PR_ERR_HIP if a launch fails.
 */
int pr_l2fit(const pr_complex* samples, int64_t n, int32_t degree, int32_t nr, int32_t nt,
             pr_complex* coeffs, void* stream);

/*
 * pr_density_local -- pr_density for roots in local disk coordinates:
 * a root w of polynomial i counts only if |w|^2 < rmax2 (the zero lies in
 * the disk the polynomial approximates f on); it is mapped to
 * z = c_i + rho_i w (re and im each a correctly rounded FP64 multiply then
 * add) and binned exactly as pr_density bins z.
 *   centers [n] pr_complex c_i, radii [n] double rho_i (DEVICE arrays).
 * Other arguments and errors as pr_density; PR_ERR_INVALID_ARG also for
 * NULL centers/radii or rmax2 not > 0.
 */
int pr_density_local(const pr_complex* roots, const int32_t* degrees, const uint32_t* status,
                     uint32_t skip_mask, int64_t n, int32_t dmax, const pr_complex* centers,
                     const double* radii, double rmax2, double x0, double x1, double y0,
                     double y1, int32_t width, int32_t height, int32_t* hist, void* stream);

/* Static English text for a return code. */
const char* pr_strerror(int code);

/* Library version, major * 10000 + minor * 100 + patch. */
int pr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PROOTS_H */
