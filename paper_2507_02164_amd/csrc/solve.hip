// solve.hip -- batched polynomial roots by single-shift QR iteration on the
// Frobenius companion matrix, one polynomial per lane (gfx950).
//
// Method (arXiv 2507.02164):
//   Sec. II-B   the roots of z^d + b_{d-1} z^{d-1} + ... + b_0 are the
//               eigenvalues of its companion matrix; Alg. 1 finds them by
//               single-shift QR iteration with bottom deflation.
//   Sec. II-C   each QR step A - sI = QR, A <- RQ + sI is done in place:
//               complex Givens rotations [[c, s], [-conj s, conj c]] that map
//               (a, b) to (sqrt(|a|^2 + |b|^2), 0) are applied to two rows at
//               a time, then their conjugate transposes to two columns at a
//               time; the Appendix shows the matrix stays upper Hessenberg.
//
// GPU design:
//   * One polynomial per lane.  The active upper-Hessenberg matrix lives in
//     VGPRs as a band (on/above-diagonal entries plus the subdiagonal: 26
//     complex entries at degree 6).  Every index is a compile-time constant:
//     the level m is a template parameter and all loops are unrolled, so no
//     entry is ever addressed at run time (no scratch).
//   * Loops are trimmed to the band: in the row pass of rotation r only
//     columns r-1..m-1 of rows r-1, r are nonzero; in the column pass only
//     rows 0..r of columns r-1, r.  The entry a rotation annihilates is
//     stored as an exact zero and the diagonal entry it produces as the real
//     rho.  The skipped products are products with exact zeros, so this is
//     the same arithmetic as the dense loops of Alg. 2.
//   * The column rotation r-1 is applied right after the row rotation r (a
//     lag of one): it touches only rows <= r-1 and the entry (r-1, r-1)
//     that row rotation r has just finished, so every operation sees the
//     same operands as in the row-pass-then-column-pass order, while only
//     two Givens pairs are live at a time.
//   * Convergence (the paper uses a fixed count): level m deflates once
//     cabs1(h[m-1][m-2]) <= eps (cabs1(h[m-1][m-1]) + cabs1(h[m-2][m-2])),
//     evaluated in FP64, eps = 2^-52 for FP64 sweeps and 2^-23 for FP32
//     sweeps.  Exceptional shift s = h[m-1][m-1] + cabs1(h[m-1][m-2])
//     (0.75 + 0.5i) on the 10th and 20th step of a level; after `cap` steps
//     the level deflates anyway and NOT_CONVERGED is set.
//   * Shift (the paper takes the bottom-right entry): by default the
//     eigenvalue of the trailing 2 x 2 block nearest that entry (Wilkinson's
//     shift; still one complex shift per step, only its value differs: about
//     45 more instructions per step and a fifth fewer steps per polynomial,
//     a 2 x 2 block deflating in one), and, on each polynomial's very first
//     step, the root nearest 0 of b0 + b1 z + b2 z^2 (both rules would start
//     from 0).  PR_FLAG_RAYLEIGH_SHIFT and the fixed-step mode take the
//     bottom-right entry throughout.
//   * FP32 form: sweeps in FP32, test in FP64, then every root is polished
//     by Newton steps r <- r - p(r)/p'(r) in FP64 on the original
//     coefficients.
//   * Mixed degrees: polynomials are sorted by degree within tiles of
//     consecutive indices, so that nearly every wave holds one degree;
//     either one wave per 64 consecutive polynomials of a sorted tile
//     (solve_sliced_kernel, the default) or persistent waves walking the
//     tiles, each degree cut into its own slices (solve_tiled_kernel).
//   * Binning epilogue (Sec. III's roots-to-pixels path, optional): once
//     the status is final, the wave counts every lane's roots with merged
//     atomics -- the same decisions and counts as the density kernel over
//     the stored roots, without a second launch.  The FP32 form bins its
//     polished roots from registers.  The FP64 form keeps one pixel index
//     per deflated root in registers (kBinKeep: 6 more VGPRs, still 3 waves
//     per SIMD, and about 1% faster than reading stored roots back).  Only
//     the FP64 fallback launch, which re-solves a sparse subset, stores its
//     roots as they deflate and reads them back at the end (kBinReread: no
//     extra registers across the QR loops).  The matrix's diagonal cannot
//     stand in for the deflated roots: the identity steps of lanes that ride
//     along preserve values, not the sign of zeros or entries next to an
//     overflowed one.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "cplx.hpp"
#include "internal.hpp"

namespace proots {
namespace {

// One-wave blocks: a finished wave's slot refills at once (256-lane blocks
// measured 6% slower).
constexpr int kBlock = 64;

// ---------------------------------------------------------------- Givens
// (c, s) = (conj a, conj b) / rho, rho = sqrt(|a|^2 + |b|^2): the only pair
// for which the Sec. II-C rotation maps (a, b) to (rho, 0).  Computed
// branch-free (a branch here would split the fully unrolled QR step into
// basic blocks and stretch register lifetimes across them).  A pair whose
// |a|^2 + |b|^2 is zero -- or, in FP32, below the smallest normal number
// (both entries under about 1e-19) -- gets the identity instead (the
// caller's `go` mask): the identity is unitary too, so the eigenvalues are
// untouched and only that lane's step is skipped.  This lets FP32 use the
// hardware reciprocal square root directly (it is accurate to 1 ulp on
// normal inputs; the library routine adds a rescaling for subnormal ones).
// The price of branch-free code is the range: |a|^2 + |b|^2 must not
// overflow (entries below about 1e154 in FP64, 1e19 in FP32), otherwise NaN
// propagates and the level ends NOT_CONVERGED.
// FP64: the hardware estimate y0 refined once by the third-order series
// 1/sqrt(x) = y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3e^2/8 + ...), e = 1 - x y0^2,
// which takes its relative error eps to about 5 eps^3 / 16 (the estimate's
// eps measured at most 2^-24.2 on gfx950 over the whole normal range; the
// refined value is within 0.99 ulp, as the library routine); x must be
// positive and finite, which the `go` mask guarantees for every value used.
__device__ __forceinline__ double rsqrt_t(double x)
{
    const double y0 = __builtin_amdgcn_rsq(x);
    const double e = __builtin_fma(-x * y0, y0, 1.0);
    return __builtin_fma(y0 * e, __builtin_fma(e, 0.375, 0.5), y0);
}
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ bool rotates(double n2) { return n2 > 0.0; }
__device__ __forceinline__ bool rotates(float n2) { return n2 >= 0x1p-126f; }

// Scalar select on values already computed (a conditional operator on a
// struct, or on an expression, may be emitted as a branch).
template <typename T>
__device__ __forceinline__ T pick(bool p, T a, T b)
{
    return p ? a : b;
}

// (x, y) <- (c x + s y, -conj(s) x + conj(c) y): rows r-1, r (Alg. 2 row loop).
template <typename T>
__device__ __forceinline__ void rot_rows(cx<T>& x, cx<T>& y, cx<T> c, cx<T> s)
{
    T xr = x.re, xi = x.im, yr = y.re, yi = y.im;
    x.re = c.re * xr - c.im * xi + s.re * yr - s.im * yi;
    x.im = c.re * xi + c.im * xr + s.re * yi + s.im * yr;
    y.re = c.re * yr + c.im * yi - s.re * xr - s.im * xi;
    y.im = c.re * yi - c.im * yr - s.re * xi + s.im * xr;
}

// (x, y) <- (conj(c) x + conj(s) y, -s x + c y): columns r-1, r (Alg. 2 column loop).
template <typename T>
__device__ __forceinline__ void rot_cols(cx<T>& x, cx<T>& y, cx<T> c, cx<T> s)
{
    T xr = x.re, xi = x.im, yr = y.re, yi = y.im;
    x.re = c.re * xr + c.im * xi + s.re * yr + s.im * yi;
    x.im = c.re * xi - c.im * xr + s.re * yi - s.im * yr;
    y.re = c.re * yr - c.im * yi - s.re * xr + s.im * xi;
    y.im = c.re * yi + c.im * yr - s.re * xi - s.im * xr;
}

// rot_cols whose x is a diagonal entry receiving its last update of the QR
// step: the shift d is added back inside the same multiply-add chain
// (A <- RQ + sI without a separate pass over the diagonal).
template <typename T>
__device__ __forceinline__ void rot_cols_diag(cx<T>& x, cx<T>& y, cx<T> c, cx<T> s, cx<T> d)
{
    T xr = x.re, xi = x.im, yr = y.re, yi = y.im;
    x.re = d.re + c.re * xr + c.im * xi + s.re * yr + s.im * yi;
    x.im = d.im + c.re * xi - c.im * xr + s.re * yi - s.im * yr;
    y.re = c.re * yr - c.im * yi - s.re * xr + s.im * xi;
    y.im = c.re * yi + c.im * yr - s.re * xi - s.im * xr;
}

// Column rotation of the row whose left entry x a rotating lane has just
// annihilated (x == 0 exactly): (x, y) <- (conj(s) y, c y), 10 operations
// instead of 16.  A lane that did not rotate has (c, s) = (1, 0) and keeps
// its x, which need not be zero, by selection.  Used for the bottom row of
// the last column rotation, whose y is the last diagonal entry: the shift d
// is added back in the same chain.
template <typename T>
__device__ __forceinline__ void rot_cols_zero(cx<T>& x, cx<T>& y, cx<T> c, cx<T> s, bool go,
                                              cx<T> d)
{
    T yr = y.re, yi = y.im;
    const T xr = s.re * yr + s.im * yi;
    const T xi = s.re * yi - s.im * yr;
    x.re = pick(go, xr, x.re);
    x.im = pick(go, xi, x.im);
    y.re = d.re + c.re * yr - c.im * yi;
    y.im = d.im + c.re * yi + c.im * yr;
}

// The same inside the row loop, where y is also known: row rotation r has
// just made it the real rho (or left a zero pair alone), so for a lane with
// go = true (x, y) <- (conj(s) rho, c rho) takes 4 multiplies and 3 selects.
template <typename T>
__device__ __forceinline__ void rot_cols_zero_real(cx<T>& x, cx<T>& y, cx<T> c, cx<T> s, bool go)
{
    const T yr = y.re;
    x.re = pick(go, s.re * yr, x.re);
    x.im = pick(go, -s.im * yr, x.im);
    y.im = pick(go, c.im * yr, y.im);
    y.re = c.re * yr;  // (c, s) = (1, 0) when go is false
}

// One shifted QR step on the leading M x M block (Alg. 1 body via Sec. II-C),
// executed by every lane of the wave.  Lanes with act == false take the
// identity rotation (c, s) = (1, 0) and shift 0 throughout, which leaves
// the values of their matrix unchanged (1*x + 0*y == x for finite y; a zero
// may change sign); the entries a real rotation overwrites are selected.
// Running the step wave-uniformly, with no lane-divergent branch around it,
// matters: a divergent branch would keep
// the pre-step matrix of the lanes that skip it alive next to the post-step
// matrix of the lanes that take it, doubling the register footprint.
//
// AHEAD (run-ahead level loop): lanes with act && !act_last are one level
// below, M-1, and take the step of their leading (M-1) x (M-1) block inside
// this one.  Their last rotation (rows M-2, M-1) is the identity, and row and
// column M-1, which hold the root they have already emitted and its
// coupling, keep their values: the shift is neither taken from nor given
// back to h[M-1][M-1], and h[M-2][M-2], whose last update is then column
// rotation M-2, gets its shift back there.  The leading block goes through
// the same operations as in the level-(M-1) step; the entries of column M-1
// above it are rotated too, which changes nothing the lane still needs.
template <typename T, int DM, int M, bool AHEAD = false>
__device__ __forceinline__ void qr_step(cx<T> (&h)[DM][DM], cx<T> sh, bool act, bool act_last)
{
    // the shortened rotation of the annihilated row, inside the loop and at
    // its end; inside the loop in FP64 it measured 170 VGPRs instead of 160
    // (one wave per SIMD fewer), so FP64 takes the plain rotation there
    constexpr bool kZeroInLoop = std::is_same<T, float>::value;
    // shift of the bottom row (lanes at level M) and of the run-ahead lanes'
    // bottom row M-2 at its last update
    const cx<T> shl = AHEAD ? cx<T>{pick(act_last, sh.re, T(0)), pick(act_last, sh.im, T(0))} : sh;
    const cx<T> shb = AHEAD ? cx<T>{pick(act_last, T(0), sh.re), pick(act_last, T(0), sh.im)}
                            : cx<T>{T(0), T(0)};
#pragma unroll
    for (int i = 0; i < M; ++i) {
        const cx<T> si = (i == M - 1) ? shl : sh;
        h[i][i].re -= si.re;
        h[i][i].im -= si.im;
    }
    cx<T> cprev, sprev;
    bool goprev = false;
#pragma unroll
    for (int r = 1; r < M; ++r) {
        const cx<T> a = h[r - 1][r - 1], b = h[r][r - 1];
        const T n2 = a.re * a.re + a.im * a.im + b.re * b.re + b.im * b.im;
        const T inv = rsqrt_t(n2);
        // a lane rotates only if it acts this trip and (a, b) is not
        // (numerically) zero -- NaN fails the test too; otherwise
        // (c, s) = (1, 0) and both entries stay
        const bool go = (r == M - 1 ? act_last : act) && rotates(n2);
        // masking by arithmetic, two selects in all: a rotating lane takes
        // 1/rho and 0, a lane that keeps its entries 0 and 1, so that
        // c = conj(a)/rho or 1, s = conj(b)/rho or 0, and the rotation maps
        // (h[r-1][r-1], h[r][r-1]) to (rho, 0) or leaves them (their values;
        // an entry whose square overflowed would turn NaN, as its rotation
        // would anyway)
        const T ig = pick(go, inv, T(0));
        const T keep = pick(go, T(0), T(1));
        const cx<T> c = {a.re * ig + keep, -a.im * ig};
        const cx<T> s = {b.re * ig, -b.im * ig};
        h[r - 1][r - 1] = {n2 * ig + keep * a.re, keep * a.im};
        h[r][r - 1] = {keep * b.re, keep * b.im};
#pragma unroll
        for (int j = r; j < M; ++j)
            rot_rows(h[r - 1][j], h[r][j], c, s);
        if (r >= 2) {
            // lagged column rotation r-1 on rows 0..r-1 (row r-1 enters with
            // h[r-1][r-2] == 0 for lanes that took row rotation r-1)
            // AHEAD, last one: row M-2's diagonal entry is complex for the
            // run-ahead lanes (their row rotation M-1 was the identity) and
            // takes its last update here, with their shift
            const bool kAheadLast = AHEAD && r == M - 1;
#pragma unroll
            for (int j = 0; j < (kZeroInLoop || kAheadLast ? r - 1 : r); ++j) {
                if (j == r - 2)  // h[r-2][r-2] takes its last update: add the shift back
                    rot_cols_diag(h[j][r - 2], h[j][r - 1], cprev, sprev, sh);
                else
                    rot_cols(h[j][r - 2], h[j][r - 1], cprev, sprev);
            }
            if (kAheadLast)
                rot_cols_zero(h[r - 1][r - 2], h[r - 1][r - 1], cprev, sprev, goprev, shb);
            else if (kZeroInLoop)
                rot_cols_zero_real(h[r - 1][r - 2], h[r - 1][r - 1], cprev, sprev, goprev);
        }
        cprev = c;
        sprev = s;
        goprev = go;
    }
#pragma unroll
    for (int j = 0; j < M - 2; ++j)
        rot_cols(h[j][M - 2], h[j][M - 1], cprev, sprev);
    rot_cols_diag(h[M - 2][M - 2], h[M - 2][M - 1], cprev, sprev, shl);
    rot_cols_zero(h[M - 1][M - 2], h[M - 1][M - 1], cprev, sprev, goprev, shl);
    // every diagonal entry got the shift back in its last update above
}

// Wilkinson's shift: the eigenvalue of [[a, b], [c, e]] nearest e.  With
// D = a - e the eigenvalues are e + (D + R)/2 and e + (D - R)/2, R^2 =
// D^2 + 4 b c; taking R on the side of D (Re(conj(D) R) >= 0, so
// |D + R| >= |D - R|), the nearer one is e + (D - R)/2, evaluated as it
// stands, without the division of the cancellation-free form: near
// convergence D and R nearly cancel and the shift is then off by about the
// rounding of |D|, no worse than e itself, and it measured the same steps
// per level as the divided form in both precisions.  The square root of
// q = D^2 + 4bc: w = sqrt((|q| + |Re q|)/2) and v = Im q / (2w), as (w, v)
// for Re q >= 0 and (v, w) otherwise (both square to q, without
// cancellation).  Where |q|^2 overflows (entries beyond about 2^31 in FP32)
// the result is not finite and the caller takes e instead.
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x)
{
    return x > 0.0 ? x * rsqrt_t(x) : 0.0;  // x == +inf gives NaN: not finite, as wanted
}
// Reciprocal for a shift's value (accuracy of a few ulp is plenty): the
// hardware estimate, refined once in FP64.  0 gives +inf, which the callers
// reject as not finite.
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x)
{
    const double y0 = __builtin_amdgcn_rcp(x);
    return __builtin_fma(y0, __builtin_fma(-x, y0, 1.0), y0);
}
template <typename T>
__device__ __forceinline__ cx<T> wilkinson(cx<T> a, cx<T> b, cx<T> c, cx<T> e)
{
    const T dr = a.re - e.re, di = a.im - e.im;
    const T qr = dr * dr - di * di + T(4) * (b.re * c.re - b.im * c.im);
    const T qi = T(2) * dr * di + T(4) * (b.re * c.im + b.im * c.re);
    const T u = (sqrt_t(qr * qr + qi * qi) + abs_t(qr)) * T(0.5);
    const T iw = pick(u > T(0), rsqrt_t(u), T(0));
    const T w = u * iw, v = qi * T(0.5) * iw;
    const bool pos = qr >= T(0);
    T rr = pick(pos, w, v), ri = pick(pos, v, w);
    const bool flip = dr * rr + di * ri < T(0);
    rr = pick(flip, -rr, rr);
    ri = pick(flip, -ri, ri);
    return {e.re + T(0.5) * (dr - rr), e.im + T(0.5) * (di - ri)};
}

// First shift of a polynomial (default shift rule): the root nearest 0 of
// b0 + b1 z + b2 z^2, b the monic coefficients, an estimate of the smallest
// root -- the eigenvalue the first unshifted steps would isolate slowly (the
// trailing block of the companion matrix is [[0, 0], [1, 0]], so the
// bottom-entry and Wilkinson shifts both start at 0).  The roots are
// 2 b0 / (-b1 -+ D), D^2 = b1^2 - 4 b0 b2; the denominator of larger modulus,
// -b1 - D with Re(conj(b1) D) >= 0, gives the smaller root.  D is taken as in
// `wilkinson`.  ok is false where the denominator is zero or the value is
// not finite; the caller then keeps the other shift (0 at this point, the
// root when b0 == 0).
template <typename T>
__device__ __forceinline__ cx<T> quad_start(cx<T> b0, cx<T> b1, cx<T> b2, bool& ok)
{
    const T qr = b1.re * b1.re - b1.im * b1.im - T(4) * (b0.re * b2.re - b0.im * b2.im);
    const T qi = T(2) * b1.re * b1.im - T(4) * (b0.re * b2.im + b0.im * b2.re);
    const T u = (sqrt_t(qr * qr + qi * qi) + abs_t(qr)) * T(0.5);
    const T iw = pick(u > T(0), rsqrt_t(u), T(0));
    const T w = u * iw, v = qi * T(0.5) * iw;
    const bool pos = qr >= T(0);
    T dr = pick(pos, w, v), di = pick(pos, v, w);
    const bool flip = b1.re * dr + b1.im * di < T(0);
    dr = pick(flip, -dr, dr);
    di = pick(flip, -di, di);
    const T er = -b1.re - dr, ei = -b1.im - di;
    const T n = er * er + ei * ei;
    const T g = T(2) * rcp_t(n);
    const cx<T> z = {(b0.re * er + b0.im * ei) * g, (b0.im * er - b0.re * ei) * g};
    ok = n > T(0) && __builtin_isfinite(z.re) && __builtin_isfinite(z.im);
    return z;
}

template <typename T>
struct Eps;
template <>
struct Eps<double> {
    static constexpr double v = 0x1p-52;
};
template <>
struct Eps<float> {
    static constexpr double v = 0x1p-23;
};

// One trip at level M (wave-uniform).  A lane at level M whose bottom
// subdiagonal entry is negligible, or that has used up its steps, deflates:
// h[M-1][M-1] goes to `emit`, the step count is recorded and the lane drops
// to level M-1.  Every other lane at level M takes one shifted QR step; lanes
// below level M ride along with the identity.
template <typename T, int DM, int M, typename Emit>
__device__ __forceinline__ void trip(cx<T> (&h)[DM][DM], int& m, int& its, int d, int cap,
                                     bool exc, bool fixed, bool wilk, uint32_t& st,
                                     int32_t* __restrict__ iters, int64_t n, int64_t i,
                                     Emit&& emit)
{
    const bool here = m == M;
    const double hh = cabs1_d(h[M - 1][M - 2]);
    const double tt = cabs1_d(h[M - 1][M - 1]) + cabs1_d(h[M - 2][M - 2]);
    // fixed-step mode (Alg. 2): no test, exactly `cap` steps per level
    const bool conv = !fixed && hh <= Eps<T>::v * tt;
    const bool done = here && (conv || its == cap);
    if (done) {
        if (!conv && !fixed)
            st |= PR_ST_NOT_CONVERGED;
        if (iters)
            iters[(int64_t)(M - 2) * n + i] = its;
        emit(M - 1, h[M - 1][M - 1]);
    }
    const bool act = here && !done;
    const bool ex = exc && (its == 10 || its == 20);
    const bool first = here && its == 0 && d == M;
    m = done ? M - 1 : m;
    its = done ? 0 : its + (act ? 1 : 0);
    // The trip in which a level's last lane deflates has no lane left to
    // step: the whole step, shift included, is skipped (a wave-uniform
    // branch; the matrix is left as it is, as the masked step would leave it).
    if (!__ballot(act))
        return;
    cx<T> mu = h[M - 1][M - 1];
    if (wilk) {  // wave-uniform: a scalar branch
        const cx<T> w = wilkinson(h[M - 2][M - 2], h[M - 2][M - 1], h[M - 1][M - 2], mu);
        const bool fin = __builtin_isfinite(w.re) && __builtin_isfinite(w.im);
        mu = {pick(fin, w.re, mu.re), pick(fin, w.im, mu.im)};
        // the polynomial's first step: its companion row is untouched (the
        // identity steps of the levels above keep values), h[0][M-1-k] =
        // -b_k of the (scaled) monic polynomial
        if (__ballot(first)) {  // wave-uniform
            const cx<T> b0 = {-h[0][M - 1].re, -h[0][M - 1].im};
            const cx<T> b1 = {-h[0][M - 2].re, -h[0][M - 2].im};
            cx<T> b2 = {T(1), T(0)};
            if constexpr (M >= 3)
                b2 = {-h[0][M - 3].re, -h[0][M - 3].im};
            bool ok;
            const cx<T> z = quad_start(b0, b1, b2, ok);
            const bool take = first && ok;
            mu = {pick(take, z.re, mu.re), pick(take, z.im, mu.im)};
        }
    }
    // the exceptional shift (10th and 20th step of a level), computed in
    // FP64 only when some lane of the wave takes it
    if (__ballot(ex && act)) {  // wave-uniform
        const T ere = (T)((double)h[M - 1][M - 1].re + hh * 0.75);
        const T eim = (T)((double)h[M - 1][M - 1].im + hh * 0.5);
        mu = {pick(ex, ere, mu.re), pick(ex, eim, mu.im)};
    }
    const cx<T> sh = {pick(act, mu.re, T(0)), pick(act, mu.im, T(0))};
    qr_step<T, DM, M>(h, sh, act, act);
}

// A trip with run-ahead lanes (M >= 4).  As `trip` for the lanes at level
// M; the lanes at level L = M-1 -- those already there and those that have
// just deflated in this trip -- are not idle: they take the deflation test
// and the shifted step of level L, on their leading block (see qr_step).  A
// lane that deflated early thus gets on with its next level while the
// wave's slower lanes finish this one.  Each lane takes exactly the tests,
// shifts and steps it takes in lock-step, in the same order; only the trip
// it takes them in changes.  (Levels 3 and 2 keep lock-step trips: their
// steps are cheap enough that the second test and the selects below would
// cost more than their idle lanes.)
template <typename T, int DM, int M, typename Emit>
__device__ __forceinline__ void trip_ahead(cx<T> (&h)[DM][DM], int& m, int& its, int d, int cap,
                                           bool exc, bool fixed, bool wilk, uint32_t& st,
                                           int32_t* __restrict__ iters, int64_t n, int64_t i,
                                           Emit&& emit)
{
    static_assert(M >= 4, "run-ahead trips are taken from level 4 up");
    constexpr int L = M - 1;
    const bool here = m == M;
    const double hh = cabs1_d(h[M - 1][M - 2]);
    const double tt = cabs1_d(h[M - 1][M - 1]) + cabs1_d(h[M - 2][M - 2]);
    // fixed-step mode (Alg. 2): no test, exactly `cap` steps per level
    const bool conv = !fixed && hh <= Eps<T>::v * tt;
    const bool done = here && (conv || its == cap);
    if (done) {
        if (!conv && !fixed)
            st |= PR_ST_NOT_CONVERGED;
        if (iters)
            iters[(int64_t)(M - 2) * n + i] = its;
        emit(M - 1, h[M - 1][M - 1]);
    }
    // the lanes at level L and their test there (itb: their steps at L)
    const bool below = m == L || done;
    const int itb = done ? 0 : its;
    const double hhb = cabs1_d(h[L - 1][L - 2]);
    const double ttb = cabs1_d(h[L - 1][L - 1]) + cabs1_d(h[L - 2][L - 2]);
    const bool convb = !fixed && hhb <= Eps<T>::v * ttb;
    const bool done_b = below && (convb || itb == cap);
    if (done_b) {
        if (!convb && !fixed)
            st |= PR_ST_NOT_CONVERGED;
        if (iters)
            iters[(int64_t)(L - 2) * n + i] = itb;
        emit(L - 1, h[L - 1][L - 1]);
    }
    const bool act = here && !done;
    const bool act_b = below && !done_b;
    const bool stp = act || act_b;
    const int its_s = act_b ? itb : its;  // steps taken so far at the level stepped
    const bool ex = exc && (its_s == 10 || its_s == 20);
    const bool first = its_s == 0 && ((act && d == M) || (act_b && d == L));
    m = done_b ? L - 1 : (done ? M - 1 : m);
    its = done_b ? 0 : (stp ? its_s + 1 : (done ? 0 : its));
    if (!__ballot(stp))
        return;
    // the trailing 2 x 2 block [[p, q], [c, e]] of the level the lane steps
    const cx<T> p = {pick(act_b, h[L - 2][L - 2].re, h[M - 2][M - 2].re),
                     pick(act_b, h[L - 2][L - 2].im, h[M - 2][M - 2].im)};
    const cx<T> q = {pick(act_b, h[L - 2][L - 1].re, h[M - 2][M - 1].re),
                     pick(act_b, h[L - 2][L - 1].im, h[M - 2][M - 1].im)};
    const cx<T> c = {pick(act_b, h[L - 1][L - 2].re, h[M - 1][M - 2].re),
                     pick(act_b, h[L - 1][L - 2].im, h[M - 1][M - 2].im)};
    const cx<T> e = {pick(act_b, h[L - 1][L - 1].re, h[M - 1][M - 1].re),
                     pick(act_b, h[L - 1][L - 1].im, h[M - 1][M - 1].im)};
    cx<T> mu = e;
    if (wilk) {  // wave-uniform: a scalar branch
        const cx<T> w = wilkinson(p, q, c, mu);
        const bool fin = __builtin_isfinite(w.re) && __builtin_isfinite(w.im);
        mu = {pick(fin, w.re, mu.re), pick(fin, w.im, mu.im)};
        // the polynomial's first step (see trip), at the level stepped: the
        // companion row of degree k holds h[0][k-1-j] = -b_j
        if (__ballot(first)) {  // wave-uniform
            const cx<T> b0 = {pick(act_b, -h[0][L - 1].re, -h[0][M - 1].re),
                              pick(act_b, -h[0][L - 1].im, -h[0][M - 1].im)};
            const cx<T> b1 = {pick(act_b, -h[0][L - 2].re, -h[0][M - 2].re),
                              pick(act_b, -h[0][L - 2].im, -h[0][M - 2].im)};
            const cx<T> b2 = {pick(act_b, -h[0][L - 3].re, -h[0][M - 3].re),
                              pick(act_b, -h[0][L - 3].im, -h[0][M - 3].im)};
            bool ok;
            const cx<T> z = quad_start(b0, b1, b2, ok);
            const bool take = first && ok;
            mu = {pick(take, z.re, mu.re), pick(take, z.im, mu.im)};
        }
    }
    // the exceptional shift (10th and 20th step of a level)
    if (__ballot(ex && stp)) {  // wave-uniform
        const double hx = act_b ? hhb : hh;
        const T ere = (T)((double)e.re + hx * 0.75);
        const T eim = (T)((double)e.im + hx * 0.5);
        mu = {pick(ex, ere, mu.re), pick(ex, eim, mu.im)};
    }
    const cx<T> sh = {pick(stp, mu.re, T(0)), pick(stp, mu.im, T(0))};
    qr_step<T, DM, M, true>(h, sh, stp, act);
}

// Alg. 1's level loop for a wave of independent lanes, level by level: the
// wave keeps taking trips at level M while any of its lanes is still at
// level M (a wave-uniform condition), then moves on to M-1.  Lanes that
// deflate early, or whose degree is below M, ride along with the identity --
// or, with AHEAD, run one level ahead (see trip_ahead).  Keeping the wave
// level-synchronous wastes less work on lane divergence than letting every
// lane run its own level (a trip would then execute the union of the levels
// present), and a separate loop per level lets each loop carry only its own
// M x M block in registers.  The loop body holds two trips (with the
// wave-uniform exit test between them): a one-trip body ends with the
// rotated entries in other registers than it started with, and the copies
// back at the loop edge cost both instructions and, above all, registers;
// over two trips the register assignment closes up.
template <typename T, int DM, int M, bool AHEAD, typename Emit>
__device__ __forceinline__ void iterate_from(cx<T> (&h)[DM][DM], int& m, int& its, int d, int cap,
                                             bool exc, bool fixed, bool wilk, uint32_t& st,
                                             int32_t* __restrict__ iters, int64_t n, int64_t i,
                                             Emit&& emit)
{
    if constexpr (M >= 2) {
        if constexpr (AHEAD && M >= 4) {
            while (__ballot(m == M)) {
                trip_ahead<T, DM, M>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i, emit);
                if (!__ballot(m == M))
                    break;
                trip_ahead<T, DM, M>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i, emit);
            }
        } else {
            while (__ballot(m == M)) {
                trip<T, DM, M>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i, emit);
                if (!__ballot(m == M))
                    break;
                trip<T, DM, M>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i, emit);
            }
        }
        iterate_from<T, DM, M - 1, AHEAD>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i,
                                          emit);
    }
}

template <typename T, int DM, bool AHEAD, typename Emit>
__device__ __forceinline__ void iterate(cx<T> (&h)[DM][DM], int d, int cap, bool exc,
                                        bool fixed, bool wilk, uint32_t& st,
                                        int32_t* __restrict__ iters, int64_t n, int64_t i,
                                        Emit&& emit)
{
    int m = d, its = 0;
    iterate_from<T, DM, DM, AHEAD>(h, m, its, d, cap, exc, fixed, wilk, st, iters, n, i, emit);
}

// Companion matrix, first-row form: h[0][j] = -b_{d-1-j} for j < d, ones on
// the subdiagonal of the leading d x d block -- of the scaled polynomial
// q(w) = p(2^s w) / 2^(s d), i.e. h[0][j] = -b_{d-1-j} 2^(-s (j+1)) (exact:
// a power-of-two scale), whose roots are w = z / 2^s.  Built from value
// selects on the run-time degree, so every matrix entry is written at a
// fixed location (a store whose address depended on d would force the
// matrix out of registers).
template <typename T, int DM>
__device__ __forceinline__ void companion(cx<T> (&h)[DM][DM], int d,
                                          const cx<double> (&b)[DM + 1], int s)
{
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        cx<double> v = {0.0, 0.0};
#pragma unroll
        for (int D = j + 1; D <= DM; ++D)
            if (d == D)
                v = b[D - 1 - j];
        const int e = -s * (j + 1);
        h[0][j] = {(T)(-__builtin_ldexp(v.re, e)), (T)(-__builtin_ldexp(v.im, e))};
    }
#pragma unroll
    for (int i = 1; i < DM; ++i)
        h[i][i - 1] = {i < d ? T(1) : T(0), T(0)};
}

// Range of the sweeps.  The Givens pair squares matrix entries, so FP32
// sweeps overflow for entries beyond about 2^63 and lose tiny ones below
// about 2^-63 (FP64: 2^511), and a companion matrix whose first row spans
// many binades loses relative accuracy on its small roots.  A polynomial
// whose root bound lies outside [2^lo, 2^hi] of FreeRange (FP32: 2^-3 ..
// 2^10, FP64: 2^-24 .. 2^24) is therefore solved as q(w) = p(2^s w) / 2^(s d), with s
// the exponent of a bound on its root moduli (Fujiwara: |z| <= 2 max_k
// |b_{d-k}|^(1/k)), so that the sweeps see roots of modulus about 1; the
// roots come back as z = 2^s w, exactly.  Ordinary polynomials get s = 0 and
// the very same arithmetic as without scaling.  s need not be exact (any
// power of two scales exactly), so the k-th roots use the hardware
// reciprocal estimate.
template <typename T>
struct FreeRange;
template <>
struct FreeRange<float> {  // below 2^-3 FP32 sweeps lose the small roots' digits
    static constexpr int lo = -3, hi = 10;
};
template <>
struct FreeRange<double> {
    static constexpr int lo = -24, hi = 24;
};

template <typename T, int DM>
__device__ __forceinline__ int root_scale(const cx<double> (&b)[DM + 1], int d)
{
    float bound = -1e30f;  // log2 of the root bound, up to rounding
#pragma unroll
    for (int j = 0; j < DM; ++j) {
        const double m = cabs1_d(b[j]);
        if (j < d && m > 0.0) {
            const float k = (float)(d - j);  // b_j = b_{d-k}
            const float e = (float)(__builtin_amdgcn_frexp_exp(m) + 1);  // >= log2(2m)
            bound = fmaxf(bound, e * __builtin_amdgcn_rcpf(k));
        }
    }
    const int s = bound > -1e29f ? (int)ceilf(bound) : 0;
    return (s > FreeRange<T>::hi || s < FreeRange<T>::lo) ? s : 0;
}

// Load a_0..a_d (zeros above d), validate, and normalise to b = a / a_d.
template <int DM>
__device__ __forceinline__ uint32_t load_poly(const double2* __restrict__ coeffs, int64_t n,
                                              int64_t i, int d, cx<double> (&a)[DM + 1],
                                              cx<double> (&b)[DM + 1])
{
    uint32_t st = 0;
    cx<double> lead = {0.0, 0.0};
    // Each row that some lane of the wave needs is read by every lane, and
    // the rows above a lane's degree are ignored: the loads sit under
    // wave-uniform conditions only, so they are all in flight before the
    // first is used (a load per row under its own lane condition waited for
    // each one), and rows above every lane's degree are not read at all.
    double2 v[DM + 1];
#pragma unroll
    for (int k = 0; k <= DM; ++k) {
        v[k] = make_double2(0.0, 0.0);
        if (__ballot(k <= d))
            v[k] = coeffs[(int64_t)k * n + i];
    }
#pragma unroll
    for (int k = 0; k <= DM; ++k) {
        const bool in = k <= d;
        a[k] = {in ? v[k].x : 0.0, in ? v[k].y : 0.0};
        if (in && !finite(a[k]))
            st |= PR_ST_NONFINITE;
        if (k == d)
            lead = a[k];
    }
    if (!st && lead.re == 0.0 && lead.im == 0.0)
        st |= PR_ST_ZERO_LEADING;
    const bool monic = lead.re == 1.0 && lead.im == 0.0;
#pragma unroll
    for (int k = 0; k <= DM; ++k)
        b[k] = (k < d && !monic && !st) ? cdiv(a[k], lead) : a[k];
    return st;
}

// Newton polish in FP64 on the original coefficients a (zeros above the
// degree, so Horner from DM gives the same value as from the degree):
// r <- r - p(r) / p'(r), a step skipped where |p'(r)|^2 is zero, subnormal
// or not finite (and then counted as unconverged unless p(r) == 0).
// The roots K0..K0+G-1 are polished together: their Horner recurrences are
// independent, and interleaving them hides the FP64 multiply-add latency
// that a single chain would wait on.  The step needs 1/|p'|^2 only to the
// accuracy of a correction: the hardware reciprocal estimate refined once
// (relative error about 2^-48) instead of a correctly rounded division.
// last2 receives |last step|^2.
constexpr int kPolishGroup = 2;  // 1, 3 and 6 measured no faster

// x y + z for complex FP64 values as four fused multiply-adds (each part's
// two products accumulated into z's part in one chain).
__device__ __forceinline__ cx<double> mul_add(cx<double> x, cx<double> y, cx<double> z)
{
    return {__builtin_fma(x.re, y.re, __builtin_fma(-x.im, y.im, z.re)),
            __builtin_fma(x.re, y.im, __builtin_fma(x.im, y.re, z.im))};
}
template <int DM, int K0, int G>
__device__ __forceinline__ void polish_group(cx<double> (&r)[DM], const cx<double> (&a)[DM + 1],
                                             int steps, double (&last2)[DM])
{
    // the last step's correction and whether it could be taken; last2 is
    // formed from them once, after the loop (0 when no step was asked for)
    cx<double> delta[G], p[G];
    bool step[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        delta[g] = {0.0, 0.0};
        p[g] = {0.0, 0.0};
        step[g] = true;
    }
    for (int s = 0; s < steps; ++s) {
        cx<double> dp[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            p[g] = a[DM];
            dp[g] = {0.0, 0.0};
        }
#pragma unroll
        for (int k = DM - 1; k >= 0; --k)
#pragma unroll
            for (int g = 0; g < G; ++g) {
                dp[g] = mul_add(dp[g], r[K0 + g], p[g]);
                p[g] = mul_add(p[g], r[K0 + g], a[k]);
            }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double den = norm2(dp[g]);
            delta[g] = {0.0, 0.0};
            step[g] = den >= 0x1p-1022 && isfinite(den);
            if (step[g]) {
                const cx<double> q = p[g] * conj(dp[g]);
                const double y0 = __builtin_amdgcn_rcp(den);
                const double inv = __builtin_fma(y0, __builtin_fma(-den, y0, 1.0), y0);
                delta[g] = {q.re * inv, q.im * inv};
            }
            r[K0 + g] = r[K0 + g] - delta[g];
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // a step that cannot be taken counts as converged only at an exact
        // root
        const bool at_root = p[g].re == 0.0 && p[g].im == 0.0;
        last2[K0 + g] = step[g] ? norm2(delta[g]) : (at_root ? 0.0 : __builtin_inf());
    }
}

// All groups of roots below the lane's degree d; a group that no lane of
// the wave needs (degrees below K0 across the wave) is skipped.
template <int DM, int K0>
__device__ __forceinline__ void polish_all(cx<double> (&r)[DM], const cx<double> (&a)[DM + 1],
                                           int steps, double (&last2)[DM], int d)
{
    if constexpr (K0 < DM) {
        constexpr int G = (DM - K0) < kPolishGroup ? (DM - K0) : kPolishGroup;
        if (__ballot(K0 < d))
            polish_group<DM, K0, G>(r, a, steps, last2);
        polish_all<DM, K0 + G>(r, a, steps, last2, d);
    }
}

// Binning epilogue variants (template argument of the kernels).
constexpr int kBinNone = 0;
constexpr int kBinReread = 1;  // FP64: roots stored, read back for binning
constexpr int kBinKeep = 2;    // pixel indices kept in registers (roots optional)

// Everything a lane needs to solve one polynomial.
struct PolyIO {
    const double2* coeffs;
    const double2* coeffs_again;  // same array, second pointer: the polish of the paired-lane
                                  // and persistent-tile launches re-reads it
    const int32_t* degrees;
    int64_t n;
    double2* roots;
    const double2* roots_again;  // same array, second pointer: kBinReread reads it back
    uint32_t* status;
    int32_t* iters;
    int cap;
    uint32_t flags;
    int polish_steps;
    double polish_tol;
    BinWindow win;  // binning epilogue only
    uint32_t skip_mask;
    uint32_t status_or;   // or-ed into every status written (the FP64 fallback's mark)
    uint32_t defer_mask;  // binning: polynomials whose status has one of these bits are left
                          // to the FP64 fallback launch, which bins them after solving again
};

// Status bits that send an FP32 result to the FP64 fallback.
constexpr uint32_t kFallbackBits = PR_ST_NOT_CONVERGED | PR_ST_POLISH_UNCONVERGED;

// The FP32 form's copy of its wave's original coefficients, row k of lane l
// at [k][l], written when they are first read and read back by the polish:
// 7 KiB per one-wave block, so the 5 waves per SIMD that the registers allow
// still fit the CU's 160 KiB of LDS.  Reading them again from memory instead
// fetched about twice their bytes where a wave's polynomials are scattered
// over a degree-sorted tile (each 128-byte line is shared with the waves of
// other degrees, which finish at other times).
template <int DM>
__device__ __forceinline__ double2 (*coeff_stash())[kBlock]
{
    __shared__ double2 stash[DM + 1][kBlock];
    return stash;
}

// Solve polynomial i on this lane.  valid == false: the lane has no
// polynomial to solve and only rides along in the wave's level loops.
// FP32 selects the FP32-sweep + FP64-polish form; BIN != kBinNone adds the
// binning epilogue (kBinKeep lets io.roots be null).  STASH (FP32 form,
// one-wave blocks): the polish takes the coefficients from coeff_stash
// rather than from memory.  No early return: every lane of the wave reaches
// the wave-uniform loops and the epilogue's ballots.
template <bool FP32, int DM, int BIN, bool AHEAD = false, bool STASH = true>
__device__ __forceinline__ void solve_poly(const PolyIO& io, int64_t i, bool valid)
{
    using T = typename std::conditional<FP32, float, double>::type;
    const int64_t n = io.n;
    const bool store = BIN != kBinKeep || io.roots != nullptr;  // wave-uniform
    int bins[DM];
#pragma unroll
    for (int k = 0; k < DM; ++k)
        bins[k] = -1;
    const double qnan = __builtin_nan("");
    int d = valid ? (io.degrees ? io.degrees[i] : DM) : 0;
    uint32_t st = 0;
    if (valid && (d < 1 || d > DM))
        st = PR_ST_BAD_DEGREE;
    cx<double> a[DM + 1], b[DM + 1];
#pragma unroll
    for (int k = 0; k <= DM; ++k)
        a[k] = b[k] = {0.0, 0.0};
    if (valid && !st)
        st = load_poly<DM>(io.coeffs, n, i, d, a, b);
    if constexpr (FP32 && STASH) {
        // a holds the rows up to the degree and zeros above it
#pragma unroll
        for (int k = 0; k <= DM; ++k)
            coeff_stash<DM>()[k][threadIdx.x] = make_double2(a[k].re, a[k].im);
    }
    const bool ok = valid && !st;
    const int dd = ok ? d : 0;  // 0: this lane takes no level
    if (valid) {
        if (store)
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k >= dd)
                    io.roots[(int64_t)k * n + i] = make_double2(qnan, qnan);
        if (io.iters)
#pragma unroll
            for (int m = 2; m <= DM; ++m)
                if (m > dd)
                    io.iters[(int64_t)(m - 2) * n + i] = 0;
    }
    cx<T> h[DM][DM];
#pragma unroll
    for (int r = 0; r < DM; ++r)
#pragma unroll
        for (int c = (r > 0 ? r - 1 : 0); c < DM; ++c)
            h[r][c] = {T(0), T(0)};
    const int sc = ok ? root_scale<T, DM>(b, d) : 0;  // roots come back as 2^sc w
    companion<T, DM>(h, dd, b, sc);
    const bool fixed = (io.flags & PR_FLAG_FIXED_STEPS) != 0;
    const bool exc = !(io.flags & PR_FLAG_NO_EXCEPTIONAL_SHIFT) && !fixed;
    const bool wilk = !(io.flags & PR_FLAG_RAYLEIGH_SHIFT) && !fixed;

    if constexpr (!FP32) {
        iterate<double, DM, AHEAD>(h, dd, io.cap, exc, fixed, wilk, st, io.iters, n, i, [&](int k, cx<double> w) {
            const cx<double> v = {__builtin_ldexp(w.re, sc), __builtin_ldexp(w.im, sc)};
            if (store)
                io.roots[(int64_t)k * n + i] = make_double2(v.re, v.im);
            if constexpr (BIN == kBinKeep) {
                // k is a compile-time constant after inlining
                const int b = pixel_of(v.re, v.im, io.win);
#pragma unroll
                for (int q = 0; q < DM; ++q)
                    if (q == k)
                        bins[q] = b;
            }
        });
        if (ok) {
            const cx<double> v0 = {__builtin_ldexp(h[0][0].re, sc), __builtin_ldexp(h[0][0].im, sc)};
            if (store)
                io.roots[i] = make_double2(v0.re, v0.im);
            if constexpr (BIN == kBinKeep)
                bins[0] = pixel_of(v0.re, v0.im, io.win);
            if constexpr (BIN == kBinReread) {
                bins[0] = pixel_of(v0.re, v0.im, io.win);
#pragma unroll
                for (int k = 1; k < DM; ++k)
                    if (k < dd) {
                        const double2 v = io.roots_again[(int64_t)k * n + i];
                        bins[k] = pixel_of(v.x, v.y, io.win);
                    }
            }
        }
    } else {
        cx<float> e[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            e[k] = {0.0f, 0.0f};
        iterate<float, DM, AHEAD>(h, dd, io.cap, exc, fixed, wilk, st, io.iters, n, i, [&](int k, cx<float> v) {
            // k is a compile-time constant after inlining
#pragma unroll
            for (int q = 0; q < DM; ++q)
                if (q == k)
                    e[q] = v;
        });
        e[0] = h[0][0];
        if (ok) {
            // The original coefficients again: from the LDS copy, or
            // (!STASH) read again through a second pointer, so that the
            // compiler cannot keep the first load alive across the QR loop.
            // That read is their last use, so it is nontemporal; the first
            // read is an ordinary one so that they may still be in L2 here.
            // The roots are stored nontemporally below: as ordinary stores
            // they would evict coefficients that other waves are about to
            // read.  (Rows read as in load_poly, so that the loads overlap.)
            double2 v[DM + 1];
#pragma unroll
            for (int k = 0; k <= DM; ++k) {
                if constexpr (STASH) {
                    v[k] = coeff_stash<DM>()[k][threadIdx.x];
                } else {
                    v[k] = make_double2(0.0, 0.0);
                    if (__ballot(k <= d))
                        v[k] = load_stream(io.coeffs_again + (int64_t)k * n + i);
                }
            }
#pragma unroll
            for (int k = 0; k <= DM; ++k) {
                // a_k 2^(s (k - d)): the coefficients of 2^(-s d) p(2^s w),
                // so that the polish below runs in the sweeps' variable w
                const bool in = k <= d;
                const int e = sc * (k - d);
                a[k] = {in ? __builtin_ldexp(v[k].x, e) : 0.0, in ? __builtin_ldexp(v[k].y, e) : 0.0};
            }
            cx<double> r[DM];
            double last2[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                r[k] = {(double)e[k].re, (double)e[k].im};
            polish_all<DM, 0>(r, a, io.polish_steps, last2, d);
            const double tol2 = io.polish_tol * io.polish_tol;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k < d) {
                    if (!(last2[k] <= tol2 * norm2(r[k])))
                        bad = true;
                } else {
                    r[k] = {qnan, qnan};
                }
            }
            // Two polished roots on top of each other: one root was lost.
#pragma unroll
            for (int j = 0; j < DM; ++j)
#pragma unroll
                for (int k = j + 1; k < DM; ++k)
                    if (k < d) {
                        double sep2 = norm2(r[j] - r[k]);
                        double mag = fmax(norm2(r[j]), 1.0) * 1e-16;  // (1e-8 max(|r_j|, 1))^2
                        if (sep2 <= mag)
                            bad = true;
                    }
            if (bad)
                st |= PR_ST_POLISH_UNCONVERGED;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                r[k] = {__builtin_ldexp(r[k].re, sc), __builtin_ldexp(r[k].im, sc)};  // z = 2^s w
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d) {
                    if (store)
                        store_stream(io.roots + (int64_t)k * n + i, make_double2(r[k].re, r[k].im));
                    if constexpr (BIN != kBinNone)
                        bins[k] = pixel_of(r[k].re, r[k].im, io.win);
                }
        }
    }
    st |= io.status_or;
    if (valid)
        io.status[i] = st;
    if constexpr (BIN != kBinNone) {
        const bool keep = valid && !(st & (io.skip_mask | io.defer_mask));
#pragma unroll
        for (int k = 0; k < DM; ++k)
            run_count(keep ? bins[k] : -1, io.win.hist);
    }
}

// Two polynomials per lane (FP32 form, index order; PR_FLAG_PAIRED_LANES):
// lane l of block b solves polynomials 128 b + l and 128 b + 64 + l, their two
// matrices stepped in the same level loop -- two independent instruction
// streams per wave, at twice the registers per lane.  Same arithmetic per
// polynomial as the one-per-lane kernel.
template <int DM, int M, typename E0, typename E1>
__device__ __forceinline__ void iterate_pair_from(cx<float> (&h0)[DM][DM], cx<float> (&h1)[DM][DM],
                                                  int (&m)[2], int (&its)[2], const int (&d)[2],
                                                  int cap, bool exc, bool fixed, bool wilk,
                                                  uint32_t (&st)[2], int32_t* __restrict__ iters,
                                                  int64_t n, const int64_t (&i)[2], E0&& emit0,
                                                  E1&& emit1)
{
    if constexpr (M >= 2) {
        while (__ballot(m[0] == M || m[1] == M)) {
            trip<float, DM, M>(h0, m[0], its[0], d[0], cap, exc, fixed, wilk, st[0], iters, n,
                               i[0], emit0);
            trip<float, DM, M>(h1, m[1], its[1], d[1], cap, exc, fixed, wilk, st[1], iters, n,
                               i[1], emit1);
            if (!__ballot(m[0] == M || m[1] == M))
                break;
            trip<float, DM, M>(h0, m[0], its[0], d[0], cap, exc, fixed, wilk, st[0], iters, n,
                               i[0], emit0);
            trip<float, DM, M>(h1, m[1], its[1], d[1], cap, exc, fixed, wilk, st[1], iters, n,
                               i[1], emit1);
        }
        iterate_pair_from<DM, M - 1>(h0, h1, m, its, d, cap, exc, fixed, wilk, st, iters, n, i,
                                     emit0, emit1);
    }
}

template <int DM, int BIN>
__device__ __forceinline__ void solve_pair(const PolyIO& io, const int64_t (&i)[2],
                                           const bool (&valid)[2])
{
    const int64_t n = io.n;
    const bool store = BIN != kBinKeep || io.roots != nullptr;  // wave-uniform
    const double qnan = __builtin_nan("");
    const bool fixed = (io.flags & PR_FLAG_FIXED_STEPS) != 0;
    const bool exc = !(io.flags & PR_FLAG_NO_EXCEPTIONAL_SHIFT) && !fixed;
    const bool wilk = !(io.flags & PR_FLAG_RAYLEIGH_SHIFT) && !fixed;
    int d[2], dd[2], sc[2], m[2], its[2];
    uint32_t st[2];
    bool ok[2];
    cx<float> h[2][DM][DM];
    cx<float> e[2][DM];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        d[p] = valid[p] ? (io.degrees ? io.degrees[i[p]] : DM) : 0;
        st[p] = 0;
        if (valid[p] && (d[p] < 1 || d[p] > DM))
            st[p] = PR_ST_BAD_DEGREE;
        cx<double> a[DM + 1], b[DM + 1];
#pragma unroll
        for (int k = 0; k <= DM; ++k)
            a[k] = b[k] = {0.0, 0.0};
        if (valid[p] && !st[p])
            st[p] = load_poly<DM>(io.coeffs, n, i[p], d[p], a, b);
        ok[p] = valid[p] && !st[p];
        dd[p] = ok[p] ? d[p] : 0;
        if (valid[p]) {
            if (store)
#pragma unroll
                for (int k = 0; k < DM; ++k)
                    if (k >= dd[p])
                        io.roots[(int64_t)k * n + i[p]] = make_double2(qnan, qnan);
            if (io.iters)
#pragma unroll
                for (int mm = 2; mm <= DM; ++mm)
                    if (mm > dd[p])
                        io.iters[(int64_t)(mm - 2) * n + i[p]] = 0;
        }
#pragma unroll
        for (int r = 0; r < DM; ++r)
#pragma unroll
            for (int c = (r > 0 ? r - 1 : 0); c < DM; ++c)
                h[p][r][c] = {0.0f, 0.0f};
        sc[p] = ok[p] ? root_scale<float, DM>(b, d[p]) : 0;
        companion<float, DM>(h[p], dd[p], b, sc[p]);
#pragma unroll
        for (int k = 0; k < DM; ++k)
            e[p][k] = {0.0f, 0.0f};
        m[p] = dd[p];
        its[p] = 0;
    }
    auto emit0 = [&](int k, cx<float> v) {
#pragma unroll
        for (int q = 0; q < DM; ++q)
            if (q == k)
                e[0][q] = v;
    };
    auto emit1 = [&](int k, cx<float> v) {
#pragma unroll
        for (int q = 0; q < DM; ++q)
            if (q == k)
                e[1][q] = v;
    };
    iterate_pair_from<DM, DM>(h[0], h[1], m, its, dd, io.cap, exc, fixed, wilk, st, io.iters, n,
                              i, emit0, emit1);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        int bins[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            bins[k] = -1;
        e[p][0] = h[p][0][0];
        if (ok[p]) {
            cx<double> a[DM + 1];
#pragma unroll
            for (int k = 0; k <= DM; ++k) {
                a[k] = {0.0, 0.0};
                if (k <= d[p]) {
                    const double2 v = load_stream(io.coeffs_again + (int64_t)k * n + i[p]);
                    const int ex = sc[p] * (k - d[p]);
                    a[k] = {__builtin_ldexp(v.x, ex), __builtin_ldexp(v.y, ex)};
                }
            }
            cx<double> r[DM];
            double last2[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                r[k] = {(double)e[p][k].re, (double)e[p][k].im};
            polish_all<DM, 0>(r, a, io.polish_steps, last2, d[p]);
            const double tol2 = io.polish_tol * io.polish_tol;
            bool bad = false;
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                if (k < d[p]) {
                    if (!(last2[k] <= tol2 * norm2(r[k])))
                        bad = true;
                } else {
                    r[k] = {qnan, qnan};
                }
            }
#pragma unroll
            for (int j = 0; j < DM; ++j)
#pragma unroll
                for (int k = j + 1; k < DM; ++k)
                    if (k < d[p]) {
                        double sep2 = norm2(r[j] - r[k]);
                        double mag = fmax(norm2(r[j]), 1.0) * 1e-16;
                        if (sep2 <= mag)
                            bad = true;
                    }
            if (bad)
                st[p] |= PR_ST_POLISH_UNCONVERGED;
#pragma unroll
            for (int k = 0; k < DM; ++k)
                r[k] = {__builtin_ldexp(r[k].re, sc[p]), __builtin_ldexp(r[k].im, sc[p])};
#pragma unroll
            for (int k = 0; k < DM; ++k)
                if (k < d[p]) {
                    if (store)
                        store_stream(io.roots + (int64_t)k * n + i[p],
                                     make_double2(r[k].re, r[k].im));
                    if constexpr (BIN != kBinNone)
                        bins[k] = pixel_of(r[k].re, r[k].im, io.win);
                }
        }
        st[p] |= io.status_or;
        if (valid[p])
            io.status[i[p]] = st[p];
        if constexpr (BIN != kBinNone) {
            const bool keep = valid[p] && !(st[p] & (io.skip_mask | io.defer_mask));
#pragma unroll
            for (int k = 0; k < DM; ++k)
                run_count(keep ? bins[k] : -1, io.win.hist);
        }
    }
}

template <int DM, int BIN>
__global__ __launch_bounds__(kBlock) void solve_pair_kernel(PolyIO io)
{
    const int64_t i0 = (int64_t)blockIdx.x * (2 * kBlock) + threadIdx.x;
    const int64_t i[2] = {i0, i0 + kBlock};
    const bool valid[2] = {i[0] < io.n, i[1] < io.n};
    solve_pair<DM, BIN>(io, i, valid);
}

// No occupancy hints: the register allocation as it comes (FP32 96 VGPRs, 5
// waves per SIMD; FP64 158, 3 waves) measured faster than any forced
// occupancy, which spills.
// One lane per polynomial in index order (all polynomials of one degree, or
// no degree array).
template <bool FP32, int DM, int BIN, bool AHEAD>
__global__ __launch_bounds__(kBlock) void solve_flat_kernel(PolyIO io)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    solve_poly<FP32, DM, BIN, AHEAD>(io, i, i < io.n);
}

// Mixed degrees, one persistent launch.  Each block is one wave and walks
// tiles of `tile` consecutive polynomials (grid-stride, no work counter to
// reset).  Per tile it counting-sorts the polynomials by degree with
// ballots (deterministic order, no atomics) into an LDS index list in which
// every degree bucket is padded to a multiple of 64, then solves the list 64
// entries at a time: each slice holds one degree, so no lane idles through
// levels above its degree.  The gathers stay inside the tile, which the
// caches hold.  SELECT (the FP64 fallback): only polynomials whose status
// has a kFallbackBits bit enter the list, so a sparse selection costs little
// more than reading the status array.
constexpr int kTileMax = 4096;
constexpr int kWave = 64;
static_assert(kWave == kBlock, "solve_poly's LDS copy of the coefficients is indexed by threadIdx.x");
constexpr int kBatch = 8;  // chunks of 64 degrees read together by the sliced kernel

template <bool FP32, int DM, int BIN, bool SELECT>
__global__ __launch_bounds__(kWave) void solve_tiled_kernel(PolyIO io, int tile)
{
    // bucket of tile entry t: its degree (0 = invalid degree), or -1 when
    // the entry is not part of this launch's list
    auto bucket = [&](int64_t g) -> int {
        if constexpr (SELECT)
            if (!(io.status[g] & kFallbackBits))
                return -1;
        const int d = io.degrees ? io.degrees[g] : DM;
        return (d >= 1 && d <= DM) ? d : 0;
    };
    __shared__ uint16_t list[kTileMax + (DM + 1) * kWave];
    const int lane = threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes < this lane
    for (int64_t base = (int64_t)blockIdx.x * tile; base < io.n;
         base += (int64_t)gridDim.x * tile) {
        const int cnt_t = (int)((io.n - base) < tile ? (io.n - base) : tile);
        // pass 1: bucket sizes (bucket 0 = invalid degree)
        int count[DM + 1];
#pragma unroll
        for (int b = 0; b <= DM; ++b)
            count[b] = 0;
        for (int t0 = 0; t0 < cnt_t; t0 += kWave) {
            const int t = t0 + lane;
            const int bk = t < cnt_t ? bucket(base + t) : -1;
#pragma unroll
            for (int b = 0; b <= DM; ++b)
                count[b] += __builtin_popcountll(__ballot(bk == b));
        }
        int start[DM + 1];
        int total = 0;
#pragma unroll
        for (int b = 0; b <= DM; ++b) {
            start[b] = total;
            total += (count[b] + kWave - 1) / kWave * kWave;
        }
        for (int t = lane; t < total; t += kWave)
            list[t] = 0xFFFF;
        __syncthreads();
        // pass 2: scatter tile-local indices into their buckets
        for (int t0 = 0; t0 < cnt_t; t0 += kWave) {
            const int t = t0 + lane;
            const int bk = t < cnt_t ? bucket(base + t) : -1;
#pragma unroll
            for (int b = 0; b <= DM; ++b) {
                const uint64_t m = __ballot(bk == b);
                if (bk == b)
                    list[start[b] + __builtin_popcountll(m & below)] = (uint16_t)t;
                start[b] += __builtin_popcountll(m);
            }
        }
        __syncthreads();
        for (int s = 0; s < total; s += kWave) {
            const uint16_t e = list[s + lane];
            const bool valid = e != 0xFFFF;
            solve_poly<FP32, DM, BIN, false, false>(io, base + (valid ? e : 0), valid);
        }
        __syncthreads();
    }
}

// Mixed degrees, one block (one wave) per (tile, slice): no loop around the
// solve, so the kernel keeps the flat kernel's register allocation (FP32 94
// VGPRs, 5 waves per SIMD; FP64 156-168, 3 waves) where the persistent tile
// loop above costs 10-20 more (one wave per SIMD fewer).  Block b takes slot
// `slot` of tile t: the tile's polynomials are sorted by degree, highest
// first (index order within a degree), and slot s takes sorted positions
// 64 s .. 64 s + 63; a slot past the tile's end exits at once.  So every
// slice but the tile's last is full, and only the slices at a degree
// boundary mix degrees.  Blocks are dealt to the 8 XCDs round-robin, so
// consecutive blocks of one XCD (b = xcd + 8 q) take the slots of one tile in
// turn: a tile's slices run together on one XCD and share its L2, which holds
// the tile's coefficients for all of them.
template <bool FP32, int DM, int BIN, bool AHEAD>
__global__ __launch_bounds__(kWave) void solve_sliced_kernel(PolyIO io, int tile, int slots,
                                                             int64_t ntiles)
{
    const int64_t b = blockIdx.x;
    const int64_t q = b >> 3;
    const int64_t g = q / slots;  // tile group: tiles 8 g .. 8 g + 7, one per XCD
    // Each group takes its slots in an order rotated by g.  With the same
    // order in every group, slot s (whose cost follows its degree) fell on
    // the same position modulo 8 or 16 of every XCD's block sequence at tiles
    // of 512 or 1024, and the wave counters showed about 30% fewer resident
    // waves and up to 11% more time: in-order workgroup dispatch over a
    // fixed cycle of shader engines would give one engine all the costly
    // slices.  Rotated, the same work ran 8-12% faster at those tiles.
    const int slot = (int)((q + g) % slots);
    const int64_t t = g * 8 + (b & 7);
    if (t >= ntiles)
        return;
    const int64_t base = t * tile;
    const int cnt_t = (int)((io.n - base) < tile ? (io.n - base) : tile);
    const int lane = threadIdx.x;
    auto degree_bucket = [](int d) -> int { return (d >= 1 && d <= DM) ? d : 0; };
    // buckets of tile entries t0 + u*64 + lane, u < kBatch (-1 past the
    // tile).  A whole batch inside the tile takes its loads unconditionally,
    // so that they are all in flight before the first is used; only the
    // tile's last, partial batch loads lane by lane.
    auto load_buckets = [&](int t0, int (&bk)[kBatch]) {
        if (t0 + kBatch * kWave <= cnt_t) {  // wave-uniform
#pragma unroll
            for (int u = 0; u < kBatch; ++u)
                bk[u] = degree_bucket(io.degrees[base + t0 + u * kWave + lane]);
        } else {
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const int tt = t0 + u * kWave + lane;
                bk[u] = tt < cnt_t ? degree_bucket(io.degrees[base + tt]) : -1;
            }
        }
    };
    // bucket sizes (bucket 0 = invalid degree).  The tile's degrees are read
    // kBatch chunks of 64 at a time, every load of a batch issued before the
    // first is used: one memory round trip per batch instead of one per
    // chunk (a chunk-by-chunk loop kept the waves of this kernel waiting on
    // memory for about 40% of their cycles).
    int count[DM + 1];
#pragma unroll
    for (int k = 0; k <= DM; ++k)
        count[k] = 0;
    for (int t0 = 0; t0 < cnt_t; t0 += kBatch * kWave) {
        int bk[kBatch];
        load_buckets(t0, bk);
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
#pragma unroll
            for (int k = 0; k <= DM; ++k)
                count[k] += __builtin_popcountll(__ballot(bk[u] == k));
    }
    // The tile in sorted order: degree DM first, down to degree 1, then the
    // invalid degrees, each bucket in index order.  The slot takes sorted
    // positions p0 .. p0 + 63.  Only the tile's last slice is partly empty; a
    // slice at a bucket boundary holds two (or, for buckets of fewer than 64,
    // more) degrees, whose lower-degree lanes wait for their level (or, with
    // run-ahead, step one level below inside the higher level's trips).
    const int p0 = slot * kWave;
    if (p0 >= cnt_t)
        return;
    // the slice's tile-local indices, in sorted order
    __shared__ uint16_t list[kWave];
    list[lane] = 0xFFFF;
    __syncthreads();
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes < this lane
    int start = 0;  // sorted position of bucket k's first member
#pragma unroll 1
    for (int k = DM; k >= 0; --k) {
        int ck = 0;  // count[k], by selects (no dynamic index into registers)
#pragma unroll
        for (int j = 0; j <= DM; ++j)
            ck = j == k ? count[j] : ck;
        // ranks r0 .. r1 - 1 of bucket k fall in the slice
        const int r0 = p0 - start > 0 ? p0 - start : 0;
        const int r1 = p0 + kWave - start < ck ? p0 + kWave - start : ck;
        if (r0 < r1) {  // wave-uniform
            int rank = 0;
            for (int t0 = 0; t0 < cnt_t && rank < r1; t0 += kBatch * kWave) {
                int bk[kBatch];
                load_buckets(t0, bk);
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int tt = t0 + u * kWave + lane;
                    const uint64_t m = __ballot(bk[u] == k);
                    const int r = rank + __builtin_popcountll(m & below);
                    if (bk[u] == k && r >= r0 && r < r1)
                        list[start + r - p0] = (uint16_t)tt;
                    rank += __builtin_popcountll(m);
                }
            }
        }
        start += ck;
        if (start >= p0 + kWave)
            break;
    }
    __syncthreads();
    const uint16_t e = list[lane];
    const bool valid = e != 0xFFFF;
    solve_poly<FP32, DM, BIN, AHEAD>(io, base + (valid ? e : 0), valid);
}

template <bool FP32, int DM, int BIN, bool AHEAD>
hipError_t launch_one_per_lane(const PolyIO& io, const SolveArgs& a, hipStream_t stream)
{
    if (a.degrees && a.tile > 0) {
        const int tile = a.tile;
        const int64_t tiles = (a.n + tile - 1) / tile;
        const int slots = (tile + kWave - 1) / kWave;  // the slices of a full tile
        const int64_t sliced = (tiles + 7) / 8 * 8 * slots;
        hipLaunchKernelGGL((solve_sliced_kernel<FP32, DM, BIN, AHEAD>), dim3((unsigned)sliced),
                           dim3(kWave), 0, stream, io, tile, slots, tiles);
    } else {
        const int64_t blocks = (a.n + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((solve_flat_kernel<FP32, DM, BIN, AHEAD>), dim3((unsigned)blocks),
                           dim3(kBlock), 0, stream, io);
    }
    return hipGetLastError();
}

template <bool FP32, int DM, int BIN>
hipError_t launch_layout(const PolyIO& io, const SolveArgs& a, hipStream_t stream)
{
    if (a.degrees && a.tile > 0) {
        const int tile = a.tile;
        const int64_t tiles = (a.n + tile - 1) / tile;
        const int slots = (tile + kWave - 1) / kWave;  // the slices of a full tile
        const int64_t sliced = (tiles + 7) / 8 * 8 * slots;
        if (a.grid_blocks == 0 && sliced <= 0x7fffffff) {
            if (a.flags & PR_FLAG_RUN_AHEAD)
                return launch_one_per_lane<FP32, DM, BIN, true>(io, a, stream);
            return launch_one_per_lane<FP32, DM, BIN, false>(io, a, stream);
        } else {
            const int64_t want = a.grid_blocks > 0 ? a.grid_blocks : a.fallback_grid;
            const int64_t grid = want < tiles ? want : tiles;
            hipLaunchKernelGGL((solve_tiled_kernel<FP32, DM, BIN, false>), dim3((unsigned)grid),
                               dim3(kWave), 0, stream, io, tile);
        }
    } else if (FP32 && BIN != kBinReread && (a.flags & PR_FLAG_PAIRED_LANES)) {
        const int64_t blocks = (a.n + 2 * kBlock - 1) / (2 * kBlock);
        hipLaunchKernelGGL((solve_pair_kernel<DM, BIN == kBinReread ? kBinNone : BIN>),
                           dim3((unsigned)blocks), dim3(kBlock), 0, stream, io);
    } else if (a.flags & PR_FLAG_RUN_AHEAD) {
        return launch_one_per_lane<FP32, DM, BIN, true>(io, a, stream);
    } else {
        return launch_one_per_lane<FP32, DM, BIN, false>(io, a, stream);
    }
    return hipGetLastError();
}

template <bool FP32, int DM>
hipError_t launch_dm(const SolveArgs& a, hipStream_t stream)
{
    PolyIO io;
    io.coeffs = reinterpret_cast<const double2*>(a.coeffs);
    io.coeffs_again = io.coeffs;
    io.degrees = a.degrees;
    io.n = a.n;
    io.roots = reinterpret_cast<double2*>(a.roots);
    io.roots_again = io.roots;
    io.status = a.status;
    io.iters = a.iters;
    io.cap = a.cap;
    io.flags = a.flags;
    io.polish_steps = a.polish_steps;
    io.polish_tol = a.polish_tol;
    io.win = a.win;
    io.skip_mask = a.skip_mask;
    io.status_or = 0;
    const bool fallback = FP32 && (a.flags & PR_FLAG_FP64_FALLBACK);
    io.defer_mask = fallback ? kFallbackBits : 0;
    hipError_t e;
    if (!a.win.hist) {
        e = launch_layout<FP32, DM, kBinNone>(io, a, stream);
    } else if constexpr (!FP32) {
        // FP64 with lanes running ahead and the roots stored: the pixels are
        // taken from the stored roots at the end instead of being kept in
        // registers through the level loops (168 VGPRs instead of 174, so 3
        // waves per SIMD instead of 2)
        if (a.roots && (a.flags & PR_FLAG_RUN_AHEAD))
            e = launch_layout<FP32, DM, kBinReread>(io, a, stream);
        else
            e = launch_layout<FP32, DM, kBinKeep>(io, a, stream);
    } else {
        e = launch_layout<FP32, DM, kBinKeep>(io, a, stream);
    }
    if (e != hipSuccess || !fallback)
        return e;
    // FP64 fallback: a second launch over the polynomials the first one
    // flagged, in tiles, with the same options; it bins what it solves
    io.status_or = PR_ST_RESOLVED_FP64;
    io.defer_mask = 0;
    const int tile = a.fallback_tile;
    const int64_t tiles = (a.n + tile - 1) / tile;
    const int64_t grid = a.fallback_grid < tiles ? a.fallback_grid : tiles;
    if (!a.win.hist)
        hipLaunchKernelGGL((solve_tiled_kernel<false, DM, kBinNone, true>), dim3((unsigned)grid),
                           dim3(kWave), 0, stream, io, tile);
    else if (a.roots)
        hipLaunchKernelGGL((solve_tiled_kernel<false, DM, kBinReread, true>),
                           dim3((unsigned)grid), dim3(kWave), 0, stream, io, tile);
    else
        hipLaunchKernelGGL((solve_tiled_kernel<false, DM, kBinKeep, true>), dim3((unsigned)grid),
                           dim3(kWave), 0, stream, io, tile);
    return hipGetLastError();
}

template <bool FP32>
hipError_t launch_form(const SolveArgs& a, hipStream_t stream)
{
    switch (a.dmax) {
    case 1: return launch_dm<FP32, 1>(a, stream);
    case 2: return launch_dm<FP32, 2>(a, stream);
    case 3: return launch_dm<FP32, 3>(a, stream);
    case 4: return launch_dm<FP32, 4>(a, stream);
    case 5: return launch_dm<FP32, 5>(a, stream);
    case 6: return launch_dm<FP32, 6>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_solve_fp64(const SolveArgs& a, hipStream_t stream)
{
    return launch_form<false>(a, stream);
}

hipError_t launch_solve_fp32_polish(const SolveArgs& a, hipStream_t stream)
{
    return launch_form<true>(a, stream);
}

int max_tile() { return kTileMax; }

}  // namespace proots
