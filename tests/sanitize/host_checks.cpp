// Host-side argument checks of the C ABI and the sorted-density workspace
// arithmetic, exercised on their own (the CPU test-suite compiles this file
// with address and undefined-behaviour sanitizers and runs it).  Prints
// "host checks ok" and exits 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <initializer_list>
#include <limits>

#include "sortplan.hpp"
#include "validate.hpp"

static int failures = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);      \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

using namespace proots;

static void windows()
{
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const double inf = std::numeric_limits<double>::infinity();
    int image = 0;
    double sx = 0, sy = 0;
    CHECK(check_window(-1, 1, -2, 2, 8, 16, &image, sx, sy) == PR_OK && sx == 4.0 && sy == 4.0);
    CHECK(check_window(-1, 1, -1, 1, 8, 8, nullptr, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(nan, 1, -1, 1, 8, 8, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(-1, inf, -1, 1, 8, 8, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(1, -1, -1, 1, 8, 8, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(-1, 1, 1, 1, 8, 8, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(-1, 1, -1, 1, 0, 8, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(-1, 1, -1, 1, 8, -3, &image, sx, sy) == PR_ERR_INVALID_ARG);
    // 65536 x 65536 pixels: the product overflows int32 and is refused
    CHECK(check_window(-1, 1, -1, 1, 65536, 65536, &image, sx, sy) == PR_ERR_INVALID_ARG);
    CHECK(check_window(-1, 1, -1, 1, 46340, 46340, &image, sx, sy) == PR_OK);
    // a window so narrow that width / (x1 - x0) overflows
    CHECK(check_window(0, 4.9e-324, -1, 1, 1 << 30, 1, &image, sx, sy) == PR_ERR_INVALID_ARG);
}

static void solve_options()
{
    pr_solve_opts o;
    CHECK(check_solve_opts(nullptr, 4096, o) == PR_OK && o.precision == PR_FP64);
    pr_solve_opts in{};
    in.precision = 7;
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_UNSUPPORTED);
    in = pr_solve_opts{};
    in.max_iter_per_level = 1001;
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_INVALID_ARG);
    in = pr_solve_opts{};
    in.polish_steps = -1;
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_INVALID_ARG);
    in = pr_solve_opts{};
    in.polish_tol = std::numeric_limits<double>::quiet_NaN();
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_INVALID_ARG);
    in = pr_solve_opts{};
    in.flags = 1u << 31;
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_UNSUPPORTED);
    in = pr_solve_opts{};
    in.tile = 4097;
    CHECK(check_solve_opts(&in, 4096, o) == PR_ERR_INVALID_ARG);
    in = pr_solve_opts{};
    in.precision = PR_FP32_POLISH;
    in.flags = PR_FLAG_FP64_FALLBACK | PR_FLAG_RAYLEIGH_SHIFT;
    in.tile = -1;
    in.max_iter_per_level = 1000;
    CHECK(check_solve_opts(&in, 4096, o) == PR_OK && o.tile == -1);
    CHECK(check_batch(-1, 6) == PR_ERR_INVALID_ARG);
    CHECK(check_batch(5, 0) == PR_ERR_INVALID_ARG && check_batch(5, 7) == PR_ERR_INVALID_ARG);
    CHECK(check_batch(std::numeric_limits<int64_t>::max(), 6) == PR_OK);
}

// Every plan the density entry points can ask for: regions 256-aligned,
// large enough for what the kernels index, and summing to the workspace.
static void plans()
{
    using namespace proots::sortbin;
    const int64_t ns[] = {0, 1, 7, 1023, 1024, 1025, 65536, 1000003, 16 << 20, 357913941,
                          357913942, (int64_t)1 << 39};
    const int sizes[][2] = {{1, 1}, {256, 256}, {640, 480}, {1920, 1080}, {4096, 4096},
                            {4097, 4096}, {46340, 46340}, {16384, 1}};
    for (int64_t n : ns)
        for (int dmax = 1; dmax <= 6; ++dmax)
            for (const auto& wh : sizes) {
                const Plan p = make_plan(n, dmax, wh[0], wh[1]);
                const int64_t npix = (int64_t)wh[0] * wh[1];
                const int64_t R = dmax * n;
                if (n == 0 || R >= ((int64_t)1 << 31) || npix > ((int64_t)kMaxTiles << kTileShift)) {
                    CHECK(p.direct && workspace_bytes(p) == 0);
                    continue;
                }
                CHECK(!p.direct);
                CHECK(p.ntiles >= 1 && (int64_t)p.ntiles * kTilePixels >= npix);
                CHECK(p.nchunks * kChunk >= n && (p.nchunks - 1) * kChunk < n);
                CHECK(p.nblocks >= 1 && p.nblocks <= kMaxBlocks && p.nblocks <= p.nchunks);
                CHECK(p.seg_len >= kMinSegment);
                // segments: sum over tiles of ceil(c_t / L) <= R / L + T
                CHECK(p.max_segments >= p.ntiles + (R + p.seg_len - 1) / p.seg_len);
                CHECK(p.ctrl_bytes >= 12 * (p.ntiles + 1));
                CHECK(p.runs_bytes >= 4 * (int64_t)p.ntiles * p.nblocks);
                CHECK(p.pix_bytes >= 4 * R && p.sorted_bytes >= 2 * R + 16);
                CHECK(p.partial_bytes >= p.max_segments * kTilePixels * 4);
                for (int64_t b : {p.ctrl_bytes, p.runs_bytes, p.pix_bytes, p.sorted_bytes,
                                  p.partial_bytes})
                    CHECK(b % 256 == 0);
                CHECK(workspace_bytes(p) == p.ctrl_bytes + p.runs_bytes + p.pix_bytes +
                                                p.sorted_bytes + p.partial_bytes);
            }
}

int main()
{
    windows();
    solve_options();
    plans();
    if (failures) {
        std::printf("%d host check(s) failed\n", failures);
        return 1;
    }
    std::printf("host checks ok\n");
    return 0;
}
