// sortplan.hpp -- sizes and layout of the tile-sorted density path's
// workspace (sortbin.hip), computed on the host.
//
// Plain C++ with no HIP dependency, so that the arithmetic can be compiled
// and exercised on its own (the CPU test-suite builds it with address and
// undefined-behaviour sanitizers).
#pragma once

#include <cstdint>

namespace proots {
namespace sortbin {

constexpr int kTileShift = 14;
constexpr int kTilePixels = 1 << kTileShift;  // 64 KiB of LDS counters
constexpr uint32_t kTileMask = kTilePixels - 1;
constexpr int kMaxTiles = 1024;               // images up to 2^24 pixels
constexpr int kChunk = 1024;                  // polynomials per chunk (one scatter block)
constexpr int kMaxBlocks = 1024;              // count/scatter blocks
constexpr int64_t kMinSegment = 1 << 16;
constexpr int64_t kSegmentsPerBatch = 512;

inline int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

struct Plan {
    int ntiles;
    int nblocks;           // count and scatter blocks
    int64_t nchunks;       // chunks of kChunk polynomials (the last may hold fewer)
    int64_t roots_bound;   // dmax n
    uint32_t seg_len;
    int64_t max_segments;
    int64_t ctrl_bytes, runs_bytes, pix_bytes, sorted_bytes, partial_bytes;
    bool direct;           // count with the direct kernel, no workspace
};

inline Plan make_plan(int64_t n, int dmax, int width, int height)
{
    Plan p{};
    const int64_t npix = (int64_t)width * height;
    p.ntiles = (int)((npix + kTilePixels - 1) >> kTileShift);
    p.roots_bound = (int64_t)dmax * n;
    p.direct = p.ntiles > kMaxTiles || p.roots_bound >= ((int64_t)1 << 31) || n == 0;
    if (p.direct)
        return p;
    p.nchunks = (n + kChunk - 1) / kChunk;
    p.nblocks = (int)(p.nchunks < kMaxBlocks ? p.nchunks : kMaxBlocks);
    int64_t len = (p.roots_bound + kSegmentsPerBatch - 1) / kSegmentsPerBatch;
    len = len < kMinSegment ? kMinSegment : len;
    p.seg_len = (uint32_t)len;
    p.max_segments = p.ntiles + (p.roots_bound + len - 1) / len;
    p.ctrl_bytes = align256((int64_t)12 * (p.ntiles + 1));
    p.runs_bytes = align256((int64_t)4 * p.ntiles * p.nblocks);
    p.pix_bytes = align256(4 * p.roots_bound);
    p.sorted_bytes = align256(2 * p.roots_bound + 16);  // + the last 16-byte group's overhang
    p.partial_bytes = align256(p.max_segments * kTilePixels * 4);
    return p;
}

inline int64_t workspace_bytes(const Plan& p)
{
    return p.direct ? 0
                    : p.ctrl_bytes + p.runs_bytes + p.pix_bytes + p.sorted_bytes + p.partial_bytes;
}

}  // namespace sortbin
}  // namespace proots
