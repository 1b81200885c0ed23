// sortbin.hip -- root-density image through image tiles counted in LDS
// (arXiv 2507.02164, Sec. III: each eigenvalue is converted to a pixel
// coordinate and accumulated in video memory).
//
// The direct density kernel adds every root to the image with a device-scope
// atomic (merged within a wave where neighbouring roots share a pixel).  Roots
// spread over the image have nothing to merge and bin at the rate of those
// atomics.  This path groups the roots by image tile first -- tiles of
// kTilePixels consecutive pixels in row-major order, small enough for an LDS
// histogram -- with a counting sort into a caller-supplied workspace, counts
// each tile's roots in LDS, and adds the counts to the image with plain loads
// and stores, one thread per pixel.  Every pixel decision is pixel_of() of
// bin.hpp, as in the direct kernel, and integer addition does not depend on
// order, so the image is the same bit for bit.
//
// Launches, in order on the caller's stream:
//   1. count       the polynomials are cut into chunks of kChunk, dealt to
//                  the blocks round-robin (block b takes chunks b, b + B, ...,
//                  so that the blocks stream neighbouring memory): each
//                  root's pixel index is written to the workspace (-1 when
//                  not counted), and the block's roots per tile are counted
//                  in LDS and stored as one column of a [tiles][blocks]
//                  matrix
//   2. rowscan     one block per tile: the tile's row of block counts turned
//                  into each block's offset within the tile, and its total
//   3. plan        one block: each tile's range of the sorted array (a prefix
//                  sum of the totals) and the segments of at most seg_len
//                  entries each range is cut into (so that a dense tile is
//                  shared by several blocks)
//   4. scatter     each block walks its chunks again, in the same order: a chunk's
//                  in-tile offsets are ranked per tile in LDS, staged in tile
//                  order and written to the block's runs as contiguous stores
//                  (16-bit entries); no global atomics, so the sorted order is
//                  deterministic
//   5. accumulate  persistent blocks, one segment at a time: an LDS histogram
//                  of the tile, stored whole into the segment's partial image
//   6. reduce      one thread per pixel: the sum of its tile's partial images
//                  added to the image
//
// Workspace (bytes from sortbin_workspace, 256-aligned regions):
//   uint32 tile_total[T + 1], tile_start[T + 1], seg_start[T + 1]
//   uint32 runs[T][B]           per (tile, block): count, then offset in the tile
//   int32  pix[dmax][n]         pixel index of every root slot, -1 if none
//   uint16 sorted[R]            in-tile pixel offsets grouped by tile
//   int32  partial[S][kTilePixels]  one partial image per segment
// with T tiles, B count/scatter blocks, R = dmax n (a bound on the roots
// counted) and S = T + ceil(R / seg_len) (a bound on the segments).  Images
// of more than kMaxTiles tiles and batches of 2^31 or more root slots are
// counted by the direct kernel instead (no workspace).
#include <hip/hip_runtime.h>

#include <atomic>

#include "bin.hpp"
#include "internal.hpp"
#include "sortplan.hpp"

namespace proots {
namespace {

using namespace sortbin;

constexpr int kCountBlock = 512;
constexpr int kPlanBlock = 1024;               // >= kMaxTiles and >= kMaxBlocks
constexpr int kScatterBlock = kChunk;
constexpr int kAccBlock = 1024;
constexpr int kReduceBlock = 256;

// Lanes of a wave that add to the same LDS counter serialise on it.  Roots of
// a smooth family (neighbouring polynomials) land on the same tile, often on
// the same pixel, so up to kMergeRounds distinct counters of a wave are
// merged: the lowest pending lane's counter is broadcast, every lane holding
// it is counted with one ballot and one atomic, and the rest add their own.
// A round that finds its counter in one lane only ends the merging (the
// wave's counters are spread), so spread roots pay one round's few scalar
// instructions.
constexpr int kMergeRounds = 2;

// Add 1 at c[idx] for every lane with idx >= 0; every active lane of the wave
// calls it together.  With RANK, returns the counter's value before the
// lane's own 1 (distinct values for the lanes adding to one counter).
template <bool RANK>
__device__ __forceinline__ uint32_t lds_count(uint32_t* c, int idx)
{
    const int lane = __lane_id();
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    uint32_t rank = 0;
    uint64_t pending = __ballot(idx >= 0);
    for (int r = 0; r < kMergeRounds && pending; ++r) {
        const int leader = __builtin_ctzll(pending);
        const int li = __builtin_amdgcn_readlane(idx, leader);
        const uint64_t same = __ballot(idx == li);
        uint32_t base = 0;
        if (lane == leader)
            base = atomicAdd(&c[li], (uint32_t)__builtin_popcountll(same));
        if (RANK)
            base = __builtin_amdgcn_readlane(base, leader);
        if (idx == li) {
            rank = base + (uint32_t)__builtin_popcountll(same & below);
            idx = -1;
        }
        pending &= ~same;
        if (__builtin_popcountll(same) == 1)
            break;
    }
    if (idx >= 0)
        rank = atomicAdd(&c[idx], 1u);
    return rank;
}

// Add amt (1..8) at c[idx] for every lane with idx >= 0; every active lane of
// the wave calls it together.  Merged as lds_count, the leader adding the sum
// of its group's amounts (four ballots, one per bit of the amount).
__device__ __forceinline__ void lds_add(uint32_t* c, int idx, uint32_t amt)
{
    const int lane = __lane_id();
    uint64_t pending = __ballot(idx >= 0);
    for (int r = 0; r < kMergeRounds && pending; ++r) {
        const int leader = __builtin_ctzll(pending);
        const int li = __builtin_amdgcn_readlane(idx, leader);
        const bool mine = idx == li;
        const uint64_t same = __ballot(mine);
        uint32_t sum = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
            sum += (uint32_t)__builtin_popcountll(__ballot(mine && ((amt >> b) & 1u))) << b;
        if (lane == leader)
            atomicAdd(&c[li], sum);
        if (mine)
            idx = -1;
        pending &= ~same;
        if (__builtin_popcountll(same) == 1)
            break;
    }
    if (idx >= 0)
        atomicAdd(&c[idx], amt);
}

struct Work {
    uint32_t* tile_total;  // [T + 1]
    uint32_t* tile_start;  // [T + 1]
    uint32_t* seg_start;   // [T + 1]
    uint32_t* runs;        // [T][B]
    int32_t* pix;          // [dmax][n]
    uint16_t* sorted;      // [R]
    int32_t* partial;      // [S][kTilePixels]
};

Work work_of(void* ws, const Plan& p)
{
    char* b = static_cast<char*>(ws);
    Work w;
    w.tile_total = reinterpret_cast<uint32_t*>(b);
    w.tile_start = w.tile_total + (p.ntiles + 1);
    w.seg_start = w.tile_start + (p.ntiles + 1);
    b += p.ctrl_bytes;
    w.runs = reinterpret_cast<uint32_t*>(b);
    b += p.runs_bytes;
    w.pix = reinterpret_cast<int32_t*>(b);
    b += p.pix_bytes;
    w.sorted = reinterpret_cast<uint16_t*>(b);
    b += p.sorted_bytes;
    w.partial = reinterpret_cast<int32_t*>(b);
    return w;
}

// Polynomial i's number of roots to read: 0 when skipped by status (or i is
// past the batch), else its degree (dmax without a degree array) clamped to
// DM -- as the direct kernel.
template <int DM>
__device__ __forceinline__ int roots_of(int64_t i, int64_t n, const int32_t* __restrict__ degrees,
                                        const uint32_t* __restrict__ status, uint32_t skip_mask)
{
    int d = 0;
    if (i < n && !(status && (status[i] & skip_mask))) {
        d = degrees ? degrees[i] : DM;
        d = d > DM ? DM : d;
    }
    return d;
}

template <int DM>
__global__ __launch_bounds__(kCountBlock) void count_kernel(
    const double2* __restrict__ roots, const int32_t* __restrict__ degrees,
    const uint32_t* __restrict__ status, uint32_t skip_mask, int64_t n, BinWindow win,
    int ntiles, int64_t nchunks, uint32_t* __restrict__ runs, int32_t* __restrict__ pixout)
{
    __shared__ uint32_t cnt[kMaxTiles];
    const int tid = threadIdx.x;
    for (int t = tid; t < ntiles; t += kCountBlock)
        cnt[t] = 0;
    __syncthreads();
    for (int64_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {  // block-uniform
        for (int sub = 0; sub < kChunk; sub += kCountBlock) {
            const int64_t i = ci * kChunk + sub + tid;
            const int d = roots_of<DM>(i, n, degrees, status, skip_mask);
            // every row loaded first (coalesced, in flight together)
            double2 z[DM];
#pragma unroll
            for (int k = 0; k < DM; ++k)
                z[k] = k < d ? roots[(int64_t)k * n + i] : make_double2(__builtin_nan(""), 0.0);
#pragma unroll
            for (int k = 0; k < DM; ++k) {
                const int px = pixel_of(z[k].x, z[k].y, win);
                if (i < n)
                    pixout[(int64_t)k * n + i] = px;
                lds_count<false>(cnt, px >= 0 ? px >> kTileShift : -1);
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < ntiles; t += kCountBlock)
        runs[(int64_t)t * gridDim.x + blockIdx.x] = cnt[t];
}

// Exclusive prefix sum of v over the block (one value per thread, blockDim
// == B, a multiple of 64); returns the sum of all values in `total`.
template <int B>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* __restrict__ wave_sums,
                                                         uint32_t& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o)
            x += y;
    }
    if (lane == 63)
        wave_sums[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < B / 64; ++w) {
            const uint32_t s = wave_sums[w];
            wave_sums[w] = run;
            run += s;
        }
        wave_sums[B / 64] = run;
    }
    __syncthreads();
    total = wave_sums[B / 64];
    const uint32_t r = wave_sums[wave] + x - v;
    __syncthreads();  // wave_sums may be reused by the caller's next scan
    return r;
}

// One block per tile: row t of the [T][B] counts becomes each block's offset
// within the tile's range; the row's sum is the tile's total.
__global__ __launch_bounds__(kPlanBlock) void rowscan_kernel(uint32_t* __restrict__ runs,
                                                             int nblocks,
                                                             uint32_t* __restrict__ tile_total)
{
    __shared__ uint32_t wave_sums[kPlanBlock / 64 + 1];
    const int t = blockIdx.x, j = threadIdx.x;
    uint32_t* row = runs + (int64_t)t * nblocks;
    const uint32_t c = j < nblocks ? row[j] : 0u;
    uint32_t total;
    const uint32_t o = block_exclusive_scan<kPlanBlock>(c, wave_sums, total);
    if (j < nblocks)
        row[j] = o;
    if (j == 0)
        tile_total[t] = total;
}

// One block: tile t's range is [tile_start[t], tile_start[t+1]) and its
// segments are seg_start[t] .. seg_start[t+1] - 1.
__global__ __launch_bounds__(kPlanBlock) void plan_kernel(const uint32_t* __restrict__ tile_total,
                                                          int ntiles, uint32_t seg_len,
                                                          uint32_t* __restrict__ tile_start,
                                                          uint32_t* __restrict__ seg_start)
{
    __shared__ uint32_t wave_sums[kPlanBlock / 64 + 1];
    const int t = threadIdx.x;
    const uint32_t cnt = t < ntiles ? tile_total[t] : 0u;
    uint32_t total;
    const uint32_t start = block_exclusive_scan<kPlanBlock>(cnt, wave_sums, total);
    const uint32_t segs = (cnt + seg_len - 1) / seg_len;
    uint32_t nseg;
    const uint32_t sstart = block_exclusive_scan<kPlanBlock>(segs, wave_sums, nseg);
    if (t < ntiles) {
        tile_start[t] = start;
        seg_start[t] = sstart;
    }
    if (t == 0) {
        tile_start[ntiles] = total;
        seg_start[ntiles] = nseg;
    }
}

template <int DM>
__global__ __launch_bounds__(kScatterBlock) void scatter_kernel(
    const int32_t* __restrict__ pixin, int64_t n, int ntiles, int64_t nchunks,
    const uint32_t* __restrict__ runs, const uint32_t* __restrict__ tile_start,
    uint16_t* __restrict__ sorted)
{
    __shared__ uint32_t cnt[kMaxTiles];    // this chunk's roots per tile
    __shared__ uint32_t off[kMaxTiles];    // their offset in the staging list
    __shared__ uint32_t run[kMaxTiles];    // where the block's next entry of each tile goes
    __shared__ uint32_t stage[kScatterBlock * DM];
    __shared__ uint32_t wave_sums[kScatterBlock / 64 + 1];
    const int tid = threadIdx.x;
    for (int t = tid; t < ntiles; t += kScatterBlock)
        run[t] = tile_start[t] + runs[(int64_t)t * gridDim.x + blockIdx.x];
    for (int64_t ci = blockIdx.x; ci < nchunks; ci += gridDim.x) {  // block-uniform
        for (int t = tid; t < ntiles; t += kScatterBlock)
            cnt[t] = 0;
        __syncthreads();
        const int64_t i = ci * kChunk + tid;
        int pix[DM];
        uint32_t rank[DM];
#pragma unroll
        for (int k = 0; k < DM; ++k)
            pix[k] = i < n ? pixin[(int64_t)k * n + i] : -1;
#pragma unroll
        for (int k = 0; k < DM; ++k)
            rank[k] = lds_count<true>(cnt, pix[k] >= 0 ? pix[k] >> kTileShift : -1);
        __syncthreads();
        const uint32_t c = tid < ntiles ? cnt[tid] : 0u;
        uint32_t total;
        const uint32_t o = block_exclusive_scan<kScatterBlock>(c, wave_sums, total);
        if (tid < ntiles)
            off[tid] = o;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < DM; ++k)
            if (pix[k] >= 0)
                stage[off[pix[k] >> kTileShift] + rank[k]] = (uint32_t)pix[k];
        __syncthreads();
        for (uint32_t j = tid; j < total; j += kScatterBlock) {
            const uint32_t p = stage[j];
            const uint32_t t = p >> kTileShift;
            sorted[run[t] + (j - off[t])] = (uint16_t)(p & kTileMask);
        }
        __syncthreads();
        if (tid < ntiles)
            run[tid] += c;
    }
}

// Persistent blocks, one segment at a time.  Each thread takes the 8 entries
// of one 16-byte group per iteration (one load, so that a wave keeps 1 KiB in
// flight); the groups at the segment's ends are masked.  Equal neighbouring
// entries (the roots of neighbouring polynomials of a smooth family) are
// added as one run.
__global__ __launch_bounds__(kAccBlock) void accumulate_kernel(
    const uint32_t* __restrict__ tile_start, const uint32_t* __restrict__ seg_start, int ntiles,
    uint32_t seg_len, const uint16_t* __restrict__ sorted, int32_t* __restrict__ partial)
{
    __shared__ uint32_t h[kTilePixels];
    const int tid = threadIdx.x;
    const uint32_t nseg = seg_start[ntiles];
    const uint4* groups = reinterpret_cast<const uint4*>(sorted);
    for (uint32_t w = blockIdx.x; w < nseg; w += gridDim.x) {
        // the tile of segment w: the last t with seg_start[t] <= w (a tile
        // with no segment shares its start with the next one)
        int lo = 0, hi = ntiles - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (seg_start[mid] <= w)
                lo = mid;
            else
                hi = mid - 1;
        }
        const uint32_t begin = tile_start[lo] + (w - seg_start[lo]) * seg_len;
        const uint32_t tile_end = tile_start[lo + 1];
        const uint32_t end = tile_end - begin < seg_len ? tile_end : begin + seg_len;
        for (int k = tid; k < kTilePixels; k += kAccBlock)
            h[k] = 0;
        __syncthreads();
        const uint32_t g0 = begin >> 3, g1 = (end + 7) >> 3;
        for (uint32_t gb = g0; gb < g1; gb += kAccBlock) {  // block-uniform
            const uint32_t g = gb + tid;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (g < g1)
                v = groups[g];
            const uint32_t word[4] = {v.x, v.y, v.z, v.w};
            int off[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint32_t e = 8 * g + m;
                off[m] = (g < g1 && e >= begin && e < end)
                             ? (int)((word[m >> 1] >> (16 * (m & 1))) & 0xFFFFu) : -1;
            }
            uint32_t len = 0;
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                len += off[m] >= 0 ? 1u : 0u;
                const bool flush = off[m] >= 0 && (m == 7 || off[m + 1] != off[m]);
                lds_add(h, flush ? off[m] : -1, len);
                len = flush ? 0u : len;
            }
        }
        __syncthreads();
        int4* out = reinterpret_cast<int4*>(partial + (int64_t)w * kTilePixels);
        for (int k = tid; k < kTilePixels / 4; k += kAccBlock)
            out[k] = make_int4((int)h[4 * k], (int)h[4 * k + 1], (int)h[4 * k + 2],
                               (int)h[4 * k + 3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kReduceBlock) void reduce_kernel(const uint32_t* __restrict__ seg_start,
                                                              const int32_t* __restrict__ partial,
                                                              int64_t npix, int32_t* __restrict__ hist)
{
    const int64_t p = (int64_t)blockIdx.x * kReduceBlock + threadIdx.x;
    if (p >= npix)
        return;
    const uint32_t t = (uint32_t)(p >> kTileShift);
    const uint32_t k = (uint32_t)(p & kTileMask);
    const uint32_t s0 = seg_start[t], s1 = seg_start[t + 1];
    int32_t sum = 0;
    for (uint32_t w = s0; w < s1; ++w)
        sum += partial[(int64_t)w * kTilePixels + k];
    if (sum)
        hist[p] += sum;  // one thread per pixel: the only writer in this launch
}

template <int DM>
hipError_t launch_dm(const DensityArgs& a, const Plan& p, void* ws, int cus, hipStream_t stream)
{
    const Work w = work_of(ws, p);
    const int64_t npix = (int64_t)a.win.width * a.win.height;
    hipLaunchKernelGGL((count_kernel<DM>), dim3(p.nblocks), dim3(kCountBlock), 0, stream,
                       reinterpret_cast<const double2*>(a.roots), a.degrees, a.status, a.skip_mask,
                       a.n, a.win, p.ntiles, p.nchunks, w.runs, w.pix);
    hipLaunchKernelGGL(rowscan_kernel, dim3(p.ntiles), dim3(kPlanBlock), 0, stream, w.runs,
                       p.nblocks, w.tile_total);
    hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanBlock), 0, stream, w.tile_total, p.ntiles,
                       p.seg_len, w.tile_start, w.seg_start);
    hipLaunchKernelGGL((scatter_kernel<DM>), dim3(p.nblocks), dim3(kScatterBlock), 0, stream,
                       w.pix, a.n, p.ntiles, p.nchunks, w.runs, w.tile_start, w.sorted);
    const int64_t ab = p.max_segments < 2 * cus ? p.max_segments : 2 * cus;
    hipLaunchKernelGGL(accumulate_kernel, dim3((unsigned)ab), dim3(kAccBlock), 0, stream,
                       w.tile_start, w.seg_start, p.ntiles, p.seg_len, w.sorted, w.partial);
    hipLaunchKernelGGL(reduce_kernel, dim3((unsigned)((npix + kReduceBlock - 1) / kReduceBlock)),
                       dim3(kReduceBlock), 0, stream, w.seg_start, w.partial, npix, a.win.hist);
    return hipGetLastError();
}

// The allocation-free entry point's workspace: one array per GPU, kept until
// the process ends.  Host code never passes `scratch` itself to a kernel (in
// host code the name stands for a host-side shadow, not a device address);
// it passes the device address hipGetSymbolAddress returns for the GPU that
// is current, looked up on the first call on each GPU.
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kSortScratchBytes];

}  // namespace

void* sortbin_scratch()
{
    static std::atomic<void*> address[kMaxScratchDevices];
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices)
        return nullptr;
    void* ptr = address[dev].load(std::memory_order_acquire);
    if (ptr == nullptr) {
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr)
            return nullptr;
        address[dev].store(ptr, std::memory_order_release);
    }
    return ptr;
}

int64_t sortbin_workspace(int64_t n, int dmax, int width, int height)
{
    return sortbin::workspace_bytes(sortbin::make_plan(n, dmax, width, height));
}

hipError_t launch_density_sorted(const DensityArgs& a, void* ws, int cus, hipStream_t stream)
{
    const sortbin::Plan p = sortbin::make_plan(a.n, a.dmax, a.win.width, a.win.height);
    if (p.direct)
        return launch_density(a, stream);
    switch (a.dmax) {
    case 1: return launch_dm<1>(a, p, ws, cus, stream);
    case 2: return launch_dm<2>(a, p, ws, cus, stream);
    case 3: return launch_dm<3>(a, p, ws, cus, stream);
    case 4: return launch_dm<4>(a, p, ws, cus, stream);
    case 5: return launch_dm<5>(a, p, ws, cus, stream);
    case 6: return launch_dm<6>(a, p, ws, cus, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace proots
