// Host side of the aggregation pass: work layout and dispatch to the
// per-disparity-count instantiations (agg_dpl*.hip).
#include <algorithm>

#include "internal.h"

namespace ss {

constexpr int kChunkClocks = 16;  // clocks per census tile chunk (= lines of a row-sharing block)

hipError_t launch_agg_dpl1(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl2(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl4(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl6(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl8(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl12(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);
hipError_t launch_agg_dpl16(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s);

namespace {
hipError_t launch_agg(const AggregateArgs *a, const AggregateQueue *q, int grid, int dpad, int hl, bool wide,
                      hipStream_t s)
{
    switch (dpad / kLanesPerLine) {
    case 1: return launch_agg_dpl1(a, q, grid, hl, wide, s);
    case 2: return launch_agg_dpl2(a, q, grid, hl, wide, s);
    case 4: return launch_agg_dpl4(a, q, grid, hl, wide, s);
    case 6: return launch_agg_dpl6(a, q, grid, hl, wide, s);
    case 8: return launch_agg_dpl8(a, q, grid, hl, wide, s);
    case 12: return launch_agg_dpl12(a, q, grid, hl, wide, s);
    case 16: return launch_agg_dpl16(a, q, grid, hl, wide, s);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

bool horizontal_lanes_valid(int dpad, int hl)
{
    return (hl == 16 || hl == 32 || hl == 64) && dpad % hl == 0;
}

int aggregate_blocks(int dx, int dy, int W, int H, int hl)
{
    if (dy == 0) {
        const int lines = kBlock / hl;
        return (H + lines - 1) / lines;
    }
    const int top = (W + kChunkClocks - 1) / kChunkClocks;
    if (dx == 0) return top;
    return top + (H - 1 + kChunkClocks - 1) / kChunkClocks;
}

int aggregate_block_clocks(int dx, int dy, int blk, int W, int H, int hl)
{
    if (dy == 0) return W;
    const int top = (W + kChunkClocks - 1) / kChunkClocks;
    if (dx == 0) return H;
    if (blk < top) {
        const int g0 = blk * kChunkClocks, nvalid = std::min(kChunkClocks, W - g0);
        const int lfirst = dx > 0 ? W - g0 : g0 + 1;
        const int llast = dx > 0 ? W - (g0 + nvalid - 1) : g0 + nvalid;
        return std::min(std::max(lfirst, llast), H);
    }
    const int j0 = (blk - top) * kChunkClocks, nvalid = std::min(kChunkClocks, H - 1 - j0);
    int c = 0;
    for (int i = 0; i < nvalid; ++i) c = std::max(c, i + std::min(W, H - j0 - i - 1));
    return c;
}

int aggregate_block_work(int dx, int dy, int blk, int W, int H, int hl, int dpad)
{
    const int cost = dy == 0 ? agg_step_cost(dpad / hl, hl) : agg_step_cost(dpad / kLanesPerLine, kLanesPerLine);
    return aggregate_block_clocks(dx, dy, blk, W, H, hl) * cost;
}

namespace {
__global__ void zero_counters_kernel(unsigned *c, int n)
{
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0u;
}
}  // namespace

hipError_t launch_zero_counters(unsigned *c, int n, hipStream_t s)
{
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(zero_counters_kernel, dim3(1), dim3(64), 0, s, c, n);
    return hipGetLastError();
}

hipError_t launch_aggregate(const AggregateArgs &a, bool wide, int hl, hipStream_t s)
{
    if (a.block_begin[a.ndirs] == 0) return hipSuccess;
    return launch_agg(&a, nullptr, 0, a.Dpad, hl, wide, s);
}

hipError_t launch_aggregate_queue(const AggregateQueue &q, int dpad, bool wide, int hl, int grid, hipStream_t s)
{
    if (q.nitems == 0) return hipSuccess;
    return launch_agg(nullptr, &q, grid, dpad, hl, wide, s);
}

}  // namespace ss
