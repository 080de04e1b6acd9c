// Instantiates the aggregation kernels for 6 disparities per lane.
#include "aggregate_impl.h"

namespace ss {

template <bool WIDE, int HL>
static hipError_t launch_one(const AggregateArgs *a, const AggregateQueue *q, int grid, hipStream_t s)
{
    constexpr int DPL = 6;
    if constexpr ((kLanesPerLine * DPL) % HL == 0) {
        if (a)
            hipLaunchKernelGGL((aggregate_kernel<DPL, WIDE, HL>), dim3(a->block_begin[a->ndirs]), dim3(kBlock), 0, s, *a);
        else
            hipLaunchKernelGGL((aggregate_queue_kernel<DPL, WIDE, HL>), dim3(grid), dim3(kBlock), 0, s, *q);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

hipError_t launch_agg_dpl6(const AggregateArgs *a, const AggregateQueue *q, int grid, int hl, bool wide, hipStream_t s)
{
    switch (hl) {
    case 16: return wide ? launch_one<true, 16>(a, q, grid, s) : launch_one<false, 16>(a, q, grid, s);
    case 32: return wide ? launch_one<true, 32>(a, q, grid, s) : launch_one<false, 32>(a, q, grid, s);
    case 64: return wide ? launch_one<true, 64>(a, q, grid, s) : launch_one<false, 64>(a, q, grid, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ss
