// Stand-ins for the library's kernel launchers, linked into the sanitizer build
// of the C ABI's host code in their place.  Each counts its call and reports a
// launch failure; the checks require that no argument-error path reaches one.
#include "../../paper_2201_11924_amd/csrc/internal.h"
#include "../../paper_2201_11924_amd/csrc/net_internal.h"

int g_stub_calls = 0;

namespace ss {

#define STUB(sig) sig { ++g_stub_calls; return hipErrorInvalidValue; }

STUB(hipError_t launch_agg_dpl1(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl2(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl4(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl6(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl8(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl12(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_agg_dpl16(const AggregateArgs *, const AggregateQueue *, int, int, bool, hipStream_t))
STUB(hipError_t launch_census(const uint8_t *, int, int, int, int, int, int, void *, bool, hipStream_t, unsigned *, int))
STUB(hipError_t launch_census_pair(const uint8_t *, const uint8_t *, int, int, int, int, int, int, void *, void *, bool,
                                   hipStream_t, unsigned *, int))
STUB(hipError_t launch_census_batch(const CensusBatch &, bool, hipStream_t))
STUB(hipError_t launch_ir_noise(const uint8_t *, const float *, const float *, uint8_t *, int64_t, hipStream_t))
STUB(hipError_t launch_select(const SelectArgs &, hipStream_t))
STUB(hipError_t launch_post(const PostArgs &, hipStream_t))
STUB(hipError_t launch_select_batch(const SelectBatch &, int, int, bool, hipStream_t))
STUB(hipError_t launch_post_batch(const PostBatch &, hipStream_t))
STUB(hipError_t launch_flip_census(const void *, void *, int, int, bool, hipStream_t))
STUB(hipError_t launch_lr_full(const LRFullArgs &, hipStream_t))
STUB(hipError_t launch_volume_sum(const PathSet &, int, bool, int, int, int, int, uint16_t *, hipStream_t))
STUB(hipError_t launch_block_cost(const BlockCostArgs &, int, bool, hipStream_t))
STUB(hipError_t launch_aggregate_volume(const VolumeArgs &, hipStream_t))

// the census tile count is host arithmetic the batch plan uses (32 x 8 tiles)
int census_tiles(int W, int H) { return ((W + 31) / 32) * ((H + 7) / 8); }

namespace net {
STUB(hipError_t launch_conv(const ConvArgs &, int, int, int, hipStream_t))
STUB(hipError_t launch_infer(InferArgs, hipStream_t))
STUB(hipError_t launch_wgrad(const WgradArgs &, int, int, hipStream_t))
int wgrad_blocks(int, int, int, int, int *rsplit) { *rsplit = 1; return 1; }
STUB(hipError_t launch_wgrad_reduce(const WgradReduceArgs &, hipStream_t))
STUB(hipError_t launch_loss(const LossArgs &, int, hipStream_t))
STUB(hipError_t launch_adam(const AdamArgs &, hipStream_t))
STUB(hipError_t launch_relayout(const RelayoutArgs &, hipStream_t))
STUB(hipError_t launch_features(const FeatureArgs &, hipStream_t))
STUB(hipError_t launch_combine(const CombineArgs &, hipStream_t))
STUB(hipError_t launch_targets(const float *, const uint8_t *, const float *, float *, uint8_t *, int64_t, hipStream_t))
}  // namespace net

}  // namespace ss
