// Internal declarations shared by the library's translation units (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/simsense.h"

namespace ss {

// Lanes that cooperate on one scanline: exactly one DPP row of a wave64, so
// every cross-lane step of the path recurrence is a row-local DPP operation.
constexpr int kLanesPerLine = 16;
constexpr int kLinesPerBlock = 16;  // 256-thread blocks
constexpr int kBlock = kLanesPerLine * kLinesPerBlock;

// Disparities held by each lane; the padded disparity count is 16 * dpl.
int pick_dpl(int max_disp);
inline int padded_disp(int max_disp) { return kLanesPerLine * pick_dpl(max_disp); }
int census_bits(int cw, int ch, int mode);

// Path directions: 2 paths = horizontal pair, 4 adds the vertical pair, 8 adds
// the four diagonals (same order as the header documents).
extern const int kPathDx[8];
extern const int kPathDy[8];
int path_lines(int dx, int dy, int W, int H);
// Default lanes per horizontal line.  Horizontal lines are the longest chains of
// the aggregation, so they get more lanes than the other lines (fewer
// instructions per step, a shorter chain) when the disparity count allows; 32
// lanes measured fastest for single 1280x720 pairs with 2 and with 8 paths.
constexpr int horizontal_lanes(int dpad) { return dpad % 32 == 0 ? 32 : 16; }
bool horizontal_lanes_valid(int dpad, int hl);
// blocks of work of one direction, and the clocks block `blk` runs
int aggregate_blocks(int dx, int dy, int W, int H, int hl);
int aggregate_block_clocks(int dx, int dy, int blk, int W, int H, int hl);
// Estimated VALU instructions per clock of a wave of a line block: about 7 per
// disparity a lane holds, plus the per-step line overhead (larger for lines
// spread over more than one DPP row).  The work of a block is clocks x this.
constexpr int agg_step_cost(int dpl, int lanes_per_line) { return 7 * dpl + (lanes_per_line == 16 ? 10 : 18); }
int aggregate_block_work(int dx, int dy, int blk, int W, int H, int hl, int dpad);

struct AggregateArgs {
    const void *census_l, *census_r;  // uint32 words, or uint64 when bits > 32
    int W, H, D, Dpad, bits, p1, p2;
    int ndirs;
    int dx[8], dy[8];
    int block_begin[9];  // first block index of each direction, prefix sums
    uint8_t *out[8];     // per-direction path values, W*H*Dpad bytes, d fastest
    int max_item_work;   // largest block work of the launch (issue priorities)
};

struct SelectArgs {
    const uint8_t *paths[8];  // 8-bit path values, or 16-bit when values16
    int values16;
    int ndirs;
    int W, H, D, Dpad;
    int uniqueness_pct, lr_max_diff, subpixel;
    int small_values;     // every path value < 128 (bits + P2 <= 127)
    uint8_t *disp_int;    // W*H
    uint16_t *cost_best;  // W*H
    uint16_t *cost_second;
    uint8_t *disp_right;
    float *disp_sub;      // before masking
    float *masked;        // masked sub-pixel disparity (0 = invalid)
    uint8_t *flags;       // bits 0..2
    int no_right;         // skip the right-image disparity (no LR check, disp_right unwritten)
};

struct PostArgs {
    const float *masked;
    const uint8_t *flags_in;
    int W, H, median;
    float fb;
    float *disp;     // may be null
    float *depth;    // may be null
    uint8_t *flags;  // may be null
};

hipError_t launch_ir_noise(const uint8_t *in, const float *gamma, const float *n, uint8_t *out,
                           int64_t count, hipStream_t s);
// (zero, nzero: counters the census launch clears on the way, so the work-queue
// launch that follows needs no kernel of its own for that)
hipError_t launch_census(const uint8_t *img, int pitch, int W, int H, int cw, int ch, int mode,
                         void *out, bool out64, hipStream_t s, unsigned *zero = nullptr, int nzero = 0);
// both images of a pair in one launch (img1 may be null: img0 alone)
hipError_t launch_census_pair(const uint8_t *img0, const uint8_t *img1, int pitch, int W, int H, int cw, int ch,
                              int mode, void *out0, void *out1, bool out64, hipStream_t s, unsigned *zero = nullptr,
                              int nzero = 0);
struct AggregateQueue {
    const AggregateArgs *slots;  // per pair slot (device)
    const uint32_t *items;       // slot << 20 | block, longest first (device)
    int nitems;
    unsigned *counter;           // zero before the launch
};
hipError_t launch_aggregate(const AggregateArgs &a, bool wide, int hl, hipStream_t s);
// zeroes n <= 64 queue counters (a kernel, so that it may sit in a captured graph)
hipError_t launch_zero_counters(unsigned *c, int n, hipStream_t s);
hipError_t launch_aggregate_queue(const AggregateQueue &q, int dpad, bool wide, int hl, int grid, hipStream_t s);
hipError_t launch_select(const SelectArgs &a, hipStream_t s);
hipError_t launch_post(const PostArgs &a, hipStream_t s);
// Semi-global block matching: the block-cost volume and the aggregation fed
// from it (16-bit path values, one block per line block).
constexpr int kMaxBlockHalf = 15;  // SGBM blocks are at most 31 x 31
// lanes per horizontal line of the block-cost-fed aggregation
__host__ __device__ constexpr int volume_horizontal_lanes(int dpad)
{
    return dpad == 128 || dpad == 256 ? 64 : dpad == 64 ? 32 : kLanesPerLine;
}
struct BlockCostArgs {
    const void *census_l, *census_r;  // uint32 words, or uint64 when bits > 32
    int W, H, bits, bw, bh;
    uint16_t *vol;                    // W*H*Dpad, d fastest
};
struct VolumeArgs {
    const uint16_t *vol;
    int W, H, D, Dpad, p1, p2;
    int ndirs;
    int dx[8], dy[8];
    int block_begin[9];  // 16-line blocks, prefix sums per direction
    uint16_t *out[8];    // per-direction path values, (W*H + 1)*Dpad
};
hipError_t launch_block_cost(const BlockCostArgs &a, int dpad, bool wide, hipStream_t s);
hipError_t launch_aggregate_volume(const VolumeArgs &a, hipStream_t s);

// x-flip of a census map (words of 4 or 8 bytes)
hipError_t launch_flip_census(const void *src, void *dst, int W, int H, bool wide, hipStream_t s);
// LR check against a full right-referenced run whose winners are given in
// x-flipped order (dint_m[y][W-1-xr] = dR(xr)): rewrites flag bit 1 and the
// masked disparity, and writes the right disparities
struct LRFullArgs {
    const uint8_t *dint, *dint_m;
    const float *disp_sub;
    uint8_t *flags;      // in: bits 0 and 2 of the left selection; out: bit 1 rewritten
    float *masked;
    uint8_t *disp_right;
    int W, H, lr;
};
hipError_t launch_lr_full(const LRFullArgs &a, hipStream_t s);

// batched forms: per-slot arguments in device memory, one block per item
// (slot << 20 | index), items in device memory
struct CensusJob {
    const uint8_t *img;
    int pitch, W, H, cw, ch, mode;
    void *out;
};
struct CensusBatch {
    const CensusJob *jobs;
    const uint32_t *items;
    int nitems, max_cw, max_ch;
    unsigned *zero;  // counters cleared by the first block (nzero of them)
    int nzero;
};
struct SelectBatch {
    const SelectArgs *slots;
    const uint32_t *items;  // slot << 20 | row
    int nitems, max_width;
    int no_right;           // as SelectArgs::no_right, for every slot of the launch
};
struct PostBatch {
    const PostArgs *slots;
    const uint32_t *items;  // slot << 20 | tile (64x4 tiles, row-major)
    int nitems;
};
hipError_t launch_census_batch(const CensusBatch &b, bool out64, hipStream_t s);
hipError_t launch_select_batch(const SelectBatch &b, int dpad, int ndirs, bool small, hipStream_t s);
hipError_t launch_post_batch(const PostBatch &b, hipStream_t s);
int census_tiles(int W, int H);
struct PathSet {
    const uint8_t *p[8];
};
hipError_t launch_volume_sum(const PathSet &paths, int ndirs, bool values16, int W, int H, int D, int Dpad,
                             uint16_t *out, hipStream_t s);

// ---------------------------------------------------------------- handle
// Parameter validation (a simsense_status) and the handle's scratch layout: one
// block holding the census maps, the per-direction path values, the per-pixel
// results (and for lr_mode 1 a second set; for SGBM the block-cost volume),
// every piece 256-byte aligned.
int validate(const simsense_params *p);
struct Layout {
    size_t census, paths, per_px[7], total;
    bool right_run;  // lr_mode 1: two more census maps and a second per-pixel set
    size_t volume;   // SGBM: the block-cost volume (16-bit, d fastest)
};
Layout layout(const simsense_params *p);
// fields derived from the parameters; the buffers carved from `base` (l.total bytes)
void init_handle(simsense_handle *h, const simsense_params *params);
void carve_scratch(simsense_handle *h, uint8_t *base, const Layout &l);
// Work common to the compute entry points; each returns a simsense_status.
//  enqueue_match: census, aggregation and selection into the handle's scratch
//                 (d*, S1, S2, dR, sub-pixel, masked disparity, flags bits 0..2);
//  enqueue_post:  median + depth of a masked map into the caller's outputs.
//                 (volume_out, if set, receives the summed path costs S)
//                 (need_right = false: the learned form, which reads only d*, S1,
//                 S2 and the sub-pixel disparity, skips the right-image disparity)
int enqueue_match(simsense_handle *h, const uint8_t *left, const uint8_t *right, int pitch, hipStream_t s,
                  uint16_t *volume_out = nullptr, bool need_right = true);
int enqueue_post(simsense_handle *h, const float *masked, const uint8_t *flags_pre, const simsense_outputs *o,
                 hipStream_t s);
int profile_begin_call(simsense_handle *h);
void profile_end_call(simsense_handle *h);
void profile_mark(simsense_handle *h, int pass, bool end, hipStream_t s);

}  // namespace ss

struct simsense_handle {  // opaque to callers
    simsense_params p;
    int bits, Dpad, ndirs;
    int hlanes;  // lanes per horizontal scanline
    bool wide;
    // launch shape of the aggregation; for the persistent form, the work list
    // (line blocks longest first), its counter and the argument block on the device
    simsense_batch_tuning tuning;
    int num_cus, nitems;
    uint32_t *d_items;
    unsigned *d_counter;
    ss::AggregateArgs *d_args;
    // full right-referenced run (lr_mode 1): x-flipped census maps (the right
    // image's as the reference), that run's per-pixel results and its arguments
    void *census_ml, *census_mr;
    uint8_t *disp_int_m, *disp_right_m, *flags_m;
    uint16_t *cost_best_m, *cost_second_m;
    float *disp_sub_m, *masked_m;
    ss::AggregateArgs *d_args_m;
    // semi-global block matching: 16-bit path values fed from a block-cost volume
    bool sgbm;
    uint16_t *volume;
    void *block;
    void *census_l, *census_r;
    uint8_t *paths[8];
    uint8_t *disp_int, *disp_right, *flags_pre;
    uint16_t *cost_best, *cost_second;
    float *disp_sub, *masked;
    hipStream_t last_stream;
    // profiling: call slots of 2 events per pass
    bool profiling;
    int prof_used;
    int prof_calls;
    double prof_ms[SIMSENSE_NUM_PASSES];
    hipEvent_t *prof_events;
};
