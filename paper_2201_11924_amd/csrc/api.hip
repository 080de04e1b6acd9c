// C ABI of the depth library: parameter validation, the handle and its device
// scratch, and the order in which the passes are enqueued.
#include <algorithm>
#include <new>
#include <string.h>
#include <utility>
#include <vector>

#include "internal.h"
#include "net_internal.h"
#include "trace.h"

namespace ss {

const int kPathDx[8] = {1, -1, 0, 0, 1, -1, 1, -1};
const int kPathDy[8] = {0, 0, 1, -1, 1, 1, -1, -1};

int pick_dpl(int max_disp)
{
    static const int options[] = {1, 2, 4, 6, 8, 12, 16};
    for (int o : options)
        if (kLanesPerLine * o >= max_disp) return o;
    return 16;
}

int census_bits(int cw, int ch, int mode)
{
    const int n = cw * ch;
    return mode == 0 ? (n - 1) / 2 : n - 1;
}

int path_lines(int dx, int dy, int W, int H) { return dy == 0 ? H : (dx == 0 ? W : W + H - 1); }

int validate(const simsense_params *p)
{
    if (!p) return SIMSENSE_ERR_NULL_POINTER;
    if (p->struct_size != sizeof(simsense_params)) return SIMSENSE_ERR_ABI;
    if (p->width < 1 || p->height < 1 || p->width > 8192 || p->height > 8192)
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->max_disp < 1 || p->max_disp > 256) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->census_w < 1 || p->census_h < 1 || !(p->census_w & 1) || !(p->census_h & 1))
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->census_mode != 0 && p->census_mode != 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    // (the sides are bounded before they are multiplied)
    if (p->census_w > 65 || p->census_h > 65) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->census_w * p->census_h < 3) return SIMSENSE_ERR_INVALID_ARGUMENT;
    const int bits = census_bits(p->census_w, p->census_h, p->census_mode);
    if (bits > 64) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->block_w < 1 || p->block_h < 1 || p->block_w > 2 * kMaxBlockHalf + 1 || p->block_h > 2 * kMaxBlockHalf + 1 || !(p->block_w & 1) ||
        !(p->block_h & 1))
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    const bool block = p->block_w * p->block_h > 1;
    if (p->p1 < 0 || p->p2 < p->p1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (!block && bits + p->p2 > 255) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (block && bits * p->block_w * p->block_h + p->p2 > 8191) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->uniqueness_pct < 0 || p->uniqueness_pct > 99) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->num_paths != 2 && p->num_paths != 4 && p->num_paths != 8) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->median != 0 && p->median != 3) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->subpixel != 0 && p->subpixel != 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (!(p->focal_px == p->focal_px) || !(p->baseline_m == p->baseline_m)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->lr_mode != 0 && p->lr_mode != 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    return SIMSENSE_OK;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout(const simsense_params *p)
{
    Layout l{};
    const size_t npx = (size_t)p->width * p->height;
    const bool wide = census_bits(p->census_w, p->census_h, p->census_mode) > 32;
    l.census = align256(npx * (wide ? 8 : 4));
    const bool block = p->block_w * p->block_h > 1;
    // + one spare pixel for idle lanes; 16-bit path values for block matching
    l.paths = align256((npx + 1) * padded_disp(p->max_disp) * (block ? 2 : 1));
    l.volume = block ? align256(npx * padded_disp(p->max_disp) * 2) : 0;
    static const int px_bytes[7] = {1, 2, 2, 1, 4, 4, 1};  // dint, S1, S2, dright, dsub, masked, flags
    l.right_run = p->lr_mode == 1;
    const int sets = l.right_run ? 2 : 1;
    l.total = 2 * sets * l.census + (size_t)p->num_paths * l.paths + l.volume;
    for (int i = 0; i < 7; ++i) {
        l.per_px[i] = align256(npx * px_bytes[i]);
        l.total += sets * l.per_px[i];
    }
    return l;
}

// The handle's parameter-derived fields (no device work).
void init_handle(simsense_handle *h, const simsense_params *params)
{
    h->p = *params;
    h->bits = census_bits(params->census_w, params->census_h, params->census_mode);
    h->wide = h->bits > 32;
    h->Dpad = padded_disp(params->max_disp);
    h->hlanes = horizontal_lanes(h->Dpad);
    h->ndirs = params->num_paths;
    h->sgbm = params->block_w * params->block_h > 1;
}

// Points the handle's buffers into one block of scratch laid out by layout().
void carve_scratch(simsense_handle *h, uint8_t *base, const Layout &l)
{
    uint8_t *cur = base;
    h->census_l = cur; cur += l.census;
    h->census_r = cur; cur += l.census;
    for (int r = 0; r < h->ndirs; ++r) { h->paths[r] = cur; cur += l.paths; }
    h->disp_int = cur; cur += l.per_px[0];
    h->cost_best = (uint16_t *)cur; cur += l.per_px[1];
    h->cost_second = (uint16_t *)cur; cur += l.per_px[2];
    h->disp_right = cur; cur += l.per_px[3];
    h->disp_sub = (float *)cur; cur += l.per_px[4];
    h->masked = (float *)cur; cur += l.per_px[5];
    h->flags_pre = cur; cur += l.per_px[6];
    if (l.volume) {
        h->volume = (uint16_t *)cur;
        cur += l.volume;
    }
    if (l.right_run) {
        h->census_ml = cur; cur += l.census;
        h->census_mr = cur; cur += l.census;
        h->disp_int_m = cur; cur += l.per_px[0];
        h->cost_best_m = (uint16_t *)cur; cur += l.per_px[1];
        h->cost_second_m = (uint16_t *)cur; cur += l.per_px[2];
        h->disp_right_m = cur; cur += l.per_px[3];
        h->disp_sub_m = (float *)cur; cur += l.per_px[4];
        h->masked_m = (float *)cur; cur += l.per_px[5];
        h->flags_m = cur; cur += l.per_px[6];
    }
}

}  // namespace ss

using namespace ss;



namespace {
constexpr int kProfSlots = 256;

hipEvent_t *prof_slot(simsense_handle *h, int pass, bool end)
{
    return &h->prof_events[(size_t)h->prof_used * (2 * SIMSENSE_NUM_PASSES) + 2 * pass + (end ? 1 : 0)];
}

// waits for the recorded events and folds them into the accumulators
int prof_harvest(simsense_handle *h)
{
    for (int c = 0; c < h->prof_used; ++c)
        for (int p = 0; p < SIMSENSE_NUM_PASSES; ++p) {
            hipEvent_t b = h->prof_events[(size_t)c * 2 * SIMSENSE_NUM_PASSES + 2 * p];
            hipEvent_t e = h->prof_events[(size_t)c * 2 * SIMSENSE_NUM_PASSES + 2 * p + 1];
            if (hipEventSynchronize(e) != hipSuccess) return SIMSENSE_ERR_DEVICE;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, b, e) != hipSuccess) return SIMSENSE_ERR_DEVICE;
            h->prof_ms[p] += ms;
        }
    h->prof_calls += h->prof_used;
    h->prof_used = 0;
    return SIMSENSE_OK;
}

void prof_free(simsense_handle *h)
{
    if (!h->prof_events) return;
    for (int i = 0; i < kProfSlots * 2 * SIMSENSE_NUM_PASSES; ++i) (void)hipEventDestroy(h->prof_events[i]);
    delete[] h->prof_events;
    h->prof_events = nullptr;
}
}  // namespace

namespace ss {

int profile_begin_call(simsense_handle *h)
{
    if (h->profiling && h->prof_used == kProfSlots) return prof_harvest(h);
    return SIMSENSE_OK;
}

void profile_end_call(simsense_handle *h)
{
    if (h->profiling) ++h->prof_used;
}

void profile_mark(simsense_handle *h, int pass, bool end, hipStream_t s)
{
    if (h->profiling) (void)hipEventRecord(*prof_slot(h, pass, end), s);
}

#define SS_TRY(expr) \
    do { if ((expr) != hipSuccess) { (void)hipGetLastError(); return SIMSENSE_ERR_DEVICE; } } while (0)

// The handle's aggregation arguments (every pointer is handle scratch, so they
// are fixed for its life).
static AggregateArgs handle_aggregate_args(const simsense_handle *h)
{
    const simsense_params &p = h->p;
    AggregateArgs ag{};
    ag.census_l = h->census_l;
    ag.census_r = h->census_r;
    ag.W = p.width; ag.H = p.height; ag.D = p.max_disp; ag.Dpad = h->Dpad; ag.bits = h->bits;
    ag.p1 = p.p1; ag.p2 = p.p2;
    ag.ndirs = h->ndirs;
    ag.block_begin[0] = 0;
    for (int r = 0; r < h->ndirs; ++r) {
        ag.dx[r] = kPathDx[r];
        ag.dy[r] = kPathDy[r];
        ag.out[r] = h->paths[r];
        ag.block_begin[r + 1] = ag.block_begin[r] + aggregate_blocks(kPathDx[r], kPathDy[r], p.width, p.height, h->hlanes);
        for (int k = 0; k < ag.block_begin[r + 1] - ag.block_begin[r]; ++k)
            ag.max_item_work = std::max(ag.max_item_work, aggregate_block_work(kPathDx[r], kPathDy[r], k, p.width,
                                                                               p.height, h->hlanes, h->Dpad));
    }
    return ag;
}

// The right-referenced run is the left-referenced pass on x-flipped census maps
// with the roles swapped (the right image's map as the reference); the set of
// path directions is closed under the flip, so only the census inputs change.
static AggregateArgs right_run_args(AggregateArgs ag, const simsense_handle *h)
{
    ag.census_l = h->census_ml;
    ag.census_r = h->census_mr;
    return ag;
}

static int launch_aggregation(simsense_handle *h, const AggregateArgs &ag, AggregateArgs *d_args, hipStream_t s)
{
    if (h->tuning.blocks_per_cu > 0) {
        AggregateQueue q{};
        q.slots = d_args;
        q.items = h->d_items;
        q.nitems = h->nitems;
        q.counter = h->d_counter;
        const int grid = std::min(h->nitems, h->tuning.blocks_per_cu * h->num_cus);
        SS_TRY(launch_zero_counters(h->d_counter, 1, s));
        SS_TRY(launch_aggregate_queue(q, h->Dpad, h->wide, h->hlanes, grid, s));
    } else {
        SS_TRY(launch_aggregate(ag, h->wide, h->hlanes, s));
    }
    return SIMSENSE_OK;
}

// Block matching (SGBM): block costs of the given census maps into the volume,
// then the aggregation fed from it into the path buffers (16-bit values).
static int sgbm_aggregation(simsense_handle *h, const void *cl, const void *cr, hipStream_t s)
{
    const simsense_params &p = h->p;
    BlockCostArgs bc{};
    bc.census_l = cl; bc.census_r = cr;
    bc.W = p.width; bc.H = p.height; bc.bits = h->bits; bc.bw = p.block_w; bc.bh = p.block_h;
    bc.vol = h->volume;
    SS_TRY(launch_block_cost(bc, h->Dpad, h->wide, s));
    VolumeArgs va{};
    va.vol = h->volume;
    va.W = p.width; va.H = p.height; va.D = p.max_disp; va.Dpad = h->Dpad; va.p1 = p.p1; va.p2 = p.p2;
    va.ndirs = h->ndirs;
    va.block_begin[0] = 0;
    for (int r = 0; r < h->ndirs; ++r) {
        va.dx[r] = kPathDx[r];
        va.dy[r] = kPathDy[r];
        va.out[r] = (uint16_t *)h->paths[r];
        va.block_begin[r + 1] = va.block_begin[r] + aggregate_blocks(kPathDx[r], kPathDy[r], p.width, p.height,
                                                                     volume_horizontal_lanes(h->Dpad));
    }
    SS_TRY(launch_aggregate_volume(va, s));
    return SIMSENSE_OK;
}

// Applies a tuning: lane count, and for the persistent form the work list of
// line blocks sorted by estimated work, largest first (stable, so equal work
// keeps direction order).
static int apply_tuning(simsense_handle *h, const simsense_batch_tuning &t)
{
    const int hl = t.horizontal_lanes == 0 ? horizontal_lanes(h->Dpad) : t.horizontal_lanes;
    if (!horizontal_lanes_valid(h->Dpad, hl)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    h->hlanes = hl;
    h->tuning = t;
    const AggregateArgs ag = handle_aggregate_args(h);
    std::vector<std::pair<int, uint32_t>> lst;
    for (int r = 0; r < h->ndirs; ++r)
        for (int k = 0; k < ag.block_begin[r + 1] - ag.block_begin[r]; ++k)
            lst.push_back({aggregate_block_work(kPathDx[r], kPathDy[r], k, h->p.width, h->p.height, hl, h->Dpad),
                           (uint32_t)(ag.block_begin[r] + k)});
    std::stable_sort(lst.begin(), lst.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
    std::vector<uint32_t> items(lst.size());
    for (size_t i = 0; i < lst.size(); ++i) items[i] = lst[i].second;  // pair slot 0
    if (h->d_items) (void)hipFree(h->d_items);
    h->d_items = nullptr;
    h->nitems = (int)items.size();
    SS_TRY(hipMalloc(&h->d_items, std::max<size_t>(items.size(), 1) * sizeof(uint32_t)));
    if (!items.empty()) SS_TRY(hipMemcpy(h->d_items, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    SS_TRY(hipMemcpy(h->d_args, &ag, sizeof(ag), hipMemcpyHostToDevice));
    if (h->p.lr_mode == 1) {
        const AggregateArgs am = right_run_args(ag, h);
        SS_TRY(hipMemcpy(h->d_args_m, &am, sizeof(am), hipMemcpyHostToDevice));
    }
    return SIMSENSE_OK;
}

int enqueue_match(simsense_handle *h, const uint8_t *left, const uint8_t *right, int pitch, hipStream_t s,
                  uint16_t *volume_out, bool need_right)
{
    const simsense_params &p = h->p;
    const int W = p.width, H = p.height, D = p.max_disp;
    h->last_stream = s;
    TraceRange range("simsense match");
    profile_mark(h, SIMSENSE_PASS_CENSUS, false, s);
    const bool queue = !h->sgbm && h->tuning.blocks_per_cu > 0;
    // (the census launch also clears the work-queue counter)
    SS_TRY(launch_census_pair(left, right, pitch, W, H, p.census_w, p.census_h, p.census_mode, h->census_l,
                              h->census_r, h->wide, s, queue ? h->d_counter : nullptr, queue ? 1 : 0));
    profile_mark(h, SIMSENSE_PASS_CENSUS, true, s);

    const AggregateArgs ag = handle_aggregate_args(h);
    profile_mark(h, SIMSENSE_PASS_AGGREGATE, false, s);
    if (h->sgbm) {
        // block costs, then the aggregation fed from them
        const int rc = sgbm_aggregation(h, h->census_l, h->census_r, s);
        if (rc != SIMSENSE_OK) return rc;
    } else if (queue) {
        AggregateQueue q{};
        q.slots = h->d_args;
        q.items = h->d_items;
        q.nitems = h->nitems;
        q.counter = h->d_counter;
        const int grid = std::min(h->nitems, h->tuning.blocks_per_cu * h->num_cus);
        SS_TRY(launch_aggregate_queue(q, h->Dpad, h->wide, h->hlanes, grid, s));
    } else {
        SS_TRY(launch_aggregate(ag, h->wide, h->hlanes, s));
    }
    profile_mark(h, SIMSENSE_PASS_AGGREGATE, true, s);
    if (volume_out) {
        // the summed volume of this (left-referenced) run, before a right-referenced
        // run reuses the path buffers
        PathSet ps{};
        for (int r = 0; r < h->ndirs; ++r) ps.p[r] = h->paths[r];
        SS_TRY(launch_volume_sum(ps, h->ndirs, h->sgbm, W, H, D, h->Dpad, volume_out, s));
    }

    SelectArgs sa{};
    for (int r = 0; r < h->ndirs; ++r) sa.paths[r] = h->paths[r];
    sa.ndirs = h->ndirs;
    sa.W = W; sa.H = H; sa.D = D; sa.Dpad = h->Dpad;
    sa.uniqueness_pct = p.uniqueness_pct; sa.lr_max_diff = p.lr_max_diff; sa.subpixel = p.subpixel;
    sa.values16 = h->sgbm;
    sa.small_values = !h->sgbm && h->bits + p.p2 <= 127;
    sa.disp_int = h->disp_int; sa.cost_best = h->cost_best; sa.cost_second = h->cost_second;
    sa.disp_right = h->disp_right; sa.disp_sub = h->disp_sub; sa.masked = h->masked; sa.flags = h->flags_pre;
    sa.no_right = !need_right;
    profile_mark(h, SIMSENSE_PASS_SELECT, false, s);
    SS_TRY(launch_select(sa, s));
    if (p.lr_mode == 1) {
        // full right-referenced run into the second per-pixel set, then the check
        SS_TRY(launch_flip_census(h->census_r, h->census_ml, W, H, h->wide, s));
        SS_TRY(launch_flip_census(h->census_l, h->census_mr, W, H, h->wide, s));
        const int rc = h->sgbm ? sgbm_aggregation(h, h->census_ml, h->census_mr, s)
                               : launch_aggregation(h, right_run_args(ag, h), h->d_args_m, s);
        if (rc != SIMSENSE_OK) return rc;
        SelectArgs sm = sa;
        sm.uniqueness_pct = 0;
        sm.lr_max_diff = -1;
        sm.disp_int = h->disp_int_m; sm.cost_best = h->cost_best_m; sm.cost_second = h->cost_second_m;
        sm.disp_right = h->disp_right_m; sm.disp_sub = h->disp_sub_m; sm.masked = h->masked_m;
        sm.flags = h->flags_m;
        SS_TRY(launch_select(sm, s));
        LRFullArgs lf{};
        lf.dint = h->disp_int; lf.dint_m = h->disp_int_m; lf.disp_sub = h->disp_sub;
        lf.flags = h->flags_pre; lf.masked = h->masked; lf.disp_right = h->disp_right;
        lf.W = W; lf.H = H; lf.lr = p.lr_max_diff;
        SS_TRY(launch_lr_full(lf, s));
    }
    profile_mark(h, SIMSENSE_PASS_SELECT, true, s);
    return SIMSENSE_OK;
}

int enqueue_post(simsense_handle *h, const float *masked, const uint8_t *flags_pre, const simsense_outputs *o,
                 hipStream_t s)
{
    const simsense_params &p = h->p;
    PostArgs pa{};
    pa.masked = masked; pa.flags_in = flags_pre;
    pa.W = p.width; pa.H = p.height; pa.median = p.median;
    pa.fb = p.focal_px * p.baseline_m;
    pa.disp = o->disp; pa.depth = o->depth; pa.flags = o->flags;
    TraceRange range("simsense post");
    profile_mark(h, SIMSENSE_PASS_POST, false, s);
    if (pa.disp || pa.depth || pa.flags) SS_TRY(launch_post(pa, s));
    profile_mark(h, SIMSENSE_PASS_POST, true, s);
    return SIMSENSE_OK;
}
#undef SS_TRY

}  // namespace ss

extern "C" {

const char *simsense_strerror(int status)
{
    switch (status) {
    case SIMSENSE_OK: return "ok";
    case SIMSENSE_ERR_INVALID_ARGUMENT: return "invalid argument";
    case SIMSENSE_ERR_NULL_POINTER: return "required pointer is NULL";
    case SIMSENSE_ERR_OUT_OF_MEMORY: return "device out of memory";
    case SIMSENSE_ERR_DEVICE: return "HIP runtime or kernel launch error";
    case SIMSENSE_ERR_UNSUPPORTED: return "unsupported configuration";
    case SIMSENSE_ERR_ABI: return "struct_size mismatch (ABI)";
    case SIMSENSE_ERR_TOO_LARGE: return "scratch needed exceeds the no-allocation entry point's static buffer";
    default: return "unknown status";
    }
}

int64_t simsense_scratch_bytes(const simsense_params *params)
{
    int rc = validate(params);
    if (rc != SIMSENSE_OK) return rc;
    return (int64_t)layout(params).total;
}

int simsense_create(const simsense_params *params, simsense_handle **out)
{
    if (!out) return SIMSENSE_ERR_NULL_POINTER;
    int rc = validate(params);
    if (rc != SIMSENSE_OK) return rc;
    Layout l = layout(params);
    simsense_handle *h = new (std::nothrow) simsense_handle();
    if (!h) return SIMSENSE_ERR_OUT_OF_MEMORY;
    init_handle(h, params);
    if (hipDeviceGetAttribute(&h->num_cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess) {
        (void)hipGetLastError();
        h->num_cus = 256;
    }
    if (hipMalloc(&h->block, l.total) != hipSuccess || hipMalloc(&h->d_counter, 256) != hipSuccess ||
        hipMalloc(&h->d_args, 2 * sizeof(AggregateArgs)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(h->block);
        (void)hipFree(h->d_counter);
        delete h;
        return SIMSENSE_ERR_OUT_OF_MEMORY;
    }
    h->d_args_m = h->d_args + 1;
    carve_scratch(h, (uint8_t *)h->block, l);
    h->last_stream = nullptr;
    h->profiling = false;
    h->prof_events = nullptr;
    h->prof_used = h->prof_calls = 0;
    simsense_batch_tuning t{};
    t.struct_size = sizeof(t);
    t.horizontal_lanes = 0;
    t.blocks_per_cu = 3;
    rc = apply_tuning(h, t);
    if (rc != SIMSENSE_OK) {
        (void)simsense_destroy(h);
        return rc;
    }
    *out = h;
    return SIMSENSE_OK;
}

int simsense_destroy(simsense_handle *h)
{
    if (!h) return SIMSENSE_OK;
    int rc = SIMSENSE_OK;
    if (hipStreamSynchronize(h->last_stream) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (hipFree(h->block) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (hipFree(h->d_items) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (hipFree(h->d_counter) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (hipFree(h->d_args) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    prof_free(h);
    delete h;
    return rc;
}

int simsense_compute_ex(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch,
                        const simsense_outputs *o, void *stream)
{
    if (!h || !left || !right || !o) return SIMSENSE_ERR_NULL_POINTER;
    const simsense_params &p = h->p;
    if (pitch < p.width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    const int W = p.width, H = p.height, D = p.max_disp;
    const size_t npx = (size_t)W * H;
    TraceRange range("simsense_compute");
    int rc = profile_begin_call(h);
    if (rc != SIMSENSE_OK) return rc;
    rc = enqueue_match(h, left, right, pitch, s, o->volume);
    if (rc != SIMSENSE_OK) return rc;
    rc = enqueue_post(h, h->masked, h->flags_pre, o, s);
    if (rc != SIMSENSE_OK) return rc;
    profile_end_call(h);
#define SS_TRY(expr) \
    do { if ((expr) != hipSuccess) { (void)hipGetLastError(); return SIMSENSE_ERR_DEVICE; } } while (0)
    if (o->disp_int) SS_TRY(hipMemcpyAsync(o->disp_int, h->disp_int, npx, hipMemcpyDeviceToDevice, s));
    if (o->cost_best) SS_TRY(hipMemcpyAsync(o->cost_best, h->cost_best, npx * 2, hipMemcpyDeviceToDevice, s));
    if (o->cost_second)
        SS_TRY(hipMemcpyAsync(o->cost_second, h->cost_second, npx * 2, hipMemcpyDeviceToDevice, s));
    if (o->disp_right) SS_TRY(hipMemcpyAsync(o->disp_right, h->disp_right, npx, hipMemcpyDeviceToDevice, s));
    if (o->disp_sub) SS_TRY(hipMemcpyAsync(o->disp_sub, h->disp_sub, npx * 4, hipMemcpyDeviceToDevice, s));
    if (o->census_left)
        SS_TRY(launch_census(left, pitch, W, H, p.census_w, p.census_h, p.census_mode, o->census_left, true, s));
    if (o->census_right)
        SS_TRY(launch_census(right, pitch, W, H, p.census_w, p.census_h, p.census_mode, o->census_right, true, s));
    if (o->features) {
        net::FeatureArgs fa{};
        fa.ir = left; fa.pitch = pitch; fa.W = W;
        fa.s1 = h->cost_best; fa.s2 = h->cost_second; fa.dint = h->disp_int;
        fa.max_disp = D; fa.smax = (float)(h->ndirs * (h->bits * p.block_w * p.block_h + p.p2));
        fa.features = o->features; fa.P = (int64_t)npx;
        SS_TRY(net::launch_features(fa, s));
    }
#undef SS_TRY
    return SIMSENSE_OK;
}

int simsense_profile_enable(simsense_handle *h, int enable)
{
    if (!h) return SIMSENSE_ERR_NULL_POINTER;
    if (enable && !h->prof_events) {
        const int n = kProfSlots * 2 * SIMSENSE_NUM_PASSES;
        h->prof_events = new (std::nothrow) hipEvent_t[n]();
        if (!h->prof_events) return SIMSENSE_ERR_OUT_OF_MEMORY;
        for (int i = 0; i < n; ++i)
            if (hipEventCreate(&h->prof_events[i]) != hipSuccess) {
                (void)hipGetLastError();
                for (int k = 0; k < i; ++k) (void)hipEventDestroy(h->prof_events[k]);
                delete[] h->prof_events;
                h->prof_events = nullptr;
                return SIMSENSE_ERR_DEVICE;
            }
        h->prof_used = h->prof_calls = 0;
        for (double &v : h->prof_ms) v = 0.0;
    }
    h->profiling = enable != 0;
    return SIMSENSE_OK;
}

int simsense_profile_read(simsense_handle *h, double *ms, int32_t *calls, int32_t n)
{
    if (!h || !ms || !calls) return SIMSENSE_ERR_NULL_POINTER;
    if (n < 0) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (h->prof_events) {
        int rc = prof_harvest(h);
        if (rc != SIMSENSE_OK) return rc;
    }
    for (int i = 0; i < n && i < SIMSENSE_NUM_PASSES; ++i) ms[i] = h->prof_ms[i];
    *calls = h->prof_calls;
    for (double &v : h->prof_ms) v = 0.0;
    h->prof_calls = 0;
    return SIMSENSE_OK;
}

int simsense_compute(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch, float *depth,
                     float *disp, uint8_t *flags, void *stream)
{
    if (!depth) return SIMSENSE_ERR_NULL_POINTER;
    simsense_outputs o{};
    o.depth = depth;
    o.disp = disp;
    o.flags = flags;
    return simsense_compute_ex(h, left, right, pitch, &o, stream);
}

int simsense_ir_noise(const uint8_t *in, const float *gamma, const float *n, uint8_t *out, int64_t count,
                      void *stream)
{
    if (count < 0) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (count == 0) return SIMSENSE_OK;
    if (!in || !gamma || !n || !out) return SIMSENSE_ERR_NULL_POINTER;
    if (launch_ir_noise(in, gamma, n, out, count, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return SIMSENSE_ERR_DEVICE;
    }
    return SIMSENSE_OK;
}

int simsense_census(const simsense_params *params, const uint8_t *img, int32_t pitch, uint64_t *out,
                    void *stream)
{
    int rc = validate(params);
    if (rc != SIMSENSE_OK) return rc;
    if (!img || !out) return SIMSENSE_ERR_NULL_POINTER;
    if (pitch < params->width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (launch_census(img, pitch, params->width, params->height, params->census_w, params->census_h,
                      params->census_mode, out, true, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return SIMSENSE_ERR_DEVICE;
    }
    return SIMSENSE_OK;
}

int simsense_set_tuning(simsense_handle *h, const simsense_batch_tuning *t)
{
    if (!h || !t) return SIMSENSE_ERR_NULL_POINTER;
    if (t->struct_size != sizeof(simsense_batch_tuning)) return SIMSENSE_ERR_ABI;
    if (t->horizontal_lanes != 0 && !horizontal_lanes_valid(h->Dpad, t->horizontal_lanes))
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 8) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (h->last_stream && hipStreamSynchronize(h->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    return apply_tuning(h, *t);
}

int simsense_get_tuning(const simsense_handle *h, simsense_batch_tuning *t)
{
    if (!h || !t) return SIMSENSE_ERR_NULL_POINTER;
    *t = h->tuning;
    return SIMSENSE_OK;
}

int simsense_autotune(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch, int32_t reps,
                      simsense_batch_tuning *best, float *ms, int32_t max_candidates, int32_t *count, void *stream)
{
    if (!h || !left || !right || !best) return SIMSENSE_ERR_NULL_POINTER;
    if (reps < 1 || pitch < h->p.width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t st = (hipStream_t)stream;
    static const int lanes[3] = {16, 32, 64};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SIMSENSE_ERR_DEVICE;
    }
    const bool was_profiling = h->profiling;
    h->profiling = false;
    float best_ms = 1e30f;
    simsense_batch_tuning best_t = h->tuning;
    int c = 0, rc = SIMSENSE_OK;
    for (int li = 0; li < 3 && rc == SIMSENSE_OK; ++li) {
        if (!horizontal_lanes_valid(h->Dpad, lanes[li])) continue;
        for (int bpc = 0; bpc <= 4 && rc == SIMSENSE_OK; ++bpc) {
            simsense_batch_tuning t{};
            t.struct_size = sizeof(t);
            t.horizontal_lanes = lanes[li];
            t.blocks_per_cu = bpc;
            rc = simsense_set_tuning(h, &t);
            if (rc == SIMSENSE_OK) rc = enqueue_match(h, left, right, pitch, st);  // warm-up
            if (rc != SIMSENSE_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = SIMSENSE_ERR_DEVICE; break; }
            for (int r = 0; r < reps && rc == SIMSENSE_OK; ++r) rc = enqueue_match(h, left, right, pitch, st);
            if (rc != SIMSENSE_OK) break;
            float m = 0.0f;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&m, e0, e1) != hipSuccess) {
                rc = SIMSENSE_ERR_DEVICE;
                break;
            }
            m /= (float)reps;
            if (ms && c < max_candidates) ms[c] = m;
            ++c;
            if (m < best_ms) {
                best_ms = m;
                best_t = t;
            }
        }
    }
    h->profiling = was_profiling;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (count) *count = c;
    if (rc != SIMSENSE_OK) return rc;
    *best = best_t;
    return simsense_set_tuning(h, &best_t);
}

}  // extern "C"
