// Batches of stereo pairs of uneven sizes and disparity ranges in one hipGraph
// launch.  Per pair slot the batch owns the same scratch a handle owns; the
// argument blocks of every slot live in device tables, and each pass of the path
// is one launch over all slots:
//   counter reset -> census (every image) -> aggregation (a persistent kernel per
//   padded-disparity group, pulling line blocks from a longest-first queue) ->
//   selection (per group) -> median/depth.
// The slots are split into phases of consecutive slots; each phase runs the pass
// sequence on its own, on one of two streams in turn, and a phase's aggregation
// starts when the previous phase's has finished, so that it runs while that phase
// selects (bound by HBM) and the vector ALUs and HBM are busy at once.  The pass
// sequence is captured once into a graph; a compute call only refreshes the
// image/output pointer tables (one host-to-device copy) and launches the graph.
#include <algorithm>
#include <map>
#include <new>
#include <string.h>
#include <tuple>
#include <vector>

#include "internal.h"
#include "net_internal.h"
#include "trace.h"

using namespace ss;

namespace {

struct Slot {
    simsense_params p;
    int bits, Dpad, ndirs, hl;
    bool wide;
    size_t off_census_l, off_census_r, off_paths[8], off_dint, off_s1, off_s2, off_dright, off_dsub, off_masked,
        off_flags;
};

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// phases the plain form of a batch of n slots is split into (consecutive slots, as
// equal in number as can be; one phase for a single slot).  Measured on 256 sensor
// pairs in 64-pair batches: 2271 pairs/s with 1 phase, 2392 with 4, 2453 with 8; at
// most 7 padded-disparity groups per phase keep 8 phases within the 64 work-queue
// counters.  The learned form, whose fused-net blocks need a whole unit, runs as
// one phase (4 phases: 4% fewer pairs/s).
constexpr int kBatchPhases = 8;
int batch_phases(int n) { return std::min(n, kBatchPhases); }

}  // namespace

struct simsense_batch {
    int n;
    std::vector<Slot> slots;
    simsense_batch_tuning tuning;
    int num_cus;
    uint8_t *scratch;  // per-slot scratch
    size_t scratch_bytes;
    // device tables
    CensusJob *d_cjobs;
    AggregateArgs *d_agg;
    SelectArgs *d_sel;
    PostArgs *d_post;
    uint32_t *d_items;  // all item lists
    unsigned *d_counters;
    // pinned staging of the pointer-dependent tables (double-buffered)
    CensusJob *h_cjobs[2];
    PostArgs *h_post[2];
    hipEvent_t staged[2];
    unsigned *h_uncertain;  // pinned: the learned form's per-pair counts, read back for the fallback
    int stage_idx;
    // launch plan
    struct AggGroup { int dpad, hl; bool wide; size_t item_off; int nitems; int counter; };
    struct SelGroup { int dpad, ndirs; bool small; size_t item_off; int nitems; };
    // a phase: slots s0 .. s1-1, their item lists and groups (ranges of the vectors)
    struct Phase {
        int s0, s1;
        size_t census_item_off, post_item_off;
        int census_nitems, post_nitems;
        int agg0, nagg, sel0, nsel;
    };
    std::vector<AggGroup> agg_groups;
    std::vector<SelGroup> sel_groups;
    std::vector<Phase> phases;   // the plain form's
    std::vector<Phase> lphases;  // the learned form's (one phase: its net blocks do not share a unit)
    int max_cw, max_ch, max_w;
    bool census_wide;
    // graph (the second stream and the events join the capture of the first)
    hipStream_t capture_stream, side_stream;
    hipEvent_t ev_fork, ev_join, ev_agg[kBatchPhases];
    hipGraphExec_t exec;
    bool captured;
    hipStream_t last_stream;
    // learned form: its own graph, valid for one (net, tau, count buffer)
    hipGraphExec_t lexec;
    bool lcaptured;
    simsense_net *lnet;
    float ltau;
    unsigned *luncertain;
};

namespace {

#define B_TRY(expr) \
    do { if ((expr) != hipSuccess) { (void)hipGetLastError(); return SIMSENSE_ERR_DEVICE; } } while (0)

int validate_params(const simsense_params *p)
{
    // the single-pair validator, through the public entry point
    const int64_t r = simsense_scratch_bytes(p);
    return r < 0 ? (int)r : SIMSENSE_OK;
}

// builds the item lists and the argument tables for the current tuning
int build_plan(simsense_batch *b)
{
    const int n = b->n;
    std::vector<uint32_t> items;
    b->agg_groups.clear();
    b->sel_groups.clear();
    b->phases.clear();
    b->max_cw = b->max_ch = 1;
    b->max_w = 1;
    for (int s = 0; s < n; ++s) {
        const Slot &sl = b->slots[s];
        b->max_cw = std::max(b->max_cw, sl.p.census_w);
        b->max_ch = std::max(b->max_ch, sl.p.census_h);
        b->max_w = std::max(b->max_w, sl.p.width);
    }
    std::vector<AggregateArgs> agg(n);
    std::vector<SelectArgs> sel(n);
    int counter = 0;
    b->lphases.clear();
    auto add_phase = [&](int s0, int s1, std::vector<simsense_batch::Phase> &dest) {
        simsense_batch::Phase P{};
        P.s0 = s0;
        P.s1 = s1;
        // census: every image of the phase
        P.census_item_off = items.size();
        for (int s = P.s0; s < P.s1; ++s) {
            const Slot &sl = b->slots[s];
            const int t = census_tiles(sl.p.width, sl.p.height);
            for (int img = 0; img < 2; ++img)
                for (int i = 0; i < t; ++i) items.push_back(((uint32_t)(2 * s + img) << 20) | (uint32_t)i);
        }
        P.census_nitems = (int)(items.size() - P.census_item_off);
        // aggregation: group slots by (Dpad, wide); items largest estimated work first
        std::map<std::pair<int, bool>, std::vector<std::pair<int, uint32_t>>> groups;
        for (int s = P.s0; s < P.s1; ++s) {
            Slot &sl = b->slots[s];
            sl.hl = horizontal_lanes_valid(sl.Dpad, b->tuning.horizontal_lanes) ? b->tuning.horizontal_lanes
                                                                                  : horizontal_lanes(sl.Dpad);
            AggregateArgs &a = agg[s];
            const int scale = a.max_item_work;  // set by an earlier plan, if any
            a = AggregateArgs{};
            a.max_item_work = scale;
            a.census_l = b->scratch + sl.off_census_l;
            a.census_r = b->scratch + sl.off_census_r;
            a.W = sl.p.width; a.H = sl.p.height; a.D = sl.p.max_disp; a.Dpad = sl.Dpad; a.bits = sl.bits;
            a.p1 = sl.p.p1; a.p2 = sl.p.p2; a.ndirs = sl.ndirs;
            a.block_begin[0] = 0;
            auto &lst = groups[{sl.Dpad, sl.wide}];
            for (int r = 0; r < sl.ndirs; ++r) {
                a.dx[r] = kPathDx[r];
                a.dy[r] = kPathDy[r];
                a.out[r] = b->scratch + sl.off_paths[r];
                const int nb = aggregate_blocks(kPathDx[r], kPathDy[r], a.W, a.H, sl.hl);
                for (int k = 0; k < nb; ++k) {
                    const int work = aggregate_block_work(kPathDx[r], kPathDy[r], k, a.W, a.H, sl.hl, sl.Dpad);
                    lst.push_back({work, ((uint32_t)s << 20) | (uint32_t)(a.block_begin[r] + k)});
                }
                a.block_begin[r + 1] = a.block_begin[r] + nb;
            }
        }
        P.agg0 = (int)b->agg_groups.size();
        for (auto &kv : groups) {
            auto &lst = kv.second;
            std::stable_sort(lst.begin(), lst.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
            // the group's blocks run in one launch: its largest block sets the scale
            // of every slot's issue priorities
            const int gmax = lst.empty() ? 0 : lst.front().first;
            // (the plain form's phases set the scale; slots of equal size get the
            // same one in every plan)
            if (&dest == &b->phases)
                for (auto &e : lst) agg[e.second >> 20].max_item_work = gmax;
            simsense_batch::AggGroup gr{};
            gr.dpad = kv.first.first;
            gr.wide = kv.first.second;
            gr.hl = horizontal_lanes_valid(gr.dpad, b->tuning.horizontal_lanes) ? b->tuning.horizontal_lanes
                                                                                : horizontal_lanes(gr.dpad);
            gr.item_off = items.size();
            gr.nitems = (int)lst.size();
            gr.counter = counter++;
            for (auto &e : lst) items.push_back(e.second);
            b->agg_groups.push_back(gr);
        }
        P.nagg = (int)b->agg_groups.size() - P.agg0;
        // selection: group by (Dpad, ndirs, small)
        std::map<std::tuple<int, int, bool>, std::vector<uint32_t>> sgroups;
        for (int s = P.s0; s < P.s1; ++s) {
            const Slot &sl = b->slots[s];
            SelectArgs &a = sel[s];
            a = SelectArgs{};
            for (int r = 0; r < sl.ndirs; ++r) a.paths[r] = b->scratch + sl.off_paths[r];
            a.ndirs = sl.ndirs;
            a.W = sl.p.width; a.H = sl.p.height; a.D = sl.p.max_disp; a.Dpad = sl.Dpad;
            a.uniqueness_pct = sl.p.uniqueness_pct; a.lr_max_diff = sl.p.lr_max_diff; a.subpixel = sl.p.subpixel;
            a.small_values = sl.bits + sl.p.p2 <= 127;
            a.disp_int = b->scratch + sl.off_dint;
            a.cost_best = (uint16_t *)(b->scratch + sl.off_s1);
            a.cost_second = (uint16_t *)(b->scratch + sl.off_s2);
            a.disp_right = b->scratch + sl.off_dright;
            a.disp_sub = (float *)(b->scratch + sl.off_dsub);
            a.masked = (float *)(b->scratch + sl.off_masked);
            a.flags = b->scratch + sl.off_flags;
            auto &lst = sgroups[{sl.Dpad, sl.ndirs, a.small_values != 0}];
            for (int y = 0; y < sl.p.height; ++y) lst.push_back(((uint32_t)s << 20) | (uint32_t)y);
        }
        P.sel0 = (int)b->sel_groups.size();
        for (auto &kv : sgroups) {
            simsense_batch::SelGroup gr{};
            gr.dpad = std::get<0>(kv.first);
            gr.ndirs = std::get<1>(kv.first);
            gr.small = std::get<2>(kv.first);
            gr.item_off = items.size();
            gr.nitems = (int)kv.second.size();
            items.insert(items.end(), kv.second.begin(), kv.second.end());
            b->sel_groups.push_back(gr);
        }
        P.nsel = (int)b->sel_groups.size() - P.sel0;
        // post
        P.post_item_off = items.size();
        for (int s = P.s0; s < P.s1; ++s) {
            const Slot &sl = b->slots[s];
            const int t = ((sl.p.width + 63) / 64) * ((sl.p.height + 3) / 4);
            for (int i = 0; i < t; ++i) items.push_back(((uint32_t)s << 20) | (uint32_t)i);
        }
        P.post_nitems = (int)(items.size() - P.post_item_off);
        dest.push_back(P);
    };
    const int nph = batch_phases(n);
    for (int ph = 0; ph < nph; ++ph)
        add_phase((int)((int64_t)n * ph / nph), (int)((int64_t)n * (ph + 1) / nph), b->phases);
    add_phase(0, n, b->lphases);
    if (counter > 64) return SIMSENSE_ERR_UNSUPPORTED;  // the work-queue counters one batch holds
    b->census_wide = b->slots[0].wide;

    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    B_TRY(hipMalloc(&b->d_items, std::max<size_t>(items.size(), 1) * sizeof(uint32_t)));
    B_TRY(hipMemcpy(b->d_items, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    B_TRY(hipMemcpy(b->d_agg, agg.data(), n * sizeof(AggregateArgs), hipMemcpyHostToDevice));
    B_TRY(hipMemcpy(b->d_sel, sel.data(), n * sizeof(SelectArgs), hipMemcpyHostToDevice));
    return SIMSENSE_OK;
}

__global__ void zero_words(unsigned *c, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0u;
}

// census of one phase's images (the launch also clears its work-queue counters)
int enqueue_census_phase(simsense_batch *b, const simsense_batch::Phase &P, hipStream_t s)
{
    CensusBatch cb{};
    cb.zero = P.nagg > 0 ? b->d_counters + b->agg_groups[P.agg0].counter : nullptr;
    cb.nzero = P.nagg;
    cb.jobs = b->d_cjobs;
    cb.items = b->d_items + P.census_item_off;
    cb.nitems = P.census_nitems;
    cb.max_cw = b->max_cw;
    cb.max_ch = b->max_ch;
    B_TRY(launch_census_batch(cb, b->census_wide, s));
    return SIMSENSE_OK;
}

int enqueue_aggregate_phase(simsense_batch *b, const simsense_batch::Phase &P, hipStream_t s)
{
    for (int i = P.agg0; i < P.agg0 + P.nagg; ++i) {
        const auto &g = b->agg_groups[i];
        AggregateQueue q{};
        q.slots = b->d_agg;
        q.items = b->d_items + g.item_off;
        q.nitems = g.nitems;
        q.counter = b->d_counters + g.counter;
        const int grid = std::min(g.nitems, std::max(1, b->tuning.blocks_per_cu) * b->num_cus);
        B_TRY(launch_aggregate_queue(q, g.dpad, g.wide, g.hl, grid, s));
    }
    return SIMSENSE_OK;
}

int enqueue_select_phase(simsense_batch *b, const simsense_batch::Phase &P, hipStream_t s, bool need_right)
{
    for (int i = P.sel0; i < P.sel0 + P.nsel; ++i) {
        const auto &g = b->sel_groups[i];
        SelectBatch sb{};
        sb.slots = b->d_sel;
        sb.items = b->d_items + g.item_off;
        sb.nitems = g.nitems;
        sb.max_width = b->max_w;
        sb.no_right = !need_right;
        B_TRY(launch_select_batch(sb, g.dpad, g.ndirs, g.small, s));
    }
    return SIMSENSE_OK;
}

int enqueue_post_phase(simsense_batch *b, const simsense_batch::Phase &P, hipStream_t s)
{
    PostBatch pb{};
    pb.slots = b->d_post;
    pb.items = b->d_items + P.post_item_off;
    pb.nitems = P.post_nitems;
    B_TRY(launch_post_batch(pb, s));
    return SIMSENSE_OK;
}

// the fused net over one phase's slots: one launch for a run of slots whose
// buffers lie at equal distances (equal-sized slots do), else per slot
int enqueue_net_phase(simsense_batch *b, const simsense_batch::Phase &P, simsense_net *net, float tau, unsigned *uncertain,
                      hipStream_t s)
{
    const int c0 = P.s0, cn = P.s1 - P.s0;
    if (cn <= 0) return SIMSENSE_OK;
    const Slot &s0 = b->slots[c0];
    const int W = s0.p.width, H = s0.p.height;
    auto gap = [&](size_t Slot::*off, int k) {
        return (int64_t)(b->slots[c0 + k].*off) - (int64_t)(b->slots[c0 + k - 1].*off);
    };
    bool uniform = true;
    for (int k = 2; k < cn && uniform; ++k)
        uniform = gap(&Slot::off_dsub, k) == gap(&Slot::off_dsub, 1) &&
                  gap(&Slot::off_masked, k) == gap(&Slot::off_masked, 1) &&
                  gap(&Slot::off_flags, k) == gap(&Slot::off_flags, 1);
    // the net reads S1, S2 and d* of image i at one byte distance per image
    for (int k = 1; k < cn && uniform; ++k)
        uniform = gap(&Slot::off_s1, k) == gap(&Slot::off_s1, 1) && gap(&Slot::off_s2, k) == gap(&Slot::off_s1, 1) &&
                  gap(&Slot::off_dint, k) == gap(&Slot::off_s1, 1);
    const int per = uniform ? cn : 1;
    for (int k = 0; k < cn; k += per) {
        const Slot &sl = b->slots[c0 + k];
        // the features are built inside the net from the selection outputs
        net::InferArgs ia = net::infer_args(net, nullptr, per, H, W);
        ia.ir_jobs = b->d_cjobs + 2 * (c0 + k);  // the left images, as refreshed per call
        ia.s1 = (const uint16_t *)(b->scratch + sl.off_s1);
        ia.s2 = (const uint16_t *)(b->scratch + sl.off_s2);
        ia.dint = b->scratch + sl.off_dint;
        ia.sel_stride = per > 1 ? gap(&Slot::off_s1, 1) : 0;
        ia.max_disp = sl.p.max_disp;
        ia.smax = (float)(sl.ndirs * (sl.bits + sl.p.p2));
        ia.d2_sub = (const float *)(b->scratch + sl.off_dsub);
        ia.masked = (float *)(b->scratch + sl.off_masked);
        ia.flags = b->scratch + sl.off_flags;
        if (per > 1) {
            ia.d2_stride = gap(&Slot::off_dsub, 1) / 4;
            ia.masked_stride = gap(&Slot::off_masked, 1) / 4;
            ia.flags_stride = gap(&Slot::off_flags, 1);
        }
        ia.uncertain = uncertain + c0 + k;
        ia.tau = tau;
        B_TRY(net::launch_infer(ia, s));
    }
    return SIMSENSE_OK;
}

// The pass sequence of every phase: phase p on stream (p even: s, odd: the side
// stream), its aggregation after phase p - 1's, and the side stream joined back
// into s at the end.  With a net, the learned form: matching without the right
// disparities, then the fused net (features built from the selection outputs, the
// per-slot uncertainty counts), then median and depth.
int enqueue_phases(simsense_batch *b, hipStream_t s, simsense_net *net, float tau, unsigned *uncertain)
{
    const std::vector<simsense_batch::Phase> &phases = net ? b->lphases : b->phases;
    const int nph = (int)phases.size();
    if (net) {
        hipLaunchKernelGGL(zero_words, dim3(1), dim3(256), 0, s, uncertain, b->n);
        B_TRY(hipGetLastError());
    }
    if (nph > 1) {
        B_TRY(hipEventRecord(b->ev_fork, s));
        B_TRY(hipStreamWaitEvent(b->side_stream, b->ev_fork, 0));
    }
    int rc = SIMSENSE_OK;
    for (int ph = 0; ph < nph && rc == SIMSENSE_OK; ++ph) {
        hipStream_t st = ph % 2 == 0 ? s : b->side_stream;
        rc = enqueue_census_phase(b, phases[ph], st);
        if (rc == SIMSENSE_OK && ph > 0) B_TRY(hipStreamWaitEvent(st, b->ev_agg[ph - 1], 0));
        if (rc == SIMSENSE_OK) rc = enqueue_aggregate_phase(b, phases[ph], st);
        if (rc == SIMSENSE_OK && ph + 1 < nph) B_TRY(hipEventRecord(b->ev_agg[ph], st));
        if (rc == SIMSENSE_OK) rc = enqueue_select_phase(b, phases[ph], st, /*need_right=*/!net);
        if (rc == SIMSENSE_OK && net) rc = enqueue_net_phase(b, phases[ph], net, tau, uncertain, st);
        if (rc == SIMSENSE_OK) rc = enqueue_post_phase(b, phases[ph], st);
    }
    if (nph > 1) {
        B_TRY(hipEventRecord(b->ev_join, b->side_stream));
        B_TRY(hipStreamWaitEvent(s, b->ev_join, 0));
    }
    return rc;
}

int capture_graph(simsense_batch *b, hipGraphExec_t *exec, simsense_net *net, float tau, unsigned *uncertain)
{
    hipGraph_t graph;
    B_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_phases(b, b->capture_stream, net, tau, uncertain);
    hipError_t e = hipStreamEndCapture(b->capture_stream, &graph);
    if (rc != SIMSENSE_OK) return rc;
    B_TRY(e);
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    B_TRY(e);
    return SIMSENSE_OK;
}

int capture(simsense_batch *b)
{
    if (b->captured) {
        (void)hipGraphExecDestroy(b->exec);
        b->captured = false;
    }
    const int rc = capture_graph(b, &b->exec, nullptr, 0.0f, nullptr);
    if (rc == SIMSENSE_OK) b->captured = true;
    return rc;
}

void drop_graphs(simsense_batch *b)
{
    if (b->captured) (void)hipGraphExecDestroy(b->exec);
    if (b->lcaptured) (void)hipGraphExecDestroy(b->lexec);
    b->captured = b->lcaptured = false;
}

// refreshes the per-call pointer tables from `pairs` (through a staging buffer
// the device no longer reads) on stream st
int stage_tables(simsense_batch *b, const simsense_pair *pairs, hipStream_t st)
{
    const int n = b->n;
    const int k = b->stage_idx;
    b->stage_idx ^= 1;
    B_TRY(hipEventSynchronize(b->staged[k]));
    for (int s = 0; s < n; ++s) {
        const Slot &sl = b->slots[s];
        const simsense_pair &pr = pairs[s];
        for (int img = 0; img < 2; ++img) {
            CensusJob &j = b->h_cjobs[k][2 * s + img];
            j.img = img == 0 ? pr.left : pr.right;
            j.pitch = pr.pitch;
            j.W = sl.p.width;
            j.H = sl.p.height;
            j.cw = sl.p.census_w;
            j.ch = sl.p.census_h;
            j.mode = sl.p.census_mode;
            j.out = b->scratch + (img == 0 ? sl.off_census_l : sl.off_census_r);
        }
        PostArgs &pa = b->h_post[k][s];
        pa = PostArgs{};
        pa.masked = (const float *)(b->scratch + sl.off_masked);
        pa.flags_in = b->scratch + sl.off_flags;
        pa.W = sl.p.width;
        pa.H = sl.p.height;
        pa.median = sl.p.median;
        pa.fb = sl.p.focal_px * sl.p.baseline_m;
        pa.disp = pr.disp;
        pa.depth = pr.depth;
        pa.flags = pr.flags;
    }
    B_TRY(hipMemcpyAsync(b->d_cjobs, b->h_cjobs[k], 2 * n * sizeof(CensusJob), hipMemcpyHostToDevice, st));
    B_TRY(hipMemcpyAsync(b->d_post, b->h_post[k], n * sizeof(PostArgs), hipMemcpyHostToDevice, st));
    B_TRY(hipEventRecord(b->staged[k], st));
    return SIMSENSE_OK;
}

int check_pairs(const simsense_batch *b, const simsense_pair *pairs)
{
    for (int s = 0; s < b->n; ++s) {
        const simsense_pair &pr = pairs[s];
        if (!pr.left || !pr.right || !pr.depth) return SIMSENSE_ERR_NULL_POINTER;
        if (pr.pitch < b->slots[s].p.width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    }
    return SIMSENSE_OK;
}

void free_batch(simsense_batch *b)
{
    drop_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    for (int i = 0; i < kBatchPhases; ++i)
        if (b->ev_agg[i]) (void)hipEventDestroy(b->ev_agg[i]);
    for (int i = 0; i < 2; ++i) {
        if (b->staged[i]) (void)hipEventDestroy(b->staged[i]);
        if (b->h_cjobs[i]) (void)hipHostFree(b->h_cjobs[i]);
        if (b->h_post[i]) (void)hipHostFree(b->h_post[i]);
    }
    if (b->h_uncertain) (void)hipHostFree(b->h_uncertain);
    (void)hipFree(b->scratch);
    (void)hipFree(b->d_cjobs);
    (void)hipFree(b->d_agg);
    (void)hipFree(b->d_sel);
    (void)hipFree(b->d_post);
    (void)hipFree(b->d_items);
    (void)hipFree(b->d_counters);
    delete b;
}

}  // namespace

extern "C" {

int simsense_batch_create(const simsense_params *params, int32_t n, simsense_batch **out)
{
    if (!params || !out) return SIMSENSE_ERR_NULL_POINTER;
    if (n < 1 || n > 2048) return SIMSENSE_ERR_INVALID_ARGUMENT;  // census jobs 2n fit 12 bits
    bool wide0 = false;
    for (int s = 0; s < n; ++s) {
        const int rc = validate_params(&params[s]);
        if (rc != SIMSENSE_OK) return rc;
        if (params[s].lr_mode != 0) return SIMSENSE_ERR_UNSUPPORTED;  // batches read dR off the left volume
        if (params[s].block_w * params[s].block_h > 1) return SIMSENSE_ERR_UNSUPPORTED;  // no block matching
        const bool wide = census_bits(params[s].census_w, params[s].census_h, params[s].census_mode) > 32;
        if (s == 0) wide0 = wide;
        else if (wide != wide0) return SIMSENSE_ERR_UNSUPPORTED;  // one census word width per batch
    }
    simsense_batch *b = new (std::nothrow) simsense_batch();
    if (!b) return SIMSENSE_ERR_OUT_OF_MEMORY;
    b->n = n;
    b->slots.resize(n);
    b->tuning.struct_size = sizeof(simsense_batch_tuning);
    b->tuning.horizontal_lanes = 0;
    b->tuning.blocks_per_cu = 2;
    if (hipDeviceGetAttribute(&b->num_cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess) b->num_cus = 256;
    size_t total = 0;
    for (int s = 0; s < n; ++s) {
        Slot &sl = b->slots[s];
        sl.p = params[s];
        sl.bits = census_bits(sl.p.census_w, sl.p.census_h, sl.p.census_mode);
        sl.wide = sl.bits > 32;
        sl.Dpad = padded_disp(sl.p.max_disp);
        sl.ndirs = sl.p.num_paths;
        const size_t npx = (size_t)sl.p.width * sl.p.height;
        auto take = [&](size_t bytes) { size_t o = total; total += a256(bytes); return o; };
        sl.off_census_l = take(npx * (sl.wide ? 8 : 4));
        sl.off_census_r = take(npx * (sl.wide ? 8 : 4));
        for (int r = 0; r < sl.ndirs; ++r) sl.off_paths[r] = take((npx + 1) * sl.Dpad);
        sl.off_dint = take(npx);
        sl.off_s1 = take(npx * 2);
        sl.off_s2 = take(npx * 2);
        sl.off_dright = take(npx);
        sl.off_dsub = take(npx * 4);
        sl.off_masked = take(npx * 4);
        sl.off_flags = take(npx);
    }
    b->scratch_bytes = total;
    int rc = SIMSENSE_OK;
    if (hipMalloc(&b->scratch, total) != hipSuccess || hipMalloc(&b->d_cjobs, 2 * n * sizeof(CensusJob)) != hipSuccess ||
        hipMalloc(&b->d_agg, n * sizeof(AggregateArgs)) != hipSuccess ||
        hipMalloc(&b->d_sel, n * sizeof(SelectArgs)) != hipSuccess ||
        hipMalloc(&b->d_post, n * sizeof(PostArgs)) != hipSuccess ||
        hipMalloc(&b->d_counters, 64 * sizeof(unsigned)) != hipSuccess)
        rc = SIMSENSE_ERR_OUT_OF_MEMORY;
    for (int i = 0; i < 2 && rc == SIMSENSE_OK; ++i) {
        if (hipHostMalloc((void **)&b->h_cjobs[i], 2 * n * sizeof(CensusJob), 0) != hipSuccess ||
            hipHostMalloc((void **)&b->h_post[i], n * sizeof(PostArgs), 0) != hipSuccess ||
            hipEventCreateWithFlags(&b->staged[i], hipEventDisableTiming) != hipSuccess)
            rc = SIMSENSE_ERR_OUT_OF_MEMORY;
    }
    if (rc == SIMSENSE_OK && hipHostMalloc((void **)&b->h_uncertain, n * sizeof(unsigned), 0) != hipSuccess)
        rc = SIMSENSE_ERR_OUT_OF_MEMORY;
    if (rc == SIMSENSE_OK && (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess ||
                              hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking) != hipSuccess))
        rc = SIMSENSE_ERR_DEVICE;
    if (rc == SIMSENSE_OK && (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
                              hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess))
        rc = SIMSENSE_ERR_DEVICE;
    for (int i = 0; i < kBatchPhases && rc == SIMSENSE_OK; ++i)
        if (hipEventCreateWithFlags(&b->ev_agg[i], hipEventDisableTiming) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (rc == SIMSENSE_OK) rc = build_plan(b);
    if (rc != SIMSENSE_OK) {
        (void)hipGetLastError();
        free_batch(b);
        return rc;
    }
    *out = b;
    return SIMSENSE_OK;
}

int simsense_batch_destroy(simsense_batch *b)
{
    if (!b) return SIMSENSE_OK;
    int rc = SIMSENSE_OK;
    if (hipStreamSynchronize(b->last_stream) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    free_batch(b);
    return rc;
}

int64_t simsense_batch_scratch_bytes(const simsense_batch *b) { return b ? (int64_t)b->scratch_bytes : -2; }

int simsense_batch_set_tuning(simsense_batch *b, const simsense_batch_tuning *t)
{
    if (!b || !t) return SIMSENSE_ERR_NULL_POINTER;
    if (t->struct_size != sizeof(simsense_batch_tuning)) return SIMSENSE_ERR_ABI;
    if (t->horizontal_lanes != 0 && t->horizontal_lanes != 16 && t->horizontal_lanes != 32 &&
        t->horizontal_lanes != 64)
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (t->blocks_per_cu < 1 || t->blocks_per_cu > 8) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(b->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    b->tuning = *t;
    drop_graphs(b);
    return build_plan(b);
}

int simsense_batch_get_tuning(const simsense_batch *b, simsense_batch_tuning *t)
{
    if (!b || !t) return SIMSENSE_ERR_NULL_POINTER;
    *t = b->tuning;
    return SIMSENSE_OK;
}

int simsense_batch_compute(simsense_batch *b, const simsense_pair *pairs, void *stream)
{
    if (!b || !pairs) return SIMSENSE_ERR_NULL_POINTER;
    int rc = check_pairs(b, pairs);
    if (rc != SIMSENSE_OK) return rc;
    TraceRange range("simsense_batch_compute");
    hipStream_t st = (hipStream_t)stream;
    if (!b->captured) {
        rc = capture(b);
        if (rc != SIMSENSE_OK) return rc;
    }
    rc = stage_tables(b, pairs, st);
    if (rc != SIMSENSE_OK) return rc;
    B_TRY(hipGraphLaunch(b->exec, st));
    b->last_stream = st;
    return SIMSENSE_OK;
}

int simsense_batch_learned_compute(simsense_batch *b, simsense_net *net, const simsense_pair *pairs, float tau,
                                   unsigned *uncertain, void *stream)
{
    if (!b || !net || !pairs || !uncertain) return SIMSENSE_ERR_NULL_POINTER;
    if (!(tau >= 0.0f)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    for (int s = 1; s < b->n; ++s)
        if (b->slots[s].p.width != b->slots[0].p.width || b->slots[s].p.height != b->slots[0].p.height)
            return SIMSENSE_ERR_UNSUPPORTED;  // the net runs on equal-sized images
    if ((int64_t)b->slots[0].p.width * b->slots[0].p.height > net->max_pixels) return SIMSENSE_ERR_INVALID_ARGUMENT;
    int rc = check_pairs(b, pairs);
    if (rc != SIMSENSE_OK) return rc;
    TraceRange range("simsense_batch_learned_compute");
    hipStream_t st = (hipStream_t)stream;
    if (b->lcaptured && (b->lnet != net || b->ltau != tau || b->luncertain != uncertain)) {
        (void)hipGraphExecDestroy(b->lexec);
        b->lcaptured = false;
    }
    if (!b->lcaptured) {
        rc = capture_graph(b, &b->lexec, net, tau, uncertain);
        if (rc != SIMSENSE_OK) return rc;
        b->lcaptured = true;
        b->lnet = net;
        b->ltau = tau;
        b->luncertain = uncertain;
    }
    rc = stage_tables(b, pairs, st);
    if (rc != SIMSENSE_OK) return rc;
    B_TRY(hipGraphLaunch(b->lexec, st));
    b->last_stream = st;
    net->last_stream = st;
    return SIMSENSE_OK;
}

int simsense_batch_learned_fallback(simsense_batch *b, simsense_net *net, simsense_handle *plain,
                                    const simsense_pair *pairs, float tau, unsigned *uncertain, int32_t mode,
                                    float max_uncertain_frac, int32_t *fell_back, void *stream)
{
    if (!b || !net || !pairs || !uncertain) return SIMSENSE_ERR_NULL_POINTER;
    if (mode != SIMSENSE_FALLBACK_THRESHOLD && mode != SIMSENSE_FALLBACK_NEVER && mode != SIMSENSE_FALLBACK_ALWAYS)
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (mode == SIMSENSE_FALLBACK_THRESHOLD && !(max_uncertain_frac >= 0.0f && max_uncertain_frac <= 1.0f))
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (mode != SIMSENSE_FALLBACK_NEVER) {
        if (!plain) return SIMSENSE_ERR_NULL_POINTER;
        // the plain run writes the pair's own outputs, so it must describe the same image
        for (const Slot &sl : b->slots)
            if (plain->p.width != sl.p.width || plain->p.height != sl.p.height || plain->p.max_disp != sl.p.max_disp)
                return SIMSENSE_ERR_INVALID_ARGUMENT;
    }
    TraceRange range("simsense_batch_learned_fallback");
    int rc = simsense_batch_learned_compute(b, net, pairs, tau, uncertain, stream);
    if (rc != SIMSENSE_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int n = b->n;
    if (mode == SIMSENSE_FALLBACK_THRESHOLD) {
        // the decision needs the counts on the host: one copy and one wait
        B_TRY(hipMemcpyAsync(b->h_uncertain, uncertain, n * sizeof(unsigned), hipMemcpyDeviceToHost, st));
        B_TRY(hipStreamSynchronize(st));
    }
    const double limit = (double)max_uncertain_frac * (double)b->slots[0].p.width * (double)b->slots[0].p.height;
    for (int s = 0; s < n; ++s) {
        const bool fb = mode == SIMSENSE_FALLBACK_ALWAYS ||
                        (mode == SIMSENSE_FALLBACK_THRESHOLD && (double)b->h_uncertain[s] > limit);
        if (fell_back) fell_back[s] = fb ? 1 : 0;
        if (!fb) continue;
        const simsense_pair &pr = pairs[s];
        rc = simsense_compute(plain, pr.left, pr.right, pr.pitch, pr.depth, pr.disp, pr.flags, stream);
        if (rc != SIMSENSE_OK) return rc;
    }
    return SIMSENSE_OK;
}

int simsense_batch_autotune(simsense_batch *b, const simsense_pair *pairs, int32_t reps,
                            simsense_batch_tuning *best, float *ms, int32_t max_candidates, int32_t *count,
                            void *stream)
{
    if (!b || !pairs || !best) return SIMSENSE_ERR_NULL_POINTER;
    if (reps < 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t st = (hipStream_t)stream;
    static const int lanes[3] = {16, 32, 64};
    static const int bpc[4] = {1, 2, 3, 4};
    hipEvent_t e0, e1;
    B_TRY(hipEventCreate(&e0));
    B_TRY(hipEventCreate(&e1));
    float best_ms = 1e30f;
    simsense_batch_tuning best_t = b->tuning;
    int c = 0;
    int rc = SIMSENSE_OK;
    for (int li = 0; li < 3 && rc == SIMSENSE_OK; ++li) {
        bool usable = false;  // the lane count must fit at least one slot's disparity range
        for (const Slot &sl : b->slots) usable |= horizontal_lanes_valid(sl.Dpad, lanes[li]);
        if (!usable) continue;
        for (int bi = 0; bi < 4 && rc == SIMSENSE_OK; ++bi) {
            simsense_batch_tuning t{};
            t.struct_size = sizeof(t);
            t.horizontal_lanes = lanes[li];
            t.blocks_per_cu = bpc[bi];
            rc = simsense_batch_set_tuning(b, &t);
            if (rc != SIMSENSE_OK) break;
            rc = simsense_batch_compute(b, pairs, st);  // capture + warm-up
            if (rc != SIMSENSE_OK) break;
            if (hipEventRecord(e0, st) != hipSuccess) { rc = SIMSENSE_ERR_DEVICE; break; }
            for (int r = 0; r < reps && rc == SIMSENSE_OK; ++r) rc = simsense_batch_compute(b, pairs, st);
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
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (count) *count = c;
    if (rc != SIMSENSE_OK) return rc;
    *best = best_t;
    return simsense_batch_set_tuning(b, &best_t);
}

}  // extern "C"
