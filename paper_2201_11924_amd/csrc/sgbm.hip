// Semi-global block matching (Sec. VI-D: the matching cost of two pixels is the
// Hamming distance between their local regions): the census Hamming costs
// summed over a block centred on the pixel (samples clamped to the image),
// aggregated by the same SGM recurrence with 16-bit path values.
//
// Two kernels: block_cost_kernel writes the block-cost volume (16-bit, d
// fastest, the path buffers' layout); aggregate_volume_kernel runs the path
// recurrence of every scanline of every direction from that volume.  The
// recurrence, the line layout of a block and the cross-lane steps are those of
// the census-fed aggregation; only the cost source and the value width differ.
#include "aggregate_impl.h"

namespace ss {

namespace {

// ---------------------------------------------------------------- block costs
// 16 pixels of one row per 256-thread block, one 16-lane row per pixel, dpl
// disparities per lane.
template <int DPL, bool WIDE>
__global__ __launch_bounds__(256) void block_cost_kernel(BlockCostArgs a)
{
    using CW = CensusWord<WIDE>;
    using Word = typename CW::T;
    const int lane = threadIdx.x & 15, px = threadIdx.x >> 4;
    const int x = blockIdx.x * 16 + px, y = blockIdx.y;
    if (x >= a.W) return;
    const int W = a.W, H = a.H, d0 = lane * DPL;
    const Word *cl = (const Word *)a.census_l, *cr = (const Word *)a.census_r;
    uint32_t acc[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) acc[j] = 0;
    for (int v = -(a.bh / 2); v <= a.bh / 2; ++v) {
        const int cy = min(max(y + v, 0), H - 1);
        const Word *rl = cl + (size_t)cy * W, *rr = cr + (size_t)cy * W;
        for (int u = -(a.bw / 2); u <= a.bw / 2; ++u) {
            const int cx = min(max(x + u, 0), W - 1);
            const Word wl = rl[cx];
#pragma unroll
            for (int j = 0; j < DPL; ++j) {
                const int xs = cx - d0 - j;
                const uint32_t c = CW::hamming(wl, rr[max(xs, 0)]);
                acc[j] += xs >= 0 ? c : (uint32_t)a.bits;
            }
        }
    }
    store_u16<DPL>(a.vol + ((size_t)y * W + x) * (kLanesPerLine * DPL) + d0, acc);
}

// ---------------------------------------------------------------- aggregation
// One block of 16 lines of one direction (16 lanes per line, horizontal lines
// included), fed from the block-cost volume; the next clock's costs are loaded
// while the current clock computes.
template <int DPL, bool HORIZ>
__device__ __forceinline__ void run_lines_volume(const VolumeArgs &a, const BlockGeom &g, uint16_t *out)
{
    using LO = LineOps<kLanesPerLine>;
    constexpr int kDpad = kLanesPerLine * DPL;
    const int W = a.W, H = a.H, D = a.D;
    const int lane = threadIdx.x % kLanesPerLine, li = threadIdx.x / kLanesPerLine;
    const bool first = lane == 0, last = lane == kLanesPerLine - 1;
    const int d0 = lane * DPL;
    const uint32_t p1 = a.p1, p2 = a.p2;
    const size_t trash = (size_t)W * H * kDpad + d0;

    int row0 = 0, xm0 = 0, xlane = 0, len = 0, skew = 0;
    if (HORIZ) {
        if (li < g.nvalid) len = W;
    } else if (g.kind == 1) {
        row0 = g.ye;
        xm0 = g.g0;
        xlane = li;
        if (li < g.nvalid) {
            const int x0 = g.g0 + li;
            len = g.dx == 0 ? H : min(g.dx > 0 ? W - x0 : x0 + 1, H);
        }
    } else {
        row0 = g.ye + g.dy * (g.j0 + 1);
        xm0 = g.dx > 0 ? g.xe - (kChunk - 1) : g.xe;
        xlane = g.dx > 0 ? kChunk - 1 - li : li;
        skew = li;
        if (li < g.nvalid) len = min(W, H - g.j0 - li - 1);
    }
    auto locate = [&](int t, int &row, int &x) {
        if (HORIZ) {
            row = g.r0 + li;
            x = g.xs + t * g.dx;
        } else {
            row = row0 + t * g.dy;
            x = xm0 + t * g.dx + xlane;
        }
    };
    auto load = [&](int t, uint32_t (&c)[DPL]) {
        int row, x;
        locate(t, row, x);
        row = min(max(row, 0), H - 1);
        x = min(max(x, 0), W - 1);
        load_u16<DPL>(a.vol + ((size_t)row * W + x) * kDpad + d0, c);
    };

    uint32_t Q[DPL], cn[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) Q[j] = 0;
    load(0, cn);
    for (int t = 0; t < g.clocks; ++t) {
        uint32_t C[DPL];
#pragma unroll
        for (int j = 0; j < DPL; ++j) C[j] = cn[j];
        if (t + 1 < g.clocks) load(t + 1, cn);
        const int s = t - skew;
        int row, x;
        locate(t, row, x);
        const bool active = s >= 0 && s < len;
        const uint32_t qm_edge = LO::from_prev(Q[DPL - 1], first);
        const uint32_t qp_edge = LO::from_next(Q[0], last);
        uint32_t L[DPL];
        uint32_t m = 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            uint32_t c = d0 + j < D ? C[j] : kPadCost;
            c = s < 0 ? 0u : c;  // a line that has not started stays at Q = 0
            const uint32_t qm = j > 0 ? Q[j - 1] : qm_edge;
            const uint32_t qp = j < DPL - 1 ? Q[j + 1] : qp_edge;
            L[j] = min(min(Q[j], min(qm, qp) + p1), p2) + c;
            m = min(m, L[j]);
        }
        m = LO::line_min(m);
#pragma unroll
        for (int j = 0; j < DPL; ++j) Q[j] = L[j] - m;
        const size_t o = active ? ((size_t)row * W + x) * kDpad + d0 : trash;
        store_u16<DPL>(out + o, L);
    }
}

template <int DPL>
__global__ __launch_bounds__(kBlock) void aggregate_volume_kernel(VolumeArgs a)
{
    const int blk = (int)blockIdx.x;
    int dir = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < a.ndirs && blk >= a.block_begin[k]) dir = k;
    const BlockGeom g = block_geometry(a.dx[dir], a.dy[dir], blk - a.block_begin[dir], a.W, a.H, kLinesPerBlock);
    if (g.kind == 0) run_lines_volume<DPL, true>(a, g, a.out[dir]);
    else run_lines_volume<DPL, false>(a, g, a.out[dir]);
}

template <int DPL>
hipError_t launch_sgbm_dpl(const BlockCostArgs *bc, const VolumeArgs *va, bool wide, hipStream_t s)
{
    if (bc) {
        dim3 grid((bc->W + 15) / 16, bc->H), block(256);
        if (wide) hipLaunchKernelGGL((block_cost_kernel<DPL, true>), grid, block, 0, s, *bc);
        else hipLaunchKernelGGL((block_cost_kernel<DPL, false>), grid, block, 0, s, *bc);
    } else {
        if (va->block_begin[va->ndirs] == 0) return hipSuccess;
        hipLaunchKernelGGL((aggregate_volume_kernel<DPL>), dim3(va->block_begin[va->ndirs]), dim3(kBlock), 0, s, *va);
    }
    return hipGetLastError();
}

hipError_t launch_sgbm(const BlockCostArgs *bc, const VolumeArgs *va, int dpad, bool wide, hipStream_t s)
{
    switch (dpad / kLanesPerLine) {
    case 1: return launch_sgbm_dpl<1>(bc, va, wide, s);
    case 2: return launch_sgbm_dpl<2>(bc, va, wide, s);
    case 4: return launch_sgbm_dpl<4>(bc, va, wide, s);
    case 6: return launch_sgbm_dpl<6>(bc, va, wide, s);
    case 8: return launch_sgbm_dpl<8>(bc, va, wide, s);
    case 12: return launch_sgbm_dpl<12>(bc, va, wide, s);
    case 16: return launch_sgbm_dpl<16>(bc, va, wide, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_block_cost(const BlockCostArgs &a, int dpad, bool wide, hipStream_t s)
{
    if (a.W < 1 || a.H < 1) return hipSuccess;
    return launch_sgbm(&a, nullptr, dpad, wide, s);
}

hipError_t launch_aggregate_volume(const VolumeArgs &a, hipStream_t s)
{
    return launch_sgbm(nullptr, &a, a.Dpad, false, s);
}

}  // namespace ss
