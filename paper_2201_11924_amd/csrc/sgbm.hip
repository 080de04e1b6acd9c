// Semi-global block matching (Sec. VI-D, the block-based cost mode: two pixels
// are compared through the neighbourhoods around them): the census Hamming
// costs summed over a block centred on the pixel (samples clamped to the image),
// aggregated by the same SGM recurrence with 16-bit path values.
//
// Two kernels: block_cost_kernel writes the block-cost volume (16-bit, d
// fastest, the path buffers' layout); aggregate_volume_kernel runs the path
// recurrence of every scanline of every direction from that volume.  The
// recurrence, the line layout of a block and the cross-lane steps are those of
// the census-fed aggregation; the cost source, the value width and the load
// schedule differ.
#include "aggregate_impl.h"

namespace ss {

namespace {

// ---------------------------------------------------------------- block costs
// 16 pixels of one row per 256-thread block, one 16-lane row per pixel, DPL
// disparities per lane (lane l: l, l + 16, l + 32, ...).  The window rows come
// into LDS by direct-to-LDS loads,
// as many rows at once as fit a 12 KB tile (all of them for blocks up to
// 14 rows at D <= 128), so a block waits for memory once per tile rather than
// once per row.  A tile row holds the left census words the 16 windows cover
// and the right words they reach at every disparity; every sample is an LDS
// read.
template <int DPL, bool WIDE>
__global__ __launch_bounds__(256) void block_cost_kernel(BlockCostArgs a)
{
    using CW = CensusWord<WIDE>;
    using Word = typename CW::T;
    constexpr int kDpad = kLanesPerLine * DPL;
    constexpr int kWordDw = (int)sizeof(Word) / 4;
    constexpr int kLeftWords = 16 + 2 * kMaxBlockHalf;
    constexpr int kRowWords = kLeftWords + kLeftWords + kDpad - 1;  // left slots, then right slots
    constexpr int kRowDw = kRowWords * kWordDw;
    constexpr int kFit = 12288 / (kRowDw * 4);
    constexpr int kRows = kFit < 1 ? 1 : (kFit > 2 * kMaxBlockHalf + 1 ? 2 * kMaxBlockHalf + 1 : kFit);
    constexpr int kLoads = (kRows * kRowDw + 255) / 256;
    __shared__ __align__(16) uint32_t tile[kLoads * 256];
    const int tid = threadIdx.x, lane = tid & 15, px = tid >> 4;
    const int W = a.W, H = a.H, y = blockIdx.y, x0 = blockIdx.x * 16, x = x0 + px;
    // lane l sums disparities l, l + 16, l + 32, ...: for each of them the
    // 16 lanes of a pixel read 16 consecutive right words (no bank conflicts)
    const int hw = a.bw / 2, hh = a.bh / 2;
    // window columns (clamped to the image) and the right columns they reach;
    // right slot k holds column rlo + k (columns left of the image are never
    // counted: their samples cost the full bit count)
    const int xlo = max(x0 - hw, 0), rlo = xlo - (kDpad - 1);
    const uint32_t *cl = (const uint32_t *)a.census_l, *cr = (const uint32_t *)a.census_r;
    uint32_t acc[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) acc[j] = 0;
    const int xc = min(x, W - 1);
    const uint32_t bits = (uint32_t)a.bits;
    const bool inner = rlo >= 0;  // no sample reaches left of the image
    for (int r0 = -hh; r0 <= hh; r0 += kRows) {
        const int nrows = min(kRows, hh - r0 + 1);
        if (r0 > -hh) __syncthreads();  // the previous tile's reads are done
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const int e = tid + 256 * k;  // dword of the tile
            if (e < nrows * kRowDw) {
                const int rr = e / kRowDw, rem = e - rr * kRowDw, idx = rem / kWordDw, h = rem - idx * kWordDw;
                const int row = min(max(y + r0 + rr, 0), H - 1);
                const bool left = idx < kLeftWords;
                const int col = min(max(left ? xlo + idx : rlo + (idx - kLeftWords), 0), W - 1);
                const uint32_t *src = (left ? cl : cr) + ((size_t)row * W + col) * kWordDw + h;
                __builtin_amdgcn_global_load_lds(src, &tile[256 * k + (tid & ~63)], 4, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(vmcnt_encoding(0));
        __syncthreads();
        for (int rr = 0; rr < nrows; ++rr) {
            const Word *sl = (const Word *)tile + rr * kRowWords, *sr = sl + kLeftWords;
            for (int u = -hw; u <= hw; ++u) {
                const int cx = min(max(xc + u, 0), W - 1);
                const Word wl = sl[cx - xlo];
                const Word *rp = &sr[cx - lane - rlo];
                if (inner) {
#pragma unroll
                    for (int j = 0; j < DPL; ++j) acc[j] += CW::hamming(wl, rp[-16 * j]);
                } else {
#pragma unroll
                    for (int j = 0; j < DPL; ++j)
                        acc[j] += cx - lane - 16 * j >= 0 ? CW::hamming(wl, rp[-16 * j]) : bits;
                }
            }
        }
    }
    if (x < W) {
        uint16_t *o = a.vol + ((size_t)y * W + x) * kDpad + lane;
#pragma unroll
        for (int j = 0; j < DPL; ++j) o[16 * j] = (uint16_t)acc[j];
    }
}

// ---------------------------------------------------------------- aggregation
// A lane's DPL 16-bit costs as loaded: packed two per word (one word for DPL 1)
template <int DPL>
constexpr int packed_words() { return DPL == 1 ? 1 : DPL / 2; }

template <int DPL>
__device__ __forceinline__ void load_packed(const uint16_t *src, uint32_t (&w)[packed_words<DPL>()])
{
    constexpr int NW = packed_words<DPL>();
    if constexpr (DPL == 1) {
        w[0] = *src;
    } else {
        const uint32_t *p = (const uint32_t *)src;
        if constexpr (NW % 4 == 0) {
#pragma unroll
            for (int i = 0; i < NW; i += 4) {
                const uint4 q = *(const uint4 *)(p + i);
                w[i] = q.x; w[i + 1] = q.y; w[i + 2] = q.z; w[i + 3] = q.w;
            }
        } else if constexpr (NW % 2 == 0) {
#pragma unroll
            for (int i = 0; i < NW; i += 2) {
                const uint2 q = *(const uint2 *)(p + i);
                w[i] = q.x; w[i + 1] = q.y;
            }
        } else {
#pragma unroll
            for (int i = 0; i < NW; ++i) w[i] = p[i];
        }
    }
}

template <int DPL>
__device__ __forceinline__ uint32_t packed_cost(const uint32_t (&w)[packed_words<DPL>()], int j)
{
    if constexpr (DPL == 1) return w[0];
    else return (j & 1) ? w[j >> 1] >> 16 : w[j >> 1] & 0xFFFFu;
}

// The lines of one block of one direction (LPL lanes per line, kBlock / LPL
// lines), fed from the block-cost volume; the costs of a clock are loaded
// several clocks ahead (the ring below).
template <int DPL, bool HORIZ, int LPL = kLanesPerLine>
__device__ __forceinline__ void run_lines_volume(const VolumeArgs &a, const BlockGeom &g, uint16_t *out)
{
    using LO = LineOps<LPL>;
    constexpr int kDpad = LPL * DPL;
    const int W = a.W, H = a.H, D = a.D;
    const int lane = threadIdx.x % LPL, li = threadIdx.x / LPL;
    const bool first = lane == 0, last = lane == LPL - 1;
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
    constexpr int NP = packed_words<DPL>();
    auto load = [&](int t, uint32_t (&c)[NP]) {
        int row, x;
        locate(t, row, x);
        row = min(max(row, 0), H - 1);
        x = min(max(x, 0), W - 1);
        load_packed<DPL>(a.vol + ((size_t)row * W + x) * kDpad + d0, c);
    };

    // costs come through a ring of kRing clocks (packed as loaded), loaded
    // kRing - 1 clocks ahead: a launch of these lines holds about one wave per
    // SIMD, so each wave must keep many loads in flight to cover the memory
    // latency; the clock loop is unrolled over the ring so the slots stay in
    // fixed registers
    constexpr int kRing = DPL <= 8 ? 12 : 8;
    uint32_t Q[DPL], ring[kRing][NP];
#pragma unroll
    for (int j = 0; j < DPL; ++j) Q[j] = 0;
    auto step = [&](int t, const uint32_t (&cw)[NP]) {
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
            uint32_t c = d0 + j < D ? packed_cost<DPL>(cw, j) : kPadCost;
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
    };
    // clock t sits in slot t % kRing; clocks 0..kRing-2 are loaded up front
    // and clock t + kRing - 1 while clock t is computed
    static_for<kRing - 1>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        load(k, ring[k]);  // clamped position when k >= clocks
    });
    auto group = [&](int t0) {
        static_for<kRing>([&](auto rc) {
            constexpr int r = decltype(rc)::value;
            const int t = t0 + r;
            // (past the last clock the load is of a clamped, unused position:
            // unconditional, so every wait counts a fixed number of loads)
            load(t + kRing - 1, ring[(r + kRing - 1) % kRing]);
            step(t, ring[r]);
        });
    };
    // the first group runs ahead of the loop, so the loop is entered with the
    // loads in flight that each of its iterations leaves (the waits inside it
    // can then count exactly)
    int t0 = 0;
    if (g.clocks >= kRing) {
        group(0);
        for (t0 = kRing; t0 + kRing <= g.clocks; t0 += kRing) group(t0);
    }
    // the last clocks (fewer than kRing), already loaded
    static_for<kRing - 1>([&](auto rc) {
        constexpr int r = decltype(rc)::value;
        if (t0 + r < g.clocks) step(t0 + r, ring[r]);
    });
}

// Horizontal lines (the longest, W clocks) run with volume_horizontal_lanes()
// lanes each, so fewer disparities per lane shorten every clock and the launch
// holds more waves; the other directions keep 16 lanes per line.
template <int DPL>
__global__ __launch_bounds__(kBlock) void aggregate_volume_kernel(VolumeArgs a)
{
    constexpr int kDpad = kLanesPerLine * DPL;
    constexpr int kHL = volume_horizontal_lanes(kDpad);
    const int blk = (int)blockIdx.x;
    int dir = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < a.ndirs && blk >= a.block_begin[k]) dir = k;
    const bool horiz = a.dy[dir] == 0;
    const BlockGeom g = block_geometry(a.dx[dir], a.dy[dir], blk - a.block_begin[dir], a.W, a.H,
                                       horiz ? kBlock / kHL : kLinesPerBlock);
    if (horiz) run_lines_volume<kDpad / kHL, true, kHL>(a, g, a.out[dir]);
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
