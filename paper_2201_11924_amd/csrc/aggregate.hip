// Semi-global path aggregation (Sec. VI-D; the SGM recurrence of Hirschmueller,
// which the paper cites):
//   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d+-1) + P1, m + P2) - m,
//   m = min_k L_r(p-r,k),  C(p,d) = popcount(cL(p) ^ cR(p - d)).
//
// Every scanline of every direction is an independent sequence, so each one is
// given to 16 lanes (one DPP row of a wave64) that hold its D-vector, dpl
// consecutive disparities per lane.  A step of the recurrence is then:
//   * the matching cost recomputed from the census words (XOR + popcount), so
//     no cost volume is ever written;
//   * the d-1 / d+1 neighbours from the lane's own registers, and at the lane
//     edges through a row_shr / row_shl DPP move;
//   * the path minimum m through a row_ror butterfly (4 DPP steps);
// and the normalised state Q = L - m is kept in registers along the line.
// With Q the update is L = C + min(Q(d), min(Q(d-1), Q(d+1)) + P1, P2), which
// equals the recurrence above exactly; a line starts from Q = 0, which yields
// L = C at its first pixel.
//
// Each direction writes its path values (<= bits + P2 <= 255) as bytes into a
// buffer of its own; the selection pass sums the directions.
#include "internal.h"

namespace ss {

namespace {

constexpr uint32_t kInf = 0x10000000u;      // outside the disparity range
constexpr uint32_t kPadCost = 0x01000000u;  // cost of the padding disparities >= D

// DPP controls (GFX9 encoding)
constexpr int kRowShl1 = 0x101, kRowShr1 = 0x111;
constexpr int kRowRor1 = 0x121, kRowRor2 = 0x122, kRowRor4 = 0x124, kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xF, 0xF, false);
}

// minimum over the 16 lanes of a DPP row, returned in every lane of the row
__device__ __forceinline__ uint32_t row_min(uint32_t v)
{
    v = min(v, dpp_mov<kRowRor8>(v, v));
    v = min(v, dpp_mov<kRowRor4>(v, v));
    v = min(v, dpp_mov<kRowRor2>(v, v));
    v = min(v, dpp_mov<kRowRor1>(v, v));
    return v;
}

template <bool WIDE>
struct CensusWord;
template <>
struct CensusWord<false> {
    using T = uint32_t;
    static __device__ __forceinline__ uint32_t hamming(T a, T b) { return __popc(a ^ b); }
};
template <>
struct CensusWord<true> {
    using T = uint64_t;
    static __device__ __forceinline__ uint32_t hamming(T a, T b) { return __popcll(a ^ b); }
};

struct Line {
    int x, y, len;
};

__device__ __forceinline__ Line line_geometry(int dx, int dy, int i, int W, int H)
{
    Line ln;
    if (dy == 0) {
        ln.y = i;
        ln.x = dx > 0 ? 0 : W - 1;
        ln.len = W;
    } else if (dx == 0) {
        ln.x = i;
        ln.y = dy > 0 ? 0 : H - 1;
        ln.len = H;
    } else {
        const int ye = dy > 0 ? 0 : H - 1, xe = dx > 0 ? 0 : W - 1;
        if (i < W) {
            ln.x = i;
            ln.y = ye;
        } else {
            ln.x = xe;
            ln.y = ye + dy * (i - W + 1);
        }
        const int lx = dx > 0 ? W - ln.x : ln.x + 1;
        const int ly = dy > 0 ? H - ln.y : ln.y + 1;
        ln.len = min(lx, ly);
    }
    return ln;
}

template <int DPL>
__device__ __forceinline__ void store_bytes(uint8_t *dst, const uint32_t (&L)[DPL])
{
    if constexpr (DPL % 4 == 0) {
        uint32_t w[DPL / 4];
#pragma unroll
        for (int k = 0; k < DPL / 4; ++k)
            w[k] = (L[4 * k] & 0xFF) | ((L[4 * k + 1] & 0xFF) << 8) | ((L[4 * k + 2] & 0xFF) << 16) |
                   (L[4 * k + 3] << 24);
        if constexpr (DPL == 4) {
            *(uint32_t *)dst = w[0];
        } else if constexpr (DPL == 8) {
            *(uint2 *)dst = make_uint2(w[0], w[1]);
        } else if constexpr (DPL == 12) {
            *(uint2 *)dst = make_uint2(w[0], w[1]);
            *(uint32_t *)(dst + 8) = w[2];
        } else {
            static_assert(DPL == 16, "unsupported disparities per lane");
            *(uint4 *)dst = make_uint4(w[0], w[1], w[2], w[3]);
        }
    } else if constexpr (DPL % 2 == 0) {
#pragma unroll
        for (int k = 0; k < DPL / 2; ++k)
            *(uint16_t *)(dst + 2 * k) = (uint16_t)((L[2 * k] & 0xFF) | ((L[2 * k + 1] & 0xFF) << 8));
    } else {
#pragma unroll
        for (int k = 0; k < DPL; ++k) dst[k] = (uint8_t)L[k];
    }
}

}  // namespace

template <int DPL, bool WIDE>
__global__ __launch_bounds__(kBlock) void aggregate_kernel(AggregateArgs a)
{
    using CW = CensusWord<WIDE>;
    using Word = typename CW::T;
    // which direction this block serves (uniform)
    int dir = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k)
        if (k < a.ndirs && (int)blockIdx.x >= a.block_begin[k]) dir = k;
    const int dx = a.dx[dir], dy = a.dy[dir];
    const int lane = threadIdx.x % kLanesPerLine;
    const int line = ((int)blockIdx.x - a.block_begin[dir]) * kLinesPerBlock + threadIdx.x / kLanesPerLine;
    const int W = a.W, H = a.H;
    const int nlines = dy == 0 ? H : (dx == 0 ? W : W + H - 1);
    if (line >= nlines) return;  // whole DPP rows leave together
    Line ln = line_geometry(dx, dy, line, W, H);

    const Word *__restrict__ cl = (const Word *)a.census_l;
    const Word *__restrict__ cr = (const Word *)a.census_r;
    uint8_t *__restrict__ out = a.out[dir];
    const int d0 = lane * DPL;
    const uint32_t p1 = a.p1, p2 = a.p2, bits = a.bits;
    const int D = a.D, Dpad = a.Dpad;

    uint32_t Q[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) Q[j] = 0;

    int x = ln.x, y = ln.y;
    for (int s = 0; s < ln.len; ++s, x += dx, y += dy) {
        const size_t row = (size_t)y * W;
        const Word wl = cl[row + x];
        uint32_t C[DPL];
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int d = d0 + j;
            const int xr = x - d;
            // the load is unconditional (clamped index) so all dpl loads issue together
            const uint32_t c = CW::hamming(wl, cr[row + max(xr, 0)]);
            C[j] = d < D ? (xr >= 0 ? c : bits) : kPadCost;
        }
        const uint32_t qm_edge = dpp_mov<kRowShr1>(kInf, Q[DPL - 1]);
        const uint32_t qp_edge = dpp_mov<kRowShl1>(kInf, Q[0]);
        uint32_t L[DPL];
        uint32_t m = 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const uint32_t qm = j > 0 ? Q[j - 1] : qm_edge;
            const uint32_t qp = j < DPL - 1 ? Q[j + 1] : qp_edge;
            uint32_t t = min(qm, qp) + p1;
            t = min(min(Q[j], t), p2);
            L[j] = C[j] + t;
            m = min(m, L[j]);
        }
        m = row_min(m);
#pragma unroll
        for (int j = 0; j < DPL; ++j) Q[j] = L[j] - m;
        store_bytes<DPL>(out + (row + x) * (size_t)Dpad + d0, L);
    }
}

namespace {
template <int DPL>
hipError_t launch_agg_dpl(const AggregateArgs &a, bool wide, hipStream_t s)
{
    dim3 grid(a.block_begin[a.ndirs]), block(kBlock);
    if (wide)
        hipLaunchKernelGGL((aggregate_kernel<DPL, true>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((aggregate_kernel<DPL, false>), grid, block, 0, s, a);
    return hipGetLastError();
}
}  // namespace

hipError_t launch_aggregate(const AggregateArgs &a, bool wide, hipStream_t s)
{
    if (a.block_begin[a.ndirs] == 0) return hipSuccess;
    switch (a.Dpad / kLanesPerLine) {
    case 1: return launch_agg_dpl<1>(a, wide, s);
    case 2: return launch_agg_dpl<2>(a, wide, s);
    case 4: return launch_agg_dpl<4>(a, wide, s);
    case 6: return launch_agg_dpl<6>(a, wide, s);
    case 8: return launch_agg_dpl<8>(a, wide, s);
    case 12: return launch_agg_dpl<12>(a, wide, s);
    case 16: return launch_agg_dpl<16>(a, wide, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ss
