// Semi-global path aggregation kernels (included by the per-disparity-count
// translation units agg_dpl*.hip, which instantiate them in parallel builds).
//
// Semi-global path aggregation (Sec. VI-D; the SGM recurrence of Hirschmueller,
// which the paper cites):
//   L_r(p,d) = C(p,d) + min(L_r(p-r,d), L_r(p-r,d+-1) + P1, m + P2) - m,
//   m = min_k L_r(p-r,k),  C(p,d) = popcount(cL(p) ^ cR(p - d)).
//
// Every scanline of every direction is an independent sequence, so each one is
// given to 16 lanes (one DPP row of a wave64) that hold its D-vector, dpl
// consecutive disparities per lane.  A step of the recurrence is then:
//   * the matching cost recomputed from census words held in LDS (XOR +
//     popcount), so no cost volume is ever written;
//   * the d-1 / d+1 neighbours from the lane's own registers, and at the lane
//     edges through a row_shr / row_shl DPP move;
//   * the path minimum m through a row_ror butterfly (4 DPP steps);
// The lanes keep the un-normalised sums
//   U(p,d) = C(p,d) + min(U(p-r,d), U(p-r,d+-1) + P1, u + P2),  u = min_k U(p-r,k),
// for which induction gives L_r(p,d) = U(p,d) - u exactly (the subtraction of m
// in the recurrence only shifts every value of a step by the same amount), so a
// step needs no normalisation pass: the stored byte is U - u, written straight
// into its byte of the output word (SDWA destination select).  A line starts
// from U = 0, u = 0, which yields L = C at its first pixel; U grows by at most
// bits + P2 per pixel, so 32 bits hold it for any line of the image.
//
// A 256-thread block owns 16 lines of one direction and advances them by one
// "clock" at a time.  Lines are grouped so that at every clock the block's 16
// pixels lie in one image row and 16 consecutive columns (vertical lines, and
// diagonals entering through the top/bottom row), or all in one column of 16
// consecutive rows (horizontal lines).  Diagonals entering through a side column
// are started one clock apart so they also share a row.  The census words a
// block needs for 16 clocks are then a 16 x (Dpad + 31) word tile: it is loaded
// from global memory while the previous 16 clocks are computed from the other
// half of a double-buffered LDS tile, so the scanline loop waits on global
// memory only once per 16 steps.
//
// Each direction writes its path values (<= bits + P2 <= 255) as bytes into a
// buffer of its own, d fastest; the selection pass sums the directions.
#pragma once
#include <algorithm>
#include <type_traits>
#include <utility>

#include "internal.h"

namespace ss {

namespace {

// the neighbour value of a disparity outside the line (the identity of min: the
// neighbour term min(v(d-1), v(d+1)) then takes the one neighbour that exists)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kPadCost = 0x01000000u;  // cost of the padding disparities >= D
constexpr int kChunk = 16;                  // clocks per LDS tile (= lines per block)
static_assert(kChunk == kLinesPerBlock, "one tile slot per line");

// DPP controls (GFX9 encoding)
constexpr int kRowShl1 = 0x101, kRowShr1 = 0x111;
constexpr int kRowRor1 = 0x121, kRowRor2 = 0x122, kRowRor4 = 0x124, kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_rot(uint32_t v)
{
    // a row rotation reads a valid lane for every lane, so no old value is needed
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

// minimum over the 16 lanes of a DPP row, returned in every lane of the row
__device__ __forceinline__ uint32_t row_min(uint32_t v)
{
    v = min(v, dpp_rot<kRowRor8>(v));
    v = min(v, dpp_rot<kRowRor4>(v));
    v = min(v, dpp_rot<kRowRor2>(v));
    v = min(v, dpp_rot<kRowRor1>(v));
    return v;
}

constexpr int kWaveShl1 = 0x130, kWaveShr1 = 0x138;

// Cross-lane pieces of a line that spans LPL lanes (16: one DPP row, 32: half a
// wave, 64: the whole wave).  Lanes hold consecutive disparity blocks.
template <int LPL>
struct LineOps {
    // value of the previous lane (lane 0 of the line gets kNone)
    static __device__ __forceinline__ uint32_t from_prev(uint32_t v, bool first)
    {
        if constexpr (LPL == 16) {
            return dpp_mov<kRowShr1>(kNone, v);
        } else {
            const uint32_t r = dpp_mov<kWaveShr1>(kNone, v);
            return LPL == 32 && first ? kNone : r;
        }
    }
    // value of the next lane (the line's last lane gets kNone)
    static __device__ __forceinline__ uint32_t from_next(uint32_t v, bool last)
    {
        if constexpr (LPL == 16) {
            return dpp_mov<kRowShl1>(kNone, v);
        } else {
            const uint32_t r = dpp_mov<kWaveShl1>(kNone, v);
            return LPL == 32 && last ? kNone : r;
        }
    }
    // minimum over the line's lanes, in every lane of the line: the DPP-row
    // minimum, then rows exchanged in pairs (permlane16 swap: row 0 with row 1,
    // row 2 with row 3) and, for a whole-wave line, halves exchanged (permlane32
    // swap); a swap of a value with itself hands every lane its partner's value
    static __device__ __forceinline__ uint32_t line_min(uint32_t v)
    {
        v = row_min(v);
        if constexpr (LPL >= 32) {
            const auto s = __builtin_amdgcn_permlane16_swap(v, v, false, false);
            v = min((uint32_t)s[0], (uint32_t)s[1]);
        }
        if constexpr (LPL == 64) {
            const auto s = __builtin_amdgcn_permlane32_swap(v, v, false, false);
            v = min((uint32_t)s[0], (uint32_t)s[1]);
        }
        return v;
    }
};

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

// Path-value stores go through global-address-space pointers: a generic (flat)
// store would also count against the LDS counter and make every wait for a
// census read from LDS wait for the outstanding stores as well.
template <typename T>
__device__ __forceinline__ void gstore(uint8_t *p, T v)
{
    *(__attribute__((address_space(1))) T *)p = v;
}
// (native vector types: HIP's uint2/uint4 classes assign through a generic
// `this` pointer, which would turn the store back into a flat one)
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

typedef uint32_t u32x3_t __attribute__((ext_vector_type(3)));

// Cache policy of the path-value stores: non-temporal (NT).  The pass writes
// ~1 GB that only the selection pass reads back; stored with the default policy
// it leaves the last-level caches full of dirty lines whose write-back then
// competes with the selection's reads (measured: selection 241 -> 185 us after
// a 1280x720 D=128 8-path pass, the aggregation itself unchanged).
constexpr int kStoreAux = 2;


// byte B of w = the low byte of a - b, written in place by the subtraction
// itself (SDWA destination select; byte 0 clears the rest of the word, bytes
// 1..3 keep it)
__device__ __forceinline__ void put_byte(uint32_t &w, uint32_t a, uint32_t b, int B)
{
    if (B == 0)
        asm("v_sub_u32_sdwa %0, %1, %2 dst_sel:BYTE_0 dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:DWORD"
            : "=v"(w) : "v"(a), "v"(b));
    else if (B == 1)
        asm("v_sub_u32_sdwa %0, %1, %2 dst_sel:BYTE_1 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
            : "+v"(w) : "v"(a), "v"(b));
    else if (B == 2)
        asm("v_sub_u32_sdwa %0, %1, %2 dst_sel:BYTE_2 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
            : "+v"(w) : "v"(a), "v"(b));
    else
        asm("v_sub_u32_sdwa %0, %1, %2 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:DWORD src1_sel:DWORD"
            : "+v"(w) : "v"(a), "v"(b));
}

// disparities packed per output word: 4 when dpl allows whole words, else
// pairs (16-bit stores) or single bytes
template <int DPL>
__host__ __device__ constexpr int bytes_per_word()
{
    return DPL % 4 == 0 ? 4 : (DPL % 2 == 0 ? 2 : 1);
}

// The lane's dpl path values L = U - u as bytes at byte offset `off` of the
// buffer rs (d0 .. d0 + dpl - 1 of one pixel).  Buffer stores take a 32-bit
// offset, and one at or past the buffer's size is dropped by the hardware, so
// a lane off its line passes such an offset instead of branching.
template <int DPL>
__device__ __forceinline__ void store_path(__amdgpu_buffer_rsrc_t rs, uint32_t off, const uint32_t (&U)[DPL], uint32_t u)
{
    constexpr int G = bytes_per_word<DPL>(), NW = DPL / G;
    uint32_t w[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k)
#pragma unroll
        for (int b = 0; b < G; ++b) put_byte(w[k], U[G * k + b], u, b);
    if constexpr (G == 4) {
        if constexpr (NW == 1) {
            __builtin_amdgcn_raw_buffer_store_b32(w[0], rs, off, 0, kStoreAux);
        } else if constexpr (NW == 2) {
            __builtin_amdgcn_raw_buffer_store_b64(u32x2_t{w[0], w[1]}, rs, off, 0, kStoreAux);
        } else if constexpr (NW == 3) {
            // 12 bytes at a 4-byte-aligned offset: two stores of natural width
            __builtin_amdgcn_raw_buffer_store_b64(u32x2_t{w[0], w[1]}, rs, off, 0, kStoreAux);
            __builtin_amdgcn_raw_buffer_store_b32(w[2], rs, off + 8, 0, kStoreAux);
        } else {
            static_assert(NW == 4, "unsupported disparities per lane");
            __builtin_amdgcn_raw_buffer_store_b128(u32x4_t{w[0], w[1], w[2], w[3]}, rs, off, 0, kStoreAux);
        }
    } else if constexpr (G == 2) {
#pragma unroll
        for (int k = 0; k < NW; ++k) __builtin_amdgcn_raw_buffer_store_b16((uint16_t)w[k], rs, off + 2 * k, 0, kStoreAux);
    } else {
#pragma unroll
        for (int k = 0; k < NW; ++k) __builtin_amdgcn_raw_buffer_store_b8((uint8_t)w[k], rs, off + k, 0, kStoreAux);
    }
}

// store instructions store_path issues per step
template <int DPL>
__host__ __device__ constexpr int store_ops()
{
    return bytes_per_word<DPL>() == 4 ? (DPL == 12 ? 2 : 1) : DPL / bytes_per_word<DPL>();
}

// a buffer offset past every buffer: the store is dropped
constexpr uint32_t kNoStore = 0x80000000u;

// buffer resource word 3 for raw byte buffers (GFX9 family)
constexpr int kBufferWord3 = 0x00020000;

// s_waitcnt immediate that waits for vmcnt <= n and leaves the other counters
// alone (GFX9 encoding: vmcnt[3:0] | expcnt[6:4] | lgkmcnt[11:8] | vmcnt_hi[15:14])
__host__ __device__ constexpr int vmcnt_encoding(int n)
{
    // counts above the 6-bit maximum wait for more than needed, which is safe
    return n > 63 ? vmcnt_encoding(63) : (n & 0xF) | (0x7 << 4) | (0xF << 8) | (((n >> 4) & 0x3) << 14);
}

// dpl 16-bit values (the low halves of v) to consecutive u16 slots (global)
template <int DPL>
__device__ __forceinline__ void store_u16(uint16_t *dst, const uint32_t (&v)[DPL])
{
    uint8_t *p = (uint8_t *)dst;
    if constexpr (DPL == 1) {
        gstore(p, (uint16_t)v[0]);
    } else {
        constexpr int NW = DPL / 2;
        uint32_t w[NW];
#pragma unroll
        for (int i = 0; i < NW; ++i) w[i] = (v[2 * i] & 0xFFFFu) | (v[2 * i + 1] << 16);
        if constexpr (NW % 4 == 0) {
#pragma unroll
            for (int i = 0; i < NW; i += 4) gstore(p + 4 * i, u32x4_t{w[i], w[i + 1], w[i + 2], w[i + 3]});
        } else if constexpr (NW % 2 == 0) {
#pragma unroll
            for (int i = 0; i < NW; i += 2) gstore(p + 4 * i, u32x2_t{w[i], w[i + 1]});
        } else {
#pragma unroll
            for (int i = 0; i < NW; ++i) gstore(p + 4 * i, w[i]);
        }
    }
}

// dpl consecutive 16-bit values, widened to 32 bits
template <int DPL>
__device__ __forceinline__ void load_u16(const uint16_t *src, uint32_t (&v)[DPL])
{
    if constexpr (DPL == 1) {
        v[0] = *src;
    } else {
        constexpr int NW = DPL / 2;
        uint32_t w[NW];
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
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            v[2 * i] = w[i] & 0xFFFFu;
            v[2 * i + 1] = w[i] >> 16;
        }
    }
}

// Geometry of one block of 16 lines of one direction.
//  kind 0: horizontal; the 16 lines are rows r0..r0+15 and every line is at
//          column xs + t*dx at clock t;
//  kind 1: vertical, or diagonal entering through the top/bottom row ye: line i
//          starts at column g0 + i; at clock t every line is in row ye + t*dy and
//          line i in column g0 + t*dx + i;
//  kind 2: diagonal entering through the side column xe: line i starts at row
//          ye + dy*(j0 + i + 1) and runs one clock behind line i-1, so at clock t
//          every line is in row ye + dy*(j0 + 1 + t).
struct BlockGeom {
    int kind, dx, dy;
    int r0, g0, j0;
    int xs, xe, ye;
    int clocks;  // clocks the block runs
    int nvalid;  // lines of the block that exist
};

__device__ __forceinline__ BlockGeom block_geometry(int dx, int dy, int blk, int W, int H, int hlines)
{
    BlockGeom g{};
    g.dx = dx;
    g.dy = dy;
    g.ye = dy > 0 ? 0 : H - 1;
    g.xe = dx > 0 ? 0 : W - 1;
    if (dy == 0) {
        g.kind = 0;
        g.r0 = blk * hlines;
        g.xs = dx > 0 ? 0 : W - 1;
        g.clocks = W;
        g.nvalid = min(hlines, H - g.r0);
    } else {
        const int top_blocks = (W + kChunk - 1) / kChunk;
        if (dx == 0 || blk < top_blocks) {
            g.kind = 1;
            g.g0 = blk * kChunk;
            g.nvalid = min(kChunk, W - g.g0);
            if (dx == 0) {
                g.clocks = H;
            } else {
                // the longest line of the block starts farthest from its exit column
                const int lfirst = dx > 0 ? W - g.g0 : g.g0 + 1;
                const int llast = dx > 0 ? W - (g.g0 + g.nvalid - 1) : g.g0 + g.nvalid;
                g.clocks = min(max(lfirst, llast), H);
            }
        } else {
            g.kind = 2;
            g.j0 = (blk - top_blocks) * kChunk;
            g.nvalid = min(kChunk, H - 1 - g.j0);
            int c = 0;  // line i: skew i, length min(W, H - j0 - i - 1)
            for (int i = 0; i < g.nvalid; ++i) c = max(c, i + min(W, H - g.j0 - i - 1));
            g.clocks = c;
        }
    }
    return g;
}

// row and leftmost column of the block's 16-column window at clock t (kinds 1, 2)
__device__ __forceinline__ void window_at(const BlockGeom &g, int t, int &row, int &xm)
{
    if (g.kind == 1) {
        row = g.ye + t * g.dy;
        xm = g.g0 + t * g.dx;
    } else {
        row = g.ye + g.dy * (g.j0 + 1 + t);
        xm = g.dx > 0 ? g.xe + t - (kChunk - 1) : g.xe - t;
    }
}

}  // namespace

// One block's scanlines.  HORIZ selects the horizontal layout (kind 0);
// otherwise the block is of kind 1 or 2, whose lines share one image row per
// clock: row(t) = row0 + t*dy, leftmost column xm(t) = xm0 + t*dx, lane column
// xm(t) + xlane.  LPL lanes hold one line, DPL disparities each (LPL * DPL = Dpad).
//
// Census tiles move global -> LDS with direct-to-LDS loads into a ring of three
// tile buffers, two chunks ahead of the chunk being computed; every lane of a
// wave writes 4 consecutive bytes, so the tile is filled as a flat array of
// dwords (two per word when census words are 64-bit).
//
// A kind-2 line that has not started yet (clock < its skew) is fed zero cost:
// from U = 0 the recurrence then yields U = 0 and u = 0 until the line's first
// pixel, exactly the state a line starts from.  Lanes of lines that have ended
// (or not started) pass an offset past the buffer, whose store the hardware
// drops, so every step issues the same unconditional store (the chunk-end wait
// counts on that).
// Census words are read from the LDS tile with inline-assembly ds_read_b32: the
// tile is filled by direct-to-LDS loads, and for compiler-visible LDS reads the
// compiler would wait for every outstanding vector memory operation (those loads
// and all path-value stores) before each read.  The tile's readiness is already
// guaranteed by the explicit vmcnt wait and barrier at each chunk boundary, so the
// reads need only their own LDS counter: lds_wait() waits for it and ties the
// results to that wait.
template <int OFF>
__device__ __forceinline__ uint32_t ds_read_at(uint32_t addr)
{
    uint32_t v;
    asm volatile("ds_read_b32 %0, %1 offset:%2" : "=v"(v) : "v"(addr), "i"(OFF));
    return v;
}

template <int N, int BASE = 0, int J = 0>
__device__ __forceinline__ void ds_read_run(uint32_t addr, uint32_t (&w)[N])
{
    if constexpr (J < N) {
        w[J] = ds_read_at<BASE + 4 * J>(addr);
        ds_read_run<N, BASE, J + 1>(addr, w);
    }
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>): a loop
// whose index is a constant expression in the body (LDS offsets as immediates)
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, I...>)
{
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f)
{
    static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int N>
__device__ __forceinline__ void lds_wait(uint32_t &a, uint32_t (&w)[N])
{
    asm volatile("s_waitcnt lgkmcnt(0)" : "+v"(a));
#pragma unroll
    for (int j = 0; j < N; ++j) asm volatile("" : "+v"(w[j]));
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(size_t)p; }

// The scalars one block of lines needs, each made explicitly wavefront-uniform
// (readfirstlane) so that they live in scalar registers even when they were read
// from a work list in memory, which the compiler cannot prove uniform.
struct LineArgs {
    const uint32_t *cl, *cr;  // census words (dwords; two per word when 64-bit)
    uint8_t *out;             // this direction's path values
    int W, H, D, p1, p2, bits;
    int max_work;             // largest block work of the launch (agg_step_cost units)
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T>
__device__ __forceinline__ T *uniform(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// HDIR: 0 for lines that share an image row per clock (kinds 1 and 2); +1 / -1
// for horizontal lines running left-to-right / right-to-left.  A horizontal
// line's cR words slide by one column per clock, so the lane keeps its DPL words
// in registers and reads one new word per clock (plus cL), at offsets that are
// compile-time constants for a given direction.
template <int DPL, int LPL, bool WIDE, int HDIR, int TILE>
__device__ __forceinline__ void run_lines(const LineArgs &a, const BlockGeom &g, uint32_t (*tile)[TILE])
{
    constexpr bool HORIZ = HDIR != 0;
    using CW = CensusWord<WIDE>;
    using LO = LineOps<LPL>;
    using Word = typename CW::T;
    constexpr int kWordDw = WIDE ? 2 : 1;                // dwords per census word
    constexpr int kDpad = LPL * DPL;
    constexpr int kLines = kBlock / LPL;                 // lines per block
    constexpr int kSlots = HORIZ ? kLines : kChunk;      // tile slots: lines or clocks
    // tile layout (words): the cR windows of all slots (Dpad + 15 words each),
    // then the cL windows (16 words each)
    constexpr int kSlotR = kDpad + kChunk - 1;
    constexpr int kRdw = kSlotR * kWordDw, kLdw = kChunk * kWordDw;  // dwords per window
    constexpr int kWaves = kBlock / 64;
    constexpr int kSPW = kSlots / kWaves;                // slots loaded by each wave
    constexpr int kRl = (kRdw + 63) / 64, kLl = (kSPW * kLdw + 63) / 64;
    constexpr int kLoads = kSPW * kRl + kLl;             // load instructions per wave and chunk
    static_assert(kSPW >= 1 && kSlots % kWaves == 0, "every wave loads whole slots");
    static_assert(kSlots * (kRdw + kLdw) <= TILE, "tile too small");
    static_assert(HORIZ || LPL == kLanesPerLine, "row-sharing lines use one DPP row per line");
    const int W = a.W, H = a.H, D = a.D;
    const int lane = threadIdx.x % LPL, li = threadIdx.x / LPL;
    const bool first = lane == 0, last = lane == LPL - 1;
    const int d0 = lane * DPL;
    const uint32_t *__restrict__ cl = a.cl;
    const uint32_t *__restrict__ cr = a.cr;
    uint8_t *__restrict__ out = a.out;
    const uint32_t p1 = a.p1, p2 = a.p2, bits = a.bits;
    const bool padded = D < kDpad;
    // the census bits of a word (a word XORed with this differs from it in `bits` bits)
    const Word bits_mask = bits >= 8 * sizeof(Word) ? ~(Word)0 : (((Word)1 << bits) - 1);

    // per-block line layout
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
    const bool skewed = !HORIZ && g.kind == 2;

    // row and leftmost column of the 16-column window of tile slot `slot` of the
    // chunk that starts at clock c0
    auto slot_window = [&](int c0, int slot, int &row, int &xm) {
        if (HORIZ) {
            row = g.r0 + slot;
            const int xc = g.xs + c0 * g.dx;
            xm = g.dx > 0 ? xc : xc - (kChunk - 1);
        } else {
            row = row0 + (c0 + slot) * g.dy;
            xm = xm0 + (c0 + slot) * g.dx;
        }
    };
    // Direct-to-LDS loads of the chunk starting at clock c0 into ring buffer buf.
    // A window is contiguous in its census map, and the image position of slot s's
    // window is A0 + c0 * Sc + s * Ss (words), so a lane's byte offset is its lane
    // index plus a wave-uniform window offset.  Loads go through buffer resources
    // over the two census maps: a window position outside the image is either
    // another pixel's word or an offset outside the map (the load returns zero);
    // such words reach only disparities with x - d < 0, clocks before a line's
    // start or after its end and lines off the image, whose values the steps
    // replace or never store.
    const int lane64 = threadIdx.x & 63;
    const int s0 = uniform((int)(threadIdx.x >> 6)) * kSPW;
    const int Sc = HORIZ ? g.dx : g.dy * W + g.dx;
    const int Ss = HORIZ ? W : Sc;
    const int A0 = HORIZ ? g.r0 * W + g.xs - (g.dx > 0 ? 0 : kChunk - 1) : row0 * W + xm0;
    const uint32_t map_bytes = (uint32_t)W * H * kWordDw * 4;
    const __amdgpu_buffer_rsrc_t rs_cl = __builtin_amdgcn_make_buffer_rsrc((void *)cl, 0, map_bytes, kBufferWord3);
    const __amdgpu_buffer_rsrc_t rs_cr = __builtin_amdgcn_make_buffer_rsrc((void *)cr, 0, map_bytes, kBufferWord3);
    // a lane's byte offset within the cL loads, relative to the window of slot s0
    uint32_t lofs[kLl];
#pragma unroll
    for (int j = 0; j < kLl; ++j) {
        const int e = lane64 + 64 * j;
        lofs[j] = (uint32_t)(((e / kLdw) * Ss * kWordDw + e % kLdw) * 4);
    }
    auto stage = [&](int c0, int buf) {
        const int base = A0 + c0 * Sc + s0 * Ss;  // window position of slot s0
#pragma unroll
        for (int i = 0; i < kSPW; ++i) {
            const int w0 = (base + i * Ss - (kDpad - 1)) * kWordDw * 4;
#pragma unroll
            for (int m = 0; m < kRl; ++m) {
                auto *dst = (__attribute__((address_space(3))) void *)&tile[buf][(s0 + i) * kRdw + 64 * m];
                const uint32_t vo = (uint32_t)(w0 + 256 * m) + (uint32_t)lane64 * 4;
                if (64 * (m + 1) <= kRdw || lane64 < kRdw - 64 * m)
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_cr, dst, 4, vo, 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < kLl; ++j) {
            auto *dst = (__attribute__((address_space(3))) void *)&tile[buf][kSlots * kRdw + s0 * kLdw + 64 * j];
            const uint32_t vo = (uint32_t)(base * kWordDw * 4) + lofs[j];
            if (64 * (j + 1) <= kSPW * kLdw || lane64 < kSPW * kLdw - 64 * j)
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_cl, dst, 4, vo, 0, 0, 0);
        }
    };
    // lane's pixel, tile slot and window at clock c0 + k
    auto locate = [&](int c0, int k, int &x, int &row, int &xm, int &slot) {
        const int t = c0 + k;
        slot = HORIZ ? li : k;
        slot_window(c0, slot, row, xm);
        x = HORIZ ? g.xs + t * g.dx : xm + xlane;
    };
    // census words of one clock: cL(x) and cR(x - d) for d = d0 + DPL - 1 .. d0
    auto fetch = [&](int buf, int slot, int xo, Word &wl, Word(&wr)[DPL]) {
        const Word *sl = (const Word *)&tile[buf][0] + kSlots * kSlotR + slot * kChunk;  // cL window
        const Word *sr = (const Word *)&tile[buf][0] + slot * kSlotR;                      // cR window
        if constexpr (WIDE) {
            wl = sl[xo];
            const Word *p = sr + (xo + kDpad - d0 - DPL);
#pragma unroll
            for (int j = 0; j < DPL; ++j) wr[j] = p[j];
        } else {
            wl = ds_read_at<0>(lds_addr(sl + xo));
            ds_read_run<DPL>(lds_addr(sr + (xo + kDpad - d0 - DPL)), wr);
        }
    };
    // the words of a fetch may be used only after this
    auto ready = [&](Word &wl, Word(&wr)[DPL]) {
        if constexpr (!WIDE) lds_wait<DPL>(wl, wr);
    };

    // un-normalised path sums U of the lane's disparities and the line minimum
    // u of the previous clock's U
    uint32_t U[DPL];
#pragma unroll
    for (int j = 0; j < DPL; ++j) U[j] = 0;
    uint32_t u = 0;
    // a lane's output byte offset moves by this much per clock
    const int step_off = (HORIZ ? g.dx : g.dy * W + g.dx) * kDpad;

    const int nchunks = (g.clocks + kChunk - 1) / kChunk;
    stage(0, 0);
    if (nchunks > 1) stage(kChunk, 1);
    // chunk 0 must be in LDS: at most chunk 1's loads may still be in flight
    if (nchunks > 1) __builtin_amdgcn_s_waitcnt(vmcnt_encoding(kLoads));
    else __builtin_amdgcn_s_waitcnt(vmcnt_encoding(0));
    __syncthreads();

    // horizontal lines: the lane's sliding window of cR words, preloaded with the
    // words of clock 0 that the first step keeps (tile indices within the line's
    // slot: a column col of chunk 0 is at col - xm + kDpad - 1)
    // (dx > 0: win[i] = cR(x0 - d0 - DPL + i) for i >= 1; dx < 0:
    // win[i] = cR(x0 - d0 - DPL + 2 + i) for i <= DPL - 2; the other word is
    // shifted out by the first step)
    Word win[DPL];
    if constexpr (HORIZ) {
        constexpr int kFirst = HDIR > 0 ? 1 : 0;
        const int idx0 = (HDIR > 0 ? kDpad - 1 - d0 - DPL : kDpad - d0 - DPL + 16) + kFirst;
        if constexpr (DPL == 1) {
            (void)idx0;
        } else if constexpr (!WIDE) {
            uint32_t w[DPL - 1], a0 = lds_addr((const Word *)&tile[0][0] + li * kSlotR + idx0);
            ds_read_run<DPL - 1>(a0, w);
            lds_wait<DPL - 1>(a0, w);
#pragma unroll
            for (int i = 0; i < DPL - 1; ++i) win[kFirst + i] = w[i];
        } else {
            const Word *sl = (const Word *)&tile[0][0] + li * kSlotR + idx0;
#pragma unroll
            for (int i = 0; i < DPL - 1; ++i) win[kFirst + i] = sl[i];
        }
        win[HDIR > 0 ? 0 : DPL - 1] = 0;
    }

    for (int c = 0; c < nchunks; ++c) {
        const int buf = c % 3;
        const int c0 = c * kChunk;
        const bool ahead = c + 2 < nchunks;
        {
            // issue priority from the block's remaining work relative to the
            // launch's largest block: the blocks sharing a SIMD then drain in
            // order of remaining work and tend to finish together, instead of the
            // last one running on alone (measured: 8-path 1280x720 D=128 pass
            // 386 -> 357 us)
            const int rem100 = (g.clocks - c0) * agg_step_cost(DPL, LPL) * 100;
            if (rem100 > 43 * a.max_work) __builtin_amdgcn_s_setprio(3);
            else if (rem100 > 21 * a.max_work) __builtin_amdgcn_s_setprio(2);
            else if (rem100 > 7 * a.max_work) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
        if (ahead) stage(c0 + 2 * kChunk, (c + 2) % 3);
        // the chunk's output window: the image rows its pixels lie in (at most
        // 16), as a buffer resource, and the lane's byte offset in it at clock c0
        int rlo, nrows, off;
        if (HORIZ) {
            rlo = g.r0;
            nrows = g.nvalid;
            off = (li * W + g.xs + c0 * g.dx) * kDpad + d0;
        } else {
            const int ra = row0 + c0 * g.dy, rb = row0 + (c0 + kChunk - 1) * g.dy;
            rlo = max(min(ra, rb), 0);
            nrows = min(max(ra, rb), H - 1) - rlo + 1;
            off = ((ra - rlo) * W + xm0 + c0 * g.dx + xlane) * kDpad + d0;
        }
        const __amdgpu_buffer_rsrc_t rs =
            __builtin_amdgcn_make_buffer_rsrc(out + (size_t)rlo * W * kDpad, 0, nrows * W * kDpad, kBufferWord3);
        // census words of clock K of the chunk.  Lines sharing an image row read
        // tile slot K at a fixed column of the lane, so the LDS addresses are two
        // per-chunk registers plus immediate offsets.
        uint32_t aL = 0, aR = 0;
        if constexpr (!HORIZ && !WIDE) {
            const uint32_t tb = lds_addr(&tile[buf][0]);
            aL = tb + (uint32_t)(kSlots * kSlotR + xlane) * 4;
            aR = tb + (uint32_t)(xlane + kDpad - d0 - DPL) * 4;
        } else if constexpr (HORIZ && !WIDE) {
            // the line's slot; clock K reads cL at window column xo(K) and the one
            // new cR word (dx > 0: column x - d0; dx < 0: x - d0 - DPL + 1)
            const uint32_t tb = lds_addr(&tile[buf][0]);
            aL = tb + (uint32_t)(kSlots * kSlotR + li * kChunk) * 4;
            aR = tb + (uint32_t)(li * kSlotR + (HDIR > 0 ? kDpad - 1 - d0 : kDpad - d0 - DPL)) * 4;
        }
        // horizontal lines: cL and the new cR word of clock K
        auto fetch_slide = [&](auto kc, Word &wl, Word(&wn)[1]) {
            constexpr int K = decltype(kc)::value;
            constexpr int XO = HDIR > 0 ? K : kChunk - 1 - K;  // window column of clock K
            if constexpr (!WIDE) {
                wl = ds_read_at<XO * 4>(aL);
                wn[0] = ds_read_at<XO * 4>(aR);
            } else {
                const Word *sl = (const Word *)&tile[buf][0] + kSlots * kSlotR + li * kChunk;
                const Word *sr = (const Word *)&tile[buf][0] + li * kSlotR;
                wl = sl[XO];
                wn[0] = sr[(HDIR > 0 ? kDpad - 1 - d0 : kDpad - d0 - DPL) + XO];
            }
        };
        auto fetch_clock = [&](auto kc, Word &wl, Word(&wr)[DPL]) {
            constexpr int K = decltype(kc)::value;
            if constexpr (!HORIZ && !WIDE) {
                wl = ds_read_at<K * kChunk * 4>(aL);
                ds_read_run<DPL, K * kSlotR * 4>(aR, wr);
            } else {
                int x, row, xm, slot;
                locate(c0, K, x, row, xm, slot);
                fetch(buf, slot, x - xm, wl, wr);
            }
        };
        Word wl_n, wr_n[DPL], wn_n[1];
        if constexpr (HORIZ) fetch_slide(std::integral_constant<int, 0>{}, wl_n, wn_n);
        else fetch_clock(std::integral_constant<int, 0>{}, wl_n, wr_n);
        static_for<kChunk>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int t = c0 + k;
            const int s = t - skew;
            int x, row, xm, slot;
            locate(c0, k, x, row, xm, slot);
            Word wl;
            Word wr[DPL];
            if constexpr (HORIZ) {
                if constexpr (!WIDE) lds_wait<1>(wl_n, wn_n);
                wl = wl_n;
                // slide the window one column and take in the new word
                if constexpr (HDIR > 0) {
#pragma unroll
                    for (int j = 0; j < DPL - 1; ++j) win[j] = win[j + 1];
                    win[DPL - 1] = wn_n[0];
                } else {
#pragma unroll
                    for (int j = DPL - 1; j > 0; --j) win[j] = win[j - 1];
                    win[0] = wn_n[0];
                }
#pragma unroll
                for (int j = 0; j < DPL; ++j) wr[j] = win[j];
                if constexpr (k + 1 < kChunk) fetch_slide(std::integral_constant<int, k + 1>{}, wl_n, wn_n);
            } else {
                ready(wl_n, wr_n);
                wl = wl_n;
#pragma unroll
                for (int j = 0; j < DPL; ++j) wr[j] = wr_n[j];
                // next clock's census words are read while this clock computes
                if constexpr (k + 1 < kChunk) fetch_clock(std::integral_constant<int, k + 1>{}, wl_n, wr_n);
            }
            // (horizontal lines all span the image width: a per-lane constant and a
            // uniform test, so the check stays on the scalar unit)
            const bool active = HORIZ ? (len > 0 && t < W) : (uint32_t)s < (uint32_t)len;
            const uint32_t um_edge = LO::from_prev(U[DPL - 1], first);
            const uint32_t up_edge = LO::from_next(U[0], last);
            const uint32_t cap = u + p2;
            uint32_t Un[DPL];
            uint32_t m = kNone;
            // the block's leftmost column decides whether any lane sees x - d < 0;
            // the first chunk of skewed lines has lines that have not started
            const bool clip = (HORIZ ? x : xm) < kDpad - 1;
            const bool border = padded || clip || (skewed && c == 0);
            if (!border) {
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const uint32_t um = j > 0 ? U[j - 1] : um_edge;
                    const uint32_t up = j < DPL - 1 ? U[j + 1] : up_edge;
                    const uint32_t tt = min(min(U[j], min(um, up) + p1), cap);
                    Un[j] = tt + CW::hamming(wl, wr[DPL - 1 - j]);
                    m = min(m, Un[j]);
                }
            } else if (!padded && !(skewed && c == 0)) {
                // only x - d < 0 occurs: those disparities compare cL with a word at
                // Hamming distance `bits` from it (cL ^ mask), which costs exactly
                // `bits`, so the update keeps its fused form
                const Word wfix = wl ^ bits_mask;
                const int xd = x - d0;
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const Word wrj = j <= xd ? wr[DPL - 1 - j] : wfix;
                    const uint32_t um = j > 0 ? U[j - 1] : um_edge;
                    const uint32_t up = j < DPL - 1 ? U[j + 1] : up_edge;
                    const uint32_t tt = min(min(U[j], min(um, up) + p1), cap);
                    Un[j] = tt + CW::hamming(wl, wrj);
                    m = min(m, Un[j]);
                }
            } else {
#pragma unroll
                for (int j = 0; j < DPL; ++j) {
                    const int d = d0 + j;
                    const uint32_t cst = CW::hamming(wl, wr[DPL - 1 - j]);
                    uint32_t C = d < D ? (x - d >= 0 ? cst : bits) : kPadCost;
                    C = s < 0 ? 0u : C;  // a line that has not started stays at U = 0
                    const uint32_t um = j > 0 ? U[j - 1] : um_edge;
                    const uint32_t up = j < DPL - 1 ? U[j + 1] : up_edge;
                    const uint32_t tt = min(min(U[j], min(um, up) + p1), cap);
                    Un[j] = tt + C;
                    m = min(m, Un[j]);
                }
            }
            store_path<DPL>(rs, active ? (uint32_t)off : kNoStore, Un, u);
            off += step_off;
            u = LO::line_min(m);
#pragma unroll
            for (int j = 0; j < DPL; ++j) U[j] = Un[j];
        });
        // the next chunk's tile must have landed: only this chunk's look-ahead
        // loads and its kChunk stores may still be in flight.  The tile is written
        // by the loads themselves, so a bare s_barrier (no release fence, which
        // would also wait for every global store) orders the waves; the empty asm
        // statements keep the compiler from moving LDS reads across it.
        if (ahead) __builtin_amdgcn_s_waitcnt(vmcnt_encoding(kLoads + store_ops<DPL>() * kChunk));
        else __builtin_amdgcn_s_waitcnt(vmcnt_encoding(0));
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    }
}

template <int DPL, bool WIDE>
constexpr int agg_tile_dwords()
{
    return (kChunk * (kLanesPerLine * DPL + 2 * kChunk - 1) * (WIDE ? 2 : 1) + kBlock - 1) / kBlock * kBlock;
}

// One block of work: 16 lines (or 256/HL horizontal lines) of one direction.
template <int DPL, bool WIDE, int HL>
__device__ __forceinline__ void aggregate_block(const AggregateArgs &a, int blk, uint32_t (*tile)[agg_tile_dwords<DPL, WIDE>()])
{
    constexpr int kDpad = kLanesPerLine * DPL;
    static_assert(kDpad % HL == 0, "horizontal lanes must divide the padded disparity count");
    // the direction of block blk: the number of later directions whose first block
    // it has passed (all prefix sums loaded at once, not one load per branch)
    const int ndirs = uniform(a.ndirs);
    int bb[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) bb[k] = a.block_begin[k];
    int dir = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) dir += (k < ndirs && blk >= bb[k]) ? 1 : 0;
    dir = uniform(dir);
    LineArgs la;
    la.cl = uniform((const uint32_t *)a.census_l);
    la.cr = uniform((const uint32_t *)a.census_r);
    la.out = uniform(a.out[dir]);
    la.W = uniform(a.W); la.H = uniform(a.H); la.D = uniform(a.D);
    la.p1 = uniform(a.p1); la.p2 = uniform(a.p2); la.bits = uniform(a.bits);
    la.max_work = uniform(max(a.max_item_work, 1));
    const BlockGeom g = block_geometry(uniform(a.dx[dir]), uniform(a.dy[dir]), blk - uniform(a.block_begin[dir]),
                                       la.W, la.H, kBlock / HL);
    if (g.kind == 0) {
        // horizontal lines: more lanes per line to shorten each step
        if (g.dx > 0) run_lines<kDpad / HL, HL, WIDE, 1, agg_tile_dwords<DPL, WIDE>()>(la, g, tile);
        else run_lines<kDpad / HL, HL, WIDE, -1, agg_tile_dwords<DPL, WIDE>()>(la, g, tile);
    } else {
        run_lines<DPL, kLanesPerLine, WIDE, 0, agg_tile_dwords<DPL, WIDE>()>(la, g, tile);
    }
    __builtin_amdgcn_s_setprio(0);
}

template <int DPL, bool WIDE, int HL>
__global__ __launch_bounds__(kBlock) void aggregate_kernel(AggregateArgs a)
{
    __shared__ uint32_t tile[3][agg_tile_dwords<DPL, WIDE>()];
    aggregate_block<DPL, WIDE, HL>(a, (int)blockIdx.x, tile);
}

// Persistent form for batches: a grid sized to the machine takes work items
// (pair slot << 20 | block) from a queue in order (longest first) until it is
// empty; every block leaves once the shared counter passes the item count.
// (4 waves per SIMD: the compiler keeps the 32-bit-census form within 128
// VGPRs, so four blocks fit on a CU)
template <int DPL, bool WIDE, int HL>
__global__ __launch_bounds__(kBlock, 4) void aggregate_queue_kernel(AggregateQueue q)
{
    __shared__ uint32_t tile[3][agg_tile_dwords<DPL, WIDE>()];
    __shared__ int cur;
    for (;;) {
        if (threadIdx.x == 0) cur = (int)atomicAdd(q.counter, 1u);
        __syncthreads();
        const int i = __builtin_amdgcn_readfirstlane(cur);
        __syncthreads();
        if (i >= q.nitems) break;
        const uint32_t it = __builtin_amdgcn_readfirstlane(q.items[i]);
        aggregate_block<DPL, WIDE, HL>(q.slots[it >> 20], (int)(it & 0xFFFFFu), tile);
    }
}

}  // namespace ss
