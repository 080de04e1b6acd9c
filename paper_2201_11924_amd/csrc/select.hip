// Disparity selection and post-processing (Sec. VI-D): winner-take-all with the
// uniqueness test, quadratic sub-pixel fit, left-right consistency check,
// 3x3 median filter and depth = f*B/d.
//
// The selection pass owns one image row per 512-thread block.  Sixteen lanes
// (one DPP row) hold one pixel's aggregated costs S(d) = sum_r L_r(p,d), dpl
// disparities per lane, exactly as the aggregation pass laid them out.  The
// right-image disparity needed by the LR check, dR(xr) = argmin_d S(xr+d, d),
// gathers costs of D different left pixels; every (x, d) scatters the key
// (S << 8 | d) into an LDS array indexed by xr = x - d with an LDS atomic min,
// so the minimum key gives the lowest cost and, among equal costs, the lowest d.
#include "internal.h"

namespace ss {

namespace {

constexpr int kRowRor1 = 0x121, kRowRor2 = 0x122, kRowRor4 = 0x124, kRowRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp(uint32_t v)
{
    // a row rotation reads a valid lane for every lane: no old value, so the move
    // folds into the consuming min / or as a DPP source
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

__device__ __forceinline__ uint32_t row_min(uint32_t v)
{
    v = min(v, dpp<kRowRor8>(v));
    v = min(v, dpp<kRowRor4>(v));
    v = min(v, dpp<kRowRor2>(v));
    v = min(v, dpp<kRowRor1>(v));
    return v;
}

constexpr int kSelBlock = 512;                            // one image row per block
constexpr int kSelGroups = kSelBlock / kLanesPerLine;     // pixels in flight per row

// Pixel steps of path values held in registers (loads run ring - 1 steps
// ahead), and the waves per SIMD the register budget is sized for: one block
// per image row and three blocks per CU (six waves per SIMD) cover a 720-row
// image in one pass; the widest lanes, 16-bit values and byte values that need
// the split sums (any value >= 128) keep two steps and take the registers they
// need.
constexpr int sel_ring(int dpl, bool v16, bool small) { return (dpl <= 8 && !v16 && (small || dpl <= 4)) ? 3 : 2; }
constexpr int sel_waves_per_simd(int dpl, bool v16, bool small) { return sel_ring(dpl, v16, small) == 3 ? 6 : 2; }

// A pointer that lies in global memory.  Pointers read from a device table
// (the batch form) are generic to the compiler, whose stores through them are
// then flat stores, which also count on the LDS wait counter; stating the
// address space lets it emit global stores, as for kernel arguments.
template <typename T>
using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ global_t<T> *global_ptr(T *p)
{
    return (global_t<T> *)p;
}

template <typename T>
__device__ __forceinline__ T *uniform_ptr(T *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(((uint64_t)hi << 32) | lo);
}

// the dpl path values of one direction for this lane, as packed words: bytes,
// or 16-bit values (V16, block matching)
template <int DPL, bool V16 = false>
struct Words {
    static constexpr int N = V16 ? (DPL + 1) / 2 : (DPL + 3) / 4;
    uint32_t w[N];
};

typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// buffer resource word 3 for raw byte buffers (GFX9 family)
constexpr int kBufferWord3 = 0x00020000;
// Path values are read exactly once: non-temporal (NT) loads keep them from
// displacing other lines in the caches (measured: 185 -> 167 us for a 1280x720
// D=128 8-path selection).
constexpr int kLoadAux = 2;

// The path values of one pixel come through raw buffer loads: one resource per
// direction covers the block's image row, so all directions share one 32-bit
// offset register instead of a 64-bit address each.
template <int DPL>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t rs, uint32_t off, Words<DPL, true> &o)
{
    if constexpr (DPL == 1) {
        o.w[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, kLoadAux);
    } else if constexpr (DPL % 8 == 0) {
#pragma unroll
        for (int i = 0; i < DPL / 2; i += 4) {
            const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 4 * i, 0, kLoadAux);
            o.w[i] = v[0]; o.w[i + 1] = v[1]; o.w[i + 2] = v[2]; o.w[i + 3] = v[3];
        }
    } else if constexpr (DPL % 4 == 0) {
#pragma unroll
        for (int i = 0; i < DPL / 2; i += 2) {
            const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 4 * i, 0, kLoadAux);
            o.w[i] = v[0]; o.w[i + 1] = v[1];
        }
    } else {
#pragma unroll
        for (int i = 0; i < DPL / 2; ++i) o.w[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * i, 0, kLoadAux);
    }
}

// 16-bit path values: a sum of 8 directions stays below 2^16 (the parameters
// bound each value by 8191), so packed pairs add as whole words
template <int DPL, int NDIR>
__device__ __forceinline__ void sum_paths16(const Words<DPL, true> (&v)[NDIR], uint32_t (&S)[DPL])
{
    constexpr int N = Words<DPL, true>::N;
    uint32_t acc[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
        acc[k] = 0;
#pragma unroll
        for (int r = 0; r < NDIR; ++r) acc[k] += v[r].w[k];
    }
#pragma unroll
    for (int j = 0; j < DPL; ++j) S[j] = (j & 1) ? (acc[j / 2] >> 16) : (acc[j / 2] & 0xFFFFu);
}

template <int DPL>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t rs, uint32_t off, Words<DPL> &o)
{
    if constexpr (DPL == 4) {
        o.w[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, kLoadAux);
    } else if constexpr (DPL == 8) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kLoadAux);
        o.w[0] = v[0];
        o.w[1] = v[1];
    } else if constexpr (DPL == 12) {
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, kLoadAux);
        o.w[0] = v[0];
        o.w[1] = v[1];
        o.w[2] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 8, 0, kLoadAux);
    } else if constexpr (DPL == 16) {
        const u32x4_t v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, kLoadAux);
        o.w[0] = v[0];
        o.w[1] = v[1];
        o.w[2] = v[2];
        o.w[3] = v[3];
    } else if constexpr (DPL == 6) {
        // 6 bytes at an even offset lie in the 8 bytes from the dword below it
        // (which end inside the same pixel's values): one load, then a shift
        const u32x2_t v = __builtin_amdgcn_raw_buffer_load_b64(rs, off & ~3u, 0, kLoadAux);
        const uint32_t sh = (off & 2u) * 8;
        o.w[0] = __builtin_amdgcn_alignbit(v[1], v[0], sh);
        o.w[1] = v[1] >> sh;  // bytes 0, 1 are d0 + 4, d0 + 5; the rest is unused
    } else if constexpr (DPL == 2) {
        o.w[0] = __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, kLoadAux);
    } else {
        static_assert(DPL == 1, "unsupported disparities per lane");
        o.w[0] = __builtin_amdgcn_raw_buffer_load_b8(rs, off, 0, kLoadAux);
    }
}

// S(d) = sum over directions of the path bytes.  Bytes are split into two
// 16-bit lanes per word (bytes 0,2 and bytes 1,3) and summed there; no lane
// can carry into the next because a sum of 8 bytes is below 2^16.  When every
// path value is below 128 (bits + P2 <= 127) two directions are first added as
// whole words, since no byte of such a sum can carry.
template <int DPL, int NDIR, bool SMALL>
__device__ __forceinline__ void sum_paths(const Words<DPL> (&v)[NDIR], uint32_t (&S)[DPL])
{
    constexpr int N = Words<DPL>::N;
    uint32_t lo[N], hi[N];
#pragma unroll
    for (int k = 0; k < N; ++k) lo[k] = hi[k] = 0;
    if constexpr (SMALL) {
#pragma unroll
        for (int r = 0; r < NDIR; r += 2)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const uint32_t w = v[r].w[k] + v[r + 1].w[k];
                lo[k] += w & 0x00FF00FFu;
                hi[k] += (w >> 8) & 0x00FF00FFu;
            }
    } else {
#pragma unroll
        for (int r = 0; r < NDIR; ++r)
#pragma unroll
            for (int k = 0; k < N; ++k) {
                lo[k] += v[r].w[k] & 0x00FF00FFu;
                hi[k] += (v[r].w[k] >> 8) & 0x00FF00FFu;
            }
    }
#pragma unroll
    for (int j = 0; j < DPL; ++j) {
        const int k = j / 4, b = j % 4;
        const uint32_t src = (b & 1) ? hi[k] : lo[k];
        S[j] = (b & 2) ? (src >> 16) : (src & 0xFFFFu);
    }
}

}  // namespace

// bitwise AND over the 16 lanes of a DPP row, in every lane of the row
__device__ __forceinline__ uint32_t row_and(uint32_t v)
{
    v &= dpp<kRowRor8>(v);
    v &= dpp<kRowRor4>(v);
    v &= dpp<kRowRor2>(v);
    v &= dpp<kRowRor1>(v);
    return v;
}

// S[t] when 0 <= t < DPL, else 0xFFFF
template <int DPL>
__device__ __forceinline__ uint32_t pick_value(const uint32_t (&S)[DPL], int t)
{
    uint32_t v = 0xFFFFu;
#pragma unroll
    for (int j = 0; j < DPL; ++j) v = t == j ? S[j] : v;
    return v;
}

template <int DPL>
constexpr size_t select_lds_bytes(int W)
{
    return ((size_t)kLanesPerLine * DPL + W) * 4 + (size_t)W * 10;
}

template <int DPL, int NDIR, bool SMALL, bool V16 = false>
__device__ __forceinline__ void select_row(const SelectArgs &a, int y, uint32_t *smem, bool right)
{
    constexpr int kValBytes = V16 ? 2 : 1;
    constexpr int kDpad = kLanesPerLine * DPL;
    const int W = a.W, D = a.D;
    // LDS: right-image keys indexed by xr + Dpad (xr >= -(Dpad-1)); the row's
    // per-pixel results, written to HBM in coalesced row stores after the pixel
    // loop (the loop itself issues no global store, so its look-ahead loads are
    // waited on precisely)
    uint32_t *keyR = smem;
    float *dsub_row = (float *)(keyR + kDpad + W);
    uint16_t *s1_row = (uint16_t *)(dsub_row + W);
    uint16_t *s2_row = s1_row + W;
    uint8_t *dint_row = (uint8_t *)(s2_row + W);
    uint8_t *uniq_row = dint_row + W;
    const size_t row = (size_t)y * W;
    if (right)
        for (int i = threadIdx.x; i < kDpad + W; i += kSelBlock) keyR[i] = 0xFFFFFFFFu;
    __syncthreads();

    const int lane = threadIdx.x % kLanesPerLine, group = threadIdx.x / kLanesPerLine;
    const int d0 = lane * DPL;
    // the pixel loop keeps a ring of kRing pixel steps of path values in
    // registers, loaded kRing - 1 steps ahead; the loop is unrolled over the
    // ring so no register still awaiting its load is ever copied (a copy would
    // wait for it), and look-ahead loads are unconditional (clamped to the row's
    // last pixel) so every wait counts the same loads
    constexpr int kRing = sel_ring(DPL, V16, SMALL);
    __amdgpu_buffer_rsrc_t rs[NDIR];
#pragma unroll
    for (int r = 0; r < NDIR; ++r) {
        const uint8_t *base = uniform_ptr(a.paths[r]) + row * kDpad * kValBytes;
        rs[r] = __builtin_amdgcn_make_buffer_rsrc((void *)base, 0, W * kDpad * kValBytes, kBufferWord3);
    }
    Words<DPL, V16> ring[kRing][NDIR];
    auto load_px = [&](int x, Words<DPL, V16>(&v)[NDIR]) {
        const uint32_t off = (uint32_t)((min(x, W - 1) * kDpad + d0) * kValBytes);
#pragma unroll
        for (int r = 0; r < NDIR; ++r) load_words<DPL>(rs[r], off, v[r]);
    };
    auto process = [&](int x, const Words<DPL, V16>(&v)[NDIR]) {
        uint32_t S[DPL];
        if constexpr (V16) sum_paths16<DPL, NDIR>(v, S);
        else sum_paths<DPL, NDIR, SMALL>(v, S);
        if (D < kDpad) {
            // padding disparities: a cost above every real one (real S < 2^16 - 8)
#pragma unroll
            for (int j = 0; j < DPL; ++j) S[j] = d0 + j < D ? S[j] : 0xFFFFu;
        }

        // winner key (S << 8 | d): the minimum gives the lowest cost and, among
        // equal costs, the lowest d; the same key is scattered to xr = x - d
        uint32_t kmin = 0xFFFFFFFFu;
        const int kb = x - d0 + kDpad - (DPL - 1);  // keyR index of d0 + DPL - 1
#pragma unroll
        for (int j = 0; j < DPL; ++j) kmin = min(kmin, (S[j] << 8) | (uint32_t)(d0 + j));
        if (right) {
#pragma unroll
            for (int j = 0; j < DPL; ++j) atomicMin(&keyR[kb + (DPL - 1 - j)], (S[j] << 8) | (uint32_t)(d0 + j));
        }
        kmin = row_min(kmin);
        const int dstar = (int)(kmin & 0xFF);
        const uint32_t s1 = kmin >> 8;
        // second best: the minimum of S outside the winner's window d*-1 .. d*+1,
        // from the registers (d is in the window when d - d* + 1 is 0, 1 or 2;
        // padding disparities hold 0xFFFF)
        const int q = d0 + 1 - dstar;
        uint32_t s2 = 0xFFFFu;
#pragma unroll
        for (int j = 0; j < DPL; ++j) s2 = min(s2, (uint32_t)(q + j) <= 2u ? 0xFFFFu : S[j]);
        s2 = row_min(s2);
        // neighbours for the sub-pixel fit, S(d*-1) and S(d*+1): the lane holding
        // one picks it from its registers, every other lane contributes all ones,
        // and an AND over the row gathers both halves into one word
        const uint32_t nb = row_and((pick_value<DPL>(S, dstar - 1 - d0) << 16) | pick_value<DPL>(S, dstar + 1 - d0));
        if (lane == 0) {
            const int u = a.uniqueness_pct;
            const bool uniq = u == 0 || s2 == 0xFFFFu || 100u * s1 <= (uint32_t)(100 - u) * s2;
            float ds = (float)dstar;
            if (a.subpixel && dstar > 0 && dstar < D - 1) {
                const int am = (int)(nb >> 16) - (int)s1, bp = (int)(nb & 0xFFFF) - (int)s1;
                ds = __fadd_rn((float)dstar, __fdiv_rn((float)(am - bp), (float)(2 * (am + bp))));
            }
            s1_row[x] = (uint16_t)s1;
            s2_row[x] = (uint16_t)s2;
            dint_row[x] = (uint8_t)dstar;
            dsub_row[x] = ds;
            uniq_row[x] = uniq;
        }
    };
    // (one step's loads after the other, not interleaved by the scheduler: the
    // waits count loads in issue order)
#pragma unroll
    for (int k = 0; k < kRing - 1; ++k) {
        load_px(group + k * kSelGroups, ring[k]);
        __builtin_amdgcn_sched_barrier(0);
    }
    for (int x0 = group; x0 < W; x0 += kRing * kSelGroups) {
#pragma unroll
        for (int s = 0; s < kRing; ++s) {
            load_px(x0 + (s + kRing - 1) * kSelGroups, ring[(s + kRing - 1) % kRing]);
            const int x = x0 + s * kSelGroups;
            if (x < W) process(x, ring[s]);
        }
    }
    __syncthreads();
    const int lr = a.lr_max_diff;
    global_t<uint8_t> *const o_flags = global_ptr(a.flags), *const o_dint = global_ptr(a.disp_int);
    global_t<uint8_t> *const o_dright = global_ptr(a.disp_right);
    global_t<float> *const o_masked = global_ptr(a.masked), *const o_dsub = global_ptr(a.disp_sub);
    global_t<uint16_t> *const o_s1 = global_ptr(a.cost_best), *const o_s2 = global_ptr(a.cost_second);
    for (int x = threadIdx.x; x < W; x += kSelBlock) {
        const int d = dint_row[x];
        const int xr = x - d;
        bool lr_ok = true;
        if (right && lr >= 0) lr_ok = xr >= 0 && abs(d - (int)(keyR[xr + kDpad] & 0xFF)) <= lr;
        const bool nz = d > 0, uq = uniq_row[x] != 0;
        o_flags[row + x] = (uint8_t)(uq | (lr_ok << 1) | (nz << 2));
        o_masked[row + x] = (uq && lr_ok && nz) ? dsub_row[x] : 0.0f;
        if (right) o_dright[row + x] = (uint8_t)(keyR[x + kDpad] & 0xFF);
        o_dint[row + x] = (uint8_t)d;
        o_s1[row + x] = s1_row[x];
        o_s2[row + x] = s2_row[x];
        o_dsub[row + x] = dsub_row[x];
    }
}

template <int DPL, int NDIR, bool SMALL, bool V16>
__global__ __launch_bounds__(kSelBlock, sel_waves_per_simd(DPL, V16, SMALL)) void select_kernel(SelectArgs a)
{
    extern __shared__ uint32_t smem[];
    select_row<DPL, NDIR, SMALL, V16>(a, (int)blockIdx.x, smem, !a.no_right);
}

// batch form: one block per (pair slot, row) item
template <int DPL, int NDIR, bool SMALL>
__global__ __launch_bounds__(kSelBlock, sel_waves_per_simd(DPL, false, SMALL)) void select_batch_kernel(SelectBatch b)
{
    extern __shared__ uint32_t smem[];
    const uint32_t it = b.items[blockIdx.x];
    const SelectArgs &a = b.slots[it >> 20];
    select_row<DPL, NDIR, SMALL>(a, (int)(it & 0xFFFFFu), smem, !(b.no_right || a.no_right));
}

namespace {
template <int DPL, int NDIR>
void launch_sel3(const SelectArgs *a, const SelectBatch *b, bool small, hipStream_t s)
{
    dim3 block(kSelBlock);
    if (a) {
        const size_t lds = select_lds_bytes<DPL>(a->W);
        if (a->values16) hipLaunchKernelGGL((select_kernel<DPL, NDIR, false, true>), dim3(a->H), block, lds, s, *a);
        else if (small) hipLaunchKernelGGL((select_kernel<DPL, NDIR, true, false>), dim3(a->H), block, lds, s, *a);
        else hipLaunchKernelGGL((select_kernel<DPL, NDIR, false, false>), dim3(a->H), block, lds, s, *a);
    } else {
        const size_t lds = select_lds_bytes<DPL>(b->max_width);
        if (small) hipLaunchKernelGGL((select_batch_kernel<DPL, NDIR, true>), dim3(b->nitems), block, lds, s, *b);
        else hipLaunchKernelGGL((select_batch_kernel<DPL, NDIR, false>), dim3(b->nitems), block, lds, s, *b);
    }
}
template <int DPL>
void launch_sel2(const SelectArgs *a, const SelectBatch *b, int ndirs, bool small, hipStream_t s)
{
    if (ndirs == 2) launch_sel3<DPL, 2>(a, b, small, s);
    else if (ndirs == 4) launch_sel3<DPL, 4>(a, b, small, s);
    else launch_sel3<DPL, 8>(a, b, small, s);
}
hipError_t launch_sel(const SelectArgs *a, const SelectBatch *b, int dpad, int ndirs, bool small, hipStream_t s)
{
    switch (dpad / kLanesPerLine) {
    case 1: launch_sel2<1>(a, b, ndirs, small, s); break;
    case 2: launch_sel2<2>(a, b, ndirs, small, s); break;
    case 4: launch_sel2<4>(a, b, ndirs, small, s); break;
    case 6: launch_sel2<6>(a, b, ndirs, small, s); break;
    case 8: launch_sel2<8>(a, b, ndirs, small, s); break;
    case 12: launch_sel2<12>(a, b, ndirs, small, s); break;
    case 16: launch_sel2<16>(a, b, ndirs, small, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
}  // namespace

hipError_t launch_select(const SelectArgs &a, hipStream_t s)
{
    return launch_sel(&a, nullptr, a.Dpad, a.ndirs, a.small_values != 0, s);
}

hipError_t launch_select_batch(const SelectBatch &b, int dpad, int ndirs, bool small, hipStream_t s)
{
    if (b.nitems == 0) return hipSuccess;
    return launch_sel(nullptr, &b, dpad, ndirs, small, s);
}

// ---------------------------------------------------------------- median + depth
// median of 9 values by the 19-exchange network of Paeth (Graphics Gems, 1990);
// min/max exchanges on non-negative floats are exact.
__device__ __forceinline__ void cswap(float &a, float &b)
{
    const float lo = fminf(a, b), hi = fmaxf(a, b);
    a = lo;
    b = hi;
}

__device__ __forceinline__ float median9(float p[9])
{
    cswap(p[1], p[2]); cswap(p[4], p[5]); cswap(p[7], p[8]);
    cswap(p[0], p[1]); cswap(p[3], p[4]); cswap(p[6], p[7]);
    cswap(p[1], p[2]); cswap(p[4], p[5]); cswap(p[7], p[8]);
    cswap(p[0], p[3]); cswap(p[5], p[8]); cswap(p[4], p[7]);
    cswap(p[3], p[6]); cswap(p[1], p[4]); cswap(p[2], p[5]);
    cswap(p[4], p[7]); cswap(p[4], p[2]); cswap(p[6], p[4]);
    cswap(p[4], p[2]);
    return p[4];
}

__device__ __forceinline__ void post_block(const PostArgs &a, int bx, int by)
{
    const int x = bx * 64 + threadIdx.x % 64, y = by * 4 + threadIdx.x / 64;
    if (x >= a.W || y >= a.H) return;
    const size_t p = (size_t)y * a.W + x;
    const global_t<const float> *const masked = global_ptr((const float *)a.masked);
    float v = masked[p];
    if (a.median == 3 && x > 0 && y > 0 && x < a.W - 1 && y < a.H - 1) {
        float w[9];
        int k = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) w[k++] = masked[p + (ptrdiff_t)dy * a.W + dx];
        v = median9(w);
    }
    if (a.disp) global_ptr(a.disp)[p] = v;
    if (a.flags) global_ptr(a.flags)[p] = (uint8_t)(global_ptr(a.flags_in)[p] | (v > 0.0f ? SIMSENSE_FLAG_VALID : 0u));
    if (a.depth) global_ptr(a.depth)[p] = v > 0.0f ? __fdiv_rn(a.fb, v) : 0.0f;
}

__global__ __launch_bounds__(256) void post_kernel(PostArgs a) { post_block(a, blockIdx.x, blockIdx.y); }

// batch form: one block per (pair slot, 64x4 tile) item; tile = by * ceil(W/64) + bx
__global__ __launch_bounds__(256) void post_batch_kernel(PostBatch b)
{
    const uint32_t it = b.items[blockIdx.x];
    const PostArgs &a = b.slots[it >> 20];
    const int tile = (int)(it & 0xFFFFFu), tx = (a.W + 63) / 64;
    post_block(a, tile % tx, tile / tx);
}

hipError_t launch_post(const PostArgs &a, hipStream_t s)
{
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4), block(256);
    hipLaunchKernelGGL(post_kernel, grid, block, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_post_batch(const PostBatch &b, hipStream_t s)
{
    if (b.nitems == 0) return hipSuccess;
    hipLaunchKernelGGL(post_batch_kernel, dim3(b.nitems), dim3(256), 0, s, b);
    return hipGetLastError();
}

// ---------------------------------------------------------------- debug volume
__global__ __launch_bounds__(256) void volume_sum_kernel(PathSet paths, int ndirs, int values16,
                                                         size_t npix, int D, int Dpad, uint16_t *out)
{
    const size_t total = npix * D;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const size_t p = i / D, d = i - p * D;
        uint32_t s = 0;
        for (int r = 0; r < ndirs; ++r)
            s += values16 ? ((const uint16_t *)paths.p[r])[p * Dpad + d] : paths.p[r][p * Dpad + d];
        out[i] = (uint16_t)s;
    }
}

hipError_t launch_volume_sum(const PathSet &paths, int ndirs, bool values16, int W, int H, int D, int Dpad,
                             uint16_t *out, hipStream_t s)
{
    size_t total = (size_t)W * H * D;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(volume_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, paths, ndirs, (int)values16,
                       (size_t)W * H, D, Dpad, out);
    return hipGetLastError();
}

}  // namespace ss

namespace ss {

// ---------------------------------------------------------------- full right-referenced LR
namespace {
template <typename T>
__global__ __launch_bounds__(256) void flip_census_kernel(const T *__restrict__ src, T *__restrict__ dst, int W, int H)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x < W) dst[(size_t)y * W + x] = src[(size_t)y * W + (W - 1 - x)];
}

__global__ __launch_bounds__(256) void lr_full_kernel(LRFullArgs a)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= a.W) return;
    const size_t row = (size_t)y * a.W, p = row + x;
    const int d = a.dint[p], xr = x - d;
    bool lr_ok = true;
    if (a.lr >= 0) lr_ok = xr >= 0 && abs(d - (int)a.dint_m[row + (a.W - 1 - max(xr, 0))]) <= a.lr;
    const uint8_t f = (uint8_t)((a.flags[p] & ~2u) | (lr_ok ? 2u : 0u));
    a.flags[p] = f;
    a.masked[p] = (f & 7u) == 7u ? a.disp_sub[p] : 0.0f;
    a.disp_right[p] = a.dint_m[row + (a.W - 1 - x)];
}
}  // namespace

hipError_t launch_flip_census(const void *src, void *dst, int W, int H, bool wide, hipStream_t s)
{
    dim3 grid((W + 255) / 256, H), block(256);
    if (wide) hipLaunchKernelGGL(flip_census_kernel<uint64_t>, grid, block, 0, s, (const uint64_t *)src, (uint64_t *)dst, W, H);
    else hipLaunchKernelGGL(flip_census_kernel<uint32_t>, grid, block, 0, s, (const uint32_t *)src, (uint32_t *)dst, W, H);
    return hipGetLastError();
}

hipError_t launch_lr_full(const LRFullArgs &a, hipStream_t s)
{
    dim3 grid((a.W + 255) / 256, a.H), block(256);
    hipLaunchKernelGGL(lr_full_kernel, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace ss
