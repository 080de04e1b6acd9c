// Fused inference of the learned surrogate: all four 3x3 convolutions of the
// net and the combination with the 2-path disparity in one kernel, with no
// activation ever leaving the chip.
//
// A block (4 waves) owns a strip of kOutW output columns and a segment of rows
// of one image and slides down it one row per step.  Every layer is computed
// over the same kRingW = 128 columns (the strip plus a 4-column halo each side)
// and keeps its recent output rows in an LDS ring of 4 slots.  The layers run
// skewed by two rows, so that at step s
//   feature row s+1 is stored, layer 1 computes row s-1, layer 2 row s-3,
//   layer 3 row s-5 and layer 4 row s-7 (residual and logit -> combination),
// each from input rows that were complete before the step began: a step needs
// one barrier, at its start.
//
// Each wave owns two 16-column MFMA tiles of every layer row and keeps every
// weight of the net as MFMA A fragments in registers.  A 3x3 layer's output row
// j reads input rows j-1, j and j+1, and row j+1's output reads j, j+1, j+2, so
// for layers 2 and 3 a wave keeps the B fragments of the last three input rows
// of its tiles in registers (a 3-row register ring, phase fixed at compile time
// by unrolling the step loop three times) and reads only the newest input row
// from LDS.  Layer 1 (4 input channels, 4 taps per k step) and layer 4 read
// their B fragments from the rings.  In LDS a pixel's 32 channels are four
// 16-byte chunks; chunk c of ring pixel p sits at position c ^ ((p >> 1) & 3),
// so the 16-byte fragment reads of 8 consecutive pixels hit 8 different 4-bank
// groups.
//
// Rows and columns outside the image are stored as zeros in every ring (the
// zero padding of the next layer), so each layer sees exactly the input the
// per-layer kernels see.  The GEMM shapes, operand layouts, k order and
// epilogue roundings are those of conv3x3_kernel, so the result equals the
// per-layer forward bit for bit.
#include <algorithm>

#include "internal.h"
#include "net_internal.h"

namespace ss {
namespace net {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kTiles = 2 * kWaves;               // 16-column MFMA tiles per layer row, two per wave
constexpr int kRingW = 16 * kTiles;              // computed columns per layer row
constexpr int kHalo = 4;                         // one column per layer on each side
constexpr int kOutW = kRingW - 2 * kHalo;        // output columns per strip
// ring pixels: a zero column, the computed columns, and a zero tail that the
// last layer-4 tile reads (it starts kHalo columns in and reaches one column past)
constexpr int kRowPx = 1 + kRingW + kHalo + 1;
constexpr int kSlots = 4;                        // rows per ring
constexpr int kSkew = 2;                         // rows between consecutive layers
constexpr int kLead = 1;                         // the feature row stored at step s is s + kLead
// (the last layer-4 tile reads ring columns up to kHalo + kRingW, pixel index one more)
static_assert(kHalo + kRingW + 1 < kRowPx, "layer-4 tiles must stay inside the ring row");

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two values as one packed word, the first in the low half (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

// ReLU on the bit pattern: negative values (sign bit set) become +0, the rest
// pass unchanged; one integer max, with none of the quieting a float max needs
__device__ __forceinline__ float relu(float v) { return __int_as_float(max(__float_as_int(v), 0)); }

// lanes 16..31 (and 48..63) receive the value of lanes 0..15 (32..47): the
// swap of the odd 16-lane rows of one operand with the even rows of the other,
// both operands the same register
__device__ __forceinline__ float from_row_below(float v)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_permlane16_swap(u, u, false, false)[0]);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    bf16x8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// largest feature scale: 8 directions x (census bits + P2 <= 255)
constexpr int kMaxSmax = 8 * 255;

struct Smem {
    uint4 feat[kSlots][kRowPx];          // 8 bf16 feature channels per pixel
    uint4 act[3][kSlots][kRowPx][4];     // [layer][slot][pixel][32 bf16 channels, chunks swizzled]
    unsigned count[kWaves];
    // the learned form's feature quotients, i / 255 and i / D (8-bit inputs) and
    // i / Smax (16-bit inputs, which never exceed Smax)
    float q8[2][256];
    float q16[kMaxSmax + 1];
};

// ring slot of image row r (rows down to -16)
__device__ __forceinline__ int slot4(int r) { return (r + 16) & (kSlots - 1); }
__device__ __forceinline__ int swz(int p, int c) { return c ^ ((p >> 1) & 3); }

__device__ __forceinline__ bf16x8 act_frag(const Smem &sm, int layer, int slot, int p, int quad)
{
    return as_bf16x8(sm.act[layer][slot][p][swz(p, quad)]);
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufWord3 = 0x00020000;    // buffer resource word 3 for raw byte buffers
constexpr uint32_t kDrop = 0x80000000u;  // a buffer offset past every plane here: the access is dropped

// ReLU of two bf16 values packed in a word, as two 16-bit integer maxima: a
// value with its sign bit set (negative, -0, a negative NaN) becomes +0 and the
// rest pass unchanged.  Rounding to bf16 keeps the sign, so this equals the
// fp32 ReLU applied before the rounding, bit for bit.
__device__ __forceinline__ uint32_t relu_pk(uint32_t w)
{
    uint32_t r;
    asm("v_pk_max_i16 %0, %1, 0" : "=v"(r) : "v"(w));
    return r;
}

// Epilogue of a 32-channel ReLU layer (the bias is the accumulator's starting
// value): channels 16 mb + 4 quad .. +3 of ring pixel p (chunk 2 mb + quad / 2,
// half quad % 2); keep = all ones inside the image, 0 outside (stored as zeros).
__device__ __forceinline__ void store_relu(Smem &sm, int layer, int slot, int p, int mb, int quad, uint32_t keep,
                                           const floatx4 &acc)
{
    uint2 w;
    w.x = relu_pk(pack_bf16(acc[0], acc[1])) & keep;
    w.y = relu_pk(pack_bf16(acc[2], acc[3])) & keep;
    uint2 *dst = (uint2 *)&sm.act[layer][slot][p][0] + 2 * swz(p, 2 * mb + quad / 2) + (quad & 1);
    *dst = w;
}

}  // namespace

// The network's input channels of one pixel from the 2-path selection outputs,
// evaluated as the features pass does (same float operations, same bf16
// rounding), so both input routes give the same features bit for bit.  The
// work is split in halves, one packed word each: half 0 makes channels 0, 1
// from (IR, S1), half 1 makes channels 2, 3 from (S2, d*); a half's inputs are
// one 8-bit and one 16-bit value.  Every numerator is a small integer (IR and
// d* below 256; S1 <= Smax; S2 <= Smax or "none", which counts as Smax), so the
// correctly rounded quotients come from tables the block fills once with the
// same divisions: min(v16, Smax) is the 16-bit index in both halves.
__device__ __forceinline__ uint32_t feature_word(const Smem &sm, int half, uint32_t v8, uint32_t v16, int smax_i)
{
    const float a = sm.q16[min(v16, (uint32_t)smax_i)], b = sm.q8[half][v8];
    return half ? pack_bf16(a, b) : pack_bf16(b, a);
}

template <bool FROM_SEL>
__global__ __launch_bounds__(256, 1) void net_infer_kernel(InferArgs a)
{
    __shared__ Smem sm;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int quad = lane >> 4, col = lane & 15;
    const int W = a.W, H = a.H;
    int blk = (int)blockIdx.x;
    const int strip = blk % a.strips;
    blk /= a.strips;
    const int seg = blk % a.segs;
    const int img = blk / a.segs;
    const int x0 = strip * kOutW, xb = x0 - kHalo;
    const int y0 = seg * a.seg_rows, y1 = min(H, y0 + a.seg_rows);
    const int64_t P = (int64_t)H * W;
    const uint4 *feat = (const uint4 *)a.feat + (int64_t)img * P;
    const uint8_t *irp = a.ir;
    int irpitch = a.ir_pitch;
    if (FROM_SEL && a.ir_jobs) {
        const CensusJob *j = (const CensusJob *)a.ir_jobs + 2 * img;
        irp = j->img;
        irpitch = j->pitch;
    }
    const int64_t soff = (int64_t)img * a.sel_stride;
    const uint16_t *s1i = (const uint16_t *)((const uint8_t *)a.s1 + soff);
    const uint16_t *s2i = (const uint16_t *)((const uint8_t *)a.s2 + soff);
    const uint8_t *di = a.dint + soff;

    // every weight of the net as A fragments: lane holds co = 16 mb + col,
    // k = 32 c + 8 quad .. +7 of the layer's [COUTP][kpad(CINP)] layout
    bf16x8 w1[2][3], w2[2][9], w3[2][9], w4[3];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            w1[mb][c] = as_bf16x8(*(const uint4 *)(a.w[0] + (16 * mb + col) * kpad(8) + 32 * c + 8 * quad));
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            w2[mb][c] = as_bf16x8(*(const uint4 *)(a.w[1] + (16 * mb + col) * kpad(32) + 32 * c + 8 * quad));
            w3[mb][c] = as_bf16x8(*(const uint4 *)(a.w[2] + (16 * mb + col) * kpad(32) + 32 * c + 8 * quad));
        }
    }
    // layer 4 as a 16-row product over one input row: row m = 2 ky + c (c the
    // output channel, ky the kernel row; rows 6..15 zero), k = 32 kx + ci, so
    // each new layer-3 row feeds the three output rows it reaches
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (col < 6) v = *(const uint4 *)(a.w[3] + (col % 2) * kpad(32) + 32 * (3 * (col / 2) + kx) + 8 * quad);
        w4[kx] = as_bf16x8(v);
    }
    // The weights are used only as MFMA A operands: keep them in the
    // accumulation registers, which MFMA reads directly, so that the vector
    // registers stay free for the accumulators and the epilogues (left to
    // itself the register allocator parks weights there and copies them back
    // before every use).
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int c = 0; c < 3; ++c) asm volatile("" : "+a"(w1[mb][c]));
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            asm volatile("" : "+a"(w2[mb][c]));
            asm volatile("" : "+a"(w3[mb][c]));
        }
    }
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) asm volatile("" : "+a"(w4[kx]));
    // biases (each chain's starting value) in registers: channels 16 mb + 4 quad .. +3
    floatx4 bias[3][2];
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const float *b = a.b[l] + 16 * mb + 4 * quad;
            bias[l][mb] = floatx4{b[0], b[1], b[2], b[3]};
        }
    const float b40 = a.b[3][0], b41 = a.b[3][1];
    const bool q0 = quad == 0, q1 = quad == 1;

    // Wait for the weight loads here, once: otherwise the waits the compiler
    // places before their first use inside the loop would, on every step, also
    // wait for that step's own feature and disparity loads.  (vmcnt 0, the
    // other counters at their maximum.)
    __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));

    const int smax_i = (int)a.smax;
    if constexpr (FROM_SEL) {
        for (int i = threadIdx.x; i < 256; i += 256) {
            sm.q8[0][i] = (float)i / 255.0f;
            sm.q8[1][i] = (float)i / (float)a.max_disp;
        }
        for (int i = threadIdx.x; i <= smax_i; i += 256) sm.q16[i] = (float)i / a.smax;
    }
    // zero every ring (the zero columns stay zero for good)
    for (int i = threadIdx.x; i < kSlots * kRowPx; i += 256) (&sm.feat[0][0])[i] = make_uint4(0, 0, 0, 0);
    for (int i = threadIdx.x; i < 3 * kSlots * kRowPx * 4; i += 256) (&sm.act[0][0][0][0])[i] = make_uint4(0, 0, 0, 0);

    // The global loads of a step (the feature row stored next step, the 2-path
    // disparities of this step's layer-4 row) are issued at its start together
    // with the stores of the previous step's outputs, and nothing waits on them
    // until the layers have run.  Loads use clamped addresses and are issued
    // unconditionally; out-of-image values are zeroed where they are consumed.
    //
    // Feature rows: threads q and q + 128 (the wave-uniform `half`) handle the
    // two halves of pixel xb + q of the row: 8 bytes of a given feature map, or
    // from the selection outputs one packed word of channels each (the raw
    // values are loaded here and turned into features when they are stored, a
    // step later, so no load is waited on early).
    const int half = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 7);
    const int fq = threadIdx.x & (kRingW - 1), fx = min(max(xb + fq, 0), W - 1);
    const bool fq_inside = xb + fq >= 0 && xb + fq < W;
    // (loads through buffer resources: 32-bit offsets, the bases in scalar registers)
    const __amdgpu_buffer_rsrc_t rs_feat =
        __builtin_amdgcn_make_buffer_rsrc((void *)feat, 0, FROM_SEL ? 0 : (int)(16 * P), kBufWord3);
    auto fetch = [&](int r) {
        const uint32_t px = (uint32_t)min(max(r, 0), H - 1) * (uint32_t)W + (uint32_t)fx;
        const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(rs_feat, 16 * px + 8 * half, 0, 0);
        return make_uint2(v[0], v[1]);
    };
    const uint8_t *p8 = half ? di : irp;
    const int64_t pitch8 = half ? (int64_t)W : (int64_t)irpitch;
    const __amdgpu_buffer_rsrc_t rs16 =
        __builtin_amdgcn_make_buffer_rsrc((void *)(half ? s2i : s1i), 0, FROM_SEL ? (int)(2 * P) : 0, kBufWord3);
    auto fetch_raw = [&](int r, uint32_t &v8, uint32_t &v16) {
        const int row = min(max(r, 0), H - 1);
        // the 8-bit plane may have a pitch: a resource over the row
        const __amdgpu_buffer_rsrc_t r8 = __builtin_amdgcn_make_buffer_rsrc((void *)(p8 + row * pitch8), 0, W, kBufWord3);
        v8 = __builtin_amdgcn_raw_buffer_load_b8(r8, fx, 0, 0);
        v16 = __builtin_amdgcn_raw_buffer_load_b16(rs16, 2 * ((uint32_t)row * (uint32_t)W + (uint32_t)fx), 0, 0);
    };

    // step range: layer 4 (row s - 7) covers rows y0 .. y1-1, so the features
    // (row s + 1) run from y0 - 4 to y1 + 3
    constexpr int D1 = 1, D2 = D1 + kSkew, D3 = D2 + kSkew, D4 = D3 + kSkew;  // row lag of layers 1..4
    const int s0 = y0 - 4 - kLead, s_end = y1 - 1 + D4;
    const int nsteps = s_end - s0 + 1;

    uint2 next = make_uint2(0, 0);
    uint32_t raw_8 = 0, raw_16 = 0;
    if constexpr (FROM_SEL) fetch_raw(s0 + kLead, raw_8, raw_16);
    else next = fetch(s0 + kLead);
    unsigned unsure = 0;
    // layer-4 results of the previous step: row prow (-1: none), this wave's tiles,
    // and the 2-path disparities of that row (loaded during that step)
    float pres[2] = {0.0f, 0.0f}, pz[2] = {0.0f, 0.0f}, pd2[2] = {0.0f, 0.0f};
    int prow = -1;
    const int t_first = 2 * wave;
    // Outputs and the 2-path disparities go through buffer resources over this
    // image's planes: an access at an offset past its plane is dropped by the
    // hardware (a load returns 0), so every lane issues the same accesses and a
    // step has no branches.  A missing array gets an empty resource.  (Planes
    // are below 2^31 bytes: 8 bytes x 8192 x 8192 pixels at most.)
    const int64_t img_px = (int64_t)img * P;
    const __amdgpu_buffer_rsrc_t rs_out = __builtin_amdgcn_make_buffer_rsrc(
        a.out ? (void *)(a.out + img_px * 2) : nullptr, 0, a.out ? (int)(8 * P) : 0, kBufWord3);
    const __amdgpu_buffer_rsrc_t rs_masked = __builtin_amdgcn_make_buffer_rsrc(
        a.masked ? (void *)(a.masked + img * a.masked_stride) : nullptr, 0, a.masked ? (int)(4 * P) : 0, kBufWord3);
    const __amdgpu_buffer_rsrc_t rs_flags = __builtin_amdgcn_make_buffer_rsrc(
        a.masked ? (void *)(a.flags + img * a.flags_stride) : nullptr, 0, a.masked ? (int)P : 0, kBufWord3);
    const __amdgpu_buffer_rsrc_t rs_d2 = __builtin_amdgcn_make_buffer_rsrc(
        a.d2_sub ? (void *)(a.d2_sub + img * a.d2_stride) : nullptr, 0, a.d2_sub ? (int)(4 * P) : 0, kBufWord3);
    // the lanes that write a layer-4 result: quad 1 (rows (2, c) of the
    // product), output columns of the strip inside the image
    bool out_lane[2];
    int out_x[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int o = 16 * (t_first + k) + col;
        out_x[k] = x0 + o;
        out_lane[k] = quad == 1 && o < kOutW && x0 + o < W;
    }
    auto flush = [&]() {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const float d = __fadd_rn(pd2[k], pres[k]);
            const bool ok = pz[k] > 0.0f && d > 0.0f;
            const uint32_t dv = ok ? __builtin_bit_cast(uint32_t, d) : 0u;
            const uint32_t fv = ok ? (uint32_t)(SIMSENSE_FLAG_UNIQUE | SIMSENSE_FLAG_LR | SIMSENSE_FLAG_NONZERO) : 0u;
            const bool st = prow >= 0 && out_lane[k];
            const uint32_t px = (uint32_t)prow * (uint32_t)W + (uint32_t)out_x[k];
            __builtin_amdgcn_raw_buffer_store_b64(
                u32x2{__builtin_bit_cast(uint32_t, pres[k]), __builtin_bit_cast(uint32_t, pz[k])}, rs_out,
                st ? 8 * px : kDrop, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(dv, rs_masked, st ? 4 * px : kDrop, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b8((uint8_t)fv, rs_flags, st ? px : kDrop, 0, 0);
        }
    };
    // the 2-path disparity of this wave's output tiles, column col, clamped into the image
    int d2x[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) d2x[k] = min(max(x0 + 16 * (t_first + k) + col, 0), W - 1);

    // layer-4 partial sums carried from step to step, per tile: row (ky, c) of
    // the 16-row product holds output channel c of the output row that the
    // current input row reaches with kernel row ky
    floatx4 acc4[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    // register rings of B fragments: [row slot][tile][kx] of layers 2 and 3;
    // image row r lives in slot (r - s0 + 12) % 3
    bf16x8 c2[3][2][3], c3[3][2][3];

    auto step = [&](auto phase_c, int s) {
        constexpr int PH = decltype(phase_c)::value;  // (s - s0) % 3
        const int j1 = s - D1, j2 = s - D2, j3 = s - D3, j4 = s - D4;
        __syncthreads();  // every row written last step is complete; its slots' readers are done
        // Global memory, in an order that never waits on this step's own
        // accesses: the feature row loaded last step goes to LDS, the previous
        // step's layer-4 row goes out (with the disparities loaded last step),
        // then this step's loads are issued; each is consumed a step later.
        const int r = s + kLead;
        // one wait for last step's loads (and stores), in every wave, so that no
        // later point of the step waits on memory
        __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));
        const bool fok = fq_inside && r >= 0 && r < H;
        if constexpr (FROM_SEL) {
            // (the ring's channels 4..7 keep the zeros they were given at the start)
            const uint32_t w = feature_word(sm, half, raw_8, raw_16, smax_i);
            ((uint32_t *)&sm.feat[slot4(r)][fq + 1])[half] = fok ? w : 0u;
        } else {
            ((uint2 *)&sm.feat[slot4(r)][fq + 1])[half] = fok ? next : make_uint2(0, 0);
        }
        flush();
        prow = -1;
        if constexpr (FROM_SEL) fetch_raw(r + 1, raw_8, raw_16);
        else next = fetch(r + 1);
        {
            const uint32_t row = (uint32_t)min(max(j4, 0), H - 1) * (uint32_t)W;
#pragma unroll
            for (int k = 0; k < 2; ++k)
                pd2[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs_d2, 4 * (row + d2x[k]), 0, 0));
        }

        // newest input rows of layers 2 and 3 into their register rings
        {
            const int sl1 = slot4(j2 + 1), sl2 = slot4(j3 + 1);
            constexpr int N2 = (PH + 1) % 3, N3 = (PH + 2) % 3;
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int kx = 0; kx < 3; ++kx) {
                    const int p = 16 * (t_first + k) + col + kx;
                    c2[N2][k][kx] = act_frag(sm, 0, sl1, p, quad);
                    c3[N3][k][kx] = act_frag(sm, 1, sl2, p, quad);
                }
        }

        // Every layer runs every step, in one branch-free block, so that one
        // layer's epilogue and LDS traffic can overlap the next layer's matrix
        // products.  A row outside the image is stored as zeros (the same
        // epilogue, with its inside flag false); rows a segment does not need
        // (warm-up and drain) are computed from whatever the rings hold and
        // land in ring slots that no needed row is read from.
        const bool in1 = j1 >= 0 && j1 < H, in2 = j2 >= 0 && j2 < H, in3 = j3 >= 0 && j3 < H;
        bool colin[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int xq = xb + 16 * (t_first + k) + col;
            colin[k] = xq >= 0 && xq < W;
        }
        // layer-1 B fragments: k = 32 c + 8 quad .. +7 is tap 4 c + quad (zero
        // beyond the 9 taps), 8 channels, of feature rows j1-1 .. j1+1
        bf16x8 bf[2][3];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int tap = 4 * c + quad, tc = tap < 9 ? tap : 8;
                uint4 v = sm.feat[slot4(j1 - 1 + tc / 3)][16 * (t_first + k) + col + tc % 3];
                // taps 9..11 (quads 1..3) are padding, whose weights are zero:
                // features built here are finite, so their products are +0 as
                // the zeros of the per-layer kernel's padding are; given feature
                // maps might not be, so those are masked to zero
                if (c == 2 && !FROM_SEL) {
                    const uint32_t m = quad == 0 ? ~0u : 0u;
                    v = make_uint4(v.x & m, v.y & m, v.z & m, v.w & m);
                }
                bf[k][c] = as_bf16x8(v);
            }
        // layer-4 B fragments: the newest layer-3 row (j4 + 1, computed last
        // step), tiles kHalo columns in, three column shifts
        bf16x8 bq[2][3];
#pragma unroll
        for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int kx = 0; kx < 3; ++kx)
                bq[k][kx] = act_frag(sm, 2, slot4(j4 + 1), kHalo + 16 * (t_first + k) + col + kx, quad);

        // Matrix work, ordered so that the products over input rows already in
        // registers (layer 2, kernel rows 0 and 1) run while this step's LDS
        // reads are in flight; each chain still sums bias, tap 0, ..., tap 8 in
        // that order.  Layers 2 and 3 read tap c = 3 ky + kx from ring slot
        // (F + ky) % 3, F = (PH + 2) % 3 for layer 2 (rows j2-1 .. j2+1) and PH
        // for layer 3 (rows j3-1 .. j3+1); four independent chains per layer.
        floatx4 acc1[2][2], acc2[2][2], acc3[2][2];
        auto mid_taps = [&](const bf16x8(&wl)[2][9], const bf16x8(&cache)[3][2][3], auto first_slot, auto c_begin,
                            auto c_end, floatx4(&acc)[2][2]) {
            constexpr int F = decltype(first_slot)::value;
#pragma unroll
            for (int c = decltype(c_begin)::value; c < decltype(c_end)::value; ++c)
#pragma unroll
                for (int k = 0; k < 2; ++k)
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
                        acc[k][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl[mb][c], cache[(F + c / 3) % 3][k][c % 3],
                                                                             acc[k][mb], 0, 0, 0);
        };
        auto epilogue = [&](int layer, int j, bool rowin, const floatx4(&acc)[2][2]) {
            const int sl = slot4(j);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int q = 16 * (t_first + k) + col;
                const uint32_t keep = rowin && colin[k] ? ~0u : 0u;
                store_relu(sm, layer, sl, q + 1, 0, quad, keep, acc[k][0]);
                store_relu(sm, layer, sl, q + 1, 1, quad, keep, acc[k][1]);
            }
        };
        using F2 = std::integral_constant<int, (PH + 2) % 3>;
        using F3 = std::integral_constant<int, PH % 3>;
        using C0 = std::integral_constant<int, 0>;
        using C6 = std::integral_constant<int, 6>;
        using C9 = std::integral_constant<int, 9>;
        auto start = [&](floatx4(&acc)[2][2], int layer) {
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) acc[k][mb] = bias[layer][mb];
        };
        start(acc2, 1);
        mid_taps(w2, c2, F2{}, C0{}, C6{}, acc2);
        // (the compiler's scheduler would otherwise hoist layer 1, whose
        // operands come from LDS, above these products)
        __builtin_amdgcn_sched_barrier(0);
        // layer 1
        start(acc1, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int k = 0; k < 2; ++k)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
                    acc1[k][mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1[mb][c], bf[k][c], acc1[k][mb], 0, 0, 0);
        // layer 2's newest input row, then layer 3
        mid_taps(w2, c2, F2{}, C6{}, C9{}, acc2);
        epilogue(0, j1, in1, acc1);
        start(acc3, 2);
        mid_taps(w3, c3, F3{}, C0{}, C9{}, acc3);
        epilogue(1, j2, in2, acc2);

        // layer 4 on input row j4 + 1: rows (0, c) start output row j4 + 2 from
        // the bias, rows (1, c) continue row j4 + 1, rows (2, c) finish row j4
        // (the per-output order of the products is the per-layer kernel's:
        // bias, then taps 0..8)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx)
#pragma unroll
            for (int k = 0; k < 2; ++k)
                acc4[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w4[kx], bq[k][kx], acc4[k], 0, 0, 0);
        // layer 3's row goes to a slot layer 4 does not read this step
        epilogue(2, j3, in3, acc3);
        prow = j4 >= y0 && j4 < y1 ? j4 : -1;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            // lanes of quad 1 hold rows 4, 5 = (2, c): output channels 0 (residual)
            // and 1 (logit) of row j4, pixel col
            pres[k] = acc4[k][0];
            pz[k] = acc4[k][1];
            unsure += prow >= 0 && out_lane[k] && fabsf(pz[k]) < a.tau ? 1u : 0u;
            // move the partial sums one kernel row on: (1, c) -> (2, c) (lanes
            // 0-15, elements 2, 3 -> lanes 16-31, elements 0, 1), (0, c) -> (1, c),
            // and (0, c) restarts from the bias
            const float m2 = from_row_below(acc4[k][2]), m3 = from_row_below(acc4[k][3]);
            const floatx4 c = acc4[k];
            acc4[k][0] = q0 ? b40 : q1 ? m2 : c[0];
            acc4[k][1] = q0 ? b41 : q1 ? m3 : c[1];
            acc4[k][2] = q0 ? c[0] : c[2];
            acc4[k][3] = q0 ? c[1] : c[3];
        }
    };

    for (int r = 0; r < nsteps; r += 3) {
        step(std::integral_constant<int, 0>{}, s0 + r);
        if (r + 1 < nsteps) step(std::integral_constant<int, 1>{}, s0 + r + 1);
        if (r + 2 < nsteps) step(std::integral_constant<int, 2>{}, s0 + r + 2);
    }
    flush();
    if (!a.uncertain) return;
    // one atomic per block: per-wave sums, then the block's total
    unsigned v = unsure;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) sm.count[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned c = sm.count[0] + sm.count[1] + sm.count[2] + sm.count[3];
        if (c) atomicAdd(a.uncertain + img, c);
    }
}

int infer_grid(const InferArgs &a) { return a.batch * a.segs * a.strips; }

hipError_t launch_infer(InferArgs a, hipStream_t s)
{
    a.strips = (a.W + kOutW - 1) / kOutW;
    if (!a.feat && (a.max_disp < 1 || a.max_disp > 256 || !(a.smax >= 1.0f && a.smax <= (float)kMaxSmax) ||
                    a.smax != (float)(int)a.smax))
        return hipErrorInvalidValue;  // the feature tables cover these ranges only
    if (a.seg_rows <= 0) {
        // Rows per block.  One block runs per compute unit at a time and a block
        // of r rows takes r + 12 steps (the pipeline's warm-up and drain), so
        // the launch takes about ceil(blocks / CUs) x (r + 12) steps: pick the
        // number of row segments per image that minimises it.
        static int num_cus = 0;
        if (num_cus == 0) {
            int dev = 0, n = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                num_cus = n;
            else
                num_cus = 256;
        }
        const int64_t per_seg = (int64_t)a.batch * a.strips;
        int64_t best = -1;
        for (int segs = 1; segs <= a.H; ++segs) {
            const int rows = (a.H + segs - 1) / segs;
            if (segs > 1 && (a.H + rows - 1) / rows != segs) continue;  // the same rows as a smaller count
            const int64_t t = ((per_seg * segs + num_cus - 1) / num_cus) * (rows + 12);
            if (best < 0 || t < best) {
                best = t;
                a.seg_rows = rows;
            }
        }
    }
    a.segs = (a.H + a.seg_rows - 1) / a.seg_rows;
    const int64_t blocks = (int64_t)a.batch * a.segs * a.strips;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    if (a.feat) hipLaunchKernelGGL(net_infer_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(net_infer_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace net
}  // namespace ss
