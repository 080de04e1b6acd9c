// Fused inference of the learned surrogate: all four 3x3 convolutions of the
// net and the combination with the 2-path disparity in one kernel, with no
// activation ever leaving the chip.
//
// A block owns a strip of kOutW output columns and a segment of rows of one
// image and slides down it one row per step.  Each layer keeps the last three
// rows of its output for the strip (plus a 4-column halo on each side) in an
// LDS ring, so a step computes exactly one new row of every layer:
//   feature row r  ->  layer-1 row r-1  ->  layer-2 row r-2  ->  layer-3 row r-3
//   ->  layer-4 row r-4 (residual and logit) -> combination -> HBM.
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

constexpr int kTiles = 6;                       // 16-column MFMA tiles per ring row
constexpr int kRingW = 16 * kTiles;             // computed columns per layer row
constexpr int kHalo = 4;                        // one column per remaining layer
constexpr int kOutW = kRingW - 2 * kHalo - 8;   // output columns per strip (5 tiles)
constexpr int kRowPx = kRingW + 2;              // + one zero column on each side
constexpr int kOutTiles = kOutW / 16;
static_assert(kOutW % 16 == 0, "output strip must be whole tiles");
static_assert(kHalo + kOutW + kHalo <= kRingW, "ring too narrow for the halo");

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two values as one packed word, the first in the low half (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    bf16x8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// Layers 2 and 3 keep their weights in registers; layers 1 and 4 read theirs
// from LDS (rows padded by 16 bytes so a fragment read spreads over the banks).
constexpr int kW1Row = kpad(8) / 8 + 1, kW4Row = kpad(32) / 8 + 1;  // uint4 per padded row

struct Smem {
    uint4 feat[3][kRowPx];          // 8 bf16 feature channels per pixel
    uint4 act[3][3][kRowPx][4];     // [layer][ring slot][pixel][32 bf16 channels, chunks swizzled]
    uint4 w1[32][kW1Row];
    uint4 w4[16][kW4Row];
    float4 bias[3][8];              // layers 1..3, 32 channels each
    float b4[2];                    // layer 4, channels 0 and 1
    unsigned count[4];
};

__device__ __forceinline__ int slot_of(int j) { return (j + 6) % 3; }  // rows j >= -6

// A pixel's 32 channels are four 16-byte chunks; chunk c of ring pixel p is
// stored at position c ^ ((p >> 2) & 3), so that the 16 lanes reading one
// chunk of 16 consecutive pixels (64 bytes apart) hit 16 different 4-bank groups.
__device__ __forceinline__ int swz(int p, int c) { return c ^ ((p >> 2) & 3); }

// One 32-channel ReLU layer row: 6 tiles x 2 output-channel blocks = 12 units,
// three per wave (units 3w .. 3w+2, unit u = tile u/2, channel block u%2); a
// wave's units touch two tiles, whose B fragments it loads once per k step.
// PAR = wave & 1 fixes which channel block and tile each unit uses, so that all
// register arrays are indexed by constants.  B fragments are loaded two k
// steps ahead of the products that use them.
template <int NK, bool FIRST, int PAR>
__device__ __forceinline__ void layer_row(Smem &sm, const bf16x8 (&wa)[2][9], int in_layer, int out_layer, int j,
                                          int xb, int W, int wave, int quad, int col)
{
    const int u0 = 3 * wave;
    const int ta = u0 / 2, tb = (u0 + 2) / 2;
    constexpr int kMb[3] = {PAR, 1 - PAR, PAR};
    constexpr bool kUseB[3] = {false, PAR == 1, true};

    // B fragment of k step c for tiles ta (va) and tb (vb)
    auto load_b = [&](int c, uint4 &va, uint4 &vb) {
        if (FIRST) {
            // k = 32c + 8 quad .. +7 -> tap 4c + quad (zero beyond the 9 taps), 8 channels
            const int tap = 4 * c + quad, tc = tap < 9 ? tap : 8;
            const int slot = slot_of(j - 1 + tc / 3), dx = tc % 3 - 1;
            va = sm.feat[slot][16 * ta + col + dx + 1];
            vb = sm.feat[slot][16 * tb + col + dx + 1];
            if (tap >= 9) va = vb = make_uint4(0, 0, 0, 0);
        } else {
            // k = 32c + 8 quad .. +7 -> tap c, channels 8 quad .. +7
            const int slot = slot_of(j - 1 + c / 3), dx = c % 3 - 1;
            const int pa = 16 * ta + col + dx + 1, pb = 16 * tb + col + dx + 1;
            va = sm.act[in_layer][slot][pa][swz(pa, quad)];
            vb = sm.act[in_layer][slot][pb][swz(pb, quad)];
        }
    };
    floatx4 acc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
    // B fragments two k steps ahead of the products, in a ring of three
    uint4 bufa[3], bufb[3];
    load_b(0, bufa[0], bufb[0]);
    if (NK > 1) load_b(1, bufa[1], bufb[1]);
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        if (c + 2 < NK) load_b(c + 2, bufa[(c + 2) % 3], bufb[(c + 2) % 3]);
        const bf16x8 ba = as_bf16x8(bufa[c % 3]), bb = as_bf16x8(bufb[c % 3]);
        bf16x8 a0, a1;
        if (FIRST) {
            a0 = as_bf16x8(sm.w1[col][4 * c + quad]);
            a1 = as_bf16x8(sm.w1[16 + col][4 * c + quad]);
        } else {
            a0 = wa[0][c];
            a1 = wa[1][c];
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
            acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kMb[i] ? a1 : a0, kUseB[i] ? bb : ba, acc[i], 0, 0, 0);
    }
    const int slot = slot_of(j);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int mb = kMb[i], t = kUseB[i] ? tb : ta;
        const int q = 16 * t + col, x = xb + q;
        const bool inside = x >= 0 && x < W;
        const float4 bv = sm.bias[out_layer][4 * mb + quad];  // channels 16 mb + 4 quad .. +3
        const float bias[4] = {bv.x, bv.y, bv.z, bv.w};
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = inside ? fmaxf(acc[i][e] + bias[e], 0.0f) : 0.0f;
        uint2 w;
        w.x = pack_bf16(v[0], v[1]);
        w.y = pack_bf16(v[2], v[3]);
        // channels 16 mb + 4 quad .. +3: chunk 2 mb + quad / 2, half quad % 2
        uint2 *dst = (uint2 *)&sm.act[out_layer][slot][q + 1][0] + 2 * swz(q + 1, 2 * mb + quad / 2) + (quad & 1);
        *dst = w;
    }
}

template <int NK, bool FIRST>
__device__ __forceinline__ void layer_row_any(Smem &sm, const bf16x8 (&wa)[2][9], int in_layer, int out_layer, int j,
                                              int xb, int W, int wave, int quad, int col)
{
    if (wave & 1) layer_row<NK, FIRST, 1>(sm, wa, in_layer, out_layer, j, xb, W, wave, quad, col);
    else layer_row<NK, FIRST, 0>(sm, wa, in_layer, out_layer, j, xb, W, wave, quad, col);
}

__device__ __forceinline__ void zero_row(Smem &sm, int layer, int j)
{
    const int slot = slot_of(j);
    for (int i = threadIdx.x; i < kRingW * 4; i += 256) sm.act[layer][slot][1 + i / 4][i % 4] = make_uint4(0, 0, 0, 0);
}

}  // namespace

// The network's input channels of one pixel from the 2-path selection outputs,
// evaluated as the features pass does (same float operations, same bf16
// rounding), so both input routes give the same features bit for bit.
struct RawFeat {
    uint32_t ir, s1, s2, d;
};

__device__ __forceinline__ uint4 feature_of(const RawFeat &v, float smax, int max_disp)
{
    const float s2 = v.s2 == 0xFFFFu ? smax : fminf((float)v.s2, smax);
    const float f0 = (float)v.ir / 255.0f, f1 = (float)v.s1 / smax, f2 = s2 / smax, f3 = (float)v.d / (float)max_disp;
    return make_uint4(pack_bf16(f0, f1), pack_bf16(f2, f3), 0u, 0u);
}

template <bool FROM_SEL>
__global__ __launch_bounds__(256, 2) void net_infer_kernel(InferArgs a)
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

    // weights as A fragments: lane holds co = 16 mb + col, k = 32 c + 8 quad .. +7
    bf16x8 w2[2][9], w3[2][9];
    for (int i = threadIdx.x; i < 32 * (kpad(8) / 8); i += 256)
        sm.w1[i / (kpad(8) / 8)][i % (kpad(8) / 8)] = ((const uint4 *)a.w[0])[i];
    for (int i = threadIdx.x; i < 16 * (kpad(32) / 8); i += 256)
        sm.w4[i / (kpad(32) / 8)][i % (kpad(32) / 8)] = ((const uint4 *)a.w[3])[i];
    if (threadIdx.x < 96) (&sm.bias[0][0].x)[threadIdx.x] = a.b[threadIdx.x / 32][threadIdx.x % 32];
    if (threadIdx.x < 2) sm.b4[threadIdx.x] = a.b[3][threadIdx.x];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            w2[mb][c] = as_bf16x8(*(const uint4 *)(a.w[1] + (16 * mb + col) * kpad(32) + 32 * c + 8 * quad));
            w3[mb][c] = as_bf16x8(*(const uint4 *)(a.w[2] + (16 * mb + col) * kpad(32) + 32 * c + 8 * quad));
        }
    }

    // Wait for the weight loads here, once: otherwise the waits the compiler
    // places before their first use inside the loop would, on every step, also
    // wait for that step's own feature and disparity loads.  (vmcnt 0, the
    // other counters at their maximum.)
    __builtin_amdgcn_s_waitcnt((0x7 << 4) | (0xF << 8));

    // zero every ring (the side columns stay zero for good)
    for (int i = threadIdx.x; i < 3 * kRowPx; i += 256) (&sm.feat[0][0])[i] = make_uint4(0, 0, 0, 0);
    for (int i = threadIdx.x; i < 3 * 3 * kRowPx * 4; i += 256) (&sm.act[0][0][0][0])[i] = make_uint4(0, 0, 0, 0);

    // Every global load of a step is issued at its start (the next feature row,
    // this step's 2-path disparities) together with the stores of the previous
    // step's outputs, and nothing waits on them until the layers have run, so
    // memory latency hides behind the step's matrix work.  Loads use clamped
    // addresses and are issued unconditionally; out-of-image values are zeroed
    // where they are consumed.
    //
    // feature row prefetch: thread q < 128 holds pixel xb + q of the row
    const int fq = threadIdx.x & 127, fx = min(max(xb + fq, 0), W - 1);
    const bool fq_inside = fq < kRingW && xb + fq >= 0 && xb + fq < W;
    auto fetch = [&](int r) { return feat[(int64_t)min(max(r, 0), H - 1) * W + fx]; };
    // (from the selection outputs: the raw values are loaded here and turned into
    // features when they are stored, a step later, so no load is waited on early)
    auto fetch_raw = [&](int r) {
        const int64_t row = min(max(r, 0), H - 1), p = row * W + fx;
        RawFeat v;
        v.ir = irp[row * irpitch + fx];
        v.s1 = s1i[p];
        v.s2 = s2i[p];
        v.d = di[p];
        return v;
    };
    uint4 next = make_uint4(0, 0, 0, 0);
    RawFeat next_raw{0u, 0u, 0u, 0u};
    if (threadIdx.x < 128) {
        if constexpr (FROM_SEL) next_raw = fetch_raw(y0 - 4);
        else next = fetch(y0 - 4);
    }
    unsigned unsure = 0;
    // layer-4 results of the previous step: row prow (-1: none), tiles wave and wave + 4
    float pres[2] = {0.0f, 0.0f}, pz[2] = {0.0f, 0.0f}, pd2[2] = {0.0f, 0.0f};
    int prow = -1;
    auto flush = [&]() {
        if (prow < 0 || quad != 0) return;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int t = wave + 4 * k, x = x0 + 16 * t + col;
            if (t >= kOutTiles || x >= W) continue;
            const int64_t p = (int64_t)prow * W + x;
            if (a.out) {
                float2 o;
                o.x = pres[k];
                o.y = pz[k];
                *(float2 *)(a.out + ((int64_t)img * P + p) * 2) = o;
            }
            if (a.masked) {
                const float d = __fadd_rn(pd2[k], pres[k]);
                const bool ok = pz[k] > 0.0f && d > 0.0f;
                a.masked[img * a.masked_stride + p] = ok ? d : 0.0f;
                a.flags[img * a.flags_stride + p] =
                    (uint8_t)(ok ? (SIMSENSE_FLAG_UNIQUE | SIMSENSE_FLAG_LR | SIMSENSE_FLAG_NONZERO) : 0u);
            }
        }
    };
    // the 2-path disparity of tile wave + 4k, column col, clamped into the image
    const float *d2img = a.d2_sub ? a.d2_sub + img * a.d2_stride : nullptr;
    int d2x[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) d2x[k] = min(x0 + 16 * (wave + 4 * k) + col, W - 1);

    for (int r = y0 - 4; r <= y1 + 3; ++r) {
        const int j4 = r - 4;  // this step's output row
        __syncthreads();  // the previous step's readers of the feature slot are done
        if (threadIdx.x < kRingW) {
            const bool ok = fq_inside && r >= 0 && r < H;
            if constexpr (FROM_SEL) next = feature_of(next_raw, a.smax, a.max_disp);
            sm.feat[slot_of(r)][threadIdx.x + 1] = ok ? next : make_uint4(0, 0, 0, 0);
        }
        if (threadIdx.x < 128) {
            if constexpr (FROM_SEL) next_raw = fetch_raw(r + 1);
            else next = fetch(r + 1);
        }
        float d2v[2] = {0.0f, 0.0f};
        if (d2img) {
            const int64_t row = (int64_t)min(max(j4, 0), H - 1) * W;
#pragma unroll
            for (int k = 0; k < 2; ++k) d2v[k] = d2img[row + d2x[k]];
        }
        flush();
        __syncthreads();
        // layer 1, row r - 1 (needed for rows y0-3 .. y1+2)
        {
            const int j = r - 1;
            if (j >= y0 - 3) {
                if (j < 0 || j >= H) zero_row(sm, 0, j);
                else layer_row_any<3, true>(sm, w2, 0, 0, j, xb, W, wave, quad, col);
            }
        }
        __syncthreads();
        {
            const int j = r - 2;
            if (j >= y0 - 2 && j <= y1 + 1) {
                if (j < 0 || j >= H) zero_row(sm, 1, j);
                else layer_row_any<9, false>(sm, w2, 0, 1, j, xb, W, wave, quad, col);
            }
        }
        __syncthreads();
        {
            const int j = r - 3;
            if (j >= y0 - 1 && j <= y1) {
                if (j < 0 || j >= H) zero_row(sm, 2, j);
                else layer_row_any<9, false>(sm, w3, 1, 2, j, xb, W, wave, quad, col);
            }
        }
        __syncthreads();
        pd2[0] = d2v[0];
        pd2[1] = d2v[1];
        prow = -1;
        // layer 4, row r - 4: 5 output tiles at ring columns kHalo + 16 t
        if (j4 >= y0 && j4 < y1) {
            prow = j4;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int t = wave + 4 * k;
                if (t >= kOutTiles) break;
                uint4 bv[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) {
                    const int pc = kHalo + 16 * t + col + c % 3;
                    bv[c] = sm.act[2][slot_of(j4 - 1 + c / 3)][pc][swz(pc, quad)];
                }
                floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < 9; ++c)
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(sm.w4[col][4 * c + quad]),
                                                                  as_bf16x8(bv[c]), acc, 0, 0, 0);
                // lanes of quad 0 hold output channels 0 (residual) and 1 (logit) of pixel col
                pres[k] = acc[0] + sm.b4[0];
                pz[k] = acc[1] + sm.b4[1];
                const int x = x0 + 16 * t + col;
                if (quad == 0 && x < W) unsure += fabsf(pz[k]) < a.tau ? 1u : 0u;
            }
        }
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
    if (a.seg_rows <= 0) {
        // rows per block: long segments amortise the 4-row warm-up of the
        // pipeline, short ones give small batches enough blocks (about 1024)
        const int64_t want = ((int64_t)a.batch * a.strips * a.H + 1023) / 1024;
        a.seg_rows = (int)std::min<int64_t>(90, std::max<int64_t>(12, want));
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
