// Learned surrogate: a 4-layer 3x3 convolutional net (4 -> 32 -> 32 -> 32 -> 2,
// ReLU after the first three, zero padding) on features of a 2-path SGM result,
// predicting a disparity residual and a validity logit.  BF16 weights and
// activations, FP32 accumulation on the gfx950 matrix cores, hand-written
// forward, backward (data and weight) and Adam kernels.
//
// Layouts.  Activations are NHWC bf16 with the channel count padded to 8 (the
// 4 feature channels, the 2 output-gradient channels) or 32.  A convolution is
// an implicit GEMM out[co][p] = sum_k Wk[co][k] * X[k][p] with k = tap * CINP + ci
// (tap = 3*ky + kx), computed by v_mfma_f32_16x16x32_bf16 with the weights as the
// A operand (16 output channels x 32 k) and the activations as the B operand
// (32 k x 16 pixels): a lane then owns 4 consecutive output channels of one
// pixel, i.e. 8 contiguous bytes of the NHWC output.  The backward-data pass is
// the same kernel with the taps mirrored and the channel roles swapped.
#include <algorithm>
#include <math.h>
#include <string.h>

#include "internal.h"
#include "net_internal.h"

namespace ss {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// fp32 -> bf16, round to nearest even (the gfx950 conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
// two values as one packed word, the first in the low half (v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi)
{
    const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
    return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ReLU on the bit pattern: negative values (sign bit set) become +0, the rest
// pass unchanged; one integer max, with none of the quieting a float max needs
__device__ __forceinline__ float relu(float v) { return __int_as_float(max(__float_as_int(v), 0)); }

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 v)
{
    bf16x8 r;
    __builtin_memcpy(&r, &v, sizeof(r));
    return r;
}

// ------------------------------------------------------------------ forward / backward-data
// A 3x3 convolution as an implicit GEMM on v_mfma_f32_16x16x32_bf16: the weights
// are the A operand (16 output channels x 32 k, k = tap * CINP + ci, held in
// registers for the block's whole run) and the input the B operand (32 k x 16
// pixels).  A block owns 64 output columns of one image over 16 rows, taken as 4
// sub-strips of 4 rows (one row per wave, four 16-pixel tiles each).  For each
// sub-strip it stages the 6 input rows x 66 columns it reads in LDS (pixel-major,
// as in memory; positions outside the image are zeros), so every input pixel is
// loaded once per sub-strip instead of once per tap, and a B fragment (8
// channels of one pixel and tap) is one aligned 16-byte LDS read.  Each output's
// products are summed onto its starting value in k order.  A 32-channel ReLU layer
// also stores which of its stored outputs are > 0, packed 4 bytes per pixel: byte q
// holds channels 4q .. 4q+3 (bits 0-3) and 16+4q .. 16+4q+3 (bits 4-7), the eight
// channels lane quad q holds in the MFMA output layout; backward-data reads that
// byte instead of the 64-byte activation.
constexpr int kConvCols = 64;   // output columns per block
constexpr int kConvRows = 4;    // output rows per sub-strip (one per wave)
constexpr int kConvSubs = 4;    // sub-strips per block
constexpr int kConvBufWord3 = 0x00020000;    // buffer resource word 3 for raw byte buffers
constexpr uint32_t kConvDrop = 0x80000000u;  // an offset past every map here: the load returns zeros
typedef uint32_t u32x4c __attribute__((ext_vector_type(4)));
// staged pixel pitch in bf16 values: 32 channels are padded to 40 so that the
// 16-byte reads of 8 consecutive pixels hit 8 different 4-bank groups
__host__ __device__ constexpr int conv_pitch(int cinp) { return cinp == 32 ? 40 : cinp; }

template <int CINP, int COUTP, int EPI>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a)
{
    constexpr int KPAD = kpad(CINP);
    constexpr int NK = KPAD / 32;
    constexpr int MB = COUTP / 16;
    constexpr int PP = conv_pitch(CINP);
    constexpr int SR = kConvRows + 2, SC = kConvCols + 2;  // staged rows and columns
    constexpr int XC = CINP / 8;                             // 16-byte chunks per pixel
    constexpr int NCH = SR * SC * XC;                        // chunks per sub-strip
    __shared__ __align__(16) uint16_t st[SR][SC][PP];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int quad = lane >> 4, col = lane & 15;
    const uint16_t *__restrict__ wk = a.weights;

    // A fragments (weights): lane holds co = 16*mb + col, k = 32*c + 8*quad .. +7
    bf16x8 wa[MB][NK];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int c = 0; c < NK; ++c)
            wa[mb][c] = as_bf16x8(*(const uint4 *)(wk + (size_t)(16 * mb + col) * KPAD + 32 * c + 8 * quad));
    float bias[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i) bias[mb][i] = a.bias ? a.bias[16 * mb + 4 * quad + i] : 0.0f;

    const int W = a.W, H = a.H;
    const int cstrips = (W + kConvCols - 1) / kConvCols;
    const int rgroups = (H + kConvRows * kConvSubs - 1) / (kConvRows * kConvSubs);
    int blk = (int)blockIdx.x;
    const int cs = blk % cstrips;
    blk /= cstrips;
    const int rg = blk % rgroups, b = blk / rgroups;
    const int x0 = cs * kConvCols;
    const int64_t img = (int64_t)b * H * W;
    // the image's input map through a buffer resource (32-bit offsets; a position
    // outside the image gets an offset past the map and loads zeros)
    const __amdgpu_buffer_rsrc_t rs_in = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.in + img * CINP), 0, (int)((int64_t)H * W * CINP * 2), kConvBufWord3);
    // the B fragment's k = 32 c + 8 quad .. +7 is tap (32 c + 8 quad) / CINP;
    // taps past 8 are padding (zero weights), read as zeros
    int tap_r[NK], tap_c[NK], tap_ch[NK];
    uint32_t tap_keep[NK];
#pragma unroll
    for (int c = 0; c < NK; ++c) {
        const int k8 = 32 * c + 8 * quad, tap = k8 / CINP;
        const int tc = tap < 9 ? tap : 8;
        tap_r[c] = tc / 3;
        tap_c[c] = tc % 3;
        tap_ch[c] = k8 - tap * CINP;
        tap_keep[c] = tap < 9 ? ~0u : 0u;
    }

    for (int sub = 0; sub < kConvSubs; ++sub) {
        const int y0 = (rg * kConvSubs + sub) * kConvRows;
        if (y0 >= H) break;
        __syncthreads();  // the previous sub-strip's reads of the stage are done
        const int y = y0 + wave;  // this wave's output row
        // the masked epilogue's ReLU masks of this wave's four tiles (one byte per
        // lane: the lane's 8 output channels), loaded while the stage is filled
        uint32_t mk[kConvCols / 16];
#pragma unroll
        for (int t = 0; t < kConvCols / 16; ++t) {
            mk[t] = 0;
            const int x = x0 + 16 * t + col;
            if (EPI == EPI_MASK && y < H && x < W) mk[t] = a.mask[(img + (int64_t)y * W + x) * 4 + quad];
        }
        for (int e = threadIdx.x; e < NCH; e += 256) {
            const int ch = 8 * (e % XC), pxi = e / XC, c = pxi % SC, r = pxi / SC;
            const int gy = y0 - 1 + r, gx = x0 - 1 + c;
            const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
            const u32x4c v = __builtin_amdgcn_raw_buffer_load_b128(
                rs_in, in ? (uint32_t)(((gy * W + gx) * CINP + ch) * 2) : kConvDrop, 0, 0);
            *(u32x4c *)&st[r][c][ch] = v;
        }
        __syncthreads();
        if (y >= H) continue;
#pragma unroll
        for (int t = 0; t < kConvCols / 16; ++t) {
            const int x = x0 + 16 * t + col;
            const int64_t p = img + (int64_t)y * W + x;  // this lane's pixel (B operand column)
            // the bias is the accumulators' starting value (forward epilogues), so
            // the products are summed onto it in k order
            floatx4 acc[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                acc[mb] = EPI == EPI_MASK ? floatx4{0.f, 0.f, 0.f, 0.f}
                                          : floatx4{bias[mb][0], bias[mb][1], bias[mb][2], bias[mb][3]};
#pragma unroll
            for (int c = 0; c < NK; ++c) {
                // staged row wave + ky, column 16 t + col + kx
                uint4 v = *(const uint4 *)&st[wave + tap_r[c]][16 * t + col + tap_c[c]][tap_ch[c]];
                v.x &= tap_keep[c];
                v.y &= tap_keep[c];
                v.z &= tap_keep[c];
                v.w &= tap_keep[c];
                const bf16x8 bv = as_bf16x8(v);
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mb][c], bv, acc[mb], 0, 0, 0);
            }
            if (x >= W) continue;
            uint32_t mbits = 0;
            // D layout: lane holds rows (output channels) 4*quad .. +3 of column (pixel) col
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int co = 16 * mb + 4 * quad;
                if (EPI == EPI_LINEAR) {
                    if (co == 0) {
                        float *o = (float *)a.out + p * 2;
                        o[0] = acc[mb][0];
                        o[1] = acc[mb][1];
                    }
                } else {
                    float h[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        float v = acc[mb][i];
                        if (EPI == EPI_RELU) v = relu(v);
                        else v = (mk[t] >> (4 * mb + i)) & 1u ? v : 0.0f;  // the forward output was > 0
                        h[i] = v;
                    }
                    uint2 w;
                    w.x = pack_bf16(h[0], h[1]);
                    w.y = pack_bf16(h[2], h[3]);
                    *(uint2 *)((uint16_t *)a.out + p * COUTP + co) = w;
                    if (EPI == EPI_RELU && COUTP == 32) {
                        // which of the stored values are > 0 (non-zero magnitude, sign
                        // clear), as bits 4 mb + i of the lane's mask byte
                        const uint32_t q[4] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu, w.y >> 16};
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            mbits |= ((q[i] & 0x7FFFu) != 0 && !(q[i] & 0x8000u) ? 1u : 0u) << (4 * mb + i);
                    }
                }
            }
            if (EPI == EPI_RELU && COUTP == 32 && a.mask_out) a.mask_out[p * 4 + quad] = (uint8_t)mbits;
        }
    }
}

hipError_t launch_conv(const ConvArgs &a, int cinp, int coutp, int epi, hipStream_t s)
{
    // the per-image input map is read through a buffer resource with 32-bit offsets
    if ((int64_t)a.H * a.W * cinp * 2 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const int64_t cstrips = (a.W + kConvCols - 1) / kConvCols;
    const int64_t rgroups = (a.H + kConvRows * kConvSubs - 1) / (kConvRows * kConvSubs);
    const int64_t blocks = (int64_t)a.batch * cstrips * rgroups;
    if (blocks <= 0 || blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    dim3 grid((unsigned)blocks), block(256);
#define SS_CONV(CI, CO, E)                                                                \
    if (cinp == CI && coutp == CO && epi == E) {                                          \
        hipLaunchKernelGGL((conv3x3_kernel<CI, CO, E>), grid, block, 0, s, a);            \
        return hipGetLastError();                                                         \
    }
    SS_CONV(8, 32, EPI_RELU)      // layer 1
    SS_CONV(32, 32, EPI_RELU)     // layers 2, 3
    SS_CONV(32, 16, EPI_LINEAR)   // layer 4 (2 real outputs)
    SS_CONV(32, 32, EPI_MASK)     // backward-data of layers 2, 3
    SS_CONV(16, 32, EPI_MASK)     // backward-data of layer 4 (2 real gradient channels)
#undef SS_CONV
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ weight gradient
// dW[co][k] = sum_p dY[p][co] * X[p + tap(k)][ci(k)]: a GEMM with M = COUT, N = 9*CINP
// and K = pixels, on v_mfma_f32_16x16x32_bf16 with dY transposed as the A operand
// (16 output channels x 32 pixels) and the shifted inputs as the B operand (32
// pixels x 16 k).  A block owns a 32-pixel column strip of one image over a range
// of rows and walks down it.  Per output row it takes that row's dY segment and the
// next input row (34 pixels: the strip and one column each side) with 16-byte
// loads issued one row ahead, and stores them in LDS as they are (pixel-major, a
// ring of three input rows), one 16-byte store per chunk.  The operands, which
// need 8 consecutive pixels of one channel per lane, are read with the LDS
// transpose read (ds_read_b64_tr_b16): within 16 lanes, lane 4 j + a reads
// channels 4 a .. 4 a + 3 of pixel j, and lane n receives channel n of the four
// pixels; a horizontal tap is a shift of the pixel index, so each input row is
// stored once.  The bias gradient (the sum of dY over the pixels) is taken from
// the same staged rows.  Per-block partial sums go out and are reduced in a fixed
// order, so the result does not depend on the schedule.
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
constexpr int kWgBufWord3 = 0x00020000;     // buffer resource word 3 for raw byte buffers
constexpr uint32_t kWgDrop = 0x80000000u;   // an offset past every map here: the load returns zeros

// four pixels x 16 channels from a pixel-major LDS array, transposed: lane
// 16 g + n gets channel n of the four pixels (the caller passes, for its lane
// 4 j + a of the group, the address of channels 4 a .. 4 a + 3 of pixel j)
__device__ __forceinline__ bf16x4 read_tr(const uint16_t *p)
{
    return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4 *)p);
}

template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a)
{
    constexpr int NB = (9 * CINP + 15) / 16;    // N blocks of 16 (k = tap*CINP + ci)
    constexpr int MB = COUTP / 16;
    constexpr int TILES = MB * NB;
    constexpr int TPW = (TILES + 3) / 4;        // tiles per wave
    constexpr int DYC = COUTP / 8, XC = CINP / 8;  // 16-byte chunks per pixel
    static_assert(32 * DYC <= 256 && 34 * XC <= 272, "one dY and one input chunk per thread (two for 8 threads)");
    static_assert(CINP % 4 == 0, "a transpose-read lane's four channels share one tap");
    __shared__ __align__(16) uint16_t sdy[32][COUTP];      // [px][co]
    __shared__ __align__(16) uint16_t sx[3][34][CINP];     // [ring slot][input column x0 - 1 + m][ci]
    __shared__ float sbias[256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int quad = lane >> 4;
    const int W = a.W, H = a.H;
    const int strips = (W + 31) / 32;
    int blk = (int)blockIdx.x;
    const int part_r = blk % a.rsplit;
    blk /= a.rsplit;
    const int strip = blk % strips, b = blk / strips;
    const int y0 = (int)((int64_t)H * part_r / a.rsplit), y1 = (int)((int64_t)H * (part_r + 1) / a.rsplit);
    const int x0 = 32 * strip;
    const int64_t img = (int64_t)b * H * W;

    // loader roles: dY chunk (pixel t / DYC, channels 8 (t % DYC) ..) for t < 32 DYC;
    // input chunk (pixel x0 - 1 + m, m = u / XC, channels 8 (u % XC) ..) for u = t and,
    // where 34 XC > 256, u = t + 256 for the first threads
    const int t = threadIdx.x;
    const bool dy_role = t < 32 * DYC;
    const int dpx = t / DYC, dch = 8 * (t % DYC);
    const bool dy_in = dy_role && x0 + dpx < W;
    auto x_role = [&](int u, int &m, int &ch, bool &valid_col) {
        m = u / XC;
        ch = 8 * (u % XC);
        const int gx = x0 - 1 + m;
        valid_col = u < 34 * XC && gx >= 0 && gx < W;
        return u < 34 * XC;
    };
    int m0, c0, m1, c1;
    bool v0, v1;
    const bool xr0 = x_role(t, m0, c0, v0), xr1 = x_role(t + 256, m1, c1, v1);

    // loads through buffer resources over this image's maps: a chunk outside the
    // image or the row range gets an offset past the map, whose load returns zeros
    const __amdgpu_buffer_rsrc_t rs_dy = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.dy + img * COUTP), 0, (int)((int64_t)H * W * COUTP * 2), kWgBufWord3);
    const __amdgpu_buffer_rsrc_t rs_x = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(a.x + img * CINP), 0, (int)((int64_t)H * W * CINP * 2), kWgBufWord3);
    u32x4 ndy = {0, 0, 0, 0}, nx0 = ndy, nx1 = ndy;
    auto fetch = [&](int it) {
        // this iteration's rows: input row y0 - 1 + it, dY row y0 - 2 + it
        const int xrow = y0 - 1 + it, drow = y0 - 2 + it;
        const uint32_t ody = dy_in && drow >= y0 ? (uint32_t)(((drow * W + x0 + dpx) * COUTP + dch) * 2) : kWgDrop;
        const bool row_ok = xrow >= 0 && xrow < H && xrow <= y1;
        const uint32_t ox0 = v0 && row_ok ? (uint32_t)(((xrow * W + x0 - 1 + m0) * CINP + c0) * 2) : kWgDrop;
        const uint32_t ox1 = v1 && row_ok ? (uint32_t)(((xrow * W + x0 - 1 + m1) * CINP + c1) * 2) : kWgDrop;
        ndy = __builtin_amdgcn_raw_buffer_load_b128(rs_dy, ody, 0, 0);
        nx0 = __builtin_amdgcn_raw_buffer_load_b128(rs_x, ox0, 0, 0);
        nx1 = __builtin_amdgcn_raw_buffer_load_b128(rs_x, ox1, 0, 0);
    };

    // transpose-read roles of this lane in its 16-lane group: pixel j of four,
    // channels (or k) 4 a .. 4 a + 3
    const int tj = (lane & 15) >> 2, ta = 4 * (lane & 3);

    floatx4 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = floatx4{0.f, 0.f, 0.f, 0.f};
    // bias: thread t sums dY of channel t % COUTP over pixels of group t / COUTP
    constexpr int BG = 256 / COUTP, BPX = 32 / BG;
    float bsum = 0.0f;

    const int nit = y1 - y0 + 2;
    fetch(0);
    for (int it = 0; it < nit; ++it) {
        const int xrow = y0 - 1 + it, y = y0 - 2 + it;
        __syncthreads();  // the previous iteration's reads of sdy and of this ring slot are done
        const int slot = (xrow + 3) % 3;
        if (dy_role) *(u32x4 *)&sdy[dpx][dch] = ndy;
        if (xr0) *(u32x4 *)&sx[slot][m0][c0] = nx0;
        if (xr1) *(u32x4 *)&sx[slot][m1][c1] = nx1;
        if (it + 1 < nit) fetch(it + 1);
        __syncthreads();
        if (y < y0) continue;  // ring warm-up: input rows y0 - 1 and y0
        // output row y reads input rows y-1 .. y+1: ring slots (y + 2 + ky) % 3;
        // lane group quad takes pixels 8 quad .. 8 quad + 7 (two reads of four)
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave + 4 * q;
            if (tile >= TILES) break;
            const int mb = tile % MB, nb = tile / MB;
            const int px = 8 * quad + tj;
            const bf16x4 a0 = read_tr(&sdy[px][16 * mb + ta]), a1 = read_tr(&sdy[px + 4][16 * mb + ta]);
            // k columns 16 nb + ta .. +3 share one tap (taps past 8 are padding
            // columns, whose results are not stored: any in-bounds values do)
            const int kk = 16 * nb + ta;
            const int tap = min(kk / CINP, 8), ci = kk % CINP;
            const uint16_t(*xs)[CINP] = sx[(y + 2 + tap / 3) % 3];
            const int xm = px + tap % 3;
            const bf16x4 b0 = read_tr(&xs[xm][ci]), b1 = read_tr(&xs[xm + 4][ci]);
            const bf16x8 av = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
            const bf16x8 bv = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
            acc[q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[q], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < BPX; ++i) bsum += bf2f(sdy[BPX * (t / COUTP) + i][t % COUTP]);
    }
    // partial[block][co][k]
    const int col = lane & 15;
    float *part = a.partial + (size_t)blockIdx.x * COUTP * 9 * CINP;
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave + 4 * q;
        if (tile >= TILES) break;
        const int mb = tile % MB, nb = tile / MB;
        if (16 * nb + col >= 9 * CINP) continue;
#pragma unroll
        for (int i = 0; i < 4; ++i) part[(size_t)(16 * mb + 4 * quad + i) * 9 * CINP + 16 * nb + col] = acc[q][i];
    }
    // bias partial[block][co]: the pixel groups' sums in group order
    sbias[t] = bsum;
    __syncthreads();
    if (t < COUTP) {
        float s = 0.0f;
        for (int g = 0; g < BG; ++g) s += sbias[g * COUTP + t];
        a.bpartial[(size_t)blockIdx.x * COUTP + t] = s;
    }
}

// grad[off + ((tap*CIN + ci)*COUT + co)] = sum over blocks of partial[block][co][tap*CINP + ci];
// grad[boff + co] = sum over blocks of bpartial[block][co].  A block of 1024
// threads takes 64 consecutive entries of a block's partials (so each load of a
// wave is one contiguous 256-byte run) and 16 slices of the blocks: a thread sums
// its slice in block order into four running sums (every fourth block each, for
// four independent loads in flight), adds them in a fixed order, and the 16
// slices are added in order (deterministic).  Entries of padding channels are
// skipped.
constexpr int kReduceSlices = 16;

__global__ __launch_bounds__(64 * kReduceSlices) void wgrad_reduce_kernel(WgradReduceArgs a)
{
    __shared__ float qs[kReduceSlices][64];
    const int kw = 9 * a.cinp;                       // entries per output channel
    const int nw = a.coutp * kw;                     // weight entries per block partial
    const int e = blockIdx.x * 64 + (threadIdx.x & 63), sl = threadIdx.x >> 6;
    bool real = false;
    const float *src = nullptr;
    size_t stride = 0;
    int nb = 0, out = 0;
    if (e < nw) {
        const int co = e / kw, k = e - co * kw, tap = k / a.cinp, ci = k - tap * a.cinp;
        real = co < a.cout && ci < a.cin;
        src = a.partial + e;
        stride = (size_t)nw;
        nb = a.nblocks;
        out = a.woff + (tap * a.cin + ci) * a.cout + co;
    } else if (e < nw + a.coutp) {
        const int co = e - nw;
        real = co < a.cout;
        src = a.bpartial + co;
        stride = (size_t)a.coutp;
        nb = a.nbblocks;
        out = a.boff + co;
    }
    float r = 0.0f;
    if (real) {
        const int b0 = nb * sl / kReduceSlices, b1 = nb * (sl + 1) / kReduceSlices;
        float s4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        int blk = b0;
        for (; blk + 4 <= b1; blk += 4) {
#pragma unroll
            for (int j = 0; j < 4; ++j) s4[j] += src[(size_t)(blk + j) * stride];
        }
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (blk + j < b1) s4[j] += src[(size_t)(blk + j) * stride];
        r = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    qs[sl][threadIdx.x & 63] = r;
    __syncthreads();
    if (sl == 0 && real) {
        float t = qs[0][threadIdx.x];
#pragma unroll
        for (int q = 1; q < kReduceSlices; ++q) t += qs[q][threadIdx.x];
        a.grad[out] = t;
    }
}

int wgrad_blocks(int batch, int H, int W, int max_blocks, int *rsplit)
{
    // about 1280 blocks (five rounds of 256 compute units at one block each, in
    // practice several blocks per unit), each column strip split into row ranges
    const int64_t cols = (int64_t)batch * ((W + 31) / 32);
    int64_t r = (1280 + cols - 1) / cols;
    r = std::max<int64_t>(1, std::min<int64_t>({r, (int64_t)H, max_blocks / std::max<int64_t>(cols, 1)}));
    *rsplit = (int)r;
    return (int)(cols * r);
}

hipError_t launch_wgrad(const WgradArgs &a, int cinp, int coutp, hipStream_t s)
{
    const int64_t strips = (a.W + 31) / 32;
    const int64_t blocks = (int64_t)a.batch * strips * a.rsplit;
    if (blocks <= 0 || blocks > 0x7FFFFFFF || a.rsplit < 1) return hipErrorInvalidValue;
    // the per-image maps are read through buffer resources with 32-bit offsets
    if ((int64_t)a.H * a.W * std::max(cinp, coutp) * 2 >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)blocks);
    if (cinp == 8 && coutp == 32) hipLaunchKernelGGL((wgrad_kernel<8, 32>), grid, dim3(256), 0, s, a);
    else if (cinp == 32 && coutp == 32) hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, dim3(256), 0, s, a);
    else if (cinp == 32 && coutp == 16) hipLaunchKernelGGL((wgrad_kernel<32, 16>), grid, dim3(256), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const WgradReduceArgs &a, hipStream_t s)
{
    const int n = 9 * a.cinp * a.coutp + a.coutp;
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((n + 63) / 64), dim3(64 * kReduceSlices), 0, s, a);
    return hipGetLastError();

}

// ------------------------------------------------------------------ loss
// Per pixel: L1 term |r - t| on 8-path-valid pixels, BCE-with-logits term on all
// pixels; the output gradient goes to dY (bf16, 16 channels: dr, dz, 0...).
// Per-block partial sums: [l1, valid count, bce]; the final sums are taken in a
// fixed order by loss_reduce_kernel, which also stores 1/count and 1/N used by
// the gradient pass.
__global__ __launch_bounds__(256) void count_kernel(LossArgs a)
{
    __shared__ float red[256];
    const int64_t P = a.P;
    const int64_t p0 = (P * blockIdx.x) / gridDim.x, p1 = (P * (blockIdx.x + 1)) / gridDim.x;
    float c = 0.0f;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) c += a.t_valid[p] ? 1.0f : 0.0f;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[blockIdx.x * 3 + 1] = red[0];
}

// the per-block partials j (0: L1, 1: valid count, 2: BCE) summed in a fixed order:
// thread i takes blocks i nb / 256 .. (i + 1) nb / 256 - 1 in order, then a tree
__device__ __forceinline__ float reduce_partials(const float *partial, int nblocks, int j, float *red)
{
    const int i = threadIdx.x;
    const int b0 = nblocks * i / 256, b1 = nblocks * (i + 1) / 256;
    float v = 0.0f;
    for (int b = b0; b < b1; ++b) v += partial[b * 3 + j];
    red[i] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (i < st) red[i] += red[i + st];
        __syncthreads();
    }
    return red[0];
}

__global__ __launch_bounds__(256) void count_reduce_kernel(LossArgs a, int nblocks)
{
    __shared__ float red[256];
    const float c = reduce_partials(a.partial, nblocks, 1, red);
    if (threadIdx.x == 0) {
        a.scal[0] = c;
        a.scal[1] = 1.0f / fmaxf(c, 1.0f);
        a.scal[2] = 1.0f / (float)a.P;
    }
}

__global__ __launch_bounds__(256) void loss_kernel(LossArgs a)
{
    __shared__ float r1[256], r3[256];
    const int64_t P = a.P;
    const float inv_nv = a.scal[1], inv_n = a.scal[2];
    const int64_t p0 = (P * blockIdx.x) / gridDim.x, p1 = (P * (blockIdx.x + 1)) / gridDim.x;
    float l1 = 0.0f, bce = 0.0f;
    for (int64_t p = p0 + threadIdx.x; p < p1; p += 256) {
        const float r = a.out[p * 2], z = a.out[p * 2 + 1];
        const float t = a.t_res[p];
        const float v = a.t_valid[p] ? 1.0f : 0.0f;
        const float e = r - t;
        l1 += fabsf(e) * v;
        bce += fmaxf(z, 0.0f) - z * v + log1pf(expf(-fabsf(z)));
        const float dr = (e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f)) * v * inv_nv;
        const float dz = (1.0f / (1.0f + expf(-z)) - v) * inv_n;
        uint4 w = make_uint4(pack_bf16(dr, dz), 0, 0, 0);
        uint4 *dst = (uint4 *)(a.dy + p * 16);
        dst[0] = w;
        dst[1] = make_uint4(0, 0, 0, 0);
    }
    r1[threadIdx.x] = l1;
    r3[threadIdx.x] = bce;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r3[threadIdx.x] += r3[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.partial[blockIdx.x * 3 + 0] = r1[0];
        a.partial[blockIdx.x * 3 + 2] = r3[0];
    }
}

__global__ __launch_bounds__(256) void loss_reduce_kernel(LossArgs a, int nblocks)
{
    __shared__ float red[256];
    float l1 = reduce_partials(a.partial, nblocks, 0, red);
    __syncthreads();
    float bce = reduce_partials(a.partial, nblocks, 2, red);
    if (threadIdx.x == 0) {
        l1 *= a.scal[1];
        bce *= a.scal[2];
        a.loss[0] = l1 + bce;
        a.loss[1] = l1;
        a.loss[2] = bce;
    }
}

hipError_t launch_loss(const LossArgs &a, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(count_kernel, dim3(nblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(count_reduce_kernel, dim3(1), dim3(256), 0, s, a, nblocks);
    hipLaunchKernelGGL(loss_kernel, dim3(nblocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL(loss_reduce_kernel, dim3(1), dim3(256), 0, s, a, nblocks);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Adam + weight layouts
__global__ __launch_bounds__(256) void adam_kernel(AdamArgs a)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.grad[i];
    const float m = a.b1 * a.m[i] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float mh = m / a.c1, vh = v / a.c2;
    a.p[i] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

// bf16 GEMM layouts of every layer from the fp32 master parameters:
//   forward        wf[co][tap*CINP + ci]        = W[tap][ci][co]
//   backward-data  wb[ci][tap'*COUTP' + co]     = W[8 - tap'][ci][co]   (mirrored taps)
__global__ __launch_bounds__(256) void relayout_kernel(RelayoutArgs a)
{
    const int L = blockIdx.y;
    const LayerDesc d = a.layer[L];
    const int nf = d.coutp * kpad(d.cinp);
    const int i = blockIdx.x * 256 + threadIdx.x;
    const float *W = a.params + d.woff;
    if (i < nf) {
        const int co = i / kpad(d.cinp), k = i - co * kpad(d.cinp);
        const int tap = k / d.cinp, ci = k - tap * d.cinp;
        float v = 0.0f;
        if (co < d.cout && tap < 9 && ci < d.cin) v = W[(tap * d.cin + ci) * d.cout + co];
        d.wf[i] = f2bf(v);
    }
    if (d.wb) {
        const int nb = d.cinp_b * kpad(d.coutp_b);  // rows = input channels (32), k over output channels
        if (i < nb) {
            const int ci = i / kpad(d.coutp_b), k = i - ci * kpad(d.coutp_b);
            const int tap = k / d.coutp_b, co = k - tap * d.coutp_b;
            float v = 0.0f;
            if (ci < d.cin && tap < 9 && co < d.cout) v = W[((8 - tap) * d.cin + ci) * d.cout + co];
            d.wb[i] = f2bf(v);
        }
    }
    if (i < d.coutp) d.bias[i] = i < d.cout ? a.params[d.boff + i] : 0.0f;
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3((a.n + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_relayout(const RelayoutArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(relayout_kernel, dim3((32 * 320 + 255) / 256, 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------ features / combine
// features[p] = bf16 {IR/255, S1/Smax, S2/Smax, d*/D, 0, 0, 0, 0} of a 2-path result
__global__ __launch_bounds__(256) void features_kernel(FeatureArgs a)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.P) return;
    const int64_t y = p / a.W, x = p - y * a.W;
    const uint8_t *img = a.ir;
    int pitch = a.pitch;
    if (a.job) {
        const CensusJob *j = (const CensusJob *)a.job;
        img = j->img;
        pitch = j->pitch;
    }
    const float ir = (float)img[y * pitch + x];
    const float s1 = (float)a.s1[p];
    const uint32_t s2r = a.s2[p];
    const float s2 = s2r == 0xFFFFu ? a.smax : fminf((float)s2r, a.smax);
    const float f0 = ir / 255.0f, f1 = s1 / a.smax, f2 = s2 / a.smax, f3 = (float)a.dint[p] / (float)a.max_disp;
    uint4 w;
    w.x = pack_bf16(f0, f1);
    w.y = pack_bf16(f2, f3);
    w.z = 0;
    w.w = 0;
    *(uint4 *)(a.features + p * 8) = w;
}

// masked[p] = d2_sub + r where the logit is positive and the sum is positive, else 0;
// optionally counts the pixels whose logit lies within (-tau, tau) (per block,
// then one atomic add per block: an integer count, so the result is exact)
__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a)
{
    __shared__ unsigned cnt[4];
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool unsure = false;
    if (p < a.P) {
        const float z = a.out[p * 2 + 1];
        const float d = __fadd_rn(a.d2_sub[p], a.out[p * 2]);
        const bool ok = z > 0.0f && d > 0.0f;
        a.masked[p] = ok ? d : 0.0f;
        a.flags[p] = (uint8_t)(ok ? (SIMSENSE_FLAG_UNIQUE | SIMSENSE_FLAG_LR | SIMSENSE_FLAG_NONZERO) : 0u);
        unsure = fabsf(z) < a.tau;
    }
    if (!a.uncertain) return;
    const unsigned long long ball = __ballot(unsure);
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = (unsigned)__popcll(ball);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned c = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        if (c) atomicAdd(a.uncertain, c);
    }
}

hipError_t launch_features(const FeatureArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(features_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// t_res = d8_sub - d2_sub; t_valid = the 8-path result passed uniqueness, LR and d* > 0
__global__ __launch_bounds__(256) void targets_kernel(const float *d8_sub, const uint8_t *flags8, const float *d2_sub,
                                                      float *t_res, uint8_t *t_valid, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= n) return;
    t_res[p] = __fsub_rn(d8_sub[p], d2_sub[p]);
    t_valid[p] = (flags8[p] & 7u) == 7u;
}

hipError_t launch_targets(const float *d8_sub, const uint8_t *flags8, const float *d2_sub, float *t_res,
                          uint8_t *t_valid, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d8_sub, flags8, d2_sub,
                       t_res, t_valid, n);
    return hipGetLastError();
}

hipError_t launch_combine(const CombineArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(combine_kernel, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace net
}  // namespace ss
