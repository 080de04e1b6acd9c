// IR noise model (Sec. VI-C, Eq. (7)) and census transform (Sec. VI-D).
#include "internal.h"

namespace ss {

// ---------------------------------------------------------------- IR noise
// out = clip(rint(gamma * in + n), 0, 255); product and sum are separately
// rounded fp32 operations, the integer decision is a round-half-even.
__global__ __launch_bounds__(256) void ir_noise_kernel(const uint8_t *__restrict__ in,
                                                       const float *__restrict__ gamma,
                                                       const float *__restrict__ n,
                                                       uint8_t *__restrict__ out, int64_t count)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        float v = __fadd_rn(__fmul_rn(gamma[i], (float)in[i]), n[i]);
        float r = rintf(v);
        r = r > 0.0f ? r : 0.0f;  // also maps NaN to 0
        r = r < 255.0f ? r : 255.0f;
        out[i] = (uint8_t)r;
    }
}

hipError_t launch_ir_noise(const uint8_t *in, const float *gamma, const float *n, uint8_t *out,
                           int64_t count, hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(ir_noise_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, gamma, n, out, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------- census
// A 32x8 output tile per block; the tile plus its window halo is staged in LDS
// with clamp-to-edge addressing, then each thread walks its window.  Bit k of a
// word is the k-th comparison of the window in row-major order:
//   full:               [I(p) > I(p+o)]       for every o != 0
//   center-symmetric:   [I(p+o) > I(p-o)]     for every o before the centre
constexpr int kCensusTx = 32, kCensusTy = 8;

template <typename Word>
__device__ __forceinline__ void census_tile(const uint8_t *__restrict__ img, int pitch, int W, int H, int cw, int ch,
                                            int mode, Word *__restrict__ out, int bx, int by, uint8_t *tile)
{
    const int rw = cw / 2, rh = ch / 2;
    const int tw = kCensusTx + cw - 1, th = kCensusTy + ch - 1;
    const int x0 = bx * kCensusTx - rw, y0 = by * kCensusTy - rh;
    const int tid = threadIdx.y * kCensusTx + threadIdx.x;
    for (int i = tid; i < tw * th; i += kCensusTx * kCensusTy) {
        int ty = i / tw, tx = i - ty * tw;
        int gx = min(max(x0 + tx, 0), W - 1), gy = min(max(y0 + ty, 0), H - 1);
        tile[i] = img[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int x = bx * kCensusTx + threadIdx.x, y = by * kCensusTy + threadIdx.y;
    if (x >= W || y >= H) return;
    // window centre inside the tile
    const int cx = threadIdx.x + rw, cy = threadIdx.y + rh;
    Word word = 0;
    int k = 0;
    if (mode == 0) {
        // offsets before the centre: every row above it, then the left half of its row
        for (int oy = -rh; oy <= 0; ++oy) {
            const int oxe = oy < 0 ? rw : -1;
            const uint8_t *pa = &tile[(cy + oy) * tw + cx];
            const uint8_t *pb = &tile[(cy - oy) * tw + cx];
            for (int ox = -rw; ox <= oxe; ++ox) {
                word |= (Word)(pa[ox] > pb[-ox]) << k;
                ++k;
            }
        }
    } else {
        const int c = tile[cy * tw + cx];
        for (int oy = -rh; oy <= rh; ++oy)
            for (int ox = -rw; ox <= rw; ++ox) {
                if (ox == 0 && oy == 0) continue;
                word |= (Word)(c > tile[(cy + oy) * tw + cx + ox]) << k;
                ++k;
            }
    }
    out[(size_t)y * W + x] = word;
}

// The same transform for a window size fixed at compile time (center-symmetric
// mode): the comparisons unroll with constant LDS offsets, and the word is built
// from the last comparison down, w = (w << 1) | [a > b], where [a > b] is the
// sign bit of b - a and the shift-and-insert is one v_alignbit.
template <int CW, int CH>
__device__ __forceinline__ void cs_offsets(int k, int &oy, int &ox)
{
    constexpr int rw = CW / 2, rh = CH / 2;
    if (k < rh * CW) {
        oy = -rh + k / CW;
        ox = -rw + k % CW;
    } else {
        oy = 0;
        ox = -rw + (k - rh * CW);
    }
}

template <typename Word, int CW, int CH>
__device__ __forceinline__ void census_tile_cs(const uint8_t *__restrict__ img, int pitch, int W, int H,
                                               Word *__restrict__ out, int bx, int by, uint8_t *tile)
{
    constexpr int rw = CW / 2, rh = CH / 2;
    constexpr int tw = kCensusTx + CW - 1, th = kCensusTy + CH - 1;
    constexpr int kBits = (CW * CH - 1) / 2;
    static_assert(kBits <= 8 * (int)sizeof(Word), "word too narrow");
    const int x0 = bx * kCensusTx - rw, y0 = by * kCensusTy - rh;
    const int tid = threadIdx.y * kCensusTx + threadIdx.x;
    for (int i = tid; i < tw * th; i += kCensusTx * kCensusTy) {
        const int ty = i / tw, tx = i - ty * tw;
        const int gx = min(max(x0 + tx, 0), W - 1), gy = min(max(y0 + ty, 0), H - 1);
        tile[i] = img[(size_t)gy * pitch + gx];
    }
    __syncthreads();
    const int x = bx * kCensusTx + threadIdx.x, y = by * kCensusTy + threadIdx.y;
    if (x >= W || y >= H) return;
    const uint8_t *ctr = &tile[(threadIdx.y + rh) * tw + threadIdx.x + rw];
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int k = kBits - 1; k >= 0; --k) {
        int oy, ox;
        cs_offsets<CW, CH>(k, oy, ox);
        const uint32_t d = (uint32_t)ctr[-oy * tw - ox] - (uint32_t)ctr[oy * tw + ox];  // sign = [a > b]
        if (kBits > 32) hi = __builtin_amdgcn_alignbit(hi, lo, 31);
        lo = __builtin_amdgcn_alignbit(lo, d, 31);
    }
    if constexpr (sizeof(Word) == 8) out[(size_t)y * W + x] = ((uint64_t)hi << 32) | lo;
    else out[(size_t)y * W + x] = lo;
}

// the window sizes with a compiled center-symmetric form; others (and the full
// census) take the general loop
template <typename Word>
__device__ __forceinline__ void census_any(const uint8_t *img, int pitch, int W, int H, int cw, int ch, int mode,
                                           Word *out, int bx, int by, uint8_t *tile)
{
    if (mode == 0) {
        if (cw == 7 && ch == 9) return census_tile_cs<Word, 7, 9>(img, pitch, W, H, out, bx, by, tile);
        if (cw == 9 && ch == 7) return census_tile_cs<Word, 9, 7>(img, pitch, W, H, out, bx, by, tile);
        if (cw == 5 && ch == 5) return census_tile_cs<Word, 5, 5>(img, pitch, W, H, out, bx, by, tile);
        if (cw == 7 && ch == 7) return census_tile_cs<Word, 7, 7>(img, pitch, W, H, out, bx, by, tile);
        if constexpr (sizeof(Word) == 8)
            if (cw == 9 && ch == 9) return census_tile_cs<Word, 9, 9>(img, pitch, W, H, out, bx, by, tile);
    }
    census_tile<Word>(img, pitch, W, H, cw, ch, mode, out, bx, by, tile);
}

// one launch for one or two images of the same size (blockIdx.z picks the image)
template <typename Word>
__global__ __launch_bounds__(256) void census_kernel(const uint8_t *__restrict__ img0, const uint8_t *__restrict__ img1,
                                                     int pitch, int W, int H, int cw, int ch, int mode,
                                                     Word *__restrict__ out0, Word *__restrict__ out1, unsigned *zero,
                                                     int nzero)
{
    extern __shared__ uint8_t tile[];
    const int tid = threadIdx.y * kCensusTx + threadIdx.x;
    if (blockIdx.x == 0 && blockIdx.y == 0 && blockIdx.z == 0 && tid < nzero) zero[tid] = 0u;
    const bool second = blockIdx.z != 0;
    census_any<Word>(second ? img1 : img0, pitch, W, H, cw, ch, mode, second ? out1 : out0, blockIdx.x, blockIdx.y, tile);
}

// batch form: one block per (job, 32x8 tile) item; tile = by * ceil(W/32) + bx
template <typename Word>
__global__ __launch_bounds__(256) void census_batch_kernel(CensusBatch b)
{
    extern __shared__ uint8_t tile[];
    const int tid = threadIdx.y * kCensusTx + threadIdx.x;
    if (blockIdx.x == 0 && tid < b.nzero) b.zero[tid] = 0u;
    const uint32_t it = b.items[blockIdx.x];
    const CensusJob &j = b.jobs[it >> 20];
    const int t = (int)(it & 0xFFFFFu), tx = (j.W + kCensusTx - 1) / kCensusTx;
    census_any<Word>(j.img, j.pitch, j.W, j.H, j.cw, j.ch, j.mode, (Word *)j.out, t % tx, t / tx, tile);
}

hipError_t launch_census_batch(const CensusBatch &b, bool out64, hipStream_t s)
{
    if (b.nitems == 0) return hipSuccess;
    if (b.nzero < 0 || b.nzero > kCensusTx * kCensusTy) return hipErrorInvalidValue;
    const size_t lds = (size_t)(kCensusTx + b.max_cw - 1) * (kCensusTy + b.max_ch - 1);
    if (out64)
        hipLaunchKernelGGL(census_batch_kernel<uint64_t>, dim3(b.nitems), dim3(kCensusTx, kCensusTy), lds, s, b);
    else
        hipLaunchKernelGGL(census_batch_kernel<uint32_t>, dim3(b.nitems), dim3(kCensusTx, kCensusTy), lds, s, b);
    return hipGetLastError();
}

int census_tiles(int W, int H) { return ((W + kCensusTx - 1) / kCensusTx) * ((H + kCensusTy - 1) / kCensusTy); }

hipError_t launch_census_pair(const uint8_t *img0, const uint8_t *img1, int pitch, int W, int H, int cw, int ch,
                              int mode, void *out0, void *out1, bool out64, hipStream_t s, unsigned *zero, int nzero)
{
    if (nzero < 0 || nzero > kCensusTx * kCensusTy || (nzero > 0 && !zero)) return hipErrorInvalidValue;
    dim3 grid((W + kCensusTx - 1) / kCensusTx, (H + kCensusTy - 1) / kCensusTy, img1 ? 2 : 1);
    dim3 block(kCensusTx, kCensusTy);
    size_t lds = (size_t)(kCensusTx + cw - 1) * (kCensusTy + ch - 1);
    if (out64)
        hipLaunchKernelGGL(census_kernel<uint64_t>, grid, block, lds, s, img0, img1, pitch, W, H, cw, ch, mode,
                           (uint64_t *)out0, (uint64_t *)out1, zero, nzero);
    else
        hipLaunchKernelGGL(census_kernel<uint32_t>, grid, block, lds, s, img0, img1, pitch, W, H, cw, ch, mode,
                           (uint32_t *)out0, (uint32_t *)out1, zero, nzero);
    return hipGetLastError();
}

hipError_t launch_census(const uint8_t *img, int pitch, int W, int H, int cw, int ch, int mode, void *out,
                         bool out64, hipStream_t s, unsigned *zero, int nzero)
{
    return launch_census_pair(img, nullptr, pitch, W, H, cw, ch, mode, out, nullptr, out64, s, zero, nzero);
}

}  // namespace ss
