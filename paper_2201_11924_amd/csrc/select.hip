// Disparity selection and post-processing (Sec. VI-D): winner-take-all with the
// uniqueness test, quadratic sub-pixel fit, left-right consistency check,
// 3x3 median filter and depth = f*B/d.
//
// The selection pass owns one image row per 256-thread block.  Sixteen lanes
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
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t row_min(uint32_t v)
{
    v = min(v, dpp<kRowRor8>(v));
    v = min(v, dpp<kRowRor4>(v));
    v = min(v, dpp<kRowRor2>(v));
    v = min(v, dpp<kRowRor1>(v));
    return v;
}

__device__ __forceinline__ uint32_t row_or(uint32_t v)
{
    v |= dpp<kRowRor8>(v);
    v |= dpp<kRowRor4>(v);
    v |= dpp<kRowRor2>(v);
    v |= dpp<kRowRor1>(v);
    return v;
}

// adds the dpl path-value bytes at src to S
template <int DPL>
__device__ __forceinline__ void add_bytes(const uint8_t *src, uint32_t (&S)[DPL])
{
    if constexpr (DPL % 4 == 0) {
        uint32_t w[DPL / 4];
        if constexpr (DPL == 4) {
            w[0] = *(const uint32_t *)src;
        } else if constexpr (DPL == 8) {
            uint2 v = *(const uint2 *)src;
            w[0] = v.x;
            w[1] = v.y;
        } else if constexpr (DPL == 12) {
            uint2 v = *(const uint2 *)src;
            w[0] = v.x;
            w[1] = v.y;
            w[2] = *(const uint32_t *)(src + 8);
        } else {
            uint4 v = *(const uint4 *)src;
            w[0] = v.x;
            w[1] = v.y;
            w[2] = v.z;
            w[3] = v.w;
        }
#pragma unroll
        for (int k = 0; k < DPL / 4; ++k)
#pragma unroll
            for (int b = 0; b < 4; ++b) S[4 * k + b] += (w[k] >> (8 * b)) & 0xFF;
    } else if constexpr (DPL % 2 == 0) {
#pragma unroll
        for (int k = 0; k < DPL / 2; ++k) {
            uint32_t h = *(const uint16_t *)(src + 2 * k);
            S[2 * k] += h & 0xFF;
            S[2 * k + 1] += h >> 8;
        }
    } else {
#pragma unroll
        for (int k = 0; k < DPL; ++k) S[k] += src[k];
    }
}

}  // namespace

template <int DPL>
__global__ __launch_bounds__(kBlock) void select_kernel(SelectArgs a)
{
    extern __shared__ uint32_t smem[];
    const int W = a.W, D = a.D, Dpad = a.Dpad;
    uint32_t *keyR = smem;                     // W
    float *dsub_row = (float *)(keyR + W);     // W
    uint8_t *dint_row = (uint8_t *)(dsub_row + W);  // W
    uint8_t *uniq_row = dint_row + W;          // W
    const int y = blockIdx.x;
    const size_t row = (size_t)y * W;
    for (int x = threadIdx.x; x < W; x += kBlock) keyR[x] = 0xFFFFFFFFu;
    __syncthreads();

    const int lane = threadIdx.x % kLanesPerLine, group = threadIdx.x / kLanesPerLine;
    const int d0 = lane * DPL;
    for (int x = group; x < W; x += kLinesPerBlock) {
        const size_t pix = row + x;
        uint32_t S[DPL];
#pragma unroll
        for (int j = 0; j < DPL; ++j) S[j] = 0;
        for (int r = 0; r < a.ndirs; ++r) add_bytes<DPL>(a.paths[r] + pix * Dpad + d0, S);

        uint32_t key[DPL];
        uint32_t kmin = 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int d = d0 + j;
            key[j] = d < D ? (S[j] << 8) | (uint32_t)d : 0xFFFFFFFFu;
            kmin = min(kmin, key[j]);
        }
        kmin = row_min(kmin);
        const int dstar = (int)(kmin & 0xFF);
        const uint32_t s1 = kmin >> 8;
        uint32_t s2 = 0xFFFFFFFFu, nb = 0;
#pragma unroll
        for (int j = 0; j < DPL; ++j) {
            const int d = d0 + j;
            if (d < D && (d - dstar >= 2 || dstar - d >= 2)) s2 = min(s2, S[j]);
            if (d == dstar - 1) nb |= S[j] << 16;
            if (d == dstar + 1 && d < D) nb |= S[j];
            if (d < D && x - d >= 0) atomicMin(&keyR[x - d], key[j]);
        }
        s2 = row_min(s2);
        nb = row_or(nb);
        if (lane == 0) {
            const int u = a.uniqueness_pct;
            const bool uniq = u == 0 || s2 == 0xFFFFFFFFu || 100u * s1 <= (uint32_t)(100 - u) * s2;
            float ds = (float)dstar;
            if (a.subpixel && dstar > 0 && dstar < D - 1) {
                const int am = (int)(nb >> 16) - (int)s1, bp = (int)(nb & 0xFFFF) - (int)s1;
                ds = __fadd_rn((float)dstar, __fdiv_rn((float)(am - bp), (float)(2 * (am + bp))));
            }
            a.disp_int[pix] = (uint8_t)dstar;
            a.cost_best[pix] = (uint16_t)s1;
            a.cost_second[pix] = (uint16_t)min(s2, 0xFFFFu);
            a.disp_sub[pix] = ds;
            dint_row[x] = (uint8_t)dstar;
            dsub_row[x] = ds;
            uniq_row[x] = uniq;
        }
    }
    __syncthreads();
    const int lr = a.lr_max_diff;
    for (int x = threadIdx.x; x < W; x += kBlock) {
        const int d = dint_row[x];
        const int xr = x - d;
        bool lr_ok = true;
        if (lr >= 0) lr_ok = xr >= 0 && abs(d - (int)(keyR[max(xr, 0)] & 0xFF)) <= lr;
        const bool nz = d > 0, uq = uniq_row[x] != 0;
        a.flags[row + x] = (uint8_t)(uq | (lr_ok << 1) | (nz << 2));
        a.masked[row + x] = (uq && lr_ok && nz) ? dsub_row[x] : 0.0f;
        a.disp_right[row + x] = (uint8_t)(keyR[x] & 0xFF);
    }
}

hipError_t launch_select(const SelectArgs &a, hipStream_t s)
{
    dim3 grid(a.H), block(kBlock);
    size_t lds = (size_t)a.W * 10;
    switch (a.Dpad / kLanesPerLine) {
#define SS_CASE(N) \
    case N: hipLaunchKernelGGL(select_kernel<N>, grid, block, lds, s, a); break;
        SS_CASE(1) SS_CASE(2) SS_CASE(4) SS_CASE(6) SS_CASE(8) SS_CASE(12) SS_CASE(16)
#undef SS_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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

__global__ __launch_bounds__(256) void post_kernel(PostArgs a)
{
    const int x = blockIdx.x * 64 + threadIdx.x % 64, y = blockIdx.y * 4 + threadIdx.x / 64;
    if (x >= a.W || y >= a.H) return;
    const size_t p = (size_t)y * a.W + x;
    float v = a.masked[p];
    if (a.median == 3 && x > 0 && y > 0 && x < a.W - 1 && y < a.H - 1) {
        float w[9];
        int k = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) w[k++] = a.masked[p + (ptrdiff_t)dy * a.W + dx];
        v = median9(w);
    }
    if (a.disp) a.disp[p] = v;
    if (a.flags) a.flags[p] = (uint8_t)(a.flags_in[p] | (v > 0.0f ? SIMSENSE_FLAG_VALID : 0u));
    if (a.depth) a.depth[p] = v > 0.0f ? __fdiv_rn(a.fb, v) : 0.0f;
}

hipError_t launch_post(const PostArgs &a, hipStream_t s)
{
    dim3 grid((a.W + 63) / 64, (a.H + 3) / 4), block(256);
    hipLaunchKernelGGL(post_kernel, grid, block, 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- debug volume
__global__ __launch_bounds__(256) void volume_sum_kernel(PathSet paths, int ndirs,
                                                         size_t npix, int D, int Dpad, uint16_t *out)
{
    const size_t total = npix * D;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        const size_t p = i / D, d = i - p * D;
        uint32_t s = 0;
        for (int r = 0; r < ndirs; ++r) s += paths.p[r][p * Dpad + d];
        out[i] = (uint16_t)s;
    }
}

hipError_t launch_volume_sum(const PathSet &paths, int ndirs, int W, int H, int D, int Dpad,
                             uint16_t *out, hipStream_t s)
{
    size_t total = (size_t)W * H * D;
    size_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(volume_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, paths, ndirs,
                       (size_t)W * H, D, Dpad, out);
    return hipGetLastError();
}

}  // namespace ss
