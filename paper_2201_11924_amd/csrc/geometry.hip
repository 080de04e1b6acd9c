// The steps either side of the depth path that Sec. VI-D integrates with it:
// rectification of the raw IR images (a per-pixel remap with bilinear
// interpolation) and registration of the depth map into the RGB camera (each
// valid depth pixel back-projected, moved by the IR->RGB extrinsics, projected
// and z-buffered; Table II's output is such a 1920x1080 map).
//
// Both are evaluated in float32 operation by operation, in the order the
// header documents, so the results are reproducible bit for bit.
#include <math.h>

#include "internal.h"

namespace ss {

namespace {

__global__ __launch_bounds__(256) void rectify_kernel(const uint8_t *__restrict__ in, int in_pitch, int W, int H,
                                                      const float *__restrict__ map_x, const float *__restrict__ map_y,
                                                      int out_w, int out_h, uint8_t *__restrict__ out, int out_pitch)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= out_w) return;
    const float sx = map_x[(size_t)y * out_w + x], sy = map_y[(size_t)y * out_w + x];
    float r = 0.0f;
    if (sx >= 0.0f && sy >= 0.0f && sx <= (float)(W - 1) && sy <= (float)(H - 1)) {
        const int x0 = (int)floorf(sx), y0 = (int)floorf(sy);
        const int x1 = min(x0 + 1, W - 1), y1 = min(y0 + 1, H - 1);
        const float fx = __fsub_rn(sx, (float)x0), fy = __fsub_rn(sy, (float)y0);
        const float i00 = in[(size_t)y0 * in_pitch + x0], i01 = in[(size_t)y0 * in_pitch + x1];
        const float i10 = in[(size_t)y1 * in_pitch + x0], i11 = in[(size_t)y1 * in_pitch + x1];
        const float top = __fadd_rn(i00, __fmul_rn(fx, __fsub_rn(i01, i00)));
        const float bot = __fadd_rn(i10, __fmul_rn(fx, __fsub_rn(i11, i10)));
        const float v = __fadd_rn(top, __fmul_rn(fy, __fsub_rn(bot, top)));
        r = fminf(fmaxf(rintf(v), 0.0f), 255.0f);
    }
    out[(size_t)y * out_pitch + x] = (uint8_t)r;
}

struct RegisterArgs {
    const float *depth;
    int W, H;
    simsense_camera ir, rgb;
    float rt[12];
    int out_w, out_h;
    uint32_t *out;  // float32 bits; positive floats order like their bit patterns
};

constexpr uint32_t kEmpty = 0x7F800000u;  // +inf: larger than every depth

__global__ __launch_bounds__(256) void fill_kernel(uint32_t *p, int64_t n, uint32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void register_kernel(RegisterArgs a)
{
    const int u = blockIdx.x * 256 + threadIdx.x, v = blockIdx.y;
    if (u >= a.W) return;
    const float z = a.depth[(size_t)v * a.W + u];
    if (!(z > 0.0f)) return;
    const float X = __fdiv_rn(__fmul_rn(__fsub_rn((float)u, a.ir.cx), z), a.ir.fx);
    const float Y = __fdiv_rn(__fmul_rn(__fsub_rn((float)v, a.ir.cy), z), a.ir.fy);
    float P[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float s = __fadd_rn(__fmul_rn(a.rt[3 * r + 0], X), __fmul_rn(a.rt[3 * r + 1], Y));
        P[r] = __fadd_rn(__fadd_rn(s, __fmul_rn(a.rt[3 * r + 2], z)), a.rt[9 + r]);
    }
    if (!(P[2] > 0.0f)) return;
    const float ux = __fadd_rn(__fmul_rn(a.rgb.fx, __fdiv_rn(P[0], P[2])), a.rgb.cx);
    const float uy = __fadd_rn(__fmul_rn(a.rgb.fy, __fdiv_rn(P[1], P[2])), a.rgb.cy);
    const float rx = rintf(ux), ry = rintf(uy);
    if (!(rx >= 0.0f && ry >= 0.0f && rx <= (float)(a.out_w - 1) && ry <= (float)(a.out_h - 1))) return;
    atomicMin(&a.out[(size_t)ry * a.out_w + (size_t)rx], __float_as_uint(P[2]));
}

__global__ __launch_bounds__(256) void finalize_kernel(uint32_t *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n && p[i] == kEmpty) p[i] = 0u;
}

}  // namespace

}  // namespace ss

using namespace ss;

extern "C" {

int simsense_rectify(const uint8_t *in, int32_t in_pitch, int32_t in_w, int32_t in_h, const float *map_x,
                     const float *map_y, int32_t out_w, int32_t out_h, uint8_t *out, int32_t out_pitch, void *stream)
{
    if (!in || !map_x || !map_y || !out) return SIMSENSE_ERR_NULL_POINTER;
    if (in_w < 1 || in_h < 1 || out_w < 1 || out_h < 1 || in_w > 65536 || in_h > 65536 || out_w > 65536 ||
        out_h > 65536 || in_pitch < in_w || out_pitch < out_w)
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    dim3 grid((out_w + 255) / 256, out_h), block(256);
    hipLaunchKernelGGL(rectify_kernel, grid, block, 0, (hipStream_t)stream, in, in_pitch, in_w, in_h, map_x, map_y,
                       out_w, out_h, out, out_pitch);
    return hipGetLastError() == hipSuccess ? SIMSENSE_OK : SIMSENSE_ERR_DEVICE;
}

int simsense_register_depth(const float *depth, int32_t width, int32_t height, const simsense_camera *ir,
                            const float *rt, const simsense_camera *rgb, int32_t out_w, int32_t out_h, float *out,
                            void *stream)
{
    if (!depth || !ir || !rt || !rgb || !out) return SIMSENSE_ERR_NULL_POINTER;
    if (width < 1 || height < 1 || out_w < 1 || out_h < 1 || width > 65536 || height > 65536 || out_w > 65536 ||
        out_h > 65536)
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (!(ir->fx != 0.0f) || !(ir->fy != 0.0f)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    RegisterArgs a{};
    a.depth = depth;
    a.W = width; a.H = height;
    a.ir = *ir; a.rgb = *rgb;
    for (int i = 0; i < 12; ++i) a.rt[i] = rt[i];
    a.out_w = out_w; a.out_h = out_h;
    a.out = (uint32_t *)out;
    const int64_t n = (int64_t)out_w * out_h;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(fill_kernel, dim3(nb), dim3(256), 0, s, a.out, n, kEmpty);
    hipLaunchKernelGGL(register_kernel, dim3((width + 255) / 256, height), dim3(256), 0, s, a);
    hipLaunchKernelGGL(finalize_kernel, dim3(nb), dim3(256), 0, s, a.out, n);
    return hipGetLastError() == hipSuccess ? SIMSENSE_OK : SIMSENSE_ERR_DEVICE;
}

}  // extern "C"
