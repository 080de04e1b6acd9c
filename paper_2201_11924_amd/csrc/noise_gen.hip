// On-device IR noise for simulated cameras (Sec. VI-C): the multiplicative
// speckle gamma and the additive thermal noise n of Eq. (7), drawn on the GPU
// (Eq. (8) and the fit of Sec. VII-C give the distributions; Table X's noise
// scale s maps gamma -> 1 + s (gamma - 1) and n -> s n), then applied to the
// clean image in the same pass, so a rendered IR pair goes to the census with
// no host round trip.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11), counter (pixel, stream,
// attempt, 0), key (seed low, seed high); uniforms from the top 23 bits,
// ((x >> 9) + 0.5) 2^-23; normals by Box-Muller and the gamma by the method of
// Marsaglia and Tsang (2000), both in double precision and rounded to float32.
#include <math.h>

#include "internal.h"

namespace ss {

namespace {

struct Philox {
    static __device__ __forceinline__ void round(uint32_t (&c)[4], uint32_t k0, uint32_t k1)
    {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    static __device__ __forceinline__ void draw(uint32_t (&c)[4], uint32_t k0, uint32_t k1)
    {
#pragma unroll
        for (int r = 0; r < 10; ++r) {
            if (r > 0) {
                k0 += 0x9E3779B9u;
                k1 += 0xBB67AE85u;
            }
            round(c, k0, k1);
        }
    }
};

__device__ __forceinline__ double u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

__device__ __forceinline__ double box_muller(uint32_t a, uint32_t b)
{
    const double kTwoPi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(u01(a))) * cos(kTwoPi * u01(b));
}

struct NoiseArgs {
    int gain_model;
    float k, theta, gain_sd, mu, sigma, scale;
    uint32_t key0, key1, stream;
};

// gamma' and n' of pixel i
__device__ __forceinline__ void draws(const NoiseArgs &a, uint32_t i, float &gamma, float &n)
{
    double g = 1.0;
    if (a.gain_model == 1) {
        const double d = (double)a.k - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
        g = d * (double)a.theta;
        for (uint32_t att = 0; att < 64; ++att) {
            uint32_t w[4] = {i, a.stream, att, 0u};
            Philox::draw(w, a.key0, a.key1);
            const double x = box_muller(w[0], w[1]);
            double v = 1.0 + c * x;
            if (v <= 0.0) continue;
            v = v * v * v;
            if (log(u01(w[2])) < 0.5 * x * x + d - d * v + d * log(v)) {
                g = d * v * (double)a.theta;
                break;
            }
        }
    } else if (a.gain_model == 2) {
        uint32_t w[4] = {i, a.stream, 0u, 0u};
        Philox::draw(w, a.key0, a.key1);
        g = 1.0 + (double)a.gain_sd * box_muller(w[0], w[1]);
    }
    uint32_t w[4] = {i, a.stream, 0xFFFFFFFFu, 0u};
    Philox::draw(w, a.key0, a.key1);
    const float nz = (float)((double)a.mu + (double)a.sigma * box_muller(w[0], w[1]));
    const float gf = (float)g;
    gamma = __fadd_rn(1.0f, __fmul_rn(a.scale, __fsub_rn(gf, 1.0f)));
    n = __fmul_rn(a.scale, nz);
}

__global__ __launch_bounds__(256) void noise_draws_kernel(NoiseArgs a, int64_t count, float *gamma, float *n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    float g, z;
    draws(a, (uint32_t)i, g, z);
    gamma[i] = g;
    n[i] = z;
}

// Eq. (7) with this pixel's draws: product and sum each rounded to float32,
// rounded to the nearest integer (ties to even) and clipped to [0, 255]
__global__ __launch_bounds__(256) void noise_apply_kernel(NoiseArgs a, const uint8_t *in, int in_pitch, int W, int H,
                                                          uint8_t *out, int out_pitch)
{
    const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
    if (x >= W) return;
    float g, z;
    draws(a, (uint32_t)((int64_t)y * W + x), g, z);
    const float prod = __fmul_rn(g, (float)in[(size_t)y * in_pitch + x]);
    float r = rintf(__fadd_rn(prod, z));
    r = r > 0.0f ? r : 0.0f;
    r = r < 255.0f ? r : 255.0f;
    out[(size_t)y * out_pitch + x] = (uint8_t)r;
}

NoiseArgs noise_args(const simsense_noise_params &p)
{
    NoiseArgs a{};
    a.gain_model = p.gain_model;
    a.k = p.k; a.theta = p.theta; a.gain_sd = p.gain_sd; a.mu = p.mu; a.sigma = p.sigma; a.scale = p.scale;
    a.key0 = (uint32_t)p.seed;
    a.key1 = (uint32_t)(p.seed >> 32);
    a.stream = p.stream;
    return a;
}

int validate_noise(const simsense_noise_params *p)
{
    if (!p) return SIMSENSE_ERR_NULL_POINTER;
    if (p->struct_size != sizeof(simsense_noise_params)) return SIMSENSE_ERR_ABI;
    if (p->gain_model < 0 || p->gain_model > 2) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p->gain_model == 1 && !(p->k >= 1.0f && p->theta > 0.0f)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (!(p->gain_sd >= 0.0f) || !(p->sigma >= 0.0f) || !(p->scale >= 0.0f) || !(p->mu == p->mu))
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    return SIMSENSE_OK;
}

}  // namespace

}  // namespace ss

using namespace ss;

extern "C" {

int simsense_noise_draws(const simsense_noise_params *params, int64_t count, float *gamma, float *n, void *stream)
{
    int rc = validate_noise(params);
    if (rc != SIMSENSE_OK) return rc;
    if (count < 0 || count > ((int64_t)1 << 32)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (count == 0) return SIMSENSE_OK;
    if (!gamma || !n) return SIMSENSE_ERR_NULL_POINTER;
    hipLaunchKernelGGL(noise_draws_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                       noise_args(*params), count, gamma, n);
    if (hipGetLastError() != hipSuccess) return SIMSENSE_ERR_DEVICE;
    return SIMSENSE_OK;
}

int simsense_ir_noise_generate(const simsense_noise_params *params, const uint8_t *in, int32_t in_pitch,
                               int32_t width, int32_t height, uint8_t *out, int32_t out_pitch, void *stream)
{
    int rc = validate_noise(params);
    if (rc != SIMSENSE_OK) return rc;
    if (width < 1 || height < 1 || width > 65536 || height > 65536) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (in_pitch < width || out_pitch < width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (!in || !out) return SIMSENSE_ERR_NULL_POINTER;
    dim3 grid((width + 255) / 256, height), block(256);
    hipLaunchKernelGGL(noise_apply_kernel, grid, block, 0, (hipStream_t)stream, noise_args(*params), in, in_pitch,
                       width, height, out, out_pitch);
    if (hipGetLastError() != hipSuccess) return SIMSENSE_ERR_DEVICE;
    return SIMSENSE_OK;
}

}  // extern "C"
