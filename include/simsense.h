/*
 * simsense.h - C ABI of the MI355X (gfx950) depth-from-active-stereo library.
 *
 * The library computes the depth stage of the active stereo sensor simulator of
 * "Close the Optical Sensing Domain Gap by Physics-Grounded Active Stereo Sensor
 * Simulation" (Sec. VI-C and VI-D): an IR stereo pair, rectified and with the
 * IR noise model applied, goes through a census transform, a Hamming matching
 * cost, semi-global path aggregation with penalties P1/P2, winner-take-all
 * disparity with a uniqueness test, quadratic sub-pixel refinement, a
 * left-right consistency check and a median filter, and is converted to depth
 * by depth = f * B / d.
 *
 * Conventions shared by every entry point:
 *  - Every image, map and buffer argument is a DEVICE pointer owned by the
 *    caller (for example the storage of a torch tensor) unless stated
 *    otherwise.  Images are row-major; `pitch` is the row stride in elements.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Work is enqueued asynchronously on it; no entry point synchronises.
 *  - Return value: SIMSENSE_OK (0) or a negative simsense_status.  Argument
 *    errors are detected on the host before anything is enqueued; device
 *    errors surface as SIMSENSE_ERR_DEVICE from the call that observes them.
 *  - A handle may be used by one stream at a time; distinct handles are
 *    independent and may run concurrently on different streams.
 */
#ifndef SIMSENSE_H
#define SIMSENSE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum simsense_status {
    SIMSENSE_OK = 0,
    SIMSENSE_ERR_INVALID_ARGUMENT = -1, /* a parameter is out of its documented range */
    SIMSENSE_ERR_NULL_POINTER = -2,     /* a required pointer is NULL */
    SIMSENSE_ERR_OUT_OF_MEMORY = -3,    /* device allocation failed */
    SIMSENSE_ERR_DEVICE = -4,           /* a HIP runtime call or kernel launch failed */
    SIMSENSE_ERR_UNSUPPORTED = -5,      /* valid but not supported by this build */
    SIMSENSE_ERR_ABI = -6,              /* struct_size does not match this library */
    SIMSENSE_ERR_TOO_LARGE = -7         /* the parameters need more scratch than
                                           simsense_compute_noalloc's static buffer holds */
} simsense_status;

/*
 * Parameters of the depth path.  The paper states the module's key parameters
 * are adjustable (Sec. VI-D) and sweeps the maximum disparity (Table II).
 *
 *  struct_size      sizeof(simsense_params); checked for ABI compatibility.
 *  width, height    image size in pixels, 1..8192 each.
 *  max_disp         D: disparities 0..D-1 are searched, 1 <= D <= 256 (Table II "Max Disparity").
 *  census_w/_h      census window, odd, window columns x rows (default 7 x 9).
 *  census_mode      0 = center-symmetric census (the paper's choice, Sec. VI-D;
 *                   (w*h-1)/2 bits), 1 = full census (w*h-1 bits); at most 64 bits.
 *  p1, p2           SGM penalties for a disparity change of 1 and of more than 1;
 *                   0 <= p1 <= p2 and bits + p2 <= 255 (path values are stored in 8 bits;
 *                   see block_w for the SGBM bound).
 *  uniqueness_pct   u in 0..99: a pixel is kept only if 100*S1 <= (100-u)*S2, S2 being
 *                   the best aggregated cost at least two disparities away; 0 disables.
 *  lr_max_diff      left-right check tolerance in pixels; negative disables.
 *  num_paths        2 (horizontal), 4 (+ vertical) or 8 (+ diagonals).
 *  median           0 (off) or 3 (3x3 median of the masked disparity map).
 *  subpixel         0 or 1 (quadratic fit through d*-1, d*, d*+1).
 *  focal_px         focal length in pixels; baseline_m  stereo baseline (depth is in its unit).
 *  lr_mode          right-image disparity of the left-right check (Sec. VI-D names the check,
 *                   not how the right disparity is found): 0 = read off the left-referenced
 *                   volume, dR(xr) = argmin_d S(xr+d, d); 1 = a full right-referenced SGM run
 *                   (cost of right pixel xr against left pixel xr+d, the same paths and
 *                   penalties), which doubles the matching work.  Batches support 0 only.
 *  block_w/_h       matching block, odd, 1..31 each.  1 x 1 is SGM: the cost of a pixel pair
 *                   is their census Hamming distance.  Larger blocks give semi-global block
 *                   matching (SGBM, Sec. VI-D: the Hamming distance between the pixels' local
 *                   regions): the Hamming costs summed over the block centred on the pixel,
 *                   block samples outside the image clamped to the edge.  SGBM keeps 16-bit
 *                   path values and requires bits * block_w * block_h + p2 <= 8191; it runs
 *                   the aggregation with one block per line block (the tuning is not used),
 *                   and is not available to batches or the learned path.
 */
typedef struct simsense_params {
    uint32_t struct_size;
    int32_t width, height, max_disp;
    int32_t census_w, census_h, census_mode;
    int32_t p1, p2;
    int32_t uniqueness_pct, lr_max_diff;
    int32_t num_paths, median, subpixel;
    float focal_px, baseline_m;
    int32_t lr_mode;
    int32_t block_w, block_h;
} simsense_params;

/* Bits of the per-pixel flag byte written by the compute calls. */
#define SIMSENSE_FLAG_UNIQUE 1u  /* passed the uniqueness test */
#define SIMSENSE_FLAG_LR 2u      /* passed the left-right check */
#define SIMSENSE_FLAG_NONZERO 4u /* integer disparity > 0 (finite depth) */
#define SIMSENSE_FLAG_VALID 8u   /* final output disparity > 0 (after the median) */

typedef struct simsense_handle simsense_handle; /* opaque */

/* Optional outputs of simsense_compute_ex; every pointer may be NULL.
 * Layouts are row-major width x height with pitch = width unless noted. */
typedef struct simsense_outputs {
    float *depth;        /* fp32 depth, 0 where invalid */
    float *disp;         /* fp32 final disparity (masked, median-filtered), 0 where invalid */
    uint8_t *flags;      /* SIMSENSE_FLAG_* bits */
    uint8_t *disp_int;   /* integer winner d* */
    uint16_t *cost_best; /* S1 = S(d*) */
    uint16_t *cost_second; /* S2, 0xFFFF when no disparity is two or more away from d* */
    uint8_t *disp_right; /* right-image integer disparity used by the LR check */
    float *disp_sub;     /* fp32 sub-pixel disparity before masking and median */
    uint64_t *census_left, *census_right; /* census words, bit k = k-th window comparison */
    uint16_t *volume;    /* summed path costs S, width*height*max_disp, d fastest */
    uint16_t *features;  /* input of the learned surrogate: bf16, 8 channels per pixel (pixel-major):
                            IR / 255, S1 / Smax, S2 / Smax (1 where no S2), d* / D, then 4 zeros;
                            Smax = num_paths * (census bits + p2) */
} simsense_outputs;

/* Allocates a handle and its device scratch for one parameter set on the
 * current HIP device.  Validates every field; *out is set only on success. */
int simsense_create(const simsense_params *params, simsense_handle **out);

/* Releases the handle and its scratch; waits for work queued on the handle's
 * last stream first.  NULL is accepted. */
int simsense_destroy(simsense_handle *h);

/* Runs the whole depth path of Sec. VI-D on one rectified, noise-applied uint8
 * pair (`left`, `right`, pitch >= width bytes).  Writes `depth` (required) and,
 * when non-NULL, `disp` and `flags`. */
int simsense_compute(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch,
                     float *depth, float *disp, uint8_t *flags, void *stream);

/* As simsense_compute, with every intermediate result of the path available. */
int simsense_compute_ex(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch,
                        const simsense_outputs *out, void *stream);

/* IR noise model, Sec. VI-C Eq. (7): out = clip(rint(gamma * in + n), 0, 255) per
 * pixel, with the product and the sum each rounded to fp32 (no fused
 * multiply-add) and ties rounded to even.  `gamma` (the speckle gain, Eq. (8))
 * and `n` (the thermal term) are the caller's fp32 draws, `count` elements. */
int simsense_ir_noise(const uint8_t *in, const float *gamma, const float *n, uint8_t *out,
                      int64_t count, void *stream);

/* On-device IR noise for simulated cameras (Sec. VI-C: I' = gamma * I + n, Eq. (7);
 * Eq. (8) and the D415 fit of Sec. VII-C give the distributions, Table X the noise
 * scale).  Draws come from Philox4x32-10 (Salmon et al., SC'11) with counter
 * (pixel index y*width+x, stream, attempt, 0) and key (seed low, seed high), so
 * they depend only on (seed, stream, pixel).
 *  gain_model  0: gamma = 1; 1: gamma ~ Gamma(k, theta), k >= 1, by the method of
 *              Marsaglia and Tsang (at most 64 attempts, then the mode-free value
 *              (k - 1/3) theta); 2: gamma ~ Normal(1, gain_sd^2).
 *  mu, sigma   n ~ Normal(mu, sigma^2) in DN (Box-Muller).
 *  scale       s >= 0: gamma' = 1 + s (gamma - 1), n' = s n (1 = the fitted noise).
 * Uniforms are ((x >> 9) + 0.5) 2^-23; normals and gammas are computed in double
 * and rounded to float32; gamma' and n' are formed in float32. */
typedef struct simsense_noise_params {
    uint32_t struct_size;
    int32_t gain_model;
    float k, theta, gain_sd;
    float mu, sigma;
    float scale;
    uint64_t seed;
    uint32_t stream;
} simsense_noise_params;

/* gamma' and n' of pixels 0..count-1 (device float arrays; count <= 2^32). */
int simsense_noise_draws(const simsense_noise_params *params, int64_t count, float *gamma, float *n, void *stream);

/* Draws and applies the noise in one pass: out = clip(rint(gamma' * in + n')), the
 * product and the sum each rounded to float32, ties to even, clipped to [0, 255]
 * (the arithmetic of simsense_ir_noise).  Images are device uint8, row pitches in
 * bytes (>= width); width, height <= 65536.  Asynchronous on `stream`. */
int simsense_ir_noise_generate(const simsense_noise_params *params, const uint8_t *in, int32_t in_pitch,
                               int32_t width, int32_t height, uint8_t *out, int32_t out_pitch, void *stream);

/* The steps either side of the matching that Sec. VI-D integrates with it.
 *
 * Rectification: out(x, y) = bilinear sample of `in` at (map_x(x,y), map_y(x,y)),
 * the per-pixel source coordinates a calibration tool produces (device float32,
 * out_w x out_h, pitch out_w); sources outside [0, in_w-1] x [0, in_h-1] give 0.
 * Evaluated in float32 as top = i00 + fx (i01 - i00), bottom likewise, then
 * top + fy (bottom - top), every operation rounded, then rounded to the nearest
 * integer (ties to even) and clipped to [0, 255].  Images are device uint8 with
 * row pitches in bytes. */
int simsense_rectify(const uint8_t *in, int32_t in_pitch, int32_t in_w, int32_t in_h, const float *map_x,
                     const float *map_y, int32_t out_w, int32_t out_h, uint8_t *out, int32_t out_pitch, void *stream);

/* Pinhole intrinsics in pixels. */
typedef struct simsense_camera {
    float fx, fy, cx, cy;
} simsense_camera;

/* Depth registration into the RGB camera.  Every pixel (u, v) of `depth` (device
 * float32, width x height, pitch width; the rectified left IR camera) with z > 0 is
 * back-projected, X = (u-cx) z / fx, Y = (v-cy) z / fy, Z = z, moved by `rt` (host,
 * 12 floats: R row-major then t; X' = R X + t with each row summed left to right),
 * dropped if Z' <= 0, projected with `rgb`, rounded to the nearest pixel (ties to
 * even) and z-buffered: out (device float32, out_w x out_h) holds the smallest Z'
 * per pixel, 0 where no point lands.  All float32, operation by operation. */
int simsense_register_depth(const float *depth, int32_t width, int32_t height, const simsense_camera *ir,
                            const float *rt, const simsense_camera *rgb, int32_t out_w, int32_t out_h, float *out,
                            void *stream);

/* Census transform alone (Sec. VI-D): one uint64 word per pixel, bit k = k-th
 * comparison of the window enumerated row-major from its top-left corner;
 * samples outside the image clamp to the edge.  Uses width, height and the
 * census fields of `params`. */
int simsense_census(const simsense_params *params, const uint8_t *img, int32_t pitch, uint64_t *out,
                    void *stream);

/* Per-pass device timing.  While enabled, every compute call on `h` records a
 * HIP event pair around each of its passes on the call's stream (census,
 * aggregation, selection, post-processing).  simsense_profile_read waits for
 * the recorded events, writes the accumulated milliseconds of pass i to ms[i]
 * and the number of timed calls to *calls (both for at most n passes), and
 * resets the accumulators.  Events are created by the enable call.  With
 * lr_mode 1 the aggregation pass times the left-referenced aggregation and the
 * selection pass everything after it (left selection, the right-referenced
 * aggregation and selection, and the check). */
#define SIMSENSE_PASS_CENSUS 0
#define SIMSENSE_PASS_AGGREGATE 1
#define SIMSENSE_PASS_SELECT 2
#define SIMSENSE_PASS_POST 3
#define SIMSENSE_NUM_PASSES 4
int simsense_profile_enable(simsense_handle *h, int enable);
int simsense_profile_read(simsense_handle *h, double *ms, int32_t *calls, int32_t n);

/* ------------------------------------------------------------------------
 * Learned surrogate (a project addition, not in the paper): a 4-layer 3x3
 * convolutional net, 4 -> 32 -> 32 -> 32 -> 2 channels with ReLU after the first
 * three and zero padding, BF16 weights and activations with FP32 accumulation,
 * that reads the features of a 2-path (horizontal) SGM result (see
 * simsense_outputs.features) and predicts a disparity residual (channel 0) and a
 * validity logit (channel 1).  It stands in for the six non-horizontal paths of
 * the paper's aggregation (Sec. VI-D); 8-path SGM stays the reference.
 *
 * Parameters are a flat fp32 vector of simsense_net_num_params() values, layer
 * by layer: weights [ky][kx][ci][co] (out(y,x) += in(y+ky-1, x+kx-1, ci) * w),
 * then biases [co].  Training minimises the mean absolute residual error over
 * pixels where the 8-path result is valid plus the mean binary cross-entropy
 * of the logit against that validity, with Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * ---------------------------------------------------------------------- */
typedef struct simsense_net simsense_net; /* opaque */

int64_t simsense_net_num_params(void);

/* Allocates a net for up to `max_pixels` = batch * height * width pixels per call
 * (about 450 bytes of device memory per pixel) with He-uniform weights drawn from
 * `seed` and zero biases; Adam state zero.  Synchronous. */
int simsense_net_create(int64_t max_pixels, uint64_t seed, simsense_net **out);
int simsense_net_destroy(simsense_net *net);

/* HOST buffers of `count` = simsense_net_num_params() floats.  get waits for the
 * net's last stream; NULL buffers are skipped.  set copies parameters (and Adam
 * moments, zero when NULL) and the step counter, then rebuilds the bf16 layouts;
 * synchronous.  Together they checkpoint and resume training exactly. */
int simsense_net_get_state(simsense_net *net, float *params, float *m, float *v, int64_t count, int64_t *step);
int simsense_net_set_state(simsense_net *net, const float *params, const float *m, const float *v,
                           int64_t count, int64_t step);
/* HOST buffer: the gradient computed by the last training step. */
int simsense_net_get_grads(simsense_net *net, float *grads, int64_t count);
/* Tensors the last simsense_net_forward or simsense_net_train_step left in the
 * net, copied to a HOST buffer of exactly `bytes` (waits for the net's last
 * stream); for checking the layers one by one.  P = batch * height * width of
 * that call, NHWC pixel order:
 *   SIMSENSE_NET_ACTIVATION, layer 0..2: bf16 [P][32], layer l's output after its
 *     ReLU (the input of layer l + 1);
 *   SIMSENSE_NET_OUTPUT, layer 3: fp32 [P][2], residual and logit;
 *   SIMSENSE_NET_OUTPUT_GRAD (training step only), layer 3: bf16 [P][16], the loss
 *     gradient at the net output in channels 0 and 1 (the rest 0); layer 0..2:
 *     bf16 [P][32], the gradient at layer l's pre-activation output (the
 *     backward-data result times the ReLU derivative).
 * Returns SIMSENSE_ERR_INVALID_ARGUMENT for another (what, layer) or size. */
#define SIMSENSE_NET_ACTIVATION 0
#define SIMSENSE_NET_OUTPUT 1
#define SIMSENSE_NET_OUTPUT_GRAD 2
int simsense_net_read_tensor(simsense_net *net, int32_t what, int32_t layer, void *host, int64_t bytes);

/* Forward pass.  `features`: bf16 [batch][height][width][8] (device); `out`: fp32
 * [batch][height][width][2] (device): residual, logit. */
int simsense_net_forward(simsense_net *net, const uint16_t *features, int32_t batch, int32_t height,
                         int32_t width, float *out, void *stream);

/* Fused inference for the learned depth path: the four convolutions and the
 * combination with the 2-path disparity in one kernel, with no activation
 * written to memory; it allocates nothing and needs no max_pixels room.
 * `features`: bf16 [batch][height][width][8] (device).  `out` (device,
 * nullable): fp32 [batch][height][width][2], equal bit for bit to
 * simsense_net_forward's.  `d2_sub`, `masked`, `flags` (device, all NULL or all
 * set, [batch][height][width]): masked = d2_sub + residual where the logit and
 * that sum are both positive, else 0; flags = 7 (unique, LR, nonzero) there,
 * else 0.  `uncertain` (device, nullable, [batch]): the number of pixels whose
 * logit lies within (-tau, tau) is ADDED to each image's counter. */
int simsense_net_infer(simsense_net *net, const uint16_t *features, int32_t batch, int32_t height, int32_t width,
                       const float *d2_sub, float *out, float *masked, uint8_t *flags, float tau,
                       unsigned *uncertain, void *stream);

/* One Adam step on a batch.  `target_residual` fp32 and `target_valid` uint8 (0/1)
 * are [batch][height][width] (device).  `loss` (device, nullable) receives
 * {total, l1, bce} of the forward pass before the update. */
int simsense_net_train_step(simsense_net *net, const uint16_t *features, const float *target_residual,
                            const uint8_t *target_valid, int32_t batch, int32_t height, int32_t width,
                            float lr, float *loss, void *stream);

/* Training targets from an 8-path and a 2-path result of the same pair (device,
 * `count` pixels): target_residual = d8_sub - d2_sub, target_valid = 1 where the
 * 8-path flags have the uniqueness, LR and nonzero bits. */
int simsense_net_targets(const float *d8_sub, const uint8_t *flags8, const float *d2_sub, float *target_residual,
                         uint8_t *target_valid, int64_t count, void *stream);

/* The learned depth path: matching with the handle's parameters (normally
 * num_paths = 2), features, the net, then disparity = d2_sub + residual where the
 * logit is positive and the sum is positive (else invalid), then the handle's
 * median and depth.  Writes the outputs requested in `out` that this path
 * produces: depth, disp, flags, disp_sub (the 2-path sub-pixel map), disp_int,
 * features.  width * height must not exceed the net's max_pixels. */
int simsense_learned_compute(simsense_handle *h, simsense_net *net, const uint8_t *left, const uint8_t *right,
                             int32_t pitch, const simsense_outputs *out, void *stream);

/* ------------------------------------------------------------------------
 * Batches (a project addition): many pairs of uneven sizes and disparity
 * ranges, as from many simulated cameras, computed by one graph launch.  Each
 * pass of the path runs once over every pair; the aggregation pass is a
 * persistent kernel that takes line blocks of all pairs from a queue, longest
 * first.  The batch owns per-pair scratch like a handle (simsense_scratch_bytes
 * of each pair's parameters).
 * ---------------------------------------------------------------------- */
typedef struct simsense_batch simsense_batch; /* opaque */

/* One pair of a batch call: device pointers owned by the caller. */
typedef struct simsense_pair {
    const uint8_t *left, *right; /* rectified, noise-applied IR images */
    int32_t pitch;               /* row stride in bytes, >= width */
    float *depth;                /* required */
    float *disp;                 /* nullable */
    uint8_t *flags;              /* nullable */
} simsense_pair;

/* Launch shape of the batch kernels.
 *  horizontal_lanes  lanes that hold one horizontal scanline's disparity vector:
 *                    16, 32 or 64 (a quarter, half or whole wavefront), 0 = the
 *                    default for each disparity range; pairs whose padded
 *                    disparity count it does not divide keep their default.
 *  blocks_per_cu     resident blocks per compute unit of the persistent
 *                    aggregation kernel, 1..8. */
typedef struct simsense_batch_tuning {
    uint32_t struct_size;
    int32_t horizontal_lanes;
    int32_t blocks_per_cu;
} simsense_batch_tuning;

/* `params`: host array of n parameter sets (1 <= n <= 2048), one per pair slot;
 * all must use the same census word width (<= 32 bits or > 32 bits). */
int simsense_batch_create(const simsense_params *params, int32_t n, simsense_batch **out);
int simsense_batch_destroy(simsense_batch *b);
int64_t simsense_batch_scratch_bytes(const simsense_batch *b);
/* `pairs`: host array of n entries, read during the call.  Asynchronous on `stream`. */
int simsense_batch_compute(simsense_batch *b, const simsense_pair *pairs, void *stream);
/* The learned form on a batch of equal-sized pairs (normally num_paths = 2): the
 * batch's matching, then the net on chunks of as many pairs as the net's
 * max_pixels allows, then disparity = d2_sub + residual where the logit is
 * positive, then median and depth, all in one graph launch.  `uncertain`
 * (device, n counters) receives per pair the number of pixels whose logit lies
 * within (-tau, tau); a caller falls back to plain SGM for pairs where it is
 * large.  The graph is kept for one (net, tau, uncertain) triple. */
int simsense_batch_learned_compute(simsense_batch *b, simsense_net *net, const simsense_pair *pairs, float tau,
                                   unsigned *uncertain, void *stream);
/* The learned form with plain SGM as its fallback: simsense_batch_learned_compute
 * on every pair, then for each pair that falls back, simsense_compute with the
 * `plain` handle (normally the same parameters with num_paths = 8) on the same
 * images, writing the pair's own depth / disp / flags over the learned result.
 * `plain` must have the slots' width, height and max_disp (it may be NULL with
 * mode NEVER).  Modes:
 *   SIMSENSE_FALLBACK_THRESHOLD  pairs whose count of pixels with a logit within
 *                                (-tau, tau) exceeds max_uncertain_frac (0..1) of
 *                                their pixels; the counts are copied to the host,
 *                                so the call waits once for the learned pass;
 *   SIMSENSE_FALLBACK_NEVER      none (the learned result stands; no wait);
 *   SIMSENSE_FALLBACK_ALWAYS     every pair (no wait).
 * `fell_back` (host, nullable, n entries) receives 1 for pairs recomputed, else 0.
 * The plain runs are enqueued on `stream` after the learned pass. */
#define SIMSENSE_FALLBACK_THRESHOLD 0
#define SIMSENSE_FALLBACK_NEVER 1
#define SIMSENSE_FALLBACK_ALWAYS 2
int simsense_batch_learned_fallback(simsense_batch *b, simsense_net *net, simsense_handle *plain,
                                    const simsense_pair *pairs, float tau, unsigned *uncertain, int32_t mode,
                                    float max_uncertain_frac, int32_t *fell_back, void *stream);
int simsense_batch_set_tuning(simsense_batch *b, const simsense_batch_tuning *t);
int simsense_batch_get_tuning(const simsense_batch *b, simsense_batch_tuning *t);
/* Times every tuning candidate (horizontal_lanes in {16, 32, 64} x blocks_per_cu in
 * {1, 2, 3, 4}) over `reps` launches on `pairs`, writes the mean milliseconds of
 * candidate i to ms[i] (host, up to max_candidates) and their number to *count,
 * keeps the fastest and returns it in *best.  Synchronous. */
int simsense_batch_autotune(simsense_batch *b, const simsense_pair *pairs, int32_t reps,
                            simsense_batch_tuning *best, float *ms, int32_t max_candidates, int32_t *count,
                            void *stream);

/* Launch shape of one handle's aggregation pass (the results do not depend on
 * it).  Same struct as the batch tuning, with blocks_per_cu 0 meaning one
 * block per line block of work (a grid of all of them, in direction order) and
 * 1..8 a persistent grid of that many blocks per compute unit that takes line
 * blocks longest first.  Default: horizontal_lanes 0, blocks_per_cu 3.
 * Synchronous (uploads the work list); returns SIMSENSE_ERR_INVALID_ARGUMENT
 * for values outside those ranges or a lane count that does not divide the
 * padded disparity count. */
int simsense_set_tuning(simsense_handle *h, const simsense_batch_tuning *t);
int simsense_get_tuning(const simsense_handle *h, simsense_batch_tuning *t);
/* Times every candidate (the valid horizontal_lanes of {16, 32, 64} x
 * blocks_per_cu in {0, 1, 2, 3, 4}) over `reps` matching passes (census ..
 * selection) of the given pair, writes the mean milliseconds of candidate i to
 * ms[i] (host, up to max_candidates) and their number to *count, keeps the
 * fastest and returns it in *best.  Synchronous. */
int simsense_autotune(simsense_handle *h, const uint8_t *left, const uint8_t *right, int32_t pitch, int32_t reps,
                      simsense_batch_tuning *best, float *ms, int32_t max_candidates, int32_t *count, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): simsense_compute without
 * a handle.  Same arguments and results as simsense_create + simsense_compute +
 * simsense_destroy with `params` (bit for bit: the same kernels, the aggregation
 * launched one block per line block), but the scratch lives in one static device
 * array of SIMSENSE_NOALLOC_SCRATCH_BYTES per GPU, which the library holds from
 * its first call on that GPU until the process ends; the call allocates nothing.
 * Parameters whose scratch (simsense_scratch_bytes) exceeds it return
 * SIMSENSE_ERR_TOO_LARGE before anything is enqueued (64 MiB holds, for example,
 * 320x240 with D = 64 and 8 paths, or 640x480 with D = 64 and 2 paths).  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on one GPU
 * (on different streams, or from different threads) race and must not be issued;
 * calls queued in order on one stream are safe.  Asynchronous on `stream`. */
#define SIMSENSE_NOALLOC_SCRATCH_BYTES (64ll << 20)
int simsense_compute_noalloc(const simsense_params *params, const uint8_t *left, const uint8_t *right,
                             int32_t pitch, float *depth, float *disp, uint8_t *flags, void *stream);

/* Human-readable name of a status code (static storage). */
const char *simsense_strerror(int status);

/* Bytes of device scratch a handle with these parameters allocates, or a
 * negative status if the parameters are invalid. */
int64_t simsense_scratch_bytes(const simsense_params *params);

#ifdef __cplusplus
}
#endif
#endif /* SIMSENSE_H */
