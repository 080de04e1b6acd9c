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
    SIMSENSE_ERR_ABI = -6               /* struct_size does not match this library */
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
 *                   0 <= p1 <= p2 and bits + p2 <= 255 (path values are stored in 8 bits).
 *  uniqueness_pct   u in 0..99: a pixel is kept only if 100*S1 <= (100-u)*S2, S2 being
 *                   the best aggregated cost at least two disparities away; 0 disables.
 *  lr_max_diff      left-right check tolerance in pixels; negative disables.
 *  num_paths        2 (horizontal), 4 (+ vertical) or 8 (+ diagonals).
 *  median           0 (off) or 3 (3x3 median of the masked disparity map).
 *  subpixel         0 or 1 (quadratic fit through d*-1, d*, d*+1).
 *  focal_px         focal length in pixels; baseline_m  stereo baseline (depth is in its unit).
 */
typedef struct simsense_params {
    uint32_t struct_size;
    int32_t width, height, max_disp;
    int32_t census_w, census_h, census_mode;
    int32_t p1, p2;
    int32_t uniqueness_pct, lr_max_diff;
    int32_t num_paths, median, subpixel;
    float focal_px, baseline_m;
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
 * resets the accumulators.  Events are created by the enable call. */
#define SIMSENSE_PASS_CENSUS 0
#define SIMSENSE_PASS_AGGREGATE 1
#define SIMSENSE_PASS_SELECT 2
#define SIMSENSE_PASS_POST 3
#define SIMSENSE_NUM_PASSES 4
int simsense_profile_enable(simsense_handle *h, int enable);
int simsense_profile_read(simsense_handle *h, double *ms, int32_t *calls, int32_t n);

/* Human-readable name of a status code (static storage). */
const char *simsense_strerror(int status);

/* Bytes of device scratch a handle with these parameters allocates, or a
 * negative status if the parameters are invalid. */
int64_t simsense_scratch_bytes(const simsense_params *params);

#ifdef __cplusplus
}
#endif
#endif /* SIMSENSE_H */
