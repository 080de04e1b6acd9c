// Internal declarations of the learned surrogate's kernels (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ss {
namespace net {

// GEMM depth of a 3x3 convolution over CINP padded channels, rounded up to the
// 32-deep k-step of v_mfma_f32_16x16x32_bf16.
__host__ __device__ constexpr int kpad(int cinp) { return (9 * cinp + 31) / 32 * 32; }

// conv epilogues
// EPI_RELU:   out = bf16(max(acc + bias, 0)), COUTP channels
// EPI_LINEAR: out = fp32 acc + bias, channels 0 and 1 only
// EPI_MASK:   out = bf16(acc * (mask > 0)), COUTP channels (the ReLU derivative)
enum { EPI_RELU = 0, EPI_LINEAR = 1, EPI_MASK = 2 };

struct ConvArgs {
    const uint16_t *in;       // bf16 NHWC, CINP channels
    const uint16_t *weights;  // bf16 [COUTP][kpad(CINP)]
    const float *bias;        // fp32 [COUTP] or null
    const uint8_t *mask;      // backward-data: the ReLU masks of its output channels, packed as below
    uint8_t *mask_out;        // ReLU layers (or null): their outputs' masks, packed; 32 channels only
    void *out;                // bf16 NHWC COUTP channels, or fp32 [P][2] for the linear layer
    int batch, H, W;
};

struct WgradArgs {
    const uint16_t *x;   // layer input, bf16 NHWC CINP channels
    const uint16_t *dy;  // gradient at the layer output, bf16 NHWC COUTP channels
    float *partial;      // [blocks][COUTP][9*CINP]
    float *bpartial;     // [blocks][COUTP]
    int batch, H, W;
    int rsplit;          // row ranges per 32-pixel column strip (blocks = batch x strips x rsplit)
};

struct WgradReduceArgs {
    const float *partial, *bpartial;
    float *grad;  // flat gradient, the oracle's parameter order
    int nblocks, nbblocks;
    int cin, cout, cinp, coutp;
    int woff, boff;
};

struct LossArgs {
    const float *out;        // [P][2] residual, logit
    const float *t_res;      // [P]
    const uint8_t *t_valid;  // [P]
    uint16_t *dy;            // bf16 [P][16] gradient at the net output
    float *partial;          // [blocks][3]
    float *scal;             // [3]: valid count, 1/count, 1/P
    float *loss;             // [3]: total, l1, bce (device)
    int64_t P;
};

struct AdamArgs {
    float *p, *m, *v;
    const float *grad;
    int n;
    float lr, b1, b2, eps, c1, c2;  // c1 = 1 - b1^t, c2 = 1 - b2^t
};

struct LayerDesc {
    int cin, cout, cinp, coutp;  // real and padded channel counts
    int cinp_b, coutp_b;         // backward-data GEMM: rows (input channels), k channels (output grads)
    int woff, boff;              // offsets in the flat parameter vector
    uint16_t *wf, *wb;           // forward / backward-data bf16 layouts (wb may be null)
    float *bias;                 // fp32 [coutp]
};

struct RelayoutArgs {
    const float *params;
    LayerDesc layer[4];
};

struct FeatureArgs {
    const uint8_t *ir;  // left image
    int pitch, W;
    const void *job;    // when set: a census job (device) whose image and pitch replace ir / pitch
    const uint16_t *s1, *s2;
    const uint8_t *dint;
    int max_disp;
    float smax;
    uint16_t *features;  // bf16 [P][8]
    int64_t P;
};

struct CombineArgs {
    const float *d2_sub, *out;
    float *masked;
    uint8_t *flags;
    int64_t P;
    unsigned *uncertain;  // nullable: pixels with |logit| < tau are counted here
    float tau;
};

// Fused inference (all four layers, then the combination with the 2-path
// disparity) on `batch` images whose per-pixel outputs lie `*_stride` elements
// apart; masked / flags / d2_sub / out / uncertain may each be null.
struct InferArgs {
    const uint16_t *feat;  // bf16 [batch][H][W][8], or null: built from the selection outputs below
    // the feature inputs when feat is null (the learned form): left image (from
    // `ir`/`ir_pitch`, or when ir_jobs is set from census jobs 2 i of image i),
    // S1, S2, d* (image i's at i * sel_stride bytes past image 0's), and the
    // scales of the features
    const uint8_t *ir;
    int ir_pitch;
    const void *ir_jobs;
    const uint16_t *s1, *s2;
    const uint8_t *dint;
    int64_t sel_stride;
    int max_disp;
    float smax;
    const uint16_t *w[4];  // forward layouts, bf16 [COUTP][kpad(CINP)]
    const float *b[4];     // fp32 [COUTP]
    const float *d2_sub;
    int64_t d2_stride;
    float *masked;
    int64_t masked_stride;
    uint8_t *flags;
    int64_t flags_stride;
    unsigned *uncertain;   // one counter per image: pixels with |logit| < tau
    float tau;
    float *out;            // fp32 [batch][H][W][2] residual and logit, or null
    int batch, H, W;
    int seg_rows;          // rows per block (0 = default); segs / strips are set by the launcher
    int segs, strips;
};

hipError_t launch_conv(const ConvArgs &a, int cinp, int coutp, int epi, hipStream_t s);
hipError_t launch_infer(InferArgs a, hipStream_t s);
// blocks of the backward-weight pass for a batch shape (at most max_blocks), and its row split
int wgrad_blocks(int batch, int H, int W, int max_blocks, int *rsplit);
hipError_t launch_wgrad(const WgradArgs &a, int cinp, int coutp, hipStream_t s);
hipError_t launch_wgrad_reduce(const WgradReduceArgs &a, hipStream_t s);
hipError_t launch_loss(const LossArgs &a, int nblocks, hipStream_t s);
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
hipError_t launch_relayout(const RelayoutArgs &a, hipStream_t s);
hipError_t launch_features(const FeatureArgs &a, hipStream_t s);
hipError_t launch_combine(const CombineArgs &a, hipStream_t s);
hipError_t launch_targets(const float *d8_sub, const uint8_t *flags8, const float *d2_sub, float *t_res,
                          uint8_t *t_valid, int64_t n, hipStream_t s);

}  // namespace net
}  // namespace ss

#include "../../include/simsense.h"

struct simsense_net {
    int64_t max_pixels;
    int64_t step;
    void *block;
    float *params, *m, *v, *grad;
    uint16_t *wf[4], *wb[4];
    float *bias[4];
    uint16_t *feat;        // [P][8] features of the learned depth path
    uint16_t *act[3];      // [P][32] outputs of layers 1..3
    float *out;            // [P][2]
    uint16_t *dy4;         // [P][16]
    uint16_t *g[3];        // [P][32] gradient at the output of layer l (ReLU-masked), l = 0..2
    uint8_t *relu_mask[3]; // [P][4] which outputs of layers 1..3 are > 0, packed (see conv3x3_kernel)
    int64_t last_P;        // pixels of the last forward or training call
    float *wpart, *bpart;  // weight / bias gradient partials
    float *lpart, *scal, *loss;
    float *t_res;          // targets of the learned depth path's own use (training helpers)
    uint8_t *t_valid;
    hipStream_t last_stream;
};

namespace ss {
namespace net {
// the net's four convolutions on `batch` images of height x width into n->out
int enqueue_forward(simsense_net *n, const uint16_t *x0, int batch, int H, int W, hipStream_t s);
// fused-inference arguments for the net's current weights (outputs unset,
// per-image strides of one image)
InferArgs infer_args(const simsense_net *n, const uint16_t *feat, int batch, int H, int W);
}  // namespace net
}  // namespace ss
