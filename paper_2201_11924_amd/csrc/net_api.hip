// C ABI of the learned surrogate: the net handle (parameters, Adam state,
// activations), its forward and training step, and the learned depth path
// (2-path matching -> features -> net -> combine -> median/depth).
#include <math.h>
#include <new>
#include <string.h>

#include "internal.h"
#include "net_internal.h"
#include "trace.h"

namespace ss {
namespace net {

struct LayerShape {
    int cin, cout, cinp, coutp;
};
constexpr LayerShape kLayers[4] = {{4, 32, 8, 32}, {32, 32, 32, 32}, {32, 32, 32, 32}, {32, 2, 32, 16}};
constexpr int kNumParams = 9 * 4 * 32 + 32 + 2 * (9 * 32 * 32 + 32) + 9 * 32 * 2 + 2;  // 20258
constexpr int kLossBlocks = 2048, kMaxWgradBlocks = 2048;

int woff(int l)
{
    int o = 0;
    for (int i = 0; i < l; ++i) o += 9 * kLayers[i].cin * kLayers[i].cout + kLayers[i].cout;
    return o;
}
int boff(int l) { return woff(l) + 9 * kLayers[l].cin * kLayers[l].cout; }

}  // namespace net
}  // namespace ss

using namespace ss;
using namespace ss::net;



namespace {

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

// host-side deterministic init: He-uniform weights from a splitmix64 stream, zero biases
uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void init_params(float *host, uint64_t seed)
{
    uint64_t s = seed;
    for (int l = 0; l < 4; ++l) {
        const int nw = 9 * kLayers[l].cin * kLayers[l].cout;
        const double bound = sqrt(6.0 / (9.0 * kLayers[l].cin));
        for (int i = 0; i < nw; ++i) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            host[woff(l) + i] = (float)((2.0 * u - 1.0) * bound);
        }
        for (int i = 0; i < kLayers[l].cout; ++i) host[boff(l) + i] = 0.0f;
    }
}

RelayoutArgs relayout_args(simsense_net *n)
{
    RelayoutArgs r{};
    r.params = n->params;
    for (int l = 0; l < 4; ++l) {
        LayerDesc &d = r.layer[l];
        d.cin = kLayers[l].cin;
        d.cout = kLayers[l].cout;
        d.cinp = kLayers[l].cinp;
        d.coutp = kLayers[l].coutp;
        d.cinp_b = kLayers[l].cinp;   // rows of the backward-data GEMM: this layer's input channels
        d.coutp_b = kLayers[l].coutp; // its k runs over this layer's (padded) output channels
        d.woff = woff(l);
        d.boff = boff(l);
        d.wf = n->wf[l];
        d.wb = l > 0 ? n->wb[l] : nullptr;
        d.bias = n->bias[l];
    }
    return r;
}

#define NET_TRY(expr) \
    do { if ((expr) != hipSuccess) { (void)hipGetLastError(); return SIMSENSE_ERR_DEVICE; } } while (0)

}  // namespace

int ss::net::enqueue_forward(simsense_net *n, const uint16_t *x0, int batch, int H, int W, hipStream_t s)
{
    ConvArgs c{};
    c.batch = batch; c.H = H; c.W = W;
    const uint16_t *in = x0;
    for (int l = 0; l < 3; ++l) {
        c.in = in; c.weights = n->wf[l]; c.bias = n->bias[l]; c.mask = nullptr; c.out = n->act[l];
        c.mask_out = n->relu_mask[l];
        NET_TRY(launch_conv(c, kLayers[l].cinp, kLayers[l].coutp, EPI_RELU, s));
        in = n->act[l];
    }
    c.in = in; c.weights = n->wf[3]; c.bias = n->bias[3]; c.out = n->out;
    NET_TRY(launch_conv(c, 32, 16, EPI_LINEAR, s));
    return SIMSENSE_OK;
}

InferArgs ss::net::infer_args(const simsense_net *n, const uint16_t *feat, int batch, int H, int W)
{
    InferArgs a{};
    a.feat = feat;
    for (int l = 0; l < 4; ++l) {
        a.w[l] = n->wf[l];
        a.b[l] = n->bias[l];
    }
    const int64_t P = (int64_t)H * W;
    a.d2_stride = a.masked_stride = a.flags_stride = P;
    a.batch = batch; a.H = H; a.W = W;
    return a;
}

namespace {

int check_shape(simsense_net *n, int batch, int H, int W)
{
    if (batch < 1 || H < 1 || W < 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if ((int64_t)batch * H * W > n->max_pixels) return SIMSENSE_ERR_INVALID_ARGUMENT;
    return SIMSENSE_OK;
}

}  // namespace

extern "C" {

int64_t simsense_net_num_params(void) { return kNumParams; }

int simsense_net_create(int64_t max_pixels, uint64_t seed, simsense_net **out)
{
    if (!out) return SIMSENSE_ERR_NULL_POINTER;
    if (max_pixels < 1 || max_pixels > ((int64_t)1 << 31)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    simsense_net *n = new (std::nothrow) simsense_net();
    if (!n) return SIMSENSE_ERR_OUT_OF_MEMORY;
    n->max_pixels = max_pixels;
    const size_t P = (size_t)max_pixels;
    const int wblocks = kMaxWgradBlocks;
    size_t sz[48];
    int k = 0;
    for (int i = 0; i < 4; ++i) sz[k++] = a256(kNumParams * sizeof(float));          // params, m, v, grad
    for (int l = 0; l < 4; ++l) sz[k++] = a256(kLayers[l].coutp * kpad(kLayers[l].cinp) * 2);  // wf
    for (int l = 0; l < 4; ++l) sz[k++] = a256(kLayers[l].cinp * kpad(kLayers[l].coutp) * 2);  // wb
    for (int l = 0; l < 4; ++l) sz[k++] = a256(kLayers[l].coutp * sizeof(float));              // bias
    sz[k++] = a256(P * 16);          // feat
    for (int l = 0; l < 3; ++l) sz[k++] = a256(P * 64);  // act
    sz[k++] = a256(P * 8);           // out
    sz[k++] = a256(P * 32);          // dy4
    for (int l = 0; l < 3; ++l) sz[k++] = a256(P * 64);  // g[l]
    sz[k++] = a256((size_t)wblocks * 32 * 9 * 32 * sizeof(float));  // wpart
    sz[k++] = a256((size_t)wblocks * 32 * sizeof(float));           // bpart
    sz[k++] = a256((size_t)kLossBlocks * 3 * sizeof(float));        // lpart
    sz[k++] = a256(3 * sizeof(float));                              // scal
    sz[k++] = a256(3 * sizeof(float));                              // loss
    sz[k++] = a256(P * 4);           // t_res
    sz[k++] = a256(P);               // t_valid
    for (int l = 0; l < 3; ++l) sz[k++] = a256(P * 4);  // relu_mask
    static_assert(sizeof(sz) / sizeof(sz[0]) >= 4 + 4 + 4 + 4 + 1 + 3 + 1 + 1 + 3 + 5 + 2 + 3, "one size per buffer");
    size_t total = 0;
    for (int i = 0; i < k; ++i) total += sz[i];
    if (hipMalloc(&n->block, total) != hipSuccess) {
        (void)hipGetLastError();
        delete n;
        return SIMSENSE_ERR_OUT_OF_MEMORY;
    }
    uint8_t *cur = (uint8_t *)n->block;
    k = 0;
    auto take = [&]() { void *p = cur; cur += sz[k++]; return p; };
    n->params = (float *)take(); n->m = (float *)take(); n->v = (float *)take(); n->grad = (float *)take();
    for (int l = 0; l < 4; ++l) n->wf[l] = (uint16_t *)take();
    for (int l = 0; l < 4; ++l) n->wb[l] = (uint16_t *)take();
    for (int l = 0; l < 4; ++l) n->bias[l] = (float *)take();
    n->feat = (uint16_t *)take();
    for (int l = 0; l < 3; ++l) n->act[l] = (uint16_t *)take();
    n->out = (float *)take();
    n->dy4 = (uint16_t *)take();
    for (int l = 0; l < 3; ++l) n->g[l] = (uint16_t *)take();
    n->wpart = (float *)take();
    n->bpart = (float *)take();
    n->lpart = (float *)take();
    n->scal = (float *)take();
    n->loss = (float *)take();
    n->t_res = (float *)take();
    n->t_valid = (uint8_t *)take();
    for (int l = 0; l < 3; ++l) n->relu_mask[l] = (uint8_t *)take();
    n->last_stream = nullptr;
    n->step = 0;
    n->last_P = 0;
    float *host = new (std::nothrow) float[kNumParams];
    if (!host) { (void)hipFree(n->block); delete n; return SIMSENSE_ERR_OUT_OF_MEMORY; }
    init_params(host, seed);
    int rc = SIMSENSE_OK;
    if (hipMemcpy(n->params, host, kNumParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(n->m, 0, kNumParams * sizeof(float)) != hipSuccess ||
        hipMemset(n->v, 0, kNumParams * sizeof(float)) != hipSuccess ||
        hipMemset(n->grad, 0, kNumParams * sizeof(float)) != hipSuccess ||
        launch_relayout(relayout_args(n), nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
        rc = SIMSENSE_ERR_DEVICE;
    delete[] host;
    if (rc != SIMSENSE_OK) {
        (void)hipGetLastError();
        (void)hipFree(n->block);
        delete n;
        return rc;
    }
    *out = n;
    return SIMSENSE_OK;
}

int simsense_net_destroy(simsense_net *n)
{
    if (!n) return SIMSENSE_OK;
    int rc = SIMSENSE_OK;
    if (hipStreamSynchronize(n->last_stream) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    if (hipFree(n->block) != hipSuccess) rc = SIMSENSE_ERR_DEVICE;
    delete n;
    return rc;
}

int simsense_net_get_state(simsense_net *n, float *params, float *m, float *v, int64_t count, int64_t *step)
{
    if (!n) return SIMSENSE_ERR_NULL_POINTER;
    if (count != kNumParams) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(n->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    const size_t b = kNumParams * sizeof(float);
    if (params && hipMemcpy(params, n->params, b, hipMemcpyDeviceToHost) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if (m && hipMemcpy(m, n->m, b, hipMemcpyDeviceToHost) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if (v && hipMemcpy(v, n->v, b, hipMemcpyDeviceToHost) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if (step) *step = n->step;
    return SIMSENSE_OK;
}

int simsense_net_set_state(simsense_net *n, const float *params, const float *m, const float *v, int64_t count,
                           int64_t step)
{
    if (!n || !params) return SIMSENSE_ERR_NULL_POINTER;
    if (count != kNumParams || step < 0) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(n->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    const size_t b = kNumParams * sizeof(float);
    if (hipMemcpy(n->params, params, b, hipMemcpyHostToDevice) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if ((m ? hipMemcpy(n->m, m, b, hipMemcpyHostToDevice) : hipMemset(n->m, 0, b)) != hipSuccess)
        return SIMSENSE_ERR_DEVICE;
    if ((v ? hipMemcpy(n->v, v, b, hipMemcpyHostToDevice) : hipMemset(n->v, 0, b)) != hipSuccess)
        return SIMSENSE_ERR_DEVICE;
    n->step = step;
    if (launch_relayout(relayout_args(n), nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return SIMSENSE_ERR_DEVICE;
    }
    return SIMSENSE_OK;
}

int simsense_net_get_grads(simsense_net *n, float *grads, int64_t count)
{
    if (!n || !grads) return SIMSENSE_ERR_NULL_POINTER;
    if (count != kNumParams) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(n->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    if (hipMemcpy(grads, n->grad, kNumParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return SIMSENSE_ERR_DEVICE;
    return SIMSENSE_OK;
}

int simsense_net_read_tensor(simsense_net *n, int32_t what, int32_t layer, void *host, int64_t bytes)
{
    if (!n || !host) return SIMSENSE_ERR_NULL_POINTER;
    const int64_t P = n->last_P;
    const void *src = nullptr;
    int64_t size = 0;
    if (what == SIMSENSE_NET_ACTIVATION && layer >= 0 && layer < 3) {
        src = n->act[layer];
        size = P * 32 * 2;
    } else if (what == SIMSENSE_NET_OUTPUT && layer == 3) {
        src = n->out;
        size = P * 2 * 4;
    } else if (what == SIMSENSE_NET_OUTPUT_GRAD && layer >= 0 && layer < 3) {
        src = n->g[layer];
        size = P * 32 * 2;
    } else if (what == SIMSENSE_NET_OUTPUT_GRAD && layer == 3) {
        src = n->dy4;
        size = P * 16 * 2;
    } else {
        return SIMSENSE_ERR_INVALID_ARGUMENT;
    }
    if (P == 0 || bytes != size) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (hipStreamSynchronize(n->last_stream) != hipSuccess) return SIMSENSE_ERR_DEVICE;
    NET_TRY(hipMemcpy(host, src, (size_t)size, hipMemcpyDeviceToHost));
    return SIMSENSE_OK;
}

int simsense_net_forward(simsense_net *n, const uint16_t *features, int32_t batch, int32_t height, int32_t width,
                         float *out, void *stream)
{
    if (!n || !features || !out) return SIMSENSE_ERR_NULL_POINTER;
    int rc = check_shape(n, batch, height, width);
    if (rc != SIMSENSE_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    n->last_stream = s;
    n->last_P = (int64_t)batch * height * width;
    rc = enqueue_forward(n, features, batch, height, width, s);
    if (rc != SIMSENSE_OK) return rc;
    NET_TRY(hipMemcpyAsync(out, n->out, (size_t)batch * height * width * 2 * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
    return SIMSENSE_OK;
}

int simsense_net_train_step(simsense_net *n, const uint16_t *features, const float *target_residual,
                            const uint8_t *target_valid, int32_t batch, int32_t height, int32_t width, float lr,
                            float *loss, void *stream)
{
    if (!n || !features || !target_residual || !target_valid) return SIMSENSE_ERR_NULL_POINTER;
    int rc = check_shape(n, batch, height, width);
    if (rc != SIMSENSE_OK) return rc;
    if (!(lr >= 0.0f) || !isfinite(lr)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    n->last_stream = s;
    TraceRange range("simsense_net_train_step");
    const int64_t P = (int64_t)batch * height * width;
    n->last_P = P;
    rc = enqueue_forward(n, features, batch, height, width, s);
    if (rc != SIMSENSE_OK) return rc;

    LossArgs la{};
    la.out = n->out; la.t_res = target_residual; la.t_valid = target_valid; la.dy = n->dy4;
    la.partial = n->lpart; la.scal = n->scal; la.loss = n->loss; la.P = P;
    NET_TRY(launch_loss(la, kLossBlocks, s));

    int rsplit = 1;
    const int wblocks = wgrad_blocks(batch, height, width, kMaxWgradBlocks, &rsplit);
    // gradient at each layer's output, layer inputs
    const uint16_t *dy = n->dy4;
    const uint16_t *xin[4] = {features, n->act[0], n->act[1], n->act[2]};
    for (int l = 3; l >= 0; --l) {
        WgradArgs wa{};
        wa.x = xin[l]; wa.dy = dy; wa.partial = n->wpart; wa.bpartial = n->bpart;
        wa.batch = batch; wa.H = height; wa.W = width; wa.rsplit = rsplit;
        NET_TRY(launch_wgrad(wa, kLayers[l].cinp, kLayers[l].coutp, s));
        WgradReduceArgs ra{};
        ra.partial = n->wpart; ra.bpartial = n->bpart; ra.grad = n->grad;
        ra.nblocks = wblocks; ra.nbblocks = wblocks;
        ra.cin = kLayers[l].cin; ra.cout = kLayers[l].cout; ra.cinp = kLayers[l].cinp; ra.coutp = kLayers[l].coutp;
        ra.woff = woff(l); ra.boff = boff(l);
        NET_TRY(launch_wgrad_reduce(ra, s));
        if (l > 0) {
            // gradient at the previous layer's output: backward-data conv, masked by its ReLU
            ConvArgs c{};
            c.in = dy; c.weights = n->wb[l]; c.bias = nullptr; c.mask = n->relu_mask[l - 1]; c.out = n->g[l - 1];
            c.batch = batch; c.H = height; c.W = width;
            NET_TRY(launch_conv(c, kLayers[l].coutp, kLayers[l].cinp, EPI_MASK, s));
            dy = n->g[l - 1];
        }
    }
    n->step += 1;
    AdamArgs ad{};
    ad.p = n->params; ad.m = n->m; ad.v = n->v; ad.grad = n->grad; ad.n = kNumParams;
    ad.lr = lr; ad.b1 = 0.9f; ad.b2 = 0.999f; ad.eps = 1e-8f;
    // bias corrections from the same (float32) decay rates the moments use
    ad.c1 = (float)(1.0 - pow((double)ad.b1, (double)n->step));
    ad.c2 = (float)(1.0 - pow((double)ad.b2, (double)n->step));
    NET_TRY(launch_adam(ad, s));
    NET_TRY(launch_relayout(relayout_args(n), s));
    if (loss) NET_TRY(hipMemcpyAsync(loss, n->loss, 3 * sizeof(float), hipMemcpyDeviceToDevice, s));
    return SIMSENSE_OK;
}

int simsense_net_targets(const float *d8_sub, const uint8_t *flags8, const float *d2_sub, float *t_res,
                         uint8_t *t_valid, int64_t count, void *stream)
{
    if (count < 0) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (count == 0) return SIMSENSE_OK;
    if (!d8_sub || !flags8 || !d2_sub || !t_res || !t_valid) return SIMSENSE_ERR_NULL_POINTER;
    NET_TRY(launch_targets(d8_sub, flags8, d2_sub, t_res, t_valid, count, (hipStream_t)stream));
    return SIMSENSE_OK;
}

int simsense_net_infer(simsense_net *n, const uint16_t *features, int32_t batch, int32_t height, int32_t width,
                       const float *d2_sub, float *out, float *masked, uint8_t *flags, float tau,
                       unsigned *uncertain, void *stream)
{
    if (!n || !features) return SIMSENSE_ERR_NULL_POINTER;
    if (batch < 1 || height < 1 || width < 1) return SIMSENSE_ERR_INVALID_ARGUMENT;
    const int set = (d2_sub != nullptr) + (masked != nullptr) + (flags != nullptr);
    if (set != 0 && set != 3) return SIMSENSE_ERR_NULL_POINTER;
    if ((int64_t)batch * height * width > ((int64_t)1 << 40)) return SIMSENSE_ERR_INVALID_ARGUMENT;
    hipStream_t s = (hipStream_t)stream;
    n->last_stream = s;
    InferArgs a = infer_args(n, features, batch, height, width);
    a.d2_sub = d2_sub; a.masked = masked; a.flags = flags; a.out = out;
    a.uncertain = uncertain; a.tau = tau;
    NET_TRY(launch_infer(a, s));
    return SIMSENSE_OK;
}

int simsense_learned_compute(simsense_handle *h, simsense_net *n, const uint8_t *left, const uint8_t *right,
                             int32_t pitch, const simsense_outputs *o, void *stream)
{
    if (!h || !n || !left || !right || !o) return SIMSENSE_ERR_NULL_POINTER;
    const simsense_params &p = h->p;
    if (pitch < p.width) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if ((int64_t)p.width * p.height > n->max_pixels) return SIMSENSE_ERR_INVALID_ARGUMENT;
    if (p.block_w * p.block_h > 1) return SIMSENSE_ERR_UNSUPPORTED;  // the net was trained on SGM costs
    hipStream_t s = (hipStream_t)stream;
    n->last_stream = s;
    TraceRange range("simsense_learned_compute");
    const int64_t P = (int64_t)p.width * p.height;
    int rc = profile_begin_call(h);
    if (rc != SIMSENSE_OK) return rc;
    rc = enqueue_match(h, left, right, pitch, s, nullptr, /*need_right=*/false);
    if (rc != SIMSENSE_OK) return rc;
    const float smax = (float)(h->ndirs * (h->bits + p.p2));
    if (o->features) {
        // the features themselves only when asked for: the net builds its own
        FeatureArgs fa{};
        fa.ir = left; fa.pitch = pitch; fa.W = p.width;
        fa.s1 = h->cost_best; fa.s2 = h->cost_second; fa.dint = h->disp_int;
        fa.max_disp = p.max_disp; fa.smax = smax;
        fa.features = o->features; fa.P = P;
        NET_TRY(launch_features(fa, s));
    }
    InferArgs ia = infer_args(n, nullptr, 1, p.height, p.width);
    ia.ir = left; ia.ir_pitch = pitch;
    ia.s1 = h->cost_best; ia.s2 = h->cost_second; ia.dint = h->disp_int;
    ia.max_disp = p.max_disp; ia.smax = smax;
    ia.d2_sub = h->disp_sub; ia.masked = h->masked; ia.flags = h->flags_pre;
    NET_TRY(launch_infer(ia, s));
    rc = enqueue_post(h, h->masked, h->flags_pre, o, s);
    if (rc != SIMSENSE_OK) return rc;
    profile_end_call(h);
    if (o->disp_sub) NET_TRY(hipMemcpyAsync(o->disp_sub, h->disp_sub, P * 4, hipMemcpyDeviceToDevice, s));
    if (o->disp_int) NET_TRY(hipMemcpyAsync(o->disp_int, h->disp_int, P, hipMemcpyDeviceToDevice, s));
    return SIMSENSE_OK;
}

}  // extern "C"
