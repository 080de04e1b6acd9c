// Host-side checks of the C ABI built with AddressSanitizer and
// UndefinedBehaviorSanitizer: parameter validation, scratch layout arithmetic at
// the largest sizes, every documented argument error of every entry point, and
// the cleanup paths of the create calls when device allocation fails (on a
// machine without a GPU every HIP allocation fails).  The library's host
// sources are linked in, the kernel launchers are replaced by stubs that count
// their calls: no argument-error path may reach a launch.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/simsense.h"

extern int g_stub_calls;

#define CHECK(cond)                                                               \
    do {                                                                          \
        if (!(cond)) {                                                            \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            exit(1);                                                              \
        }                                                                         \
    } while (0)

static simsense_params base()
{
    simsense_params p{};
    p.struct_size = sizeof(p);
    p.width = 320; p.height = 240; p.max_disp = 64;
    p.census_w = 7; p.census_h = 9; p.census_mode = 0;
    p.p1 = 7; p.p2 = 86; p.uniqueness_pct = 10; p.lr_max_diff = 1;
    p.num_paths = 8; p.median = 3; p.subpixel = 1;
    p.focal_px = 400.0f; p.baseline_m = 0.055f;
    p.lr_mode = 0; p.block_w = 1; p.block_h = 1;
    return p;
}

int main()
{
    for (int s = 1; s >= -8; --s) CHECK(simsense_strerror(s) != nullptr);

    // scratch sizes over a grid of valid parameters, up to the largest ones
    const int sizes[][2] = {{1, 1}, {1, 8192}, {8192, 1}, {1280, 720}, {8192, 8192}};
    const int disps[] = {1, 2, 15, 16, 17, 100, 128, 192, 255, 256};
    for (auto &wh : sizes)
        for (int D : disps)
            for (int paths : {2, 4, 8})
                for (int lr : {0, 1})
                    for (int blk : {1, 3, 31}) {
                        simsense_params p = base();
                        p.width = wh[0]; p.height = wh[1]; p.max_disp = D; p.num_paths = paths; p.lr_mode = lr;
                        p.block_w = p.block_h = blk;
                        if (blk > 1) { p.census_w = 3; p.census_h = 3; p.p1 = 20; p.p2 = 200; }
                        const int64_t b = simsense_scratch_bytes(&p);
                        CHECK(b > 0);
                        CHECK(b >= (int64_t)wh[0] * wh[1] * paths);
                    }

    // every documented parameter error
    struct Bad { const char *what; void (*set)(simsense_params &); int code; };
    const Bad bad[] = {
        {"width 0", [](simsense_params &p) { p.width = 0; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"height 8193", [](simsense_params &p) { p.height = 8193; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"D 0", [](simsense_params &p) { p.max_disp = 0; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"D 257", [](simsense_params &p) { p.max_disp = 257; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"even census", [](simsense_params &p) { p.census_w = 6; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"census mode", [](simsense_params &p) { p.census_mode = 2; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"> 64 bits", [](simsense_params &p) { p.census_w = 11; p.census_h = 13; p.census_mode = 1; },
         SIMSENSE_ERR_INVALID_ARGUMENT},
        {"huge census", [](simsense_params &p) { p.census_w = 2147483647; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"p1 < 0", [](simsense_params &p) { p.p1 = -1; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"p2 < p1", [](simsense_params &p) { p.p1 = 10; p.p2 = 9; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"bits + p2", [](simsense_params &p) { p.p2 = 240; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"uniqueness", [](simsense_params &p) { p.uniqueness_pct = 100; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"paths", [](simsense_params &p) { p.num_paths = 3; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"median", [](simsense_params &p) { p.median = 5; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"subpixel", [](simsense_params &p) { p.subpixel = 2; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"focal nan", [](simsense_params &p) { p.focal_px = __builtin_nanf(""); }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"lr mode", [](simsense_params &p) { p.lr_mode = 2; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"block even", [](simsense_params &p) { p.block_w = 2; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"block 33", [](simsense_params &p) { p.block_h = 33; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"block bound", [](simsense_params &p) { p.block_w = p.block_h = 31; p.p2 = 200; }, SIMSENSE_ERR_INVALID_ARGUMENT},
        {"struct size", [](simsense_params &p) { p.struct_size = 4; }, SIMSENSE_ERR_ABI},
    };
    for (const Bad &b : bad) {
        simsense_params p = base();
        b.set(p);
        if (simsense_scratch_bytes(&p) != b.code) {
            fprintf(stderr, "scratch_bytes accepted: %s\n", b.what);
            return 1;
        }
        simsense_handle *h = (simsense_handle *)0x1;
        CHECK(simsense_create(&p, &h) == b.code);
        CHECK(h == (simsense_handle *)0x1);
        simsense_batch *bt = nullptr;
        CHECK(simsense_batch_create(&p, 1, &bt) == b.code && bt == nullptr);
        float d;
        uint8_t img;
        CHECK(simsense_compute_noalloc(&p, &img, &img, 320, &d, nullptr, nullptr, nullptr) == b.code);
        CHECK(simsense_census(&p, &img, 320, (uint64_t *)&d, nullptr) == b.code);
    }

    // NULL pointers and ranges of the other entry points
    simsense_params p = base();
    CHECK(simsense_scratch_bytes(nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_create(&p, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_destroy(nullptr) == SIMSENSE_OK);
    CHECK(simsense_compute(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr) ==
          SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_compute_ex(nullptr, nullptr, nullptr, 0, nullptr, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_ir_noise(nullptr, nullptr, nullptr, nullptr, -1, nullptr) == SIMSENSE_ERR_INVALID_ARGUMENT);
    CHECK(simsense_ir_noise(nullptr, nullptr, nullptr, nullptr, 0, nullptr) == SIMSENSE_OK);
    CHECK(simsense_ir_noise(nullptr, nullptr, nullptr, nullptr, 3, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_profile_enable(nullptr, 1) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_set_tuning(nullptr, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_batch_create(&p, 0, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    simsense_batch *bt = nullptr;
    CHECK(simsense_batch_create(&p, 0, &bt) == SIMSENSE_ERR_INVALID_ARGUMENT);
    CHECK(simsense_batch_create(&p, 2049, &bt) == SIMSENSE_ERR_INVALID_ARGUMENT);
    CHECK(simsense_batch_destroy(nullptr) == SIMSENSE_OK);
    CHECK(simsense_batch_compute(nullptr, nullptr, nullptr) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_batch_learned_fallback(nullptr, nullptr, nullptr, nullptr, 0.5f, nullptr, 0, 0.1f, nullptr,
                                          nullptr) == SIMSENSE_ERR_NULL_POINTER);
    simsense_net *net = nullptr;
    CHECK(simsense_net_num_params() == 20258);
    CHECK(simsense_net_create(0, 0, &net) == SIMSENSE_ERR_INVALID_ARGUMENT && net == nullptr);
    CHECK(simsense_net_create(((int64_t)1 << 31) + 1, 0, &net) == SIMSENSE_ERR_INVALID_ARGUMENT);
    CHECK(simsense_net_destroy(nullptr) == SIMSENSE_OK);
    CHECK(simsense_net_read_tensor(nullptr, 0, 0, nullptr, 0) == SIMSENSE_ERR_NULL_POINTER);
    CHECK(simsense_net_targets(nullptr, nullptr, nullptr, nullptr, nullptr, -1, nullptr) ==
          SIMSENSE_ERR_INVALID_ARGUMENT);
    CHECK(simsense_noise_draws(nullptr, 1, nullptr, nullptr, nullptr) != SIMSENSE_OK);
    CHECK(simsense_rectify(nullptr, 0, 0, 0, nullptr, nullptr, 0, 0, nullptr, 0, nullptr) != SIMSENSE_OK);
    float d;
    uint8_t img;
    p.width = 1280; p.height = 720; p.max_disp = 128;
    CHECK(simsense_compute_noalloc(&p, &img, &img, 1280, &d, nullptr, nullptr, nullptr) == SIMSENSE_ERR_TOO_LARGE);
    CHECK(g_stub_calls == 0);

    // valid parameters on a machine without a GPU: every create fails to
    // allocate and must release whatever it took on the way (checked by the
    // leak sanitizer at exit); the error is reported, nothing is launched
    int ndev = 0;
    const bool no_gpu = hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0;
    (void)hipGetLastError();
    if (no_gpu) {
        simsense_params q = base();
        simsense_handle *h = nullptr;
        CHECK(simsense_create(&q, &h) != SIMSENSE_OK && h == nullptr);
        q.lr_mode = 1;
        CHECK(simsense_create(&q, &h) != SIMSENSE_OK && h == nullptr);
        simsense_params qs[3] = {base(), base(), base()};
        qs[1].width = 97; qs[1].max_disp = 37; qs[2].num_paths = 2;
        CHECK(simsense_batch_create(qs, 3, &bt) != SIMSENSE_OK && bt == nullptr);
        CHECK(simsense_net_create(1000, 1, &net) != SIMSENSE_OK && net == nullptr);
        CHECK(g_stub_calls == 0);
    }
    printf("C ABI host checks clean (%s)\n", no_gpu ? "no GPU: allocation failure paths included" : "GPU present");
    return 0;
}
