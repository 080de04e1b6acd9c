/*
 * Drives every entry point of the CPU oracle over small, ragged and degenerate
 * inputs, built with AddressSanitizer and UndefinedBehaviorSanitizer (no
 * recovery): an out-of-bounds access, a leak, a signed overflow or an invalid
 * shift anywhere in the oracle ends the run with an error.  Results are not
 * checked here (the Python tests pin them); the run only has to be clean.
 *
 * The oracle sources are compiled into this file directly.
 */
#include "../../oracle/sgm_oracle.c"
#include "../../oracle/noise_oracle.c"
#include "../../oracle/geometry_oracle.c"

#include <stdio.h>

static uint32_t rng_state = 12345u;
static uint32_t next_u32(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 17;
    rng_state ^= rng_state << 5;
    return rng_state;
}

static void run_sgm(int W, int H, int D, int cw, int ch, int mode, int paths, int lr_mode, int bw, int bh,
                    int median, int subpixel, int uniq, int keep_volume)
{
    const size_t npx = (size_t)W * H;
    uint8_t *l = malloc(npx), *r = malloc(npx);
    for (size_t i = 0; i < npx; ++i) {
        l[i] = (uint8_t)(next_u32() & 0xFF);
        r[i] = (uint8_t)(next_u32() & 0xFF);
    }
    const int bits = orc_census_bits(cw, ch, mode);
    orc_params p = {W, H, D, cw, ch, mode, 7, bits * bw * bh + 86 > 255 && bw * bh == 1 ? 255 - bits : 86,
                    uniq, 1, paths, median, subpixel, 400.0f, 0.055f, lr_mode, bw, bh};
    orc_result res;
    res.census_l = malloc(npx * 8);
    res.census_r = malloc(npx * 8);
    res.S = keep_volume ? malloc(npx * D * sizeof(uint32_t)) : NULL;
    res.dint = malloc(npx * 4);
    res.s1 = malloc(npx * 4);
    res.s2 = malloc(npx * 4);
    res.dright = malloc(npx * 4);
    res.flags = malloc(npx);
    res.dsub = malloc(npx * 8);
    res.disp = malloc(npx * 8);
    res.depth = malloc(npx * 8);
    if (orc_sgm(&p, l, r, &res) != 0) {
        fprintf(stderr, "orc_sgm failed\n");
        exit(1);
    }
    free(res.census_l); free(res.census_r); free(res.S); free(res.dint); free(res.s1); free(res.s2);
    free(res.dright); free(res.flags); free(res.dsub); free(res.disp); free(res.depth);
    free(l);
    free(r);
}

int main(void)
{
    /* shapes: thin, tiny, ragged; disparity ranges from 1 to beyond the width */
    static const int shapes[][3] = {{1, 1, 1}, {1, 9, 3}, {9, 1, 5}, {2, 3, 2}, {17, 5, 37}, {33, 21, 16},
                                    {40, 24, 64}, {5, 40, 2}};
    static const int windows[][3] = {{3, 3, 0}, {5, 5, 0}, {7, 9, 0}, {9, 7, 0}, {9, 9, 0}, {7, 9, 1},
                                     {5, 3, 1}, {3, 5, 1}, {1, 3, 0}, {3, 1, 1}};
    int n = 0;
    for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s)
        for (size_t w = 0; w < sizeof(windows) / sizeof(windows[0]); ++w) {
            const int W = shapes[s][0], H = shapes[s][1], D = shapes[s][2];
            const int paths = 2 << (int)((s + w) % 3);
            run_sgm(W, H, D, windows[w][0], windows[w][1], windows[w][2], paths, (int)(w & 1), 1, 1,
                    (w % 2) ? 3 : 0, (int)(s & 1), (int)(10 * (w % 3)), (int)(s % 2));
            ++n;
        }
    /* block matching, both LR modes */
    run_sgm(23, 11, 9, 5, 5, 0, 8, 0, 3, 3, 3, 1, 10, 1);
    run_sgm(23, 11, 9, 5, 5, 0, 4, 1, 5, 3, 3, 1, 0, 0);
    run_sgm(3, 2, 4, 7, 9, 0, 8, 1, 31, 31, 3, 1, 10, 0);
    n += 3;

    /* noise model and the on-device generator's oracle */
    {
        const int64_t cnt = 1000;
        uint8_t in[1000], out[1000];
        float g[1000], nn[1000];
        for (int i = 0; i < cnt; ++i) in[i] = (uint8_t)(next_u32() & 0xFF);
        for (int model = 0; model < 3; ++model) {
            orc_noise_params np = {model, 3.98f, 0.254f, 0.05f, -0.231f, 0.83f, 1.5f, 7u, 0u, 3u};
            orc_noise_draws(&np, cnt, g, nn);
            orc_ir_noise(in, g, nn, out, cnt);
        }
        ++n;
    }
    /* rectification and registration, including maps that leave the image */
    {
        enum { IW = 13, IH = 7, OW = 11, OH = 9 };
        uint8_t img[IW * IH], rect[OW * OH];
        float mx[OW * OH], my[OW * OH], depth[IW * IH], reg[OW * OH];
        for (int i = 0; i < IW * IH; ++i) {
            img[i] = (uint8_t)(next_u32() & 0xFF);
            depth[i] = (next_u32() % 4 == 0) ? 0.0f : 0.2f + (float)(next_u32() % 1000) * 0.01f;
        }
        for (int i = 0; i < OW * OH; ++i) {
            mx[i] = (float)((int)(next_u32() % 40) - 10) * 0.77f;
            my[i] = (float)((int)(next_u32() % 30) - 10) * 0.61f;
        }
        orc_rectify(img, IW, IW, IH, mx, my, OW, OH, rect);
        const orc_camera ir = {20.0f, 20.0f, 6.0f, 3.0f}, rgb = {15.0f, 15.0f, 5.0f, 4.0f};
        const float rt[12] = {1, 0, 0, 0, 1, 0, 0, 0, 1, -0.05f, 0.01f, 0.0f};
        orc_register_depth(depth, IW, IH, &ir, rt, &rgb, OW, OH, reg);
        ++n;
    }
    printf("oracle sanitizer run clean: %d cases\n", n);
    return 0;
}
