/*
 * CPU oracle of the steps either side of the depth path (Sec. VI-D names
 * rectification before matching and depth registration to the RGB frame after
 * it; Table II's output is the registered 1920x1080 depth).  TEST
 * INFRASTRUCTURE ONLY; it shares no code with the GPU library.
 *
 * Readings (the paper gives no formulas):
 *  - rectification applies per-output-pixel source coordinates (map_x, map_y),
 *    as produced by a calibration tool, with bilinear interpolation; sources
 *    outside [0, W-1] x [0, H-1] give 0; the interpolation is evaluated in
 *    float32 as two horizontal lerps and one vertical lerp, each a + f*(b-a)
 *    with every operation rounded (no fused multiply-add), then rounded to the
 *    nearest integer (ties to even) and clipped to [0, 255];
 *  - registration back-projects every valid depth pixel (u, v, z > 0) of the
 *    rectified left camera, X = (u-cx) z / fx, Y = (v-cy) z / fy, Z = z, moves it
 *    to the RGB camera, X' = R X + t (row sums left to right), drops Z' <= 0,
 *    projects u' = fx' X'/Z' + cx', v' = fy' Y'/Z' + cy', rounds to the nearest
 *    pixel (ties to even) and keeps the smallest Z' per RGB pixel; empty pixels
 *    are 0.  All in float32, operation by operation.
 */
#include <math.h>
#include <stdint.h>

void orc_rectify(const uint8_t *in, int in_pitch, int W, int H, const float *map_x, const float *map_y, int out_w,
                 int out_h, uint8_t *out)
{
    for (int y = 0; y < out_h; ++y)
        for (int x = 0; x < out_w; ++x) {
            const float sx = map_x[(int64_t)y * out_w + x], sy = map_y[(int64_t)y * out_w + x];
            float r = 0.0f;
            if (sx >= 0.0f && sy >= 0.0f && sx <= (float)(W - 1) && sy <= (float)(H - 1)) {
                const int x0 = (int)floorf(sx), y0 = (int)floorf(sy);
                const int x1 = x0 + 1 < W ? x0 + 1 : W - 1, y1 = y0 + 1 < H ? y0 + 1 : H - 1;
                volatile float fx = sx - (float)x0, fy = sy - (float)y0;
                const float i00 = in[(int64_t)y0 * in_pitch + x0], i01 = in[(int64_t)y0 * in_pitch + x1];
                const float i10 = in[(int64_t)y1 * in_pitch + x0], i11 = in[(int64_t)y1 * in_pitch + x1];
                volatile float dt = i01 - i00, db = i11 - i10;
                volatile float mt = fx * dt, mb = fx * db;
                volatile float top = i00 + mt, bot = i10 + mb;
                volatile float dv = bot - top;
                volatile float mv = fy * dv;
                volatile float v = top + mv;
                r = rintf(v);
                if (r < 0.0f) r = 0.0f;
                if (r > 255.0f) r = 255.0f;
            }
            out[(int64_t)y * out_w + x] = (uint8_t)r;
        }
}

typedef struct orc_camera {
    float fx, fy, cx, cy;
} orc_camera;

void orc_register_depth(const float *depth, int W, int H, const orc_camera *ir, const float *rt, const orc_camera *rgb,
                        int out_w, int out_h, float *out)
{
    for (int64_t i = 0; i < (int64_t)out_w * out_h; ++i) out[i] = 0.0f;
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            const float z = depth[(int64_t)v * W + u];
            if (!(z > 0.0f)) continue;
            volatile float du = (float)u - ir->cx, dv = (float)v - ir->cy;
            volatile float pu = du * z, pv = dv * z;
            volatile float X = pu / ir->fx, Y = pv / ir->fy, Z = z;
            float P[3];
            for (int r = 0; r < 3; ++r) {
                volatile float a = rt[3 * r + 0] * X;
                volatile float b = rt[3 * r + 1] * Y;
                volatile float c = rt[3 * r + 2] * Z;
                volatile float s = a + b;
                volatile float s2 = s + c;
                volatile float s3 = s2 + rt[9 + r];
                P[r] = s3;
            }
            if (!(P[2] > 0.0f)) continue;
            volatile float qx = P[0] / P[2], qy = P[1] / P[2];
            volatile float mx = rgb->fx * qx, my = rgb->fy * qy;
            volatile float ux = mx + rgb->cx, uy = my + rgb->cy;
            const float rx = rintf(ux), ry = rintf(uy);
            if (!(rx >= 0.0f && ry >= 0.0f && rx <= (float)(out_w - 1) && ry <= (float)(out_h - 1))) continue;
            const int64_t o = (int64_t)ry * out_w + (int64_t)rx;
            if (out[o] == 0.0f || P[2] < out[o]) out[o] = P[2];
        }
}
