/*
 * CPU oracle of the SimSense depth path (Sec. VI-C noise model, Sec. VI-D stereo
 * matching).  TEST INFRASTRUCTURE ONLY: it exists so that the GPU library can be
 * checked against an independent, plain, slow, obviously-correct definition.
 * Nothing in the product path may link, load or call it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Every function is a direct, unblocked, unfused transcription of the
 * definition it cites; integer work is int32/int64, floating point is double
 * unless the definition fixes another precision (the noise model's rounding
 * decision is taken in float32, the precision the GPU path decides it in).
 *
 * Readings of the paper where it is silent (the same readings the GPU path
 * implements):
 *  - census window is census_w (columns) x census_h (rows), offsets enumerated
 *    row-major from the top-left, bit k at position k;
 *    full mode: bit = [I(p) > I(p+o)] for every o != 0;
 *    center-symmetric mode: for every o before the centre in raster order,
 *    bit = [I(p+o) > I(p-o)]; samples outside the image clamp to the edge.
 *  - cost C(x,y,d) = popcount(cL(x,y) ^ cR(x-d,y)), and the number of census
 *    bits where x-d < 0; disparities 0..D-1; for block matching (SGBM) the
 *    pixel costs summed over a block with clamped samples.
 *  - path recurrence in its normalised form, first pixel of a path L = C.
 *  - winner: lowest d on ties; uniqueness second best over |d-d*| >= 2,
 *    valid iff 100*S1 <= (100-u)*S2; sub-pixel parabola through d*-1, d*, d*+1;
 *    right disparity from the left volume (or, as an option, from a full
 *    right-referenced run), LR on integer disparities;
 *    d* = 0 is invalid; 3x3 median on the masked map with the border copied;
 *    depth = f*B/d.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- noise */
/* Eq. (7): I_noisy = gamma * I_clean + n per pixel.  Product and sum are each
 * rounded to float32 (no fused multiply-add), the result is rounded to the
 * nearest integer with ties to even and clipped to the 8-bit range. */
void orc_ir_noise(const uint8_t *in, const float *gamma, const float *n, uint8_t *out, int64_t count)
{
    for (int64_t i = 0; i < count; ++i) {
        volatile float prod = gamma[i] * (float)in[i];
        volatile float sum = prod + n[i];
        float r = rintf(sum);
        if (!(r > 0.0f)) r = 0.0f; /* also maps NaN to 0 */
        if (r > 255.0f) r = 255.0f;
        out[i] = (uint8_t)r;
    }
}

/* ---------------------------------------------------------------- census */
int orc_census_bits(int cw, int ch, int mode)
{
    int n = cw * ch;
    return mode == 0 ? (n - 1) / 2 : n - 1;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

static int pix(const uint8_t *img, int W, int H, int pitch, int x, int y)
{
    return img[(size_t)clampi(y, 0, H - 1) * pitch + clampi(x, 0, W - 1)];
}

/* Center-symmetric census transform (Zabih & Woodfill, the variant the paper
 * uses, Sec. VI-D) or the full census, one word per pixel. */
void orc_census(const uint8_t *img, int W, int H, int pitch, int cw, int ch, int mode, uint64_t *out)
{
    int rw = cw / 2, rh = ch / 2;
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            uint64_t word = 0;
            int k = 0;
            int centre = pix(img, W, H, pitch, x, y);
            for (int dy = -rh; dy <= rh; ++dy) {
                for (int dx = -rw; dx <= rw; ++dx) {
                    if (dx == 0 && dy == 0) {
                        if (mode == 0) goto done; /* CS: only offsets before the centre */
                        continue;
                    }
                    int bit;
                    if (mode == 0)
                        bit = pix(img, W, H, pitch, x + dx, y + dy) > pix(img, W, H, pitch, x - dx, y - dy);
                    else
                        bit = centre > pix(img, W, H, pitch, x + dx, y + dy);
                    word |= (uint64_t)bit << k;
                    ++k;
                }
            }
        done:
            out[(size_t)y * W + x] = word;
        }
    }
}

/* ---------------------------------------------------------------- cost */
int orc_popcount(uint64_t v) { return __builtin_popcountll(v); }

/* Hamming matching cost, C[(y*W + x)*D + d]. */
void orc_cost(const uint64_t *cl, const uint64_t *cr, int W, int H, int D, int bits, uint16_t *C)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d) {
                int c = bits;
                if (x - d >= 0) c = orc_popcount(cl[(size_t)y * W + x] ^ cr[(size_t)y * W + x - d]);
                C[((size_t)y * W + x) * D + d] = (uint16_t)c;
            }
}

/* ---------------------------------------------------------------- aggregation */
/* One SGM path r = (dx, dy) (Hirschmueller 2008, cited in Sec. VI-D):
 *   L(p,d) = C(p,d) + min(L(p-r,d), L(p-r,d-1)+P1, L(p-r,d+1)+P1, m(p-r)+P2) - m(p-r),
 *   m(q) = min_k L(q,k);  L(p,d) = C(p,d) where p-r lies outside the image.
 * Pixels are visited so that p-r is always finished before p. */
void orc_path(const uint16_t *C, int W, int H, int D, int dx, int dy, int P1, int P2, uint16_t *L)
{
    int y0 = dy >= 0 ? 0 : H - 1, y1 = dy >= 0 ? H : -1, ys = dy >= 0 ? 1 : -1;
    int x0 = dx >= 0 ? 0 : W - 1, x1 = dx >= 0 ? W : -1, xs = dx >= 0 ? 1 : -1;
    for (int y = y0; y != y1; y += ys) {
        for (int x = x0; x != x1; x += xs) {
            size_t p = ((size_t)y * W + x) * D;
            int qx = x - dx, qy = y - dy;
            if (qx < 0 || qx >= W || qy < 0 || qy >= H) {
                for (int d = 0; d < D; ++d) L[p + d] = C[p + d];
                continue;
            }
            size_t q = ((size_t)qy * W + qx) * D;
            int m = 1 << 30;
            for (int k = 0; k < D; ++k)
                if (L[q + k] < m) m = L[q + k];
            for (int d = 0; d < D; ++d) {
                int best = L[q + d];
                if (d > 0 && L[q + d - 1] + P1 < best) best = L[q + d - 1] + P1;
                if (d < D - 1 && L[q + d + 1] + P1 < best) best = L[q + d + 1] + P1;
                if (m + P2 < best) best = m + P2;
                L[p + d] = (uint16_t)(C[p + d] + best - m);
            }
        }
    }
}

/* Path directions: 2 paths = horizontal pair; 4 adds the vertical pair; 8 adds
 * the four diagonals. */
static const int PATH_DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
static const int PATH_DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};

void orc_path_dir(int i, int *dx, int *dy)
{
    *dx = PATH_DX[i];
    *dy = PATH_DY[i];
}

/* S(p,d) = sum over the chosen paths of L_r(p,d). */
void orc_aggregate(const uint16_t *C, int W, int H, int D, int num_paths, int P1, int P2, uint32_t *S)
{
    size_t n = (size_t)W * H * D;
    uint16_t *L = (uint16_t *)malloc(n * sizeof(uint16_t));
    memset(S, 0, n * sizeof(uint32_t));
    for (int r = 0; r < num_paths; ++r) {
        orc_path(C, W, H, D, PATH_DX[r], PATH_DY[r], P1, P2, L);
        for (size_t i = 0; i < n; ++i) S[i] += L[i];
    }
    free(L);
}

/* ---------------------------------------------------------------- winner and checks */
/* Winner-take-all with the uniqueness test and the quadratic sub-pixel fit.
 *   d*  = argmin_d S (lowest d on ties), S1 = S(d*),
 *   S2  = min over |d-d*| >= 2 of S (-1 when no such d exists),
 *   valid_u iff u == 0 or S2 < 0 or 100*S1 <= (100-u)*S2,
 *   dsub = d* + (a-b) / (2(a+b)) with a = S(d*-1)-S1, b = S(d*+1)-S1 for
 *   0 < d* < D-1, else d*. */
void orc_wta(const uint32_t *S, int W, int H, int D, int uniqueness_pct, int subpixel,
             int32_t *dint, int32_t *s1, int32_t *s2, uint8_t *valid_u, double *dsub)
{
    for (size_t p = 0; p < (size_t)W * H; ++p) {
        const uint32_t *v = S + p * D;
        int best = 0;
        for (int d = 1; d < D; ++d)
            if (v[d] < v[best]) best = d;
        int64_t second = -1;
        for (int d = 0; d < D; ++d)
            if (abs(d - best) >= 2 && (second < 0 || v[d] < second)) second = v[d];
        dint[p] = best;
        s1[p] = (int32_t)v[best];
        s2[p] = (int32_t)second;
        valid_u[p] = (uint8_t)(uniqueness_pct == 0 || second < 0 ||
                               100 * (int64_t)v[best] <= (int64_t)(100 - uniqueness_pct) * second);
        double f = best;
        if (subpixel && best > 0 && best < D - 1) {
            double a = (double)v[best - 1] - (double)v[best];
            double b = (double)v[best + 1] - (double)v[best];
            f = best + (a - b) / (2.0 * (a + b));
        }
        dsub[p] = f;
    }
}

/* Right-image disparity read off the left-referenced volume:
 *   dR(xr) = argmin over 0 <= d <= min(D-1, W-1-xr) of S(xr+d, d), lowest d. */
void orc_right_disp(const uint32_t *S, int W, int H, int D, int32_t *dR)
{
    for (int y = 0; y < H; ++y)
        for (int xr = 0; xr < W; ++xr) {
            int best = 0;
            uint32_t bv = S[((size_t)y * W + xr) * D + 0];
            for (int d = 1; d < D && xr + d < W; ++d) {
                uint32_t v = S[((size_t)y * W + xr + d) * D + d];
                if (v < bv) { bv = v; best = d; }
            }
            dR[(size_t)y * W + xr] = best;
        }
}

/* Right-referenced matching cost: the right pixel xr against the left pixel
 * xr + d, CR[(y*W + xr)*D + d] = popcount(cR(xr,y) ^ cL(xr+d,y)), and the number
 * of census bits where xr + d > W-1. */
void orc_cost_right(const uint64_t *cl, const uint64_t *cr, int W, int H, int D, int bits, uint16_t *CR)
{
    for (int y = 0; y < H; ++y)
        for (int xr = 0; xr < W; ++xr)
            for (int d = 0; d < D; ++d) {
                int c = bits;
                if (xr + d <= W - 1) c = orc_popcount(cr[(size_t)y * W + xr] ^ cl[(size_t)y * W + xr + d]);
                CR[((size_t)y * W + xr) * D + d] = (uint16_t)c;
            }
}

/* Semi-global block matching cost (Sec. VI-D, the block-based cost mode, which
 * compares the neighbourhoods around the two pixels): the pixel costs summed over a bw x bh block
 * centred on the pixel, block samples outside the image clamped to the edge,
 *   CB(x,y,d) = sum_{|u|<=bw/2, |v|<=bh/2} C(clamp(x+u), clamp(y+v), d). */
void orc_block_cost(const uint16_t *C, int W, int H, int D, int bw, int bh, uint16_t *CB)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x)
            for (int d = 0; d < D; ++d) {
                int sum = 0;
                for (int v = -(bh / 2); v <= bh / 2; ++v)
                    for (int u = -(bw / 2); u <= bw / 2; ++u) {
                        int cx = clampi(x + u, 0, W - 1), cy = clampi(y + v, 0, H - 1);
                        sum += C[((size_t)cy * W + cx) * D + d];
                    }
                CB[((size_t)y * W + x) * D + d] = (uint16_t)sum;
            }
}

/* Right disparity from a full right-referenced SGM run: the right-referenced
 * cost (block-summed like the left one when bw x bh > 1) aggregated over the
 * same paths with the same penalties, then the winner of each right pixel
 * (lowest d on ties). */
void orc_right_disp_full(const uint64_t *cl, const uint64_t *cr, int W, int H, int D, int bits, int num_paths,
                         int P1, int P2, int bw, int bh, int32_t *dR)
{
    size_t n = (size_t)W * H * D;
    uint16_t *CR = (uint16_t *)malloc(n * sizeof(uint16_t));
    uint32_t *SR = (uint32_t *)malloc(n * sizeof(uint32_t));
    orc_cost_right(cl, cr, W, H, D, bits, CR);
    if (bw * bh > 1) {
        uint16_t *CB = (uint16_t *)malloc(n * sizeof(uint16_t));
        orc_block_cost(CR, W, H, D, bw, bh, CB);
        memcpy(CR, CB, n * sizeof(uint16_t));
        free(CB);
    }
    orc_aggregate(CR, W, H, D, num_paths, P1, P2, SR);
    for (size_t p = 0; p < (size_t)W * H; ++p) {
        int best = 0;
        for (int d = 1; d < D; ++d)
            if (SR[p * D + d] < SR[p * D + best]) best = d;
        dR[p] = best;
    }
    free(CR);
    free(SR);
}

/* Left-right consistency on integer disparities:
 *   valid iff lr < 0, or x - d* >= 0 and |d* - dR(x - d*)| <= lr. */
void orc_lr_check(const int32_t *dint, const int32_t *dR, int W, int H, int lr, uint8_t *valid_lr)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            int ok = 1;
            if (lr >= 0) {
                int xr = x - dint[p];
                ok = xr >= 0 && abs(dint[p] - dR[(size_t)y * W + xr]) <= lr;
            }
            valid_lr[p] = (uint8_t)ok;
        }
}

/* 3x3 median of the masked disparity map; the one-pixel border is copied. */
void orc_median3(const double *in, int W, int H, double *out)
{
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            if (x == 0 || y == 0 || x == W - 1 || y == H - 1) {
                out[p] = in[p];
                continue;
            }
            double v[9];
            int k = 0;
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) v[k++] = in[(size_t)(y + dy) * W + x + dx];
            for (int i = 1; i < 9; ++i) /* insertion sort */
                for (int j = i; j > 0 && v[j - 1] > v[j]; --j) {
                    double t = v[j]; v[j] = v[j - 1]; v[j - 1] = t;
                }
            out[p] = v[4];
        }
}

/* depth = f*B/d for d > 0, else 0. */
void orc_depth(const double *disp, int64_t count, double focal_px, double baseline_m, double *depth)
{
    double fb = focal_px * baseline_m;
    for (int64_t i = 0; i < count; ++i) depth[i] = disp[i] > 0.0 ? fb / disp[i] : 0.0;
}

/* ---------------------------------------------------------------- whole path */
typedef struct orc_params {
    int32_t width, height, max_disp;
    int32_t census_w, census_h, census_mode;
    int32_t p1, p2, uniqueness_pct, lr_max_diff, num_paths, median, subpixel;
    float focal_px, baseline_m;
    int32_t lr_mode; /* 0: right disparity read off the left volume; 1: full right-referenced run */
    int32_t block_w, block_h; /* matching block; 1 x 1 = SGM, larger = SGBM */
} orc_params;

typedef struct orc_result {
    uint64_t *census_l, *census_r; /* W*H */
    uint32_t *S;                   /* W*H*D (optional; NULL to skip keeping it) */
    int32_t *dint, *s1, *s2, *dright;
    uint8_t *flags;                /* bit0 uniqueness, bit1 LR, bit2 d*>0, bit3 final */
    double *dsub, *disp, *depth;   /* disp = after masking and median */
} orc_result;

/* The depth path of Sec. VI-D on a rectified, already-noised pair. */
int orc_sgm(const orc_params *pp, const uint8_t *left, const uint8_t *right, orc_result *r)
{
    int W = pp->width, H = pp->height, D = pp->max_disp;
    size_t npx = (size_t)W * H, nvol = npx * D;
    int bits = orc_census_bits(pp->census_w, pp->census_h, pp->census_mode);
    uint16_t *C = (uint16_t *)malloc(nvol * sizeof(uint16_t));
    int bw = pp->block_w > 0 ? pp->block_w : 1, bh = pp->block_h > 0 ? pp->block_h : 1;
    uint32_t *S = r->S ? r->S : (uint32_t *)malloc(nvol * sizeof(uint32_t));
    uint8_t *vu = (uint8_t *)malloc(npx), *vlr = (uint8_t *)malloc(npx);
    double *masked = (double *)malloc(npx * sizeof(double));
    if (!C || !S || !vu || !vlr || !masked) return -1;

    orc_census(left, W, H, W, pp->census_w, pp->census_h, pp->census_mode, r->census_l);
    orc_census(right, W, H, W, pp->census_w, pp->census_h, pp->census_mode, r->census_r);
    orc_cost(r->census_l, r->census_r, W, H, D, bits, C);
    if (bw * bh > 1) {
        uint16_t *CB = (uint16_t *)malloc(nvol * sizeof(uint16_t));
        if (!CB) return -1;
        orc_block_cost(C, W, H, D, bw, bh, CB);
        memcpy(C, CB, nvol * sizeof(uint16_t));
        free(CB);
    }
    orc_aggregate(C, W, H, D, pp->num_paths, pp->p1, pp->p2, S);
    orc_wta(S, W, H, D, pp->uniqueness_pct, pp->subpixel, r->dint, r->s1, r->s2, vu, r->dsub);
    if (pp->lr_mode == 1)
        orc_right_disp_full(r->census_l, r->census_r, W, H, D, bits, pp->num_paths, pp->p1, pp->p2, bw, bh,
                            r->dright);
    else
        orc_right_disp(S, W, H, D, r->dright);
    orc_lr_check(r->dint, r->dright, W, H, pp->lr_max_diff, vlr);
    for (size_t p = 0; p < npx; ++p) {
        int nz = r->dint[p] > 0;
        int ok = vu[p] && vlr[p] && nz;
        masked[p] = ok ? r->dsub[p] : 0.0;
        r->flags[p] = (uint8_t)(vu[p] | (vlr[p] << 1) | (nz << 2));
    }
    if (pp->median == 3)
        orc_median3(masked, W, H, r->disp);
    else
        memcpy(r->disp, masked, npx * sizeof(double));
    for (size_t p = 0; p < npx; ++p)
        if (r->disp[p] > 0.0) r->flags[p] |= 8;
    orc_depth(r->disp, (int64_t)npx, (double)pp->focal_px, (double)pp->baseline_m, r->depth);

    free(C);
    if (!r->S) free(S);
    free(vu);
    free(vlr);
    free(masked);
    return 0;
}
