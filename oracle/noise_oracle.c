/*
 * CPU oracle of the on-device IR noise generator (Sec. VI-C: multiplicative
 * speckle gamma and additive thermal noise n, I' = gamma * I + n, Eq. (7); the
 * distributions of Eq. (8) and the fit of Sec. VII-C; the noise-scale knob of
 * Table X).  TEST INFRASTRUCTURE ONLY: nothing in the product path may link,
 * load or call it, and it shares no code with the GPU library.
 *
 * Random numbers come from one counter-based generator, Philox4x32-10 (Salmon,
 * Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11),
 * written here from its published definition; the GPU library implements the
 * same generator independently.  Per image pixel i and attempt a, the counter is
 * (i, stream, a, 0) and the key (seed low, seed high).  Conversions:
 *   uniform  u(x) = ((x >> 9) + 0.5) * 2^-23, exactly representable, in (0, 1);
 *   normal   Box-Muller in double, z = sqrt(-2 ln u0) * cos(2 pi u1);
 *   gamma    Marsaglia and Tsang (ACM TOMS 26(3), 2000) for shape k >= 1 in double:
 *            d = k - 1/3, c = 1 / sqrt(9 d); attempt a draws x (normal, words 0-1)
 *            and u (uniform, word 2); v = (1 + c x)^3; accept when v > 0 and
 *            ln u < x^2 / 2 + d - d v + d ln v; gamma = d v theta; at most 64
 *            attempts (then d theta).
 * Draws are rounded to float32.  gain models: 0 none (gamma = 1), 1 gamma(k,
 * theta), 2 normal(1, gain_sd^2); n ~ normal(mu, sigma^2) from the attempt
 * counter 0xFFFFFFFF.  Noise scale s: gamma' = 1 + s (gamma - 1), n' = s n, each
 * operation rounded to float32.
 */
#include <math.h>
#include <stdint.h>

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0], n1 = lo1, n2 = hi0 ^ c[3] ^ k[1], n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

/* Philox4x32 with 10 rounds: out = f(counter, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]}, k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

double orc_u01(uint32_t x) { return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0); }

static double box_muller(uint32_t a, uint32_t b)
{
    const double kTwoPi = 6.283185307179586476925286766559;
    return sqrt(-2.0 * log(orc_u01(a))) * cos(kTwoPi * orc_u01(b));
}

typedef struct orc_noise_params {
    int32_t gain_model; /* 0 none, 1 gamma(k, theta), 2 normal(1, gain_sd) */
    float k, theta, gain_sd, mu, sigma, scale;
    uint32_t seed_lo, seed_hi, stream;
} orc_noise_params;

/* The draws gamma', n' of `count` pixels. */
void orc_noise_draws(const orc_noise_params *p, int64_t count, float *gamma, float *n)
{
    const uint32_t key[2] = {p->seed_lo, p->seed_hi};
    for (int64_t i = 0; i < count; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, p->stream, 0u, 0u}, w[4];
        double g = 1.0;
        if (p->gain_model == 1) {
            const double d = (double)p->k - 1.0 / 3.0, c = 1.0 / sqrt(9.0 * d);
            g = d * (double)p->theta;
            for (uint32_t a = 0; a < 64; ++a) {
                ctr[2] = a;
                orc_philox4x32_10(ctr, key, w);
                const double x = box_muller(w[0], w[1]);
                double v = 1.0 + c * x;
                if (v <= 0.0) continue;
                v = v * v * v;
                if (log(orc_u01(w[2])) < 0.5 * x * x + d - d * v + d * log(v)) {
                    g = d * v * (double)p->theta;
                    break;
                }
            }
        } else if (p->gain_model == 2) {
            ctr[2] = 0;
            orc_philox4x32_10(ctr, key, w);
            g = 1.0 + (double)p->gain_sd * box_muller(w[0], w[1]);
        }
        ctr[2] = 0xFFFFFFFFu;
        orc_philox4x32_10(ctr, key, w);
        const float nz = (float)((double)p->mu + (double)p->sigma * box_muller(w[0], w[1]));
        volatile float gf = (float)g;
        volatile float gm1 = gf - 1.0f;
        volatile float sg = p->scale * gm1;
        gamma[i] = 1.0f + sg;
        n[i] = p->scale * nz;
    }
}
