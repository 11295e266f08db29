/*
 * Seeded synthetic inputs for the block lower-triangular Toeplitz workloads.
 *
 * This module holds no arithmetic of the matvec method: it only draws the
 * numbers that both the HIP path and the oracle consume.  Every value is a
 * pure function of (seed, stream, index), so any entry can be regenerated on
 * its own (counter-based generation).
 *
 * Raw 64-bit values come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): the output
 * function is the published mix64 finaliser applied to a Weyl sequence with
 * increment gamma = 0x9E3779B97F4A7C15.
 *   key(seed, stream) = mix64(seed + gamma * (stream + 1))
 *   raw(n)            = mix64(key + gamma * (n + 1))
 *   unif(n)           = ((raw(n) >> 11) + 0.5) * 2^-53       in (0, 1)
 * Standard normals use the Box-Muller transform on a pair of uniforms
 * (the cosine branch only):
 *   normal(i) = sqrt(-2 ln unif(2i)) * cos(2 pi unif(2i+1)).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define SM_GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t stream)
{
    return mix64(seed + SM_GAMMA * (stream + 1));
}

static inline double unif(uint64_t key, uint64_t n)
{
    uint64_t r = mix64(key + SM_GAMMA * (n + 1));
    return ((double)(r >> 11) + 0.5) * 0x1.0p-53;
}

static inline double normal_at(uint64_t key, uint64_t i)
{
    const double two_pi = 6.283185307179586476925286766559;
    double a = unif(key, 2 * i), b = unif(key, 2 * i + 1);
    return sqrt(-2.0 * log(a)) * cos(two_pi * b);
}

/* out[i] = normal(offset + i) for i < count */
void synth_normal(uint64_t seed, uint64_t stream, uint64_t offset, int64_t count, double *out)
{
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = normal_at(key, offset + (uint64_t)i);
}

/* out[i] = (float) normal(offset + i) */
void synth_normal_f32(uint64_t seed, uint64_t stream, uint64_t offset, int64_t count, float *out)
{
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = (float)normal_at(key, offset + (uint64_t)i);
}

/* out[i] = unif(offset + i) */
void synth_uniform(uint64_t seed, uint64_t stream, uint64_t offset, int64_t count, double *out)
{
    uint64_t key = stream_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = unif(key, offset + (uint64_t)i);
}

/*
 * First block column of the operator, time-outer: out[k][s][p] for
 * k < nt, s < nd, p < nm, equal to normal((k*nd + s)*nm + p) * exp(-k/tau).
 * tau <= 0 means no decay.  Rows [k0, k0+nk) only, written from out[0].
 */
void synth_blocks(uint64_t seed, uint64_t stream, int64_t nt, int64_t nd, int64_t nm,
                  double tau, int64_t k0, int64_t nk, double *out)
{
    uint64_t key = stream_key(seed, stream);
    int64_t per = nd * nm;
    (void)nt;
#pragma omp parallel for schedule(static) collapse(2)
    for (int64_t kk = 0; kk < nk; ++kk)
        for (int64_t e = 0; e < per; ++e) {
            int64_t k = k0 + kk;
            double w = tau > 0 ? exp(-(double)k / tau) : 1.0;
            out[kk * per + e] = normal_at(key, (uint64_t)(k * per + e)) * w;
        }
}
