/*
 * Seeded synthetic star-schema columns.
 *
 * This module is shared input plumbing: it draws random columns and nothing
 * else.  It holds none of the filter / join / aggregation arithmetic, so both
 * the HIP path and the CPU oracle can consume its buffers without sharing any
 * of the method's code.
 *
 * Generator: counter-based SplitMix64.  Every value is a pure function of
 * (seed, column id, row), so any slice of a column can be produced
 * independently and in parallel, and the same (seed, column, row) always
 * yields the same value.
 *
 *   stream(seed, col) = mix(seed * G + mix(col + C0))
 *   draw(seed, col, row) = mix(stream(seed, col) + (row + 1) * G)
 *
 * with G = 0x9E3779B97F4A7C15 (the SplitMix64 increment) and mix() the
 * SplitMix64 output finaliser (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).
 *
 * A uniform integer in [lo, hi) is lo + floor(draw * (hi - lo) / 2^64)
 * (multiply-high); the bias is below 2^-40 for every range used here and is
 * irrelevant to parity, because both sides read the same buffers.
 */
#include <stdint.h>
#include <math.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t col) {
    return mix64(seed * GOLDEN + mix64(col + 0x632BE59BD9B4E019ULL));
}

static inline uint64_t draw(uint64_t key, uint64_t row) {
    return mix64(key + (row + 1) * GOLDEN);
}

static inline int64_t in_range(uint64_t r, int64_t lo, int64_t hi) {
    uint64_t span = (uint64_t)(hi - lo);
    return lo + (int64_t)(uint64_t)(((unsigned __int128)r * span) >> 64);
}

uint64_t tqpgen_draw(uint64_t seed, uint64_t col, int64_t row) {
    return draw(stream_key(seed, col), (uint64_t)row);
}

/* Uniform double in [0, 1) with 53 random bits. */
double tqpgen_unit(uint64_t seed, uint64_t col, int64_t row) {
    return (double)(tqpgen_draw(seed, col, row) >> 11) * (1.0 / 9007199254740992.0);
}

void tqpgen_i32(uint64_t seed, uint64_t col, int64_t row0, int64_t n,
                int64_t lo, int64_t hi, int32_t* out) {
    uint64_t key = stream_key(seed, col);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = (int32_t)in_range(draw(key, (uint64_t)(row0 + i)), lo, hi);
}

void tqpgen_i64(uint64_t seed, uint64_t col, int64_t row0, int64_t n,
                int64_t lo, int64_t hi, int64_t* out) {
    uint64_t key = stream_key(seed, col);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = in_range(draw(key, (uint64_t)(row0 + i)), lo, hi);
}

void tqpgen_i8(uint64_t seed, uint64_t col, int64_t row0, int64_t n,
               int64_t lo, int64_t hi, int8_t* out) {
    uint64_t key = stream_key(seed, col);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = (int8_t)in_range(draw(key, (uint64_t)(row0 + i)), lo, hi);
}

/* A seeded permutation of 0..n-1 (Fisher-Yates, Durstenfeld form): for
 * i = n-1 down to 1, swap a[i] with a[j], j uniform in [0, i]. */
void tqpgen_perm_i32(uint64_t seed, uint64_t col, int64_t n, int32_t* out) {
    uint64_t key = stream_key(seed, col);
    for (int64_t i = 0; i < n; ++i) out[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = in_range(draw(key, (uint64_t)i), 0, i + 1);
        int32_t t = out[i];
        out[i] = out[j];
        out[j] = t;
    }
}
