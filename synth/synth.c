/*
 * Seeded, counter-based synthetic inputs shaped like the Gaia AVU-GSR
 * observation matrix (Section 3 of the paper: every row holds 5 astrometric,
 * 3x4 attitude, 6 instrumental and 1 global coefficient, rows sorted by star).
 *
 * This file draws random numbers and nothing else: star assignment, attitude
 * start index, instrumental column indices, coefficient values, a "true"
 * solution vector and observation noise.  It contains no part of the solver's
 * arithmetic (no products with the matrix, no norms, no LSQR); the right-hand
 * side b = A x_true + e is formed by whoever consumes these arrays.
 *
 * Generator: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) used as a counter-based generator: draw
 * number i of stream key K is mix64(K + (i + 1) * GAMMA), where mix64 is the
 * SplitMix64 output function.  Every value therefore depends only on
 * (seed, stream, index), so any row range can be generated independently and
 * in parallel with bit-identical results.
 *
 *   uniform(K, i)  = (draw(K, i) >> 11) * 2^-53                in [0, 1)
 *   normal(K, i)   = Box-Muller (cosine branch) of the two uniforms
 *                    u1 = ((draw(K, 2i) >> 11) + 1) * 2^-53     in (0, 1]
 *                    u2 =  (draw(K, 2i+1) >> 11) * 2^-53
 *                    sqrt(-2 ln u1) * cos(2 pi u2)
 *   below(K, i, k) = floor(draw(K, i) * k / 2^64)              in [0, k)
 *
 * Built with plain gcc; OpenMP only splits independent index ranges.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SYN_GAMMA 0x9E3779B97F4A7C15ULL

enum {
    SYN_STREAM_VALS = 1,
    SYN_STREAM_ATT = 2,
    SYN_STREAM_INSTR = 3,
    SYN_STREAM_XTRUE = 4,
    SYN_STREAM_NOISE = 5,
    SYN_STREAM_OBS = 6,
    SYN_STREAM_XREF = 7,
    SYN_STREAM_STARS = 8,
    SYN_STREAM_PRIMARY = 9,     /* selection of the stars the constraint rows touch */
    SYN_STREAM_CON_VALS = 10,   /* coefficients of the constraint rows              */
    SYN_STREAM_RHS_X = 64,      /* + j for right-hand side j   */
    SYN_STREAM_RHS_NOISE = 4096 /* + j for right-hand side j   */
};

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t key, uint64_t i)
{
    return mix64(key + (i + 1) * SYN_GAMMA);
}

uint64_t syn_key(uint64_t seed, uint64_t stream)
{
    return mix64(mix64(seed + SYN_GAMMA) ^ (stream * 0xD1B54A32D192ED03ULL));
}

uint64_t syn_draw(uint64_t key, uint64_t i) { return draw(key, i); }

double syn_uniform(uint64_t key, uint64_t i)
{
    return (double)(draw(key, i) >> 11) * 0x1.0p-53;
}

double syn_normal(uint64_t key, uint64_t i)
{
    const double u1 = (double)((draw(key, 2 * i) >> 11) + 1) * 0x1.0p-53;
    const double u2 = (double)(draw(key, 2 * i + 1) >> 11) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

uint32_t syn_below(uint64_t key, uint64_t i, uint32_t k)
{
    return (uint32_t)(((unsigned __int128)draw(key, i) * k) >> 64);
}

/* Fill out[i] = normal(key(seed, stream), first + i) * scale for i < count. */
void syn_fill_normal(uint64_t seed, uint64_t stream, int64_t first, int64_t count,
                     double scale, double *out)
{
    const uint64_t key = syn_key(seed, stream);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = scale * syn_normal(key, (uint64_t)(first + i));
}

/* Observations per star: obs_lo + below(key, s, obs_hi - obs_lo + 1). */
void syn_star_counts(uint64_t seed, int64_t n_stars, int32_t obs_lo, int32_t obs_hi,
                     int32_t *counts)
{
    const uint64_t key = syn_key(seed, SYN_STREAM_OBS);
    const uint32_t span = (uint32_t)(obs_hi - obs_lo + 1);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < n_stars; ++s)
        counts[s] = (obs_hi == obs_lo) ? obs_lo
                                       : obs_lo + (int32_t)syn_below(key, (uint64_t)s, span);
}

/*
 * Rows [row_begin, row_end) of a system with n_dfa attitude degrees of freedom
 * per axis and n_instr instrumental columns:
 *   att[r]      = below(ATT, r, n_dfa - 3)      attitude start t in [0, n_dfa-4]
 *   instr[r*6+j]= 6 distinct draws below(INSTR, r*64 + c, n_instr), c = 0,1,...
 *                 (rejection of repeats), stored in ascending order
 *   vals[r*24+k]= normal(VALS, r*24 + k)
 * Output arrays are indexed from row_begin (i.e. att[0] is row row_begin).
 * Any of the output pointers may be NULL to skip that array.
 */
void syn_rows(uint64_t seed, int32_t n_dfa, int32_t n_instr, int64_t row_begin, int64_t row_end,
              int32_t *att, int32_t *instr, double *vals)
{
    const uint64_t k_att = syn_key(seed, SYN_STREAM_ATT);
    const uint64_t k_ins = syn_key(seed, SYN_STREAM_INSTR);
    const uint64_t k_val = syn_key(seed, SYN_STREAM_VALS);
    const int64_t count = row_end - row_begin;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < count; ++q) {
        const int64_t r = row_begin + q;
        if (att)
            att[q] = (int32_t)syn_below(k_att, (uint64_t)r, (uint32_t)(n_dfa - 3));
        if (instr) {
            int32_t got[6];
            int n = 0;
            for (int c = 0; c < 64 && n < 6; ++c) {
                const int32_t cand =
                    (int32_t)syn_below(k_ins, (uint64_t)r * 64u + (uint64_t)c, (uint32_t)n_instr);
                int dup = 0;
                for (int e = 0; e < n; ++e)
                    dup |= (got[e] == cand);
                if (!dup)
                    got[n++] = cand;
            }
            /* 64 draws without 6 distinct values: complete with the smallest unused. */
            for (int32_t cand = 0; n < 6; ++cand) {
                int dup = 0;
                for (int e = 0; e < n; ++e)
                    dup |= (got[e] == cand);
                if (!dup)
                    got[n++] = cand;
            }
            for (int a = 1; a < 6; ++a) { /* insertion sort, ascending */
                const int32_t v = got[a];
                int b = a - 1;
                while (b >= 0 && got[b] > v) {
                    got[b + 1] = got[b];
                    --b;
                }
                got[b + 1] = v;
            }
            memcpy(instr + q * 6, got, sizeof got);
        }
        if (vals) {
            double *dst = vals + q * 24;
            for (int k = 0; k < 24; ++k)
                dst[k] = syn_normal(k_val, (uint64_t)r * 24u + (uint64_t)k);
        }
    }
}

/* Star number of rows [row_begin, row_end) given per-star row offsets
 * (row_ptr[s] = first row of star s, row_ptr[n_stars] = n_rows). */
void syn_star_of_rows(const int64_t *row_ptr, int64_t n_stars, int64_t row_begin, int64_t row_end,
                      int32_t *star)
{
    int64_t lo = 0, hi = n_stars; /* first star whose range contains row_begin */
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (row_ptr[mid + 1] <= row_begin)
            lo = mid + 1;
        else
            hi = mid;
    }
    int64_t s = lo;
    for (int64_t r = row_begin; r < row_end; ++r) {
        while (row_ptr[s + 1] <= r)
            ++s;
        star[r - row_begin] = (int32_t)s;
    }
}

/* Stars selected for the constraint rows: star s is selected when
 * uniform(PRIMARY, s) < frac.  Writes the selected star numbers (ascending) to
 * `out` when it is not NULL; returns how many there are. */
int64_t syn_primary_stars(uint64_t seed, int64_t n_stars, double frac, int32_t *out)
{
    const uint64_t key = syn_key(seed, SYN_STREAM_PRIMARY);
    int64_t n = 0;
    for (int64_t s = 0; s < n_stars; ++s)
        if (syn_uniform(key, (uint64_t)s) < frac) {
            if (out)
                out[n] = (int32_t)s;
            ++n;
        }
    return n;
}
