/*
 * Seeded synthetic comment-text rows, the heavy part of the input generator.
 * It holds none of the codec arithmetic: it only draws words and lays out
 * rows.  Both the oracle tests and the GPU path consume what it writes.
 *
 * Row r draws from its own counter-based stream (splitmix64 keyed by the seed
 * and the row index), so any range of rows can be generated independently and
 * in parallel with the same result:
 *   T = 40 + (next() mod 71)                       target length in [40, 110]
 *   repeat: k = Zipf rank from one uniform draw (inverse CDF over `cdf`),
 *           append (a space, unless the row is empty) + word k,
 *   until the row holds at least T bytes; then append '\n'.
 */
#include <stdint.h>
#include <string.h>

static uint64_t splitmix64(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* uniform double in [0, 1) from the top 53 bits */
static double unit(uint64_t *s) { return (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0); }

/* Generate rows [row0, row1) into out (capacity cap).  Returns bytes written,
 * or -1 when cap is too small.  row_len (nullable) receives each row's length. */
int64_t zfgen_text_rows(uint64_t seed, const double *cdf, uint32_t K, const uint8_t *words,
                        const uint32_t *word_off, const uint32_t *word_len, uint64_t row0,
                        uint64_t row1, uint8_t *out, uint64_t cap) {
    uint64_t at = 0;
    for (uint64_t r = row0; r < row1; r++) {
        uint64_t st = seed * 0xD1B54A32D192ED03ull ^ (r + 1) * 0x9E3779B97F4A7C15ull;
        uint32_t T = 40 + (uint32_t)(splitmix64(&st) % 71u);
        uint32_t len = 0;
        while (len < T) {
            double u = unit(&st);
            uint32_t lo = 0, hi = K - 1; /* first k with cdf[k] > u */
            while (lo < hi) {
                uint32_t mid = lo + (hi - lo) / 2;
                if (cdf[mid] > u) hi = mid;
                else lo = mid + 1;
            }
            uint32_t wl = word_len[lo];
            if (at + len + wl + 2 > cap) return -1;
            if (len) out[at + len++] = ' ';
            memcpy(out + at + len, words + word_off[lo], wl);
            len += wl;
        }
        out[at + len++] = '\n';
        at += len;
    }
    return (int64_t)at;
}
