/*
 * zfo.c -- the oracle (test infrastructure only; see zfo.h).
 *
 * Plain C99, single-threaded, no SIMD, no cleverness.  Every stream is built
 * and read one field at a time with byte-wise little-endian helpers and a
 * bit-at-a-time packer, so each function can be checked against its
 * definition by eye.
 *
 * ---------------------------------------------------------------- container
 * Column blob, all integers little-endian:
 *   [0,64)   header: "ZFC1", u16 version=1, u8 dtype, u8 codec (0 if the
 *            chunks mix codecs), u64 n_elems, u64 plain_bytes, u32 n_chunks,
 *            u32 dict_count, u64 dict_off, u64 total_bytes, u32 table_crc,
 *            u32 0, u32 0, u32 header_crc (CRC-32 of bytes [0,60)).
 *   [64, 64+32*n_chunks)  chunk table, one 32-byte entry per chunk:
 *            u64 plain_off, u64 comp_off, u32 plain_len, u32 comp_len,
 *            u32 n_elems, u8 codec, u8 schedule hint (a tile choice for the
 *            decoder; the decoded bytes do not depend on it; this encoder
 *            writes 0), 2 zero bytes.
 *   dictionary (when dict_count > 0) at dict_off = align16(end of table):
 *            dict_count entries of elem_size bytes, sorted ascending and
 *            unique (integers by signed value, FIXED16 by memcmp).
 *   chunk streams, each at a 16-aligned comp_off, in chunk order; the gap
 *            bytes are zero; total_bytes = align16(end of the last stream).
 *   table_crc = CRC-32 over the chunk table followed by the dictionary.
 *
 * The codec streams are described above their encoders below.
 */
#include "zfo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define FOR_BLOCK 2048u /* values per FOR / bit-packing block */
#define RLE_GROUP 64u   /* runs per RLE group record */
#define LZ_MAX_CHUNK 65536u
#define LZ_HASH_BITS 16
#define LZ_CHAIN 16

/* ------------------------------------------------------------ byte helpers */
static void put8(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; }
static void put16(uint8_t *p, uint32_t v) { p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); }
static void put32(uint8_t *p, uint32_t v) {
    for (int i = 0; i < 4; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static void put64(uint8_t *p, uint64_t v) {
    for (int i = 0; i < 8; i++) p[i] = (uint8_t)(v >> (8 * i));
}
static uint32_t get16(const uint8_t *p) { return (uint32_t)p[0] | ((uint32_t)p[1] << 8); }
static uint32_t get32(const uint8_t *p) {
    uint32_t v = 0;
    for (int i = 0; i < 4; i++) v |= (uint32_t)p[i] << (8 * i);
    return v;
}
static uint64_t get64(const uint8_t *p) {
    uint64_t v = 0;
    for (int i = 0; i < 8; i++) v |= (uint64_t)p[i] << (8 * i);
    return v;
}
static uint64_t align16(uint64_t x) { return (x + 15u) & ~(uint64_t)15u; }

/* ---------------------------------------------------------------- CRC-32 */
/* IEEE 802.3 CRC-32 (reflected polynomial 0xEDB88320, initial value and final
 * xor 0xFFFFFFFF), computed one bit at a time from its definition. */
uint32_t zfo_crc32(const uint8_t *p, uint64_t n) {
    uint32_t c = 0xFFFFFFFFu;
    for (uint64_t i = 0; i < n; i++) {
        c ^= p[i];
        for (int k = 0; k < 8; k++) c = (c & 1u) ? (c >> 1) ^ 0xEDB88320u : (c >> 1);
    }
    return c ^ 0xFFFFFFFFu;
}

uint32_t zfo_elem_size(uint32_t dtype) {
    switch (dtype) {
    case ZFO_I32: return 4;
    case ZFO_I64: return 8;
    case ZFO_BYTES: return 1;
    case ZFO_FIXED16: return 16;
    case ZFO_F64: return 8;
    default: return 0;
    }
}

/* number of bits needed to write v; bitlen(0) = 0 */
static uint32_t bitlen64(uint64_t v) {
    uint32_t n = 0;
    while (v) { n++; v >>= 1; }
    return n;
}

/* width of the integer type in bits (32 for I32, 64 for I64) */
static uint32_t int_bits(uint32_t dtype) { return dtype == ZFO_I32 ? 32u : 64u; }
static uint64_t mask_bits(uint32_t w) { return w >= 64 ? ~(uint64_t)0 : (((uint64_t)1 << w) - 1); }

/* read element j of an integer column as a two's complement value held in
 * 64 bits (I32 is sign-extended) */
static int64_t load_int(const uint8_t *p, uint32_t dtype, uint64_t j) {
    if (dtype == ZFO_I32) return (int64_t)(int32_t)get32(p + 4 * j);
    return (int64_t)get64(p + 8 * j);
}
static void store_int(uint8_t *p, uint32_t dtype, uint64_t j, uint64_t v) {
    if (dtype == ZFO_I32) put32(p + 4 * j, (uint32_t)v);
    else put64(p + 8 * j, v);
}

/* ------------------------------------------------------------ growing buffer */
typedef struct { uint8_t *p; uint64_t n, cap; int bad; } buf_t;
static void buf_reserve(buf_t *b, uint64_t need) {
    if (b->bad || need <= b->cap) return;
    uint64_t cap = b->cap ? b->cap : 256;
    while (cap < need) cap *= 2;
    uint8_t *q = (uint8_t *)realloc(b->p, cap);
    if (!q) { b->bad = 1; return; }
    memset(q + b->cap, 0, cap - b->cap);
    b->p = q;
    b->cap = cap;
}
/* grow to length n (new bytes are zero) */
static void buf_resize(buf_t *b, uint64_t n) {
    buf_reserve(b, n);
    if (!b->bad && n > b->n) b->n = n;
}

/* ------------------------------------------------------------- bit packing */
/* The packed stream is a sequence of little-endian u32 words; stream bit k is
 * bit (k mod 32) of word floor(k/32).  Field j of width w occupies stream bits
 * [j*w, j*w + w), least significant bit first (Sec. 2.1, bit-packing).
 * Both directions go one bit at a time. */
static void pack_bits(uint8_t *words, uint64_t j, uint32_t w, uint64_t v) {
    for (uint32_t k = 0; k < w; k++) {
        uint64_t bit = (uint64_t)j * w + k;
        if ((v >> k) & 1u) words[4 * (bit / 32) + (bit % 32) / 8] |= (uint8_t)(1u << (bit % 8));
    }
}
static uint64_t unpack_bits(const uint8_t *words, uint64_t j, uint32_t w) {
    uint64_t v = 0;
    for (uint32_t k = 0; k < w; k++) {
        uint64_t bit = (uint64_t)j * w + k;
        uint64_t b = (words[4 * (bit / 32) + (bit % 32) / 8] >> (bit % 8)) & 1u;
        v |= b << k;
    }
    return v;
}
static uint64_t packed_words(uint64_t nfields, uint32_t w) { return (nfields * w + 31) / 32; }

/* ============================================================== FOR + BP
 * Frame of reference plus bit-packing (Sec. 2.1: the reference is the block
 * minimum and the width follows from the minimum and maximum).
 * Stream for a chunk of n values, B = 2048, nb = ceil(n/B) blocks:
 *   block directory, 16 bytes per block at offset 16*b:
 *       i64 ref (the block minimum; I32 sign-extended), u32 w, u32 poff
 *   payload of block b at byte offset poff (16-aligned): the fields
 *       d_j = x_j - ref (mod 2^bits), packed at width w = bitlen(max d).
 *   poff_0 = align16(16*nb), poff_{b+1} = align16(poff_b + 4*words_b);
 *   comp_len = poff_last + 4*words_last.
 * Decode: x_j = ref + field_j (mod 2^bits). */
static void enc_for_bp(buf_t *s, const uint8_t *x, uint32_t dtype, uint32_t n) {
    uint32_t nb = (n + FOR_BLOCK - 1) / FOR_BLOCK;
    uint64_t mask = mask_bits(int_bits(dtype));
    uint64_t pos = align16((uint64_t)16 * nb);
    buf_resize(s, pos);
    uint64_t end = pos;
    for (uint32_t b = 0; b < nb && !s->bad; b++) {
        uint32_t j0 = b * FOR_BLOCK, nv = n - j0 < FOR_BLOCK ? n - j0 : FOR_BLOCK;
        int64_t ref = load_int(x, dtype, j0);
        for (uint32_t j = 1; j < nv; j++) {
            int64_t v = load_int(x, dtype, j0 + j);
            if (v < ref) ref = v;
        }
        uint64_t dmax = 0;
        for (uint32_t j = 0; j < nv; j++) {
            uint64_t d = ((uint64_t)load_int(x, dtype, j0 + j) - (uint64_t)ref) & mask;
            if (d > dmax) dmax = d;
        }
        uint32_t w = bitlen64(dmax);
        uint64_t nw = packed_words(nv, w);
        buf_resize(s, pos + 4 * nw);
        if (s->bad) return;
        put64(s->p + 16 * (uint64_t)b, (uint64_t)ref);
        put32(s->p + 16 * (uint64_t)b + 8, w);
        put32(s->p + 16 * (uint64_t)b + 12, (uint32_t)pos);
        for (uint32_t j = 0; j < nv; j++) {
            uint64_t d = ((uint64_t)load_int(x, dtype, j0 + j) - (uint64_t)ref) & mask;
            pack_bits(s->p + pos, j, w, d);
        }
        end = pos + 4 * nw;
        pos = align16(end);
    }
    s->n = end;
}

/* Decode FOR+BP into 64-bit unsigned values (the caller narrows). */
static int dec_for_bp_u64(const uint8_t *s, uint64_t comp_len, uint32_t n, uint32_t bits,
                          uint64_t *out) {
    uint32_t nb = (n + FOR_BLOCK - 1) / FOR_BLOCK;
    if ((uint64_t)16 * nb > comp_len) return ZFO_ECORRUPT;
    uint64_t mask = mask_bits(bits);
    for (uint32_t b = 0; b < nb; b++) {
        uint32_t j0 = b * FOR_BLOCK, nv = n - j0 < FOR_BLOCK ? n - j0 : FOR_BLOCK;
        uint64_t ref = get64(s + 16 * (uint64_t)b);
        uint32_t w = get32(s + 16 * (uint64_t)b + 8);
        uint64_t poff = get32(s + 16 * (uint64_t)b + 12);
        if (w > bits || poff % 16 != 0 || poff < (uint64_t)16 * nb) return ZFO_ECORRUPT;
        if (poff + 4 * packed_words(nv, w) > comp_len) return ZFO_ECORRUPT;
        for (uint32_t j = 0; j < nv; j++)
            out[j0 + j] = (ref + unpack_bits(s + poff, j, w)) & mask;
    }
    return ZFO_OK;
}

/* =================================================================== ANS
 * Asymmetric numeral systems (Sec. 2.1: entropy coding; Sec. 3.1: a serial
 * state machine per chunk), here range ANS over the chunk's bytes with a
 * static order-0 model, the byte sequence dealt round-robin to 64 interleaved
 * coders (byte i to coder i mod 64), each with its own 32-bit state.
 * Model: M = 4096 (12 bits).  For byte counts c_s over the chunk's n bytes,
 *   f_s = 0 if c_s = 0, else max(1, floor(c_s * M / n));
 *   if sum f < M: the byte with the largest count (ties: the smallest byte)
 *       gets the difference;
 *   while sum f > M: the byte with the largest f (ties: the smallest byte)
 *       loses one;
 *   cum_s = sum of f_t for t < s.
 * Coder (state x in [L, L * 2^16), L = 2^16), one step per byte:
 *   encode byte s: while x >= 2^20 * f_s: emit the low 16 bits of x;
 *       x = x >> 16; then x = floor(x / f_s) * M + (x mod f_s) + cum_s;
 *   decode: slot = x mod M, s = the byte with cum_s <= slot < cum_s + f_s,
 *       x = f_s * floor(x / M) + slot - cum_s, then while x < L:
 *       x = x * 2^16 + the next 16-bit word.
 * The 64 coders share one word stream.  Decoding takes the bytes in order
 * i = 0, 1, ..., n-1, byte i by coder i mod 64, and each renormalisation
 * reads the next word of the stream; encoding takes the bytes in the reverse
 * order (i = n-1 down to 0), every coder starting from x = L, and the stream
 * is its emitted words reversed.  A valid stream leaves every coder at x = L
 * with every word read.
 * Stream of a chunk of n bytes:
 *   u32 n, u32 nw (16-bit words), u32 0, u32 0; u16 f[256];
 *   u32 state[64] (coder j's state after encoding, where decoding starts);
 *   u16 words[nw] at byte 784, in the order the decoder reads them.
 *   comp_len = 784 + 2*nw. */
#define ANS_M 4096u
#define ANS_L 65536u
#define ANS_LANES 64u
#define ANS_HDR 784u

static void ans_model(const uint8_t *x, uint32_t n, uint32_t f[256]) {
    uint64_t c[256] = {0};
    for (uint32_t i = 0; i < n; i++) c[x[i]]++;
    uint32_t sum = 0;
    for (int s = 0; s < 256; s++) {
        f[s] = 0;
        if (c[s]) {
            uint64_t q = c[s] * ANS_M / n;
            f[s] = q ? (uint32_t)q : 1u;
        }
        sum += f[s];
    }
    if (sum < ANS_M) {
        int best = -1;
        for (int s = 0; s < 256; s++)
            if (c[s] && (best < 0 || c[s] > c[best])) best = s;
        f[best] += ANS_M - sum;
        sum = ANS_M;
    }
    while (sum > ANS_M) {
        int best = -1;
        for (int s = 0; s < 256; s++)
            if (f[s] > 1 && (best < 0 || f[s] > f[best])) best = s;
        f[best]--;
        sum--;
    }
}

static void enc_ans(buf_t *s, const uint8_t *x, uint32_t n) {
    uint32_t f[256], cum[256];
    ans_model(x, n, f);
    cum[0] = 0;
    for (int t = 1; t < 256; t++) cum[t] = cum[t - 1] + f[t - 1];
    /* emitted words in emission order; a byte emits at most one word (after
     * one shift x < 2^16 <= 2^20 * f) */
    uint16_t *em = (uint16_t *)malloc(sizeof(uint16_t) * ((uint64_t)n + 1));
    uint64_t state[ANS_LANES], nw = 0;
    if (!em) { s->bad = 1; return; }
    for (uint32_t j = 0; j < ANS_LANES; j++) state[j] = ANS_L;
    for (int64_t i = (int64_t)n - 1; i >= 0; i--) {
        uint64_t *xs = &state[i % ANS_LANES];
        uint32_t sy = x[i];
        uint64_t xmax = ((uint64_t)(ANS_L >> 12) << 16) * f[sy];
        while (*xs >= xmax) {
            em[nw++] = (uint16_t)(*xs & 0xFFFFu);
            *xs >>= 16;
        }
        *xs = (*xs / f[sy]) * ANS_M + (*xs % f[sy]) + cum[sy];
    }
    buf_resize(s, ANS_HDR + 2 * nw);
    if (!s->bad) {
        put32(s->p, n);
        put32(s->p + 4, (uint32_t)nw);
        for (int t = 0; t < 256; t++) put16(s->p + 16 + 2 * t, f[t]);
        for (uint32_t j = 0; j < ANS_LANES; j++) put32(s->p + 528 + 4 * j, (uint32_t)state[j]);
        for (uint64_t k = 0; k < nw; k++) put16(s->p + ANS_HDR + 2 * k, em[nw - 1 - k]);
    }
    free(em);
}

static int dec_ans(const uint8_t *s, uint64_t comp_len, uint32_t n, uint8_t *out) {
    if (comp_len < ANS_HDR) return ZFO_ECORRUPT;
    uint64_t nw = get32(s + 4);
    if (get32(s) != n || ANS_HDR + 2 * nw != comp_len) return ZFO_ECORRUPT;
    uint32_t f[256], cum[256], sum = 0;
    for (int t = 0; t < 256; t++) {
        f[t] = get16(s + 16 + 2 * t);
        cum[t] = sum;
        sum += f[t];
    }
    if (sum != ANS_M) return ZFO_ECORRUPT;
    uint64_t state[ANS_LANES], w = 0;
    for (uint32_t j = 0; j < ANS_LANES; j++) state[j] = get32(s + 528 + 4 * j);
    for (uint64_t i = 0; i < n; i++) {
        uint64_t *xs = &state[i % ANS_LANES];
        uint32_t slot = (uint32_t)(*xs % ANS_M), sy = 0;
        while (!(cum[sy] <= slot && slot < cum[sy] + f[sy])) sy++;
        *xs = f[sy] * (*xs / ANS_M) + slot - cum[sy];
        while (*xs < ANS_L) {
            if (w >= nw) return ZFO_ECORRUPT;
            *xs = (*xs << 16) | get16(s + ANS_HDR + 2 * w++);
        }
        out[i] = (uint8_t)sy;
    }
    for (uint32_t j = 0; j < ANS_LANES; j++)
        if (state[j] != ANS_L) return ZFO_ECORRUPT;
    return w == nw ? ZFO_OK : ZFO_ECORRUPT;
}

/* ============================================================= Float2Int
 * Decimal floating point to integers (Sec. 2.1 names Float2Int: significant
 * digits and exponent split into integers; it fixes no layout, so this one is
 * the zf format's).  In block b a float64 value v is represented by the
 * integer d with
 *     bits(v) == bits((double)d / 10^e_b)
 * (IEEE binary64 division, round to nearest even; 10^e exact for e <= 18;
 * (double)d the round-to-nearest conversion of the int64 d).  Values with no
 * such d -- NaN, infinities, -0.0, more digits than e_b allows, magnitudes of
 * 2^62 * 10^-e_b or more -- are exceptions, stored raw.  The d of a block are
 * then FOR + bit-packed (Float2Int nested with bit-packing, Table 2).
 * Stream for a chunk of n values, B = 2048, nb = ceil(n/B) blocks:
 *   block directory, 32 bytes per block at offset 32*b:
 *       i64 ref, u32 w, u32 poff, u32 xoff, u16 nx, u8 e, u8 0, 8 zero bytes
 *   payload at poff (16-aligned): field_j = d_j - ref packed at width w, an
 *       exception holding field 0;
 *   exceptions at xoff (16-aligned): nx records of 16 bytes
 *       {u32 j (index in the block, strictly increasing), u32 0, u64 bits};
 *   blocks in order, each its payload then its exceptions;
 *   poff_0 = align16(32*nb); xoff_b = align16(poff_b + 4*words_b);
 *   poff_{b+1} = align16(xoff_b + 16*nx_b); comp_len = xoff_last + 16*nx_last.
 * The encoder's choice of e_b: for e = 0..18 every value gets
 * d = nearbyint(v * 10^e) when |v * 10^e| < 2^62 and the round trip above
 * holds, else it is an exception; cost(e) = nv*w(e) + 128*nx(e) bits, where
 * w(e) is the bit length of max(d) - min(d) over the non-exceptions; the
 * smallest cost wins, ties going to the smaller e; ref = min(d) (0 when every
 * value is an exception).
 * Decode: x_j = bits of (double)(int64)(ref + field_j) / 10^e, then every
 * exception record overwrites its x_j. */
static const double F2I_P10[19] = {1e0,  1e1,  1e2,  1e3,  1e4,  1e5,  1e6,  1e7,  1e8, 1e9,
                                   1e10, 1e11, 1e12, 1e13, 1e14, 1e15, 1e16, 1e17, 1e18};
#define F2I_EMAX 18u

static uint64_t f64_bits(double v) {
    uint64_t b;
    memcpy(&b, &v, 8);
    return b;
}
static double f64_from(uint64_t b) {
    double v;
    memcpy(&v, &b, 8);
    return v;
}

/* the d of value bits b at exponent e, if it round-trips */
static int f2i_digits(uint64_t b, uint32_t e, int64_t *d) {
    double m = f64_from(b) * F2I_P10[e];
    if (!(fabs(m) < 4611686018427387904.0)) return 0; /* 2^62; false for NaN */
    int64_t k = (int64_t)nearbyint(m);
    if (f64_bits((double)k / F2I_P10[e]) != b) return 0;
    *d = k;
    return 1;
}

static void enc_f2i_bp(buf_t *s, const uint8_t *x, uint32_t n) {
    uint32_t nb = (n + FOR_BLOCK - 1) / FOR_BLOCK;
    uint64_t pos = align16((uint64_t)32 * nb);
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * FOR_BLOCK);
    uint8_t *ok = (uint8_t *)malloc(FOR_BLOCK);
    if (!d || !ok) { s->bad = 1; free(d); free(ok); return; }
    buf_resize(s, pos);
    uint64_t end = pos;
    for (uint32_t b = 0; b < nb && !s->bad; b++) {
        uint32_t j0 = b * FOR_BLOCK, nv = n - j0 < FOR_BLOCK ? n - j0 : FOR_BLOCK;
        /* pick e */
        uint32_t best_e = 0;
        uint64_t best_cost = 0;
        for (uint32_t e = 0; e <= F2I_EMAX; e++) {
            uint32_t nx = 0, any = 0;
            int64_t lo = 0, hi = 0;
            for (uint32_t j = 0; j < nv; j++) {
                int64_t k;
                if (!f2i_digits(get64(x + 8 * (uint64_t)(j0 + j)), e, &k)) { nx++; continue; }
                if (!any || k < lo) lo = k;
                if (!any || k > hi) hi = k;
                any = 1;
            }
            uint32_t w = any ? bitlen64((uint64_t)hi - (uint64_t)lo) : 0;
            uint64_t cost = (uint64_t)nv * w + (uint64_t)128 * nx;
            if (e == 0 || cost < best_cost) { best_cost = cost; best_e = e; }
        }
        /* encode with best_e */
        uint32_t e = best_e, nx = 0, any = 0;
        int64_t ref = 0, hi = 0;
        for (uint32_t j = 0; j < nv; j++) {
            ok[j] = (uint8_t)f2i_digits(get64(x + 8 * (uint64_t)(j0 + j)), e, &d[j]);
            if (!ok[j]) { nx++; continue; }
            if (!any || d[j] < ref) ref = d[j];
            if (!any || d[j] > hi) hi = d[j];
            any = 1;
        }
        uint32_t w = any ? bitlen64((uint64_t)hi - (uint64_t)ref) : 0;
        uint64_t nw = packed_words(nv, w);
        uint64_t xoff = align16(pos + 4 * nw);
        buf_resize(s, xoff + (uint64_t)16 * nx);
        if (s->bad) break;
        uint8_t *de = s->p + 32 * (uint64_t)b;
        put64(de, (uint64_t)ref);
        put32(de + 8, w);
        put32(de + 12, (uint32_t)pos);
        put32(de + 16, (uint32_t)xoff);
        put16(de + 20, nx);
        put8(de + 22, e);
        uint32_t xi = 0;
        for (uint32_t j = 0; j < nv; j++) {
            if (ok[j]) {
                pack_bits(s->p + pos, j, w, (uint64_t)d[j] - (uint64_t)ref);
            } else {
                uint8_t *r = s->p + xoff + (uint64_t)16 * xi++;
                put32(r, j);
                put64(r + 8, get64(x + 8 * (uint64_t)(j0 + j)));
            }
        }
        end = xoff + (uint64_t)16 * nx;
        pos = align16(end);
    }
    free(d);
    free(ok);
    s->n = end;
}

static int dec_f2i_bp(const uint8_t *s, uint64_t comp_len, uint32_t n, uint8_t *out) {
    uint32_t nb = (n + FOR_BLOCK - 1) / FOR_BLOCK;
    if ((uint64_t)32 * nb > comp_len) return ZFO_ECORRUPT;
    for (uint32_t b = 0; b < nb; b++) {
        uint32_t j0 = b * FOR_BLOCK, nv = n - j0 < FOR_BLOCK ? n - j0 : FOR_BLOCK;
        const uint8_t *de = s + 32 * (uint64_t)b;
        uint64_t ref = get64(de);
        uint32_t w = get32(de + 8);
        uint64_t poff = get32(de + 12), xoff = get32(de + 16);
        uint32_t nx = get16(de + 20), e = de[22];
        if (w > 64 || e > F2I_EMAX || nx > nv) return ZFO_ECORRUPT;
        if (poff % 16 || poff < (uint64_t)32 * nb || poff + 4 * packed_words(nv, w) > comp_len)
            return ZFO_ECORRUPT;
        if (xoff % 16 || xoff < (uint64_t)32 * nb || xoff + (uint64_t)16 * nx > comp_len)
            return ZFO_ECORRUPT;
        for (uint32_t j = 0; j < nv; j++) {
            int64_t k = (int64_t)(ref + unpack_bits(s + poff, j, w));
            put64(out + 8 * (uint64_t)(j0 + j), f64_bits((double)k / F2I_P10[e]));
        }
        for (uint32_t i = 0; i < nx; i++) {
            const uint8_t *r = s + xoff + (uint64_t)16 * i;
            uint32_t j = get32(r);
            if (j >= nv || (i > 0 && j <= get32(r - 16))) return ZFO_ECORRUPT;
            put64(out + 8 * (uint64_t)(j0 + j), get64(r + 8));
        }
    }
    return ZFO_OK;
}

/* ============================================================ dictionary
 * Dictionary encoding (Sec. 2.1; the FP example of Sec. 3.1 decodes with the
 * dictionary as a lookup table held in metadata).  The column dictionary is
 * the sorted set of distinct values; the code of a value is its index in it.
 * A DICT_BP chunk stream is exactly the FOR_BP stream of its u32 code
 * sequence (read as I32): dictionary encoding nested with bit-packing.
 * Decode: x_j = dict[code_j]; a code >= dict_count is corrupt. */
static uint32_t g_sort_es; /* element size for the qsort comparator */
static uint32_t g_sort_dtype;
static int cmp_entry(const void *a, const void *b) {
    if (g_sort_dtype == ZFO_FIXED16) return memcmp(a, b, 16);
    int64_t x = load_int((const uint8_t *)a, g_sort_dtype, 0);
    int64_t y = load_int((const uint8_t *)b, g_sort_dtype, 0);
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* sorted unique values of x[0..n) -> *dict (malloc'd), *count */
static int build_dict(const uint8_t *x, uint64_t n, uint32_t dtype, uint8_t **dict,
                      uint32_t *count) {
    uint32_t es = zfo_elem_size(dtype);
    uint8_t *tmp = (uint8_t *)malloc(n ? n * es : 1);
    if (!tmp) return ZFO_ENOMEM;
    memcpy(tmp, x, n * es);
    g_sort_es = es;
    g_sort_dtype = dtype;
    qsort(tmp, n, es, cmp_entry);
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; i++)
        if (m == 0 || cmp_entry(tmp + (m - 1) * es, tmp + i * es) != 0) {
            memmove(tmp + m * es, tmp + i * es, es);
            m++;
        }
    if (m > 0xFFFFFFFFu) { free(tmp); return ZFO_EUNSUP; }
    *dict = tmp;
    *count = (uint32_t)m;
    return ZFO_OK;
}

/* index of value v in the sorted dictionary (binary search; v is present) */
static uint32_t dict_code(const uint8_t *dict, uint32_t count, uint32_t dtype, const uint8_t *v) {
    uint32_t es = zfo_elem_size(dtype), lo = 0, hi = count;
    while (hi - lo > 1) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (cmp_entry(dict + (uint64_t)mid * es, v) <= 0) lo = mid;
        else hi = mid;
    }
    return lo;
}

/* ============================================================ RLE + delta
 * Run-length encoding (Sec. 2.1: a value and a count per run), with the run
 * values delta-encoded (Sec. 2.1: differences to the previous value over a
 * stored base) and the deltas bit-packed with a frame of reference.  The runs
 * of a chunk are maximal.  Every RLE_GROUP consecutive runs form a group whose
 * record carries its own output offset and value base, so groups decode
 * independently; the output offset of a run is the exclusive prefix sum of
 * the counts (the `presum` of Sec. 3.2).
 * Stream:
 *   header 16 bytes: u32 n_runs, u32 n_groups = ceil(n_runs/64),
 *                    u32 runs_off, u32 0
 *   group records, 32 bytes each at offset 16 + 32*g:
 *       u32 out_off (element index of the group's first run in the chunk),
 *       u32 w, u32 doff (byte offset of the packed deltas, 4-aligned), u32 0,
 *       i64 base (value of the first run), i64 dmin
 *   packed deltas of group g at doff: nr_g - 1 fields of width w, field j-1
 *       = delta_j - dmin (mod 2^bits) for j = 1 .. nr_g-1, where
 *       delta_j = v_j - v_{j-1} (mod 2^bits) and dmin is the smallest delta
 *       read as a signed integer; w = bitlen(max field); groups of one run
 *       store w = 0 and dmin = 0.  Groups follow each other at 4-byte steps
 *       starting at 16 + 32*n_groups.
 *   run lengths: u32[n_runs] at runs_off = align16(end of deltas).
 *   comp_len = runs_off + 4*n_runs.
 * DELTA_BP is the same stream for runs that are all of length one (every
 * value is its own run, equal neighbours included): n_runs = n, runs_off = 0,
 * no run array, comp_len = end of the deltas. */
static void enc_rle_delta(buf_t *s, const uint8_t *x, uint32_t dtype, uint32_t n, int unit_runs) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    /* runs */
    uint64_t *val = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint32_t *len = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!val || !len) { free(val); free(len); s->bad = 1; return; }
    uint32_t nr = 0;
    for (uint32_t j = 0; j < n; j++) {
        uint64_t v = (uint64_t)load_int(x, dtype, j) & mask;
        if (!unit_runs && nr > 0 && val[nr - 1] == v) len[nr - 1]++;
        else { val[nr] = v; len[nr] = 1; nr++; }
    }
    uint32_t ng = (nr + RLE_GROUP - 1) / RLE_GROUP;
    uint64_t pos = 16 + (uint64_t)32 * ng;
    buf_resize(s, pos);
    uint32_t out_off = 0;
    for (uint32_t g = 0; g < ng && !s->bad; g++) {
        uint32_t r0 = g * RLE_GROUP, cnt = nr - r0 < RLE_GROUP ? nr - r0 : RLE_GROUP;
        /* signed minimum delta, then the field width */
        int64_t dmin = 0;
        for (uint32_t j = 1; j < cnt; j++) {
            uint64_t d = (val[r0 + j] - val[r0 + j - 1]) & mask;
            int64_t sd = bits == 32 ? (int64_t)(int32_t)(uint32_t)d : (int64_t)d;
            if (j == 1 || sd < dmin) dmin = sd;
        }
        uint64_t fmax = 0;
        for (uint32_t j = 1; j < cnt; j++) {
            uint64_t d = (val[r0 + j] - val[r0 + j - 1]) & mask;
            uint64_t f = (d - (uint64_t)dmin) & mask;
            if (f > fmax) fmax = f;
        }
        uint32_t w = bitlen64(fmax);
        uint64_t nw = packed_words(cnt - 1, w);
        buf_resize(s, pos + 4 * nw);
        if (s->bad) break;
        uint8_t *rec = s->p + 16 + (uint64_t)32 * g;
        put32(rec + 0, out_off);
        put32(rec + 4, w);
        put32(rec + 8, (uint32_t)pos);
        put32(rec + 12, 0);
        /* base is the first run value as a signed integer (I32 sign-extended) */
        int64_t base = bits == 32 ? (int64_t)(int32_t)(uint32_t)val[r0] : (int64_t)val[r0];
        put64(rec + 16, (uint64_t)base);
        put64(rec + 24, (uint64_t)dmin);
        for (uint32_t j = 1; j < cnt; j++) {
            uint64_t d = (val[r0 + j] - val[r0 + j - 1]) & mask;
            pack_bits(s->p + pos, j - 1, w, (d - (uint64_t)dmin) & mask);
        }
        pos += 4 * nw;
        for (uint32_t j = 0; j < cnt; j++) out_off += len[r0 + j];
    }
    if (!s->bad) {
        put32(s->p + 0, nr);
        put32(s->p + 4, ng);
        put32(s->p + 12, 0);
        if (unit_runs) {
            put32(s->p + 8, 0);
            s->n = pos;
        } else {
            uint64_t roff = align16(pos);
            buf_resize(s, roff + 4 * (uint64_t)nr);
            if (!s->bad) {
                put32(s->p + 8, (uint32_t)roff);
                for (uint32_t j = 0; j < nr; j++) put32(s->p + roff + 4 * (uint64_t)j, len[j]);
                s->n = roff + 4 * (uint64_t)nr;
            }
        }
    }
    free(val);
    free(len);
}

static int dec_rle_delta(const uint8_t *s, uint64_t comp_len, uint32_t dtype, uint32_t n,
                         int unit_runs, uint8_t *dst) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    if (comp_len < 16) return ZFO_ECORRUPT;
    uint32_t nr = get32(s), ng = get32(s + 4), roff = get32(s + 8);
    if (ng != (nr + RLE_GROUP - 1) / RLE_GROUP) return ZFO_ECORRUPT;
    if (16 + (uint64_t)32 * ng > comp_len) return ZFO_ECORRUPT;
    if (unit_runs) {
        if (nr != n || roff != 0) return ZFO_ECORRUPT;
    } else {
        if (roff % 4 != 0 || roff < 16 + (uint64_t)32 * ng) return ZFO_ECORRUPT;
        if ((uint64_t)roff + 4 * (uint64_t)nr > comp_len) return ZFO_ECORRUPT;
    }
    uint64_t produced = 0;
    for (uint32_t g = 0; g < ng; g++) {
        const uint8_t *rec = s + 16 + (uint64_t)32 * g;
        uint32_t out_off = get32(rec), w = get32(rec + 4), doff = get32(rec + 8);
        uint64_t base = get64(rec + 16), dmin = get64(rec + 24);
        uint32_t r0 = g * RLE_GROUP, cnt = nr - r0 < RLE_GROUP ? nr - r0 : RLE_GROUP;
        if (w > bits || doff % 4 != 0) return ZFO_ECORRUPT;
        if ((uint64_t)doff + 4 * packed_words(cnt - 1, w) > comp_len) return ZFO_ECORRUPT;
        /* the record's offset must equal the sum of all earlier runs */
        if (out_off != produced) return ZFO_ECORRUPT;
        uint64_t v = base & mask;
        for (uint32_t j = 0; j < cnt; j++) {
            if (j > 0) v = (v + dmin + unpack_bits(s + doff, j - 1, w)) & mask;
            uint32_t r = unit_runs ? 1u : get32(s + roff + 4 * (uint64_t)(r0 + j));
            if (r == 0 || produced + r > n) return ZFO_ECORRUPT;
            for (uint32_t k = 0; k < r; k++) store_int(dst, dtype, produced + k, v);
            produced += r;
        }
    }
    if (produced != n) return ZFO_ECORRUPT;
    return ZFO_OK;
}

/* ============================================================ DeltaStride
 * DeltaStride (Sec. 5, a Group-Parallel RLE variant for increasing integer
 * keys): the column is cut into runs that are arithmetic progressions, each a
 * (start, stride, count) triple, and the triples are nested with bit-packing.
 * Runs are maximal from the left: a run starting at element i takes
 * stride d = x[i+1] - x[i] (mod 2^bits) and extends while the next difference
 * equals d; a run that starts on the last element has count 1 and stride 0.
 * Every RLE_GROUP consecutive runs form a group with its own output offset and
 * start value, so groups decode independently.  Within a group the start of
 * run j >= 1 is predicted as the value run j-1 would produce next,
 * s_{j-1} + d_{j-1} * r_{j-1}; the stored gap is the difference to it
 * (0 for runs that continue a progression after a lone element, small for
 * nearly increasing keys).
 * Stream:
 *   header 16 bytes: u32 n_runs, u32 n_groups = ceil(n_runs/64),
 *                    u32 runs_off, u32 0
 *   group records, 32 bytes each at offset 16 + 32*g:
 *       u32 out_off (element index of the group's first run in the chunk),
 *       u32 poff (byte offset of the group's payload, 8-aligned),
 *       u32 widths (bits 0-7: gap width wg, bits 8-15: stride width wd),
 *       u32 0, i64 base (start of the group's first run), i64 dmin
 *   payload of group g at poff: i64 gmin, then cnt-1 gap fields of width wg
 *       (field j-1 = gap_j - gmin mod 2^bits, j = 1 .. cnt-1), then, from the
 *       next u32 word, cnt stride fields of width wd (field j = d_j - dmin
 *       mod 2^bits); gmin, dmin are the smallest gap and stride read as
 *       signed integers (0 when there is none); a width is the bit length of
 *       the largest field.
 *   run lengths: u32[n_runs] at runs_off = align16(end of the payloads).
 *   comp_len = runs_off + 4*n_runs.
 * Decode: s_0 = base, s_j = s_{j-1} + d_{j-1} r_{j-1} + gap_j; run j writes
 * s_j + d_j t for t = 0 .. r_j - 1 (all mod 2^bits). */
static int64_t as_signed(uint64_t v, uint32_t bits) {
    return bits == 32 ? (int64_t)(int32_t)(uint32_t)v : (int64_t)v;
}

static void enc_dstride(buf_t *s, const uint8_t *x, uint32_t dtype, uint32_t n) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    uint64_t *st = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint64_t *sd = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    uint32_t *len = (uint32_t *)malloc(sizeof(uint32_t) * (n ? n : 1));
    if (!st || !sd || !len) { free(st); free(sd); free(len); s->bad = 1; return; }
    /* maximal progressions from the left */
    uint32_t nr = 0;
    for (uint32_t i = 0; i < n;) {
        uint64_t a = (uint64_t)load_int(x, dtype, i) & mask, d = 0;
        uint32_t r = 1;
        if (i + 1 < n) {
            d = (((uint64_t)load_int(x, dtype, i + 1)) - a) & mask;
            r = 2;
            while (i + r < n && ((((uint64_t)load_int(x, dtype, i + r)) -
                                  (uint64_t)load_int(x, dtype, i + r - 1)) & mask) == d)
                r++;
        }
        st[nr] = a;
        sd[nr] = d;
        len[nr] = r;
        nr++;
        i += r;
    }
    uint32_t ng = (nr + RLE_GROUP - 1) / RLE_GROUP;
    uint64_t pos = 16 + (uint64_t)32 * ng;
    buf_resize(s, pos);
    uint32_t out_off = 0;
    for (uint32_t g = 0; g < ng && !s->bad; g++) {
        uint32_t r0 = g * RLE_GROUP, cnt = nr - r0 < RLE_GROUP ? nr - r0 : RLE_GROUP;
        /* gaps of runs 1 .. cnt-1 against the predicted start */
        uint64_t gap[RLE_GROUP];
        for (uint32_t j = 1; j < cnt; j++) {
            uint64_t pred = (st[r0 + j - 1] + sd[r0 + j - 1] * (uint64_t)len[r0 + j - 1]) & mask;
            gap[j] = (st[r0 + j] - pred) & mask;
        }
        int64_t gmin = 0, dmin = 0;
        for (uint32_t j = 1; j < cnt; j++)
            if (j == 1 || as_signed(gap[j], bits) < gmin) gmin = as_signed(gap[j], bits);
        for (uint32_t j = 0; j < cnt; j++)
            if (j == 0 || as_signed(sd[r0 + j], bits) < dmin) dmin = as_signed(sd[r0 + j], bits);
        uint64_t gmax = 0, dmax = 0;
        for (uint32_t j = 1; j < cnt; j++) {
            uint64_t f = (gap[j] - (uint64_t)gmin) & mask;
            if (f > gmax) gmax = f;
        }
        for (uint32_t j = 0; j < cnt; j++) {
            uint64_t f = (sd[r0 + j] - (uint64_t)dmin) & mask;
            if (f > dmax) dmax = f;
        }
        uint32_t wg = bitlen64(gmax), wd = bitlen64(dmax);
        pos = (pos + 7) & ~(uint64_t)7;
        uint64_t gw = packed_words(cnt - 1, wg), dw = packed_words(cnt, wd);
        buf_resize(s, pos + 8 + 4 * (gw + dw));
        if (s->bad) break;
        uint8_t *rec = s->p + 16 + (uint64_t)32 * g;
        put32(rec + 0, out_off);
        put32(rec + 4, (uint32_t)pos);
        put32(rec + 8, wg | (wd << 8));
        put32(rec + 12, 0);
        put64(rec + 16, (uint64_t)as_signed(st[r0], bits));
        put64(rec + 24, (uint64_t)dmin);
        put64(s->p + pos, (uint64_t)gmin);
        for (uint32_t j = 1; j < cnt; j++)
            pack_bits(s->p + pos + 8, j - 1, wg, (gap[j] - (uint64_t)gmin) & mask);
        for (uint32_t j = 0; j < cnt; j++)
            pack_bits(s->p + pos + 8 + 4 * gw, j, wd, (sd[r0 + j] - (uint64_t)dmin) & mask);
        pos += 8 + 4 * (gw + dw);
        for (uint32_t j = 0; j < cnt; j++) out_off += len[r0 + j];
    }
    if (!s->bad) {
        uint64_t roff = align16(pos);
        buf_resize(s, roff + 4 * (uint64_t)nr);
        if (!s->bad) {
            put32(s->p + 0, nr);
            put32(s->p + 4, ng);
            put32(s->p + 8, (uint32_t)roff);
            put32(s->p + 12, 0);
            for (uint32_t j = 0; j < nr; j++) put32(s->p + roff + 4 * (uint64_t)j, len[j]);
            s->n = roff + 4 * (uint64_t)nr;
        }
    }
    free(st);
    free(sd);
    free(len);
}

static int dec_dstride(const uint8_t *s, uint64_t comp_len, uint32_t dtype, uint32_t n, uint8_t *dst) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    if (comp_len < 16) return ZFO_ECORRUPT;
    uint32_t nr = get32(s), ng = get32(s + 4), roff = get32(s + 8);
    if (ng != (nr + RLE_GROUP - 1) / RLE_GROUP) return ZFO_ECORRUPT;
    if (16 + (uint64_t)32 * ng > comp_len) return ZFO_ECORRUPT;
    if (roff % 4 != 0 || roff < 16 + (uint64_t)32 * ng) return ZFO_ECORRUPT;
    if ((uint64_t)roff + 4 * (uint64_t)nr > comp_len) return ZFO_ECORRUPT;
    uint64_t produced = 0;
    for (uint32_t g = 0; g < ng; g++) {
        const uint8_t *rec = s + 16 + (uint64_t)32 * g;
        uint32_t out_off = get32(rec), poff = get32(rec + 4), widths = get32(rec + 8);
        uint32_t wg = widths & 0xFFu, wd = (widths >> 8) & 0xFFu;
        uint64_t base = get64(rec + 16), dmin = get64(rec + 24);
        uint32_t r0 = g * RLE_GROUP, cnt = nr - r0 < RLE_GROUP ? nr - r0 : RLE_GROUP;
        if (wg > bits || wd > bits || (widths >> 16) != 0 || poff % 8 != 0) return ZFO_ECORRUPT;
        uint64_t gw = packed_words(cnt - 1, wg), dw = packed_words(cnt, wd);
        if ((uint64_t)poff + 8 + 4 * (gw + dw) > comp_len) return ZFO_ECORRUPT;
        if (out_off != produced) return ZFO_ECORRUPT;
        uint64_t gmin = get64(s + poff);
        uint64_t start = base & mask, prev_d = 0;
        uint32_t prev_r = 0;
        for (uint32_t j = 0; j < cnt; j++) {
            uint64_t d = (dmin + unpack_bits(s + poff + 8 + 4 * gw, j, wd)) & mask;
            if (j > 0)
                start = (start + prev_d * (uint64_t)prev_r + gmin +
                         unpack_bits(s + poff + 8, j - 1, wg)) & mask;
            uint32_t r = get32(s + roff + 4 * (uint64_t)(r0 + j));
            if (r == 0 || produced + r > n) return ZFO_ECORRUPT;
            for (uint32_t t = 0; t < r; t++)
                store_int(dst, dtype, produced + t, (start + d * (uint64_t)t) & mask);
            produced += r;
            prev_d = d;
            prev_r = r;
        }
    }
    if (produced != n) return ZFO_ECORRUPT;
    return ZFO_OK;
}

/* =============================== DeltaStride | [Delta | RLE | [BP, BP], BP]
 * The order-key tree of the paper's table of applied schemes (Sec. 5): a
 * DeltaStride stage with two outputs, the first nested as Delta | RLE with
 * both of RLE's outputs bit-packed, the second bit-packed.
 * DeltaStride stage: the chunk's stride d is the most frequent difference
 * x[i+1] - x[i] (mod 2^bits; ties to the smaller one read as unsigned; 0 for a
 * chunk of one value); runs are maximal from the left, a run extending while
 * the next difference equals d.  Its outputs are the run starts S[0..R) and
 * the run counts C[0..R); run k writes S[k] + d*t, t = 0 .. C[k]-1.
 * Delta: D[0] = S[0], D[k] = S[k] - S[k-1] (mod 2^bits), so S is the running
 * sum of D.  RLE of D: maximal runs, values V[0..Q) and lengths L[0..Q).
 * Bit-packing of V, L and C: per group of 64 (one wavefront), the group's
 * smallest value (V read as signed) is the reference and each field holds
 * value - reference at the width of the largest such difference.
 * Every 64 consecutive runs of either level form a group whose record holds
 * its output offset (and, for D's runs, the running sum before it), so
 * groups decode independently.
 * Stream:
 *   header 32 bytes: u32 R, u32 ngB = ceil(R/64), u32 Q, u32 ngA = ceil(Q/64),
 *       i64 d, u32 b_off = 32 + 32*ngA, u32 0
 *   D's run groups, 32 bytes each at 32 + 32*g:
 *       u32 out_off (index in S of the group's first element), u32 poff
 *       (byte offset of the group's payload, 4-aligned), u32 widths (bits
 *       0-7: V width wv, bits 8-15: L width wl), u32 lmin,
 *       i64 base (S[out_off - 1]; 0 for the first group), i64 vmin
 *   the runs' groups, 16 bytes each at b_off + 16*g:
 *       u32 out_off (element index of the group's first run), u32 poff,
 *       u32 wc (C width), u32 cmin
 *   payloads from b_off + 16*ngB on, first D's groups then the runs' groups,
 *   each group's starting at the word after the previous one's:
 *       D group: cnt V fields (V_j - vmin), then from the next u32 word cnt L
 *           fields (L_j - lmin);
 *       runs group: cnt C fields (C_j - cmin).
 *   comp_len = end of the last payload.
 * Decode: S from D's groups (S[k] = S[k-1] + V_j over the L_j positions of
 * run j, starting from the group's base), then the output from the runs'
 * groups. */
typedef struct {
    uint32_t n;
    uint64_t *v; /* values */
    uint32_t *c; /* counts */
} runs_t;

static void runs_free(runs_t *r) { free(r->v); free(r->c); }

/* group g of a value array: reference (smallest, read as signed) and width */
static void group_for(const uint64_t *v, uint32_t cnt, uint32_t bits, uint64_t *ref, uint32_t *w) {
    uint64_t mask = mask_bits(bits);
    int64_t lo = 0;
    for (uint32_t j = 0; j < cnt; j++)
        if (j == 0 || as_signed(v[j], bits) < lo) lo = as_signed(v[j], bits);
    uint64_t fmax = 0;
    for (uint32_t j = 0; j < cnt; j++) {
        uint64_t f = (v[j] - (uint64_t)lo) & mask;
        if (f > fmax) fmax = f;
    }
    *ref = (uint64_t)lo;
    *w = bitlen64(fmax);
}

static void group_for32(const uint32_t *c, uint32_t cnt, uint32_t *ref, uint32_t *w) {
    uint32_t lo = c[0], hi = c[0];
    for (uint32_t j = 1; j < cnt; j++) {
        if (c[j] < lo) lo = c[j];
        if (c[j] > hi) hi = c[j];
    }
    *ref = lo;
    *w = bitlen64(hi - lo);
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : x > y;
}

static void enc_dstree(buf_t *s, const uint8_t *x, uint32_t dtype, uint32_t n) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    /* the stride: the most frequent difference, ties to the smaller */
    uint64_t d = 0;
    if (n > 1) {
        uint64_t *df = (uint64_t *)malloc(sizeof(uint64_t) * (n - 1));
        if (!df) { s->bad = 1; return; }
        for (uint32_t i = 0; i + 1 < n; i++)
            df[i] = ((uint64_t)load_int(x, dtype, i + 1) - (uint64_t)load_int(x, dtype, i)) & mask;
        qsort(df, n - 1, sizeof(uint64_t), cmp_u64);
        uint32_t best = 0;
        for (uint32_t i = 0; i < n - 1;) {
            uint32_t k = i;
            while (k < n - 1 && df[k] == df[i]) k++;
            if (k - i > best) { best = k - i; d = df[i]; }
            i = k;
        }
        free(df);
    }
    /* DeltaStride runs */
    runs_t st = {0, (uint64_t *)malloc(sizeof(uint64_t) * n), (uint32_t *)malloc(sizeof(uint32_t) * n)};
    runs_t dr = {0, (uint64_t *)malloc(sizeof(uint64_t) * n), (uint32_t *)malloc(sizeof(uint32_t) * n)};
    if (!st.v || !st.c || !dr.v || !dr.c) { runs_free(&st); runs_free(&dr); s->bad = 1; return; }
    for (uint32_t i = 0; i < n;) {
        uint32_t r = 1;
        while (i + r < n && ((((uint64_t)load_int(x, dtype, i + r)) -
                              (uint64_t)load_int(x, dtype, i + r - 1)) & mask) == d)
            r++;
        st.v[st.n] = (uint64_t)load_int(x, dtype, i) & mask;
        st.c[st.n] = r;
        st.n++;
        i += r;
    }
    /* Delta of the starts, then RLE */
    for (uint32_t k = 0; k < st.n; k++) {
        uint64_t dk = k == 0 ? st.v[0] : (st.v[k] - st.v[k - 1]) & mask;
        if (dr.n > 0 && dr.v[dr.n - 1] == dk) dr.c[dr.n - 1]++;
        else { dr.v[dr.n] = dk; dr.c[dr.n] = 1; dr.n++; }
    }
    uint32_t R = st.n, Q = dr.n, ngA = (Q + 63) / 64, ngB = (R + 63) / 64;
    uint64_t b_off = 32 + (uint64_t)32 * ngA, pos = b_off + (uint64_t)16 * ngB;
    buf_resize(s, pos);
    uint32_t at = 0; /* index in S */
    for (uint32_t g = 0; g < ngA && !s->bad; g++) {
        uint32_t j0 = 64 * g, cnt = Q - j0 < 64 ? Q - j0 : 64;
        uint64_t vmin;
        uint32_t wv, lmin, wl;
        group_for(dr.v + j0, cnt, bits, &vmin, &wv);
        group_for32(dr.c + j0, cnt, &lmin, &wl);
        uint64_t vw = packed_words(cnt, wv), lw = packed_words(cnt, wl);
        buf_resize(s, pos + 4 * (vw + lw));
        if (s->bad) break;
        uint8_t *rec = s->p + 32 + (uint64_t)32 * g;
        put32(rec, at);
        put32(rec + 4, (uint32_t)pos);
        put32(rec + 8, wv | (wl << 8));
        put32(rec + 12, lmin);
        put64(rec + 16, at == 0 ? 0 : (uint64_t)as_signed(st.v[at - 1], bits));
        put64(rec + 24, vmin);
        for (uint32_t j = 0; j < cnt; j++) {
            pack_bits(s->p + pos, j, wv, (dr.v[j0 + j] - vmin) & mask);
            pack_bits(s->p + pos + 4 * vw, j, wl, dr.c[j0 + j] - lmin);
            at += dr.c[j0 + j];
        }
        pos += 4 * (vw + lw);
    }
    uint32_t out = 0;
    for (uint32_t g = 0; g < ngB && !s->bad; g++) {
        uint32_t j0 = 64 * g, cnt = R - j0 < 64 ? R - j0 : 64;
        uint32_t cmin, wc;
        group_for32(st.c + j0, cnt, &cmin, &wc);
        uint64_t cw = packed_words(cnt, wc);
        buf_resize(s, pos + 4 * cw);
        if (s->bad) break;
        uint8_t *rec = s->p + b_off + (uint64_t)16 * g;
        put32(rec, out);
        put32(rec + 4, (uint32_t)pos);
        put32(rec + 8, wc);
        put32(rec + 12, cmin);
        for (uint32_t j = 0; j < cnt; j++) {
            pack_bits(s->p + pos, j, wc, st.c[j0 + j] - cmin);
            out += st.c[j0 + j];
        }
        pos += 4 * cw;
    }
    if (!s->bad) {
        put32(s->p, R);
        put32(s->p + 4, ngB);
        put32(s->p + 8, Q);
        put32(s->p + 12, ngA);
        put64(s->p + 16, (uint64_t)as_signed(d, bits));
        put32(s->p + 24, (uint32_t)b_off);
        put32(s->p + 28, 0);
        s->n = pos;
    }
    runs_free(&st);
    runs_free(&dr);
}

static int dec_dstree(const uint8_t *s, uint64_t comp_len, uint32_t dtype, uint32_t n, uint8_t *dst) {
    uint32_t bits = int_bits(dtype);
    uint64_t mask = mask_bits(bits);
    if (comp_len < 32) return ZFO_ECORRUPT;
    uint32_t R = get32(s), ngB = get32(s + 4), Q = get32(s + 8), ngA = get32(s + 12);
    uint64_t d = get64(s + 16) & mask, b_off = get32(s + 24);
    if (R == 0 || R > n || Q == 0 || Q > R || ngB != (R + 63) / 64 || ngA != (Q + 63) / 64) return ZFO_ECORRUPT;
    if (b_off != 32 + (uint64_t)32 * ngA || get32(s + 28) != 0) return ZFO_ECORRUPT;
    if (b_off + (uint64_t)16 * ngB > comp_len) return ZFO_ECORRUPT;
    uint64_t *S = (uint64_t *)malloc(sizeof(uint64_t) * R);
    if (!S) return ZFO_ENOMEM;
    int rc = ZFO_OK;
    /* S from D's run groups */
    uint64_t k = 0;
    for (uint32_t g = 0; g < ngA && rc == ZFO_OK; g++) {
        const uint8_t *rec = s + 32 + (uint64_t)32 * g;
        uint32_t out_off = get32(rec), poff = get32(rec + 4), widths = get32(rec + 8), lmin = get32(rec + 12);
        uint32_t wv = widths & 0xFFu, wl = (widths >> 8) & 0xFFu;
        uint64_t v = get64(rec + 16) & mask, vmin = get64(rec + 24);
        uint32_t cnt = Q - 64 * g < 64 ? Q - 64 * g : 64;
        uint64_t vw = packed_words(cnt, wv), lw = packed_words(cnt, wl);
        if (wv > bits || wl > 32 || (widths >> 16) || poff % 4 || out_off != k ||
            (uint64_t)poff + 4 * (vw + lw) > comp_len) { rc = ZFO_ECORRUPT; break; }
        for (uint32_t j = 0; j < cnt; j++) {
            uint64_t vj = (vmin + unpack_bits(s + poff, j, wv)) & mask;
            uint64_t lj = (uint64_t)lmin + unpack_bits(s + poff + 4 * vw, j, wl);
            if (lj == 0 || lj > 0xFFFFFFFFu || k + lj > R) { rc = ZFO_ECORRUPT; break; }
            for (uint64_t t = 0; t < lj; t++) {
                v = (v + vj) & mask;
                S[k++] = v;
            }
        }
    }
    if (rc == ZFO_OK && k != R) rc = ZFO_ECORRUPT;
    /* the output from the runs' groups */
    uint64_t p = 0;
    for (uint32_t g = 0; g < ngB && rc == ZFO_OK; g++) {
        const uint8_t *rec = s + b_off + (uint64_t)16 * g;
        uint32_t out_off = get32(rec), poff = get32(rec + 4), wc = get32(rec + 8), cmin = get32(rec + 12);
        uint32_t cnt = R - 64 * g < 64 ? R - 64 * g : 64;
        uint64_t cw = packed_words(cnt, wc);
        if (wc > 32 || poff % 4 || out_off != p || (uint64_t)poff + 4 * cw > comp_len) { rc = ZFO_ECORRUPT; break; }
        for (uint32_t j = 0; j < cnt; j++) {
            uint64_t cj = (uint64_t)cmin + unpack_bits(s + poff, j, wc);
            if (cj == 0 || cj > 0xFFFFFFFFu || p + cj > n) { rc = ZFO_ECORRUPT; break; }
            for (uint64_t t = 0; t < cj; t++) store_int(dst, dtype, p + t, (S[64 * g + j] + d * t) & mask);
            p += cj;
        }
    }
    if (rc == ZFO_OK && p != n) rc = ZFO_ECORRUPT;
    free(S);
    return rc;
}

/* ======================================================= String-dictionary
 * String-dictionary (Sec. 2.1; Sec. 5: the text is cut into words at spaces
 * and periods, each distinct word is a dictionary entry, the word indices are
 * bit-packed, and each word decodes as one group of the Group-Parallel
 * pattern).  Tokens: every byte belongs to exactly one token; a token is a
 * run of bytes other than ' ' and '.' followed by one ' ' or '.', or the
 * chunk's final bytes when they end without one; a run longer than
 * SD_MAX_TOKEN bytes is cut into pieces of SD_MAX_TOKEN (the piece that ends
 * with the separator may be shorter).  Entries are the distinct tokens in
 * order of first appearance.
 * Stream:
 *   header 32 bytes: u32 n_tokens, u32 n_entries, u32 w (code width =
 *       bitlen(n_entries - 1)), u32 n_groups = ceil(n_tokens/64),
 *       u32 ent_off, u32 bytes_off, u32 codes_off, u32 n_bytes (sum of the
 *       entry lengths)
 *   group offsets: u32[n_groups] at 32, the output byte offset of token 64g
 *   entries: u32[n_entries] at ent_off = align16(32 + 4*n_groups), entry k =
 *       byte offset of its bytes (bits 0-23) | length 1..64 (bits 24-31)
 *   entry bytes at bytes_off = ent_off + 4*n_entries, n_bytes of them, then
 *       zero bytes up to codes_off = align16(bytes_off + n_bytes + 4)
 *   codes at codes_off: n_tokens fields of width w (entry index of token i)
 *   comp_len = codes_off + 4*ceil(n_tokens*w/32).
 * Decode: token i writes entry code_i's bytes at the group offset plus the
 * lengths of the earlier tokens of its group. */
#define SD_MAX_TOKEN 64u

static int sd_is_sep(uint8_t c) { return c == ' ' || c == '.'; }

/* length of the token starting at byte i of x[0..n) */
static uint32_t sd_token_len(const uint8_t *x, uint32_t n, uint32_t i) {
    uint32_t k = 0;
    while (i + k < n && k < SD_MAX_TOKEN) {
        k++;
        if (sd_is_sep(x[i + k - 1])) break;
    }
    return k;
}

static uint64_t sd_hash(const uint8_t *p, uint32_t len) {
    uint64_t h = 1469598103934665603ull;  /* FNV-1a */
    for (uint32_t k = 0; k < len; k++) h = (h ^ p[k]) * 1099511628211ull;
    return h;
}

static void enc_sdict(buf_t *s, const uint8_t *x, uint32_t n) {
    /* tokens */
    uint32_t nt = 0;
    for (uint32_t i = 0; i < n; i += sd_token_len(x, n, i)) nt++;
    uint32_t *tstart = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    uint32_t *tlen = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    uint32_t *code = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1));
    uint32_t *efirst = (uint32_t *)malloc(sizeof(uint32_t) * (nt ? nt : 1)); /* token that defines entry k */
    uint64_t cap = 16;
    while (cap < 2 * (uint64_t)nt) cap *= 2;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * cap);  /* entry index or -1 */
    if (!tstart || !tlen || !code || !efirst || !slot) {
        free(tstart); free(tlen); free(code); free(efirst); free(slot);
        s->bad = 1;
        return;
    }
    for (uint64_t k = 0; k < cap; k++) slot[k] = -1;
    uint32_t ne = 0, nbytes = 0;
    for (uint32_t i = 0, t = 0; i < n; t++) {
        uint32_t L = sd_token_len(x, n, i);
        tstart[t] = i;
        tlen[t] = L;
        /* find the token among the entries (open addressing) */
        uint64_t h = sd_hash(x + i, L) & (cap - 1);
        while (slot[h] >= 0) {
            uint32_t f = efirst[slot[h]];
            if (tlen[f] == L && memcmp(x + tstart[f], x + i, L) == 0) break;
            h = (h + 1) & (cap - 1);
        }
        if (slot[h] < 0) {
            slot[h] = ne;
            efirst[ne] = t;
            ne++;
            nbytes += L;
        }
        code[t] = (uint32_t)slot[h];
        i += L;
    }
    uint32_t w = ne > 1 ? bitlen64(ne - 1) : 0;
    uint32_t ng = (nt + 63) / 64;
    uint64_t ent_off = align16(32 + 4 * (uint64_t)ng);
    uint64_t bytes_off = ent_off + 4 * (uint64_t)ne;
    uint64_t codes_off = align16(bytes_off + nbytes + 4);
    buf_resize(s, codes_off + 4 * packed_words(nt, w));
    if (!s->bad) {
        uint8_t *p = s->p;
        put32(p + 0, nt);
        put32(p + 4, ne);
        put32(p + 8, w);
        put32(p + 12, ng);
        put32(p + 16, (uint32_t)ent_off);
        put32(p + 20, (uint32_t)bytes_off);
        put32(p + 24, (uint32_t)codes_off);
        put32(p + 28, nbytes);
        for (uint32_t g = 0; g < ng; g++) put32(p + 32 + 4 * (uint64_t)g, tstart[64 * g]);
        uint32_t at = 0;
        for (uint32_t k = 0; k < ne; k++) {
            uint32_t f = efirst[k];
            put32(p + ent_off + 4 * (uint64_t)k, at | (tlen[f] << 24));
            memcpy(p + bytes_off + at, x + tstart[f], tlen[f]);
            at += tlen[f];
        }
        for (uint32_t t = 0; t < nt; t++) pack_bits(p + codes_off, t, w, code[t]);
        s->n = codes_off + 4 * packed_words(nt, w);
    }
    free(tstart); free(tlen); free(code); free(efirst); free(slot);
}

static int dec_sdict(const uint8_t *s, uint64_t comp_len, uint32_t plain_len, uint8_t *out) {
    if (comp_len < 32) return ZFO_ECORRUPT;
    uint32_t nt = get32(s), ne = get32(s + 4), w = get32(s + 8), ng = get32(s + 12);
    uint32_t ent_off = get32(s + 16), bytes_off = get32(s + 20), codes_off = get32(s + 24);
    uint32_t nbytes = get32(s + 28);
    if (ng != (nt + 63) / 64 || ne == 0 || w > 32) return ZFO_ECORRUPT;
    if (w != (ne > 1 ? bitlen64(ne - 1) : 0)) return ZFO_ECORRUPT;
    if (ent_off != align16(32 + 4 * (uint64_t)ng) || bytes_off != ent_off + 4 * (uint64_t)ne ||
        codes_off != align16((uint64_t)bytes_off + nbytes + 4) ||
        (uint64_t)codes_off + 4 * packed_words(nt, w) != comp_len)
        return ZFO_ECORRUPT;
    uint64_t p = 0;
    for (uint32_t t = 0; t < nt; t++) {
        if (t % 64 == 0 && get32(s + 32 + 4 * (uint64_t)(t / 64)) != p) return ZFO_ECORRUPT;
        uint64_t c = unpack_bits(s + codes_off, t, w);
        if (c >= ne) return ZFO_ECORRUPT;
        uint32_t e = get32(s + ent_off + 4 * c), off = e & 0xFFFFFFu, len = e >> 24;
        if (len == 0 || len > SD_MAX_TOKEN || (uint64_t)off + len > nbytes) return ZFO_ECORRUPT;
        if (p + len > plain_len) return ZFO_ECORRUPT;
        memcpy(out + p, s + bytes_off + off, len);
        p += len;
    }
    if (p != plain_len) return ZFO_ECORRUPT;
    return ZFO_OK;
}

/* ============================================ String-dictionary | BP | ANS
 * A nested scheme (Sec. 5, the comment column's String-dictionary, then
 * bit-packing, then ANS): the SDICT_BP stream whose packed entry indices
 * (the ncb = 4*ceil(n_tokens*w/32) bytes at codes_off) are replaced by ANS
 * streams of those bytes, cut into pieces of SD_ANS_PIECE bytes (the last
 * one shorter) so that the pieces decode independently.  Every header field
 * keeps its SDICT_BP meaning.  At codes_off: u32 n_pieces =
 * ceil(ncb / SD_ANS_PIECE), then u32 end[n_pieces] (the end of each piece's
 * ANS stream, counted from the first stream's start at codes_off + 4 +
 * 4*n_pieces), then the streams, each followed by zero bytes up to a
 * multiple of 4 (so every stream starts 4-aligned; the padding is counted in
 * the ends).  No index bytes (w = 0): nothing at codes_off,
 * comp_len = codes_off. */
#define SD_ANS_PIECE 65536u

/* The ncb = inner->n - co packed index bytes at co of an inner stream
 * replaced by the piece table and the pieces' ANS streams, as described
 * above; the inner bytes before co are kept. */
static void ans_pieces_encode(buf_t *s, const buf_t *inner, uint32_t co) {
    uint64_t ncb = inner->n - co;  /* index bytes */
    uint32_t np = (uint32_t)((ncb + SD_ANS_PIECE - 1) / SD_ANS_PIECE);
    uint64_t at = co + (np ? 4 + 4 * (uint64_t)np : 0);
    buf_resize(s, at);
    if (!s->bad) memcpy(s->p, inner->p, co);
    if (np && !s->bad) put32(s->p + co, np);
    for (uint32_t k = 0; k < np && !s->bad; k++) {
        uint64_t lo = (uint64_t)k * SD_ANS_PIECE, hi = lo + SD_ANS_PIECE < ncb ? lo + SD_ANS_PIECE : ncb;
        buf_t a = {0};
        enc_ans(&a, inner->p + co + lo, (uint32_t)(hi - lo));
        if (a.bad) { s->bad = 1; free(a.p); break; }
        uint64_t padded = (a.n + 3) & ~(uint64_t)3;
        buf_resize(s, at + padded);
        if (!s->bad) {
            memcpy(s->p + at, a.p, a.n);
            at += padded;
            put32(s->p + co + 4 + 4 * (uint64_t)k, (uint32_t)(at - (co + 4 + 4 * (uint64_t)np)));
        }
        free(a.p);
    }
    if (!s->bad) s->n = at;
}

/* Inverse of ans_pieces_encode: inner (co + ncb bytes) = the stream's first
 * co bytes followed by the decoded index bytes. */
static int ans_pieces_decode(const uint8_t *s, uint64_t comp_len, uint32_t co, uint64_t ncb, uint8_t *inner) {
    uint32_t np = (uint32_t)((ncb + SD_ANS_PIECE - 1) / SD_ANS_PIECE);
    if (co > comp_len) return ZFO_ECORRUPT;
    if (np == 0 && comp_len != co) return ZFO_ECORRUPT;
    if (np && (co + 4 + 4 * (uint64_t)np > comp_len || get32(s + co) != np)) return ZFO_ECORRUPT;
    memcpy(inner, s, co);
    int rc = ZFO_OK;
    uint64_t base = co + 4 + 4 * (uint64_t)np, prev = 0;
    for (uint32_t k = 0; k < np && rc == ZFO_OK; k++) {
        uint64_t end = get32(s + co + 4 + 4 * (uint64_t)k);
        uint64_t lo = (uint64_t)k * SD_ANS_PIECE, hi = lo + SD_ANS_PIECE < ncb ? lo + SD_ANS_PIECE : ncb;
        if (end < prev + ANS_HDR || base + end > comp_len || (k + 1 == np && base + end != comp_len)) {
            rc = ZFO_ECORRUPT;
        } else {
            uint64_t alen = ANS_HDR + 2 * (uint64_t)get32(s + base + prev + 4);
            if (((alen + 3) & ~(uint64_t)3) != end - prev) rc = ZFO_ECORRUPT;
            else rc = dec_ans(s + base + prev, alen, (uint32_t)(hi - lo), inner + co + lo);
        }
        prev = end;
    }
    return rc;
}

static void enc_sdict_ans(buf_t *s, const uint8_t *x, uint32_t n) {
    buf_t inner = {0};
    enc_sdict(&inner, x, n);
    if (inner.bad) { free(inner.p); s->bad = 1; return; }
    ans_pieces_encode(s, &inner, get32(inner.p + 24));
    free(inner.p);
}

static int dec_sdict_ans(const uint8_t *s, uint64_t comp_len, uint32_t plain_len, uint8_t *out) {
    if (comp_len < 32) return ZFO_ECORRUPT;
    uint32_t nt = get32(s), w = get32(s + 8), co = get32(s + 24);
    if (w > 32 || co > comp_len) return ZFO_ECORRUPT;
    uint64_t ncb = 4 * packed_words(nt, w);
    uint8_t *inner = (uint8_t *)malloc(co + ncb + 1);
    if (!inner) return ZFO_ENOMEM;
    int rc = ans_pieces_decode(s, comp_len, co, ncb, inner);
    if (rc == ZFO_OK) rc = dec_sdict(inner, co + ncb, plain_len, out);
    free(inner);
    return rc;
}

/* =============================== String-dictionary over a column dictionary
 * The paper builds one word dictionary for a whole column (Sec. 5: the
 * comment column's 1,878 distinct words, indices bit-packed) from the
 * frequent byte sequences of the data (Sec. 2.1).  Here the dictionary lives
 * in the container's dictionary area, shared by every chunk, and each chunk
 * keeps only its bit-packed indices and group offsets, so chunks still decode
 * on their own.  Tokens are cut as for SDICT_BP, except that a newline also
 * ends a token: the byte column holds rows ended by '\n', a row is one value
 * of the column, and no token spans two values.
 * Column dictionary (dtype BYTES, at the container's dict_off, dict_count =
 * number of entries):
 *   u32 n_bytes, u32 0, u32 0, u32 0
 *   u32 entry[dict_count] at 16: byte offset (bits 0-23) | length 1..64
 *       (bits 24-31)
 *   n_bytes entry bytes at 16 + 4*dict_count, then zero bytes up to
 *   16 + 4*dict_count + align16(n_bytes).  The first entry starts at byte 4,
 *   each next one at align4(end of the previous + 3), and n_bytes is the
 *   larger of align4(end of the last + 3) and the last start + 16: every
 *   entry has at least three zero bytes before and after it, and 16 bytes
 *   from its start lie within n_bytes (a decoder may read whole dwords
 *   around an entry, or 16 bytes from its start).  A dictionary whose
 *   entries lack those zero bytes or 16 bytes is corrupt.
 *   Entries: the distinct tokens of the column's SDICT_COL / SDICT_COL_ANS
 *   chunks, by decreasing number of occurrences, ties by first appearance;
 *   at most 2^24 entries and 2^24 - 1 entry bytes.
 * Chunk stream:
 *   header 16 bytes: u32 n_tokens, u32 w (= bitlen(dict_count - 1)),
 *       u32 n_groups = ceil(n_tokens/64), u32 codes_off = align16(16 + 4*n_groups)
 *   group offsets: u32[n_groups] at 16, the output byte offset of token 64g
 *   codes at codes_off: n_tokens fields of width w (entry index of token i)
 *   comp_len = codes_off + 4*ceil(n_tokens*w/32).
 * SDICT_COL_ANS: the same stream with the packed codes replaced exactly as
 * SDICT_ANS replaces them (piece table and 64 KiB ANS pieces at codes_off). */
#define SDC_MAX_ENTRIES (1u << 24)
#define SDC_MAX_BYTES ((1u << 24) - 1)

static int sdc_is_sep(uint8_t c) { return c == ' ' || c == '.' || c == '\n'; }

static uint32_t sdc_token_len(const uint8_t *x, uint32_t n, uint32_t i) {
    uint32_t k = 0;
    while (i + k < n && k < SD_MAX_TOKEN) {
        k++;
        if (sdc_is_sep(x[i + k - 1])) break;
    }
    return k;
}

/* Distinct tokens: open-addressing table of (position of the first
 * occurrence in the column, length, count). */
typedef struct {
    uint64_t *pos;    /* first occurrence, byte offset in the column */
    uint32_t *len, *count, *code;
    int64_t *slot;    /* token id or -1 */
    uint64_t cap, n;
    const uint8_t *src;
    int bad;
} tdict_t;

static void tdict_free(tdict_t *d) {
    free(d->pos); free(d->len); free(d->count); free(d->code); free(d->slot);
    memset(d, 0, sizeof *d);
}

/* id of the token src[at, at+L), added (count 0) if new; -1 on failure */
static int64_t tdict_find(tdict_t *d, uint64_t at, uint32_t L, int add) {
    if (add && 2 * (d->n + 1) > d->cap) {
        uint64_t nc = d->cap ? 2 * d->cap : 1024;
        int64_t *ns = (int64_t *)malloc(sizeof(int64_t) * nc);
        uint64_t *np = (uint64_t *)realloc(d->pos, sizeof(uint64_t) * nc);
        uint32_t *nl = (uint32_t *)realloc(d->len, sizeof(uint32_t) * nc);
        uint32_t *nn = (uint32_t *)realloc(d->count, sizeof(uint32_t) * nc);
        if (np) d->pos = np;
        if (nl) d->len = nl;
        if (nn) d->count = nn;
        if (!ns || !np || !nl || !nn) { free(ns); d->bad = 1; return -1; }
        for (uint64_t k = 0; k < nc; k++) ns[k] = -1;
        for (uint64_t t = 0; t < d->n; t++) {
            uint64_t h = sd_hash(d->src + d->pos[t], d->len[t]) & (nc - 1);
            while (ns[h] >= 0) h = (h + 1) & (nc - 1);
            ns[h] = (int64_t)t;
        }
        free(d->slot);
        d->slot = ns;
        d->cap = nc;
    }
    if (!d->cap) return -1;
    uint64_t h = sd_hash(d->src + at, L) & (d->cap - 1);
    while (d->slot[h] >= 0) {
        uint64_t t = (uint64_t)d->slot[h];
        if (d->len[t] == L && memcmp(d->src + d->pos[t], d->src + at, L) == 0) return (int64_t)t;
        h = (h + 1) & (d->cap - 1);
    }
    if (!add) return -1;
    d->slot[h] = (int64_t)d->n;
    d->pos[d->n] = at;
    d->len[d->n] = L;
    d->count[d->n] = 0;
    return (int64_t)d->n++;
}

static const tdict_t *g_sort_dict;
static int tdict_order(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    const tdict_t *d = g_sort_dict;
    if (d->count[x] != d->count[y]) return d->count[x] > d->count[y] ? -1 : 1;
    return d->pos[x] < d->pos[y] ? -1 : d->pos[x] > d->pos[y];
}

/* Build the column dictionary from the chunks coded with SDICT_COL or
 * SDICT_COL_ANS; fills d (codes = entry index of each token id) and the
 * dictionary area bytes.  Returns ZFO_OK, ZFO_EUNSUP (too many entries or
 * bytes) or ZFO_ENOMEM. */
static int tdict_build(const uint8_t *src, const uint32_t *chunk_elems, uint32_t n_chunks,
                       const uint32_t *codecs, uint32_t codec, tdict_t *d, uint8_t **area,
                       uint64_t *area_len, uint32_t *n_entries) {
    memset(d, 0, sizeof *d);
    d->src = src;
    uint64_t off = 0;
    for (uint32_t i = 0; i < n_chunks; i++) {
        uint32_t c = codecs ? codecs[i] : codec, n = chunk_elems[i];
        if (c == ZFO_SDICT_COL || c == ZFO_SDICT_COL_ANS) {
            for (uint32_t k = 0; k < n;) {
                uint32_t L = sdc_token_len(src + off, n, k);
                int64_t t = tdict_find(d, off + k, L, 1);
                if (t < 0) { tdict_free(d); return ZFO_ENOMEM; }
                d->count[t]++;
                k += L;
            }
        }
        off += n;
    }
    if (d->n > SDC_MAX_ENTRIES) { tdict_free(d); return ZFO_EUNSUP; }
    /* entry bytes with the zero guards: 4 before the first, then each entry
     * and at least 3 zero bytes, up to a multiple of 4 */
    uint64_t *ord = (uint64_t *)malloc(sizeof(uint64_t) * (d->n ? d->n : 1));
    d->code = (uint32_t *)malloc(sizeof(uint32_t) * (d->n ? d->n : 1));
    if (!ord || !d->code) { free(ord); tdict_free(d); return ZFO_ENOMEM; }
    for (uint64_t t = 0; t < d->n; t++) ord[t] = t;
    g_sort_dict = d;
    qsort(ord, d->n, sizeof(uint64_t), tdict_order);
    /* entry starts in dictionary order: 4, then align4(end + 3) */
    uint64_t nb = 4, last = 4;
    for (uint64_t k = 0; k < d->n; k++) {
        last = nb;
        nb = (nb + d->len[ord[k]] + 3 + 3) & ~(uint64_t)3;
    }
    if (nb < last + 16) nb = last + 16;
    if (nb > SDC_MAX_BYTES) { free(ord); tdict_free(d); return ZFO_EUNSUP; }
    uint64_t len = 16 + 4 * d->n + align16(nb);
    uint8_t *a = (uint8_t *)calloc(len, 1);
    if (!a) { free(ord); tdict_free(d); return ZFO_ENOMEM; }
    put32(a, (uint32_t)nb);
    uint64_t at = 4;
    for (uint64_t k = 0; k < d->n; k++) {
        uint64_t t = ord[k];
        d->code[t] = (uint32_t)k;
        put32(a + 16 + 4 * k, (uint32_t)at | (d->len[t] << 24));
        memcpy(a + 16 + 4 * d->n + at, src + d->pos[t], d->len[t]);
        at = (at + d->len[t] + 3 + 3) & ~(uint64_t)3;
    }
    free(ord);
    *area = a;
    *area_len = len;
    *n_entries = (uint32_t)d->n;
    return ZFO_OK;
}

/* chunk x = column bytes [x0, x0 + n) */
static void enc_sdict_col(buf_t *s, tdict_t *d, uint64_t x0, uint32_t n, uint32_t ne) {
    const uint8_t *x = d->src + x0;
    uint32_t nt = 0;
    for (uint32_t i = 0; i < n; i += sdc_token_len(x, n, i)) nt++;
    uint32_t w = ne > 1 ? bitlen64(ne - 1) : 0;
    uint32_t ng = (nt + 63) / 64;
    uint64_t co = align16(16 + 4 * (uint64_t)ng);
    buf_resize(s, co + 4 * packed_words(nt, w));
    if (s->bad) return;
    uint8_t *p = s->p;
    put32(p, nt);
    put32(p + 4, w);
    put32(p + 8, ng);
    put32(p + 12, (uint32_t)co);
    for (uint32_t i = 0, t = 0; i < n; t++) {
        uint32_t L = sdc_token_len(x, n, i);
        if (t % 64 == 0) put32(p + 16 + 4 * (uint64_t)(t / 64), i);
        int64_t id = tdict_find(d, x0 + i, L, 0);
        if (id < 0) { s->bad = 1; return; }
        pack_bits(p + co, t, w, d->code[id]);
        i += L;
    }
    s->n = co + 4 * packed_words(nt, w);
}

static int dec_sdict_col(const uint8_t *s, uint64_t comp_len, uint32_t plain_len, const uint8_t *dict,
                         uint32_t dict_count, uint8_t *out) {
    if (comp_len < 16 || !dict || dict_count == 0) return ZFO_ECORRUPT;
    uint32_t nt = get32(s), w = get32(s + 4), ng = get32(s + 8), co = get32(s + 12);
    if (ng != (nt + 63) / 64 || w != (dict_count > 1 ? bitlen64(dict_count - 1) : 0) ||
        co != align16(16 + 4 * (uint64_t)ng) || (uint64_t)co + 4 * packed_words(nt, w) != comp_len)
        return ZFO_ECORRUPT;
    uint32_t nb = get32(dict);
    const uint8_t *ents = dict + 16, *bytes = dict + 16 + 4 * (uint64_t)dict_count;
    uint64_t p = 0;
    for (uint32_t t = 0; t < nt; t++) {
        if (t % 64 == 0 && get32(s + 16 + 4 * (uint64_t)(t / 64)) != p) return ZFO_ECORRUPT;
        uint64_t c = unpack_bits(s + co, t, w);
        if (c >= dict_count) return ZFO_ECORRUPT;
        uint32_t e = get32(ents + 4 * c), off = e & 0xFFFFFFu, len = e >> 24;
        if (len == 0 || len > SD_MAX_TOKEN || (uint64_t)off + len > nb) return ZFO_ECORRUPT;
        if (p + len > plain_len) return ZFO_ECORRUPT;
        memcpy(out + p, bytes + off, len);
        p += len;
    }
    if (p != plain_len) return ZFO_ECORRUPT;
    return ZFO_OK;
}

static void enc_sdict_col_ans(buf_t *s, tdict_t *d, uint64_t x0, uint32_t n, uint32_t ne) {
    buf_t inner = {0};
    enc_sdict_col(&inner, d, x0, n, ne);
    if (inner.bad) { free(inner.p); s->bad = 1; return; }
    ans_pieces_encode(s, &inner, get32(inner.p + 12));
    free(inner.p);
}

static int dec_sdict_col_ans(const uint8_t *s, uint64_t comp_len, uint32_t plain_len, const uint8_t *dict,
                             uint32_t dict_count, uint8_t *out) {
    if (comp_len < 16) return ZFO_ECORRUPT;
    uint32_t nt = get32(s), w = get32(s + 4), co = get32(s + 12);
    if (w > 32 || co > comp_len) return ZFO_ECORRUPT;
    uint64_t ncb = 4 * packed_words(nt, w);
    uint8_t *inner = (uint8_t *)malloc(co + ncb + 1);
    if (!inner) return ZFO_ENOMEM;
    int rc = ans_pieces_decode(s, comp_len, co, ncb, inner);
    if (rc == ZFO_OK) rc = dec_sdict_col(inner, co + ncb, plain_len, dict, dict_count, out);
    free(inner);
    return rc;
}

/* ================================================================= LZ77
 * LZ77 family (Sec. 2.1): repeated byte sequences become pointers to earlier
 * output.  A chunk holds at most 65536 plain bytes and decodes on its own
 * (Sec. 3.1: independent file chunks are what the Non-Parallel pattern
 * parallelises over).  The chunk is a list of sequences; sequence i is
 * ll_i literal bytes followed by a match of ml_i bytes (ml_i = 0: none)
 * copied from off_i bytes back.
 * Stream:
 *   header 16 bytes: u32 n_seq, u32 n_lit, u32 n_ext, u32 plain_len
 *   offs:  u16[n_seq] at 16                (0 when the sequence has no match)
 *   ext:   u16[n_ext] at 16 + 2*n_seq      (extended lengths, in order)
 *   tags:  u8[n_seq]  at 16 + 2*n_seq + 2*n_ext
 *   lits:  u8[n_lit]  right after the tags
 *   comp_len = 16 + 3*n_seq + 2*n_ext + n_lit.
 * tag bits 0..2 = lc: ll = lc for lc < 7; lc = 7 takes the next ext e, ll = 7 + e.
 * tag bits 3..7 = mc: mc = 0 no match; 1..30: ml = mc + 3; 31 takes the next
 * ext e (after the literal one, if any), ml = 34 + e.
 * Decode in order: copy ll literals, then for j = 0 .. ml-1 ascending
 * out[p + j] = out[p - off + j] (so an overlapping match repeats its period);
 * 1 <= off <= p.  Corrupt: off out of range, off != 0 without a match, any
 * write past plain_len, and at the end p != plain_len, or the literal or ext
 * cursors short of n_lit or n_ext.
 * Encoder: greedy, hash of the 4 bytes at a position, chains of the most
 * recent earlier positions (depth 16), longest match, ties to the nearest. */
static uint32_t lz_hash(const uint8_t *p) {
    uint32_t v = (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
                 ((uint32_t)p[3] << 24);
    return (v * 2654435761u) >> (32 - LZ_HASH_BITS);
}

typedef struct { uint32_t ll, ml, off; } lz_seq;

static void enc_lz77(buf_t *s, const uint8_t *x, uint32_t n) {
    int32_t *head = (int32_t *)malloc(sizeof(int32_t) << LZ_HASH_BITS);
    int32_t *prev = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    lz_seq *seq = (lz_seq *)malloc(sizeof(lz_seq) * (n + 1));
    if (!head || !prev || !seq) { free(head); free(prev); free(seq); s->bad = 1; return; }
    for (uint32_t i = 0; i < (1u << LZ_HASH_BITS); i++) head[i] = -1;
    uint32_t nseq = 0, i = 0, lit_start = 0;
    while (i < n) {
        uint32_t best = 0, best_off = 0;
        if (i + 4 <= n) {
            int32_t c = head[lz_hash(x + i)];
            for (int d = 0; d < LZ_CHAIN && c >= 0; d++) {
                uint32_t l = 0;
                while (i + l < n && x[(uint32_t)c + l] == x[i + l]) l++;
                if (l > best) { best = l; best_off = i - (uint32_t)c; }
                c = prev[c];
            }
        }
        if (best >= 4) {
            seq[nseq].ll = i - lit_start;
            seq[nseq].ml = best;
            seq[nseq].off = best_off;
            nseq++;
            for (uint32_t k = i; k < i + best; k++)
                if (k + 4 <= n) { uint32_t h = lz_hash(x + k); prev[k] = head[h]; head[h] = (int32_t)k; }
            i += best;
            lit_start = i;
        } else {
            if (i + 4 <= n) { uint32_t h = lz_hash(x + i); prev[i] = head[h]; head[h] = (int32_t)i; }
            i++;
        }
    }
    if (lit_start < n || nseq == 0) {
        seq[nseq].ll = n - lit_start;
        seq[nseq].ml = 0;
        seq[nseq].off = 0;
        nseq++;
    }
    if (n == 0) nseq = 0;
    uint32_t next = 0, nlit = 0;
    for (uint32_t k = 0; k < nseq; k++) {
        next += (seq[k].ll >= 7) + (seq[k].ml >= 34);
        nlit += seq[k].ll;
    }
    uint64_t total = 16 + 3 * (uint64_t)nseq + 2 * (uint64_t)next + nlit;
    buf_resize(s, total);
    if (!s->bad) {
        put32(s->p + 0, nseq);
        put32(s->p + 4, nlit);
        put32(s->p + 8, next);
        put32(s->p + 12, n);
        uint8_t *offs = s->p + 16, *ext = offs + 2 * (uint64_t)nseq,
                *tags = ext + 2 * (uint64_t)next, *lits = tags + nseq;
        uint32_t e = 0, lp = 0, pos = 0;
        for (uint32_t k = 0; k < nseq; k++) {
            uint32_t lc, mc;
            if (seq[k].ll < 7) lc = seq[k].ll;
            else { lc = 7; put16(ext + 2 * (uint64_t)e++, seq[k].ll - 7); }
            if (seq[k].ml == 0) mc = 0;
            else if (seq[k].ml <= 33) mc = seq[k].ml - 3;
            else { mc = 31; put16(ext + 2 * (uint64_t)e++, seq[k].ml - 34); }
            put8(tags + k, lc | (mc << 3));
            put16(offs + 2 * (uint64_t)k, seq[k].off);
            memcpy(lits + lp, x + pos, seq[k].ll);
            lp += seq[k].ll;
            pos += seq[k].ll + seq[k].ml;
        }
        s->n = total;
    }
    free(head);
    free(prev);
    free(seq);
}

static int dec_lz77(const uint8_t *s, uint64_t comp_len, uint32_t plain_len, uint8_t *out) {
    if (comp_len < 16) return ZFO_ECORRUPT;
    uint32_t nseq = get32(s), nlit = get32(s + 4), next = get32(s + 8), plen = get32(s + 12);
    if (plen != plain_len || plain_len > LZ_MAX_CHUNK) return ZFO_ECORRUPT;
    if (16 + 3 * (uint64_t)nseq + 2 * (uint64_t)next + nlit != comp_len) return ZFO_ECORRUPT;
    const uint8_t *offs = s + 16, *ext = offs + 2 * (uint64_t)nseq,
                  *tags = ext + 2 * (uint64_t)next, *lits = tags + nseq;
    uint64_t p = 0, lp = 0, e = 0;
    for (uint32_t k = 0; k < nseq; k++) {
        uint32_t tag = tags[k], lc = tag & 7u, mc = tag >> 3, off = get16(offs + 2 * (uint64_t)k);
        uint64_t ll = lc, ml = 0;
        if (lc == 7) { if (e >= next) return ZFO_ECORRUPT; ll = 7 + get16(ext + 2 * e++); }
        if (mc == 31) { if (e >= next) return ZFO_ECORRUPT; ml = 34 + get16(ext + 2 * e++); }
        else if (mc > 0) ml = mc + 3;
        if (lp + ll > nlit || p + ll > plain_len) return ZFO_ECORRUPT;
        for (uint64_t j = 0; j < ll; j++) out[p + j] = lits[lp + j];
        p += ll;
        lp += ll;
        if (ml == 0) {
            if (off != 0) return ZFO_ECORRUPT;
            continue;
        }
        if (off == 0 || off > p || p + ml > plain_len) return ZFO_ECORRUPT;
        for (uint64_t j = 0; j < ml; j++) out[p + j] = out[p - off + j];
        p += ml;
    }
    if (p != plain_len || lp != nlit || e != next) return ZFO_ECORRUPT;
    return ZFO_OK;
}

/* ============================================================ per stream */
static int codec_allows(uint32_t codec, uint32_t dtype) {
    switch (codec) {
    case ZFO_PLAIN: return zfo_elem_size(dtype) != 0;
    case ZFO_FOR_BP:
    case ZFO_DELTA_BP:
    case ZFO_RLE_DELTA_BP: return dtype == ZFO_I32 || dtype == ZFO_I64;
    case ZFO_DICT_BP: return dtype == ZFO_I32 || dtype == ZFO_I64 || dtype == ZFO_FIXED16;
    case ZFO_LZ77: return zfo_elem_size(dtype) != 0;
    case ZFO_F2I_BP: return dtype == ZFO_F64;
    case ZFO_ANS: return zfo_elem_size(dtype) != 0;
    case ZFO_DSTRIDE_BP:
    case ZFO_DSTREE: return dtype == ZFO_I32 || dtype == ZFO_I64;
    case ZFO_SDICT_BP:
    case ZFO_SDICT_ANS:
    case ZFO_SDICT_COL:
    case ZFO_SDICT_COL_ANS: return dtype == ZFO_BYTES;
    default: return 0;
    }
}

int zfo_decode_stream(uint32_t codec, uint32_t dtype, const uint8_t *s, uint64_t comp_len,
                      uint32_t n, const uint8_t *dict, uint32_t dict_count, void *dstv) {
    uint8_t *dst = (uint8_t *)dstv;
    uint32_t es = zfo_elem_size(dtype);
    if (!codec_allows(codec, dtype) || n == 0) return ZFO_ECORRUPT;
    uint64_t plain = (uint64_t)n * es;
    switch (codec) {
    case ZFO_PLAIN:
        if (comp_len != plain) return ZFO_ECORRUPT;
        memcpy(dst, s, plain);
        return ZFO_OK;
    case ZFO_LZ77:
        if (plain > LZ_MAX_CHUNK) return ZFO_ECORRUPT;
        return dec_lz77(s, comp_len, (uint32_t)plain, dst);
    case ZFO_DELTA_BP:
    case ZFO_RLE_DELTA_BP:
        return dec_rle_delta(s, comp_len, dtype, n, codec == ZFO_DELTA_BP, dst);
    case ZFO_F2I_BP:
        return dec_f2i_bp(s, comp_len, n, dst);
    case ZFO_ANS:
        return dec_ans(s, comp_len, (uint32_t)plain, dst);
    case ZFO_DSTRIDE_BP:
        return dec_dstride(s, comp_len, dtype, n, dst);
    case ZFO_DSTREE:
        return dec_dstree(s, comp_len, dtype, n, dst);
    case ZFO_SDICT_BP:
        return dec_sdict(s, comp_len, (uint32_t)plain, dst);
    case ZFO_SDICT_ANS:
        return dec_sdict_ans(s, comp_len, (uint32_t)plain, dst);
    case ZFO_SDICT_COL:
        return dec_sdict_col(s, comp_len, (uint32_t)plain, dict, dict_count, dst);
    case ZFO_SDICT_COL_ANS:
        return dec_sdict_col_ans(s, comp_len, (uint32_t)plain, dict, dict_count, dst);
    case ZFO_FOR_BP:
    case ZFO_DICT_BP: {
        uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * n);
        if (!tmp) return ZFO_ENOMEM;
        uint32_t bits = codec == ZFO_DICT_BP ? 32u : int_bits(dtype);
        int rc = dec_for_bp_u64(s, comp_len, n, bits, tmp);
        for (uint32_t j = 0; rc == ZFO_OK && j < n; j++) {
            if (codec == ZFO_FOR_BP) store_int(dst, dtype, j, tmp[j]);
            else if (tmp[j] >= dict_count || !dict) rc = ZFO_ECORRUPT;
            else memcpy(dst + (uint64_t)j * es, dict + tmp[j] * es, es);
        }
        free(tmp);
        return rc;
    }
    }
    return ZFO_ECORRUPT;
}

/* ============================================================= container */
void zfo_free(void *p) { free(p); }

int zfo_encode(const void *srcv, uint64_t n_elems, uint32_t dtype, uint32_t codec,
               const uint32_t *chunk_elems, uint32_t n_chunks, const uint32_t *codecs,
               uint8_t **out, uint64_t *out_len) {
    const uint8_t *src = (const uint8_t *)srcv;
    uint32_t es = zfo_elem_size(dtype);
    if (!es || !out || !out_len) return ZFO_EINVAL;
    uint64_t sum = 0;
    int any_dict = 0, any_tdict = 0;
    for (uint32_t i = 0; i < n_chunks; i++) {
        uint32_t c = codecs ? codecs[i] : codec;
        if (chunk_elems[i] == 0 || !codec_allows(c, dtype)) return ZFO_EINVAL;
        if (c == ZFO_LZ77 && (uint64_t)chunk_elems[i] * es > LZ_MAX_CHUNK) return ZFO_EINVAL;
        if ((uint64_t)chunk_elems[i] * es > 0xFFFFFFFFu) return ZFO_EINVAL;
        any_dict |= c == ZFO_DICT_BP;
        any_tdict |= c == ZFO_SDICT_COL || c == ZFO_SDICT_COL_ANS;
        sum += chunk_elems[i];
    }
    if (sum != n_elems) return ZFO_EINVAL;
    int mixed = 0;
    for (uint32_t i = 1; i < n_chunks; i++)
        if ((codecs ? codecs[i] : codec) != (codecs ? codecs[0] : codec)) mixed = 1;

    uint8_t *dict = NULL;
    uint32_t dict_count = 0;
    uint64_t dl = 0;  /* dictionary area bytes */
    tdict_t td;
    memset(&td, 0, sizeof td);
    if (any_dict) {
        int rc = build_dict(src, n_elems, dtype, &dict, &dict_count);
        if (rc) return rc;
        dl = (uint64_t)dict_count * es;
    } else if (any_tdict) {
        int rc = tdict_build(src, chunk_elems, n_chunks, codecs, codec, &td, &dict, &dl, &dict_count);
        if (rc) return rc;
    }
    uint64_t table_end = 64 + (uint64_t)32 * n_chunks;
    uint64_t dict_off = dict_count ? align16(table_end) : 0;
    uint64_t pos = align16(dict_count ? dict_off + dl : table_end);

    buf_t b = {0};
    buf_resize(&b, pos);
    uint64_t plain_off = 0;
    uint32_t *codes = NULL;
    for (uint32_t i = 0; i < n_chunks && !b.bad; i++) {
        uint32_t c = codecs ? codecs[i] : codec, n = chunk_elems[i];
        const uint8_t *x = src + plain_off;
        buf_t s = {0};
        switch (c) {
        case ZFO_PLAIN:
            buf_resize(&s, (uint64_t)n * es);
            if (!s.bad) memcpy(s.p, x, (uint64_t)n * es);
            break;
        case ZFO_FOR_BP: enc_for_bp(&s, x, dtype, n); break;
        case ZFO_DICT_BP:
            codes = (uint32_t *)realloc(codes, sizeof(uint32_t) * n);
            if (!codes) { s.bad = 1; break; }
            for (uint32_t j = 0; j < n; j++)
                codes[j] = dict_code(dict, dict_count, dtype, x + (uint64_t)j * es);
            {
                /* the code sequence as an I32 column */
                uint8_t *cb = (uint8_t *)malloc((uint64_t)4 * n);
                if (!cb) { s.bad = 1; break; }
                for (uint32_t j = 0; j < n; j++) put32(cb + 4 * (uint64_t)j, codes[j]);
                enc_for_bp(&s, cb, ZFO_I32, n);
                free(cb);
            }
            break;
        case ZFO_DELTA_BP: enc_rle_delta(&s, x, dtype, n, 1); break;
        case ZFO_RLE_DELTA_BP: enc_rle_delta(&s, x, dtype, n, 0); break;
        case ZFO_LZ77: enc_lz77(&s, x, n * es); break;
        case ZFO_F2I_BP: enc_f2i_bp(&s, x, n); break;
        case ZFO_ANS: enc_ans(&s, x, n * es); break;
        case ZFO_DSTRIDE_BP: enc_dstride(&s, x, dtype, n); break;
        case ZFO_DSTREE: enc_dstree(&s, x, dtype, n); break;
        case ZFO_SDICT_BP: enc_sdict(&s, x, n); break;
        case ZFO_SDICT_ANS: enc_sdict_ans(&s, x, n); break;
        case ZFO_SDICT_COL: enc_sdict_col(&s, &td, plain_off, n, dict_count); break;
        case ZFO_SDICT_COL_ANS: enc_sdict_col_ans(&s, &td, plain_off, n, dict_count); break;
        }
        if (s.bad || s.n > 0xFFFFFFFFu) { free(s.p); b.bad = 1; break; }
        buf_resize(&b, pos + s.n);
        if (!b.bad) {
            memcpy(b.p + pos, s.p, s.n);
            uint8_t *e = b.p + 64 + (uint64_t)32 * i;
            put64(e + 0, plain_off);
            put64(e + 8, pos);
            put32(e + 16, n * es);
            put32(e + 20, (uint32_t)s.n);
            put32(e + 24, n);
            put8(e + 28, c);
        }
        free(s.p);
        pos = align16(pos + s.n);
        plain_off += (uint64_t)n * es;
    }
    free(codes);
    tdict_free(&td);
    buf_resize(&b, pos);
    if (b.bad) { free(b.p); free(dict); return ZFO_ENOMEM; }
    if (dict_count) memcpy(b.p + dict_off, dict, dl);
    free(dict);

    uint8_t *h = b.p;
    memcpy(h, "ZFC1", 4);
    put16(h + 4, 1);
    put8(h + 6, dtype);
    /* the column codec byte is 0 when the chunks mix codecs */
    uint32_t col_codec = n_chunks == 0 ? codec : (codecs ? codecs[0] : codec);
    put8(h + 7, mixed ? 0 : col_codec);
    put64(h + 8, n_elems);
    put64(h + 16, n_elems * es);
    put32(h + 24, n_chunks);
    put32(h + 28, dict_count);
    put64(h + 32, dict_off);
    put64(h + 40, pos);
    /* table CRC covers the chunk table followed by the dictionary */
    uint64_t tl = (uint64_t)32 * n_chunks;
    uint8_t *tmp = (uint8_t *)malloc(tl + dl + 1);
    if (!tmp) { free(b.p); return ZFO_ENOMEM; }
    memcpy(tmp, h + 64, tl);
    if (dl) memcpy(tmp + tl, h + dict_off, dl);
    put32(h + 48, zfo_crc32(tmp, tl + dl));
    free(tmp);
    put32(h + 52, 0);
    put32(h + 56, 0);
    put32(h + 60, zfo_crc32(h, 60));
    *out = b.p;
    *out_len = pos;
    return ZFO_OK;
}

int zfo_inspect(const uint8_t *blob, uint64_t len, zfo_info *info) {
    if (!blob || len < 64) return ZFO_ECORRUPT;
    if (memcmp(blob, "ZFC1", 4) != 0 || get16(blob + 4) != 1) return ZFO_ECORRUPT;
    if (get32(blob + 60) != zfo_crc32(blob, 60)) return ZFO_ECORRUPT;
    zfo_info in;
    in.dtype = blob[6];
    in.codec = blob[7];
    in.n_elems = get64(blob + 8);
    in.plain_bytes = get64(blob + 16);
    in.n_chunks = get32(blob + 24);
    in.dict_count = get32(blob + 28);
    in.dict_off = get64(blob + 32);
    in.total_bytes = get64(blob + 40);
    uint32_t es = zfo_elem_size(in.dtype);
    if (!es || in.plain_bytes != in.n_elems * es || in.total_bytes != len) return ZFO_ECORRUPT;
    uint64_t tl = (uint64_t)32 * in.n_chunks;
    if (64 + tl > len) return ZFO_ECORRUPT;
    uint64_t dl = (uint64_t)in.dict_count * es;
    if (in.dict_count && in.dtype == ZFO_BYTES) {
        /* a token dictionary: its size follows from its entry-byte count */
        if (in.dict_off % 16 != 0 || in.dict_off < 64 + tl || in.dict_off + 16 > len) return ZFO_ECORRUPT;
        uint32_t nb = get32(blob + in.dict_off);
        if (nb > SDC_MAX_BYTES || in.dict_count > SDC_MAX_ENTRIES) return ZFO_ECORRUPT;
        dl = 16 + 4 * (uint64_t)in.dict_count + align16(nb);
        if (in.dict_off + dl > len) return ZFO_ECORRUPT;
        /* every entry inside the bytes with three zero bytes on each side */
        const uint8_t *ents = blob + in.dict_off + 16, *bytes = ents + 4 * (uint64_t)in.dict_count;
        for (uint32_t k = 0; k < in.dict_count; k++) {
            uint32_t e = get32(ents + 4 * (uint64_t)k), off = e & 0xFFFFFFu, el = e >> 24;
            if (el == 0 || el > SD_MAX_TOKEN || off < 3 || (uint64_t)off + el + 3 > nb || (uint64_t)off + 16 > nb)
                return ZFO_ECORRUPT;
            for (uint32_t q = 1; q <= 3; q++)
                if (bytes[off - q] != 0 || bytes[off + el + q - 1] != 0) return ZFO_ECORRUPT;
        }
    }
    if (in.dict_count) {
        if (in.dict_off % 16 != 0 || in.dict_off < 64 + tl || in.dict_off + dl > len)
            return ZFO_ECORRUPT;
    } else if (in.dict_off != 0) return ZFO_ECORRUPT;
    uint8_t *tmp = (uint8_t *)malloc(tl + dl + 1);
    if (!tmp) return ZFO_ENOMEM;
    memcpy(tmp, blob + 64, tl);
    if (dl) memcpy(tmp + tl, blob + in.dict_off, dl);
    uint32_t crc = zfo_crc32(tmp, tl + dl);
    free(tmp);
    if (crc != get32(blob + 48)) return ZFO_ECORRUPT;
    /* chunks tile the plain bytes in order and sit inside the blob */
    uint64_t plain_off = 0, elems = 0;
    for (uint32_t i = 0; i < in.n_chunks; i++) {
        zfo_chunk c;
        zfo_get_chunk(blob, len, i, &c);
        if (c.plain_off != plain_off || c.n_elems == 0 || (uint64_t)c.n_elems * es != c.plain_len)
            return ZFO_ECORRUPT;
        if (c.comp_off % 16 != 0 || c.comp_off < 64 + tl || c.comp_off + c.comp_len > len)
            return ZFO_ECORRUPT;
        if (!codec_allows(c.codec, in.dtype)) return ZFO_ECORRUPT;
        if ((c.codec == ZFO_DICT_BP || c.codec == ZFO_SDICT_COL || c.codec == ZFO_SDICT_COL_ANS) &&
            in.dict_count == 0)
            return ZFO_ECORRUPT;
        plain_off += c.plain_len;
        elems += c.n_elems;
    }
    if (plain_off != in.plain_bytes || elems != in.n_elems) return ZFO_ECORRUPT;
    if (info) *info = in;
    return ZFO_OK;
}

int zfo_get_chunk(const uint8_t *blob, uint64_t len, uint32_t i, zfo_chunk *c) {
    if (len < 64 || i >= get32(blob + 24) || 64 + (uint64_t)32 * (i + 1) > len) return ZFO_EINVAL;
    const uint8_t *e = blob + 64 + (uint64_t)32 * i;
    c->plain_off = get64(e);
    c->comp_off = get64(e + 8);
    c->plain_len = get32(e + 16);
    c->comp_len = get32(e + 20);
    c->n_elems = get32(e + 24);
    c->codec = e[28];
    return ZFO_OK;
}

int zfo_decode_chunks(const uint8_t *blob, uint64_t len, uint32_t first, uint32_t count,
                      void *dstv, uint64_t dst_len) {
    zfo_info in;
    int rc = zfo_inspect(blob, len, &in);
    if (rc) return rc;
    if ((uint64_t)first + count > in.n_chunks) return ZFO_EINVAL;
    uint8_t *dst = (uint8_t *)dstv;
    uint64_t need = 0;
    for (uint32_t i = first; i < first + count; i++) {
        zfo_chunk c;
        zfo_get_chunk(blob, len, i, &c);
        need += c.plain_len;
    }
    if (need != dst_len) return ZFO_EINVAL;
    uint64_t at = 0;
    const uint8_t *dict = in.dict_count ? blob + in.dict_off : NULL;
    for (uint32_t i = first; i < first + count; i++) {
        zfo_chunk c;
        zfo_get_chunk(blob, len, i, &c);
        rc = zfo_decode_stream(c.codec, in.dtype, blob + c.comp_off, c.comp_len, c.n_elems, dict,
                               in.dict_count, dst + at);
        if (rc) return rc;
        at += c.plain_len;
    }
    return ZFO_OK;
}

int zfo_decode(const uint8_t *blob, uint64_t len, void *dst, uint64_t dst_len) {
    zfo_info in;
    int rc = zfo_inspect(blob, len, &in);
    if (rc) return rc;
    if (dst_len != in.plain_bytes) return ZFO_EINVAL;
    return zfo_decode_chunks(blob, len, 0, in.n_chunks, dst, dst_len);
}
