/*
 * zfo -- the oracle: a plain, single-threaded, obviously-correct CPU encoder
 * and decoder for every codec of the zf column format.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The GPU product path never links,
 * calls or includes anything from here, and this code includes nothing from
 * the product.
 *
 * Every codec here is lossless, so the plain definition of a decode is the
 * original column itself (ZipFlow paper, Sec. 2.1: dictionary, delta, RLE,
 * FOR + bit-packing, LZ77).  The byte layout of each stream is the zf format,
 * which the paper leaves open; it is written out in the comments of zfo.c.
 */
#ifndef ZFO_H
#define ZFO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dtypes */
#define ZFO_I32 1
#define ZFO_I64 2
#define ZFO_BYTES 3
#define ZFO_FIXED16 4
#define ZFO_F64 5

/* codecs */
#define ZFO_PLAIN 1
#define ZFO_FOR_BP 2
#define ZFO_DICT_BP 3
#define ZFO_DELTA_BP 4
#define ZFO_RLE_DELTA_BP 5
#define ZFO_LZ77 6
#define ZFO_F2I_BP 7
#define ZFO_ANS 8
#define ZFO_DSTRIDE_BP 9
#define ZFO_SDICT_BP 10
#define ZFO_SDICT_ANS 11
#define ZFO_SDICT_COL 12
#define ZFO_SDICT_COL_ANS 13
#define ZFO_DSTREE 14

/* status */
#define ZFO_OK 0
#define ZFO_EINVAL 1
#define ZFO_EUNSUP 2
#define ZFO_ECORRUPT 3
#define ZFO_ENOMEM 4

typedef struct {
    uint32_t dtype, codec, n_chunks, dict_count;
    uint64_t n_elems, plain_bytes, dict_off, total_bytes;
} zfo_info;

typedef struct {
    uint64_t plain_off, comp_off;
    uint32_t plain_len, comp_len, n_elems, codec;
} zfo_chunk;

uint32_t zfo_crc32(const uint8_t *p, uint64_t n);
uint32_t zfo_elem_size(uint32_t dtype);

/* Encode a whole column.  chunk_elems[i] values go into chunk i;
 * codecs (nullable) gives a per-chunk codec, else `codec` is used for all.
 * *out is malloc'd; free it with zfo_free. */
int zfo_encode(const void *src, uint64_t n_elems, uint32_t dtype, uint32_t codec,
               const uint32_t *chunk_elems, uint32_t n_chunks, const uint32_t *codecs,
               uint8_t **out, uint64_t *out_len);
void zfo_free(void *p);

/* Validate a column blob and report its header. */
int zfo_inspect(const uint8_t *blob, uint64_t len, zfo_info *info);
int zfo_get_chunk(const uint8_t *blob, uint64_t len, uint32_t i, zfo_chunk *c);

/* Decode a whole column into dst (dst_len must equal plain_bytes). */
int zfo_decode(const uint8_t *blob, uint64_t len, void *dst, uint64_t dst_len);
/* Decode chunks [first, first+count) into dst (their plain bytes, in order). */
int zfo_decode_chunks(const uint8_t *blob, uint64_t len, uint32_t first, uint32_t count,
                      void *dst, uint64_t dst_len);

/* Single-stream decoders, for streams assembled by hand in tests.  `dict`
 * is needed by DICT_BP only.  Return ZFO_OK or ZFO_ECORRUPT. */
int zfo_decode_stream(uint32_t codec, uint32_t dtype, const uint8_t *s, uint64_t comp_len,
                      uint32_t n_elems, const uint8_t *dict, uint32_t dict_count, void *dst);

#ifdef __cplusplus
}
#endif
#endif
