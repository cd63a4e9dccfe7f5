/*
 * zf.h -- C ABI of the zf library: compressed column chunks move from pinned
 * host memory to an MI355X over PCIe and are decoded there by HIP kernels.
 *
 * The calls follow the problem statement of the ZipFlow paper (Sec. 3,
 * "Design"): columns are compressed on the CPU and kept in CPU memory;
 * online, the compressed bytes cross PCIe and a device-specific decoder
 * expands them in GPU memory, with copies and decodes of successive blocks
 * overlapped (Sec. 3.3) and kernels instantiated per device (Sec. 4).
 *
 * Conventions for every call:
 *   - plain C types only; pointers are host pointers unless named d_*;
 *     a zf_stream_t is a hipStream_t (NULL = the legacy default stream).
 *   - every call returns a zf_status; on failure the out-parameters are left
 *     untouched and zf_last_error() holds a message for the calling thread.
 *   - no C++ exception crosses this boundary.
 *
 * Column byte format (little-endian), shared by every codec:
 *   64-byte header: "ZFC1", u16 version = 1, u8 dtype, u8 codec (0 when the
 *     chunks mix codecs), u64 n_elems, u64 plain_bytes, u32 n_chunks,
 *     u32 dict_count, u64 dict_off, u64 total_bytes, u32 table_crc,
 *     u32 0, u32 0, u32 header_crc (CRC-32 of header bytes [0,60)).
 *   chunk table at 64: per chunk 32 bytes {u64 plain_off, u64 comp_off,
 *     u32 plain_len, u32 comp_len, u32 n_elems, u8 codec, u8 schedule hint
 *     (0 = tuned default, 1..4 = tile granularity chosen at encode time;
 *     decoding does not depend on it), 2 zero bytes}.
 *   dictionary (dict_count > 0) at dict_off: sorted unique values (dtype
 *     BYTES: the token dictionary described at ZF_SDICT_COL).
 *   chunk streams at 16-aligned comp_off.  table_crc = CRC-32 of the chunk
 *   table followed by the dictionary.  The per-codec streams are described
 *   at zf_codec below.
 */
#ifndef ZF_H
#define ZF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ZF_OK = 0,
    ZF_E_INVALID = 1,     /* bad argument (null pointer, size mismatch, bad enum) */
    ZF_E_UNSUPPORTED = 2, /* valid request this library does not handle        */
    ZF_E_CORRUPT = 3,     /* stream failed validation on the host or the device */
    ZF_E_NOMEM = 4,       /* host or device allocation failed                   */
    ZF_E_HIP = 5,         /* a HIP runtime call failed                          */
    ZF_E_TOO_SMALL = 6,   /* a caller buffer is smaller than required           */
    ZF_E_STATE = 7        /* call out of order (e.g. plan already failed)       */
} zf_status;

typedef enum {
    ZF_I32 = 1,     /* int32 values                        */
    ZF_I64 = 2,     /* int64 values                        */
    ZF_BYTES = 3,   /* byte column (e.g. text)             */
    ZF_FIXED16 = 4, /* 16-byte fixed-width strings, CHAR(16) */
    ZF_F64 = 5      /* IEEE binary64 values                 */
} zf_dtype;

/*
 * Codecs (Sec. 2.1 defines the algorithms; Sec. 3.1 classifies them as
 * Fully-Parallel, Group-Parallel or Non-Parallel):
 *  ZF_PLAIN         raw bytes.
 *  ZF_FOR_BP        [FP] frame of reference + bit-packing, blocks of 2048:
 *                   16-byte directory {i64 ref = block minimum, u32 w, u32 poff}
 *                   per block, payload of w-bit fields, LSB-first in LE u32
 *                   words; value = ref + field (mod 2^bits).  I32, I64.
 *  ZF_DICT_BP       [FP] dictionary + bit-packing: the column dictionary is
 *                   the sorted distinct values; a chunk is the FOR_BP stream
 *                   of the dictionary indices; value = dict[code].
 *                   I32, I64, FIXED16.
 *  ZF_DELTA_BP      [GP] delta + bit-packing: ZF_RLE_DELTA_BP with every run
 *                   of length one and no run array.  I32, I64.
 *  ZF_RLE_DELTA_BP  [GP] RLE; run values delta-coded and bit-packed; groups
 *                   of 64 runs, each with a 32-byte record {u32 out_off,
 *                   u32 w, u32 doff, u32 0, i64 base, i64 dmin}; header
 *                   {u32 n_runs, u32 n_groups, u32 runs_off, u32 0}; u32 run
 *                   lengths at runs_off.  I32, I64.
 *  ZF_LZ77          [NP] LZ77 sequences in chunks of <= 65536 bytes; header
 *                   {u32 n_seq, u32 n_lit, u32 n_ext, u32 plain_len}, u16
 *                   offsets[n_seq], u16 ext[n_ext], u8 tags[n_seq], literals.
 *                   Tag bits 0-2: literal count (7 = 7 + next ext), bits 3-7:
 *                   match code (0 none, 1..30 -> length code+3, 31 -> 34 +
 *                   next ext).  Any dtype (decoded as bytes).
 *  ZF_F2I_BP        [FP] Float2Int + bit-packing (Sec. 2.1; layout ours):
 *                   per block of 2048 values an exponent e <= 18 and
 *                   integers d with bits(v) == bits((double)d / 10^e) (IEEE
 *                   division), FOR + bit-packed; values with no such d are
 *                   exceptions stored raw.  32-byte directory {i64 ref, u32 w,
 *                   u32 poff, u32 xoff, u16 nx, u8 e, u8 0, 8 zero bytes};
 *                   exception records {u32 index in block (increasing), u32 0,
 *                   u64 bits} at xoff.  F64.
 *  ZF_ANS           [NP] range ANS over the chunk's bytes (Sec. 2.1), static
 *                   order-0 model with M = 4096 (frequencies quantised from
 *                   the byte counts), byte i coded by coder i mod 64, state
 *                   in [2^16, 2^32), 16-bit renormalisation.  Header {u32 n,
 *                   u32 nw, u32 0, u32 0}, u16 f[256], u32 final state[64],
 *                   then nw u16 words shared by the coders, in the order
 *                   the decoder reads them (byte order: each renormalisation
 *                   takes the next word).  Any dtype (decoded as bytes).
 *  ZF_DSTRIDE_BP    [GP] DeltaStride (Sec. 5): runs that are arithmetic
 *                   progressions (start, stride, count), maximal from the
 *                   left; groups of 64 runs, each with a 32-byte record
 *                   {u32 out_off, u32 poff, u32 widths (gap width bits 0-7,
 *                   stride width bits 8-15), u32 0, i64 base (first start),
 *                   i64 dmin}; at poff (8-aligned) an i64 gmin, the cnt-1
 *                   gap fields, then from the next u32 word the cnt stride
 *                   fields, FOR-bit-packed.  Start j >= 1 = start j-1 +
 *                   stride j-1 * count j-1 + gap j.  Header and u32 run
 *                   lengths as ZF_RLE_DELTA_BP.  I32, I64.
 *  ZF_DSTREE        [GP, two stages] DeltaStride | [Delta | RLE | [BP, BP],
 *                   BP], the order-key scheme of Sec. 5: stride d = the
 *                   chunk's most frequent neighbour difference (ties to the
 *                   smaller, unsigned); maximal runs of step d give starts S
 *                   and counts C; D = S[0], S[1] - S[0], ... is run-length
 *                   coded into values V and lengths L; V, L, C bit-packed per
 *                   group of 64 against the group minimum.  Header {u32 R,
 *                   u32 ngB, u32 Q, u32 ngA, i64 d, u32 b_off = 32 + 32 ngA,
 *                   u32 0}; D groups {u32 out_off, u32 poff, u32 widths (V
 *                   bits 0-7, L bits 8-15), u32 lmin, i64 base, i64 vmin} at
 *                   32; run groups {u32 out_off, u32 poff, u32 wc, u32 cmin}
 *                   at b_off; payloads after them (V fields, then L fields
 *                   from the next word; C fields).  The starts are decoded
 *                   into the plan's scratch area by one launch and expanded
 *                   by the next.  I32, I64.
 *  ZF_SDICT_BP      [GP] String-dictionary (Sec. 2.1, Sec. 5): tokens end
 *                   after ' ' or '.' (at most 64 bytes; the chunk's last may
 *                   end without one); distinct tokens in order of first
 *                   appearance are the entries.  Header {u32 n_tokens,
 *                   n_entries, w, n_groups, ent_off, bytes_off, codes_off,
 *                   n_bytes}; u32 output offset per 64 tokens at 32; u32
 *                   entries {offset bits 0-23, length bits 24-31} at ent_off
 *                   = align16(32 + 4 n_groups); entry bytes at bytes_off,
 *                   zero-padded to codes_off = align16(bytes_off + n_bytes +
 *                   4); n_tokens entry indices of w = bitlen(n_entries - 1)
 *                   bits at codes_off.  BYTES.
 *  ZF_SDICT_ANS     [GP, two stages] String-dictionary | bit-packing | ANS
 *                   (Sec. 5): the ZF_SDICT_BP stream with its packed entry
 *                   indices (4 ceil(n_tokens w / 32) bytes) replaced by the
 *                   ZF_ANS stream of those bytes (nothing when w = 0).  The
 *                   indices are ANS-decoded into the plan's scratch area by
 *                   one launch and expanded by the next (with the persistent
 *                   kernel: one persistent launch for the kinds up to RLE,
 *                   then one for the rest).  BYTES.
 *  ZF_SDICT_COL     [GP] String-dictionary over one dictionary for the whole
 *                   column (Sec. 5: one word dictionary for the comment
 *                   column; Sec. 2.1: it holds the data's frequent byte
 *                   sequences).  Tokens as ZF_SDICT_BP, except that '\n' (the
 *                   end of a row value) also ends one.  The column dictionary
 *                   sits in the container's dictionary area (dict_count =
 *                   entries): {u32 n_bytes, 3 u32 0, u32 entries {offset bits
 *                   0-23, length bits 24-31}, n_bytes entry bytes (the first
 *                   entry at 4, each next at align4(previous end + 3),
 *                   n_bytes = max(align4(last end + 3), last start + 16): at
 *                   least three zero bytes on each side of every entry and 16
 *                   bytes from each start within n_bytes), zero padding to a
 *                   multiple of 16}; entries
 *                   are the distinct tokens of the column's ZF_SDICT_COL /
 *                   ZF_SDICT_COL_ANS chunks by decreasing count, ties by first
 *                   appearance; at most 2^24 entries and 2^24 - 1 bytes
 *                   (ZF_E_UNSUPPORTED beyond).  Chunk: header {u32 n_tokens,
 *                   u32 w = bitlen(dict_count - 1), u32 n_groups, u32
 *                   codes_off = align16(16 + 4 n_groups)}, u32 output offset
 *                   per 64 tokens at 16, packed indices at codes_off.  BYTES.
 *  ZF_SDICT_COL_ANS [GP, two stages] ZF_SDICT_COL | bit-packing | ANS: the
 *                   packed indices replaced as in ZF_SDICT_ANS.  BYTES.
 */
typedef enum {
    ZF_AUTO = 0,
    ZF_PLAIN = 1,
    ZF_FOR_BP = 2,
    ZF_DICT_BP = 3,
    ZF_DELTA_BP = 4,
    ZF_RLE_DELTA_BP = 5,
    ZF_LZ77 = 6,
    ZF_F2I_BP = 7,
    ZF_ANS = 8,
    ZF_DSTRIDE_BP = 9,
    ZF_SDICT_BP = 10,
    ZF_SDICT_ANS = 11,
    ZF_SDICT_COL = 12,
    ZF_SDICT_COL_ANS = 13,
    ZF_DSTREE = 14
} zf_codec;

typedef void *zf_stream_t;              /* a hipStream_t */
typedef struct zf_column zf_column_t;   /* compressed column, host memory */
typedef struct zf_plan zf_plan_t;       /* schedule + device workspace     */

typedef struct {
    uint32_t chunk_bytes_min;     /* uneven chunks: log-uniform plain size in  */
    uint32_t chunk_bytes_max;     /*  [min, max]; min == max gives fixed size  */
    uint64_t seed;                /* seed of the chunk-size draw               */
    int32_t n_threads;            /* encoder threads; 0 = all host cores       */
    int32_t pinned;               /* 1: hipHostMalloc (default); 0: malloc     */
    const uint32_t *chunk_elems;  /* explicit chunking (overrides the above)   */
    uint32_t n_chunk_elems;
    const uint32_t *chunk_codecs; /* per-chunk codec for explicit chunking     */
    const char *mlp_weights;      /* cost model for ZF_AUTO (NULL: $ZF_MLP_WEIGHTS;
                                     without one, ZF_AUTO keeps the smallest
                                     stream of the applicable codecs)         */
    int32_t fallback_device;      /* ZF_AUTO with a cost model: HIP device on
                                     which near-ties are timed; -1 (default):
                                     the network's choice stands              */
    float fallback_margin;        /* near-tie: the two lowest predicted log
                                     times differ by less than this (default
                                     0.05, about 5%); <= 0 turns timing off   */
} zf_encode_opts;

/* Defaults: chunks of 1 MiB plain (LZ77: 64 KiB), all cores, pinned, no
 * near-tie timing (fallback_device -1, fallback_margin 0.05). */
void zf_encode_opts_default(zf_encode_opts *opts);

/*
 * Compress n_elems values of `dtype` at src (host memory, read only, not
 * retained) into a new column (Sec. 3: compression runs on the CPU and the
 * result stays in CPU memory).  Chunks are encoded in parallel.  With codec
 * ZF_AUTO each chunk takes the codec the cost model predicts cheapest.
 * n_elems == 0 makes an empty column.  The column owns its memory (pinned by
 * default) until zf_column_free.  Errors: ZF_E_INVALID (dtype/codec mix,
 * null pointers, chunking that does not sum to n_elems, LZ77 chunks above
 * 65536 bytes), ZF_E_NOMEM.
 * ZF_AUTO with a cost model: each chunk's statistics (zf_chunk_features) go
 * through the network and the chunk takes the applicable (codec, schedule)
 * with the lowest predicted transfer + decode time; the schedule is stored in
 * the chunk table (LZ77 chunks are split at the chosen chunk size).  With
 * fallback_device >= 0, a chunk whose two best predictions are within
 * fallback_margin is encoded both ways on its own, each candidate's
 * zf_transfer_and_decompress time is measured on that device (median of three
 * after one untimed run) and the faster is kept (Sec. 3.3: measured search
 * behind the learned choice); errors of that device come back as ZF_E_HIP.
 */
zf_status zf_compress_host(const void *src, uint64_t n_elems, zf_dtype dtype, zf_codec codec,
                           const zf_encode_opts *opts /* nullable */, zf_column_t **out);

/* The 32 statistics the cost model reads for a chunk of n_elems values at
 * src (host memory), computed on its first 65,536 values: sizes, value range
 * and FOR widths, distinct count and top frequencies, byte and value entropy,
 * order, runs and deltas, text shape, repeats of 4-byte strings, and
 * closed-form size estimates per codec.  out receives ZF_FEATURES floats. */
#define ZF_FEATURES 32
zf_status zf_chunk_features(const void *src, uint64_t n_elems, zf_dtype dtype, float *out);

/* Adopt a serialised column (copied; `pinned` as in zf_encode_opts).  The
 * header, CRCs, chunk table and every stream's directory are validated;
 * ZF_E_CORRUPT on failure. */
zf_status zf_column_from_bytes(const void *buf, uint64_t len, int32_t pinned, zf_column_t **out);
/* Serialised bytes of a column (owned by the column). */
const void *zf_column_bytes(const zf_column_t *col, uint64_t *len);
uint64_t zf_column_plain_bytes(const zf_column_t *col);
uint64_t zf_column_n_elems(const zf_column_t *col);
uint32_t zf_column_n_chunks(const zf_column_t *col);
int32_t zf_column_dtype(const zf_column_t *col);
void zf_column_free(zf_column_t *col);

/* Kernel kinds: one decode routine per pattern class and value width. */
typedef enum {
    ZF_KIND_LZ77 = 0,
    ZF_KIND_ANS,     /* range ANS, one chunk per wavefront */
    ZF_KIND_RLE64,   /* RLE_DELTA_BP, DELTA_BP and DSTRIDE_BP, int64 */
    ZF_KIND_RLE32,   /* RLE_DELTA_BP, DELTA_BP and DSTRIDE_BP, int32 */
    ZF_KIND_SDICT,   /* SDICT_BP (String-dictionary), bytes */
    ZF_KIND_DICT128,
    ZF_KIND_DICT64,
    ZF_KIND_DICT32,
    ZF_KIND_FOR64,
    ZF_KIND_FOR32,
    ZF_KIND_F2I,     /* Float2Int + bit-packing, float64 */
    ZF_KIND_PLAIN,
    ZF_KIND_TREE,    /* DSTREE output stage (its run starts decode in RLE32/RLE64) */
    ZF_KIND_COUNT
} zf_kind;

/* Tile shape of one kind, the device geometry of Sec. 4 (<L,S,C>): `unit`
 * is the work of one wavefront (FP: 2048-value blocks; GP: output elements;
 * PLAIN: bytes; LZ77: output bytes per block of the copy step, 4, 8 or 16,
 * one chunk per wavefront; the persistent kernel always uses 4; SDICT:
 * output bytes, in whole groups of 64 tokens),
 * `waves_per_block`
 * the wavefronts per workgroup (S/64; SDICT: at most 12, or 14 and 16, which
 * run the units over column dictionaries as two workgroups per compute unit
 * over contiguous ranges of units, each sharing an LDS copy of the hottest
 * records of a column dictionary and staging through 2 KiB buffers, and
 * the other units in a second launch of 4-wave workgroups).  A lane always owns 16 output bytes per
 * step (C).  Zero fields take the tune cache's value, else a default. */
typedef struct {
    uint32_t unit;
    uint32_t waves_per_block;
} zf_tile;

typedef struct {
    uint64_t slot_bytes;     /* staging slot size for transfers (default 256 MiB) */
    int32_t n_slots;         /* staging slots, >= 1 (default 2: double buffering)   */
    int32_t use_graphs;      /* 1: one hipGraph per batch (default); 0: plain launches */
    int32_t persistent;      /* 1: a persistent multi-codec kernel per batch (two
                                ordered launches when two-stage chunks are present),
                                its waves pulling units from one queue per XCD;
                                0: one launch per kernel kind (default)             */
    int32_t order;           /* 0: Johnson order (default); 1: column order          */
    double pcie_gbps;        /* transfer-time estimate for ordering (0: 55)          */
    zf_tile tiles[ZF_KIND_COUNT];
    uint32_t waves_per_cu;   /* persistent kernel: waves in flight per CU (0: 16)    */
    const char *tune_cache;  /* tile cache (JSON); NULL: $ZF_TUNE_CACHE, else the
                                tune_gfx950.json next to libzf.so, else defaults    */
} zf_plan_opts;

void zf_plan_opts_default(zf_plan_opts *opts);

/*
 * Build a plan for decoding `cols` on HIP device `device`: per-chunk tiles
 * from the tune cache (Sec. 4, device geometry scheduling), batches of chunks
 * no larger than one staging slot, the batch order by Johnson's rule on
 * (transfer, decode) estimates (Sec. 3.3), and the device workspace (tables,
 * staging slots, error word, graphs, and a 16-byte record per entry of every
 * column token dictionary: the entry's first 15 bytes, zero past its length,
 * then its length, which the String-dictionary kernel reads instead of the
 * image's entry for tokens of up to 15 bytes).  The columns must outlive the
 * plan and must not change, and a device image given to
 * zf_decompress_async must hold these same columns.  Errors: ZF_E_INVALID,
 * ZF_E_CORRUPT (host validation of every stream header), ZF_E_NOMEM,
 * ZF_E_HIP.
 */
zf_status zf_plan(const zf_column_t *const *cols, uint32_t n_cols, int32_t device,
                  const zf_plan_opts *opts /* nullable */, zf_plan_t **out);
void zf_plan_free(zf_plan_t *plan);

/*
 * Batches of a plan in execution order (Sec. 3.3: each batch is a two-stage
 * job, its PCIe copy then its decode, and the plan orders the batches by
 * Johnson's rule for the two-machine flow shop).  For batch k (0-based, in
 * execution order) zf_plan_batch_info fills:
 *   t_h2d_ms   copy-time estimate: compressed bytes / the plan's PCIe rate
 *              (zf_plan_opts.pcie_gbps, default 55 GB/s);
 *   t_dec_ms   decode-time estimate: per chunk, plain bytes / the measured
 *              rate of its kernel kind in the tune cache (plain_GBps);
 *   comp_bytes, plain_bytes, n_chunks   the batch's chunks;
 *   index      the batch's position in column order, before ordering.
 * Errors: ZF_E_INVALID (null pointer, k >= zf_plan_n_batches).
 */
typedef struct {
    double t_h2d_ms, t_dec_ms;
    uint64_t comp_bytes, plain_bytes;
    uint32_t n_chunks, index;
} zf_batch_info;
uint32_t zf_plan_n_batches(const zf_plan_t *plan);
zf_status zf_plan_batch_info(const zf_plan_t *plan, uint32_t k, zf_batch_info *info);

/*
 * Johnson's rule (Sec. 3.3), the order zf_plan gives its batches: jobs with
 * a[i] < b[i] first, by increasing a; then the others, by decreasing b; equal
 * keys keep the lower index first.  a, b: n first- and second-stage times
 * (host arrays, read only); order: n job indices written by the call (host
 * array owned by the caller).  Host only, no device needed.  Errors:
 * ZF_E_INVALID (null pointer with n > 0, a NaN time).
 */
zf_status zf_johnson_order(const double *a, const double *b, uint32_t n, uint32_t *order);

/*
 * The work units the planner cuts one chunk into, each decoded by one
 * wavefront (the device geometry of Sec. 4).  units[i] = {kind (a zf_kind),
 * a, b, c}: FP kinds (FOR, DICT, F2I): first 2048-value block, block count,
 * 0; RLE32, RLE64, TREE: first group, first element, end element; SDICT:
 * first group of 64 tokens, end group, 0; PLAIN: first byte, end byte, 0;
 * LZ77 and ANS: 0, 0, 0 (the whole stream).  A two-stage chunk lists its
 * first-stage units first (ANS pieces of SDICT_ANS / SDICT_COL_ANS, the run
 * starts of DSTREE in RLE32 / RLE64), then the units of its output stage.
 * Tiles come from opts (nullable: the tune cache, as zf_plan takes them)
 * and the chunk's schedule hint.  units: caller-owned host array of cap
 * entries; with units NULL and cap 0 only *n_units is set.  Host only, no
 * device needed.  Errors: ZF_E_INVALID (null column or n_units, chunk out
 * of range), ZF_E_TOO_SMALL (cap below the unit count).
 */
typedef struct {
    uint32_t kind, a, b, c;
} zf_unit;
zf_status zf_chunk_units(const zf_column_t *col, uint32_t chunk, const zf_plan_opts *opts,
                         zf_unit *units, uint32_t cap, uint32_t *n_units);

/* Device image for zf_decompress_async: column c's serialised bytes go at
 * byte offset zf_plan_image_offset(plan, c) of a device buffer of
 * zf_plan_image_bytes(plan) bytes (offsets are 256-aligned). */
uint64_t zf_plan_image_bytes(const zf_plan_t *plan);
uint64_t zf_plan_image_offset(const zf_plan_t *plan, uint32_t col);

/*
 * Decode every column of the plan from a device image already in HBM
 * (d_comp, laid out as above) into d_out[c] (device buffers of exactly
 * zf_column_plain_bytes(cols[c]) bytes, 16-aligned), enqueued on `stream`.
 * The image must hold the same bytes the plan was built from; kernels
 * re-check every offset they use against the plan's sizes, never read or
 * write out of bounds, and latch corruption into the plan's error word
 * (reported by zf_sync).  Returns after enqueueing.  A plan serves one
 * stream at a time.
 */
zf_status zf_decompress_async(zf_plan_t *plan, const void *d_comp, uint64_t comp_bytes,
                              void *const *d_out, zf_stream_t stream);

typedef struct {
    double h2d_ms;       /* sum of copy durations                       */
    double decode_ms;    /* sum of decode durations                     */
    double wall_ms;      /* first copy start to last decode end         */
    uint64_t plain_bytes, comp_bytes;
} zf_timing;

/*
 * Transfer and decode (Sec. 3.3): for each batch in plan order, the copy
 * stream waits for its staging slot to be free, copies the batch's
 * compressed chunks from the columns' pinned memory over PCIe, and signals;
 * `stream` waits for that signal and runs the batch's decode graph.  With two
 * slots the copy of batch k+1 overlaps the decode of batch k.  Outputs as in
 * zf_decompress_async.  `timing` (nullable) is filled by zf_sync.
 */
zf_status zf_transfer_and_decompress(zf_plan_t *plan, void *const *d_out, zf_stream_t stream,
                                     zf_timing *timing);

/*
 * Kernel times inside a decode (measurement, Sec. 5.1): after
 * zf_plan_profile(plan, 1), every zf_decompress_async of the plan records a
 * HIP event on its stream before and after each kernel kind's launch (the
 * persistent kernel as a whole).  zf_plan_kind_ms then fills
 * ms[ZF_KIND_COUNT + 1] (host array owned by the caller) with the durations,
 * in ms, of the most recent such call: entry k for kind k, entry
 * ZF_KIND_COUNT for the persistent kernel, -1 where nothing was launched; it
 * waits for those events.  zf_plan_profile(plan, 0) stops recording.
 * Errors: ZF_E_INVALID (null pointer), ZF_E_STATE (no profiled decode since
 * profiling was switched on), ZF_E_HIP.
 */
zf_status zf_plan_profile(zf_plan_t *plan, int32_t on);
zf_status zf_plan_kind_ms(zf_plan_t *plan, double *ms);

/* Wait for the plan's work on `stream`; read the device error word:
 * ZF_E_CORRUPT if any kernel found a corrupt stream (sticky until
 * zf_plan_clear_error). */
zf_status zf_sync(zf_plan_t *plan, zf_stream_t stream);
void zf_plan_clear_error(zf_plan_t *plan);

/*
 * Learned (codec, schedule) choice: a cost-model network of 32 chunk
 * statistics -> 64 -> 64 -> 24 scores (6 codecs x 4 schedules; each a
 * predicted log of transfer + decode time), relu hidden layers, FP32.
 * Parameters are one flat device array of ZF_MLP_PARAMS floats:
 * W1 (64x32), b1 (64), W2 (64x64), b2 (64), W3 (24x64), b3 (24), row-major.
 * Inputs x are n x 32 row-major; outputs y are n x 24.  All pointers are
 * device pointers owned by the caller; calls are enqueued on `stream`.
 */
#define ZF_MLP_IN 32
#define ZF_MLP_HIDDEN 64
#define ZF_MLP_OUT 24
#define ZF_MLP_PARAMS 7832

/* y = network(x) for n samples. */
zf_status zf_mlp_forward(const float *d_params, const float *d_x, uint32_t n, float *d_y,
                         zf_stream_t stream);
/* Bytes of device workspace zf_mlp_grad needs for n samples. */
uint64_t zf_mlp_grad_work_bytes(uint32_t n);
/* Loss (1/n) sum_i (y_i[k_i] - t_i)^2 into *d_loss and its gradient with
 * respect to every parameter into d_grad (ZF_MLP_PARAMS floats).  Summation
 * order is fixed, so results are bit-reproducible.  A k_i outside [0, 24)
 * makes the loss NaN and contributes no gradient.  ZF_E_TOO_SMALL when
 * work_bytes < zf_mlp_grad_work_bytes(n). */
zf_status zf_mlp_grad(const float *d_params, const float *d_x, const int32_t *d_k, const float *d_t,
                      uint32_t n, float *d_grad, float *d_loss, void *d_work, uint64_t work_bytes,
                      zf_stream_t stream);
/*
 * zf_mlp_grad without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
 * zf_mlp_grad; the per-workgroup partial gradients go to a static device
 * array of the library (ceil(ZF_MLP_STATIC_MAX_N / 64) x 7833 floats, about
 * 8 MB, held on each device the call runs on until the process ends).  The
 * call allocates nothing; it runs on the current device (the stream must
 * belong to it).  n > ZF_MLP_STATIC_MAX_N: ZF_E_UNSUPPORTED; null pointers
 * or n == 0: ZF_E_INVALID.  Every call on one device shares that array, so
 * calls that overlap on one device (concurrent streams, threads) race; calls
 * ordered on one stream do not.
 */
#define ZF_MLP_STATIC_MAX_N 16384
zf_status zf_mlp_grad_noalloc(const float *d_params, const float *d_x, const int32_t *d_k,
                              const float *d_t, uint32_t n, float *d_grad, float *d_loss,
                              zf_stream_t stream);
/* One Adam step (step counts from 1) on the parameters in place; d_m and
 * d_v are the moment estimates (ZF_MLP_PARAMS floats each, zero at start). */
zf_status zf_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, uint32_t step,
                      float lr, float beta1, float beta2, float eps, zf_stream_t stream);

const char *zf_status_str(zf_status s);
const char *zf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
