// Column container: CRC-32, layout, parsing and host-side validation.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

#include "zf_internal.hpp"

namespace zf {

static thread_local std::string g_last_error;

void set_last_error(const std::string &m) { g_last_error = m; }
const std::string &last_error() { return g_last_error; }

void fail(zf_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{st, buf};
}

uint32_t elem_size(uint32_t dtype) {
    switch (dtype) {
    case D_I32: return 4;
    case D_I64: return 8;
    case D_BYTES: return 1;
    case D_FIXED16: return 16;
    case D_F64: return 8;
    }
    return 0;
}

bool codec_allows(uint32_t codec, uint32_t dtype) {
    if (!elem_size(dtype)) return false;
    switch (codec) {
    case C_PLAIN:
    case C_LZ77: return true;
    case C_FOR_BP:
    case C_DELTA_BP:
    case C_RLE_DELTA_BP:
    case C_DSTRIDE_BP:
    case C_DSTREE: return dtype == D_I32 || dtype == D_I64;
    case C_SDICT_BP:
    case C_SDICT_ANS:
    case C_SDICT_COL:
    case C_SDICT_COL_ANS: return dtype == D_BYTES;
    case C_DICT_BP: return dtype != D_BYTES && dtype != D_F64;
    case C_F2I_BP: return dtype == D_F64;
    case C_ANS: return true;
    }
    return false;
}

Kind kind_of(uint32_t codec, uint32_t dtype) {
    switch (codec) {
    case C_PLAIN: return K_PLAIN;
    case C_FOR_BP: return dtype == D_I32 ? K_FOR32 : K_FOR64;
    case C_DICT_BP: return dtype == D_I32 ? K_DICT32 : dtype == D_I64 ? K_DICT64 : K_DICT128;
    case C_DELTA_BP:
    case C_RLE_DELTA_BP:
    case C_DSTRIDE_BP: return dtype == D_I32 ? K_RLE32 : K_RLE64;
    case C_SDICT_BP:
    case C_SDICT_ANS:
    case C_SDICT_COL:
    case C_SDICT_COL_ANS: return K_SDICT;
    case C_LZ77: return K_LZ;
    case C_F2I_BP: return K_F2I;
    case C_ANS: return K_ANS;
    case C_DSTREE: return K_TREE;
    }
    fail(ZF_E_CORRUPT, "unknown codec %u", codec);
}

// CRC-32 (IEEE, reflected 0xEDB88320), byte-at-a-time with a 256-entry table.
static uint32_t g_crc_table[256];
static bool g_crc_ready = [] {
    for (uint32_t i = 0; i < 256; i++) {
        uint32_t c = i;
        for (int k = 0; k < 8; k++) c = (c >> 1) ^ (0xEDB88320u & (0u - (c & 1u)));
        g_crc_table[i] = c;
    }
    return true;
}();

uint32_t crc32(const uint8_t *p, uint64_t n, uint32_t crc) {
    uint32_t c = ~crc;
    for (uint64_t i = 0; i < n; i++) c = g_crc_table[(c ^ p[i]) & 0xFFu] ^ (c >> 8);
    return ~c;
}

void HostBuf::alloc(uint64_t bytes, bool pin) {
    release();
    uint64_t nb = bytes ? bytes : 16;
    if (pin) {
        void *q = nullptr;
        hipError_t e = hipHostMalloc(&q, nb, hipHostMallocDefault);
        if (e != hipSuccess || !q)
            fail(e == hipErrorOutOfMemory ? ZF_E_NOMEM : ZF_E_HIP,
                 "hipHostMalloc(%llu) failed: %s", (unsigned long long)nb, hipGetErrorString(e));
        p = static_cast<uint8_t *>(q);
    } else {
        p = static_cast<uint8_t *>(std::aligned_alloc(256, align_up(nb, 256)));
        if (!p) fail(ZF_E_NOMEM, "host allocation of %llu bytes failed", (unsigned long long)nb);
    }
    n = bytes;
    pinned = pin;
}

void HostBuf::release() {
    if (p) {
        if (pinned) (void)hipHostFree(p);
        else std::free(p);
    }
    p = nullptr;
    n = 0;
}

// ---------------------------------------------------------------- layout
void assemble_column(HostBuf &out, bool pinned, uint32_t dtype, uint64_t n_elems,
                     const std::vector<EncodedChunk> &chunks, const uint8_t *dict,
                     uint32_t dict_count, uint64_t dict_len) {
    const uint32_t es = elem_size(dtype);
    const uint64_t nc = chunks.size();
    const uint64_t table_end = 64 + 32 * nc;
    const uint64_t dict_off = dict_count ? align_up(table_end, 16) : 0;
    uint64_t pos = align_up(dict_count ? dict_off + dict_len : table_end, 16);
    std::vector<uint64_t> comp_off(nc);
    for (uint64_t i = 0; i < nc; i++) {
        comp_off[i] = pos;
        pos = align_up(pos + chunks[i].bytes.size(), 16);
    }
    out.alloc(pos, pinned);
    uint8_t *b = out.p;
    std::memset(b, 0, table_end);
    if (dict_count) {
        std::memset(b + table_end, 0, dict_off - table_end);
        std::memcpy(b + dict_off, dict, dict_len);
    }
    uint64_t plain_off = 0;
    bool mixed = false;
    for (uint64_t i = 0; i < nc; i++) {
        const EncodedChunk &c = chunks[i];
        uint64_t gap_from = i == 0 ? (dict_count ? dict_off + dict_len : table_end)
                                   : comp_off[i - 1] + chunks[i - 1].bytes.size();
        std::memset(b + gap_from, 0, comp_off[i] - gap_from);
        std::memcpy(b + comp_off[i], c.bytes.data(), c.bytes.size());
        uint8_t *e = b + 64 + 32 * i;
        wr64(e, plain_off);
        wr64(e + 8, comp_off[i]);
        wr32(e + 16, c.n_elems * es);
        wr32(e + 20, uint32_t(c.bytes.size()));
        wr32(e + 24, c.n_elems);
        e[28] = c.codec;
        e[29] = c.sched;
        plain_off += uint64_t(c.n_elems) * es;
        mixed |= c.codec != chunks[0].codec;
    }
    uint64_t tail = nc ? comp_off[nc - 1] + chunks[nc - 1].bytes.size()
                       : (dict_count ? dict_off + dict_len : table_end);
    std::memset(b + tail, 0, pos - tail);

    std::memcpy(b, "ZFC1", 4);
    wr16(b + 4, 1);
    b[6] = uint8_t(dtype);
    b[7] = (nc == 0 || mixed) ? 0 : chunks[0].codec;
    wr64(b + 8, n_elems);
    wr64(b + 16, n_elems * es);
    wr32(b + 24, uint32_t(nc));
    wr32(b + 28, dict_count);
    wr64(b + 32, dict_off);
    wr64(b + 40, pos);
    uint32_t tcrc = crc32(b + 64, 32 * nc);
    if (dict_count) tcrc = crc32(b + dict_off, dict_len, tcrc);
    wr32(b + 48, tcrc);
    wr32(b + 52, 0);
    wr32(b + 56, 0);
    wr32(b + 60, crc32(b, 60));
}

// ------------------------------------------------------------- validation
static uint64_t words_for(uint64_t fields, uint32_t w) { return (fields * w + 31) / 32; }

// An ANS stream of L bytes decoding to n bytes: header sizes and
// frequencies that sum to M (the coders' states and words are checked by
// the decoder as it reads them).
static void check_ans(const uint8_t *s, uint64_t L, uint64_t n, uint32_t i) {
    ZF_REQUIRE(L >= kAnsHdr && rd32(s) == n && kAnsHdr + 2ull * rd32(s + 4) == L, ZF_E_CORRUPT,
               "chunk %u: ANS header does not match its sizes", i);
    uint32_t sum = 0;
    for (uint32_t t = 0; t < 256; t++) sum += rd16(s + 16 + 2 * t);
    ZF_REQUIRE(sum == kAnsM, ZF_E_CORRUPT, "chunk %u: ANS frequencies sum to %u", i, sum);
}

// The packed entry indices of a nested String-dictionary stream: nothing
// when there are none, else the piece table at co and one ANS stream per
// kSdAnsPiece bytes of them, each 4-aligned.
static void check_ans_pieces(const uint8_t *s, uint64_t L, uint64_t co, uint64_t ncb, uint32_t i) {
    if (ncb == 0) {
        ZF_REQUIRE(co == L, ZF_E_CORRUPT, "chunk %u: String-dictionary codes size", i);
        return;
    }
    const uint32_t np = uint32_t((ncb + kSdAnsPiece - 1) / kSdAnsPiece);
    ZF_REQUIRE(co + 4 + 4ull * np <= L && rd32(s + co) == np, ZF_E_CORRUPT,
               "chunk %u: String-dictionary ANS piece table", i);
    const uint64_t base = co + 4 + 4ull * np;
    uint64_t prev = 0;
    for (uint32_t k = 0; k < np; k++) {
        const uint64_t end = rd32(s + co + 4 + 4ull * k);
        const uint64_t len = std::min<uint64_t>(kSdAnsPiece, ncb - uint64_t(k) * kSdAnsPiece);
        ZF_REQUIRE(end >= prev + kAnsHdr && base + end <= L && (k + 1 < np || base + end == L),
                   ZF_E_CORRUPT, "chunk %u: String-dictionary ANS piece %u", i, k);
        const uint64_t alen = kAnsHdr + 2ull * rd32(s + base + prev + 4);  // without padding
        ZF_REQUIRE(align_up(alen, 4) == end - prev, ZF_E_CORRUPT,
                   "chunk %u: String-dictionary ANS piece %u padding", i, k);
        check_ans(s + base + prev, alen, len, i);
        prev = end;
    }
}

void check_stream(const ColumnView &v, const uint8_t *blob, uint32_t i) {
    const ChunkInfo &c = v.chunks[i];
    const uint8_t *s = blob + c.comp_off;
    const uint32_t n = c.n_elems, L = c.comp_len;
    switch (c.codec) {
    case C_PLAIN:
        ZF_REQUIRE(L == c.plain_len, ZF_E_CORRUPT, "chunk %u: plain stream length", i);
        return;
    case C_FOR_BP:
    case C_DICT_BP: {
        const uint32_t bits = (c.codec == C_DICT_BP || v.dtype == D_I32) ? 32 : 64;
        const uint64_t nb = (n + kForBlock - 1) / kForBlock;
        ZF_REQUIRE(16 * nb <= L, ZF_E_CORRUPT, "chunk %u: block directory overruns", i);
        for (uint64_t b = 0; b < nb; b++) {
            uint32_t w = rd32(s + 16 * b + 8), poff = rd32(s + 16 * b + 12);
            uint64_t nv = std::min<uint64_t>(kForBlock, n - b * kForBlock);
            ZF_REQUIRE(w <= bits && poff % 16 == 0 && poff >= 16 * nb &&
                           poff + 4 * words_for(nv, w) <= L,
                       ZF_E_CORRUPT, "chunk %u block %llu: bad directory entry", i,
                       (unsigned long long)b);
        }
        return;
    }
    case C_DELTA_BP:
    case C_RLE_DELTA_BP: {
        const uint32_t bits = v.dtype == D_I32 ? 32 : 64;
        ZF_REQUIRE(L >= 16, ZF_E_CORRUPT, "chunk %u: short RLE header", i);
        uint32_t nr = rd32(s), ng = rd32(s + 4), roff = rd32(s + 8);
        ZF_REQUIRE(ng == (uint64_t(nr) + kRleGroup - 1) / kRleGroup && 16 + 32ull * ng <= L,
                   ZF_E_CORRUPT, "chunk %u: bad group count", i);
        if (c.codec == C_DELTA_BP)
            ZF_REQUIRE(nr == n && roff == 0, ZF_E_CORRUPT, "chunk %u: delta header", i);
        else
            ZF_REQUIRE(nr >= 1 && roff % 4 == 0 && roff >= 16 + 32ull * ng &&
                           roff + 4ull * nr <= L,
                       ZF_E_CORRUPT, "chunk %u: run array out of range", i);
        uint64_t prev = 0;
        for (uint32_t g = 0; g < ng; g++) {
            const uint8_t *r = s + 16 + 32ull * g;
            uint32_t off = rd32(r), w = rd32(r + 4), doff = rd32(r + 8);
            uint32_t cnt = std::min<uint32_t>(kRleGroup, nr - g * kRleGroup);
            ZF_REQUIRE(w <= bits && doff % 4 == 0 && doff + 4 * words_for(cnt - 1, w) <= L,
                       ZF_E_CORRUPT, "chunk %u group %u: bad record", i, g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < n), ZF_E_CORRUPT,
                       "chunk %u group %u: output offset out of order", i, g);
            prev = off;
        }
        return;
    }
    case C_DSTRIDE_BP: {
        const uint32_t bits = v.dtype == D_I32 ? 32 : 64;
        ZF_REQUIRE(L >= 16, ZF_E_CORRUPT, "chunk %u: short DeltaStride header", i);
        uint32_t nr = rd32(s), ng = rd32(s + 4), roff = rd32(s + 8);
        ZF_REQUIRE(ng == (uint64_t(nr) + kRleGroup - 1) / kRleGroup && 16 + 32ull * ng <= L,
                   ZF_E_CORRUPT, "chunk %u: bad group count", i);
        ZF_REQUIRE(nr >= 1 && roff % 4 == 0 && roff >= 16 + 32ull * ng && roff + 4ull * nr <= L,
                   ZF_E_CORRUPT, "chunk %u: run array out of range", i);
        uint64_t prev = 0;
        for (uint32_t g = 0; g < ng; g++) {
            const uint8_t *r = s + 16 + 32ull * g;
            const uint32_t off = rd32(r), poff = rd32(r + 4), widths = rd32(r + 8);
            const uint32_t wg = widths & 0xFFu, wd = (widths >> 8) & 0xFFu;
            const uint32_t cnt = std::min<uint32_t>(kRleGroup, nr - g * kRleGroup);
            ZF_REQUIRE(wg <= bits && wd <= bits && (widths >> 16) == 0 && poff % 8 == 0 &&
                           poff + 8 + 4 * (words_for(cnt - 1, wg) + words_for(cnt, wd)) <= L,
                       ZF_E_CORRUPT, "chunk %u group %u: bad record", i, g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < n), ZF_E_CORRUPT,
                       "chunk %u group %u: output offset out of order", i, g);
            prev = off;
        }
        return;
    }
    case C_DSTREE: {
        // header, both levels' group records (widths, payloads in range,
        // output offsets from 0 and increasing); the run lengths and counts
        // are checked by the kernels as they expand them
        const uint32_t bits = v.dtype == D_I32 ? 32 : 64;
        ZF_REQUIRE(L >= 32, ZF_E_CORRUPT, "chunk %u: short DeltaStride tree header", i);
        const uint32_t R = rd32(s), ngB = rd32(s + 4), Q = rd32(s + 8), ngA = rd32(s + 12), b_off = rd32(s + 24);
        ZF_REQUIRE(R >= 1 && R <= n && Q >= 1 && Q <= R && ngB == (uint64_t(R) + 63) / 64 &&
                       ngA == (uint64_t(Q) + 63) / 64 && b_off == 32 + 32ull * ngA && rd32(s + 28) == 0 &&
                       b_off + 16ull * ngB <= L,
                   ZF_E_CORRUPT, "chunk %u: DeltaStride tree header does not match its sizes", i);
        uint64_t prev = 0;
        for (uint32_t g = 0; g < ngA; g++) {
            const uint8_t *r = s + 32 + 32ull * g;
            const uint32_t off = rd32(r), poff = rd32(r + 4), widths = rd32(r + 8);
            const uint32_t wv = widths & 0xFFu, wl = (widths >> 8) & 0xFFu, cnt = std::min(64u, Q - 64 * g);
            ZF_REQUIRE(wv <= bits && wl <= 32 && (widths >> 16) == 0 && poff % 4 == 0 &&
                           poff + 4 * (words_for(cnt, wv) + words_for(cnt, wl)) <= L,
                       ZF_E_CORRUPT, "chunk %u start group %u: bad record", i, g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < R), ZF_E_CORRUPT,
                       "chunk %u start group %u: output offset out of order", i, g);
            prev = off;
        }
        prev = 0;
        for (uint32_t g = 0; g < ngB; g++) {
            const uint8_t *r = s + b_off + 16ull * g;
            const uint32_t off = rd32(r), poff = rd32(r + 4), wc = rd32(r + 8), cnt = std::min(64u, R - 64 * g);
            ZF_REQUIRE(wc <= 32 && poff % 4 == 0 && poff + 4 * words_for(cnt, wc) <= L, ZF_E_CORRUPT,
                       "chunk %u run group %u: bad record", i, g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < n), ZF_E_CORRUPT,
                       "chunk %u run group %u: output offset out of order", i, g);
            prev = off;
        }
        return;
    }
    case C_SDICT_BP:
    case C_SDICT_ANS: {
        ZF_REQUIRE(L >= 32, ZF_E_CORRUPT, "chunk %u: short String-dictionary header", i);
        const uint32_t nt = rd32(s), ne = rd32(s + 4), w = rd32(s + 8), ng = rd32(s + 12);
        const uint32_t eo = rd32(s + 16), bo = rd32(s + 20), co = rd32(s + 24), nb = rd32(s + 28);
        const uint32_t wneed = ne > 1 ? 32 - uint32_t(__builtin_clz(ne - 1)) : 0;
        ZF_REQUIRE(ne >= 1 && nt >= 1 && w == wneed && ng == (uint64_t(nt) + 63) / 64 &&
                       eo == align_up(32 + 4ull * ng, 16) && bo == eo + 4ull * ne &&
                       co == align_up(uint64_t(bo) + nb + 4, 16) && co <= L && nb <= 0xFFFFFFu,
                   ZF_E_CORRUPT, "chunk %u: String-dictionary header does not match its sizes", i);
        const uint64_t ncb = 4 * words_for(nt, w);  // packed entry-index bytes
        if (c.codec == C_SDICT_BP)
            ZF_REQUIRE(co + ncb == L, ZF_E_CORRUPT, "chunk %u: String-dictionary codes size", i);
        else
            check_ans_pieces(s, L, co, ncb, i);
        for (uint32_t k = 0; k < ne; k++) {
            const uint32_t e = rd32(s + eo + 4ull * k), len = e >> 24;
            ZF_REQUIRE(len >= 1 && len <= kSdMaxToken && (e & 0xFFFFFFu) + uint64_t(len) <= nb,
                       ZF_E_CORRUPT, "chunk %u: String-dictionary entry %u", i, k);
        }
        uint64_t prev = 0;
        for (uint32_t g = 0; g < ng; g++) {
            const uint32_t off = rd32(s + 32 + 4ull * g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < c.plain_len), ZF_E_CORRUPT,
                       "chunk %u group %u: output offset out of order", i, g);
            prev = off;
        }
        return;
    }
    case C_SDICT_COL:
    case C_SDICT_COL_ANS: {
        ZF_REQUIRE(L >= 16, ZF_E_CORRUPT, "chunk %u: short String-dictionary header", i);
        const uint32_t nt = rd32(s), w = rd32(s + 4), ng = rd32(s + 8), co = rd32(s + 12);
        const uint32_t ne = v.dict_count;
        const uint32_t wneed = ne > 1 ? 32 - uint32_t(__builtin_clz(ne - 1)) : 0;
        ZF_REQUIRE(ne >= 1 && nt >= 1 && w == wneed && ng == (uint64_t(nt) + 63) / 64 &&
                       co == align_up(16 + 4ull * ng, 16) && co <= L,
                   ZF_E_CORRUPT, "chunk %u: String-dictionary header does not match its sizes", i);
        const uint64_t ncb = 4 * words_for(nt, w);
        if (c.codec == C_SDICT_COL)
            ZF_REQUIRE(co + ncb == L, ZF_E_CORRUPT, "chunk %u: String-dictionary codes size", i);
        else
            check_ans_pieces(s, L, co, ncb, i);
        uint64_t prev = 0;
        for (uint32_t g = 0; g < ng; g++) {
            const uint32_t off = rd32(s + 16 + 4ull * g);
            ZF_REQUIRE(g == 0 ? off == 0 : (off > prev && off < c.plain_len), ZF_E_CORRUPT,
                       "chunk %u group %u: output offset out of order", i, g);
            prev = off;
        }
        return;
    }
    case C_F2I_BP: {
        const uint64_t nb = (n + kForBlock - 1) / kForBlock;
        ZF_REQUIRE(32 * nb <= L, ZF_E_CORRUPT, "chunk %u: block directory overruns", i);
        for (uint64_t b = 0; b < nb; b++) {
            const uint8_t *d = s + 32 * b;
            const uint32_t w = rd32(d + 8), poff = rd32(d + 12), xoff = rd32(d + 16);
            const uint32_t nx = rd16(d + 20), e = d[22];
            const uint64_t nv = std::min<uint64_t>(kForBlock, n - b * kForBlock);
            ZF_REQUIRE(w <= 64 && e <= 18 && nx <= nv && poff % 16 == 0 && poff >= 32 * nb &&
                           poff + 4 * words_for(nv, w) <= L && xoff % 16 == 0 && xoff >= 32 * nb &&
                           xoff + 16ull * nx <= L,
                       ZF_E_CORRUPT, "chunk %u block %llu: bad directory entry", i,
                       (unsigned long long)b);
        }
        return;
    }
    case C_ANS: check_ans(s, L, c.plain_len, i); return;
    case C_LZ77: {
        ZF_REQUIRE(L >= 16 && c.plain_len <= kLzMaxChunk, ZF_E_CORRUPT, "chunk %u: LZ77 sizes", i);
        uint64_t ns = rd32(s), nl = rd32(s + 4), ne = rd32(s + 8), pl = rd32(s + 12);
        ZF_REQUIRE(pl == c.plain_len && 16 + 3 * ns + 2 * ne + nl == L, ZF_E_CORRUPT,
                   "chunk %u: LZ77 header does not match its sizes", i);
        return;
    }
    }
    fail(ZF_E_CORRUPT, "chunk %u: unknown codec %u", i, c.codec);
}

ColumnView parse_column(const uint8_t *p, uint64_t len) {
    ZF_REQUIRE(p && len >= 64, ZF_E_CORRUPT, "column shorter than its header");
    ZF_REQUIRE(std::memcmp(p, "ZFC1", 4) == 0 && rd16(p + 4) == 1, ZF_E_CORRUPT,
               "bad magic or version");
    ZF_REQUIRE(rd32(p + 60) == crc32(p, 60), ZF_E_CORRUPT, "header CRC mismatch");
    ColumnView v;
    v.dtype = p[6];
    v.codec = p[7];
    v.n_elems = rd64(p + 8);
    v.plain_bytes = rd64(p + 16);
    v.n_chunks = rd32(p + 24);
    v.dict_count = rd32(p + 28);
    v.dict_off = rd64(p + 32);
    v.total_bytes = rd64(p + 40);
    const uint32_t es = elem_size(v.dtype);
    ZF_REQUIRE(es && v.plain_bytes == v.n_elems * es && v.total_bytes == len, ZF_E_CORRUPT,
               "header sizes inconsistent");
    const uint64_t tl = 32ull * v.n_chunks;
    uint64_t dl = uint64_t(v.dict_count) * es;
    ZF_REQUIRE(64 + tl <= len, ZF_E_CORRUPT, "chunk table overruns the column");
    if (v.dict_count && v.dtype == D_BYTES) {
        // a token dictionary: its size follows from its entry-byte count
        ZF_REQUIRE(v.dict_off % 16 == 0 && v.dict_off >= 64 + tl && v.dict_off + 16 <= len, ZF_E_CORRUPT,
                   "dictionary out of range");
        const uint32_t nb = rd32(p + v.dict_off);
        ZF_REQUIRE(nb < (1u << 24) && v.dict_count <= (1u << 24), ZF_E_CORRUPT, "token dictionary too large");
        dl = 16 + 4ull * v.dict_count + align_up(nb, 16);
    }
    v.dict_bytes = dl;
    if (v.dict_count)
        ZF_REQUIRE(v.dict_off % 16 == 0 && v.dict_off >= 64 + tl && v.dict_off + dl <= len,
                   ZF_E_CORRUPT, "dictionary out of range");
    else
        ZF_REQUIRE(v.dict_off == 0, ZF_E_CORRUPT, "dictionary offset without dictionary");
    uint32_t tcrc = crc32(p + 64, tl);
    if (v.dict_count) tcrc = crc32(p + v.dict_off, dl, tcrc);
    ZF_REQUIRE(tcrc == rd32(p + 48), ZF_E_CORRUPT, "chunk table CRC mismatch");
    if (v.dict_count && v.dtype == D_BYTES) {
        const uint8_t *d = p + v.dict_off;
        const uint32_t nb = rd32(d);
        ZF_REQUIRE(rd32(d + 4) == 0 && rd32(d + 8) == 0 && rd32(d + 12) == 0, ZF_E_CORRUPT,
                   "token dictionary header");
        // every entry inside the bytes with three zero bytes on each side
        const uint8_t *bytes = d + 16 + 4ull * v.dict_count;
        for (uint32_t k = 0; k < v.dict_count; k++) {
            const uint32_t e = rd32(d + 16 + 4ull * k), elen = e >> 24, off = e & 0xFFFFFFu;
            ZF_REQUIRE(elen >= 1 && elen <= kSdMaxToken && off >= 3 && off + uint64_t(elen) + 3 <= nb &&
                           off + 16ull <= nb,
                       ZF_E_CORRUPT, "token dictionary entry %u", k);
            for (uint32_t q = 1; q <= 3; q++)
                ZF_REQUIRE(bytes[off - q] == 0 && bytes[off + elen + q - 1] == 0, ZF_E_CORRUPT,
                           "token dictionary entry %u: no zero bytes around it", k);
        }
    }
    v.chunks.resize(v.n_chunks);
    uint64_t plain = 0, elems = 0;
    for (uint32_t i = 0; i < v.n_chunks; i++) {
        const uint8_t *e = p + 64 + 32ull * i;
        ChunkInfo &c = v.chunks[i];
        c.plain_off = rd64(e);
        c.comp_off = rd64(e + 8);
        c.plain_len = rd32(e + 16);
        c.comp_len = rd32(e + 20);
        c.n_elems = rd32(e + 24);
        c.codec = e[28];
        c.sched = e[29];
        ZF_REQUIRE(c.sched <= 4, ZF_E_CORRUPT, "chunk %u: schedule hint %u", i, c.sched);
        ZF_REQUIRE(c.plain_off == plain && c.n_elems > 0 && uint64_t(c.n_elems) * es == c.plain_len,
                   ZF_E_CORRUPT, "chunk %u: plain range", i);
        ZF_REQUIRE(c.comp_off % 16 == 0 && c.comp_off >= 64 + tl && c.comp_off + c.comp_len <= len,
                   ZF_E_CORRUPT, "chunk %u: stream out of range", i);
        ZF_REQUIRE(codec_allows(c.codec, v.dtype), ZF_E_CORRUPT, "chunk %u: codec %u for dtype %u",
                   i, c.codec, v.dtype);
        ZF_REQUIRE((c.codec != C_DICT_BP && c.codec != C_SDICT_COL && c.codec != C_SDICT_COL_ANS) ||
                       v.dict_count > 0,
                   ZF_E_CORRUPT, "chunk %u: dictionary chunk without dictionary", i);
        plain += c.plain_len;
        elems += c.n_elems;
        check_stream(v, p, i);
    }
    ZF_REQUIRE(plain == v.plain_bytes && elems == v.n_elems, ZF_E_CORRUPT,
               "chunks do not cover the column");
    return v;
}

}  // namespace zf
