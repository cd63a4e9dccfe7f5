// Device-side work tables: written by the host planner, read by the kernels.
// Plain structs only; the same definitions compile on both sides.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace zf {

constexpr uint32_t kForBlock = 2048;   // values per FOR / bit-packing block
constexpr uint32_t kRleGroup = 64;     // runs per RLE group record (one wave)
constexpr uint32_t kLzMaxChunk = 65536;
constexpr uint32_t kMaxCols = 256;     // output table size: columns per plan + 1
// Output-table slot of the plan's scratch area (the decoded entry indices of
// String-dictionary | BP | ANS chunks, the first of their two decode stages)
constexpr uint32_t kScratchCol = kMaxCols - 1;
// ANS: M = 2^12 model, state in [2^16, 2^32), 64 interleaved coders, stream
// header of 16 + 512 (frequencies) + 256 (states) + 256 (word offsets) bytes.
constexpr uint32_t kAnsM = 4096, kAnsL = 65536, kAnsLanes = 64, kAnsHdr = 784;
// ANS: LDS per wave, the model (1280 dwords) and 1 KiB of output staging
constexpr uint32_t kAnsLdsWords = 1536;
// String-dictionary: longest token
constexpr uint32_t kSdMaxToken = 64;

// Codec / dtype codes, as in zf.h.
enum : uint8_t { C_PLAIN = 1, C_FOR_BP = 2, C_DICT_BP = 3, C_DELTA_BP = 4, C_RLE_DELTA_BP = 5, C_LZ77 = 6,
                 C_F2I_BP = 7, C_ANS = 8, C_DSTRIDE_BP = 9, C_SDICT_BP = 10, C_SDICT_ANS = 11,
                 C_SDICT_COL = 12, C_SDICT_COL_ANS = 13, C_DSTREE = 14,
                 // internal: the first decode stage of a C_DSTREE chunk (its run starts)
                 C_DSTREE_STARTS = 200 };
enum : uint8_t { D_I32 = 1, D_I64 = 2, D_BYTES = 3, D_FIXED16 = 4, D_F64 = 5 };

// Kernel kinds: one device routine per (codec class, value width).  The
// order is the order of the persistent queue: slow units first, so that the
// long serial LZ77 chunks start early and the short streaming units fill in.
enum Kind : uint32_t {
    K_LZ = 0,
    K_ANS,     // range ANS, 64 interleaved coders per chunk
    K_RLE64,   // RLE_DELTA_BP, DELTA_BP, DSTRIDE_BP and the DSTREE starts, int64
    K_RLE32,   // RLE_DELTA_BP, DELTA_BP, DSTRIDE_BP and the DSTREE starts, int32
    K_SDICT,   // String-dictionary, bytes
    K_DICT128,
    K_DICT64,
    K_DICT32,
    K_FOR64,
    K_FOR32,
    K_F2I,     // Float2Int + bit-packing, float64
    K_PLAIN,
    K_TREE,    // DSTREE second stage (after the RLE kinds wrote its run starts)
    K_COUNT
};

// One chunk of one column, as seen from the device.
struct ChunkDesc {
    uint64_t comp_off;    // stream offset from the launch's comp base
    uint64_t out_off;     // byte offset of the chunk in its column's output
    uint64_t dict_off;    // dictionary offset from the launch's dict base
    uint32_t comp_len;    // stream bytes
    uint32_t n_elems;     // values in the chunk
    uint32_t dict_count;  // dictionary entries (DICT_BP)
    uint16_t col;         // column index (output table slot)
    uint8_t codec;
    uint8_t dtype;
    uint64_t aux_off;     // SDICT_ANS, SDICT_COL_ANS: offset of the decoded entry indices in the scratch area
    uint64_t dict_bytes;  // size of the column's dictionary area
    uint64_t fat_off;     // SDICT_COL, SDICT_COL_ANS: offset of the column's entry table in LaunchArgs::fat
};
static_assert(sizeof(ChunkDesc) == 64, "ChunkDesc layout");

// The plan's copy of a column token dictionary, one 16-byte record per
// entry: the entry's first 15 bytes (zero past its length), then its length.
constexpr uint32_t kFatBytes = 16;
constexpr uint32_t kFatInline = 15;

// One unit of work for one wavefront.
//   FOR / DICT / F2I: a = first block, b = number of blocks
//   RLE / DELTA: a = first group, b = first element, c = end element
//   LZ77, ANS: the whole chunk
//   PLAIN: a = first byte, b = end byte
struct Tile {
    uint32_t chunk;
    uint32_t a, b, c;
};
static_assert(sizeof(Tile) == 16, "Tile layout");

// Device error word bits.
enum : uint32_t { ERR_CORRUPT = 1u, ERR_BOUNDS = 2u };

// Arguments of one decode launch (a batch or the whole image).
struct LaunchArgs {
    const uint8_t *comp;          // base of the compressed streams
    const uint8_t *dict;          // base of the dictionaries
    uint8_t *const *out_tab;      // device table: column -> output pointer
    const ChunkDesc *chunks;
    const Tile *tiles;            // tiles grouped by kind
    uint32_t *err;                // device error word
    uint32_t *counter;            // persistent-kernel queue heads: 2 launches x 8 XCDs, 32 dwords apart
    const uint8_t *fat;           // the plan's 16-byte entry records of the column token dictionaries
    uint32_t kind_begin[K_COUNT + 1];
    uint32_t two_stage;           // some units read the scratch area that earlier kinds write
    uint32_t sdict_codecs;        // String-dictionary tiles: bit 0 some over a column dictionary, bit 1 some not
};

// Host side: events recorded around each kind's launch of a profiled decode
// (index K_COUNT: the persistent kernel).
struct KindEvents {
    hipEvent_t e0[K_COUNT + 1] = {}, e1[K_COUNT + 1] = {};
    bool used[K_COUNT + 1] = {};
};

}  // namespace zf
