// Host-side internals of libzf: errors, the column container, helpers.
#pragma once
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "zf.h"
#include "zf_device.hpp"

namespace zf {

struct Error {
    zf_status st;
    std::string msg;
};
[[noreturn]] void fail(zf_status st, const char *fmt, ...);
void set_last_error(const std::string &m);

#define ZF_HIP(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) ::zf::fail(ZF_E_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define ZF_REQUIRE(cond, st, ...)                \
    do {                                         \
        if (!(cond)) ::zf::fail(st, __VA_ARGS__); \
    } while (0)

// Run `body` and turn exceptions into a status + thread-local message.
template <class F>
zf_status guard(F &&body) {
    try {
        body();
        return ZF_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.st;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return ZF_E_NOMEM;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return ZF_E_INVALID;
    } catch (...) {
        set_last_error("unknown error");
        return ZF_E_INVALID;
    }
}

// ------------------------------------------------------------ little endian
inline uint32_t rd32(const uint8_t *p) { uint32_t v; std::memcpy(&v, p, 4); return v; }
inline uint64_t rd64(const uint8_t *p) { uint64_t v; std::memcpy(&v, p, 8); return v; }
inline uint16_t rd16(const uint8_t *p) { uint16_t v; std::memcpy(&v, p, 2); return v; }
inline void wr32(uint8_t *p, uint32_t v) { std::memcpy(p, &v, 4); }
inline void wr64(uint8_t *p, uint64_t v) { std::memcpy(p, &v, 8); }
inline void wr16(uint8_t *p, uint16_t v) { std::memcpy(p, &v, 2); }
inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Bytes of packed entry indices per ANS piece of the nested
// String-dictionary | BP | ANS scheme (each piece decodes on its own).
constexpr uint32_t kSdAnsPiece = 65536;

uint32_t elem_size(uint32_t dtype);
bool codec_allows(uint32_t codec, uint32_t dtype);
uint32_t crc32(const uint8_t *p, uint64_t n, uint32_t crc = 0);
Kind kind_of(uint32_t codec, uint32_t dtype);

// ------------------------------------------------------------------ memory
struct HostBuf {
    uint8_t *p = nullptr;
    uint64_t n = 0;
    bool pinned = false;
    HostBuf() = default;
    HostBuf(const HostBuf &) = delete;
    HostBuf &operator=(const HostBuf &) = delete;
    ~HostBuf() { release(); }
    void alloc(uint64_t bytes, bool pin);
    void release();
};

// ------------------------------------------------------------------ column
struct ChunkInfo {
    uint64_t plain_off, comp_off;
    uint32_t plain_len, comp_len, n_elems;
    uint8_t codec;
    uint8_t sched;  // schedule hint: 0 = tuned default, 1..4 = chosen granularity
};

struct ColumnView {
    uint32_t dtype = 0, codec = 0, n_chunks = 0, dict_count = 0;
    uint64_t n_elems = 0, plain_bytes = 0, dict_off = 0, total_bytes = 0;
    uint64_t dict_bytes = 0;  // size of the dictionary area
    std::vector<ChunkInfo> chunks;
};

// Parse and validate header, CRCs, chunk table and every stream's directory.
ColumnView parse_column(const uint8_t *p, uint64_t len);
// Validate the directory of chunk i's stream (host side; throws ZF_E_CORRUPT).
void check_stream(const ColumnView &v, const uint8_t *blob, uint32_t i);

// Lay out a column: header, table, dictionary (dict_len bytes), streams
// (16-aligned).
struct EncodedChunk {
    std::vector<uint8_t> bytes;
    uint32_t n_elems;
    uint8_t codec;
    uint8_t sched = 0;
};
void assemble_column(HostBuf &out, bool pinned, uint32_t dtype, uint64_t n_elems,
                     const std::vector<EncodedChunk> &chunks, const uint8_t *dict,
                     uint32_t dict_count, uint64_t dict_len);

}  // namespace zf

struct zf_column {
    zf::HostBuf buf;
    zf::ColumnView view;
};
