// Tile shapes per kernel kind: defaults, the autotuner's cache, overrides.
#pragma once
#include <string>

#include "zf_internal.hpp"

namespace zf {

struct TileShape {
    uint32_t unit[K_COUNT];  // FP: blocks; GP: elements; PLAIN: bytes; LZ77: bytes per block
    uint32_t wpb[K_COUNT];   // waves per workgroup
    uint32_t wpcu;           // persistent kernel: waves per CU
    double rate_gbps[K_COUNT];  // measured decode rate (GB/s of plain output) of the tuned tile
};

TileShape default_tiles();
bool read_tune_cache(const std::string &path, TileShape &t);
TileShape resolve_tiles(const zf_plan_opts &o);
const char *kind_name(uint32_t k);
// Unit size of a chunk whose encoder chose schedule `sched` (1..4).
uint32_t scheduled_unit(uint32_t kind, uint32_t sched, uint32_t tuned);

}  // namespace zf
