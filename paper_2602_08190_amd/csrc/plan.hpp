// The plan: work tables, batches, order, device workspace, graphs.
#pragma once
#include <vector>

#include "zf_internal.hpp"

struct zf_plan;
namespace zf {

// lz_blk: output bytes per block of the per-kind LZ77 kernel (4, 8 or 16).
hipError_t launch_decode(const LaunchArgs &A, uint32_t persistent_waves, const uint32_t *waves_per_block,
                         uint32_t lz_blk, hipStream_t st, KindEvents *ev = nullptr);
hipError_t launch_set_out_tab(uint8_t **d_tab, uint8_t *const *ptrs, uint32_t n, uint8_t *scratch, hipStream_t st);

struct CopyOp {
    const uint8_t *src;  // pinned host bytes of a column
    uint64_t dst_off;    // offset in the staging slot (or dictionary area)
    uint64_t len;
};

// Host-side work tables of one launch (a batch, or the whole image).
struct WorkTables {
    std::vector<ChunkDesc> chunks;
    std::vector<Tile> tiles[K_COUNT];
    uint64_t plain_bytes = 0, comp_bytes = 0;
    uint64_t scratch_bytes = 0;  // scratch area the launch's two-stage chunks use
    double t_dec = 0;  // decode-time estimate, seconds
};

void release_plan(zf_plan_t *P);
// Johnson's two-machine order of jobs with first-stage times a, second b.
std::vector<uint32_t> johnson(const std::vector<double> &a, const std::vector<double> &b);
// The units add_chunk cuts chunk ci of col into, in kind order (host only).
std::vector<zf_unit> chunk_units(const zf_column &col, uint32_t ci, const zf_plan_opts &o);

struct Batch {
    WorkTables w;
    std::vector<CopyOp> copies;
    uint64_t slot_used = 0;
    double t_h2d = 0;
    uint32_t index = 0;     // position in column order, before ordering
    LaunchArgs args{};      // comp base = its slot
    int slot = 0;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

}  // namespace zf

struct zf_plan {
    int device = 0;
    zf_plan_opts opts{};
    std::vector<const zf_column *> cols;
    std::vector<uint64_t> image_off;
    uint64_t image_bytes = 0;

    // launch configuration
    uint32_t persistent_waves = 0;  // 0: per-kind launches
    uint32_t lz_blk = 16;         // LZ77 bytes per block
    uint32_t waves_per_block[zf::K_COUNT] = {4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4, 4};
    uint32_t cu_count = 0;

    // device memory
    uint8_t *d_tables = nullptr;
    uint8_t **d_out_tab = nullptr;
    uint32_t *d_err = nullptr;      // error word, then the queue counter
    std::vector<uint8_t *> d_slots;
    uint64_t slot_bytes = 0;
    uint8_t *d_dict = nullptr;
    uint8_t *d_scratch = nullptr;  // shared by every launch (they run in stream order)
    uint8_t *d_fat = nullptr;      // 16-byte entry records of the column token dictionaries
    uint64_t scratch_bytes = 0;
    uint64_t dict_bytes = 0;
    std::vector<zf::CopyOp> dict_copies;

    zf::LaunchArgs image_args{};    // comp/dict bases filled per call
    std::vector<zf::Batch> batches; // in execution order

    hipStream_t copy_stream = nullptr;
    std::vector<hipEvent_t> slot_full, slot_free;
    std::vector<hipEvent_t> ev_h2d0, ev_h2d1, ev_dec0, ev_dec1;
    hipEvent_t ev_start = nullptr, ev_end = nullptr, ev_dict = nullptr;
    zf_timing *pending_timing = nullptr;
    bool timing_valid = false;
    // per-kind events of profiled image decodes (zf_plan_profile)
    bool profile = false, kinds_recorded = false;
    zf::KindEvents kind_ev;

    ~zf_plan() { zf::release_plan(this); }
};
