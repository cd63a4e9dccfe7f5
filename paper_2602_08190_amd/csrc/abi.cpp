// extern "C" entry points declared in zf.h.  Each one validates its
// arguments, runs inside zf::guard (no exception crosses the boundary) and
// leaves its out-parameters untouched on failure.
#include <memory>

#include "features.hpp"
#include "plan.hpp"

namespace zf {
const std::string &last_error();
void compress_host(const void *src, uint64_t n_elems, uint32_t dtype, uint32_t codec,
                   const zf_encode_opts &o, zf_column_t *col, const uint8_t *forced_sched);
void build_plan(zf_plan_t *P, const zf_column *const *cols, uint32_t n_cols, int device,
                const zf_plan_opts &o);
void decompress_async(zf_plan_t *P, const void *d_comp, uint64_t comp_bytes, void *const *d_out,
                      hipStream_t st);
void transfer_and_decompress(zf_plan_t *P, void *const *d_out, hipStream_t st, zf_timing *timing);
void sync_plan(zf_plan_t *P, hipStream_t st);
void clear_error(zf_plan_t *P);
void set_profile(zf_plan_t *P, bool on);
void kind_ms(zf_plan_t *P, double *ms);
}  // namespace zf

using namespace zf;

extern "C" {

void zf_encode_opts_default(zf_encode_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->pinned = 1;
    o->fallback_device = -1;
    o->fallback_margin = 0.05f;
}

void zf_plan_opts_default(zf_plan_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->slot_bytes = 256ull << 20;
    o->n_slots = 2;
    o->use_graphs = 1;
    o->persistent = 0;
    o->order = 0;
    o->pcie_gbps = 0;
}

zf_status zf_compress_host(const void *src, uint64_t n_elems, zf_dtype dtype, zf_codec codec,
                           const zf_encode_opts *opts, zf_column_t **out) {
    return guard([&] {
        ZF_REQUIRE(out, ZF_E_INVALID, "null output pointer");
        zf_encode_opts o;
        zf_encode_opts_default(&o);
        if (opts) o = *opts;
        auto col = std::make_unique<zf_column>();
        compress_host(src, n_elems, uint32_t(dtype), uint32_t(codec), o, col.get(), nullptr);
        *out = col.release();
    });
}

zf_status zf_chunk_features(const void *src, uint64_t n_elems, zf_dtype dtype, float *out) {
    return guard([&] {
        ZF_REQUIRE(out && (src || n_elems == 0), ZF_E_INVALID, "null pointer");
        ZF_REQUIRE(elem_size(uint32_t(dtype)) != 0, ZF_E_INVALID, "unknown dtype %d", int(dtype));
        chunk_features(src, n_elems, uint32_t(dtype), out);
    });
}

zf_status zf_column_from_bytes(const void *buf, uint64_t len, int32_t pinned, zf_column_t **out) {
    return guard([&] {
        ZF_REQUIRE(buf && out, ZF_E_INVALID, "null pointer");
        ColumnView v = parse_column(static_cast<const uint8_t *>(buf), len);
        auto col = std::make_unique<zf_column>();
        col->buf.alloc(len, pinned != 0);
        std::memcpy(col->buf.p, buf, len);
        col->view = std::move(v);
        *out = col.release();
    });
}

const void *zf_column_bytes(const zf_column_t *col, uint64_t *len) {
    if (!col) return nullptr;
    if (len) *len = col->buf.n;
    return col->buf.p;
}
uint64_t zf_column_plain_bytes(const zf_column_t *col) { return col ? col->view.plain_bytes : 0; }
uint64_t zf_column_n_elems(const zf_column_t *col) { return col ? col->view.n_elems : 0; }
uint32_t zf_column_n_chunks(const zf_column_t *col) { return col ? col->view.n_chunks : 0; }
int32_t zf_column_dtype(const zf_column_t *col) { return col ? int32_t(col->view.dtype) : 0; }
void zf_column_free(zf_column_t *col) { delete col; }

zf_status zf_plan(const zf_column_t *const *cols, uint32_t n_cols, int32_t device,
                  const zf_plan_opts *opts, zf_plan_t **out) {
    return guard([&] {
        ZF_REQUIRE(out, ZF_E_INVALID, "null output pointer");
        zf_plan_opts o;
        zf_plan_opts_default(&o);
        if (opts) o = *opts;
        auto P = std::make_unique<zf_plan_t>();
        build_plan(P.get(), cols, n_cols, device, o);
        *out = P.release();
    });
}

void zf_plan_free(zf_plan_t *plan) { delete plan; }

uint64_t zf_plan_image_bytes(const zf_plan_t *plan) { return plan ? plan->image_bytes : 0; }
uint64_t zf_plan_image_offset(const zf_plan_t *plan, uint32_t col) {
    return (plan && col < plan->image_off.size()) ? plan->image_off[col] : 0;
}

uint32_t zf_plan_n_batches(const zf_plan_t *plan) { return plan ? uint32_t(plan->batches.size()) : 0; }

zf_status zf_plan_batch_info(const zf_plan_t *plan, uint32_t k, zf_batch_info *info) {
    return guard([&] {
        ZF_REQUIRE(plan && info, ZF_E_INVALID, "null pointer");
        ZF_REQUIRE(k < plan->batches.size(), ZF_E_INVALID, "batch %u of %zu", k, plan->batches.size());
        const Batch &b = plan->batches[k];
        zf_batch_info r{};
        r.t_h2d_ms = b.t_h2d * 1e3;
        r.t_dec_ms = b.w.t_dec * 1e3;
        r.comp_bytes = b.w.comp_bytes;
        r.plain_bytes = b.w.plain_bytes;
        r.n_chunks = 0;
        for (const ChunkDesc &c : b.w.chunks) r.n_chunks += c.col != kScratchCol;
        r.index = b.index;
        *info = r;
    });
}

zf_status zf_johnson_order(const double *a, const double *b, uint32_t n, uint32_t *order) {
    return guard([&] {
        ZF_REQUIRE((a && b && order) || n == 0, ZF_E_INVALID, "null pointer");
        for (uint32_t i = 0; i < n; i++)
            ZF_REQUIRE(a[i] == a[i] && b[i] == b[i], ZF_E_INVALID, "job %u has a NaN time", i);
        const std::vector<uint32_t> o = johnson(std::vector<double>(a, a + n), std::vector<double>(b, b + n));
        std::copy(o.begin(), o.end(), order);
    });
}

zf_status zf_chunk_units(const zf_column_t *col, uint32_t chunk, const zf_plan_opts *opts, zf_unit *units,
                         uint32_t cap, uint32_t *n_units) {
    return guard([&] {
        ZF_REQUIRE(col && n_units, ZF_E_INVALID, "null pointer");
        zf_plan_opts o;
        if (opts)
            o = *opts;
        else
            zf_plan_opts_default(&o);
        const std::vector<zf_unit> u = chunk_units(*col, chunk, o);
        if (units || cap) {
            ZF_REQUIRE(units, ZF_E_INVALID, "null units with cap %u", cap);
            ZF_REQUIRE(cap >= u.size(), ZF_E_TOO_SMALL, "%zu units, room for %u", u.size(), cap);
            std::copy(u.begin(), u.end(), units);
        }
        *n_units = uint32_t(u.size());
    });
}

zf_status zf_decompress_async(zf_plan_t *plan, const void *d_comp, uint64_t comp_bytes,
                              void *const *d_out, zf_stream_t stream) {
    return guard([&] {
        ZF_REQUIRE(plan, ZF_E_INVALID, "null plan");
        decompress_async(plan, d_comp, comp_bytes, d_out, static_cast<hipStream_t>(stream));
    });
}

zf_status zf_transfer_and_decompress(zf_plan_t *plan, void *const *d_out, zf_stream_t stream,
                                     zf_timing *timing) {
    return guard([&] {
        ZF_REQUIRE(plan, ZF_E_INVALID, "null plan");
        transfer_and_decompress(plan, d_out, static_cast<hipStream_t>(stream), timing);
    });
}

zf_status zf_sync(zf_plan_t *plan, zf_stream_t stream) {
    return guard([&] {
        ZF_REQUIRE(plan, ZF_E_INVALID, "null plan");
        sync_plan(plan, static_cast<hipStream_t>(stream));
    });
}

zf_status zf_plan_profile(zf_plan_t *plan, int32_t on) {
    return guard([&] {
        ZF_REQUIRE(plan, ZF_E_INVALID, "null plan");
        set_profile(plan, on != 0);
    });
}

zf_status zf_plan_kind_ms(zf_plan_t *plan, double *ms) {
    return guard([&] {
        ZF_REQUIRE(plan && ms, ZF_E_INVALID, "null pointer");
        double t[ZF_KIND_COUNT + 1];
        kind_ms(plan, t);
        std::copy(t, t + ZF_KIND_COUNT + 1, ms);
    });
}

void zf_plan_clear_error(zf_plan_t *plan) {
    if (plan) clear_error(plan);
}

const char *zf_status_str(zf_status s) {
    switch (s) {
    case ZF_OK: return "ok";
    case ZF_E_INVALID: return "invalid argument";
    case ZF_E_UNSUPPORTED: return "unsupported";
    case ZF_E_CORRUPT: return "corrupt stream";
    case ZF_E_NOMEM: return "out of memory";
    case ZF_E_HIP: return "HIP runtime error";
    case ZF_E_TOO_SMALL: return "buffer too small";
    case ZF_E_STATE: return "bad state";
    }
    return "unknown status";
}

const char *zf_last_error(void) { return last_error().c_str(); }

}  // extern "C"
