// zf_plan: per-chunk work units with device-specific tile shapes (Sec. 4),
// batches no larger than a staging slot, Johnson's order over the batches'
// (transfer, decode) estimates (Sec. 3.3), and the device workspace.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "plan.hpp"
#include "tune.hpp"

namespace zf {

// Output-balanced Group-Parallel units over n elements whose ng groups start
// at gof(g): about `unit` outputs each, cut at a group boundary when one is
// near, so a unit rarely rescans a group.  Tile {chunk, first group, first
// element, end element}.
template <class GroupOffset>
static void gp_tiles(std::vector<Tile> &T, uint32_t idx, uint32_t ng, uint32_t n, uint32_t unit,
                     GroupOffset gof) {
    uint32_t e = 0, g = 0;
    while (e < n) {
        while (g + 1 < ng && gof(g + 1) <= e) g++;
        const uint64_t target = uint64_t(e) + unit;
        uint32_t e_end;
        if (target >= n) {
            e_end = n;
        } else {
            uint32_t gb = g + 1;
            while (gb < ng && gof(gb) < target) gb++;
            e_end = (gb < ng && gof(gb) <= target + unit) ? gof(gb) : uint32_t(target);
        }
        T.push_back({idx, g, e, e_end});
        e = e_end;
    }
}

// The 16-byte entry records of a column token dictionary (host validated:
// every entry of 1..64 bytes lies inside the entry bytes): an entry's first
// 15 bytes, zero past its length, then its length, so that one aligned
// 16-byte read gives a token of up to 15 bytes and its length.
static void fat_records(const zf_column &col, std::vector<uint8_t> &out) {
    const uint8_t *d = col.buf.p + col.view.dict_off;
    const uint32_t ne = col.view.dict_count;
    const uint8_t *bytes = d + 16 + 4ull * ne;
    const size_t at = out.size();
    out.resize(at + uint64_t(kFatBytes) * ne, 0);
    for (uint32_t k = 0; k < ne; k++) {
        const uint32_t e = rd32(d + 16 + 4ull * k), len = e >> 24, off = e & 0xFFFFFFu;
        uint8_t *r = out.data() + at + uint64_t(kFatBytes) * k;
        std::memcpy(r, bytes + off, std::min(len, kFatInline));
        r[kFatInline] = uint8_t(len);
    }
}

static void add_chunk(WorkTables &w, const zf_column &col, uint32_t ci, uint32_t col_idx,
                      uint64_t comp_off, uint64_t dict_off, const TileShape &ts, uint64_t fat_off = 0) {
    const ChunkInfo &c = col.view.chunks[ci];
    ChunkDesc d{};
    d.comp_off = comp_off;
    d.out_off = c.plain_off;
    d.dict_off = dict_off;
    d.comp_len = c.comp_len;
    d.n_elems = c.n_elems;
    d.dict_count = col.view.dict_count;
    d.dict_bytes = col.view.dict_bytes;
    d.col = uint16_t(col_idx);
    d.codec = c.codec;
    d.dtype = uint8_t(col.view.dtype);
    const bool col_dict = c.codec == C_SDICT_COL || c.codec == C_SDICT_COL_ANS;
    d.fat_off = col_dict ? fat_off : 0;
    if (c.codec == C_SDICT_ANS || c.codec == C_SDICT_COL_ANS) {
        // first stage: ANS-decode the packed entry indices into the scratch
        // area; the String-dictionary stage reads them from there
        const uint8_t *s = col.buf.p + c.comp_off;
        const uint32_t nt = rd32(s), wd = rd32(s + (col_dict ? 4 : 8)), co = rd32(s + (col_dict ? 12 : 24));
        const uint64_t ncb = 4 * ((uint64_t(nt) * wd + 31) / 32);
        d.aux_off = w.scratch_bytes;
        if (ncb) {
            // one ANS unit per piece (the host checked the piece table)
            const uint32_t np = rd32(s + co);
            const uint64_t base = co + 4 + 4ull * np;
            uint64_t prev = 0;
            for (uint32_t k = 0; k < np; k++) {
                const uint64_t end = rd32(s + co + 4 + 4ull * k);
                ChunkDesc a = d;
                a.comp_off = comp_off + base + prev;
                a.comp_len = uint32_t(kAnsHdr + 2ull * rd32(s + base + prev + 4));  // without padding
                a.n_elems = uint32_t(std::min<uint64_t>(kSdAnsPiece, ncb - uint64_t(k) * kSdAnsPiece));
                a.out_off = d.aux_off + uint64_t(k) * kSdAnsPiece;
                a.col = uint16_t(kScratchCol);
                a.codec = C_ANS;
                a.dtype = D_BYTES;
                a.aux_off = 0;
                w.tiles[K_ANS].push_back({uint32_t(w.chunks.size()), 0, 0, 0});
                w.chunks.push_back(a);
                prev = end;
            }
            w.scratch_bytes = align_up(d.aux_off + ncb, 256);
        }
    }
    if (c.codec == C_DSTREE) {
        // first stage: the run starts S (R values) into the scratch area, as
        // units of the RLE kind of the column's width; the second stage
        // (kind TREE, launched after the RLE kinds) reads them there
        const uint8_t *s = col.buf.p + c.comp_off;
        const uint32_t R = rd32(s), ngA = rd32(s + 12);
        const uint32_t es = col.view.dtype == D_I32 ? 4 : 8;
        const Kind ks = col.view.dtype == D_I32 ? K_RLE32 : K_RLE64;
        d.aux_off = w.scratch_bytes;
        ChunkDesc a = d;
        a.out_off = d.aux_off;
        a.n_elems = R;
        a.col = uint16_t(kScratchCol);
        a.codec = C_DSTREE_STARTS;
        const uint32_t aidx = uint32_t(w.chunks.size());
        w.chunks.push_back(a);
        gp_tiles(w.tiles[ks], aidx, ngA, R, ts.unit[ks], [&](uint32_t g) { return rd32(s + 32 + 32ull * g); });
        w.scratch_bytes = align_up(d.aux_off + uint64_t(R) * es, 256);
    }
    const uint32_t idx = uint32_t(w.chunks.size());
    w.chunks.push_back(d);
    const Kind k = kind_of(c.codec, col.view.dtype);
    std::vector<Tile> &T = w.tiles[k];
    const uint32_t unit = scheduled_unit(k, c.sched, ts.unit[k]);
    switch (k) {
    case K_PLAIN:
        for (uint64_t a = 0; a < c.plain_len; a += unit)
            T.push_back({idx, uint32_t(a), uint32_t(std::min<uint64_t>(c.plain_len, a + unit)), 0});
        break;
    case K_FOR32:
    case K_FOR64:
    case K_DICT32:
    case K_DICT64:
    case K_DICT128:
    case K_F2I: {
        const uint32_t nb = (c.n_elems + kForBlock - 1) / kForBlock;
        for (uint32_t b = 0; b < nb; b += unit) T.push_back({idx, b, std::min(unit, nb - b), 0});
        break;
    }
    case K_RLE32:
    case K_RLE64: {
        const uint8_t *s = col.buf.p + c.comp_off;
        gp_tiles(T, idx, rd32(s + 4), c.n_elems, unit, [&](uint32_t g) { return rd32(s + 16 + 32ull * g); });
        break;
    }
    case K_TREE: {
        const uint8_t *s = col.buf.p + c.comp_off;
        const uint32_t b_off = rd32(s + 24);
        gp_tiles(T, idx, rd32(s + 4), c.n_elems, unit, [&](uint32_t g) { return rd32(s + b_off + 16ull * g); });
        break;
    }
    case K_SDICT: {
        // whole groups of 64 tokens, about `unit` output bytes per unit
        const uint8_t *s = col.buf.p + c.comp_off;
        const uint32_t ng = rd32(s + (col_dict ? 8 : 12)), n = c.plain_len, go = col_dict ? 16 : 32;
        auto gof = [&](uint32_t g) { return g < ng ? rd32(s + go + 4ull * g) : n; };
        for (uint32_t g = 0; g < ng;) {
            uint32_t gb = g + 1;
            while (gb < ng && gof(gb) - gof(g) < unit && gb - g < 63) gb++;  // at most 63 groups per unit
            T.push_back({idx, g, gb, 0});
            g = gb;
        }
        break;
    }
    case K_LZ:
    case K_ANS: T.push_back({idx, 0, 0, 0}); break;
    default: break;
    }
    w.plain_bytes += c.plain_len;
    w.comp_bytes += c.comp_len;
    w.t_dec += double(c.plain_len) / (ts.rate_gbps[k] * 1e9);
}

// Johnson's rule (Sec. 3.3): batches whose copy is shorter than their decode
// first, by increasing copy time; the rest by decreasing decode time; equal
// keys keep the lower batch index first (stable sorts of ascending indices).
std::vector<uint32_t> johnson(const std::vector<double> &a, const std::vector<double> &b) {
    std::vector<uint32_t> first, rest;
    for (uint32_t i = 0; i < a.size(); i++) (a[i] < b[i] ? first : rest).push_back(i);
    std::stable_sort(first.begin(), first.end(), [&](uint32_t x, uint32_t y) { return a[x] < a[y]; });
    std::stable_sort(rest.begin(), rest.end(), [&](uint32_t x, uint32_t y) { return b[x] > b[y]; });
    first.insert(first.end(), rest.begin(), rest.end());
    return first;
}

std::vector<zf_unit> chunk_units(const zf_column &col, uint32_t ci, const zf_plan_opts &o) {
    ZF_REQUIRE(ci < col.view.n_chunks, ZF_E_INVALID, "chunk %u of %u", ci, col.view.n_chunks);
    WorkTables w;
    add_chunk(w, col, ci, 0, 0, 0, resolve_tiles(o));
    std::vector<zf_unit> u;
    for (uint32_t k = 0; k < K_COUNT; k++)
        for (const Tile &t : w.tiles[k]) u.push_back({k, t.a, t.b, t.c});
    return u;
}

// Size in bytes of a launch's flattened tables.
static uint64_t table_bytes(const WorkTables &w) {
    uint64_t n = align_up(w.chunks.size() * sizeof(ChunkDesc), 256);
    for (int k = 0; k < K_COUNT; k++) n += w.tiles[k].size() * sizeof(Tile);
    return align_up(n, 256);
}

// Copy a launch's tables into host staging at `off`; fill its LaunchArgs.
static void flatten(const WorkTables &w, std::vector<uint8_t> &host, uint64_t off, uint8_t *d_base,
                    LaunchArgs &A) {
    uint8_t *h = host.data() + off;
    std::memcpy(h, w.chunks.data(), w.chunks.size() * sizeof(ChunkDesc));
    A.chunks = reinterpret_cast<const ChunkDesc *>(d_base + off);
    uint64_t t = align_up(w.chunks.size() * sizeof(ChunkDesc), 256);
    A.tiles = reinterpret_cast<const Tile *>(d_base + off + t);
    uint32_t u = 0;
    for (int k = 0; k < K_COUNT; k++) {
        A.kind_begin[k] = u;
        std::memcpy(h + t + uint64_t(u) * sizeof(Tile), w.tiles[k].data(), w.tiles[k].size() * sizeof(Tile));
        u += uint32_t(w.tiles[k].size());
    }
    A.kind_begin[K_COUNT] = u;
    A.two_stage = w.scratch_bytes > 0;
    A.sdict_codecs = 0;
    for (const Tile &t : w.tiles[K_SDICT]) {
        const uint32_t c = w.chunks[t.chunk].codec;
        A.sdict_codecs |= c == C_SDICT_COL || c == C_SDICT_COL_ANS ? 1u : 2u;
    }
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        ZF_HIP(hipGetDevice(&prev));
        if (prev != dev) ZF_HIP(hipSetDevice(dev));
    }
    ~DeviceGuard() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

void build_plan(zf_plan_t *P, const zf_column *const *cols, uint32_t n_cols, int device,
                const zf_plan_opts &o) {
    ZF_REQUIRE(cols && n_cols >= 1 && n_cols <= kScratchCol, ZF_E_INVALID,
               "a plan needs 1..%u columns", kScratchCol);
    for (uint32_t c = 0; c < n_cols; c++) ZF_REQUIRE(cols[c], ZF_E_INVALID, "column %u is null", c);
    ZF_REQUIRE(o.n_slots >= 1, ZF_E_INVALID, "n_slots must be >= 1");
    P->device = device;
    P->opts = o;
    P->cols.assign(cols, cols + n_cols);

    const TileShape ts = resolve_tiles(o);

    DeviceGuard dg(device);
    hipDeviceProp_t prop;
    ZF_HIP(hipGetDeviceProperties(&prop, device));
    P->cu_count = uint32_t(prop.multiProcessorCount);
    for (uint32_t k = 0; k < K_COUNT; k++) P->waves_per_block[k] = ts.wpb[k];
    P->lz_blk = ts.unit[K_LZ];
    P->persistent_waves = o.persistent ? P->cu_count * ts.wpcu : 0;

    // ---- the entry records of every column token dictionary
    std::vector<uint8_t> fat;
    std::vector<uint64_t> fat_at(n_cols, 0);
    for (uint32_t c = 0; c < n_cols; c++)
        if (cols[c]->view.dtype == D_BYTES && cols[c]->view.dict_count) {
            fat_at[c] = fat.size();
            fat_records(*cols[c], fat);
        }

    // ---- image layout and its tables
    WorkTables image;
    P->image_off.resize(n_cols);
    uint64_t at = 0;
    for (uint32_t c = 0; c < n_cols; c++) {
        P->image_off[c] = at;
        at = align_up(at + cols[c]->buf.n, 256);
    }
    P->image_bytes = at;
    for (uint32_t c = 0; c < n_cols; c++) {
        const zf_column &col = *cols[c];
        for (uint32_t i = 0; i < col.view.n_chunks; i++)
            add_chunk(image, col, i, c, P->image_off[c] + col.view.chunks[i].comp_off,
                      P->image_off[c] + col.view.dict_off, ts, fat_at[c]);
    }

    // ---- staged mode: dictionaries, then batches of whole chunks
    std::vector<uint64_t> dict_at(n_cols, 0);
    uint64_t dict_total = 0;
    for (uint32_t c = 0; c < n_cols; c++) {
        const zf_column &col = *cols[c];
        if (!col.view.dict_count) continue;
        const uint64_t len = col.view.dict_bytes;
        dict_at[c] = dict_total;
        P->dict_copies.push_back({col.buf.p + col.view.dict_off, dict_total, len});
        dict_total = align_up(dict_total + len, 256);
    }
    P->dict_bytes = dict_total;

    uint64_t slot = o.slot_bytes ? o.slot_bytes : (256ull << 20);
    for (uint32_t c = 0; c < n_cols; c++)
        for (auto &ch : cols[c]->view.chunks) slot = std::max<uint64_t>(slot, align_up(ch.comp_len, 256));
    P->slot_bytes = slot;

    std::vector<Batch> batches;
    Batch cur;
    int64_t range_col = -1;
    uint64_t range_src = 0, range_dst = 0;  // current contiguous copy
    uint32_t range_next_chunk = 0;
    auto close = [&]() {
        if (!cur.w.chunks.empty()) batches.push_back(std::move(cur));
        cur = Batch{};
        range_col = -1;
    };
    for (uint32_t c = 0; c < n_cols; c++) {
        const zf_column &col = *cols[c];
        for (uint32_t i = 0; i < col.view.n_chunks; i++) {
            const ChunkInfo &ch = col.view.chunks[i];
            const bool extends = range_col == int64_t(c) && range_next_chunk == i;
            uint64_t need = extends ? range_dst + (ch.comp_off + ch.comp_len - range_src)
                                    : align_up(cur.slot_used, 256) + ch.comp_len;
            if (need > slot) {
                close();
                need = ch.comp_len;
            }
            if (!(range_col == int64_t(c) && range_next_chunk == i)) {
                range_col = c;
                range_src = ch.comp_off;
                range_dst = align_up(cur.slot_used, 256);
                cur.copies.push_back({col.buf.p + range_src, range_dst, 0});
            }
            const uint64_t dst = range_dst + (ch.comp_off - range_src);
            cur.copies.back().len = ch.comp_off + ch.comp_len - range_src;
            cur.slot_used = dst + ch.comp_len;
            range_next_chunk = i + 1;
            add_chunk(cur.w, col, i, c, dst, dict_at[c], ts, fat_at[c]);
        }
    }
    close();
    const double pcie = (o.pcie_gbps > 0 ? o.pcie_gbps : 55.0) * 1e9;
    std::vector<double> ta, tb;
    for (uint32_t i = 0; i < batches.size(); i++) {
        Batch &b = batches[i];
        uint64_t bytes = 0;
        for (auto &cp : b.copies) bytes += cp.len;
        b.index = i;
        b.t_h2d = double(bytes) / pcie;
        ta.push_back(b.t_h2d);
        tb.push_back(b.w.t_dec);
    }
    std::vector<uint32_t> order(batches.size());
    std::iota(order.begin(), order.end(), 0u);
    if (o.order == 0) order = johnson(ta, tb);
    for (uint32_t k = 0; k < order.size(); k++) P->batches.push_back(std::move(batches[order[k]]));

    // ---- device memory
    uint64_t tb_total = table_bytes(image);
    for (auto &b : P->batches) tb_total += table_bytes(b.w);
    std::vector<uint8_t> host(tb_total, 0);
    ZF_HIP(hipMalloc(&P->d_tables, std::max<uint64_t>(tb_total, 256)));
    ZF_HIP(hipMalloc(&P->d_out_tab, sizeof(uint8_t *) * kMaxCols));
    // error word, then the persistent queue heads from byte 256 (2 x 8 of
    // them, 128 bytes apart)
    ZF_HIP(hipMalloc(&P->d_err, 256 + 16 * 128));
    ZF_HIP(hipMemset(P->d_err, 0, 256 + 16 * 128));
    uint64_t off = 0;
    flatten(image, host, off, P->d_tables, P->image_args);
    off += table_bytes(image);
    for (auto &b : P->batches) {
        flatten(b.w, host, off, P->d_tables, b.args);
        off += table_bytes(b.w);
    }
    ZF_HIP(hipMemcpy(P->d_tables, host.data(), tb_total, hipMemcpyHostToDevice));

    const int ns = o.n_slots;
    if (!P->batches.empty()) {
        P->d_slots.assign(std::min<size_t>(ns, P->batches.size()), nullptr);
        for (auto &sp : P->d_slots) ZF_HIP(hipMalloc(&sp, slot));
    }
    if (dict_total) ZF_HIP(hipMalloc(&P->d_dict, dict_total));
    if (!fat.empty()) {
        ZF_HIP(hipMalloc(&P->d_fat, fat.size()));
        ZF_HIP(hipMemcpy(P->d_fat, fat.data(), fat.size(), hipMemcpyHostToDevice));
    }
    P->scratch_bytes = image.scratch_bytes;
    for (auto &b : P->batches) P->scratch_bytes = std::max(P->scratch_bytes, b.w.scratch_bytes);
    if (P->scratch_bytes) ZF_HIP(hipMalloc(&P->d_scratch, P->scratch_bytes));

    auto fill = [&](LaunchArgs &A) {
        A.out_tab = P->d_out_tab;
        A.err = P->d_err;
        A.counter = P->d_err + 64;
        A.fat = P->d_fat;
    };
    fill(P->image_args);
    for (uint32_t k = 0; k < P->batches.size(); k++) {
        Batch &b = P->batches[k];
        b.slot = int(k % P->d_slots.size());
        fill(b.args);
        b.args.comp = P->d_slots[b.slot];
        b.args.dict = P->d_dict;
    }

    // ---- streams, events, graphs
    ZF_HIP(hipStreamCreateWithFlags(&P->copy_stream, hipStreamNonBlocking));
    const size_t nsl = P->d_slots.size();
    P->slot_full.resize(nsl);
    P->slot_free.resize(nsl);
    for (size_t s = 0; s < nsl; s++) {
        ZF_HIP(hipEventCreateWithFlags(&P->slot_full[s], hipEventDisableTiming));
        ZF_HIP(hipEventCreateWithFlags(&P->slot_free[s], hipEventDisableTiming));
    }
    auto mk = [&](std::vector<hipEvent_t> &v) {
        v.resize(P->batches.size());
        for (auto &e : v) ZF_HIP(hipEventCreate(&e));
    };
    mk(P->ev_h2d0);
    mk(P->ev_h2d1);
    mk(P->ev_dec0);
    mk(P->ev_dec1);
    ZF_HIP(hipEventCreate(&P->ev_start));
    ZF_HIP(hipEventCreate(&P->ev_end));
    ZF_HIP(hipEventCreateWithFlags(&P->ev_dict, hipEventDisableTiming));

    if (o.use_graphs && !P->batches.empty()) {
        hipStream_t cap;
        ZF_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        try {
            for (auto &b : P->batches) {
                ZF_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
                hipError_t le = launch_decode(b.args, P->persistent_waves, P->waves_per_block, P->lz_blk, cap);
                hipError_t ce = hipStreamEndCapture(cap, &b.graph);
                ZF_HIP(le);
                ZF_HIP(ce);
                ZF_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
            }
        } catch (...) {
            (void)hipStreamDestroy(cap);
            throw;
        }
        ZF_HIP(hipStreamDestroy(cap));
    }
}

void release_plan(zf_plan_t *P) {
    zf_plan_t &p = *P;
    int device = p.device;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != device) (void)hipSetDevice(device);
    if (p.copy_stream) (void)hipStreamSynchronize(p.copy_stream);
    for (auto &b : p.batches) {
        if (b.exec) (void)hipGraphExecDestroy(b.exec);
        if (b.graph) (void)hipGraphDestroy(b.graph);
    }
    auto kill = [](std::vector<hipEvent_t> &v) {
        for (auto e : v)
            if (e) (void)hipEventDestroy(e);
    };
    kill(p.slot_full);
    kill(p.slot_free);
    kill(p.ev_h2d0);
    kill(p.ev_h2d1);
    kill(p.ev_dec0);
    kill(p.ev_dec1);
    for (auto e : {p.ev_start, p.ev_end, p.ev_dict})
        if (e) (void)hipEventDestroy(e);
    for (uint32_t k = 0; k <= K_COUNT; k++)
        for (auto e : {p.kind_ev.e0[k], p.kind_ev.e1[k]})
            if (e) (void)hipEventDestroy(e);
    if (p.copy_stream) (void)hipStreamDestroy(p.copy_stream);
    for (auto sp : p.d_slots)
        if (sp) (void)hipFree(sp);
    if (p.d_dict) (void)hipFree(p.d_dict);
    if (p.d_tables) (void)hipFree(p.d_tables);
    if (p.d_out_tab) (void)hipFree(p.d_out_tab);
    if (p.d_scratch) (void)hipFree(p.d_scratch);
    if (p.d_fat) (void)hipFree(p.d_fat);
    if (p.d_err) (void)hipFree(p.d_err);
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
}

}  // namespace zf
