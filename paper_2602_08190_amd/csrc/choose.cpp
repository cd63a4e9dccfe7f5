// Measured (codec, schedule) choice for ZF_AUTO near-ties (Sec. 3.3: the
// learned model stands in for measurement, and exhaustive measurement backs
// it up): a candidate is encoded on its own, exactly as a chunk of the column
// would be, and its transfer + decode time is taken from the pipeline's own
// events on the given device.
#include <algorithm>
#include <cstring>

#include "plan.hpp"

namespace zf {

void compress_host(const void *src, uint64_t n_elems, uint32_t dtype, uint32_t codec,
                   const zf_encode_opts &o, zf_column_t *col, const uint8_t *forced_sched);
void transfer_and_decompress(zf_plan_t *P, void *const *d_out, hipStream_t st, zf_timing *timing);
void sync_plan(zf_plan_t *P, hipStream_t st);
void build_plan(zf_plan_t *P, const zf_column *const *cols, uint32_t n_cols, int device,
                const zf_plan_opts &o);

namespace {
struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        ZF_HIP(hipGetDevice(&prev));
        if (prev != dev) ZF_HIP(hipSetDevice(dev));
    }
    ~DeviceScope() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};
struct DeviceBuffer {
    void *p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};
struct Stream {
    hipStream_t s = nullptr;
    ~Stream() {
        if (s) (void)hipStreamDestroy(s);
    }
};
}  // namespace

// Median of three timed runs (after one untimed) of h2d + decode, in ms, for
// n values at x encoded with `codec` and schedule `sched` (1..4).  LZ77's
// schedule is its chunk size (8, 16, 32 or 64 KiB), the others' a tile unit.
double time_choice(const uint8_t *x, uint32_t n, uint32_t dtype, uint32_t codec, uint32_t sched, int device,
                   int threads) {
    const uint32_t es = elem_size(dtype);
    ZF_REQUIRE(es && n > 0 && sched >= 1 && sched <= 4, ZF_E_INVALID, "bad candidate");
    std::vector<uint32_t> ce;
    if (codec == C_LZ77) {
        const uint32_t per = std::max<uint32_t>(1, (8192u << (sched - 1)) / es);
        for (uint32_t a = 0; a < n; a += per) ce.push_back(std::min(per, n - a));
    } else {
        ce.push_back(n);
    }
    std::vector<uint32_t> cc(ce.size(), codec);
    std::vector<uint8_t> sc(ce.size(), uint8_t(sched));
    zf_encode_opts o;
    std::memset(&o, 0, sizeof o);
    o.pinned = 1;
    o.n_threads = threads;
    o.chunk_elems = ce.data();
    o.n_chunk_elems = uint32_t(ce.size());
    o.chunk_codecs = cc.data();
    zf_column col;
    compress_host(x, n, dtype, codec, o, &col, sc.data());

    DeviceScope scope(device);
    zf_plan_opts po;
    zf_plan_opts_default(&po);
    po.slot_bytes = std::max<uint64_t>(1u << 20, col.buf.n);
    const zf_column *cols[1] = {&col};
    zf_plan_t P;
    build_plan(&P, cols, 1, device, po);
    DeviceBuffer out;
    ZF_HIP(hipMalloc(&out.p, (col.view.plain_bytes + 15) & ~uint64_t(15)));
    Stream st;
    ZF_HIP(hipStreamCreateWithFlags(&st.s, hipStreamNonBlocking));
    void *outs[1] = {out.p};
    double t[4];
    for (int r = 0; r < 4; r++) {
        zf_timing tm{};
        transfer_and_decompress(&P, outs, st.s, &tm);
        sync_plan(&P, st.s);
        t[r] = tm.h2d_ms + tm.decode_ms;
    }
    std::sort(t + 1, t + 4);
    return t[2];
}

}  // namespace zf
