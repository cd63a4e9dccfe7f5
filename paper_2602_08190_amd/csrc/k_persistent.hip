// The persistent multi-codec kernel, the small helper kernels and the host
// entry that enqueues a launch's decode.
#include "kernels.hpp"

namespace zf {

// Persistent: every wave pulls units from one queue until it is empty.
// Units are ordered by kind, the costliest kinds first.
__global__ __launch_bounds__(256) void k_decode_persistent(LaunchArgs A) {
    __shared__ __attribute__((aligned(16))) uint32_t lz_rows[4][kAnsLdsWords > kSdBufWords ? kAnsLdsWords : kSdBufWords];
    uint32_t *mine = lz_rows[threadIdx.x / 64];
    const uint32_t n = A.kind_begin[K_COUNT];
    for (;;) {
        uint32_t u = 0;
        if (lane_id() == 0) u = atomicAdd(A.counter, 1u);
        u = first32(u);
        if (u >= n) return;
        uint32_t kind = 0;
        while (kind + 1 < K_COUNT && u >= A.kind_begin[kind + 1]) kind++;
        run_unit<0>(A, kind, u, mine);
    }
}

__global__ void k_zero_counter(uint32_t *c) { *c = 0; }

struct OutTable {
    uint8_t *p[kMaxCols];
};
__global__ void k_set_out_tab(uint8_t **tab, OutTable t, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) tab[i] = t.p[i];
}

// ============================================================ host side
hipError_t launch_set_out_tab(uint8_t **d_tab, uint8_t *const *ptrs, uint32_t n, uint8_t *scratch,
                              hipStream_t st) {
    OutTable t{};
    for (uint32_t i = 0; i < n && i < kScratchCol; i++) t.p[i] = ptrs[i];
    t.p[kScratchCol] = scratch;
    hipLaunchKernelGGL(k_set_out_tab, dim3(1), dim3(kMaxCols), 0, st, d_tab, t, kMaxCols);
    return hipGetLastError();
}

// Enqueue the decode of one launch's units.  persistent_waves > 0 selects
// the persistent kernel with that many waves in flight.  With `ev`, an event
// is recorded on `st` before and after each kind's launch (slot K_COUNT: the
// persistent kernel), and ev->used says which were recorded.
hipError_t launch_decode(const LaunchArgs &A, uint32_t persistent_waves, const uint32_t *wpb,
                         uint32_t lz_blk, hipStream_t st, KindEvents *ev) {
    if (ev)
        for (uint32_t k = 0; k <= K_COUNT; k++) ev->used[k] = false;
    if (A.kind_begin[K_COUNT] == 0) return hipSuccess;
    auto mark = [&](uint32_t k, bool end) -> hipError_t {
        if (!ev) return hipSuccess;
        if (!end) ev->used[k] = true;
        return hipEventRecord(end ? ev->e1[k] : ev->e0[k], st);
    };
    hipError_t e = hipSuccess;
    if (persistent_waves) {
        if ((e = mark(K_COUNT, false)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(1), 0, st, A.counter);
        const uint32_t blocks = (persistent_waves + 3) / 4;
        hipLaunchKernelGGL(k_decode_persistent, dim3(blocks), dim3(256), 0, st, A);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return mark(K_COUNT, true);
    }
    // launch order: the slow serial kinds first
    // (TREE after the RLE kinds, which write its chunks' run starts; SDICT
    // after ANS, which writes its chunks' entry indices)
    static const uint32_t order[K_COUNT] = {K_LZ,     K_ANS,    K_RLE32, K_RLE64, K_TREE, K_SDICT, K_DICT128,
                                            K_DICT64, K_DICT32, K_FOR64, K_FOR32, K_F2I,  K_PLAIN};
    for (uint32_t i = 0; i < K_COUNT; i++) {
        const uint32_t k = order[i];
        if (A.kind_begin[k + 1] == A.kind_begin[k]) continue;
        if ((e = mark(k, false)) != hipSuccess) return e;
        switch (k) {
        case K_LZ: launch_lz(A, wpb[K_LZ], lz_blk, st); break;
        case K_ANS: launch_ans(A, wpb[K_ANS], st); break;
        case K_RLE32: launch_rle32(A, wpb[K_RLE32], st); break;
        case K_RLE64: launch_rle64(A, wpb[K_RLE64], st); break;
        case K_TREE: launch_tree(A, wpb[K_TREE], st); break;
        case K_SDICT: launch_sdict(A, wpb[K_SDICT], st); break;
        case K_DICT128: launch_dict128(A, wpb[K_DICT128], st); break;
        case K_DICT64: launch_dict64(A, wpb[K_DICT64], st); break;
        case K_DICT32: launch_dict32(A, wpb[K_DICT32], st); break;
        case K_FOR64: launch_for64(A, wpb[K_FOR64], st); break;
        case K_FOR32: launch_for32(A, wpb[K_FOR32], st); break;
        case K_F2I: launch_f2i(A, wpb[K_F2I], st); break;
        case K_PLAIN: launch_plain(A, wpb[K_PLAIN], st); break;
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = mark(k, true)) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace zf
