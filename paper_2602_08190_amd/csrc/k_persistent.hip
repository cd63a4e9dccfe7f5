// The persistent multi-codec kernel, the small helper kernels and the host
// entry that enqueues a launch's decode.
#include "kernels.hpp"

namespace zf {

// Persistent: waves pull units of [ub, ue) from eight queues, one per XCD,
// until all are empty.  Units are ordered by kind, the costliest kinds first;
// the range is dealt to the queues in blocks of kPersistBlock consecutive
// units, round robin, so every XCD works through the kinds in that order and
// neighbouring tiles of a chunk stay on one XCD (and its L2).  A workgroup
// starts on the queue of its own XCD (workgroups are dealt to the XCDs in
// turn) and moves on to the others' when it is empty.  ctr: the eight
// counters, 32 dwords apart.
constexpr uint32_t kPersistBlock = 16;
// Its register budget is the union of every kind's routine (about 140 VGPRs
// unconstrained, 2 to 3 waves per SIMD); it is held to 128 (4 waves per SIMD,
// a few spills), the fastest of 2, 4 and 6 waves per SIMD on the fact table.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_decode_persistent(
    LaunchArgs A, uint32_t ub, uint32_t ue, uint32_t *ctr) {
    __shared__ __attribute__((aligned(16))) uint32_t lz_rows[4][kAnsLdsWords > kSdBufAlloc ? kAnsLdsWords : kSdBufAlloc];
    uint32_t *mine = lz_rows[threadIdx.x / 64];
    const uint32_t n = ue - ub, nblk = (n + kPersistBlock - 1) / kPersistBlock;
    const uint32_t x0 = blockIdx.x % 8;
    for (uint32_t k = 0; k < 8; k++) {
        const uint32_t x = (x0 + k) % 8;
        // queue x holds blocks x, x + 8, x + 16, ... of the range
        const uint32_t qlen = x < nblk ? ((nblk - x + 7) / 8) * kPersistBlock : 0u;
        for (;;) {
            uint32_t i = 0;
            if (lane_id() == 0) i = atomicAdd(ctr + 32 * x, 1u);
            i = first32(i);
            if (i >= qlen) break;
            const uint32_t u = ub + ((i / kPersistBlock) * 8 + x) * kPersistBlock + i % kPersistBlock;
            if (u >= ue) continue;  // the last block's tail
            uint32_t kind = 0;
            while (kind + 1 < K_COUNT && u >= A.kind_begin[kind + 1]) kind++;
            run_unit<0>(A, kind, u, mine);
        }
    }
}

__global__ void k_zero_counters(uint32_t *c) {
    if (threadIdx.x < 16) c[32 * threadIdx.x] = 0;
}

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
        // two-stage chunks: the kinds up to RLE (LZ77, ANS, RLE) write the
        // scratch area that String-dictionary and TREE units read, so they
        // get a launch of their own first; otherwise one launch takes all
        if ((e = mark(K_COUNT, false)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, A.counter);
        const uint32_t blocks = (persistent_waves + 3) / 4, all = A.kind_begin[K_COUNT];
        const uint32_t cut = A.two_stage ? A.kind_begin[K_SDICT] : all;
        if (cut > 0)
            hipLaunchKernelGGL(k_decode_persistent, dim3(blocks), dim3(256), 0, st, A, 0u, cut, A.counter);
        if (all > cut)
            hipLaunchKernelGGL(k_decode_persistent, dim3(blocks), dim3(256), 0, st, A, cut, all,
                               A.counter + 8 * 32);
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
