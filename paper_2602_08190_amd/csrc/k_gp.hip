// Group-Parallel decodes: RLE + delta, DeltaStride (and its order-key tree),
// String-dictionary.
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_RLE32, launch_rle32)
ZF_DEFINE_LAUNCHER(K_RLE64, launch_rle64)
ZF_DEFINE_LAUNCHER(K_TREE, launch_tree)
// String-dictionary: tiles mapped XCD-aware (the tiles of a chunk share its
// dictionary, so neighbouring tiles go to the same XCD and its L2); each
// wave's staging buffer is dynamic shared memory, kSdBufAlloc dwords.
// skip_col: the tiles over a column dictionary are another launch's.
__global__ __launch_bounds__(1024) void k_decode_sdict(LaunchArgs A, uint32_t skip_col) {
    const uint32_t waves = blockDim.x / 64;
    const uint32_t u = A.kind_begin[K_SDICT] + xcd_block(blockIdx.x, gridDim.x) * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[K_SDICT + 1]) return;
    extern __shared__ uint32_t sd_smem[];
    const Tile t = A.tiles[u];
    const ChunkDesc &ck = A.chunks[t.chunk];
    if (skip_col && (ck.codec == C_SDICT_COL || ck.codec == C_SDICT_COL_ANS)) return;
    unit_sdict<true>(A, t, ck, sd_smem + (threadIdx.x / 64) * kSdBufAlloc);
}
// 14 or 16 waves: the tiles over a column dictionary go to two workgroups
// per compute unit, each taking a contiguous range of the kind's tiles (its
// waves take every W-th, skipping the others), with staging buffers of
// kSdSmallBuf dwords; the other tiles go to a launch of k_decode_sdict.  A workgroup first copies the hottest
// records of its first tile's column dictionary (the entries are ordered by
// decreasing count, so records 0, 1, ...) into the rest of its half of the
// LDS, after a zero row; its tiles over that dictionary read those records
// there (the frequent tokens, most of a Zipf text's tokens) and the others
// from global memory.
constexpr size_t kSdHotLds = 80 * 1024;  // per workgroup
template <uint32_t W>
constexpr uint32_t sd_hot_records() { return uint32_t((kSdHotLds - W * kSdSmallBuf * sizeof(uint32_t)) / 16) - 1; }
template <uint32_t W>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(W / 2, W / 2))) void k_decode_sdict_hot(
    LaunchArgs A) {
    constexpr uint32_t R = sd_hot_records<W>();
    const uint32_t begin = A.kind_begin[K_SDICT], n = A.kind_begin[K_SDICT + 1] - begin;
    const uint32_t lo = begin + uint32_t(uint64_t(n) * blockIdx.x / gridDim.x);
    const uint32_t hi = begin + uint32_t(uint64_t(n) * (blockIdx.x + 1) / gridDim.x);
    if (lo >= hi) return;  // the whole workgroup
    extern __shared__ u32x4 sd_hot[];
    const ChunkDesc &c0 = A.chunks[A.tiles[lo].chunk];
    const bool col0 = c0.codec == C_SDICT_COL || c0.codec == C_SDICT_COL_ANS;
    const uint32_t hn = col0 ? min(c0.dict_count, R) : 0u;
    const u32x4 *rec = reinterpret_cast<const u32x4 *>(A.fat + c0.fat_off);
    if (threadIdx.x == 0) sd_hot[0] = u32x4{0u, 0u, 0u, 0u};
    for (uint32_t r = threadIdx.x; r < hn; r += blockDim.x) sd_hot[1 + r] = rec[r];
    __syncthreads();
    const uint32_t w = first32(threadIdx.x / 64);
    uint32_t *buf = reinterpret_cast<uint32_t *>(sd_hot + R + 1) + w * kSdSmallBuf;
    for (uint32_t u = lo + w; u < hi; u += W) {
        const Tile t = A.tiles[u];
        const ChunkDesc &ck = A.chunks[t.chunk];
        if (ck.codec == C_SDICT_COL || ck.codec == C_SDICT_COL_ANS)
            unit_sdict_hot(A, t, ck, buf, sd_hot, col0 && ck.fat_off == c0.fat_off ? hn : 0u);
    }
}
template <uint32_t W>
static void launch_sdict_hot(const LaunchArgs &A, uint32_t n, hipStream_t st) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_decode_sdict_hot<W>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(kSdHotLds));
    const uint32_t blocks = min(2u * uint32_t(cus), (n + W - 1) / W);
    hipLaunchKernelGGL(k_decode_sdict_hot<W>, dim3(blocks), dim3(64 * W), kSdHotLds, st, A);
}
void launch_sdict(const LaunchArgs &A, uint32_t waves, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_SDICT + 1] - A.kind_begin[K_SDICT];
    if (!n) return;
    uint32_t skip_col = 0;
    if (waves >= 14) {
        if (A.sdict_codecs & 1u) {
            if (waves >= 16) launch_sdict_hot<16>(A, n, st);
            else launch_sdict_hot<14>(A, n, st);
            skip_col = 1;
        }
        if (!(A.sdict_codecs & 2u)) return;
        waves = 4;  // the other tiles
    }
    waves = waves > 12 ? 12u : waves;  // 12 staging buffers: 60.2 KiB of LDS per workgroup
    hipLaunchKernelGGL(k_decode_sdict, dim3((n + waves - 1) / waves), dim3(64 * waves),
                       waves * kSdBufAlloc * sizeof(uint32_t), st, A, skip_col);
}
}  // namespace zf
