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
__global__ __launch_bounds__(1024) void k_decode_sdict(LaunchArgs A) {
    const uint32_t waves = blockDim.x / 64;
    const uint32_t u = A.kind_begin[K_SDICT] + xcd_block(blockIdx.x, gridDim.x) * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[K_SDICT + 1]) return;
    extern __shared__ uint32_t sd_smem[];
    const Tile t = A.tiles[u];
    unit_sdict<true>(A, t, A.chunks[t.chunk], sd_smem + (threadIdx.x / 64) * kSdBufAlloc);
}
void launch_sdict(const LaunchArgs &A, uint32_t waves, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_SDICT + 1] - A.kind_begin[K_SDICT];
    if (!n) return;
    waves = waves > 12 ? 12u : waves;  // 12 staging buffers: 60.2 KiB of LDS per workgroup
    hipLaunchKernelGGL(k_decode_sdict, dim3((n + waves - 1) / waves), dim3(64 * waves),
                       waves * kSdBufAlloc * sizeof(uint32_t), st, A);
}
}  // namespace zf
