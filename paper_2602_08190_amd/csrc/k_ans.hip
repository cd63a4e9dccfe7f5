// ANS decode (Non-Parallel: 64 interleaved coders per chunk).
#include "kernels.hpp"

namespace zf {
// One chunk per wave; each wave's model and output staging (kAnsLdsWords
// dwords) are dynamic LDS.
__global__ __launch_bounds__(1024) void k_decode_ans(LaunchArgs A) {
    const uint32_t waves = blockDim.x / 64;
    const uint32_t u = A.kind_begin[K_ANS] + blockIdx.x * waves + first32(threadIdx.x / 64);
    if (u >= A.kind_begin[K_ANS + 1]) return;
    extern __shared__ uint32_t ans_smem[];
    unit_ans(A, A.chunks[A.tiles[u].chunk], ans_smem + (threadIdx.x / 64) * kAnsLdsWords);
}

void launch_ans(const LaunchArgs &A, uint32_t waves, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_ANS + 1] - A.kind_begin[K_ANS];
    if (!n) return;
    waves = waves > 16 ? 16 : waves;
    const size_t lds = size_t(waves) * kAnsLdsWords * sizeof(uint32_t);  // at most 96 KiB
    if (lds > 65536)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_decode_ans),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL(k_decode_ans, dim3((n + waves - 1) / waves), dim3(64 * waves), lds, st, A);
}
}  // namespace zf
