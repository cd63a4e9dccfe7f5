// LZ77 decode (Non-Parallel) and plain copies.
#include "kernels.hpp"

namespace zf {
// blk: output bytes per block (4, 8 or 16; other values select 16).
void launch_lz(const LaunchArgs &A, uint32_t waves, uint32_t blk, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_LZ + 1] - A.kind_begin[K_LZ];
    if (!n) return;
    blk = (blk == 4 || blk == 8) ? blk : 16;
    const dim3 grid((n + waves - 1) / waves), block(64 * waves);
    const size_t lds = size_t(waves) * 64 * blk * sizeof(uint32_t);  // at most 64 KiB
    if (blk == 4) hipLaunchKernelGGL(k_decode_lz<4>, grid, block, lds, st, A);
    else if (blk == 8) hipLaunchKernelGGL(k_decode_lz<8>, grid, block, lds, st, A);
    else hipLaunchKernelGGL(k_decode_lz<16>, grid, block, lds, st, A);
}
ZF_DEFINE_LAUNCHER(K_PLAIN, launch_plain)
}  // namespace zf
