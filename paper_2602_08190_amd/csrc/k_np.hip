// LZ77 decode (Non-Parallel) and plain copies.
#include "kernels.hpp"

namespace zf {
// lanes: lanes per chunk (16, 32 or 64; other values select 64).
void launch_lz(const LaunchArgs &A, uint32_t waves, uint32_t lanes, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_LZ + 1] - A.kind_begin[K_LZ];
    if (!n) return;
    const uint32_t per = lanes == 16 ? 4 : lanes == 32 ? 2 : 1, units = waves * per;
    const dim3 grid((n + units - 1) / units), block(64 * waves);
    if (per == 4) hipLaunchKernelGGL(k_decode_lz<16>, grid, block, 0, st, A);
    else if (per == 2) hipLaunchKernelGGL(k_decode_lz<32>, grid, block, 0, st, A);
    else hipLaunchKernelGGL(k_decode_lz<64>, grid, block, 0, st, A);
}
ZF_DEFINE_LAUNCHER(K_PLAIN, launch_plain)
}  // namespace zf
