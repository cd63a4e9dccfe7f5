// LZ77 decode (Non-Parallel) and plain copies.
#include "kernels.hpp"

namespace zf {
// knob: 16, 32 or 64 = lanes per chunk (16 output bytes per lane step);
// 4 or 8 = output bytes per lane step with 64 lanes per chunk.
void launch_lz(const LaunchArgs &A, uint32_t waves, uint32_t knob, hipStream_t st) {
    const uint32_t n = A.kind_begin[K_LZ + 1] - A.kind_begin[K_LZ];
    if (!n) return;
    const uint32_t per = knob == 16 ? 4 : knob == 32 ? 2 : 1, units = waves * per;
    const dim3 grid((n + units - 1) / units), block(64 * waves);
    const uint32_t blk = (knob == 4 || knob == 8) ? knob : 16;
    const size_t lds = waves * (blk == 4 ? sizeof(LzWave<4>) : blk == 8 ? sizeof(LzWave<8>) : sizeof(LzWave<16>));
    if (lds > 65536) {  // LDS beyond the default dynamic limit (160 KiB per CU)
        const void *f = knob == 16 ? reinterpret_cast<const void *>(&k_decode_lz<16, 16>)
                      : knob == 32 ? reinterpret_cast<const void *>(&k_decode_lz<32, 16>)
                      : knob == 4  ? reinterpret_cast<const void *>(&k_decode_lz<64, 4>)
                      : knob == 8  ? reinterpret_cast<const void *>(&k_decode_lz<64, 8>)
                                   : reinterpret_cast<const void *>(&k_decode_lz<64, 16>);
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    }
    if (knob == 16) hipLaunchKernelGGL((k_decode_lz<16, 16>), grid, block, lds, st, A);
    else if (knob == 32) hipLaunchKernelGGL((k_decode_lz<32, 16>), grid, block, lds, st, A);
    else if (knob == 4) hipLaunchKernelGGL((k_decode_lz<64, 4>), grid, block, lds, st, A);
    else if (knob == 8) hipLaunchKernelGGL((k_decode_lz<64, 8>), grid, block, lds, st, A);
    else hipLaunchKernelGGL((k_decode_lz<64, 16>), grid, block, lds, st, A);
}
ZF_DEFINE_LAUNCHER(K_PLAIN, launch_plain)
}  // namespace zf
