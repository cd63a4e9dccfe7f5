// Group-Parallel decodes: RLE + delta, DeltaStride, String-dictionary.
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_RLE32, launch_rle32)
ZF_DEFINE_LAUNCHER(K_RLE64, launch_rle64)
ZF_DEFINE_LAUNCHER(K_SDICT, launch_sdict)
}  // namespace zf
