// RLE + delta decode (Group-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_RLE32, launch_rle32)
ZF_DEFINE_LAUNCHER(K_RLE64, launch_rle64)
}  // namespace zf
