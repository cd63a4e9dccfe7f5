// LZ77 decode (Non-Parallel) and plain copies.
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_LZ, launch_lz)
ZF_DEFINE_LAUNCHER(K_PLAIN, launch_plain)
}  // namespace zf
