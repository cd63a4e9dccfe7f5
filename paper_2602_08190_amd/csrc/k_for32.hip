// FOR decode of 32-bit values (Fully-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_FOR32, launch_for32)
}  // namespace zf
