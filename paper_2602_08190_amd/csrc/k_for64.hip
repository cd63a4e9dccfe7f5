// FOR decode of 64-bit values (Fully-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_FOR64, launch_for64)
}  // namespace zf
