// Dictionary decode of 64-bit values (Fully-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_DICT64, launch_dict64)
}  // namespace zf
