// Dictionary decode of 32-bit values (Fully-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_DICT32, launch_dict32)
}  // namespace zf
