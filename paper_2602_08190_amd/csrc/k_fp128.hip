// Dictionary decode of CHAR(16) values (Fully-Parallel).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_DICT128, launch_dict128)
}  // namespace zf
