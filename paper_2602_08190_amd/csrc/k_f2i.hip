// Float2Int + bit-packing decode (Fully-Parallel, float64 output).
#include "kernels.hpp"

namespace zf {
ZF_DEFINE_LAUNCHER(K_F2I, launch_f2i)
}  // namespace zf
