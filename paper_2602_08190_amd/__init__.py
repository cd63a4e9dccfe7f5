"""zf: compressed column chunks streamed from pinned host memory over PCIe
and decoded on an MI355X by hand-written HIP kernels (the ZipFlow method's
hot path, built for gfx950).

The native library is ``libzf.so`` (C ABI in ``include/zf.h``); ``zf`` is its
Python binding.
"""
from . import zf  # noqa: F401
