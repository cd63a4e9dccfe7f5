"""Python binding of libzf (``include/zf.h``): argument marshalling only.

Every step of the hot path runs in the native library and its HIP kernels;
PyTorch tensors are used only as device buffers (their data pointers) and
streams (their HIP stream handles).  If ``libzf.so`` cannot be loaded the
binding raises instead of falling back to anything else.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzf.so")

# dtypes and codecs (zf.h)
I32, I64, BYTES, FIXED16, F64 = 1, 2, 3, 4, 5
AUTO, PLAIN, FOR_BP, DICT_BP, DELTA_BP, RLE_DELTA_BP, LZ77, F2I_BP, ANS, DSTRIDE_BP, SDICT_BP, SDICT_ANS = \
    0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11
SDICT_COL, SDICT_COL_ANS, DSTREE = 12, 13, 14
CODEC_NAMES = {PLAIN: "PLAIN", FOR_BP: "FOR_BP", DICT_BP: "DICT_BP", DELTA_BP: "DELTA_BP",
               RLE_DELTA_BP: "RLE_DELTA_BP", LZ77: "LZ77", F2I_BP: "F2I_BP", ANS: "ANS",
               DSTRIDE_BP: "DSTRIDE_BP", SDICT_BP: "SDICT_BP", SDICT_ANS: "SDICT_ANS",
               SDICT_COL: "SDICT_COL", SDICT_COL_ANS: "SDICT_COL_ANS", DSTREE: "DSTREE"}
ELEM_SIZE = {I32: 4, I64: 8, BYTES: 1, FIXED16: 16, F64: 8}
OK, E_INVALID, E_UNSUPPORTED, E_CORRUPT, E_NOMEM, E_HIP, E_TOO_SMALL, E_STATE = range(8)


class ZfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"zf status {status}: {msg}")
        self.status = status


class EncodeOpts(ctypes.Structure):
    _fields_ = [("chunk_bytes_min", ctypes.c_uint32), ("chunk_bytes_max", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("n_threads", ctypes.c_int32),
                ("pinned", ctypes.c_int32), ("chunk_elems", ctypes.c_void_p),
                ("n_chunk_elems", ctypes.c_uint32), ("chunk_codecs", ctypes.c_void_p),
                ("mlp_weights", ctypes.c_char_p), ("fallback_device", ctypes.c_int32),
                ("fallback_margin", ctypes.c_float)]


# kernel kinds (zf_kind), in enum order
KINDS = ["LZ77", "ANS", "RLE64", "RLE32", "SDICT", "DICT128", "DICT64", "DICT32", "FOR64", "FOR32", "F2I",
         "PLAIN", "TREE"]
KIND_GROUPS = {"FP": ["FOR32", "FOR64", "DICT32", "DICT64", "DICT128", "F2I"],
               "GP": ["RLE32", "RLE64", "SDICT", "TREE"],
               "NP": ["LZ77", "ANS"]}


class Tile(ctypes.Structure):
    _fields_ = [("unit", ctypes.c_uint32), ("waves_per_block", ctypes.c_uint32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("slot_bytes", ctypes.c_uint64), ("n_slots", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("order", ctypes.c_int32), ("pcie_gbps", ctypes.c_double),
                ("tiles", Tile * len(KINDS)), ("waves_per_cu", ctypes.c_uint32),
                ("tune_cache", ctypes.c_char_p)]


class Timing(ctypes.Structure):
    _fields_ = [("h2d_ms", ctypes.c_double), ("decode_ms", ctypes.c_double),
                ("wall_ms", ctypes.c_double), ("plain_bytes", ctypes.c_uint64),
                ("comp_bytes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Unit(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("a", ctypes.c_uint32), ("b", ctypes.c_uint32),
                ("c", ctypes.c_uint32)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("t_h2d_ms", ctypes.c_double), ("t_dec_ms", ctypes.c_double),
                ("comp_bytes", ctypes.c_uint64), ("plain_bytes", ctypes.c_uint64),
                ("n_chunks", ctypes.c_uint32), ("index", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# every symbol zf.h declares, with (restype, argtypes)
_vp, _u32, _u64, _i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32
SIGNATURES = {
    "zf_encode_opts_default": (None, [ctypes.POINTER(EncodeOpts)]),
    "zf_compress_host": (_i32, [_vp, _u64, _i32, _i32, ctypes.POINTER(EncodeOpts),
                                ctypes.POINTER(_vp)]),
    "zf_column_from_bytes": (_i32, [_vp, _u64, _i32, ctypes.POINTER(_vp)]),
    "zf_chunk_features": (_i32, [_vp, _u64, _i32, _vp]),
    "zf_column_bytes": (_vp, [_vp, ctypes.POINTER(_u64)]),
    "zf_column_plain_bytes": (_u64, [_vp]),
    "zf_column_n_elems": (_u64, [_vp]),
    "zf_column_n_chunks": (_u32, [_vp]),
    "zf_column_dtype": (_i32, [_vp]),
    "zf_column_free": (None, [_vp]),
    "zf_plan_opts_default": (None, [ctypes.POINTER(PlanOpts)]),
    "zf_plan": (_i32, [ctypes.POINTER(_vp), _u32, _i32, ctypes.POINTER(PlanOpts),
                       ctypes.POINTER(_vp)]),
    "zf_plan_free": (None, [_vp]),
    "zf_plan_image_bytes": (_u64, [_vp]),
    "zf_plan_image_offset": (_u64, [_vp, _u32]),
    "zf_plan_n_batches": (_u32, [_vp]),
    "zf_plan_batch_info": (_i32, [_vp, _u32, ctypes.POINTER(BatchInfo)]),
    "zf_johnson_order": (_i32, [_vp, _vp, _u32, _vp]),
    "zf_chunk_units": (_i32, [_vp, _u32, ctypes.POINTER(PlanOpts), _vp, _u32, ctypes.POINTER(_u32)]),
    "zf_decompress_async": (_i32, [_vp, _vp, _u64, ctypes.POINTER(_vp), _vp]),
    "zf_transfer_and_decompress": (_i32, [_vp, ctypes.POINTER(_vp), _vp,
                                          ctypes.POINTER(Timing)]),
    "zf_sync": (_i32, [_vp, _vp]),
    "zf_plan_clear_error": (None, [_vp]),
    "zf_plan_profile": (_i32, [_vp, _i32]),
    "zf_plan_kind_ms": (_i32, [_vp, _vp]),
    "zf_mlp_forward": (_i32, [_vp, _vp, _u32, _vp, _vp]),
    "zf_mlp_grad_work_bytes": (_u64, [_u32]),
    "zf_mlp_grad": (_i32, [_vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _u64, _vp]),
    "zf_mlp_grad_noalloc": (_i32, [_vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp]),
    "zf_mlp_adam": (_i32, [_vp, _vp, _vp, _vp, _u32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                           ctypes.c_float, _vp]),
    "zf_status_str": (ctypes.c_char_p, [_i32]),
    "zf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libzf.so (building it first only when no build exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        msg = lib().zf_last_error().decode(errors="replace")
        raise ZfError(rc, msg)


def dtype_of(x):
    if x.dtype == np.int32:
        return I32
    if x.dtype == np.int64:
        return I64
    if x.dtype == np.float64:
        return F64
    if x.dtype == np.uint8 and x.ndim == 1:
        return BYTES
    if x.dtype == np.uint8 and x.ndim == 2 and x.shape[1] == 16:
        return FIXED16
    raise TypeError(f"unsupported column {x.dtype} {x.shape}")


class Column:
    """A compressed column in host memory (pinned unless asked otherwise)."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle)

    @classmethod
    def compress(cls, x, codec, chunk_elems=None, chunk_codecs=None, chunk_bytes=None, seed=0,
                 threads=0, pinned=True, mlp_weights=None, fallback_device=None, fallback_margin=None):
        x = np.ascontiguousarray(x)
        o = EncodeOpts()
        lib().zf_encode_opts_default(ctypes.byref(o))
        o.pinned = 1 if pinned else 0
        o.n_threads = threads
        o.seed = seed
        keep = []
        if mlp_weights is not None:
            keep.append(mlp_weights.encode())
            o.mlp_weights = keep[-1]
        if fallback_device is not None:
            o.fallback_device = fallback_device
        if fallback_margin is not None:
            o.fallback_margin = fallback_margin
        if chunk_bytes is not None:
            o.chunk_bytes_min, o.chunk_bytes_max = chunk_bytes
        if chunk_elems is not None:
            ce = np.ascontiguousarray(chunk_elems, dtype=np.uint32)
            keep.append(ce)
            o.chunk_elems = ce.ctypes.data
            o.n_chunk_elems = ce.size
            if chunk_codecs is not None:
                cc = np.ascontiguousarray(chunk_codecs, dtype=np.uint32)
                keep.append(cc)
                o.chunk_codecs = cc.ctypes.data
        h = ctypes.c_void_p()
        _check(lib().zf_compress_host(x.ctypes.data, x.shape[0], dtype_of(x), codec,
                                      ctypes.byref(o), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_bytes(cls, buf, pinned=True):
        a = np.ascontiguousarray(np.frombuffer(bytes(buf), np.uint8) if not isinstance(buf, np.ndarray) else buf)
        h = ctypes.c_void_p()
        _check(lib().zf_column_from_bytes(a.ctypes.data, a.size, 1 if pinned else 0, ctypes.byref(h)))
        return cls(h.value)

    @property
    def handle(self):
        return self._h

    def bytes(self):
        n = ctypes.c_uint64()
        p = lib().zf_column_bytes(self._h, ctypes.byref(n))
        return np.ctypeslib.as_array((ctypes.c_uint8 * n.value).from_address(p)).copy() if n.value else np.zeros(0, np.uint8)

    def host_pointer(self):
        n = ctypes.c_uint64()
        p = lib().zf_column_bytes(self._h, ctypes.byref(n))
        return p, n.value

    @property
    def plain_bytes(self):
        return lib().zf_column_plain_bytes(self._h)

    @property
    def n_elems(self):
        return lib().zf_column_n_elems(self._h)

    @property
    def n_chunks(self):
        return lib().zf_column_n_chunks(self._h)

    @property
    def dtype(self):
        return lib().zf_column_dtype(self._h)

    def free(self):
        if self._h and self._h.value:
            lib().zf_column_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def chunk_features(x):
    """The 32 cost-model statistics of a chunk (numpy column)."""
    x = np.ascontiguousarray(x)
    out = np.zeros(32, np.float32)
    _check(lib().zf_chunk_features(x.ctypes.data, x.shape[0], dtype_of(x), out.ctypes.data))
    return out


def johnson_order(a, b):
    """The library's Johnson order of jobs with stage times a (copy), b (decode)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert a.shape == b.shape and a.ndim == 1
    order = np.zeros(a.size, np.uint32)
    _check(lib().zf_johnson_order(a.ctypes.data, b.ctypes.data, a.size, order.ctypes.data))
    return order.tolist()


def _ptr(x):
    """Device pointer of a torch tensor, or an int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _set_tiles(o, tiles):
    """tiles: {kind or group name: {"unit": u, "waves_per_block": w}} into PlanOpts o."""
    for name, shape in (tiles or {}).items():
        for kind in KIND_GROUPS.get(name, [name]):
            t = o.tiles[KINDS.index(kind)]
            t.unit = shape.get("unit", 0)
            t.waves_per_block = shape.get("waves_per_block", 0)


def chunk_units(col, chunk, tiles=None, tune_cache=None):
    """[(kind name, a, b, c)] of the wavefront units the planner cuts chunk
    `chunk` of `col` into (zf_chunk_units; host only)."""
    o = PlanOpts()
    lib().zf_plan_opts_default(ctypes.byref(o))
    _set_tiles(o, tiles)
    keep = tune_cache.encode() if tune_cache else None
    o.tune_cache = keep
    n = ctypes.c_uint32()
    _check(lib().zf_chunk_units(col.handle, chunk, ctypes.byref(o), None, 0, ctypes.byref(n)))
    arr = (Unit * max(n.value, 1))()
    _check(lib().zf_chunk_units(col.handle, chunk, ctypes.byref(o), arr, n.value, ctypes.byref(n)))
    return [(KINDS[u.kind], u.a, u.b, u.c) for u in arr[:n.value]]


class Plan:
    """Work tables, batches and device workspace for decoding `cols`."""

    def __init__(self, cols, device=0, slot_bytes=256 << 20, n_slots=2, use_graphs=True,
                 persistent=False, order=0, pcie_gbps=0.0, tiles=None, waves_per_cu=0,
                 tune_cache=None):
        """tiles: {kind or group name: {"unit": u, "waves_per_block": w}}, where a
        kind is one of KINDS and a group one of KIND_GROUPS."""
        self.cols = list(cols)
        o = PlanOpts()
        lib().zf_plan_opts_default(ctypes.byref(o))
        o.slot_bytes = slot_bytes
        o.n_slots = n_slots
        o.use_graphs = 1 if use_graphs else 0
        o.persistent = 1 if persistent else 0
        o.order = order
        o.pcie_gbps = pcie_gbps
        _set_tiles(o, tiles)
        o.waves_per_cu = waves_per_cu
        self._tune = tune_cache.encode() if tune_cache else None
        o.tune_cache = self._tune
        arr = (ctypes.c_void_p * len(self.cols))(*[c.handle.value for c in self.cols])
        h = ctypes.c_void_p()
        _check(lib().zf_plan(arr, len(self.cols), device, ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._timing = Timing()

    @property
    def image_bytes(self):
        return lib().zf_plan_image_bytes(self._h)

    def image_offset(self, c):
        return lib().zf_plan_image_offset(self._h, c)

    def profile(self, on=True):
        """Record per-kind kernel times in zf_decompress_async (zf_plan_profile)."""
        _check(lib().zf_plan_profile(self._h, 1 if on else 0))

    def kind_ms(self):
        """{kind name or "PERSISTENT": ms} of the most recent profiled decode."""
        ms = np.zeros(len(KINDS) + 1, np.float64)
        _check(lib().zf_plan_kind_ms(self._h, ms.ctypes.data))
        names = KINDS + ["PERSISTENT"]
        return {names[k]: float(ms[k]) for k in range(len(names)) if ms[k] >= 0}

    def batches(self):
        """The plan's batches in execution order (zf_plan_batch_info)."""
        out = []
        for k in range(lib().zf_plan_n_batches(self._h)):
            b = BatchInfo()
            _check(lib().zf_plan_batch_info(self._h, k, ctypes.byref(b)))
            out.append(b.as_dict())
        return out

    def _outs(self, outs):
        return (ctypes.c_void_p * len(outs))(*[_ptr(t) for t in outs])

    def decompress_async(self, d_comp, comp_bytes, outs, stream=None):
        _check(lib().zf_decompress_async(self._h, _ptr(d_comp), comp_bytes, self._outs(outs),
                                         _stream(stream)))

    def transfer_and_decompress(self, outs, stream=None, timing=True):
        t = ctypes.byref(self._timing) if timing else None
        _check(lib().zf_transfer_and_decompress(self._h, self._outs(outs), _stream(stream), t))

    def sync(self, stream=None):
        _check(lib().zf_sync(self._h, _stream(stream)))
        return self._timing.as_dict()

    def clear_error(self):
        lib().zf_plan_clear_error(self._h)

    def free(self):
        if self._h and self._h.value:
            lib().zf_plan_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def first_codec(col):
    """Codec of a column's first chunk (byte 28 of its first chunk-table
    entry), read in place; PLAIN for a column without chunks."""
    if col.n_chunks == 0:
        return PLAIN
    return ctypes.string_at(col.host_pointer()[0] + 64 + 28, 1)[0]


def chunk_table(col):
    """(n_elems, codec, schedule) of every chunk, read in place from the
    column's 32-byte chunk-table entries (bytes 24..27, 28 and 29)."""
    n = col.n_chunks
    raw = ctypes.string_at(col.host_pointer()[0] + 64, 32 * n)
    return [(int.from_bytes(raw[32 * i + 24:32 * i + 28], "little"), raw[32 * i + 28], raw[32 * i + 29])
            for i in range(n)]


def kind_of_column(col):
    """Kernel kind of a single-codec column (its first chunk's codec)."""
    codec = first_codec(col)
    dt = col.dtype
    if codec == PLAIN:
        return "PLAIN"
    if codec == LZ77:
        return "LZ77"
    if codec == F2I_BP:
        return "F2I"
    if codec == ANS:
        return "ANS"
    if codec in (SDICT_BP, SDICT_ANS, SDICT_COL, SDICT_COL_ANS):
        return "SDICT"
    if codec == DSTREE:
        return "TREE"
    if codec in (DELTA_BP, RLE_DELTA_BP, DSTRIDE_BP):
        return "RLE32" if dt == I32 else "RLE64"
    if codec == DICT_BP:
        return {I32: "DICT32", I64: "DICT64", FIXED16: "DICT128"}[dt]
    return "FOR32" if dt == I32 else "FOR64"


# ---------------------------------------------------------- torch helpers
def torch_dtype_shape(col):
    """(torch dtype, shape) of a decoded column."""
    import torch
    n = col.n_elems
    dt = col.dtype
    if dt == I32:
        return torch.int32, (n,)
    if dt == I64:
        return torch.int64, (n,)
    if dt == F64:
        return torch.float64, (n,)
    if dt == FIXED16:
        return torch.uint8, (n, 16)
    return torch.uint8, (n,)


def empty_outputs(cols, device="cuda"):
    import torch
    outs = []
    for c in cols:
        dt, shape = torch_dtype_shape(c)
        outs.append(torch.empty(shape, dtype=dt, device=device))
    return outs


def upload_image(plan, cols, device="cuda"):
    """Copy the columns' bytes into a device image laid out for `plan`."""
    import torch
    img = torch.empty(max(1, plan.image_bytes), dtype=torch.uint8, device=device)
    for i, c in enumerate(cols):
        b = torch.from_numpy(c.bytes())
        off = plan.image_offset(i)
        img[off:off + b.numel()].copy_(b)
    return img


# ------------------------------------------------------------ cost model
MLP_IN, MLP_HIDDEN, MLP_OUT, MLP_PARAMS = 32, 64, 24, 7832


def mlp_forward(params, x, y, stream=None):
    _check(lib().zf_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(y), _stream(stream)))


def mlp_grad_work_bytes(n):
    return lib().zf_mlp_grad_work_bytes(n)


MLP_STATIC_MAX_N = 16384


def mlp_grad_noalloc(params, x, k, t, grad, loss, stream=None):
    _check(lib().zf_mlp_grad_noalloc(_ptr(params), _ptr(x), _ptr(k), _ptr(t), x.shape[0], _ptr(grad),
                                     _ptr(loss), _stream(stream)))


def mlp_grad(params, x, k, t, grad, loss, work, stream=None):
    _check(lib().zf_mlp_grad(_ptr(params), _ptr(x), _ptr(k), _ptr(t), x.shape[0], _ptr(grad),
                             _ptr(loss), _ptr(work), work.numel() * work.element_size(),
                             _stream(stream)))


def mlp_adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().zf_mlp_adam(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                             _stream(stream)))
