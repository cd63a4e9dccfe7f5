"""ctypes binding of the oracle codecs in ``zfo.c``.

Test infrastructure only (see ``oracle/__init__.py``)."""
import ctypes
import os

import numpy as np

from . import build as _build

I32, I64, BYTES, FIXED16, F64 = 1, 2, 3, 4, 5
PLAIN, FOR_BP, DICT_BP, DELTA_BP, RLE_DELTA_BP, LZ77, F2I_BP, ANS, DSTRIDE_BP, SDICT_BP, SDICT_ANS = \
    1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11
SDICT_COL, SDICT_COL_ANS = 12, 13
DSTREE = 14
OK, EINVAL, EUNSUP, ECORRUPT, ENOMEM = 0, 1, 2, 3, 4
ELEM_SIZE = {I32: 4, I64: 8, BYTES: 1, FIXED16: 16, F64: 8}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"oracle {what}: status {code}")
        self.code = code


class _Info(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_uint32), ("codec", ctypes.c_uint32),
                ("n_chunks", ctypes.c_uint32), ("dict_count", ctypes.c_uint32),
                ("n_elems", ctypes.c_uint64), ("plain_bytes", ctypes.c_uint64),
                ("dict_off", ctypes.c_uint64), ("total_bytes", ctypes.c_uint64)]


class _Chunk(ctypes.Structure):
    _fields_ = [("plain_off", ctypes.c_uint64), ("comp_off", ctypes.c_uint64),
                ("plain_len", ctypes.c_uint32), ("comp_len", ctypes.c_uint32),
                ("n_elems", ctypes.c_uint32), ("codec", ctypes.c_uint32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.zfo_crc32.argtypes = [vp, u64]
        L.zfo_crc32.restype = u32
        L.zfo_encode.argtypes = [vp, u64, u32, u32, vp, u32, vp,
                                 ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(u64)]
        L.zfo_free.argtypes = [vp]
        L.zfo_inspect.argtypes = [vp, u64, ctypes.POINTER(_Info)]
        L.zfo_get_chunk.argtypes = [vp, u64, u32, ctypes.POINTER(_Chunk)]
        L.zfo_decode.argtypes = [vp, u64, vp, u64]
        L.zfo_decode_chunks.argtypes = [vp, u64, u32, u32, vp, u64]
        L.zfo_decode_stream.argtypes = [u32, u32, vp, u64, u32, vp, u32, vp]
        _lib = L
    return _lib


def _buf(a):
    a = np.ascontiguousarray(a)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _as_bytes(blob):
    return np.frombuffer(bytes(blob), dtype=np.uint8) if not isinstance(blob, np.ndarray) else blob


def crc32(data):
    a, p = _buf(np.frombuffer(bytes(data), dtype=np.uint8))
    return lib().zfo_crc32(p, a.size)


def dtype_of(x):
    """zf dtype code of a numpy column."""
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


def encode(x, codec, chunk_elems=None, codecs=None):
    """Encode numpy column x -> column blob (np.uint8).  chunk_elems: list of
    per-chunk element counts (default: one chunk)."""
    x = np.ascontiguousarray(x)
    dt = dtype_of(x)
    n = x.shape[0]
    if chunk_elems is None:
        chunk_elems = [n] if n else []
    ce, cep = _buf(np.asarray(chunk_elems, dtype=np.uint32))
    cc, ccp = (None, None)
    if codecs is not None:
        cc, ccp = _buf(np.asarray(codecs, dtype=np.uint32))
    _, xp = _buf(x)
    out = ctypes.c_void_p()
    olen = ctypes.c_uint64()
    rc = lib().zfo_encode(xp, n, dt, codec, cep, ce.size, ccp, ctypes.byref(out), ctypes.byref(olen))
    if rc:
        raise OracleError(rc, "encode")
    try:
        res = np.frombuffer(ctypes.string_at(out, olen.value), dtype=np.uint8).copy()
    finally:
        lib().zfo_free(out)
    return res


def inspect(blob):
    b, bp = _buf(_as_bytes(blob))
    info = _Info()
    rc = lib().zfo_inspect(bp, b.size, ctypes.byref(info))
    if rc:
        raise OracleError(rc, "inspect")
    return {k: getattr(info, k) for k, _ in _Info._fields_}


def chunks(blob):
    b, bp = _buf(_as_bytes(blob))
    info = inspect(b)
    out = []
    for i in range(info["n_chunks"]):
        c = _Chunk()
        lib().zfo_get_chunk(bp, b.size, i, ctypes.byref(c))
        out.append({k: getattr(c, k) for k, _ in _Chunk._fields_})
    return out


def _shape_out(nbytes, dtype):
    es = ELEM_SIZE[dtype]
    if dtype == I32:
        return np.empty(nbytes // 4, dtype=np.int32)
    if dtype == I64:
        return np.empty(nbytes // 8, dtype=np.int64)
    if dtype == F64:
        return np.empty(nbytes // 8, dtype=np.float64)
    if dtype == FIXED16:
        return np.empty((nbytes // es, 16), dtype=np.uint8)
    return np.empty(nbytes, dtype=np.uint8)


def decode(blob):
    b, bp = _buf(_as_bytes(blob))
    info = inspect(b)
    out = _shape_out(info["plain_bytes"], info["dtype"])
    _, op = _buf(out)
    rc = lib().zfo_decode(bp, b.size, op, info["plain_bytes"])
    if rc:
        raise OracleError(rc, "decode")
    return out


def decode_chunks(blob, first, count):
    b, bp = _buf(_as_bytes(blob))
    info = inspect(b)
    cs = chunks(b)[first:first + count]
    nbytes = sum(c["plain_len"] for c in cs)
    out = _shape_out(nbytes, info["dtype"])
    _, op = _buf(out)
    rc = lib().zfo_decode_chunks(bp, b.size, first, count, op, nbytes)
    if rc:
        raise OracleError(rc, "decode_chunks")
    return out


def decode_chunks_into(blob, first, count, out, byte_off, nbytes):
    """Decode chunks [first, first + count) of a column blob (contiguous
    np.uint8) into the bytes of numpy array `out` from byte `byte_off`;
    nbytes = the chunks' plain bytes.  For running many chunk ranges at once
    on host threads (the C call holds no Python lock)."""
    assert blob.dtype == np.uint8 and blob.flags.c_contiguous and out.flags.c_contiguous
    assert 0 <= byte_off and byte_off + nbytes <= out.nbytes
    rc = lib().zfo_decode_chunks(ctypes.c_void_p(blob.ctypes.data), blob.size, first, count,
                                 ctypes.c_void_p(out.ctypes.data + byte_off), nbytes)
    if rc:
        raise OracleError(rc, "decode_chunks")


def decode_stream(codec, dtype, stream, n_elems, dictionary=None, dict_count=0):
    """Decode one raw codec stream (no container).  Returns (status, output)."""
    s, sp = _buf(_as_bytes(stream) if len(stream) else np.zeros(1, np.uint8))
    slen = len(stream)
    out = _shape_out(n_elems * ELEM_SIZE[dtype], dtype)
    _, op = _buf(out)
    dp = None
    if dictionary is not None:
        d, dp = _buf(_as_bytes(dictionary))
    rc = lib().zfo_decode_stream(codec, dtype, sp, slen, n_elems, dp, dict_count, op)
    return rc, out
