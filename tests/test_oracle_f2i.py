"""Float2Int + bit-packing in the oracle, pinned to things other than itself:
hand-computed streams, a pure-Python reader of the stream (struct, Python
floats and integers) that re-derives every value and re-runs the choice of
exponent by brute force, bit-exact round trips over special values, and
rejection of corrupt streams."""
import math
import struct

import numpy as np

import oracle.zfo as z

B = 2048


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def bits(v):
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def from_bits(b):
    return struct.unpack("<d", struct.pack("<Q", b))[0]


def py_digits(b, e):
    """The integer d with bits(float(d) / 10.0**e) == b, if any (Python's own
    IEEE arithmetic; 10.0**e is exact for e <= 18)."""
    v = from_bits(b)
    m = v * (10.0 ** e)
    if not abs(m) < 2.0 ** 62:
        return None
    k = int(round(m))  # Python rounds half to even, as nearbyint does
    if bits(float(k) / (10.0 ** e)) != b:
        return None
    return k


def py_read(stream, n):
    """Decode one F2I_BP stream with Python only; also returns per-block
    (e, ref, w, nx)."""
    nb = (n + B - 1) // B
    out, meta = [], []
    for b in range(nb):
        nv = min(B, n - b * B)
        ref, w, poff, xoff, nx, e, pad = struct.unpack_from("<qIIIHBB", stream, 32 * b)
        words = stream[poff:poff + 4 * ((nv * w + 31) // 32)]
        big = int.from_bytes(words, "little")
        vals = []
        for j in range(nv):
            f = (big >> (j * w)) & ((1 << w) - 1)
            k = (ref + f + 2 ** 63) % 2 ** 64 - 2 ** 63  # int64 wrap
            vals.append(bits(float(k) / (10.0 ** e)))
        for i in range(nx):
            j, zero, raw = struct.unpack_from("<IIQ", stream, xoff + 16 * i)
            vals[j] = raw
        out += vals
        meta.append((e, ref, w, nx))
    return np.array(out, dtype=np.uint64).view(np.float64), meta


def py_best_e(block_bits):
    """Brute force over e of the cost nv*w + 128*nx (ties to the smaller e)."""
    best = None
    for e in range(19):
        ds = [py_digits(b, e) for b in block_bits]
        ok = [d for d in ds if d is not None]
        w = (max(ok) - min(ok)).bit_length() if ok else 0
        cost = len(ds) * w + 128 * (len(ds) - len(ok))
        if best is None or cost < best[0]:
            best = (cost, e, min(ok) if ok else 0, w, len(ds) - len(ok))
    return best[1:]


def test_golden_streams(golden):
    gd = golden("f2i_examples.json")
    for ex in gd["examples"]:
        x = np.array([float(v) for v in ex["values"]], dtype=np.float64)
        blob = z.encode(x, z.F2I_BP)
        assert stream_of(blob).hex() == ex["stream_hex"]
        rc, out = z.decode_stream(z.F2I_BP, z.F64, bytes.fromhex(ex["stream_hex"]), len(x))
        assert rc == z.OK and np.array_equal(out.view(np.uint64), x.view(np.uint64))


SPECIALS = [0.0, -0.0, float("inf"), float("-inf"), float("nan"), 5e-324, -5e-324, 2.2250738585072014e-308,
            1.7976931348623157e308, 0.1, 0.2, 0.30000000000000004, 1e18, 4.611686018427388e18,
            9.2e18, -9.2e18, 123456789.123, 1 / 3, math.pi, 2.0 ** 53, 2.0 ** 53 + 2]


def columns():
    r = np.random.default_rng(7)
    yield np.array(SPECIALS * 3, dtype=np.float64)
    for digits in (0, 1, 2, 4, 7, 12):
        # decimals with `digits` places, as parsed from text
        ints = r.integers(-10 ** 9, 10 ** 9, size=5000)
        yield np.array([float(f"{i / 10 ** digits:.{digits}f}") for i in ints], dtype=np.float64)
    yield np.round(r.uniform(900, 105000, size=4500), 2)           # prices
    yield np.round(r.integers(0, 11, size=3000) / 100, 2)           # discounts 0.00..0.10
    yield r.random(2100)                                            # full-precision doubles
    yield r.integers(0, 2 ** 64, size=2100, dtype=np.uint64).view(np.float64)  # any bits
    mix = np.round(r.uniform(-50, 50, size=6000), 3)
    mix[r.integers(0, 6000, size=40)] = np.array(SPECIALS * 2)[:40]
    yield mix


def test_round_trip_is_bit_exact_and_python_reader_agrees():
    for x in columns():
        n = len(x)
        ce = [n] if n <= 5000 else [1234, n - 1234]
        blob = z.encode(x, z.F2I_BP, ce)
        y = z.decode(blob)
        assert np.array_equal(y.view(np.uint64), x.view(np.uint64))
        at = 0
        for i, m in enumerate(ce):
            py, meta = py_read(stream_of(blob, i), m)
            assert np.array_equal(py.view(np.uint64), x[at:at + m].view(np.uint64))
            # the encoder's exponent, reference, width and exception count are
            # the brute-force optimum
            for b, (e, ref, w, nx) in enumerate(meta):
                blk = [int(v) for v in x[at + b * B:at + min(m, (b + 1) * B)].view(np.uint64)]
                assert (e, ref, w, nx) == py_best_e(blk)
            at += m


def test_brute_force_tiny_blocks():
    """Every block of two values drawn from a small set of decimals and
    specials round-trips and matches the Python reader."""
    pool = [0.0, -0.0, 0.5, 1.25, -3.0, 0.1, 1e-5, 7.0e15, float("nan"), float("inf")]
    for a in pool:
        for b in pool:
            x = np.array([a, b], dtype=np.float64)
            blob = z.encode(x, z.F2I_BP)
            y = z.decode(blob)
            assert np.array_equal(y.view(np.uint64), x.view(np.uint64))
            py, meta = py_read(stream_of(blob), 2)
            assert np.array_equal(py.view(np.uint64), x.view(np.uint64))
            assert meta[0] == py_best_e([int(v) for v in x.view(np.uint64)])


def test_corrupt_streams_rejected():
    x = np.round(np.linspace(-5, 5, 3000), 2)
    s = bytearray(stream_of(z.encode(x, z.F2I_BP)))
    n = len(x)
    assert z.decode_stream(z.F2I_BP, z.F64, bytes(s), n)[0] == z.OK
    for off, val in ((22, 19), (8, 65), (12, 33), (16, 40)):   # e, w, poff, xoff
        t = bytearray(s)
        t[off:off + 1] = bytes([val])
        assert z.decode_stream(z.F2I_BP, z.F64, bytes(t), n)[0] == z.ECORRUPT
    # exception records out of order
    y = np.array([0.5, -0.0, float("nan"), 1.5], dtype=np.float64)
    s2 = bytearray(stream_of(z.encode(y, z.F2I_BP)))
    _, meta = py_read(bytes(s2), 4)
    xoff = struct.unpack_from("<I", s2, 16)[0]
    s2[xoff:xoff + 4], s2[xoff + 16:xoff + 20] = s2[xoff + 16:xoff + 20], s2[xoff:xoff + 4]
    assert z.decode_stream(z.F2I_BP, z.F64, bytes(s2), 4)[0] == z.ECORRUPT
