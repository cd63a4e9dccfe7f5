"""The oracle pinned to things other than itself: hand-computed streams,
independent re-derivations of what each stream must hold (Python integers,
numpy library routines), brute force on tiny inputs, and extremes."""
import itertools

import numpy as np
import pytest

import oracle.zfo as z
from paper_2602_08190_amd import datagen as g


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def _vals(x, dtype):
    return np.array(x, dtype=np.int32 if dtype == "i32" else np.int64)


# --------------------------------------------------------------- FOR + BP
def test_for_bp_golden(golden):
    gd = golden("for_bp_examples.json")
    for ex in gd["examples"]:
        x = _vals(ex["values"], ex["dtype"])
        blob = z.encode(x, z.FOR_BP)
        assert stream_of(blob).hex() == ex["stream_hex"], ex["name"]
        rc, out = z.decode_stream(z.FOR_BP, z.I32, bytes.fromhex(ex["stream_hex"]), len(x))
        assert rc == z.OK and (out == x).all()
    for ex in gd["decode_only"]:
        rc, out = z.decode_stream(z.FOR_BP, z.I32, bytes.fromhex(ex["stream_hex"]), ex["n"])
        assert rc == z.OK and list(out) == ex["values"], ex["name"]


def _check_for_stream(s, x, bits):
    """Re-derive every field of a FOR_BP stream with Python integers: the
    reference is the block minimum, the width is bitlen(max - min), and field
    j sits at bits [j*w, j*w+w) of the little-endian payload."""
    n = len(x)
    nb = (n + 2047) // 2048
    for b in range(nb):
        blk = [int(v) for v in x[b * 2048:(b + 1) * 2048]]
        ref = int.from_bytes(s[16 * b:16 * b + 8], "little", signed=True)
        w = int.from_bytes(s[16 * b + 8:16 * b + 12], "little")
        poff = int.from_bytes(s[16 * b + 12:16 * b + 16], "little")
        assert ref == min(blk)
        assert w == (max(blk) - min(blk)).bit_length()
        assert poff % 16 == 0
        payload = int.from_bytes(s[poff:poff + 4 * ((len(blk) * w + 31) // 32)], "little")
        for j, v in enumerate(blk):
            assert (payload >> (j * w)) & ((1 << w) - 1) == v - ref


def test_for_bp_fields_rederived():
    for dt, lo, hi in [(np.int32, -2**31, 2**31), (np.int64, -2**63, 2**63)]:
        r = g.rng(5)
        for n, span in [(1, 1), (7, 9), (2048, 4096), (2049, 1 << 20), (5000, 3)]:
            base = int(r.integers(lo // 2, hi // 2))
            x = (base + r.integers(0, span, size=n)).astype(dt)
            s = stream_of(z.encode(x, z.FOR_BP))
            _check_for_stream(s, x, 32 if dt == np.int32 else 64)
            assert (z.decode(z.encode(x, z.FOR_BP)) == x).all()


def test_for_bp_brute_force_tiny():
    for n in range(1, 5):
        for vals in itertools.product(range(8), repeat=n):
            x = np.array(vals, dtype=np.int32)
            b = z.encode(x, z.FOR_BP)
            assert (z.decode(b) == x).all()
            _check_for_stream(stream_of(b), x, 32)


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_for_bp_extremes(dt):
    info = np.iinfo(dt)
    bits = info.bits
    cases = [
        [5, 5, 5],                              # w = 0
        [0, (1 << 31) - 1],                     # w = 31
        [info.min, info.max],                   # w = bits
        [info.min, info.min, info.min + 1],
        [info.max, info.max - 1],
    ]
    if bits == 64:
        cases.append([0, (1 << 63) - 1])        # w = 63
    for c in cases:
        x = np.array(c, dtype=dt)
        s = stream_of(z.encode(x, z.FOR_BP))
        w = int.from_bytes(s[8:12], "little")
        assert w == (int(max(c)) - int(min(c))).bit_length()
        assert (z.decode(z.encode(x, z.FOR_BP)) == x).all()


def test_for_bp_chunking_and_config1_roundtrip():
    x = g.for_bp_column()
    b = z.encode(x, z.FOR_BP, [1 << 20])
    s = stream_of(b)
    # uniform draws over a 4096-value range give w = 12 in every block
    assert all(int.from_bytes(s[16 * k + 8:16 * k + 12], "little") == 12 for k in range(512))
    assert (z.decode(b) == x).all()
    b2 = z.encode(x, z.FOR_BP, [1000, 300000, (1 << 20) - 301000])
    assert (z.decode(b2) == x).all()
    assert (z.decode_chunks(b2, 1, 1) == x[1000:301000]).all()


# ------------------------------------------------------------ dictionary
def test_dict_golden(golden):
    gd = golden("dict_bp_example.json")
    x = np.zeros((4, 16), np.uint8)
    for i, w in enumerate(gd["values"]):
        x[i, :len(w)] = np.frombuffer(w.encode(), np.uint8)
    b = z.encode(x, z.DICT_BP)
    info = z.inspect(b)
    assert info["dict_count"] == 3
    d = b[info["dict_off"]:info["dict_off"] + 48].reshape(3, 16)
    assert [bytes(r).rstrip(b"\0").decode() for r in d] == gd["dictionary"]
    assert stream_of(b).hex() == gd["stream_hex"]
    assert (z.decode(b) == x).all()


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_dict_matches_numpy_unique(dt):
    r = g.rng(11)
    vals = r.integers(-2**30, 2**30, size=300).astype(dt)
    x = vals[r.integers(0, 300, size=20000)]
    b = z.encode(x, z.DICT_BP, [7000, 13000])
    info = z.inspect(b)
    uniq = np.unique(x)
    d = np.frombuffer(bytes(b[info["dict_off"]:info["dict_off"] + uniq.nbytes]), dtype=dt)
    assert (d == uniq).all()
    # the code stream is the FOR_BP stream of the dictionary indices
    codes = np.searchsorted(uniq, x).astype(np.int32)
    assert stream_of(b, 0) == stream_of(z.encode(codes[:7000], z.FOR_BP))
    assert (z.decode(b) == x).all()


def test_dict_fixed16_roundtrip():
    x = g.fixed16_column(10000, 25, 3)
    b = z.encode(x, z.DICT_BP, [2048, 7952])
    assert z.inspect(b)["dict_count"] == len({bytes(r) for r in x})
    assert (z.decode(b) == x).all()


def test_dict_code_out_of_range_is_corrupt():
    gd_stream = bytes.fromhex("00000000000000000200000010000000" + "62000000")
    dic = np.zeros((2, 16), np.uint8)     # only 2 entries, but code 2 is used
    rc, _ = z.decode_stream(z.DICT_BP, z.FIXED16, gd_stream, 4, dic, 2)
    assert rc == z.ECORRUPT
    dic3 = np.zeros((3, 16), np.uint8)
    rc, _ = z.decode_stream(z.DICT_BP, z.FIXED16, gd_stream, 4, dic3, 3)
    assert rc == z.OK


# ----------------------------------------------------------- RLE + delta
def test_rle_golden(golden):
    for ex in golden("rle_examples.json")["examples"]:
        x = np.array(ex["values"], np.int32)
        b = z.encode(x, z.RLE_DELTA_BP)
        assert stream_of(b).hex() == ex["stream_hex"], ex["name"]
        rc, out = z.decode_stream(z.RLE_DELTA_BP, z.I32, bytes.fromhex(ex["stream_hex"]), len(x))
        assert rc == z.OK and list(out) == ex["values"]
        # run starts = exclusive prefix sum of the counts
        assert list(np.concatenate([[0], np.cumsum(ex["run_lengths"])[:-1]])) == ex["run_starts"]


def _runs_numpy(x):
    """Maximal runs via numpy: boundaries where neighbours differ."""
    edge = np.flatnonzero(np.diff(x)) + 1
    starts = np.concatenate([[0], edge])
    lens = np.diff(np.concatenate([starts, [len(x)]]))
    return x[starts], lens


def _check_rle_stream(s, x, bits, unit_runs=False):
    """Re-derive an RLE_DELTA_BP stream with Python integers."""
    M = (1 << bits) - 1
    vals, lens = (x, np.ones(len(x), np.int64)) if unit_runs else _runs_numpy(x)
    nr, ng, roff = (int.from_bytes(s[k:k + 4], "little") for k in (0, 4, 8))
    assert nr == len(vals) and ng == (nr + 63) // 64
    if unit_runs:
        assert roff == 0
    else:
        runs = np.frombuffer(s[roff:roff + 4 * nr], np.uint32)
        assert (runs == lens).all()
    start = 0
    for gi in range(ng):
        rec = s[16 + 32 * gi:48 + 32 * gi]
        out_off, w, doff = (int.from_bytes(rec[k:k + 4], "little") for k in (0, 4, 8))
        base = int.from_bytes(rec[16:24], "little", signed=True)
        dmin = int.from_bytes(rec[24:32], "little", signed=True)
        gv = [int(v) for v in vals[64 * gi:64 * gi + 64]]
        assert out_off == start and base == gv[0]
        nf = len(gv) - 1
        payload = int.from_bytes(s[doff:doff + 4 * ((nf * w + 31) // 32)], "little")
        v = base & M
        for j in range(1, len(gv)):
            v = (v + dmin + ((payload >> ((j - 1) * w)) & ((1 << w) - 1))) & M
            assert v == gv[j] & M
        start += int(lens[64 * gi:64 * gi + 64].sum())


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_rle_rederived_and_roundtrip(dt):
    bits = np.iinfo(dt).bits
    for seed, mean in [(1, 8), (2, 1.5), (3, 300)]:
        x = g.sorted_runs_column(30000, mean, seed, dtype=dt)
        b = z.encode(x, z.RLE_DELTA_BP, [16384, 30000 - 16384])
        assert (z.decode(b) == x).all()
        _check_rle_stream(stream_of(b, 0), x[:16384], bits)
        _check_rle_stream(stream_of(b, 1), x[16384:], bits)
    info = np.iinfo(dt)
    x = np.array([info.min, info.max, info.min, 0, 0, info.max, -1, -1], dt)
    b = z.encode(x, z.RLE_DELTA_BP)
    assert (z.decode(b) == x).all()
    _check_rle_stream(stream_of(b), x, bits)


@pytest.mark.parametrize("dt", [np.int32, np.int64])
def test_delta_bp_rederived(dt):
    r = g.rng(4)
    x = np.cumsum(r.integers(-50, 100, size=5000)).astype(dt)
    b = z.encode(x, z.DELTA_BP, [1000, 4000])
    assert (z.decode(b) == x).all()
    _check_rle_stream(stream_of(b, 1), x[1000:], np.iinfo(dt).bits, unit_runs=True)


def test_rle_brute_force_tiny():
    for n in range(1, 9):
        for vals in itertools.combinations_with_replacement(range(4), n):
            x = np.array(vals, np.int32)  # every non-decreasing sequence over [0,4)
            b = z.encode(x, z.RLE_DELTA_BP)
            assert (z.decode(b) == x).all()
            _check_rle_stream(stream_of(b), x, 32)


@pytest.mark.parametrize("kind,kw", [("even", dict(x=2)), ("even", dict(x=7)),
                                     ("random", dict(lo=1, hi=64)), ("outlier", dict(big=1024)),
                                     ("mixed", {})])
def test_rle_run_families(kind, kw):
    runs = g.runs_family(kind, 3000, 9, **kw)
    x = g.column_from_runs(runs, 10)
    b = z.encode(x, z.RLE_DELTA_BP)
    assert (z.decode(b) == x).all()
    _check_rle_stream(stream_of(b), x, 32)


def _rle_stream(runs, vals, base_bad=False):
    # a one-group stream assembled field by field
    import struct
    nr = len(runs)
    d = [(vals[j] - vals[j - 1]) for j in range(1, nr)]
    dmin = min(d) if d else 0
    f = [v - dmin for v in d]
    w = max(f).bit_length() if f else 0
    payload = sum(v << (j * w) for j, v in enumerate(f))
    nw = (len(f) * w + 31) // 32
    doff = 48
    roff = (doff + 4 * nw + 15) // 16 * 16
    s = struct.pack("<IIII", nr, 1, roff, 0) + struct.pack("<IIIIqq", 0, w, doff, 0, vals[0], dmin)
    s += payload.to_bytes(4 * nw, "little") + bytes(roff - doff - 4 * nw)
    s += struct.pack(f"<{nr}I", *runs)
    return s


def test_rle_corrupt_streams():
    good = _rle_stream([2, 3], [4, 9])
    rc, out = z.decode_stream(z.RLE_DELTA_BP, z.I32, good, 5)
    assert rc == z.OK and list(out) == [4, 4, 9, 9, 9]
    assert z.decode_stream(z.RLE_DELTA_BP, z.I32, _rle_stream([2, 0, 3], [4, 5, 9]), 5)[0] == z.ECORRUPT
    assert z.decode_stream(z.RLE_DELTA_BP, z.I32, good, 6)[0] == z.ECORRUPT   # sum < n
    assert z.decode_stream(z.RLE_DELTA_BP, z.I32, good, 4)[0] == z.ECORRUPT   # sum > n
    assert z.decode_stream(z.RLE_DELTA_BP, z.I32, good[:-1], 5)[0] == z.ECORRUPT


# ------------------------------------------------------------------ LZ77
def test_lz77_golden(golden):
    for ex in golden("lz77_examples.json")["examples"]:
        x = np.frombuffer(ex["plain"].encode(), np.uint8)
        b = z.encode(x, z.LZ77)
        assert stream_of(b).hex() == ex["stream_hex"], ex["name"]
        rc, out = z.decode_stream(z.LZ77, z.BYTES, bytes.fromhex(ex["stream_hex"]), len(x))
        assert rc == z.OK and bytes(out) == ex["plain"].encode()


def test_lz77_brute_force_ab():
    for n in range(1, 13):
        for t in itertools.product(b"ab", repeat=n):
            x = np.frombuffer(bytes(t), np.uint8)
            assert bytes(z.decode(z.encode(x, z.LZ77))) == bytes(t)


def test_lz77_text_roundtrip_and_ratio():
    x = g.text_column(1 << 20, seed=2)
    b = z.encode(x, z.LZ77, [65536] * 16)
    assert (z.decode(b) == x).all()
    ratio = x.size / b.size
    assert 1.8 < ratio < 4.0


def test_lz77_other_dtypes():
    x = g.sorted_runs_column(40000, 8, 1)
    b = z.encode(x, z.LZ77, [16384, 16384, 40000 - 32768])
    assert (z.decode(b) == x).all()


def _lz_stream(seqs, lits, plain_len):
    import struct
    offs, ext, tags = [], [], []
    for ll, ml, off in seqs:
        lc = ll if ll < 7 else 7
        if ll >= 7:
            ext.append(ll - 7)
        if ml == 0:
            mc = 0
        elif ml <= 33:
            mc = ml - 3
        else:
            mc = 31
            ext.append(ml - 34)
        tags.append(lc | (mc << 3))
        offs.append(off)
    return (struct.pack("<IIII", len(seqs), len(lits), len(ext), plain_len) +
            struct.pack(f"<{len(offs)}H", *offs) + struct.pack(f"<{len(ext)}H", *ext) +
            bytes(tags) + bytes(lits))


def test_lz77_corrupt_streams():
    ok = _lz_stream([(3, 9, 3), (1, 0, 0)], b"abcX", 13)
    rc, out = z.decode_stream(z.LZ77, z.BYTES, ok, 13)
    assert rc == z.OK and bytes(out) == b"abcabcabcabcX"
    bad = [
        _lz_stream([(3, 9, 0), (1, 0, 0)], b"abcX", 13),   # offset 0 with a match
        _lz_stream([(3, 9, 4), (1, 0, 0)], b"abcX", 13),   # offset beyond output
        _lz_stream([(3, 9, 3), (1, 0, 5)], b"abcX", 13),   # offset without a match
        _lz_stream([(3, 10, 3), (1, 0, 0)], b"abcX", 13),  # overruns the chunk
        _lz_stream([(3, 9, 3)], b"abc", 13),               # ends short
    ]
    for s in bad:
        assert z.decode_stream(z.LZ77, z.BYTES, s, 13)[0] == z.ECORRUPT
    assert z.decode_stream(z.LZ77, z.BYTES, ok + b"\0", 13)[0] == z.ECORRUPT  # trailing byte


# -------------------------------------------------------------- container
def test_container_header_bit_flips_rejected():
    x = g.for_bp_column(5000, 1)
    b = z.encode(x, z.FOR_BP, [2048, 2952])
    z.inspect(b)
    table_end = 64 + 32 * 2
    for byte in range(table_end):
        for bit in range(8):
            c = b.copy()
            c[byte] ^= 1 << bit
            with pytest.raises(z.OracleError):
                z.inspect(c)


def test_container_crc_known_value():
    # the standard CRC-32 check value of the ASCII digits 1..9
    assert z.crc32(b"123456789") == 0xCBF43926


def test_container_mixed_codecs_and_plain():
    x = g.sorted_runs_column(10000, 8, 1)
    b = z.encode(x, 0, [2048, 4096, 3856], codecs=[z.PLAIN, z.RLE_DELTA_BP, z.LZ77])
    assert z.inspect(b)["codec"] == 0
    assert (z.decode(b) == x).all()


def test_empty_column():
    x = np.zeros(0, np.int32)
    b = z.encode(x, z.FOR_BP, [])
    info = z.inspect(b)
    assert info["n_chunks"] == 0 and info["plain_bytes"] == 0
    assert z.decode(b).size == 0
