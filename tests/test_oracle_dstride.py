"""DeltaStride in the oracle, pinned to things other than itself: streams
derived by hand (tests/golden/dstride_examples.json), the properties that
define a left-to-right maximal split into progressions, brute-force round
trips over every short sequence of a small alphabet, the closed-form stream
size of evenly spaced key blocks, and rejection of corrupt streams."""
import itertools
import struct

import numpy as np

import oracle.zfo as z

DT = {"i32": np.int32, "i64": np.int64}


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def runs_of(stream):
    """(count, stride) of every run, read from the stream's fields."""
    nr, ng, roff, _ = struct.unpack_from("<4I", stream, 0)
    lens = struct.unpack_from(f"<{nr}I", stream, roff)
    strides = []
    for g in range(ng):
        _, poff, widths, _, _, dmin = struct.unpack_from("<4Iqq", stream, 16 + 32 * g)
        wg, wd = widths & 0xFF, (widths >> 8) & 0xFF
        cnt = min(64, nr - 64 * g)
        gw = ((cnt - 1) * wg + 31) // 32
        bits = int.from_bytes(stream[poff + 8 + 4 * gw:poff + 8 + 4 * gw + 4 * ((cnt * wd + 31) // 32)],
                              "little")
        strides += [dmin + ((bits >> (j * wd)) & ((1 << wd) - 1)) for j in range(cnt)]
    return list(lens), strides


def test_hand_derived_streams(golden):
    for e in golden("dstride_examples.json")["examples"]:
        x = np.array(e["values"], DT[e["dtype"]])
        s = stream_of(z.encode(x, z.DSTRIDE_BP))
        r = e["record"]
        nr = len(e["runs"])
        assert struct.unpack_from("<4I", s, 0) == (nr, 1, e["runs_off"], 0), e["name"]
        assert struct.unpack_from("<4Iqq", s, 16) == (r["out_off"], r["poff"], r["widths"], 0,
                                                      r["base"], r["dmin"]), e["name"]
        assert struct.unpack_from("<q", s, r["poff"])[0] == e["gmin"]
        words = list(struct.unpack_from(f"<{(len(s) - r['poff'] - 8 - 4 * nr) // 4}I", s, r["poff"] + 8))
        assert words[:len(e.get("gap_words", []))] == e.get("gap_words", [])
        assert words[len(e.get("gap_words", [])):len(e.get("gap_words", [])) + len(e.get("stride_words", []))] \
            == e.get("stride_words", [])
        assert list(struct.unpack_from(f"<{nr}I", s, e["runs_off"])) == [c for _, _, c in e["runs"]]
        assert len(s) == e["comp_len"]
        rc, out = z.decode_stream(z.DSTRIDE_BP, z.I32 if e["dtype"] == "i32" else z.I64, s, len(x))
        assert rc == z.OK and np.array_equal(out.view(x.dtype), x)


def _check_split(x, bits):
    """A left-to-right maximal split: the counts cover x; inside a run the
    step is the run's stride; a run of one element is the last element; a
    run never continues into the next one."""
    lens, strides = runs_of(stream_of(z.encode(x, z.DSTRIDE_BP)))
    m = (1 << bits) - 1
    assert sum(lens) == len(x)
    i = 0
    for j, (r, d) in enumerate(zip(lens, strides)):
        assert r >= 1
        if r == 1:
            assert i == len(x) - 1 and d == 0
        for t in range(1, r):
            assert (int(x[i + t]) - int(x[i + t - 1])) & m == d & m
        if r >= 2 and i + r < len(x):
            assert (int(x[i + r]) - int(x[i + r - 1])) & m != d & m
        i += r


def test_brute_force_short_sequences():
    alphabet = [-2, -1, 0, 1, 2]
    for n in range(1, 6):
        for t in itertools.product(alphabet, repeat=n):
            x = np.array(t, np.int32)
            blob = z.encode(x, z.DSTRIDE_BP)
            assert np.array_equal(z.decode(blob), x), t
            _check_split(x, 32)


def test_random_and_wrapping_round_trips():
    r = np.random.default_rng(7)
    for dt, bits in ((np.int32, 32), (np.int64, 64)):
        info = np.iinfo(dt)
        for trial in range(40):
            n = int(r.integers(1, 3000))
            kind = trial % 4
            if kind == 0:    # nearly increasing keys
                x = np.cumsum(r.integers(0, 3, n)).astype(dt)
            elif kind == 1:  # random values (runs of two)
                x = r.integers(info.min, info.max, n, dtype=dt, endpoint=True)
            elif kind == 2:  # progressions that wrap
                x = (np.arange(n, dtype=np.uint64) * np.uint64(r.integers(1, 1 << 40)) +
                     np.uint64(info.max - 5)).astype(np.dtype(dt).newbyteorder("=")) if bits == 64 else \
                    (np.arange(n, dtype=np.int64) * int(r.integers(1, 1 << 20)) + info.max - 5).astype(dt)
            else:            # blocks of consecutive keys with random jumps
                x = np.cumsum(np.where(r.random(n) < 0.1, r.integers(2, 1000, n), 1)).astype(dt)
            blob = z.encode(x, z.DSTRIDE_BP, chunk_elems=[n])
            assert np.array_equal(z.decode(blob), x)
            if n < 400:
                _check_split(x, bits)


def test_evenly_spaced_key_blocks_have_a_closed_form_size():
    # blocks of 8 consecutive keys every 32: one run per block, every gap 24
    # and every stride 1, so both widths are 0 and a group costs its record
    # and the 8-byte gmin.
    for nb in (1, 63, 64, 65, 1000):
        x = (np.arange(nb * 8) // 8 * 32 + np.arange(nb * 8) % 8 + 1).astype(np.int32)
        s = stream_of(z.encode(x, z.DSTRIDE_BP, chunk_elems=[len(x)]))
        ng = (nb + 63) // 64
        end = 16 + 32 * ng
        for _ in range(ng):
            end = (end + 7) // 8 * 8 + 8
        assert len(s) == (end + 15) // 16 * 16 + 4 * nb
        lens, strides = runs_of(s)
        assert lens == [8] * nb and strides == [1] * nb


def test_corrupt_streams_are_rejected(golden):
    e = golden("dstride_examples.json")["examples"][0]
    x = np.array(e["values"], np.int32)
    good = bytearray(stream_of(z.encode(x, z.DSTRIDE_BP)))
    assert z.decode_stream(z.DSTRIDE_BP, z.I32, bytes(good), len(x))[0] == z.OK

    def bad(mut):
        s = bytearray(good)
        mut(s)
        return z.decode_stream(z.DSTRIDE_BP, z.I32, bytes(s), len(x))[0]
    assert bad(lambda s: struct.pack_into("<I", s, 64, 0)) == z.ECORRUPT          # zero count
    assert bad(lambda s: struct.pack_into("<I", s, 64, 9)) == z.ECORRUPT          # counts overrun n
    assert bad(lambda s: struct.pack_into("<I", s, 16 + 8, 33)) == z.ECORRUPT     # width > 32
    assert bad(lambda s: struct.pack_into("<I", s, 16 + 4, 44)) == z.ECORRUPT     # poff not 8-aligned
    assert bad(lambda s: struct.pack_into("<I", s, 16, 1)) == z.ECORRUPT          # out_off != 0
    assert bad(lambda s: struct.pack_into("<I", s, 4, 2)) == z.ECORRUPT           # group count
    assert z.decode_stream(z.DSTRIDE_BP, z.I32, bytes(good), len(x) + 1)[0] == z.ECORRUPT
