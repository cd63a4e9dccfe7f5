"""The order-key tree DeltaStride | [Delta | RLE | [BP, BP], BP] in the oracle,
pinned to things other than itself: hand-derived streams, every part of
generated streams read back by an independent reader and checked against a
numpy derivation of what each stage must hold (the stride, the runs, the
deltas of the starts and their runs), brute-force round trips of every short
sequence over a small alphabet, the closed-form size of evenly spaced key
blocks, and rejection of corrupt streams."""
import itertools
import struct

import numpy as np

import oracle.zfo as z
from paper_2602_08190_amd import datagen as g


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


DT = {"i32": np.int32, "i64": np.int64}


def expected_stream(e):
    h = e["header"]
    out = bytearray(struct.pack("<IIIIqII", h["R"], h["ngB"], h["Q"], h["ngA"], h["d"], h["b_off"], 0))
    for a in e["a_records"]:
        out += struct.pack("<IIIIqq", a["out_off"], a["poff"], a["widths"], a["lmin"], a["base"], a["vmin"])
    for b in e["b_records"]:
        out += struct.pack("<IIII", b["out_off"], b["poff"], b["wc"], b["cmin"])
    out += struct.pack(f"<{len(e['words'])}I", *e["words"])
    assert len(out) == e["comp_len"]
    return bytes(out)


def test_golden_streams(golden):
    for e in golden("dstree_examples.json")["examples"]:
        x = np.array(e["values"], DT[e["dtype"]])
        got = stream_of(z.encode(x, z.DSTREE, [len(x)]))
        assert got == expected_stream(e), e["name"]
        rc, out = z.decode_stream(z.DSTREE, z.I32 if e["dtype"] == "i32" else z.I64, got, len(x))
        assert rc == z.OK and np.array_equal(out, x)


# ------------------------------------------------------ independent reader
def fields(words, n, w):
    """n fields of width w, LSB first, from little-endian u32 words."""
    big = int.from_bytes(words, "little")
    return [(big >> (j * w)) & ((1 << w) - 1) for j in range(n)]


def read_parts(s, bits):
    R, ngB, Q, ngA, d, b_off, zero = struct.unpack_from("<IIIIqII", s, 0)
    assert zero == 0 and b_off == 32 + 32 * ngA and ngA == -(-Q // 64) and ngB == -(-R // 64)
    m = (1 << bits) - 1
    V, L, A = [], [], []
    end = b_off + 16 * ngB
    for g_ in range(ngA):
        out_off, poff, widths, lmin, base, vmin = struct.unpack_from("<IIIIqq", s, 32 + 32 * g_)
        cnt = min(64, Q - 64 * g_)
        wv, wl = widths & 0xFF, widths >> 8
        vw, lw = (cnt * wv + 31) // 32, (cnt * wl + 31) // 32
        assert poff == end  # payloads follow each other word by word
        V += [(vmin + f) & m for f in fields(s[poff:poff + 4 * vw], cnt, wv)]
        L += [lmin + f for f in fields(s[poff + 4 * vw:poff + 4 * (vw + lw)], cnt, wl)]
        A.append((out_off, base & m))
        end = poff + 4 * (vw + lw)
    C, B = [], []
    for g_ in range(ngB):
        out_off, poff, wc, cmin = struct.unpack_from("<IIII", s, b_off + 16 * g_)
        cnt = min(64, R - 64 * g_)
        cw = (cnt * wc + 31) // 32
        assert poff == end
        C += [cmin + f for f in fields(s[poff:poff + 4 * cw], cnt, wc)]
        B.append(out_off)
        end = poff + 4 * cw
    assert end == len(s)
    return dict(R=R, Q=Q, d=d & m, V=V, L=L, C=C, A=A, B=B)


def derive(x, bits):
    """What each stage must hold, from numpy."""
    m = (1 << bits) - 1
    u = [int(v) & m for v in x.tolist()]
    if len(u) > 1:
        df = np.array([(b - a) & m for a, b in zip(u, u[1:])], dtype=object)
        vals, counts = np.unique(df.astype(np.uint64), return_counts=True)
        d = int(vals[np.flatnonzero(counts == counts.max())[0]])  # unique() sorts: the first is the smallest
    else:
        d = 0
    brk = [0] + [i + 1 for i in range(len(u) - 1) if (u[i + 1] - u[i]) & m != d] + [len(u)]
    S = [u[a] for a in brk[:-1]]
    C = [b - a for a, b in zip(brk[:-1], brk[1:])]
    D = [S[0]] + [(b - a) & m for a, b in zip(S, S[1:])]
    V, L = [], []
    for v in D:
        if V and V[-1] == v:
            L[-1] += 1
        else:
            V.append(v)
            L.append(1)
    return dict(d=d, S=S, C=C, V=V, L=L)


def cases():
    r = g.rng(11)
    out = []
    for dt, bits in ((np.int32, 32), (np.int64, 64)):
        i = np.arange(20000)
        keys = (32 * (i // 8) + i % 8 + 1).astype(dt)
        out += [(keys, bits), (keys[r.random(keys.size) > 0.01], bits),
                (g.key_column(9000, 3, dtype=dt), bits),
                (r.integers(-100, 100, size=3000).astype(dt), bits),
                (np.arange(5000, dtype=dt) * 7 - 3, bits),
                (np.iinfo(dt).max - np.arange(300, dtype=dt), bits)]
    # a progression across the int32 wrap
    out.append(((np.arange(1000, dtype=np.int64) * 3 + 2**31 - 1500).astype(np.int64).astype(np.int32), 32))
    return out


def test_parts_read_back_against_numpy():
    for x, bits in cases():
        s = stream_of(z.encode(x, z.DSTREE, [len(x)]))
        p = read_parts(s, bits)
        want = derive(x, bits)
        assert p["d"] == want["d"]
        assert p["C"] == want["C"] and p["R"] == len(want["S"])
        assert p["V"] == want["V"] and p["L"] == want["L"] and p["Q"] == len(want["V"])
        # group records: D groups start at the running count of L, with the
        # start before them as base; the runs' groups at the running count of C
        m = (1 << bits) - 1
        at = np.concatenate([[0], np.cumsum(want["L"])])
        for g_, (out_off, base) in enumerate(p["A"]):
            assert out_off == at[64 * g_]
            assert base == (0 if out_off == 0 else want["S"][out_off - 1] & m)
        cat = np.concatenate([[0], np.cumsum(want["C"])])
        assert p["B"] == [int(cat[64 * g_]) for g_ in range(len(p["B"]))]
        # and the whole tree decodes to x
        assert np.array_equal(z.decode(z.encode(x, z.DSTREE, [len(x)])), x)


def test_brute_force_short_sequences():
    for dt, top in ((np.int32, 5), (np.int64, 4)):
        for n in range(1, top + 1):
            for t in itertools.product(range(-2, 3), repeat=n):
                x = np.array(t, dt)
                assert np.array_equal(z.decode(z.encode(x, z.DSTREE, [n])), x), t


def test_closed_form_size_of_even_key_blocks():
    # m blocks of 8 consecutive keys, each 32 past the previous: d = 1, R = m,
    # D = [1, 32, 32, ...] so Q = 2 (one D group: two V fields at width 5 and
    # two L fields at width bitlen(m - 2), one word each), every C = 8 (width
    # 0, no words): 32 + 32 + 16 ceil(m / 64) + 8 bytes
    for m in (3, 64, 65, 1000, 4097):
        i = np.arange(8 * m)
        x = (32 * (i // 8) + i % 8 + 1).astype(np.int32)
        s = stream_of(z.encode(x, z.DSTREE, [len(x)]))
        assert len(s) == 32 + 32 + 16 * (-(-m // 64)) + 8, m


def test_corrupt_streams_rejected():
    i = np.arange(5000)
    x = (32 * (i // 8) + i % 8 + 1).astype(np.int32)
    x = x[g.rng(5).random(x.size) > 0.05]
    good = bytearray(stream_of(z.encode(x, z.DSTREE, [len(x)])))
    n = len(x)
    assert z.decode_stream(z.DSTREE, z.I32, bytes(good), n)[0] == z.OK
    R, ngB, Q, ngA = struct.unpack_from("<IIII", good, 0)
    b_off = struct.unpack_from("<I", good, 24)[0]
    assert ngA >= 2 and ngB >= 2

    def bad(off, fmt, val):
        s = bytearray(good)
        struct.pack_into(fmt, s, off, val)
        return z.decode_stream(z.DSTREE, z.I32, bytes(s), n)[0]
    assert bad(0, "<I", R + 1) == z.ECORRUPT              # run count
    assert bad(8, "<I", Q + 64) == z.ECORRUPT             # D run count vs its groups
    assert bad(24, "<I", b_off + 16) == z.ECORRUPT        # runs' records offset
    assert bad(32 + 8, "<I", 33) == z.ECORRUPT            # V width above 32 bits
    assert bad(32 + 32 + 0, "<I", 1) == z.ECORRUPT        # second D group's output offset
    assert bad(b_off + 16, "<I", 3) == z.ECORRUPT         # second runs group's output offset
    assert bad(b_off + 12, "<I", 0) == z.ECORRUPT         # a zero count (cmin 0 with a 0 field)
    assert bad(b_off + 4, "<I", len(good)) == z.ECORRUPT  # payload past the end
    assert z.decode_stream(z.DSTREE, z.I32, bytes(good[:-4]), n)[0] == z.ECORRUPT
