"""String-dictionary over a column dictionary (SDICT_COL) in the oracle,
pinned to things other than itself: streams and dictionaries derived by hand
(tests/golden/sdict_col_examples.json), the properties that define the
tokens (separators space, period and row end) and the entry order (count,
then first appearance, over the whole column), independence of the chunking
from the dictionary, brute-force round trips over every short string of a
small alphabet and every chunking of it, the token list of generated text
against a regular-expression split, and rejection of corrupt streams and
dictionaries.  The nested SDICT_COL | bit-packing | ANS stream is pinned to
its two separately pinned parts."""
import collections
import itertools
import re
import struct

import numpy as np
import pytest

import oracle.zfo as z
from paper_2602_08190_amd import datagen as g

SEP = b" .\n"
PIECE = 65536


def text_of(e):
    if "text" in e:
        return e["text"].encode()
    return b"".join(p.encode() * k for p, k in e["text_parts"])


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def dictionary(blob):
    """(entries as bytes, raw entry words, n_bytes, area length) of the
    column dictionary, read from its fields."""
    info = z.inspect(blob)
    d, ne = info["dict_off"], info["dict_count"]
    b = bytes(blob)
    nb = struct.unpack_from("<I", b, d)[0]
    words = struct.unpack_from(f"<{ne}I", b, d + 16)
    base = d + 16 + 4 * ne
    ents = [b[base + (e & 0xFFFFFF):base + (e & 0xFFFFFF) + (e >> 24)] for e in words]
    return ents, list(words), nb, 16 + 4 * ne + (nb + 15) // 16 * 16


def parse(s, ents):
    nt, w, ng, co = struct.unpack_from("<4I", s, 0)
    bits = int.from_bytes(s[co:], "little")
    codes = [(bits >> (w * t)) & ((1 << w) - 1) for t in range(nt)]
    return [ents[c] for c in codes], codes


def test_hand_derived_streams(golden):
    for e in golden("sdict_col_examples.json")["examples"]:
        text = text_of(e)
        x = np.frombuffer(text, np.uint8)
        for ch in e["chunkings"]:
            blob = z.encode(x, z.SDICT_COL, chunk_elems=ch["chunk_elems"])
            info = z.inspect(blob)
            assert info["dict_count"] == len(e["dict_entries"]), e["name"]
            assert info["dict_off"] == (64 + 32 * len(ch["chunk_elems"]) + 15) // 16 * 16
            b = bytes(blob)
            d = info["dict_off"]
            assert list(struct.unpack_from("<4I", b, d)) == e["dict_header"]
            ents, words, nb, dlen = dictionary(blob)
            assert words == e["dict_entries"] and dlen == e["dict_len"]
            if "dict_bytes_hex" in e:
                assert b[d + 16 + 4 * len(words):][:nb] == bytes.fromhex(e["dict_bytes_hex"])
            assert b[d + 16 + 4 * len(words) + nb:d + dlen] == bytes(dlen - 16 - 4 * len(words) - nb)
            # the stored layout: first entry at 4, each next at align4(end + 3),
            # n_bytes = align4(last end + 3), zeros between entries
            at = last = 4
            for wd in words:
                assert wd & 0xFFFFFF == at
                last = at
                at = (at + (wd >> 24) + 3 + 3) // 4 * 4
            assert nb == max(at, last + 16)
            for i, c in enumerate(ch["chunks"]):
                s = stream_of(blob, i)
                h = c["header"]
                assert list(struct.unpack_from("<4I", s, 0)) == h, (e["name"], i)
                assert list(struct.unpack_from(f"<{h[2]}I", s, 16)) == c["group_offsets"]
                nw = (h[0] * h[1] + 31) // 32
                assert list(struct.unpack_from(f"<{nw}I", s, h[3])) == c["code_words"]
                assert len(s) == c["comp_len"]
                if "tokens" in c:
                    assert [t.decode() for t in parse(s, ents)[0]] == c["tokens"]
            assert z.decode(blob).tobytes() == text


def _check(text, chunk_elems):
    """Tokens of every chunk concatenate to it, are 1..64 bytes with a
    separator only as the last byte (a token without one is 64 bytes long or
    ends its chunk); the entries are the distinct tokens of the column,
    ordered by count (largest first), then by first appearance."""
    blob = z.encode(np.frombuffer(text, np.uint8), z.SDICT_COL, chunk_elems=chunk_elems)
    ents, _, _, _ = dictionary(blob)
    all_toks = []
    at = 0
    for i, n in enumerate(chunk_elems):
        toks, codes = parse(stream_of(blob, i), ents)
        assert b"".join(toks) == text[at:at + n]
        for k, t in enumerate(toks):
            assert 1 <= len(t) <= 64
            assert not any(c in SEP for c in t[:-1])
            if t[-1] not in SEP:
                assert len(t) == 64 or k == len(toks) - 1
        all_toks += toks
        at += n
    cnt = collections.Counter(all_toks)
    first = {}
    for k, t in enumerate(all_toks):
        first.setdefault(t, k)
    assert sorted(cnt) == sorted(ents) and len(set(ents)) == len(ents)
    assert ents == sorted(cnt, key=lambda t: (-cnt[t], first[t]))
    assert z.decode(blob).tobytes() == text


def test_brute_force_short_strings_and_chunkings():
    for n in range(1, 7):
        for t in itertools.product(b"ab .\n", repeat=n):
            text = bytes(t)
            if n <= 4:
                for cut in range(1, n):          # every two-chunk split
                    _check(text, [cut, n - cut])
            _check(text, [n])


def test_dictionary_is_shared_by_the_chunks():
    """Re-chunking a column changes the chunk streams, not how each token's
    entry is found: every chunking decodes to the text, and chunkings that
    cut no token have the same dictionary."""
    text = g.text_column(200000, 12).tobytes()
    x = np.frombuffer(text, np.uint8)
    ref = None
    for ce in ([len(x)], [100000, 100000], [1, 65535, len(x) - 65536]):
        blob = z.encode(x, z.SDICT_COL, chunk_elems=ce)
        assert z.decode(blob).tobytes() == text
        _check(text, ce) if len(ce) > 1 and ce[0] > 1 else None
    # chunk boundaries right after a separator cut no token
    cuts = [i + 1 for i, c in enumerate(text) if c in SEP]
    a, b = cuts[len(cuts) // 3], cuts[2 * len(cuts) // 3]
    d1 = dictionary(z.encode(x, z.SDICT_COL, chunk_elems=[len(x)]))[0]
    d2 = dictionary(z.encode(x, z.SDICT_COL, chunk_elems=[a, b - a, len(x) - b]))[0]
    assert d1 == d2


def test_generated_text_tokens_match_a_regex_split():
    text = g.text_column(300000, 4).tobytes()
    toks = re.findall(rb"[^ .\n]*[ .\n]|[^ .\n]+$", text)
    assert all(len(t) <= 64 for t in toks)
    blob = z.encode(np.frombuffer(text, np.uint8), z.SDICT_COL, chunk_elems=[len(text)])
    ents = dictionary(blob)[0]
    got, _ = parse(stream_of(blob), ents)
    assert got == toks
    cnt = collections.Counter(toks)
    assert len(ents) == len(cnt) and ents[0] == cnt.most_common(1)[0][0]


def test_long_runs_and_binary_bytes_round_trip():
    r = np.random.default_rng(5)
    for x in (np.frombuffer(r.bytes(30000), np.uint8),
              np.full(1000, ord("a"), np.uint8),
              np.full(1000, ord("\n"), np.uint8),
              np.frombuffer(b"." * 129 + b"a" * 129 + b"\n" * 3, np.uint8)):
        blob = z.encode(x, z.SDICT_COL, chunk_elems=[len(x) // 2, len(x) - len(x) // 2])
        assert np.array_equal(z.decode(blob), x)
        if len(x) <= 3000:
            _check(x.tobytes(), [len(x) // 2, len(x) - len(x) // 2])


def test_corrupt_streams_and_dictionaries_are_rejected():
    x = np.frombuffer(b"the cat. the dog\nthe cat ", np.uint8)
    blob = z.encode(x, z.SDICT_COL)
    info = z.inspect(blob)
    d = info["dict_off"]
    s = stream_of(blob)
    dict_area = bytes(blob[d:d + 84])
    assert len(dictionary(blob)[0]) == 5 and dictionary(blob)[3] == 84
    assert z.decode_stream(z.SDICT_COL, z.BYTES, s, len(x), dict_area, 5)[0] == z.OK

    def bad(mut=None, dmut=None, n=len(x), count=5):
        t, dd = bytearray(s), bytearray(dict_area)
        if mut:
            mut(t)
        if dmut:
            dmut(dd)
        return z.decode_stream(z.SDICT_COL, z.BYTES, bytes(t), n, bytes(dd), count)[0]
    assert bad(lambda t: struct.pack_into("<I", t, 32, 5 << 3)) == z.ECORRUPT   # code 5 >= 5 entries
    assert bad(lambda t: struct.pack_into("<I", t, 16, 1)) == z.ECORRUPT         # group offset
    assert bad(lambda t: struct.pack_into("<I", t, 4, 4)) == z.ECORRUPT          # width
    assert bad(lambda t: struct.pack_into("<I", t, 12, 48)) == z.ECORRUPT        # codes offset
    assert bad(count=4) == z.ECORRUPT                                             # width of 4 entries is 2
    assert bad(dmut=lambda dd: struct.pack_into("<I", dd, 16, 0)) == z.ECORRUPT  # entry of length 0
    assert bad(dmut=lambda dd: struct.pack_into("<I", dd, 16 + 16, 46 | (4 << 24))) == z.ECORRUPT  # past bytes
    assert bad(n=len(x) + 1) == z.ECORRUPT                                        # too few bytes
    # the container: a token dictionary's size follows its byte count
    b = bytearray(blob)
    struct.pack_into("<I", b, d, 1 << 24)
    with pytest.raises(z.OracleError):
        z.inspect(b)
    b = bytearray(blob)
    b[d + 16] ^= 1            # the table CRC covers the dictionary
    with pytest.raises(z.OracleError):
        z.inspect(b)
    # a nonzero byte next to an entry, the table CRC kept right
    import zlib
    for at in (d + 16 + 20 + 8, d + 16 + 20 + 11, d + 16 + 20 + 3):   # after "the ", before "cat.", before "the "
        b = bytearray(blob)
        b[at] = 0x41
        ne = 5
        tl = 32 * info["n_chunks"]
        crc = zlib.crc32(bytes(b[64:64 + tl]) + bytes(b[d:d + 84]))  # the dictionary area is 84 bytes
        struct.pack_into("<I", b, 48, crc)
        struct.pack_into("<I", b, 60, zlib.crc32(bytes(b[:60])))
        with pytest.raises(z.OracleError):
            z.inspect(b)


def test_nested_stream_is_sdict_col_with_ans_coded_indices():
    r = np.random.default_rng(8)
    for x in (np.frombuffer(g.text_column(1_500_000, 7).tobytes(), np.uint8),
              np.frombuffer(b"the cat. the dog\nthe cat ", np.uint8),
              np.frombuffer(r.bytes(5000), np.uint8)):
        ce = [len(x) // 3, len(x) - len(x) // 3]
        plain = z.encode(x, z.SDICT_COL, chunk_elems=ce)
        nested = z.encode(x, z.SDICT_COL_ANS, chunk_elems=ce)
        assert dictionary(plain)[:3] == dictionary(nested)[:3]
        for i in range(2):
            sd, ns = stream_of(plain, i), stream_of(nested, i)
            co = struct.unpack_from("<I", sd, 12)[0]
            assert ns[:co] == sd[:co]
            codes = np.frombuffer(sd[co:], np.uint8)
            if len(codes) == 0:
                assert len(ns) == co
                continue
            np_ = struct.unpack_from("<I", ns, co)[0]
            ends = struct.unpack_from(f"<{np_}I", ns, co + 4)
            base = co + 4 + 4 * np_
            assert np_ == (len(codes) + PIECE - 1) // PIECE and base + ends[-1] == len(ns)
            for k in range(np_):
                st = ns[base + (ends[k - 1] if k else 0):base + ends[k]]
                piece = codes[k * PIECE:(k + 1) * PIECE]
                ans = stream_of(z.encode(piece, z.ANS, chunk_elems=[len(piece)]))
                assert st == ans + bytes(len(st) - len(ans)) and len(st) % 4 == 0
        assert np.array_equal(z.decode(nested), x)


def test_nested_brute_force_round_trips():
    for n in range(1, 6):
        for t in itertools.product(b"ab .\n", repeat=n):
            x = np.frombuffer(bytes(t), np.uint8)
            assert z.decode(z.encode(x, z.SDICT_COL_ANS)).tobytes() == bytes(t)


def test_too_many_distinct_tokens_is_unsupported():
    # 2^24 entry bytes are the limit: 280,000 distinct 64-byte tokens exceed it
    r = np.random.default_rng(3)
    x = np.frombuffer(r.integers(ord("a"), ord("z") + 1, size=64 * 280000, dtype=np.uint8).tobytes(), np.uint8)
    with pytest.raises(z.OracleError) as e:
        z.encode(x, z.SDICT_COL, chunk_elems=[len(x)])
    assert e.value.code == z.EUNSUP
