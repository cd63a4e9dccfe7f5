"""String-dictionary in the oracle, pinned to things other than itself:
streams derived by hand (tests/golden/sdict_examples.json), the properties
that define the tokens and the entry order, brute-force round trips over
every short string of a small alphabet, the entry count of generated text
against a regular-expression split, and rejection of corrupt streams.  The
nested String-dictionary | bit-packing | ANS stream is pinned to its two
separately pinned parts: the String-dictionary stream up to its codes, then
the ANS streams of exactly its packed index bytes, 64 KiB per piece."""
import itertools
import re
import struct

import numpy as np

import oracle.zfo as z
from paper_2602_08190_amd import datagen as g

SEP = b" ."


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def parse(s):
    """(tokens, entries, codes) read from a stream's fields."""
    nt, ne, w, ng, eo, bo, co, nb = struct.unpack_from("<8I", s, 0)
    ents = struct.unpack_from(f"<{ne}I", s, eo)
    entries = [s[bo + (e & 0xFFFFFF):bo + (e & 0xFFFFFF) + (e >> 24)] for e in ents]
    bits = int.from_bytes(s[co:], "little")
    codes = [(bits >> (w * t)) & ((1 << w) - 1) for t in range(nt)]
    return [entries[c] for c in codes], entries, codes


def test_hand_derived_streams(golden):
    for e in golden("sdict_examples.json")["examples"]:
        text = e["text"].encode() if "text" in e else e["text_repeat"][0].encode() * e["text_repeat"][1]
        x = np.frombuffer(text, np.uint8)
        s = stream_of(z.encode(x, z.SDICT_BP))
        h = e["header"]
        assert list(struct.unpack_from("<8I", s, 0)) == h, e["name"]
        assert list(struct.unpack_from(f"<{h[3]}I", s, 32)) == e["group_offsets"]
        assert list(struct.unpack_from(f"<{h[1]}I", s, h[4])) == e["entries"]
        if "entry_bytes" in e:
            assert s[h[5]:h[5] + h[7]] == e["entry_bytes"].encode()
        nw = (h[0] * h[2] + 31) // 32
        assert list(struct.unpack_from(f"<{nw}I", s, h[6])) == e["code_words"]
        assert len(s) == e["comp_len"]
        if "tokens" in e:
            assert [t.decode() for t in parse(s)[0]] == e["tokens"]
        rc, out = z.decode_stream(z.SDICT_BP, z.BYTES, s, len(x))
        assert rc == z.OK and out.tobytes() == text


def _check_tokens(text):
    """Tokens concatenate to the text; each is 1..64 bytes with a separator
    only as its last byte; one without a final separator is 64 bytes long or
    the last token; entries are distinct and numbered by first appearance."""
    toks, entries, codes = parse(stream_of(z.encode(np.frombuffer(text, np.uint8), z.SDICT_BP)))
    assert b"".join(toks) == text
    for i, t in enumerate(toks):
        assert 1 <= len(t) <= 64
        assert not any(c in SEP for c in t[:-1])
        if t[-1] not in SEP:
            assert len(t) == 64 or i == len(toks) - 1
    assert len(set(entries)) == len(entries)
    first = []
    for c in codes:
        if c not in first:
            first.append(c)
    assert first == list(range(len(entries)))


def test_brute_force_short_strings():
    for n in range(1, 8):
        for t in itertools.product(b"ab .", repeat=n):
            text = bytes(t)
            x = np.frombuffer(text, np.uint8)
            assert z.decode(z.encode(x, z.SDICT_BP)).tobytes() == text
            if n <= 5:
                _check_tokens(text)


def test_generated_text_entries_match_a_regex_split():
    text = g.text_column(300000, 4).tobytes()
    for lo, hi in ((0, 300000), (1000, 66536), (5, 6)):
        part = text[lo:hi]
        toks = re.findall(rb"[^ .]*[ .]|[^ .]+$", part)
        assert all(len(t) <= 64 for t in toks)
        s = stream_of(z.encode(np.frombuffer(part, np.uint8), z.SDICT_BP, chunk_elems=[hi - lo]))
        got, entries, _ = parse(s)
        assert got == toks
        assert len(entries) == len(set(toks))
    _check_tokens(text[:20000])


def test_long_runs_and_binary_bytes_round_trip():
    r = np.random.default_rng(5)
    for x in (np.frombuffer(r.bytes(50000), np.uint8),
              np.full(1000, ord("a"), np.uint8),
              np.full(1000, ord(" "), np.uint8),
              np.frombuffer(b"." * 129 + b"a" * 129, np.uint8)):
        assert np.array_equal(z.decode(z.encode(x, z.SDICT_BP, chunk_elems=[len(x)])), x)
        if len(x) <= 20000:
            _check_tokens(x.tobytes())


def test_corrupt_streams_are_rejected(golden):
    x = np.frombuffer(b"the cat. the dog ran the cat", np.uint8)
    good = bytearray(stream_of(z.encode(x, z.SDICT_BP)))
    assert z.decode_stream(z.SDICT_BP, z.BYTES, bytes(good), len(x))[0] == z.OK

    def bad(mut, n=len(x)):
        s = bytearray(good)
        mut(s)
        return z.decode_stream(z.SDICT_BP, z.BYTES, bytes(s), n)[0]
    assert bad(lambda s: struct.pack_into("<I", s, 96, 7 << 21)) == z.ECORRUPT     # code 7 >= 6 entries
    assert bad(lambda s: struct.pack_into("<I", s, 48, 0)) == z.ECORRUPT           # entry of length 0
    assert bad(lambda s: struct.pack_into("<I", s, 48, 18 | (4 << 24))) == z.ECORRUPT  # entry past the bytes
    assert bad(lambda s: struct.pack_into("<I", s, 32, 1)) == z.ECORRUPT           # group offset
    assert bad(lambda s: struct.pack_into("<I", s, 8, 4)) == z.ECORRUPT            # width
    assert bad(lambda s: None, n=len(x) + 1) == z.ECORRUPT                          # too few bytes


# ----------------------------------------- String-dictionary | BP | ANS
PIECE = 65536


def pieces_of(nested, co):
    """The ANS streams of a nested stream, read from its piece table."""
    np_ = struct.unpack_from("<I", nested, co)[0]
    ends = struct.unpack_from(f"<{np_}I", nested, co + 4)
    base = co + 4 + 4 * np_
    return [nested[base + (ends[k - 1] if k else 0):base + ends[k]] for k in range(np_)], base + ends[-1]


def test_nested_stream_is_sdict_with_ans_coded_indices():
    """The nested stream is the String-dictionary stream up to its codes,
    then ANS streams (a separately pinned codec) of exactly the packed index
    bytes, cut into pieces of 65536 bytes and each zero-padded to a multiple
    of 4 bytes; it decodes to the input."""
    r = np.random.default_rng(8)
    for x in (np.frombuffer(g.text_column(2_000_000, 7).tobytes(), np.uint8),
              np.frombuffer(b"the cat. the dog ran the cat", np.uint8),
              np.frombuffer(r.bytes(5000), np.uint8)):
        sd = stream_of(z.encode(x, z.SDICT_BP, chunk_elems=[len(x)]))
        nested = stream_of(z.encode(x, z.SDICT_ANS, chunk_elems=[len(x)]))
        co = struct.unpack_from("<I", sd, 24)[0]
        assert nested[:co] == sd[:co]
        codes = np.frombuffer(sd[co:], np.uint8)
        streams, end = pieces_of(nested, co)
        assert end == len(nested) and len(streams) == (len(codes) + PIECE - 1) // PIECE
        for k, st in enumerate(streams):
            piece = codes[k * PIECE:(k + 1) * PIECE]
            ans = stream_of(z.encode(piece, z.ANS, chunk_elems=[len(piece)]))
            # each stream is stored zero-padded to a multiple of 4 bytes
            assert len(st) == (len(ans) + 3) // 4 * 4 and st == ans + bytes(len(st) - len(ans))
            rc, out = z.decode_stream(z.ANS, z.BYTES, ans, len(piece))
            assert rc == z.OK and np.array_equal(out, piece)
        rc, out = z.decode_stream(z.SDICT_ANS, z.BYTES, nested, len(x))
        assert rc == z.OK and np.array_equal(out, x)


def ab_tokens(nt, seed):
    """nt tokens, each "a " or "b " at random: two entries, so w = 1 and the
    packed indices take 4*ceil(nt/32) bytes."""
    t = np.random.default_rng(seed).integers(0, 2, nt)
    x = np.empty(2 * nt, np.uint8)
    x[0::2], x[1::2] = np.where(t == 0, ord("a"), ord("b")), ord(" ")
    return x


def test_nested_piece_boundary():
    # exactly one full piece of index bytes, then one 4-byte piece past it
    for nt, pieces, last in ((8 * PIECE, 1, PIECE), (8 * PIECE + 32, 2, 4)):
        x = ab_tokens(nt, nt)
        sd = stream_of(z.encode(x, z.SDICT_BP, chunk_elems=[len(x)]))
        nested = stream_of(z.encode(x, z.SDICT_ANS, chunk_elems=[len(x)]))
        co = struct.unpack_from("<I", sd, 24)[0]
        assert struct.unpack_from("<I", sd, 8)[0] == 1 and len(sd) - co == (nt + 31) // 32 * 4
        streams, _ = pieces_of(nested, co)
        assert len(streams) == pieces and struct.unpack_from("<I", streams[-1], 0)[0] == last
        rc, out = z.decode_stream(z.SDICT_ANS, z.BYTES, nested, len(x))
        assert rc == z.OK and np.array_equal(out, x)


def test_nested_without_index_bytes():
    # one distinct token: w = 0, no index bytes, no ANS stream
    x = np.frombuffer(b"x " * 70, np.uint8)
    s = stream_of(z.encode(x, z.SDICT_ANS))
    assert struct.unpack_from("<I", s, 8)[0] == 0 and len(s) == struct.unpack_from("<I", s, 24)[0]
    assert z.decode_stream(z.SDICT_ANS, z.BYTES, s, len(x))[1].tobytes() == x.tobytes()


def test_nested_brute_force_round_trips():
    for n in range(1, 7):
        for t in itertools.product(b"ab .", repeat=n):
            x = np.frombuffer(bytes(t), np.uint8)
            assert z.decode(z.encode(x, z.SDICT_ANS)).tobytes() == bytes(t)


def test_nested_corrupt_streams_are_rejected():
    x = np.frombuffer(g.text_column(20000, 9).tobytes(), np.uint8)
    good = bytearray(stream_of(z.encode(x, z.SDICT_ANS)))
    co = struct.unpack_from("<I", good, 24)[0]
    assert z.decode_stream(z.SDICT_ANS, z.BYTES, bytes(good), len(x))[0] == z.OK

    def bad(mut):
        s = bytearray(good)
        mut(s)
        return z.decode_stream(z.SDICT_ANS, z.BYTES, bytes(s), len(x))[0]
    assert bad(lambda s: struct.pack_into("<I", s, co, 2)) == z.ECORRUPT        # piece count
    assert bad(lambda s: struct.pack_into("<I", s, co + 8, 7)) == z.ECORRUPT    # ANS length field
    last = co + 8 + 784 + 2 * struct.unpack_from("<I", good, co + 8 + 4)[0] - 1  # end of the ANS words
    assert bad(lambda s: s.__setitem__(last, s[last] ^ 0x55)) == z.ECORRUPT  # a word
    assert bad(lambda s: struct.pack_into("<I", s, 24, co + 16)) == z.ECORRUPT  # codes offset
