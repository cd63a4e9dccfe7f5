"""ANS (range ANS, 64 interleaved coders sharing one word stream) in the
oracle, pinned to things other than itself: hand-computed streams (two with
renormalisation, one of them interleaving two coders' words), the
hand-derived frequency quantisation, brute-force round trips of every short
string over a small alphabet, the coding cost against the model's entropy,
and rejection of corrupt streams."""
import itertools
import math
import struct

import numpy as np

import oracle.zfo as z

HDR = 784


def stream_of(blob, i=0):
    c = z.chunks(blob)[i]
    return bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])


def expected_stream(n, freq, states, words):
    def per_lane(d):
        return [d.get(str(j), d.get("rest")) for j in range(64)]
    f = [0] * 256
    for k, v in freq.items():
        f[int(k)] = v
    return (struct.pack("<IIII", n, len(words), 0, 0) + struct.pack("<256H", *f) +
            struct.pack("<64I", *per_lane(states)) + struct.pack(f"<{len(words)}H", *words))


def freqs_of(stream):
    return struct.unpack_from("<256H", stream, 16)


def test_golden_streams(golden):
    gd = golden("ans_examples.json")
    ex = gd["examples"]
    x0 = np.frombuffer(ex[0]["text"].encode(), np.uint8)
    x1 = np.full(256, ord("a"), np.uint8)
    x1[[0, 64, 128, 192]] = [ord("W"), ord("X"), ord("Y"), ord("Z")]
    x2 = np.full(256, ord("a"), np.uint8)
    x2[[0, 64, 128, 192, 65, 193]] = [ord(c) for c in "PQRSTU"]
    for e, x in ((ex[0], x0), (ex[1], x1), (ex[2], x2)):
        want = expected_stream(len(x), e["freq"], e["states"], e["words"])
        got = stream_of(z.encode(x, z.ANS))
        assert got == want, e["name"]
        rc, out = z.decode_stream(z.ANS, z.BYTES, want, len(x))
        assert rc == z.OK and np.array_equal(out, x)


def test_quantisation_by_hand(golden):
    q = golden("ans_examples.json")["quantisation"]
    f = freqs_of(stream_of(z.encode(np.frombuffer(b"abc", np.uint8), z.ANS)))
    assert {i: v for i, v in enumerate(f) if v} == {int(k): v for k, v in q[0]["freq"].items()}
    others = [b for b in range(201) if b != ord("a")]
    x = np.array([ord("a")] * 9800 + others, np.uint8)
    f = freqs_of(stream_of(z.encode(x, z.ANS)))
    assert f[ord("a")] == q[1]["freq_a"] and all(f[b] == q[1]["freq_other"] for b in others)
    assert sum(f) == 4096


def test_brute_force_short_strings():
    for n in range(1, 5):
        for t in itertools.product(b"ab\xff", repeat=n):
            x = np.frombuffer(bytes(t), np.uint8)
            assert np.array_equal(z.decode(z.encode(x, z.ANS)), x)


def test_round_trips_and_cost_within_the_model_entropy():
    r = np.random.default_rng(3)
    cases = [r.choice(np.frombuffer(b"ANR", np.uint8), size=n, p=p)
             for n, p in ((50000, [0.25, 0.5, 0.25]), (70000, [0.05, 0.9, 0.05]), (129, [0.3, 0.4, 0.3]))]
    cases.append(r.integers(0, 256, size=40000).astype(np.uint8))
    cases.append(np.full(5000, 7, np.uint8))  # one symbol: f = M, no words at all
    for x in cases:
        blob = z.encode(x, z.ANS, [len(x)])
        assert np.array_equal(z.decode(blob), x)
        s = stream_of(blob)
        f = freqs_of(s)
        nw = struct.unpack_from("<I", s, 4)[0]
        # bits the model assigns to the data, plus at most 48 bits per coder
        ideal = sum(math.log2(4096 / f[b]) for b in x.tolist())
        assert 16 * nw <= ideal * 1.002 + 64 * 48, (16 * nw, ideal)
        assert 16 * nw >= ideal - 64 * 32


def test_corrupt_streams_rejected():
    x = np.random.default_rng(4).choice(np.frombuffer(b"ANR", np.uint8), size=3000)
    s = bytearray(stream_of(z.encode(x, z.ANS)))
    n = len(x)
    assert z.decode_stream(z.ANS, z.BYTES, bytes(s), n)[0] == z.OK
    bad = []
    t = bytearray(s); t[16 + 2 * ord("A")] ^= 1; bad.append(t)          # frequencies not summing to M
    t = bytearray(s); t[528] ^= 0x40; bad.append(t)                     # a final state
    t = bytearray(s); t[4] += 1; bad.append(t)                          # the word count
    t = bytearray(s[:-2]); t[4:8] = struct.pack("<I", len(t) // 2 - HDR // 2); bad.append(t)  # a word short
    t = bytearray(s); t[HDR] ^= 0xFF; t[HDR + 1] ^= 0xFF; bad.append(t)  # a word
    for t in bad:
        assert z.decode_stream(z.ANS, z.BYTES, bytes(t), n)[0] == z.ECORRUPT
