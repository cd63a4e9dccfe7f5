"""Test-only builders: raw codec streams and column containers assembled
field by field (zlib's CRC-32 is the IEEE CRC the format uses)."""
import struct
import zlib

import numpy as np

ES = {1: 4, 2: 8, 3: 1, 4: 16}


def lz_stream(seqs, lits, plain_len):
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


def random_lz(rng, plain_len, max_lit=20, small_offsets=True):
    """A random valid LZ77 sequence list covering plain_len bytes; matches
    often overlap themselves and reach into the same 64-sequence batch."""
    seqs, lits, pos = [], bytearray(), 0
    while pos < plain_len:
        ll = int(rng.integers(0, max_lit + 1)) if rng.random() < 0.8 else int(rng.integers(7, 300))
        ll = min(ll, plain_len - pos)
        if pos == 0 and ll == 0:
            ll = 1
        lits += bytes(rng.integers(0, 256, size=ll, dtype=np.uint8))
        pos += ll
        ml, off = 0, 0
        room = plain_len - pos
        if room >= 4 and rng.random() < 0.9:
            ml = int(min(room, rng.integers(4, 40) if rng.random() < 0.9 else rng.integers(34, 2000)))
            top = min(pos, 65535)
            off = int(rng.integers(1, min(top, 24) + 1)) if (small_offsets and rng.random() < 0.5) \
                else int(rng.integers(1, top + 1))
        seqs.append((ll, ml, off))
        pos += ml
    return seqs, bytes(lits)


def flat_lz(rng, plain_len, empty_every=0):
    """A random valid LZ77 sequence list whose every batch of 64 sequences is
    flat (each match reads only bytes before its batch or its own literals),
    rich in what the flat copy path must get right: matches repeating their
    own literals with a short period, long matches spanning many copy steps,
    sources far back, zero-length literal runs and (every `empty_every`-th
    sequence, if nonzero) empty sequences."""
    seqs, lits, pos, batch_start = [], bytearray(), 0, 0
    while pos < plain_len:
        if len(seqs) % 64 == 0:
            batch_start = pos
        if empty_every and pos > 0 and len(seqs) % empty_every == empty_every - 1:
            seqs.append((0, 0, 0))
            continue
        room = plain_len - pos
        kind = rng.random()
        ll = int(rng.integers(0, 12)) if rng.random() < 0.85 else int(rng.integers(7, 200))
        if pos == 0 and ll == 0:
            ll = 1
        ll = min(ll, room)
        lits += bytes(rng.integers(0, 256, size=ll, dtype=np.uint8))
        P, D = pos, pos + ll
        pos = D
        room = plain_len - pos
        ml, off = 0, 0
        if room >= 4 and kind < 0.35 and ll >= 1:
            # period over its own literals (off <= ll), often long
            off = int(rng.integers(1, min(ll, 9) + 1))
            ml = int(min(room, rng.integers(4, 40) if rng.random() < 0.7 else rng.integers(34, 3000)))
        elif room >= 4 and kind < 0.95 and batch_start >= 4:
            # a copy from before the batch, without overlap
            ml = int(min(room, batch_start, rng.integers(4, 30) if rng.random() < 0.9
                         else rng.integers(34, 2500)))
            if ml >= 4:
                q0 = int(rng.integers(max(0, D - 65535), batch_start - ml + 1))
                off = D - q0
            else:
                ml = 0
        seqs.append((ll, ml, off))
        pos += ml
    return seqs, bytes(lits)


def container(dtype, chunks, dictionary=b"", dict_count=0):
    """chunks: list of (stream_bytes, n_elems, codec)."""
    es = ES[dtype]
    n = len(chunks)
    table_end = 64 + 32 * n
    dict_off = (table_end + 15) // 16 * 16 if dict_count else 0
    pos = ((dict_off + dict_count * es) if dict_count else table_end)
    pos = (pos + 15) // 16 * 16
    offs = []
    for s, _, _ in chunks:
        offs.append(pos)
        pos = (pos + len(s) + 15) // 16 * 16
    blob = bytearray(pos)
    if dict_count:
        blob[dict_off:dict_off + len(dictionary)] = dictionary
    plain_off = 0
    n_elems = 0
    for i, (s, ne, codec) in enumerate(chunks):
        blob[offs[i]:offs[i] + len(s)] = s
        struct.pack_into("<QQIIIB3x", blob, 64 + 32 * i, plain_off, offs[i], ne * es, len(s), ne, codec)
        plain_off += ne * es
        n_elems += ne
    codecs = {c for _, _, c in chunks}
    struct.pack_into("<4sHBBQQIIQQ", blob, 0, b"ZFC1", 1, dtype, codecs.pop() if len(codecs) == 1 else 0,
                     n_elems, n_elems * es, n, dict_count, dict_off, pos)
    tcrc = zlib.crc32(bytes(blob[64:table_end]) + (bytes(blob[dict_off:dict_off + dict_count * es]) if dict_count else b""))
    struct.pack_into("<III", blob, 48, tcrc, 0, 0)
    struct.pack_into("<I", blob, 60, zlib.crc32(bytes(blob[:60])))
    return np.frombuffer(bytes(blob), np.uint8)
