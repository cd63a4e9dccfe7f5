"""A lane-by-lane CPU model of the Group-Parallel decode wave (RLE_DELTA_BP,
DELTA_BP and DSTRIDE_BP; int32 and int64), run over product-encoded streams
for every unit cut a plan can make: the unit starts at any group and any
element, partial last groups, every output misalignment.  It follows the
kernel's steps: the run lengths' wave scan, the run values (RLE: inclusive
scan of base, dmin + field; DeltaStride: base + exclusive scan of stride *
count + inclusive scan of the gaps, value c + stride * p), the window slots of
64 lanes x 16 bytes, the carry of the last run start across lanes and
windows, and the lane permutes that fetch a run's value.  Every value any
lane reads from another lane is read from a lane whose value was set for all
64 lanes, as in the kernel; a lane never reads a value that only exists on
some lanes.  Parity with the oracle here shows the algorithm and the unit
cuts are right, independent of the GPU."""
import struct

import numpy as np
import pytest

import oracle.zfo as zo
from paper_2602_08190_amd import datagen as g
from paper_2602_08190_amd import zf

G = 64


def field(words, bit, w, bits):
    """w-bit field at `bit` of a little-endian u32 word stream (0 past it)."""
    if w == 0:
        return 0
    k = bit >> 5
    v = 0
    for d in range(3):
        if k + d < len(words):
            v |= int(words[k + d]) << (32 * d)
    return (v >> (bit & 31)) & ((1 << w) - 1)


def chunk_streams(col):
    b = col.bytes()
    out = []
    for c in zo.chunks(b):
        out.append((b[c["comp_off"]:c["comp_off"] + c["comp_len"]].tobytes(), c))
    return out


def group_values(s, codec, g, nr, n, bits):
    """Per-lane values of group g as the wave computes them: (goff, next_off,
    cnt, r[64], v[64], dstr[64])."""
    M = (1 << bits) - 1
    rec = 16 + 32 * g
    goff, a1, a2 = struct.unpack_from("<III", s, rec)
    base, dmin = struct.unpack_from("<QQ", s, rec + 16)
    ng = struct.unpack_from("<I", s, 4)[0]
    roff = struct.unpack_from("<I", s, 8)[0]
    next_off = struct.unpack_from("<I", s, rec + 32)[0] if g + 1 < ng else n
    cnt = min(G, nr - g * G)
    lanes = np.arange(G)
    act = lanes < cnt
    if codec == zf.DELTA_BP:
        r = np.where(act, 1, 0)
    else:
        runs = np.frombuffer(s, np.uint32, count=nr, offset=roff)
        r = np.array([int(runs[g * G + l]) if act[l] else 0 for l in range(G)], dtype=object)
    if codec == zf.DSTRIDE_BP:
        poff, widths = a1, a2
        wg, ws = widths & 0xFF, (widths >> 8) & 0xFF
        gmin = struct.unpack_from("<Q", s, poff)[0]
        nwg = ((cnt - 1) * wg + 31) // 32
        gw = np.frombuffer(s, np.uint32, count=nwg, offset=poff + 8)
        sw = np.frombuffer(s, np.uint32, count=(cnt * ws + 31) // 32, offset=poff + 8 + 4 * nwg)
        dstr = [(dmin + field(sw, l * ws, ws, bits)) & M if act[l] else 0 for l in range(G)]
        f = [(dstr[l] * int(r[l])) & M if act[l] else 0 for l in range(G)]
        gap = [(gmin + field(gw, (l - 1) * wg, wg, bits)) & M if act[l] and l >= 1 else 0 for l in range(G)]
        F = np.cumsum(np.array(f, dtype=object))
        Gs = np.cumsum(np.array(gap, dtype=object))
        incl_r = np.cumsum(np.array([int(x) for x in r], dtype=object))
        start_abs = [(goff + int(incl_r[l]) - int(r[l])) & 0xFFFFFFFF for l in range(G)]
        st = [(base + (int(F[l]) - f[l]) + int(Gs[l])) & M for l in range(G)]
        v = [(st[l] - dstr[l] * start_abs[l]) & M for l in range(G)]
    else:
        w, doff = a1, a2
        words = np.frombuffer(s, np.uint32, count=((cnt - 1) * w + 31) // 32, offset=doff) if cnt > 1 else []
        delta = [base if l == 0 else (dmin + field(words, (l - 1) * w, w, bits)) & M for l in range(G)]
        v = list(np.cumsum(np.array([delta[l] if act[l] else 0 for l in range(G)], dtype=object)) % (M + 1))
        dstr = [0] * G
    return goff, next_off, cnt, [int(x) for x in r], [int(x) for x in v], [int(x) for x in dstr]


def run_unit(s, codec, n, bits, g0, e0, e1, out, mis_elems):
    """One wave's unit: groups from g0, elements [e0, e1); writes out[]."""
    R = 16 // (bits // 8)
    SPAN = 64 * R
    M = (1 << bits) - 1
    nr, ng = struct.unpack_from("<II", s, 0)
    g = g0
    while True:
        goff, next_off, cnt, r, v, dstr = group_values(s, codec, g, nr, n, bits)
        assert not (g == g0 and goff > e0)
        more = next_off < e1
        incl = np.cumsum(r)
        end_abs = [goff + int(incl[l]) for l in range(G)]
        start_abs = [end_abs[l] - r[l] for l in range(G)]
        act = [l < cnt for l in range(G)]
        assert goff + int(incl[cnt - 1]) == next_off
        a, bnd = max(e0, goff), min(e1, next_off)
        if a < bnd:
            mis = (mis_elems + a) % R          # the output pointer's misalignment at a
            carry = 1 + sum(1 for l in range(G) if act[l] and end_abs[l] <= a)
            W0 = a - mis
            while W0 < bnd:
                slot = np.zeros((R, G), dtype=np.int64)
                for l in range(G):
                    rel = start_abs[l] - W0
                    if act[l] and 0 <= rel < SPAN and start_abs[l] >= a:
                        slot[rel % R, rel // R] = l + 1
                last = [0] * G
                for l in range(G):
                    for i in range(R):
                        if slot[i, l]:
                            last[l] = slot[i, l]
                # last_nonzero_below: the highest lane below with a nonzero last
                nz = [l for l in range(G) if last[l]]
                cur = []
                for l in range(G):
                    below = [k for k in nz if k < l]
                    cur.append(last[below[-1]] if below else carry)
                if nz:
                    carry = last[nz[-1]]
                for l in range(G):
                    c = cur[l]
                    for i in range(R):
                        c = slot[i, l] if slot[i, l] else c
                        src = c - 1
                        assert 0 <= src < cnt, "a lane read a run outside the group"
                        p = W0 + R * l + i
                        val = v[src]
                        if codec == zf.DSTRIDE_BP:
                            val = (val + dstr[src] * (p & 0xFFFFFFFF)) & M
                        if a <= p < bnd:
                            out[p] = val
                W0 += SPAN
        if not more:
            return
        g += 1


def units(s, n, unit):
    """Output-balanced units as the planner cuts them: about `unit` outputs,
    cut at a group boundary when one is within another `unit`."""
    ng = struct.unpack_from("<I", s, 4)[0]
    gof = [struct.unpack_from("<I", s, 16 + 32 * k)[0] for k in range(ng)]
    e, gg, res = 0, 0, []
    while e < n:
        while gg + 1 < ng and gof[gg + 1] <= e:
            gg += 1
        target = e + unit
        if target >= n:
            e_end = n
        else:
            gb = gg + 1
            while gb < ng and gof[gb] < target:
                gb += 1
            e_end = gof[gb] if (gb < ng and gof[gb] <= target + unit) else target
        res.append((gg, e, e_end))
        e = e_end
    return res


CASES = [
    ("keys32", zf.DSTRIDE_BP, lambda: g.key_column(9000, 8, dtype=np.int32)),
    ("keys64", zf.DSTRIDE_BP, lambda: g.key_column(9000, 8, dtype=np.int64)),
    ("wrap64", zf.DSTRIDE_BP, lambda: (np.arange(3000, dtype=np.int64) * 977 + np.iinfo(np.int64).max - 3000)
     .astype(np.uint64).astype(np.int64)),
    ("rand64", zf.DSTRIDE_BP, lambda: g.rng(4).integers(-2**63, 2**63 - 1, size=1500, dtype=np.int64)),
    ("runs32", zf.RLE_DELTA_BP, lambda: g.sorted_runs_column(6000, 8, 5)),
    ("runs64", zf.RLE_DELTA_BP, lambda: g.sorted_runs_column(6000, 8, 5).astype(np.int64) * 3_000_000_001),
    ("delta32", zf.DELTA_BP, lambda: np.cumsum(g.rng(6).integers(-5, 9, size=3000)).astype(np.int32)),
]


@pytest.mark.parametrize("name,codec,make", CASES, ids=[c[0] for c in CASES])
def test_wave_model_every_cut(name, codec, make):
    x = make()
    bits = x.dtype.itemsize * 8
    n = len(x)
    # uneven chunks so that the last group of each is partial
    ce = [n // 3 + 7, n // 3 - 5, n - (n // 3 + 7) - (n // 3 - 5)]
    col = zf.Column.compress(x, codec, chunk_elems=ce, pinned=False)
    want = zo.decode(col.bytes())
    assert np.array_equal(want, x)
    M = (1 << bits) - 1
    for (s, c) in chunk_streams(col):
        ref = [int(t) & M for t in want[c["plain_off"] // (bits // 8):][:c["n_elems"]]]
        nr = struct.unpack_from("<I", s, 0)[0]
        assert nr % G != 0 or name == "delta32"   # a partial last group, as in the keys workloads
        for unit in (64, 100, 333, 4096):
            for mis in range(16 // (bits // 8)):
                out = [None] * c["n_elems"]
                for (g0, e0, e1) in units(s, c["n_elems"], unit):
                    run_unit(s, codec, c["n_elems"], bits, g0, e0, e1, out, mis)
                assert out == ref, (name, unit, mis)
