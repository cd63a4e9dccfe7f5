"""Index maps of the paper's <L,S,C> schedules (Sec. 4), modelled in Python:
every output index is covered exactly once, for the paper's examples; then
the units zf's planner cuts real chunks into, checked against those maps
(Fully-Parallel) and against the invariants of its output-balanced
Group-Parallel and whole-group String-dictionary cuts."""


def fp_indices(L, S, C, n_blocks):
    """Fully-Parallel: block k, thread t, loop l, element c -> one index; the
    tile is L*S*C and successive loop steps are S*C apart."""
    out = []
    tile = L * S * C
    for k in range(n_blocks):
        for t in range(S):
            for l in range(L):
                for c in range(C):
                    out.append(k * tile + l * S * C + t * C + c)
    return out


def gp_groups(L, S, C, n_groups):
    """Group-Parallel: C threads (C/S blocks) share a group; a block steps
    over groups by L*S/C."""
    blocks_per_group = C // S
    stride = L * S // C
    owner = {}
    for blk in range(L):
        g = blk // blocks_per_group
        while g < n_groups:
            owner.setdefault(g, set()).add(blk)
            g += stride
    return owner


def test_fp_example_2_2_4():
    idx = fp_indices(2, 2, 4, 3)
    assert sorted(idx) == list(range(3 * 16))
    # thread 0 of block 0 touches [0..4) then [8..12): stride S*C = 8
    assert fp_indices(2, 2, 4, 1)[:8] == [0, 1, 2, 3, 8, 9, 10, 11]


def test_gp_example_8_4_16():
    owner = gp_groups(8, 4, 16, 4)
    assert owner[0] == owner[2] == {0, 1, 2, 3}
    assert owner[1] == owner[3] == {4, 5, 6, 7}


# ------------------------------------------------- the planner's own cutting
# The tests below read the units zf's planner cuts real chunks into
# (zf_chunk_units, host only) and check them against the maps above and
# against the invariants of its Group-Parallel and String-dictionary cuts.
import struct  # noqa: E402

import numpy as np  # noqa: E402
import pytest  # noqa: E402

import oracle.zfo as zo  # noqa: E402
from paper_2602_08190_amd import datagen as g  # noqa: E402
from paper_2602_08190_amd import zf  # noqa: E402

BLOCK = 2048  # values per FOR / bit-packing block (zf.h, ZF_FOR_BP)


def chunk_streams(col):
    blob = col.bytes()
    return [(c, bytes(blob[c["comp_off"]:c["comp_off"] + c["comp_len"]])) for c in zo.chunks(blob)]


@pytest.mark.parametrize("kind,dtype,es", [("FOR32", np.int32, 4), ("FOR64", np.int64, 8),
                                           ("DICT128", None, 16)])
@pytest.mark.parametrize("unit", [1, 2, 3, 8])
def test_fp_units_follow_the_fp_map(kind, dtype, es, unit):
    # a wavefront is S = 64 lanes, each owning C = 16 / es values per step,
    # stepping L = unit * 2048 / (64 C) times: its tile is unit blocks
    n = 5 * BLOCK + 700
    r = g.rng(3)
    if dtype is None:
        x = g.fixed16_column(n, seed=4)
        col = zf.Column.compress(x, zf.DICT_BP, chunk_elems=[n // 3, n - n // 3], pinned=False)
    else:
        x = r.integers(0, 1000, size=n).astype(dtype)
        col = zf.Column.compress(x, zf.FOR_BP, chunk_elems=[n // 3, n - n // 3], pinned=False)
    C = 16 // es
    L = unit * BLOCK // (64 * C)
    for ci, (c, _) in enumerate(chunk_streams(col)):
        units = zf.chunk_units(col, ci, tiles={kind: {"unit": unit}})
        assert all(u[0] == kind for u in units)
        m = c["n_elems"]
        model = fp_indices(L, 64, C, len(units))
        tile = L * 64 * C
        for j, (_, a, b, _c) in enumerate(units):
            want = sorted(i for i in model[j * tile:(j + 1) * tile] if i < m)
            assert list(range(a * BLOCK, min(m, (a + b) * BLOCK))) == want, (ci, j)
        assert sorted(i for i in model if i < m) == list(range(m))


def rle_group_starts(s):
    ng = struct.unpack_from("<I", s, 4)[0]
    return [struct.unpack_from("<I", s, 16 + 32 * k)[0] for k in range(ng)]


def check_gp_units(units, gof, n, unit):
    """Units {first group, first element, end element} tile [0, n) in order;
    the first group holds the first element; each unit but the last covers
    at least `unit` and at most 2 `unit` elements, and a unit that ends
    elsewhere than `unit` past its start ends at a group start."""
    ng = len(gof)
    e = 0
    for j, (g0, a, b) in enumerate(units):
        assert a == e and b > a
        assert gof[g0] <= a and (g0 + 1 == ng or gof[g0 + 1] > a)
        if b < n:
            assert unit <= b - a <= 2 * unit
            assert b - a == unit or b in gof
        e = b
    assert e == n


@pytest.mark.parametrize("unit", [64, 1000, 4096])
def test_gp_units_tile_each_chunk(unit):
    x = g.sorted_runs_column(60000, mean_run=6, seed=5)
    col = zf.Column.compress(x, zf.RLE_DELTA_BP, chunk_elems=[25000, 35000], pinned=False)
    for ci, (c, s) in enumerate(chunk_streams(col)):
        units = zf.chunk_units(col, ci, tiles={"RLE32": {"unit": unit}})
        assert {u[0] for u in units} == {"RLE32"}
        check_gp_units([u[1:] for u in units], rle_group_starts(s), c["n_elems"], unit)


def test_tree_units_tile_starts_then_output():
    x = g.orderkey_column(40000, seed=6)
    col = zf.Column.compress(x, zf.DSTREE, chunk_elems=[40000], pinned=False)
    (c, s), = chunk_streams(col)
    unit = 512
    units = zf.chunk_units(col, 0, tiles={"RLE32": {"unit": unit}, "TREE": {"unit": unit}})
    kinds = [u[0] for u in units]
    k = kinds.index("TREE")
    assert set(kinds[:k]) == {"RLE32"} and set(kinds[k:]) == {"TREE"}
    R, ngB, Q, ngA = struct.unpack_from("<IIII", s, 0)
    b_off = struct.unpack_from("<I", s, 24)[0]
    starts_gof = [struct.unpack_from("<I", s, 32 + 32 * j)[0] for j in range(ngA)]
    out_gof = [struct.unpack_from("<I", s, b_off + 16 * j)[0] for j in range(ngB)]
    check_gp_units([u[1:] for u in units[:k]], starts_gof, R, unit)
    check_gp_units([u[1:] for u in units[k:]], out_gof, c["n_elems"], unit)


@pytest.mark.parametrize("unit", [256, 4096, 1 << 20])
def test_sdict_units_are_whole_groups(unit):
    text = g.text_column(300_000, seed=7)
    col = zf.Column.compress(text, zf.SDICT_COL_ANS, chunk_elems=[100_000, 200_000], pinned=False)
    for ci, (c, s) in enumerate(chunk_streams(col)):
        units = zf.chunk_units(col, ci, tiles={"SDICT": {"unit": unit}})
        ans = [u for u in units if u[0] == "ANS"]
        sd = [u for u in units if u[0] == "SDICT"]
        assert units == ans + sd and len(ans) >= 1
        ng = struct.unpack_from("<I", s, 8)[0]
        gof = [struct.unpack_from("<I", s, 16 + 4 * j)[0] for j in range(ng)] + [c["plain_len"]]
        at = 0
        for _, a, b, _c in sd:
            assert a == at and a < b and b - a <= 63
            # as few groups as reach `unit` output bytes (or 63 groups)
            assert b - a == 1 or gof[b - 1] - gof[a] < unit
            if b < ng:
                assert gof[b] - gof[a] >= unit or b - a == 63
            at = b
        assert at == ng


def test_plain_and_whole_chunk_units():
    x = np.frombuffer(g.rng(8).bytes(100_000), np.uint8).copy()
    col = zf.Column.compress(x, zf.PLAIN, chunk_elems=[100_000], pinned=False)
    assert zf.chunk_units(col, 0, tiles={"PLAIN": {"unit": 16384}}) == \
        [("PLAIN", a, min(a + 16384, 100_000), 0) for a in range(0, 100_000, 16384)]
    lz = zf.Column.compress(x, zf.LZ77, chunk_elems=[60_000, 40_000], pinned=False)
    assert [zf.chunk_units(lz, i) for i in range(2)] == [[("LZ77", 0, 0, 0)]] * 2
    with pytest.raises(zf.ZfError):
        zf.chunk_units(lz, 2)
