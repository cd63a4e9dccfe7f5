"""The autotuner's search logic on the CPU, on cost tables whose answers are
known: the grid sizes (the paper's Table 3 counts L x S x C candidates; on
wave64 hardware S runs 64..1024, five values), the coordinate search
against brute force on a separable convex table (it must land on the
optimum from every start) and on a two-basin table (it must stop at a local
optimum, in fewer probes than the grid), and the 1% tie rule."""
import itertools
import math

from paper_2602_08190_amd import autotune as A


def test_grid_sizes():
    sizes = {grp: len(A.UNITS[grp]) * len(A.WPB) for grp in A.UNITS}
    # FP: L (blocks per wave) x S (lanes per workgroup, 64..1024) x C (one 16-byte lane step)
    assert A.WPB == [1, 2, 4, 8, 16] and [64 * w for w in A.WPB] == [64, 128, 256, 512, 1024]
    assert sizes == {"FP": 25, "GP": 30, "PLAIN": 20, "NP": 15, "ANS": 5, "SDICT": 30}
    for kind, grp in A.GROUP.items():
        assert A.DEFAULT[grp] in A.UNITS[grp], kind


def grids():
    units, wpbs = A.UNITS["GP"], A.WPB
    for a, b in itertools.product(range(len(units)), range(len(wpbs))):
        yield units, wpbs, {(u, w): 1.0 + (math.log2(u) - math.log2(units[a])) ** 2
                            + 0.5 * (math.log2(w) - math.log2(wpbs[b])) ** 2
                            for u in units for w in wpbs}, (units[a], wpbs[b])


def test_coordinate_search_finds_the_optimum_of_a_convex_table():
    for units, wpbs, grid, best in grids():
        for start in itertools.product(units, wpbs):
            shape, t, probes = A.coordinate_search(lambda u, w: grid[(u, w)], units, wpbs, start)
            assert shape == best and t == grid[best]
            assert probes <= len(grid)


def test_coordinate_search_stops_at_a_local_optimum():
    units, wpbs = A.UNITS["GP"], A.WPB
    # two basins: a shallow one near the small corner, the deep one at the far corner
    def cost(u, w):
        i, j = units.index(u), wpbs.index(w)
        return min(2.0 + (i - 1) ** 2 + (j - 1) ** 2, 1.0 + (i - 5) ** 2 + (j - 4) ** 2)
    grid = {(u, w): cost(u, w) for u in units for w in wpbs}
    assert A.choose(grid) == (units[5], wpbs[4])
    shape, t, probes = A.coordinate_search(cost, units, wpbs, (units[0], wpbs[0]))
    assert shape == (units[1], wpbs[1]) and t == 2.0 and probes < len(grid)
    i, j = units.index(shape[0]), wpbs.index(shape[1])
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        if 0 <= i + di < len(units) and 0 <= j + dj < len(wpbs):
            assert cost(units[i + di], wpbs[j + dj]) >= t
    # from the default start it reaches the deep basin
    shape, t, _ = A.coordinate_search(cost, units, wpbs, (A.DEFAULT["GP"], 4))
    assert shape == (units[5], wpbs[4]) and t == 1.0


def test_tie_rule_prefers_the_smaller_workgroup():
    grid = {(1, 1): 1.009, (1, 2): 1.0, (2, 4): 1.005, (4, 1): 1.02}
    assert A.choose(grid) == (1, 1)                     # within 1%: smallest workgroup
    grid[(1, 1)] = 1.02
    assert A.choose(grid) == (1, 2)                     # (1, 1) and (4, 1) are now 2% off
    assert A.choose({(8, 4): 2.0, (16, 4): 2.0}) in ((8, 4), (16, 4))
