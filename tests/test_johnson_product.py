"""The library's batch order (zf_johnson_order, the rule zf_plan applies to
its batches, Sec. 3.3) against the oracle's Johnson order on the same stage
times: the paper's A/B example, ties, random vectors, degenerate cases."""
import numpy as np
import pytest

from oracle import johnson as J
from paper_2602_08190_amd import zf


def test_paper_example(golden):
    ex = golden("johnson_example.json")
    a, b = ex["transfer"], ex["decode"]
    got = zf.johnson_order(a, b)
    assert [ex["names"][i] for i in got] == ex["johnson_order"]
    assert got == J.johnson_order(a, b)


def test_random_and_ties_equal_oracle():
    r = np.random.default_rng(7)
    for trial in range(400):
        n = int(r.integers(1, 40))
        # small integer times make ties (a == b, equal a, equal b) common
        hi = int(r.choice([3, 6, 50]))
        a = r.integers(0, hi, size=n).astype(float)
        b = r.integers(0, hi, size=n).astype(float)
        if trial % 3 == 0:
            a = a * 0.37 + r.random(n) * 1e-3
        assert zf.johnson_order(a, b) == J.johnson_order(a.tolist(), b.tolist()), (a, b)


def test_order_is_optimal_where_brute_force_reaches():
    r = np.random.default_rng(8)
    for trial in range(60):
        n = int(r.integers(1, 7))
        a = r.integers(1, 20, size=n).tolist()
        b = r.integers(1, 20, size=n).tolist()
        best, _ = J.brute_force_best(a, b)
        assert J.makespan(zf.johnson_order(a, b), a, b) == best


def test_degenerate():
    assert zf.johnson_order([], []) == []
    assert zf.johnson_order([5.0], [1.0]) == [0]
    # all jobs equal: index order
    assert zf.johnson_order([2.0] * 5, [2.0] * 5) == [0, 1, 2, 3, 4]
    with pytest.raises(zf.ZfError):
        zf.johnson_order([float("nan")], [1.0])
