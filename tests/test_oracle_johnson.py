"""Johnson's rule (Sec. 3.3) pinned to the paper's A/B example and to brute
force: Johnson (1954) proved the rule optimal for the two-machine flow shop
with an unlimited buffer between the stages."""
import numpy as np

from oracle import johnson as J


def test_paper_example(golden):
    ex = golden("johnson_example.json")
    a, b = ex["transfer"], ex["decode"]
    assert J.makespan([0, 1], a, b) == ex["makespan_A_then_B"]
    assert J.makespan([1, 0], a, b) == ex["makespan_B_then_A"]
    assert [ex["names"][i] for i in J.johnson_order(a, b)] == ex["johnson_order"]


def test_johnson_optimal_unbounded():
    r = np.random.default_rng(0)
    for trial in range(150):
        n = int(r.integers(1, 8))
        a = r.integers(1, 20, size=n).tolist()
        b = r.integers(1, 20, size=n).tolist()
        best, _ = J.brute_force_best(a, b)
        assert J.makespan(J.johnson_order(a, b), a, b) == best


def test_makespan_closed_forms():
    # one job: a + b; identical jobs: a + n*b when decode dominates, n*a + b otherwise
    assert J.makespan([0], [3], [5]) == 8
    assert J.makespan(list(range(4)), [2] * 4, [5] * 4) == 2 + 4 * 5
    assert J.makespan(list(range(4)), [5] * 4, [2] * 4) == 4 * 5 + 2
    # with one slot there is no overlap at all
    assert J.makespan([0, 1, 2], [1, 2, 3], [4, 5, 6], slots=1) == sum([1, 2, 3, 4, 5, 6])


def test_bounded_buffer_never_beats_unbounded():
    r = np.random.default_rng(1)
    for trial in range(60):
        n = int(r.integers(2, 7))
        a = r.integers(1, 20, size=n).tolist()
        b = r.integers(1, 20, size=n).tolist()
        o = J.johnson_order(a, b)
        assert J.makespan(o, a, b, slots=2) >= J.makespan(o, a, b)
        best2, _ = J.brute_force_best(a, b, slots=2)
        assert best2 >= J.brute_force_best(a, b)[0]
