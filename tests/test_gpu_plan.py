"""The plan's batch order (Sec. 3.3): zf_plan orders its batches by
Johnson's rule on its own (copy, decode) estimates; the order it reports
must equal the oracle's Johnson order of those estimates, including the
paper's A/B case built from real columns, and the staged decode must stay
bit-exact in every order."""
import sys

import numpy as np
import pytest

import oracle.zfo as zo
from oracle import johnson as J
from paper_2602_08190_amd import datagen as g
from paper_2602_08190_amd import zf

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def by_index(bs):
    n = len(bs)
    a, b = [0.0] * n, [0.0] * n
    for x in bs:
        a[x["index"]], b[x["index"]] = x["t_h2d_ms"], x["t_dec_ms"]
    return a, b


def staged_check(cols, **kw):
    plan = zf.Plan(cols, device=0, **kw)
    outs = zf.empty_outputs(cols)
    plan.transfer_and_decompress(outs)
    plan.sync()
    for i, (c, o) in enumerate(zip(cols, outs)):
        assert np.array_equal(o.cpu().numpy(), zo.decode(c.bytes())), f"column {i}"
    return plan


def test_paper_ab_case_on_real_batches():
    """Batch A: incompressible bytes (long copy, short decode); batch B: a
    long-run column (short copy, long decode).  Johnson runs B first."""
    log("plan A/B")
    a_bytes = np.frombuffer(np.random.default_rng(5).bytes(8 << 20), np.uint8).copy()
    b_runs = g.sorted_runs_column(1 << 23, 4096, 6)
    cols = [zf.Column.compress(a_bytes, zf.PLAIN, chunk_bytes=(8 << 20, 8 << 20)),
            zf.Column.compress(b_runs, zf.RLE_DELTA_BP, chunk_bytes=(32 << 20, 32 << 20))]
    plan = staged_check(cols, slot_bytes=8 << 20)
    bs = plan.batches()
    assert len(bs) == 2
    a, b = by_index(bs)
    assert a[0] > b[0] and a[1] < b[1], (a, b)   # the paper's shape of the two jobs
    assert [x["index"] for x in bs] == [1, 0] == J.johnson_order(a, b)
    assert J.makespan([1, 0], a, b) < J.makespan([0, 1], a, b)
    # column order keeps A first and still decodes right
    plan = staged_check(cols, slot_bytes=8 << 20, order=1)
    assert [x["index"] for x in plan.batches()] == [0, 1]


def test_mixed_table_order_equals_oracle():
    log("plan mixed")
    r = g.rng(12)
    xs = [g.for_bp_column(1 << 21, 3), g.sorted_runs_column(1 << 21, 64, 4),
          g.fixed16_column(1 << 18, 25, 5), g.text_column(6 << 20, 6),
          r.integers(0, 1 << 31, size=1 << 20, dtype=np.int64)]
    codecs = [zf.FOR_BP, zf.RLE_DELTA_BP, zf.DICT_BP, zf.SDICT_BP, zf.FOR_BP]
    cols = [zf.Column.compress(x, c, chunk_bytes=(64 << 10, 2 << 20), seed=7 + i)
            for i, (x, c) in enumerate(zip(xs, codecs))]
    for slot in (1 << 20, 3 << 20):
        plan = staged_check(cols, slot_bytes=slot)
        bs = plan.batches()
        assert len(bs) >= 4
        a, b = by_index(bs)
        assert [x["index"] for x in bs] == J.johnson_order(a, b)
        assert sum(x["n_chunks"] for x in bs) == sum(c.n_chunks for c in cols)
        assert sum(x["plain_bytes"] for x in bs) == sum(c.plain_bytes for c in cols)
