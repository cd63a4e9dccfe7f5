"""Host logic of bench.py that needs no GPU: the refusal of several GPUs and
the lookup of HBM traffic per kernel group in the committed counter summary."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_several_gpus_exit_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""


def test_group_traffic_sums_its_launches():
    ans, sd = bench.read_traffic("sdict_ans/ANS"), bench.read_traffic("sdict_ans/SDICT")
    if ans is None or sd is None:   # counters taken on other kernel sources
        assert bench.group_traffic("sdict_ans", "ANS+SDICT") is None
        return
    assert bench.group_traffic("sdict_ans", "ANS+SDICT") == ans + sd
    assert bench.group_traffic("fact", "SDICT") == bench.read_traffic("fact/SDICT")
    assert bench.group_traffic("fact", "NO_SUCH_KIND") is None
    assert bench.group_traffic("sdict_ans", "ANS+NO_SUCH_KIND") is None


def test_oracle_full_decode_and_compare():
    """The whole-output check: chunk ranges decoded on host threads equal the
    oracle's one-call decode, and a flipped byte is reported where it is."""
    import numpy as np
    import torch

    import oracle.zfo as zo
    from paper_2602_08190_amd import datagen as g
    from paper_2602_08190_amd import zf
    xs = [g.for_bp_column(300000, 1), g.text_column(700000, 3), g.fixed16_column(50000, 25, 2)]
    codecs = [zf.FOR_BP, zf.SDICT_BP, zf.DICT_BP]
    cols = [zf.Column.compress(x, c, chunk_bytes=(16 << 10, 256 << 10), seed=5 + i, pinned=False)
            for i, (x, c) in enumerate(zip(xs, codecs))]
    ref, secs = bench.cpu_baseline_all_cores(cols, 3)
    assert secs > 0
    for x, c, r in zip(xs, cols, ref):
        assert c.n_chunks > 3
        assert np.array_equal(r, zo.decode(c.bytes()).view(np.uint8).reshape(-1))
        assert np.array_equal(r, np.ascontiguousarray(x).view(np.uint8).reshape(-1))
    outs = [torch.from_numpy(np.ascontiguousarray(x).copy()) for x in xs]
    assert all(v["ok"] for v in bench.compare_outputs(torch, outs, ref, 2))
    outs[1][12345] ^= 1
    res = bench.compare_outputs(torch, outs, ref, 2)
    assert res[0]["ok"] and res[2]["ok"] and not res[1]["ok"]
    assert res[1]["first_mismatch"] == 12345 and res[1]["mismatching_bytes"] == 1


def test_host_description_and_manifest():
    import numpy as np
    d = bench.host_description(2)
    assert d["threads_used"] == 2 and "cpu_model" in d
    m = bench.sha256_manifest([np.arange(10, dtype=np.int32)], ["a"], 1)
    import hashlib
    assert m["a"] == hashlib.sha256(np.arange(10, dtype=np.int32).tobytes()).hexdigest()
    assert 1 <= bench.host_threads() <= 16
    assert bench.pct([1, 2, 3, 4, 5], 50) == 3
