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
