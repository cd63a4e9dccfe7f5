"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (image decode from HBM, per-kind launches, tiles from the tune cache),
for the FOR+bit-packing column (2^20 int32), the run-sorted date column
(2^26 int32 in 64 KiB chunks), the 1 GiB comment text as LZ77 in 64 KiB
chunks, and the 16-column fact table (8.5 GB, mixed codecs, uneven chunks).

At these sizes the oracle decodes a sample: the first and last chunk of every
column and 12 more drawn with a fixed seed, each compared element by element
with the GPU's output at that chunk's offset.  Every output is also compared
whole with the column it was encoded from (decode(encode(x)) == x holds at any
size); the whole-table comparison with the oracle's own decode is bench.py's
verify step."""
import numpy as np
import pytest

import bench
import oracle.zfo as zo
from paper_2602_08190_amd import zf

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def log(*a):
    print(*a, flush=True)


def check_full(cols, xs, names):
    import torch
    plan = zf.Plan(cols, device=0)
    img = zf.upload_image(plan, cols)
    outs = zf.empty_outputs(cols)
    plan.decompress_async(img, img.numel(), outs)
    plan.sync()
    r = np.random.default_rng(77)
    for c, x, o, name in zip(cols, xs, outs, names):
        ob = o.view(torch.uint8).reshape(-1)
        want = torch.from_numpy(np.ascontiguousarray(x).view(np.uint8).reshape(-1)).to(o.device)
        assert ob.numel() == want.numel(), name
        if not torch.equal(ob, want):
            bad = torch.nonzero(ob != want)[:4].flatten().tolist()
            raise AssertionError(f"{name}: GPU output differs from the encoded column at bytes {bad}")
        del want
        blob = c.bytes()
        cs = zo.chunks(blob)
        pick = sorted({0, len(cs) - 1, *r.integers(0, len(cs), size=12).tolist()})
        for i in pick:
            ref = np.ascontiguousarray(zo.decode_chunks(blob, i, 1)).view(np.uint8).reshape(-1)
            a, n = cs[i]["plain_off"], cs[i]["plain_len"]
            got = ob[a:a + n].cpu().numpy()
            assert np.array_equal(got, ref), f"{name}: chunk {i} differs from the oracle"
        log(f"{name}: {ob.numel()} bytes equal to the input; {len(pick)} chunks equal to the oracle")
    plan.free()


@pytest.mark.parametrize("kind,n", [("for", 1 << 20), ("rle", 1 << 26), ("lz", 1 << 30)])
def test_single_workloads_full_size(kind, n):
    log("full size", kind, n)
    cols, xs, names, _ = bench.single(kind, n)
    check_full(cols, xs, names)


def test_fact_table_full_size():
    log("full size fact table")
    from paper_2602_08190_amd import datagen as g
    cols, xs, names, _ = bench.fact_table(g.FACT_ROWS)
    check_full(cols, xs, names)
