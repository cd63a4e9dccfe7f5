"""Parameter sweeps of single codecs on the GPU, for the measurements the
paper reports per pattern (Sec. 5.2):

    python -m paper_2602_08190_amd.sweeps ans [--mib 1024]
    python -m paper_2602_08190_amd.sweeps text [--mib 1024]

ANS: decode throughput of a flag column ('A', 'N', 'R') from HBM, over the
frequency skew (the paper's L_RETURNFLAG-shaped workload made more and more
imbalanced) and over the chunk size (parallelism against ratio).
text: the comment-text column under LZ77 (64 KiB chunks, its largest), and
String-dictionary and String-dictionary | BP | ANS over the chunk size (the
per-chunk dictionary against parallelism), and both over one column
dictionary."""
import argparse
import json
import sys

import numpy as np

from . import datagen as g
from . import zf


def log(*a):
    print("[sweep]", *a, file=sys.stderr, flush=True)


def time_decode(torch, col, reps=10):
    plan = zf.Plan([col], device=0)
    img = zf.upload_image(plan, [col])
    outs = zf.empty_outputs([col])
    plan.decompress_async(img, img.numel(), outs)
    plan.sync()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        plan.decompress_async(img, img.numel(), outs)
    b.record(s)
    torch.cuda.synchronize()
    plan.sync()
    return a.elapsed_time(b) / reps, outs[0]


def ans(mib):
    import torch
    n = mib << 20
    rows = []
    skews = [(1 / 3, 1 / 3), (0.25, 0.5), (0.1, 0.8), (0.02, 0.96), (0.005, 0.99)]
    for pa, pn in skews:
        x = g.returnflag_column(n, pa, pn, 9)
        col = zf.Column.compress(x, zf.ANS)
        ms, out = time_decode(torch, col)
        assert np.array_equal(out[:1 << 16].cpu().numpy(), x[:1 << 16])
        comp = col.host_pointer()[1]
        rows.append({"sweep": "skew", "p": [round(pa, 3), round(pn, 3), round(1 - pa - pn, 3)],
                     "chunk_bytes": 65536, "ratio": round(n / comp, 3), "ms": round(ms, 4),
                     "plain_GBps": round(n / ms / 1e6, 1)})
        log(rows[-1])
        col.free()
    x = g.returnflag_column(n, 0.25, 0.5, 9)
    for kib in (4, 16, 64, 256, 1024):
        col = zf.Column.compress(x, zf.ANS, chunk_bytes=(kib << 10, kib << 10))
        ms, out = time_decode(torch, col)
        comp = col.host_pointer()[1]
        rows.append({"sweep": "chunk", "p": [0.25, 0.5, 0.25], "chunk_bytes": kib << 10,
                     "ratio": round(n / comp, 3), "ms": round(ms, 4), "plain_GBps": round(n / ms / 1e6, 1)})
        log(rows[-1])
        col.free()
    return {"workload": f"{mib} MiB flag column, decode from HBM, one kernel per launch", "rows": rows}


def text(mib):
    import torch
    n = mib << 20
    x = g.text_column(n, 2)
    rows = []

    def one(codec, name, kib):
        col = zf.Column.compress(x, codec, chunk_bytes=(kib << 10, kib << 10))
        ms, out = time_decode(torch, col)
        assert np.array_equal(out[:1 << 16].cpu().numpy(), x[:1 << 16])
        rows.append({"codec": name, "chunk_bytes": kib << 10, "ratio": round(n / col.host_pointer()[1], 3),
                     "ms": round(ms, 4), "plain_GBps": round(n / ms / 1e6, 1)})
        log(rows[-1])
        col.free()
    one(zf.LZ77, "LZ77", 64)
    for kib in (64, 256, 1024, 4096, 16384):
        one(zf.SDICT_BP, "SDICT_BP", kib)
    for kib in (256, 1024, 4096):
        one(zf.SDICT_ANS, "SDICT_ANS", kib)
    for kib in (64, 1024, 4096):
        one(zf.SDICT_COL, "SDICT_COL", kib)
    for kib in (64, 1024, 4096):
        one(zf.SDICT_COL_ANS, "SDICT_COL_ANS", kib)
    return {"workload": f"{mib} MiB comment text (Zipf 1.1 over 10,000 words), decode from HBM", "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["ans", "text"])
    ap.add_argument("--mib", type=int, default=1024)
    a = ap.parse_args()
    print(json.dumps(ans(a.mib) if a.what == "ans" else text(a.mib)))


if __name__ == "__main__":
    main()
