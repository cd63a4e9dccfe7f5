"""Tile autotuner: per kernel kind, time the decode of a representative
column over a power-of-two grid of tile shapes (the paper's <L,S,C> search
space, Sec. 5.5 and Table 3) and keep the fastest ("native config").

Two searches run on the same measurements:
  * brute force over the whole grid;
  * a coordinate search that starts from the default shape and moves one
    knob at a time to a neighbouring value while that improves the time
    (the monotone structure the paper exploits to cut its search to about
    ten probes).
Ties within 1% of the fastest go to the smaller workgroup.  The result is
the tile cache libzf reads (``tune_gfx950.json`` next to
libzf.so, or ``$ZF_TUNE_CACHE``); the kinds tuned in a run replace their
entries, the others are kept.

Two kinds of measurement:
  * --workload columns (default): one representative column per kind,
    decoded alone;
  * --workload fact: the batched fact table; each kind's time is taken inside
    the whole table's decode (events around its launch), with the other kinds
    at their cached tiles, so a tile is chosen for the kind's neighbours and
    uneven chunks as well.

    python -m paper_2602_08190_amd.autotune [--out PATH] [--scale 1.0]
                                            [--workload columns|fact] [--kinds K ...]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

from . import datagen as g
from . import zf

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_gfx950.json")

WPB = [1, 2, 4, 8, 16]                       # S = 64 .. 1024 lanes
UNITS = {
    "FP": [1, 2, 4, 8, 16],                  # L: 2048-value blocks per wave
    "GP": [256, 512, 1024, 2048, 4096, 8192],
    "PLAIN": [16384, 65536, 262144, 1048576],
    "NP": [4, 8, 16],                        # LZ77: output bytes per block
    "ANS": [0],                              # one chunk per wave, no unit knob
    "SDICT": [1024, 2048, 4096, 8192, 16384, 32768],  # output bytes per wave (whole groups, <= 63)
}
GROUP = {"FOR32": "FP", "FOR64": "FP", "DICT32": "FP", "DICT64": "FP", "DICT128": "FP",
         "RLE32": "GP", "RLE64": "GP", "LZ77": "NP", "PLAIN": "PLAIN", "F2I": "FP",
         "ANS": "ANS", "SDICT": "SDICT"}
DEFAULT = {"FP": 2, "GP": 4096, "PLAIN": 65536, "NP": 16, "ANS": 0, "SDICT": 4096}


def log(*a):
    print("[autotune]", *a, file=sys.stderr, flush=True)


def workloads(scale):
    """One representative column per kernel kind (seeded)."""
    n = lambda k: max(1 << 16, int(k * scale))  # noqa: E731
    r = g.rng(77)
    d32 = r.integers(-2**31, 2**31, size=256, dtype=np.int64).astype(np.int32)
    d64 = r.integers(-2**62, 2**62, size=256, dtype=np.int64)
    return {
        "FOR32": (g.for_bp_column(n(1 << 26), 0), zf.FOR_BP),
        "FOR64": (r.integers(100, 10**7, size=n(1 << 25), dtype=np.int64), zf.FOR_BP),
        "DICT32": (d32[r.integers(0, 256, size=n(1 << 26))], zf.DICT_BP),
        "DICT64": (d64[r.integers(0, 256, size=n(1 << 25))], zf.DICT_BP),
        "DICT128": (g.fixed16_column(n(1 << 24), 25, 5), zf.DICT_BP),
        "RLE32": (g.sorted_runs_column(n(1 << 26), 8, 1), zf.RLE_DELTA_BP),
        "RLE64": (g.sorted_runs_column(n(1 << 25), 8, 2, dtype=np.int64), zf.RLE_DELTA_BP),
        "LZ77": (g.text_column(n(1 << 30), 2), zf.LZ77),
        "F2I": (g.decimal_column(n(1 << 25), 5, 90000, 10500000), zf.F2I_BP),
        "ANS": (g.returnflag_column(n(1 << 28), 0.25, 0.5, 9), zf.ANS),
        "SDICT": (g.text_column(n(1 << 30), 2), zf.SDICT_COL),
        "PLAIN": (np.frombuffer(g.rng(5).bytes(n(1 << 28)), np.uint8), zf.PLAIN),
    }


class Timer:
    """Times one column's decode for a given tile shape; the device image is
    uploaded once (its layout does not depend on the tiles)."""

    def __init__(self, torch, col, reps=5):
        self.torch = torch
        self.col = col
        self.reps = reps
        self.out = zf.empty_outputs([col])
        self.img = zf.upload_image(zf.Plan([col], device=0), [col])
        self.cache = {}

    def __call__(self, kind, unit, wpb):
        key = (unit, wpb)
        if key in self.cache:
            return self.cache[key]
        T = self.torch
        plan = zf.Plan([self.col], device=0, tiles={kind: {"unit": unit, "waves_per_block": wpb}},
                       tune_cache=os.devnull)
        s = T.cuda.current_stream()
        plan.decompress_async(self.img, self.img.numel(), self.out)
        T.cuda.synchronize()
        a, b = T.cuda.Event(enable_timing=True), T.cuda.Event(enable_timing=True)
        a.record(s)
        for _ in range(self.reps):
            plan.decompress_async(self.img, self.img.numel(), self.out)
        b.record(s)
        T.cuda.synchronize()
        plan.sync()
        ms = a.elapsed_time(b) / self.reps
        self.cache[key] = ms
        return ms


def coordinate_search(measure, units, wpbs, start):
    """Move one knob at a time to a neighbouring grid value while it helps.
    Returns (best shape, best time, number of distinct probes)."""
    ui, wi = units.index(start[0]), wpbs.index(start[1])
    seen = {}

    def probe(a, b):
        if (a, b) not in seen:
            seen[(a, b)] = measure(units[a], wpbs[b])
        return seen[(a, b)]

    best = probe(ui, wi)
    improved = True
    while improved:
        improved = False
        for da, db in ((-1, 0), (1, 0), (0, -1), (0, 1)):
            a, b = ui + da, wi + db
            if 0 <= a < len(units) and 0 <= b < len(wpbs):
                t = probe(a, b)
                if t < best:
                    best, ui, wi, improved = t, a, b, True
    return (units[ui], wpbs[wi]), best, len(seen)


def choose(grid):
    """The brute-force winner of a {(unit, wpb): ms} grid: the smallest
    workgroup among the shapes within 1% of the fastest (whole workgroups
    retire together, so smaller ones refill a CU sooner when unit times vary,
    as they do on bigger inputs than the probe), then the faster."""
    fastest = min(grid.values())
    return min((k for k, v in grid.items() if v <= fastest * 1.01), key=lambda k: (k[1], grid[k]))


def report(kind, grid, plain, t0):
    grp = GROUP[kind]
    units = UNITS[grp]
    bu, bw = choose(grid)
    (cu, cw), ct, probes = coordinate_search(lambda u, w: grid[(u, w)], units, WPB, (DEFAULT[grp], 4))
    dflt = grid[(DEFAULT[grp], 4)]
    log(f"{kind:8s} best unit={bu} wpb={bw} {grid[(bu, bw)]:.3f} ms "
        f"({plain / grid[(bu, bw)] / 1e6:.0f} GB/s; default {dflt:.3f} ms; coordinate search "
        f"{probes} probes -> {ct:.3f} ms) in {time.time() - t0:.1f}s")
    return {
        "unit": bu, "waves_per_block": bw,
        "ms": round(grid[(bu, bw)], 4), "plain_GBps": round(plain / grid[(bu, bw)] / 1e6, 1),
        "default_ms": round(dflt, 4),
        "brute_force_candidates": len(grid),
        "coordinate_search": {"unit": cu, "waves_per_block": cw, "ms": round(ct, 4), "probes": probes},
        "grid_ms": {f"{u}x{w}": round(v, 4) for (u, w), v in sorted(grid.items())},
    }


def tune(scale=1.0, kinds=None):
    import torch
    assert torch.cuda.is_available(), "the autotuner measures on the GPU"
    zf.lib()
    res = {}
    for kind, (x, codec) in workloads(scale).items():
        if kinds and kind not in kinds:
            continue
        units = UNITS[GROUP[kind]]
        col = zf.Column.compress(x, codec)
        timer = Timer(torch, col)
        grid = {}
        t0 = time.time()
        for u in units:
            for w in WPB:
                grid[(u, w)] = timer(kind, u, w)
        res[kind] = report(kind, grid, col.plain_bytes, t0)
        res[kind]["measured"] = "column decoded alone"
        col.free()
    return res


def tune_fact(scale=1.0, kinds=None, reps=3):
    """Each kind's tile chosen on its in-step time in the fact table's decode."""
    import torch
    assert torch.cuda.is_available(), "the autotuner measures on the GPU"
    zf.lib()
    rows = max(1 << 16, int(g.FACT_ROWS * scale))
    cols = []
    for i, (name, kind, _) in enumerate(g.FACT_COLUMNS):
        x = g.fact_column(i, rows)
        cols.append(zf.Column.compress(x, getattr(zf, g.FACT_CODECS[kind]), chunk_bytes=(16 << 10, 4 << 20),
                                       seed=3000 + i))
        log(f"column {i} {name} ready")
    present = sorted({zf.kind_of_column(c) for c in cols} |
                     ({"ANS"} if any(zf.first_codec(c) in (zf.SDICT_ANS, zf.SDICT_COL_ANS) for c in cols) else set()))
    img = zf.upload_image(zf.Plan(cols, device=0), cols)
    outs = zf.empty_outputs(cols)
    plain = {k: sum(c.plain_bytes for c in cols if zf.kind_of_column(c) == k) for k in present}
    plain["ANS"] = plain.get("ANS") or plain.get("SDICT", 0)   # the stage feeds the String-dictionary text
    res = {}
    for kind in present:
        if kinds and kind not in kinds:
            continue
        units = UNITS[GROUP[kind]]
        grid = {}
        t0 = time.time()
        for u in units:
            for w in WPB:
                plan = zf.Plan(cols, device=0, tiles={kind: {"unit": u, "waves_per_block": w}})
                plan.profile(True)
                ts = []
                for _ in range(reps + 1):
                    plan.decompress_async(img, img.numel(), outs)
                    ts.append(plan.kind_ms()[kind])
                plan.sync()
                grid[(u, w)] = sorted(ts[1:])[len(ts[1:]) // 2]
        res[kind] = report(kind, grid, plain[kind], t0)
        res[kind]["measured"] = "inside the fact table's decode (%d rows)" % rows
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--kinds", nargs="*")
    ap.add_argument("--workload", default="columns", choices=["columns", "fact"])
    a = ap.parse_args()
    res = tune_fact(a.scale, a.kinds) if a.workload == "fact" else tune(a.scale, a.kinds)
    out = {"arch": "gfx950", "method": "brute force over the grid; coordinate search reported beside it",
           "kinds": {}}
    if os.path.exists(a.out):
        with open(a.out) as f:
            out = json.load(f)
    out["kinds"].update(res)
    with open(a.out, "w") as f:
        json.dump(out, f, indent=1)
    log("wrote", a.out, "kinds", sorted(res))


if __name__ == "__main__":
    main()
