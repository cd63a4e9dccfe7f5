"""Learned (codec, schedule) selection: data, training, evaluation.

* collect: synthetic columns of five families (uniform ints, Zipf ints,
  sorted ints with runs, low-cardinality ints, Zipf text), cut into chunks; for
  each chunk, the 32 statistics (zf_chunk_features) and, for every applicable
  (codec, schedule), the transfer + decode time the pipeline itself measures
  (zf_transfer_and_decompress timing: copy events + decode events), median of
  three runs.
* train: the 32-64-64-24 network on log time, masked squared error on the
  measured output, Adam; every forward/backward/update runs in the library's
  HIP kernels (zf_mlp_grad, zf_mlp_adam).
* evaluate: regret of the network's choice against exhaustive measured search
  on held-out columns, next to the choice without a model.

    python -m paper_2602_08190_amd.learn collect --cols 0 64 --out d0.npz
    python -m paper_2602_08190_amd.learn train --data d*.npz --weights w.bin --report r.json
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import datagen as g
from . import zf

FAMILIES = ["uniform", "zipf", "runs", "lowcard", "text"]
CODECS = [zf.PLAIN, zf.FOR_BP, zf.DICT_BP, zf.DELTA_BP, zf.RLE_DELTA_BP, zf.LZ77]
N_COLS = 256
CHUNKS_PER_COL = 16
CHUNK_BYTES = 8 << 20            # every chunk holds 8 MiB of plain data
LZ_SUB = [8192, 16384, 32768, 65536]
UNIT = {"FP": [1, 2, 4, 8], "GP": [1024, 2048, 4096, 8192], "PLAIN": [16384, 65536, 262144, 1048576]}
DEFAULT_SCHED = {zf.PLAIN: 1, zf.FOR_BP: 1, zf.DICT_BP: 1, zf.DELTA_BP: 2, zf.RLE_DELTA_BP: 2,
                 zf.LZ77: 3}
TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_gfx950.json")


def tuned_sched(path=TUNE_CACHE):
    """Schedule index of each codec under the autotuner's tile cache (what the
    library runs when no model picks a schedule); LZ77 keeps 64 KiB chunks."""
    try:
        with open(path) as f:
            kinds = json.load(f)["kinds"]
    except (OSError, ValueError, KeyError):
        return dict(DEFAULT_SCHED)

    def near(grp, kind):
        u = kinds.get(kind, {}).get("unit", UNIT[grp][0])
        return int(np.argmin([abs(math.log2(max(u, 1)) - math.log2(x)) for x in UNIT[grp]]))
    return {zf.PLAIN: near("PLAIN", "PLAIN"), zf.FOR_BP: near("FP", "FOR32"),
            zf.DICT_BP: near("FP", "DICT32"), zf.DELTA_BP: near("GP", "RLE32"),
            zf.RLE_DELTA_BP: near("GP", "RLE32"), zf.LZ77: 3}


def log(*a):
    print("[learn]", *a, file=sys.stderr, flush=True)


# --------------------------------------------------------------- columns
def family_of(i):
    """52 uniform, 51 each of the others, interleaved."""
    return FAMILIES[i % 5]


def column_params(i):
    r = g.rng(1000 + i)
    fam = family_of(i)
    if fam == "uniform":
        return dict(fam=fam, w=int(r.integers(4, 32)), lo=int(r.integers(-2**30, 2**30)))
    if fam == "zipf":
        return dict(fam=fam, s=float(r.uniform(0.5, 2.0)),
                    vals=r.integers(-2**31, 2**31, size=1 << 16, dtype=np.int64).astype(np.int32))
    if fam == "runs":
        return dict(fam=fam, mean=float(math.exp(r.uniform(0, math.log(4096)))),
                    cycle=int(math.exp(r.uniform(math.log(16), math.log(1 << 20)))))
    if fam == "lowcard":
        k = int(r.integers(2, 257))
        return dict(fam=fam, vals=r.integers(-2**31, 2**31, size=k, dtype=np.int64).astype(np.int32))
    return dict(fam=fam, s=float(r.uniform(0.9, 1.5)),
                vocab=int(math.exp(r.uniform(math.log(1000), math.log(20000)))))


_zipf_cdf = {}


_text = {}


def chunk_data(i, j, p, chunk_bytes=CHUNK_BYTES):
    """Chunk j of column i (chunk_bytes of plain data), on its own seed."""
    r = g.rng((1000 + i) * 100 + j)
    n = chunk_bytes // 4
    fam = p["fam"]
    if fam == "uniform":
        return (p["lo"] + r.integers(0, 1 << p["w"], size=n, dtype=np.int64)).astype(np.int32)
    if fam == "zipf":
        key = ("z", round(p["s"], 6))
        if key not in _zipf_cdf:
            _zipf_cdf[key] = g.zipf_cdf(1 << 16, p["s"])
        ranks = np.searchsorted(_zipf_cdf[key], r.random(n))
        return p["vals"][np.minimum(ranks, (1 << 16) - 1)]
    if fam == "runs":
        runs = g.run_lengths_geometric(n, p["mean"], (1000 + i) * 100 + j)
        start = int(r.integers(0, p["cycle"]))
        v = ((start + np.arange(runs.size, dtype=np.int64)) % p["cycle"]).astype(np.int32)
        return np.repeat(v, runs)
    if fam == "lowcard":
        return p["vals"][r.integers(0, len(p["vals"]), size=n)]
    if i not in _text:
        _text.clear()
        _text[i] = g.TextSource(1000 + i, vocab=p["vocab"], s=p["s"])
    rows = chunk_bytes // 40 + 16  # rows are at least 40 bytes
    return _text[i].rows(j * rows, (j + 1) * rows)[:chunk_bytes].copy()


def kind_group(codec):
    if codec in (zf.FOR_BP, zf.DICT_BP):
        return "FP"
    if codec in (zf.DELTA_BP, zf.RLE_DELTA_BP):
        return "GP"
    if codec == zf.PLAIN:
        return "PLAIN"
    return "NP"


def applicable(codec, x):
    dt = zf.dtype_of(x)
    if codec in (zf.FOR_BP, zf.DELTA_BP, zf.RLE_DELTA_BP):
        return dt in (zf.I32, zf.I64)
    if codec == zf.DICT_BP:
        return dt != zf.BYTES
    return True


def time_column(col, tiles, reps=3):
    """Median (h2d_ms + decode_ms) of the pipeline's own timing."""
    plan = zf.Plan([col], device=0, slot_bytes=max(1 << 20, col.host_pointer()[1]), tiles=tiles,
                   tune_cache=os.devnull)
    outs = zf.empty_outputs([col])
    ts = []
    for _ in range(reps + 1):
        plan.transfer_and_decompress(outs)
        t = plan.sync()
        ts.append(t["h2d_ms"] + t["decode_ms"])
    plan.free()
    return float(np.median(ts[1:])), outs[0]


def collect(cols, out_path, check=True, chunk_bytes=CHUNK_BYTES, chunks_per_col=CHUNKS_PER_COL):
    import torch
    assert torch.cuda.is_available(), "timings are measured on the GPU"
    zf.lib()
    X, T, S, ids = [], [], [], []
    t0 = time.time()
    for i in cols:
        p = column_params(i)
        for j in range(chunks_per_col):
            x = chunk_data(i, j, p, chunk_bytes)
            feats = zf.chunk_features(x)
            times = np.full(24, np.nan)
            sizes = np.full(24, np.nan)
            for ci, codec in enumerate(CODECS):
                if not applicable(codec, x):
                    continue
                grp = kind_group(codec)
                if codec == zf.LZ77:
                    variants = []
                    for s, sub in enumerate(LZ_SUB):
                        per = sub // x.itemsize if x.ndim == 1 else sub // 16
                        ce = [per] * (len(x) // per) + ([len(x) % per] if len(x) % per else [])
                        variants.append((s, zf.Column.compress(x, codec, chunk_elems=ce), None))
                else:
                    try:
                        col = zf.Column.compress(x, codec, chunk_elems=[len(x)])
                    except zf.ZfError:
                        continue  # e.g. too many distinct values for DICT_BP
                    name = {"FP": "FP", "GP": "GP", "PLAIN": "PLAIN"}[grp]
                    variants = [(s, col, {name: {"unit": UNIT[grp][s]}}) for s in range(4)]
                for s, col, tiles in variants:
                    ms, out = time_column(col, tiles)
                    if check and s == 0:
                        got = out[:4096].cpu().numpy()
                        assert np.array_equal(got, x[:4096]), "decode mismatch while collecting"
                    times[ci * 4 + s] = ms
                    sizes[ci * 4 + s] = col.host_pointer()[1]
                for _, col, _ in variants:
                    col.free()
            X.append(feats)
            T.append(times)
            S.append(sizes)
            ids.append((i, j))
        log(f"column {i} ({p['fam']}) done, {time.time() - t0:.0f}s")
        # written after every column, so a cut-off run keeps what it measured
        np.savez(out_path, X=np.array(X, np.float32), T=np.array(T), S=np.array(S),
                 ids=np.array(ids, np.int32), fam=np.array([family_of(i) for i, _ in ids]))


# ----------------------------------------------------------------- train
def load(paths):
    parts = [np.load(p) for p in paths]
    return {k: np.concatenate([q[k] for q in parts]) for k in ("X", "T", "S", "ids", "fam")}


def split(d, test_every=5):
    """Column-level split: columns with (id // 5) % 5 == 4 are held out (one
    column in five of every family)."""
    test = (d["ids"][:, 0] // 5) % test_every == test_every - 1
    return ~test, test


def he_uniform(seed, sizes=(32, 64, 64, 24)):
    """Flat initial parameters: W ~ U(+-sqrt(6/fan_in)), zero biases."""
    r = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = math.sqrt(6.0 / a)
        parts.append(r.uniform(-lim, lim, size=(b, a)).reshape(-1))
        parts.append(np.zeros(b))
    return np.concatenate(parts).astype(np.float32)


def train(d, train_mask, epochs=150, batch=2048, lr=2e-3, seed=0):
    import torch
    Xc = d["X"][train_mask].astype(np.float64)
    mean = Xc.mean(axis=0)
    std = Xc.std(axis=0)
    scale = np.where(std > 1e-6, 1.0 / np.maximum(std, 1e-6), 0.0)
    rows, ks, ts = [], [], []
    for x, t in zip(d["X"][train_mask], d["T"][train_mask]):
        z = (x - mean) * scale
        for k in np.flatnonzero(np.isfinite(t)):
            rows.append(z)
            ks.append(k)
            ts.append(math.log(t[k] * 1000.0))  # log microseconds
    Xs = np.array(rows, np.float32)
    K = np.array(ks, np.int32)
    Tt = np.array(ts, np.float32)
    n = len(K)
    dev = torch.device("cuda")
    P = torch.from_numpy(he_uniform(seed)).to(dev)
    Mo, Vo, G = torch.zeros_like(P), torch.zeros_like(P), torch.empty_like(P)
    L = torch.empty(1, dtype=torch.float32, device=dev)
    batch = min(batch, n)
    W = torch.empty(zf.mlp_grad_work_bytes(batch) // 4 + 1, dtype=torch.float32, device=dev)
    r = np.random.default_rng(seed)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = r.permutation(n)
        Xd = torch.from_numpy(Xs[perm]).to(dev)
        Kd = torch.from_numpy(K[perm]).to(dev)
        Td = torch.from_numpy(Tt[perm]).to(dev)
        for a in range(0, n - batch + 1, batch):
            step += 1
            zf.mlp_grad(P, Xd[a:a + batch], Kd[a:a + batch], Td[a:a + batch], G, L, W)
            zf.mlp_adam(P, G, Mo, Vo, step, lr=lr)
        if ep % 10 == 0 or ep == epochs - 1:
            hist.append((ep, float(L.item())))
    return mean.astype(np.float32), scale.astype(np.float32), P.cpu().numpy(), hist, n


def predict(mean, scale, params, X):
    import torch
    dev = torch.device("cuda")
    Z = ((X - mean) * scale).astype(np.float32)
    Pd = torch.from_numpy(params).to(dev)
    Xd = torch.from_numpy(Z).to(dev)
    Y = torch.empty((len(Z), 24), dtype=torch.float32, device=dev)
    zf.mlp_forward(Pd, Xd, Y)
    return Y.cpu().numpy()


def save_weights(path, mean, scale, params):
    with open(path, "wb") as f:
        f.write(b"ZFMLP1\0\0")
        f.write(np.asarray(mean, "<f4").tobytes())
        f.write(np.asarray(scale, "<f4").tobytes())
        f.write(np.asarray(params, "<f4").tobytes())


STATIC = {"uniform": zf.FOR_BP, "zipf": zf.DICT_BP, "runs": zf.RLE_DELTA_BP, "lowcard": zf.DICT_BP,
          "text": zf.LZ77}


def evaluate(d, mask, Y, margin=0.05):
    T = d["T"][mask]
    S = d["S"][mask]
    fams = d["fam"][mask]
    best = np.nanmin(T, axis=1)
    Ym = np.where(np.isfinite(T), Y, np.inf)
    pick = np.argmin(Ym, axis=1)
    chosen = T[np.arange(len(T)), pick]
    # fallback: when the two best predictions are within `margin` (log), both
    # are measured and the faster one is kept
    order = np.argsort(Ym, axis=1)
    close = (Ym[np.arange(len(T)), order[:, 1]] - Ym[np.arange(len(T)), order[:, 0]]) < margin
    fb = np.where(close, np.minimum(chosen, T[np.arange(len(T)), order[:, 1]]), chosen)

    def pick_codec(codec_of_row, sched_of_codec):
        idx = np.array([CODECS.index(c) * 4 + sched_of_codec[c] for c in codec_of_row])
        return T[np.arange(len(T)), idx]

    def smallest_stream(sched):
        idx = []
        for row in S:
            cands = [(row[c * 4 + sched[CODECS[c]]], c) for c in range(6)
                     if np.isfinite(row[c * 4 + sched[CODECS[c]]])]
            c = min(cands)[1]
            idx.append(c * 4 + sched[CODECS[c]])
        return T[np.arange(len(T)), np.array(idx)]

    reg = lambda t: float(np.sum(t) / np.sum(best) - 1.0)  # noqa: E731
    tuned = tuned_sched()
    fam_reg = {f: {"mlp": float(np.sum(chosen[fams == f]) / np.sum(best[fams == f]) - 1.0),
                   "smallest_stream_tuned": float(np.sum(smallest_stream(tuned)[fams == f])
                                                  / np.sum(best[fams == f]) - 1.0)}
               for f in np.unique(fams)}
    return {"chunks": int(len(T)), "regret_mlp": reg(chosen), "regret_mlp_fallback": reg(fb),
            "fallback_rate": float(np.mean(close)),
            # the library without a model: the smallest stream, with the tile
            # cache's schedule (tuned) or the fixed default schedule
            "regret_smallest_stream_tuned": reg(smallest_stream(tuned)),
            "regret_smallest_stream_default": reg(smallest_stream(DEFAULT_SCHED)),
            "regret_static_rule_tuned": reg(pick_codec([STATIC[f] for f in fams], tuned)),
            "regret_always_plain_tuned": reg(pick_codec([zf.PLAIN] * len(T), tuned)),
            "exact_best_rate": float(np.mean(pick == np.nanargmin(T, axis=1))),
            "total_best_ms": float(np.sum(best)), "total_mlp_ms": float(np.sum(chosen)),
            "per_family": fam_reg, "tuned_schedule": {str(k): v for k, v in tuned.items()}}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd")
    c = sub.add_parser("collect")
    c.add_argument("--cols", nargs=2, type=int, default=[0, N_COLS])
    c.add_argument("--out", required=True)
    t = sub.add_parser("train")
    t.add_argument("--data", nargs="+", required=True)
    t.add_argument("--weights", required=True)
    t.add_argument("--report", required=True)
    t.add_argument("--epochs", type=int, default=150)
    a = ap.parse_args()
    if a.cmd == "collect":
        collect(range(*a.cols), a.out)
    elif a.cmd == "train":
        d = load(a.data)
        tr, te = split(d)
        t0 = time.time()
        mean, scale, params, hist, n = train(d, tr, epochs=a.epochs)
        train_s = time.time() - t0
        save_weights(a.weights, mean, scale, params)
        rep = {"train_samples": n, "train_chunks": int(tr.sum()), "test_chunks": int(te.sum()),
               "train_seconds": round(train_s, 1), "loss_history": hist,
               "test": evaluate(d, te, predict(mean, scale, params, d["X"][te])),
               "train": evaluate(d, tr, predict(mean, scale, params, d["X"][tr]))}
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
        print(json.dumps(rep["test"]))


if __name__ == "__main__":
    main()
