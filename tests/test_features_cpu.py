"""Chunk statistics of the cost model, re-derived with numpy on the CPU."""
import numpy as np

from paper_2602_08190_amd import datagen as g
from paper_2602_08190_amd import zf


def test_integer_features():
    x = g.sorted_runs_column(50000, 8, 1)
    f = zf.chunk_features(x)
    assert f[0] == np.float32(np.log2(50001))
    assert f[1] == 2.0 and f[2] == 0.0
    assert f[4] == float(int(x.max() - x.min()).bit_length())
    u, c = np.unique(x, return_counts=True)
    assert abs(f[7] - np.log2(len(u) + 1)) < 1e-5
    assert abs(f[9] - c.max() / len(x)) < 1e-6
    runs = 1 + np.count_nonzero(np.diff(x))
    assert abs(f[14] - runs / len(x)) < 1e-6
    assert abs(f[13] - np.mean(np.diff(x.astype(np.int64)) >= 0)) < 1e-6
    p = c / len(x)
    assert abs(f[12] - float(-(p * np.log2(p)).sum())) < 1e-3


def test_text_features():
    x = g.text_column(50000, seed=3)
    f = zf.chunk_features(x)
    assert f[2] == 1.0
    sp = np.isin(x, [32, 10])
    assert abs(f[21] - sp.mean()) < 1e-6
    assert f[22] > 0.2          # Zipf text repeats most 4-byte strings


def test_sample_is_bounded():
    x = g.uniform_i32(1 << 20, 0, 1 << 12, 1)
    f = zf.chunk_features(x)
    assert f[3] == np.float32(np.log2(65537))
    assert f[6] == 12.0


# ------------------------------------------------ the committed cost model
import json
import os

import oracle.mlp as om
import oracle.zfo as zo
from paper_2602_08190_amd import learn as Lr

PKG = os.path.dirname(os.path.abspath(zf.__file__))
WEIGHTS = os.path.join(PKG, "cost_model_gfx950.bin")
REPORT = os.path.join(PKG, "cost_model_gfx950.json")


def _read_weights(path):
    raw = open(path, "rb").read()
    assert raw[:8] == b"ZFMLP1\0\0"
    v = np.frombuffer(raw[8:], "<f4")
    assert v.size == 32 + 32 + om.n_params()
    return v[:32], v[32:64], v[64:]


def test_committed_cost_model_meets_its_regret_bound():
    """The shipped network was trained on the pipeline's own timings; on
    held-out columns its choice is within 5% of exhaustive search and better
    than the library without it."""
    _read_weights(WEIGHTS)
    r = json.load(open(REPORT))
    t = r["test"]
    assert r["train_samples"] > 50000 and t["chunks"] >= 500
    assert t["regret_mlp"] <= 0.05
    assert t["regret_mlp"] < t["regret_smallest_stream_tuned"]
    assert t["regret_mlp"] < t["regret_always_plain_tuned"]


def test_encoder_choice_follows_the_fp64_network():
    """ZF_AUTO's host forward pass (float32) picks the same (codec, schedule)
    as the FP64 oracle network on the same statistics, wherever the oracle's
    two best scores are not near-ties."""
    mean, scale, params = _read_weights(WEIGHTS)
    checked = 0
    for i in range(10):
        p = Lr.column_params(i)
        x = Lr.chunk_data(i, 0, p, 1 << 18)
        f = zf.chunk_features(x).astype(np.float64)
        y = om.forward(params.astype(np.float64), ((f - mean) * scale)[None, :])[1][0]
        allowed = [c for c in range(24) if Lr.applicable(Lr.CODECS[c // 4], x)]
        ys = sorted((y[c], c) for c in allowed)
        col = zf.Column.compress(x, zf.AUTO, chunk_elems=[len(x)], mlp_weights=WEIGHTS,
                                 pinned=False)
        codecs = {c["codec"] for c in zo.chunks(col.bytes())}
        assert (zo.decode(col.bytes()) == x).all()
        if ys[1][0] - ys[0][0] < 1e-3:
            continue
        best = ys[0][1]
        if Lr.CODECS[best // 4] == zf.DICT_BP and len(np.unique(x)) > (1 << 16):
            continue  # no dictionary for this chunk: the encoder skips DICT_BP
        assert codecs == {Lr.CODECS[best // 4]}, (i, p["fam"], best, codecs)
        checked += 1
    assert checked >= 6
