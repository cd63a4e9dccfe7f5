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
