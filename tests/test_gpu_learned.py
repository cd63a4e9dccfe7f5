"""Learned (codec, schedule) choice at small scale, end to end on the GPU:
timings from the pipeline, training in the library's kernels, and the gain
over choosing without the network (smallest stream, static rule, always
PLAIN) on held-out columns."""
import numpy as np
import pytest

from paper_2602_08190_amd import learn as Lr
from paper_2602_08190_amd import zf

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def test_learned_choice_beats_no_model(tmp_path):
    out = str(tmp_path / "d.npz")
    Lr.collect(range(0, 30), out, chunk_bytes=1 << 20, chunks_per_col=2)
    d = Lr.load([out])
    assert d["X"].shape == (60, 32)
    assert np.isfinite(d["T"]).sum() > 60 * 8
    tr, te = Lr.split(d)
    assert tr.sum() > 0 and te.sum() > 0
    mean, scale, params, hist, n = Lr.train(d, tr, epochs=400, batch=256, lr=3e-3)
    assert hist[-1][1] < 0.5 * hist[0][1]          # the loss falls
    ev_tr = Lr.evaluate(d, tr, Lr.predict(mean, scale, params, d["X"][tr]))
    ev_te = Lr.evaluate(d, te, Lr.predict(mean, scale, params, d["X"][te]))
    print("train", ev_tr)
    print("test", ev_te)
    # the gain over the library without the network (smallest stream at the
    # tile cache's schedule) and over always sending PLAIN
    for ev in (ev_tr, ev_te):
        assert ev["regret_mlp"] < ev["regret_smallest_stream_tuned"]
        assert ev["regret_mlp"] < ev["regret_always_plain_tuned"]
    # the weights drive ZF_AUTO in the encoder
    w = str(tmp_path / "w.bin")
    Lr.save_weights(w, mean, scale, params)
    x = Lr.chunk_data(2, 0, Lr.column_params(2), 1 << 20)
    col = zf.Column.compress(x, zf.AUTO, chunk_elems=[len(x) // 2, len(x) - len(x) // 2],
                             mlp_weights=w)
    plan = zf.Plan([col], device=0)
    outs = zf.empty_outputs([col])
    plan.transfer_and_decompress(outs)
    plan.sync()
    assert np.array_equal(outs[0].cpu().numpy(), x)
