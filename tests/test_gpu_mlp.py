"""Cost-model kernels through the C ABI against the FP64 oracle: forward,
gradients (relative error per tensor <= 1e-5), one Adam step (<= 1e-6),
bit-reproducible reductions, and a training run whose loss falls."""
import numpy as np
import pytest

from oracle import mlp as M
from paper_2602_08190_amd import zf

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def batch(seed, n):
    r = np.random.default_rng(seed)
    X = r.normal(size=(n, 32)).astype(np.float32)
    k = r.integers(0, 24, size=n).astype(np.int32)
    t = r.normal(size=n).astype(np.float32)
    return X, k, t


def tensors(flat):
    out, at = [], 0
    for s in M.shapes():
        n = int(np.prod(s))
        out.append((at, at + n))
        at += n
    return [flat[a:b] for a, b in out]


@pytest.mark.parametrize("n", [1, 63, 64, 200, 4096])
def test_forward_and_grad_match_oracle(n):
    import torch
    p32 = M.he_uniform(5).astype(np.float32)
    X, k, t = batch(n, n)
    P, Xd, Kd, Td = dev(p32, np.float32), dev(X, np.float32), dev(k, np.int32), dev(t, np.float32)
    Y = torch.empty((n, 24), dtype=torch.float32, device="cuda")
    zf.mlp_forward(P, Xd, Y)
    _, yref = M.forward(p32.astype(np.float64), X.astype(np.float64))
    assert np.abs(Y.cpu().numpy() - yref).max() <= 1e-5 * max(1.0, np.abs(yref).max())
    G = torch.empty(M.n_params(), dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    W = torch.empty(zf.mlp_grad_work_bytes(n) // 4, dtype=torch.float32, device="cuda")
    zf.mlp_grad(P, Xd, Kd, Td, G, L, W)
    lref, gref = M.grad(p32.astype(np.float64), X.astype(np.float64), k, t.astype(np.float64))
    g = G.cpu().numpy().astype(np.float64)
    for a, b in zip(tensors(g), tensors(gref)):
        if np.linalg.norm(b) > 0:
            assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-5
        else:
            assert np.abs(a).max() == 0
    assert abs(L.item() - lref) <= 1e-5 * lref
    # bit-reproducible
    G2 = torch.empty_like(G)
    zf.mlp_grad(P, Xd, Kd, Td, G2, L, W)
    assert torch.equal(G, G2)


def test_adam_step_matches_oracle():
    import torch
    r = np.random.default_rng(1)
    p = r.normal(size=M.n_params()).astype(np.float32)
    g = r.normal(size=M.n_params()).astype(np.float32)
    m = (r.normal(size=M.n_params()) * 0.1).astype(np.float32)
    v = np.abs(r.normal(size=M.n_params()) * 0.1).astype(np.float32)
    P, G, Md, Vd = (dev(a, np.float32) for a in (p, g, m, v))
    zf.mlp_adam(P, G, Md, Vd, 7, lr=1e-3)
    pr, mr, vr = M.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                        v.astype(np.float64), 7, lr=1e-3)
    assert np.linalg.norm(P.cpu().numpy() - pr) / np.linalg.norm(pr) <= 1e-6
    assert np.linalg.norm(Md.cpu().numpy() - mr) / np.linalg.norm(mr) <= 1e-6


def test_bad_index_gives_nan_loss():
    import torch
    p32 = M.he_uniform(2).astype(np.float32)
    X, k, t = batch(3, 10)
    k[4] = 24
    P, Xd, Kd, Td = dev(p32, np.float32), dev(X, np.float32), dev(k, np.int32), dev(t, np.float32)
    G = torch.empty(M.n_params(), dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    W = torch.empty(zf.mlp_grad_work_bytes(10) // 4, dtype=torch.float32, device="cuda")
    zf.mlp_grad(P, Xd, Kd, Td, G, L, W)
    assert np.isnan(L.item())
    with pytest.raises(zf.ZfError):
        zf.mlp_grad(P, Xd, Kd, Td, G, L, W[:10])


def test_gpu_training_reduces_loss():
    import torch
    r = np.random.default_rng(0)
    n = 2048
    X = r.normal(size=(n, 32)).astype(np.float32)
    true = (r.normal(size=(32, 24)) * 0.3)
    k = r.integers(0, 24, size=n).astype(np.int32)
    t = (X.astype(np.float64) @ true)[np.arange(n), k].astype(np.float32)
    P = dev(M.he_uniform(1).astype(np.float32), np.float32)
    Md = torch.zeros_like(P)
    Vd = torch.zeros_like(P)
    Xd, Kd, Td = dev(X, np.float32), dev(k, np.int32), dev(t, np.float32)
    G = torch.empty_like(P)
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    W = torch.empty(zf.mlp_grad_work_bytes(n) // 4, dtype=torch.float32, device="cuda")
    zf.mlp_grad(P, Xd, Kd, Td, G, L, W)
    l0 = L.item()
    for s in range(1, 301):
        zf.mlp_grad(P, Xd, Kd, Td, G, L, W)
        zf.mlp_adam(P, G, Md, Vd, s, lr=3e-3)
    zf.mlp_grad(P, Xd, Kd, Td, G, L, W)
    assert L.item() < 0.2 * l0
