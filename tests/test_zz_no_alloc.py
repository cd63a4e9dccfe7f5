"""zf_mlp_grad_noalloc (the allocation-free gradient, partials in the
library's static device array) against zf_mlp_grad with a caller workspace:
two calls in a row, the second smaller, each equal bit for bit to the
workspace call on the same inputs (same kernels, same summation order) and
within the FP64 oracle's tolerance; the size limit is enforced."""
import sys

import numpy as np
import pytest

from oracle import mlp as M
from paper_2602_08190_amd import zf

from conftest import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def inputs(seed, n):
    r = np.random.default_rng(seed)
    X = r.normal(size=(n, 32)).astype(np.float32)
    k = r.integers(0, 24, size=n).astype(np.int32)
    t = r.normal(size=n).astype(np.float32)
    return X, k, t


def run_both(p32, n, seed):
    import torch
    X, k, t = inputs(seed, n)
    P, Xd, Kd, Td = dev(p32, np.float32), dev(X, np.float32), dev(k, np.int32), dev(t, np.float32)
    G0 = torch.full((M.n_params(),), 7.0, dtype=torch.float32, device="cuda")
    L0 = torch.full((1,), 7.0, dtype=torch.float32, device="cuda")
    W = torch.empty(zf.mlp_grad_work_bytes(n) // 4, dtype=torch.float32, device="cuda")
    zf.mlp_grad(P, Xd, Kd, Td, G0, L0, W)
    G1 = torch.full_like(G0, -3.0)
    L1 = torch.full_like(L0, -3.0)
    zf.mlp_grad_noalloc(P, Xd, Kd, Td, G1, L1)
    torch.cuda.synchronize()
    g0, g1 = G0.cpu().numpy(), G1.cpu().numpy()
    assert np.array_equal(g0.view(np.uint32), g1.view(np.uint32)), f"n={n}: gradients differ"
    assert L0.item() == L1.item()
    lref, gref = M.grad(p32.astype(np.float64), X.astype(np.float64), k, t.astype(np.float64))
    assert np.linalg.norm(g1 - gref) / np.linalg.norm(gref) <= 1e-5
    assert abs(L1.item() - lref) <= 1e-5 * lref


def test_noalloc_equals_workspace_call_twice_then_smaller():
    p32 = M.he_uniform(11).astype(np.float32)
    for n in (3000, 700):   # second call smaller: stale partials of the first must not leak in
        print("noalloc grad n =", n, flush=True)
        run_both(p32, n, seed=n)


def test_noalloc_limit():
    import torch
    p32 = M.he_uniform(12).astype(np.float32)
    print("noalloc grad at the limit", flush=True)
    run_both(p32, zf.MLP_STATIC_MAX_N, seed=1)
    n = zf.MLP_STATIC_MAX_N + 1
    X, k, t = inputs(2, n)
    P, Xd, Kd, Td = dev(p32, np.float32), dev(X, np.float32), dev(k, np.int32), dev(t, np.float32)
    G = torch.empty(M.n_params(), dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    with pytest.raises(zf.ZfError) as e:
        zf.mlp_grad_noalloc(P, Xd, Kd, Td, G, L)
    assert e.value.status == zf.E_UNSUPPORTED and "16384" in str(e.value)
