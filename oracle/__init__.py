"""The oracle: plain, slow, obviously-correct CPU implementations of what the
zf hot path computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The product package
never imports it, and nothing here imports the product.

* ``oracle.zfo``      -- codecs and the column container (plain C, via ctypes)
* ``oracle.johnson``  -- Johnson's two-machine flow-shop rule (Sec. 3.3)
* ``oracle.mlp``      -- the FP64 cost-model network, its gradients and Adam
"""
