"""FP64 reference of the cost-model network and its training step.

Test infrastructure only (see ``oracle/__init__.py``).

The network maps 32 chunk statistics to 24 scores (6 codecs x 4 schedules),
each a predicted log of (transfer + decode) time:

    h1 = relu(W1 x + b1)      W1: 64 x 32
    h2 = relu(W2 h1 + b2)     W2: 64 x 64
    y  = W3 h2 + b3           W3: 24 x 64

Loss over a minibatch of samples (x_i, k_i, t_i), where k_i is the one output
that was measured for sample i and t_i its measured log time:

    L = (1/B) sum_i (y_i[k_i] - t_i)^2

Gradients are ordinary backpropagation with relu'(0) = 0.  Adam (Kingma and
Ba, 2015): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; m^ = m / (1-b1^t);
v^ = v / (1-b2^t); p -= lr m^ / (sqrt(v^) + eps).

The flat parameter vector is W1, b1, W2, b2, W3, b3 (row-major), 7,832
values.
"""
import numpy as np

SIZES = (32, 64, 64, 24)


def shapes(sizes=SIZES):
    out = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        out.append((b, a))
        out.append((b,))
    return out


def n_params(sizes=SIZES):
    return sum(int(np.prod(s)) for s in shapes(sizes))


def unflatten(flat, sizes=SIZES):
    flat = np.asarray(flat, dtype=np.float64)
    out, at = [], 0
    for s in shapes(sizes):
        n = int(np.prod(s))
        out.append(flat[at:at + n].reshape(s))
        at += n
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in parts])


def he_uniform(seed, sizes=SIZES):
    """W ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), biases zero."""
    r = np.random.default_rng(seed)
    parts = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / a)
        parts.append(r.uniform(-lim, lim, size=(b, a)))
        parts.append(np.zeros(b))
    return flatten(parts)


def forward(flat, X, sizes=SIZES):
    """Returns (activations, y): activations[0] = X, then each hidden layer."""
    P = unflatten(flat, sizes)
    acts = [np.asarray(X, dtype=np.float64)]
    h = acts[0]
    nl = len(sizes) - 1
    for layer in range(nl):
        W, b = P[2 * layer], P[2 * layer + 1]
        z = h @ W.T + b
        h = np.maximum(z, 0.0) if layer < nl - 1 else z
        if layer < nl - 1:
            acts.append(h)
    return acts, h


def loss(flat, X, k, t, sizes=SIZES):
    _, y = forward(flat, X, sizes)
    B = len(k)
    e = y[np.arange(B), k] - t
    return float(np.mean(e * e))


def grad(flat, X, k, t, sizes=SIZES):
    """(loss, flat gradient) by backpropagation."""
    P = unflatten(flat, sizes)
    acts, y = forward(flat, X, sizes)
    B = len(k)
    e = y[np.arange(B), k] - t
    dy = np.zeros_like(y)
    dy[np.arange(B), k] = 2.0 * e / B
    grads = [None] * len(P)
    d = dy
    nl = len(sizes) - 1
    for layer in reversed(range(nl)):
        h = acts[layer]
        grads[2 * layer] = d.T @ h
        grads[2 * layer + 1] = d.sum(axis=0)
        if layer > 0:
            d = (d @ P[2 * layer]) * (h > 0)
    return float(np.mean(e * e)), flatten(grads)


def adam(flat, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1).  Returns new (params, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
