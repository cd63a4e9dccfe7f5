"""Seeded synthetic inputs, shaped like the paper's star-schema columns.

This module holds none of the codecs' arithmetic; it only draws data.  The
oracle tests and the GPU path both consume exactly what it returns.

All integer draws use numpy's PCG64; the text rows use the counter-based
generator in ``datagen_text.c`` (one independent stream per row), so large
columns build in parallel and identically on every machine.
"""
import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATE_CYCLE = 2557  # distinct day values of the date-like columns


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------- integers
def uniform_i32(n, lo, span, seed):
    """n int32 values uniform in [lo, lo + span)."""
    return rng(seed).integers(lo, lo + span, size=n, dtype=np.int64).astype(np.int32)


def for_bp_column(n=1 << 20, seed=0):
    """FOR+bit-packing workload: uniform in [10^6, 10^6 + 4096)."""
    return uniform_i32(n, 10 ** 6, 4096, seed)


def run_lengths_geometric(n_total, mean_run, seed):
    """Run lengths ~ Geometric(p = 1/mean) on {1, 2, ...}, cut to n_total."""
    g = rng(seed)
    out = []
    have = 0
    while have < n_total:
        k = max(1024, int((n_total - have) / mean_run * 1.1) + 16)
        r = g.geometric(1.0 / mean_run, size=k).astype(np.int64)
        out.append(r)
        have += int(r.sum())
    r = np.concatenate(out)
    c = np.cumsum(r)
    m = int(np.searchsorted(c, n_total)) + 1
    r = r[:m].copy()
    r[-1] -= int(c[m - 1] - n_total)
    return r


def sorted_runs_column(n, mean_run=8, seed=1, cycle=DATE_CYCLE, dtype=np.int32):
    """Date-like column: run k has value (k mod cycle) and a geometric length,
    so the column climbs through `cycle` distinct values, then restarts."""
    r = run_lengths_geometric(n, mean_run, seed)
    v = (np.arange(r.size, dtype=np.int64) % cycle).astype(dtype)
    return np.repeat(v, r)


def runs_family(kind, n_runs, seed, **kw):
    """Run-length families of the paper's RLE microbenchmark (Sec. 5.2):
    even-X (all runs X), random[L,R] (uniform), outlier (mostly 1 with a few
    long runs), mixed (an even and a random family concatenated)."""
    g = rng(seed)
    if kind == "even":
        return np.full(n_runs, kw.get("x", 2), dtype=np.int64)
    if kind == "random":
        return g.integers(kw.get("lo", 1), kw.get("hi", 64) + 1, size=n_runs).astype(np.int64)
    if kind == "outlier":
        r = np.ones(n_runs, dtype=np.int64)
        k = max(1, int(n_runs * kw.get("frac", 0.01)))
        idx = g.choice(n_runs, size=k, replace=False)
        r[idx] = kw.get("big", 1024)
        return r
    if kind == "mixed":
        h = n_runs // 2
        return np.concatenate([runs_family("even", h, seed, x=kw.get("x", 8)),
                               runs_family("random", n_runs - h, seed + 1,
                                           lo=kw.get("lo", 1), hi=kw.get("hi", 256))])
    raise ValueError(kind)


def column_from_runs(runs, seed, dtype=np.int32, distinct=True):
    """Expand run lengths into a column; neighbouring runs get different values
    (so the runs are maximal) drawn as a random walk."""
    g = rng(seed)
    steps = g.integers(1, 1000, size=runs.size).astype(np.int64)
    v = np.cumsum(steps) if distinct else g.integers(0, 4, size=runs.size)
    return np.repeat(v.astype(dtype), runs)


# ---------------------------------------------------------------- strings
def distinct_words(k, seed, lmin=3, lmax=10):
    """k distinct lowercase words of lmin..lmax letters."""
    g = rng(seed)
    words, seen = [], set()
    while len(words) < k:
        n = int(g.integers(lmin, lmax + 1))
        w = bytes(g.integers(97, 123, size=n, dtype=np.uint8))
        if w not in seen:
            seen.add(w)
            words.append(w)
    return words


def fixed16_dictionary(k=25, seed=0):
    """k distinct CHAR(16) values (5..15 letters, zero padded)."""
    ws = distinct_words(k, seed, 5, 15)
    d = np.zeros((k, 16), dtype=np.uint8)
    for i, w in enumerate(ws):
        d[i, :len(w)] = np.frombuffer(w, dtype=np.uint8)
    return d


def fixed16_column(n, k=25, seed=0):
    d = fixed16_dictionary(k, seed)
    idx = rng(seed + 7919).integers(0, k, size=n)
    return d[idx]


def zipf_cdf(K, s):
    """CDF of the finite Zipf law p_k ~ k^-s over ranks 1..K."""
    p = np.arange(1, K + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(p / p.sum())
    c[-1] = 1.0
    return c


_gen = None


def _genlib():
    global _gen
    if _gen is None:
        path = os.path.join(HERE, "libzfgen.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build_gen()
        L = ctypes.CDLL(path)
        L.zfgen_text_rows.restype = ctypes.c_int64
        L.zfgen_text_rows.argtypes = [ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p,
                                      ctypes.c_uint64]
        _gen = L
    return _gen


class TextSource:
    """Zipf comment-text rows over a seeded vocabulary of `vocab` distinct
    words of 3..10 lowercase letters."""

    def __init__(self, seed, vocab=10000, s=1.1):
        self.seed = seed
        words = distinct_words(vocab, seed)
        self.cdf = zipf_cdf(vocab, s)
        self.wlen = np.array([len(w) for w in words], dtype=np.uint32)
        self.woff = np.zeros(vocab, dtype=np.uint32)
        self.woff[1:] = np.cumsum(self.wlen)[:-1]
        self.wbytes = np.frombuffer(b"".join(words), dtype=np.uint8).copy()

    def rows(self, row0, row1):
        cap = (row1 - row0) * 128 + 64
        out = np.empty(cap, dtype=np.uint8)
        c = ctypes.c_void_p
        n = _genlib().zfgen_text_rows(
            self.seed, self.cdf.ctypes.data_as(c), self.cdf.size, self.wbytes.ctypes.data_as(c),
            self.woff.ctypes.data_as(c), self.wlen.ctypes.data_as(c), row0, row1,
            out.ctypes.data_as(c), cap)
        if n < 0:
            raise RuntimeError("text buffer too small")
        return out[:n]

    def rows_parallel(self, n_rows, threads=None, block=1 << 20):
        threads = threads or min(16, os.cpu_count() or 1)
        starts = list(range(0, n_rows, block))
        parts = [None] * len(starts)

        def work(ids):
            for i in ids:
                parts[i] = self.rows(starts[i], min(n_rows, starts[i] + block))

        ts = [threading.Thread(target=work, args=(list(range(t, len(starts), threads)),))
              for t in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        return np.concatenate(parts) if parts else np.empty(0, np.uint8)

    def nbytes(self, nbytes):
        """Exactly nbytes of text (the last row is cut)."""
        est = nbytes // 60 + 1024
        t = self.rows_parallel(est)
        while t.size < nbytes:
            est *= 2
            t = self.rows_parallel(est)
        return t[:nbytes].copy()


def text_column(nbytes=1 << 30, seed=2):
    """Comment-text byte column: Zipf(1.1) words from a 10,000-word vocabulary,
    rows of 40..120 bytes."""
    return TextSource(seed).nbytes(nbytes)


# ------------------------------------------------------------- fact table
# 16 columns: (name, kind, parameters).  Int32 keys over spans 2^12 .. 2^31,
# int64 cents in [100, 10^7), three date-like columns with mean runs 8/64/512,
# three CHAR(16) columns with 25 values each, and one comment-text column.
FACT_COLUMNS = [
    ("key_12", "u32", dict(lo=10 ** 6, span=1 << 12)),
    ("key_16", "u32", dict(lo=10 ** 6, span=1 << 16)),
    ("key_20", "u32", dict(lo=10 ** 6, span=1 << 20)),
    ("key_24", "u32", dict(lo=10 ** 6, span=1 << 24)),
    ("key_25", "u32", dict(lo=10 ** 6, span=1 << 25)),
    ("key_31", "u32", dict(lo=-(1 << 30), span=1 << 31)),
    ("cents_a", "cents", {}),
    ("cents_b", "cents", {}),
    ("cents_c", "cents", {}),
    ("date_8", "date", dict(mean=8)),
    ("date_64", "date", dict(mean=64)),
    ("date_512", "date", dict(mean=512)),
    ("flag_a", "char16", {}),
    ("flag_b", "char16", {}),
    ("flag_c", "char16", {}),
    ("comment", "text", {}),
]
FACT_ROWS = 45_450_000
# codec of each kind of fact-table column (names of zf codecs): the text
# column takes the comment column's scheme, String-dictionary | bit-packing |
# ANS over one dictionary for the column
FACT_CODECS = {"u32": "FOR_BP", "cents": "FOR_BP", "date": "RLE_DELTA_BP", "char16": "DICT_BP",
               "text": "SDICT_COL_ANS"}


def fact_column(i, rows=FACT_ROWS, seed=3):
    name, kind, p = FACT_COLUMNS[i]
    s = seed * 1000 + i
    if kind == "u32":
        return uniform_i32(rows, p["lo"], p["span"], s)
    if kind == "cents":
        return rng(s).integers(100, 10 ** 7, size=rows, dtype=np.int64)
    if kind == "date":
        return sorted_runs_column(rows, p["mean"], s)
    if kind == "char16":
        return fixed16_column(rows, 25, s)
    if kind == "text":
        return TextSource(s).rows_parallel(rows)
    raise ValueError(kind)


def decimal_column(n, seed, lo, hi, scale=100, specials=0):
    """float64 decimals with log10(scale) places, as read from text: integers
    uniform in [lo, hi) divided by `scale` (IEEE division gives the nearest
    double to each decimal).  `specials` values at random positions are
    replaced by NaN, infinities, -0.0 and full-precision doubles."""
    r = rng(seed)
    x = r.integers(lo, hi, size=n).astype(np.float64) / float(scale)
    if specials:
        pool = np.array([np.nan, np.inf, -np.inf, -0.0, 1.0 / 3.0, np.pi, 5e-324, 1e300])
        x[r.integers(0, n, size=specials)] = pool[r.integers(0, len(pool), size=specials)]
    return x


def returnflag_column(n, p_a, p_n, seed):
    """Bytes 'A', 'N', 'R' with probabilities p_a, p_n and 1 - p_a - p_n
    (a flag column with a skewed distribution, the paper's ANS workload)."""
    r = rng(seed)
    u = r.random(n)
    out = np.full(n, ord("R"), np.uint8)
    out[u < p_a + p_n] = ord("N")
    out[u < p_a] = ord("A")
    return out


def orderkey_column(n, seed, drop=0.01, block=8, spacing=32, dtype=np.int32, start=1):
    """Sparse order keys: the first `block` keys of every `spacing` (the key
    layout of the TPC-H orders table), each key then removed with
    probability `drop` (deleted orders), so some blocks are shorter and some
    gaps wider; n keys are returned."""
    g = rng(seed)
    m = int(n / (1.0 - drop)) + block + 64
    i = np.arange(m, dtype=np.int64)
    keys = start + spacing * (i // block) + i % block
    keep = g.random(m) >= drop
    out = keys[keep][:n]
    while out.size < n:  # rare: more drops than expected
        m *= 2
        i = np.arange(m, dtype=np.int64)
        keys = start + spacing * (i // block) + i % block
        out = keys[g.random(m) >= drop][:n]
    return out.astype(dtype)


def key_column(n, seed, mean_run=8, max_jump=64, dtype=np.int32, start=1):
    """Nearly increasing primary keys: blocks of consecutive keys with
    geometric lengths (mean `mean_run`), each block starting a uniform
    1..max_jump past the end of the previous one."""
    g = rng(seed)
    r = run_lengths_geometric(n, mean_run, seed)
    jumps = g.integers(1, max_jump + 1, size=r.size).astype(np.int64)
    jumps[0] = 0
    block_start = start + np.cumsum(np.concatenate([[0], r[:-1]])) + np.cumsum(jumps)
    first = np.repeat(block_start, r)
    within = np.arange(n, dtype=np.int64) - np.repeat(np.cumsum(r) - r, r)
    return (first + within).astype(dtype)
