"""Benchmark of the zf hot path on one MI355X.

Default workload: the batched 16-column fact table (45.45M rows, ~8.0 GiB
plain): six int32 key columns (FOR_BP), three int64 cents columns (FOR_BP),
three date-like columns with runs (RLE_DELTA_BP), three CHAR(16) flag columns
(DICT_BP) and one comment-text column (String-dictionary over one dictionary
for the column, bit-packing and ANS: SDICT_COL_ANS; --text-codec picks another
String-dictionary variant or LZ77), in uneven chunks of 16 KiB - 4 MiB.
Synthetic, seeded data.

One step decodes the whole table from its compressed image already in HBM
(zf_decompress_async: one kernel per kind, or the persistent kernel with
--persistent 1).  The metric names two rates: the end-to-end effective rate
of H2D + decode from pinned host memory, and the decode HBM rate.  `value` is
the second, (compressed bytes read + plain bytes written) / step time, since
its inputs are resident in HBM when the timed region starts; the PCIe-
inclusive rate is reported beside it under "e2e" with the raw uncompressed
copy it is compared with.  Also reported: plain bytes decoded per second,
per-step median and p10/p90, each kernel kind's time inside the step (HIP
events around its launch), the dominant kernel's HBM roofline, the whole
output checked against the oracle (decoded chunk-parallel on the host
cores, which also times the oracle on all cores), the oracle on one core on a
bounded sample, the host and ROCm description and a sha256 manifest of the
generated inputs.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload fact|for|rle|lz|f2i|ans|keys|sdict|sdict_ans|copy]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "end-to-end effective GB/s (H2D+decode) vs raw PCIe copy; decode HBM GB/s"
HBM_PEAK_GBPS = 8000.0
PCIE_PEAK_GBPS = 63.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_hash():
    from paper_2602_08190_amd.profiling import kernel_sha
    return kernel_sha()


# ------------------------------------------------------------- workloads
TEXT_CODECS = {"sdict": "SDICT_BP", "sdict_ans": "SDICT_ANS", "sdict_col": "SDICT_COL",
               "sdict_col_ans": "SDICT_COL_ANS", "lz77": "LZ77"}


def fact_table(rows, text_codec="sdict_col_ans"):
    """The 16-column table.  The comment text is String-dictionary coded (the
    paper's choice for comment columns, Sec. 5) on the same uneven chunks as
    the other columns: one dictionary for the column, nested with bit-packing
    and ANS (sdict_col_ans, the paper's comment-column scheme; the default),
    or not (sdict_col), or one dictionary per chunk (sdict, sdict_ans);
    text_codec="lz77" codes it as LZ77 in 64 KiB chunks."""
    from paper_2602_08190_amd import datagen as g
    from paper_2602_08190_amd import zf
    codec_of = {k: getattr(zf, v) for k, v in g.FACT_CODECS.items()}
    codec_of["text"] = getattr(zf, TEXT_CODECS[text_codec])
    cols, xs, names = [], [], []
    for i, (name, kind, _) in enumerate(g.FACT_COLUMNS):
        t = time.time()
        x = g.fact_column(i, rows)
        t1 = time.time()
        c = zf.Column.compress(x, codec_of[kind], chunk_bytes=(16 << 10, 4 << 20), seed=3000 + i)
        log(f"column {i:2d} {name:9s} {x.nbytes / 2**20:8.1f} MiB -> {c.host_pointer()[1] / 2**20:8.1f} MiB"
            f"  ({c.n_chunks} chunks, gen {t1 - t:.1f}s, encode {time.time() - t1:.1f}s)")
        cols.append(c)
        xs.append(x)
        names.append(name)
    text = ("LZ77 in 64 KiB chunks" if text_codec == "lz77" else f"String-dictionary, {TEXT_CODECS[text_codec]}")
    desc = (f"batched 16-column fact table, {rows} rows: 6 int32 keys (FOR_BP), 3 int64 cents "
            f"(FOR_BP), 3 run-sorted dates (RLE_DELTA_BP), 3 CHAR(16) flags (DICT_BP), 1 Zipf "
            f"comment text ({text}); uneven chunks 16 KiB-4 MiB")
    return cols, xs, names, desc


def single(kind, n):
    from paper_2602_08190_amd import datagen as g
    from paper_2602_08190_amd import zf
    if kind == "for":
        x = g.for_bp_column(n, 0)
        c = zf.Column.compress(x, zf.FOR_BP, chunk_bytes=(4 << 20, 4 << 20))
        desc = f"FOR_BP int32, {n} values uniform in [10^6, 10^6+4096), w=12, 4 MiB chunks"
    elif kind == "rle":
        x = g.sorted_runs_column(n, 8, 1)
        c = zf.Column.compress(x, zf.RLE_DELTA_BP, chunk_elems=[16384] * (n // 16384) +
                               ([n % 16384] if n % 16384 else []))
        desc = f"RLE_DELTA_BP int32, {n} values, geometric(8) runs, 64 KiB chunks"
    elif kind == "lz":
        x = g.text_column(n, 2)
        c = zf.Column.compress(x, zf.LZ77)
        desc = f"LZ77 text, {n} bytes, Zipf(1.1) over 10,000 words, 64 KiB chunks"
    elif kind == "f2i":
        x = g.decimal_column(n, 5, 90000, 10500000)
        c = zf.Column.compress(x, zf.F2I_BP)
        desc = (f"F2I_BP float64, {n} prices with 2 decimal places uniform in [900, 105000), "
                f"1 MiB chunks")
    elif kind == "ans":
        x = g.returnflag_column(n, 0.25, 0.5, 9)
        c = zf.Column.compress(x, zf.ANS)
        desc = (f"ANS bytes, {n} flags 'A'/'N'/'R' with probabilities 0.25/0.5/0.25, 64 KiB chunks, "
                f"64 interleaved coders per chunk")
    elif kind == "sdict":
        x = g.text_column(n, 2)
        c = zf.Column.compress(x, zf.SDICT_BP)
        desc = (f"SDICT_BP text, {n} bytes, Zipf(1.1) over 10,000 words, String-dictionary per 1 MiB "
                f"chunk (tokens end at spaces and periods)")
    elif kind == "sdict_ans":
        x = g.text_column(n, 2)
        c = zf.Column.compress(x, zf.SDICT_ANS)
        desc = (f"SDICT_ANS text, {n} bytes, Zipf(1.1) over 10,000 words: String-dictionary | "
                f"bit-packing | ANS per 1 MiB chunk (two launches: ANS stage into scratch, then "
                f"String-dictionary)")
    elif kind in ("sdict_col", "sdict_col_ans"):
        x = g.text_column(n, 2)
        codec = zf.SDICT_COL if kind == "sdict_col" else zf.SDICT_COL_ANS
        c = zf.Column.compress(x, codec)
        desc = (f"{zf.CODEC_NAMES[codec]} text, {n} bytes, Zipf(1.1) over 10,000 words: one String-dictionary "
                f"for the column (tokens end at spaces, periods and row ends), 1 MiB chunks"
                + (" (two launches: ANS stage into scratch, then String-dictionary)" if codec == zf.SDICT_COL_ANS
                   else ""))
    elif kind == "keys":
        x = g.key_column(n, 11)
        c = zf.Column.compress(x, zf.DSTRIDE_BP)
        desc = (f"DSTRIDE_BP int32, {n} nearly increasing keys (blocks of consecutive keys, "
                f"geometric(8) lengths, jumps uniform 1..64), 1 MiB chunks")
    elif kind == "orderkey":
        x = g.orderkey_column(n, 12)
        c = zf.Column.compress(x, zf.DSTREE)
        desc = (f"DSTREE int32, {n} sparse order keys (the first 8 of every 32, 1% deleted): DeltaStride | "
                f"[Delta | RLE | [BP, BP], BP], 1 MiB chunks (two launches: the run starts into scratch, "
                f"then the output)")
    elif kind == "copy":
        x = np.frombuffer(np.random.default_rng(0).bytes(n), np.uint8)
        c = zf.Column.compress(x, zf.PLAIN, chunk_bytes=(4 << 20, 4 << 20))
        desc = f"PLAIN copy probe, {n} bytes"
    else:
        raise ValueError(kind)
    return [c], [x], [kind], desc


# ------------------------------------------------------------- CPU oracle
def host_threads():
    """Host threads for the chunk-parallel oracle: the CPUs this process may
    run on, at most 16 (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_description(threads):
    d = {"threads_used": threads, "cpus_visible": os.cpu_count()}
    try:
        models, sockets = set(), set()
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                models.add(line.split(":", 1)[1].strip())
            elif line.startswith("physical id"):
                sockets.add(line.split(":", 1)[1].strip())
        d["cpu_model"] = "; ".join(sorted(models))
        d["sockets"] = len(sockets) or None
    except OSError:
        pass
    try:
        cpus = sorted(os.sched_getaffinity(0))
        nodes = set()
        base = "/sys/devices/system/node"
        for nd in os.listdir(base):
            if nd.startswith("node"):
                lst = open(os.path.join(base, nd, "cpulist")).read().strip()
                ids = set()
                for part in lst.split(","):
                    if "-" in part:
                        a, b = part.split("-")
                        ids.update(range(int(a), int(b) + 1))
                    elif part:
                        ids.add(int(part))
                if ids & set(cpus):
                    nodes.add(nd)
        d["numa_nodes"] = sorted(nodes)
    except OSError:
        pass
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                d["mem_total_GiB"] = round(int(line.split()[1]) / 2**20, 1)
    except OSError:
        pass
    return d


def gpu_description(torch):
    import glob
    props = torch.cuda.get_device_properties(0)
    d = {"name": torch.cuda.get_device_name(0) or getattr(props, "gcnArchName", ""),
         "arch": getattr(props, "gcnArchName", ""), "compute_units": props.multi_processor_count}
    try:
        d["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        pass
    d["torch"] = torch.__version__
    # the current engine and memory clock levels from the driver's sysfs
    # tables (the level in use is marked with '*'; no helper program is run)
    clocks = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        for name in ("pp_dpm_sclk", "pp_dpm_mclk"):
            try:
                lines = open(f"{dev}/{name}").read().splitlines()
            except OSError:
                continue
            cur = [ln.split(":", 1)[1].strip(" *") for ln in lines if ln.rstrip().endswith("*")]
            if cur:
                clocks[f"{dev.split('/')[-2]} {name[7:]}"] = cur[0]
    d["clocks"] = clocks or "unavailable (no readable clock table)"
    return d


def cpu_single_thread(cols, budget_s=12.0):
    """The oracle (single-threaded C) decoding runs of consecutive chunks from
    every column for about budget_s seconds in total."""
    import oracle.zfo as zo
    per_col = budget_s / len(cols)
    total_bytes, total_s, nchunks = 0, 0.0, 0
    for c in cols:
        b = c.bytes()
        cs = zo.chunks(b)
        first, k, spent = len(cs) // 3, 1, 0.0
        while spent < per_col:
            k = min(k, len(cs) - first)
            t = time.perf_counter()
            zo.decode_chunks(b, first, k)
            dt = time.perf_counter() - t
            spent += dt
            total_s += dt
            total_bytes += sum(x["plain_len"] for x in cs[first:first + k])
            nchunks += k
            first = (first + k) % len(cs)
            k *= 2
    return {"value": round(total_bytes / total_s / 1e9, 4), "unit": "GB/s", "cores": 1,
            "sample": f"{nchunks} chunks in runs of consecutive chunks, about {per_col:.1f} s of "
                      f"decoding per column over all {len(cols)} columns, {total_bytes / 2**20:.0f} "
                      f"MiB plain decoded from host memory in {total_s:.1f} s"}


def cpu_baseline_all_cores(cols, threads):
    """The CPU baseline on all host threads: every chunk of every column
    decoded by the oracle, chunk ranges spread over `threads` host threads
    (the oracle itself is single-threaded).  Returns (outputs as flat uint8
    arrays, wall seconds); the outputs also serve as the reference the GPU's
    whole output is compared with."""
    import concurrent.futures as cf
    import oracle.zfo as zo
    blobs = [c.bytes() for c in cols]
    outs, jobs = [], []
    for ci, b in enumerate(blobs):
        info = zo.inspect(b)
        cs = zo.chunks(b)
        out = np.empty(info["plain_bytes"], np.uint8)
        outs.append(out)
        piece = max(1, info["plain_bytes"] // (threads * 4))
        i = 0
        while i < len(cs):
            j, nb = i, 0
            while j < len(cs) and (nb < piece or j == i):
                nb += cs[j]["plain_len"]
                j += 1
            jobs.append((ci, i, j - i, cs[i]["plain_off"], nb))
            i = j
    t = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda jb: zo.decode_chunks_into(blobs[jb[0]], jb[1], jb[2], outs[jb[0]], jb[3], jb[4]),
                    jobs))
    return outs, time.perf_counter() - t


def compare_outputs(torch, outs, ref, threads):
    """Whole-output check: each GPU column against the oracle's bytes.
    Returns per-column {"ok", "first_mismatch"}."""
    import concurrent.futures as cf
    host = [o.view(torch.uint8).reshape(-1).cpu().numpy() for o in outs]

    def one(i):
        a, b = host[i], ref[i]
        if a.size == b.size and np.array_equal(a, b):
            return {"ok": True}
        if a.size != b.size:
            return {"ok": False, "first_mismatch": f"size {a.size} != {b.size}"}
        bad = np.flatnonzero(a != b)
        return {"ok": False, "first_mismatch": int(bad[0]), "mismatching_bytes": int(bad.size)}
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, range(len(outs))))


def sha256_manifest(xs, names, threads):
    import concurrent.futures as cf
    import hashlib

    def one(x):
        return hashlib.sha256(np.ascontiguousarray(x).view(np.uint8).reshape(-1)).hexdigest()
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return dict(zip(names, ex.map(one, xs)))


def pct(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q))


def group_traffic(workload, group):
    """HBM bytes per decode of one kernel group ("ANS+SDICT" sums its two
    launches), or None if any launch has no current counter reading."""
    parts = [read_traffic(f"{workload}/{k}") for k in group.split("+")]
    return None if None in parts else sum(parts)


def read_traffic(key):
    """HBM bytes per launch of one kernel from the committed counter summary
    (profiles/traffic.txt), if it was taken on the current kernel sources."""
    p = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(p):
        return None
    kv = {}
    for line in open(p):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_sha") != kernel_hash():
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="fact", choices=["fact", "for", "rle", "lz", "f2i", "ans", "keys", "orderkey", "sdict",
                                                              "sdict_ans", "sdict_col", "sdict_col_ans", "copy"])
    ap.add_argument("--rows", type=int, default=None)
    ap.add_argument("--text-codec", default="sdict_col_ans", choices=sorted(TEXT_CODECS),
                    help="codec of the fact table's comment column")
    ap.add_argument("--no-e2e", action="store_true")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU baseline (the oracle on all host threads, whose outputs the whole "
                         "GPU output is compared with, and on one core)")
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0,
                    help="persistent kernel: waves in flight per CU (0: the tune cache's)")
    ap.add_argument("--untuned", action="store_true",
                    help="plan with the built-in default tile of every kind instead of the tune cache")
    ap.add_argument("--e2e-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: decoding needs no exchange between GPUs, and a "
              "multi-GPU run is not implemented (each GPU would decode its own chunks over its "
              "own PCIe link).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_08190_amd import datagen as g
    from paper_2602_08190_amd import zf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    zf.lib()
    threads = host_threads()
    t0 = time.time()
    if args.workload == "fact":
        cols, xs, names, desc = fact_table(args.rows or g.FACT_ROWS, args.text_codec)
    else:
        n = args.rows or {"for": 1 << 28, "rle": 1 << 26, "lz": 1 << 30, "f2i": 1 << 26,
                           "ans": 1 << 30, "keys": 1 << 26, "orderkey": 1 << 26, "sdict": 1 << 30, "sdict_ans": 1 << 30,
                           "sdict_col": 1 << 30, "sdict_col_ans": 1 << 30, "copy": 1 << 30}[args.workload]
        cols, xs, names, desc = single(args.workload, n)
    plain = sum(c.plain_bytes for c in cols)
    comp = sum(c.host_pointer()[1] for c in cols)
    log(f"data ready in {time.time() - t0:.1f}s: plain {plain / 2**30:.2f} GiB, compressed "
        f"{comp / 2**30:.2f} GiB (ratio {plain / comp:.2f}x)")
    manifest = sha256_manifest(xs, names, threads)

    plan = zf.Plan(cols, device=0, persistent=bool(args.persistent), waves_per_cu=args.waves_per_cu,
                   **({"tune_cache": os.devnull} if args.untuned else {}))
    img = zf.upload_image(plan, cols)
    outs = zf.empty_outputs(cols)
    stream = torch.cuda.current_stream()

    # one decode, checked against the input on a sample of rows
    plan.decompress_async(img, img.numel(), outs)
    plan.sync()
    r = np.random.default_rng(0)
    for x, o in zip(xs, outs):
        idx = r.integers(0, len(x), size=4096)
        got = o[torch.from_numpy(idx).to(o.device)].cpu().numpy()
        if x.dtype == np.float64:  # bit for bit
            got, want = got.view(np.uint64), x[idx].view(np.uint64)
        else:
            want = x[idx]
        assert np.array_equal(got, want), "decode mismatch"
    log("sampled check against the input: ok")

    # CPU baseline on all host threads; its outputs are the reference for the
    # whole GPU output
    verify, ref, cpu_all = None, None, None
    if not args.no_cpu:
        ref, secs = cpu_baseline_all_cores(cols, threads)
        cpu_all = {"value": round(plain / secs / 1e9, 4), "unit": "GB/s", "cores": threads,
                   "seconds": round(secs, 2)}
        log(f"oracle, all chunks on {threads} host threads: {secs:.2f} s ({plain / secs / 1e9:.2f} GB/s)")
        res = compare_outputs(torch, outs, ref, threads)
        inputs_ok = [np.array_equal(rf, np.ascontiguousarray(x).view(np.uint8).reshape(-1))
                     for rf, x in zip(ref, xs)]
        verify = {"image_decode_vs_oracle": "ok" if all(v["ok"] for v in res) else
                  {n: v for n, v in zip(names, res) if not v["ok"]},
                  "oracle_vs_input": "ok" if all(inputs_ok) else
                  [n for n, ok in zip(names, inputs_ok) if not ok],
                  "bytes_compared": plain}
        log(f"whole output vs oracle: {verify['image_decode_vs_oracle']}; oracle vs input: "
            f"{verify['oracle_vs_input']}")

    # timed steps: decode of the whole table from HBM, an event per step
    for _ in range(args.warmup):
        plan.decompress_async(img, img.numel(), outs)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record(stream)
    for k in range(args.steps):
        plan.decompress_async(img, img.numel(), outs)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    plan.sync()
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    ms = evs[0].elapsed_time(evs[-1]) / args.steps
    alg_bytes = comp + plain  # every compressed byte read once, every plain byte written once
    hbm_gbps = alg_bytes / (ms * 1e-3) / 1e9
    plain_gbps = plain / (ms * 1e-3) / 1e9
    log(f"decode from HBM: {ms:.3f} ms/step (median {pct(step_ms, 50):.3f}), {hbm_gbps:.1f} GB/s HBM, "
        f"{plain_gbps:.1f} GB/s plain")

    # kernel times inside the step: events before and after each kind's launch
    prof_steps = max(5, args.steps // 2)
    plan.profile(True)
    per = {}
    for _ in range(prof_steps):
        plan.decompress_async(img, img.numel(), outs)
        for k, v in plan.kind_ms().items():
            per.setdefault(k, []).append(v)
    plan.profile(False)
    plan.sync()
    groups = {}
    for c in cols:
        key = zf.kind_of_column(c)
        if zf.first_codec(c) in (zf.SDICT_ANS, zf.SDICT_COL_ANS):
            key = "ANS+SDICT"  # two ordered launches: the ANS stage, then String-dictionary
        if zf.first_codec(c) == zf.DSTREE:
            key = ("RLE32" if c.dtype == zf.I32 else "RLE64") + "+TREE"  # the run starts, then the output
        if args.persistent:
            key = "PERSISTENT"
        groups[key] = groups.get(key, 0) + c.host_pointer()[1] + c.plain_bytes
    kinds = {}
    for key, kb in groups.items():
        series = [sum(v) for v in zip(*[per[k] for k in key.split("+")])]
        med = pct(series, 50)
        kinds[key] = {"ms_median": round(med, 4), "ms_p10": round(pct(series, 10), 4),
                      "ms_p90": round(pct(series, 90), 4), "algorithmic_bytes": kb,
                      "GBps": round(kb / (med * 1e-3) / 1e9, 1),
                      "frac_of_hbm_peak": round(kb / (med * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        log(f"kernel {key:8s} in the step: {med:.3f} ms, {kinds[key]['GBps']:.1f} GB/s of algorithmic bytes")
    for key in groups:
        if "+" in key:   # the launches of a two-stage group, each on its own
            for k in key.split("+"):
                kinds[key][f"{k}_ms_median"] = round(pct(per[k], 50), 4)
    dom = max(kinds, key=lambda k: kinds[k]["ms_median"])

    # the same decode with the persistent kernel (same image, same outputs)
    pers = None
    if not args.persistent:
        plan_p = zf.Plan(cols, device=0, persistent=True, waves_per_cu=args.waves_per_cu,
                         **({"tune_cache": os.devnull} if args.untuned else {}))
        assert all(plan_p.image_offset(i) == plan.image_offset(i) for i in range(len(cols)))
        for _ in range(max(1, args.warmup)):
            plan_p.decompress_async(img, img.numel(), outs)
        torch.cuda.synchronize()
        pe = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        pe[0].record(stream)
        for k in range(args.steps):
            plan_p.decompress_async(img, img.numel(), outs)
            pe[k + 1].record(stream)
        torch.cuda.synchronize()
        plan_p.sync()
        pms = [pe[k].elapsed_time(pe[k + 1]) for k in range(args.steps)]
        pers = {"ms_per_step": round(pe[0].elapsed_time(pe[-1]) / args.steps, 4),
                "ms_median": round(pct(pms, 50), 4),
                "vs_per_kind": round((pe[0].elapsed_time(pe[-1]) / args.steps) / ms, 3)}
        plan_p.free()
        log(f"persistent kernel: {pers['ms_per_step']:.3f} ms/step ({pers['vs_per_kind']:.2f}x the per-kind step)")

    result = {
        "metric": METRIC, "value": round(hbm_gbps, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.workload == "f2i" else "u32",
        "data": "synthetic",
        "config": {"workload": desc, "plain_bytes": plain, "comp_bytes": comp,
                   "ratio": round(plain / comp, 3),
                   "chunks": sum(c.n_chunks for c in cols),
                   "launch": "persistent" if args.persistent else "per-kind",
                   "tiles": "built-in defaults" if args.untuned else "tune cache"},
        "value_is": "decode HBM GB/s = (compressed + plain bytes) / step time, inputs in HBM",
        "decode_plain_GBps": round(plain_gbps, 2),
        "step_ms": {"median": round(pct(step_ms, 50), 4), "p10": round(pct(step_ms, 10), 4),
                    "p90": round(pct(step_ms, 90), 4)},
        "roofline": {"bound": "hbm", "achieved": kinds[dom]["GBps"], "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": kinds[dom]["frac_of_hbm_peak"],
                     "traffic": group_traffic(args.workload, dom),
                     "kernel": {"LZ77": "k_decode_lz (LZ77)", "ANS": "k_decode_ans",
                                "ANS+SDICT": "k_decode_ans then the String-dictionary kernel (k_decode_sdict_hot<16u> "
                                             "at 16 waves per workgroup, else k_decode_sdict)",
                                "RLE32+TREE": "k_decode_kind<RLE32> then k_decode_kind<TREE>",
                                "RLE64+TREE": "k_decode_kind<RLE64> then k_decode_kind<TREE>",
                                "PERSISTENT": "k_decode_persistent"}.get(dom, f"k_decode_kind<{dom}>"),
                     "algorithmic_bytes_per_launch": kinds[dom]["algorithmic_bytes"],
                     "avg_launch_ms": kinds[dom]["ms_median"],
                     "timing": f"median of {prof_steps} steps, HIP events around the launch inside the step"},
        "kernels": kinds,
    }
    if pers is not None:
        result["persistent_launch"] = pers
    if verify is not None:
        result["verify"] = verify

    if not args.no_e2e:
        # PCIe end to end: pinned host -> staging slots -> decode, pipelined
        walls = []
        for rep in range(args.e2e_reps):
            plan.transfer_and_decompress(outs, timing=True)
            walls.append(plan.sync())
        walls.sort(key=lambda t: t["wall_ms"])
        tm = walls[len(walls) // 2]
        eff = plain / (tm["wall_ms"] * 1e-3) / 1e9
        if ref is not None:
            res = compare_outputs(torch, outs, ref, threads)
            result["verify"]["staged_decode_vs_oracle"] = "ok" if all(v["ok"] for v in res) else \
                {n: v for n, v in zip(names, res) if not v["ok"]}
            log(f"staged output vs oracle: {result['verify']['staged_decode_vs_oracle']}")
        # raw copy of the plain bytes from pinned memory, 256 MiB pieces
        hosts = [torch.from_numpy(np.ascontiguousarray(x).view(np.uint8).reshape(-1)).pin_memory()
                 for x in xs]
        flat = [o.view(torch.uint8).reshape(-1) for o in outs]
        raws = []
        for rep in range(args.e2e_reps):
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for h, d in zip(hosts, flat):
                for s in range(0, h.numel(), 256 << 20):
                    d[s:s + (256 << 20)].copy_(h[s:s + (256 << 20)], non_blocking=True)
            b.record(stream)
            torch.cuda.synchronize()
            raws.append(a.elapsed_time(b))
        raw_ms = pct(raws, 50)
        raw = plain / (raw_ms * 1e-3) / 1e9
        del hosts
        wall = [t["wall_ms"] for t in walls]
        result["e2e"] = {
            "effective_GBps": round(eff, 2), "raw_copy_GBps": round(raw, 2),
            "vs_raw_copy": round(eff / raw, 3), "wall_ms": round(tm["wall_ms"], 2),
            "wall_ms_p10": round(pct(wall, 10), 2), "wall_ms_p90": round(pct(wall, 90), 2),
            "h2d_ms": round(tm["h2d_ms"], 2), "decode_ms": round(tm["decode_ms"], 2),
            "pcie_GBps_compressed": round(comp / (tm["h2d_ms"] * 1e-3) / 1e9, 2),
            "pcie_frac_of_63": round(comp / (tm["h2d_ms"] * 1e-3) / 1e9 / PCIE_PEAK_GBPS, 3),
            "reps": args.e2e_reps}
        log(f"end to end: {eff:.1f} GB/s effective vs raw copy {raw:.1f} GB/s "
            f"(x{eff / raw:.2f}); wall {tm['wall_ms']:.1f} ms, h2d {tm['h2d_ms']:.1f} ms, "
            f"decode {tm['decode_ms']:.1f} ms")

    if not args.no_cpu:
        log("CPU oracle baseline, one core ...")
        one = cpu_single_thread(cols)
        log(f"oracle on one core: {one['value']} GB/s")
        if cpu_all is not None:
            result["cpu_baseline"] = {
                "value": cpu_all["value"], "unit": "GB/s", "cores": threads, "kind": "oracle",
                "sample": f"every chunk of the workload ({plain / 2**30:.2f} GiB plain) decoded from host "
                          f"memory by the single-threaded oracle, chunk ranges spread over {threads} "
                          f"host threads, in {cpu_all['seconds']} s; rate = plain bytes / wall time",
                "one_core": one}
        else:
            result["cpu_baseline"] = dict(one, kind="oracle")
    result["host"] = host_description(threads)
    result["gpu"] = gpu_description(torch)
    result["inputs_sha256"] = manifest
    print(json.dumps(result), flush=True)
    if verify is not None and any(v != "ok" for k, v in result["verify"].items() if k != "bytes_compared"):
        log("output mismatch against the oracle")
        sys.exit(1)


if __name__ == "__main__":
    main()
