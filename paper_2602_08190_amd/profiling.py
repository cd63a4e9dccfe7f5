"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2602_08190_amd.profiling stats <run_kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2602_08190_amd.profiling traffic <pmc_root> <out_dir> "<command>"
    python -m paper_2602_08190_amd.profiling counters <out.txt> <kernel> "<command>" <csv> [<csv> ...]
    python -m paper_2602_08190_amd.profiling copies <stats.csv> <trace.csv> <out.txt> "<command>"

`traffic` expects <pmc_root>/pmc_<workload>_<COUNTER>/run_counter_collection.csv
for COUNTER in FETCH_SIZE, WRITE_SIZE and workloads including `copy` (the
PLAIN copy probe of exactly 1 GiB, which calibrates both counters).
"""
import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
KIND_OF_ID = ["LZ77", "ANS", "RLE64", "RLE32", "SDICT", "DICT128", "DICT64", "DICT32", "FOR64", "FOR32", "F2I",
              "PLAIN", "TREE"]


def kernel_sha():
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith(".hip") or name in ("kernels.hpp", "zf_device.hpp"):
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def stats(csv_path, out_path, command):
    rows = list(csv.DictReader(open(csv_path)))
    lines = [f"# rocprofv3 --kernel-trace --stats summary ({os.path.basename(csv_path)})",
             f"# command: {command}", f"# kernel sources sha: {kernel_sha()}", "",
             f"{'kernel':58s} {'calls':>6s} {'avg_us':>11s} {'total_us':>12s} {'pct':>7s}"]
    for r in rows:
        name = r["Name"]
        for kid, kind in enumerate(KIND_OF_ID):
            name = name.replace(f"k_decode_kind<{kid}u>", f"k_decode_kind<{kid}u={kind}>")
        name = name if len(name) <= 58 else name[:55] + "..."
        lines.append(f"{name:58s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:11.1f} "
                     f"{float(r['TotalDurationNs']) / 1e3:12.1f} {float(r['Percentage']):7.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def _kernel_of(kernel_id):
    """Name fragment of the per-kind decode kernel (LZ77 has its own)."""
    kind = KIND_OF_ID[kernel_id]
    return {"LZ77": "k_decode_lz<", "ANS": "k_decode_ans", "SDICT": "k_decode_sdict"}.get(
        kind, f"k_decode_kind<{kernel_id}u>")


def _per_dispatch(path, kernel_id):
    agg = collections.defaultdict(float)
    frag = _kernel_of(kernel_id)
    for r in csv.DictReader(open(path)):
        if frag in r["Kernel_Name"]:
            agg[r["Dispatch_Id"]] += float(r["Counter_Value"])
    v = sorted(agg.values())
    return v[len(v) // 2] * 1024 if v else None  # KiB -> bytes


def traffic(root, out_dir, command):
    def f(w, c):
        return os.path.join(root, f"pmc_{w}_{c}", "run_counter_collection.csv")
    workloads = sorted({d[4:].rsplit("_", 2)[0] for d in os.listdir(root)
                        if d.startswith("pmc_") and d.endswith(("_FETCH_SIZE", "_WRITE_SIZE"))})
    copy_id = KIND_OF_ID.index("PLAIN")
    sf = (1 << 30) / _per_dispatch(f("copy", "FETCH_SIZE"), copy_id)
    sw = (1 << 30) / _per_dispatch(f("copy", "WRITE_SIZE"), copy_id)
    lines = ["# HBM traffic per launch of each decode kernel, from rocprofv3 PMC counters",
             "# (one counter per run; FETCH_SIZE and WRITE_SIZE in KiB, summed over the agent's",
             "# instances per dispatch, median dispatch), scaled by what each counter reads for the",
             "# PLAIN copy kernel moving exactly 1 GiB in and 1 GiB out.",
             f"# command per counter C and workload W: {command}",
             f"# scale: FETCH_SIZE x {sf:.4f}, WRITE_SIZE x {sw:.4f}",
             f"kernel_sha: {kernel_sha()}"]
    for w in workloads:
        if not os.path.exists(f(w, "FETCH_SIZE")) or not os.path.exists(f(w, "WRITE_SIZE")):
            continue
        for kid, kind in enumerate(KIND_OF_ID):
            rd = _per_dispatch(f(w, "FETCH_SIZE"), kid)
            wr = _per_dispatch(f(w, "WRITE_SIZE"), kid)
            if rd is None or wr is None:
                continue
            lines.append(f"# {w}/{kind}: read {rd * sf / 2**30:.3f} GiB, write {wr * sw / 2**30:.3f} GiB")
            lines.append(f"{w}/{kind}: {rd * sf + wr * sw:.0f}")
    with open(os.path.join(out_dir, "traffic.txt"), "w") as fo:
        fo.write("\n".join(lines) + "\n")


def counters(csv_paths, fragments, out_path, command):
    """Median per-dispatch value of every counter in the given
    run_counter_collection.csv files for the kernels whose names contain each
    of the comma-separated `fragments` (each dispatch's value summed over the
    agent's instances), one section per kernel."""
    lines = [f"# rocprofv3 --pmc counters, median per dispatch, of kernels matching {fragments}",
             f"# command (one run per counter set): {command}", f"# kernel sources sha: {kernel_sha()}"]
    for fragment in fragments.split(","):
        rows = {}
        for path in csv_paths:
            per = collections.defaultdict(lambda: collections.defaultdict(float))
            for r in csv.DictReader(open(path)):
                if fragment in r["Kernel_Name"]:
                    per[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
            for name, d in per.items():
                v = sorted(d.values())
                rows[name] = (v[len(v) // 2], len(v))
        lines += ["", f"## {fragment}"]
        for name in sorted(rows):
            lines.append(f"{name:32s} {rows[name][0]:18.0f}   ({rows[name][1]} dispatches)")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def copies(stats_csv, trace_csv, out_path, command, piece_bytes=256 << 20):
    """Host-to-device copy summary: calls and durations per direction, and
    the link rate from the raw-copy leg's fixed-size pieces (the copies whose
    byte count is piece_bytes, or, when the trace has no sizes, the longest
    copies, which are those pieces)."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 --memory-copy-trace --stats summary ({os.path.basename(stats_csv)}, "
             f"{os.path.basename(trace_csv)})", f"# command: {command}", "",
             f"{'direction':32s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s}"]
    for r in rows:
        lines.append(f"{r['Name']:32s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.1f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.2f}")
    tr = [r for r in csv.DictReader(open(trace_csv)) if "HOST_TO_DEVICE" in r.get("Direction", r.get("Kind", ""))
          or "HOST_TO_DEVICE" in " ".join(r.values())]
    size_key = next((k for k in ("Size", "Bytes", "Copy_Bytes") if tr and k in tr[0]), None)
    dur = lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9  # noqa: E731
    if size_key:
        pieces = [r for r in tr if int(r[size_key]) == piece_bytes]
    else:
        d = sorted(dur(r) for r in tr)
        cut = d[-1] * 0.85 if d else 0
        pieces = [r for r in tr if dur(r) >= cut]
    if pieces:
        t = sum(dur(r) for r in pieces) / len(pieces)
        lines += ["", f"raw-copy pieces of {piece_bytes >> 20} MiB: {len(pieces)} copies, average {t * 1e3:.3f} ms "
                  f"-> {piece_bytes / t / 1e9:.1f} GB/s host to device "
                  f"({'by byte count' if size_key else 'the longest copies'})"]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "copies":
        # copies <run_memory_copy_stats.csv> <run_memory_copy_trace.csv> <out.txt> "<command>"
        copies(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif sys.argv[1] == "counters":
        # counters <out.txt> <kernel fragment> "<command>" <csv> [<csv> ...]
        counters(sys.argv[5:], sys.argv[3], sys.argv[2], sys.argv[4])
