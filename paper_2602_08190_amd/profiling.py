"""Summaries of rocprofv3 output for the profiles/ folder.

    python -m paper_2602_08190_amd.profiling stats <run_kernel_stats.csv> <out.txt> "<command>"
    python -m paper_2602_08190_amd.profiling traffic <pmc_root> <out_dir> "<command>"
    python -m paper_2602_08190_amd.profiling counters <out.txt> <kernel> "<command>" <csv> [<csv> ...]

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


def counters(csv_paths, fragment, out_path, command):
    """Median per-dispatch value of every counter in the given
    run_counter_collection.csv files for kernels whose name contains
    `fragment` (each dispatch's value summed over the agent's instances)."""
    rows = {}
    for path in csv_paths:
        per = collections.defaultdict(lambda: collections.defaultdict(float))
        for r in csv.DictReader(open(path)):
            if fragment in r["Kernel_Name"]:
                per[r["Counter_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
        for name, d in per.items():
            v = sorted(d.values())
            rows[name] = (v[len(v) // 2], len(v))
    lines = [f"# rocprofv3 --pmc counters of kernels matching '{fragment}', median per dispatch",
             f"# command (one run per counter set): {command}", f"# kernel sources sha: {kernel_sha()}", ""]
    for name in sorted(rows):
        lines.append(f"{name:32s} {rows[name][0]:18.0f}   ({rows[name][1]} dispatches)")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "counters":
        # counters <out.txt> <kernel fragment> "<command>" <csv> [<csv> ...]
        counters(sys.argv[5:], sys.argv[3], sys.argv[2], sys.argv[4])
