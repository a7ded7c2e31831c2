"""Summaries of rocprofv3 output for the solver's kernels (plain text, for
the profile records kept with the sources).

    python -m paper_1802_10323_amd.profiling stats  --csv <run_kernel_stats.csv> --out <txt> --command "<cmd>"
    python -m paper_1802_10323_amd.profiling traffic --fetch <fetch run_counter_collection.csv>
        --write <write run_counter_collection.csv> --copy-bytes <B> --workload <name>
        --out <txt> --command "<cmd>" [--command "<cmd>"]

`traffic` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch)
into HBM bytes per launch of each solver stage.  Each counter is scaled by
what it reads for a plain device copy of known size in the same run (the
runtime's copy kernel, `__amd_rocclr_copyBuffer`, at its largest grid in
the run, moving `--copy-bytes` bytes each way): factor = true bytes /
counter bytes.  Solver dispatches
come five per solve in stage order (forward t1, forward t2, elimination,
backward t2, backward t1).
"""
import argparse
import csv
import hashlib
import os
import statistics
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
STAGES = ("fwd_t1", "fwd_t2", "tridiag", "inv_t2", "inv_t1")
COPY_KERNEL = "__amd_rocclr_copyBuffer"
SOLVER_TAG = "poisson_dev::"


def kernel_source_hash():
    """Hash of every kernel source file: a stored counter reading applies
    only to the kernels it was taken on."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".h", ".hip")):
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    return name.replace("poisson_dev::", "").split("(")[0]


def read_counters(path, counter):
    """[(dispatch id, kernel name, value)] in dispatch order; plain copies
    other than the largest (the field-sized ones) are dropped."""
    per = defaultdict(float)
    names = {}
    grid = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            d = int(r["Dispatch_Id"])
            per[d] += float(r["Counter_Value"])
            names[d] = r["Kernel_Name"]
            grid[d] = int(r["Grid_Size"])
    big = max([grid[d] for d in names if names[d] == COPY_KERNEL] or [0])
    return [(d, names[d], per[d]) for d in sorted(per)
            if names[d] != COPY_KERNEL or grid[d] == big]


def stage_values(rows):
    """Per stage: (kernel name, [counter values]) of the solver dispatches."""
    solver = [(n, v) for _, n, v in rows if SOLVER_TAG in n]
    out = {s: [None, []] for s in STAGES}
    for i, (n, v) in enumerate(solver):
        s = STAGES[i % len(STAGES)]
        out[s][0] = n
        out[s][1].append(v)
    return out


def copy_factor(rows, copy_bytes):
    vals = [v for _, n, v in rows if n == COPY_KERNEL]
    if not vals:
        raise SystemExit("no plain copy dispatch in the counter file")
    med = statistics.median(vals) * 1024.0
    return copy_bytes / med, statistics.median(vals), len(vals)


def cmd_traffic(a):
    fetch = read_counters(a.fetch, "FETCH_SIZE")
    write = read_counters(a.write, "WRITE_SIZE")
    ff, fmed, fn = copy_factor(fetch, a.copy_bytes)
    wf, wmed, wn = copy_factor(write, a.copy_bytes)
    fs, ws = stage_values(fetch), stage_values(write)
    lines = [f"# HBM traffic per launch of each solver stage, workload {a.workload}",
             "# from rocprofv3 hardware counters (KiB per dispatch), one pass per counter:"]
    lines += [f"#   {c}" for c in a.command]
    lines += [f"# calibration: plain copy of {a.copy_bytes} B each way in the same runs "
              f"({COPY_KERNEL}): FETCH_SIZE median {fmed:.0f} KiB over {fn} copies -> "
              f"factor {ff:.4f}; WRITE_SIZE median {wmed:.0f} KiB over {wn} copies -> "
              f"factor {wf:.4f}",
              "# bytes_per_launch = fetch_KiB * 1024 * fetch factor + write_KiB * 1024 * write factor "
              "(medians over the launches of the stage)",
              f"kernel_source_hash {kernel_source_hash()}",
              f"copy_factors fetch {ff:.6f} write {wf:.6f}"]
    for s in STAGES:
        name, fv = fs[s]
        _, wv = ws[s]
        if not fv or not wv:
            continue
        fk, wk = statistics.median(fv), statistics.median(wv)
        total = fk * 1024 * ff + wk * 1024 * wf
        lines.append(f"stage {s} kernel {short_name(name).replace(' ', '')} launches {len(fv)} "
                     f"fetch_KiB {fk:.0f} write_KiB {wk:.0f} bytes_per_launch {total:.0f}")
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text, end="")


def cmd_stats(a):
    rows = []
    with open(a.csv) as fh:
        for r in csv.DictReader(fh):
            rows.append(r)
    lines = ["# rocprofv3 --kernel-trace --stats summary", "# command:"]
    lines += [f"#   {c}" for c in a.command]
    lines.append(f"# kernel sources {kernel_source_hash()}")
    # whole template argument lists (kind, direction, form of each
    # instantiation), without the spaces
    names = [short_name(r["Name"]).replace(", ", ",").removeprefix("void ") for r in rows]
    w = min(100, max([60] + [len(n) for n in names]))
    names = [n[:w] for n in names]
    lines.append(f"{'kernel':{w}s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s} {'pct':>6s}")
    for r, name in zip(rows, names):
        lines.append(f"{name:{w}s} {int(r['Calls']):6d} "
                     f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                     f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                     f"{float(r['Percentage']):6.2f}")
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text, end="")


def cmd_counters(a):
    """Per solver stage, the median per launch of every counter in one
    counter file (any counters, e.g. address-translation ones)."""
    names = set()
    with open(a.csv) as fh:
        for r in csv.DictReader(fh):
            names.add(r["Counter_Name"])
    names = sorted(names)
    per = {c: stage_values(read_counters(a.csv, c)) for c in names}
    what = "kernel (medians over its launches)" if a.kernels else "solver stage"
    lines = [f"# hardware counters per launch of each {what}, workload {a.workload}",
             "# command:"]
    lines += [f"#   {c}" for c in a.command]
    lines.append(f"kernel_source_hash {kernel_source_hash()}")
    if a.kernels:
        # per kernel instead of per solver stage: medians over its launches
        # of the launches that did work (more than one wave)
        per_k = {}
        with open(a.csv) as fh:
            for r in csv.DictReader(fh):
                k = short_name(r["Kernel_Name"]).replace(" ", "")
                per_k.setdefault(k, {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        for k, cs in sorted(per_k.items()):
            if not any(x in k for x in a.kernels.split(",")):
                continue
            vals = " ".join(f"{c} {statistics.median(v):.0f}" for c, v in sorted(cs.items()))
            lines.append(f"kernel {k} {vals}")
        text = "\n".join(lines) + "\n"
        with open(a.out, "w") as fh:
            fh.write(text)
        print(text, end="")
        return
    for s in STAGES:
        kname = next((per[c][s][0] for c in names if per[c][s][0]), None)
        if kname is None:
            continue
        vals = " ".join(f"{c} {statistics.median(per[c][s][1]):.0f}" for c in names if per[c][s][1])
        lines.append(f"stage {s} kernel {short_name(kname).replace(' ', '')} {vals}")
    text = "\n".join(lines) + "\n"
    with open(a.out, "w") as fh:
        fh.write(text)
    print(text, end="")


def read_traffic(path):
    """{stage: bytes per launch} from a traffic summary, with its source hash."""
    out, src = {}, None
    with open(path) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "kernel_source_hash":
                src = f[1]
            elif f[0] == "stage":
                out[f[1]] = float(f[f.index("bytes_per_launch") + 1])
    return src, out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--command", action="append", default=[])
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--command", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--kernels", default="",
                   help="comma list of name fragments: summarise these kernels, not the solver stages")
    a = ap.parse_args()
    {"traffic": cmd_traffic, "stats": cmd_stats, "counters": cmd_counters}[a.what](a)


if __name__ == "__main__":
    main()
