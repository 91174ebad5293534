"""Summaries of rocprofv3 output for the smoother roofline.

    python -m paper_1805_10167_amd.profiling summarize \
        --stats DIR --fetch DIR --write DIR --kernel NAME --out FILE --cmd "..."
    python -m paper_1805_10167_amd.profiling counters \
        --stats DIR --pmc DIR [DIR ...] --kernel NAME --out FILE --cmd "..."
    python -m paper_1805_10167_amd.profiling trace \
        --stats DIR --kernels NAME ... --alg-bytes B ... --source FILE --out FILE --cmd "..."

reads the kernel-trace CSV of one run (average duration per kernel and grid
size) and the counter CSVs of two --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB
per dispatch).  Counter values are scaled by what the same counters report
for a plain copy of known size in the same run (the runtime's copyBuffer
kernel), so that they read as HBM bytes.  The summary records a hash of the
kernel source; `traffic_for` returns the figures only while that source is
unchanged.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
HEADERS = ["hhg_internal.hpp", "hhg_kernels.hpp", "hhg_mesh.hpp", "hhg_device.hpp"]
# the files a profiled kernel is built from, by the source file holding it
SOURCES = {name: [name] + HEADERS for name in ("kernels.hip", "net.hip", "stokes.hip", "transport.hip", "p2.hip")}
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def source_hash(files=("kernels.hip",)):
    """Hash of the given csrc files (the kernel's source and its headers)."""
    h = hashlib.sha256()
    for name in files:
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def _csv(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise FileNotFoundError("no *%s under %s" % (suffix, d))
    return list(csv.DictReader(open(files[0])))


def kernel_durations(trace_dir):
    """(kernel name, grid) -> list of durations in ns."""
    out = defaultdict(list)
    for r in _csv(trace_dir, "kernel_trace.csv"):
        out[(r["Kernel_Name"], int(r["Grid_Size_X"]))].append(
            int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return out


def counter_values(pmc_dir):
    """(kernel name, grid) -> list of counter values (KiB per dispatch)."""
    out = defaultdict(list)
    for r in _csv(pmc_dir, "counter_collection.csv"):
        out[(r["Kernel_Name"], int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return out


def _plain(name):
    """Kernel name without the "void " that template instances carry."""
    return name[5:] if name.startswith("void ") else name


def _largest(d, name):
    keys = [k for k in d if _plain(k[0]).startswith(_plain(name))]
    if not keys:
        raise KeyError(name)
    return max(keys, key=lambda k: k[1])


def summarize(stats_dir, fetch_dir, write_dir, kernel, copy_bytes, cmd, source="kernels.hip"):
    dur = kernel_durations(stats_dir)
    fetch = counter_values(fetch_dir)
    write = counter_values(write_dir)
    kd = _largest(dur, kernel)
    kf, kw = _largest(fetch, kernel), _largest(write, kernel)
    cf, cw = _largest(fetch, COPY_KERNEL), _largest(write, COPY_KERNEL)
    mean = lambda v: sum(v) / len(v)
    for tab, key, name in ((fetch, cf, "FETCH_SIZE"), (write, cw, "WRITE_SIZE")):
        # the calibration copy must be the only copy of its grid in the run:
        # copies of other sizes on the same grid would skew the scale
        if max(tab[key]) > 1.01 * min(tab[key]):
            raise ValueError("%s of the copy dispatches on grid %d ranges from %.0f to %.0f KiB: the run holds "
                             "copies other than the calibration copy; profile without them"
                             % (name, key[1], min(tab[key]), max(tab[key])))
    fetch_scale = copy_bytes / (mean(fetch[cf]) * 1024.0)
    write_scale = copy_bytes / (mean(write[cw]) * 1024.0)
    fetch_b = mean(fetch[kf]) * 1024.0 * fetch_scale
    write_b = mean(write[kw]) * 1024.0 * write_scale
    top = sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:12]
    return {
        "kernel": kernel, "grid": kd[1], "dispatches": len(dur[kd]),
        "avg_duration_us": mean(dur[kd]) / 1e3,
        "fetch_bytes": fetch_b, "write_bytes": write_b, "traffic_bytes": fetch_b + write_b,
        "fetch_scale": fetch_scale, "write_scale": write_scale,
        "copy_bytes": copy_bytes, "source_files": SOURCES[source],
        "source_hash": source_hash(SOURCES[source]), "command": cmd,
        "top_kernels_us": [[k[0].split("(")[0][:80], k[1], len(v), sum(v) / 1e3, mean(v) / 1e3]
                           for k, v in top],
    }


def trace_summary(stats_dir, kernels, bytes_per_dispatch, cmd, out, source):
    """Average duration of the largest-grid dispatches of each kernel in
    `kernels`, with the achieved rate of its algorithmic bytes per dispatch
    (0: not stated)."""
    dur = kernel_durations(stats_dir)
    mean = lambda v: sum(v) / len(v)
    lines = ["# rocprofv3 kernel trace: %s" % ", ".join(kernels), "", "command: " + cmd,
             "kernel source hash: %s (%s)" % (source_hash(SOURCES[source]), ", ".join(SOURCES[source])), "",
             "kernel, grid, dispatches, average us, algorithmic MB per dispatch, TB/s:"]
    rec = []
    for name, nb in zip(kernels, bytes_per_dispatch):
        kd = _largest(dur, name)
        us = mean(dur[kd]) / 1e3
        rate = nb / (us * 1e-6) / 1e12 if nb else 0.0
        lines.append("  %-60s %8d %7d %9.2f %9.1f %6.2f" % (kd[0].split("(")[0][:60], kd[1], len(dur[kd]), us,
                                                            nb / 1e6, rate))
        rec.append({"kernel": kd[0].split("(")[0], "grid": kd[1], "dispatches": len(dur[kd]),
                    "avg_duration_us": us, "alg_bytes": nb, "tb_per_s": rate})
    top = sorted(dur.items(), key=lambda kv: -sum(kv[1]))[:16]
    lines += ["", "top kernels by total time (name, grid, dispatches, total us, avg us):"]
    for k, v in top:
        lines.append("  %-70s %9d %7d %10.1f %9.2f" % (k[0].split("(")[0][:70], k[1], len(v), sum(v) / 1e3,
                                                      mean(v) / 1e3))
    lines += ["", "json: " + json.dumps({"kernels": rec, "command": cmd, "source_files": SOURCES[source],
                                         "source_hash": source_hash(SOURCES[source])})]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_summary(s, path):
    lines = ["# rocprofv3 summary: %s (grid %d)" % (s["kernel"], s["grid"]), "",
             "command: %s" % s["command"],
             "kernel source hash: %s (%s)" % (s["source_hash"], ", ".join(s["source_files"])), "",
             "average duration: %.2f us over %d dispatches" % (s["avg_duration_us"], s["dispatches"]),
             "HBM fetch: %.1f MB, write: %.1f MB per dispatch" % (s["fetch_bytes"] / 1e6,
                                                                 s["write_bytes"] / 1e6),
             "counter scale (plain copy of %d bytes): FETCH_SIZE x%.3f, WRITE_SIZE x%.3f"
             % (s["copy_bytes"], s["fetch_scale"], s["write_scale"]), "",
             "top kernels by total time (name, grid, dispatches, total us, avg us):"]
    for row in s["top_kernels_us"]:
        lines.append("  %-80s %9d %6d %10.1f %9.2f" % tuple(row))
    lines += ["", "json: " + json.dumps({k: v for k, v in s.items() if k != "top_kernels_us"})]
    open(path, "w").write("\n".join(lines) + "\n")


def traffic_for(path):
    """HBM bytes per dispatch recorded in a summary, or None if the kernel
    source has changed since (or the file is missing)."""
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("json: "):
            s = json.loads(line[6:])
            files = s.get("source_files", ["kernels.hip"])
            return s["traffic_bytes"] if s.get("source_hash") == source_hash(files) else None
    return None


def counter_table(pmc_dir):
    """(kernel name, grid) -> {counter name: [values per dispatch]}."""
    out = defaultdict(lambda: defaultdict(list))
    for r in _csv(pmc_dir, "counter_collection.csv"):
        out[(r["Kernel_Name"], int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def counters_summary(stats_dir, pmc_dirs, kernel, cmd, out, source="net.hip"):
    """Average duration and counters of the largest-grid dispatches of
    `kernel`; MFMA operation counters (units of 512 flops) are turned into
    achieved matrix-core TFLOP/s."""
    dur = kernel_durations(stats_dir)
    kd = _largest(dur, kernel)
    avg_ns = sum(dur[kd]) / len(dur[kd])
    vals = {}
    for d in pmc_dirs:
        tab = counter_table(d)
        kk = _largest(tab, kernel)
        for name, v in tab[kk].items():
            vals[name] = sum(v) / len(v)
    lines = ["# rocprofv3 counters: %s (grid %d)" % (kd[0], kd[1]), "",
             "command: " + cmd, "kernel source hash: " + source_hash(SOURCES[source]), "",
             "average duration: %.2f us over %d dispatches" % (avg_ns / 1e3, len(dur[kd])), "",
             "counters (average per dispatch):"]
    for name in sorted(vals):
        lines.append("  %-34s %.4g" % (name, vals[name]))
    mops = [v for n, v in vals.items() if n.startswith("SQ_INSTS_VALU_MFMA_MOPS_")]
    rec = {"kernel": kd[0], "grid": kd[1], "avg_duration_us": avg_ns / 1e3, "counters": vals,
           "command": cmd, "source_files": SOURCES[source], "source_hash": source_hash(SOURCES[source])}
    if mops:
        flops = 512.0 * sum(mops)
        rec["mfma_flops"] = flops
        rec["mfma_tflops"] = flops / avg_ns / 1e3
        lines += ["", "matrix-core work: %.4g flop per dispatch (MOPS x 512) -> %.2f TFLOP/s achieved"
                  % (flops, rec["mfma_tflops"])]
    lines += ["", "json: " + json.dumps(rec)]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def cycle_breakdown(stats_dir, cycles, finest, cmd, out):
    """Kernel time of `cycles` V-cycles by kernel and level.  The launches of
    each kernel are grouped by grid size; within one kernel the grids are
    distinct per level and shrink with it, so the k-th largest grid of a
    kernel is taken as level finest - k (kernels launched on fewer levels,
    e.g. the coarse solve, are labelled by the same rank)."""
    dur = kernel_durations(stats_dir)
    by_name = defaultdict(list)
    for (name, grid), v in dur.items():
        by_name[name.split("(")[0]].append((grid, v))
    rows = []
    for name, lst in by_name.items():
        lst.sort(key=lambda gv: -gv[0])
        for rank, (grid, v) in enumerate(lst):
            rows.append((finest - rank, name, grid, len(v) / cycles, sum(v) / 1e3 / cycles))
    rows.sort(key=lambda r: (-r[0], -r[4]))
    per_level = defaultdict(float)
    for lvl, _, _, _, us in rows:
        per_level[lvl] += us
    total = sum(per_level.values())
    lines = ["# rocprofv3 per-level kernel time of one V-cycle", "", "command: " + cmd,
             "cycles in the trace: %d; finest level %d" % (cycles, finest), "",
             "kernel time per cycle by level (us):"]
    for lvl in sorted(per_level, reverse=True):
        lines.append("  level %2d  %9.1f  (%4.1f%%)" % (lvl, per_level[lvl], 100 * per_level[lvl] / total))
    lines += ["  total     %9.1f" % total, "",
              "by kernel (level, name, grid, launches per cycle, us per cycle):"]
    for lvl, name, grid, cnt, us in rows:
        lines.append("  %2d  %-70s %9d %6.1f %9.1f" % (lvl, name[:70], grid, cnt, us))
    lines += ["", "json: " + json.dumps({"cycles": cycles, "finest": finest, "command": cmd,
                                         "per_level_us": {str(k): v for k, v in per_level.items()},
                                         "total_us": total})]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["summarize", "counters", "cycle", "trace"])
    ap.add_argument("--kernels", nargs="*", default=[])
    ap.add_argument("--alg-bytes", nargs="*", type=float, default=[])
    ap.add_argument("--cycles", type=int, default=1)
    ap.add_argument("--finest", type=int, default=10)
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--kernel", default="")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--source", default=None, help="csrc file holding the kernel")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.mode == "summarize":
        s = summarize(a.stats, a.fetch, a.write, a.kernel, a.copy_bytes, a.cmd,
                      a.source or "kernels.hip")
        write_summary(s, a.out)
    elif a.mode == "trace":
        nb = a.alg_bytes + [0.0] * (len(a.kernels) - len(a.alg_bytes))
        trace_summary(a.stats, a.kernels, nb, a.cmd, a.out, a.source or "stokes.hip")
    elif a.mode == "cycle":
        cycle_breakdown(a.stats, a.cycles, a.finest, a.cmd, a.out)
    else:
        counters_summary(a.stats, a.pmc, a.kernel, a.cmd, a.out, a.source or "net.hip")
    print(open(a.out).read())


if __name__ == "__main__":
    main()
