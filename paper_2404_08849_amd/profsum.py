"""Summaries of rocprofv3 runs of the benchmark, and the record bench.py reads back.

A profile directory holds the outputs of five runs of one workload (kernel
trace of the timed benchmark, FETCH_SIZE and WRITE_SIZE counter passes of the
same launch shapes, and the two counter passes over a plain device copy of
known size), the benchmark's JSON line from the traced run and the commands.
`summarize` turns it into a short markdown file: per-kernel durations, the
dominant kernel's average against the benchmark's own HIP-event figure, and
its HBM traffic per launch, each counter divided by what that counter reads
per byte actually copied by the copy kernel.

The file ends with a `record` block (key: value lines) that the benchmark
reads to report `traffic`; it carries a digest of the library sources and is
ignored once they change.

    python -m paper_2404_08849_amd.profsum DIR OUT.md
"""
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))


def source_digest():
    """sha256 over every library source and the build script (names + bytes)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [os.path.join(HERE, "build.py")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_record(path):
    """key -> value (str) from the ```record block of a summary, or {}."""
    if not os.path.exists(path):
        return {}
    rec, inside = {}, False
    with open(path) as fh:
        for line in fh:
            s = line.strip()
            if s == "```record":
                inside = True
            elif inside and s == "```":
                break
            elif inside and ":" in s:
                k, v = s.split(":", 1)
                rec[k.strip()] = v.strip()
    return rec


def kernel_instance(kernel, policy_real, vpl):
    """Regex for the template instance of a library kernel (class, FP type, values per lane)."""
    return re.compile(r"mpdc::%s<(?:\d+, )?%s, %d[,>]" % (re.escape(kernel), policy_real, vpl))


def _csv(path_glob):
    paths = glob.glob(path_glob, recursive=True)
    if not paths:
        raise FileNotFoundError(path_glob)
    with open(paths[0]) as fh:
        return list(csv.DictReader(fh))


def _short(name):
    for pat in (r"mpdc::\w+<[^>]*>", r"mpdc::\w+", r"__amd_rocclr_\w+"):
        m = re.search(pat, name)
        if m:
            return m.group(0)
    return name[:60]


def _counter(rows, counter, pred):
    vals = [float(r["Counter_Value"]) for r in rows if r["Counter_Name"] == counter and pred(r["Kernel_Name"])]
    return vals


def summarize(d, out):
    bench = None
    with open(os.path.join(d, "bench_trace.json")) as fh:
        for line in fh:
            if line.startswith("{"):
                bench = json.loads(line)
    if bench is None:
        raise RuntimeError("no benchmark JSON line in bench_trace.json")
    with open(os.path.join(d, "commands.txt")) as fh:
        commands = fh.read().strip()
    rf = bench["roofline"]
    kernel = rf["kernel"]
    dycore = ["k_cell_a", "k_vertex", "k_cell_b", "k_edge"]
    tracer = ["k_tr_low", "k_tr_limit", "k_tr_update"]
    names = tracer if kernel in tracer else dycore
    shapes = bench["launch_shapes"]["mix"]
    if isinstance(shapes, dict):   # coupled runs: shapes per model
        shapes = shapes["tracer" if kernel in tracer else "dycore"]
    vpl, group = shapes[names.index(kernel)]
    inst = kernel_instance(kernel, "float", vpl)

    stats = _csv(os.path.join(d, "trace", "**", "*kernel_stats.csv"))
    trace = _csv(os.path.join(d, "trace", "**", "*kernel_trace.csv"))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in trace
            if inst.search(r["Kernel_Name"])]
    stat = [r for r in stats if inst.search(r["Name"])]
    if not stat:
        raise RuntimeError("dominant kernel instance not in the trace")
    avg_ms = float(stat[0]["AverageNs"]) * 1e-6

    fetch = _csv(os.path.join(d, "fetch", "**", "*counter_collection.csv"))
    write = _csv(os.path.join(d, "write", "**", "*counter_collection.csv"))
    cfetch = _csv(os.path.join(d, "copy_fetch", "**", "*counter_collection.csv"))
    cwrite = _csv(os.path.join(d, "copy_write", "**", "*counter_collection.csv"))
    with open(os.path.join(d, "copy.json")) as fh:
        copy = json.loads([l for l in fh if l.startswith("{")][-1])
    copy_bytes = copy["copy_calibration_bytes_each_way"]
    is_copy = lambda n: "copyBuffer" in n
    cf = _counter(cfetch, "FETCH_SIZE", is_copy)
    cw = _counter(cwrite, "WRITE_SIZE", is_copy)
    # counters read KiB per dispatch; the copy kernel moves copy_bytes each way
    f_factor = (sum(cf) / len(cf)) * 1024.0 / copy_bytes
    w_factor = (sum(cw) / len(cw)) * 1024.0 / copy_bytes
    kf = _counter(fetch, "FETCH_SIZE", inst.search)
    kw = _counter(write, "WRITE_SIZE", inst.search)
    fetch_b = sum(kf) / len(kf) * 1024.0 / f_factor
    write_b = sum(kw) / len(kw) * 1024.0 / w_factor
    traffic = fetch_b + write_b

    L = []
    L.append("# %s, %s: kernel durations and HBM traffic (MI355X)" % (kernel, bench["config"]["workload"]))
    L.append("")
    L.append("Commands (run from the repository root; rocprofv3 writes CSV):")
    L.append("")
    L.append("```")
    L.append(commands)
    L.append("```")
    L.append("")
    L.append("Launch shapes (values per lane, cells or threads per work-group), mixed policy: %s; "
             "all-FP64: %s." % (bench["launch_shapes"]["mix"], bench["launch_shapes"]["dbl"]))
    L.append("")
    L.append("## Kernel trace (rocprofv3 --kernel-trace --stats)")
    L.append("")
    L.append("| kernel instance | calls | average us | share % |")
    L.append("|---|---:|---:|---:|")
    for r in stats:
        L.append("| %s | %s | %.2f | %.2f |" % (_short(r["Name"]), r["Calls"], float(r["AverageNs"]) * 1e-3,
                                            float(r["Percentage"])))
    L.append("")
    in_step = rf.get("ms_per_launch_in_step")
    L.append("Dominant kernel of the mixed step: `%s` (values per lane %d, group %d).  "
             "Profiler average %.2f us over %d dispatches (trace: min %.2f, max %.2f us); the benchmark's "
             "HIP-event average in the same run: %.2f us over back-to-back launches of the first RK stage "
             "(used for `achieved`)%s."
             % (_short(stat[0]["Name"]), vpl, group, avg_ms * 1e3, len(durs), min(durs) * 1e3, max(durs) * 1e3,
                rf["ms_per_launch"] * 1e3,
                ", %.2f us between the launches of whole steps (event and launch overhead included)"
                % (in_step * 1e3) if in_step else ""))
    L.append("")
    L.append("## HBM traffic (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE)")
    L.append("")
    L.append("Copy calibration: a device copy of %d bytes reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB "
             "per dispatch, i.e. %.3f and %.3f counter bytes per byte moved."
             % (copy_bytes, sum(cf) / len(cf), sum(cw) / len(cw), f_factor, w_factor))
    L.append("")
    L.append("| kernel instance | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM read MB | HBM write MB |")
    L.append("|---|---:|---:|---:|---:|")
    per = defaultdict(lambda: [[], []])
    for r in fetch:
        if r["Counter_Name"] == "FETCH_SIZE" and "mpdc::" in r["Kernel_Name"]:
            per[_short(r["Kernel_Name"])][0].append(float(r["Counter_Value"]))
    for r in write:
        if r["Counter_Name"] == "WRITE_SIZE" and "mpdc::" in r["Kernel_Name"]:
            per[_short(r["Kernel_Name"])][1].append(float(r["Counter_Value"]))
    for k in sorted(per):
        f, w = per[k]
        if not f or not w:
            continue
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        L.append("| %s | %.0f | %.0f | %.2f | %.2f |" % (k, fm, wm, fm * 1024 / f_factor / 1e6,
                                                        wm * 1024 / w_factor / 1e6))
    L.append("")
    alg = rf.get("bytes_per_launch_mean", rf["bytes_per_launch"])   # the dispatches span all RK stages
    L.append("Dominant kernel: algorithmic bytes per launch %.3f MB (mean over the RK stages; %.3f MB in the "
             "first stage, the one timed back to back); measured HBM traffic per launch %.3f MB "
             "(read %.3f + write %.3f), ratio %.2f."
             % (alg / 1e6, rf["bytes_per_launch"] / 1e6, traffic / 1e6, fetch_b / 1e6, write_b / 1e6,
                traffic / alg))
    L.append("")
    L.append("```record")
    L.append("workload: %s" % bench["config"]["workload"])
    L.append("kernel: %s" % kernel)
    L.append("values_per_lane: %d" % vpl)
    L.append("group: %d" % group)
    L.append("profiler_avg_us: %.3f" % (avg_ms * 1e3))
    L.append("traffic_bytes_per_launch: %.0f" % traffic)
    L.append("fetch_factor: %.4f" % f_factor)
    L.append("write_factor: %.4f" % w_factor)
    L.append("source_sha256: %s" % bench.get("source_sha256", ""))
    L.append("```")
    with open(out, "w") as fh:
        fh.write("\n".join(L) + "\n")
    return out


if __name__ == "__main__":
    if len(sys.argv) != 3:
        sys.exit(__doc__)
    print(summarize(sys.argv[1], sys.argv[2]))
