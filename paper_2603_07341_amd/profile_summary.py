"""Text summaries of rocprofv3 runs of the benchmark, for profiles/.

The benchmark brackets a 1 GiB plain device copy with marks 0 and 1 and its
timed window with marks 2 and 3 (empty k_mark dispatches, see
paces_profile_mark).  Given the output folders of three runs of the same
command -- a kernel trace with --stats, a FETCH_SIZE counter run and a
WRITE_SIZE counter run -- this module writes one summary:

  * the window's per-kernel dispatch count and time (trace) and HBM bytes
    (counters, each scaled so that the copy reads as 1 GiB fetched and
    1 GiB written);
  * per stage of the step (select, expand+build, transfer, propagate,
    observe) the counted bytes and kernel time per timed step, stages being
    assigned in dispatch order from the first kernel of each stage;
  * the middle Clenshaw term's mean bytes and duration per launch;
  * the whole-run --stats table.

Lines "key: value" are read back by bench.py, which uses them only when the
kernel sources (comments ignored) and the window (growth, warm-up and timed
steps, |S| at both ends, from the bench's JSON line) are the same.

    python -m paper_2603_07341_amd.profile_summary --trace DIR --fetch DIR \
        --write DIR --bench-json FILE --command CMD --out FILE

The dispatches of a run between the copy's first mark and the window's
last mark can be kept as a small CSV (`... extract trace DIR OUT`,
`... extract FETCH_SIZE DIR OUT`, `... extract WRITE_SIZE DIR OUT`) and
given to --trace / --fetch / --write in place of the folders.
"""
import argparse
import csv
import re
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
MID = "k_cheb_term<double, 1, 1, true>"
GIB = float(1 << 30)

# first kernel of each stage of a step, in dispatch order (a step from the
# previous graph starts its expansion with k_warm_old and turns psi into
# phi in place there: its transfer stage is only the fold of the dropped
# weight, counted with the expansion)
STAGE_START = [("k_begin_step", "select"), ("k_fill_u64", "expand+build"),
               ("k_warm_old", "expand+build"),
               ("k_transfer", "transfer"), ("k_bounds", "build"),
               ("k_cheb_term", "propagate"), ("k_pop_norm", "observe")]


def source_hash():
    """Hash of the step kernels' code, comments and blank lines ignored."""
    h = hashlib.sha256()
    for f in ["kernels.hip", "warm.hip", "device.hpp", "kernels.hpp",
              "warm.hpp", "common.hpp"]:
        with open(os.path.join(HERE, "csrc", f)) as fh:
            for line in fh:
                code = line.split("//")[0].rstrip()
                if code:
                    h.update((code + "\n").encode())
    return h.hexdigest()[:16]


def _csv(folder, suffix):
    files = sorted(glob.glob(os.path.join(folder, "**", "*" + suffix),
                             recursive=True))
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, folder))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _between(disp, lo, hi):
    """Dispatches strictly between marks lo and hi (dispatch order)."""
    marks = [d for d in disp if "k_mark" in d["name"]]
    if len(marks) < hi + 1:
        raise SystemExit("found %d marks, need %d" % (len(marks), hi + 1))
    a, b = marks[lo]["id"], marks[hi]["id"]
    return [d for d in disp if a < d["id"] < b]


_KNAME = re.compile(r"k_\w+(?:<[^()]*>)?")


def short_name(name):
    """Kernel name without return type, namespaces and parameter list
    ("k_cheb_term<double, 1, 1, true>"); names of other kernels as given."""
    m = _KNAME.search(name)
    return m.group(0) if m else name


def trace_dispatches(folder):
    out = []
    for r in _csv(folder, "kernel_trace.csv"):
        out.append({"id": int(r["Dispatch_Id"]),
                    "name": short_name(r["Kernel_Name"]),
                    "ns": int(r["End_Timestamp"]) - int(r["Start_Timestamp"])})
    return sorted(out, key=lambda d: d["id"])


def counter_dispatches(folder, counter):
    out = {}
    for r in _csv(folder, "counter_collection.csv"):
        if r["Counter_Name"] != counter:
            continue
        i = int(r["Dispatch_Id"])
        d = out.setdefault(i, {"id": i, "name": short_name(r["Kernel_Name"]),
                               "kib": 0.0})
        d["kib"] += float(r["Counter_Value"])
    return sorted(out.values(), key=lambda d: d["id"])


def write_window_rows(folder, kind, counter, path):
    """The dispatches between marks 0 and 3 of one run as a small CSV (id,
    name, value: ns or KiB), so that the summary can be redone from them."""
    disp = (trace_dispatches(folder) if kind == "trace"
            else counter_dispatches(folder, counter))
    key = "ns" if kind == "trace" else "kib"
    marks = [d for d in disp if "k_mark" in d["name"]]
    if len(marks) < 4:
        raise SystemExit("found %d marks, need 4" % len(marks))
    lo, hi = marks[0]["id"], marks[3]["id"]
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["id", "name", key])
        for d in disp:
            if lo <= d["id"] <= hi:
                w.writerow([d["id"], d["name"], d[key]])


def read_window_rows(path):
    seen, out = set(), []
    with open(path, newline="") as fh:
        r = csv.DictReader(fh)
        key = [f for f in r.fieldnames if f in ("ns", "kib")][0]
        for x in r:
            i = int(x["id"])
            if i not in seen:  # one row per dispatch
                seen.add(i)
                out.append({"id": i, "name": x["name"], key: float(x[key])})
    return sorted(out, key=lambda d: d["id"])


def stage_of(names):
    """Stage of each dispatch of a window given in order."""
    cur, out = "select", []
    for n in names:
        for prefix, st in STAGE_START:
            if n.startswith(prefix):
                cur = "expand+build" if st == "build" else st
                break
        out.append(cur)
    return out


def per_kernel(disp, key):
    agg = {}
    for d in disp:
        a = agg.setdefault(d["name"], [0, 0.0])
        a[0] += 1
        a[1] += d[key]
    return agg


def _load(path, kind, counter=None):
    if os.path.isfile(path):
        return read_window_rows(path)
    return (trace_dispatches(path) if kind == "trace"
            else counter_dispatches(path, counter))


def summarize(args):
    trace = _load(args.trace, "trace")
    fetch = _load(args.fetch, "counter", "FETCH_SIZE")
    write = _load(args.write, "counter", "WRITE_SIZE")
    with open(args.bench_json) as fh:
        line = [l for l in fh if l.strip().startswith("{")][-1]
    bench = json.loads(line)
    steps = int(bench["steps"])
    cfg = bench["config"]
    # calibration: the copy between marks 0 and 1 moves 1 GiB each way (the
    # fill that makes its source also lies between the marks: only the
    # copy dispatch counts)
    cf = sum(d["kib"] for d in _between(fetch, 0, 1)
             if "copyBuffer" in d["name"]) * 1024.0
    cw = sum(d["kib"] for d in _between(write, 0, 1)
             if "copyBuffer" in d["name"]) * 1024.0
    sf, sw = GIB / cf, GIB / cw
    tw, fw, ww = (_between(trace, 2, 3), _between(fetch, 2, 3),
                  _between(write, 2, 3))
    t_by = per_kernel(tw, "ns")
    f_by = per_kernel(fw, "kib")
    w_by = per_kernel(ww, "kib")
    L = []
    L.append("# %s" % args.title)
    L.append("#")
    L.append("# commands (each its own run; cd /tmp && export TMPDIR=/tmp first):")
    L.append("#   rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- %s" % args.command)
    L.append("#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> -o run -- %s" % args.command)
    L.append("#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out> -o run -- %s" % args.command)
    L.append("# summary: python -m paper_2603_07341_amd.profile_summary (this file's figures)")
    L.append("# calibration: the 1 GiB copy between marks 0 and 1 reads FETCH_SIZE %.1f KiB and"
             % (cf / 1024.0))
    L.append("# WRITE_SIZE %.1f KiB: fetch counts scaled by %.3f, write counts by %.3f"
             % (cw / 1024.0, sf, sw))
    L.append("# bench line of the trace run: value %.4g updates/s, %.3f ms/step, roofline frac %.3f"
             % (bench["value"], bench["ms_per_step"], bench["roofline"]["frac"]))
    L.append("kernel_sha: %s" % source_hash())
    for f in ("grown_steps", "S_start", "S_end"):
        L.append("window_%s: %d" % (f, int(cfg[f])))
    L.append("window_warmup: %d" % int(bench["warmup"]))
    L.append("window_steps: %d" % steps)
    L.append("window_S_mean: %.1f" % float(cfg["S_mean"]))
    # middle Clenshaw term
    n_mid = t_by.get(MID, [0, 0.0])[0]
    if n_mid:
        fb = f_by[MID][1] * 1024.0 * sf / f_by[MID][0]
        wb = w_by[MID][1] * 1024.0 * sw / w_by[MID][0]
        us = t_by[MID][1] / n_mid / 1e3
        L.append("mid_term_launches: %d" % n_mid)
        L.append("mid_term_avg_us: %.2f" % us)
        L.append("mid_term_fetch_bytes_per_launch: %.0f" % fb)
        L.append("mid_term_write_bytes_per_launch: %.0f" % wb)
        L.append("mid_term_bytes_per_launch: %.0f" % (fb + wb))
        L.append("mid_term_counted_bytes_per_row: %.2f" % ((fb + wb) / float(cfg["S_mean"])))
        L.append("mid_term_counted_rate_gbs: %.1f" % ((fb + wb) / (us * 1e-6) / 1e9))
    # stages per timed step
    st_t, st_b = {}, {}
    for d, s in zip(tw, stage_of([d["name"] for d in tw])):
        st_t[s] = st_t.get(s, 0.0) + d["ns"] * 1e-6
    for src, sc in ((fw, sf), (ww, sw)):
        for d, s in zip(src, stage_of([d["name"] for d in src])):
            st_b[s] = st_b.get(s, 0.0) + d["kib"] * 1024.0 * sc
    for s in ("select", "expand+build", "transfer", "propagate", "observe"):
        L.append("stage %s bytes: %.0f" % (s, st_b.get(s, 0.0) / steps))
        L.append("stage %s kernel_ms: %.4f" % (s, st_t.get(s, 0.0) / steps))
    L.append("")
    L.append("## timed window, per kernel (trace time; counted bytes fetch x %.3f + write x %.3f)" % (sf, sw))
    L.append("   %-44s %6s %10s %9s %11s %7s %6s" % ("kernel", "calls", "total ms", "avg us", "MB", "TB/s", "frac"))
    rows = sorted(t_by.items(), key=lambda kv: -kv[1][1])
    for name, (n, ns) in rows:
        mb = (f_by.get(name, [0, 0.0])[1] * sf + w_by.get(name, [0, 0.0])[1] * sw) * 1024.0 / 1e6
        ms = ns * 1e-6
        tbs = mb * 1e6 / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
        L.append("   %-44s %6d %10.3f %9.1f %11.1f %7.2f %6.2f" % (
            name[:44], n, ms, ns / n / 1e3, mb, tbs, tbs / 8.0))
    L.append("")
    L.append("## whole process (rocprofv3 --stats of the trace run), top kernels")
    try:
        if args.stats and os.path.isfile(args.stats):
            with open(args.stats, newline="") as fh:
                stats = list(csv.DictReader(fh))
        else:
            stats = _csv(args.stats or args.trace, "kernel_stats.csv")
        L.append("   %-44s %8s %12s %10s %7s" % ("kernel", "calls", "total ms", "avg us", "%"))
        for r in stats[:25]:
            L.append("   %-44s %8s %12.3f %10.1f %7.2f" % (
                short_name(r["Name"])[:44], r["Calls"],
                float(r["TotalDurationNs"]) / 1e6,
                float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    except (SystemExit, KeyError) as e:
        L.append("   (no stats table: %s)" % e)
    text = "\n".join(L) + "\n"
    with open(args.out, "w") as fh:
        fh.write(text)
    return text


def summarize_tail(args):
    """The last launches of one kernel in a whole run (kernel trace and the
    two counter runs of the same command), against the states of the steps
    they belong to (records saved by the run): time, counted bytes per
    launch and per state, and the rate by the algorithmic bytes per state."""
    import numpy as np
    trace = trace_dispatches(args.trace)
    fetch = {d["id"]: d for d in counter_dispatches(args.fetch, "FETCH_SIZE")}
    write = {d["id"]: d for d in counter_dispatches(args.write, "WRITE_SIZE")}
    t_k = [d for d in trace if d["name"] == args.kernel]
    f_k = [d for d in sorted(fetch.values(), key=lambda d: d["id"])
           if d["name"] == args.kernel]
    w_k = [d for d in sorted(write.values(), key=lambda d: d["id"])
           if d["name"] == args.kernel]
    n = min(args.last, len(t_k), len(f_k), len(w_k))
    if n == 0:
        raise SystemExit("no launches of %s" % args.kernel)
    us = sum(d["ns"] for d in t_k[-n:]) / n / 1e3
    fb = sum(d["kib"] for d in f_k[-n:]) / n * 1024.0 * args.fetch_scale
    wb = sum(d["kib"] for d in w_k[-n:]) / n * 1024.0 * args.write_scale
    rec = np.load(args.records)
    rows = float(rec[-args.steps:, 7].mean())
    L = ["# %s" % args.title, "#",
         "# commands (each its own run; cd /tmp && export TMPDIR=/tmp first):",
         "#   rocprofv3 --kernel-trace --stats --output-format csv -d <out> -o run -- %s" % args.command,
         "#   rocprofv3 --pmc FETCH_SIZE --output-format csv -d <out> -o run -- %s" % args.command,
         "#   rocprofv3 --pmc WRITE_SIZE --output-format csv -d <out> -o run -- %s" % args.command,
         "# summary: python -m paper_2603_07341_amd.profile_summary tail (this file's figures)",
         "# counter scales: fetch x %.3f, write x %.3f (a plain 1 GiB copy on the same GPU)"
         % (args.fetch_scale, args.write_scale),
         "kernel_sha: %s" % source_hash(),
         "kernel: %s" % args.kernel,
         "launches_used: %d (the last of %d)" % (n, len(t_k)),
         "steps_used: %d (the last of %d), mean states %.0f" % (args.steps, len(rec), rows),
         "avg_us: %.1f" % us,
         "counted_fetch_bytes_per_launch: %.0f" % fb,
         "counted_write_bytes_per_launch: %.0f" % wb,
         "counted_bytes_per_state: %.1f" % ((fb + wb) / rows),
         "counted_rate_tbs: %.2f" % ((fb + wb) / (us * 1e-6) / 1e12),
         "algorithmic_bytes_per_state: %d" % args.alg_bytes,
         "algorithmic_rate_tbs: %.2f" % (args.alg_bytes * rows / (us * 1e-6) / 1e12),
         "algorithmic_frac_of_8tbs: %.3f" % (args.alg_bytes * rows / (us * 1e-6) / 8e12),
         "", "## whole run, top kernels by trace time",
         "   %-44s %6s %11s %9s" % ("kernel", "calls", "total ms", "avg us")]
    agg = per_kernel(trace, "ns")
    for name, (c, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:16]:
        L.append("   %-44s %6d %11.1f %9.1f" % (name[:44], c, ns / 1e6, ns / c / 1e3))
    out = "\n".join(L) + "\n"
    with open(args.out, "w") as fh:
        fh.write(out)
    return out


def main(argv=None):
    argv = sys.argv[1:] if argv is None else argv
    if argv and argv[0] == "tail":
        ap = argparse.ArgumentParser()
        ap.add_argument("--trace", required=True)
        ap.add_argument("--fetch", required=True)
        ap.add_argument("--write", required=True)
        ap.add_argument("--records", required=True)
        ap.add_argument("--kernel", default=MID)
        ap.add_argument("--last", type=int, default=40)
        ap.add_argument("--steps", type=int, default=5)
        ap.add_argument("--alg-bytes", type=int, default=108)
        ap.add_argument("--fetch-scale", type=float, default=2.0)
        ap.add_argument("--write-scale", type=float, default=1.0)
        ap.add_argument("--command", required=True)
        ap.add_argument("--title", required=True)
        ap.add_argument("--out", required=True)
        sys.stdout.write(summarize_tail(ap.parse_args(argv[1:])))
        return
    if argv and argv[0] == "extract":
        # extract trace DIR OUT | extract FETCH_SIZE DIR OUT | extract WRITE_SIZE DIR OUT
        what, folder, out = argv[1], argv[2], argv[3]
        if what == "trace":
            write_window_rows(folder, "trace", None, out)
        else:
            write_window_rows(folder, "counter", what, out)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True,
                    help="rocprofv3 output folder, or a window CSV written "
                         "by --extract")
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--stats", default=None,
                    help="folder holding the trace run's kernel_stats.csv "
                         "(default: --trace)")
    ap.add_argument("--bench-json", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", default="Timed window of the ring16 bench step "
                    "(16-site Holstein ring, cutoff 12, g 1.2, J -1, k 4, "
                    "theta 1e-8, dt 0.01, complex128), MI355X")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    sys.stdout.write(summarize(args))


if __name__ == "__main__":
    main()
