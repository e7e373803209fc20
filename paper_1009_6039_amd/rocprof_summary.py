"""Short text summaries of rocprofv3 output for the solver's kernels.

  stats    kernel-trace CSV -> per-kernel table for the whole command, and the
           average duration of one kernel over the solves of the last K steps
           (the timed steps of bench.py's headline arm, which runs last)
  traffic  FETCH_SIZE and WRITE_SIZE counter CSVs of the solver run and of a plain
           copy of known size -> HBM bytes per dispatch of one kernel, scaled so
           the copy reads and writes its own size; ends with a JSON line that
           bench.py reads, keyed by a hash of the kernel sources

A solve's kernels run from k_setup_sums to k_outputs; launches outside those
segments (the warm-start network and its head) are not counted in the window.

  python -m paper_1009_6039_amd.rocprof_summary stats --trace T.csv --kernel 'k_passC<512>' \\
      --steps 3 --title ... --command ...
  python -m paper_1009_6039_amd.rocprof_summary traffic --fetch F.csv --write W.csv \\
      --copy-fetch CF.csv --copy-write CW.csv --copy-mib 512 --kernel 'k_passC<512>' --steps 1 ...
"""

import argparse
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# the translation units of the Strain passes (row A, column B, row C) and what they include
KERNEL_SOURCES = ["csrc/strain.h", "csrc/k_pass_a.hip", "csrc/k_pass_b.hip", "csrc/k_pass_c.hip",
                  "csrc/k_strain.hip", "csrc/fft.h", "csrc/common.h", "csrc/kernels.h"]


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short_name(name):
    m = re.search(r"(k_\w+(?:<[^>]*>)?|__amd_rocclr_\w+)", name)
    return m.group(1) if m else name[:40]


def solve_windows(names, steps):
    """Indices of the kernels of the last `steps` solves (k_setup_sums .. k_outputs)."""
    starts = [i for i, n in enumerate(names) if n == "k_setup_sums"]
    keep = set()
    for s in starts[-steps:]:
        i = s
        while i < len(names):
            keep.add(i)
            if names[i] == "k_outputs":
                break
            i += 1
    return keep


def stats(args):
    rows = list(csv.DictReader(open(args.trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    names = [short_name(r["Kernel_Name"]) for r in rows]
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3 for r in rows]
    agg = {}
    for n, d in zip(names, dur):
        a = agg.setdefault(n, [0, 0.0])
        a[0] += 1
        a[1] += d
    total = sum(a[1] for a in agg.values())
    win = solve_windows(names, args.steps)
    wd = [dur[i] for i in sorted(win) if names[i] == args.kernel]
    out = ["# %s" % args.title, "", "Command (repository root, MI355X):", "", "    " + args.command, ""]
    if args.note:
        out += [args.note, ""]
    out += ["| Kernel | Calls | Total ms | Avg us | % |", "|---|---:|---:|---:|---:|"]
    for n, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:args.top]:
        out.append("| %s | %d | %.1f | %.2f | %.1f |" % (n, c, t * 1e-3, t / c, 100.0 * t / total))
    out += ["", "Kernel busy time over the whole command: %.1f ms." % (total * 1e-3), ""]
    if wd:
        out.append("%s over the solves of the last %d steps (the timed steps of the headline arm): "
                   "%d launches, %.2f us average, %.1f ms total."
                   % (args.kernel, args.steps, len(wd), sum(wd) / len(wd), sum(wd) * 1e-3))
        out += ["", "window_avg_us %s: %.3f" % (args.kernel, sum(wd) / len(wd))]
    print("\n".join(out))


def counters(path, counter):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(short_name(r["Kernel_Name"]), float(r["Counter_Value"])) for r in rows]


def copy_scale(path, counter, mib):
    vals = [v for n, v in counters(path, counter) if n.startswith("__amd_rocclr_copy")]
    if not vals:
        raise SystemExit("no copy dispatch in " + path)
    return mib * 1024.0 / max(vals)  # KiB the copy moved / KiB the counter read


def traffic(args):
    fs = copy_scale(args.copy_fetch, "FETCH_SIZE", args.copy_mib)
    ws = copy_scale(args.copy_write, "WRITE_SIZE", args.copy_mib)
    F = counters(args.fetch, "FETCH_SIZE")
    W = counters(args.write, "WRITE_SIZE")
    per = {}
    for label, data, scale in (("read", F, fs), ("write", W, ws)):
        names = [n for n, _ in data]
        win = solve_windows(names, args.steps)
        for i in sorted(win):
            n, v = data[i]
            a = per.setdefault(n, {"read": [0, 0.0], "write": [0, 0.0]})
            a[label][0] += 1
            a[label][1] += v * 1024.0 * scale
    out = ["# %s" % args.title, "", "Commands (repository root, MI355X), one counter per run:", ""]
    out += ["    " + c for c in args.command]
    out += ["", "Counter scale from a plain device copy of %d MiB: FETCH_SIZE x %.4f, WRITE_SIZE x %.4f "
            "(bytes the copy moved / bytes the counter reported)." % (args.copy_mib, fs, ws), ""]
    if args.note:
        out += [args.note, ""]
    out += ["Over the solve kernels of the last %d step(s):" % args.steps, "",
            "| Kernel | Dispatches | Read MB | Written MB | MB / dispatch |", "|---|---:|---:|---:|---:|"]
    for n, a in sorted(per.items(), key=lambda kv: -(kv[1]["read"][1] + kv[1]["write"][1]))[:args.top]:
        d = max(a["read"][0], a["write"][0])
        out.append("| %s | %d | %.1f | %.1f | %.2f |" % (n, d, a["read"][1] / 1e6, a["write"][1] / 1e6,
                                                         (a["read"][1] + a["write"][1]) / d / 1e6))
    k = per.get(args.kernel)
    if k:
        d = max(k["read"][0], k["write"][0])
        rec = {"kernel": args.kernel, "dispatches": d, "read_bytes_per_launch": k["read"][1] / d,
               "write_bytes_per_launch": k["write"][1] / d,
               "traffic_bytes_per_launch": (k["read"][1] + k["write"][1]) / d,
               "source_sha256": kernel_source_hash(), "variant": args.variant}
        if args.algorithmic_bytes_per_launch:
            rec["algorithmic_bytes_per_launch"] = args.algorithmic_bytes_per_launch
            rec["traffic_over_algorithmic"] = rec["traffic_bytes_per_launch"] / args.algorithmic_bytes_per_launch
        out += ["", "traffic_record: " + json.dumps(rec)]
    print("\n".join(out))


def read_traffic_record(path, kernel):
    """The traffic record of a summary if its kernel sources are the current ones, else None."""
    try:
        with open(path) as fh:
            for line in fh:
                if line.startswith("traffic_record: "):
                    rec = json.loads(line[len("traffic_record: "):])
                    if rec.get("kernel") == kernel and rec.get("source_sha256") == kernel_source_hash():
                        return rec
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("--trace", required=True)
    s.add_argument("--kernel", required=True)
    s.add_argument("--steps", type=int, default=3)
    s.add_argument("--title", required=True)
    s.add_argument("--command", required=True)
    s.add_argument("--note", default="")
    s.add_argument("--top", type=int, default=24)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--steps", type=int, default=1)
    t.add_argument("--title", required=True)
    t.add_argument("--command", action="append", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--algorithmic-bytes-per-launch", type=float, default=0.0)
    t.add_argument("--variant", type=int, default=0, help="launch-geometry variant of the kernel profiled")
    t.add_argument("--top", type=int, default=12)
    a = ap.parse_args()
    stats(a) if a.cmd == "stats" else traffic(a)


if __name__ == "__main__":
    main()
