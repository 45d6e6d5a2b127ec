"""Text summaries of rocprofv3 runs of bench.py (kernel trace statistics and
HBM traffic from the FETCH_SIZE / WRITE_SIZE counters), and the lookup that
bench.py uses to attach the measured traffic to its roofline line.

rocprofv3 writes one SQLite database per run (``-d DIR -o run``).  Traffic
is the counter value (KiB per dispatch) scaled by what the same counter
reads for a plain device copy of known size in the same run (bench.py
--copy-probe BYTES), per kernel launch.  A summary records a hash of the
kernel sources it was measured on; once they change, the lookup returns
None so that no stale traffic is reported.

    python -m paper_1907_13088_amd.profsum --trace T.db --fetch F.db --write W.db \\
        --copy-bytes N --bench-json bench.json --kernel REGEX --out profiles/NAME.md \\
        --cmd-trace "..." --cmd-fetch "..." --cmd-write "..." [--sq S.db --cmd-sq "..."]
    python -m paper_1907_13088_amd.profsum --trace T.db --title TITLE --cmd-trace "..." \\
        [--bench-json bench.json] --out profiles/NAME.md
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
# sources that determine the 2D sweep pass kernels and their launch shapes
SWEEP_SOURCES = ("csrc/k2s_impl.h", "csrc/stencil2d.h", "csrc/mx_internal.h", "csrc/k2s.hip",
                 "csrc/k2s_f32_all.hip", "csrc/k2f_impl.h", "csrc/k2f.hip", "csrc/k2fs_impl.h", "csrc/k2fs.hip",
                 "csrc/mx_api.cpp")


def source_sha(files=SWEEP_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_per_launch(path: str, category: str = None):
    """Measured HBM bytes per launch of the summarised kernel, or None when
    the summary is missing, covers another kernel category or was taken on
    other kernel sources."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m1 = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    m2 = re.search(r"^source_sha256:\s*([0-9a-f]+)", txt, re.M)
    m3 = re.search(r"^category:\s*(\S+)", txt, re.M)
    if not m1 or not m2 or m2.group(1) != source_sha():
        return None
    if category is not None and (not m3 or m3.group(1) != category):
        return None
    return float(m1.group(1))


def _short(n: str) -> str:
    n = n.replace("(anonymous namespace)::", "")
    n = re.sub(r"\(.*", "", n)
    return n.replace("void ", "").replace("mx::", "")


def _stats(db):
    cur = sqlite3.connect(db).cursor()
    return list(cur.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))


def _counter(db, name):
    cur = sqlite3.connect(db).cursor()
    per = {}
    for k, v in cur.execute("select kernel_name, value from counters_collection where counter_name = ?", (name,)):
        per.setdefault(k, []).append(float(v))
    return per


def _calibrate(fetch, write, copy_bytes):
    """Per-dispatch counters of both runs and the bytes per counter unit,
    from the largest copy kernel (the probe of copy_bytes)."""
    f = _counter(fetch, "FETCH_SIZE")
    w = _counter(write, "WRITE_SIZE")
    copyk = [k for k in f if "copy" in k.lower() and k in w]
    if not copyk:
        raise SystemExit("no copy kernel in the counter runs (run bench.py with --copy-probe)")
    ck = max(copyk, key=lambda k: max(f[k]))
    # the probe is the largest copy of the run (the run may hold smaller
    # copies of the same kernel); it reads and writes copy_bytes
    fcopy, wcopy = max(f[ck]), max(w[ck])
    return f, w, ck, fcopy, wcopy, copy_bytes / fcopy, copy_bytes / wcopy


def _sq_table(db, cmd):
    """Per-kernel means of the SQ counters of one counter run (instruction
    counts are per dispatch, summed over the wavefronts)."""
    cur = sqlite3.connect(db).cursor()
    per = {}
    for k, n, v in cur.execute("select kernel_name, counter_name, value from counters_collection"):
        per.setdefault(k, {}).setdefault(n, []).append(float(v))
    names = sorted({n for d in per.values() for n in d})
    L = ["SQ counters per dispatch (means; instruction counts summed over wavefronts):", "",
         "command: `" + cmd + "`", "",
         "| kernel | " + " | ".join(names) + " |", "|---|" + "---:|" * len(names)]
    for k in sorted(per, key=lambda k: -statistics.mean(per[k].get("SQ_WAVES", [0.0]))):
        if "copy" in k.lower() or "elementwise" in k.lower():
            continue
        L.append(f"| {_short(k)} | " + " | ".join(f"{statistics.mean(per[k][n]):.4g}" if n in per[k] else "-"
                                                 for n in names) + " |")
    return L + [""]


def summarize(trace, fetch, write, copy_bytes, bench_json, kernel_re, out, cmds, sq=None):
    st = _stats(trace)
    f, w, ck, fcopy, wcopy, ff, fw = _calibrate(fetch, write, copy_bytes)
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1]) if bench_json else None
    L = []
    L.append("# rocprofv3 summary: 2D field step, 4096 x 4096 TE+TM FP32, m = 20, p = 3 (MI355X, 1 GPU)")
    L.append("")
    L.append("kernel trace command: `" + cmds[0] + "`")
    L.append("")
    L.append("| kernel | calls | avg us | total ms | % |")
    L.append("|---|---:|---:|---:|---:|")
    sel_calls, sel_total, sel_names = 0, 0.0, []
    for n, c, tot, avg, pct in st:
        L.append(f"| {_short(n)} | {c} | {avg:.1f} | {tot / 1e3:.2f} | {pct:.1f} |")
        if re.search(kernel_re, n):
            sel_calls += c
            sel_total += tot
            sel_names.append(_short(n))
    L.append("")
    if bench:
        L.append("library HIP-event averages inside the timed region of the same command (bench.py output):")
        L.append("")
        L.append("| category | launches | avg us | algorithmic GB/s |")
        L.append("|---|---:|---:|---:|")
        for k, v in bench["kernels"].items():
            L.append(f"| {k} | {v['launches']} | {v['avg_us']} | {v['GBps']} |")
        L.append("")
    L.append("HBM traffic per dispatch (one counter per run):")
    L.append("")
    L.append("fetch command: `" + cmds[1] + "`")
    L.append("")
    L.append("write command: `" + cmds[2] + "`")
    L.append("")
    L.append(f"calibration: a plain {copy_bytes}-byte device copy ({_short(ck)}) reads FETCH_SIZE = {fcopy:.0f} "
             f"and WRITE_SIZE = {wcopy:.0f} per dispatch, so one unit is {ff:.1f} B read and {fw:.1f} B written")
    L.append("")
    L.append("| kernel | dispatches | read MB | written MB | traffic MB |")
    L.append("|---|---:|---:|---:|---:|")
    sel_rd, sel_wr = [], []
    for k in sorted(f, key=lambda k: -statistics.mean(f[k])):
        if k == ck or k not in w:
            continue
        rd = statistics.mean(f[k]) * ff
        wr = statistics.mean(w[k]) * fw
        L.append(f"| {_short(k)} | {len(f[k])} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {(rd + wr) / 1e6:.1f} |")
        if re.search(kernel_re, k):
            sel_rd += [v * ff for v in f[k]]
            sel_wr += [v * fw for v in w[k]]
    L.append("")
    if not sel_calls or not sel_rd:
        raise SystemExit(f"kernel /{kernel_re}/ not found in the runs")
    cat = bench["roofline"].get("category", "sweep") if bench else "sweep"
    L.append(f"dominant kernel: {', '.join('`' + n + '`' for n in sel_names)} (library category {cat}), "
             f"{sel_calls} calls, rocprofv3 average {sel_total / sel_calls:.1f} us")
    if bench:
        r = bench["roofline"]
        L.append(f"bench.py HIP-event average of the same launches: {r['avg_launch_us']} us, "
                 f"algorithmic {r['bytes_per_launch'] / 1e6:.1f} MB per launch ({r['achieved']} GB/s)")
    L.append("")
    if sq:
        L += _sq_table(sq, cmds[3])
    L.append(f"traffic_bytes_per_launch: {statistics.mean(sel_rd) + statistics.mean(sel_wr):.0f}")
    L.append(f"category: {cat}")
    L.append(f"source_sha256: {source_sha()}")
    open(out, "w").write("\n".join(L) + "\n")
    return out


def trace_summary(trace, title, cmd, out, bench_json=None, fetch=None, write=None, copy_bytes=None,
                  cmd_fetch=None, cmd_write=None):
    """Kernel statistics of one rocprofv3 --kernel-trace --stats run, and,
    given the two counter runs, the HBM traffic per dispatch of every kernel."""
    L = [f"# rocprofv3 summary: {title} (MI355X, 1 GPU)", "", "kernel trace command: `" + cmd + "`", "",
         "| kernel | calls | avg us | total ms | % |", "|---|---:|---:|---:|---:|"]
    for n, c, tot, avg, pct in _stats(trace):
        L.append(f"| {_short(n)} | {c} | {avg:.1f} | {tot / 1e3:.2f} | {pct:.1f} |")
    if bench_json:
        L += ["", "bench.py output of the same command:", "", "```",
              open(bench_json).read().strip().splitlines()[-1], "```"]
    if fetch and write:
        f, w, ck, fcopy, wcopy, ff, fw = _calibrate(fetch, write, copy_bytes)
        L += ["", "HBM traffic per dispatch (one counter per run):", "", "fetch command: `" + cmd_fetch + "`", "",
              "write command: `" + cmd_write + "`", "",
              f"calibration: a plain {copy_bytes}-byte device copy ({_short(ck)}) reads FETCH_SIZE = {fcopy:.0f} "
              f"and WRITE_SIZE = {wcopy:.0f} per dispatch, so one unit is {ff:.1f} B read and {fw:.1f} B written",
              "", "| kernel | dispatches | read MB | written MB | traffic MB |", "|---|---:|---:|---:|---:|"]
        for k in sorted(f, key=lambda k: -statistics.mean(f[k])):
            if k == ck or k not in w:
                continue
            rd = statistics.mean(f[k]) * ff
            wr = statistics.mean(w[k]) * fw
            L.append(f"| {_short(k)} | {len(f[k])} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | {(rd + wr) / 1e6:.1f} |")
    open(out, "w").write("\n".join(L) + "\n")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--title", default=None, help="trace-only summary with this title")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-bytes", type=int)
    ap.add_argument("--bench-json", default=None)
    ap.add_argument("--kernel", help="regex of the dominant kernel's name")
    ap.add_argument("--out", required=True)
    ap.add_argument("--cmd-trace", required=True)
    ap.add_argument("--cmd-fetch")
    ap.add_argument("--cmd-write")
    ap.add_argument("--sq", help="counter run of SQ counters (instruction counts) to tabulate")
    ap.add_argument("--cmd-sq")
    a = ap.parse_args()
    if a.title:
        print(trace_summary(a.trace, a.title, a.cmd_trace, a.out, a.bench_json, a.fetch, a.write, a.copy_bytes,
                            a.cmd_fetch, a.cmd_write))
        return
    print(summarize(a.trace, a.fetch, a.write, a.copy_bytes, a.bench_json, a.kernel, a.out,
                    (a.cmd_trace, a.cmd_fetch, a.cmd_write, a.cmd_sq), sq=a.sq))


if __name__ == "__main__":
    main()
