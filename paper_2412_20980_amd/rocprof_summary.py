"""Summaries of rocprofv3 results for the profiles/ folder.

  python -m paper_2412_20980_amd.rocprof_summary \\
      --trace T_results.db [--fetch F_results.db --write W_results.db \\
      --copy-fetch CF_results.db --copy-write CW_results.db --copy-bytes N] \\
      --last-passes K --workload NAME --tuning SG,BS,SW,BB --command "..." \\
      --out-md profiles/X.md [--out-traffic profiles/NAME_traffic.json]

Reads rocprofv3's SQLite output (kernel dispatches, and FETCH_SIZE /
WRITE_SIZE counters in KiB per dispatch) and writes
  * a Markdown table of per-kernel calls, average and total duration over the
    whole run;
  * the last K fitness passes of the run (the ones the benchmark times with
    events): each pass's kernels, their summed duration per pass and, from the
    counter runs of the same command, the HBM traffic of one pass: FETCH_SIZE
    and WRITE_SIZE summed over the pass's kernels, each scaled by bytes /
    counter measured on a plain copy of known size.
A pass is the dispatches of the fitness kernels from one k_dead_transpose up
to the next dispatch of any other kernel.
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import re
import sqlite3
import sys

# kernels of one batched-fitness pass (bit-parallel path)
FITNESS_KERNELS = ("k_dead_transpose", "k_seed", "k_pull_band", "k_collect_pending", "k_pull_worklist",
                   "k_collect_pairs", "k_pairs_hook", "k_pairs_count", "k_pairs_reduce")
PASS_MARKER = "k_dead_transpose"  # launched first in every pass, once


def short(name: str) -> str:
    m = re.search(r"(k_\w+|__amd\w+|elementwise_kernel|copy\w*)", name)
    return m.group(1) if m else name[:48]


def _columns(c, table):
    return [r[1] for r in c.execute(f"pragma table_info({table})").fetchall()]


def dispatches(db: str):
    """(name, duration ns, start ns or None) of every kernel dispatch in
    dispatch order."""
    c = sqlite3.connect(db)
    cols = _columns(c, "kernels")
    order = next((x for x in ("start", "dispatch_id", "id") if x in cols), None)
    start = "start" if "start" in cols else "NULL"
    q = f"select name, duration, {start} from kernels" + (f" order by {order}" if order else "")
    return c.execute(q).fetchall()


def counter_rows(db: str, counter: str):
    """(name, value) per dispatch of one counter, in dispatch order (rows of
    the same dispatch summed)."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, name, counter_value from pmc_events where counter_name = ? "
                     "order by dispatch_id", (counter,)).fetchall()
    per = collections.OrderedDict()
    for did, name, val in rows:
        if did in per:
            per[did][1] += val
        else:
            per[did] = [short(name), val]
    return [tuple(v) for v in per.values()]


def kernel_table(db: str) -> str:
    d = collections.defaultdict(list)
    for name, dur, _ in dispatches(db):
        d[short(name)].append(dur)
    total = sum(sum(v) for v in d.values())
    lines = ["| kernel | calls | avg us | total us | % |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {k} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {sum(v) / 1e3:.1f} | "
                     f"{100.0 * sum(v) / total:.1f} |")
    return "\n".join(lines)


def last_passes(seq, K: int):
    """Indices of the dispatches of the last K passes in a sequence of
    (kernel name, ...) items: a pass starts at PASS_MARKER and runs while the
    kernels are fitness kernels."""
    starts = [i for i, it in enumerate(seq) if it[0] == PASS_MARKER]
    if len(starts) < K:
        raise SystemExit(f"only {len(starts)} passes in the run, {K} asked for")
    out = []
    for s in starts[-K:]:
        i = s
        idx = []
        while i < len(seq) and seq[i][0] in FITNESS_KERNELS and (i == s or seq[i][0] != PASS_MARKER):
            idx.append(i)
            i += 1
        out.append(idx)
    return out


def copy_factor(db: str, counter: str, copy_bytes: int) -> float:
    """bytes / counter-byte on the plain copy: the largest dispatch."""
    vals = sorted((v for _, v in counter_rows(db, counter)), reverse=True)
    if not vals:
        raise SystemExit(f"no {counter} values in {db}")
    return copy_bytes / (vals[0] * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--last-passes", type=int, default=0, help="K: summarise the last K fitness passes")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--tuning", default="", help="launch shapes of the profiled run: SG,BS,SW,BB")
    ap.add_argument("--command", required=True)
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-traffic")
    ap.add_argument("--source-sha256", default="")
    a = ap.parse_args(argv)

    md = [f"# rocprofv3 kernel trace: {a.workload}", "",
          f"Kernel sources (sha256 of the fitness-pass sources, first 16 hex digits): `{a.source_sha256}`", "",
          "Commands:", "", "```", a.command, "```", "", "## All dispatches of the run", "",
          kernel_table(a.trace), ""]
    traffic = None
    if a.last_passes > 0:
        K = a.last_passes
        seq = [(short(n), d, st) for n, d, st in dispatches(a.trace)]
        passes = last_passes(seq, K)
        per_kernel = collections.defaultdict(float)
        calls = collections.Counter()
        pass_sum = []
        spans = []
        for idx in passes:
            pass_sum.append(sum(seq[i][1] for i in idx))
            for i in idx:
                per_kernel[seq[i][0]] += seq[i][1]
                calls[seq[i][0]] += 1
            if seq[idx[0]][2] is not None:
                spans.append(seq[idx[-1]][2] + seq[idx[-1]][1] - seq[idx[0]][2])
        pass_ms = sum(pass_sum) / K / 1e6
        span_ms = sum(spans) / K / 1e6 if spans else None
        md += [f"## The last {K} fitness passes", "",
               f"Kernel time per pass (sum of the pass's dispatch durations): {pass_ms * 1e3:.1f} us"
               + (f"; first dispatch start to last dispatch end: {span_ms * 1e3:.1f} us" if span_ms else "") + ".",
               ""]
        rows = ["| kernel | calls per pass | us per pass |", "|---|---:|---:|"]
        for k in FITNESS_KERNELS:
            if calls[k]:
                rows.append(f"| {k} | {calls[k] / K:.2f} | {per_kernel[k] / K / 1e3:.2f} |")
        md += rows + [""]
        if a.fetch and a.write:
            ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes) if a.copy_fetch else 1.0
            wf = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes) if a.copy_write else 1.0
            f_seq = counter_rows(a.fetch, "FETCH_SIZE")
            w_seq = counter_rows(a.write, "WRITE_SIZE")
            fk, wk = collections.defaultdict(float), collections.defaultdict(float)
            for idx in last_passes(f_seq, K):
                for i in idx:
                    fk[f_seq[i][0]] += f_seq[i][1]
            for idx in last_passes(w_seq, K):
                for i in idx:
                    wk[w_seq[i][0]] += w_seq[i][1]
            f_pass = sum(fk.values()) / K * 1024.0 * ff
            w_pass = sum(wk.values()) / K * 1024.0 * wf
            md += ["## HBM traffic of one fitness pass", "",
                   f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch) over the last {K} passes of the counter runs, "
                   f"per pass, scaled by the copy calibration (a plain copy of {a.copy_bytes} bytes): fetch factor "
                   f"{ff:.4f}, write factor {wf:.4f}.", "",
                   "| kernel | fetch KiB/pass | write KiB/pass | GB/s at its trace time |", "|---|---:|---:|---:|"]
            for k in FITNESS_KERNELS:
                if fk[k] or wk[k]:
                    t = per_kernel[k] / K
                    rate = (fk[k] * ff + wk[k] * wf) / K * 1024.0 / t if t else 0.0
                    md.append(f"| {k} | {fk[k] / K:.0f} | {wk[k] / K:.0f} | {rate:.0f} |")
            md += ["", f"Per pass: fetch {f_pass / 1e6:.2f} MB, write {w_pass / 1e6:.2f} MB, total "
                       f"{(f_pass + w_pass) / 1e6:.2f} MB; at the traced kernel time {pass_ms * 1e3:.1f} us that is "
                       f"{(f_pass + w_pass) / (pass_ms * 1e-3) / 1e9:.0f} GB/s "
                       f"({(f_pass + w_pass) / (pass_ms * 1e-3) / 8e12:.3f} of 8 TB/s).", ""]
            tuning = None
            if a.tuning:
                sg, bs, sw, bb = (int(x) for x in a.tuning.split(","))
                tuning = {"sweep_grid": sg, "band_scan": bs, "sweeps": sw, "band_blocks": bb}
            traffic = {"workload": a.workload, "source_sha256": a.source_sha256, "tuning": tuning,
                       "passes": K, "pass_ms": pass_ms, "pass_span_ms": span_ms,
                       "fetch_bytes_per_pass": f_pass, "write_bytes_per_pass": w_pass,
                       "bytes_per_pass": f_pass + w_pass, "fetch_factor": ff, "write_factor": wf,
                       "command": a.command}
    if a.out_traffic and traffic:
        with open(a.out_traffic, "w") as f:
            json.dump(traffic, f, indent=1)
    os.makedirs(os.path.dirname(os.path.abspath(a.out_md)), exist_ok=True)
    with open(a.out_md, "w") as f:
        f.write("\n".join(md) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
