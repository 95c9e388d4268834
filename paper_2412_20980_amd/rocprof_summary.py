"""Summaries of rocprofv3 results for the profiles/ folder.

  python -m paper_2412_20980_amd.rocprof_summary \\
      --trace T_results.db [--fetch F_results.db --write W_results.db \\
      --copy-fetch CF_results.db --copy-write CW_results.db --copy-bytes N] \\
      --workload NAME --command "..." --out-md profiles/X.md [--out-traffic profiles/fitness_traffic.json]

Reads rocprofv3's SQLite output (kernel dispatches, and FETCH_SIZE /
WRITE_SIZE counters in KiB per dispatch) and writes
  * a Markdown table of per-kernel calls, average and total duration;
  * optionally the HBM traffic of one batched-fitness pass: FETCH_SIZE and
    WRITE_SIZE summed over the pass's kernels, per pass, each scaled by
    bytes / counter measured on a plain copy of known size.
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
                   "k_collect_pairs", "k_pairs_hook", "k_pairs_count", "k_pairs_reduce",
                   "k_root_final")
PASS_MARKER = "k_dead_transpose"  # launched once per pass


def short(name: str) -> str:
    m = re.search(r"(k_\w+|__amd\w+|elementwise_kernel|copy\w*)", name)
    return m.group(1) if m else name[:48]


def dispatches(db: str):
    c = sqlite3.connect(db)
    return c.execute("select name, duration from kernels").fetchall()


def counters(db: str):
    c = sqlite3.connect(db)
    return c.execute("select name, dispatch_id, counter_name, counter_value from pmc_events").fetchall()


def kernel_table(db: str) -> str:
    d = collections.defaultdict(list)
    for name, dur in dispatches(db):
        d[short(name)].append(dur)
    total = sum(sum(v) for v in d.values())
    lines = ["| kernel | calls | avg us | total us | % |", "|---|---:|---:|---:|---:|"]
    for k, v in sorted(d.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {k} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {sum(v) / 1e3:.1f} | "
                     f"{100.0 * sum(v) / total:.1f} |")
    return "\n".join(lines)


def per_kernel_counter(db: str, counter: str):
    d = collections.defaultdict(float)
    n = collections.Counter()
    for name, _, cname, val in counters(db):
        if cname == counter:
            d[short(name)] += val
            n[short(name)] += 1
    return d, n


def copy_factor(db: str, counter: str, copy_bytes: int) -> float:
    """bytes / counter-byte on the plain copy: the largest dispatches."""
    vals = sorted((val for _, _, cname, val in counters(db) if cname == counter), reverse=True)
    if not vals:
        raise SystemExit(f"no {counter} values in {db}")
    kib = vals[0]
    return copy_bytes / (kib * 1024.0)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out-md", required=True)
    ap.add_argument("--out-traffic")
    ap.add_argument("--source-sha256", default="")
    a = ap.parse_args(argv)

    md = [f"# rocprofv3 kernel trace: {a.workload}", "", "Command:", "", "```", a.command, "```", "",
          kernel_table(a.trace), ""]
    if a.fetch and a.write:
        fetch, nf = per_kernel_counter(a.fetch, "FETCH_SIZE")
        write, nw = per_kernel_counter(a.write, "WRITE_SIZE")
        passes = nf[PASS_MARKER]
        ff = copy_factor(a.copy_fetch, "FETCH_SIZE", a.copy_bytes) if a.copy_fetch else 1.0
        wf = copy_factor(a.copy_write, "WRITE_SIZE", a.copy_bytes) if a.copy_write else 1.0
        # a standalone pass (bench's roofline unit) also builds the removed-node
        # bit sets from genes: add the mask kernel's average per dispatch
        mk = "k_mask_build_lds"
        f_mask = fetch[mk] / nf[mk] if nf[mk] else 0.0
        w_mask = write[mk] / nw[mk] if nw[mk] else 0.0
        f_pass = (sum(fetch[k] for k in FITNESS_KERNELS) / passes + f_mask) * 1024.0 * ff
        w_pass = (sum(write[k] for k in FITNESS_KERNELS) / passes + w_mask) * 1024.0 * wf
        md += ["## HBM traffic of one batched-fitness pass", "",
               f"FETCH_SIZE and WRITE_SIZE (KiB per dispatch) summed over the pass's kernels and divided by "
               f"the {passes} passes profiled; scaled by the copy calibration (a plain copy of "
               f"{a.copy_bytes} bytes): fetch factor {ff:.4f}, write factor {wf:.4f}.", "",
               "| kernel | fetch KiB/pass | write KiB/pass |", "|---|---:|---:|"]
        md.append(f"| {mk} (per dispatch) | {f_mask:.0f} | {w_mask:.0f} |")
        for k in FITNESS_KERNELS:
            md.append(f"| {k} | {fetch[k] / passes:.0f} | {write[k] / passes:.0f} |")
        md += ["", f"Per pass: fetch {f_pass / 1e6:.2f} MB, write {w_pass / 1e6:.2f} MB, "
                   f"total {(f_pass + w_pass) / 1e6:.2f} MB.", ""]
        if a.out_traffic:
            with open(a.out_traffic, "w") as f:
                json.dump({"workload": a.workload, "source_sha256": a.source_sha256,
                           "fetch_bytes_per_pass": f_pass, "write_bytes_per_pass": w_pass,
                           "bytes_per_pass": f_pass + w_pass, "passes_profiled": passes,
                           "fetch_factor": ff, "write_factor": wf, "command": a.command}, f, indent=1)
    os.makedirs(os.path.dirname(os.path.abspath(a.out_md)), exist_ok=True)
    with open(a.out_md, "w") as f:
        f.write("\n".join(md) + "\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
