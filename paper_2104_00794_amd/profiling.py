"""Summaries of rocprofv3 output for the measurement records under ``profiles/``.

Three kinds of summary are written, all short markdown text:

* kernel statistics of one run (``rocprofv3 --kernel-trace --stats``): calls,
  total and average duration per kernel;
* HBM traffic of one kernel: the per-dispatch ``FETCH_SIZE`` and ``WRITE_SIZE``
  counters (two separate ``--pmc`` runs), each scaled by the factor that makes
  the same counter report the known size of a plain device copy.  The summary
  records the SHA-256 of the kernel source it was measured with; ``bench.py``
  reports the traffic only while that source is unchanged;
* other hardware counters of chosen kernels (``--pmc`` runs), mean per dispatch.

Usage (from the repository root)::

    python -m paper_2104_00794_amd.profiling kernels DB OUT --title T --cmd C
    python -m paper_2104_00794_amd.profiling counters OUT --db DB [--db DB ...] --kernel K [--kernel K ...] \\
        --title T --cmd C [--cmd C ...]
    python -m paper_2104_00794_amd.profiling traffic OUT --kernel K --workload W \\
        --fetch-db DB --write-db DB --copy-fetch-db DB --copy-write-db DB \\
        --copy-bytes N --alg-bytes N --cmd C [--cmd C ...]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import os
import re
import sqlite3
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kernels.hip")


def kernel_source_sha256() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _db(path: str) -> str:
    """A results database, or the single one inside a rocprofv3 output folder."""
    if os.path.isdir(path):
        found = sorted(glob.glob(os.path.join(path, "**", "*_results.db"), recursive=True))
        if len(found) != 1:
            raise FileNotFoundError("expected one *_results.db under %s, found %d" % (path, len(found)))
        return found[0]
    return path


def kernel_stats(db: str):
    con = sqlite3.connect(_db(db))
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage from top_kernels"))
    con.close()
    return rows


def counter_mean(db: str, counter: str, kernel: str) -> tuple:
    """Mean value per dispatch of `counter` over the dispatches of kernels whose
    name contains `kernel`, and the dispatch count."""
    con = sqlite3.connect(_db(db))
    vals = [v for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection")
            if c == counter and kernel in k]
    con.close()
    if not vals:
        raise ValueError("no %s samples for a kernel matching %r" % (counter, kernel))
    return sum(vals) / len(vals), len(vals)


def write_kernel_summary(db: str, out: str, title: str, cmd: str) -> str:
    lines = ["# %s" % title, "", "Command (repository root, one MI355X):", "", "```", cmd, "```", "",
             "rocprofv3 --kernel-trace --stats (its top_kernels table); durations in microseconds.", "",
             "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, n, tot, avg, pct in kernel_stats(db):
        short = name.replace("tpx::", "").replace("void ", "").split("(")[0]
        lines.append("| `%s` | %d | %.1f | %.3f | %.2f |" % (short, n, tot, avg, pct))
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def write_traffic_summary(out: str, kernel: str, workload: str, fetch_db: str, write_db: str,
                          copy_fetch_db: str, copy_write_db: str, copy_bytes: float, alg_bytes: float,
                          cmds) -> str:
    fetch_kib, nf = counter_mean(fetch_db, "FETCH_SIZE", kernel)
    write_kib, nw = counter_mean(write_db, "WRITE_SIZE", kernel)
    cf_kib, _ = counter_mean(copy_fetch_db, "FETCH_SIZE", "copyBuffer")
    cw_kib, _ = counter_mean(copy_write_db, "WRITE_SIZE", "copyBuffer")
    f_fetch = copy_bytes / (cf_kib * 1024.0)
    f_write = copy_bytes / (cw_kib * 1024.0)
    fetch_b = fetch_kib * 1024.0 * f_fetch
    write_b = write_kib * 1024.0 * f_write
    total = fetch_b + write_b
    lines = [
        "# HBM traffic of `%s`, workload %s" % (kernel, workload), "",
        "Commands (repository root, one MI355X; each counter in its own run):", "", "```", *cmds, "```", "",
        "Calibration: a device copy of %d bytes reads as FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB per "
        "dispatch, so the counters are scaled by %.4f (fetch) and %.4f (write)." % (copy_bytes, cf_kib, cw_kib,
                                                                                  f_fetch, f_write), "",
        "| quantity | per launch |", "|---|---|",
        "| FETCH_SIZE (raw, %d dispatches) | %.1f KiB |" % (nf, fetch_kib),
        "| WRITE_SIZE (raw, %d dispatches) | %.1f KiB |" % (nw, write_kib),
        "| bytes read (scaled) | %.0f |" % fetch_b,
        "| bytes written (scaled) | %.0f |" % write_b,
        "| algorithmic bytes | %.0f |" % alg_bytes,
        "| traffic / algorithmic | %.3f |" % (total / alg_bytes), "",
        "traffic_bytes_per_launch = %.0f" % total,
        "kernel_source_sha256 = %s" % kernel_source_sha256(),
    ]
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def counter_table(db: str):
    """{(kernel name, counter): (mean per dispatch, dispatches)} of one --pmc run."""
    con = sqlite3.connect(_db(db))
    acc = {}
    for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
        tot, n = acc.get((k, c), (0.0, 0))
        acc[(k, c)] = (tot + v, n + 1)
    con.close()
    return {key: (tot / n, n) for key, (tot, n) in acc.items()}


def write_counter_summary(dbs, out: str, title: str, kernels, cmds, notes=()) -> str:
    """Mean per-dispatch values of every counter in the --pmc runs `dbs`, for
    the kernels whose names contain one of `kernels`."""
    rows = {}
    counters = []
    for db in dbs:
        for (k, c), (mean, n) in counter_table(db).items():
            tag = next((t for t in kernels if t in k), None)
            if tag is None:
                continue
            rows.setdefault(tag, {})[c] = (mean, n)
            if c not in counters:
                counters.append(c)
    lines = ["# %s" % title, "", "Commands (repository root, one MI355X; each counter set in its own run):", "",
             "```", *cmds, "```", "", "Mean value per dispatch (dispatch count in parentheses).", "",
             "| kernel | " + " | ".join(counters) + " |", "|---" * (len(counters) + 1) + "|"]
    for tag in kernels:
        if tag not in rows:
            continue
        cells = ["%.4g (%d)" % rows[tag][c] if c in rows[tag] else "" for c in counters]
        lines.append("| `%s` | " % tag + " | ".join(cells) + " |")
    lines += [""] + list(notes)
    text = "\n".join(lines) + "\n"
    with open(out, "w") as f:
        f.write(text)
    return text


def traffic_path(workload: str, kernel_tag: str) -> str:
    return os.path.join(PROFILES, "%s_%s_traffic.md" % (kernel_tag, workload))


def read_traffic(workload: str, kernel_tag: str) -> Optional[float]:
    """Measured traffic per launch, or None if absent or taken with other kernel source."""
    path = traffic_path(workload, kernel_tag)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"^traffic_bytes_per_launch = (\d+)", text, re.M)
    h = re.search(r"^kernel_source_sha256 = ([0-9a-f]{64})", text, re.M)
    if not t or not h or h.group(1) != kernel_source_sha256():
        return None
    return float(t.group(1))


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="what", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("db")
    k.add_argument("out")
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("out")
    for a in ("--kernel", "--workload", "--fetch-db", "--write-db", "--copy-fetch-db", "--copy-write-db"):
        t.add_argument(a, required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--alg-bytes", type=float, required=True)
    t.add_argument("--cmd", action="append", required=True)
    c = sub.add_parser("counters")
    c.add_argument("out")
    c.add_argument("--db", action="append", required=True)
    c.add_argument("--kernel", action="append", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--cmd", action="append", required=True)
    c.add_argument("--note", action="append", default=[])
    a = ap.parse_args(argv)
    if a.what == "kernels":
        print(write_kernel_summary(a.db, a.out, a.title, a.cmd))
    elif a.what == "counters":
        print(write_counter_summary(a.db, a.out, a.title, a.kernel, a.cmd, a.note))
    else:
        print(write_traffic_summary(a.out, a.kernel, a.workload, a.fetch_db, a.write_db, a.copy_fetch_db,
                                    a.copy_write_db, a.copy_bytes, a.alg_bytes, a.cmd))


if __name__ == "__main__":
    main()
