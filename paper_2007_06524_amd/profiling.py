"""Summaries of rocprofv3 output for the solver's kernels.

    python -m paper_2007_06524_amd.profiling --trace DIR [--fetch DIR] [--write DIR]
        [--copy-mib M] [--out FILE] [--title TEXT] [--command TEXT ...] [--digest]

DIR is a rocprofv3 output directory (CSV files from --output-format csv, or
the rocpd SQLite database).  The summary is a Markdown table per kernel:
launches, average duration, and, when counter runs are given, the average
FETCH_SIZE / WRITE_SIZE per launch.  Counter values are scaled by the ratio
of the known traffic of the calibration copy kernel (an elementwise kernel
that reads and writes M MiB, launched first by bench.py --copy-probe-mib M)
to what the same counter reports for it.  With --digest the summary records
a digest of the kernel sources, so that a reader (bench.py) can tell whether
the counters still describe the kernels as built.
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import os
import sqlite3


def _csv_rows(directory, suffix):
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _col(row, *names):
    low = {k.lower(): k for k in row}
    for n in names:
        if n.lower() in low:
            return row[low[n.lower()]]
    raise KeyError(names)


def kernel_durations(directory):
    """{kernel name: [durations in ns]}"""
    out = collections.defaultdict(list)
    rows = _csv_rows(directory, "kernel_trace.csv")
    if rows:
        for r in rows:
            name = _col(r, "Kernel_Name", "kernel_name")
            t0 = int(_col(r, "Start_Timestamp", "start"))
            t1 = int(_col(r, "End_Timestamp", "end"))
            out[name].append(t1 - t0)
        return out
    for db in glob.glob(os.path.join(directory, "**", "*.db"), recursive=True):
        con = sqlite3.connect(db)
        for name, t0, t1 in con.execute("select name, start, end from kernels"):
            out[name].append(int(t1) - int(t0))
    return out


def kernel_counters(directory, counter):
    """{kernel name: [counter value per dispatch]}"""
    out = collections.defaultdict(list)
    rows = _csv_rows(directory, "counter_collection.csv")
    if rows:
        for r in rows:
            if _col(r, "Counter_Name", "counter_name") != counter:
                continue
            out[_col(r, "Kernel_Name", "kernel_name")].append(float(_col(r, "Counter_Value", "value")))
        return out
    for db in glob.glob(os.path.join(directory, "**", "*.db"), recursive=True):
        con = sqlite3.connect(db)
        for name, val in con.execute(
                "select kernel_name, value from counters_collection where counter_name = ?", (counter,)):
            out[name].append(float(val))
    return out


def _short(name, width=72):
    name = name.replace("kp::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def _calibration(counts, copy_mib):
    """Scale factor: known KiB of the copy kernel / reported KiB."""
    if not copy_mib:
        return None
    cand = [k for k in counts if "elementwise" in k and counts[k]]
    if not cand:
        return None
    known = copy_mib * 1024.0
    best = max(cand, key=lambda k: max(counts[k]))
    reported = max(counts[best])
    return known / reported if reported > 0 else None


def kernel_source_digest(root=None):
    """sha256 over the GPU kernel sources (csrc/*.hip and csrc/*.h, sorted by name)."""
    import hashlib
    root = root or os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(root, "csrc", "*.hip")) + glob.glob(os.path.join(root, "csrc", "*.h"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


DIGEST_LINE = "Kernel source digest (sha256 of csrc/*.hip and csrc/*.h): "


def measured_traffic(summary_path, pattern):
    """Fetch and write bytes per launch of the kernel matching `pattern` (a regular
    expression; of several rows the one with the most launches) in a summary this
    module wrote, with the kernel source digest recorded there; None if absent."""
    import re
    if not os.path.exists(summary_path):
        return None
    digest, best = None, None
    with open(summary_path) as fh:
        for line in fh:
            if line.startswith(DIGEST_LINE):
                digest = line[len(DIGEST_LINE):].strip()
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) != 7 or not re.search(pattern, cells[0]):
                continue
            try:
                launches, fetch, write = int(cells[1]), float(cells[5]), float(cells[6])
            except ValueError:
                continue
            if best is None or launches > best["launches"]:
                best = {"kernel": cells[0].strip("`"), "launches": launches,
                        "fetch_bytes": fetch * 1e6, "write_bytes": write * 1e6}
    if best is None:
        return None
    best["digest"] = digest
    return best


def summarize(trace, fetch=None, write=None, copy_mib=0, title="", commands=(), digest=None):
    dur = kernel_durations(trace)
    fc = kernel_counters(fetch, "FETCH_SIZE") if fetch else {}
    wc = kernel_counters(write, "WRITE_SIZE") if write else {}
    ff = _calibration(fc, copy_mib)
    wf = _calibration(wc, copy_mib)
    total = sum(sum(v) for v in dur.values())
    lines = []
    if title:
        lines += [f"# {title}", ""]
    if commands:
        lines += ["Commands (run from the repository root on the GPU box):", "", "```"]
        lines += list(commands)
        lines += ["```", ""]
    if digest:
        lines += [DIGEST_LINE + digest, ""]
    if fetch or write:
        lines += [f"Counter calibration (copy kernel of {copy_mib} MiB read + {copy_mib} MiB written): "
                  f"FETCH_SIZE x {ff:.3f}, WRITE_SIZE x {wf:.3f}" if ff and wf else
                  "Counter calibration: not available", ""]
    hdr = "| kernel | launches | avg us | total ms | % |"
    sep = "|---|---:|---:|---:|---:|"
    if fetch or write:
        hdr += " fetch MB/launch | write MB/launch |"
        sep += "---:|---:|"
    lines += [hdr, sep]
    for name, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        row = (f"| `{_short(name)}` | {len(v)} | {sum(v) / len(v) / 1e3:.1f} | {sum(v) / 1e6:.3f} | "
               f"{100.0 * sum(v) / total:.1f} |")
        if fetch or write:
            def mb(counts, fac):
                vals = counts.get(name)
                if not vals:
                    return "-"
                avg = sum(vals) / len(vals) * (fac or 1.0)
                return f"{avg * 1024 / 1e6:.1f}"
            row += f" {mb(fc, ff)} | {mb(wc, wf)} |"
        lines.append(row)
    return "\n".join(lines) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=int, default=0)
    ap.add_argument("--title", default="")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--out")
    ap.add_argument("--digest", action="store_true",
                    help="record the digest of the kernel sources the profile was taken with")
    a = ap.parse_args(argv)
    text = summarize(a.trace, a.fetch, a.write, a.copy_mib, a.title, a.command,
                     kernel_source_digest() if a.digest else None)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(text)
    else:
        print(text)


if __name__ == "__main__":
    main()
