"""Turns rocprofv3 CSV output into the short markdown summaries kept in profiles/.

Usage (after the rocprofv3 runs named in the summary it writes):
  python3 -m paper_2009_12584_amd.rocprof_summary --stats DIR --fetch DIR --write DIR \
      --kernel-hash HASH --out FILE [--commands TEXT]

--stats   directory of a `rocprofv3 --kernel-trace --stats --output-format csv` run
--fetch   directory of a `rocprofv3 --pmc FETCH_SIZE --output-format csv` run
--write   directory of a `rocprofv3 --pmc WRITE_SIZE --output-format csv` run

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are calibrated with the copy
probe kernel of the same runs, whose true read and write byte counts are
known: bytes = counter KiB * 1024 * (true copy bytes / copy counter bytes).
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
from collections import defaultdict

COPY_KERNEL = "k_copy_probe"


def _one(dirname, suffix):
    files = glob.glob(os.path.join(dirname, "*" + suffix))
    if not files:
        raise FileNotFoundError("no *%s in %s" % (suffix, dirname))
    return files[0]


def short_name(name: str) -> str:
    """'void mclbm::k_step<float, 8, 2, 0, false>(mclbm::Inst, ...)' -> 'k_step<float, 8, 2, 0, false>'."""
    n = re.sub(r"^void ", "", name)
    n = re.sub(r"^\(anonymous namespace\)::", "", n)
    n = re.sub(r"^mclbm::", "", n)
    n = re.sub(r"^\(anonymous namespace\)::", "", n)
    depth, out = 0, []
    for ch in n:
        if ch == "(" and depth == 0:
            break
        depth += ch == "<"
        depth -= ch == ">"
        out.append(ch)
    return "".join(out).strip()


def kernel_stats(dirname):
    rows = []
    with open(_one(dirname, "_kernel_stats.csv")) as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                         float(r["Percentage"])))
    return rows


def pmc_means(dirname, counter):
    acc = defaultdict(list)
    with open(_one(dirname, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter:
                acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def copy_bytes(dirname, counter):
    """True bytes per copy-probe dispatch, from its grid size (16 B per lane)."""
    with open(_one(dirname, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if COPY_KERNEL in r["Kernel_Name"] and r["Counter_Name"] == counter:
                return int(r["Grid_Size"]) * 16
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--kernel-hash", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--commands", default="")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args()

    lines = ["# %s" % a.title, "", "kernel source hash: `%s`" % a.kernel_hash, ""]
    if a.commands:
        lines += ["Commands (run from the repository root on the GPU box):", "", "```"]
        lines += [c.strip() for c in a.commands.split(";;") if c.strip()]
        lines += ["```", ""]
    lines += ["## Kernel time (`--kernel-trace --stats`)", "", "| kernel | calls | avg us | % time |",
              "|---|---|---|---|"]
    for name, calls, avg, pct in kernel_stats(a.stats)[: a.top]:
        lines.append("| %s | %d | %.2f | %.2f |" % (name, calls, avg, pct))
    lines.append("")
    if a.fetch and a.write:
        fetch = pmc_means(a.fetch, "FETCH_SIZE")
        write = pmc_means(a.write, "WRITE_SIZE")
        true_copy = copy_bytes(a.fetch, "FETCH_SIZE")
        copy_fetch = fetch.get(next((k for k in fetch if COPY_KERNEL in k), ""), None)
        copy_write = write.get(next((k for k in write if COPY_KERNEL in k), ""), None)
        kf = true_copy / (copy_fetch * 1024) if true_copy and copy_fetch else 1.0
        kw = true_copy / (copy_write * 1024) if true_copy and copy_write else 1.0
        lines += ["## HBM traffic per dispatch (`--pmc FETCH_SIZE`, `--pmc WRITE_SIZE`)", "",
                  "Calibration: the copy probe moves %d B each way per dispatch; FETCH_SIZE reads %.1f KiB "
                  "(factor %.3f), WRITE_SIZE reads %.1f KiB (factor %.3f)." % (
                      true_copy or 0, copy_fetch or 0, kf, copy_write or 0, kw), "",
                  "| kernel | fetch MB | write MB | total MB |", "|---|---|---|---|"]
        for k in sorted(set(fetch) & set(write), key=lambda k: -(fetch[k] * kf + write[k] * kw)):
            fb = fetch[k] * 1024 * kf / 1e6
            wb = write[k] * 1024 * kw / 1e6
            lines.append("| %s | %.3f | %.3f | %.3f |" % (k, fb, wb, fb + wb))
        lines.append("")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
