"""Turns rocprofv3 CSV output into the short markdown summaries kept in profiles/.

Usage (after the rocprofv3 runs named in the summary it writes):
  python3 -m paper_2009_12584_amd.rocprof_summary --stats DIR --fetch DIR --write DIR \
      --kernel-hash HASH --out FILE [--commands TEXT]

--stats   directory of a `rocprofv3 --kernel-trace --stats --output-format csv` run
--fetch   directory of a `rocprofv3 --pmc FETCH_SIZE --output-format csv` run
--write   directory of a `rocprofv3 --pmc WRITE_SIZE --output-format csv` run
--issue   directory of a `rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU
          SQ_INSTS_LDS SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR GRBM_GUI_ACTIVE` run

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are calibrated with the copy
probe kernel of the same runs, whose true read and write byte counts are
known: bytes = counter KiB * 1024 * (true copy bytes / copy counter bytes).

The issue table gives wavefront instructions per wave and the VALU issue
fraction: SQ_INSTS_VALU over the cycles the dispatch had, at one VALU
wavefront instruction per compute unit and cycle (4 SIMDs, each taking 4
cycles for a 64-wide instruction); the cycles are GRBM_GUI_ACTIVE, which
counts on every XCD, divided by the XCD count of the agent.
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


def pmc_table(dirname):
    """Per kernel: mean of every counter over its dispatches, and the mean
    dispatch duration in ns."""
    acc = defaultdict(lambda: defaultdict(list))
    dur = defaultdict(dict)
    with open(_one(dirname, "_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = short_name(r["Kernel_Name"])
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            dur[k][r["Dispatch_Id"]] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    out = {}
    for k, c in acc.items():
        m = {n: sum(v) / len(v) for n, v in c.items()}
        m["ns"] = sum(dur[k].values()) / len(dur[k])
        out[k] = m
    return out


def agent_field(dirname, field, default):
    try:
        with open(_one(dirname, "_agent_info.csv")) as f:
            for r in csv.DictReader(f):
                if r.get("Name", "").startswith("gfx") and r.get(field):
                    return int(r[field])
    except (OSError, ValueError):
        pass
    return default


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
    ap.add_argument("--issue")
    ap.add_argument("--kernel-hash", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="rocprofv3 summary")
    ap.add_argument("--commands", default="")
    ap.add_argument("--top", type=int, default=12)
    a = ap.parse_args()

    lines = ["# %s" % a.title, "", "kernel source hash: `%s`" % a.kernel_hash, ""]
    if a.commands:
        lines += ["Commands (run from the repository root on an MI355X):", "", "```"]
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
    if a.issue:
        t = pmc_table(a.issue)
        xcc = agent_field(a.issue, "Num_Xcc", 8)
        cus = agent_field(a.issue, "Cu_Count", 256)
        lines += ["## Instruction issue (`--pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS "
                  "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR GRBM_GUI_ACTIVE`)", "",
                  "Per wavefront: instructions issued.  Clock = GRBM_GUI_ACTIVE / %d XCDs / dispatch "
                  "duration.  VALU issue = SQ_INSTS_VALU / (%d CUs x cycles)." % (xcc, cus), "",
                  "| kernel | waves | VALU/wave | SALU/wave | LDS/wave | VMEM rd/wave | VMEM wr/wave | "
                  "us | clock GHz | VALU issue |", "|---|---|---|---|---|---|---|---|---|---|"]
        # the step kernels and the copy probe; the clock and issue columns
        # only for dispatches long enough (50 us) that the counters' window
        # is the dispatch
        rows = [(k, m) for k, m in t.items() if m.get("SQ_WAVES") and "SQ_INSTS_VALU" in m and
                (k.startswith("k_step") or k.startswith("k_batch") or COPY_KERNEL in k)]
        for k, m in sorted(rows, key=lambda km: -km[1]["ns"]):
            w = m["SQ_WAVES"]
            cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / xcc
            long_enough = cyc > 0 and m["ns"] >= 50e3
            ghz = "%.2f" % (cyc / m["ns"]) if long_enough else "-"
            util = "%.2f" % (m["SQ_INSTS_VALU"] / (cus * cyc)) if long_enough else "-"
            lines.append("| %s | %d | %.0f | %.0f | %.1f | %.1f | %.1f | %.1f | %s | %s |" % (
                k, w, m["SQ_INSTS_VALU"] / w, m.get("SQ_INSTS_SALU", 0) / w, m.get("SQ_INSTS_LDS", 0) / w,
                m.get("SQ_INSTS_VMEM_RD", 0) / w, m.get("SQ_INSTS_VMEM_WR", 0) / w, m["ns"] / 1e3, ghz, util))
        lines.append("")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
