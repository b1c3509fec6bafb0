"""Condense rocprofv3 CSV output into the short text summaries kept under profiles/.

Three summaries:

* kernel statistics (``--kernel-trace --stats``): calls and average / min / max
  duration per kernel;
* HBM bytes from two counter runs (``--pmc FETCH_SIZE``, then ``--pmc
  WRITE_SIZE``, both in KiB per dispatch).  Each counter is scaled by what it
  reads for a plain device copy of known size in the same run (the largest
  ``__amd_rocclr_copyBuffer`` dispatch, ``bench.py --calibrate-copy``: 1 GiB read
  and 1 GiB written), so the scaled figure is in bytes of HBM traffic;
* vector-ALU issue from one counter run (``--pmc SQ_WAVES SQ_INSTS_VALU
  VALUBusy``): wavefronts, VALU instructions issued (counted once per
  wavefront instruction) and the share of the kernel's time the CUs' vector
  ALUs were busy, per dispatch.

The counter summaries record the SHA-256 of the HIP source the counters were
taken on; ``bench.py`` uses their figures only while that source is unchanged.

    python -m paper_2208_12795_amd.rocprof_summary stats  <dir> <prefix> <out.md> --command "..."
    python -m paper_2208_12795_amd.rocprof_summary traffic <fetch_dir> <write_dir> <prefix> <out.md> --command "..."
    python -m paper_2208_12795_amd.rocprof_summary valu <dir> <prefix> <out.md> --command "..."
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

COPY_KERNEL = "__amd_rocclr_copyBuffer"
CALIB_BYTES = 1 << 30
HIP_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "etpic.hip")


def source_sha256(path: str = HIP_SOURCE) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def short_name(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "")
    if n.startswith("void "):
        n = n[5:]
    return n.split("(")[0]


def load_counters(path: str) -> dict:
    per = collections.defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            per[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return per


def load_counter_table(path: str) -> dict:
    """kernel -> counter -> list of per-dispatch values (a run of several counters)"""
    per = collections.defaultdict(lambda: collections.defaultdict(list))
    with open(path) as f:
        for r in csv.DictReader(f):
            per[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return per


def stats_summary(prof_dir: str, prefix: str, command: str) -> str:
    with open(os.path.join(prof_dir, f"{prefix}_kernel_stats.csv")) as f:
        rows = list(csv.DictReader(f))
    out = ["# rocprofv3 kernel statistics", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | % of GPU time |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(out) + "\n"


def traffic_summary(fetch_dir: str, write_dir: str, prefix: str, command: str, sha: str) -> str:
    fetch = load_counters(os.path.join(fetch_dir, f"{prefix}_counter_collection.csv"))
    write = load_counters(os.path.join(write_dir, f"{prefix}_counter_collection.csv"))
    f_copy, w_copy = max(fetch[COPY_KERNEL]), max(write[COPY_KERNEL])
    sf = CALIB_BYTES / 1024 / f_copy
    sw = CALIB_BYTES / 1024 / w_copy
    out = ["# HBM traffic per dispatch from FETCH_SIZE / WRITE_SIZE", "", "Commands (one counter per run):", "",
           "```", command, "```", "",
           f"source_sha256: {sha}", "",
           f"Copy calibration (`{COPY_KERNEL}`, {CALIB_BYTES} B read and written): FETCH_SIZE {f_copy:.0f} KiB, "
           f"WRITE_SIZE {w_copy:.0f} KiB per dispatch; scale factors {sf:.4f} (fetch), {sw:.4f} (write).", "",
           "| kernel | dispatches | FETCH_SIZE KiB (raw mean) | WRITE_SIZE KiB (raw mean) | HBM bytes (scaled) |",
           "|---|---|---|---|---|"]
    tagged = []
    for k in sorted(set(fetch) & set(write), key=lambda k: -sum(fetch[k]) / len(fetch[k])):
        if k == COPY_KERNEL:
            continue
        fm = sum(fetch[k]) / len(fetch[k])
        wm = sum(write[k]) / len(write[k])
        tot = (fm * sf + wm * sw) * 1024
        out.append(f"| `{short_name(k)}` | {len(fetch[k])} | {fm:.0f} | {wm:.0f} | {tot:.4g} |")
        tagged.append(f"traffic_bytes {short_name(k)}: {int(round(tot))}")
    return "\n".join(out + ["", "Machine-readable:", "", "```"] + tagged + ["```"]) + "\n"


def valu_summary(prof_dir: str, prefix: str, command: str, sha: str) -> str:
    per = load_counter_table(os.path.join(prof_dir, f"{prefix}_counter_collection.csv"))
    out = ["# Vector-ALU issue per dispatch from SQ_WAVES / SQ_INSTS_VALU / VALUBusy", "", "Command:", "", "```",
           command, "```", "", f"source_sha256: {sha}", "",
           "SQ_INSTS_VALU counts one per wavefront instruction; a wavefront (64 lanes) occupies a 16-lane SIMD "
           "for 4 cycles per VALU instruction, so the issue ceiling is 256 CUs x 4 SIMDs x 2.4 GHz / 4 = "
           "614.4e9 wavefront instructions per second.  VALUBusy is rocprofv3's derived share of the "
           "dispatch's GPU-active time the CUs' vector ALUs were busy.", "",
           "| kernel | dispatches | wavefronts | VALU instructions | per wavefront | VALUBusy % |",
           "|---|---|---|---|---|---|"]
    tagged = []
    rows = []
    for k, d in per.items():
        if "SQ_INSTS_VALU" not in d or "SQ_WAVES" not in d:
            continue
        mean = {c: sum(v) / len(v) for c, v in d.items()}
        rows.append((k, len(d["SQ_INSTS_VALU"]), mean))
    for k, nd, mean in sorted(rows, key=lambda r: -r[2]["SQ_INSTS_VALU"]):
        waves, insts = mean["SQ_WAVES"], mean["SQ_INSTS_VALU"]
        busy = mean.get("VALUBusy")
        out.append(f"| `{short_name(k)}` | {nd} | {waves:.0f} | {insts:.4g} | {insts / max(waves, 1):.1f} | "
                   f"{'' if busy is None else f'{busy:.1f}'} |")
        tagged.append(f"valu_insts {short_name(k)}: {int(round(insts))}")
        if busy is not None:
            tagged.append(f"valu_busy {short_name(k)}: {busy:.2f}")
    return "\n".join(out + ["", "Machine-readable:", "", "```"] + tagged + ["```"]) + "\n"


def _tagged(path: str, tag: str, kernel: str, sha: str | None):
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^source_sha256: ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(1) != (sha or source_sha256()):
        return None
    m = re.search(r"^" + tag + " " + re.escape(kernel) + r": ([0-9.]+)$", text, re.M)
    return m.group(1) if m else None


def read_valu(path: str, kernel: str, sha: str | None = None):
    """(VALU instructions per dispatch, VALUBusy %) of `kernel` from a VALU
    summary, or None if the file is missing, lacks the kernel, or was taken on
    another source."""
    n = _tagged(path, "valu_insts", kernel, sha)
    if n is None:
        return None
    b = _tagged(path, "valu_busy", kernel, sha)
    return int(n), (None if b is None else float(b))


def read_traffic(path: str, kernel: str, sha: str | None = None):
    """Scaled HBM bytes per dispatch of `kernel` from a traffic summary, or None
    if the file is missing, lacks the kernel, or was taken on another source."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"^source_sha256: ([0-9a-f]{64})$", text, re.M)
    if not m or m.group(1) != (sha or source_sha256()):
        return None
    m = re.search(r"^traffic_bytes " + re.escape(kernel) + r": (\d+)$", text, re.M)
    return int(m.group(1)) if m else None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("prefix")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_dir")
    t.add_argument("write_dir")
    t.add_argument("prefix")
    t.add_argument("out")
    t.add_argument("--command", required=True)
    t.add_argument("--sha", default=None, help="SHA-256 of the HIP source profiled (default: the current one)")
    v = sub.add_parser("valu")
    v.add_argument("dir")
    v.add_argument("prefix")
    v.add_argument("out")
    v.add_argument("--command", required=True)
    v.add_argument("--sha", default=None, help="SHA-256 of the HIP source profiled (default: the current one)")
    a = ap.parse_args()
    if a.mode == "stats":
        text = stats_summary(a.dir, a.prefix, a.command)
    elif a.mode == "valu":
        text = valu_summary(a.dir, a.prefix, a.command, a.sha or source_sha256())
    else:
        text = traffic_summary(a.fetch_dir, a.write_dir, a.prefix, a.command, a.sha or source_sha256())
    with open(a.out, "w") as f:
        f.write(text)
    print(text)


if __name__ == "__main__":
    main()
