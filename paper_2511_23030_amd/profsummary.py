"""Summarise a rocprofv3 run: per-kernel calls and durations from the
``top_kernels`` view of its rocpd database, as a Markdown table.

python -m paper_2511_23030_amd.profsummary <run_results.db>
python -m paper_2511_23030_amd.profsummary traffic <fetch.csv> <write.csv> <kernel regex>
    <copy regex> <copy bytes> <source file> <out.json> <command>
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short_name(n: str) -> str:
    n = n.replace("dcgs::(anonymous namespace)::", "").replace("void ", "")
    return re.split(r"\(", n, maxsplit=1)[0]


def summary(db: str, limit: int = 20) -> str:
    c = sqlite3.connect(db)
    rows = list(c.execute("select name, total_calls, total_duration, average, percentage "
                          "from top_kernels limit ?", (limit,)))
    out = ["| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows:
        out.append(f"| `{short_name(n)}` | {calls} | {tot:.0f} | {avg:.1f} | {pct:.1f} |")
    return "\n".join(out)




def _counter_rows(csv_path: str, counter: str):
    """(kernel name, value) per dispatch of one counter from a rocprofv3
    counter_collection.csv."""
    import csv
    with open(csv_path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") == counter:
                yield row.get("Kernel_Name", ""), float(row["Counter_Value"])


def traffic(fetch_csv: str, write_csv: str, kernel_regex: str, copy_regex: str,
            copy_bytes: float) -> dict:
    """HBM bytes per launch of the kernels matching kernel_regex: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch) averaged over its dispatches, each
    scaled by bytes / counter of a plain copy kernel that moves copy_bytes
    (read once, written once)."""
    out = {}
    for name, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        k_vals, c_vals = [], []
        for kname, v in _counter_rows(path, name):
            if re.search(kernel_regex, kname):
                k_vals.append(v)
            elif re.search(copy_regex, kname):
                c_vals.append(v)
        if not k_vals or not c_vals:
            raise ValueError(f"{name}: kernel or copy dispatches not found")
        scale = copy_bytes / (max(c_vals) * 1024.0)
        out[name] = {"kernel_kib_avg": sum(k_vals) / len(k_vals), "dispatches": len(k_vals),
                     "copy_kib": max(c_vals), "scale": scale,
                     "bytes_per_launch": sum(k_vals) / len(k_vals) * 1024.0 * scale}
    out["bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + \
        out["WRITE_SIZE"]["bytes_per_launch"]
    return out


def source_digest(path: str) -> str:
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _main(argv):
    if len(argv) < 2 or argv[1] in ("-h", "--help"):
        print(__doc__)
        return
    if argv[1] == "traffic":
        # traffic <fetch.csv> <write.csv> <kernel regex> <copy regex> <copy bytes> <source> <out.json> <command>
        import json
        t = traffic(argv[2], argv[3], argv[4], argv[5], float(argv[6]))
        t["source_sha256"] = source_digest(argv[7])
        t["source"] = argv[7]
        t["kernel_regex"] = argv[4]
        t["command"] = argv[9]
        with open(argv[8], "w") as f:
            json.dump(t, f, indent=1)
        print(json.dumps(t, indent=1))
    else:
        print(summary(argv[1]))



def trace_summary(trace_csv: str, focus_regex: str, limit: int = 16) -> str:
    """Markdown of a rocprofv3 kernel_trace.csv: per kernel and launch size
    (grid threads), calls and average/min/max duration."""
    import csv
    from collections import defaultdict
    d = defaultdict(list)
    with open(trace_csv, newline="") as f:
        for r in csv.DictReader(f):
            n = short_name(r["Kernel_Name"])
            g = int(r.get("Grid_Size_X") or 0) * int(r.get("Grid_Size_Y") or 1) * \
                int(r.get("Grid_Size_Z") or 1)
            d[(n, g)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in d.values())
    rows = sorted(d.items(), key=lambda kv: -sum(kv[1]))[:limit]
    out = ["| kernel | grid threads | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|---|"]
    for (n, g), v in rows:
        out.append(f"| `{n}` | {g} | {len(v)} | {sum(v) / 1e3:.1f} | {sum(v) / len(v):.1f} | "
                   f"{min(v):.1f} | {max(v):.1f} | {100 * sum(v) / total:.1f} |")
    foc = [(k, v) for k, v in d.items() if re.search(focus_regex, k[0])]
    if foc:
        (n, g), v = max(foc, key=lambda kv: kv[0][1])
        out.append("")
        out.append(f"Largest launch of `{n}` (grid {g} threads): {len(v)} calls, average "
                   f"{sum(v) / len(v) / 1e3:.3f} ms.")
    return "\n".join(out)


if __name__ == "__main__":
    _main(sys.argv)
