"""Summarise a rocprofv3 run: per-kernel calls and durations from the
``top_kernels`` view of its rocpd database, as a Markdown table.

python -m paper_2511_23030_amd.profsummary <run_results.db> [title]
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


if __name__ == "__main__":
    print(summary(sys.argv[1]))
