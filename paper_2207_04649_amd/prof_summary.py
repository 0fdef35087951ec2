"""Summarise a rocprofv3 kernel trace (rocpd SQLite output) per kernel."""
from __future__ import annotations

import re
import sqlite3
import sys


def short_name(name: str) -> str:
    m = re.search(r'(k_\w+)(<[^>]*>)?', name)
    return m.group(0) if m else name.split('(')[0][:60]


def summary(db: str) -> list[tuple]:
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    return [(short_name(n), cnt, avg / 1e3, mn / 1e3, mx / 1e3, tot / 1e6) for n, cnt, avg, mn, mx, tot in rows]


def render(db: str, command: str = "") -> str:
    out = []
    if command:
        out.append(f"command: {command}")
    out.append(f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_ms':>10s}")
    for n, cnt, avg, mn, mx, tot in summary(db):
        out.append(f"{n[:40]:40s} {cnt:6d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {tot:10.3f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(render(sys.argv[1], " ".join(sys.argv[2:])))
