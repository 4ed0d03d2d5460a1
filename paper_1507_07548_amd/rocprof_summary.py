"""Writes a short per-kernel summary (calls, average and total duration) from
a rocprofv3 --kernel-trace results database (`*_results.db`)."""
import sqlite3
import sys


def summarize(db_path, top=12):
    con = sqlite3.connect(db_path)
    rows = con.execute("select name, count(*), avg(duration), sum(duration) from kernels "
                       "group by name order by sum(duration) desc").fetchall()
    total = sum(r[3] for r in rows)
    out = ["| kernel | calls | avg us | total ms | % time |", "|---|---|---|---|---|"]
    for name, calls, avg, tot in rows[:top]:
        out.append(f"| `{name.split('(')[0]}` | {calls} | {avg / 1e3:.1f} | {tot / 1e6:.2f} | {100 * tot / total:.1f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1]))
