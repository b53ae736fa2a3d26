"""Summarise a rocprofv3 kernel-trace database (rocpd SQLite) into a short
text table: per kernel name, launches, average/total duration."""
import sqlite3
import sys


def main(db, top=20):
    c = sqlite3.connect(db)
    rows = c.execute("select name, count(*), avg(duration), sum(duration), min(duration), max(duration) "
                     "from kernels group by name order by sum(duration) desc").fetchall()
    tot = sum(r[3] for r in rows)
    print("busy = launches longer than 5% of the kernel's longest (PCG launches queued after")
    print("convergence return at once; the library's own event timing leaves them out too)")
    print(f"{'launches':>8} {'avg_us':>10} {'busy_n':>7} {'busy_avg_us':>11} {'max_us':>9} {'total_ms':>9} {'pct':>6}  kernel")
    for r in rows[:top]:
        busy = c.execute("select count(*), avg(duration) from kernels where name = ? and duration > 0.05 * ?",
                         (r[0], r[5])).fetchone()
        print(f"{r[1]:8d} {r[2]/1e3:10.2f} {busy[0]:7d} {busy[1]/1e3:11.2f} {r[5]/1e3:9.2f} {r[3]/1e6:9.3f} "
              f"{100*r[3]/tot:6.2f}  {r[0][:110]}")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 20)
