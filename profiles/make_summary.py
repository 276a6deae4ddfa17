"""Write a short text summary of a rocprofv3 kernel-trace database.

    python profiles/make_summary.py <results.db> <out.txt> "<command that made it>"
"""
import sqlite3
import sys


def main(db, out, cmd):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels").fetchall()
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --kernel-trace --stats summary\n# command: {cmd}\n")
        fh.write("# kernel | calls | total_ms | avg_ms | percent  (top_kernels view: durations in us)\n")
        for name, n, tot, avg, pct in rows:
            short = name.split("(")[0].replace("void ", "")
            fh.write(f"{short} | {n} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {pct:.2f}\n")


if __name__ == "__main__":
    main(*sys.argv[1:4])
