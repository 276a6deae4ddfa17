"""Short summaries of rocprofv3 output, written under profiles/.

Kernel-trace statistics (text):
    python -m paper_2002_01392_amd.profsummary trace <results.db> <out.txt> "<command>"

MFMA use per kernel class from one counter run (SQ_INSTS_VALU_MFMA_F64,
SQ_INSTS_VALU_MFMA_MOPS_F64, SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE;
utilisation = busy cycles / (active cycles x SIMDs), FP64 MFMA peak 78.6 TF/s):
    python -m paper_2002_01392_amd.profsummary mfma <counters.csv> <out.txt> <simds> "<command>"

HBM traffic per launch from two counter runs (FETCH_SIZE, then WRITE_SIZE,
both in KiB per dispatch), each scaled by what the same counter reads for the
largest plain device copy in the run (a 1 GiB copy: it reads and writes
exactly 1 GiB), one JSON file per kernel class:
    python -m paper_2002_01392_amd.profsummary pmc <fetch.csv> <write.csv> <workload> \\
        <kernel source hash> "<fetch command>" "<write command>"
"""
import collections
import csv
import json
import os
import sqlite3
import statistics
import sys

# summaries go to the repository's profiles/ folder
HERE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")

# kernel name prefix -> timing class of the library (the y kernel serves three
# classes of equal traffic pattern; it is reported as one)
CLASSES = {"fcns::k_x_nl<": "x_nl", "fcns::k_x_nlw<": "x_nl", "fcns::k_x_nlw_q<": "x_nl",
           "fcns::k_z_stageA<": "z_stageA", "fcns::k_z_stageB<": "z_stageB",
           "fcns::k_z_back<": "z_back", "fcns::k_z_pass<": "z_pass", "fcns::k_y<": "y"}
COPY_BYTES = 1 << 30


def trace(db, out, cmd):
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels").fetchall()
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --kernel-trace --stats summary\n# command: {cmd}\n")
        fh.write("# kernel | calls | total_ms | avg_ms | percent  (top_kernels view: durations in us)\n")
        for name, n, tot, avg, pct in rows:
            short = name.split("(")[0].replace("void ", "")
            fh.write(f"{short} | {n} | {tot / 1e3:.2f} | {avg / 1e3:.4f} | {pct:.2f}\n")


def _per_dispatch(path, counter):
    out = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            out.append((r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    return out


def _per_launch(rows):
    """Median per kernel name (template variants of a class differ, e.g. the
    first RK stage's stage A reads one state array less; a median keeps
    the odd dispatch outside the step out), then the mean over the names
    weighted by their dispatches."""
    by = collections.defaultdict(list)
    for n, v in rows:
        by[n].append(v)
    tot = sum(len(v) for v in by.values())
    return sum(statistics.median(v) * len(v) for v in by.values()) / tot


def pmc(fetch_csv, write_csv, workload, src_hash, cmd_fetch, cmd_write):
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")
    cf = max(v for n, g, v in fetch if "copyBuffer" in n)
    cw = max(v for n, g, v in write if "copyBuffer" in n)
    kf = COPY_BYTES / (cf * 1024.0)
    kw = COPY_BYTES / (cw * 1024.0)
    for prefix, cls in CLASSES.items():
        fr = [(n, g, v) for n, g, v in fetch if n.replace("void ", "").startswith(prefix)]
        wr = [(n, g, v) for n, g, v in write if n.replace("void ", "").startswith(prefix)]
        if not fr or not wr:
            continue
        # the dispatches of the largest grid (the workload's own launches),
        # per launch as in _per_launch
        gmax = max(g for _, g, _ in fr)
        fv = [(n, v) for n, g, v in fr if g == gmax]
        wv = [(n, v) for n, g, v in wr if g == gmax]
        fb = _per_launch(fv) * 1024.0 * kf
        wb = _per_launch(wv) * 1024.0 * kw
        rec = {"kernel_class": cls, "workload": workload, "source_hash": src_hash,
               "hbm_bytes_per_launch": int(fb + wb), "read_bytes": int(fb),
               "write_bytes": int(wb), "dispatches": len(fv),
               "calibration": {"copy_bytes": COPY_BYTES, "fetch_kib": cf, "write_kib": cw,
                               "fetch_factor": kf, "write_factor": kw},
               "commands": [cmd_fetch, cmd_write]}
        with open(os.path.join(HERE, f"pmc_{cls}_{workload}.json"), "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")


def mfma(path, out, simds, cmd):
    simds = int(simds)
    rows = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"].replace("void ", "")
        cls = next((c for pre, c in CLASSES.items() if name.startswith(pre)), None)
        if cls is None:
            continue
        rows[(cls, int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    with open(out, "w") as fh:
        fh.write(f"# rocprofv3 --pmc MFMA summary (FC extension on the matrix cores)\n# command: {cmd}\n")
        fh.write("# class | dispatches | MFMA F64 insts / dispatch | MFMA FP64 flop / dispatch | "
                 "MFMA busy %  (median over the dispatches of the largest grid)\n")
        best = {}
        for (cls, grid), d in rows.items():
            if cls not in best or grid > best[cls][0]:
                best[cls] = (grid, d)
        for cls, (grid, d) in sorted(best.items()):
            med = {k: statistics.median(v) for k, v in d.items()}
            n = len(next(iter(d.values())))
            flop = med.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512
            util = 100.0 * med.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / max(
                med.get("GRBM_GUI_ACTIVE", 1.0) * simds, 1.0)
            fh.write(f"{cls} | {n} | {med.get('SQ_INSTS_VALU_MFMA_F64', 0):.0f} | {flop:.3e} | {util:.3f}\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:5])
    elif sys.argv[1] == "pmc":
        pmc(*sys.argv[2:8])
    elif sys.argv[1] == "mfma":
        mfma(*sys.argv[2:6])
    else:
        raise SystemExit(__doc__)
