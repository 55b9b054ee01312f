"""Summaries of rocprofv3 output databases (ROCm 7 rocpd SQLite files).

  python -m paper_2401_15758_amd.profile_summary stats DB [--match S] [--grid X]
      per-kernel launches, total and average duration, share of kernel time,
      as a markdown table; --match keeps kernels whose name contains S, --grid
      keeps launches whose grid_x (work-items) equals X.

  python -m paper_2401_15758_amd.profile_summary traffic FETCH_DB WRITE_DB --kernel S --grid X
      [--grid-y Y] --calib-mib M [--tiling JSON] [--workload W] [--sources F ...] [--out JSON]
      HBM bytes per launch of the launches of kernel S with grid_x X (and
      grid_y Y), from a FETCH_SIZE run and a WRITE_SIZE run (KiB per dispatch,
      summed over the counter's instances).  Each counter is scaled by what it reads on the run's
      calibration dispatch: the last elementwise copy kernel, which reads and
      writes M MiB.  --sources records the sha256 of the kernel's source files, so
      that a reader can tell whether the record still matches the code.
"""
import argparse
import hashlib
import json
import sqlite3
import sys


def _kernels(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration, grid_x, dispatch_id, grid_y from kernels order by dispatch_id").fetchall()
    con.close()
    return rows


def short_name(name):
    """Kernel name without return type, anonymous namespace and parameter list."""
    n = name.replace("(anonymous namespace)::", "")
    n = n[5:] if n.startswith("void ") else n
    return n.split("(")[0]


def stats(db, match=None, grid=None):
    rows = _kernels(db)
    total_all = sum(r[1] for r in rows)
    sel = [r for r in rows if (match is None or match in r[0]) and (grid is None or r[2] == grid)]
    agg = {}
    for name, dur, *_ in sel:
        a = agg.setdefault(name, [0, 0])
        a[0] += 1
        a[1] += dur
    out = [f"Total kernel time {total_all / 1e6:.2f} ms over {len(rows)} launches"
           + (f"; selected {sum(a[1] for a in agg.values()) / 1e6:.2f} ms" if (match or grid) else "") + ".", "",
           "| kernel | calls | total ms | avg us | % of all |", "|---|---|---|---|---|"]
    for name, (n, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        out.append(f"| `{short_name(name)}` | {n} | {t / 1e6:.2f} | {t / n / 1e3:.2f} | {100 * t / total_all:.1f} |")
    return "\n".join(out)


def _counter_per_dispatch(db, counter):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, sum(counter_value) from pmc_events where counter_name = ? "
                       "group by dispatch_id", (counter,)).fetchall()
    con.close()
    return dict(rows)


def traffic(fetch_db, write_db, kernel, grid, calib_mib, tiling=None, workload=None, sources=(), grid_y=None):
    rec = {"kernel": kernel, "grid_x": grid, "grid_y": grid_y, "workload": workload, "tiling": tiling or {}}
    if sources:
        h = hashlib.sha256()
        for s in sources:
            with open(s, "rb") as f:
                h.update(f.read())
        rec["source_sha256"] = h.hexdigest()
    copy_kib = calib_mib * 1024.0
    for db, counter, key in ((fetch_db, "FETCH_SIZE", "fetch"), (write_db, "WRITE_SIZE", "write")):
        per = _counter_per_dispatch(db, counter)
        ks = _kernels(db)
        sel = [per[d] for name, _, g, d, gy in ks
               if kernel in name and g == grid and (grid_y is None or gy == grid_y) and d in per]
        copies = [per[d] for name, _, g, d, _ in ks if "elementwise" in name.lower() and d in per]
        if not sel or not copies:
            raise SystemExit(f"{db}: no {counter} values for {kernel!r} at grid {grid} or no calibration copy")
        calib = copies[-1]
        scale = copy_kib / calib
        raw = sum(sel) / len(sel)
        rec[f"{key}_launches"] = len(sel)
        rec[f"{key}_kib_raw"] = raw
        rec[f"{key}_calib_kib"] = calib
        rec[f"{key}_scale"] = scale
        rec[f"{key}_bytes_per_launch"] = raw * scale * 1024.0
    rec["bytes_per_launch"] = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return rec


def main(argv=None):
    ap = argparse.ArgumentParser(description="rocprofv3 database summaries")
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--match")
    s.add_argument("--grid", type=int)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_db")
    t.add_argument("write_db")
    t.add_argument("--kernel", required=True)
    t.add_argument("--grid", type=int, required=True)
    t.add_argument("--grid-y", type=int)
    t.add_argument("--calib-mib", type=int, required=True)
    t.add_argument("--tiling")
    t.add_argument("--workload")
    t.add_argument("--sources", nargs="*", default=())
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats(a.db, a.match, a.grid))
        return
    rec = traffic(a.fetch_db, a.write_db, a.kernel, a.grid, a.calib_mib,
                  json.loads(a.tiling) if a.tiling else None, a.workload, a.sources, a.grid_y)
    if a.out:
        try:
            with open(a.out) as f:
                doc = json.load(f)
        except (OSError, ValueError):
            doc = {}
        recs = [r for r in doc.get("records", []) if not (r.get("kernel") == rec["kernel"]
                                                          and r.get("workload") == rec["workload"])]
        doc["records"] = recs + [rec]
        with open(a.out, "w") as f:
            json.dump(doc, f, indent=1)
    json.dump(rec, sys.stdout, indent=1)
    print()


if __name__ == "__main__":
    main()
