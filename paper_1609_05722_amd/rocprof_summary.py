"""Summarise rocprofv3 output databases (rocpd SQLite) as short text.

    python -m paper_1609_05722_amd.rocprof_summary stats  RESULTS.db [--kernel SUBSTR]
    python -m paper_1609_05722_amd.rocprof_summary pmc    RESULTS.db [--kernel SUBSTR]
    python -m paper_1609_05722_amd.rocprof_summary traffic FETCH.db WRITE.db \
        --kernel SUBSTR --copy-kernel SUBSTR --copy-bytes N --kernel-source FILE \
        --size S --out FILE.json

`stats` lists per-kernel dispatch counts and durations (what
`rocprofv3 --stats` reports); `pmc` lists the mean of every counter per
kernel; `traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch) into HBM
bytes per launch of one kernel, each counter scaled by what it reads for a
plain device copy of known size in the same run.
"""
import argparse
import hashlib
import json
import re
import sqlite3
import sys


def code_hash(path):
    """First 16 hex digits of the SHA-256 of a C/HIP source with its comments
    and whitespace removed: it changes when the code does, not when a
    comment does."""
    with open(path) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return hashlib.sha256(" ".join(text.split()).encode()).hexdigest()[:16]


def short_name(name):
    """A kernel name without its namespaces and trailing parameter list, so
    that its template arguments fit a line."""
    m = re.search(r"fused_step_kernelILi(\d)ENS0_7MathP16ILi(\d)ELi(\d)EDF16([b_])"
                  r"(?:Li(\d+)EEELi(\d)E)?", name)
    if m:   # mangled (the demangler leaves the 16-bit float types alone)
        p16 = "__bf16" if m.group(4) == "b" else "_Float16"
        if m.group(5):   # waves per workgroup and mode (0 step, 1 gradient, 2 + energy)
            return "fused_step_kernel<%s, MathP16<%s, %s, %s, %s>, %s>" % (
                m.group(1), m.group(2), m.group(3), p16, m.group(5), m.group(6))
        return "fused_step_kernel<%s, MathP16<%s, %s, %s> >" % (
            m.group(1), m.group(2), m.group(3), p16)
    for ns in ("fe::(anonymous namespace)::", "fe::"):
        name = name.replace(ns, "")
    if name.startswith("void "):
        name = name[5:]
    cut = name.find(">(")
    return name[:cut + 1] if cut > 0 else name


def kernel_stats(db, like=None, by_grid=False):
    """Dispatch counts and durations per kernel, or per (kernel, grid) with
    by_grid (one kernel launched on different workloads has one line per
    launch shape; `grid` is the work-item count of the launch)."""
    con = sqlite3.connect(db)
    grid = "grid_x * grid_y * grid_z" if by_grid else "0"
    group = "name, grid_x * grid_y * grid_z" if by_grid else "name"
    q = ("select name, %s, count(*), avg(duration), min(duration), max(duration), "
         "sum(duration) from kernels group by %s order by sum(duration) desc" % (grid, group))
    rows = list(con.execute(q))
    total = sum(r[6] for r in rows) or 1
    out = []
    for name, grid, n, avg, mn, mx, tot in rows:
        if like and like not in name:
            continue
        out.append({"kernel": name, "grid": grid, "calls": n, "avg_us": avg / 1e3,
                    "min_us": mn / 1e3, "max_us": mx / 1e3, "total_ms": tot / 1e6,
                    "pct": 100.0 * tot / total})
    return out


def pmc_means(db, like=None):
    con = sqlite3.connect(db)
    q = ("select name, counter_name, count(*), avg(counter_value), sum(counter_value), "
         "count(distinct dispatch_id) from pmc_events group by name, counter_name")
    out = {}
    for name, cn, n, avg, tot, nd in con.execute(q):
        if like and like not in name:
            continue
        # per dispatch: sum over the counter's instances, averaged over dispatches
        out.setdefault(name, {})[cn] = {"per_dispatch": tot / max(nd, 1),
                                        "instances": n // max(nd, 1), "dispatches": nd}
    return out


def dispatch_values(db, counter, like):
    """Per-dispatch value of one counter (summed over its instances) for
    every dispatch of the kernels whose name contains `like`."""
    con = sqlite3.connect(db)
    q = ("select dispatch_id, sum(counter_value) from pmc_events where counter_name = ? "
         "and name like ? group by dispatch_id")
    vals = [v for _, v in con.execute(q, (counter, "%" + like + "%"))]
    if not vals:
        raise SystemExit("no %s for kernels matching %r in %s" % (counter, like, db))
    return vals


def traffic(args):
    fk = dispatch_values(args.fetch_db, "FETCH_SIZE", args.kernel)
    wk = dispatch_values(args.write_db, "WRITE_SIZE", args.kernel)
    fetch_k, write_k = sum(fk) / len(fk), sum(wk) / len(wk)
    # the reference is the largest dispatch of the copy kernel (the copy of
    # known size; smaller dispatches of the same kernel are runtime blits)
    copy_fetch = max(dispatch_values(args.fetch_db, "FETCH_SIZE", args.copy_kernel))
    copy_write = max(dispatch_values(args.write_db, "WRITE_SIZE", args.copy_kernel))
    f_scale = args.copy_bytes / (copy_fetch * 1024.0)
    w_scale = args.copy_bytes / (copy_write * 1024.0)
    rec = {
        "kernel": args.kernel, "kernel_code_sha256_16": code_hash(args.kernel_source),
        "size": args.size,
        "fetch_kib_per_dispatch": fetch_k, "write_kib_per_dispatch": write_k,
        "dispatches": [len(fk), len(wk)],
        "copy_kernel": args.copy_kernel, "copy_bytes": args.copy_bytes,
        "copy_fetch_kib": copy_fetch, "copy_write_kib": copy_write,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "bytes_per_launch": fetch_k * 1024.0 * f_scale + write_k * 1024.0 * w_scale,
        "iterations_checked": True,
    }
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s1 = sub.add_parser("stats")
    s1.add_argument("db")
    s1.add_argument("--kernel")
    s1.add_argument("--by-grid", action="store_true",
                    help="one line per kernel and launch shape (work-items)")
    s2 = sub.add_parser("pmc")
    s2.add_argument("db")
    s2.add_argument("--kernel")
    s3 = sub.add_parser("traffic")
    s3.add_argument("fetch_db")
    s3.add_argument("write_db")
    s3.add_argument("--kernel", required=True)
    s3.add_argument("--copy-kernel", required=True)
    s3.add_argument("--copy-bytes", type=float, required=True)
    s3.add_argument("--kernel-source", required=True)
    s3.add_argument("--size", type=int, required=True)
    s3.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        for r in kernel_stats(a.db, a.kernel, a.by_grid):
            grid = " grid=%-9d" % r["grid"] if a.by_grid else ""
            print("%-70s%s calls=%-6d avg=%9.2f us min=%9.2f max=%9.2f total=%9.3f ms %5.1f%%"
                  % (short_name(r["kernel"])[:70], grid, r["calls"], r["avg_us"], r["min_us"],
                     r["max_us"], r["total_ms"], r["pct"]))
    elif a.cmd == "pmc":
        for k, v in pmc_means(a.db, a.kernel).items():
            print(short_name(k)[:100])
            for cn, d in sorted(v.items()):
                print("    %-34s per_dispatch=%16.1f  (instances=%d, dispatches=%d)"
                      % (cn, d["per_dispatch"], d["instances"], d["dispatches"]))
    else:
        traffic(a)


if __name__ == "__main__":
    sys.exit(main())
