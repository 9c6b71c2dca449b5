"""Helpers to read rocprofv3 result databases (kernel durations, counters).

Used to summarize runs of ``rocprofv3 --kernel-trace --stats`` and
``rocprofv3 --pmc ...`` into the short text summaries kept with the project.
"""
import glob
import hashlib
import os
import sqlite3

HERE = os.path.dirname(os.path.abspath(__file__))


def _db(path):
    if os.path.isdir(path):
        dbs = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
        if not dbs:
            raise FileNotFoundError("no rocprofv3 database under %s" % path)
        path = dbs[0]
    return sqlite3.connect(path)


def kernel_stats(path):
    """[(name, launches, avg_us, min_us, max_us, total_us)] sorted by total time."""
    c = _db(path)
    q = ("select name, count(*), avg(end-start), min(end-start), max(end-start), sum(end-start) "
         "from kernels group by name order by sum(end-start) desc")
    return [(r[0], r[1], r[2] / 1e3, r[3] / 1e3, r[4] / 1e3, r[5] / 1e3) for r in c.execute(q)]


def counter_values(path):
    """{(kernel_name, counter): [value per dispatch]}"""
    c = _db(path)
    out = {}
    q = "select kernel_name, counter_name, dispatch_id, sum(value) from counters_collection " \
        "group by kernel_name, counter_name, dispatch_id order by dispatch_id"
    for name, ctr, _, v in c.execute(q):
        out.setdefault((name, ctr), []).append(v)
    return out


def source_hash(files):
    """sha256 over the given source files (relative to the package csrc/)."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _avg_for(values, substr):
    """Average per-dispatch value over the kernels whose name contains substr."""
    rows = [v for (name, _), vs in values.items() if substr in name for v in vs]
    return sum(rows) / len(rows) if rows else None


def traffic_record(kernel_substr, fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes,
                   sources, algorithmic_bytes, label):
    """HBM bytes per launch of a kernel from FETCH_SIZE / WRITE_SIZE runs (KiB
    per dispatch), each scaled by what the same counter reads for a plain copy
    of copy_bytes in each direction."""
    fetch = _avg_for(counter_values(fetch_dir), kernel_substr)
    write = _avg_for(counter_values(write_dir), kernel_substr)
    cf = max(v for vs in counter_values(copy_fetch_dir).values() for v in vs)
    cw = max(v for vs in counter_values(copy_write_dir).values() for v in vs)
    fs = copy_bytes / (cf * 1024.0)
    ws = copy_bytes / (cw * 1024.0)
    return {"kernel": label, "source_sha256": source_hash(sources),
            "fetch_kib_per_launch": fetch, "write_kib_per_launch": write,
            "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes_each_way": copy_bytes,
            "fetch_scale": fs, "write_scale": ws,
            "traffic_bytes_per_launch": fetch * 1024.0 * fs + write * 1024.0 * ws,
            "algorithmic_bytes_per_launch": algorithmic_bytes}


def stats_markdown(path, top=12):
    lines = ["| kernel | launches | avg us | min us | max us | total us |", "|---|---|---|---|---|---|"]
    for name, n, avg, mn, mx, tot in kernel_stats(path)[:top]:
        short = name if len(name) <= 90 else name[:87] + "..."
        lines.append("| %s | %d | %.1f | %.1f | %.1f | %.1f |" % (short.replace("|", "/"), n, avg, mn, mx, tot))
    return "\n".join(lines)


def counters_markdown(dirs, kernels):
    """Average per-dispatch value of every counter in the runs under dirs,
    for each kernel whose name contains one of the substrings."""
    lines = ["| kernel | counter | avg per dispatch | dispatches |", "|---|---|---|---|"]
    merged = {}
    for d in dirs:
        for key, vs in counter_values(d).items():
            merged.setdefault(key, []).extend(vs)
    for sub in kernels:
        for (name, ctr), vs in sorted(merged.items(), key=lambda kv: (kv[0][1], kv[0][0])):
            if sub in name:
                short = sub
                lines.append("| %s | %s | %.4g | %d |" % (short, ctr, sum(vs) / len(vs), len(vs)))
    return "\n".join(lines)


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="summarise rocprofv3 result databases")
    sub = ap.add_subparsers(dest="cmd", required=True)
    st = sub.add_parser("stats", help="markdown table of kernel durations")
    st.add_argument("dir")
    st.add_argument("--top", type=int, default=12)
    tr = sub.add_parser("traffic", help="HBM bytes per launch of one kernel (JSON)")
    tr.add_argument("--kernel", required=True, help="substring of the kernel name")
    tr.add_argument("--label", required=True)
    tr.add_argument("--fetch", required=True)
    tr.add_argument("--write", required=True)
    tr.add_argument("--copy-fetch", required=True)
    tr.add_argument("--copy-write", required=True)
    tr.add_argument("--copy-bytes", type=int, default=1 << 29)
    tr.add_argument("--sources", nargs="+", required=True)
    tr.add_argument("--alg-bytes", type=float, required=True)
    ct = sub.add_parser("counters", help="markdown table of counter averages per kernel")
    ct.add_argument("dirs", nargs="+")
    ct.add_argument("--kernel", action="append", required=True, help="substring of a kernel name")
    a = ap.parse_args(argv)
    if a.cmd == "stats":
        print(stats_markdown(a.dir, a.top))
    elif a.cmd == "counters":
        print(counters_markdown(a.dirs, a.kernel))
    else:
        rec = traffic_record(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes,
                             a.sources, a.alg_bytes, a.label)
        print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
