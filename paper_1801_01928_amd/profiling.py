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
