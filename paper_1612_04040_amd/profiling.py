"""Summaries of rocprofv3 results (measurement support, not part of the method).

``python -m paper_1612_04040_amd.profiling trace DB...`` prints per-kernel
dispatch counts and mean durations from rocprofv3 ``--kernel-trace`` result
databases; ``counters DB...`` prints per-kernel mean counter values from
``--pmc`` runs.  ``traffic`` combines a FETCH_SIZE and a WRITE_SIZE run into
HBM bytes per dispatch, each counter scaled by what it reads for the plain
dword copy kernel (``ls::copy_f32_kernel``, 1 GiB read and 1 GiB written in
the bench's calibration pass), and records them in profiles/traffic.json
under the kernel source digest they were taken on.
"""
import argparse
import collections
import json
import os
import re
import sqlite3
import sys

CALIB_KERNEL = "ls::copy_f32_kernel"
CALIB_BYTES = 1 << 30
CALIB_DISPATCHES = 3  # the calibration pass: the last three copy dispatches of the run


def _rows(db, query):
    con = sqlite3.connect(db)
    try:
        return con.execute(query).fetchall()
    finally:
        con.close()


def short_name(k):
    k = k.replace("void ", "")
    return k.split("(")[0]


def kernel_durations(db):
    """{kernel: (dispatches, mean duration in us)} from a kernel-trace database."""
    rows = _rows(db, "select name, start, end from kernels")
    acc = collections.defaultdict(list)
    for name, start, end in rows:
        acc[short_name(name)].append((end - start) / 1e3)
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def kernel_counters(db):
    """{(kernel, counter): (dispatches, mean value)} from a --pmc database."""
    rows = _rows(db, "select kernel_name, counter_name, value from counters_collection")
    acc = collections.defaultdict(list)
    for k, c, v in rows:
        acc[(short_name(k), c)].append(v)
    return {key: (len(v), sum(v) / len(v)) for key, v in acc.items()}


def _mean_over(counters, prefix, name):
    """Dispatch-weighted mean of counter `name` over the kernels whose names
    match the regular expression `prefix` at their start (a plain name
    prefix is such an expression)."""
    n = tot = 0.0
    for (k, c), (d, v) in counters.items():
        if c == name and re.match(prefix, k):
            n += d
            tot += d * v
    if n == 0:
        raise KeyError(f"no {name} samples for kernels starting with {prefix}")
    return tot / n, int(n)


def _calibration(db, counter):
    """Mean counter value (KiB) of the calibration copies: the last
    CALIB_DISPATCHES dispatches of the copy kernel (a run may use the same
    kernel earlier for copies of other sizes)."""
    rows = _rows(db, "select dispatch_id, kernel_name, counter_name, value "
                     "from counters_collection")
    vals = [v for d, k, c, v in sorted(rows)
            if c == counter and short_name(k).startswith(CALIB_KERNEL)]
    if len(vals) < CALIB_DISPATCHES:
        raise KeyError(f"fewer than {CALIB_DISPATCHES} {CALIB_KERNEL} samples of {counter}")
    return sum(vals[-CALIB_DISPATCHES:]) / CALIB_DISPATCHES


def traffic(fetch_db, write_db, prefix):
    """HBM bytes per dispatch of the kernels matching `prefix` at the start of
    their names (all their variants together), calibrated by the copy kernel."""
    f = kernel_counters(fetch_db)
    w = kernel_counters(write_db)
    f_cal = _calibration(fetch_db, "FETCH_SIZE") * 1024.0
    w_cal = _calibration(write_db, "WRITE_SIZE") * 1024.0
    rf, wf = CALIB_BYTES / f_cal, CALIB_BYTES / w_cal
    fm, nf = _mean_over(f, prefix, "FETCH_SIZE")
    wm, nw = _mean_over(w, prefix, "WRITE_SIZE")
    fk, wk = fm * 1024.0 * rf, wm * 1024.0 * wf
    return {"read_bytes": fk, "write_bytes": wk, "bytes_per_launch": fk + wk,
            "fetch_scale": rf, "write_scale": wf, "dispatches": [nf, nw]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db", nargs="+")
    c = sub.add_parser("counters")
    c.add_argument("db", nargs="+")
    tr = sub.add_parser("traffic")
    tr.add_argument("fetch_db")
    tr.add_argument("write_db")
    tr.add_argument("--kernel", required=True,
                    help="kernel name prefix (a regular expression matched at the start)")
    tr.add_argument("--key", required=True, help="kernel/workload key in traffic.json")
    tr.add_argument("--digest", required=True, help="kernel source digest of the run")
    tr.add_argument("--out", default=os.path.join(os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), "profiles", "traffic.json"))
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        for db in a.db:
            for k, (n, us) in sorted(kernel_durations(db).items(), key=lambda kv: -kv[1][0] * kv[1][1]):
                print(f"{k[:100]:100s} dispatches={n:6d} mean_us={us:10.3f}")
    elif a.cmd == "counters":
        for db in a.db:
            for (k, cn), (n, v) in sorted(kernel_counters(db).items()):
                print(f"{k[:100]:100s} {cn:20s} dispatches={n:6d} mean={v:16.1f}")
    else:
        names = {k for k, _ in kernel_counters(a.fetch_db)}
        match = sorted(n for n in names if re.match(a.kernel, n))
        if not match:
            print(f"no kernel starting with {a.kernel}", file=sys.stderr)
            return 1
        rec = traffic(a.fetch_db, a.write_db, a.kernel)
        rec["kernels"] = match
        rec["source_digest"] = a.digest
        data = {}
        if os.path.exists(a.out):
            with open(a.out) as fh:
                data = json.load(fh)
        data[a.key] = rec
        with open(a.out, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
