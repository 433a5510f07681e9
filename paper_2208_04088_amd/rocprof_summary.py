"""Summaries of rocprofv3 result databases (SQLite, rocpd schema) for the
step kernel: per-kernel dispatch durations, and the HBM traffic per launch
from FETCH_SIZE and WRITE_SIZE counter runs, each calibrated against the
plain copy kernel of known size that the same run launches.

    python -m paper_2208_04088_amd.rocprof_summary trace RESULTS.db
    python -m paper_2208_04088_amd.rocprof_summary traffic --fetch F.db --write W.db \\
        --kernel "k_step<float, false, false>" --copy-bytes 2147483648 \\
        --workload NAME --precision fp32 --rows 6 --strip 62 --out profiles/traffic_NAME_fp32.json

The counters report KiB per dispatch.  On this part FETCH_SIZE counts half
and WRITE_SIZE all of the bytes a streaming copy moves, so each is scaled by
the copy's reading: bytes = counter * (copy bytes / copy counter).
"""
import argparse
import collections
import json
import os
import sqlite3
import statistics


def kernel_durations(db):
    """{kernel name: [durations in ns]} over all dispatches."""
    c = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, dur in c.execute("select name, duration from kernels"):
        out[name].append(dur)
    return out


def counter_values(db):
    """{(kernel name, counter): [values per dispatch]}."""
    c = sqlite3.connect(db)
    out = collections.defaultdict(list)
    for name, cn, v in c.execute("select name, counter_name, counter_value from pmc_events"):
        out[(name, cn)].append(v)
    return out


def _pick(names, key):
    hits = [n for n in names if key in n]
    if len(hits) != 1:
        raise SystemExit(f"kernel '{key}' matches {len(hits)} names: {hits}")
    return hits[0]


def short_name(name):
    """Kernel name without its parameter list."""
    if not name.endswith(")"):
        return name
    depth = 0
    for i in range(len(name) - 1, -1, -1):
        depth += {")": 1, "(": -1}.get(name[i], 0)
        if depth == 0:
            return name[:i]
    return name


def trace_table(db):
    rows = []
    for name, d in sorted(kernel_durations(db).items(), key=lambda kv: -sum(kv[1])):
        rows.append((short_name(name), len(d), sum(d) / len(d) / 1e3, statistics.median(d) / 1e3,
                     min(d) / 1e3, max(d) / 1e3))
    return rows


def traffic(fetch_db, write_db, kernel, copy_kernel, copy_bytes):
    f, w = counter_values(fetch_db), counter_values(write_db)
    fk = _pick({n for n, _ in f}, kernel)
    wk = _pick({n for n, _ in w}, kernel)
    fc = _pick({n for n, _ in f}, copy_kernel)
    wc = _pick({n for n, _ in w}, copy_kernel)
    fetch_factor = copy_bytes / 1024 / statistics.mean(f[(fc, "FETCH_SIZE")])
    write_factor = copy_bytes / 1024 / statistics.mean(w[(wc, "WRITE_SIZE")])
    fetch_kib = statistics.mean(f[(fk, "FETCH_SIZE")])
    write_kib = statistics.mean(w[(wk, "WRITE_SIZE")])
    return {
        "fetch_kib": round(fetch_kib, 1), "write_kib": round(write_kib, 1),
        "dispatches": [len(f[(fk, "FETCH_SIZE")]), len(w[(wk, "WRITE_SIZE")])],
        "fetch_factor": round(fetch_factor, 4), "write_factor": round(write_factor, 4),
        "traffic_bytes_per_launch": round(1024 * (fetch_kib * fetch_factor + write_kib * write_factor)),
    }


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    q = sub.add_parser("traffic")
    q.add_argument("--fetch", required=True)
    q.add_argument("--write", required=True)
    q.add_argument("--kernel", required=True)
    q.add_argument("--copy-kernel", default="k_copy16")
    q.add_argument("--copy-bytes", type=int, required=True)
    q.add_argument("--workload", required=True)
    q.add_argument("--precision", required=True)
    q.add_argument("--rows", type=int, required=True)
    q.add_argument("--strip", type=int, required=True)
    q.add_argument("--out", required=True)
    q.add_argument("--source", default="step_kernel.h", help="kernel source the fingerprint covers")
    q.add_argument("--key", default=None, help="entry name (default: <rows>x<strip>)")
    a = ap.parse_args()
    if a.cmd == "trace":
        print(f"{'kernel':<58} {'calls':>6} {'avg us':>9} {'median':>9} {'min':>9} {'max':>9}")
        for r in trace_table(a.db):
            print(f"{r[0][-58:]:<58} {r[1]:>6} {r[2]:>9.2f} {r[3]:>9.2f} {r[4]:>9.2f} {r[5]:>9.2f}")
        return
    from paper_2208_04088_amd.build import kernel_fingerprint
    d = {}
    if os.path.exists(a.out):
        with open(a.out) as fh:
            d = json.load(fh)
    fp = kernel_fingerprint(a.source)
    if d.get("kernel_fingerprint") != fp:
        d = {}
    d.update({"kernel_fingerprint": fp, "workload": a.workload, "precision": a.precision,
              "copy_kernel": a.copy_kernel, "copy_bytes": a.copy_bytes})
    t = traffic(a.fetch, a.write, a.kernel, a.copy_kernel, a.copy_bytes)
    t["kernel"] = a.kernel
    key = a.key or f"{a.rows}x{a.strip}"
    d.setdefault("shapes", {})[key] = t
    with open(a.out, "w") as fh:
        json.dump(d, fh, indent=1)
    print(json.dumps(d["shapes"][key]))


if __name__ == "__main__":
    main()
