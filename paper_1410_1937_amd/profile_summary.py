"""Summaries of rocprofv3 databases (rocpd SQLite) written by profile_run or
bench.py runs, as the text tables kept under profiles/.

    python3 -m paper_1410_1937_amd.profile_summary trace DB [PATTERN]
        per kernel: dispatches, mean and median duration (us), total (ms);
        the CG sweeps and the network's convolutions also get the median
        over full launches (> 20 us): launches queued past the solver's
        stopping point return at once
    python3 -m paper_1410_1937_amd.profile_summary pmc DB [PATTERN]
        per kernel: mean per dispatch of every collected counter
    python3 -m paper_1410_1937_amd.profile_summary traffic FETCH_DB WRITE_DB [PATTERN]
        HBM bytes per launch: FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
        median over full sweeps) each scaled by what that counter reads for
        the calibration copies (the three largest k_stream_copy dispatches,
        of --copy-mib MiB each: profile_run's default, 1024)

Names are shortened (namespaces and argument lists dropped).
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3
import statistics
import sys


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("nfa::", "")
    if name.startswith("void "):
        name = name[5:]
    return name.split("(", 1)[0] if name.startswith("k_") else name[:60]


def _is_sweep(name: str) -> bool:
    """Kernels that return at once when the solver state says done (launches
    queued past the stopping point), so that only longer launches are full."""
    return name.startswith(("k_cg_a", "k_cg_b", "k_tconv"))


def trace(db: str, pat: str | None):
    c = sqlite3.connect(db)
    agg = collections.defaultdict(list)
    for n, d in c.execute("select name, duration from kernels"):
        n = _short(n)
        if pat and not re.search(pat, n):
            continue
        agg[n].append(d / 1000.0)
    print("| kernel | dispatches | mean (us) | median (us) | median of full sweeps (us) | total (ms) |")
    print("|---|---|---|---|---|---|")
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        full = [x for x in v if x > 20.0] if _is_sweep(n) else []
        fm = f"{statistics.median(full):.1f}" if full else ""
        print(f"| `{n}` | {len(v)} | {sum(v) / len(v):.1f} | {statistics.median(v):.1f} | {fm} | {sum(v) / 1000:.2f} |")


def _counters(db: str, pat: str | None):
    c = sqlite3.connect(db)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for kn, d, cn, v in c.execute("select kernel_name, dispatch_id, counter_name, value from counters_collection"):
        kn = _short(kn)
        if pat and not re.search(pat, kn) and kn != "k_stream_copy":
            continue
        per[(kn, d)][cn] += v
        disp[kn].add(d)
    return per, disp


def pmc(db: str, pat: str | None):
    per, disp = _counters(db, pat)
    names = sorted({cn for cs in per.values() for cn in cs})
    print("| kernel | dispatches | " + " | ".join(names) + " |")
    print("|---|---|" + "---|" * len(names))
    for kn in sorted(disp):
        ds = sorted(disp[kn])
        means = [sum(per[(kn, d)].get(cn, 0.0) for d in ds) / len(ds) for cn in names]
        print(f"| `{kn}` | {len(ds)} | " + " | ".join(f"{m:.4g}" for m in means) + " |")


def _per_dispatch(db: str, counter: str, pat: str | None):
    per, disp = _counters(db, pat)
    return {kn: [per[(kn, d)].get(counter, 0.0) for d in sorted(ds)] for kn, ds in disp.items()}


def traffic(fetch_db: str, write_db: str, pat: str | None, copy_mib: int):
    f = _per_dispatch(fetch_db, "FETCH_SIZE", pat)
    w = _per_dispatch(write_db, "WRITE_SIZE", pat)
    copy_kib = copy_mib * 1024.0
    cf = sorted(f.get("k_stream_copy", []))[-3:]
    cw = sorted(w.get("k_stream_copy", []))[-3:]
    if not cf or not cw:
        sys.exit("no k_stream_copy dispatches to calibrate with")
    ff, fw = copy_kib / statistics.median(cf), copy_kib / statistics.median(cw)
    print(f"Calibration: k_stream_copy of {copy_mib} MiB: FETCH_SIZE reads {statistics.median(cf):.0f} KiB "
          f"(factor {ff:.4f}), WRITE_SIZE {statistics.median(cw):.0f} KiB (factor {fw:.4f}).\n")
    print("| kernel | dispatches | FETCH KiB (raw, median) | WRITE KiB (raw, median) | fetched bytes | written bytes "
          "| traffic bytes |")
    print("|---|---|---|---|---|---|---|")
    lines = []
    for kn in sorted(set(f) & set(w)):
        if kn == "k_stream_copy":
            continue
        fv, wv = f[kn], w[kn]
        if _is_sweep(kn):   # full sweeps only (early exits read almost nothing)
            top = max(fv)
            fv = [x for x in fv if x > 0.2 * top]
            topw = max(wv)
            wv = [x for x in wv if x > 0.2 * topw]
        fm, wm = statistics.median(fv), statistics.median(wv)
        fb, wb = fm * 1024 * ff, wm * 1024 * fw
        print(f"| `{kn}` | {len(f[kn])} | {fm:.0f} | {wm:.0f} | {fb:.4g} | {wb:.4g} | {fb + wb:.4g} |")
        lines.append(f"traffic_bytes_per_launch {kn}: {fb + wb:.0f}")
    print()
    for ln in lines:
        print(ln)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=("trace", "pmc", "traffic"))
    ap.add_argument("db")
    ap.add_argument("rest", nargs="*")
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    if a.mode == "trace":
        trace(a.db, a.rest[0] if a.rest else None)
    elif a.mode == "pmc":
        pmc(a.db, a.rest[0] if a.rest else None)
    else:
        if not a.rest:
            sys.exit("traffic needs FETCH_DB WRITE_DB")
        traffic(a.db, a.rest[0], a.rest[1] if len(a.rest) > 1 else None, a.copy_mib)
    return 0


if __name__ == "__main__":
    sys.exit(main())
