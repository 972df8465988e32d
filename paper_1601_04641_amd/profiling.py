"""Summaries of rocprofv3 output for the SSCN sweeps.

* ``traffic``: HBM bytes per launch of the timed real-time sweeps of a bench.py run, from
  two counter runs of the same command (``rocprofv3 --pmc FETCH_SIZE`` and
  ``rocprofv3 --pmc WRITE_SIZE``, CSV output).  Both counters are scaled by what they read
  for a plain device copy of a known size (by default the runtime's copy kernel, which
  bench.py's bandwidth probe runs on 1 GiB through torch), so the result is in bytes.
  Writes the JSON that bench.py reports as ``roofline.traffic`` when the mapping matches.
* ``stats``: a markdown table of a ``--kernel-trace --stats`` summary, with algorithmic
  GB/s for the sweep kernels of one grid (one read and one write of psi per launch).
* ``counters``: the mean per dispatch of every counter of one or more ``--pmc`` runs, per
  sweep kernel.

    python -m paper_1601_04641_amd.profiling traffic --fetch F.csv --write W.csv \\
        --bench B.json --out profiles/traffic.json
    python -m paper_1601_04641_amd.profiling stats --stats S_kernel_stats.csv --points N
"""
from __future__ import annotations

import argparse
import csv
import json
import re
import sys
from collections import defaultdict

_KERNEL = re.compile(r"gpk::(k_sweep_lines|k_sweep_z|k_stream_lines|k_stream_yz)<(float|double), ([^>]*)>")


def classify(name: str):
    """(kind, precision, complex_coefficients) of a single-grid sweep kernel, else None.
    kind: x_sweep (a line sweep that applies the potential step), y_sweep, z_sweep, yz_fused;
    precision: c64 (float) / c128 (double); complex coefficients = real time."""
    m = _KERNEL.search(name)
    if not m:
        return None
    fam, real, rest = m.group(1), m.group(2), [a.strip() for a in m.group(3).split(",")]
    prec = "c64" if real == "float" else "c128"
    if fam == "k_sweep_lines":      # <R, M, SW, CC, NSTEP, WIDE, MAXW>
        return ("x_sweep" if int(rest[3]) != 0 else "y_sweep"), prec, rest[2] == "true"
    if fam == "k_stream_lines":     # <R, H, CC, NSTEP>
        return ("x_sweep" if int(rest[2]) != 0 else "y_sweep"), prec, rest[1] == "true"
    if fam == "k_sweep_z":          # <R, MZ, CC, NORM, EPI>
        return "z_sweep", prec, rest[1] == "true"
    return "yz_fused", prec, rest[2] == "true"   # k_stream_yz<R, H, MZ, CC, ...>


def in_mapping(name: str, mapping) -> bool:
    """Whether an exact-sweep kernel is the one a context with this line mapping
    [m_x, sw_x, m_y, sw_y, segments_z, m_z] launches."""
    m = _KERNEL.search(name)
    if not m:
        return False
    fam, rest = m.group(1), [a.strip() for a in m.group(3).split(",")]
    if fam == "k_sweep_lines":
        want = mapping[0:2] if int(rest[3]) != 0 else mapping[2:4]
        return [int(rest[0]), int(rest[1])] == list(want)
    if fam == "k_sweep_z":
        return int(rest[0]) == mapping[5]
    return False


def read_counter(path: str, counter: str):
    """{kernel name: [values per dispatch]} of one counter from a counter_collection CSV."""
    out = defaultdict(list)
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                out[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return out


def traffic(fetch_csv: str, write_csv: str, bench_json: str, copy_bytes: int = 1 << 30,
            calib_kernel: str = "__amd_rocclr_copyBuffer"):
    """Traffic per launch of the timed sweeps.  Calibration: the dispatches of `calib_kernel`
    (a name prefix) that move about `copy_bytes` (counter values above a quarter of that
    size in KiB; the runtime's device copy serves small transfers too)."""
    fetch = read_counter(fetch_csv, "FETCH_SIZE")
    write = read_counter(write_csv, "WRITE_SIZE")
    big = copy_bytes / 1024 / 4
    copies = [k for k in fetch if k.startswith(calib_kernel)]
    f_copy = [v for k in copies for v in fetch[k] if v > big]
    w_copy = [v for k in copies for v in write.get(k, []) if v > big]
    if not f_copy or not w_copy:
        raise SystemExit(f"no {calib_kernel} dispatch of {copy_bytes} bytes in the counter runs")
    f_kib, w_kib = sum(f_copy) / len(f_copy), sum(w_copy) / len(w_copy)
    fs, ws = copy_bytes / (f_kib * 1024), copy_bytes / (w_kib * 1024)
    line = None
    with open(bench_json) as f:
        for ln in f:
            ln = ln.strip()
            if ln.startswith("{"):
                line = json.loads(ln)
    if line is None:
        raise SystemExit(f"no JSON line in {bench_json}")
    nx, ny, nz = line["config"]["grid"]
    npts = nx * ny * nz
    maps = {"c128" if line["dtype"] == "f64" else "c64": line["config"]["mapping"]}
    if "precision_form" in line:
        maps["c64"] = line["precision_form"]["mapping"]
    if "complex128" in line:
        maps["c128"] = line["complex128"]["mapping"]
    out = {"workload": line["config"]["workload"], "grid": [nx, ny, nz],
           "calibration": {"kernel": calib_kernel, "dispatches": len(f_copy), "bytes_read": copy_bytes,
                           "bytes_written": copy_bytes, "FETCH_SIZE_KiB": f_kib, "WRITE_SIZE_KiB": w_kib,
                           "fetch_scale": fs, "write_scale": ws}}
    for prec, mapping in maps.items():
        esz = 8 if prec == "c64" else 16
        alg = 2 * esz * npts
        entry = {"mapping": mapping, "algorithmic_bytes": alg, "detail": {}}
        for name in fetch:
            c = classify(name)
            if c is None or c[1] != prec or not c[2] or name not in write:
                continue
            kind = c[0]
            fk = sum(fetch[name]) / len(fetch[name])
            wk = sum(write[name]) / len(write[name])
            rb, wb = fk * 1024 * fs, wk * 1024 * ws
            d = {"kernel": name.split("(")[0].replace("void ", ""), "dispatches": len(fetch[name]),
                 "FETCH_SIZE_KiB": fk, "WRITE_SIZE_KiB": wk, "read_bytes": rb,
                 "write_bytes": wb, "traffic_over_algorithmic": (rb + wb) / alg}
            if in_mapping(name, mapping):
                entry[kind] = rb + wb
                entry["detail"][kind] = d
            else:   # another mapping or the halo-truncated kernels
                entry.setdefault("other", []).append(d)
        out[prec] = entry
    return out


def counter_table(csvs, kernels=None):
    """Markdown table of the mean value per dispatch of every counter in the given
    counter_collection CSVs, one row per sweep kernel (or per kernel whose name contains
    one of `kernels`)."""
    vals = defaultdict(lambda: defaultdict(list))
    for path in csvs:
        with open(path, newline="") as f:
            for row in csv.DictReader(f):
                vals[row["Kernel_Name"]][row["Counter_Name"]].append(float(row["Counter_Value"]))
    names = sorted({c for d in vals.values() for c in d})
    lines = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for k in sorted(vals):
        keep = classify(k) is not None if kernels is None else any(s in k for s in kernels)
        if not keep:
            continue
        d = vals[k]
        n = max(len(v) for v in d.values())
        cells = [f"{sum(d[c]) / len(d[c]):.4g}" if d.get(c) else "" for c in names]
        lines.append(f"| `{k.split('(')[0].replace('void ', '')}` | {n} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names[0])


def stats_table(stats_csv: str, points: int = 0, top: int = 30):
    """Markdown table of the `top` kernels by total time; algorithmic GB/s for sweep kernels
    when `points` (the grid's point count) is given."""
    rows = []
    with open(stats_csv, newline="") as f:
        for r in csv.DictReader(f):
            rows.append((_col(r, "Name", "KERNEL_NAME"), int(_col(r, "Calls", "CALLS")),
                         float(_col(r, "TotalDurationNs", "TOTAL_DURATION")),
                         float(_col(r, "AverageNs", "AVERAGE")), float(_col(r, "Percentage", "PERCENTAGE"))))
    rows.sort(key=lambda t: -t[2])
    lines = ["| kernel | calls | average us | share | algorithmic GB/s |", "|---|---|---|---|---|"]
    for name, calls, _tot, avg, pct in rows[:top]:
        short = name.split("(")[0].replace("void ", "")
        gbps = ""
        c = classify(name)
        if points and c is not None and c[0] != "yz_fused":
            gbps = f"{2 * (8 if c[1] == 'c64' else 16) * points / (avg * 1e-9) / 1e9:.0f}"
        lines.append(f"| `{short}` | {calls} | {avg / 1e3:.1f} | {pct:.1f}% | {gbps} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--bench", required=True, help="the stdout of one of the two bench.py runs")
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--calib-kernel", default="__amd_rocclr_copyBuffer",
                   help="name prefix of the copy kernel whose dispatches of --copy-bytes calibrate the counters")
    t.add_argument("--out", default=None)
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+", help="counter_collection CSVs of one or more --pmc runs")
    c.add_argument("--kernels", nargs="*", default=None, help="name fragments to keep (default: the sweeps)")
    s = sub.add_parser("stats")
    s.add_argument("--stats", required=True)
    s.add_argument("--points", type=int, default=0)
    s.add_argument("--top", type=int, default=30)
    a = ap.parse_args(argv)
    if a.cmd == "traffic":
        res = traffic(a.fetch, a.write, a.bench, a.copy_bytes, a.calib_kernel)
        text = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)
    elif a.cmd == "counters":
        print(counter_table(a.csv, a.kernels))
    else:
        print(stats_table(a.stats, a.points, a.top))


if __name__ == "__main__":
    sys.exit(main())
