"""Summaries of rocprofv3 CSV output for the kernels of this library.

  python -m paper_1801_02417_amd.profile_summary stats  <kernel_stats.csv>
      per kernel: dispatches, average / min / max duration (us), share of GPU time
  python -m paper_1801_02417_amd.profile_summary pmc    <counter_collection.csv> [...]
      per kernel: dispatches and the mean of every collected counter per dispatch
  python -m paper_1801_02417_amd.profile_summary traffic --fetch F.csv --write W.csv
         --cal-fetch CF.csv --cal-write CW.csv --out traffic.json
      HBM bytes per launch of each pass's kernel of the 256^2 / 2e5-visibility iteration:
      FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by what the same counters read for
      a plain device copy of known size (bench.py --calibrate-copy), stored with the SHA-256 of
      the kernel's source file so that a later change of the kernel invalidates the figure.
  python -m paper_1801_02417_amd.profile_summary bandwidth --trace kernel_trace.csv --fetch F.csv
         --write W.csv --cal-fetch CF.csv --cal-write CW.csv [--min-dispatches 8]
      per kernel, over the dispatches of its most frequent grid size (the launches of the
      profiled form rather than set-up work): average duration from the kernel trace, HBM bytes
      from the scaled counters, and the achieved HBM bandwidth as a share of 8 TB/s.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 256 << 20          # bench.py --calibrate-copy moves 64 Mi floats each way

# pass id (as in psara_profile_passes) -> (kernel name prefix, source file)
PASS_KERNELS = {
    0: ("void psara::fft_pass_kernel<float, 512, 0, 0>", "kernels_fft.hip"),
    4: ("void psara::fft_pass_kernel<float, 512, 1, -1>", "kernels_fft.hip"),
    5: ("void psara::degrid_kernel<float, 0, 8>", "kernels_grid.hip"),
    6: ("void psara::grid_kernel<float, 0, 8>", "kernels_grid.hip"),
    7: ("void psara::fft_pass_kernel<float, 512, 2, -1>", "kernels_fft.hip"),
    8: ("void psara::fft_pass_kernel<float, 512, 3, -1>", "kernels_fft.hip"),
    9: ("void psara::fft_pass_kernel<float, 512, 4, 0>", "kernels_fft.hip"),
    10: ("void psara::degrid_grid_kernel<float, 0, 8>", "kernels_grid.hip"),
}


def short(name: str) -> str:
    return name.split("(")[0]


def stats(path: str) -> None:
    rows = list(csv.DictReader(open(path)))
    print(f"| kernel | dispatches | avg us | min us | max us | % time |")
    print(f"|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
              f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")


def pmc_means(paths) -> dict:
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in paths:
        for r in csv.DictReader(open(p)):
            agg[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return {k: {c: (sum(v) / len(v), len(v)) for c, v in d.items()} for k, d in agg.items()}


def pmc(paths) -> None:
    m = pmc_means(paths)
    counters = sorted({c for d in m.values() for c in d})
    print("| kernel | dispatches | " + " | ".join(counters) + " |")
    print("|---|---|" + "---|" * len(counters))
    for k in sorted(m):
        n = max(v[1] for v in m[k].values())
        print(f"| {short(k)} | {n} | " + " | ".join(f"{m[k][c][0]:.6g}" if c in m[k] else "-" for c in counters) + " |")


def _counter(means: dict, prefix: str, counter: str) -> float:
    for k, d in means.items():
        if k.startswith(prefix) and counter in d:
            return d[counter][0]
    raise KeyError(f"{counter} of {prefix} not found")


def traffic(a) -> None:
    fetch, write = pmc_means([a.fetch]), pmc_means([a.write])
    cf, cw = pmc_means([a.cal_fetch]), pmc_means([a.cal_write])
    copy = "__amd_rocclr_copyBuffer"
    f_scale = COPY_BYTES / (_counter(cf, copy, "FETCH_SIZE") * 1024.0)
    w_scale = COPY_BYTES / (_counter(cw, copy, "WRITE_SIZE") * 1024.0)
    out = {"workload": "256x256x4 Stokes, 2e5 visibilities, FP32", "fetch_scale": f_scale, "write_scale": w_scale,
           "passes": {}}
    for pid, (prefix, src) in PASS_KERNELS.items():
        fb = _counter(fetch, prefix, "FETCH_SIZE") * 1024.0 * f_scale
        wb = _counter(write, prefix, "WRITE_SIZE") * 1024.0 * w_scale
        with open(os.path.join(HERE, "csrc", src), "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
        out["passes"][str(pid)] = {"kernel": prefix, "fetch_bytes": round(fb), "write_bytes": round(wb),
                                   "hbm_bytes_per_launch": round(fb + wb), "source": src, "source_sha256": sha}
    with open(a.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


HBM_PEAK_GBS = 8000.0


def _grid(r: dict) -> int:
    if "Grid_Size" in r:
        return int(r["Grid_Size"])
    return int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y", 1) or 1) * int(r.get("Grid_Size_Z", 1) or 1)


def _per_launch_counter(path: str, counter: str) -> dict:
    """(kernel, grid size) -> mean counter value per dispatch."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[(r["Kernel_Name"], _grid(r))].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in agg.items()}


def bandwidth(a) -> None:
    dur = collections.defaultdict(list)
    for r in csv.DictReader(open(a.trace)):
        dur[(r["Kernel_Name"], _grid(r))].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    fetch = _per_launch_counter(a.fetch, "FETCH_SIZE")
    write = _per_launch_counter(a.write, "WRITE_SIZE")
    cf, cw = pmc_means([a.cal_fetch]), pmc_means([a.cal_write])
    copy = "__amd_rocclr_copyBuffer"
    f_scale = COPY_BYTES / (_counter(cf, copy, "FETCH_SIZE") * 1024.0)
    w_scale = COPY_BYTES / (_counter(cw, copy, "WRITE_SIZE") * 1024.0)
    best = {}
    for (k, g), v in dur.items():
        if len(v) >= a.min_dispatches and (k not in best or len(v) > len(dur[(k, best[k])])):
            best[k] = g
    rows = []
    for k, g in best.items():
        d = dur[(k, g)]
        us = sum(d) / len(d) / 1e3
        fb = fetch.get((k, g), float("nan")) * 1024.0 * f_scale
        wb = write.get((k, g), float("nan")) * 1024.0 * w_scale
        gbs = (fb + wb) / (us * 1e-6) / 1e9
        rows.append((sum(d), short(k), g, len(d), us, fb / 1e6, wb / 1e6, gbs))
    rows.sort(reverse=True)
    print(f"FETCH_SIZE scaled by {f_scale:.4f}, WRITE_SIZE by {w_scale:.4f} (plain-copy calibration)\n")
    print("| kernel | grid (threads) | dispatches | avg us | fetch MB | write MB | HBM GB/s | % of 8 TB/s |")
    print("|---|---|---|---|---|---|---|---|")
    for _, k, g, nd, us, f, w, gbs in rows:
        print(f"| {k} | {g} | {nd} | {us:.2f} | {f:.2f} | {w:.2f} | {gbs:.0f} | {100 * gbs / HBM_PEAK_GBS:.1f} |")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    p = sub.add_parser("pmc")
    p.add_argument("csv", nargs="+")
    t = sub.add_parser("traffic")
    for name in ("--fetch", "--write", "--cal-fetch", "--cal-write", "--out"):
        t.add_argument(name, required=True)
    b = sub.add_parser("bandwidth")
    for name in ("--trace", "--fetch", "--write", "--cal-fetch", "--cal-write"):
        b.add_argument(name, required=True)
    b.add_argument("--min-dispatches", type=int, default=8)
    a = ap.parse_args()
    if a.cmd == "bandwidth":
        bandwidth(a)
    elif a.cmd == "stats":
        stats(a.csv)
    elif a.cmd == "pmc":
        pmc(a.csv)
    else:
        traffic(a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
