"""Summaries of rocprofv3 output for the kernels of the solve.

  python -m paper_1912_13403_amd.profiling stats DIR
      per-kernel calls / total / average duration from the *_kernel_trace.csv
      that `rocprofv3 --kernel-trace --stats --output-format csv -d DIR`
      wrote, or from the *_results.db of the default (rocpd) output format.

  python -m paper_1912_13403_amd.profiling traffic FETCH_DIR WRITE_DIR OUT.json
      mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of every kernel from two
      `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs of
      `bench.py --copy-calibration`, with the calibration factors: what each
      counter reads for the plain 2 GiB device copy that run starts with,
      divided by the bytes that copy moves.  bench.py divides a kernel's
      counters by these factors to get its HBM bytes per launch.

  python -m paper_1912_13403_amd.profiling mfma DIR [SIMDS]
      per-kernel matrix-core utilisation from one `rocprofv3 --pmc
      SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_F64 SQ_INSTS_VALU_MFMA_MOPS_F32
      GRBM_GUI_ACTIVE` run: busy = sum of SQ_VALU_MFMA_BUSY_CYCLES /
      ((GRBM_GUI_ACTIVE / 8) x SIMDS) (the graphics-active count is summed over
      the 8 XCDs; SIMDS = 1024 on the 256 compute units of the MI355X), and the
      FP64 and FP32 matrix flops the hardware executed (MOPS x 512).

  python -m paper_1912_13403_amd.profiling timeline DIR [GAP_MS]
      phases of every multi-task solve in a kernel trace (one solve per
      bt2_group_kernel launch; solves are told apart by idle gaps of the
      device longer than GAP_MS, default 2): wall time, device-busy time and
      the largest kernels from the start of the solve to its first grouped
      panel QR (factor and standard form), to the first bulge-chasing launch
      (full -> band), to the last one's end (bulge chasing), to the grouped
      stage-2 back-transform (tridiagonal eigensolver, occupations), its
      duration, and to the end (stage-1 back-transform, L^-T, density).
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

COPY_BYTES = 8 << 28  # bench.py --copy-calibration: 2^28 doubles read and written
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _find(d, pattern):
    hits = sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no {pattern} under {d}")
    return hits[0]


def _short(name):
    name = name.replace("(anonymous namespace)::", "")
    if name.startswith("void "):
        name = name[5:]
    i = name.find("(")
    return name[:i] if i > 0 else name


def _stats_db(path):
    """name -> (calls, total_ms, mean_us) from a rocpd database (the default
    output format of rocprofv3)."""
    import sqlite3
    con = sqlite3.connect(path)
    agg = {}
    q = ("select coalesce(s.display_name, s.kernel_name), d.start, d.end "
         "from rocpd_kernel_dispatch d "
         "join rocpd_info_kernel_symbol s on d.kernel_id = s.id")
    for name, t0, t1 in con.execute(q):
        a = agg.setdefault(_short(name), [0, 0.0])
        a[0] += 1
        a[1] += (t1 - t0) * 1e-6
    con.close()
    return {k: (v[0], v[1], 1e3 * v[1] / v[0]) for k, v in agg.items()}


def stats(d):
    """name -> (calls, total_ms, mean_us) from a kernel trace csv, or from the
    rocpd database when no csv was written."""
    try:
        path = _find(d, "*kernel_trace.csv")
    except FileNotFoundError:
        return _stats_db(_find(d, "*_results.db"))
    agg = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = _short(row.get("Kernel_Name", ""))
            t = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-6
            a = agg.setdefault(name, [0, 0.0])
            a[0] += 1
            a[1] += t
    return {k: (v[0], v[1], 1e3 * v[1] / v[0]) for k, v in agg.items()}


def print_stats(d, top=25):
    st = stats(d)
    tot = sum(v[1] for v in st.values())
    print(f"{'total ms':>10} {'%':>5} {'calls':>7} {'mean us':>10}  kernel")
    for k, (c, t, m) in sorted(st.items(), key=lambda kv: -kv[1][1])[:top]:
        print(f"{t:10.2f} {100 * t / tot:5.1f} {c:7d} {m:10.1f}  {k}")
    print(f"{tot:10.2f} total kernel time (ms)")


def _counter(d, counter):
    path = _find(d, "*counter_collection.csv")
    per = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            if row.get("Counter_Name") != counter:
                continue
            key = (row.get("Dispatch_Id") or row.get("Correlation_Id"), _short(row["Kernel_Name"]))
            per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    return per


def _source_sha(kernel):
    sys.path.insert(0, ROOT)
    import bench  # noqa: E402  (the same hash bench.py checks)
    return bench.kernel_source_sha(kernel)


def traffic(fetch_dir, write_dir, out_path, workload="cfg2_n16384"):
    res = {"workload": workload, "copy_bytes": COPY_BYTES, "kernels": {}}
    for counter, d, fkey in (("FETCH_SIZE", fetch_dir, "fetch"), ("WRITE_SIZE", write_dir, "write")):
        per = _counter(d, counter)
        by = {}
        for (_, name), v in per.items():
            by.setdefault(name, []).append(v)
        # the calibration copy is the torch elementwise copy with the largest reading
        copies = [v for (_, name), v in per.items() if "copy" in name.lower()]
        if not copies:
            raise RuntimeError(f"no copy kernel in the {counter} run")
        res[f"copy_factor_{fkey}"] = max(copies) * 1024.0 / COPY_BYTES
        for name, vals in by.items():
            k = res["kernels"].setdefault(name, {})
            k[f"{fkey}_kib_per_dispatch"] = sum(vals) / len(vals)
            k["dispatches"] = len(vals)
    for name, k in res["kernels"].items():
        k["source_sha1"] = _source_sha(name)
    res["kernels"] = {k: v for k, v in res["kernels"].items()
                      if "fetch_kib_per_dispatch" in v and "write_kib_per_dispatch" in v
                      and v["source_sha1"]}
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1, sort_keys=True)
    return res


def mfma(d, simds=1024, xcds=8):
    """name -> dict(dispatches, util (fraction of SIMD-cycles with the matrix
    core busy), fp64 and fp32 matrix flops per dispatch).  GRBM_GUI_ACTIVE
    is counted by each XCD's graphics block and summed over the xcds; the
    busy cycles are summed over all SIMDs."""
    busy = _counter(d, "SQ_VALU_MFMA_BUSY_CYCLES")
    gui = _counter(d, "GRBM_GUI_ACTIVE")
    mops = _counter(d, "SQ_INSTS_VALU_MFMA_MOPS_F64")
    try:
        mops32 = _counter(d, "SQ_INSTS_VALU_MFMA_MOPS_F32")
    except FileNotFoundError:
        mops32 = {}
    out = {}
    for key, b in busy.items():
        g = gui.get(key, 0.0)
        a = out.setdefault(key[1], [0, 0.0, 0.0, 0.0, 0.0])
        a[0] += 1
        a[1] += b
        a[2] += g / xcds
        a[3] += mops.get(key, 0.0) * 512.0
        a[4] += mops32.get(key, 0.0) * 512.0
    return {k: {"dispatches": v[0], "util": v[1] / (v[2] * simds) if v[2] > 0 else None,
                "fp64_mfma_flops_per_dispatch": v[3] / v[0],
                "fp32_mfma_flops_per_dispatch": v[4] / v[0]} for k, v in out.items()}


def print_mfma(d, simds=1024, top=12):
    st = mfma(d, simds)
    print(f"{'disp':>5} {'MFMA busy':>10} {'FP64 MFMA flops/disp':>22} {'FP32 MFMA flops/disp':>22}"
          f"  kernel")
    for k, v in sorted(st.items(), key=lambda kv: -(kv[1]["fp64_mfma_flops_per_dispatch"]
                                                    + kv[1]["fp32_mfma_flops_per_dispatch"])
                       * kv[1]["dispatches"])[:top]:
        u = "n/a" if v["util"] is None else f"{100 * v['util']:.1f} %"
        print(f"{v['dispatches']:5d} {u:>10} {v['fp64_mfma_flops_per_dispatch']:22.4e} "
              f"{v['fp32_mfma_flops_per_dispatch']:22.4e}  {k}")


def _busy(iv):
    tot, cs, ce = 0, None, None
    for a, b in sorted(iv):
        if cs is None or a > ce:
            if cs is not None:
                tot += ce - cs
            cs, ce = a, b
        else:
            ce = max(ce, b)
    return tot + (ce - cs if cs is not None else 0)


def timeline(d, gap_ms=2.0, top=6):
    path = _find(d, "*kernel_trace.csv")
    rows = []
    with open(path) as fh:
        for row in csv.DictReader(fh):
            rows.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]),
                         _short(row.get("Kernel_Name", ""))))
    rows.sort()
    # segments separated by idle gaps; a solve is a run of segments ending
    # with the one that holds its bt2_group_kernel
    solves, cur, end = [], [], None
    for r in rows:
        if cur and r[0] - end > gap_ms * 1e6 and any(x[2] == "bt2_group_kernel" for x in cur):
            solves.append(cur)
            cur = []
        cur.append(r)
        end = r[1] if end is None else max(end, r[1])
    if any(x[2] == "bt2_group_kernel" for x in cur):
        solves.append(cur)
    out = []
    for k, sv in enumerate(solves):
        # the solve starts at its first kernel after the previous solve's torch
        # work (input copies and the like carry no library kernel names)
        sv = [r for r in sv if not r[2].startswith(("at::", "__amd_rocclr"))]
        first = lambda nm: next(r[0] for r in sv if r[2].startswith(nm))
        lastend = lambda nm: max(r[1] for r in sv if r[2].startswith(nm))
        t0, t1 = sv[0][0], max(r[1] for r in sv)
        marks = [("start", t0), ("panel QR group", first("panel_qr_group_kernel")),
                 ("bulge chasing", first("sb2st_group_kernel")),
                 ("chasing end", lastend("sb2st_group_kernel")),
                 ("stage-2 back-transform", first("bt2_group_kernel")),
                 ("its end", lastend("bt2_group_kernel")), ("end", t1)]
        phases = []
        for (n0, x0), (n1, x1) in zip(marks, marks[1:]):
            ks = [r for r in sv if x0 <= r[0] < x1]
            agg = {}
            for r in ks:
                agg[r[2]] = agg.get(r[2], 0.0) + (r[1] - r[0]) * 1e-6
            phases.append((n0, n1, (x1 - x0) * 1e-6, _busy([(r[0], r[1]) for r in ks]) * 1e-6,
                           len(ks), sorted(agg.items(), key=lambda kv: -kv[1])[:top]))
        out.append(((t1 - t0) * 1e-6, phases))
    return out


def print_timeline(d, gap_ms=2.0):
    for k, (wall, phases) in enumerate(timeline(d, gap_ms)):
        print(f"solve {k}: {wall:.1f} ms")
        for n0, n1, w, b, nk, top in phases:
            print(f"  {n0:>22} -> {n1:<22} {w:8.1f} ms  busy {b:8.1f} ms  {nk:6d} launches")
            for name, ms in top:
                print(f"  {'':>22}    {ms:8.1f} ms  {name}")


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        print_stats(sys.argv[2])
    elif len(sys.argv) >= 5 and sys.argv[1] == "traffic":
        r = traffic(sys.argv[2], sys.argv[3], sys.argv[4])
        print(json.dumps({k: r[k] for k in r if k != "kernels"}))
    elif len(sys.argv) >= 3 and sys.argv[1] == "mfma":
        print_mfma(sys.argv[2], int(sys.argv[3]) if len(sys.argv) >= 4 else 1024)
    elif len(sys.argv) >= 3 and sys.argv[1] == "timeline":
        print_timeline(sys.argv[2], float(sys.argv[3]) if len(sys.argv) >= 4 else 2.0)
    else:
        print(__doc__)
        sys.exit(2)
