"""Summaries of rocprofv3 CSV output for the profiles/ folder.

  python profile_summary.py trace <kernel_trace.csv> <out.md> "<command>" "<title>" [note]
      per-kernel totals and, for the solve-phase kernels, per launch size
      (one grid size per multigrid level).

  python profile_summary.py counters <fetch_counter_collection.csv> <write_counter_collection.csv>
                            <out.json> <out.md> <kernel> <algorithmic_bytes> "<fetch cmd>" "<write cmd>"
                            [grid] [title]
      FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the launches of the kernels
      whose name matches the regular expression <kernel> with the given grid
      (default: the largest grid), each scaled by the factor that maps the same
      counter, read on a 1 GiB read + 1 GiB write elementwise kernel, to its
      known byte count.

  python profile_summary.py mfma <counter_collection.csv> <out.md> "<command>" "<title>"
      FP32 and FP64 matrix-core work per dispatch (SQ_INSTS_VALU_MFMA_MOPS_F32 /
      _F64 x 512 flops) over the dispatch duration, against the matrix peak of
      the dispatch's precision.
"""
import csv
import hashlib
import json
import os
import re
import statistics
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
SOLVE_KERNELS = ("k_cheb", "k_sell_spmv", "k_patch", "k_packed", "k_spmv_dot")
CALIBRATION_BYTES = 1 << 30


def short(name):
    return name.split("(")[0]


def trace(path, out, cmd, title, note=""):
    rows = list(csv.DictReader(open(path)))
    byname, bygrid = defaultdict(list), defaultdict(list)
    for r in rows:
        name = short(r["Kernel_Name"])
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        byname[name].append(d)
        if any(k in name for k in SOLVE_KERNELS):
            bygrid[(name, int(r["Grid_Size_X"]) if "Grid_Size_X" in r else int(r["Grid_Size"]))].append(d)
    tot = sum(sum(v) for v in byname.values())
    L = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", cmd, "```", ""]
    if note:
        L += [note, ""]
    L += [f"Kernel dispatches: {len(rows)}; total kernel time {tot / 1e3:.1f} ms (setup and timed solves).", "",
          "## All kernels by total time", "", "| kernel | calls | total ms | avg us |", "|---|---|---|---|"]
    for name, v in sorted(byname.items(), key=lambda kv: -sum(kv[1]))[:30]:
        L.append(f"| `{name}` | {len(v)} | {sum(v) / 1e3:.2f} | {statistics.mean(v):.1f} |")
    L += ["", "## Solve-phase kernels by launch size (grid = threads; one grid size per level; the 40 largest "
              "totals)", "",
          "| kernel | grid | calls | total ms | avg us | min us | max us |", "|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(bygrid.items(), key=lambda kv: -sum(kv[1]))[:40]:
        L.append(f"| `{name}` | {grid} | {len(v)} | {sum(v) / 1e3:.2f} | {statistics.mean(v):.1f} | "
                 f"{min(v):.1f} | {max(v):.1f} |")
    open(out, "w").write("\n".join(L) + "\n")


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, grid, value)} for one counter."""
    out = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        v = float(r["Counter_Value"])
        name, grid = short(r["Kernel_Name"]), int(r["Grid_Size"])
        if key in out:
            v += out[key][2]
        out[key] = (name, grid, v)
    return out


def _kernel_and_calibration(path, counter, kernel, grid=None):
    d = _per_dispatch(path, counter)
    ks = [(g, v) for (n, g, v) in d.values() if re.search(kernel, n)]
    gmax = max(g for g, _ in ks) if grid is None else grid
    vals = [v for g, v in ks if g == gmax]
    assert vals, f"no launch of {kernel} with grid {gmax}"
    cal = [v for (n, g, v) in d.values() if "MulFunctor" in n and g * 1 >= (1 << 25)]
    return gmax, vals, cal


def source_hash():
    from bench import kernel_source_hash
    return kernel_source_hash()


def counters(fetch_csv, write_csv, out_json, out_md, kernel, alg_bytes, fetch_cmd, write_cmd, grid=None,
             title=None):
    alg_bytes = float(alg_bytes)
    grid = int(grid) if grid else None
    gf, fv, fcal = _kernel_and_calibration(fetch_csv, "FETCH_SIZE", kernel, grid)
    gw, wv, wcal = _kernel_and_calibration(write_csv, "WRITE_SIZE", kernel, grid)
    assert gf == gw and fcal and wcal, "kernel or calibration launches missing"
    f_factor = CALIBRATION_BYTES / (statistics.median(fcal) * 1024)
    w_factor = CALIBRATION_BYTES / (statistics.median(wcal) * 1024)
    fetch_b = statistics.mean(fv) * 1024 * f_factor
    write_b = statistics.mean(wv) * 1024 * w_factor
    d = {"kernel": kernel, "grid": gf, "launches_fetch": len(fv), "launches_write": len(wv),
         "fetch_kib_per_launch_raw": statistics.mean(fv), "write_kib_per_launch_raw": statistics.mean(wv),
         "calibration_fetch_kib_raw": statistics.median(fcal), "calibration_write_kib_raw": statistics.median(wcal),
         "fetch_factor": f_factor, "write_factor": w_factor,
         "hbm_bytes_per_launch": fetch_b + write_b, "algorithmic_bytes_per_launch": alg_bytes,
         "traffic_over_algorithmic": (fetch_b + write_b) / alg_bytes,
         "kernel_source_hash": source_hash(), "command_fetch": fetch_cmd, "command_write": write_cmd}
    json.dump(d, open(out_json, "w"), indent=1)
    L = [f"# {title}" if title else f"# HBM traffic of `{kernel}` (largest grid, {gf} threads)", "",
         f"Launches of the kernels matching `{kernel}` with a grid of {gf} threads.", "",
         "Commands (from the repository root, one MI355X):", "", "```", fetch_cmd, write_cmd, "```", "",
         "| quantity | value |", "|---|---|",
         f"| FETCH_SIZE per launch (raw, KiB) | {d['fetch_kib_per_launch_raw']:.0f} ({len(fv)} launches) |",
         f"| WRITE_SIZE per launch (raw, KiB) | {d['write_kib_per_launch_raw']:.0f} ({len(wv)} launches) |",
         f"| calibration kernel (1 GiB read, 1 GiB write): FETCH_SIZE / WRITE_SIZE KiB | "
         f"{d['calibration_fetch_kib_raw']:.0f} / {d['calibration_write_kib_raw']:.0f} |",
         f"| scale factors fetch / write | {f_factor:.4f} / {w_factor:.4f} |",
         f"| HBM bytes per launch (scaled) | {fetch_b + write_b:.4e} |",
         f"| algorithmic bytes per launch | {alg_bytes:.4e} |",
         f"| traffic / algorithmic | {d['traffic_over_algorithmic']:.3f} |", "",
         "WRITE_SIZE counts the lines the L2 writes back during the dispatch; lines still dirty in the L2 "
         "when the kernel ends (at most the 8 x 4 MB of L2) are written back later and counted with a later "
         "dispatch, so the write figure can fall short of the bytes the kernel stores.", ""]
    open(out_md, "w").write("\n".join(L) + "\n")
    print(json.dumps(d))


PEAK_TFLOPS = {"F64": 78.6, "F32": 157.3}   # MI355X dense matrix-core peaks


def mfma(path, out, cmd, title):
    """Matrix-core work per dispatch from SQ_INSTS_VALU_MFMA_MOPS_F32 / _F64
    (units of 512 flops) over the dispatch duration, against the peak of the
    dispatch's own precision (the one with the larger count)."""
    per = defaultdict(dict)
    for r in csv.DictReader(open(path)):
        key = (int(r["Dispatch_Id"]), short(r["Kernel_Name"]), int(r["Grid_Size"]))
        per[key][r["Counter_Name"]] = float(r["Counter_Value"])
        per[key]["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    L = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```", cmd, "```", "",
         "| dispatch | kernel | workgroups | precision | MFMA flops | ms | TFLOP/s | of matrix peak |",
         "|---|---|---|---|---|---|---|---|"]
    tot = defaultdict(lambda: [0.0, 0])
    for (did, name, grid), v in sorted(per.items()):
        fl = {p: v.get(f"SQ_INSTS_VALU_MFMA_MOPS_{p}", 0.0) * 512 for p in PEAK_TFLOPS}
        p = max(fl, key=fl.get)
        ns = v["ns"]
        tot[p][0] += fl[p]
        tot[p][1] += ns
        L.append(f"| {did} | `{name}` | {grid // 256} | {p} | {fl[p]:.3e} | {ns / 1e6:.1f} | "
                 f"{fl[p] / ns / 1e3:.2f} | {fl[p] / ns / 1e3 / PEAK_TFLOPS[p]:.3f} |")
    L.append("")
    for p, (f, t) in sorted(tot.items()):
        if t:
            L.append(f"{p} total: {f:.3e} flops in {t / 1e6:.1f} ms = {f / t / 1e3:.2f} TFLOP/s "
                     f"({f / t / 1e3 / PEAK_TFLOPS[p]:.3f} of the {PEAK_TFLOPS[p]} TFLOP/s {p} matrix peak).")
    L.append("")
    open(out, "w").write("\n".join(L) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(*sys.argv[2:])
    elif sys.argv[1] == "counters":
        counters(*sys.argv[2:])
    elif sys.argv[1] == "mfma":
        mfma(*sys.argv[2:])
    else:
        sys.exit(__doc__)
