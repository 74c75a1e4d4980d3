"""Summaries of rocprofv3 CSV output for the committed profiles.

    python -m paper_1901_07993_amd.prof_summary stats TRACE.csv OUT.md --title T --cmd C [--group P ...]
        per-kernel totals of the last factorization in a kernel trace (a
        factorization starts at its k_chol_scatter launch), plus the span;
        each --group P adds the totals of all kernels whose names start
        with P (e.g. every variant of the numeric kernel)
    python -m paper_1901_07993_amd.prof_summary traffic FETCH.csv WRITE.csv OUT.json \
            --kernel k_numeric_f64 --copy-mib N --cmd C [--hash H]
        HBM bytes per dispatch of one kernel from FETCH_SIZE / WRITE_SIZE
        counter runs, each scaled by the factor that maps the same counter
        on a plain device copy of N MiB (issued before any library kernel)
        to its known size
    python -m paper_1901_07993_amd.prof_summary mfma COUNTERS.csv TRACE.csv OUT.json \
            --kernel k_numeric_f64 --peak-tflops P --cmd C
        MFMA busy fraction and MFMA flop rate of one kernel (MfmaUtil and
        MfmaFlopsF64 counters, dispatch times from the same run's trace)
"""
from __future__ import annotations

import argparse
import collections
import csv
import json


def _short(name: str) -> str:
    return name.replace("lif::(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def stats(trace: str, out: str, title: str, cmd: str, groups=()) -> None:
    rows = list(csv.DictReader(open(trace)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    starts = [i for i, r in enumerate(rows) if "k_chol_scatter" in r["Kernel_Name"]]
    seg = rows[starts[-1]:] if starts else rows
    t0 = int(seg[0]["Start_Timestamp"])
    t1 = max(int(r["End_Timestamp"]) for r in seg)
    agg = collections.defaultdict(lambda: [0, 0])
    busy = 0
    for r in seg:
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        agg[_short(r["Kernel_Name"])][0] += 1
        agg[_short(r["Kernel_Name"])][1] += d
        busy += d
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommand (repository root, one MI355X):\n\n```\n{cmd}\n```\n\n")
        f.write(f"Last factorization of the run: {len(seg)} kernels, span {(t1 - t0) / 1e6:.2f} ms, "
                f"summed kernel time {busy / 1e6:.2f} ms (the leaf inverse runs on a second stream, so "
                f"kernels overlap; the profiler adds time between launches).\n\n")
        f.write("| kernel | calls | total ms | avg us | % of summed |\n|---|---:|---:|---:|---:|\n")
        for n, (c, d) in sorted(agg.items(), key=lambda x: -x[1][1]):
            f.write(f"| `{n}` | {c} | {d / 1e6:.3f} | {d / c / 1e3:.1f} | {100 * d / busy:.1f} |\n")
        for g in groups:
            c = sum(v[0] for n, v in agg.items() if n.startswith(g))
            d = sum(v[1] for n, v in agg.items() if n.startswith(g))
            if c:
                f.write(f"\nAll `{g}*` kernels together: {c} calls, {d / 1e6:.3f} ms, average "
                        f"{d / c / 1e3:.1f} us per call, {100 * d / busy:.1f} % of the summed time.\n")


def _counter(path: str, name: str):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == name]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return rows


def _calibration(rows, copy_mib: float) -> float:
    """Known bytes / counted bytes of the probe copy: the first copy dispatch
    before any library kernel whose count is at least a quarter of the
    probe's size (smaller copies are the runtime's own)."""
    want = copy_mib * 2 ** 20
    for r in rows:
        if "lif::" in r["Kernel_Name"]:
            break
        counted = float(r["Counter_Value"]) * 1024.0
        if "copyBuffer" in r["Kernel_Name"] and counted >= 0.25 * want:
            return want / counted
    raise SystemExit("no probe copy dispatch before the first library kernel")


def traffic(fetch: str, write: str, out: str, kernel: str, copy_mib: float, cmd: str, khash: str) -> None:
    res = {"kernel": kernel, "command": cmd, "copy_probe_mib": copy_mib, "kernel_hash": khash}
    for key, path, cname in (("fetch", fetch, "FETCH_SIZE"), ("write", write, "WRITE_SIZE")):
        rows = _counter(path, cname)
        scale = _calibration(rows, copy_mib)
        vals = [float(r["Counter_Value"]) * 1024.0 for r in rows if _short(r["Kernel_Name"]).startswith(kernel)]
        res[f"{key}_dispatches"] = len(vals)
        res[f"{key}_bytes_per_dispatch_raw"] = sum(vals) / max(len(vals), 1)
        res[f"{key}_calibration"] = scale
        res[f"{key}_bytes_per_dispatch"] = scale * sum(vals) / max(len(vals), 1)
    res["bytes_per_launch"] = res["fetch_bytes_per_dispatch"] + res["write_bytes_per_dispatch"]
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


def mfma(counters: str, trace: str, out: str, kernel: str, peak_tflops: float, cmd: str,
         flops_counter: str = "MfmaFlopsF64") -> None:
    """MFMA busy fraction and MFMA flop rate of one kernel from a counter run
    that also traced the kernels (durations by dispatch id): the derived
    counters MfmaUtil (MFMA busy cycles over active cycles and SIMDs, in %)
    and MfmaFlopsF64 / MfmaFlopsF32 / MfmaFlopsBF16 (512 flops per MFMA op
    of that type), weighted by dispatch time."""
    dur = {}
    for r in csv.DictReader(open(trace)):
        if _short(r["Kernel_Name"]).startswith(kernel):
            dur[int(r["Dispatch_Id"])] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    util, flops = {}, {}
    for r in csv.DictReader(open(counters)):
        if not _short(r["Kernel_Name"]).startswith(kernel):
            continue
        d = int(r["Dispatch_Id"])
        if r["Counter_Name"] == "MfmaUtil":
            util[d] = util.get(d, 0.0) + float(r["Counter_Value"])
        elif r["Counter_Name"] == flops_counter:
            flops[d] = flops.get(d, 0.0) + float(r["Counter_Value"])
    ids = sorted(set(util) & set(flops) & set(dur))
    t = sum(dur[i] for i in ids)
    res = {"kernel": kernel, "command": cmd, "dispatches": len(ids), "kernel_seconds": t / 1e9,
           "flops_counter": flops_counter,
           "mfma_util_pct_time_weighted": sum(util[i] * dur[i] for i in ids) / t if t else None,
           "mfma_flops": sum(flops[i] for i in ids),
           "mfma_tflops": sum(flops[i] for i in ids) / (t / 1e9) / 1e12 if t else None,
           "peak_tflops": peak_tflops}
    res["frac_of_peak"] = res["mfma_tflops"] / peak_tflops if res["mfma_tflops"] else None
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
        f.write("\n")


def _last_factorization(rows, id_key):
    """Rows of the last factorization (from its k_chol_scatter dispatch on)."""
    rows = sorted(rows, key=lambda r: int(r[id_key]))
    starts = [i for i, r in enumerate(rows) if "k_chol_scatter" in r["Kernel_Name"]]
    return rows[starts[-1]:] if starts else rows


def hbm(trace: str, fetch: str, write: str, out: str, copy_mib: float, peak_gbps: float, title: str,
        cmd: str) -> None:
    """Per kernel of the last factorization: HBM bytes per dispatch (FETCH_SIZE
    + WRITE_SIZE, each calibrated on the probe copy) from the two counter runs,
    mean duration per dispatch from the trace run of the same command, and
    their ratio against the HBM peak."""
    dur = collections.defaultdict(list)
    for r in _last_factorization(list(csv.DictReader(open(trace))), "Dispatch_Id"):
        dur[_short(r["Kernel_Name"])].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    byts = collections.defaultdict(lambda: [0.0, 0])
    for path, cname in ((fetch, "FETCH_SIZE"), (write, "WRITE_SIZE")):
        rows = _counter(path, cname)
        scale = _calibration(rows, copy_mib)
        per = collections.defaultdict(list)
        for r in _last_factorization(rows, "Dispatch_Id"):
            per[_short(r["Kernel_Name"])].append(scale * float(r["Counter_Value"]) * 1024.0)
        for k, v in per.items():
            byts[k][0] += sum(v) / len(v)
            byts[k][1] = len(v)
    total_t = sum(sum(v) for v in dur.values())
    with open(out, "w") as f:
        f.write(f"# {title}\n\nCommands (repository root, one MI355X):\n\n```\n{cmd}\n```\n\n")
        f.write("Bytes per dispatch: FETCH_SIZE + WRITE_SIZE of the counter runs, each scaled by the factor "
                f"that maps the same counter on a {copy_mib:g} MiB device copy to its size; duration per "
                "dispatch: the kernel trace of the same command. Both over the last factorization of the "
                f"run. HBM peak {peak_gbps:g} GB/s.\n\n")
        f.write("| kernel | dispatches | % of kernel time | MB per dispatch | us per dispatch | GB/s | "
                "% of HBM peak |\n|---|---:|---:|---:|---:|---:|---:|\n")
        for k, d in sorted(dur.items(), key=lambda x: -sum(x[1])):
            if k not in byts:
                continue
            b = byts[k][0]
            t = sum(d) / len(d)
            gbps = b / t if t else 0.0
            f.write(f"| `{k}` | {len(d)} | {100 * sum(d) / total_t:.1f} | {b / 1e6:.2f} | {t / 1e3:.1f} | "
                    f"{gbps:.0f} | {100 * gbps / peak_gbps:.1f} |\n")


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("trace")
    s.add_argument("out")
    s.add_argument("--title", required=True)
    s.add_argument("--cmd", required=True)
    s.add_argument("--group", action="append", default=[])
    t = sub.add_parser("traffic")
    t.add_argument("fetch")
    t.add_argument("write")
    t.add_argument("out")
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-mib", type=float, required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--hash", default="")
    h = sub.add_parser("hbm")
    h.add_argument("trace")
    h.add_argument("fetch")
    h.add_argument("write")
    h.add_argument("out")
    h.add_argument("--copy-mib", type=float, required=True)
    h.add_argument("--peak-gbps", type=float, default=8000.0)
    h.add_argument("--title", required=True)
    h.add_argument("--cmd", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("counters")
    m.add_argument("trace")
    m.add_argument("out")
    m.add_argument("--kernel", required=True)
    m.add_argument("--peak-tflops", type=float, required=True)
    m.add_argument("--cmd", required=True)
    m.add_argument("--flops-counter", default="MfmaFlopsF64")
    a = ap.parse_args()
    if a.what == "stats":
        stats(a.trace, a.out, a.title, a.cmd, a.group)
    elif a.what == "traffic":
        traffic(a.fetch, a.write, a.out, a.kernel, a.copy_mib, a.cmd, a.hash)
    elif a.what == "hbm":
        hbm(a.trace, a.fetch, a.write, a.out, a.copy_mib, a.peak_gbps, a.title, a.cmd)
    else:
        mfma(a.counters, a.trace, a.out, a.kernel, a.peak_tflops, a.cmd, a.flops_counter)


if __name__ == "__main__":
    main()
