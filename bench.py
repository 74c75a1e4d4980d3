"""Benchmark: seconds per inverse factorization and leaf-GEMM rate on one GPU.

Workload: the quasi-linear helix chain, 5000 residues x 20 s-type Gaussian
centres (n = 100,000), b = 64 leaf blocks, block truncation tau = 1e-10,
localized inverse factorization with binary recursion down to 4096-row
leaves (inverse Cholesky leaves), refinement with m = 4 and the paper's
stopping rule, all FP64.  Synthetic, seeded input (the paper's Ergo overlap
matrices are not available).

A step is one complete lif_localized call on the resident S (the handle is
created, S uploaded and truncated, before the timed region).  Output: one
JSON line, which also carries the FP32 / BF16 schedules on the chain, RINCH,
IRSI and the regular-form recursion on the same S, the per-kernel rooflines of
the leaf factorization and the symbolic phases, the FP64-against-BF16
comparison on the 20,000-molecule water cluster, and the CPU oracle's time.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--no-cpu-baseline]
    python bench.py --water-only fp64_sym,bf16_schedule_sym [--water-count N]
    python bench.py --fit-sweep 30000,35000,40000     (largest cluster that fits)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "s per inverse factorization + leaf-GEMM GFLOP/s at ‖Z*SZ−I‖≤1e-10, FP64 vs mixed"
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_BPS = 8.0e12
KERNEL_SOURCES = ("paper_1901_07993_amd/csrc/spgemm.hip", "paper_1901_07993_amd/csrc/tile_mma.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "numeric_f64_chain5000_traffic.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per numeric-kernel launch from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(count: int = 5000) -> dict:
    """The block-sparse FP64 oracle (oracle/blocked.py: the same LIF steps on
    block lists, numpy) on the chain of ``count`` residues (n = 20 count,
    tau = 1e-10, 4096-row leaves): by default the whole workload (about 10 s
    on 16 cores); a shorter chain is scaled to 5000 residues by the residue
    ratio (its cost grows about linearly with the chain)."""
    import numpy as np
    from gen import config_matrix
    from oracle import blocked

    S, cfg = config_matrix(1, count=count)
    t0 = time.perf_counter()
    c0 = time.process_time()
    blocked.lif(S, cfg["tau"], base_rows=4096)
    dt = time.perf_counter() - t0
    cpu = time.process_time() - c0   # CPU time of every thread of the process
    scale = 5000 / count
    avail = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": dt * scale, "unit": "s", "cores": max(1, round(cpu / dt)), "kind": "oracle",
            "sample": f"block-sparse numpy oracle LIF on chain-{count} (n={S.n}, tau=1e-10, 4096-row leaves), "
                      f"one factorization: {dt:.2f} s measured" +
                      (f", x {scale:g} (residues) to chain-5000" if scale != 1 else " (the whole workload)"),
            "sample_seconds": dt, "cores_effective": cpu / dt, "cores_available": avail,
            "cpu_model": cpu_model(), "np_version": np.__version__}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def rel_diff(A, B) -> float:
    """||A - B||_F / ||B||_F of two block lists (host arrays sorted by (row,
    col)); blocks present in one list only count whole.  Reductions run
    through torch on the host (several threads), in chunks of blocks."""
    import numpy as np
    import torch
    nb = (int(B.n) + int(B.b) - 1) // int(B.b)
    ka = np.asarray(A.brow, np.int64) * nb + np.asarray(A.bcol, np.int64)
    kb = np.asarray(B.brow, np.int64) * nb + np.asarray(B.bcol, np.int64)
    _, ia, ib = np.intersect1d(ka, kb, assume_unique=True, return_indices=True)
    chunk = 1 << 15

    def sumsq(vals, idx=None):
        tot = 0.0
        n = len(vals) if idx is None else len(idx)
        for s in range(0, n, chunk):
            v = vals[s:s + chunk] if idx is None else vals[idx[s:s + chunk]]
            t = torch.from_numpy(np.ascontiguousarray(v))
            tot += float(torch.sum(t * t))
        return tot

    num = 0.0
    for s in range(0, len(ia), chunk):
        d = torch.from_numpy(A.vals[ia[s:s + chunk]]) - torch.from_numpy(B.vals[ib[s:s + chunk]])
        num += float(torch.sum(d * d))
    only_a = np.setdiff1d(np.arange(len(ka)), ia, assume_unique=True)
    only_b = np.setdiff1d(np.arange(len(kb)), ib, assume_unique=True)
    num += sumsq(A.vals, only_a) + sumsq(B.vals, only_b)
    return (num / sumsq(B.vals)) ** 0.5


def time_method(lif, Sd, tau, meth, steps, **kw):
    """(seconds per call, info of the last call) of one untimed and `steps`
    timed calls of a Factorization method on the device matrix Sd."""
    import torch
    f = lif.Factorization(Sd, tau=tau, base_rows=4096, **kw)
    getattr(f, meth)()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        info = getattr(f, meth)()
    torch.cuda.synchronize()
    s = (time.perf_counter() - t0) / steps
    f.close()
    return s, info


WATER_VARIANTS = {
    # name: (precision, precision switch, symmetric delta update, inputs of
    # the delta update in reduced iterations)
    "fp64": ("FP64", 0.0, 0, "FP64"), "fp64_sym": ("FP64", 0.0, 1, "FP64"),
    "fp32_schedule": ("MIXED_FP32", 1e-2, 0, "FP64"), "bf16_schedule": ("MIXED_BF16", 1e-2, 0, "FP64"),
    "fp32_schedule_sym": ("MIXED_FP32", 1e-2, 1, "FP64"), "bf16_schedule_sym": ("MIXED_BF16", 1e-2, 1, "FP64"),
    "bf16_schedule_sym_f32update": ("MIXED_BF16", 1e-2, 1, "MIXED_FP32"),
    "fp32_schedule_sym_f32update": ("MIXED_FP32", 1e-2, 1, "MIXED_FP32"),
}
# the same with IRSI instead of LIF (the method of the small water workload,
# from Z_0 = I / sqrt(beta), beta the Gershgorin bound): "irsi_" + a name above
for _k, _v in list(WATER_VARIANTS.items()):
    WATER_VARIANTS["irsi_" + _k] = _v
PEAK_TFLOPS = {"FP64": 78.6, "MIXED_FP32": 157.3, "MIXED_BF16": 2500.0}


def water_comparison(lif, count, which=("fp64_sym", "bf16_schedule_sym", "irsi_fp64_sym", "irsi_bf16_schedule_sym"),
                     z_diff=True, residuals=True):
    """FP64 against the scheduled reduced-precision corrections on a water
    cluster (tau = 1e-8, b = 64, paper stop; LIF to 4096-row leaves, and
    IRSI for the "irsi_" variants): the metric's comparison, on the
    compute-bound products where reduced precision pays.  One handle holds S and its memory pool for all runs
    (lif_set_opts between them): one untimed warm-up per method (LIF, and
    IRSI from c = 1 / sqrt(beta) for the "irsi_" variants), then one timed
    factorization per variant.  Reported per run: seconds, the untruncated
    residual against the truncated S that was factorized and, for the FP64
    runs, against S before that truncation (Table 1 leaves open which one it
    used), node iterations, the leaf-GEMM rate of each precision on its own,
    the memory peak and, for reduced runs, ||Z - Z_fp64||_F / ||Z_fp64||_F
    against the same method's FP64 factor.  A variant
    that fails (out of memory, say) is reported with its error."""
    import torch
    from gen import config_matrix
    print(f"# generating water-{count}", file=sys.stderr, flush=True)
    S, cfg = config_matrix(2, count=count)
    Sd = type("DevBlocks", (), dict(n=S.n, b=S.b, brow=torch.from_numpy(S.brow).cuda(),
                                    bcol=torch.from_numpy(S.bcol).cuda(), vals=torch.from_numpy(S.vals).cuda()))
    out = {"workload": f"water-{count}: {count} molecules x 7 s-Gaussians, n={S.n}, b=64, tau={cfg['tau']}, "
                       f"LIF to 4096-row leaves, and IRSI from I / sqrt(beta) (\"irsi_\" variants), m=4, "
                       f"paper stop", "n": S.n, "nnzb_S": int(S.nnzb),
           "tau_floor_note": "with per-block truncation at tau = 1e-8 the residual settles near 1e-5 (the floor); "
                             "the 1e-10 target is the tau = 0 runs' gate",
           "device_memory_gib": torch.cuda.get_device_properties(0).total_memory / 2 ** 30}
    first = WATER_VARIANTS[which[0]]
    f = lif.Factorization(Sd, tau=cfg["tau"], base_rows=4096, prec=getattr(lif, first[0]), prec_switch=first[1],
                          sym_delta=first[2], update_prec=getattr(lif, first[3]), start=lif.START_INV_SQRT_GERSH,
                          timing=1)
    warm = set()
    for name in which:
        irsi = name.startswith("irsi_")
        if irsi in warm:
            continue
        warm.add(irsi)
        pname, sw, sym, upd = WATER_VARIANTS[name]
        f.set_opts(prec=getattr(lif, pname), prec_switch=sw, sym_delta=sym, update_prec=getattr(lif, upd),
                   start=lif.START_INV_SQRT_GERSH)
        try:
            f.refine() if irsi else f.localized()
        except lif.LifError as e:
            print(f"# water-{count} warm-up of {name}: {e}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    print(f"# water-{count} warm-up done", file=sys.stderr, flush=True)
    t64 = {}   # FP64 seconds by (method, symmetric delta)
    Zref = {}  # FP64 factor by method
    for name in which:
        pname, sw, sym, upd = WATER_VARIANTS[name]
        irsi = name.startswith("irsi_")
        f.set_opts(prec=getattr(lif, pname), prec_switch=sw, sym_delta=sym, update_prec=getattr(lif, upd),
                   start=lif.START_INV_SQRT_GERSH)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            info = f.refine() if irsi else f.localized()
        except lif.LifError as e:
            out[name] = {"error": str(e)}
            print(f"# water-{count} {name}: {e}", file=sys.stderr, flush=True)
            continue
        torch.cuda.synchronize()
        s = time.perf_counter() - t0
        # the residual against S before its truncation for the FP64 runs (an
        # untruncated residual of this size costs about as much as a
        # factorization; the mixed runs' factors differ from FP64's by 1e-3)
        res = f.residual() if residuals else None
        res_u = f.residual_against(Sd) if residuals and pname == "FP64" else None
        r = {"s_per_factorization": s, "residual": res, "residual_untruncated_S": res_u,
             "iterations_total": info["iterations_total"], "iterations_reduced": info["iterations_reduced"],
             "iterations_redone": info["iterations_redone"], "nnzb_Z": info["nnzb_Z"],
             "mem_peak_gib": info["mem_peak_bytes"] / 2 ** 30, "sym_delta": sym,
             "method": "irsi" if irsi else "lif",
             "products_compacted": info["products_compacted"], "pair_panels": info["pair_panels"]}
        fl, sec = info["flops_leaf_gemm"], info["seconds_leaf_gemm"]
        flr, secr = info["flops_leaf_gemm_reduced"], info["seconds_leaf_gemm_reduced"]
        r["leaf_gemm_seconds"] = sec
        r["leaf_gemm_reduced_seconds"] = secr
        if sec - secr > 0:
            r["leaf_gemm_fp64_tflops"] = (fl - flr) / (sec - secr) / 1e12
            r["leaf_gemm_fp64_frac_of_peak"] = r["leaf_gemm_fp64_tflops"] / PEAK_TFLOPS["FP64"]
        # the reduced launches by input precision (with update_prec the
        # delta update's FP32 products join the correction's BF16 ones)
        fl32, sec32 = info["flops_leaf_gemm_fp32"], info["seconds_leaf_gemm_fp32"]
        n32 = info["leaf_gemm_launches_fp32"]
        nred = info["leaf_gemm_launches_reduced"]
        for tag, p_fl, p_sec, p_n, peak in (("bf16", flr - fl32, secr - sec32, nred - n32, "MIXED_BF16"),
                                            ("fp32", fl32, sec32, n32, "MIXED_FP32")):
            if p_n > 0 and p_sec > 0:
                r[f"leaf_gemm_{tag}_seconds"] = p_sec
                r[f"leaf_gemm_{tag}_tflops"] = p_fl / p_sec / 1e12
                r[f"leaf_gemm_{tag}_frac_of_peak"] = r[f"leaf_gemm_{tag}_tflops"] / PEAK_TFLOPS[peak]
                r[f"leaf_gemm_{tag}_launches"] = p_n
        if pname == "FP64":
            t64[(irsi, sym)] = s
            if z_diff and irsi not in Zref:
                Zref[irsi] = f.get_Z()
        else:
            if (irsi, sym) in t64:
                r["speedup_vs_fp64_same_update"] = t64[(irsi, sym)] / s
            if (irsi, 0) in t64:
                r["speedup_vs_fp64"] = t64[(irsi, 0)] / s
            if z_diff and irsi in Zref:
                r["rel_diff_vs_fp64_Z"] = rel_diff(f.get_Z(), Zref[irsi])
        out[name] = r
        print(f"# water-{count} {name}: {s:.2f} s, residual {res} (untruncated S {res_u})",
              file=sys.stderr, flush=True)
    f.close()
    del Zref
    torch.cuda.empty_cache()
    return out


def fit_sweep(lif, counts, variant):
    """The largest water cluster that one GPU factorizes (the survey's
    largest single-GPU case: tau = 1e-8, b = 64, LIF to 4096-row leaves,
    by default FP32 corrections under the schedule): one factorization per
    size, in increasing order, until one does not fit in the device memory
    (reported with its error).  Per size: seconds (first factorization on
    its handle, so including the memory pool's hipMalloc calls), memory
    peak, blocks of Z, node iterations, the residual and each precision's
    leaf-GEMM rate; the untruncated residual after it (its own error, if
    it does not fit, does not end the sweep)."""
    import torch
    from gen import config_matrix
    pname, sw, sym, upd = WATER_VARIANTS[variant]
    rows = []
    for count in counts:
        print(f"# generating water-{count}", file=sys.stderr, flush=True)
        S, cfg = config_matrix(2, count=count)
        Sd = type("DevBlocks", (), dict(n=S.n, b=S.b, brow=torch.from_numpy(S.brow).cuda(),
                                        bcol=torch.from_numpy(S.bcol).cuda(), vals=torch.from_numpy(S.vals).cuda()))
        row = {"count": count, "n": S.n, "nnzb_S": int(S.nnzb)}
        del S
        f = lif.Factorization(Sd, tau=cfg["tau"], base_rows=4096, prec=getattr(lif, pname), prec_switch=sw,
                              sym_delta=sym, update_prec=getattr(lif, upd), timing=1)
        try:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = f.localized()
            torch.cuda.synchronize()
            row.update(fits=True, s_per_factorization=time.perf_counter() - t0,
                       mem_peak_gib=info["mem_peak_bytes"] / 2 ** 30, nnzb_Z=info["nnzb_Z"],
                       iterations_total=info["iterations_total"], iterations_reduced=info["iterations_reduced"])
            fl, sec = info["flops_leaf_gemm"], info["seconds_leaf_gemm"]
            flr, secr = info["flops_leaf_gemm_reduced"], info["seconds_leaf_gemm_reduced"]
            if sec - secr > 0:
                row["leaf_gemm_fp64_tflops"] = (fl - flr) / (sec - secr) / 1e12
            if secr > 0:
                row[f"leaf_gemm_{pname.split('_')[-1].lower()}_tflops"] = flr / secr / 1e12
                row["leaf_gemm_reduced_frac_of_peak"] = flr / secr / 1e12 / PEAK_TFLOPS[pname]
        except lif.LifError as e:
            row.update(fits=False, error=str(e))
        if row["fits"]:
            try:
                row["residual"] = f.residual()
            except lif.LifError as e:
                row["residual_error"] = str(e)
        f.close()
        del Sd
        torch.cuda.empty_cache()
        rows.append(row)
        print(f"# water-{count}: {row}", file=sys.stderr, flush=True)
        if not row["fits"]:
            break
    return {"fit_sweep": rows, "variant": variant, "device_memory_gib":
            torch.cuda.get_device_properties(0).total_memory / 2 ** 30, "data": "synthetic"}


def cpl_sweep(counts, steps):
    """Critical-path task counts (the one-GPU shadow of Sec. 3) and times of
    the four methods on chains of the given lengths."""
    import torch
    from gen import config_matrix
    from paper_1901_07993_amd import lif
    rows = []
    for count in counts:
        S, cfg = config_matrix(1, count=count)
        Sd = type("DevBlocks", (), dict(n=S.n, b=S.b, brow=torch.from_numpy(S.brow).cuda(),
                                        bcol=torch.from_numpy(S.bcol).cuda(), vals=torch.from_numpy(S.vals).cuda()))
        row = {"count": count, "n": S.n}
        for name, meth, kw in (("lif", "localized", {}), ("rinch", "rinch", {}), ("irsi", "refine", {}),
                               ("recursive_regular", "localized", {"refinement": lif.REFINE_NONLOCAL})):
            s_v, inf = time_method(lif, Sd, cfg["tau"], meth, steps, **kw)
            row[name] = {"s": s_v, "cpl_tasks": inf["cpl_tasks"], "cpl_products": inf["cpl_products"],
                         "iterations_total": inf["iterations_total"]}
            print(f"# chain-{count} {name}: {s_v * 1e3:.1f} ms, {inf['cpl_tasks']} tasks on the critical path",
                  file=sys.stderr, flush=True)
        rows.append(row)
    return {"cpl_sweep": rows, "unit": "tasks", "data": "synthetic"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--count", type=int, default=5000, help="chain residues (5000 = the full workload)")
    ap.add_argument("--no-residual", action="store_true", help="skip the untruncated residual after timing")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32 / BF16 runs")
    ap.add_argument("--no-rinch", action="store_true", help="skip the recursive inverse Cholesky run")
    ap.add_argument("--rinch-steps", type=int, default=2)
    ap.add_argument("--no-variants", action="store_true",
                    help="skip IRSI and the regular-form recursive factorization on the same matrix")
    ap.add_argument("--sym-delta", action="store_true",
                    help="chain runs with opts.sym_delta = 1 (upper-triangle delta update)")
    ap.add_argument("--no-water", action="store_true",
                    help="skip the FP64 vs scheduled mixed-precision comparison on the water cluster")
    ap.add_argument("--water-count", type=int, default=20000,
                    help="molecules of that water cluster (20000 = the n = 140000 workload)")
    ap.add_argument("--water-only", type=str, default="",
                    help="comma-separated subset of fp64,fp64_sym,fp32_schedule,bf16_schedule,"
                         "fp32_schedule_sym,bf16_schedule_sym,bf16_schedule_sym_f32update,"
                         "fp32_schedule_sym_f32update: run only the water "
                         "comparison with these (one JSON line) and exit")
    ap.add_argument("--cpl-sweep", type=str, default="",
                    help="comma-separated chain lengths: print critical-path task counts and times of "
                         "LIF, RINCH, IRSI and the regular-form recursion per size (one JSON line) and exit")
    ap.add_argument("--fit-sweep", type=str, default="",
                    help="comma-separated water-cluster sizes (molecules), increasing: factorize each once "
                         "until one does not fit in the device memory (one JSON line) and exit")
    ap.add_argument("--fit-variant", type=str, default="fp32_schedule_sym",
                    help="precision variant of --fit-sweep (a name of the water comparison)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding the recursion over several "
              "GPUs is a design that is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from gen import config_matrix
    from paper_1901_07993_amd import lif

    lif.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.water_only:
        import torch
        from paper_1901_07993_amd import lif as lifmod
        lifmod.load()
        assert torch.cuda.is_available(), "bench.py needs a GPU"
        print(json.dumps({"water": water_comparison(lifmod, args.water_count, tuple(args.water_only.split(",")),
                                                    z_diff=not args.no_residual, residuals=not args.no_residual)}),
              flush=True)
        return
    if args.fit_sweep:
        from paper_1901_07993_amd import lif as lifmod
        lifmod.load()
        print(json.dumps(fit_sweep(lifmod, [int(x) for x in args.fit_sweep.split(",")], args.fit_variant)),
              flush=True)
        return
    if args.cpl_sweep:
        print(json.dumps(cpl_sweep([int(x) for x in args.cpl_sweep.split(",")], args.rinch_steps)), flush=True)
        return
    print(f"# generating chain-{args.count}", file=sys.stderr, flush=True)
    S, cfg = config_matrix(1, count=args.count)
    Sd = type("DevBlocks", (), dict(n=S.n, b=S.b, brow=torch.from_numpy(S.brow).cuda(),
                                    bcol=torch.from_numpy(S.bcol).cuda(), vals=torch.from_numpy(S.vals).cuda()))
    def run(prec, stop, tol, prec_switch=0.0):
        f = lif.Factorization(Sd, tau=cfg["tau"], base_rows=4096, stop=stop, tol=tol, prec=prec, timing=1,
                              prec_switch=prec_switch, sym_delta=1 if args.sym_delta else 0)
        torch.cuda.synchronize()
        for w in range(args.warmup):
            info = f.localized()
            print(f"# prec {prec} warmup {w}: {info['seconds_total']:.3f} s, top iterations {info['iterations_top']}",
                  file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for k in range(args.steps):
            infos.append(f.localized())
            print(f"# prec {prec} step {k}: {infos[-1]['seconds_total']:.3f} s", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        res = None if args.no_residual else f.residual()
        res_u = None if args.no_residual else f.residual_against(Sd)
        Z = None if args.no_residual else f.get_Z()
        run.detail = None
        if prec == lif.FP64:
            # after the timed steps: three more with every leaf factorization
            # and symbolic phase timed as well (more events per step, so not
            # part of the headline), for their rooflines
            f.set_opts(timing=2)
            run.detail = [f.localized() for _ in range(3)]
        f.close()
        run.res_u = res_u
        return (t1 - t0) / args.steps, infos, res, Z

    step_s, infos, res, Z64 = run(lif.FP64, lif.STOP_PAPER, 1e-10)
    res_u64 = run.res_u
    detail64 = run.detail
    ms = step_s * 1e3
    flops = sum(i["flops_leaf_gemm"] for i in infos)
    gemm_s = sum(i["seconds_leaf_gemm"] for i in infos)
    launches = sum(i["leaf_gemm_launches"] for i in infos)
    last = infos[-1]
    achieved = flops / gemm_s / 1e12 if gemm_s > 0 else 0.0
    traffic = measured_traffic()
    mixed = {}
    if not args.no_mixed:
        # the precision schedule: reduced-precision corrections while
        # ||delta||_F > 1e-2, FP64 iterations and the paper's rule after, so
        # the run stops at the same floor as the FP64 one
        for name, prec in (("fp32", lif.MIXED_FP32), ("bf16", lif.MIXED_BF16)):
            s_m, inf_m, res_m, Zm = run(prec, lif.STOP_PAPER, 1e-10, prec_switch=1e-2)
            fl = sum(i["flops_leaf_gemm"] for i in inf_m)
            gs = sum(i["seconds_leaf_gemm"] for i in inf_m)
            mixed[name] = {"s_per_factorization": s_m, "speedup_vs_fp64": step_s / s_m,
                           "leaf_gemm_gflops": fl / gs / 1e9 if gs > 0 else None,
                           "iterations_top": inf_m[-1]["iterations_top"],
                           "iterations_total": inf_m[-1]["iterations_total"],
                           "iterations_reduced": inf_m[-1]["iterations_reduced"], "prec_switch": 1e-2,
                           "stagnated": inf_m[-1]["stagnated"], "delta_tracked": inf_m[-1]["delta_tracked"],
                           "residual": res_m, "residual_untruncated_S": run.res_u,
                           "rel_diff_vs_fp64_Z": None if Zm is None else rel_diff(Zm, Z64)}
    rinch = None
    if not args.no_rinch:
        # the paper's recursive inverse Cholesky on the same matrix (the
        # sequential recursion LIF shortens): one warm-up, then timed runs
        f = lif.Factorization(Sd, tau=cfg["tau"], base_rows=4096, prec=lif.FP64, timing=1)
        f.rinch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.rinch_steps):
            inf_r = f.rinch()
        torch.cuda.synchronize()
        s_r = (time.perf_counter() - t0) / args.rinch_steps
        rinch = {"s_per_factorization": s_r, "depth": inf_r["levels"], "nnzb_Z": inf_r["nnzb_Z"],
                 "cpl_tasks": inf_r["cpl_tasks"], "cpl_products": inf_r["cpl_products"],
                 "residual": None if args.no_residual else f.residual(),
                 "leaf_gemm_gflops": (inf_r["flops_leaf_gemm"] / inf_r["seconds_leaf_gemm"] / 1e9
                                      if inf_r["seconds_leaf_gemm"] > 0 else None),
                 "lif_speedup": s_r / step_s}
        f.close()
    variants = None
    if not args.no_variants:
        # the other methods of the paper on the same matrix: IRSI (Sec. 2.2)
        # and the recursive factorization with the regular correction
        # (Sec. 2.3), with their critical-path shadows beside LIF's
        variants = {"lif": {"s_per_factorization": step_s, "cpl_tasks": last["cpl_tasks"],
                            "cpl_products": last["cpl_products"]}}
        if rinch:
            variants["rinch"] = {"s_per_factorization": rinch["s_per_factorization"],
                                 "cpl_tasks": rinch["cpl_tasks"], "cpl_products": rinch["cpl_products"]}
        for name, meth, kw in (("irsi", "refine", {}),
                               ("recursive_regular", "localized", {"refinement": lif.REFINE_NONLOCAL})):
            s_v, inf_v = time_method(lif, Sd, cfg["tau"], meth, args.rinch_steps, **kw)
            variants[name] = {"s_per_factorization": s_v, "lif_speedup": s_v / step_s,
                              "cpl_tasks": inf_v["cpl_tasks"], "cpl_products": inf_v["cpl_products"],
                              "iterations_top": inf_v["iterations_top"],
                              "iterations_total": inf_v["iterations_total"], "nnzb_Z": inf_v["nnzb_Z"]}
    rooflines = []
    if detail64:
        d = detail64
        lf, ls = sum(i["flops_leaf_factorization"] for i in d), sum(i["seconds_leaf_factorization"] for i in d)
        sb, ss = sum(i["bytes_symbolic"] for i in d), sum(i["seconds_symbolic"] for i in d)
        nl = sum(i["symbolic_launches"] for i in d)
        if ls > 0:
            rooflines.append({"kernel": "k_potrf + k_step + k_trinv (batched leaf inverse Cholesky, one interval per "
                                        "factorization: the serial steps with the inverse's columns beside them)",
                              "bound": "mfma", "achieved": lf / ls / 1e12, "peak": PEAK_FP64_MFMA_TFLOPS,
                              "unit": "TFLOP/s", "frac": lf / ls / 1e12 / PEAK_FP64_MFMA_TFLOPS,
                              "flops_per_factorization": lf / len(d), "seconds_per_factorization": ls / len(d)})
        if ss > 0:
            rooflines.append({"kernel": "k_symbolic_* + k_scan_pair* (symbolic phases of every product)",
                              "bound": "hbm", "achieved": sb / ss / 1e9, "peak": PEAK_HBM_BPS / 1e9, "unit": "GB/s",
                              "frac": sb / ss / PEAK_HBM_BPS, "bytes_per_factorization": sb / len(d),
                              "seconds_per_factorization": ss / len(d), "launches_per_factorization": nl / len(d)})
    water = None
    if not args.no_water:
        water = water_comparison(lif, args.water_count)
    out = {
        "metric": METRIC,
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"chain-{args.count}: helix of {args.count} residues x 20 s-Gaussians, n={S.n}, "
                               f"b=64, tau=1e-10, LIF to 4096-row inverse-Cholesky leaves, m=4, paper stop, FP64",
                   "n": S.n, "b": 64, "tau": cfg["tau"], "method": "lif", "precision": "fp64",
                   "parallelism": "single-gpu"},
        "leaf_gemm_gflops": flops / gemm_s / 1e9 if gemm_s > 0 else None,
        "leaf_gemm_seconds_per_step": gemm_s / args.steps,
        "leaf_gemm_flops_per_step": flops / args.steps,
        "residual": res,
        "residual_untruncated_S": res_u64,
        "delta_tracked": last["delta_tracked"],
        "iterations_top": last["iterations_top"],
        "levels": last["levels"],
        "iterations_total": last["iterations_total"],
        "nnzb_Z": last["nnzb_Z"],
        "products_per_step": last["products_total"],
        "iterations_redone": last.get("iterations_redone"),
        "mixed": mixed,
        "rinch": rinch,
        "variants": variants,
        "water": water,
        "rooflines_other_kernels": rooflines,
        "roofline": {"bound": "mfma", "kernel": "k_numeric_f64 (leaf GEMM, v_mfma_f64_16x16x4f64)",
                     "achieved": achieved, "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_MFMA_TFLOPS,
                     "flops_per_launch": flops / max(launches, 1),
                     "avg_launch_us": gemm_s / max(launches, 1) * 1e6,
                     "launches_per_step": launches / args.steps,
                     "traffic": traffic,
                     # two b x b FP64 operand blocks per block product: b / 8 flop per byte
                     "operand_bytes_per_launch": flops / max(launches, 1) / 8.0,
                     "traffic_GBps": (traffic / (gemm_s / max(launches, 1)) / 1e9
                                      if traffic and gemm_s > 0 else None),
                     "traffic_frac_of_hbm_peak": (traffic / (gemm_s / max(launches, 1)) / PEAK_HBM_BPS
                                                  if traffic and gemm_s > 0 else None)},
    }
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
