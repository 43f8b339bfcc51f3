#!/usr/bin/env python3
"""Benchmark: perturbative-triples energy E(T) of one LNO-sized domain on one
MI355X, in triples GFLOP/s.

One step is one full ltriples_energy call on the domain (operand layouts,
density-fitting integral builds, every occupied triplet of the four spin
blocks, FP64 energy epilogue and reductions), with the inputs resident in HBM.
The printed JSON line also carries:
  roofline      the triplet-contraction GEMM kernel against the matrix-core
                peak of its dtype, timed live with HIP events on the library's
                stream; traffic from the committed counter summary when it was
                taken on the current kernel source (else null)
  fp64_gpu      the same path in FP64 (the "plain FP64 GPU" baseline), timed
                on a stratified item sample and scaled to the whole domain;
                with --autotune 1 its tiles are tuned on that sample first
  parity        per-item values of the timed run against the FP64 CPU oracle
                on the CPU-baseline items, and against the FP64 GPU run
  cpu_baseline  the FP64 CPU oracle timed on the host on a small item sample
  backward      the adjoint pass (dE/dT1, dE/dT2, dE/dB, dE/df_ov, dE/deps)
                on the gradient workload (20,18,160,162,640), FP32 and FP64,
                with a sampled check against the oracle gradient

Other workloads (not the headline line): --workload large runs the largest
domain (60,58,500,502,2000); --workload batch runs the set of 64 uneven
domains through ltriples_energy_batched, eager and as a captured hipGraph
(first call with capture, then replays); --workload rhf runs a closed-shell
domain (40 occupied, 300 virtual, 1200 auxiliary) through
ltriples_energy_rhf; --workload naf times the natural-auxiliary-function
compression that produces B^Q.

Profiling aids (not headline measurements): --sample-items K restricts the
timed step to K sampled triplets per spin block, --prefix-items K to the
first K per block in the whole-domain order; --copy-calibration runs only a
plain 1 GiB device copy (for scaling HBM byte counters); --traffic-from
writes the HBM traffic summary from counter csv files (no GPU).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "(T) triples GFLOP/s & MFMA util vs plain FP64 GPU, at |ΔE(T)|≤1e-6 Eh"
# dense matrix-core peaks of MI355X (TFLOP/s)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "bf16": 2500.0}
# matrix-core products per algorithmic multiply-add
MFMA_PRODUCTS = {"fp64": 1, "fp32": 1, "bf16x3": 3, "bf16": 1}
GEMM_SOURCES = {"bf16x3": "lt_gemm_bf16.hip", "bf16": "lt_gemm_bf16.hip", "fp32": "lt_gemm.hip",
                "fp64": "lt_gemm.hip"}
TOL = {"fp64": 1e-11, "fp32": 1e-8, "bf16x3": 1e-6, "bf16": None}


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [p.get("num_threads", 0) for p in threadpool_info() if p.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count() or 1


def kernel_source_hash(precision):
    src = os.path.join(ROOT, "paper_2311_10048_amd", "csrc", GEMM_SOURCES[precision])
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def committed_traffic(precision, workload):
    """Per-launch HBM bytes of the contraction kernel from the committed
    counter summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{precision}_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash(precision):
        return None
    return t


def copy_calibration():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n, "launches": 3}), flush=True)


def library_gemm(steps):
    """Profiling aid: the vendor library's plain BF16 GEMM (torch.matmul, BF16
    output) on the contraction's average shape, for comparison with the
    triplet contraction kernel.  K = 2304 is three times the mean contraction
    depth of the LNO domain (767), i.e. the three BF16 products of one
    split multiply-add laid end to end; N = 362400 is four triplets' output
    columns of a mixed G launch."""
    import torch
    out = []
    for M, K, N in ((300, 2304, 362400), (320, 2304, 362400), (8192, 8192, 8192)):
        A = torch.randn(M, K, device="cuda", dtype=torch.bfloat16)
        B = torch.randn(K, N, device="cuda", dtype=torch.bfloat16).contiguous()
        C = torch.empty(M, N, device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            torch.matmul(A, B, out=C)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            torch.matmul(A, B, out=C)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        out.append({"M": M, "K": K, "N": N, "ms": round(ms, 4), "TFLOP/s": round(2.0 * M * N * K / ms / 1e9, 1)})
        del A, B, C
    print(json.dumps({"library_gemm_bf16": out}), flush=True)


def _csv_rows(path, kernel):
    import csv
    with open(path) as f:
        return [r for r in csv.DictReader(f) if kernel in r["Kernel_Name"]]


def traffic_from(pmc_dir, trace_csv, precision, workload, dst=None):
    """Write profiles/traffic_<precision>_<workload>.json from rocprofv3
    counter runs (fetch/write of the sampled bench, cfetch/cwrite of
    --copy-calibration, csv output under pmc_dir) and the kernel trace of the
    full bench (trace_csv).  Bytes per work-group are taken per launch grid
    from the sampled run, whose contraction launches have the full step's
    grids; each launch of the full step is priced at its grid's figure
    (launches whose grid the sample lacks at the sample's mean per
    work-group), scaled by the counters' reading of a plain device copy."""
    kern = "k_tgemm_bf16" if precision in ("bf16x3", "bf16") else "k_tgemm<"
    raw = {}
    for c in ("fetch", "write"):
        for r in _csv_rows(os.path.join(pmc_dir, f"{c}_counter_collection.csv"), kern):
            g = int(r["Grid_Size"])
            raw.setdefault(g, {"fetch": [], "write": []})[c].append(float(r["Counter_Value"]))
    cal = {}
    for c in ("fetch", "write"):
        v = [float(r["Counter_Value"]) for r in
             _csv_rows(os.path.join(pmc_dir, f"c{c}_counter_collection.csv"), "__amd_rocclr_copyBuffer")]
        cal[c] = (float(1 << 30) / 1024.0) / (sum(v) / len(v))
    per_wg = {g: {c: 1024.0 * cal[c] * (sum(v[c]) / len(v[c])) / (g / 256) for c in ("fetch", "write")}
              for g, v in raw.items()}
    wgs = sum(g / 256 * len(v["fetch"]) for g, v in raw.items())
    mean_wg = {c: sum(per_wg[g][c] * g / 256 * len(raw[g]["fetch"]) for g in raw) / wgs for c in ("fetch", "write")}
    trace = [int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y") or 1) * int(r.get("Grid_Size_Z") or 1)
             for r in _csv_rows(trace_csv, kern)]
    mix = {}
    tot = {"fetch": 0.0, "write": 0.0}
    for g in trace:
        mix[g] = mix.get(g, 0) + 1
        for c in ("fetch", "write"):
            tot[c] += (per_wg[g][c] if g in per_wg else mean_wg[c]) * (g / 256)
    n = len(trace)
    out = {
        "kernel": kern, "precision": precision, "workload": workload,
        "bytes_per_launch": (tot["fetch"] + tot["write"]) / n,
        "fetch_bytes_per_launch": tot["fetch"] / n, "write_bytes_per_launch": tot["write"] / n,
        "fetch_scale": round(cal["fetch"], 4), "write_scale": round(cal["write"], 4),
        "sampled_raw_KiB_per_launch_by_grid": {
            str(g): {"launches": len(v["fetch"]), "FETCH_SIZE": sum(v["fetch"]) / len(v["fetch"]),
                     "WRITE_SIZE": sum(v["write"]) / len(v["write"])} for g, v in sorted(raw.items())},
        "full_trace_launches_by_grid": {str(g): k for g, k in sorted(mix.items())},
        "unsampled_grid_launches": sum(k for g, k in mix.items() if g not in per_wg),
        "source_hash": kernel_source_hash(precision),
        "method": "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two rocprofv3 --pmc runs of bench.py on "
                  "sampled triplets (same launch grids as the full step), per work-group per grid, priced over "
                  "the full step's launches from its kernel trace, scaled by the counters' reading of a plain "
                  "1 GiB device copy (bench.py --copy-calibration)",
    }
    if dst is None:
        dst = os.path.join(ROOT, "profiles", f"traffic_{precision}_{workload}.json")
    with open(dst, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({"wrote": dst, "bytes_per_launch": out["bytes_per_launch"], "launches": n}))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "fp64", "bf16x3", "bf16"])
    ap.add_argument("--workload", default="lno",
                    choices=["tiny", "lno", "grad", "large", "batch", "rhf", "naf", "central", "latency",
                             "batch_rates", "groups"])
    ap.add_argument("--fp64-sample", type=int, default=24, help="items per block for the FP64 GPU comparison")
    ap.add_argument("--cpu-sample", type=int, default=3, help="items per block for the CPU oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--backward-fp64", action="store_true", help="also time the FP64 adjoint in the backward leg")
    ap.add_argument("--backward-bf16x3", action="store_true",
                    help="also time the BF16X3 adjoint (split-product recompute) in the backward leg")
    ap.add_argument("--autotune", type=int, default=1,
                    help="1: tile shapes of the contraction kernels tuned during the warmup step (results unchanged)")
    ap.add_argument("--sample-items", type=int, default=0, help="profiling aid: K sampled triplets per block")
    ap.add_argument("--prefix-items", type=int, default=0,
                    help="profiling aid: the first K triplets per block in the whole-domain order")
    ap.add_argument("--copy-calibration", action="store_true", help="profiling aid: plain 1 GiB device copy")
    ap.add_argument("--group-budget", type=float, default=0.0,
                    help="batch workload: launch-group budget in GiB (options.group_budget; 0 = no groups)")
    ap.add_argument("--library-gemm", action="store_true",
                    help="profiling aid: the library BF16 GEMM on the contraction's average shape")
    ap.add_argument("--traffic-from", nargs=2, metavar=("PMC_DIR", "TRACE_CSV"),
                    help="profiling aid (no GPU): write the HBM traffic summary from counter and trace csv files")
    args = ap.parse_args()
    if args.traffic_from:
        traffic_from(*args.traffic_from, args.precision, args.workload)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): "
              "the (T) energy of one domain is measured on a single MI355X; sharding across GPUs "
              "is a design note, not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2311_10048_amd as lt
    import synth

    lt.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.library_gemm:
        library_gemm(max(args.steps, 20))
        return
    if args.workload == "latency":
        run_latency(args, lt, synth, torch)
        return
    if args.workload == "batch":
        run_batch(args, lt, synth, torch)
        return
    if args.workload == "batch_rates":
        run_batch_rates(args, lt, synth, torch)
        return
    if args.workload == "groups":
        run_groups(args, lt, synth, torch)
        return
    if args.workload == "rhf":
        run_rhf(args, lt, synth, torch)
        return
    if args.workload == "naf":
        run_naf(args, lt, synth, torch)
        return
    if args.workload == "central":
        run_central(args, lt, synth, torch)
        return
    dev = torch.device("cuda:0")
    prec = lt.PRECISIONS[args.precision]

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    t0 = time.time()
    dom = synth.config_domain(args.workload)
    log(f"generated {args.workload} domain {dom.dims} in {time.time() - t0:.1f} s")
    tens = {k: torch.from_numpy(v).to(dev) for k, v in dom.arrays().items()}
    torch.cuda.synchronize()
    d = lt.make_domain(dom.dims, tens)
    step_items = None
    if args.sample_items > 0:
        step_items = synth.sample_items(dom.noa, dom.nob, args.sample_items, seed=99)
    elif args.prefix_items > 0:
        step_items = synth.first_items(dom.noa, dom.nob, args.prefix_items)
    ostep, _keep0 = lt.make_options(items=step_items)
    F_all, n_all = lt.ltriples_flops(d, ostep)
    ws = torch.empty(lt.ltriples_workspace_size(d, prec, ostep), dtype=torch.uint8, device=dev)
    e_items = torch.zeros(n_all, 3, dtype=torch.float64, device=dev)
    log(f"items {n_all}, algorithmic flops {F_all:.4e}, workspace {ws.numel() / 1e9:.1f} GB")

    def step():
        st = lt.Stats()
        e, parts = lt.ltriples_energy(tens, dom.dims, prec, items=step_items, e_items=e_items, workspace=ws,
                                      stats=st, autotune=bool(args.autotune))
        return e, parts, st

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    stats = []
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    tw = time.perf_counter()
    ev0.record()
    for k in range(args.steps):
        e, parts, st = step()
        stats.append(st)
        log(f"step {k + 1}/{args.steps}: {st.total_ms / 1e3:.2f} s")
    ev1.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - tw) * 1e3
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    E = float(e.item())
    parts = parts.cpu().numpy()
    value = F_all / (ms_per_step * 1e-3) / 1e9

    # roofline of the contraction kernel: the step's algorithmic flops F (the
    # block formulas over the full virtual cube) per launch over the launches'
    # average HIP-event duration (events on the library's stream); the flops
    # the kernel executes (2 M N K over the pair-packed outputs) give frac_executed
    gemm_ms = sum(s.triples_gemm_ms for s in stats)
    gemm_flops = sum(s.triples_gemm_flops for s in stats)
    launches = sum(s.triples_gemm_launches for s in stats)
    achieved_exec = gemm_flops / (gemm_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    avg_ms = gemm_ms / max(launches, 1)
    per_step = max(launches // max(len(stats), 1), 1)
    F_launch = F_all / per_step
    achieved = F_launch / (avg_ms * 1e-3) / 1e12
    traffic = None
    # the committed counter summary prices the whole-domain step only
    tr = committed_traffic(args.precision, args.workload) if step_items is None else None
    if tr is not None:
        traffic = tr["bytes_per_launch"]
    kname = "k_tgemm_bf16" if args.precision.startswith("bf16") else "k_tgemm"
    roofline = {"bound": "mfma", "kernel": f"{kname} (triplet contraction GEMM)",
                "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "avg_launch_ms": round(avg_ms, 4),
                "launches_per_step": per_step,
                "flops_per_launch": F_launch,
                "achieved_executed": round(achieved_exec, 2),
                "frac_executed": round(achieved_exec / peak, 4),
                "executed_flops_per_launch": gemm_flops / max(launches, 1),
                "kernel_source_hash": kernel_source_hash(args.precision)}
    # matrix-core utilisation counts every product the split performs
    mfma_util = MFMA_PRODUCTS[args.precision] * achieved_exec / peak
    phase = {"setup_ms": round(stats[-1].setup_ms, 2), "triples_gemm_ms": round(stats[-1].triples_gemm_ms, 2),
             "epilogue_ms": round(stats[-1].epilogue_ms, 2), "total_ms": round(stats[-1].total_ms, 2)}
    log(f"E = {E:.10e}  {ms_per_step / 1e3:.2f} s/step  {value:.1f} GFLOP/s  gemm {achieved:.1f} TFLOP/s (F)")

    full_items = step_items if step_items is not None else None

    def positions(items):
        if full_items is None:
            return _item_index(dom.noa, dom.nob, items)
        lut = {tuple(r): n for n, r in enumerate(np.asarray(full_items).reshape(-1, 4).tolist())}
        return np.asarray([lut[tuple(r)] for r in np.asarray(items).reshape(-1, 4).tolist()], dtype=np.int64)

    # ---- FP64 GPU path on a stratified sample, scaled to the domain -----------------------
    fp64 = None
    try:
        items64 = synth.sample_items(dom.noa, dom.nob, args.fp64_sample, seed=2311)
        if step_items is not None:
            items64 = step_items
        need64 = 0
        if args.fp64_sample > 0 and len(items64):
            o64, _keep = lt.make_options(items=items64)
            need64 = lt.ltriples_workspace_size(d, lt.LT_FP64, o64)
            del ws
            torch.cuda.empty_cache()
            if need64 > torch.cuda.mem_get_info(dev)[0] - (1 << 30):
                fp64 = {"skipped": f"FP64 workspace of {need64 / 1e9:.1f} GB does not fit beside the inputs"}
                log(fp64["skipped"])
        if args.fp64_sample > 0 and len(items64) and fp64 is None:
            F_s, n_s = lt.ltriples_flops(d, o64)
            ws64 = torch.empty(need64, dtype=torch.uint8, device=dev)
            ei64 = torch.zeros(n_s, 3, dtype=torch.float64, device=dev)
            tune64 = bool(args.autotune)
            if tune64:
                # the FP64 contraction gets its tiles tuned on the sample it is timed on, as the
                # step above had its own tuned in the warmup: an untimed tuning call first
                lt.ltriples_energy(tens, dom.dims, lt.LT_FP64, items=items64, e_items=ei64, workspace=ws64,
                                   autotune=True)
                torch.cuda.synchronize()
            st64 = lt.Stats()
            lt.ltriples_energy(tens, dom.dims, lt.LT_FP64, items=items64, e_items=ei64, workspace=ws64, stats=st64,
                               autotune=tune64)
            torch.cuda.synchronize()
            per_flop_ms = (st64.triples_gemm_ms + st64.epilogue_ms) / F_s
            est_ms = st64.setup_ms + per_flop_ms * F_all
            mine = e_items.cpu().numpy()[positions(items64)]
            ref64 = ei64.cpu().numpy()
            s_mine, s_ref = mine.sum(), ref64.sum()
            fp64 = {"sample_items": int(n_s), "sample_ms": round(st64.total_ms, 2),
                    "est_full_s": round(est_ms / 1e3, 2), "speedup_vs_fp64": round(est_ms / ms_per_step, 3),
                    "sample_rel_diff_vs_fp64": float(abs(s_mine - s_ref) / max(1.0, abs(s_ref))),
                    "gemm_tflops": round(st64.triples_gemm_flops / (st64.triples_gemm_ms * 1e-3) / 1e12, 2),
                    "tiles": "tuned" if tune64 else "default"}
            log(f"fp64 sample: est {est_ms / 1e3:.1f} s for the domain, speedup {est_ms / ms_per_step:.2f}x")
            del ws64
    except Exception as ex:   # a failed side leg must not lose the measured step
        fp64 = {"error": f"{type(ex).__name__}: {ex}"}
        log(f"fp64 leg failed: {ex}")

    # ---- CPU oracle baseline + parity on its items ------------------------------------------
    cpu = None
    parity = None
    try:
        if not args.no_cpu_baseline and args.cpu_sample > 0:
            from oracle import blocks
            itc = synth.sample_items(dom.noa, dom.nob, args.cpu_sample, seed=11)
            if step_items is not None:
                itc = step_items[:4]
            oc, _k2 = lt.make_options(items=itc)
            F_c, n_c = lt.ltriples_flops(d, oc)
            tc = time.perf_counter()
            ref = blocks.energy(dom, items=itc, return_items=True)
            dt = time.perf_counter() - tc
            cpu = {"value": round(F_c / dt / 1e9, 3), "unit": "GFLOP/s", "cores": _blas_threads(), "kind": "oracle",
                   "sample": f"{n_c} occupied triplets ({args.cpu_sample} per spin block) of the same domain, "
                             f"{F_c:.3e} flops in {dt:.1f} s, NumPy FP64",
                   "seconds": round(dt, 2), "est_full_domain_s": round(dt * F_all / F_c, 1),
                   "cpu_model": _cpu_model(), "single_thread": _single_thread_tiny(lt, synth),
                   "single_thread_grad": _single_thread_grad(lt, synth)}
            g = e_items.cpu().numpy()[positions(itc)]
            r = ref["items"]
            tot = np.abs(g.sum(axis=1) - r.sum(axis=1)) / np.maximum(1.0, np.abs(r.sum(axis=1)))
            tol = TOL[args.precision]
            parity = {"oracle_items": int(n_c), "max_rel_err_item_E": float(tot.max()), "tolerance": tol,
                      "pass": None if tol is None else bool(tot.max() <= tol)}
            log(f"cpu oracle {dt:.1f} s for {n_c} items; max item rel err {tot.max():.2e}")
    except Exception as ex:   # a failed side leg must not lose the measured step
        cpu = {"error": f"{type(ex).__name__}: {ex}"}
        log(f"cpu-baseline leg failed: {ex}")

    backward = None
    try:
        if not args.no_backward and step_items is None:
            backward = run_backward(lt, synth, torch, log, fp64=args.backward_fp64, bf16x3=args.backward_bf16x3)
    except Exception as ex:   # a failed side leg must not lose the measured step
        backward = {"error": f"{type(ex).__name__}: {ex}"}
        log(f"backward leg failed: {ex}")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": f"{args.workload} domain: noa={dom.noa} nob={dom.nob} nva={dom.nva} "
                               f"nvb={dom.nvb} naux={dom.naux}, "
                               + (f"all {n_all} occupied triplets" if step_items is None
                                  else f"{n_all} {'sampled' if args.sample_items > 0 else 'leading'} triplets (profiling run)"),
                   "algorithmic_flops": F_all, "precision": args.precision,
                   "wall_ms_per_step": round(wall_ms / args.steps, 2)},
        "E": E,
        "parts": parts.tolist(),
        "phases": phase,
        "roofline": roofline,
        "mfma_util": round(mfma_util, 4),
        "fp64_gpu": fp64,
        "parity": parity,
        "cpu_baseline": cpu,
        "backward": backward,
    }
    print(json.dumps(out), flush=True)


def run_batch(args, lt, synth, torch):
    """The 64 uneven domains through ltriples_energy_batched, as two calls of
    32 domains (even- and odd-indexed, so the halves carry similar work): eager
    steps, then the graph path (the first call of each half captures its
    launch sequence and runs it; later calls replay it).  Inputs are generated
    and copied to the device one domain at a time."""
    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    prec = lt.PRECISIONS[args.precision]
    shapes = synth.batch_shapes()
    t0 = time.time()
    tens, dims, F = [], [], []
    for n in range(len(shapes)):
        dom = synth.batch_domain(n, shapes)
        tens.append({k: torch.from_numpy(v).cuda() for k, v in dom.arrays().items()})
        dims.append(dom.dims)
        F.append(lt.ltriples_flops(lt.make_domain(dom.dims, tens[-1]), None)[0])
        del dom
    torch.cuda.synchronize()
    halves = [list(range(0, len(shapes), 2)), list(range(1, len(shapes), 2))]
    Ftot = sum(F)
    log(f"generated and uploaded {len(shapes)} domains in {time.time() - t0:.1f} s, F = {Ftot:.4e}")
    gbudget = int(args.group_budget * (1 << 30))
    opts, _ = lt.make_options(group_budget=gbudget)
    need = max(lt.ltriples_workspace_size_batched([dims[n] for n in h], [tens[n] for n in h], prec, opts)
               for h in halves)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    outs = [(torch.empty(len(h), dtype=torch.float64, device="cuda"),
             torch.empty(len(h), 4, 3, dtype=torch.float64, device="cuda")) for h in halves]
    log(f"workspace {need / 1e9:.1f} GB (shared by the two halves)")

    def step(graph, label):
        ms = 0.0
        for k, h in enumerate(halves):
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record()
            lt.ltriples_energy_batched([tens[n] for n in h], [dims[n] for n in h], prec, graph=graph,
                                       workspace=ws, out=outs[k], autotune=bool(args.autotune) and not graph,
                                       group_budget=gbudget)
            ev1.record()
            torch.cuda.synchronize()
            ms += ev0.elapsed_time(ev1)
            log(f"{label}: half {k + 1}/2 done ({ev0.elapsed_time(ev1) / 1e3:.2f} s)")
        e = np.zeros(len(shapes))
        for k, h in enumerate(halves):
            e[h] = outs[k][0].cpu().numpy()
        return ms, e

    for w in range(args.warmup):
        step(False, f"warmup {w + 1}")
    eager = [step(False, f"eager step {k + 1}") for k in range(args.steps)]
    lt.ltriples_graph_reset()
    first = step(True, "graph first call")
    replays = [step(True, f"graph replay {k + 1}") for k in range(args.steps)]
    lt.ltriples_graph_reset()
    e_eager, e_graph = eager[-1][1], replays[-1][1]
    same = bool(np.array_equal(e_eager, e_graph)) and bool(np.array_equal(e_eager, first[1]))
    ms = sum(x[0] for x in eager) / len(eager)
    rms = sum(x[0] for x in replays) / len(replays)
    log(f"eager {ms / 1e3:.2f} s, graph first call {first[0] / 1e3:.2f} s, replay {rms / 1e3:.2f} s, "
        f"graph == eager: {same}")
    res = {
        "metric": METRIC, "value": round(Ftot / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"batch: {len(dims)} uneven domains (nocc 10-40, nvir 80-320, naux 4 nvir), "
                               "two ltriples_energy_batched calls of 32 domains per step",
                   "algorithmic_flops": Ftot, "precision": args.precision,
                   "group_budget_GiB": args.group_budget, "workspace_GB": round(need / 1e9, 2)},
        "graph": {"first_call_ms": round(first[0], 2), "replay_ms": round(rms, 2),
                  "replay_GFLOP/s": round(Ftot / (rms * 1e-3) / 1e9, 1), "bitwise_equal_to_eager": same},
        "E_per_domain": [float(x) for x in e_eager],
    }
    print(json.dumps(res), flush=True)


def run_batch_rates(args, lt, synth, torch):
    """Where the 64-domain set loses against one large domain: eleven of its
    domains, spread over the virtual sizes (smallest to largest nva), each
    timed alone through ltriples_energy with phase statistics (setup,
    contractions, epilogues); one untimed call first.  Prints one JSON line
    per domain and a summary line."""
    prec = lt.PRECISIONS[args.precision]
    shapes = synth.batch_shapes()
    order = sorted(range(len(shapes)), key=lambda n: shapes[n][2])
    pick = [order[i] for i in (0, 1, 8, 16, 24, 32, 40, 48, 56, 62, 63)]
    out = []
    for n in pick:
        dom = synth.batch_domain(n, shapes)
        t = {k: torch.from_numpy(v).cuda() for k, v in dom.arrays().items()}
        F = lt.ltriples_flops(lt.make_domain(dom.dims, t), None)[0]
        for _ in range(max(args.warmup, 1) + 1):
            st = lt.Stats()
            lt.ltriples_energy(t, dom.dims, prec, stats=st)
            torch.cuda.synchronize()
        s = st.as_dict()
        row = {"domain": n, "dims": list(dom.dims), "F": F, "total_ms": round(s["total_ms"], 2),
               "setup_ms": round(s["setup_ms"], 2), "contraction_ms": round(s["triples_gemm_ms"], 2),
               "epilogue_ms": round(s["epilogue_ms"], 2), "contraction_launches": s["triples_gemm_launches"],
               "TFLOP/s": round(F / s["total_ms"] / 1e9, 1),
               "contraction_TFLOP/s_on_F": round(F / max(s["triples_gemm_ms"], 1e-9) / 1e9, 1)}
        out.append(row)
        print(json.dumps(row), flush=True)
        del t, dom
        torch.cuda.empty_cache()
    print(json.dumps({"workload": "batch_rates", "precision": args.precision, "domains": len(out)}), flush=True)


def run_groups(args, lt, synth, torch):
    """Launch groups (options.group_budget) against domains one after
    another, on three sets of small domains where launches are smallest: 64
    tiny domains (4-8 occupied, 20-60 virtual), 32 small ones (8-14, 60-120)
    and the 16 smallest domains of the 64-domain set; eager and graph-replayed
    calls with a preallocated workspace, energies compared bitwise."""
    prec = lt.PRECISIONS[args.precision]
    rng = np.random.default_rng(11)
    sets = {}
    no, nv = rng.integers(4, 9, 64), rng.integers(20, 61, 64)
    sets["64 tiny domains (4-8 occupied, 20-60 virtual)"] = [
        (int(a), int(a) - 1, int(v), int(v) + 1, 3 * int(v)) for a, v in zip(no, nv)]
    no, nv = rng.integers(8, 15, 32), rng.integers(60, 121, 32)
    sets["32 small domains (8-14 occupied, 60-120 virtual)"] = [
        (int(a), int(a) - 1, int(v), int(v) + 1, 4 * int(v)) for a, v in zip(no, nv)]
    shapes = synth.batch_shapes()
    F = sorted((lt.ltriples_flops(lt.make_domain(s, {f: (1 << 40) for f in lt.ARRAY_FIELDS}))[0], n)
               for n, s in enumerate(shapes))
    sets["the 16 smallest domains of the 64-domain set"] = [shapes[n] for _, n in F[:16]]
    reps = max(args.steps, 5)
    for name, sh in sets.items():
        doms = [synth.make_domain(*s, seed=synth.BASE_SEED + 900 + k) for k, s in enumerate(sh)]
        tens = [{k: torch.from_numpy(v).cuda() for k, v in d.arrays().items()} for d in doms]
        dims = [d.dims for d in doms]
        Ft = sum(lt.ltriples_flops(lt.make_domain(d, t))[0] for d, t in zip(dims, tens))
        res, energies = {}, []
        for budget in (0, 1 << 50):
            opts, _ = lt.make_options(group_budget=budget)
            ws = torch.empty(lt.ltriples_workspace_size_batched(dims, tens, prec, opts), dtype=torch.uint8,
                             device="cuda")
            out = (torch.empty(len(dims), dtype=torch.float64, device="cuda"),
                   torch.empty(len(dims), 4, 3, dtype=torch.float64, device="cuda"))
            for graph in (False, True):
                lt.ltriples_graph_reset()
                for _ in range(2):
                    lt.ltriples_energy_batched(tens, dims, prec, graph=graph, workspace=ws, out=out,
                                               group_budget=budget)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    lt.ltriples_energy_batched(tens, dims, prec, graph=graph, workspace=ws, out=out,
                                               group_budget=budget)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                energies.append(out[0].cpu().numpy().copy())
                key = ("groups" if budget else "one after another") + (", graph" if graph else ", eager")
                res[key] = {"ms": round(ms, 2), "TFLOP/s": round(Ft / ms / 1e9, 1)}
            lt.ltriples_graph_reset()
            res["workspace_GB " + ("groups" if budget else "one after another")] = round(ws.numel() / 1e9, 2)
            del ws
        same = all(np.array_equal(energies[0], e) for e in energies)
        print(json.dumps({"set": name, "domains": len(dims), "F": Ft, "precision": args.precision, **res,
                          "bitwise_equal": same}), flush=True)
        del tens, doms
        torch.cuda.empty_cache()


def run_latency(args, lt, synth, torch):
    """Call latency on the small domain (5,4,30,31,120): eager single-domain
    calls against replays of the same launch sequence captured in a hipGraph
    (a one-domain ltriples_energy_batched call with options.graph), both
    with a preallocated workspace; energies compared bitwise."""

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    prec = lt.PRECISIONS[args.precision]
    dom = synth.config_domain("tiny")
    tens = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in dom.arrays().items()}
    d = lt.make_domain(dom.dims, tens)
    ws = torch.empty(max(lt.ltriples_workspace_size(d, prec), 1), dtype=torch.uint8, device=dev)
    n = max(args.steps, 50)

    def timed(fn):
        for _ in range(max(args.warmup, 3)):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(n):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) * 1e3 / n, r

    ms_eager, (e0, _) = timed(lambda: lt.ltriples_energy(tens, dom.dims, prec, workspace=ws))
    lt.ltriples_graph_reset()
    import ctypes
    arr = lt._domain_array([dom.dims], [tens])
    opts, _k = lt.make_options()
    opts.graph = 1
    sz = ctypes.c_size_t(0)
    lt._check(lt.load_library().ltriples_workspace_size_batched(arr, 1, prec, ctypes.byref(opts), ctypes.byref(sz)))
    wsb = torch.empty(max(sz.value, 1), dtype=torch.uint8, device=dev)
    out = (torch.empty(1, dtype=torch.float64, device=dev), torch.empty(1, 4, 3, dtype=torch.float64, device=dev))
    ms_graph, (e1, _) = timed(lambda: lt.ltriples_energy_batched([tens], [dom.dims], prec, graph=True,
                                                                 workspace=wsb, out=out))
    same = float(e0.item()) == float(e1[0].item())
    log(f"tiny {dom.dims}: eager {ms_eager:.3f} ms per call, graph replay {ms_graph:.3f} ms, same E: {same}")
    print(json.dumps({"workload": f"tiny domain {dom.dims}, call latency", "precision": args.precision,
                      "calls": n, "eager_ms_per_call": round(ms_eager, 4),
                      "graph_replay_ms_per_call": round(ms_graph, 4), "bitwise_equal": same}), flush=True)


def run_rhf(args, lt, synth, torch):
    """Closed-shell (SOMO-free) LNO-sized domain through ltriples_energy_rhf
    (spin-adapted); parity and CPU baseline on sampled aaa/aab triplets of the
    same data through the open-shell entry point and the oracle."""
    from oracle import blocks

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    prec = lt.PRECISIONS[args.precision]
    t0 = time.time()
    dom = synth.rhf_config_domain("rhf")
    dims = (dom.noa, dom.nva, dom.naux)
    log(f"generated rhf domain (no, nv, naux) = {dims} in {time.time() - t0:.1f} s")
    tens = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in synth.rhf_arrays(dom).items()}
    rd = lt.make_rhf_domain(dims, tens)
    F, n = lt.ltriples_rhf_flops(rd)
    # the same energy through the spin-block form (E = 2 E_aaa + 2 E_aab) costs the
    # open-shell count of the alpha == beta domain over its aaa and aab blocks
    dfake = lt.make_domain((dom.noa, dom.noa, dom.nva, dom.nva, dom.naux), {k: (1 << 40) for k in lt.ARRAY_FIELDS})
    F_sb = 0.5 * lt.ltriples_flops(dfake)[0]
    ws = torch.empty(lt.ltriples_rhf_workspace_size(rd, prec), dtype=torch.uint8, device=dev)
    log(f"items {n}, algorithmic flops {F:.4e}, workspace {ws.numel() / 1e9:.1f} GB")

    def step():
        st = lt.Stats()
        e, parts = lt.ltriples_energy_rhf(tens, dims, prec, workspace=ws, stats=st)
        return e, parts, st

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    stats = []
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for k in range(args.steps):
        e, parts, st = step()
        stats.append(st)
        log(f"step {k + 1}/{args.steps}: {st.total_ms / 1e3:.2f} s")
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    E = float(e.item())
    gemm_ms = sum(x.triples_gemm_ms for x in stats)
    gemm_flops = sum(x.triples_gemm_flops for x in stats)
    launches = sum(x.triples_gemm_launches for x in stats)
    achieved = gemm_flops / (gemm_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    kname = "k_tgemm_bf16" if args.precision.startswith("bf16") else "k_tgemm"
    roofline = {"bound": "mfma", "kernel": f"{kname} (triplet contraction GEMM)", "achieved": round(achieved, 2),
                "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                "avg_launch_ms": round(gemm_ms / max(launches, 1), 4),
                "launches_per_step": launches // max(len(stats), 1),
                "flops_per_launch": gemm_flops / max(launches, 1),
                "kernel_source_hash": kernel_source_hash(args.precision)}
    log(f"E = {E:.10e}  {ms / 1e3:.2f} s/step  {F / (ms * 1e-3) / 1e9:.1f} GFLOP/s  gemm {achieved:.1f} TFLOP/s")
    del ws
    torch.cuda.empty_cache()

    # sampled aaa and aab triplets of the same data: GPU spin-block path vs the oracle
    parity = cpu = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        items = [r for r in synth.sample_items(dom.noa, dom.nob, args.cpu_sample, seed=11).tolist() if r[0] in (0, 1)]
        full = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in dom.arrays().items()}
        ei = torch.zeros(len(items), 3, dtype=torch.float64, device=dev)
        lt.ltriples_energy(full, dom.dims, prec, items=items, e_items=ei)
        torch.cuda.synchronize()
        d = lt.make_domain(dom.dims, full)
        oc, _k = lt.make_options(items=items)
        F_c, n_c = lt.ltriples_flops(d, oc)
        tc = time.perf_counter()
        ref = blocks.energy(dom, items=items, return_items=True)
        dt = time.perf_counter() - tc
        g = ei.cpu().numpy()
        r = ref["items"]
        err = np.abs(g.sum(axis=1) - r.sum(axis=1)) / np.maximum(1.0, np.abs(r.sum(axis=1)))
        tol = TOL[args.precision]
        parity = {"oracle_items": int(n_c), "max_rel_err_item_E": float(err.max()), "tolerance": tol,
                  "pass": None if tol is None else bool(err.max() <= tol)}
        cpu = {"value": round(F_c / dt / 1e9, 3), "unit": "GFLOP/s", "cores": _blas_threads(), "kind": "oracle",
               "sample": f"{n_c} aaa/aab triplets of the same closed-shell data, {F_c:.3e} flops in {dt:.1f} s, "
                         "NumPy FP64", "seconds": round(dt, 2)}
        log(f"cpu oracle {dt:.1f} s for {n_c} items; max item rel err {err.max():.2e}")
    out = {
        "metric": METRIC, "value": round(F / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": f"rhf domain (closed shell, spin-adapted): no={dom.noa} nv={dom.nva} "
                               f"naux={dom.naux}, all {n} unordered occupied triples i<=j<=k",
                   "algorithmic_flops": F, "precision": args.precision,
                   "spin_block_flops": F_sb,
                   "spin_block_flops_per_s": round(F_sb / (ms * 1e-3) / 1e9, 1)},
        "E": E, "parts": parts.cpu().numpy().tolist(), "roofline": roofline,
        "mfma_util": round(MFMA_PRODUCTS[args.precision] * achieved / peak, 4),
        "parity": parity, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_naf(args, lt, synth, torch):
    """Natural-auxiliary-function step of an LNO-sized domain: 340 orbitals
    per spin (40+300 and 38+302), 2400 auxiliary functions with a decaying
    spectrum, eps 1e-2.  The oracle runs the same input on the host as the
    CPU baseline and parity reference."""
    from oracle import naf

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    shape, eps = (40, 300, 38, 302, 2400), 1e-2
    t0 = time.time()
    Ja, Jb = synth.make_naf_input(*shape, seed=synth.BASE_SEED + 6000, decay=250.0, rotate=False)
    log(f"generated NAF input {shape} in {time.time() - t0:.1f} s")
    ta, tb = torch.from_numpy(Ja).to(dev), torch.from_numpy(Jb).to(dev)
    inp = lt.make_naf_input(shape, ta, tb)
    ws = torch.empty(lt.ltriples_naf_workspace_size(inp), dtype=torch.uint8, device=dev)
    for w in range(args.warmup):
        lt.ltriples_naf(ta, tb, shape, eps, workspace=ws)
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    times = []
    for k in range(args.steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        m, out = lt.ltriples_naf(ta, tb, shape, eps, workspace=ws)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t) * 1e3)
        log(f"step {k + 1}/{args.steps}: {times[-1]:.1f} ms, {m} NAFs kept")
    ms = sum(times) / len(times)
    na, nb, nx = shape[0] + shape[1], shape[2] + shape[3], shape[4]
    # W build (pairs p <= q, both spins) and the two factor GEMMs, 2 flops per multiply-add
    flops = 2.0 * nx * nx * (na * (na + 1) / 2 + nb * (nb + 1) / 2) + 2.0 * m * nx * (na * na + nb * nb)
    parity = cpu = None
    if not args.no_cpu_baseline:
        tc = time.perf_counter()
        lam, U, m_ref, Bref = naf.naf(Ja, Jb, eps)
        dt = time.perf_counter() - tc
        ev = out["eigenvalues"].cpu().numpy()
        rng = np.random.default_rng(3)
        idx = rng.choice(na * na, size=200, replace=False)
        # (pq|rs) on sampled pairs of spin a, from the full [m][n][n] factors
        full = np.zeros((m, na, na))
        o = shape[0]
        full[:, :o, :o] = out["Boo_a"].cpu().numpy()
        full[:, :o, o:] = out["Bov_a"].cpu().numpy()
        full[:, o:, :o] = full[:, :o, o:].transpose(0, 2, 1)
        full[:, o:, o:] = out["Bvv_a"].cpu().numpy()
        Xg = full.reshape(m, -1)[:, idx]
        Xr = Bref[0].reshape(m_ref, -1)[:, idx]
        gerr = float(np.max(np.abs(Xg.T @ Xg - Xr.T @ Xr)) / np.max(np.abs(Xr.T @ Xr)))
        parity = {"naux_gpu": int(m), "naux_oracle": int(m_ref),
                  "max_rel_err_eigenvalues": float(np.max(np.abs(ev - lam)) / abs(lam[0])),
                  "max_rel_err_sampled_integrals": gerr,
                  "pass": bool(m == m_ref and gerr <= 1e-12)}
        cpu = {"value": round(dt * 1e3, 1), "unit": "ms", "cores": _blas_threads(), "kind": "oracle",
               "sample": "the whole input (NumPy FP64: W over p <= q pairs, eigh, factors)"}
        log(f"oracle {dt:.1f} s; naux {m} vs {m_ref}; integrals {gerr:.2e}")
    res = {"metric": "natural-auxiliary-function step time", "value": round(ms, 2), "unit": "ms", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": False,
           "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"NAF of an LNO-sized domain: {na} + {nb} orbitals, {nx} auxiliary functions, "
                                  f"eps {eps}, {m} kept", "flops": flops},
           "achieved_TFLOP/s": round(flops / (ms * 1e-3) / 1e12, 2), "parity": parity, "cpu_baseline": cpu}
    print(json.dumps(res), flush=True)


def run_backward(lt, synth, torch, log, fp64=False, bf16x3=False):
    """Adjoint pass on the gradient workload: FP32 (timed after one warmup),
    with bf16x3 the BF16X3 adjoint (split-product recompute, FP32 reverse
    GEMMs; timed after one warmup) and with fp64 FP64; 3F / t in GFLOP/s;
    sampled items against the oracle gradient in every precision run."""
    from oracle import grad as ograd
    dom = synth.config_domain("grad")
    tens = {k: torch.from_numpy(v).cuda() for k, v in dom.arrays().items()}
    d = lt.make_domain(dom.dims, tens)
    F, n = lt.ltriples_flops(d)
    res = {"workload": f"grad domain: noa={dom.noa} nob={dom.nob} nva={dom.nva} nvb={dom.nvb} naux={dom.naux}, "
                       f"all {n} occupied triplets", "algorithmic_flops_3F": 3 * F}
    legs = [("fp32", lt.LT_FP32)] + ([("bf16x3", lt.LT_BF16X3)] if bf16x3 else []) \
        + ([("fp64", lt.LT_FP64)] if fp64 else [])
    for name, prec in legs:
        ws = torch.empty(lt.ltriples_backward_workspace_size(d, prec), dtype=torch.uint8, device="cuda")
        reps = 1 if name == "fp64" else 2
        for r in range(reps):
            st = lt.Stats()
            g = lt.ltriples_backward(tens, dom.dims, prec, workspace=ws, stats=st)
            torch.cuda.synchronize()
        res[name] = {"ms": round(st.total_ms, 1), "GFLOP/s": round(3 * F / (st.total_ms * 1e-3) / 1e9, 1),
                     "gemm_ms": round(st.triples_gemm_ms, 1), "epilogue_ms": round(st.epilogue_ms, 1)}
        log(f"backward {name}: {st.total_ms / 1e3:.2f} s")
        del ws, g
    items = synth.sample_items(dom.noa, dom.nob, 1, seed=77)
    tc = time.perf_counter()
    _, ref = ograd.energy_and_grad(dom, items=items, fock=True)
    dt = time.perf_counter() - tc
    err = {}
    for name, prec in (("fp32", lt.LT_FP32), ("fp64", lt.LT_FP64)) + ((("bf16x3", lt.LT_BF16X3),) if bf16x3 else ()):
        g = lt.ltriples_backward(tens, dom.dims, prec, items=items)
        torch.cuda.synchronize()
        worst = 0.0
        for k in lt.GRAD_FIELDS + lt.FOCK_GRAD_FIELDS:
            r = ref[k]
            if r.size:
                worst = max(worst, float(np.max(np.abs(g[k].cpu().numpy() - r)) / np.max(np.abs(r))))
        err[name] = worst
    res["parity"] = {"oracle_items": int(len(items)), "max_rel_err_fp64": err["fp64"], "tol_fp64": 1e-10,
                     "max_rel_err_fp32": err["fp32"], "tol_fp32": 1e-5,
                     "pass": bool(err["fp64"] <= 1e-10 and err["fp32"] <= 1e-5
                                  and err.get("bf16x3", 0.0) <= 1e-5), "oracle_seconds": round(dt, 1)}
    if bf16x3:
        res["parity"].update({"max_rel_err_bf16x3": err["bf16x3"], "tol_bf16x3": 1e-5})
    log("backward parity: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()))
    return res


def _cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or the platform string."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def _single_thread_grad(lt, synth):
    """The oracle's energy with one BLAS thread on a bounded sample of the
    gradient domain (20,18,160,162,640): one triplet per spin block, with the
    rate scaled to the whole domain's algorithmic count."""
    from oracle import blocks
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        return None
    dom = synth.config_domain("grad")
    fake = lt.make_domain(dom.dims, {k: (1 << 40) for k in lt.ARRAY_FIELDS})
    items = synth.sample_items(dom.noa, dom.nob, 1, seed=31)
    F_s = lt.ltriples_flops(fake, lt.make_options(items=items)[0])[0]
    F = lt.ltriples_flops(fake)[0]
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        blocks.energy(dom, items=items)
        dt = time.perf_counter() - t
    return {"workload": f"grad domain {dom.dims}, {len(items)} triplets (one per spin block)", "threads": 1,
            "seconds": round(dt, 3), "GFLOP/s": round(F_s / dt / 1e9, 3),
            "est_full_domain_s": round(dt * F / F_s, 1)}


def _single_thread_tiny(lt, synth):
    """The oracle on the whole small domain (5,4,30,31,120) with one BLAS
    thread: seconds and GFLOP/s of the algorithmic count."""
    from oracle import blocks
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        return None
    dom = synth.config_domain("tiny")
    F = lt.ltriples_flops(lt.make_domain(dom.dims, {k: (1 << 40) for k in lt.ARRAY_FIELDS}))[0]
    with threadpool_limits(limits=1):
        blocks.energy(dom)                    # warm caches and imports
        t = time.perf_counter()
        blocks.energy(dom)
        dt = time.perf_counter() - t
    return {"workload": f"tiny domain {dom.dims}, all triplets", "threads": 1, "seconds": round(dt, 3),
            "GFLOP/s": round(F / dt / 1e9, 3)}


def run_central(args, lt, synth, torch):
    """The (T) share of one central orbital of the LNO-sized domain
    (eq. local_pt): an alpha orbital given as a seeded unit vector over the
    domain's occupied alpha orbitals, with a seeded four-point Laplace
    quadrature (the cost does not depend on the points).  Parity: the same
    share through the FP64 GPU path (which the GPU tests hold to the oracle at
    1e-11 on smaller domains); CPU baseline: the oracle on a restricted
    central vector (one nonzero coefficient) of the small domain."""
    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    prec = lt.PRECISIONS[args.precision]
    dom = synth.config_domain("lno")
    tens = {k: torch.from_numpy(v).to(dev) for k, v in dom.arrays().items()}
    c, s, w = synth.central_inputs(dom.noa, 4, seed=synth.BASE_SEED + 7000)
    cd = torch.from_numpy(c).to(dev)
    d = lt.make_domain(dom.dims, tens)
    cen, keepq = lt.make_central(0, cd, s, w)
    ws = torch.empty(lt.ltriples_central_workspace_size(d, cen, prec), dtype=torch.uint8, device=dev)
    log(f"central share of lno {dom.dims}: workspace {ws.numel() / 1e9:.1f} GB")

    def step():
        st = lt.Stats()
        e, parts = lt.ltriples_energy_central(tens, dom.dims, 0, cd, s, w, prec, workspace=ws, stats=st,
                                              autotune=bool(args.autotune))
        return e, parts, st

    for k in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {k + 1}/{args.warmup} done")
    stats = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for k in range(args.steps):
        e, parts, st = step()
        stats.append(st)
        log(f"step {k + 1}/{args.steps}: {st.total_ms / 1e3:.3f} s")
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    E = float(e.item())
    F = stats[-1].algorithmic_flops
    gemm_ms = sum(x.triples_gemm_ms for x in stats)
    launches = sum(x.triples_gemm_launches for x in stats)
    per_step = max(launches // len(stats), 1)
    avg = gemm_ms / max(launches, 1)
    achieved = F / per_step / (avg * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.precision]
    del ws
    torch.cuda.empty_cache()
    ref = None
    if prec != lt.LT_FP64:
        e64, _ = lt.ltriples_energy_central(tens, dom.dims, 0, cd, s, w, lt.LT_FP64)
        torch.cuda.synchronize()
        ref = float(e64.item())
    tol = TOL[args.precision]
    parity = None if ref is None else {"fp64_gpu": ref, "rel_err": abs(E - ref) / max(1.0, abs(ref)),
                                       "tolerance": tol, "pass": None if tol is None else
                                       bool(abs(E - ref) / max(1.0, abs(ref)) <= tol)}
    out = {"metric": METRIC, "value": round(F / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True,
           "scaling": "strong", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
           "config": {"workload": f"central-orbital share of the lno domain {dom.dims}: alpha central orbital, "
                                  f"4 Laplace points, {stats[-1].n_items} triplets", "algorithmic_flops": F,
                      "precision": args.precision},
           "E": E, "parts": parts.cpu().numpy().tolist(),
           "roofline": {"bound": "mfma", "kernel": "k_tgemm_bf16" if args.precision.startswith("bf16") else "k_tgemm",
                        "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                        "frac": round(achieved / peak, 4), "traffic": None, "avg_launch_ms": round(avg, 4),
                        "launches_per_step": per_step},
           "phases": {"setup_ms": round(stats[-1].setup_ms, 2), "triples_gemm_ms": round(stats[-1].triples_gemm_ms, 2),
                      "epilogue_ms": round(stats[-1].epilogue_ms, 2)},
           "parity": parity}
    print(json.dumps(out), flush=True)


def _item_index(noa, nob, items):
    """Positions of (block, p, q, r) items in the library's full enumeration
    order (block, then lexicographic)."""
    c0 = noa * (noa - 1) * (noa - 2) // 6
    c1 = noa * (noa - 1) // 2 * nob
    c2 = nob * (nob - 1) // 2 * noa
    base = [0, c0, c0 + c1, c0 + c1 + c2]
    idx = []
    for b, p, q, r in np.asarray(items).reshape(-1, 4):
        if b in (0, 3):
            n = nob if b == 3 else noa
            k = 0
            for i in range(p):
                k += (n - 1 - i) * (n - 2 - i) // 2
            for j in range(p + 1, q):
                k += n - 1 - j
            k += r - q - 1
        else:
            n = noa if b == 1 else nob
            m = nob if b == 1 else noa
            k = 0
            for i in range(p):
                k += (n - 1 - i) * m
            k += (q - p - 1) * m + r
        idx.append(base[b] + k)
    return np.asarray(idx, dtype=np.int64)


if __name__ == "__main__":
    main()
