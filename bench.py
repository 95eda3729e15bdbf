"""Benchmark of the GLS grid on one MI355X.

A step is one pass of the whole hot path over the precision-study workload
(n = 1000 samples, p = 4, m = 1,000,000 SNPs, t = 1,000 traits, synthetic data
drawn by `synth`; the largest of the paper-shaped grids that stays resident on
one GPU): rotation of every SNP by Z^T (genotype bytes on the int8 MFMAs
against Z in int8 digits, exact integer sums) and the solve of the
10^9-problem grid (trait rotation, per-trait prologue, fused contraction +
FP64 p x p solve), with b left in HBM. Inputs (genotypes as uint8, traits as
FP64) are resident in HBM before timing starts; the host eigendecomposition of
the kinship matrix is setup and is not timed.

The headline value is the FP64 form's throughput (GLS problems/s), the
paper's arithmetic; the FP32 and split-BF16 forms are timed the same way and
reported beside it, each with its fused kernel's fraction of the MFMA peak of
its own precision. A short run
of the serving workload (500 requests at 16/s on a resident m = 1e6 cohort)
adds the p50/p99 request latency under "serving". The
oracle (plain FP64 C, dense Cholesky per problem) is timed on the host cores
on a bounded sample as a reference point.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published dense peaks
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16x3": 2500.0, "bf16x6": 2500.0}
DEFAULT_FORMS = "f64,f32,bf16x3,bf16x6"
# BF16 MFMA products executed per algorithmic product
MFMA_MULT = {"f64": 1, "f32": 1, "bf16x3": 3, "bf16x6": 6}
HBM_GBPS = 8000.0


def fused_traffic(form: str, workload: str):
    """HBM bytes per launch of a form's fused kernel on a workload from the committed
    counter profile, or None when there is none or the kernel sources changed since
    the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "fused_%s_traffic_%s.json" % (form, workload))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for s in rec["sources"]:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return rec["traffic_bytes"] if h.hexdigest() == rec["sources_sha256"] else None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, phi, xl, budget_s: float = 12.0):
    """Time the oracle on a bounded sample of the workload, about budget_s seconds:
    every problem is passed as its own trait row, so that each pays its own O(n^3)
    factorisation (Table 1, LAPACK row) even where a trait is drawn twice."""
    import oracle

    oracle.build(force=False)
    threads = os.cpu_count() or 1
    import synth

    rng = np.random.default_rng(0)
    y, h2 = synth.traits(w, 0, w.t)
    count = threads
    while True:
        jj = rng.choice(w.t, size=count, replace=count > w.t)
        ii = rng.choice(w.m, size=jj.size, replace=False)
        xr = synth.snp_columns(w, ii)
        t0 = time.perf_counter()
        oracle.gls(phi, xl, xr, y[jj], h2[jj], nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= budget_s / 3 or count >= w.m:
            break
        count = int(min(w.m, max(count * 2, count * budget_s / max(dt, 1e-3))))
    # one thread, a few problems of the same sample
    k1 = min(8, jj.size)
    t1 = time.perf_counter()
    oracle.gls(phi, xl, xr[:k1], y[jj[:k1]], h2[jj[:k1]], nthreads=1)
    dt1 = time.perf_counter() - t1
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    # for context: Eq. (1) through the eigendecomposition of Phi (rotations by
    # Z^T, then per problem the weighted p x p normal equations) in numpy FP64 on
    # the same host, eigendecomposition excluded as setup
    from oracle import rotated

    lam, z = np.linalg.eigh(phi)
    mm, tt = 2000, 100
    xr_m = synth.snp_columns(w, rng.choice(w.m, size=mm, replace=False))
    t2 = time.perf_counter()
    rotated.gls_rotated(xl, xr_m, y[:tt], h2[:tt], z, lam)
    dt2 = time.perf_counter() - t2
    return {"value": jj.size / dt, "unit": "GLS problems/s", "cores": threads, "kind": "oracle",
            "sample": "%d problems (i, j) of the %s workload (distinct SNPs, traits drawn at random), "
                      "each factorising its own n x n M_j; %.1f s on %d threads" % (jj.size, w.name, dt, threads),
            "single_thread_value": k1 / dt1, "cpu_model": model,
            "method_on_host": {"value": mm * tt / dt2, "unit": "GLS problems/s",
                               "kind": "Eq. 1 through the eigendecomposition of Phi (rotate by Z^T, weighted "
                                               "p x p normal equations per problem) in numpy FP64, "
                                               "eigendecomposition excluded",
                               "sample": "%d SNPs x %d traits of the %s workload; %.2f s" % (mm, tt, w.name, dt2)}}


def stream_bench(args):
    """Streamed grid: n = 1000, p = 4, m = 1e6 resident, t = 1e4 in trait blocks of 1000,
    b (1e10 x 4 FP32) streamed slab by slab to pinned host memory and checksummed."""
    import torch

    import synth
    from paper_1210_7683_amd import costmodel as cm
    from paper_1210_7683_amd import gwas

    w = synth.WORKLOADS[args.workload]
    form = args.forms.split(",")[0]
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    ev, z = np.linalg.eigh(phi)
    log("inputs (%d SNPs, %d traits) drawn in %.1f s" % (w.m, w.t, time.perf_counter() - t0))
    cohort = gwas.Cohort(z, ev, xl, w.m, forms=(form,), max_traits=1000, timing=True,
                         host_threads=min(16, os.cpu_count() or 1))
    xr_d = torch.from_numpy(xr).cuda()
    cohort.rotate(0, xr_d)
    del xr_d
    y_d = torch.from_numpy(y).cuda()
    torch.cuda.synchronize()
    # host-link reference: one 1 GiB pinned device -> host copy
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty(1 << 28, dtype=torch.float32, pin_memory=True)
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    link = 3 * (1 << 30) / (time.perf_counter() - t0) / 1e9
    del src, dst
    # check: the first trait block's first slabs against b computed resident in HBM
    check = cohort.solve(y_d[:1000], h2[:1000], form=form, i0=0, m=3 * 16384).cpu().numpy()
    expect = [gwas.checksum(check[k * 16384:(k + 1) * 16384]) for k in range(3)]
    cohort.reset_stats()
    t0 = time.perf_counter()
    sums = cohort.solve_stream(y_d, h2, form=form)
    wall = time.perf_counter() - t0
    st = cohort.stats()
    cohort.close()
    problems = w.m * w.t
    ok = sums[:3] == expect
    fused_s = st["fused_ms"] * 1e-3
    line = {
        "metric": "GLS problems solved/s, b streamed to pinned host memory",
        "value": problems / wall, "unit": "GLS problems/s", "n_gpus": 1, "dtype": form,
        "config": {"workload": w.name, "n": w.n, "p": w.p, "m": w.m, "t": w.t, "trait_block": 1000,
                   "slab_snps": 16384, "form": form},
        "wall_s": wall, "d2h_gbps": st["bytes_d2h"] / wall / 1e9, "pinned_copy_gbps": link,
        "kernel_only_gls_per_s": problems / fused_s, "fused_ms_total": st["fused_ms"],
        "fused_frac_of_wall": fused_s / wall, "slabs": len(sums),
        "checksum_sum": int(sum(sums) % (1 << 64)), "checksums_match_resident": ok,
        "bytes_d2h": st["bytes_d2h"],
    }
    log("streamed %d slabs in %.2f s: %.3e GLS/s end to end, D2H %.1f GB/s (pinned copy %.1f GB/s), "
        "kernels %.2f s; checksums match: %s" % (len(sums), wall, problems / wall, line["d2h_gbps"], link,
                                                 fused_s, ok))
    print(json.dumps(line), flush=True)


def single_trait_bench(args):
    """Few traits (t = 1, 2, 3) against m = 1e6 resident SNPs, n = 1000, p = 4:
    the dot-product kernel, bound by reading the rotated SNP store once. A step
    is one solve of the m x t grid (the rotation is the cohort's one-time setup,
    timed separately); the roofline is HBM bytes per launch over its duration.
    The headline is t = 1; traits beyond the workload's one come from the same
    generator (the paper-shape workload's first traits)."""
    import torch

    import synth
    from paper_1210_7683_amd import gwas

    w = synth.WORKLOADS[args.workload]
    forms = [f for f in args.forms.split(",") if f in ("f32", "f64")] or ["f32"]
    ts = [int(v) for v in args.small_t.split(",")]
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    if max(ts) > w.t:
        y2, h22 = synth.traits("paper_m1e6", 0, max(ts) - w.t)
        y, h2 = np.vstack([y, y2]), np.concatenate([h2, h22])
    ev, z = np.linalg.eigh(phi)
    log("inputs (%d SNPs, %d traits) drawn in %.1f s" % (w.m, y.shape[0], time.perf_counter() - t0))
    xr_d = torch.from_numpy(xr).cuda()
    y_d = torch.from_numpy(y).cuda()
    results = {}
    for form in forms:
        cohort = gwas.Cohort(z, ev, xl, w.m, forms=(form,), timing=True)
        cohort.rotate(0, xr_d)
        dt = torch.float64 if form == "f64" else torch.float32
        torch.cuda.synchronize()
        rot_ms = cohort.stats()["rotate_ms"]
        for t in ts:
            b = torch.empty((w.m, t, w.p), dtype=dt, device="cuda")
            for _ in range(args.warmup):
                cohort.solve(y_d[:t], h2[:t], form=form, out=b)
            torch.cuda.synchronize()
            cohort.reset_stats()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                cohort.solve(y_d[:t], h2[:t], form=form, out=b)
            e1.record()
            torch.cuda.synchronize()
            st = cohort.stats()
            ms = e0.elapsed_time(e1) / args.steps
            fused_ms = st["fused_ms"] / max(1, st["fused_launches"])
            esz = 8 if form == "f64" else 4
            bytes_launch = w.m * (w.n * esz + t * w.p * esz)   # X'_R rows once + b
            key = form if t == ts[0] else "%s_t%d" % (form, t)
            results[key] = {"t": t, "gls_per_s": w.m * t / (ms * 1e-3), "ms_per_step": ms, "fused_ms": fused_ms,
                            "hbm_gbps": bytes_launch / (fused_ms * 1e-3) / 1e9,
                            "dot_launches": st["dot_launches"] // max(1, args.steps),
                            "rotate_once_ms": rot_ms, "finite": bool(torch.isfinite(b).all().item())}
            log("%s t=%d: %.3f ms/solve (kernel %.3f ms, %.0f GB/s), %.3g GLS/s, dot kernel %s; rotation once %.1f ms" %
                (form, t, ms, fused_ms, results[key]["hbm_gbps"], results[key]["gls_per_s"],
                 bool(st["dot_launches"]), rot_ms))
            del b
        cohort.close()
    head = forms[0]
    r = results[head]
    line = {"metric": "GLS problems/s, single trait (t = 1) against a resident cohort",
            "value": r["gls_per_s"], "unit": "GLS problems/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": head, "data": "synthetic",
            "config": {"workload": w.name, "n": w.n, "p": w.p, "m": w.m, "t": r["t"], "form": head,
                       "step": "solve of the m x t grid, rotated SNPs resident, b in HBM"},
            "roofline": {"bound": "hbm", "achieved": r["hbm_gbps"], "peak": HBM_GBPS, "unit": "GB/s",
                         "frac": r["hbm_gbps"] / HBM_GBPS, "traffic": None,
                         "kernel": "fused_gemv_kernel<%s, p=4, t=%d>" % (head, r["t"])},
            "forms": results}
    print(json.dumps(line), flush=True)


def snp_stream_bench(args):
    """SNPs streamed from pinned host memory (not resident): n = 1000, p = 4,
    m = 4e6 genotypes (4 GB uint8) through a store of 2^20 rotated SNPs, t = 100
    traits; each block is copied, rotated and solved while the previous block's
    b (4e8 x 4 FP32 in all, 6.4 GB) goes to pinned host memory. One step is the
    whole grid."""
    import torch

    import synth
    from paper_1210_7683_amd import gwas

    w = synth.WORKLOADS[args.workload]
    form = args.forms.split(",")[0]
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = torch.from_numpy(synth.snps(w)).pin_memory()
    y, h2 = synth.traits(w)
    ev, z = np.linalg.eigh(phi)
    log("inputs (%d SNPs, %d traits) drawn and pinned in %.1f s" % (w.m, w.t, time.perf_counter() - t0))
    cap = 1 << 20
    cohort = gwas.Cohort(z, ev, xl, cap, forms=(form,), timing=True, host_threads=min(16, os.cpu_count() or 1))
    y_d = torch.from_numpy(y).cuda()
    for _ in range(max(1, args.warmup)):
        cohort.solve_snp_stream(xr[: cap], y_d, h2, form=form)
    torch.cuda.synchronize()
    cohort.reset_stats()
    w0 = time.perf_counter()
    sums = cohort.solve_snp_stream(xr, y_d, h2, form=form)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    st = cohort.stats()
    problems = w.m * w.t
    res = {"metric": "GLS problems/s, SNPs streamed from host memory through the rotated store",
           "value": problems / wall, "unit": "GLS problems/s", "n_gpus": 1, "dtype": form,
           "config": {"workload": w.name, "n": w.n, "p": w.p, "m": w.m, "t": w.t, "form": form,
                      "store_snps": cap, "block_snps": cap // 2},
           "wall_s": wall, "h2d_gbps": st["bytes_h2d"] / wall / 1e9, "d2h_gbps": st["bytes_d2h"] / wall / 1e9,
           "rotate_s": st["rotate_ms"] * 1e-3, "fused_s": st["fused_ms"] * 1e-3, "slabs": len(sums),
           "bytes_h2d": st["bytes_h2d"], "bytes_d2h": st["bytes_d2h"]}
    log("streamed %d SNPs x %d traits in %.3f s: %.3e GLS/s; H2D %.1f GB/s, D2H %.1f GB/s; "
        "rotation %.3f s, fused %.3f s (kernel sums)" % (w.m, w.t, wall, res["value"], res["h2d_gbps"],
                                                        res["d2h_gbps"], res["rotate_s"], res["fused_s"]))
    cohort.close()
    print(json.dumps(res), flush=True)


def serve_bench(args):
    """Serving: resident cohort n = 1000, m = 1e6; Poisson arrivals; each request a
    trait block with t ~ log-uniform[1, 512], its own h2 and p - 1 ~ U{1..7}; b
    streamed to pinned host memory and checksummed; p50/p99 latency at a fixed rate."""
    line = run_serving(args.workload, args.forms.split(",")[0], args.rate, args.requests, args.warmup_requests,
                       args.slots, args.ring_slots, args.skip_checksum, args.grid_wgs)
    print(json.dumps(line), flush=True)


def run_serving(workload, form, rate, requests, warmup_requests, slots=8, ring_slots=0, skip_checksum=False,
                grid_wgs=0):
    import torch

    import synth
    from paper_1210_7683_amd import gwas

    w = synth.WORKLOADS[workload]
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)       # intercept + 6 covariates: p up to 8
    xr = synth.snps(w)
    ev, z = np.linalg.eigh(phi)
    reqs = synth.requests(w, warmup_requests + requests, rate)
    log("inputs drawn in %.1f s; %d requests at %.1f/s" % (time.perf_counter() - t0, len(reqs), rate))
    cohort = gwas.Cohort(z, ev, xl, w.m, forms=(form,))
    xr_d = torch.from_numpy(xr).cuda()
    cohort.rotate(0, xr_d)
    torch.cuda.synchronize()
    del xr_d
    srv = gwas.Server(cohort, form=form, max_slots=slots, max_traits=512,
                      host_threads=min(16, os.cpu_count() or 1), ring_slots=ring_slots,
                      skip_checksum=skip_checksum, grid_wgs=grid_wgs)
    start = gwas.clock() + 0.2
    tickets = []
    for i, r in enumerate(reqs):
        delay = start + r.arrival_s - gwas.clock()
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(r.y, r.h2, r.p))
        if (i + 1) % 500 == 0:
            log("serving: %d of %d requests submitted" % (i + 1, len(reqs)))
    res = [srv.wait(tk, timeout=600) for tk in tickets]
    sst = srv.stats()
    srv.close()
    cohort.close()
    meas = list(range(warmup_requests, len(reqs)))
    lat = np.array([res[k]["t_done"] - (start + reqs[k].arrival_s) for k in meas])
    qwait = np.array([res[k]["t_admit"] - (start + reqs[k].arrival_s) for k in meas])
    problems = sum(res[k]["problems"] for k in meas)
    bytes_b = sum(res[k]["problems"] * reqs[k].p * (8 if form == "f64" else 4) for k in meas)
    t_first = start + reqs[meas[0]].arrival_s
    t_last = max(res[k]["t_done"] for k in meas)
    span = t_last - t_first
    ok = all(res[k]["state"] == "done" for k in range(len(reqs)))
    line = {
        "metric": "serving: p50/p99 latency and GLS problems/s at a fixed arrival rate",
        "value": problems / span, "unit": "GLS problems/s", "n_gpus": 1, "dtype": form,
        "config": {"workload": w.name, "n": w.n, "m": w.m, "rate_hz": rate,
                   "requests": len(meas), "warmup_requests": warmup_requests, "slots": slots,
                   "t": "log-uniform[1,512]", "p": "2..8", "form": form},
        "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_max_s": float(lat.max()), "queue_wait_p99_s": float(np.percentile(qwait, 99)),
        "mean_traits": float(np.mean([reqs[k].y.shape[0] for k in meas])),
        "d2h_gbps": bytes_b / span / 1e9, "window_s": span, "all_done": ok,
        "server": sst, "checksummed": not skip_checksum,
        # the grouped launches: slabs per launch, and the serving kernel's own rate over
        # every request (warm-up ones included), algorithmic 2 (p + 1) n flops per problem
        "items_per_launch": sst["items"] / max(1, sst["rounds"]),
        "kernel_gls_per_s": sum(r["problems"] for r in res) / max(1e-9, sst["kernel_s"]),
        "kernel_tflops": sum(res[k]["problems"] * 2 * (reqs[k].p + 1) * w.n for k in range(len(reqs)))
                         / max(1e-9, sst["kernel_s"]) / 1e12,
    }
    log("serving at %.1f req/s: p50 %.3f s, p99 %.3f s, %.3e GLS/s, b to host %.1f GB/s; %.2f slabs per "
        "launch, kernel %.1f TFLOP/s" % (rate, line["latency_p50_s"], line["latency_p99_s"], line["value"],
                                        line["d2h_gbps"], line["items_per_launch"], line["kernel_tflops"]))
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper_m1e6")
    ap.add_argument("--forms", default=DEFAULT_FORMS, help="headline form first")
    ap.add_argument("--f32-flush", type=int, default=None,
                    help="FP32 form: 2 = FP64 folds (the library default), 0 = FP32 accumulation only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true",
                    help="paper-shape bench: skip the short serving run that reports p50/p99 latency")
    ap.add_argument("--serving-requests", type=int, default=500,
                    help="paper-shape bench: measured requests of the short serving run")
    ap.add_argument("--small-t", default="1,2,3", help="single_trait workload: trait counts to time")
    ap.add_argument("--rate", type=float, default=16.0, help="serving: request arrival rate (1/s)")
    ap.add_argument("--requests", type=int, default=200, help="serving: measured requests")
    ap.add_argument("--warmup-requests", type=int, default=20)
    ap.add_argument("--slots", type=int, default=8, help="serving: requests in flight")
    ap.add_argument("--ring-slots", type=int, default=0, help="serving: pinned ring slots (0: library default)")
    ap.add_argument("--skip-checksum", action="store_true", help="serving: do not checksum ring slabs")
    ap.add_argument("--grid-wgs", type=int, default=0, help="serving: persistent workgroups (0: two per CU)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="one step of each form in --forms plus a plain 1 GiB device copy (for counter "
                         "calibration), no timing output; meant to run under rocprofv3")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the GLS grid shards along SNPs with no exchange, "
              "and the bench measures one GPU's share (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_1210_7683_amd import costmodel as cm
    from paper_1210_7683_amd import gwas

    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.workload.startswith("stream"):
        if args.forms == DEFAULT_FORMS:
            args.forms = "bf16x3"
        return stream_bench(args)
    if args.workload.startswith("snp_stream"):
        if args.forms == DEFAULT_FORMS:
            args.forms = "f32"
        return snp_stream_bench(args)
    if args.workload.startswith("single_trait"):
        if args.forms == DEFAULT_FORMS:
            args.forms = "f32,f64"
        return single_trait_bench(args)
    if args.workload.startswith("serve"):
        if args.forms == DEFAULT_FORMS:
            args.forms = "f32"
        return serve_bench(args)
    forms = args.forms.split(",")
    w = synth.WORKLOADS[args.workload]
    log("workload %s: n=%d p=%d m=%d t=%d" % (w.name, w.n, w.p, w.m, w.t))
    t0 = time.perf_counter()
    phi, xl = synth.kinship(w), synth.covariates(w)
    xr = synth.snps(w)
    y, h2 = synth.traits(w)
    ev, z = np.linalg.eigh(phi)
    log("inputs drawn and Phi eigendecomposed in %.1f s" % (time.perf_counter() - t0))

    xr_d = torch.from_numpy(xr).cuda()
    y_d = torch.from_numpy(y).cuda()
    torch.cuda.synchronize()
    problems = w.m * w.t
    flops_gls = cm.flops_per_gls_contraction(w.n, w.p)
    if args.profile_pass:
        for form in forms:
            with gwas.Cohort(z, ev, xl, w.m, forms=(form,), f32_flush=args.f32_flush) as cohort:
                b = torch.empty((w.m, w.t, w.p), dtype=torch.float64 if form == "f64" else torch.float32,
                                device="cuda")
                cohort.rotate(0, xr_d)
                cohort.solve(y_d, h2, form=form, out=b)
                torch.cuda.synchronize()
                del b
            log("profile pass: one %s step" % form)
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("profile pass done: a 1 GiB device copy")
        return
    results = {}
    for form in forms:
        # one cohort per form, holding only that form's rotated SNPs, so a step's
        # rotation writes exactly what the form's solve reads
        cohort = gwas.Cohort(z, ev, xl, w.m, forms=(form,), timing=True, f32_flush=args.f32_flush)
        dt = torch.float64 if form == "f64" else torch.float32
        b = torch.empty((w.m, w.t, w.p), dtype=dt, device="cuda")

        def step():
            cohort.rotate(0, xr_d)
            cohort.solve(y_d, h2, form=form, out=b)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        cohort.reset_stats()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        evs[0].record()
        for k in range(args.steps):
            step()
            evs[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)])
        ms = evs[0].elapsed_time(evs[-1]) / args.steps
        st = cohort.stats()
        fused_ms = st["fused_ms"] / max(1, st["fused_launches"])
        rot_ms = st["rotate_ms"] / max(1, st["rotate_launches"])
        mult = MFMA_MULT[form]
        achieved = mult * flops_gls * problems / (fused_ms * 1e-3) / 1e12
        results[form] = {
            "gls_per_s": problems / (ms * 1e-3),
            "ms_per_step": ms,
            "step_ms_median": float(np.median(step_ms)),
            "step_ms_min": float(step_ms.min()),
            "step_ms_max": float(step_ms.max()),
            "wall_ms_per_step": wall * 1e3 / args.steps,
            "fused_ms": fused_ms,
            "rotate_ms": rot_ms,
            "solve_only_gls_per_s": problems / (fused_ms * 1e-3),
            "fused_tflops": achieved,
            "mfma_frac": achieved / PEAK_TFLOPS[form],
            # the paper's convention, (5 + 2(p-1)) n flops per problem over the whole step
            # (its 40-core node: about 25 GFLOP/s on this count)
            "paper_convention_tflops": cm.flops_per_gls_paper(w.n, w.p) * problems / (ms * 1e-3) / 1e12,
            "non_spd": st["non_spd"],
            "finite": bool(torch.isfinite(b).all()),
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_TFLOPS[form], "unit": "TFLOP/s",
                         "frac": achieved / PEAK_TFLOPS[form], "traffic": fused_traffic(form, w.name),
                         "flops_per_launch": mult * flops_gls * problems,
                         "flops_counted": "executed BF16 products" if mult > 1 else "algorithmic"},
        }
        log("%s: %.3f ms/step (fused %.3f ms, rotate %.3f ms) -> %.3e GLS/s, fused %.1f TFLOP/s "
            "= %.1f%% of %s peak" % (form, ms, fused_ms, rot_ms, results[form]["gls_per_s"],
                                      achieved, 100 * achieved / PEAK_TFLOPS[form], form))
        del b
        cohort.close()
        torch.cuda.empty_cache()

    head = forms[0]
    r = results[head]
    mult = MFMA_MULT[head]
    line = {
        "metric": "GLS problems solved/s + MFMA % of peak, FP64 vs FP32 vs split-BF16; p99",
        "value": r["gls_per_s"],
        "unit": "GLS problems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "p": w.p, "m": w.m, "t": w.t,
                   "form": head, "step": "rotate all SNPs + solve the full grid, b in HBM"},
        "roofline": {"bound": "mfma", "achieved": r["fused_tflops"], "peak": PEAK_TFLOPS[head],
                     "unit": "TFLOP/s", "frac": r["mfma_frac"], "traffic": fused_traffic(head, w.name),
                     "kernel": "fused_dma_kernel<%s, p=4>" % head,
                     "flops_per_launch": mult * flops_gls * problems},
        "forms": results,
    }
    if not args.no_serving:
        # the metric's p99: a short run of the serving workload (the full one is
        # --workload serve_m1e6), reported beside the grid's throughput
        log("serving: %d requests at %.0f/s on the resident m = 1e6 cohort ..." % (args.serving_requests, args.rate))
        s = run_serving("serve_m1e6", "f32", args.rate, args.serving_requests, 20)
        line["serving"] = {"workload": "serve_m1e6", "form": "f32", "rate_hz": args.rate,
                           "requests": s["config"]["requests"], "latency_p50_s": s["latency_p50_s"],
                           "latency_p99_s": s["latency_p99_s"], "gls_per_s": s["value"],
                           "d2h_gbps": s["d2h_gbps"], "all_done": s["all_done"],
                           "items_per_launch": s["items_per_launch"], "kernel_tflops": s["kernel_tflops"]}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline(w, phi, xl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
