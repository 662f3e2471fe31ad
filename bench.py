"""Benchmark of the RAS-PML GMRES hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload k640]

A step is one complete pass of the hot path on one synthetic problem:
setup (geometry, global and local operators, batched band factorisation
of every subdomain), right-hand side b = M f, FGMRES(100) preconditioned
by RAS-PML to a confirmed true relative residual <= 1e-6, and teardown.
The source f is resident in HBM before the timed region.  The default
workload is k = 640, h = 1/1280 (1,703,025 unknowns), 32 x 32 subdomains,
overlap = PML width = ceil(ln k / (k h)) = 13 cells, global PML 13 cells,
g(x) = 10 k x^3, Gaussian source exp(-|x - (0.5,0.5)|^2 / 0.05^2), mixed
precision (complex64 local factors and solves, complex128 Krylov work).

Printed: one JSON line with the metric (time to a 1e-6 residual, seconds
per solve), the FP64 GPU path beside it, RAS-PML applies/s in both
precisions, the roofline of the dominant kernel (batched band solves,
HIP-event durations on the launch stream) and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-6 residual & RAS-PML applies/s at k=640; mixed vs FP64 GPU"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (k, n_int, P)
    "k640": (640.0, 1280, 32),
    "k160": (160.0, 320, 16),
    "k20": (20.0, 40, 2),
}


def measured_traffic(workload):
    """HBM bytes per band-solve launch from the committed rocprofv3 PMC
    summary (FETCH_SIZE and WRITE_SIZE runs scaled by a copy of known size),
    or None when the kernel source changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_band_solve_%s_pmc.json" % workload)
    src = os.path.join(ROOT, "paper_2602_00735_amd", "csrc", "k_solve.hip")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("k_solve_hip_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return rec["traffic_bytes_per_dispatch"]


def log_width(k, h):
    return int(math.ceil(math.log(k) / (k * h) - 1e-12))


# factorisation kernel variants as ras_pml_tuning numbers them
LU_VARIANTS = ("mfma", "mfma_register_capped", "valu_one_column")
# fused Arnoldi variants as RAS_KNOB_ARNOLDI numbers them
ARNOLDI_VARIANTS = {0: "e8", 1: "e16", 2: "lean_e12", -1: "first_that_fits", -2: "unfused"}


def progress(msg):
    """A line on stderr when a phase of the run ends."""
    print("[bench] %s" % msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="k640", choices=sorted(WORKLOADS))
    ap.add_argument("--source", default="gaussian", choices=["gaussian", "paper"])
    ap.add_argument("--applies", type=int, default=50)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (default: tune once before the warmup, outside the "
                         "timed region, and set every timed handle up from its cache)")
    ap.add_argument("--no-section4", action="store_true",
                    help="skip Section 4's own covering at k = 300 and 1200 (wide bands)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 32-problem batch (seeded multi-source problems, one handle)")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the k-sweep at kh = 1/2 with the Section 3 (iii) widths: "
                         "subdomain boundary conditions (Tables 1/2 set-up) and the growth of "
                         "iterations and time with k (Tables 3/4 set-up); one JSON line per run")
    ap.add_argument("--sweep-max-k", type=float, default=1280.0)
    ap.add_argument("--paper-tables", action="store_true",
                    help="only run Section 4's own covering: grid (2k)^2, N = (k/150)^2 "
                         "subdomains with 300-cell cores, widths from the width rule, a global "
                         "PML of three wavelengths, the smoothed point source, rtol 1e-10, "
                         "at most 500 iterations: Tables 1/2 (C_kappa = 3/8, three subdomain "
                         "conditions, Richardson and GMRES) and Tables 3/4 (C_kappa = 1/2, "
                         "Richardson, setup and solve seconds); one JSON line per run")
    ap.add_argument("--paper-max-k", type=float, default=2400.0)
    ap.add_argument("--warmstart", action="store_true",
                    help="only run the learned warm start at k = 320, h = 1/640, 16x16 subdomains: "
                         "solve --ws-train seeded problems, train the encoder-decoder on the "
                         "(source, k^2 u) pairs, compare GMRES from the network's guess with GMRES "
                         "from zero on --ws-test held-out seeds")
    ap.add_argument("--ws-train", type=int, default=4096)
    ap.add_argument("--ws-test", type=int, default=256)
    ap.add_argument("--ws-epochs", type=int, default=4)
    ap.add_argument("--ws-batch", type=int, default=8)
    ap.add_argument("--ws-source", default="gaussian", choices=["gaussian", "narrow"],
                    help="gaussian: 1-4 Gaussians of width 0.03; narrow: 1-4 of the paper's "
                         "smoothed point sources (width pi/(4k)), which radiate")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (PMC traffic calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole hot path on a single "
              "MI355X (sharding across GPUs is designed, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2602_00735_amd as rp
    from paper_2602_00735_amd import inputs

    if args.calibrate_copy:
        # 1 GiB read + 1 GiB written per copy, three dispatches
        n = 1 << 27
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 8 * n, "bytes_written": 8 * n,
                          "dispatches": 3}))
        return

    if args.paper_tables:
        paper_tables(args.paper_max_k)
        return
    if args.sweep:
        sweep(args.sweep_max_k)
        return
    if args.warmstart:
        warmstart(args)
        return

    k, n_int, P = WORKLOADS[args.workload]
    h = 1.0 / n_int
    L = log_width(k, h)
    G = 4 if args.workload == "k20" else L
    grid, subs = (n_int, n_int), (P, P)
    if args.source == "gaussian":
        f_h = inputs.centre_gaussian(n_int, G, 0.05)
    else:
        f_h = inputs.paper(k, n_int, G)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f = torch.from_numpy(f_h).to(dev)
    ndof = f.numel()
    stream = torch.cuda.current_stream()

    import tempfile
    cache = None if args.no_tune else os.path.join(
        tempfile.gettempdir(), "ras_pml_tune_%s_%d.json" % (args.workload, os.getpid()))
    tuning = {}
    if cache is not None:
        for name, prec in (("mixed", rp.RAS_MIXED), ("fp64", rp.RAS_FP64)):
            if name == "fp64" and args.no_fp64:
                continue
            Ht = rp.ras_pml_setup(k, h, grid, subs, L, L, rp.default_opts(global_pml=G, precision=prec))
            rp.ras_pml_autotune(Ht, cache)
            tuning[name] = rp.ras_pml_tuning(Ht)
            tuning[name]["times_ms"] = rp.ras_pml_tune_report(Ht)
            Ht.close()

    def one_solve(precision, timing=False, f=f, graph=False, repeat=False):
        flags = (rp.RAS_FLAG_TIMING if timing else 0) | (rp.RAS_FLAG_GRAPH_STEPS if graph else 0)
        opts = rp.default_opts(global_pml=G, precision=precision, flags=flags)
        if cache is not None:
            opts.tune_cache = os.fsencode(cache)
        t0 = time.perf_counter()
        H = rp.ras_pml_setup(k, h, grid, subs, L, L, opts)
        b = torch.empty_like(f)
        x = torch.zeros_like(f)
        rp.ras_pml_rhs(H, f, b)
        t1 = time.perf_counter()
        rc, it, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-6, restart=100, maxit=500)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        stats = rp.ras_pml_get_stats(H)
        res = dict(rc=rc, iters=it, relres=rr, setup_s=t1 - t0, solve_s=t2 - t1,
                   total_s=t2 - t0, stats=stats, x=x, alloc_s=stats["alloc_ms"] / 1000.0)
        if repeat:
            # a second solve on the same handle (Krylov workspace and, with
            # graph steps, the recorded graph already there)
            x2 = torch.zeros_like(f)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            rc2, it2, _, _ = rp.gmres_solve(H, b, x2, rtol=1e-6, restart=100, maxit=500)
            torch.cuda.synchronize()
            res["repeat_solve_s"] = time.perf_counter() - t3
            res["repeat_same"] = bool(rc2 == rc and it2 == it and torch.equal(x2, x))
        H.close()
        return res

    # ---------------------------------------------------------------- warmup
    for _ in range(args.warmup):
        one_solve(rp.RAS_MIXED)
    # ---------------------------------------------------------------- timed
    # (no per-launch events inside: each event record drains the queue and
    # writes the caches back, which adds ~0.15 ms to every band solve)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [one_solve(rp.RAS_MIXED) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(r["rc"] == rp.RAS_OK for r in runs), [r["rc"] for r in runs]
    ms_per_step = 1000.0 * elapsed / args.steps
    mixed = runs[-1]
    # per-kernel breakdown: one more solve, untimed, with per-launch events
    st = one_solve(rp.RAS_MIXED, timing=True)["stats"]
    progress("timed steps done: %.4f s per solve" % (ms_per_step / 1000.0))

    # ---------------------------------------------------------------- graph steps
    # the same solve with every eight FGMRES steps replayed from a HIP graph
    # (RAS_FLAG_GRAPH_STEPS), timed like the steps above, and a second solve
    # on each handle (the eager and the graph-replayed one)
    one_solve(rp.RAS_MIXED, graph=True)
    ng = max(3, min(args.steps, 10))
    gruns = [one_solve(rp.RAS_MIXED, graph=True, repeat=True) for _ in range(ng)]
    eruns = [one_solve(rp.RAS_MIXED, repeat=True) for _ in range(3)]
    g_ms = 1000.0 * float(np.median([r["total_s"] for r in gruns]))
    graph_blk = {
        "ms_per_step": round(g_ms, 3),
        "solve_s": round(float(np.median([r["solve_s"] for r in gruns])), 5),
        "repeat_solve_s": round(float(np.median([r["repeat_solve_s"] for r in gruns])), 5),
        "eager_repeat_solve_s": round(float(np.median([r["repeat_solve_s"] for r in eruns])), 5),
        "eager_solve_s": round(float(np.median([r["solve_s"] for r in runs])), 5),
        "iters": gruns[-1]["iters"],
        "identical_to_eager": bool(all(torch.equal(r["x"], mixed["x"]) for r in gruns)
                                   and all(r["repeat_same"] for r in gruns + eruns)),
        "note": "ms_per_step: median of setup + first solve (which records the graph) over "
                "%d handles; repeat: a second solve on the same handle" % ng}
    progress("graph-replayed steps done: %.4f s per solve" % (g_ms / 1000.0))

    # ---------------------------------------------------------------- roofline
    # the dominant kernel alone: back-to-back batched band solves on the
    # launch stream, HIP events around the loop
    nroof = 20

    def band_loop(precision):
        o = rp.default_opts(global_pml=G, precision=precision)
        if cache is not None:
            o.tune_cache = os.fsencode(cache)
        Hr = rp.ras_pml_setup(k, h, grid, subs, L, L, o)
        nbytes = rp.ras_pml_get_stats(Hr)["solve_bytes"]
        vr = torch.from_numpy(inputs.random_vector(ndof, 2)).to(dev)
        for _ in range(2):
            rp.ras_pml_local_solve(Hr, vr, None)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(nroof):
            rp.ras_pml_local_solve(Hr, vr, None)
        e1.record(stream)
        torch.cuda.synchronize()
        Hr.close()
        return e0.elapsed_time(e1) / nroof, nbytes

    solve_avg_ms, solve_bytes = band_loop(rp.RAS_MIXED)
    achieved = solve_bytes / (solve_avg_ms * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(ms_per_step / 1000.0, 6),
        "unit": "s per solve to a true relative residual <= 1e-6 (setup + solve, mixed precision)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "c64 local factors/solves + c128 SpMV/Krylov",
        "data": "synthetic (seeded Gaussian source on the mesh nodes)",
        "config": {
            "workload": "RAS-PML FGMRES(100) rtol 1e-6, k=%g h=1/%d (%d unknowns), %dx%d "
                        "subdomains, overlap=pml=%d cells, global PML %d cells, g=10k x^3, "
                        "%s source, impedance subdomain BC, linear PoU"
                        % (k, n_int, ndof, P, P, L, G, args.source),
            "k": k, "h": "1/%d" % n_int, "subdomains": [P, P], "overlap": L, "pml_width": L,
            "global_pml": G, "restart": 100, "rtol": 1e-6, "source": args.source,
        },
        "mixed": {"iters": mixed["iters"], "relres": mixed["relres"],
                  "setup_s": round(mixed["setup_s"], 5), "solve_s": round(mixed["solve_s"], 5),
                  "device_alloc_s": round(mixed["alloc_s"], 5),
                  "breakdown_note": "per-kernel sums over one extra solve with per-launch "
                                    "events (which slow each launch a little)",
                  "per_step_breakdown_ms": {
                      "band_solves": round(st["solve_ms"], 3), "pou_sum": round(st["sum_ms"], 3),
                      "spmv": round(st["spmv_ms"], 3), "mgs": round(st["mgs_ms"], 3),
                      "givens": round(st["givens_ms"], 3)},
                  "setup_assemble_ms": round(st["setup_assemble_ms"], 3),
                  "setup_factor_ms": round(st["setup_factor_ms"], 3)},
        "graph_steps": graph_blk,
        "tuning": {name: {"band_solve_deep_prefetch": t["solve_deep"],
                          "band_solve_queue": t["solve_queue"],
                          "arnoldi_variant": ARNOLDI_VARIANTS.get(t["arnoldi"], t["arnoldi"]),
                          "factor_classes": [{"tiles": g[0], "subdomains": g[1],
                                              "variant": LU_VARIANTS[g[2]]} for g in t["ldlt"]],
                          "times_ms": t["times_ms"]}
                   for name, t in tuning.items()},
        "roofline": {"kernel": "k_band_solve (batched forward/backward band sweeps)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.workload),
                     "algorithmic_bytes_per_launch": solve_bytes,
                     "avg_launch_ms": round(solve_avg_ms, 4), "launches": nroof,
                     "timing": "HIP events around %d back-to-back launches on the launch "
                               "stream" % nroof},
    }

    # ---------------------------------------------------------------- FP64 path
    if not args.no_fp64:
        one_solve(rp.RAS_FP64)
        r64 = one_solve(rp.RAS_FP64)
        ms64, b64 = band_loop(rp.RAS_FP64)
        d = (mixed["x"] - r64["x"]).norm().item() / r64["x"].norm().item()
        out["fp64"] = {"iters": r64["iters"], "relres": r64["relres"],
                       "setup_s": round(r64["setup_s"], 5), "solve_s": round(r64["solve_s"], 5),
                       "total_s": round(r64["total_s"], 5), "device_alloc_s": round(r64["alloc_s"], 5),
                       "band_solve_avg_ms": round(ms64, 4),
                       "band_solve_GBs": round(b64 / (ms64 * 1e-3) / 1e9, 1)}
        out["mixed_vs_fp64_solution_rel_l2"] = d
        out["speedup_mixed_over_fp64_time_to_solution"] = round(r64["total_s"] / mixed["total_s"], 3)
        out["speedup_mixed_over_fp64"] = {
            "setup": round(r64["setup_s"] / mixed["setup_s"], 3),
            "solve_phase": round(r64["solve_s"] / mixed["solve_s"], 3),
            "total": round(r64["total_s"] / mixed["total_s"], 3)}

    # ---------------------------------------------------------------- Richardson
    # the preconditioner as a fixed-point iteration (Algorithm 1), mixed
    # precision, same problem and stopping test; solve time only
    o = rp.default_opts(global_pml=G, precision=rp.RAS_MIXED)
    if cache is not None:
        o.tune_cache = os.fsencode(cache)
    H = rp.ras_pml_setup(k, h, grid, subs, L, L, o)
    b = torch.empty_like(f)
    rp.ras_pml_rhs(H, f, b)
    x = torch.zeros_like(f)
    rp.ras_pml_richardson(H, b, x, rtol=1e-6, maxit=2)
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, it, rr, _ = rp.ras_pml_richardson(H, b, x, rtol=1e-6, maxit=500)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["richardson"] = {"iters": it, "relres": rr, "converged": rc == rp.RAS_OK,
                         "solve_s": round(ts, 5), "ms_per_iteration": round(1000 * ts / max(1, it), 4),
                         "fgmres_iters_same_problem": mixed["iters"]}
    H.close()

    # ---------------------------------------------------------------- applies/s
    applies = {}
    for name, prec in (("mixed", rp.RAS_MIXED), ("fp64", rp.RAS_FP64)):
        if name == "fp64" and args.no_fp64:
            continue
        o = rp.default_opts(global_pml=G, precision=prec)
        if cache is not None:
            o.tune_cache = os.fsencode(cache)
        H = rp.ras_pml_setup(k, h, grid, subs, L, L, o)
        v = torch.from_numpy(inputs.random_vector(ndof, 1)).to(dev)
        z = torch.empty_like(v)
        rp.ras_pml_apply(H, v, z)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.applies):
            rp.ras_pml_apply(H, v, z)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.applies
        # the same applies replayed from a captured graph
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            rp.ras_pml_apply(H, v, z)
        g.replay()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.applies):
            g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        gms = e0.elapsed_time(e1) / args.applies
        applies[name] = {"applies_per_s": round(1000.0 / ms, 2), "ms_per_apply": round(ms, 4),
                         "graph_replayed_applies_per_s": round(1000.0 / gms, 2)}
        del g
        H.close()
    out["applies"] = applies
    progress("applies done")

    # ---------------------------------------------------------------- 32-problem batch
    if not args.no_batch:
        out["batch32"] = batch32(dev, args.no_fp64)

    # ---------------------------------------------------------------- Section 4 source
    # the paper's smoothed point source (radiates at every k), same workload
    # and solver, beside the Gaussian of the headline
    fsrc = {args.source: f_h}
    if args.source == "gaussian":
        fsrc["paper"] = inputs.paper(k, n_int, G)
        f_paper = torch.from_numpy(fsrc["paper"]).to(dev)
        blk = {}
        for name, prec in (("mixed", rp.RAS_MIXED), ("fp64", rp.RAS_FP64)):
            if name == "fp64" and args.no_fp64:
                continue
            one_solve(prec, f=f_paper)
            r = one_solve(prec, f=f_paper)
            assert r["rc"] == rp.RAS_OK, r["rc"]
            blk[name] = {"iters": r["iters"], "relres": r["relres"], "setup_s": round(r["setup_s"], 5),
                         "solve_s": round(r["solve_s"], 5), "total_s": round(r["total_s"], 5),
                         "x": r["x"]}
        out["paper_source"] = blk
        progress("paper source done")

    # ---------------------------------------------------------------- Section 4's covering
    # the paper's own subdomains (300-cell cores, bands of ~350: the wide
    # kernels) at k = 300 and 1200, Table 4's constants, Richardson to 1e-10
    if not args.no_section4:
        sec = []
        section4_run(300.0, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")    # warm-up
        for ks4 in (300.0, 1200.0):
            r = section4_run(ks4, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")
            sec.append({key: r[key] for key in ("k", "grid", "subdomains", "ovlp", "pml",
                                                 "W_max", "iters", "relres", "converged",
                                                 "setup_s", "solve_s")})
        out["section4_covering"] = sec
        progress("Section 4 covering done")

    # ---------------------------------------------------------------- CPU oracle
    if not args.no_cpu:
        xs = {args.source: {"mixed": mixed["x"]}}
        if "fp64" in out:
            xs[args.source]["fp64"] = r64["x"]
        if "paper_source" in out:
            xs["paper"] = {name: blk["x"] for name, blk in out["paper_source"].items()}
        cb, errs = cpu_oracle(k, n_int, P, L, G, fsrc, xs, args.workload)
        out["cpu_baseline"] = cb
        out["solution_rel_l2_vs_oracle"] = errs[args.source]
        if "paper_source" in out:
            for name, blk in out["paper_source"].items():
                blk["rel_l2_vs_oracle"] = errs["paper"].get(name)
                blk["oracle_iters"] = errs["paper"]["oracle_iters"]
    for blk in out.get("paper_source", {}).values():
        blk.pop("x", None)
    if cache is not None and os.path.exists(cache):
        os.remove(cache)
    print(json.dumps(out), flush=True)


def sweep(max_k):
    """k = 80 ... max_k at kh = 1/2 (about 12.6 points per wavelength), k/20
    subdomains per side (40-cell cores, N proportional to k^2), the Section 4
    source (smoothed point source at the centre), a global PML of three
    wavelengths, rtol 1e-10, at most 500 iterations, mixed precision.
      - "bc": overlap and PML from the width rule with C_delta = 1/6,
        C_kappa = 3/8 (the Tables 1/2 constants); RAS-PML-Imp, RAS-PML-Drch
        and RAS-Imp (no subdomain PML); Richardson and GMRES(100).
      - "growth": C_delta = 1/6, C_kappa = 1/2 (Tables 3/4); RAS-PML-Imp
        Richardson; setup and solve seconds."""
    import torch
    import paper_2602_00735_amd as rp
    from paper_2602_00735_amd import inputs
    torch.cuda.set_device(0)
    ks = [k for k in (80.0, 160.0, 320.0, 640.0, 1280.0) if k <= max_k]

    def run(k, bc, pml, c_kappa, solver):
        n = int(round(2 * k))
        h = 1.0 / n
        P = int(round(k / 20))
        G = int(math.floor(3 * 2 * math.pi / k / h + 1e-9))
        o = rp.default_opts(global_pml=G, bc=bc, precision=rp.RAS_MIXED, width_c_kappa=c_kappa)
        t0 = time.perf_counter()
        H = rp.ras_pml_setup(k, h, (n, n), (P, P), rp.RAS_WIDTH_RULE, pml, o)
        f = torch.from_numpy(inputs.paper(k, n, G)).to("cuda")
        b = torch.empty_like(f)
        x = torch.zeros_like(f)
        rp.ras_pml_rhs(H, f, b)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        if solver == "richardson":
            rc, it, rr, _ = rp.ras_pml_richardson(H, b, x, rtol=1e-10, maxit=500, check=False)
        else:
            rc, it, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-10, restart=100, maxit=500,
                                           check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        d = H.desc()[0]
        H.close()
        return {"k": k, "grid": n, "subdomains": P * P, "ovlp": d[20], "pml": d[21],
                "global_pml": G, "solver": solver, "iters": it,
                "relres": rr if math.isfinite(rr) else None,
                "converged": rc == rp.RAS_OK, "status": rc,
                "setup_s": round(t1 - t0, 4), "solve_s": round(t2 - t1, 4)}

    variants = (("RAS-PML-Imp", rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE),
                ("RAS-PML-Drch", rp.RAS_BC_DRCH, rp.RAS_WIDTH_RULE),
                ("RAS-Imp", rp.RAS_BC_IMP, 0))
    run(80.0, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")        # warm-up
    for k in ks:
        for name, bc, pml in variants:
            for solver in ("richardson", "gmres"):
                r = run(k, bc, pml, 3.0 / 8.0, solver)
                r.update(sweep="bc", variant=name)
                print(json.dumps(r), flush=True)
    for k in ks:
        r = run(k, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")
        r.update(sweep="growth", variant="RAS-PML-Imp",
                 total_per_k=round((r["setup_s"] + r["solve_s"]) / k, 6))
        print(json.dumps(r), flush=True)


def section4_run(k, bc, pml, c_kappa, solver, overlap=None):
    """One run of Section 4's covering (see paper_tables): setup, right-hand
    side and solve of a fresh handle; returns the run's figures.  overlap and
    pml in cells, or RAS_WIDTH_RULE (the default overlap)."""
    import torch
    import paper_2602_00735_amd as rp
    from paper_2602_00735_amd import inputs
    n = int(round(2 * k))
    h = 1.0 / n
    P = int(round(k / 150))
    G = int(math.floor(3 * 2 * math.pi / k / h + 1e-9))
    o = rp.default_opts(global_pml=G, bc=bc, precision=rp.RAS_MIXED, width_c_kappa=c_kappa)
    ov = rp.RAS_WIDTH_RULE if overlap is None else overlap
    t0 = time.perf_counter()
    H = rp.ras_pml_setup(k, h, (n, n), (P, P), ov, pml, o)
    f = torch.from_numpy(inputs.paper(k, n, G)).to("cuda")
    b = torch.empty_like(f)
    x = torch.zeros_like(f)
    rp.ras_pml_rhs(H, f, b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if solver == "richardson":
        rc, it, rr, _ = rp.ras_pml_richardson(H, b, x, rtol=1e-10, maxit=500, check=False)
    else:
        rc, it, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-10, restart=100, maxit=500,
                                       check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    desc = H.desc()
    d = desc[0]
    H.close()
    del f, b, x
    torch.cuda.empty_cache()
    return {"k": k, "grid": n, "subdomains": P * P, "ovlp": d[20], "pml": d[21],
            "global_pml": G, "band_max": max(e[1] for e in desc) + 1,
            "W_max": max(e[2] for e in desc), "solver": solver, "iters": it,
            "relres": rr if math.isfinite(rr) else None,
            "converged": rc == rp.RAS_OK, "status": rc,
            "setup_s": round(t1 - t0, 4), "solve_s": round(t2 - t1, 4)}


def paper_tables(max_k):
    """Section 4's covering on one GPU: k = 300 ... max_k, grid (2k)^2 (12
    points per wavelength), P = k/150 subdomains per side (300-cell cores of
    the interior grid; the covering divides the grid with its global PML),
    overlap and PML from the width rule, a global PML of three wavelengths,
    g = 10 k x^3, the smoothed point source, rtol 1e-10, at most 500
    iterations, mixed precision.  Subdomain bands of 323..375: the wide
    kernels.
      - "tables12": C_delta = 1/6, C_kappa = 3/8; RAS-PML-Imp, RAS-PML-Drch
        and RAS-Imp; Richardson and GMRES(100) (GMRES up to k = 1200, whose
        Krylov basis still fits beside the factors).
      - "table4": C_delta = 1/6, C_kappa = 1/2; RAS-PML-Imp Richardson;
        setup and solve seconds.
      - "table3": RAS-PML-Imp Richardson with the PML a fixed two
        wavelengths and the overlap two thirds of a wavelength or from the
        rule, and with the rule's PML (C_kappa = 1/2) and an overlap of a
        third of a wavelength (the fourth column pair of Table 3 is
        Table 4's set-up)."""
    import torch
    import paper_2602_00735_amd as rp
    torch.cuda.set_device(0)
    ks = [k for k in (300.0, 600.0, 1200.0, 2400.0) if k <= max_k]
    run = section4_run

    run(300.0, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")       # warm-up
    for k in ks:
        r = run(k, rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE, 0.5, "richardson")
        r.update(table="table4", variant="RAS-PML-Imp",
                 total_per_k=round((r["setup_s"] + r["solve_s"]) / k, 6))
        print(json.dumps(r), flush=True)
    for k in ks:
        cells = lambda wavelengths: int(math.floor(wavelengths * 2 * math.pi / k * 2 * k + 1e-9))
        for name, pml, ov in (("pml 2 wavelengths, ovlp 2/3 wavelength", cells(2.0), cells(2.0 / 3.0)),
                              ("pml 2 wavelengths, ovlp rule", cells(2.0), None),
                              ("pml rule, ovlp 1/3 wavelength", rp.RAS_WIDTH_RULE, cells(1.0 / 3.0))):
            r = run(k, rp.RAS_BC_IMP, pml, 0.5, "richardson", overlap=ov)
            r.update(table="table3", variant=name)
            print(json.dumps(r), flush=True)
    variants = (("RAS-PML-Imp", rp.RAS_BC_IMP, rp.RAS_WIDTH_RULE),
                ("RAS-PML-Drch", rp.RAS_BC_DRCH, rp.RAS_WIDTH_RULE),
                ("RAS-Imp", rp.RAS_BC_IMP, 0))
    for k in ks:
        for name, bc, pml in variants:
            for solver in ("richardson", "gmres"):
                if solver == "gmres" and k > 1200.0:
                    continue
                r = run(k, bc, pml, 3.0 / 8.0, solver)
                r.update(table="tables12", variant=name)
                print(json.dumps(r), flush=True)


def warmstart(args):
    """Learned warm start (config: k = 320, h = 1/640, 16 x 16 subdomains,
    overlap = PML = global PML = ceil(ln k / (k h)) = 12 cells, sources of 1-4
    Gaussians of width 0.03 as in the 32-problem batch, mixed precision,
    GMRES(100) to rtol 1e-6).  Training seeds 1..N, held-out seeds from
    100001.  One JSON line per phase."""
    import numpy as np
    import torch
    import paper_2602_00735_amd as rp
    from paper_2602_00735_amd import inputs
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    k, n, P = 320.0, 640, 16
    h = 1.0 / n
    L = log_width(k, h)
    G = L
    H = rp.ras_pml_setup(k, h, (n, n), (P, P), L, L, rp.default_opts(global_pml=G))
    assert H.grid_side() == n
    channels = (16, 32, 64, 64, 64)

    draw = inputs.warm_draw if args.ws_source == "gaussian" else inputs.warm_draw_narrow
    # sources and targets at unit scale (the map f -> u is linear)
    fscale = 1.0 if args.ws_source == "gaussian" else 16.0 * k * k / math.pi ** 3

    def problem(seed):
        f = torch.from_numpy(inputs.batch_source(n, G, draw(seed, k))).to(dev)
        b = torch.empty_like(f)
        rp.ras_pml_rhs(H, f, b)
        return f, b

    # ------------------------------------------------------------ data
    N = args.ws_train
    X = torch.empty((N, n, n, 2), dtype=torch.float32, device=dev)
    T = torch.empty_like(X)
    t0 = time.perf_counter()
    its = []
    for i in range(N):
        f, b = problem(1 + i)
        x = torch.zeros_like(f)
        rc, it, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-6, restart=100, maxit=500)
        assert rc == rp.RAS_OK
        its.append(it)
        rp.ras_pml_grid_sample(H, f, 1.0 / fscale, X[i])
        rp.ras_pml_grid_sample(H, x, k * k / fscale, T[i])
        if (i + 1) % 512 == 0:
            torch.cuda.synchronize()
            print(json.dumps({"phase": "data", "solved": i + 1, "s": round(time.perf_counter() - t0, 1),
                              "mean_iters": round(float(np.mean(its)), 2)}), flush=True)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0

    # ------------------------------------------------------------ training
    net = rp.WSNet(n, channels, args.ws_batch)
    net.set_weights(inputs.ws_init_weights(rp.ws_shapes(channels), 0))
    rng = np.random.default_rng(0)
    Bt = args.ws_batch
    steps_per_epoch = N // Bt
    xb = torch.empty((Bt, n, n, 2), dtype=torch.float32, device=dev)
    tb = torch.empty_like(xb)
    # algorithmic flops of one training step: forward, input gradient (all but
    # the first convolution) and weight gradient of every 3 x 3 convolution
    # and its algorithmic HBM bytes: every convolution reads its input and
    # writes its output (bf16, channels padded to 16; the network's input and
    # its output and output gradient are two fp32 channels, 8 bytes a pixel),
    # the input gradient reads the masked output gradient and writes the
    # input gradient, the weight gradient reads input and masked gradient,
    # and the kernel that writes a masked gradient reads the activation for
    # its ReLU mask
    lv = (0, 1, 2, 3, 4, 3, 2, 1, 0, 0)
    cp = lambda c: (c + 15) // 16 * 16
    flops = nbytes = 0.0
    for li, (ci, co) in enumerate(rp.ws_shapes(channels)):
        m = Bt * (n >> lv[li]) ** 2
        flops += (3 if li > 0 else 2) * 2.0 * m * 9 * ci * co
        a = 8.0 * m if li == 0 else 2.0 * m * cp(ci)
        b = 8.0 * m if li == 9 else 2.0 * m * cp(co)
        nbytes += (a + b) * (3 if li > 0 else 2) + (b if li < 9 else 0)
    t0 = time.perf_counter()
    step_times = []
    for ep in range(args.ws_epochs):
        lr = 1e-3 if ep < args.ws_epochs - 1 else 3e-4
        perm = rng.permutation(N)
        losses = []
        te = time.perf_counter()
        for st in range(steps_per_epoch):
            idx = torch.from_numpy(perm[st * Bt:(st + 1) * Bt]).to(dev)
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(T, 0, idx, out=tb)
            want = st % 64 == 0
            loss = net.train_step(xb, tb, lr, want_loss=want)
            if want:
                losses.append(loss)
        torch.cuda.synchronize()
        dt = time.perf_counter() - te
        step_times.append(dt / steps_per_epoch)
        print(json.dumps({"phase": "train", "epoch": ep + 1, "lr": lr, "s": round(dt, 2),
                          "loss_first": losses[0], "loss_last": losses[-1]}), flush=True)
    t_train = time.perf_counter() - t0
    # one step timed alone with HIP events (the training step's kernels)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        net.gradient(xb, tb, want_grad=False)
    e1.record()
    torch.cuda.synchronize()
    grad_ms = e0.elapsed_time(e1) / 10
    e0.record()
    for _ in range(10):
        net.forward(xb)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10

    # ------------------------------------------------------------ held-out
    res = {"zero": [], "warm": []}
    used = 0
    for i in range(args.ws_test):
        f, b = problem(100001 + i)
        x = torch.zeros_like(f)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        rc, it0, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-6, restart=100, maxit=500)
        torch.cuda.synchronize()
        tb_ = time.perf_counter()
        x0 = torch.empty_like(f)
        u = rp.ras_pml_warm_start(H, net, f, b, x0, fscale)
        rc1, it1, rr1, _ = rp.gmres_solve(H, b, x0, rtol=1e-6, restart=100, maxit=500)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        assert rc == rp.RAS_OK and rc1 == rp.RAS_OK
        used += int(u)
        res["zero"].append((it0, tb_ - ta))
        res["warm"].append((it1, tc - tb_))
    z = np.array(res["zero"])
    w = np.array(res["warm"])
    out = {
        "phase": "result",
        "workload": "learned warm start: k=320 h=1/640 16x16 subdomains overlap=pml=%d, "
                    "1-4 %s, GMRES(100) rtol 1e-6, mixed precision"
                    % (L, "Gaussians (width 0.03)" if args.ws_source == "gaussian"
                       else "smoothed point sources (width pi/(4k))"),
        "network": {"levels": 5, "channels": channels, "grid": n, "weights": net.nweights,
                    "dtype": "bf16 weights/activations, fp32 accumulation and Adam"},
        "training": {"pairs": N, "epochs": args.ws_epochs, "batch": Bt, "data_s": round(t_data, 1),
                     "train_s": round(t_train, 1), "samples_per_s": round(N * args.ws_epochs / t_train, 1),
                     "mean_iters_from_zero": round(float(np.mean(its)), 2)},
        "kernels": {"train_step_ms": round(grad_ms, 3), "forward_ms": round(fwd_ms, 3),
                    "train_step_tflops": round(flops / (grad_ms * 1e-3) / 1e12, 2),
                    "bf16_mfma_peak_tflops": 2500.0,
                    "mfma_frac": round(flops / (grad_ms * 1e-3) / 1e12 / 2500.0, 4),
                    "train_step_algorithmic_GB": round(nbytes / 1e9, 3),
                    "train_step_GBs": round(nbytes / (grad_ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(nbytes / (grad_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "bound": "hbm (about 70 flop per byte at 16 channels, below the bf16 ridge)"},
        "held_out": {"seeds": args.ws_test, "guess_kept": used,
                     "iters_zero_mean": round(float(z[:, 0].mean()), 2),
                     "iters_warm_mean": round(float(w[:, 0].mean()), 2),
                     "time_zero_ms_mean": round(1000 * float(z[:, 1].mean()), 3),
                     "time_warm_ms_mean": round(1000 * float(w[:, 1].mean()), 3),
                     "note": "warm times include the network's forward pass and the residual test"},
    }
    net.close()
    H.close()
    print(json.dumps(out), flush=True)


def batch32(dev, no_fp64):
    """The 32 seeded multi-source problems (seeds 0..31: k from {40, 80, 160},
    h = 1/(2k), G = overlap = PML = L, P = ceil(Nc / 22)) in one handle: setup,
    right-hand sides and one GMRES(100) call to rtol 1e-6 for all of them,
    timed end to end after one untimed run."""
    import numpy as np
    import torch
    import paper_2602_00735_amd as rp
    from paper_2602_00735_amd import inputs
    ks, hs, grids, subs, ovs, fs = [], [], [], [], [], []
    for seed in range(32):
        d = inputs.batch_draw(seed)
        k = d["k"]
        n = int(round(2 * k))
        L = log_width(k, 1.0 / n)
        P = -(-(n + 2 * L) // 22)
        ks.append(k); hs.append(1.0 / n); grids.append((n, n)); subs.append((P, P)); ovs.append(L)
        fs.append(inputs.batch_source(n, L, d))
    f = torch.from_numpy(np.concatenate(fs)).to(dev)
    res = {"problems": 32, "unknowns": int(f.numel()),
           "subdomains": int(sum(P * Q for P, Q in subs))}
    import tempfile
    for name, prec in (("mixed", rp.RAS_MIXED), ("fp64", rp.RAS_FP64)):
        if name == "fp64" and no_fp64:
            continue
        # the tuner on this batch (bands 36..68: window classes of 3..5
        # tiles), its timings reported; the timed runs use its choices
        cache = os.path.join(tempfile.gettempdir(), "ras_pml_tune_batch32_%s_%d.json"
                             % (name, os.getpid()))
        Ht = rp.ras_pml_setup_batch(ks, hs, grids, subs, ovs, ovs, rp.default_opts(precision=prec))
        rp.ras_pml_autotune(Ht, cache)
        tun = rp.ras_pml_tuning(Ht)
        times = rp.ras_pml_tune_report(Ht)
        Ht.close()
        opts = rp.default_opts(precision=prec)
        opts.tune_cache = os.fsencode(cache)
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = rp.ras_pml_setup_batch(ks, hs, grids, subs, ovs, ovs, opts)
            b = torch.empty_like(f)
            x = torch.zeros_like(f)
            rp.ras_pml_rhs(H, f, b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            rc, it, rr, _ = rp.gmres_solve(H, b, x, rtol=1e-6, restart=100, maxit=500)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            per = [rp.ras_pml_batch_result(H, m) for m in range(32)]
            alloc = rp.ras_pml_get_stats(H)["alloc_ms"] / 1000.0
            H.close()
        res[name] = {"total_s": round(t2 - t0, 5), "setup_s": round(t1 - t0, 5),
                     "solve_s": round(t2 - t1, 5), "device_alloc_s": round(alloc, 5),
                     "status": rc,
                     "iters_max": max(p[0] for p in per), "iters_min": min(p[0] for p in per),
                     "all_converged": all(p[2] for p in per),
                     "relres_max": max(p[1] for p in per),
                     "tuning": {"band_solve_deep_prefetch": tun["solve_deep"],
                                "band_solve_queue": tun["solve_queue"],
                                "factor_classes": [{"tiles": g[0], "subdomains": g[1],
                                                    "variant": LU_VARIANTS[g[2]]}
                                                   for g in tun["ldlt"]],
                                "times_ms": times}}
        os.remove(cache)
    return res


def cpu_oracle(k, n_int, P, L, G, fsrc, xs, workload):
    """The CPU oracle on the whole workload, outside the timed region: every
    subdomain assembled and factorised (complex128), then its GMRES(100) to
    rtol 1e-6 on each source.  Returns the cpu_baseline record (setup + solve
    of the Gaussian, on every host thread the oracle uses; one apply on one
    thread beside it) and the relative l2 distance of each GPU solution from
    the oracle's."""
    import numpy as np
    from oracle import band, fem, geometry, gmres, ras
    from paper_2602_00735_amd import inputs
    pb = geometry.Problem(k=k, n_int=n_int, G=G, Px=P, Py=P, delta=L, kappa=L, sigma=10 * k)
    cores = band.nthreads()
    t0 = time.perf_counter()
    R = ras.RasPml(pb)
    t_setup = time.perf_counter() - t0
    progress("oracle setup %.1f s" % t_setup)
    errs, solves = {}, {}
    for src, f in fsrc.items():
        b = fem.rhs(R.M1, f)
        t0 = time.perf_counter()
        ref = gmres.gmres(lambda x: R.A @ x, R.apply, b, rtol=1e-6, restart=100, maxit=500)
        solves[src] = (time.perf_counter() - t0, ref.iters, ref.relres)
        progress("oracle GMRES (%s source) %.1f s, %d iterations" % (src, solves[src][0], ref.iters))
        xr = ref.x
        e = {"oracle_iters": ref.iters, "oracle_relres": ref.relres}
        for name, x in xs.get(src, {}).items():
            e[name] = float(np.linalg.norm(x.cpu().numpy() - xr) / np.linalg.norm(xr))
        errs[src] = e
    v = inputs.random_vector(pb.ndof, 1)
    t0 = time.perf_counter()
    R.apply(v)
    t_apply = time.perf_counter() - t0
    band.set_threads(1)
    t0 = time.perf_counter()
    R.apply(v)
    t_apply1 = time.perf_counter() - t0
    band.set_threads(None)
    progress("oracle applies %.2f s (%d threads), %.2f s (1 thread)" % (t_apply, cores, t_apply1))
    head = next(iter(fsrc))
    ts, it, rr = solves[head]
    cb = {"value": round(t_setup + ts, 3),
          "unit": "s per solve to a true relative residual <= 1e-6 (setup + solve, measured)",
          "cores": cores, "kind": "oracle",
          "sample": "the whole workload (no sampling): all %d subdomains assembled and "
                    "factorised in complex128, then GMRES(100) to rtol 1e-6 from zero on the "
                    "%s source (%d iterations)" % (P * P, head, it),
          "setup_s": round(t_setup, 3), "solve_s": round(ts, 3), "iters": it,
          "relres": rr, "apply_s": round(t_apply, 4),
          "apply_1thread_s": round(t_apply1, 4), "host_cpus": os.cpu_count()}
    if "paper" in solves and head != "paper":
        cb["paper_source_solve_s"] = round(solves["paper"][0], 3)
    del R
    return cb, errs


if __name__ == "__main__":
    main()
