"""DDPS benchmark: time-to-solution on one MI355X.

A step is one pass of the whole hot path on a resident system: refresh the
matrix values (device scan, stages 1/3/5), factor the blocks and compute the
spikes (stages 2/4), and solve Ax = f to ||f - Ax||_inf / ||f||_inf <= tol
(stage 6 with the Figure 2 preconditioner).  The inputs (CSR and f) are in HBM
before the timed region starts.

Workload: 3D 7-point upwind convection-diffusion, 32 x 32 x 512 grid
(n = 524,288), velocity (1,1,10), p = 64 slabs of 8 planes (block n 8192,
band 1024, 1024 coupling columns per side), f = A x*, x* ~ U[-1,1].

The timed configuration (`value`) is the mixed-precision solver (factors and
spikes on bf16 MFMA with split FP32 operands, FP64 refinement); the plain
FP64 solver is timed on the same GPU in the same run for the speedup.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode M] [--no-cpu]
       python bench.py --config c4 [--mode M]   (learned-guess time sequence)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {"f64": 78.6e12, "f32": 157.3e12, "bf16x3": 2.5e15, "bf16": 2.5e15}
HBM_PEAK = 8.0e12
TOL = 1e-10


WORKLOADS = {
    "c2": "3D 7-point upwind conv-diff 32x32x512 (n=524288), v=(1,1,10), p=64 slabs of 8 planes, "
          "f=A x*, x*~U[-1,1], tol 1e-10",
    "c3": "2D anisotropic (eps_y 1e-3) lognormal(0,1.5) diffusion 2048x2048 (n=4194304), p=123 uneven slabs "
          "of U{4..28} grid rows (block n 8192-57344, band 2048), f=A x*, tol 1e-10",
    "c5": "3D lognormal(0,1) diffusion + reaction 0.1, 40x40x4096 (n=6553600), p=512 slabs of 8 planes "
          "(block n 12800, band 1600), 8 right-hand sides, f=A x*, tol 1e-10",
    "c1": "2D upwind conv-diff 64x64, v=(20,20), p=4 slabs of 16 rows, f=A x*, tol 1e-10",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(name):
    from workloads import configs
    return configs.BUILDERS[name]()


def run_mode(d, mode, steps, warmup, tol, inner_tol, timing_kind="gemm", graph_steps=None, exec_form=None,
             inner_prec=0, tune_cache=None):
    import torch
    from paper_1008_1700_amd import ddps
    A = d["A"]
    fh = d["f"]
    k = 1 if fh.ndim == 1 else fh.shape[1]
    S = ddps.Solver(A, d["part_ptr"], dtype=mode, inner_tol=inner_tol, outer="refine", max_rhs=k,
                    inner_prec=inner_prec)
    if k == 1:
        f = torch.from_numpy(np.ascontiguousarray(fh)).cuda()
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    else:
        f = torch.from_numpy(np.ascontiguousarray(fh.T)).cuda()        # row j = right-hand side j
        x = torch.zeros(k, A.n, dtype=torch.float64, device="cuda")
    val = S.val
    log(f"{mode}: setup done, n={A.n}")
    if exec_form is None:
        tune = ddps.ddps_autotune(S.h, tune_cache)   # execution form (stream groups, tiles), untimed
    else:
        ddps.ddps_set_execution(S.h, exec_form[0], False, exec_form[1])
        tune = dict(streams=exec_form[0], tile_policy=exec_form[1], factor_ms=None)

    def step():
        ddps.ddps_refactor_values(S.h, val)
        ddps.ddps_factor(S.h)
        if k == 1:
            return S.solve(f, x, tol, check=False)
        return ddps.ddps_solve_many(S.h, f, x, tol, check=False)

    log(f"{mode}: execution form {tune}")
    for _ in range(warmup):
        step()
    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        infos.append(step())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"{mode}: {steps} timed steps, {(t1 - t0) * 1e3 / steps:.1f} ms each")
    rc, info = infos[-1]
    xs = x.cpu().numpy()
    # one more (untimed) step with every factor GEMM launch timed by HIP events
    # on its stream; while they are timed the stream groups run one after
    # another, so each interval holds its own kernel only (the timed steps
    # above run the groups concurrently and carry no per-launch events)
    ddps.ddps_timing_read(S.h, timing_kind)            # clear
    ddps.ddps_timing_enable(S.h, timing_kind, True)
    step()
    torch.cuda.synchronize()
    ddps.ddps_timing_enable(S.h, timing_kind, False)
    tim = ddps.ddps_timing_read(S.h, timing_kind)
    # one more (untimed) step with the solve-phase GEMV launches timed
    gemv = dict(launches=0, ms=0.0, bytes=0.0, per_kind={})
    for kind in ("sweep", "reduced", "retrieval"):
        ddps.ddps_timing_read(S.h, kind)
        ddps.ddps_timing_enable(S.h, kind, True)
    step()
    torch.cuda.synchronize()
    for kind in ("sweep", "reduced", "retrieval"):
        ddps.ddps_timing_enable(S.h, kind, False)
        tk = ddps.ddps_timing_read(S.h, kind)
        gemv["launches"] += tk["launches"]
        gemv["ms"] += tk["ms"]
        gemv["bytes"] += tk["bytes"]
        gemv["per_kind"][kind] = dict(launches=tk["launches"], ms=tk["ms"],
                                      GBps=tk["bytes"] / (tk["ms"] * 1e-3) / 1e9 if tk["ms"] > 0 else None)
    graph_ms = None
    if graph_steps:
        ddps.ddps_set_execution(S.h, tune["streams"], True, tune["tile_policy"])
        step()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(graph_steps):
            step()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) * 1e3 / graph_steps
    Ssp = A.scipy()
    X = xs if k == 1 else xs.T
    r = fh - Ssp @ X
    nf = np.linalg.norm(fh, np.inf, axis=0)
    xst = d["x_star"]
    out = dict(
        mode=mode, rc=rc, ms_per_step=(t1 - t0) * 1e3 / steps, rhs=k,
        factor_ms=info.t_factor_ms, solve_ms=info.t_solve_ms,
        outer_iters=info.outer_iters, inner_iters_avg=info.inner_iters_avg,
        applications=info.applications,
        relres_inf=float(np.max(np.max(np.abs(r), axis=0) / nf)),
        relerr_xstar=float(np.max(np.linalg.norm(X - xst, axis=0) / np.linalg.norm(xst, axis=0))),
        kernel=dict(kind=timing_kind, launches_per_step=tim["launches"], ms_per_step=tim["ms"],
                    flops_per_step=tim["flops"], bytes_per_step=tim["bytes"],
                    timing="one untimed step after the timed steps, per-launch HIP events, "
                           "stream groups one after another"),
        mem_gb=ddps.ddps_memory(S.h) / 1e9,
        inner_tol=inner_tol, gemv=gemv,
        exec=dict(tune, graph_ms_per_step=graph_ms),
    )
    S.close()
    del f, x
    torch.cuda.empty_cache()
    return out


def recorded_traffic(config, mode, launches_per_step):
    """HBM bytes per grouped-GEMM launch from the counter runs recorded in
    profiles/*_traffic.md (rocprofv3 FETCH_SIZE and WRITE_SIZE, each scaled
    by what the counter reads for a plain copy of known size).  None when no
    record matches this workload and mode, or when the GEMM source changed
    since the counters were taken (its hash differs)."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1008_1700_amd", "csrc", "k_gemm.hip")
    try:
        md5 = hashlib.md5(open(src, "rb").read()).hexdigest()
    except OSError:
        return None, None
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        for line in open(path):
            if not line.startswith("traffic: "):
                continue
            rec = json.loads(line[len("traffic: "):])
            if rec.get("config") != config or rec.get("mode") != mode:
                continue
            if rec.get("k_gemm_md5") != md5:
                return None, os.path.basename(path) + " (stale: GEMM source changed)"
            per_launch = rec["fetch_kib_per_launch"] * 1024 * rec["fetch_scale"] + \
                rec["write_kib_per_launch"] * 1024 * rec["write_scale"]
            return per_launch, os.path.basename(path)
    return None, None


def band_lu_spike_flops(d):
    """Leading-order algorithmic flops of stages 2 and 4: 2 n_i b^2 for the
    band LU plus 4 n_i b w_top + 2 n_i b w_bot for the spikes."""
    b = d["b"]
    part = d["part_ptr"]
    p = len(part) - 1
    tot = 0.0
    for i in range(p):
        ni = part[i + 1] - part[i]
        wt = b if i > 0 else 0
        wb = b if i < p - 1 else 0
        tot += 2.0 * ni * b * b + 4.0 * ni * b * wt + 2.0 * ni * b * wb
    return tot


def cpu_baseline(d, budget_s=25.0):
    """The CPU oracle timed on a bounded sample: block 0 of the workload,
    exact band LU (stage 2), spikes for a subset of its coupling columns
    (stage 4), and a block solve (6.1); scaled to the whole workload."""
    import scipy.sparse as sp
    from oracle import ddps_oracle as O
    A = d["A"]
    part = d["part_ptr"]
    p = len(part) - 1
    S = A.scipy()
    lo, hi = part[0], part[1]
    Aii = S[lo:hi, lo:hi].tocsr()
    t0 = time.perf_counter()
    fac = O.factor_block(Aii)
    t_fac = time.perf_counter() - t0
    Ri = S[lo:hi, :].tocsc()
    cols = np.arange(hi, min(hi + d["b"], A.n))
    ncols_total = 2 * d["b"]
    sample = 128
    t0 = time.perf_counter()
    Rt = Ri[:, cols[:sample]].toarray()
    O.block_solve(fac, Rt)
    t_spk = (time.perf_counter() - t0) * (ncols_total / sample)
    t0 = time.perf_counter()
    O.block_solve(fac, np.ones(hi - lo))
    t_sweep = time.perf_counter() - t0
    per_block = t_fac + t_spk + t_sweep
    total = per_block * p
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        th = max((x.get("num_threads", 1) for x in threadpool_info()), default=cores)
    except Exception:
        th = cores
    return dict(value=total * 1e3, unit="ms", cores=int(th), kind="oracle",
                sample=(f"block 0 of {p}: exact band LU, spikes for {sample} of its {ncols_total} coupling "
                        f"columns scaled x{ncols_total // sample}, one block solve; per-block time x {p} "
                        f"blocks (reduced solve not included); host cores available {cores}"),
                measured_s=per_block)


def run_c4(args):
    """C4: 300 implicit-Euler steps of 2D convection-diffusion on 1024^2 with a
    rotating velocity, p = 64.  Steps 1..200 solve with the previous-step
    guess and record training pairs; the network trains on the GPU; steps
    201..300 are solved with both guesses from the same factors."""
    import torch
    from paper_1008_1700_amd import ddps, guess
    from workloads import configs, pde
    nx = ny = 1024
    p = 64
    A1, _ = configs.c4_matrix(1, nx, ny)
    part = pde.slab_partition(ny, ny // p, nx)
    kinds = configs.c4_kinds(A1, nx)
    itol = args.inner_tol_f64 if args.mode == "f64" else args.inner_tol
    S = ddps.Solver(A1, part, dtype=args.mode, inner_tol=itol, outer="refine", guess=True,
                    inner_prec=args.inner_prec if args.mode != "f64" else 0)
    tune = ddps.ddps_autotune(S.h, args.tune_cache)
    log(f"c4: n={A1.n} p={p} mode={args.mode} exec={tune}")
    t0 = time.perf_counter()
    out = guess.run_sequence(S, lambda st: configs.c4_step_values(st, kinds, nx), steps=args.c4_steps,
                             train_steps=args.c4_train, dt=configs.C4_DT, source=1.0, tol=args.tol,
                             hidden=512, epochs=args.c4_epochs, batch_rows=512, lr=1e-3, seed=0, log=log)
    wall = time.perf_counter() - t0
    S.close()
    recs = out["records"]
    ev = [r for r in recs if "r_learn" in r]
    mean = lambda k, rs: float(np.mean([r[k] for r in rs])) if rs else None
    res = {
        "metric": "C4 learned initial guess: reduced-solve start residual and solve time per step, "
                  "learned (judged) vs previous-step guess, steps after training",
        "value": mean("learn_ms", ev), "unit": "ms", "higher_is_better": False,
        "n_gpus": 1, "dtype": {"f64": "f64", "f32": "f32+f64", "bf16x3": "bf16x3+f64", "bf16": "bf16+f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": "2D implicit-Euler upwind conv-diff 1024x1024, dt 1e-3, |v|=50 rotating 1.2 deg/step, "
                               "p=64, source 1, u0=0, tol 1e-10", "steps": args.c4_steps, "train_steps": args.c4_train,
                   "net": "4 layers 4098-512-512-512-2048 bf16/FP32-accumulate, Adam", "epochs": args.c4_epochs,
                   "inner_prec": args.inner_prec if args.mode != "f64" else 0},
        "eval_steps": len(ev),
        "solve_ms_prev": mean("prev_ms", ev), "solve_ms_learned": mean("learn_ms", ev),
        "inner_iters_prev": mean("prev_inner", ev), "inner_iters_learned": mean("learn_inner", ev),
        "judge_resid_prev_median": float(np.median([r["r_prev"] for r in ev])) if ev else None,
        "judge_resid_learned_median": float(np.median([r["r_learn"] for r in ev])) if ev else None,
        "learned_chosen": sum(bool(r["learned"]) for r in ev),
        "guess_ms": mean("guess_ms", ev), "features_ms": mean("features_ms", recs),
        "factor_ms": mean("factor_ms", recs), "train_s": out["train_s"],
        "loss_first_last": [out["loss"][0], out["loss"][-1]] if out["loss"] else None,
        "max_relres": max(r["relres"] for r in recs), "wall_s": wall,
    }
    print(json.dumps(res), flush=True)


def copy_probe(gib=1.0):
    """A plain device-to-device copy of a known size, for scaling the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE) of a profiled run."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_each_way": n * 8, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="bf16x3", choices=["f64", "f32", "bf16x3", "bf16"])
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-baseline", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tol", type=float, default=TOL)
    # defaults: the fastest tolerance of a sweep for each mode on this workload
    ap.add_argument("--inner-tol", type=float, default=1e-6, help="reduced-solve tolerance, timed mode")
    ap.add_argument("--inner-tol-f64", type=float, default=1e-9, help="reduced-solve tolerance, FP64 mode")
    ap.add_argument("--inner-prec", type=int, default=0,
                    help="inner BiCGStab preconditioner of the timed mode (0 none, 1 interface-local)")
    ap.add_argument("--graph-steps", type=int, default=2, help="extra steps timed with the factor graph")
    ap.add_argument("--exec", default=None, help="fixed execution form 'streams,tile_policy' instead of the autotuner")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON file of the autotuner's choices (reused when present, so counter runs repeat the form)")
    ap.add_argument("--copy-probe", action="store_true", help="only run the calibration copy (3 x 1 GiB)")
    ap.add_argument("--c4-steps", type=int, default=300)
    ap.add_argument("--c4-train", type=int, default=200)
    ap.add_argument("--c4-epochs", type=int, default=200)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus must be 1)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.copy_probe:
        copy_probe()
        return
    if args.config == "c4":
        run_c4(args)
        return
    exec_form = tuple(int(v) for v in args.exec.split(",")) if args.exec else None
    log(f"building workload {args.config}")
    d = build_workload(args.config)
    log(f"n={d['A'].n} nnz={d['A'].nnz} p={len(d['part_ptr']) - 1}")
    itol = args.inner_tol_f64 if args.mode == "f64" else args.inner_tol
    iprec = args.inner_prec if args.mode != "f64" else 0
    res = run_mode(d, args.mode, args.steps, args.warmup, args.tol, itol, graph_steps=args.graph_steps,
                   exec_form=exec_form, inner_prec=iprec, tune_cache=args.tune_cache)
    log(f"{args.mode}: {json.dumps(res)}")
    base = None
    if not args.no_baseline and args.mode != "f64":
        from paper_1008_1700_amd import ddps
        try:
            base = run_mode(d, "f64", args.steps, args.warmup, args.tol, args.inner_tol_f64,
                            graph_steps=args.graph_steps, exec_form=exec_form, tune_cache=args.tune_cache)
        except ddps.DDPSError as e:
            # FP64 factors and spikes beyond the device memory: the paper's failure F1
            base = dict(mode="f64", status=str(e), ms_per_step=None)
        log(f"f64: {json.dumps(base)}")
    k = res["kernel"]
    kms = k["ms_per_step"]
    peak = PEAKS[args.mode]
    # achieved: the band-LU + spike algorithmic flops of stages 2 and 4 per
    # step over the summed durations of the grouped GEMM launches of one
    # factorisation (HIP events on each launch's stream, in the GEMM-timed
    # step whose stream groups run one after another).  mfma_rate counts the
    # products the launches execute (tile-granular triangles; three bf16
    # products per split product).
    alg = band_lu_spike_flops(d)
    achieved = alg / (kms * 1e-3) if kms > 0 else 0.0
    split = 3.0 if args.mode == "bf16x3" else 1.0
    traffic, traffic_src = recorded_traffic(args.config, args.mode, k["launches_per_step"])
    roof = dict(bound="mfma", achieved=achieved / 1e12, peak=peak / 1e12, unit="TFLOP/s",
                frac=achieved / peak, traffic=traffic,
                kernel="k_gemm_dl / k_gemm_bf16 / k_gemm_std (grouped GEMM of stages 2 and 4)",
                launches_per_step=k["launches_per_step"], kernel_ms_per_step=kms,
                stream_groups=res["exec"]["streams"], launch_timing=k.get("timing"),
                avg_launch_us=kms * 1e3 / max(k["launches_per_step"], 1),
                algorithmic_flops_per_step=alg,
                mfma_rate=k["flops_per_step"] * split / (kms * 1e-3) / 1e12 if kms > 0 else None,
                traffic_unit="HBM bytes per launch", traffic_source=traffic_src,
                factor_phase_rate=alg / (res["factor_ms"] * 1e-3) / 1e12)
    g = res.get("gemv")
    roof_gemv = None
    if g and g["ms"] > 0:
        bw = g["bytes"] / (g["ms"] * 1e-3)
        roof_gemv = dict(bound="hbm", achieved=bw / 1e9, peak=HBM_PEAK / 1e9, unit="GB/s", frac=bw / HBM_PEAK,
                         kernel="k_gemv (reduced products, block sweeps, retrieval)", launches=g["launches"],
                         algorithmic_bytes=g["bytes"], ms=g["ms"], per_kind=g["per_kind"])
    cpu = None if args.no_cpu else cpu_baseline(d)
    out = {
        "metric": "DDPS time-to-solution @rel.resid 1e-10, mixed vs plain FP64" + (
            " (C2 3D conv-diff 32x32x512, p=64)" if args.config == "c2" else f" ({args.config})"),
        "value": res["ms_per_step"],
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32+f64", "bf16x3": "bf16x3+f64", "bf16": "bf16+f64"}[args.mode],
        "data": "synthetic",
        "config": {"workload": WORKLOADS.get(args.config, args.config), "mode": args.mode, "inner_prec": iprec},
        "solve": {k2: v for k2, v in res.items() if k2 != "kernel"},
        "plain_f64": base and {k2: v for k2, v in base.items() if k2 != "kernel"},
        "speedup_vs_f64": (base["ms_per_step"] / res["ms_per_step"]) if base and base.get("ms_per_step") else None,
        "algorithmic_flops_factor": band_lu_spike_flops(d),
        "roofline": roof,
        "roofline_gemv": roof_gemv,
        "cpu_baseline": cpu,
    }
    if cpu:
        out["cpu_baseline"]["gpu_speedup"] = cpu["value"] / res["ms_per_step"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
