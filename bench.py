"""DDPS benchmark: time-to-solution on one MI355X.

A step is one pass of the whole hot path on a resident system: refresh the
matrix values (device scan, stages 1/3/5), factor the blocks and compute the
spikes (stages 2/4), and solve Ax = f to ||f - Ax||_inf / ||f||_inf <= tol
(stage 6 with the Figure 2 preconditioner).  The inputs (CSR and f) are in HBM
before the timed region starts.

Default workload (the full combination): 3D 7-point variable-coefficient
diffusion-reaction, lognormal(0,1) coefficients, reaction 0.1, on a
40 x 40 x 4096 grid (n = 6,553,600), p = 512 slabs of 8 planes (block n
12,800, band 1600), 8 right-hand sides f = A x*, x* ~ U[-1,1].

The timed configuration (`value`) is the mixed-precision solver (factors and
spikes on bf16 MFMA with split FP32 operands, FP64 refinement, the inner
BiCGStab preconditioned by the interface-local I - N) with the learned guess
of the reduced solves, trained beforehand (untimed, reported) on plain solves
of 32 random right-hand sides of the same matrix.  The same solver without
the learned guess, the plain FP64 solver (the paper's method: unpreconditioned
inner BiCGStab; spike tips only and re-solved retrieval, which is what fits in
memory), and FP64 with the same inner preconditioner are timed on the same GPU
in the same run.  So is the path with incomplete block factors (ILU(0) of
every block, FP32 tips, the outer BiCGStab), reported under "ilu0".

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode M] [--config c5|c2|c3|c1] [--no-cpu]
       python bench.py --config c4 [--mode M]   (learned-guess time sequence)
       python bench.py --ilu-only               (only the incomplete-factor leg)
       python bench.py --delta-sweep            (outer iterations against the drop tolerance)
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
             inner_prec=0, tune_cache=None, retrieval=0, tune_budget=60.0, learned=None, compare_steps=0,
             backward_error_block=None, kappa=False, reduced="bicgstab"):
    """Set up one solver on the workload, tune its execution form, and time
    `steps` whole-path steps (refresh values, factor, solve) after `warmup`.
    learned: None, or dict(K, epochs, budget_s) -- the learned guess of a
    fixed matrix is trained first (untimed, reported) and attached during
    the timed steps; compare_steps more steps then run without it."""
    import torch
    from paper_1008_1700_amd import ddps
    A = d["A"]
    fh = d["f"]
    k = 1 if fh.ndim == 1 else fh.shape[1]
    S = ddps.Solver(A, d["part_ptr"], dtype=mode, inner_tol=inner_tol, outer="refine", max_rhs=k,
                    inner_prec=inner_prec, retrieval=retrieval, reduced=reduced)
    if k == 1:
        f = torch.from_numpy(np.ascontiguousarray(fh)).cuda()
        x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    else:
        f = torch.from_numpy(np.ascontiguousarray(fh.T)).cuda()        # row j = right-hand side j
        x = torch.zeros(k, A.n, dtype=torch.float64, device="cuda")
    val = S.val
    log(f"{mode}: setup done, n={A.n}, retrieval={retrieval}, reduced={reduced}, "
        f"{ddps.ddps_memory(S.h) / 1e9:.1f} GB")
    if exec_form is None:
        tune = ddps.ddps_autotune(S.h, tune_cache, tune_budget)   # execution form (stream groups, tiles), untimed
    else:
        ddps.ddps_set_execution(S.h, exec_form[0], False, exec_form[1])
        tune = dict(streams=exec_form[0], tile_policy=exec_form[1], factor_ms=None)

    def step():
        ddps.ddps_refactor_values(S.h, val)
        ddps.ddps_factor(S.h)
        if k == 1:
            return S.solve(f, x, tol, check=False)
        return ddps.ddps_solve_many(S.h, f, x, tol, check=False)

    def timed(nsteps):
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(nsteps):
            infos.append(step())
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / nsteps, infos[-1]

    log(f"{mode}: execution form {tune}")
    G = None
    gstats = None
    if learned:
        from paper_1008_1700_amd import guess
        ddps.ddps_factor(S.h)
        G, gstats = guess.train_rhs_guess(S, A, K=learned["K"], seed=learned.get("seed", 3), tol=tol,
                                          epochs=learned["epochs"], time_budget_s=learned["budget_s"], log=log)
        G.attach(True)
    for _ in range(warmup):
        step()
    c0 = ddps.ddps_guess_counts(S.h)
    ms, (rc, info) = timed(steps)
    log(f"{mode}: {steps} timed steps, {ms:.1f} ms each (factor {info.t_factor_ms:.1f}, solve {info.t_solve_ms:.1f},"
        f" {info.applications} applications, {info.inner_iters_avg:.2f} inner its)")
    xs = x.cpu().numpy()
    compare = None
    if G is not None:
        c1 = ddps.ddps_guess_counts(S.h)
        gstats["chosen_in_timed_steps"] = {q: c1[q] - c0[q] for q in c1}
        gstats["trial"] = ddps.ddps_guess_trial(S.h)
        G.attach(False)
        if compare_steps > 0:
            step()
            ms2, (rc2, info2) = timed(compare_steps)
            compare = dict(ms_per_step=ms2, steps=compare_steps, rc=rc2, factor_ms=info2.t_factor_ms,
                           solve_ms=info2.t_solve_ms, applications=info2.applications,
                           inner_iters_avg=info2.inner_iters_avg, relres_inf=info2.relres_inf)
            log(f"{mode}: without the learned guess {ms2:.1f} ms per step (solve {info2.t_solve_ms:.1f}, "
                f"{info2.inner_iters_avg:.2f} inner its)")
        G.attach(True)
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
    if G is not None:
        G.close()
    Ssp = A.scipy()
    X = xs if k == 1 else xs.T
    r = fh - Ssp @ X
    nf = np.linalg.norm(fh, np.inf, axis=0)
    xst = d["x_star"]
    out = dict(
        mode=mode, retrieval=retrieval, reduced=reduced, rc=rc, ms_per_step=ms, rhs=k,
        factor_ms=info.t_factor_ms, solve_ms=info.t_solve_ms,
        outer_iters=info.outer_iters, inner_iters_avg=info.inner_iters_avg,
        applications=info.applications, loosened_steps=info.loosened_steps, undone_steps=info.undone_steps,
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
    if gstats is not None:
        out["learned_guess"] = gstats
        out["without_learned_guess"] = compare
    if backward_error_block is not None:
        out["factor_backward_error"] = factor_backward_error(S, d, backward_error_block)
        log(f"{mode}: factor backward error {out['factor_backward_error']}")
    if kappa:
        out["kappa_inf"] = kappa_inf_certificate(S, d)
        log(f"{mode}: kappa_inf {out['kappa_inf']}")
    S.close()
    del f, x
    torch.cuda.empty_cache()
    return out


def run_ilu(d, mode, steps, warmup, tol, inner_tol, inner_prec=1):
    """The same whole path with incomplete block factors (ILU(0) of every
    A_ii, Section 3's L~_i U~_i; tips only, re-solved retrieval) and the
    outer BiCGStab that wins back what they leave: `steps` timed steps
    (refresh values, factor, solve) after `warmup`, then one untimed step
    with the ILU block solves timed by HIP events."""
    import torch
    from paper_1008_1700_amd import ddps
    A = d["A"]
    fh = d["f"]
    k = 1 if fh.ndim == 1 else fh.shape[1]
    S = ddps.Solver(A, d["part_ptr"], dtype=mode, inner_tol=inner_tol, outer="bicgstab", max_rhs=k,
                    inner_prec=inner_prec, retrieval=1, block_factor="ilu0")
    f = torch.from_numpy(np.ascontiguousarray(fh.T if k > 1 else fh)).cuda()
    x = torch.zeros((k, A.n) if k > 1 else (A.n,), dtype=torch.float64, device="cuda")
    log(f"ilu0 {mode}: setup done, {ddps.ddps_memory(S.h) / 1e9:.1f} GB")

    def step():
        x.zero_()
        ddps.ddps_refactor_values(S.h, S.val)
        ddps.ddps_factor(S.h)
        return ddps.ddps_solve_many(S.h, f.reshape(k, A.n), x.reshape(k, A.n), tol, check=False)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rc, info = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    log(f"ilu0 {mode}: {ms:.1f} ms per step (factor {info.t_factor_ms:.1f}, solve {info.t_solve_ms:.1f}, "
        f"{info.outer_iters} outer its, {info.applications} applications)")
    xs = x.reshape(k, A.n).cpu().numpy().T
    sweeps = dict(launches=0, ms=0.0, bytes=0.0)
    for kind in ("sweep", "retrieval"):
        ddps.ddps_timing_read(S.h, kind)
        ddps.ddps_timing_enable(S.h, kind, True)
    step()
    torch.cuda.synchronize()
    for kind in ("sweep", "retrieval"):
        ddps.ddps_timing_enable(S.h, kind, False)
        tk = ddps.ddps_timing_read(S.h, kind)
        for q in ("launches", "ms", "bytes"):
            sweeps[q] += tk[q]
    r = fh.reshape(A.n, k) - A.scipy() @ xs
    nf = np.linalg.norm(fh.reshape(A.n, k), np.inf, axis=0)
    xst = d["x_star"].reshape(A.n, k)
    out = dict(mode=mode, block_factor="ilu0", rc=rc, ms_per_step=ms, steps=steps, factor_ms=info.t_factor_ms,
               solve_ms=info.t_solve_ms, outer_iters=info.outer_iters, applications=info.applications,
               inner_iters_avg=info.inner_iters_avg, inner_tol=inner_tol, inner_prec=inner_prec,
               relres_inf=float(np.max(np.max(np.abs(r), axis=0) / nf)),
               relerr_xstar=float(np.max(np.linalg.norm(xs - xst, axis=0) / np.linalg.norm(xst, axis=0))),
               block_solve=dict(kernel="k_ilu_solve", launches=sweeps["launches"],
                                avg_launch_us=sweeps["ms"] * 1e3 / max(sweeps["launches"], 1),
                                algorithmic_bytes_per_launch=sweeps["bytes"] / max(sweeps["launches"], 1),
                                GBps=sweeps["bytes"] / (sweeps["ms"] * 1e-3) / 1e9 if sweeps["ms"] > 0 else None),
               mem_gb=ddps.ddps_memory(S.h) / 1e9)
    S.close()
    del f, x
    torch.cuda.empty_cache()
    return out


SWEEP_DELTAS = [0.99, 0.9, 0.6, 0.3, 0.1, 1e-5]   # the drop tolerances of the paper's Table 6


def run_delta_sweep(args):
    """Outer iterations against the drop tolerance delta (Section 4, Table 6:
    p = 16, outer BiCGStab to ||f - Ax||_inf / ||f||_inf <= 1e-5 within 1000
    iterations, inner unpreconditioned BiCGStab to 1e-4 within 100) on a
    general sparse matrix: an unstructured mesh-like M-matrix (random
    geometric graph of 400,000 points, about 8 neighbours, lognormal(0,1)
    coupling magnitudes, diagonal dominance margin 0.02-0.04) reordered by
    reverse Cuthill-McKee and cut into 16 equal slabs.  FP64 exact block
    factors, bf16x3 exact block factors (FP32 storage) and FP64 ILU(0) block
    factors, all with the spike tips only.  F2 marks a run that ends above
    the tolerance, as in the paper."""
    import torch
    from paper_1008_1700_amd import ddps
    from workloads import pde
    A = pde.random_geometric(400000, 8, 7, sigma=1.0, margin=0.02, margin_rand=0.02)
    gs = ddps.GeneralSystem(A.n, A.row_ptr, A.col, A.val, 16)
    p = len(gs.part_ptr) - 1
    log(f"delta sweep: n={A.n} nnz={A.nnz} bandwidth after RCM {gs.b}, p={p}")
    xs = np.random.default_rng(8).uniform(-1, 1, A.n)
    f = torch.from_numpy(gs.to_perm(A.scipy() @ xs)).cuda()
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    tol = 1e-5
    rows = []
    for form, dtype in (("lu", "f64"), ("lu", "bf16x3"), ("ilu0", "f64")):
        for dl in SWEEP_DELTAS:
            S = ddps.Solver(gs, gs.part_ptr, dtype=dtype, delta=dl, outer="bicgstab", inner_tol=1e-4,
                            inner_maxit=100, outer_maxit=1000, retrieval=1, block_factor=form)
            S.factor()
            S.factor()
            # the mask of kept columns is set by the factorisation (dropping rule)
            m, t, _ = ddps.ddps_reduced_layout(S.h)
            mask = torch.empty(max(m, 1), dtype=torch.float64, device="cuda")
            cidx = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
            if m:
                ddps.ddps_reduced_layout(S.h, cidx, mask)
            x.zero_()
            rc, info = S.solve(f, x, tol, check=False)
            r = dict(block_factor=form, dtype=dtype, delta=dl, kept_columns=int(mask[:m].sum().item()) if m else 0,
                     outer_iters=info.outer_iters, applications=info.applications,
                     inner_iters_avg=info.inner_iters_avg, relres_inf=info.relres_inf,
                     status="ok" if info.relres_inf <= tol else "F2", factor_ms=info.t_factor_ms,
                     solve_ms=info.t_solve_ms, rc=rc)
            log(f"delta sweep {form} {dtype} delta={dl:g}: {json.dumps(r)}")
            rows.append(r)
            S.close()
    torch.cuda.empty_cache()
    print(json.dumps(dict(metric="DDPS outer BiCGStab iterations against the drop tolerance (Table 6 setting)",
                          unit="outer iterations", higher_is_better=False, n_gpus=1, dtype="f64, bf16x3+f64",
                          data="synthetic",
                          config={"workload": "random geometric graph, n=400000, ~8 neighbours, lognormal(0,1) "
                                              "couplings, RCM + 16 equal slabs", "n": A.n, "nnz": A.nnz,
                                  "bandwidth": gs.b, "t": t, "p": p, "tol": tol, "inner_tol": 1e-4},
                          sweep=rows)), flush=True)


def factor_backward_error(S, d, blk):
    """||A_ii - L~ U~||_F / ||A_ii||_F for block `blk` from the GPU's factor
    tiles (the diagonal tiles hold L_kk^{-1} and U_kk^{-1}, inverted back here
    in float64), tile by tile in the padded block layout, plus the largest
    tile-wise relative error of the off-diagonal factors against the same
    products formed from A and the GPU's own diagonal factors."""
    import scipy.linalg as sla
    import torch
    from paper_1008_1700_amd import ddps
    A = d["A"].scipy()
    part = d["part_ptr"]
    t, tiles, pads = ddps.ddps_block_shape(S.h, len(part) - 1)
    T, pad = tiles[blk], pads[blk]
    lo, hi = int(part[blk]), int(part[blk + 1])
    buf = torch.empty(t * t, dtype=torch.float64, device="cuda")

    def tile(kind, k):
        ddps.ddps_get_tile(S.h, blk, k, kind, buf)
        return buf.cpu().numpy().reshape(t, t).T.copy()

    def a_tile(kr, kc):
        # rows/columns of the padded block (pad identity rows on top)
        out = np.zeros((t, t))
        r0, c0 = kr * t - pad, kc * t - pad
        rs, cs = max(r0, 0), max(c0, 0)
        re, ce = min(r0 + t, hi - lo), min(c0 + t, hi - lo)
        if re > rs and ce > cs:
            out[rs - r0:re - r0, cs - c0:ce - c0] = A[lo + rs:lo + re, lo + cs:lo + ce].toarray()
        if kr == kc:
            for i in range(min(pad - kr * t, t)):
                out[i, i] = 1.0
        return out

    num = den = 0.0
    Lp = Up = None     # L_{k,k-1}, U_{k-1,k}
    for k in range(T):
        D = tile(0, k)
        Lk = sla.inv(np.tril(D, -1) + np.eye(t))
        Uk = sla.inv(np.triu(D))
        Akk = a_tile(k, k)
        E = Akk - Lk @ Uk - (Lp @ Up if k > 0 else 0.0)
        num += float(np.sum(E * E))
        den += float(np.sum(Akk * Akk))
        if k < T - 1:
            Ll, Uu = tile(1, k), tile(2, k)
            Alo, Aup = a_tile(k + 1, k), a_tile(k, k + 1)
            E1, E2 = Alo - Ll @ Uk, Aup - Lk @ Uu
            num += float(np.sum(E1 * E1) + np.sum(E2 * E2))
            den += float(np.sum(Alo * Alo) + np.sum(Aup * Aup))
            Lp, Up = Ll, Uu
    return dict(block=blk, rel_fro=float(np.sqrt(num / den)), t=t, tile_rows=T)


def kappa_inf_certificate(S, d):
    """Two-sided bounds on kappa_inf(A) = ||A||_inf ||A^{-1}||_inf from one
    GPU solve of A y = 1, checked on the CPU: for a matrix with nonpositive
    off-diagonal entries, y > 0 with A y > 0 certifies a nonsingular
    M-matrix, whose inverse is nonnegative, so ||A^{-1}||_inf = ||A^{-1} 1||_inf
    lies between ||y||_inf / ||A y||_inf and ||y||_inf / min(A y) (Berman &
    Plemmons, Ch. 6); A y is formed in float64 on the host and widened by its
    rounding bound.  None if the certificate fails."""
    import torch
    from paper_1008_1700_amd import ddps
    A = d["A"].scipy()
    n = A.shape[0]
    coo = A.tocoo()
    if np.any(coo.data[coo.row != coo.col] > 0):
        return None
    ones = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(ones)
    ddps.ddps_factor(S.h)
    # any y > 0 with A y > 0 certifies; a residual of 1e-10 makes the bracket
    # tight without driving a badly conditioned system to the FP64 floor
    if S.opt.max_rhs > 1:
        ddps.ddps_solve_many(S.h, ones.reshape(1, n), y.reshape(1, n), 1e-10, check=False)
    else:
        S.solve(ones, y, 1e-10, check=False)
    yh = y.cpu().numpy()
    if not np.all(yh > 0):
        return None
    r = A @ yh
    kmax = int(np.max(np.diff(A.indptr)))
    u = np.finfo(np.float64).eps / 2
    err = kmax * u / (1 - kmax * u) * (abs(A) @ yh)
    rmin = float(np.min(r - err))
    if not rmin > 0:
        return None
    ainf = float(np.max(abs(A) @ np.ones(n)))
    ym = float(np.max(yh))
    return dict(lo=ainf * ym / float(np.max(r + err)), hi=ainf * ym / rmin, norm_A_inf=ainf)


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


def _oracle_block_job(args):
    """One sampled block of the CPU oracle in a worker process with
    single-threaded BLAS: stage 2 (exact band LU), stage 4 for `ncols` of the
    block's coupling columns, and one block solve (6.1).  Returns the three
    durations in seconds."""
    n, row_ptr, col, val, lo, hi, ncols = args     # the CSR rows [lo, hi) of A
    import scipy.sparse as sp
    from oracle import ddps_oracle as O
    rows = sp.csr_matrix((val, col, row_ptr), shape=(hi - lo, n))
    Aii = rows[:, lo:hi].tocsr()
    t0 = time.perf_counter()
    fac = O.factor_block(Aii)
    t1 = time.perf_counter()
    coo = rows.tocoo()
    off = (coo.col < lo) | (coo.col >= hi)
    Ri = sp.csc_matrix((coo.data[off], (coo.row[off], coo.col[off])), shape=(hi - lo, n))
    cols = np.unique(coo.col[off])[:ncols]
    if cols.size:
        O.block_solve(fac, Ri[:, cols].toarray())
    t2 = time.perf_counter()
    O.block_solve(fac, np.ones(hi - lo))
    t3 = time.perf_counter()
    return t1 - t0, t2 - t1, t3 - t2, int(cols.size)


def cpu_baseline(d, budget_s=25.0):
    """The CPU oracle (as it stands) timed on a bounded sample of the
    workload: a process pool with one worker per host core and one BLAS
    thread per worker runs, for `cores` sampled blocks at once, the block's
    exact band LU (stage 2), its spikes for a subset of the coupling columns
    (stage 4, LAPACK band solves) and one block solve (6.1).  The full
    figure is extrapolated: per-block column time scaled to all 2b coupling
    columns, then one pool round per `cores` blocks.  The reduced solve (6.3)
    and retrieval (6.5) are not included."""
    import concurrent.futures as cf
    import multiprocessing as mp
    A = d["A"]
    part = d["part_ptr"]
    p = len(part) - 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count() or 1
    b = d["b"]
    ncols = 128
    # sampled blocks: evenly spread over the partition (interior blocks have
    # couplings on both sides)
    nsamp = max(1, min(p, cores))
    idx = np.unique(np.linspace(0, p - 1, nsamp).round().astype(int))
    def rows_of(i):
        lo, hi = int(part[i]), int(part[i + 1])
        a, b2 = A.row_ptr[lo], A.row_ptr[hi]
        return (A.n, A.row_ptr[lo:hi + 1] - a, A.col[a:b2].copy(), A.val[a:b2].copy(), lo, hi, ncols)

    jobs = [rows_of(i) for i in idx]
    # one BLAS thread per worker: the workers are started with these set
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS")
    saved = {k2: os.environ.get(k2) for k2 in keys}
    for k2 in keys:
        os.environ[k2] = "1"
    try:
        t0 = time.perf_counter()
        with cf.ProcessPoolExecutor(max_workers=len(jobs), mp_context=mp.get_context("spawn")) as ex:
            res = list(ex.map(_oracle_block_job, jobs))
        wall = time.perf_counter() - t0
    finally:
        for k2, v in saved.items():
            if v is None:
                os.environ.pop(k2, None)
            else:
                os.environ[k2] = v
    fac = np.array([r[0] for r in res])
    spk = np.array([r[1] * (2 * b / max(r[3], 1)) if r[3] else 0.0 for r in res])
    sol = np.array([r[2] for r in res])
    per_block = fac + spk + sol              # seconds per block on one core
    rounds = int(np.ceil(p / len(jobs)))
    total = float(np.mean(per_block)) * rounds  # each round runs len(jobs) blocks side by side
    return dict(value=total * 1e3, unit="ms", cores=int(len(jobs)), kind="oracle", extrapolated=True,
                sample=(f"{len(jobs)} of {p} blocks (evenly spread), one process and one BLAS thread per block on "
                        f"{cores} host cores: exact band LU, spikes for {ncols} of the 2b = {2 * b} coupling "
                        f"columns (scaled x{2 * b / ncols:g}), one block solve; full figure = mean per-block time x "
                        f"{rounds} rounds of {len(jobs)} blocks; reduced solve and retrieval not included"),
                measured_wall_s=wall, per_block_s=dict(factor=float(np.mean(fac)), spikes_scaled=float(np.mean(spk)),
                                                       block_solve=float(np.mean(sol))))


# The paper's own figures (Tables 2 and 3 of the paper: total solve times of
# the DDPS method, delta = 0.9, 16 MPI processes on a Xeon X5560 cluster, on
# matrices of a public collection): context on different hardware and
# different matrices, not a target.
PAPER_CONTEXT = {
    "hardware": "Intel Xeon X5560 2.8 GHz cluster, InfiniBand, 16 MPI processes (one per core)",
    "note": "different matrices and machine; the paper's Tables 2-3, context only",
    "ddps_16proc_total_s": {"ATMOSMODL n=1489752": 100.7, "RAJAT31 n=4690002": 45.1, "TORSO3 n=259156": 2.1,
                            "XENON2 n=157464": 2.9, "LANGUAGE n=399130": 2.0},
    "pardiso_1core_total_s": {"ATMOSMODL n=1489752": 1291.0, "RAJAT31 n=4690002": 57.9},
}


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
                    inner_prec=args.inner_prec if args.mode != "f64" else 0, reduced=args.reduced)
    tune = ddps.ddps_autotune(S.h, args.tune_cache, args.tune_budget)
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
        "selection_resid_prev_median": float(np.median([r["r_prev"] for r in ev])) if ev else None,
        "selection_resid_learned_median": float(np.median([r["r_learn"] for r in ev])) if ev else None,
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


TUNE_CACHE = os.path.join(ROOT, "paper_1008_1700_amd", "tune_cache.json")
# (mixed, FP64) reduced-solve tolerances: the fastest of a sweep on each
# workload (C5: mixed 1e-4 1646 ms vs 1e-5 1715 ms vs 1e-6 1842 ms; FP64
# 1e-5 4272 ms, 1e-6..1e-9 4309-4314 ms; C2: mixed 1e-6, FP64 1e-9)
INNER_TOL = {"c5": (1e-4, 1e-5), "c2": (1e-6, 1e-9), "c3": (1e-6, 1e-9), "c1": (1e-6, 1e-9)}
# reduced-solve tolerance of the incomplete-factor leg: the fastest of a sweep
# on the 3D benchmark workload (1e-4 .. 1e-1)
ILU_INNER_TOL = 5e-2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", default="bf16x3", choices=["f64", "f32", "bf16x3", "bf16"])
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-baseline", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--baseline-steps", type=int, default=3, help="timed steps of the plain FP64 run (at most --steps)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tol", type=float, default=TOL)
    # defaults: the fastest reduced-solve tolerance of a sweep for each mode
    # and workload (INNER_TOL)
    ap.add_argument("--inner-tol", type=float, default=None, help="reduced-solve tolerance, timed mode")
    ap.add_argument("--inner-tol-f64", type=float, default=None, help="reduced-solve tolerance, FP64 mode")
    ap.add_argument("--inner-prec", type=int, default=1,
                    help="inner BiCGStab preconditioner of the timed mode (0 none, the paper's method; "
                         "1 interface-local I - N).  The plain FP64 baseline always runs the paper's method; "
                         "with 1, FP64 is also timed with the same preconditioner")
    ap.add_argument("--graph-steps", type=int, default=0, help="extra steps timed with the factor graph")
    ap.add_argument("--exec", default=None, help="fixed execution form 'streams,tile_policy' instead of the autotuner")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="JSON file of the autotuner's choices (reused when present, so counter runs repeat the form)")
    ap.add_argument("--copy-probe", action="store_true", help="only run the calibration copy (3 x 1 GiB)")
    ap.add_argument("--retrieval", type=int, default=0, help="timed mode: 0 spikes kept, 1 re-solve with tips only")
    ap.add_argument("--retrieval-f64", type=int, default=-1,
                    help="FP64 baseline: 0 spikes kept, 1 re-solve with tips only, -1 re-solve where full spikes "
                         "do not fit (C3, C5)")
    ap.add_argument("--tune-budget", type=float, default=60.0, help="autotuner time budget per handle (s)")
    ap.add_argument("--no-learned", action="store_true", help="time the mixed solver without the learned guess")
    ap.add_argument("--reduced", default="bicgstab", choices=["bicgstab", "direct"],
                    help="reduced solve of the timed mode (the FP64 baseline keeps BiCGStab)")
    ap.add_argument("--guess-k", type=int, default=32, help="random right-hand sides the learned guess trains on")
    ap.add_argument("--guess-epochs", type=int, default=100)
    ap.add_argument("--guess-budget", type=float, default=30.0, help="training time budget (s)")
    ap.add_argument("--compare-steps", type=int, default=3, help="steps timed without the learned guess")
    ap.add_argument("--c4-steps", type=int, default=300)
    ap.add_argument("--c4-train", type=int, default=200)
    ap.add_argument("--c4-epochs", type=int, default=200)
    ap.add_argument("--no-ilu", action="store_true", help="skip the incomplete-factor (ILU(0)) run")
    ap.add_argument("--ilu-only", action="store_true", help="only run the incomplete-factor leg (one JSON line)")
    ap.add_argument("--ilu-steps", type=int, default=1)
    ap.add_argument("--ilu-inner-tol", type=float, default=None, help="reduced-solve tolerance of the ILU(0) leg")
    ap.add_argument("--delta-sweep", action="store_true",
                    help="only the drop-tolerance sweep on a general sparse matrix (one JSON line)")
    args = ap.parse_args()
    it_mix, it_f64 = INNER_TOL.get(args.config, INNER_TOL["c2"])
    args.inner_tol = it_mix if args.inner_tol is None else args.inner_tol
    args.inner_tol_f64 = it_f64 if args.inner_tol_f64 is None else args.inner_tol_f64
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (--gpus must be 1)",
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
    if args.delta_sweep:
        run_delta_sweep(args)
        return
    exec_form = tuple(int(v) for v in args.exec.split(",")) if args.exec else None
    log(f"building workload {args.config}")
    d = build_workload(args.config)
    log(f"n={d['A'].n} nnz={d['A'].nnz} p={len(d['part_ptr']) - 1}")
    ilu_mode = "f64" if args.mode == "f64" else "f32"
    if args.ilu_only:
        ilu = run_ilu(d, ilu_mode, args.ilu_steps, 1, args.tol, args.ilu_inner_tol or ILU_INNER_TOL, args.inner_prec)
        print(json.dumps(dict(metric="DDPS time-to-solution @rel.resid 1e-10, ILU(0) block factors", value=ilu["ms_per_step"],
                              unit="ms", higher_is_better=False, n_gpus=1, dtype=ilu_mode,
                              config={"workload": WORKLOADS.get(args.config, args.config)}, ilu0=ilu)), flush=True)
        return
    itol = args.inner_tol_f64 if args.mode == "f64" else args.inner_tol
    iprec = args.inner_prec
    learned = None if (args.no_learned or args.mode == "f64" or args.reduced == "direct" or
                       len(d["part_ptr"]) < 3) else dict(
        K=args.guess_k, epochs=args.guess_epochs, budget_s=args.guess_budget, seed=3)
    res = run_mode(d, args.mode, args.steps, args.warmup, args.tol, itol, graph_steps=args.graph_steps,
                   exec_form=exec_form, inner_prec=iprec, tune_cache=args.tune_cache,
                   retrieval=args.retrieval if args.mode != "f64" else max(args.retrieval_f64, 0),
                   tune_budget=args.tune_budget, learned=learned, compare_steps=args.compare_steps,
                   backward_error_block=1 if len(d["part_ptr"]) > 2 else 0, kappa=True, reduced=args.reduced)
    log(f"{args.mode}: {json.dumps(res)}")
    base = None
    rf64 = args.retrieval_f64 if args.retrieval_f64 >= 0 else (1 if args.config in ("c3", "c5") else 0)
    if not args.no_baseline and args.mode != "f64":
        from paper_1008_1700_amd import ddps
        try:
            nb = max(1, min(args.steps, args.baseline_steps))
            base = run_mode(d, "f64", nb, 1, args.tol, args.inner_tol_f64, exec_form=exec_form,
                            tune_cache=args.tune_cache, retrieval=rf64, tune_budget=args.tune_budget)
            base["timed_steps"] = nb
        except ddps.DDPSError as e:
            # FP64 factors beyond the device memory: the paper's failure F1
            base = dict(mode="f64", status=str(e), ms_per_step=None)
        log(f"f64: {json.dumps(base)}")
    # the same inner preconditioner on FP64, so that the precision's share of
    # the speedup is stated on its own
    base_same = None
    if not args.no_baseline and args.mode != "f64" and iprec and base and base.get("ms_per_step"):
        nb = max(1, min(args.steps, args.baseline_steps))
        base_same = run_mode(d, "f64", nb, 1, args.tol, args.inner_tol_f64, exec_form=exec_form, inner_prec=iprec,
                             tune_cache=args.tune_cache, retrieval=rf64, tune_budget=args.tune_budget)
        base_same["timed_steps"] = nb
        log(f"f64 inner_prec {iprec}: {json.dumps(base_same)}")
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
    ilu = None
    if not args.no_ilu and len(d["part_ptr"]) > 2:
        ilu = run_ilu(d, ilu_mode, args.ilu_steps, 1, args.tol, args.ilu_inner_tol or ILU_INNER_TOL, iprec)
        ilu["vs_exact_factors"] = ilu["ms_per_step"] / res["ms_per_step"]
        log(f"ilu0: {json.dumps(ilu)}")
    cpu = None if args.no_cpu else cpu_baseline(d)
    speed = (base["ms_per_step"] / res["ms_per_step"]) if base and base.get("ms_per_step") else None
    speed_same = (base_same["ms_per_step"] / res["ms_per_step"]) if base_same else None
    kappa = res.get("kappa_inf")
    learned_on = "learned_guess" in res
    out = {
        "metric": "DDPS time-to-solution @rel.resid 1e-10, mixed" + ("+learned" if learned_on else "")
                  + " vs plain FP64",
        "note": ("the timed solver preconditions its inner BiCGStab with the interface-local I - N "
                 "(beside the method); plain_f64 is the paper's method in FP64, and "
                 "speedup_vs_f64_same_inner_prec compares with FP64 using the same preconditioner")
                if iprec and args.mode != "f64" else None,
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
        "config": {"workload": WORKLOADS.get(args.config, args.config), "mode": args.mode,
                   "retrieval": res["retrieval"], "inner_prec": iprec, "learned_guess": learned_on},
        "speedup_vs_f64": speed,
        "speedup_vs_f64_same_inner_prec": speed_same,
        "target_speedup": 3.0,
        "target_met": bool(speed is not None and speed >= 3.0),
        "solve": {k2: v for k2, v in res.items() if k2 != "kernel"},
        "plain_f64": base and {k2: v for k2, v in base.items() if k2 != "kernel"},
        "f64_same_inner_prec": base_same and {k2: v for k2, v in base_same.items() if k2 != "kernel"},
        "kappa_inf": kappa,
        "error_bound_inf": (kappa["hi"] * res["relres_inf"]) if kappa else None,
        "algorithmic_flops_factor": alg,
        "roofline": roof,
        "roofline_gemv": roof_gemv,
        "ilu0": ilu,
        "cpu_baseline": cpu,
        "paper_context": PAPER_CONTEXT,
    }
    if cpu:
        out["cpu_baseline"]["gpu_speedup"] = cpu["value"] / res["ms_per_step"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
