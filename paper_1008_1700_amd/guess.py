"""Learned initial guess of the reduced solve over a sequence of systems.

Over the time steps of an implicit integrator the systems A_n x = f_n change
slowly, and so do the interface solutions z^ of step 6.3.  This helper keeps
the previous step's z^ (the fallback guess), records training pairs while
plain solves run, trains the per-interface network on the GPU, and at later
steps proposes z^_0 = z^prev + s_j net([r_j / s_j, z^prev_j / q_j, cos, sin])
from the reduced residual r = g^ - G^ z^prev of the fallback guess
(s_j = max |r_j|, q_j = max |z^prev_j|), keeping whichever of the two
candidates has the smaller reduced residual ||g^ - G^ z^_0||_2 (the selection rule).

Orchestration only: every numerical step runs in libddps.so
(ddps_reduced_rhs, ddps_guess_*, ddps_mlp_*, ddps_reduced_residual,
ddps_reduced_restrict, ddps_set_guess); torch supplies the device buffers.
"""
from __future__ import annotations

import numpy as np

from . import ddps


class LearnedGuess:
    def __init__(self, h, p, hidden=512, capacity_steps=200, seed=0, max_batch=4096, stream=None):
        import torch
        self.torch = torch
        self.h = h
        self.m, self.t, _ = ddps.ddps_reduced_layout(h)
        self.nif = p - 1
        self.d_in = 4 * self.t + 2
        self.d_out = 2 * self.t
        self.capacity = capacity_steps
        self.max_batch = max(max_batch, self.nif)
        dev = dict(device="cuda")
        f32 = dict(dtype=torch.float32, **dev)
        f64 = dict(dtype=torch.float64, **dev)
        rows = capacity_steps * self.nif
        self.Xd = torch.zeros(rows, self.d_in, **f32)      # recorded features
        self.Td = torch.zeros(rows, self.d_out, **f32)     # recorded targets
        self.Sd = torch.zeros(rows, **f32)                 # recorded scales
        self.X = torch.zeros(self.nif, self.d_in, **f32)
        self.S = torch.zeros(self.nif, **f32)
        self.Y = torch.zeros(self.nif, self.d_out, **f32)
        self.ghat = torch.zeros(max(self.m, 1), **f64)
        self.rprev = torch.zeros(max(self.m, 1), **f64)
        self.zprev = torch.zeros(max(self.m, 1), **f64)
        self.znew = torch.zeros(max(self.m, 1), **f64)
        self.zlearn = torch.zeros(max(self.m, 1), **f64)
        self.count = 0            # recorded steps
        self.recording = False
        self.rng = np.random.default_rng(seed)
        self.net = ddps.ddps_mlp_create(self.d_in, hidden, self.d_out, self.max_batch, seed=seed, stream=stream)

    # -- per step -------------------------------------------------------
    def begin_step(self, f, cos_t=0.0, sin_t=0.0, record=False):
        """g^ of f (steps 6.1-6.2 with the current factors), the reduced
        residual of the previous-step guess and the network inputs of this
        step; with record=True the inputs go to the dataset."""
        self.recording = record and self.count < self.capacity
        ddps.ddps_reduced_rhs(self.h, 1, f, self.ghat)
        self.r_prev = ddps.ddps_reduced_residual(self.h, 1, self.ghat, self.zprev, self.rprev)[0]
        if self.recording:
            r0 = self.count * self.nif
            X, S = self.Xd[r0:r0 + self.nif], self.Sd[r0:r0 + self.nif]
        else:
            X, S = self.X, self.S
        ddps.ddps_guess_features(self.h, 1, self.rprev, self.zprev, cos_t, sin_t, self.d_in, X, S)
        self._cur = (X, S)

    def use_previous(self):
        """Seed the reduced solve with the previous step's z^."""
        ddps.ddps_set_guess(self.h, self.zprev, 1)

    def propose(self):
        """Network guess vs previous-step guess, judged by the reduced
        residual; the winner seeds the reduced solve.  Returns the two
        residuals and the choice."""
        X, S = self._cur
        ddps.ddps_mlp_forward(self.net, self.nif, X, self.Y)
        ddps.ddps_guess_compose(self.h, 1, self.zprev, self.Y, S, self.zlearn)
        r_prev = self.r_prev
        r_learn = ddps.ddps_reduced_residual(self.h, 1, self.ghat, self.zlearn)[0]
        learned = bool(r_learn < r_prev)
        ddps.ddps_set_guess(self.h, self.zlearn if learned else self.zprev, 1)
        return dict(r_prev=r_prev, r_learn=r_learn, learned=learned)

    def end_step(self, x):
        """Record the step's interface solution (the restriction of x to the
        reduced layout) as target and as the next step's fallback guess."""
        ddps.ddps_reduced_restrict(self.h, 1, x, self.znew)
        if self.recording:
            X, S = self._cur
            r0 = self.count * self.nif
            ddps.ddps_guess_target(self.h, 1, self.znew, self.zprev, S, self.Td[r0:r0 + self.nif])
            self.count += 1
        self.zprev, self.znew = self.znew, self.zprev
        self.recording = False

    # -- training ---------------------------------------------------------
    def train(self, epochs=200, batch_rows=512, lr=1e-3):
        """Adam on the recorded pairs; minibatches are contiguous row ranges
        visited in a random order each epoch.  Returns the loss history."""
        rows = self.count * self.nif
        if rows == 0:
            return []
        b = max(1, min(batch_rows, self.max_batch, rows))
        starts = np.arange(0, rows, b)
        hist = []
        for e in range(epochs):
            tot = 0.0
            last = e == epochs - 1 or e == 0
            for s0 in self.rng.permutation(starts):
                s1 = min(rows, s0 + b)
                loss = ddps.ddps_mlp_train_step(self.net, s1 - s0, self.Xd[s0:s1], self.Td[s0:s1], lr,
                                                want_loss=last)
                if last:
                    tot += loss * (s1 - s0)
            if last:
                hist.append(tot / rows)
        return hist

    def close(self):
        if self.net:
            ddps.ddps_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_sequence(S, values_fn, steps, train_steps, dt, source, tol, hidden=512, epochs=200, lr=1e-3,
                 batch_rows=512, seed=0, log=None):
    """Implicit time stepping u_n = A_n^{-1} (u_{n-1} + dt * source), u_0 = 0,
    with one DDPS solve per step on the handle of Solver S (same pattern for
    every A_n; values_fn(step) -> (CSR values of A_n, theta_n)).

    Steps 1..train_steps solve with the previous-step guess and record
    training pairs; the network is then trained; each later step is solved
    twice from the same factors: with the previous-step guess, then with the
    judged learned guess (whose solution continues the sequence).  Returns
    per-step records and the training-loss history."""
    import time
    import torch
    nif = S.p - 1
    LG = LearnedGuess(S.h, S.p, hidden=hidden, capacity_steps=train_steps, seed=seed,
                      max_batch=max(batch_rows, nif), stream=S.stream.cuda_stream)
    n = S.n
    u = torch.zeros(n, dtype=torch.float64, device="cuda")
    f = torch.empty_like(u)
    x = torch.zeros_like(u)
    recs = []
    hist = []
    t_train = 0.0
    try:
        for step in range(1, steps + 1):
            val, th = values_fn(step)
            S.val.copy_(torch.from_numpy(val))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ddps.ddps_refactor_values(S.h, S.val)
            ddps.ddps_factor(S.h)
            torch.add(u, dt * source, out=f)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            train = step <= train_steps
            LG.begin_step(f, np.cos(th), np.sin(th), record=train)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            rec = dict(step=step, factor_ms=(t1 - t0) * 1e3, features_ms=(t2 - t1) * 1e3)
            LG.use_previous()
            _, info = S.solve(f, x, tol)
            rec.update(prev_inner=info.inner_iters_total, prev_ms=info.t_solve_ms, prev_apps=info.applications)
            if not train and LG.count > 0:
                t0 = time.perf_counter()
                jr = LG.propose()
                torch.cuda.synchronize()
                t_guess = (time.perf_counter() - t0) * 1e3
                _, info = S.solve(f, x, tol)
                rec.update(jr, learn_inner=info.inner_iters_total, learn_ms=info.t_solve_ms,
                           learn_apps=info.applications, guess_ms=t_guess)
            rec["relres"] = info.relres_inf
            LG.end_step(x)
            u, x = x, u
            recs.append(rec)
            if step == train_steps:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                hist = LG.train(epochs=epochs, batch_rows=batch_rows, lr=lr)
                torch.cuda.synchronize()
                t_train = time.perf_counter() - t0
                if log:
                    log(f"trained on {LG.count * nif} pairs in {t_train:.2f} s, loss {hist[0]:.3e} -> {hist[-1]:.3e}")
            elif log and step % 25 == 0:
                log(f"step {step}: {rec}")
    finally:
        LG.close()
    return dict(records=recs, loss=hist, train_s=t_train, u=u)


class RhsGuess:
    """Learned guess for one matrix without a time sequence.

    The reduced solution of a right-hand side is z^ = G^^{-1} g^, one linear
    map for every right-hand side and every preconditioner application of the
    same factors.  Training pairs come from plain solves of random right-hand
    sides: the input row of interface j is [r_j / s_j, g^_j / q_j, 0, 0] with
    r = g^ - G^ g^ the residual of the zero-order guess g^ (G^ = I + G(c,c)),
    and the target is (z^_j - g^_j) / s_j, z^ the restriction of the solution
    (exact coupling: the reduced solution is the solution on c).  Once
    trained, the network is attached to the handle (ddps_set_guess_model),
    which then tries it in every application, judged against z0 = 0 and
    z0 = g^ by the reduced residual.

    Orchestration only: every numerical step runs in libddps.so."""

    def __init__(self, h, p, max_rhs, capacity_rhs, hidden=512, seed=0, batch_rows=512, stream=None):
        import torch
        self.torch = torch
        self.h = h
        self.m, self.t, _ = ddps.ddps_reduced_layout(h)
        self.nif = p - 1
        self.d_in = 4 * self.t + 2
        self.d_out = 2 * self.t
        self.kmax = max_rhs
        R = 1 if max_rhs <= 1 else 2 if max_rhs <= 2 else 4 if max_rhs <= 4 else 8
        self.max_batch = max(batch_rows, R * self.nif)
        rows = capacity_rhs * self.nif
        f32 = dict(dtype=torch.float32, device="cuda")
        f64 = dict(dtype=torch.float64, device="cuda")
        self.Xd = torch.zeros(rows, self.d_in, **f32)
        self.Td = torch.zeros(rows, self.d_out, **f32)
        self.Sd = torch.zeros(rows, **f32)
        self.ghat = torch.zeros(max_rhs, max(self.m, 1), **f64)
        self.rb = torch.zeros_like(self.ghat)
        self.zh = torch.zeros_like(self.ghat)
        self.rows = 0
        self.rng = np.random.default_rng(seed)
        self.net = ddps.ddps_mlp_create(self.d_in, hidden, self.d_out, self.max_batch, seed=seed, stream=stream)

    def record(self, F, X):
        """Pairs of k right-hand sides F and their solutions X ((k, n)
        contiguous float64 device tensors) into the dataset."""
        k = F.shape[0]
        r0, r1 = self.rows, self.rows + k * self.nif
        if r1 > self.Xd.shape[0]:
            raise ValueError("training set full")
        ddps.ddps_reduced_rhs(self.h, k, F, self.ghat)
        ddps.ddps_reduced_residual(self.h, k, self.ghat, self.ghat, self.rb)
        ddps.ddps_guess_features(self.h, k, self.rb, self.ghat, 0.0, 0.0, self.d_in, self.Xd[r0:r1], self.Sd[r0:r1])
        ddps.ddps_reduced_restrict(self.h, k, X, self.zh)
        ddps.ddps_guess_target(self.h, k, self.zh, self.ghat, self.Sd[r0:r1], self.Td[r0:r1])
        self.rows = r1

    def train(self, epochs=100, batch_rows=512, lr=1e-3, time_budget_s=None):
        """Adam on the recorded pairs (contiguous minibatches in a random
        order per epoch); returns the mean loss of the first and last epochs
        and the epochs run (fewer when the time budget runs out)."""
        import time
        rows = self.rows
        if rows == 0:
            return dict(loss=[], epochs=0)
        b = max(1, min(batch_rows, self.max_batch, rows))
        starts = np.arange(0, rows, b)
        hist = []
        t0 = time.perf_counter()
        done = 0
        for e in range(epochs):
            last = e == epochs - 1 or (time_budget_s is not None and time.perf_counter() - t0 > time_budget_s)
            want = last or e == 0
            tot = 0.0
            for s0 in self.rng.permutation(starts):
                s1 = min(rows, s0 + b)
                loss = ddps.ddps_mlp_train_step(self.net, s1 - s0, self.Xd[s0:s1], self.Td[s0:s1], lr,
                                                want_loss=want)
                if want:
                    tot += loss * (s1 - s0)
            if want:
                hist.append(tot / rows)
            done = e + 1
            if last:
                break
        return dict(loss=hist, epochs=done)

    def attach(self, on=True):
        ddps.ddps_set_guess_model(self.h, self.net if on else None)

    def close(self):
        if self.net:
            ddps.ddps_set_guess_model(self.h, None)
            ddps.ddps_mlp_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def train_rhs_guess(S, A, K=32, seed=3, tol=1e-10, hidden=512, epochs=100, lr=1e-3, batch_rows=512,
                    time_budget_s=None, log=None):
    """The learned guess of a fixed matrix (the solver S's handle, A its CSR
    on the host): K random right-hand sides f = A x, x ~ U[-1, 1] from
    default_rng(seed), solved in batches of S's max_rhs with the plain
    method, recorded and trained on.  Returns (RhsGuess, stats)."""
    import time
    import torch
    kmax = S.opt.max_rhs
    G = RhsGuess(S.h, S.p, kmax, K, hidden=hidden, seed=seed, batch_rows=batch_rows, stream=S.stream.cuda_stream)
    rng = np.random.default_rng(seed)
    As = A.scipy()
    t0 = time.perf_counter()
    solve_ms = 0.0
    done = 0
    while done < K:
        k = min(kmax, K - done)
        Xs = rng.uniform(-1.0, 1.0, (A.n, k))
        F = torch.from_numpy(np.ascontiguousarray((As @ Xs).T)).cuda()
        X = torch.zeros_like(F)
        rc, info = ddps.ddps_solve_many(S.h, F, X, tol)
        solve_ms += info.t_solve_ms
        G.record(F, X)
        done += k
        del F, X
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tr = G.train(epochs=epochs, batch_rows=batch_rows, lr=lr, time_budget_s=time_budget_s)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    stats = dict(K=K, pairs=G.rows, collect_s=t1 - t0, solve_ms_total=solve_ms, train_s=t2 - t1,
                 epochs=tr["epochs"], loss_first_last=[tr["loss"][0], tr["loss"][-1]] if tr["loss"] else None)
    if log:
        log(f"learned guess: {G.rows} pairs from {K} right-hand sides in {t1 - t0:.1f} s, trained "
            f"{tr['epochs']} epochs in {t2 - t1:.1f} s, loss {stats['loss_first_last']}")
    return G, stats
