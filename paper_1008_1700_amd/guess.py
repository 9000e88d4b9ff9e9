"""Learned initial guess of the reduced solve over a sequence of systems.

Over the time steps of an implicit integrator the systems A_n x = f_n change
slowly, and so do the interface solutions z^ of step 6.3.  This helper keeps
the previous step's z^ (the fallback guess), records training pairs while
plain solves run, trains the per-interface network on the GPU, and at later
steps proposes z^_0 = z^prev + s_j net([r_j / s_j, z^prev_j / q_j, cos, sin])
from the reduced residual r = g^ - G^ z^prev of the fallback guess
(s_j = max |r_j|, q_j = max |z^prev_j|), keeping whichever of the two
candidates has the smaller reduced residual ||g^ - G^ z^_0||_2 (the judge).

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
