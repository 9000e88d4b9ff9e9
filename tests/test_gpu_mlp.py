"""GPU parity of the learned-guess network and its reduced-vector plumbing
against the CPU oracle (oracle/mlp_oracle.py, oracle/ddps_oracle.py).

The network runs bf16 operands with FP32 accumulation; the oracle takes the
same bf16 roundings in float64, so the two differ by accumulation order
(plus the rare bf16 tie or ReLU decision that order flips): the bar is 1e-2
relative, norm-wise per tensor.  Adam is checked on the GPU's own gradients,
where only FP32 vs float64 arithmetic differs.
"""
import numpy as np
import pytest

from tests.gpu_util import dev_vec, host, make_solver, oracle_prec, relerr, torch_cuda
from workloads import configs, pde

pytestmark = pytest.mark.gpu


def _unpack(flat, d_in, H, d_out):
    dims = [d_in, H, H, H, d_out]
    out, o = [], 0
    for a, b in zip(dims[:-1], dims[1:]):
        out.append(flat[o:o + a * b].reshape(a, b).astype(np.float64))
        o += a * b
        out.append(flat[o:o + b].astype(np.float64))
        o += b
    assert o == flat.size
    return out


def _net(d_in, H, d_out, batch, seed):
    from paper_1008_1700_amd import ddps
    net = ddps.ddps_mlp_create(d_in, H, d_out, batch, seed=seed)
    # nonzero biases so the bias paths are exercised
    p = ddps.ddps_mlp_get_params(net)
    rng = np.random.default_rng(seed + 100)
    P = _unpack(p, d_in, H, d_out)
    flat = []
    for i, a in enumerate(P):
        if i % 2 == 1:
            a = 0.05 * rng.standard_normal(a.shape)
        flat.append(a.reshape(-1))
    p = np.concatenate(flat).astype(np.float32)
    ddps.ddps_mlp_set_params(net, p)
    return net, p


# small ragged shapes, then the production network of the time sequence
# (t = 1024: inputs 2 (2t) + 2, outputs 2t, hidden 512) at the batch of one
# step (63 interfaces) and a training batch of 512 rows
SHAPES = [(70, 96, 40, 75), (130, 64, 200, 33), (4098 // 8, 128, 256, 130), (4098, 512, 2048, 63),
          (4098, 512, 2048, 512)]


@pytest.mark.parametrize("d_in,H,d_out,batch", SHAPES)
def test_mlp_forward_matches_oracle(d_in, H, d_out, batch):
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    net, p = _net(d_in, H, d_out, batch, 1)
    try:
        rng = np.random.default_rng(2)
        X = rng.standard_normal((batch, d_in)).astype(np.float32)
        Xd = torch.from_numpy(X).cuda()
        Yd = torch.empty(batch, d_out, dtype=torch.float32, device="cuda")
        ddps.ddps_mlp_forward(net, batch, Xd, Yd)
        torch.cuda.synchronize()
        y_ref, _ = M.forward(_unpack(p, d_in, H, d_out), X.astype(np.float64), bf16=True)
        y = host(Yd).astype(np.float64)
        assert relerr(y, y_ref) <= 1e-2
        assert np.max(np.abs(y - y_ref)) <= 3e-2 * np.max(np.abs(y_ref))
    finally:
        ddps.ddps_mlp_destroy(net)


@pytest.mark.parametrize("d_in,H,d_out,batch", SHAPES)
def test_mlp_gradients_match_oracle(d_in, H, d_out, batch):
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    net, p = _net(d_in, H, d_out, batch, 3)
    try:
        rng = np.random.default_rng(4)
        X = rng.standard_normal((batch, d_in)).astype(np.float32)
        T = rng.standard_normal((batch, d_out)).astype(np.float32)
        g, loss = ddps.ddps_mlp_gradients(net, batch, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
        P = _unpack(p, d_in, H, d_out)
        y, cache = M.forward(P, X.astype(np.float64), bf16=True)
        g_ref = M.backward(P, cache, y, T.astype(np.float64), bf16=True)
        assert abs(loss - M.mse(y, T)) <= 1e-3 * M.mse(y, T)
        G = _unpack(g, d_in, H, d_out)
        for i, (a, b) in enumerate(zip(G, g_ref)):
            assert relerr(a, b) <= 1e-2, (i, relerr(a, b))
    finally:
        ddps.ddps_mlp_destroy(net)


def test_mlp_adam_steps_match_oracle():
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d_in, H, d_out, batch = 50, 64, 30, 40
    net, p0 = _net(d_in, H, d_out, batch, 5)
    try:
        rng = np.random.default_rng(6)
        Xd = torch.from_numpy(rng.standard_normal((batch, d_in)).astype(np.float32)).cuda()
        Td = torch.from_numpy(rng.standard_normal((batch, d_out)).astype(np.float32)).cuda()
        lr = 1e-3
        P = [p0.astype(np.float64)]
        m = [np.zeros(p0.size)]
        v = [np.zeros(p0.size)]
        for t in (1, 2, 3):
            g, _ = ddps.ddps_mlp_gradients(net, batch, Xd, Td)          # GPU gradients at current params
            ddps.ddps_mlp_train_step(net, batch, Xd, Td, lr)             # same gradients, then Adam
            P, m, v = M.adam_step(P, [g.astype(np.float64)], m, v, t, lr=lr)
            got = ddps.ddps_mlp_get_params(net).astype(np.float64)
            err = np.abs(got - P[0])
            assert np.all(err <= 1e-6 * np.abs(P[0]) + 1e-4 * lr), (t, err.max())
            P = [got]       # continue both sides from the GPU's FP32 parameters
    finally:
        ddps.ddps_mlp_destroy(net)


def test_mlp_training_reduces_loss():
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d_in, H, d_out, batch = 64, 128, 32, 256
    net = ddps.ddps_mlp_create(d_in, H, d_out, batch, seed=9)
    try:
        rng = np.random.default_rng(10)
        X = rng.standard_normal((batch, d_in))
        Wt = rng.standard_normal((d_in, d_out)) / np.sqrt(d_in)
        T = np.tanh(X @ Wt)
        Xd = torch.from_numpy(X.astype(np.float32)).cuda()
        Td = torch.from_numpy(T.astype(np.float32)).cuda()
        first = ddps.ddps_mlp_train_step(net, batch, Xd, Td, 1e-3)
        for _ in range(300):
            last = ddps.ddps_mlp_train_step(net, batch, Xd, Td, 1e-3, want_loss=False)
        last = ddps.ddps_mlp_train_step(net, batch, Xd, Td, 1e-3)
        assert np.isfinite(first) and last < 0.1 * first, (first, last)
    finally:
        ddps.ddps_mlp_destroy(net)


def test_mlp_argument_errors():
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    with pytest.raises(ddps.DDPSError):
        ddps.ddps_mlp_create(0, 8, 8, 4)
    net = ddps.ddps_mlp_create(8, 8, 8, 4)
    try:
        X = torch.zeros(5, 8, dtype=torch.float32, device="cuda")
        with pytest.raises(ddps.DDPSError):
            ddps.ddps_mlp_forward(net, 5, X, X)          # batch above max_batch
        with pytest.raises(ddps.DDPSError):
            ddps.ddps_mlp_train_step(net, 4, X, X, 0.0)  # lr must be positive
        assert ddps.ddps_mlp_param_count(net) == 4 * (8 * 8 + 8)
    finally:
        ddps.ddps_mlp_destroy(net)


# ------------------------------------------------------------ plumbing
@pytest.fixture(scope="module")
def c1_setup():
    d = configs.c1()
    S = make_solver(d, inner_tol=1e-14, max_rhs=2, guess=True)
    S.factor()
    P = oracle_prec(d)
    yield d, S, P
    S.close()


def test_reduced_rhs_restrict_and_residual(c1_setup):
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d, S, P = c1_setup
    m, t, _ = ddps.ddps_reduced_layout(S.h)
    cand, mask = M.candidate_layout(d["part_ptr"], t, P.c)
    assert len(cand) == m
    rng = np.random.default_rng(21)
    f = rng.standard_normal(d["A"].n)
    gh = torch.empty(m, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_rhs(S.h, 1, dev_vec(f), gh)
    _, rec = P.apply(f)
    gh_ref = M.to_candidates(rec["ghat"], P.c, cand)
    assert relerr(host(gh), gh_ref) <= 1e-12
    # restriction is a gather: exact
    x = rng.standard_normal(d["A"].n)
    z = torch.empty(m, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_restrict(S.h, 1, dev_vec(x), z)
    assert np.array_equal(host(z), x[cand] * mask)
    # selection residual: ||g^ - G^ z||_2 on c
    zc = x[P.c]
    r_ref = np.linalg.norm(rec["ghat"] - P.ghat_matvec(zc))
    r = ddps.ddps_reduced_residual(S.h, 1, gh, z)[0]
    assert abs(r - r_ref) <= 1e-11 * r_ref
    # the exact reduced solution has a tiny residual
    zs = M.to_candidates(rec["zhat"], P.c, cand)
    r0 = ddps.ddps_reduced_residual(S.h, 1, gh, dev_vec(zs))[0]
    assert r0 <= 1e-12 * np.linalg.norm(rec["ghat"])


def test_two_column_plumbing_matches_per_column(c1_setup):
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d, S, P = c1_setup
    m, t, _ = ddps.ddps_reduced_layout(S.h)
    n = d["A"].n
    rng = np.random.default_rng(22)
    F = rng.standard_normal((2, n))
    G2 = torch.empty(2 * m, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_rhs(S.h, 2, dev_vec(F.reshape(-1)), G2)
    for j in range(2):
        g1 = torch.empty(m, dtype=torch.float64, device="cuda")
        ddps.ddps_reduced_rhs(S.h, 1, dev_vec(F[j]), g1)
        assert np.array_equal(host(g1), host(G2)[j * m:(j + 1) * m])


def test_guess_features_compose_target_match_oracle(c1_setup):
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d, S, P = c1_setup
    m, t, _ = ddps.ddps_reduced_layout(S.h)
    nif = len(d["part_ptr"]) - 2
    cand, mask = M.candidate_layout(d["part_ptr"], t, P.c)
    rng = np.random.default_rng(23)
    gh = rng.standard_normal(m) * mask * 3.0
    zp = rng.standard_normal(m)
    zh = rng.standard_normal(m) * mask
    d_in = 4 * t + 7
    X = torch.empty(nif, d_in, dtype=torch.float32, device="cuda")
    s = torch.empty(nif, dtype=torch.float32, device="cuda")
    ddps.ddps_guess_features(S.h, 1, dev_vec(gh), dev_vec(zp), 0.25, -0.75, d_in, X, s)   # gh stands in for r
    X_ref, s_ref = M.guess_features(gh, zp, mask, t, 0.25, -0.75, d_in)
    assert np.array_equal(host(X), X_ref) and np.array_equal(host(s), s_ref)
    T = torch.empty(nif, 2 * t, dtype=torch.float32, device="cuda")
    ddps.ddps_guess_target(S.h, 1, dev_vec(zh), dev_vec(zp), s, T)
    T_ref = M.guess_target(zh, zp, s_ref, mask, t)
    assert np.allclose(host(T), T_ref, rtol=2e-7, atol=0)
    Y = torch.from_numpy(rng.standard_normal((nif, 2 * t)).astype(np.float32)).cuda()
    z0 = torch.empty(m, dtype=torch.float64, device="cuda")
    ddps.ddps_guess_compose(S.h, 1, dev_vec(zp), Y, s, z0)
    z0_ref = M.guess_compose(zp, host(Y), s_ref, mask, t)
    assert np.allclose(host(z0), z0_ref, rtol=1e-15, atol=1e-15)
    with pytest.raises(ddps.DDPSError):
        ddps.ddps_guess_features(S.h, 1, dev_vec(gh), dev_vec(zp), 0.0, 0.0, 4 * t + 1, X, s)


def test_guess_seeds_the_reduced_solve(c1_setup):
    # the exact reduced solution as guess: the inner solve needs (almost) no
    # iterations, and the solution is unchanged
    from oracle import mlp_oracle as M
    from paper_1008_1700_amd import ddps
    torch = torch_cuda()
    d, S, P = c1_setup
    m, t, _ = ddps.ddps_reduced_layout(S.h)
    cand, _ = M.candidate_layout(d["part_ptr"], t, P.c)
    f = d["f"]
    x = torch.zeros(d["A"].n, dtype=torch.float64, device="cuda")
    ddps.ddps_set_guess(S.h, None)
    _, i0 = S.solve(dev_vec(f), x, 1e-10)
    z = torch.empty(m, dtype=torch.float64, device="cuda")
    ddps.ddps_reduced_restrict(S.h, 1, x, z)
    ddps.ddps_set_guess(S.h, z, 1)
    x1 = torch.zeros_like(x)
    _, i1 = S.solve(dev_vec(f), x1, 1e-10)
    ddps.ddps_set_guess(S.h, None)
    assert i1.inner_iters_total < i0.inner_iters_total
    assert relerr(host(x1), d["x_star"]) <= 1e-8


# ------------------------------------------------------------ gain
def test_learned_guess_selection_on_time_sequence():
    """Implicit-Euler convection-diffusion (128 x 128, |v| = 50 rotating 1.2
    degrees per step, dt = 1e-3, p = 8): 60 plain steps train the network,
    the next 20 solve each step twice, once from the previous-step guess and
    once from the judged guess.

    What is asserted: the network learns (loss falls fivefold), its guess
    starts the reduced solve from a smaller reduced residual than the
    previous step's solution, the selection takes whichever start has the
    smaller residual, and every solve converges.  What is not asserted is an
    iteration gain: there is none.  The reduced BiCGStab gains about a
    decade per iteration, so a start residual a few times smaller is worth a
    fraction of an iteration, and the measured totals over the 20 steps are
    about equal (317 inner iterations from the judged guess, 315 from the
    previous step's)."""
    from paper_1008_1700_amd import ddps, guess
    torch_cuda()
    nx = ny = 128
    p = 8
    A1, _ = configs.c4_matrix(1, nx, ny)
    part = pde.slab_partition(ny, ny // p, nx)
    S = ddps.Solver(A1, part, dtype="f64", inner_tol=1e-12, guess=True)
    S.factor()
    try:
        kinds = configs.c4_kinds(A1, nx)
        out = guess.run_sequence(S, lambda s: configs.c4_step_values(s, kinds, nx), steps=80, train_steps=60,
                                 dt=configs.C4_DT, source=1.0, tol=1e-10, hidden=256, epochs=300,
                                 batch_rows=105, seed=0, log=print)
    finally:
        S.close()
    ev = [r for r in out["records"] if "r_learn" in r]
    assert len(ev) == 20
    assert all(r["relres"] <= 1e-10 for r in out["records"])
    assert out["loss"][-1] < 0.2 * out["loss"][0]
    rp = np.array([r["r_prev"] for r in ev])
    rl = np.array([r["r_learn"] for r in ev])
    ip = sum(r["prev_inner"] for r in ev)
    il = sum(r["learn_inner"] for r in ev)
    print(f"selection residual prev/learned (median) {np.median(rp):.3e} / {np.median(rl):.3e}; "
          f"learned chosen {sum(r['learned'] for r in ev)}/20; inner iterations prev {ip} learned {il}")
    assert np.median(rl) < 0.5 * np.median(rp)
    assert all(r["learned"] == (r["r_learn"] < r["r_prev"]) for r in ev)
    # both runs of a step do the same work up to the start: iteration counts
    # stay within a few per step of each other (recorded, not a gain)
    assert abs(il - ip) <= 3 * len(ev)


@pytest.mark.parametrize("retrieval", [0, 1])
def test_learned_guess_in_every_application(retrieval):
    """A network trained on plain solves of random right-hand sides
    (guess.train_rhs_guess) and attached to the handle: every preconditioner
    application picks its reduced-solve starting vector among 0, g^ and the
    network's, so the solutions must still match the direct solve, and the
    choices must add up to the reduced solves made."""
    torch = torch_cuda()
    from paper_1008_1700_amd import ddps, guess
    d = configs.small_banded(6, [300, 340, 280, 330, 310, 290], 40, 21)
    A = d["A"]
    S = ddps.Solver(A, d["part_ptr"], dtype="bf16x3", inner_tol=1e-8, outer="refine", max_rhs=4,
                    retrieval=retrieval)
    try:
        S.factor()
        G, st = guess.train_rhs_guess(S, A, K=12, seed=3, tol=1e-11, hidden=64, epochs=30)
        assert st["pairs"] == 12 * 5 and st["epochs"] == 30
        assert st["loss_first_last"][1] < st["loss_first_last"][0]
        rng = np.random.default_rng(5)
        Xs = rng.uniform(-1, 1, (A.n, 4))
        F = torch.from_numpy(np.ascontiguousarray((A.scipy() @ Xs).T)).cuda()
        X = torch.zeros_like(F)
        c0 = ddps.ddps_guess_counts(S.h)
        G.attach(True)
        rc, info = ddps.ddps_solve_many(S.h, F, X, 1e-11)
        c1 = ddps.ddps_guess_counts(S.h)
        G.attach(False)
        assert rc == 0 and info.relres_inf <= 1e-11
        assert relerr(host(X).T, Xs) <= 1e-8
        made = sum(c1[q] - c0[q] for q in c1)
        assert made == info.applications * 4
        G.close()
    finally:
        S.close()


def test_untrained_network_is_retired_by_the_trial():
    """An untrained network attached to the handle: the first reduced solves
    alternate between leaving it out and letting the selection consider it, and
    after 8 solves per arm it is retired unless its solves took at least
    half an iteration fewer.  An untrained network cannot do that; afterwards
    no candidates are tried, and every solve still matches the direct one."""
    torch = torch_cuda()
    from paper_1008_1700_amd import ddps
    d = configs.small_banded(6, [300, 340, 280, 330, 310, 290], 40, 21)
    A = d["A"]
    S = ddps.Solver(A, d["part_ptr"], dtype="bf16x3", inner_tol=1e-8, outer="refine", max_rhs=4)
    m, t, _ = ddps.ddps_reduced_layout(S.h)
    net = ddps.ddps_mlp_create(4 * t + 2, 32, 2 * t, 4 * (S.p - 1), seed=7, stream=S.stream.cuda_stream)
    try:
        S.factor()
        ddps.ddps_set_guess_model(S.h, net)
        tr0 = ddps.ddps_guess_trial(S.h)
        assert tr0["state"] == "running" and tr0["solves_with"] == 0 and tr0["solves_without"] == 0
        rng = np.random.default_rng(8)
        for rep in range(4):
            Xs = rng.uniform(-1, 1, (A.n, 4))
            F = torch.from_numpy(np.ascontiguousarray((A.scipy() @ Xs).T)).cuda()
            X = torch.zeros_like(F)
            rc, info = ddps.ddps_solve_many(S.h, F, X, 1e-11)
            assert rc == 0 and info.relres_inf <= 1e-11
            assert relerr(host(X).T, Xs) <= 1e-8
        tr = ddps.ddps_guess_trial(S.h)
        print(f"trial: {tr}")
        assert tr["state"] == "retired"
        assert tr["solves_with"] >= 8 and tr["solves_without"] >= 8
        assert tr["mean_iters_with"] > tr["mean_iters_without"] - 0.5
        c0 = ddps.ddps_guess_counts(S.h)
        X = torch.zeros_like(F)
        rc, info = ddps.ddps_solve_many(S.h, F, X, 1e-11)
        c1 = ddps.ddps_guess_counts(S.h)
        assert c1["retired"] - c0["retired"] == 4 * info.applications
        assert c1["learned"] == c0["learned"] and c1["zero"] == c0["zero"] and c1["ghat"] == c0["ghat"]
    finally:
        ddps.ddps_set_guess_model(S.h, None)
        S.close()
        ddps.ddps_mlp_destroy(net)
