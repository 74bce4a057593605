"""Ragged batch of independent 1D Euler problems (one launch per
stage, graph-captured step) against the oracle run problem by problem."""
import numpy as np
import pytest
import torch

from gpu_util import rel_err, run_tolerance, say, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_2306_09760_amd import solver
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return solver


def _small_batch(W, seed=0, nprob=12, nmin=9, nmax=700):
    return W.shock_tube_batch(seed=seed, nprob=nprob, nmin=nmin, nmax=nmax)


def _oracle(ora, meta, p, bc="transmissive", **kw):
    N = int(meta["lengths"][p])
    return ora.Problem(system="euler", ndim=1, n=(N,), h=(meta["h"][p],), bc=bc, **kw)


def _cols(U, meta, p):
    o = meta["offsets"]
    return U[:, o[p]:o[p + 1]]


@pytest.mark.parametrize("weights,xi", [("fe", 100.0), ("fe", 1e6), ("z", 100.0), ("js", 100.0)])
@pytest.mark.parametrize("tile", [128, 256])
def test_batch_residual(lib, ora, W, weights, xi, tile):
    prob, U, meta = _small_batch(W)
    say("batch residual", weights, xi, tile)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights=weights, xi=xi)
    B.tile = tile
    R = to_host(B.residual(to_dev(U)))
    for p in range(len(meta["lengths"])):
        ref = _oracle(ora, meta, p, weights=weights, xi=xi).residual(_cols(U, meta, p))
        n, pt = rel_err(_cols(R, meta, p), ref)
        assert n <= 1e-12 and pt <= 1e-10, (p, n, pt)


@pytest.mark.parametrize("diff", ["mnd6", "md6"])
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
@pytest.mark.parametrize("tile", [128, 256])
def test_batch_residual_short_problems(lib, ora, W, diff, bc, tile):
    """Problems of 9 to 40 nodes: tiles are packed across problem ends, so
    every tile holds the nodes and ghost slots of several problems."""
    prob, U, meta = _small_batch(W, seed=4, nprob=64, nmin=9, nmax=40)
    say("batch residual, short problems", diff, bc, tile)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0, diff=diff, bc=bc)
    B.tile = tile
    R = to_host(B.residual(to_dev(U)))
    for p in range(len(meta["lengths"])):
        ref = _oracle(ora, meta, p, bc=bc, weights="fe", xi=100.0, diff=diff).residual(_cols(U, meta, p))
        n, pt = rel_err(_cols(R, meta, p), ref)
        assert n <= 1e-12 and pt <= 1e-10, (p, n, pt)


@pytest.mark.parametrize("n", [9, 5000])
def test_batch_single_problem(lib, ora, W, n):
    """A batch of one problem: of the minimum length (one tile of mostly
    ghost slots) and of 5000 nodes (many tiles, one problem each)."""
    prob, U, meta = W.shock_tube_batch(seed=7, nprob=1, nmin=n, nmax=n)
    say("batch of one problem", n)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    R = to_host(B.residual(Ud))
    O = _oracle(ora, meta, 0, weights="fe", xi=100.0)
    n_, pt = rel_err(_cols(R, meta, 0), O.residual(_cols(U, meta, 0)))
    assert n_ <= 1e-12 and pt <= 1e-10, (n_, pt)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.rk3_steps(Ud, t, 1.0, 0.5, 2)
    Uo = _cols(U, meta, 0)
    for _ in range(2):
        dt = O.cfl_dt(Uo, 0.5)
        Uo, bad = O.rk3_step(Uo, dt)
    n_, pt = rel_err(_cols(to_host(Ud), meta, 0), Uo)
    assert n_ <= 1e-12 and pt <= 1e-12, (n_, pt)


@pytest.mark.parametrize("graph,fused", [(False, False), (True, False), (False, True)])
def test_batch_steps_to_time_match_per_problem_runs(lib, ora, W, graph, fused):
    prob, U, meta = _small_batch(W, seed=1, nprob=10, nmin=64, nmax=300)
    t_end = 0.05
    say("batch run to time, graph =", graph, "fused =", fused)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    B.set_graph(graph)
    Ud = to_dev(U)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t, steps = B.run_to_time(Ud, t_end, cfl=0.5, check_every=16, status=status, fused=fused)
    assert bool((t == t_end).all().item())
    assert int(status.item()) == 0
    Ug = to_host(Ud)
    for p in range(len(meta["lengths"])):
        O = _oracle(ora, meta, p, weights="fe", xi=100.0)
        Uo, s, tt, bad = O.run_to_time(_cols(U, meta, p), t_end, cfl=0.5)
        assert bad == 0 and tt == t_end
        Of = _oracle(ora, meta, p, weights="fe", xi=100.0, variant="fma")
        Uf, *_ = Of.run_to_time(_cols(U, meta, p), t_end, cfl=0.5)
        tol, ptol, spread = run_tolerance(Uo, Uf)
        n, pt = rel_err(_cols(Ug, meta, p), Uo)
        assert n <= tol and pt <= ptol, (p, n, pt, spread)


def test_graph_replay_equals_eager_steps(lib, W):
    prob, U, meta = _small_batch(W, seed=2, nprob=40, nmin=100, nmax=2000)
    say("graph vs eager")
    res = []
    for graph in (False, True):
        B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
        B.set_graph(graph)
        Ud = to_dev(U)
        t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
        out = []
        for k in range(6):
            B.rk3_step(Ud, t, 0.2, 0.5)
            torch.cuda.synchronize()
            out.append(to_host(Ud).copy())  # eager work between replays
        res.append(out)
    for a, b in zip(*res):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("nmin,nmax,tile", [(9, 40, 128), (9, 40, 256), (200, 2000, 256), (200, 2000, 128)])
def test_rk3_steps_equal_single_steps(lib, W, nmin, nmax, tile):
    """rk3_steps (the CFL maximum of each step taken by the previous step's
    last stage) gives bitwise the states and times of single rk3_step calls,
    also while problems finish and with many problems per tile."""
    prob, U, meta = _small_batch(W, seed=6, nprob=48, nmin=nmin, nmax=nmax)
    say("rk3_steps vs rk3_step", nmin, nmax, tile)
    t_end = 100.0  # even problems stay far from it over 20 steps
    # odd problems start just before t_end (they finish in their first step),
    # the last one at t_end (finished from the start), the rest at 0
    t0 = np.zeros(48)
    t0[1::2] = t_end * (1.0 - 1e-6)
    t0[-1] = t_end
    res = []
    for fused in (False, True):
        B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
        B.tile = tile
        Ud = to_dev(U)
        t = torch.from_numpy(t0.copy()).cuda()
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        out = []
        for chunk in (1, 5, 14):
            if fused:
                B.rk3_steps(Ud, t, t_end, 0.5, chunk, status)
            else:
                for _ in range(chunk):
                    B.rk3_step(Ud, t, t_end, 0.5, status)
            out.append((to_host(Ud).copy(), t.cpu().numpy().copy()))
        assert int(status.item()) == 0
        res.append(out)
    finished = res[0][-1][1] >= t_end
    assert finished[1::2].all() and not finished[0:-1:2].any()
    for (ua, ta), (ub, tb) in zip(*res):
        assert np.array_equal(ta, tb)
        assert np.array_equal(ua, ub)


def test_finished_problems_are_untouched(lib, ora, W):
    """A finished problem shares its tiles with live neighbours (tiles are
    packed across problem ends): it stays bitwise unchanged, they advance one
    step as the oracle does."""
    prob, U, meta = _small_batch(W, seed=3, nprob=6, nmin=50, nmax=80)
    say("finished problems")
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    t[2] = 1.0  # already past t_end
    B.rk3_step(Ud, t, 0.1, 0.5)
    Ug = to_host(Ud)
    assert np.array_equal(_cols(Ug, meta, 2), _cols(U, meta, 2))
    for p in (0, 1, 3, 4, 5):
        O = _oracle(ora, meta, p, weights="fe", xi=100.0)
        dt = min(O.cfl_dt(_cols(U, meta, p), 0.5), 0.1)
        U1, bad = O.rk3_step(_cols(U, meta, p), dt)
        n, pt = rel_err(_cols(Ug, meta, p), U1)
        assert n <= 1e-12 and pt <= 1e-12, (p, n, pt)


def test_full_config2_batch_sampled(lib, ora, W):
    """The 4096-problem batch at full size: residual and one step on 48
    sampled problems (longest, shortest and random) vs the oracle."""
    prob, U, meta = W.shock_tube_batch(seed=0)
    L = meta["lengths"]
    rng = np.random.default_rng(5)
    sample = sorted(set([int(np.argmax(L)), int(np.argmin(L))] + list(rng.choice(len(L), 46, replace=False))))
    say("config2 full batch sampled", len(sample))
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    B.autotune(Ud)
    R = to_host(B.residual(Ud))
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    B.rk3_step(Ud, t, 0.2, 0.5)
    Ug = to_host(Ud)
    for p in sample:
        O = _oracle(ora, meta, p, weights="fe", xi=100.0)
        n, pt = rel_err(_cols(R, meta, p), O.residual(_cols(U, meta, p)))
        assert n <= 1e-12 and pt <= 1e-10, ("residual", p, n, pt)
        dt = O.cfl_dt(_cols(U, meta, p), 0.5)
        U1, bad = O.rk3_step(_cols(U, meta, p), dt)
        n, pt = rel_err(_cols(Ug, meta, p), U1)
        assert n <= 1e-12 and pt <= 1e-12, ("step", p, n, pt)


def test_full_config2_batch_rk3_steps_equal_single_steps(lib, W):
    """The benchmark's call at full size (4096 problems, autotuned tile):
    rk3_steps gives bitwise the states and times of single rk3_step calls;
    single steps are checked against the oracle above."""
    prob, U, meta = W.shock_tube_batch(seed=0)
    say("config2 full batch, rk3_steps vs rk3_step")
    res = []
    for fused in (False, True):
        B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
        Ud = to_dev(U)
        B.autotune(Ud)
        t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        if fused:
            B.rk3_steps(Ud, t, 0.2, 0.5, 4, status)
        else:
            for _ in range(4):
                B.rk3_step(Ud, t, 0.2, 0.5, status)
        assert int(status.item()) == 0
        res.append((to_host(Ud), t.cpu().numpy()))
    assert np.array_equal(res[0][1], res[1][1])
    assert np.array_equal(res[0][0], res[1][0])
