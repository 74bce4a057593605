"""Ragged batch of independent 1D Euler problems (one launch per
stage, graph-captured step) against the oracle run problem by problem."""
import numpy as np
import pytest
import torch

from concurrent.futures import ThreadPoolExecutor

from gpu_util import (StepRatio, check_step, end_bar, other_roundings, rel_err, say, to_dev,
                      to_host)

T_END2 = 0.2

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


def _shadow_batch_step(B, Ud, t, t_end, meta, probs, make_oracle, status, ratio=None):
    """One rk3_step of the batch from its current state, checked for the
    listed problems against the oracle's step from the same state (dt from
    the oracle's CFL bound on it, clipped at t_end); finished problems must
    stay bitwise unchanged.  With a StepRatio, the FMA build's step from the
    same state is taken too.  Returns the number of live problems checked."""
    Ub = to_host(Ud).copy()
    tb = t.cpu().numpy().copy()
    B.rk3_step(Ud, t, t_end, 0.5, status)
    Ua = to_host(Ud)
    ta = t.cpu().numpy()
    live = 0
    for p in probs:
        if tb[p] >= t_end:
            assert np.array_equal(_cols(Ua, meta, p), _cols(Ub, meta, p)) and ta[p] == tb[p]
            continue
        O = make_oracle(p)
        Up = _cols(Ub, meta, p)
        dt = O.cfl_dt(Up, 0.5)
        if not dt < t_end - tb[p]:
            dt = t_end - tb[p]
        assert ta[p] == pytest.approx(tb[p] + dt, rel=1e-14, abs=1e-15), (p, ta[p], tb[p], dt)
        U1, bad = O.rk3_step(Up, dt)
        assert bad == 0
        e = check_step(_cols(Ua, meta, p), U1, what=f"problem {p} at t = {tb[p]:.6g}")
        if ratio is not None:
            Uf, _ = make_oracle(p, "fma").rk3_step(Up, dt)
            ratio.add(e[0], rel_err(Uf, U1)[0])
        live += 1
    return live


def _exact_density_l1(meta, p, U, t_end):
    """Mean |rho - rho_exact| of problem p's state at t_end (exact Riemann
    solution of its two initial states, jump at x = 0.5)."""
    from oracle import exact_riemann as er
    N = int(meta["lengths"][p])
    x = np.arange(N) * meta["h"][p]
    (rl, ul, pl), (rr, ur, pr) = meta["states"][p]
    rho_ex, _, _ = er.sample(x, t_end, 0.5, rl, ul, pl, rr, ur, pr)
    return float(np.mean(np.abs(U[0] - rho_ex)))


def _end_check_dt_sequence(ora, meta, p, Ug, U0, dts, t_end, kw, ratio=1.0):
    """End state of problem p after a CFL-driven run against the oracle run
    through the same step sizes (the GPU's dt of every step, each pinned to
    the oracle's CFL bound at the shadowed steps): 1e-9, else 2 max(1,
    ratio) times the spread of other valid roundings of that run (the FMA
    build, and both builds from the one-ulp-perturbed initial state, the
    same step sizes); where that bar exceeds the cap, the end state is
    unpinned element by element and the GPU's and the oracle's L1 density
    distances from the exact Riemann solution must agree to 2 max(1, ratio)
    times the largest L1 deviation of those roundings.  Returns (error,
    spread or None).

    The free-running oracle is not the reference here: its step size is a
    maximum over the state, taken where the state is most sensitive to
    rounding (at a shock), and feeds every node; over thousands of steps two
    valid roundings then choose measurably different step sequences (on one
    tube, 7.8e-5 apart at the end with the GPU's rounding against the
    oracle's, while the oracle driven by the GPU's steps lands 2.9e-6 from
    the GPU, inside the 3.6e-6 of the FMA build)."""
    O = _oracle(ora, meta, p, **kw)
    Of = _oracle(ora, meta, p, variant="fma", **kw)
    Uo, bad = O.run_dt_sequence(U0, dts)
    assert bad == 0
    assert abs(float(np.sum(dts)) - t_end) <= 1e-12 * t_end
    n, pt = rel_err(Ug, Uo)
    if n <= 1e-9 and pt <= 1e-9:
        return n, None
    alts = other_roundings(Uo, lambda X: O.run_dt_sequence(X, dts)[0],
                           lambda X: Of.run_dt_sequence(X, dts)[0], U0, Ug, ratio)
    tol, ptol, spread, informative = end_bar(Uo, alts, ratio)
    if informative:
        assert n <= tol and pt <= ptol, (p, n, pt, spread, ratio)
    else:
        # the end state is unpinned element by element; the GPU's and the
        # oracle's L1 density distances from the exact solution must agree
        # as closely as the other roundings' do
        lg = _exact_density_l1(meta, p, Ug, t_end)
        lo = _exact_density_l1(meta, p, Uo, t_end)
        dev = max(float(np.mean(np.abs(A[0] - Uo[0]))) for A in alts)
        assert abs(lg - lo) <= 2 * max(1.0, ratio) * dev, (p, lg, lo, dev, spread, ratio)
    return n, spread


def _end_check_problem(ora, meta, p, Ug, U0, t_end, kw, ratio=1.0):
    """End state of problem p after a run to t_end against the oracle's run:
    1e-9, else 2 max(1, ratio) times the spread of other valid roundings of
    the run (gpu_util.other_roundings); where that bar exceeds the cap, the
    GPU's and the oracle's L1 density distances from the exact Riemann
    solution must agree to 2 max(1, ratio) times the largest L1 deviation of
    those roundings' density from the oracle's.  Returns (error, spread or
    None)."""
    O = _oracle(ora, meta, p, **kw)
    Of = _oracle(ora, meta, p, variant="fma", **kw)
    Uo, s, tt, bad = O.run_to_time(U0, t_end, cfl=0.5)
    assert bad == 0 and tt == t_end
    n, pt = rel_err(Ug, Uo)
    if n <= 1e-9 and pt <= 1e-9:
        return n, None
    alts = other_roundings(Uo, lambda X: O.run_to_time(X, t_end, cfl=0.5)[0],
                           lambda X: Of.run_to_time(X, t_end, cfl=0.5)[0], U0, Ug, ratio)
    tol, ptol, spread, informative = end_bar(Uo, alts, ratio)
    if informative:
        assert n <= tol and pt <= ptol, (p, n, pt, spread, ratio)
    else:
        lg = _exact_density_l1(meta, p, Ug, t_end)
        lo = _exact_density_l1(meta, p, Uo, t_end)
        dev = max(float(np.mean(np.abs(A[0] - Uo[0]))) for A in alts)
        assert abs(lg - lo) <= 2 * max(1.0, ratio) * dev, (p, lg, lo, dev, spread, ratio)
    return n, spread


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
    # the same run stepped singly, every step shadowed (single steps give
    # bitwise the fused call's states and times): the end states agree
    B1 = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    U1 = to_dev(U)
    t1 = torch.zeros(B1.nprob, dtype=torch.float64, device="cuda")
    while bool((t1 < t_end).any().item()):
        B1.rk3_step(U1, t1, t_end, 0.5)
    assert torch.equal(t1, t) and torch.equal(U1, Ud)


def test_batch_run_shadowed_every_step(lib, ora, W):
    """The same kind of batch to t = 0.05, every step shadowed for every
    problem by the oracle's step from the GPU's state."""
    prob, U, meta = _small_batch(W, seed=1, nprob=10, nmin=64, nmax=300)
    t_end = 0.05
    say("batch run, every step shadowed")
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    make = lambda p, v="plain": _oracle(ora, meta, p, weights="fe", xi=100.0, variant=v)  # noqa: E731
    ratio = StepRatio()
    steps = 0
    while bool((t < t_end).any().item()):
        _shadow_batch_step(B, Ud, t, t_end, meta, range(B.nprob), make, status, ratio)
        steps += 1
    assert int(status.item()) == 0
    say("  steps", steps, "step ratio", ratio.value)
    Ug = to_host(Ud)
    for p in range(B.nprob):
        n, spread = _end_check_problem(ora, meta, p, _cols(Ug, meta, p), _cols(U, meta, p), t_end,
                                       dict(weights="fe", xi=100.0), ratio.value)
        say("  problem", p, "end state", n, "spread", spread)


def _config2_subset(W, cap=4e7):
    """A stratified subset of the 4096-tube batch (seed 0): eight length bins
    over [256, 4096], eight tubes from each, spread evenly over the bin's
    tubes ordered by estimated work (3 N steps, steps from the initial wave
    speeds), among tubes of estimated work <= cap (82 % of the batch; the
    heaviest tubes are checked by the shadowed full-batch run)."""
    prob, U, meta = W.shock_tube_batch(seed=0)
    L, h, S = meta["lengths"], meta["h"], meta["states"]
    rate = np.max(np.abs(S[:, :, 1]) + np.sqrt(1.4 * S[:, :, 2] / S[:, :, 0]), axis=1) / h
    work = 3 * L * np.ceil(T_END2 * rate / 0.5)
    bins = np.linspace(256, 4097, 9)
    idx = []
    for b in range(8):
        m = np.where((L >= bins[b]) & (L < bins[b + 1]) & (work <= cap))[0]
        o = m[np.argsort(work[m], kind="stable")]
        idx += [int(o[int((k + 0.5) * len(o) / 8)]) for k in range(8)]
    return U, meta, np.array(idx)


@pytest.mark.timeout(400)
@pytest.mark.parametrize("half", [0, 1])
def test_config2_subset_run_to_end(lib, ora, W, half):
    """32 of the 64 stratified tubes (four length bins each) as one batch of
    their own to t = 0.2, stepped singly: a step shadowed about every 500
    steps (state and dt against the oracle's from the same state), and every
    tube's end state against the oracle run through the GPU's own step
    sizes (_end_check_dt_sequence)."""
    U_all, meta_all, idx = _config2_subset(W)
    idx = idx[32 * half:32 * (half + 1)]
    L = meta_all["lengths"][idx]
    offsets = np.zeros(len(idx) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(L)
    U = np.concatenate([_cols(U_all, meta_all, p) for p in idx], axis=1)
    meta = dict(lengths=L, offsets=offsets, h=meta_all["h"][idx], states=meta_all["states"][idx])
    say("config2 subset to t = 0.2, half", half, "tubes", idx.tolist())
    B = lib.BatchPlan(offsets, meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    make = lambda p, v="plain": _oracle(ora, meta, p, weights="fe", xi=100.0, variant=v)  # noqa: E731
    ratio = StepRatio()
    dts = torch.zeros((20000, B.nprob), dtype=torch.float64, device="cuda")
    steps = checked = 0
    while bool((t < T_END2).any().item()):
        assert steps < dts.shape[0]
        if steps % 500 == 0:
            checked += _shadow_batch_step(B, Ud, t, T_END2, meta, range(B.nprob), make, status, ratio)
        else:
            for _ in range(min(99, dts.shape[0] - 1 - steps)):
                B.rk3_step(Ud, t, T_END2, 0.5, status)
                B.last_dt(out=dts[steps])
                steps += 1
                if steps % 500 == 0:
                    break
            continue
        B.last_dt(out=dts[steps])
        steps += 1
    assert int(status.item()) == 0 and bool((t == T_END2).all().item())
    say("  steps", steps, "shadowed problem-steps", checked, "step ratio", ratio.value)
    Ug = to_host(Ud)
    D = dts[:steps].cpu().numpy()
    kw = dict(weights="fe", xi=100.0)
    with ThreadPoolExecutor(16) as ex:
        res = list(ex.map(lambda p: _end_check_dt_sequence(ora, meta, p, _cols(Ug, meta, p),
                                                           _cols(U, meta, p), D[:, p], T_END2, kw,
                                                           ratio.value),
                          range(B.nprob)))
    for p, (n, spread) in enumerate(res):
        say("  tube", int(idx[p]), "N", int(L[p]), "end state", "%.2e" % n, "spread", spread)


@pytest.mark.timeout(300)
def test_config2_full_batch_run_to_end_shadowed(lib, ora, W):
    """The full 4096-tube batch to t = 0.2 (the benchmark run, about 20 000
    steps for the slowest tube): at every 1000th step one single step is
    shadowed for the 12 live tubes with the most work left plus 12 random
    live tubes; at the end every tube is at t = 0.2 with a clean status."""
    prob, U, meta = W.shock_tube_batch(seed=0)
    say("config2 full batch to t = 0.2, shadowed")
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    B.autotune(Ud)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    make = lambda p, v="plain": _oracle(ora, meta, p, weights="fe", xi=100.0, variant=v)  # noqa: E731
    rng = np.random.default_rng(9)
    L = meta["lengths"]
    steps = checked = 0
    while bool((t < T_END2).any().item()):
        tt = t.cpu().numpy()
        live = np.where(tt < T_END2)[0]
        # most work left ~ N_p (t_end - t_p) / dt_p: rank by N_p (T - t_p)
        rank = live[np.argsort(-(L[live] * (T_END2 - tt[live])), kind="stable")]
        pick = sorted(set(rank[:12].tolist()) | set(rng.choice(live, min(12, len(live)), replace=False).tolist()))
        checked += _shadow_batch_step(B, Ud, t, T_END2, meta, pick, make, status)
        B.rk3_steps(Ud, t, T_END2, 0.5, 999, status)
        steps += 1000
        say("  step", steps, "live", len(live), "checked", checked)
    assert int(status.item()) == 0 and bool((t == T_END2).all().item())


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


@pytest.mark.parametrize("tile", [128, 256])
def test_capped_steps_equal_uncapped(lib, W, tile):
    """rk3_steps with the stage launches sized to the live-tile count read
    after the previous call (problems finish between the calls) gives
    bitwise the states and times of the uncapped calls; a bound below the
    live count is reported in bit 1 of the status word."""
    prob, U, meta = _small_batch(W, seed=8, nprob=48, nmin=60, nmax=900)
    say("capped rk3_steps", tile)
    t_end = 0.02  # the shortest tubes finish within the first calls, the longest later
    res, counts = [], []
    for capped in (False, True):
        B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
        B.tile = tile
        Ud = to_dev(U)
        t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
        status = torch.zeros(1, dtype=torch.int32, device="cuda")
        out, live = [], None
        for chunk in (4, 8, 16, 40, 60):
            B.rk3_steps(Ud, t, t_end, 0.5, chunk, status, max_live=live if capped else None)
            out.append((to_host(Ud).copy(), t.cpu().numpy().copy()))
            if capped:
                live = max(1, B.live_tiles())
                counts.append(live)
        assert int(status.item()) == 0
        res.append(out)
    assert counts[0] > counts[-1] >= 1  # problems finished between the calls
    assert (res[0][-1][1] >= t_end).any()
    for (ua, ta), (ub, tb) in zip(*res):
        assert np.array_equal(ta, tb)
        assert np.array_equal(ua, ub)
    # a bound below the list's length: flagged
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    B.tile = tile
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.rk3_steps(Ud, t, t_end, 0.5, 1, status)
    n = B.live_tiles()
    assert n > 1
    B.rk3_steps(Ud, t, t_end, 0.5, 2, status, max_live=n - 1)
    assert int(status.item()) & 2


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


def test_nonphysical_problem_is_stopped_and_reported(lib, ora, W):
    """A problem whose state is non-physical from the start (negative
    pressure: its wave rate is NaN) gets dt = 0 and keeps its time and state;
    the status word says so; its neighbours in the packed tiles advance as
    the oracle does; run_to_time raises."""
    prob, U, meta = _small_batch(W, seed=3, nprob=6, nmin=50, nmax=80)
    o = meta["offsets"]
    U = U.copy()
    U[2, o[3] + 10] = -1.0  # E < 0 at one node of problem 3
    say("non-physical problem in a batch")
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.rk3_step(Ud, t, 0.1, 0.5, status)
    Ug = to_host(Ud)
    assert int(status.item()) & 1
    assert float(t[3].item()) == 0.0
    assert np.array_equal(_cols(Ug, meta, 3), _cols(U, meta, 3))
    for p in (0, 1, 2, 4, 5):
        O = _oracle(ora, meta, p, weights="fe", xi=100.0)
        dt = min(O.cfl_dt(_cols(U, meta, p), 0.5), 0.1)
        assert float(t[p].item()) == pytest.approx(dt, rel=1e-14)
        U1, bad = O.rk3_step(_cols(U, meta, p), dt)
        n, pt = rel_err(_cols(Ug, meta, p), U1)
        assert n <= 1e-12 and pt <= 1e-12, (p, n, pt)
    # the fused multi-step call keeps it stopped
    B.rk3_steps(Ud, t, 0.1, 0.5, 3, status)
    assert float(t[3].item()) == 0.0
    with pytest.raises(lib._lib.WCNSError, match="non-physical"):
        B.run_to_time(to_dev(U), 0.1, cfl=0.5, check_every=4)


@pytest.mark.parametrize("first,second", [(128, 256), (256, 128)])
def test_stage_after_tile_change_uses_every_tile(lib, ora, W, first, second):
    """wcns_batch_stage takes the live list the last wcns_batch_cfl built;
    after a change of tile size that list belongs to another tiling, and the
    stage must fall back to every tile (same result as a fresh cfl)."""
    prob, U, meta = _small_batch(W, seed=5, nprob=20, nmin=60, nmax=900)
    say("stage after tile change", first, second)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    B.tile = first
    Ud = to_dev(U)
    t = torch.zeros(B.nprob, dtype=torch.float64, device="cuda")
    B.cfl(Ud, t, 0.2, 0.5)
    B.tile = second
    out = torch.empty_like(Ud)
    B.stage(1, Ud, Ud, out)
    Ug = to_host(out)
    tt = t.cpu().numpy()
    for p in range(B.nprob):
        O = _oracle(ora, meta, p, weights="fe", xi=100.0)
        Up = _cols(U, meta, p)
        ref = Up + tt[p] * O.residual(Up)
        n, pt = rel_err(_cols(Ug, meta, p), ref)
        assert n <= 1e-12 and pt <= 1e-12, (p, n, pt)


def test_auxiliary_tensors_are_checked(lib, W):
    """t, status and dt reach the kernels as raw addresses: wrong device,
    dtype or size is refused before any launch."""
    prob, U, meta = _small_batch(W, seed=0, nprob=4, nmin=20, nmax=40)
    B = lib.BatchPlan(meta["offsets"], meta["h"], weights="fe", xi=100.0)
    Ud = to_dev(U)
    err = lib._lib.WCNSError
    good_t = torch.zeros(4, dtype=torch.float64, device="cuda")
    for bad in (torch.zeros(4, dtype=torch.float64), torch.zeros(4, dtype=torch.float32, device="cuda"),
                torch.zeros(3, dtype=torch.float64, device="cuda")):
        with pytest.raises(err):
            B.rk3_step(Ud, bad, 0.1)
        with pytest.raises(err):
            B.rk3_steps(Ud, bad, 0.1, 0.5, 2)
    with pytest.raises(err):
        B.rk3_step(Ud, good_t, 0.1, status=torch.zeros(1, dtype=torch.int64, device="cuda"))
    prob1, U1, _ = W.shock_tube(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 64)
    P = lib.Plan(**prob1, weights="fe")
    U1d = to_dev(U1)
    with pytest.raises(err):
        P.rk3_step(U1d, dt=torch.full((1,), 1e-4, dtype=torch.float64))  # host dt
    with pytest.raises(err):
        P.rk3_step(U1d, dt=torch.full((1,), 1e-4, dtype=torch.float32, device="cuda"))
    with pytest.raises(err):
        P.residual(U1d, out=torch.empty(3, 10, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
