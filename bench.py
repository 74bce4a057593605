#!/usr/bin/env python
"""Throughput of the WCNS-FE residual + SSP-RK3 step on one MI355X.

Workload: a batch of 4096 independent 1D Euler shock tubes (gamma = 1.4),
N_p uniform in [256, 4096] (seed 0: 8.97 M points in total), left/right
(rho, u, p) drawn from the seed, transmissive ends, FE weights (xi = 100,
kappa = 0.5, p = 2, eps = 1e-40), characteristic projection, MND6, SSP-RK3
at CFL 0.5 with a per-problem dt.  One "step" is one SSP-RK3 step of every
problem: the per-problem dt from the CFL bound of the step's state, then the
three stage kernels.  The K timed steps are one wcns_batch_rk3_steps call,
in which the last stage of each step also takes the per-problem maximum
wave rate of the state it writes (the next step's dt), so only the first
step reads the state for its CFL bound; --single-steps times K
graph-replayed wcns_batch_rk3_step calls instead (a CFL pass over the state
in every step).  States are resident in HBM before timing starts.

Prints one JSON line with the metric (grid-point RK3-stage updates per
second), the roofline of the dominant kernel (the batch stage kernel) and
the CPU oracle timed on a bounded sample of the same workload.  The line
also carries the whole run of the batch to t = 0.2 (time to solution and the
mean rate over it, every problem to its own end) next to the K-step rate.
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

PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector (published)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E (published)
T_END = 0.2


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--weights", default="fe")
    ap.add_argument("--xi", type=float, default=100.0)
    ap.add_argument("--no-graph", action="store_true",
                    help="with --single-steps: launch each step eagerly")
    ap.add_argument("--single-steps", action="store_true",
                    help="time K wcns_batch_rk3_step calls (CFL pass per step) instead of one "
                         "wcns_batch_rk3_steps call")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the xi = 1e6 and plain-form (1D per problem, 2D, 3D) timings")
    ap.add_argument("--tile", type=int, choices=[128, 256], default=None,
                    help="midpoints per batch tile instead of the autotuner's choice "
                         "(keeps profiled runs, where timings shift, on one kernel)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--no-whole-run", action="store_true",
                    help="skip the run of the batch to t = 0.2")
    ap.add_argument("--sweeps-2d", action="store_true",
                    help="only time the 2D 1024^2 residual (x and y sweeps, fixed tiles) and "
                         "its adjoint, a few launches each (for profiler counter runs)")
    ap.add_argument("--sweep-kernels", action="store_true",
                    help="only run the grid kernels a few launches each, fixed tiles (for "
                         "profiler counter runs): the 2D 2048^2 Riemann residual (x, y sweeps), "
                         "the 3D 256^3 turbulence residual (x, y, z sweeps) and the 2D 1024^2 "
                         "residual adjoint (x, y)")
    return ap.parse_args()


def sweeps_2d(seed):
    """The 2D periodic 1024^2 residual with x tile 256 and y tile (64, 4) and
    its adjoint: one warm-up launch each, then 3 + 2 launches timed with HIP
    events."""
    import torch
    from paper_2306_09760_amd import workloads as W
    from paper_2306_09760_amd.solver import Plan
    dev = torch.device("cuda")
    prob, U_host, _ = W.adjoint2d(seed=seed, n=1024, flow_amp=0.05)
    P = Plan(**prob, weights="fe", xi=100.0)
    U = torch.from_numpy(U_host).to(dev)
    P.tiles = (256, 64, 4)
    R, Rb, Ub = torch.empty_like(U), torch.ones_like(U), torch.zeros_like(U)

    def timed(fn, n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    timed(lambda: P.residual(U, R), 1)  # warm-up
    timed(lambda: P.residual_adjoint(U, Rb, Ub), 1)
    res_ms = timed(lambda: P.residual(U, R), 3)
    adj_ms = timed(lambda: P.residual_adjoint(U, Rb, Ub), 2)
    print(json.dumps({"workload": "2D Euler periodic 1024^2, FE xi=100, tiles (256, 64, 4)",
                      "residual_ms": round(res_ms, 4), "residual_adjoint_ms": round(adj_ms, 4),
                      "state_bytes": int(U.numel() * 8)}), flush=True)


def sweep_kernels(seed):
    """Each grid kernel of the configurations at full size, one warm-up call
    and three timed calls of the residual (or residual adjoint), with the
    autotuner's tiles fixed: 2D 2048^2 (256; 128, 2), 3D 256^3 (256; 32, 8),
    2D 1024^2 adjoint.  Prints one JSON line of HIP-event times per call."""
    import torch
    from paper_2306_09760_amd import workloads as W
    from paper_2306_09760_amd.solver import Plan
    dev = torch.device("cuda")

    def timed(fn, n):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {}
    for name, (prob, U_host, _), tiles in (
            ("2d_riemann_2048", W.riemann2d(seed=seed, n=2048), (256, 128, 2)),
            ("3d_turbulence_256", W.turbulence3d(seed=seed, n=256), (256, 32, 8))):
        P = Plan(**prob, weights="fe", xi=100.0)
        P.tiles = tiles
        U = torch.from_numpy(U_host).to(dev)
        R = torch.empty_like(U)
        out[name] = {"residual_ms": round(timed(lambda: P.residual(U, R), 3), 4),
                     "tiles": list(tiles), "points": int(U.numel() // U.shape[0])}
        del P, U, R
    prob, U_host, _ = W.adjoint2d(seed=seed, n=1024, flow_amp=0.05)
    P = Plan(**prob, weights="fe", xi=100.0)
    P.tiles = (256, 128, 2)
    U = torch.from_numpy(U_host).to(dev)
    Rb, Ub = torch.ones_like(U), torch.zeros_like(U)
    out["2d_adjoint_1024"] = {"residual_adjoint_ms": round(timed(lambda: P.residual_adjoint(U, Rb, Ub), 3), 4),
                              "points": 1024 * 1024}
    del P, U, Rb, Ub
    # a plain 1 GiB device copy: the HBM counters' calibration
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


def source_digest():
    """Digest of the HIP sources: counters taken on other sources are stale."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2306_09760_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel):
    """Counter figures of ``kernel`` from the committed summary (rocprofv3
    FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy of known size, and
    the SQ instruction counters), or None if they were taken on other
    sources."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_counters.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != source_digest() or rec.get("kernel") != kernel:
        return None
    return rec


# Algorithmic work per grid-point RK3 stage of the 1D Euler batch with FE
# weights, as the scope table of the method counts it (nv = 3, one direction):
# 1040 floating-point operations besides 37 divisions, 5 square roots and 60
# tanh.  The roofline's `achieved` is priced on the 1040.
CONTRACT_FLOPS_PER_POINT_STAGE = 1040.0
CONTRACT_SPECIAL_PER_POINT_STAGE = 37 + 5 + 60

# The oracle's operation tally of one residual per node, by weight choice
# (each +, -, x, /, sqrt and tanh counts once; characteristic projection,
# MND6, LLF) on a 512-node shock tube, plus the stage combine (5 per
# variable): it counts what the oracle computes, recomputations included.
# A CPU test recomputes each entry with the oracle.
FLOPS_PER_POINT_STAGE = {
    "fe": 1286.208984375,
    "js": 706.833984375,
    "z": 767.185546875,
    "pfe": 771.216796875,
    "linear": 616.306640625,
}


_CPU_JOB = {}   # the batch, set before the worker processes fork


def _oracle_steps(probs):
    """One SSP-RK3 step (CFL 0.5) of each listed problem with the oracle."""
    import oracle
    U_host, meta, okw = _CPU_JOB["U"], _CPU_JOB["meta"], _CPU_JOB["okw"]
    o = meta["offsets"]
    npts = 0
    for p in probs:
        n = int(o[p + 1] - o[p])
        P = oracle.Problem(system="euler", ndim=1, n=(n,), h=(meta["h"][p],), **okw)
        Up = U_host[:, o[p]:o[p + 1]]
        P.rk3_step(Up, P.cfl_dt(Up, 0.5))
        npts += n
    return npts


def cpu_baseline(seed, okw):
    """The oracle on the host: one step of every ninth problem on one thread,
    then one step of every problem over all cores (forked worker processes,
    started before this process touches the GPU)."""
    import multiprocessing as mp

    from paper_2306_09760_amd import workloads as W
    _, U_host, meta = W.shock_tube_batch(seed=seed)
    nprob = len(meta["lengths"])
    _CPU_JOB.update(U=U_host, meta=meta, okw=okw)
    t0 = time.perf_counter()
    n1 = _oracle_steps(list(range(0, nprob, 9)))
    t1 = time.perf_counter() - t0
    cores = max(1, min(16, os.cpu_count() or 1))
    jobs = [list(range(k, nprob, cores)) for k in range(cores)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        pool.map(abs, range(cores))  # workers up before the clock starts
        t0 = time.perf_counter()
        nall = sum(pool.map(_oracle_steps, jobs))
        tall = time.perf_counter() - t0
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": 3 * nall / tall, "unit": "grid-point RK3-stage updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "host_cpus": os.cpu_count(),
            "sample": f"one SSP-RK3 step of all {nprob} problems of the batch ({nall} points) in "
                      f"{cores} worker processes, {tall:.1f} s wall",
            "single_thread_value": 3 * n1 / t1,
            "single_thread_sample": f"one step of every ninth problem ({n1} points, {t1:.1f} s)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the residual path has no multi-GPU form in this "
              "library (a grid would shard into slabs with halo exchanges, a batch by "
              "problems); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.sweeps_2d:
        sweeps_2d(args.seed)
        return
    if args.sweep_kernels:
        sweep_kernels(args.seed)
        return

    proto = dict(weights=args.weights, xi=args.xi, kappa=0.5, zpow=2, eps=1e-40, diff="mnd6",
                 charproj=True, gamma=1.4, bc="transmissive")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.seed, proto)

    import torch
    from paper_2306_09760_amd import workloads as W
    from paper_2306_09760_amd.solver import BatchPlan, Plan

    dev = torch.device("cuda")
    prob, U_host, meta = W.shock_tube_batch(seed=args.seed)
    lengths = meta["lengths"].astype(np.int64)
    B = BatchPlan(meta["offsets"], meta["h"], **proto)
    U0 = torch.from_numpy(U_host).to(dev)
    U = U0.clone()
    if args.tile is None:
        tile = B.autotune(U)
    else:
        B.tile = tile = args.tile
    B.set_graph(not args.no_graph)
    status = torch.zeros(1, dtype=torch.int32, device=dev)

    def reset(t):
        U.copy_(U0)
        t.zero_()

    def advance(nsteps):
        if args.single_steps:
            for _ in range(nsteps):
                B.rk3_step(U, t, T_END, 0.5, status)
        else:
            B.rk3_steps(U, t, T_END, 0.5, nsteps, status)

    t = torch.zeros(B.nprob, dtype=torch.float64, device=dev)
    advance(args.warmup)
    reset(t)
    torch.cuda.synchronize()

    # ---- timed region: K steps --------------------------------------------
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record()
    advance(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = e0.elapsed_time(e1)
    bad = int(status.item())

    # Active points per step (problems stop at t = 0.2): replay untimed with a
    # snapshot of t before every step (single steps give bitwise the same
    # times as the fused call).
    reset(t)
    active_pts = 0
    for _ in range(args.steps):
        active = (t < T_END).cpu().numpy()
        active_pts += int(lengths[active].sum())
        B.rk3_step(U, t, T_END, 0.5, status)
    torch.cuda.synchronize()
    pt_stages = 3 * active_pts
    value = pt_stages / (ms * 1e-3)

    # ---- dominant kernel: the batch stage kernel --------------------------
    # stage 2 (out = 3/4 U^n + 1/4 (U^(1) + dt R(U^(1)))) with U^(1), U^n and
    # out in three distinct buffers, as inside a step; timed right after the
    # timed steps (before the whole run heats the GPU for seconds), so that
    # it runs in the state of the timed region
    reset(t)
    B.cfl(U, t, T_END, 0.5)
    out = torch.empty_like(U)
    U1 = U0.clone()
    nk = max(args.steps, 10)
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    B.stage(2, U1, U, out)  # warm
    k0.record()
    for _ in range(nk):
        B.stage(2, U1, U, out)
    k1.record()
    torch.cuda.synchronize()
    kernel_ms = k0.elapsed_time(k1) / nk
    # template arguments: NV, direction, batch, FE specialisation, TM, W
    kernel = "sweep_kernel<3, 0, true, 1, %d, 1>" % tile
    total_pts = int(lengths.sum())

    flops_pt = CONTRACT_FLOPS_PER_POINT_STAGE
    tally_pt = FLOPS_PER_POINT_STAGE[args.weights]
    kernel_flops = flops_pt * total_pts
    achieved_tflops = kernel_flops / (kernel_ms * 1e-3) / 1e12
    tally_tflops = tally_pt * total_pts / (kernel_ms * 1e-3) / 1e12
    bytes_pt = 3 * 3 * 8  # stage 2/3 reads U^(k) and U^n, writes U^(k+1)
    hbm_gbs = bytes_pt * total_pts / (kernel_ms * 1e-3) / 1e9

    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def time_launches(fn, n):
        """Average ms of n calls after one warm call (HIP events, current stream)."""
        fn()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        for _ in range(n):
            fn()
        f1.record()
        torch.cuda.synchronize()
        return f0.elapsed_time(f1) / n

    # ---- roof probes: FP64 FMA stream and HBM streaming copy ----------------
    # (beside the stage kernel's timing, in the same state of the GPU)
    from paper_2306_09760_amd._lib import check as _check, lib as _lib
    stream = torch.cuda.current_stream().cuda_stream
    pblocks, piters = 2048, 20000
    pout = torch.empty(pblocks * 256, dtype=torch.float64, device=dev)
    ncopy = 1 << 27  # 1 GiB of doubles
    psrc = torch.ones(ncopy, dtype=torch.float64, device=dev)
    pdst = torch.empty_like(psrc)

    def run_fma():
        _check(_lib().wcns_probe_fp64_fma(pout.data_ptr(), pblocks, piters, stream), "probe")

    def run_copy():
        _check(_lib().wcns_probe_copy(psrc.data_ptr(), pdst.data_ptr(), ncopy, stream), "probe")

    fma_ms = time_launches(run_fma, 3)
    copy_ms = time_launches(run_copy, 5)
    fma_tf = pblocks * 256 * piters * 16 / (fma_ms * 1e-3) / 1e12
    copy_tbs = 16 * ncopy / (copy_ms * 1e-3) / 1e12
    probes = {"fp64_fma_tflops": round(fma_tf, 2), "fp64_fma_frac_of_published": round(fma_tf / PEAK_FP64_TFLOPS, 3),
              "copy_tbps": round(copy_tbs, 3), "copy_frac_of_published": round(copy_tbs * 1e3 / PEAK_HBM_GBS, 3),
              "stage_kernel_frac_of_probe_fp64": round(achieved_tflops / fma_tf, 3),
              "note": "register-resident FP64 FMA chains (2048 x 256 lanes) and a 1 GiB "
                      "16-byte streaming copy, timed with HIP events"}
    del pout, psrc, pdst

    # the batch at xi = 1e6 (a saturating tanh per map term: the kernel's
    # SPEC_FE_SAT instantiation), timed in the same state as the stage kernel
    ms6 = None
    if not args.no_forms:
        B6 = BatchPlan(meta["offsets"], meta["h"], **dict(proto, xi=1e6))
        B6.autotune(U0)
        t6 = torch.zeros(B6.nprob, dtype=torch.float64, device=dev)
        B6.cfl(U0, t6, T_END, 0.5)
        ms6 = time_launches(lambda: B6.stage(2, U1, U0, out), 10)
        del B6

    # ---- the whole run to t = 0.2 ----------------------------------------
    # rk3_steps calls of 256 steps with a host check of completion after
    # each (what a caller running to the end does), each call's stage
    # launches sized to the live-tile count read at the previous check,
    # timed with HIP events; then an untimed replay counts each problem's
    # live steps on the device (single steps give bitwise the times of the
    # fused call), which gives the exact number of grid-point stage updates.
    whole = None
    if not args.no_whole_run:
        reset(t)
        chunk = 256
        torch.cuda.synchronize()
        r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        rwall0 = time.perf_counter()
        r0.record()
        issued = 0
        live = None
        while True:
            B.rk3_steps(U, t, T_END, 0.5, chunk, status, max_live=live)
            issued += chunk
            if bool((t >= T_END).all().item()):
                break
            live = max(1, B.live_tiles())
        r1.record()
        torch.cuda.synchronize()
        run_ms = r0.elapsed_time(r1)
        run_wall = time.perf_counter() - rwall0
        run_bad = int(status.item())
        reset(t)
        Lt = torch.from_numpy(lengths).to(dev)
        live_steps = torch.zeros(B.nprob, dtype=torch.int64, device=dev)
        for _ in range(issued):
            live_steps += (t < T_END)
            B.rk3_steps(U, t, T_END, 0.5, 1, status)
        torch.cuda.synchronize()
        run_pts = 3 * int((live_steps * Lt).sum())
        whole = {"t_end": T_END, "time_to_solution_s": run_ms * 1e-3, "wall_s": run_wall,
                 "steps_issued": issued, "steps_longest_problem": int(live_steps.max()),
                 "steps_shortest_problem": int(live_steps.min()),
                 "grid_point_stage_updates": run_pts,
                 "value": run_pts / (run_ms * 1e-3),
                 "fraction_of_k_step_rate": (run_pts / (run_ms * 1e-3)) / value,
                 "status_word": run_bad,
                 "note": "every problem to t = 0.2 by rk3_steps calls of 256 steps, a host "
                         "check of completion after each, the stage launches of each call "
                         "sized to the live tiles at the previous check; updates counted per "
                         "problem over its live steps"}


    # ---- adjoint / forward time on the 2D periodic problem ----------------
    adjoint = None
    if not args.no_adjoint:
        from paper_2306_09760_amd import rollout as RO
        prob5, U5, _ = W.adjoint2d(seed=args.seed, n=1024, flow_amp=0.05)
        P5 = Plan(**prob5, weights=args.weights, xi=args.xi)
        U5d = torch.from_numpy(U5).to(dev)
        P5.autotune(U5d)
        dt5 = P5.cfl_dt(U5d, 0.5).clone()
        lam = torch.ones_like(U5d)
        Uf = U5d.clone()
        # Each form runs `warm` untimed steps first: this section follows host
        # work (the workload, the autotuner) that leaves the GPU idle, and its
        # clock takes some milliseconds of load to come back up.
        reps, warm = 20, 10
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

        def timed(step):
            for _ in range(warm):
                step()
            a0.record()
            for _ in range(reps):
                step()
            a1.record()
            torch.cuda.synchronize()
            return a0.elapsed_time(a1) / reps

        fwd_ms = timed(lambda: P5.rk3_step(Uf, dt=dt5))
        adj_ms = timed(lambda: P5.rk3_step_adjoint(U5d, lam, dt5))
        # the same step reversed from stored stage states (no recomputation)
        S1, S2 = torch.empty_like(U5d), torch.empty_like(U5d)
        Us = U5d.clone()
        P5.rk3_step_stages(Us, S1, S2, dt=dt5)
        adj_st_ms = timed(lambda: P5.rk3_step_adjoint(U5d, lam, dt5, stages=(S1, S2)))
        del S1, S2, Us

        # 100-step differentiable rollout of J = 1/2 ||rho(T)||^2-type loss:
        # forward, then backward with every state stored (no recompute) and
        # with 9 checkpoints besides U0 (binomial recompute)
        nsteps = 100

        def roll(snap, stages=False):
            X = U5d.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            UT = RO.rollout(P5, X, dt5, nsteps, snap, stages=stages)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            UT[0].sum().backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            return (t1 - t0) * 1e3, (t2 - t1) * 1e3

        roll(nsteps - 1)  # warm
        f_all, b_all = roll(nsteps - 1)
        f_rev, b_rev = roll(9)
        f_st, b_st = roll(0, stages=True)
        adjoint = {"workload": "2D Euler periodic 1024^2, smooth rho, u, v, p, FE xi=%g" % args.xi,
                   "forward_step_ms": round(fwd_ms, 4), "adjoint_step_ms": round(adj_ms, 4),
                   "ratio": round(adj_ms / fwd_ms, 3),
                   "adjoint_step_ms_stages_stored": round(adj_st_ms, 4),
                   "ratio_stages_stored": round(adj_st_ms / fwd_ms, 3),
                   "rollout_steps": nsteps,
                   "rollout_forward_ms": round(f_all, 2),
                   "rollout_backward_ms_all_states_stored": round(b_all, 2),
                   "rollout_backward_ms_9_checkpoints": round(b_rev, 2),
                   "recomputed_steps_9_checkpoints": RO.schedule_cost(nsteps, 9),
                   "rollout_forward_ms_stages_stored": round(f_st, 2),
                   "rollout_backward_ms_stages_stored": round(b_st, 2),
                   "ratio_rollout_no_recompute": round(b_all / f_all, 3),
                   "ratio_rollout_with_recompute": round(b_rev / f_rev, 3),
                   "ratio_rollout_stages_stored": round(b_st / f_all, 3),
                   "note": "adjoint_step_ms recomputes the step's two stage states; "
                           "*_stages_stored reverses from the stage states the forward kept; "
                           "each step time is the mean of %d steps after %d untimed" % (reps, warm)}

    # ---- other forms on the same GPU --------------------------------------
    forms = None
    if not args.no_forms:
        forms = {"batch_stage_xi_%g" % args.xi: {
            "kernel_ms": round(kernel_ms, 4), "pt_stage_per_s": total_pts / (kernel_ms * 1e-3)}}
        forms["batch_stage_xi_1e6"] = {"kernel_ms": round(ms6, 4),
                                       "pt_stage_per_s": total_pts / (ms6 * 1e-3)}
        # plain form on the batch workload: the first 256 tubes, one plan each
        o = meta["offsets"]
        plains = []
        for p in range(256):
            n = int(lengths[p])
            Pp = Plan(system="euler", ndim=1, n=(n,), h=(float(meta["h"][p]),),
                      **{k: v for k, v in proto.items()})
            plains.append((Pp, U0[:, o[p]:o[p + 1]].clone()))
        npl = int(lengths[:256].sum())

        def plain_steps():
            for Pp, Up in plains:
                Pp.rk3_step(Up)
        msp = time_launches(plain_steps, 3)
        forms["plain_1d_one_plan_per_tube"] = {
            "workload": "first 256 tubes of the batch (%d points), one plan and one CFL step each" % npl,
            "ms_per_step": round(msp, 4), "pt_stage_per_s": 3 * npl / (msp * 1e-3)}
        del plains
        # plain form on structured grids
        r2d = W.riemann2d(seed=args.seed, n=2048)
        for name, (pk, Uh, _), scheme in (
                ("plain_2d_riemann_2048", r2d, "wcns"),
                ("plain_2d_riemann_2048_weno", r2d, "weno"),
                ("plain_3d_turbulence_256", W.turbulence3d(seed=args.seed, n=256), "wcns")):
            Pg = Plan(**pk, weights=args.weights, xi=args.xi, scheme=scheme)
            Ug = torch.from_numpy(Uh).to(dev)
            tiles = Pg.autotune(Ug)
            msg = time_launches(lambda: Pg.rk3_step(Ug), 3)
            npg = int(np.prod(Uh.shape[1:]))
            forms[name] = {"ms_per_step": round(msg, 4), "pt_stage_per_s": 3 * npg / (msg * 1e-3),
                           "tiles": list(tiles)}
            del Pg, Ug
        if adjoint is not None:
            n5 = 1024 * 1024
            forms["adjoint_2d_1024"] = {
                "forward_pt_stage_per_s": 3 * n5 / (adjoint["forward_step_ms"] * 1e-3),
                "adjoint_pt_stage_per_s": 3 * n5 / (adjoint["adjoint_step_ms"] * 1e-3)}

    cnt = measured_counters(kernel)
    line = {
        "metric": "grid-point RK3-stage updates/s (FP64), % HBM roofline; adjoint/forward time ratio",
        "value": value,
        "unit": "grid-point RK3-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "batch of 4096 independent 1D Euler shock tubes, N_p uniform in "
                        "[256,4096], FE weights, MND6, SSP-RK3 CFL 0.5, per-problem dt",
            "nprob": int(B.nprob), "total_points": total_pts, "seed": args.seed,
            "weights": args.weights, "xi": args.xi, "tile_midpoints": int(tile),
            "step_call": ("wcns_batch_rk3_step x K" + ("" if args.no_graph else ", graph-replayed")
                          if args.single_steps else
                          "wcns_batch_rk3_steps (K steps, CFL maximum fused into the last stage)"),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tflops,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tflops / PEAK_FP64_TFLOPS,
            "traffic": cnt["bytes_per_launch"] if cnt else None,
            "kernel": kernel,
            "kernel_ms": kernel_ms,
            "flops_per_point_stage": flops_pt,
            "flops_basis": "the scope table's count for the 1D Euler FE stage (divisions, "
                           "square roots and tanh not included)",
            "frac_counting_div_sqrt_tanh_once": (CONTRACT_FLOPS_PER_POINT_STAGE +
                                                 CONTRACT_SPECIAL_PER_POINT_STAGE) * total_pts
                                                / (kernel_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "oracle_tally_flops_per_point_stage": tally_pt,
            "frac_on_oracle_tally": tally_tflops / PEAK_FP64_TFLOPS,
            "hbm_algorithmic_gbs": hbm_gbs,
            "hbm_frac": hbm_gbs / PEAK_HBM_GBS,
            "hbm_measured_gbs": (cnt["bytes_per_launch"] / (kernel_ms * 1e-3) / 1e9) if cnt else None,
            # wave instructions issued / (256 CU x 4 SIMD x 2.4 GHz / 4 cycles each)
            "valu_issue_frac": (cnt["valu_wave_insts"] * 4 / (1024 * 2.4e9 * kernel_ms * 1e-3))
                               if cnt else None,
            "fp64_share_of_valu": (cnt["fp64_wave_insts"] / cnt["valu_wave_insts"]) if cnt else None,
        },
        "cpu_baseline": cpu,
        "whole_run": whole,
        "probes": probes,
        "adjoint_forward": adjoint,
        "forms": forms,
        "status_word": bad,
        "wall_s": wall,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
