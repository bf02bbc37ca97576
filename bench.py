"""Throughput of the batched ph-AFQMC walker step on one MI355X.

A step is one full Split-2 walker step (fields, force bias, operator build,
half-steps, Krylov exponential, overlap and phaseless weight, scheduled QR,
local energy and estimator) of every walker of the production-shape
workload: M = 300 orbitals, N = 50 electrons per spin, 1500 Cholesky
vectors, 512 walkers, Krylov dimension 10, QR every 5 steps, tau = 0.05.
Inputs are seeded synthetic Hamiltonians (no molecular integrals are
available); all inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: the library
runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import afq_workloads as W  # noqa: E402

PEAK_FP64 = 78.6e12          # MI355X dense FP64 matrix peak, flop/s
PEAK_BF16 = 2.5e15           # MI355X dense BF16 matrix peak, flop/s
PRECISIONS = {"fp64": lambda a: a.PREC_FP64, "mixed": lambda a: a.PREC_MIXED,
              "mixed_fast": lambda a: a.PREC_MIXED_FAST,
              "mixed_energy": lambda a: a.PREC_MIXED_ENERGY}
DTYPES = {"fp64": "f64",
          "mixed": "bf16x3 split, f32 accumulate (contractions); f64 elsewhere",
          "mixed_fast": "bf16x2 split, f32 accumulate (contractions); f64 elsewhere",
          "mixed_energy": "bf16x3 split, f32 accumulate (local energy); f64 elsewhere"}
PEAK_HBM = 8.0e12            # bytes/s


def exchange_flops_per_walker(M, N, G):
    """Algorithmic flops of the local-energy contraction per walker:
    T_g = (Psi_T^T L_g) Theta for G Cholesky blocks plus the h block
    (real x complex: 4 N^2 M each) and the traces tr(T_g T_g) (8 N^2 each)."""
    return (G + 1) * (4.0 * N * N * M + 8.0 * N * N)


def step_flops_per_walker(M, N, G, k, reorth_every):
    """Algorithmic flops of one walker step (the production-shape count)."""
    ex = exchange_flops_per_walker(M, N, G)
    build = 2.0 * G * M * (M + 1)           # A = sum_g a_g L_g, symmetric: packed triangle
    matvec = 8.0 * k * M * M * N            # k complex operator-orbital products
    onebody = 2 * 4.0 * M * M * N           # two real x complex half-steps
    arnoldi = 8.0 * M * N * (k * k + 2 * k)
    overlap = 4.0 * N * N * M + 8.0 * N * N * M + (8.0 / 3.0) * N ** 3
    qr = (2 * (8.0 * N * N * M + 8.0 * N * N * M)) / max(1, reorth_every)
    return ex + build + matvec + onebody + arnoldi + overlap + qr


def measured_traffic(cfg, precision):
    """HBM bytes per launch of the local-energy kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by a plain-copy
    calibration), or None when the kernel source has changed since, or the
    run is not the profiled workload."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_exchange_c3_fp64_traffic.json")
    if precision != "fp64" or cfg.name != "c3" or cfg.W != 512 or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    for src, sha in rec["sources"].items():
        if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != sha:
            return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def adjoint_flops(M, N, G, W):
    """Algorithmic flops of one call pair afq_local_energy_adjoint +
    afq_force_bias_adjoint over W walkers: the Coulomb vector of every
    (g, w) (G x 2W x NM), all T_g^w (2WN x G N x M), the D_g contraction
    (G N x M x 2WN), the h gradient (W NM + M^2 N), the Coulomb-vector
    weights (G x NM x 2W) and the two batched Psi_T products (G M^2 N each)."""
    ell = 2.0 * G * (2 * W) * N * M
    tg = 2.0 * G * N * (2 * W * N) * M
    dg = 2.0 * G * N * M * (2 * W * N)
    gh = 2.0 * W * N * M + 2.0 * M * M * N
    z = 2.0 * G * N * M * 2 * W
    psi = 2 * 2.0 * G * M * M * N
    return ell + tg + dg + gh + z + psi


def _oracle_grad_worker(args):
    """One walker's gradients (local energy and Coulomb vector), repeated for
    about `budget` seconds after a warm-up call; returns (calls, seconds)."""
    w, budget = args
    from threadpoolctl import threadpool_limits
    from oracle import afq_oracle as O
    st = _CPU_STATE
    p, theta = st["p"], st["theta"]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        O.local_energy_gradient(p, theta)
        O.coulomb_vector_gradient(p, theta, st["d_ell"])
        reps = max(1, int(math.ceil(budget / (time.perf_counter() - t0))))
        t0 = time.perf_counter()
        for _ in range(reps):
            O.local_energy_gradient(p, theta)
            O.coulomb_vector_gradient(p, theta, st["d_ell"])
        return reps, time.perf_counter() - t0


def adjoint_bench(args):
    """Throughput of the hand-written adjoint (local energy and Coulomb
    vector w.r.t. h and L_g) at the c5 shape, after propagating the walkers
    away from the trial."""
    cfg = W.CONFIGS["c5"]
    log(f"generating workload {cfg.name}")
    ham, psi = W.make_system(cfg)
    cpu = None
    if not args.no_cpu:
        import multiprocessing as mp
        from oracle import afq_oracle as O
        with __import__("threadpoolctl").threadpool_limits(1):
            p = O.prepare(ham.h, ham.L, ham.e_core, psi, cfg.tau)
        rng = np.random.default_rng(0)
        phi = psi + 0.05 * (rng.normal(size=psi.shape) + 1j * rng.normal(size=psi.shape))
        _CPU_STATE.update(p=p, theta=O.overlap(psi, phi)[1],
                          d_ell=rng.normal(size=cfg.G) + 1j * rng.normal(size=cfg.G))
        nproc = args.cpu_procs or max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"CPU oracle gradient baseline on {nproc} processes")
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(nproc) as pool:
            res = pool.map(_oracle_grad_worker, [(w, 10.0) for w in range(nproc)])
        wall = time.perf_counter() - t0
        rate = sum(n / t for n, t in res) / cfg.W
        calls = sum(n for n, _ in res)
        cpu = {"value": rate, "unit": "adjoint evaluations/s (all walkers)", "cores": int(nproc),
               "kind": "oracle",
               "sample": f"{nproc} processes (one BLAS thread each) x ~10 s of one-walker "
                         f"gradients (local energy + Coulomb vector), {calls} calls after a "
                         f"warm-up call each; rate scaled to the {cfg.W}-walker batch; "
                         f"per-walker time {sum(t for _, t in res) / calls:.2f} s, "
                         f"wall {wall:.1f} s"}
    import torch
    from paper_2403_02542_amd import afq
    log("initialising the GPU library")
    ctx = afq.Context(0)
    sid = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
    ctx.init_trial(sid, psi)
    ctx.init_walkers(sid, cfg.W)
    ctx.propagate_batch(sid, tau=cfg.tau, n_steps=cfg.steps, exp_method=afq.EXP_KRYLOV,
                        exp_order=cfg.k, reorth_every=cfg.reorth_every, seed=0)
    ctx.sync()
    M, G, N, Wk = cfg.M, cfg.G, cfg.N, cfg.W
    dev = "cuda"
    dE = torch.full((Wk,), 1.0 / Wk, dtype=torch.float64, device=dev)
    d_ell = torch.randn((Wk, G), dtype=torch.complex128, device=dev)
    gh = torch.empty((M, M), dtype=torch.float64, device=dev)
    gL = torch.empty((G, M, M), dtype=torch.float64, device=dev)
    gF = torch.empty((G, M, M), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        ctx.local_energy_adjoint(sid, dE, gh, gL)
        ctx.force_bias_adjoint(sid, d_ell, gF)
    ctx.sync()
    log(f"timed: {args.steps} adjoint evaluations")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.local_energy_adjoint(sid, dE, gh, gL)
        ctx.force_bias_adjoint(sid, d_ell, gF)
    ctx.sync()
    dt = (time.perf_counter() - t0) / args.steps
    fl = adjoint_flops(M, N, G, Wk)
    out = {
        "metric": "adjoint evaluations/s at c5 (d<E_L>/dh, d<E_L>/dL_g and the Coulomb-vector "
                  "adjoint over all walkers)",
        "value": 1.0 / dt, "unit": "evaluations/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded random Cholesky Hamiltonian, walkers after "
                f"{cfg.steps} Krylov steps)",
        "config": {"workload": f"c5: M={M} N={N} G={G} walkers={Wk}", "M": M, "N": N,
                   "n_chol": G, "walkers": Wk, "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "achieved": fl / dt / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": fl / dt / PEAK_FP64, "traffic": None,
                     "kernel": "adjoint call pair (k_adj_t and the sliced D product dominate)",
                     "flops_per_call": fl},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def _oracle_system_worker(cfg):
    """One walker-step of the oracle on one system of the uneven batch (after
    one warm-up step); the system is generated inside the worker."""
    from threadpoolctl import threadpool_limits
    from oracle import afq_oracle as O
    with threadpool_limits(1):
        ham, psi = W.make_system(cfg, trial_iters=W.C4.trial_iters)
        p = O.prepare(ham.h, ham.L, ham.e_core, psi, cfg.tau)
        wk = O.init_walker(p)
        wk, _ = O.walker_step(p, wk, W.fields(0, 0, 0, cfg.W, cfg.G)[0], O.EXP_KRYLOV, cfg.k,
                              O.reorth_due(0, cfg.reorth_every))
        t0 = time.perf_counter()
        O.walker_step(p, wk, W.fields(0, 0, 1, cfg.W, cfg.G)[0], O.EXP_KRYLOV, cfg.k,
                      O.reorth_due(1, cfg.reorth_every))
        return cfg.M, time.perf_counter() - t0


def uneven_cpu_baseline(cfgs, nproc):
    """Oracle walker-step times on systems at six size quantiles, log-log
    interpolated over all systems of the batch."""
    import multiprocessing as mp
    order = sorted(range(len(cfgs)), key=lambda i: cfgs[i].M)
    pick = sorted({order[int(round(q * (len(order) - 1)))] for q in np.linspace(0, 1, 6)})
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(min(nproc, len(pick))) as pool:
        res = sorted(pool.map(_oracle_system_worker, [cfgs[i] for i in pick]))
    wall = time.perf_counter() - t0
    lm = np.log([m for m, _ in res])
    lt = np.log([t for _, t in res])
    per_step = sum(c.W * math.exp(np.interp(math.log(c.M), lm, lt)) for c in cfgs)
    rate = sum(c.W for c in cfgs) / per_step
    return {"value": rate, "unit": "walker-steps/s", "cores": 1, "kind": "oracle",
            "sample": "one walker-step (after a warm-up step) of the oracle, one BLAS thread, on "
                      f"the systems with M = {[m for m, _ in res]} "
                      f"(s per walker-step: {[round(t, 3) for _, t in res]}); the batch's step "
                      "time is the sum over all systems and walkers of the log-log interpolated "
                      f"per-walker time ({per_step:.0f} s per batch step on one core); "
                      f"wall {wall:.1f} s"}


def open_shell_bench(args):
    """Open-shell walkers beside the closed shell on the same Hamiltonian (the
    c2 shape: M = 120, G = 600, 256 walkers, Krylov k = 8, tau = 0.05, QR every
    step): N_alpha = 20, N_beta = 18 through afq_init_trial (the library runs
    them as one determinant of 2M = 240 spin orbitals), against N = 20 closed
    shell.  FP64, fields from the library's generator, HIP-event phases."""
    import torch
    from paper_2403_02542_amd import afq
    cfg = W.CONFIGS["c2"]
    nb = cfg.N - 2
    log(f"generating workload {cfg.name}")
    ham, psi = W.make_system(cfg)
    ctx = afq.Context(0)
    res = {}
    for name in ("closed_shell", "open_shell"):
        sid = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
        if name == "open_shell":
            ctx.init_trial(sid, np.hstack([psi, psi[:, :nb]]), n_beta=nb)
        else:
            ctx.init_trial(sid, psi)
        ctx.init_walkers(sid, cfg.W)
        kw = dict(tau=cfg.tau, exp_method=afq.EXP_KRYLOV, exp_order=cfg.k,
                  reorth_every=cfg.reorth_every, seed=0)
        ctx.propagate_batch(sid, n_steps=args.warmup, step0=0, **kw)
        ctx.sync()
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        t0 = time.perf_counter()
        ctx.propagate_batch(sid, n_steps=args.steps, step0=args.warmup, **kw)
        ctx.sync()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        ctx.profile(False)
        d = ctx.dims[sid]
        Mx, Nx = d["M"], d["N"]
        ex_ms = prof["exchange"][0] / max(1, prof["exchange"][1])
        fl = exchange_flops_per_walker(Mx, Nx, cfg.G) * cfg.W
        res[name] = {"value": cfg.W * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
                     "orbitals": Mx, "electrons": Nx,
                     "local_energy_ms": ex_ms,
                     "local_energy_frac_fp64_peak": fl / (ex_ms * 1e-3) / PEAK_FP64,
                     "phases_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()}}
        log(f"{name}: {res[name]['value']:.1f} walker-steps/s")
    o, c = res["open_shell"], res["closed_shell"]
    line = {"metric": "walker-steps/sec, open shell (c2 Hamiltonian, N_alpha=20, N_beta=18, "
                      "2M = 240 spin orbitals, FP64)",
            "value": o["value"], "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": o["ms_per_step"], "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic (seeded random Cholesky Hamiltonian, mean-field trial, Philox fields)",
            "config": {"workload": "c2 Hamiltonian (M=120, G=600), 256 walkers, Krylov k=8, "
                                   "tau=0.05, QR every step; open shell N_alpha=20, N_beta=18",
                       "parallelism": "1 GPU"},
            "open_shell": o, "closed_shell_same_hamiltonian": c,
            "open_over_closed_time": o["ms_per_step"] / c["ms_per_step"],
            "note": "spin-orbital form: operator, products and L over 2M functions with half of "
                    "every matrix zero; separate alpha and beta blocks would do about a quarter "
                    "to a half of this work"}
    print(json.dumps(line))


def uneven_bench(args):
    """Throughput of the 48-system uneven batch (M ~ U{40..400}, N = M/6,
    G = 5M, 64 walkers each, Krylov k = 8, tau = 0.05, QR every step)."""
    import torch
    from paper_2403_02542_amd import afq
    batch = W.C4
    cfgs = batch.configs()
    cpu = None
    if not args.no_cpu:
        nproc = args.cpu_procs or max(1, min(16, len(os.sched_getaffinity(0))))
        log("CPU oracle baseline on sampled systems")
        cpu = uneven_cpu_baseline(cfgs, nproc)
        log(f"CPU oracle: {cpu['value']:.3f} walker-steps/s")
    log("initialising the GPU library")
    ctx = afq.Context(0)
    ids = []
    for i, cfg in enumerate(cfgs):
        ham, psi = W.make_system(cfg, trial_iters=batch.trial_iters)
        sid = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
        ctx.init_trial(sid, psi)
        ctx.init_walkers(sid, batch.W)
        ids.append(sid)
        del ham
        log(f"system {i + 1}/{len(cfgs)}: M={cfg.M} N={cfg.N} G={cfg.G}")
    sched = {"auto": afq.SCHED_AUTO, "serial": afq.SCHED_SERIAL, "streams": afq.SCHED_STREAMS,
             "graph": afq.SCHED_GRAPH}[args.schedule]
    kw = dict(tau=batch.tau, exp_method=afq.EXP_KRYLOV, exp_order=batch.k,
              reorth_every=batch.reorth_every, seed=0, schedule=sched)
    if args.autotune:
        log("autotuning tiles")
        ctx.autotune(ids, **{k: v for k, v in kw.items() if k != "schedule"})
    warm = args.warmup + (args.warmup % 2)   # even: the graph's buffer state repeats
    energies = torch.zeros((len(ids), args.steps, 2), dtype=torch.float64, device="cuda")
    ew = torch.zeros((len(ids), max(1, warm), 2), dtype=torch.float64, device="cuda")
    step0 = 0

    def timed(schedule):
        nonlocal step0
        k = dict(kw, schedule=schedule)
        log(f"schedule {schedule}: warm-up {warm} steps")
        ctx.propagate_batch(ids, n_steps=warm, step0=step0, energies_out=ew, **k)
        ctx.sync()
        torch.cuda.synchronize()
        log(f"schedule {schedule}: timed {args.steps} steps")
        t0 = time.perf_counter()
        ctx.propagate_batch(ids, n_steps=args.steps, step0=step0 + warm, energies_out=energies,
                            **k)
        ctx.sync()
        torch.cuda.synchronize()
        step0 += warm + args.steps
        return time.perf_counter() - t0

    compare = {}
    if args.compare_schedules:
        for name in ("serial", "streams", "graph"):
            if name != args.schedule:
                dtn = timed({"serial": afq.SCHED_SERIAL, "streams": afq.SCHED_STREAMS,
                             "graph": afq.SCHED_GRAPH}[name])
                compare[name] = {"ms_per_step": dtn / args.steps * 1e3,
                                 "walker_steps_per_s": len(ids) * batch.W * args.steps / dtn}
    dt = timed(sched)
    n_ws = len(ids) * batch.W
    value = n_ws * args.steps / dt
    # per-size breakdown: every system alone, one step after the other
    log("per-system steps alone")
    per = []
    kw1 = dict(kw, schedule=afq.SCHED_SERIAL)
    for i, sid in enumerate(ids):
        ctx.sync()
        t1 = time.perf_counter()
        ctx.propagate_batch(sid, n_steps=2, step0=step0, **kw1)
        ctx.sync()
        ms = (time.perf_counter() - t1) / 2 * 1e3
        per.append({"M": cfgs[i].M, "N": cfgs[i].N, "G": cfgs[i].G, "ms_per_step_alone": ms,
                    "walker_steps_per_s_alone": batch.W / ms * 1e3})
    step0 += 2
    # phases (one step after the other, HIP events) for the local-energy roofline
    ctx.profile(True)
    ctx.profile_read()
    ctx.propagate_batch(ids, n_steps=2, step0=step0, **kw1)
    prof = ctx.profile_read()
    ctx.profile(False)
    ex_ms, ex_n = prof["exchange"]
    ex_fl = 2 * sum(exchange_flops_per_walker(c.M, c.N, c.G) * c.W for c in cfgs)
    achieved = ex_fl / (ex_ms / 1e3) if ex_ms > 0 else 0.0
    alone_ms = sum(p["ms_per_step_alone"] for p in per)
    out = {
        "metric": "walker-steps/sec over 48 uneven systems (M ~ U{40..400}, FP64)",
        "value": value, "unit": "walker-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": warm, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (48 seeded random Cholesky Hamiltonians, mean-field trials, Philox "
                "fields)",
        "config": {"workload": f"c4: {len(ids)} systems, M ~ U{{40..400}}, N = M//6, G = 5M, "
                               f"{batch.W} walkers each, Krylov k={batch.k}, tau={batch.tau}, "
                               f"QR every {batch.reorth_every}",
                   "schedule": args.schedule, "autotune": bool(args.autotune),
                   "parallelism": "1 GPU"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                     "kernel": "k_exchange (per system, one after the other, HIP events)",
                     "exchange_ms_per_step": ex_ms / 2},
        "sum_alone_ms_per_step": alone_ms,
        "batched_speedup_vs_alone": alone_ms / (dt / args.steps * 1e3),
        "other_schedules": compare,
        "per_size": per,
        "phases_serial_ms_per_step": {k: v[0] / 2 for k, v in prof.items()},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


_CPU_STATE = {}
_T0 = time.perf_counter()


def log(msg):
    print(f"[bench {time.perf_counter() - _T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def _oracle_worker(args):
    """Time one walker of the oracle: one warm-up step, then n_steps steps."""
    w, n_steps = args
    from threadpoolctl import threadpool_limits
    from oracle import afq_oracle as O
    st = _CPU_STATE
    cfg, p = st["cfg"], st["p"]
    with threadpool_limits(1):
        wk = O.init_walker(p)
        x0 = W.fields(0, 0, 0, cfg.W, cfg.G)[w]
        wk, _ = O.walker_step(p, wk, x0, O.EXP_KRYLOV, cfg.k, O.reorth_due(0, cfg.reorth_every))
        t0 = time.perf_counter()
        for t in range(1, 1 + n_steps):
            x = W.fields(0, 0, t, cfg.W, cfg.G)[w]
            wk, _ = O.walker_step(p, wk, x, O.EXP_KRYLOV, cfg.k, O.reorth_due(t, cfg.reorth_every))
        return time.perf_counter() - t0


def cpu_model():
    """Host CPU model name (from /proc/cpuinfo), or None."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def population_rows(est):
    """Per-step (sum W E_L, sum W) rows as the weighted estimate E_k of
    Sec. II.A, or "extinct" when no walker carries weight."""
    out = []
    for num, den in est:
        out.append({"sum_w": float(den),
                    "e_k": float(num / den) if den > 0 else "extinct"})
    return out


def run_statistics(afq, est):
    """Time average, variance and correlation length (Sec. II.A, Eq.
    (variance)) of the timed steps' estimates, from the library's host
    statistics; every timed step counts (no equilibration cut), so on a short
    run these describe the run, not a converged energy."""
    w = np.array([den for _, den in est], dtype=np.float64)
    e = np.array([num / den if den > 0 else 0.0 for num, den in est], dtype=np.float64)
    live = w > 0
    if live.sum() < 2:
        return {"note": "fewer than two steps with weight"}
    mean, var, n = afq.stats_time_average(w, e, 0)
    k = afq.stats_kappa(e[live], 5.0)
    kappa = max(1.0, k["acf"])
    return {"e_bar": mean, "sigma_e2": var, "n": n, "kappa_acf": k["acf"],
            "kappa_block": k["block"], "sigma_e_bar": float(np.sqrt(max(var, 0.0) * kappa / n)),
            "note": "every timed step counted (no equilibration cut); kappa from the steps "
                    "with weight"}


def cpu_baseline(cfg, ham, psi, n_procs, n_steps):
    """The FP64 oracle, as it stands, on a bounded sample of the workload:
    walkers are independent, so n_procs processes (one BLAS thread each, the
    oracle's fastest setting: its many small products lose to threading)
    each run one walker for n_steps steps after a warm-up step.  Must run
    before the process touches the GPU (the pool forks)."""
    import multiprocessing as mp
    from oracle import afq_oracle as O
    with __import__("threadpoolctl").threadpool_limits(1):
        p = O.prepare(ham.h, ham.L, ham.e_core, psi, cfg.tau)
    _CPU_STATE.update(cfg=cfg, p=p)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(n_procs) as pool:
        times = pool.map(_oracle_worker, [(w, n_steps) for w in range(n_procs)])
    wall = time.perf_counter() - t0
    rate = sum(n_steps / t for t in times)
    per = sum(times) / (n_procs * n_steps)
    return {"value": rate, "unit": "walker-steps/s", "cores": int(n_procs), "kind": "oracle",
            "one_thread_value": 1.0 / per, "cpu_model": cpu_model(),
            "host_cpus_visible": len(os.sched_getaffinity(0)),
            "sample": f"{n_procs} walkers (one process and one BLAS thread each; {n_procs} is "
                      f"the host CPU share of one GPU) x {n_steps} steps after one warm-up step, "
                      f"same workload and fields; per-walker step time {per:.3f} s on one thread, "
                      f"wall {wall:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(W.CONFIGS))
    ap.add_argument("--walkers", type=int, default=None)
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precision", default="fp64",
                    choices=["fp64", "mixed", "mixed_fast", "mixed_energy"])
    ap.add_argument("--energy-every", type=int, default=1,
                    help="measure the local energy every this many steps (default 1)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="with --precision fp64: skip the mixed-precision runs beside it")
    ap.add_argument("--cpu-procs", type=int, default=None,
                    help="oracle processes for the CPU baseline (default: host cores, <= 16)")
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the "
                         "HBM byte counters of a profiler) and exit")
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint entry points at the c5 shape instead of the step")
    ap.add_argument("--open-shell", action="store_true",
                    help="open-shell walkers beside the closed shell on the c2 Hamiltonian")
    ap.add_argument("--uneven", action="store_true",
                    help="time the 48-system uneven batch (c4) instead of the single system")
    ap.add_argument("--schedule", default="auto", choices=["auto", "serial", "streams", "graph"])
    ap.add_argument("--autotune", action="store_true", help="tune tile shapes before timing")
    ap.add_argument("--compare-schedules", action="store_true",
                    help="with --uneven: also time the other schedules")
    args = ap.parse_args()
    if args.adjoint and args.gpus == 1:
        adjoint_bench(args)
        return
    if args.uneven and args.gpus == 1:
        uneven_bench(args)
        return
    if args.open_shell and args.gpus == 1:
        open_shell_bench(args)
        return
    if args.copy_probe:
        import torch
        n = args.copy_probe * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8}))
        return
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (got --gpus {args.gpus}); "
              "walkers shard trivially across GPUs but no multi-GPU path is built.",
              file=sys.stderr)
        sys.exit(2)

    cfg = W.CONFIGS[args.workload]
    if args.walkers or args.tau:
        import dataclasses
        cfg = dataclasses.replace(cfg, W=args.walkers or cfg.W, tau=args.tau or cfg.tau)
    log(f"generating workload {cfg.name}")
    ham, psi = W.make_system(cfg)
    cpu = None
    if not args.no_cpu:
        ncores = len(os.sched_getaffinity(0))
        nproc = args.cpu_procs or max(1, min(16, ncores))
        log(f"CPU oracle baseline on {nproc} processes")
        cpu = cpu_baseline(cfg, ham, psi, nproc, args.cpu_steps)
        log(f"CPU oracle: {cpu['value']:.3f} walker-steps/s")

    import torch
    from paper_2403_02542_amd import afq
    log("initialising the GPU library")
    ctx = afq.Context(0)
    sid = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
    ctx.init_trial(sid, psi)
    ctx.init_walkers(sid, cfg.W)
    if args.autotune:
        log("autotuning tiles")
        ctx.autotune([sid])
    step0 = 0

    def run_mode(name, energy_every=None, tau=None):
        """Warm-up then timed steps in one precision mode (HIP-event phases)."""
        nonlocal step0
        prec = PRECISIONS[name](afq)
        kw = dict(tau=tau or cfg.tau, exp_method=afq.EXP_KRYLOV, exp_order=cfg.k,
                  reorth_every=cfg.reorth_every, seed=0, precision=prec,
                  energy_every=energy_every or args.energy_every)
        energies = torch.zeros((1, args.steps, 2), dtype=torch.float64, device="cuda")
        log(f"{name}: warm-up {args.warmup} steps")
        ctx.propagate_batch(sid, n_steps=args.warmup, step0=step0, **kw)
        ctx.sync()
        log(f"{name}: timed {args.steps} steps")
        torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.propagate_batch(sid, n_steps=args.steps, step0=step0 + args.warmup,
                            energies_out=energies, **kw)
        ctx.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = ctx.profile_read()
        ctx.profile(False)
        step0 += args.warmup + args.steps
        dt = t1 - t0
        est = energies.cpu().numpy()[0]
        ex_ms, ex_n = prof["exchange"]
        ex_flops = exchange_flops_per_walker(cfg.M, cfg.N, cfg.G) * cfg.W
        ex_avg_s = ex_ms / max(1, ex_n) / 1e3 if ex_n else float("nan")
        if name == "fp64":
            # FP64 matrix cores: the algorithmic flops against the FP64 peak
            achieved, peak, kernel, fl = ex_flops / ex_avg_s, PEAK_FP64, "k_exchange", ex_flops
        else:
            # BF16 matrix cores: each FP64-equivalent product is 6 (3 pieces)
            # or 3 (2 pieces) BF16 piece products, against the BF16 peak
            prods = 3 if name == "mixed_fast" else 6
            fl = prods * ex_flops
            achieved, peak, kernel = fl / ex_avg_s, PEAK_BF16, "k_exchange_mx"
        roof = {"bound": "mfma", "achieved": achieved / 1e12, "peak": peak / 1e12,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": measured_traffic(cfg, name), "kernel": kernel,
                "avg_launch_ms": ex_avg_s * 1e3, "flops_per_launch": fl}
        return {"value": cfg.W * args.steps / dt, "ms_per_step": 1e3 * dt / args.steps,
                "roofline": roof,
                "phases": {k: {"ms_per_step": v[0] / args.steps, "launches": v[1]}
                           for k, v in prof.items()},
                "population": population_rows(est),
                "statistics": run_statistics(afq, est),
                "first_step": step0 - args.steps}

    main_run = run_mode(args.precision)
    cnt = ctx.get_counters(sid)
    if cnt["weighted"] == 0:
        log("the walker population is extinct at the last timed step (no walker carries weight; "
            "every walker is still propagated, so the timing covers the full step)")
    others = {}
    sparse = {}
    tau_sweep = {}
    if args.precision == "fp64" and not args.no_mixed:
        for name in ("mixed_energy", "mixed"):
            r = run_mode(name)
            others[name] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                            "speedup_vs_fp64": r["value"] / main_run["value"],
                            "roofline": r["roofline"],
                            "phases_ms_per_step": {k: v["ms_per_step"]
                                                   for k, v in r["phases"].items()}}
        if args.workload == "c3" and args.energy_every <= 1:
            # the other time steps of the extrapolation sweep (same shapes;
            # the Krylov dimension and the work per step do not change)
            for tau in (0.02, 0.1):
                for name in ("fp64", "mixed_energy"):
                    r = run_mode(name, tau=tau)
                    tau_sweep.setdefault(str(tau), {})[name] = {
                        "value": r["value"], "ms_per_step": r["ms_per_step"],
                        "population": r["population"]}
        if args.energy_every <= 1 and args.steps >= 10:
            # the local energy measured every 10th step (the other steps form
            # only the Coulomb vector for the force bias), FP64 and MIXED_ENERGY
            for name in ("fp64", "mixed_energy"):
                r = run_mode(name, energy_every=10)
                sparse[name] = {"value": r["value"], "ms_per_step": r["ms_per_step"],
                                "speedup_vs_fp64_every_step": r["value"] / main_run["value"],
                                "phases_ms_per_step": {k: v["ms_per_step"]
                                                       for k, v in r["phases"].items()}}
    ms_per_step = main_run["ms_per_step"]
    step_fl = step_flops_per_walker(cfg.M, cfg.N, cfg.G, cfg.k, cfg.reorth_every) * cfg.W
    out = {
        "metric": "walker-steps/sec at M=300 (FP64 GPU; mixed and CPU oracle alongside)",
        "value": main_run["value"],
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[args.precision],
        "data": "synthetic (seeded random Cholesky Hamiltonian, mean-field trial, Philox fields)",
        "config": {"workload": f"{cfg.name}: M={cfg.M} N={cfg.N} G={cfg.G} walkers={cfg.W} "
                               f"Krylov k={cfg.k} QR every {cfg.reorth_every} tau={cfg.tau}",
                   "M": cfg.M, "N": cfg.N, "n_chol": cfg.G, "walkers": cfg.W, "k": cfg.k,
                   "tau": cfg.tau, "reorth_every": cfg.reorth_every,
                   "precision": args.precision, "energy_every": args.energy_every,
                   "autotune": bool(args.autotune),
                   "parallelism": "1 GPU"},
        "step_tflops": step_fl / (ms_per_step / 1e3) / 1e12,
        "step_frac_fp64_peak": step_fl / (ms_per_step / 1e3) / PEAK_FP64,
        "roofline": main_run["roofline"],
        "phases": main_run["phases"],
        "counters": cnt,
        "statistics": main_run["statistics"],
        "population": {"timed_steps_from": main_run["first_step"],
                       "per_step": main_run["population"],
                       "weighted_walkers_last_step": cnt["weighted"],
                       "note": "fixed E0 = trial energy, no population control: on this "
                               "synthetic workload the walkers lose their overlap with the "
                               "trial within ~10 steps and the phaseless rule / reweighting "
                               "cap zero their weights; dead walkers keep being propagated"},
        "mixed": others,
        "mixed_headline": None if "mixed_energy" not in others else {
            "form": "mixed_energy",
            "speedup_vs_fp64": others["mixed_energy"]["speedup_vs_fp64"],
            "note": "the BF16-split form that stays within 0.1 mHa per walker of the FP64 "
                    "energies (local-energy contraction in three BF16 pieces, propagation and "
                    "Coulomb vector in FP64); the 3x target is not reached: the FP64 "
                    "propagation alone bounds the ratio, and two pieces miss the bar"},
        "tau_sweep": tau_sweep,
        "energy_every_10": sparse,
        "energy_every_10_note": "different work (local energy on every 10th step only); "
                                "not comparable with the every-step speedups",
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
