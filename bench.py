"""Throughput of the batched ph-AFQMC walker step on one MI355X.

A step is one full Split-2 walker step (fields, force bias, operator build,
half-steps, Krylov exponential, overlap and phaseless weight, scheduled QR,
local energy and estimator) of every walker of the production-shape
workload: M = 300 orbitals, N = 50 electrons per spin, 1500 Cholesky
vectors, 512 walkers, Krylov dimension 10, QR every 5 steps, tau = 0.05.
Inputs are seeded synthetic Hamiltonians (no molecular integrals are
available); all inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0).  `--gpus N` with N > 1 exits: this build
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
PEAK_HBM = 8.0e12            # bytes/s


def exchange_flops_per_walker(M, N, G):
    """Algorithmic flops of the local-energy contraction per walker:
    T_g = (Psi_T^T L_g) Theta for G Cholesky blocks plus the h block
    (real x complex: 4 N^2 M each) and the traces tr(T_g T_g) (8 N^2 each)."""
    return (G + 1) * (4.0 * N * N * M + 8.0 * N * N)


def step_flops_per_walker(M, N, G, k, reorth_every):
    """Algorithmic flops of one walker step (the production-shape count)."""
    ex = exchange_flops_per_walker(M, N, G)
    build = 4.0 * G * M * M                 # A = sum_g a_g L_g, full complex M x M
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
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


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
    return {"value": rate, "unit": "walker-steps/s", "cores": int(n_procs), "kind": "oracle",
            "sample": f"{n_procs} walkers (one process and one BLAS thread each) x {n_steps} "
                      f"steps after one warm-up step, same workload and fields; "
                      f"per-walker step time {sum(times) / (n_procs * n_steps):.3f} s, "
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
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "mixed_fast"])
    ap.add_argument("--cpu-procs", type=int, default=None,
                    help="oracle processes for the CPU baseline (default: host cores, <= 16)")
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the "
                         "HBM byte counters of a profiler) and exit")
    args = ap.parse_args()
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
        print(f"bench.py: this build runs on one GPU only (got --gpus {args.gpus}); "
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
    prec = {"fp64": afq.PREC_FP64, "mixed": afq.PREC_MIXED,
            "mixed_fast": afq.PREC_MIXED_FAST}[args.precision]
    kw = dict(tau=cfg.tau, exp_method=afq.EXP_KRYLOV, exp_order=cfg.k,
              reorth_every=cfg.reorth_every, seed=0, precision=prec)
    energies = torch.zeros((1, args.steps, 2), dtype=torch.float64, device="cuda")
    log(f"warm-up: {args.warmup} steps")
    ctx.propagate_batch(sid, n_steps=args.warmup, step0=0, **kw)
    ctx.sync()
    log(f"timed: {args.steps} steps")
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.propagate_batch(sid, n_steps=args.steps, step0=args.warmup, energies_out=energies, **kw)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    dt = t1 - t0
    ms_per_step = 1e3 * dt / args.steps
    value = cfg.W * args.steps / dt
    cnt = ctx.get_counters(sid)
    est = energies.cpu().numpy()[0]
    e_last = float(est[-1, 0] / est[-1, 1]) if est[-1, 1] != 0 else float("nan")

    ex_ms, ex_n = prof["exchange"]
    ex_flops = exchange_flops_per_walker(cfg.M, cfg.N, cfg.G) * cfg.W
    ex_avg_s = ex_ms / max(1, ex_n) / 1e3
    achieved = ex_flops / ex_avg_s if ex_avg_s > 0 else 0.0
    roofline = {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP64,
                "traffic": measured_traffic(cfg, args.precision),
                "kernel": "k_exchange", "avg_launch_ms": ex_avg_s * 1e3,
                "flops_per_launch": ex_flops}
    step_fl = step_flops_per_walker(cfg.M, cfg.N, cfg.G, cfg.k, cfg.reorth_every) * cfg.W
    phases = {k: {"ms_per_step": v[0] / args.steps, "launches": v[1]} for k, v in prof.items()}

    out = {
        "metric": "walker-steps/sec at M=300 (FP64 GPU; mixed and CPU oracle alongside)",
        "value": value,
        "unit": "walker-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded random Cholesky Hamiltonian, mean-field trial, Philox fields)",
        "config": {"workload": f"{cfg.name}: M={cfg.M} N={cfg.N} G={cfg.G} walkers={cfg.W} "
                               f"Krylov k={cfg.k} QR every {cfg.reorth_every} tau={cfg.tau}",
                   "M": cfg.M, "N": cfg.N, "n_chol": cfg.G, "walkers": cfg.W, "k": cfg.k,
                   "tau": cfg.tau, "reorth_every": cfg.reorth_every, "parallelism": "1 GPU"},
        "step_tflops": step_fl / (ms_per_step / 1e3) / 1e12,
        "step_frac_fp64_peak": step_fl / (ms_per_step / 1e3) / PEAK_FP64,
        "roofline": roofline,
        "phases": phases,
        "counters": cnt,
        "energy_last_step": e_last,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
