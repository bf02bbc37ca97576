"""Walker-population report of the FP64 oracle (CPU only).

Runs the oracle on a workload shape for a few walkers and prints, per step:
the walkers that still carry weight (W > 0), the total weight, which rule
set a weight to zero that step (the reweighting cap of Sec. V.B, the
phaseless cosine of Eq. (phaseless), or a frozen non-finite walker), the
trial energy E0 against the mean local energy of the walkers with weight,
and the spread of the hybrid energy.  Walkers are independent under a fixed
E0, so each runs in its own process.

    python tests/population_report.py c2 --walkers 16 --steps 50
    python tests/population_report.py c3 --walkers 4 --steps 10
    python tests/population_report.py c2 --e0-update --pop-every 1 --steps 50

With --e0-update, E0 follows the running weighted energy estimate (the
update rule of `oracle.afq_oracle.update_e0`); with --pop-every r the
population is comb-resampled after every r-th step (`comb_resample`).
Either couples the walkers, which then run together in one process.
"""
import argparse
import dataclasses
import math
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import afq_workloads as W  # noqa: E402
from oracle import afq_oracle as O  # noqa: E402

_STATE = {}


def _walker_path(w):
    cfg, p, n_steps = _STATE["cfg"], _STATE["p"], _STATE["n"]
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        wk = O.init_walker(p)
        rows = []
        for t in range(n_steps):
            x = W.fields(cfg.seed, 0, t, cfg.W, cfg.G)[w]
            wk, info = O.walker_step(p, wk, x, O.EXP_KRYLOV, cfg.k,
                                     O.reorth_due(t, cfg.reorth_every))
            rows.append((wk.weight, info.e_loc.real, info.e_capped, info.e_hybrid.real,
                         info.zeroed_by))
        return rows


def report(rows_by_walker, e0s):
    n_w = len(rows_by_walker)
    n_steps = len(rows_by_walker[0])
    print(f"{'step':>4} {'E0':>10} {'W>0':>5} {'sum W':>11} {'cap':>4} {'phase':>5} "
          f"{'frozen':>6} {'<E_L> (W>0)':>12} {'<E_H> (W>0)':>12} {'sd E_H':>8} {'E_k':>11}")
    for t in range(n_steps):
        wts = np.array([r[t][0] for r in rows_by_walker])
        el = np.array([r[t][1] for r in rows_by_walker])
        ec = np.array([r[t][2] for r in rows_by_walker])
        eh = np.array([r[t][3] for r in rows_by_walker])
        why = [r[t][4] for r in rows_by_walker]
        live = wts > 0
        sw = wts.sum()
        ek = (wts * ec).sum() / sw if sw > 0 else float("nan")
        mel = el[live].mean() if live.any() else float("nan")
        meh = eh[live].mean() if live.any() else float("nan")
        seh = eh[live].std() if live.sum() > 1 else float("nan")
        print(f"{t + 1:>4} {e0s[t]:>10.3f} {int(live.sum()):>3}/{n_w:<2} {sw:>10.3e} "
              f"{why.count('reweight_cap'):>4} {why.count('phase'):>5} {why.count('frozen'):>6} "
              f"{mel:>12.3f} {meh:>12.3f} {seh:>8.2f} "
              f"{'extinct' if sw == 0 else f'{ek:.3f}':>11}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(W.CONFIGS))
    ap.add_argument("--walkers", type=int, default=8)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--tau", type=float, default=None)
    ap.add_argument("--procs", type=int, default=min(8, len(os.sched_getaffinity(0))))
    ap.add_argument("--e0-update", action="store_true")
    ap.add_argument("--pop-every", type=int, default=0)
    args = ap.parse_args()
    cfg = W.CONFIGS[args.workload]
    if args.tau:
        cfg = dataclasses.replace(cfg, tau=args.tau)
    n_steps = args.steps or cfg.steps
    ham, psi = W.make_system(cfg)
    p = O.prepare(ham.h, ham.L, ham.e_core, psi, cfg.tau)
    print(f"{cfg.name}: M={cfg.M} N={cfg.N} G={cfg.G} tau={cfg.tau} k={cfg.k} "
          f"QR every {cfg.reorth_every}; {args.walkers} walkers of the batch of {cfg.W}; "
          f"E_HF(trial) = E0 = {p.e0:.4f}; energy window +-{O.energy_window(2 * cfg.N, cfg.tau):.2f}; "
          f"reweighting cap at E_H < E0 - {math.log(10.0) / cfg.tau:.2f}")
    if not args.e0_update and not args.pop_every:
        _STATE.update(cfg=cfg, p=p, n=n_steps)
        with mp.get_context("fork").Pool(args.procs) as pool:
            rows = pool.map(_walker_path, range(args.walkers))
        report(rows, [p.e0] * n_steps)
        return
    wks = [O.init_walker(p) for _ in range(args.walkers)]
    rows = [[] for _ in range(args.walkers)]
    e0s = []
    state = O.E0State(p.e0) if args.e0_update else None
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        for t in range(n_steps):
            e0s.append(p.e0)
            x = W.fields(cfg.seed, 0, t, cfg.W, cfg.G)
            wks, hist = O.run(p, wks, lambda s: x, 1, O.EXP_KRYLOV, cfg.k, cfg.reorth_every,
                              step0=t, e0_state=state, pop_every=args.pop_every,
                              comb_u=lambda s: W.comb_uniform(cfg.seed, 0, s))
            h = hist[0]
            for w in range(args.walkers):
                rows[w].append((h["weight"][w], h["e_loc"][w].real, h["e_capped"][w],
                                h["e_hybrid"][w].real, h["zeroed_by"][w]))
    report(rows, e0s)


if __name__ == "__main__":
    main()
