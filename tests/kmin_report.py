"""Synthetic k_min study of the exponential methods (Sec. IV.E, Fig. expm),
with the FP64 oracle (CPU only).

For a seeded synthetic system and each time step tau, walkers are
propagated for a few steps with the exact exponential (scipy expm) and with
each method (Taylor, Chebyshev, Krylov, block Krylov) at order k on the same
fields; the energy is the weighted local energy (capped, Sec. V.A) averaged
over the steps (the estimator of Sec. II.A summed over steps).  k_min is the
smallest order whose energy differs from the exact-exponential one by less
than eps (1e-5 Ha in the paper).  The paper averages over 22 molecules in
Gaussian bases; these synthetic Hamiltonians follow the workload recipe
instead.

    python tests/kmin_report.py --walkers 32 --steps 10
    python tests/kmin_report.py --shape 60,6,240 --walkers 32 --steps 10

--shape M,N,G builds a system of the production recipe (couplings scaled
by 1 / sqrt(M)) instead of a named workload.
"""
import argparse
import dataclasses
import multiprocessing as mp
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import afq_workloads as W  # noqa: E402
from oracle import afq_oracle as O  # noqa: E402

EXACT = O.EXP_EXACT
METHODS = {"taylor": O.EXP_TAYLOR, "chebyshev": O.EXP_CHEBYSHEV, "krylov": O.EXP_KRYLOV,
           "block_krylov": O.EXP_BLOCK_KRYLOV}


def energy(p, cfg, method, k, n_walkers, n_steps, seed=0):
    """sum over steps of sum_w W E_capped / sum over steps of sum_w W."""
    wks = [O.init_walker(p) for _ in range(n_walkers)]
    num = den = 0.0
    for t in range(n_steps):
        x = W.fields(seed, 0, t, n_walkers, cfg.G)
        for w in range(n_walkers):
            wks[w], info = O.walker_step(p, wks[w], x[w], method, k,
                                         O.reorth_due(t, cfg.reorth_every))
            num += wks[w].weight * info.e_capped
            den += wks[w].weight
    return num / den if den > 0 else float("nan")


def config(name, shape, tau):
    if shape:
        M, N, G = shape
        return W.generate._cfg(f"M{M}N{N}G{G}", M, N, G, 32, tau, 8, 10, 1, scaled=True)
    return dataclasses.replace(W.CONFIGS[name], tau=tau)


def kmin_for(args):
    name, shape, tau, mname, n_walkers, n_steps, eps, kmax = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        cfg = config(name, shape, tau)
        ham, psi = W.make_system(cfg)
        p = O.prepare(ham.h, ham.L, ham.e_core, psi, tau)
        ref = energy(p, cfg, EXACT, 0, n_walkers, n_steps)
        for k in range(1, kmax + 1):
            if mname == "block_krylov" and k * cfg.N > cfg.M:
                return tau, mname, "n/a", ref
            e = energy(p, cfg, METHODS[mname], k, n_walkers, n_steps)
            if abs(e - ref) < eps:
                return tau, mname, k, ref
    return tau, mname, None, ref


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c1", choices=sorted(W.CONFIGS))
    ap.add_argument("--walkers", type=int, default=32)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--eps", type=float, default=1e-5)
    ap.add_argument("--kmax", type=int, default=16)
    ap.add_argument("--taus", default="0.01,0.05,0.1,0.2,0.3")
    ap.add_argument("--shape", default=None, help="M,N,G of a scaled synthetic system")
    args = ap.parse_args()
    taus = [float(t) for t in args.taus.split(",")]
    shape = tuple(int(v) for v in args.shape.split(",")) if args.shape else None
    jobs = [(args.workload, shape, t, m, args.walkers, args.steps, args.eps, args.kmax)
            for t in taus for m in METHODS]
    with mp.get_context("fork").Pool(min(len(jobs), len(os.sched_getaffinity(0)))) as pool:
        res = pool.map(kmin_for, jobs)
    cfg = config(args.workload, shape, taus[0])
    print(f"k_min for |E - E(expm)| < {args.eps:g} Ha: {cfg.name} (M={cfg.M} N={cfg.N} "
          f"G={cfg.G}), {args.walkers} walkers x {args.steps} steps")
    print(f"{'tau':>6} " + " ".join(f"{m:>13}" for m in METHODS) + f" {'E(expm)':>12}")
    for t in taus:
        row = {m: k for tt, m, k, _ in res if tt == t}
        ref = [r for tt, m, k, r in res if tt == t][0]
        cells = []
        for m in METHODS:
            k = row[m]
            cells.append(f"{'>' + str(args.kmax) if k is None else 'beyond kN=M' if k == 'n/a' else k:>13}")
        print(f"{t:>6.2f} " + " ".join(cells) + f" {ref:>12.5f}")


if __name__ == "__main__":
    main()
