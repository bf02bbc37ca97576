"""Shared helpers of the GPU parity tests: build the same workload for the
HIP library and the oracle, run both step by step on the same fields, and
compare with the tolerance of the FP64 path."""
import math

import numpy as np
import pytest

import afq_workloads as W
from oracle import afq_oracle as O

# FP64 parity bar (relative): GPU and oracle round differently, and the
# propagation amplifies rounding differences mildly (about x10 over 20 steps
# in the oracle's own perturbation runs), so 1e-10 leaves ample margin.
RTOL = 1e-10
NEAR = 1e-8  # threshold events closer than this are flagged, not compared


def device_ready():
    try:
        import torch
        if not torch.cuda.is_available():
            return False
        from paper_2403_02542_amd import afq
        afq.lib()
        return True
    except Exception:
        return False


def require_gpu():
    if not device_ready():
        pytest.fail("GPU test needs a HIP device and the built libafq.so")


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))


def wrap(x):
    return (x + math.pi) % (2 * math.pi) - math.pi


class Case:
    """One system on both sides."""

    def __init__(self, h, L, psi, e_core=0.0, spin=2):
        self.h, self.L, self.psi, self.e_core = h, L, psi, e_core
        self.M, self.N, self.G = h.shape[0], psi.shape[1], L.shape[0]
        self.spin = spin   # 1: (h, L, psi) in spin orbitals, one determinant

    @classmethod
    def from_config(cls, name):
        cfg = W.CONFIGS[name]
        ham, psi = W.make_system(cfg)
        return cls(ham.h, ham.L, psi, ham.e_core)

    @classmethod
    def random(cls, M, N, G, seed, sigma_h=0.1, sigma_A=0.05, e_core=0.0):
        ham = W.hamiltonian(M, G, sigma_h, sigma_A, seed, e_core)
        psi = W.rhf_trial(ham.h, ham.L, N, n_iter=3)
        return cls(ham.h, ham.L, psi, e_core)

    def gpu(self, ctx, n_walkers, phi0=None):
        sid = ctx.init_hamiltonian(self.h, self.L, self.e_core)
        if self.spin == 1:
            ctx.init_trial_spin_orbital(sid, self.psi)
        else:
            ctx.init_trial(sid, self.psi)
        ctx.init_walkers(sid, n_walkers, phi0)
        return sid

    def oracle(self, tau):
        return O.prepare(self.h, self.L, self.e_core, self.psi, tau, spin=self.spin)


def flags_from_info(p, info, weight_factor_ok=True):
    """R-25 style flags: a threshold decision within NEAR of its edge."""
    flag = False
    if np.any(np.abs(np.abs(info.f) - 1.0) < NEAR):
        flag = True
    if abs(math.cos(info.dtheta)) < NEAR:
        flag = True
    if info.e_hybrid != 0:
        arg = -p.tau * (info.e_hybrid.real - p.e0)
        if abs(arg - math.log(10.0)) < NEAR:
            flag = True
    d = O.energy_window(p.spin * p.N, p.tau)
    if min(abs(info.e_loc.real - (p.e0 - d)), abs(info.e_loc.real - (p.e0 + d))) < NEAR:
        flag = True
    return flag


def run_pair(case, ctx, *, tau, k, method, reorth, n_steps, n_walkers, track, seed=0,
             phi0=None, resync=False, live_only=False, stats=None, prop=0, fb_at=0):
    """Propagate n_walkers on the GPU and the `track` subset in the oracle,
    one step per call, on the same fields; returns the worst errors.

    resync=True restarts the oracle every step from the GPU's state, so the
    errors are those of a single step (no accumulation along the path).
    live_only=True stops comparing a walker after the step at which its
    oracle weight reaches zero: such a walker no longer enters any estimate,
    and near the vanishing overlap that zeroed it, its force bias (through
    Theta = Phi (Psi_T^T Phi)^-1) amplifies rounding step after step.
    `stats`, a dict, receives the number of compared walker-steps."""
    import torch
    sid = case.gpu(ctx, n_walkers, phi0)
    p = case.oracle(tau)
    wks = [O.init_walker(p, None if phi0 is None else phi0[w]) for w in track]
    flagged = set()
    dead = set()
    compared = 0
    worst = {"phi": 0.0, "weight": 0.0, "logdet": 0.0, "eloc": 0.0}
    for s in range(n_steps):
        if resync and s > 0:
            for t, w in enumerate(track):
                _, th = O.overlap(case.psi, st["phi"][w])
                wks[t] = O.Walker(st["phi"][w].copy(), complex(st["log_ovlp"][w]), th,
                                  float(st["weight"][w]), bool(st["alive"][w]))
        x = W.fields(seed, 0, s, n_walkers, case.G)
        xd = to_dev(x)
        ctx.propagate_batch(sid, tau=tau, n_steps=1, exp_method=method, exp_order=k,
                            reorth_every=reorth, step0=s, fields=xd, e0=p.e0, propagator=prop,
                            force_bias_at=fb_at)
        torch.cuda.synchronize()
        st = ctx.get_walkers(sid)
        el = ctx.local_energy_batch(sid)
        for t, w in enumerate(track):
            wks[t], info = O.walker_step(p, wks[t], x[w], method, k, O.reorth_due(s, reorth),
                                         prop, fb_at)
            if flags_from_info(p, info):
                flagged.add(w)
            if w in flagged or w in dead:
                continue
            wk = wks[t]
            compared += 1
            if live_only and wk.weight == 0.0:
                dead.add(w)
            worst["phi"] = max(worst["phi"], rel(st["phi"][w], wk.phi))
            worst["weight"] = max(worst["weight"], abs(st["weight"][w] - wk.weight) / max(1.0, abs(wk.weight)))
            dl = st["log_ovlp"][w] - wk.logdet
            worst["logdet"] = max(worst["logdet"], abs(dl.real) / max(1.0, abs(wk.logdet.real)),
                                  abs(wrap(dl.imag)))
            worst["eloc"] = max(worst["eloc"], abs(el[w] - info.e_loc) / max(1.0, abs(info.e_loc)))
        if live_only and len(dead) == len(track):
            print(f"  step {s + 1}/{n_steps}: every tracked walker has weight zero, stop",
                  flush=True)
            break
        if resync or s % 5 == 4 or s == n_steps - 1:
            print(f"  step {s + 1}/{n_steps}: worst so far {worst}, flagged {sorted(flagged)}"
                  + (f", weight zero from then on {sorted(dead)}" if live_only else ""),
                  flush=True)
    if stats is not None:
        stats["compared"] = compared
        stats["dead"] = sorted(dead)
    return worst, flagged, sid
