"""Mixed precision (BF16-split MFMA contractions, FP32 accumulation) against
the FP64 oracle: per-quantity errors, with the local-energy bound of 1e-4 Ha
(0.1 mHa) per walker."""
import numpy as np
import pytest

import afq_workloads as W
import gpu_common as C
from oracle import afq_oracle as O

pytestmark = pytest.mark.gpu
E_TOL = 1e-4   # Ha per walker


@pytest.fixture(scope="module")
def ctx():
    C.require_gpu()
    from paper_2403_02542_amd import afq
    c = afq.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cfg", ["c2", "c3"])
def test_mixed_local_energy(ctx, cfg):
    """Walkers after 6 FP64 steps (far from the trial); E_L from the
    BF16-split contraction vs the FP64 kernel and vs the oracle."""
    import torch
    from paper_2403_02542_amd import afq
    conf = W.CONFIGS[cfg]
    case = C.Case.from_config(cfg)
    nw = 32
    sid = case.gpu(ctx, nw)
    ctx.propagate_batch(sid, tau=conf.tau, n_steps=6, exp_order=conf.k,
                        reorth_every=conf.reorth_every, seed=1)
    torch.cuda.synchronize()
    e64 = ctx.local_energy_batch(sid)
    st = ctx.get_walkers(sid)
    p = case.oracle(conf.tau)
    errs = {}
    for prec in (afq.PREC_MIXED, afq.PREC_MIXED_FAST):
        emx = ctx.local_energy_batch(sid, precision=prec)
        errs[prec] = np.abs(emx - e64).max()
        for w in (0, nw - 1):
            _, th = O.overlap(case.psi, st["phi"][w])
            eo = O.local_energy(p, st["phi"][w], th)
            assert abs(emx[w] - eo) < E_TOL
    print(cfg, "max |E_L(mixed) - E_L(fp64)|: 3 pieces %.3e, 2 pieces %.3e"
          % (errs[afq.PREC_MIXED], errs[afq.PREC_MIXED_FAST]))
    assert errs[afq.PREC_MIXED] < E_TOL
    assert errs[afq.PREC_MIXED] < errs[afq.PREC_MIXED_FAST]


@pytest.mark.parametrize("prec_name", ["MIXED"])
def test_mixed_propagation_c2(ctx, prec_name):
    """c2 trajectories in mixed precision vs the FP64 oracle on the same
    fields: E_L within 1e-4 Ha per walker over 20 steps; the orbital and
    weight deviations are reported."""
    import torch
    from paper_2403_02542_amd import afq
    prec = getattr(afq, "PREC_" + prec_name)
    conf = W.CONFIGS["c2"]
    case = C.Case.from_config("c2")
    nw, track, steps = conf.W, [0, 100, 255], 20
    sid = case.gpu(ctx, nw)
    p = case.oracle(conf.tau)
    wks = [O.init_walker(p) for _ in track]
    worst = {"eloc": 0.0, "phi": 0.0, "weight": 0.0}
    for s in range(steps):
        x = W.fields(0, 0, s, nw, case.G)
        ctx.propagate_batch(sid, tau=conf.tau, n_steps=1, exp_order=conf.k,
                            reorth_every=conf.reorth_every, step0=s, fields=C.to_dev(x),
                            e0=p.e0, precision=prec)
        torch.cuda.synchronize()
        st = ctx.get_walkers(sid)
        el = ctx.local_energy_batch(sid, precision=prec)
        for t, w in enumerate(track):
            wks[t], info = O.walker_step(p, wks[t], x[w], O.EXP_KRYLOV, conf.k,
                                         O.reorth_due(s, conf.reorth_every))
            worst["eloc"] = max(worst["eloc"], abs(el[w] - info.e_loc))
            worst["phi"] = max(worst["phi"], C.rel(st["phi"][w], wks[t].phi))
            worst["weight"] = max(worst["weight"], abs(st["weight"][w] - wks[t].weight)
                                  / max(1.0, wks[t].weight))
    print(prec_name, "c2 20 steps:", worst, flush=True)
    assert worst["eloc"] < E_TOL
