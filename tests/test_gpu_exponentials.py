"""GPU parity of the Chebyshev exponential (Sec. IV.B, Eq. chebpoly)
against the oracle's `chebyshev`, and of its BF16-split form against the
FP64 kernel, through the C ABI."""
import numpy as np
import pytest

import afq_workloads as W
import gpu_common as C
from oracle import afq_oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    C.require_gpu()
    from paper_2403_02542_amd import afq
    c = afq.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("prop", [O.PROP_SPLIT2, O.PROP_TAYLOR])
def test_chebyshev_c1_all_walkers(ctx, prop):
    """c1 in full (16 walkers, 20 steps), Chebyshev order 8, with Split-2
    and with the refactorised propagator."""
    cfg = W.CONFIGS["c1"]
    case = C.Case.from_config("c1")
    worst, flagged, _ = C.run_pair(case, ctx, tau=cfg.tau, k=8, method=O.EXP_CHEBYSHEV,
                                   reorth=cfg.reorth_every, n_steps=cfg.steps, n_walkers=cfg.W,
                                   track=list(range(cfg.W)), prop=prop)
    print("c1 Chebyshev", prop, worst, "flagged", sorted(flagged))
    assert len(flagged) <= 2
    for key, v in worst.items():
        assert v < C.RTOL, (key, v)


def test_chebyshev_c2_subset_odd_order(ctx):
    """c2 (256 walkers), order 7 (an odd number of recurrence swaps), 3
    walkers tracked over 12 steps."""
    cfg = W.CONFIGS["c2"]
    case = C.Case.from_config("c2")
    worst, flagged, _ = C.run_pair(case, ctx, tau=cfg.tau, k=7, method=O.EXP_CHEBYSHEV,
                                   reorth=cfg.reorth_every, n_steps=12, n_walkers=cfg.W,
                                   track=[1, 99, 254])
    print("c2 Chebyshev", worst, "flagged", sorted(flagged))
    for key, v in worst.items():
        assert v < C.RTOL, (key, v)


@pytest.mark.parametrize("k", [1, 2, 9])
def test_chebyshev_mixed_step(k):
    """One MIXED step (BF16-split operator-orbital products, three pieces)
    with the Chebyshev exponential against one FP64 step from the same
    walkers on the same fields: orbitals within 1e-6 relative (orders 1 and
    2 exercise the first two terms alone)."""
    import torch
    from paper_2403_02542_amd import afq
    C.require_gpu()
    conf = W.CONFIGS["c2"]
    case = C.Case.from_config("c2")
    nw = 32
    res = {}
    for prec in (afq.PREC_FP64, afq.PREC_MIXED):
        c = afq.Context(0)
        sid = case.gpu(c, nw)
        x = C.to_dev(W.fields(0, 0, 0, nw, case.G))
        c.propagate_batch(sid, tau=conf.tau, n_steps=1, exp_method=afq.EXP_CHEBYSHEV,
                          exp_order=k, reorth_every=1, step0=0, fields=x, precision=prec)
        torch.cuda.synchronize()
        res[prec] = c.get_walkers(sid)
        c.close()
    err = max(C.rel(res[afq.PREC_MIXED]["phi"][w], res[afq.PREC_FP64]["phi"][w])
              for w in range(nw))
    print(f"Chebyshev order {k}: MIXED orbitals max rel. {err:.2e}")
    assert err < 1e-6
