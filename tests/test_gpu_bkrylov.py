"""GPU parity of the block-Krylov exponential (Sec. IV.D, Eq. bkrylov): the
walker step with AFQ_EXP_BLOCK_KRYLOV against the FP64 oracle's
`block_krylov`, on the same seeded inputs and fields, through the C ABI."""
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


def _check(worst):
    for key, v in worst.items():
        assert v < C.RTOL, (key, v)


def test_block_krylov_c1_all_walkers(ctx):
    """c1 in full (16 walkers x 20 steps, QR every step), block order 4
    (kN = 20 <= M = 24)."""
    cfg = W.CONFIGS["c1"]
    case = C.Case.from_config("c1")
    worst, flagged, _ = C.run_pair(case, ctx, tau=cfg.tau, k=4, method=O.EXP_BLOCK_KRYLOV,
                                   reorth=cfg.reorth_every, n_steps=cfg.steps, n_walkers=cfg.W,
                                   track=list(range(cfg.W)))
    print("c1 block Krylov", worst, "flagged", sorted(flagged))
    assert len(flagged) <= 2
    _check(worst)


def test_block_krylov_full_space_ragged(ctx):
    """kN = M (45 = 5 x 9): the block space is the whole orbital space and the
    step applies exp(A) exactly; QR every 3 steps, tau = 0.1, 10 walkers."""
    case = C.Case.random(45, 9, 70, seed=5, sigma_A=0.2 / np.sqrt(45))
    worst, flagged, _ = C.run_pair(case, ctx, tau=0.1, k=5, method=O.EXP_BLOCK_KRYLOV, reorth=3,
                                   n_steps=12, n_walkers=10, track=list(range(10)))
    print("full space", worst, "flagged", sorted(flagged))
    _check(worst)


def test_block_krylov_c2_subset(ctx):
    """c2 (256 walkers), block order 3, 4 walkers tracked over 20 steps."""
    cfg = W.CONFIGS["c2"]
    case = C.Case.from_config("c2")
    worst, flagged, _ = C.run_pair(case, ctx, tau=cfg.tau, k=3, method=O.EXP_BLOCK_KRYLOV,
                                   reorth=cfg.reorth_every, n_steps=20, n_walkers=cfg.W,
                                   track=[0, 77, 200, 255])
    print("c2 block Krylov", worst, "flagged", sorted(flagged))
    _check(worst)


def test_block_krylov_c3_single_steps(ctx):
    """Production shape (512 walkers, M = 300, N = 50), block order 5, the
    oracle restarted from the GPU state every step (QR steps included)."""
    cfg = W.CONFIGS["c3"]
    case = C.Case.from_config("c3")
    worst, flagged, _ = C.run_pair(case, ctx, tau=cfg.tau, k=5, method=O.EXP_BLOCK_KRYLOV,
                                   reorth=cfg.reorth_every, n_steps=5, n_walkers=cfg.W,
                                   track=[3, 400], resync=True)
    print("c3 block Krylov single step", worst, "flagged", sorted(flagged))
    _check(worst)


def test_block_krylov_independent_of_qr_schedule(ctx):
    """bkrylov{A, Psi S} = bkrylov{A, Psi} S for any invertible S, so the
    weights, overlaps and local energies do not depend on how often the
    walkers are reorthonormalised (unlike the per-orbital Krylov)."""
    import torch
    cfg = W.CONFIGS["c2"]
    case = C.Case.from_config("c2")
    p = case.oracle(cfg.tau)
    nw, steps = 64, 8
    out = []
    for every in (1, 4):
        sid = case.gpu(ctx, nw)
        for s in range(steps):
            ctx.propagate_batch(sid, tau=cfg.tau, n_steps=1, exp_method=O.EXP_BLOCK_KRYLOV,
                                exp_order=4, reorth_every=every, step0=s,
                                fields=C.to_dev(W.fields(0, 0, s, nw, case.G)), e0=p.e0)
        torch.cuda.synchronize()
        st = ctx.get_walkers(sid)
        out.append((st, ctx.local_energy_batch(sid)))
    (a, ea), (b, eb) = out
    assert np.array_equal(a["alive"], b["alive"])
    assert a["alive"].sum() > nw // 2
    live = a["alive"].astype(bool)
    assert C.rel(a["weight"][live], b["weight"][live]) < 1e-9
    assert np.abs(a["log_ovlp"][live].real - b["log_ovlp"][live].real).max() < 1e-8
    assert np.abs(C.wrap(a["log_ovlp"][live].imag - b["log_ovlp"][live].imag)).max() < 1e-8
    assert C.rel(ea[live], eb[live]) < 1e-9
    # the orbitals differ by a right factor only: same column span
    for w in np.flatnonzero(live)[:8]:
        qa, _ = np.linalg.qr(a["phi"][w])
        qb, _ = np.linalg.qr(b["phi"][w])
        assert np.linalg.norm(qa @ (qa.conj().T @ qb) - qb) < 1e-9


def test_block_krylov_arguments(ctx):
    """k N > M is refused; so is the graph schedule (the small exponential
    reads its substep count on the host)."""
    from paper_2403_02542_amd import afq
    cfg = W.CONFIGS["c1"]
    case = C.Case.from_config("c1")
    sid = case.gpu(ctx, 4)
    with pytest.raises(afq.AfqError) as e:
        ctx.propagate_batch(sid, tau=cfg.tau, n_steps=1, exp_method=O.EXP_BLOCK_KRYLOV,
                            exp_order=5)
    assert e.value.code == afq.EINVAL
    with pytest.raises(afq.AfqError) as e:
        ctx.propagate_batch([sid], tau=cfg.tau, n_steps=1, exp_method=O.EXP_BLOCK_KRYLOV,
                            exp_order=4, schedule=afq.SCHED_GRAPH)
    assert e.value.code == afq.EINVAL
    ctx.propagate_batch(sid, tau=cfg.tau, n_steps=2, exp_method=O.EXP_BLOCK_KRYLOV, exp_order=4)
