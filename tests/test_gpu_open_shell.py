"""GPU parity of open-shell walkers (spin-orbital determinants, spin factor
1 in Eqs. eloc, hyben and force_shift) against the oracle, through the
C ABI: an N_alpha = 5, N_beta = 3 system propagated step by step (set up
from spatial orbitals by afq_init_trial as well), the
spin-orbital embedding of a closed-shell system against the closed-shell
path, the BF16-split local energy on spin orbitals, and the many-system
graph schedule with a closed-shell and an open-shell system together."""
import numpy as np
import pytest
import scipy.linalg

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


def _open_shell(M=24, na=5, nb=3, G=60, seed=21):
    """A spatial system of the production recipe (couplings scaled by
    1/sqrt(M)) with an ROHF-like trial: the N_alpha lowest orbitals of the
    mean-field iteration for alpha, the first N_beta of them for beta."""
    ham = W.hamiltonian(M, G, 0.1, 0.3 / np.sqrt(M), seed, 0.0)
    pa = W.rhf_trial(ham.h, ham.L, na, n_iter=3)
    h2, L2, psi2 = W.spin_orbital_system(ham.h, ham.L, pa, pa[:, :nb])
    return C.Case(h2, L2, psi2, ham.e_core, spin=1)


@pytest.mark.parametrize("prop,method,k", [(O.PROP_SPLIT2, O.EXP_KRYLOV, 6),
                                           (O.PROP_SPLIT2, O.EXP_BLOCK_KRYLOV, 4),
                                           (O.PROP_SPLIT1, O.EXP_CHEBYSHEV, 10)])
def test_open_shell_parity(ctx, prop, method, k):
    """M = 2 x 24 spin orbitals, N = 5 + 3, G = 60: 32 walkers, 4 tracked
    over 12 steps, QR every 3 steps, against the oracle with spin = 1."""
    case = _open_shell()
    worst, flagged, _ = C.run_pair(case, ctx, tau=0.05, k=k, method=method, reorth=3,
                                   n_steps=12, n_walkers=32, track=[0, 7, 19, 31], prop=prop)
    print("open shell", prop, method, worst, "flagged", sorted(flagged))
    assert len(flagged) <= 1
    for key, v in worst.items():
        assert v < C.RTOL, (key, v)


def test_fully_polarised_parity(ctx):
    """N_alpha = 4, N_beta = 0 (every electron of one spin) set up from the
    spatial orbitals through afq_init_trial: 16 walkers, all tracked over 8
    steps against the oracle in spin orbitals."""
    M, G, na = 20, 40, 4
    ham = W.hamiltonian(M, G, 0.1, 0.3 / np.sqrt(M), 17, 0.0)
    pa = W.rhf_trial(ham.h, ham.L, na, n_iter=3)
    h2, L2, psi2 = W.spin_orbital_system(ham.h, ham.L, pa, pa[:, :0])
    case = C.Case(h2, L2, psi2, ham.e_core, spin=1)
    nw = 16
    sid = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
    ctx.init_trial(sid, pa, n_beta=0)
    ctx.init_walkers(sid, nw)
    p = case.oracle(0.05)
    assert ctx.get_e0(sid) == pytest.approx(p.e0, rel=1e-12)
    wks = [O.init_walker(p) for _ in range(nw)]
    import torch
    for s in range(8):
        x = W.fields(0, 0, s, nw, G)
        ctx.propagate_batch(sid, tau=0.05, n_steps=1, exp_order=6, reorth_every=2, step0=s,
                            fields=C.to_dev(x), e0=p.e0)
        torch.cuda.synchronize()
        st = ctx.get_walkers(sid)
        for w in range(nw):
            wks[w], info = O.walker_step(p, wks[w], x[w], O.EXP_KRYLOV, 6, O.reorth_due(s, 2))
            assert C.rel(st["phi"][w], wks[w].phi) < C.RTOL, (s, w)
            assert abs(st["weight"][w] - wks[w].weight) <= C.RTOL * max(1.0, wks[w].weight), (s, w)


def test_closed_shell_embedding_matches_closed_shell(ctx):
    """c1 written in spin orbitals (Psi_a = Psi_b) and run with spin factor 1
    follows the closed-shell run on the same fields: equal weights, E_L and
    E0, log-overlap doubled, walker diag(Phi, Phi)."""
    import torch
    case = C.Case.from_config("c1")
    h2, L2, psi2 = W.spin_orbital_system(case.h, case.L, case.psi, case.psi)
    emb = C.Case(h2, L2, psi2, case.e_core, spin=1)
    nw, tau = 16, 0.01
    sa, sb = case.gpu(ctx, nw), emb.gpu(ctx, nw)
    assert ctx.get_e0(sb) == pytest.approx(ctx.get_e0(sa), rel=1e-12)
    for s in range(10):
        x = C.to_dev(W.fields(0, 0, s, nw, case.G))
        for sid in (sa, sb):
            ctx.propagate_batch(sid, tau=tau, n_steps=1, exp_order=6, reorth_every=2, step0=s,
                                fields=x)
        torch.cuda.synchronize()
        a, b = ctx.get_walkers(sa), ctx.get_walkers(sb)
        ea, eb = ctx.local_energy_batch(sa), ctx.local_energy_batch(sb)
        assert C.rel(b["weight"], a["weight"]) < 1e-10, s
        assert C.rel(eb, ea) < 1e-10, s
        assert np.abs(b["log_ovlp"].real - 2 * a["log_ovlp"].real).max() < 1e-9, s
        for w in range(nw):
            want = scipy.linalg.block_diag(a["phi"][w], a["phi"][w])
            assert C.rel(b["phi"][w], want) < 1e-10, (s, w)
        print(f"  step {s + 1}/10: weights, E_L, log-overlaps and walkers agree", flush=True)


def _c2_open_shell(n_beta=18):
    """c2's Hamiltonian (M = 120, G = 600) in spin orbitals with its 20
    trial orbitals for alpha and the first n_beta of them for beta."""
    case = C.Case.from_config("c2")
    h2, L2, psi2 = W.spin_orbital_system(case.h, case.L, case.psi, case.psi[:, :n_beta])
    return C.Case(h2, L2, psi2, case.e_core, spin=1)


def test_open_shell_mixed_local_energy(ctx):
    """The BF16-split exchange with spin factor 1 and the FP64 Coulomb
    vector over the virtual space, on c2 in spin orbitals (M = 240,
    N = 20 + 18): after 6 FP64 steps, E_L with three pieces within 1e-4 Ha
    of the FP64 E_L for every walker (as for closed-shell c2), closer than
    with two pieces, and both FP64 and mixed E_L against the oracle."""
    import torch
    from paper_2403_02542_amd import afq
    conf = W.CONFIGS["c2"]
    case = _c2_open_shell()
    nw = 32
    sid = case.gpu(ctx, nw)
    ctx.propagate_batch(sid, tau=conf.tau, n_steps=6, exp_order=conf.k,
                        reorth_every=conf.reorth_every, seed=1)
    torch.cuda.synchronize()
    e64 = ctx.local_energy_batch(sid)
    errs = {}
    for prec in (afq.PREC_MIXED, afq.PREC_MIXED_FAST):
        errs[prec] = np.abs(ctx.local_energy_batch(sid, precision=prec) - e64).max()
    emx = ctx.local_energy_batch(sid, precision=afq.PREC_MIXED)
    print("open-shell c2 max |E_L(mixed) - E_L(fp64)|: 3 pieces %.3e, 2 pieces %.3e"
          % (errs[afq.PREC_MIXED], errs[afq.PREC_MIXED_FAST]), flush=True)
    st = ctx.get_walkers(sid)
    p = case.oracle(conf.tau)
    for w in (0, nw - 1):
        _, th = O.overlap(case.psi, st["phi"][w])
        e = O.local_energy(p, st["phi"][w], th)
        assert abs(e64[w] - e) / max(1.0, abs(e)) < C.RTOL, w
        assert abs(emx[w] - e) < 1e-4, w
    assert errs[afq.PREC_MIXED] < 1e-4
    assert errs[afq.PREC_MIXED] < errs[afq.PREC_MIXED_FAST]


def test_open_and_closed_shell_in_one_graph_batch():
    """A closed-shell and an open-shell system in one graph-schedule call
    equal each propagated alone, bitwise (the spin factor travels with each
    system through the many-system launches)."""
    import torch
    from paper_2403_02542_amd import afq
    C.require_gpu()
    cases = [C.Case.random(20, 4, 40, seed=5), _open_shell(M=16, na=4, nb=2, G=40, seed=9)]
    res = []
    for sched, alone in ((afq.SCHED_SERIAL, True), (afq.SCHED_GRAPH, False)):
        c = afq.Context(0)
        ids = [cs.gpu(c, 8) for cs in cases]
        kw = dict(tau=0.05, n_steps=4, exp_order=6, reorth_every=2, seed=1, schedule=sched)
        if alone:
            for s in ids:
                c.propagate_batch(s, **kw)
        else:
            c.propagate_batch(ids, **kw)
        c.sync()
        torch.cuda.synchronize()
        res.append([c.get_walkers(s) for s in ids])
        c.close()
    for a, b in zip(res[0], res[1]):
        for key in ("phi", "weight", "log_ovlp"):
            assert np.array_equal(a[key], b[key]), key


def test_open_shell_trial_from_spatial_orbitals(ctx):
    """afq_init_trial with N_alpha = 5 != N_beta = 3 and Psi_T = [Psi_a, Psi_b]
    over the 24 spatial orbitals rewrites the system in spin orbitals on the
    device: the run equals, bitwise, the same system embedded on the host and
    set up with afq_init_trial_spin_orbital, on the same fields."""
    import torch
    M, G, na, nb = 24, 60, 5, 3
    ham = W.hamiltonian(M, G, 0.1, 0.3 / np.sqrt(M), 21, 0.0)
    pa = W.rhf_trial(ham.h, ham.L, na, n_iter=3)
    pb = pa[:, :nb]
    h2, L2, psi2 = W.spin_orbital_system(ham.h, ham.L, pa, pb)
    nw = 16
    sa = ctx.init_hamiltonian(ham.h, ham.L, ham.e_core)
    ctx.init_trial(sa, np.hstack([pa, pb]), n_beta=nb)
    ctx.init_walkers(sa, nw)
    sb = ctx.init_hamiltonian(h2, L2, ham.e_core)
    ctx.init_trial_spin_orbital(sb, psi2)
    ctx.init_walkers(sb, nw)
    assert ctx.get_e0(sa) == ctx.get_e0(sb)
    for s in range(6):
        x = C.to_dev(W.fields(0, 0, s, nw, G))
        for sid in (sa, sb):
            ctx.propagate_batch(sid, tau=0.05, n_steps=1, exp_order=6, reorth_every=2, step0=s,
                                fields=x)
        torch.cuda.synchronize()
        a, b = ctx.get_walkers(sa), ctx.get_walkers(sb)
        assert a["phi"].shape == (nw, 2 * M, na + nb)
        for key in ("phi", "weight", "log_ovlp"):
            assert np.array_equal(a[key], b[key]), (s, key)
        assert np.array_equal(ctx.local_energy_batch(sa), ctx.local_energy_batch(sb)), s


def test_open_shell_arguments(ctx):
    from paper_2403_02542_amd import afq
    case = C.Case.from_config("c1")
    sid = ctx.init_hamiltonian(case.h, case.L, case.e_core)
    # equal counts with separate orbitals are the spin-orbital entry point's
    with pytest.raises(ValueError):
        ctx.init_trial(sid, np.hstack([case.psi, case.psi]), n_beta=case.N)
    # the beta columns must be orthonormal among themselves
    bad = np.hstack([case.psi, 2.0 * case.psi[:, :2]])
    with pytest.raises(afq.AfqError) as e:
        ctx.init_trial(sid, bad, n_beta=2)
    assert e.value.code == afq.EINVAL
    ctx.init_trial_spin_orbital(sid, case.psi)
    with pytest.raises(afq.AfqError) as e:
        ctx.init_trial_spin_orbital(sid, case.psi)
    assert e.value.code == afq.ESTATE
    ctx.init_walkers(sid, 4)
    with pytest.raises(afq.AfqError) as e:
        ctx.local_energy_adjoint(sid, np.ones(4), np.zeros((case.M, case.M)),
                                 np.zeros((case.G, case.M, case.M)))
    assert e.value.code == afq.EINVAL
    # 2M above the kernels' 512
    M = 300
    big = ctx.init_hamiltonian(np.diag(np.linspace(-2.0, 0.0, M)), np.zeros((1, M, M)), 0.0)
    psi = np.eye(M)[:, :3]
    with pytest.raises(afq.AfqError) as e:
        ctx.init_trial(big, psi, n_beta=1)
    assert e.value.code == afq.EINVAL
