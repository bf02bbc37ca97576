"""Input generators: determinism, structure and the field generator's
definition (Philox4x64-10 of Salmon et al., SC'11, with Box-Muller)."""
import math

import numpy as np
import pytest

import afq_workloads as W

M64 = (1 << 64) - 1


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds, written out from its published definition."""
    m0, m1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
    w0, w1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
    c0, c1, c2, c3 = ctr
    k0, k1 = key
    for r in range(10):
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> 64, p0 & M64
        hi1, lo1 = p1 >> 64, p1 & M64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0, k1 = (k0 + w0) & M64, (k1 + w1) & M64
    return c0, c1, c2, c3


def test_philox_known_answers():
    """Known-answer vectors of the Random123 distribution (kat_vectors)."""
    assert philox4x64_10((0, 0, 0, 0), (0, 0)) == (
        0x16554d9eca36314c, 0xdb20fe9d672d0fdc, 0xd7e772cee186176b, 0x7e68b68aec7ba23b)
    assert philox4x64_10((M64,) * 4, (M64, M64)) == (
        0x87b092c3013fe90b, 0x438c3c67be8d0224, 0x9cc7d7c69cd777b6, 0xa09caebf594f0ba0)


def test_numpy_philox_counter_convention():
    """numpy's Philox(counter=c) emits the block of counter c + 1."""
    for c in (0, 7, 123456789):
        bg = np.random.Philox(key=np.array([3, 5], dtype=np.uint64), counter=c)
        got = tuple(int(v) for v in bg.random_raw(4))
        assert got == philox4x64_10((c + 1, 0, 0, 0), (3, 5))


def test_fields_follow_definition():
    seed, sid, step, nw, ng = 0, 2, 3, 5, 10
    x = W.fields(seed, sid, step, nw, ng)
    nb = (ng + 3) // 4
    for w in range(nw):
        for b in range(nb):
            blk = philox4x64_10(((step * nw + w) * nb + b + 1, 0, 0, 0), (seed, sid))
            u = [((v >> 11) + 1) * 2.0 ** -53 for v in blk]
            z = [math.sqrt(-2 * math.log(u[0])) * math.cos(2 * math.pi * u[1]),
                 math.sqrt(-2 * math.log(u[0])) * math.sin(2 * math.pi * u[1]),
                 math.sqrt(-2 * math.log(u[2])) * math.cos(2 * math.pi * u[3]),
                 math.sqrt(-2 * math.log(u[2])) * math.sin(2 * math.pi * u[3])]
            for j in range(4):
                g = 4 * b + j
                if g < ng:
                    assert x[w, g] == pytest.approx(z[j], rel=1e-15, abs=1e-15)


def test_fields_statistics():
    x = W.fields(0, 0, 0, 2000, 50)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1.0) < 0.01


def test_hamiltonian_structure_and_determinism():
    cfg = W.CONFIGS["c1"]
    a = W.hamiltonian(cfg.M, cfg.G, cfg.sigma_h, cfg.sigma_A, 0)
    b = W.hamiltonian(cfg.M, cfg.G, cfg.sigma_h, cfg.sigma_A, 0)
    assert np.array_equal(a.h, b.h) and np.array_equal(a.L, b.L)
    assert np.array_equal(a.h, a.h.T)
    assert np.array_equal(a.L, a.L.transpose(0, 2, 1))
    d = np.diag(a.h)
    assert d.min() >= -2.0 and d.max() <= 0.0
    off = a.h[np.triu_indices(cfg.M, 1)]
    assert abs(off.std() - 0.1) < 0.02


def test_trial_is_orthonormal_mean_field():
    cfg = W.CONFIGS["c1"]
    ham, psi = W.make_system(cfg)
    assert psi.shape == (cfg.M, cfg.N)
    assert np.abs(psi.T @ psi - np.eye(cfg.N)).max() < 1e-12
    _, psi2 = W.make_system(cfg)
    assert np.array_equal(psi, psi2)
    # without interaction the trial is the lowest eigenvectors of h
    psi0 = W.rhf_trial(ham.h, np.zeros((1, cfg.M, cfg.M)), cfg.N)
    v = np.linalg.eigh(ham.h)[1][:, :cfg.N]
    assert np.abs(psi0 @ psi0.T - v @ v.T).max() < 1e-12


def test_uneven_batch_sizes():
    sizes = W.uneven_batch_sizes()
    assert len(sizes) == 48
    assert all(40 <= M <= 400 and N == M // 6 and G == 5 * M for M, N, G in sizes)


def test_comb_uniform_follows_definition():
    """Population-control uniforms: word 0 of the Philox block of counter
    step + 1 under the key (seed, sys_id + 2^32), u = (x >> 11) 2^-53."""
    for seed, sid, step in ((0, 0, 0), (0, 0, 1), (3, 2, 7), (5, 47, 123456)):
        blk = philox4x64_10((step + 1, 0, 0, 0), (seed, sid + (1 << 32)))
        u = (blk[0] >> 11) * 2.0 ** -53
        assert W.comb_uniform(seed, sid, step) == u
        assert 0.0 <= u < 1.0
