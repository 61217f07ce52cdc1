"""The seeded input generators: determinism, sizes and the geometric guarantees they give
(minimum separation, unit bonds, confinement, globule spacing)."""
import numpy as np

from workloads import make_workload, globule_workload, small_workload, confined_saw


def test_config0_ball():
    w = make_workload(0)
    assert w.n_atoms == 500 and w.L == (32, 32, 32) and w.tau == 0.8 and w.steps == 100
    x = w.x0.astype(float)
    assert np.linalg.norm(x - 16.0, axis=1).max() <= 6.0 + 1e-5
    d = np.sqrt(((x[:, None] - x[None]) ** 2).sum(-1))
    np.fill_diagonal(d, 9.0)
    assert d.min() >= 1.0 - 1e-5
    assert abs(w.v0.std() - 0.01) < 0.001
    assert w.x0.dtype == np.float32 and w.v0.dtype == np.float32


def test_determinism():
    a, b = make_workload(3), make_workload(3)
    assert (a.x0 == b.x0).all() and (a.v0 == b.v0).all() and (a.bonds == b.bonds).all()
    assert (a.target_shift == b.target_shift).all()
    assert abs(np.linalg.norm(a.target_shift) - 1) < 1e-6
    assert a.body_force.shape == (3, 96, 96, 96) and not a.body_force.any()


def test_saw_is_self_avoiding_and_confined():
    rng = np.random.default_rng(0)
    p = confined_saw(3000, 11.0, rng)
    assert len({tuple(q) for q in p}) == 3000
    assert (np.abs(np.diff(p, axis=0)).sum(1) == 1).all()
    assert ((p ** 2).sum(1) <= 121).all()


def test_globules_separated():
    w = globule_workload(96, 3, 2000, seed=4)
    x = w.x0.astype(float).reshape(3, 2000, 3)
    L = 96.0
    c = x.mean(1)
    for i in range(3):
        for j in range(i + 1, 3):
            d = np.abs(c[i] - c[j]); d = np.minimum(d, L - d)
            assert np.linalg.norm(d) > 2 * 20 * (2000 / 20000) ** (1 / 3)
    b = w.bonds
    assert len(b) == 3 * 1999
    bl = np.linalg.norm(w.x0[b[:, 0]].astype(float) - w.x0[b[:, 1]].astype(float), axis=1)
    assert np.abs(bl - 1.0).max() < 1e-4


def test_small_workload_sizes():
    w = small_workload(16, 50, seed=1)
    assert w.n_atoms == 50 and w.n_sites == 16 ** 3
