"""Implicit-solvent Coulomb (U = k_C q_i q_j / r^2, the paper's direct sum with a permittivity
growing with r) on the GPU against the oracle: forward parity with and without Lennard-Jones,
on a ball and on a bonded globule, and the adjoint's gradients with charges."""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lj", [True, False])
def test_charged_ball_parity(O, lj):
    """Mixed charges with Lennard-Jones; like charges without it (opposite charges with no
    short-range repulsion collapse onto each other, a singular and chaotic case)."""
    from workloads import seeded_charges, small_workload
    q = seeded_charges(300, 4) if lj else np.full(300, 0.5, np.float32)
    w = small_workload((24, 22, 20), 300, seed=4, tau=0.8, gamma=0.1, k_tether=0.05, mass=8.0,
                       lj=lj, coul_k=0.02, charges=q)
    steps = 20
    r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
    say("charged ball (LJ %s), %d steps:" % (lj, steps), r)
    assert max(r.values()) < 1e-5, r


def test_charged_globule_parity(O):
    from workloads import globule_workload, seeded_charges
    w = globule_workload(28, 1, 800, seed=6, tau=0.7, gamma=0.2, coul_k=0.02,
                         charges=seeded_charges(800, 6))
    steps = 10
    r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
    say("charged globule, %d steps:" % steps, r)
    assert max(r.values()) < 1e-5, r


def test_adjoint_with_charges(O):
    from test_gpu_adjoint import _check, _dfields, _gpu_grads, _oracle_grads
    from workloads import globule_workload, seeded_charges
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, coul_k=0.02,
                         charges=seeded_charges(60, 21))
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 12, 5)
    _check(outs, _oracle_grads(O, w, field, D, 12, dfields), dfields, 1e-3)
