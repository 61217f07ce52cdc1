"""The oracle's two ways of evaluating the same step agree bit for bit.

* ``or_step_sampled`` evaluates one coupled step (Section 2.2: collision and streaming of
  Eq. 1, the friction coupling and the atom update) only at requested sites and atoms: the
  collision at the Q upstream nodes of each site, the force field for each atom alone.  It is
  the reference of every full-size GPU test, where ``or_run`` over the whole lattice is too
  slow.  Here it is evaluated at every site and atom and must equal ``or_run`` for one step,
  value for value, for every option the step has (both velocity sets, both collisions,
  thermal noise, the Coulomb term, every body-force kind, tethers, bonds and exclusions).
* The coupled step sums the force field atom by atom over cell-list candidates; ``or_forces``
  is the pairwise all-pairs loop that defines it.  They must give the same bits: the
  candidates hold every partner closer than the cut-off, in the order the all-pairs loop adds
  them.
"""
import numpy as np
import pytest

from workloads import globule_workload, seeded_charges, small_workload


def _random_state(O, p, rng, amp=2e-3):
    """A pre-collision state away from equilibrium: the equilibrium of a random velocity field
    plus random non-equilibrium parts."""
    c, w = O.velocity_set(O.n_velocities(p))
    shape = O.pop_shape(p)
    u = rng.normal(0.0, amp, size=(3,) + shape[1:])
    drho = rng.normal(0.0, amp, size=shape[1:])
    cu = np.einsum("qa,a...->q...", c.astype(float), u)
    uu = (u * u).sum(0)
    rho = 1.0 + drho
    g = w[:, None, None, None] * (drho + rho * (3 * cu + 4.5 * cu * cu - 1.5 * uu))
    return g + rng.normal(0.0, 0.2 * amp, size=shape) * w[:, None, None, None]


def _case(kind, q, trt, kT, coul, bf):
    rng = np.random.default_rng([q, int(trt), int(kT), int(coul), bf, kind == "ball"])
    L = (13, 11, 12)
    if kind == "ball":
        w = small_workload(L, 60, seed=5, tau=0.7, gamma=0.3, k_tether=0.05, mass=4.0)
    else:
        w = globule_workload(L, 1, 90, seed=8, tau=0.62, gamma=0.2, mass=4.0)
    w.velocity_set = q
    w.trt_magic = 0.1875 if trt else 0.0
    w.kT, w.noise_seed = (1e-4, 77) if kT else (0.0, 0)
    if coul:
        w.coul_k = 0.02
        w.charges = seeded_charges(w.n_atoms, 3)
    w.bf_kind = bf
    w.bf_amp = 3e-5 if bf in (1, 2) else 0.0
    if bf == 3:
        w.body_force = rng.normal(0.0, 1e-4, size=(3, L[2], L[1], L[0])).astype(np.float32)
    # velocities large enough that the friction and the spread force matter
    w.v0 = (w.v0 * 3).astype(np.float32)
    return w, rng


CASES = [
    ("ball", 19, False, False, False, 0),
    ("ball", 19, True, True, True, 1),
    ("ball", 27, False, True, False, 2),
    ("ball", 27, True, False, True, 3),
    ("globule", 19, False, False, False, 1),
    ("globule", 19, True, True, False, 3),
    ("globule", 27, False, True, True, 0),
    ("globule", 27, True, False, False, 2),
]


@pytest.mark.parametrize("kind,q,trt,kT,coul,bf", CASES)
def test_sampled_step_equals_full_step_bitwise(O, kind, q, trt, kT, coul, bf):
    w, rng = _case(kind, q, trt, kT, coul, bf)
    p = O.params_from_workload(w)
    p.step0 = 5                 # the noise is counted by the step
    g0 = _random_state(O, p, rng)
    field = w.body_force
    g1, X1, V1 = O.run(p, g0, w.x0, w.v0, w.x0, w.bonds, field, 1)
    S = O.n_sites(p)
    gs, Xs, Vs = O.step_sampled(p, g0, w.x0, w.v0, w.x0, w.bonds, field, np.arange(S),
                                np.arange(w.n_atoms))
    Q = O.n_velocities(p)
    assert np.array_equal(gs.T.reshape(Q, -1), g1.reshape(Q, -1))
    assert np.array_equal(Xs, X1) and np.array_equal(Vs, V1)
    # and the step did something: the populations and velocities changed
    assert not np.array_equal(g1, g0) and not np.array_equal(V1, w.v0)


@pytest.mark.parametrize("kind,coul,shift", [("ball", False, 0), ("ball", True, 3),
                                             ("globule", False, -2), ("globule", True, 1)])
def test_force_field_by_atom_equals_pairwise_bitwise(O, kind, coul, shift):
    """Per-atom sums over cell-list candidates against the pairwise all-pairs loop, with atoms
    unwrapped several boxes away and moved onto cell boundaries and the periodic seam."""
    L = (16, 15, 17)
    if kind == "ball":
        w = small_workload(L, 300, seed=11, tau=0.8)
    else:
        w = globule_workload(L, 1, 400, seed=12)
    if coul:
        w.coul_k = 0.05
        w.charges = seeded_charges(w.n_atoms, 4)
    p = O.params_from_workload(w)
    X = w.x0.astype(np.float64) + np.array(L) * shift
    # a few atoms exactly on a cell boundary (cells are 16 / 6 wide along x) and on the seam
    nc = np.floor(np.array(L) / (2.5 * 1.001))
    X[0, 0] = L[0] / nc[0] * 2
    X[1, 1] = 0.0
    X[2, 2] = L[2] * 1.0
    F_pair = O.forces(p, X, w.x0, w.bonds)
    F_atom = O.forces_by_atom(p, X, w.x0, w.bonds)
    assert np.array_equal(F_pair, F_atom)
    assert np.abs(F_pair).max() > 0


def test_force_field_by_atom_small_box_scans_all(O):
    """Fewer than three cells along an axis: the per-atom sum scans every atom."""
    w = small_workload((7, 12, 12), 40, seed=2, radius=2.5)
    p = O.params_from_workload(w)
    assert np.array_equal(O.forces(p, w.x0, w.x0, w.bonds), O.forces_by_atom(p, w.x0, w.x0, w.bonds))
