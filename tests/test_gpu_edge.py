"""Degenerate and boundary cases against the oracle: the smallest lattices (where a site's
upstream neighbours along an axis coincide), the smallest cell grid (3 cells per axis), a single
atom, atoms exactly on nodes and on the periodic seam, unwrapped positions far outside the box,
atoms without friction (gamma = 0), relaxation times near the stability limit tau = 1/2, and a
call of zero steps."""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


def _random_pops(O, w, seed, amp=1e-3):
    p = O.params_from_workload(w)
    return np.random.default_rng(seed).normal(0, amp, size=O.pop_shape(p)).astype(np.float32)


@pytest.mark.parametrize("L", [(2, 2, 2), (2, 3, 5), (3, 2, 4)])
def test_smallest_lattices(O, L):
    from workloads import small_workload
    w = small_workload(L, 0, seed=1, tau=0.7, steps=0, bf_kind=1, bf_amp=1e-4)
    g0 = _random_pops(O, w, 5)
    r = compare(gpu_run(w, 12, g0=g0), oracle_run(O, w, 12, g0=g0), w)
    say("lattice", L, r)
    assert max(r.values()) < 1e-5, r


def test_single_atom(O):
    from workloads import small_workload
    w = small_workload((5, 4, 3), 1, seed=2, tau=0.8, gamma=0.2, k_tether=0.05, lj=False, mass=1.0)
    g0 = _random_pops(O, w, 6)
    r = compare(gpu_run(w, 30, g0=g0), oracle_run(O, w, 30, g0=g0), w)
    say("single atom", r)
    assert max(r.values()) < 1e-5, r


def test_three_cells_per_axis_atoms_on_nodes_and_seam(O):
    """L = 8 with r_c = 2.5 gives exactly 3 cells per axis, so the 27 neighbour cells wrap onto
    each other's images.  Atoms sit exactly on nodes, on the seam (x = 0, x just below L) and
    at unwrapped positions several boxes away."""
    from workloads import small_workload
    w = small_workload((8, 8, 8), 0, seed=3, tau=0.8, gamma=0.1, k_tether=0.05, lj=True, mass=8.0)
    x = np.array([[0.0, 0.0, 0.0], [7.999, 4.0, 4.0], [3.0, 3.0, 3.0], [4.5, 5.5, 2.25],
                  [-37.25, 13.5, 6.0], [16.75, -8.5, 31.0], [1.2, 6.8, 7.9], [6.1, 1.3, 0.4]],
                 np.float32)
    rng = np.random.default_rng(4)
    w.x0 = x
    w.v0 = rng.normal(0, 0.01, size=x.shape).astype(np.float32)
    g0 = _random_pops(O, w, 7)
    r = compare(gpu_run(w, 25, g0=g0), oracle_run(O, w, 25, g0=g0), w)
    say("3 cells per axis, atoms on nodes / seam / far images", r)
    assert max(r.values()) < 1e-5, r


def test_zero_friction_leaves_the_fluid_untouched(O):
    """gamma = 0 (Section 2.2's coupling switched off): the atoms move under their own forces
    only, every spread force is an exact zero, and the populations equal, value for value, those
    of the same lattice without atoms; both runs match the oracle."""
    from workloads import globule_workload, small_workload
    L = (20, 18, 16)
    w = globule_workload(L, 1, 300, seed=12, tau=0.7, gamma=0.0, bf_kind=1, bf_amp=1e-5)
    fluid = small_workload(L, 0, seed=12, tau=0.7, steps=0, bf_kind=1, bf_amp=1e-5)
    g0 = _random_pops(O, w, 8)
    a = gpu_run(w, 20, g0=g0)
    b = gpu_run(fluid, 20, g0=g0)
    assert (a["g"] == b["g"]).all()
    r = compare(a, oracle_run(O, w, 20, g0=g0), w)
    say("gamma = 0, globule of 300", r)
    assert max(r.values()) < 1e-5, r


@pytest.mark.parametrize("tau", [0.505, 0.51])
def test_relaxation_time_near_one_half(O, tau):
    """Over-relaxation near the stability limit of Eq. (1) (omega = 1/tau close to 2): the
    non-equilibrium part changes sign every step and decays only by |1 - omega| per step.  A
    lattice from a random state with Kolmogorov forcing over 100 steps, then a tethered ball
    coupled to it over 30."""
    from workloads import small_workload
    w = small_workload((24, 20, 18), 0, seed=9, tau=tau, steps=0, bf_kind=1, bf_amp=1e-5)
    g0 = _random_pops(O, w, 9)
    r = compare(gpu_run(w, 100, g0=g0), oracle_run(O, w, 100, g0=g0), w)
    say("tau", tau, "lattice, 100 steps", r)
    assert max(r.values()) < 1e-5, r
    wb = small_workload((16, 14, 12), 40, seed=10, tau=tau, gamma=0.1, k_tether=0.05, lj=False, mass=8.0)
    g0 = _random_pops(O, wb, 10)
    r = compare(gpu_run(wb, 30, g0=g0), oracle_run(O, wb, 30, g0=g0), wb)
    say("tau", tau, "tethered ball, 30 steps", r)
    assert max(r.values()) < 1e-5, r


def test_zero_steps_is_a_no_op():
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import small_workload
    w = small_workload((10, 9, 8), 20, seed=5, tau=0.8, gamma=0.1, mass=8.0)
    sim = CoupledLB.from_workload(w)
    sim.step(3)
    g = sim.populations()
    _, _, x, v = sim.read_fields()
    sim.step(0)
    _, _, x2, v2 = sim.read_fields()
    assert bool((sim.populations() == g).all()) and bool((x == x2).all()) and bool((v == v2).all())
    assert sim.step_count == 3
    sim.close()
