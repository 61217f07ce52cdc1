"""Pins of the oracle's stand-in force field and atom integrator: Newton's third law, force =
-gradient of the energy (central differences), the Lennard-Jones landmarks far from the cut-off
(U(sigma) = 0, U(2^(1/6) sigma) = -eps with zero force), force and energy falling continuously
to zero at the cut-off and nothing beyond it, the harmonic bond at rest length, minimum image,
bonded exclusion, and the symplectic-Euler map of a tethered atom (closed form as a matrix
power)."""
import numpy as np
import pytest

E0 = np.zeros((0, 2), np.int32)


def _pair_params(O, **kw):
    d = dict(L=20, tau=0.8, lj_eps=0.01, lj_sigma=1.0, lj_rc=2.5, n_atoms=2)
    d.update(kw)
    return O.make_params(**d)


def test_lj_landmarks(O):
    """With the cut-off 100 sigma away (two atoms: the minimum image picks the one pair) the
    shift that makes the force vanish at r_c changes the energy by less than 1e-12 and the force
    by less than 1e-17: the plain Lennard-Jones landmarks U(sigma) = 0 and U(2^(1/6) sigma) =
    -eps with zero force."""
    pf = _pair_params(O, lj_rc=100.0)
    for r, U_want in ((1.0, 0.0), (2 ** (1 / 6), -0.01)):
        X = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        assert abs(O.energy(pf, X, X, E0) - U_want) < 1e-12
    X = np.array([[5.0, 5.0, 5.0], [5.0 + 2 ** (1 / 6), 5.0, 5.0]])
    assert np.abs(O.forces(pf, X, X, E0)).max() < 1e-16
    p = _pair_params(O)
    # repulsive inside the minimum, attractive beyond, zero past the cut-off
    X = np.array([[5.0, 5.0, 5.0], [6.0, 5.0, 5.0]])
    F = O.forces(p, X, X, E0)
    assert F[0, 0] < 0 < F[1, 0]
    X = np.array([[5.0, 5.0, 5.0], [6.5, 5.0, 5.0]])
    F = O.forces(p, X, X, E0)
    assert F[0, 0] > 0 > F[1, 0]
    X = np.array([[5.0, 5.0, 5.0], [7.5001, 5.0, 5.0]])
    assert np.abs(O.forces(p, X, X, E0)).max() == 0.0


@pytest.mark.parametrize("kind", ["lj", "coulomb"])
def test_pair_terms_vanish_continuously_at_cutoff(O, kind):
    """Just inside r_c = 2.5 the pair force falls to zero linearly and the energy quadratically
    in the distance d to r_c (so a pair whose distance rounds to either side of r_c changes
    the force by O(d), not by a finite jump); at and beyond r_c both are exactly zero."""
    if kind == "lj":
        p = _pair_params(O)
    else:
        p = O.make_params(20, 0.8, n_atoms=2, coul_k=0.3, charges=np.array([0.7, -0.4]), lj_rc=2.5)
    F1 = U1 = None
    for d in (1e-2, 1e-3, 1e-4):
        X = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0 + 2.5 - d]])
        F = np.abs(O.forces(p, X, X, E0)).max()
        U = O.energy(p, X, X, E0)
        assert F > 0
        if F1 is not None:
            # ten times closer: ten times less force, a hundred times less energy
            assert abs(F1 / F - 10.0) < 0.2 and abs(U1 / U - 100.0) < 2.0, (d, F1 / F, U1 / U)
        F1, U1 = F, U
    for r in (2.5, 2.50001, 3.0):
        X = np.array([[5.0, 5.0, 5.0], [5.0, 5.0, 5.0 + r]])
        assert np.abs(O.forces(p, X, X, E0)).max() == 0.0 and O.energy(p, X, X, E0) == 0.0


def test_minimum_image_and_bond_exclusion(O):
    p = _pair_params(O, L=10)
    X = np.array([[0.4, 5.0, 5.0], [9.6, 5.0, 5.0]])   # 0.8 apart through the seam
    Xn = np.array([[5.4, 5.0, 5.0], [4.6, 5.0, 5.0]])
    np.testing.assert_allclose(O.forces(p, X, X, E0), O.forces(p, Xn, Xn, E0), rtol=1e-12)
    b = np.array([[0, 1]], np.int32)
    pb = _pair_params(O, L=10, n_bonds=1, lj_exclude_bonded=1, k_bond=0.0)
    assert np.abs(O.forces(pb, X, X, b)).max() == 0.0
    pb2 = _pair_params(O, L=10, n_bonds=1, lj_exclude_bonded=0, k_bond=0.0)
    np.testing.assert_allclose(O.forces(pb2, X, X, b), O.forces(p, X, X, E0), rtol=1e-14)


def test_harmonic_bond_closed_form(O):
    b = np.array([[0, 1]], np.int32)
    p = O.make_params(20, 0.8, k_bond=0.5, r0_bond=1.0, n_atoms=2, n_bonds=1)
    X = np.array([[3.0, 3.0, 3.0], [4.0, 3.0, 3.0]])
    assert np.abs(O.forces(p, X, X, b)).max() == 0.0
    X = np.array([[3.0, 3.0, 3.0], [3.0, 4.3, 3.0]])
    F = O.forces(p, X, X, b)
    np.testing.assert_allclose(F[0], [0, 0.5 * 0.3, 0], atol=1e-15)   # pulled toward atom 1
    np.testing.assert_allclose(F[1], -F[0], atol=1e-15)
    assert abs(O.energy(p, X, X, b) - 0.5 * 0.5 * 0.09) < 1e-15


def test_tether_closed_form(O):
    p = O.make_params(20, 0.8, k_tether=0.05, n_atoms=1)
    X0 = np.array([[3.0, 4.0, 5.0]])
    X = X0 + np.array([[0.1, -0.2, 0.3]])
    np.testing.assert_allclose(O.forces(p, X, X0, E0), -0.05 * (X - X0), rtol=1e-14)
    assert abs(O.energy(p, X, X0, E0) - 0.5 * 0.05 * 0.14) < 1e-16


@pytest.fixture(scope="module")
def cluster():
    from workloads import globule_workload
    w = globule_workload(24, 1, 300, seed=11, tau=0.6)
    rng = np.random.default_rng(5)
    X = w.x0.astype(float) + rng.normal(0, 0.05, size=w.x0.shape)
    return w, X


def test_newton_third_law(O, cluster):
    w, X = cluster
    p = O.params_from_workload(w)
    F = O.forces(p, X, w.x0, w.bonds)
    assert np.abs(F).max() > 1e-3
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-14)


def test_force_is_minus_energy_gradient(O, cluster):
    w, X = cluster
    p = O.params_from_workload(w)
    p.k_tether = 0.05
    F = O.forces(p, X, w.x0, w.bonds)
    h = 1e-6
    rng = np.random.default_rng(0)
    for a in rng.choice(len(X), 12, replace=False):
        for c in range(3):
            Xp = X.copy(); Xp[a, c] += h
            Xm = X.copy(); Xm[a, c] -= h
            fd = -(O.energy(p, Xp, w.x0, w.bonds) - O.energy(p, Xm, w.x0, w.bonds)) / (2 * h)
            assert abs(fd - F[a, c]) < 1e-7 + 1e-6 * abs(F[a, c]), (a, c, fd, F[a, c])


def test_lj_pair_count_brute_force(O, cluster):
    """Summed over atoms, F . X relates to the virial; here we just check against an
    independent numpy evaluation of the pair sum at the same positions."""
    w, X = cluster
    p = O.params_from_workload(w)
    p.k_bond = 0.0
    L = np.array(w.L, float)
    bonded = {(int(i), int(j)) for i, j in w.bonds} | {(int(j), int(i)) for i, j in w.bonds}
    F = np.zeros_like(X)
    for i in range(len(X)):
        r = X[i] - X
        r -= L * np.floor(r / L + 0.5)
        r2 = (r * r).sum(1)
        for j in np.nonzero((r2 < 2.5 ** 2) & (np.arange(len(X)) != i))[0]:
            if (i, int(j)) in bonded:
                continue
            # the force of the plain term minus its value at r_c, scaled by r / r_c
            dU_dr = 4 * 0.01 * (-12 / r2[j] ** 6.5 + 6 / r2[j] ** 3.5)
            dU_dr_c = 4 * 0.01 * (-12 / 2.5 ** 13 + 6 / 2.5 ** 7)
            F[i] -= dU_dr * r[j] / np.sqrt(r2[j]) - dU_dr_c * r[j] / 2.5
    np.testing.assert_allclose(O.forces(p, X, w.x0, w.bonds), F, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("k,m", [(0.05, 8.0), (0.5, 1.0), (3.0, 1.0)])
def test_symplectic_euler_tethered_atom(O, k, m):
    """gamma = 0 decouples the atom; v' = v - (k/m) x, x' = x + v' is the linear map
    [[1 - k/m, 1], [-k/m, 1]] (det 1) whose n-th power gives the trajectory."""
    p = O.make_params(12, 0.8, gamma=0.0, mass=m, k_tether=k, n_atoms=1)
    X0 = np.array([[6.0, 6.0, 6.0]])
    x = np.array([[6.3, 5.8, 6.05]])
    v = np.array([[0.01, 0.02, -0.03]])
    M = np.array([[1 - k / m, 1.0], [-k / m, 1.0]])
    assert abs(np.linalg.det(M) - 1) < 1e-14
    n = 37
    _, Xn, Vn = O.run(p, np.zeros(O.pop_shape(p)), x, v, X0, E0, None, n)
    Mn = np.linalg.matrix_power(M, n)
    for c in range(3):
        want = Mn @ np.array([x[0, c] - X0[0, c], v[0, c]])
        assert abs(Xn[0, c] - X0[0, c] - want[0]) < 1e-12
        assert abs(Vn[0, c] - want[1]) < 1e-12


# ---- implicit-solvent Coulomb (permittivity proportional to r): U = k_C q_i q_j / r^2 ----------

def test_coulomb_implicit_pair_closed_form(O):
    """Two charges with the cut-off far away (1e6, where the shift is below 1e-9 of the
    energy and 1e-15 of the force): U = k q1 q2 / r^2 and F_1 = 2 k q1 q2 (X_1 - X_2) / r^4;
    off at r >= r_c."""
    q = np.array([0.7, -0.4])
    pf = O.make_params(20, 0.8, n_atoms=2, coul_k=0.3, charges=q, lj_rc=1.0e6)
    for r in (0.9, 1.7, 2.4):
        X = np.array([[5.0, 5.0, 5.0], [5.0, 5.0 + r, 5.0]])
        U = O.energy(pf, X, X, E0)
        assert abs(U - 0.3 * 0.7 * -0.4 / r ** 2) < 1e-9 * abs(U)
        F = O.forces(pf, X, X, E0)
        want = 2 * 0.3 * 0.7 * -0.4 / r ** 4 * np.array([0.0, -r, 0.0])
        np.testing.assert_allclose(F[0], want, rtol=1e-11, atol=1e-18)
        np.testing.assert_allclose(F[1], -want, rtol=1e-11, atol=1e-18)
    p = O.make_params(20, 0.8, n_atoms=2, coul_k=0.3, charges=q, lj_rc=2.5)
    X = np.array([[5.0, 5.0, 5.0], [5.0, 5.0 + 2.6, 5.0]])
    assert O.energy(p, X, X, E0) == 0.0 and np.abs(O.forces(p, X, X, E0)).max() == 0.0


def test_coulomb_newton_third_law_and_gradient(O, cluster):
    """With charges on the globule (bonded pairs excluded like LJ): forces sum to zero and
    equal -grad U by central differences."""
    from workloads import seeded_charges
    w, X = cluster
    q = seeded_charges(w.n_atoms, 3).astype(np.float64)
    p = O.make_params(w.L, w.tau, k_bond=w.k_bond, r0_bond=w.r0_bond, lj_eps=w.lj_eps,
                      lj_exclude_bonded=1, n_atoms=w.n_atoms, n_bonds=len(w.bonds),
                      coul_k=0.02, charges=q)
    F = O.forces(p, X, w.x0, w.bonds)
    p0 = O.make_params(w.L, w.tau, k_bond=w.k_bond, r0_bond=w.r0_bond, lj_eps=w.lj_eps,
                       lj_exclude_bonded=1, n_atoms=w.n_atoms, n_bonds=len(w.bonds))
    assert np.abs(F - O.forces(p0, X, w.x0, w.bonds)).max() > 1e-4   # the term is active
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-14)
    h = 1e-6
    rng = np.random.default_rng(2)
    for a in rng.choice(w.n_atoms, 8, replace=False):
        for c in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[a, c] += h
            Xm[a, c] -= h
            fd = -(O.energy(p, Xp, w.x0, w.bonds) - O.energy(p, Xm, w.x0, w.bonds)) / (2 * h)
            assert abs(fd - F[a, c]) < 1e-7 * max(1.0, abs(F[a, c])), (a, c, fd, F[a, c])
