"""Pins of the oracle's D3Q27 lattice (the higher-order velocity set the paper's outlook in
Section 4 proposes), against facts that do not come from the oracle itself: the set is all of
{-1, 0, 1}^3 with the tensor-product weights of the one-dimensional three-speed lattice, its
moments in exact arithmetic, conservation and Guo moments of the collision, brute-force
streaming, shear-wave decay at nu = (tau - 1/2)/3, the momentum ledger of a coupled run, and
for the thermal noise: an exactly orthogonal moment basis, exact conservation, the
fluctuation-dissipation variance of every mode, and equipartition."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

RNG = np.random.default_rng(2727)
NO_ATOMS = (np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2)))


def test_velocity_set_is_the_full_cube_with_product_weights(O):
    c, w = O.velocity_set(27)
    assert c.shape == (27, 3)
    assert {tuple(v) for v in c} == set(itertools.product((-1, 0, 1), repeat=3))
    # the first 19 rows are the D3Q19 set in the same order; opposite(i) = i + 1 for odd i
    c19, _ = O.velocity_set(19)
    assert (c[:19] == c19).all()
    for i in range(1, 27, 2):
        assert (c[i] == -c[i + 1]).all()
    # weights: product of the D1Q3 weights 2/3 (speed 0) and 1/6 (speed +-1) per axis
    w1 = {0: Fraction(2, 3), 1: Fraction(1, 6), -1: Fraction(1, 6)}
    wf = [w1[int(v[0])] * w1[int(v[1])] * w1[int(v[2])] for v in c]
    for i in range(27):
        assert abs(w[i] - float(wf[i])) < 1e-16
    assert sorted(set(wf)) == [Fraction(1, 216), Fraction(1, 54), Fraction(2, 27), Fraction(8, 27)]


def test_exact_moments_and_the_sixth_order_product(O):
    """Isotropy to fourth order as for D3Q19, plus sum w c_x^2 c_y^2 c_z^2 = c_s^6 = 1/27,
    which the 19-speed set (no corner velocities) lacks."""
    d = lambda a, b: 1 if a == b else 0
    for q in (19, 27):
        c, w = O.velocity_set(q)
        wf = [Fraction(x).limit_denominator(1000) for x in w]
        assert sum(wf) == 1
        for a in range(3):
            assert sum(wf[i] * int(c[i, a]) for i in range(q)) == 0
            for b in range(3):
                assert sum(wf[i] * int(c[i, a] * c[i, b]) for i in range(q)) == Fraction(d(a, b), 3)
                for g in range(3):
                    assert sum(wf[i] * int(c[i, a] * c[i, b] * c[i, g]) for i in range(q)) == 0
        for a, b, g, h in itertools.product(range(3), repeat=4):
            m4 = sum(wf[i] * int(c[i, a] * c[i, b] * c[i, g] * c[i, h]) for i in range(q))
            assert m4 == Fraction(d(a, b) * d(g, h) + d(a, g) * d(b, h) + d(a, h) * d(b, g), 9)
        m6 = sum(wf[i] * int(c[i, 0] ** 2 * c[i, 1] ** 2 * c[i, 2] ** 2) for i in range(q))
        assert m6 == (Fraction(1, 27) if q == 27 else 0)


@pytest.mark.parametrize("drho,u", [(0.0, (0.0, 0.0, 0.0)), (0.013, (0.02, -0.01, 0.005)),
                                    (-0.2, (0.1, 0.05, -0.07))])
def test_equilibrium_moments(O, drho, u):
    c, w = O.velocity_set(27)
    rho0 = 1.0
    rho = rho0 + drho
    u = np.array(u)
    f = w * rho0 + O.equilibrium(rho0, drho, u, q=27)
    assert abs(f.sum() - rho) < 1e-14
    np.testing.assert_allclose(c.T @ f, rho * u, atol=1e-15)
    Pi = np.einsum("ia,ib,i->ab", c, c, f)
    np.testing.assert_allclose(Pi, rho * (np.outer(u, u) + np.eye(3) / 3.0), atol=1e-15)


@pytest.mark.parametrize("tau,magic", [(0.55, 0.0), (0.8, 0.0), (1.7, 0.0), (0.8, 0.25), (0.6, 3 / 16)])
def test_collision_conservation_and_guo_moments(O, tau, magic):
    """Mass conserved, momentum j + F exactly; for BGK the second moment relaxes toward the
    forced equilibrium (for two relaxation times the even part does the same)."""
    c, w = O.velocity_set(27)
    rho0 = 1.0
    for trial in range(5):
        g = RNG.normal(0, 1e-3, 27)
        F = RNG.normal(0, 1e-3, 3) * (trial > 0)
        out = O.collide_node(tau, rho0, g, F, q=27, magic=magic)
        drho = g.sum()
        j = c.T @ g
        assert abs(out.sum() - drho) < 1e-17 * 27 + 1e-18
        np.testing.assert_allclose(c.T @ out, j + F, atol=1e-17)
        rho = rho0 + drho
        us = (j + 0.5 * F) / rho
        Pi = np.einsum("ia,ib,i->ab", c, c, g)
        Pi_eq = drho / 3.0 * np.eye(3) + rho * np.outer(us, us)
        want = Pi - (Pi - Pi_eq) / tau + (1 - 0.5 / tau) * (np.outer(us, F) + np.outer(F, us))
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, out), want, atol=1e-16)


def test_collision_fixed_point_and_shear_relaxation(O):
    g = O.equilibrium(1.0, 0.01, np.array([0.03, -0.02, 0.01]), q=27)
    np.testing.assert_allclose(O.collide_node(0.7, 1.0, g, np.zeros(3), q=27), g, atol=1e-17)
    c, w = O.velocity_set(27)
    neq = 1e-4 * w * c[:, 0] * c[:, 1]       # zero density and momentum
    tau = 0.8
    np.testing.assert_allclose(O.collide_node(tau, 1.0, neq, np.zeros(3), q=27), (1 - 1 / tau) * neq,
                               atol=1e-20)


def test_streaming_brute_force(O):
    c, _ = O.velocity_set(27)
    L = (5, 4, 3)
    rng = np.random.default_rng(8)
    for i in range(27):
        post = np.zeros((27, L[2], L[1], L[0]))
        x, y, z = rng.integers(L[0]), rng.integers(L[1]), rng.integers(L[2])
        post[i, z, y, x] = 1.0
        pre = O.stream(L, post)
        assert pre[i, (z + c[i, 2]) % L[2], (y + c[i, 1]) % L[1], (x + c[i, 0]) % L[0]] == 1.0
        assert pre.sum() == 1.0


def _shear_wave_rate(O, Ly, tau, steps=(10, 100), U0=1e-4):
    p = O.make_params((2, Ly, 2), tau, velocity_set=27)
    y = np.arange(Ly)
    g = np.zeros(O.pop_shape(p))
    assert g.shape[0] == 27
    for yy in y:
        g[:, :, yy, :] = O.equilibrium(1.0, 0.0, np.array([U0 * np.sin(2 * np.pi * yy / Ly), 0, 0]),
                                       q=27)[:, None, None]
    s = np.sin(2 * np.pi * y / Ly)
    amps = []
    for n in (steps[0], steps[1] - steps[0]):
        g = O.run(p, g, *NO_ATOMS, None, n)[0]
        _, u = O.observables(p, g)
        amps.append(2.0 / Ly * (u[0, 0, :, 0] * s).sum())
    return np.log(amps[0] / amps[1]) / (steps[1] - steps[0])


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_viscosity(O, tau):
    """The 27-speed lattice has the same shear viscosity nu = (tau - 1/2)/3 (within 1% at
    Ly = 32)."""
    Ly = 32
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / Ly
    rate = _shear_wave_rate(O, Ly, tau)
    assert abs(rate / (nu * k * k) - 1) < 0.01, (rate, nu * k * k)


def test_uniform_force_momentum_ledger(O):
    L = (6, 5, 4)
    p = O.make_params(L, 0.7, bf_kind=3, velocity_set=27)
    gvec = np.array([1e-5, -2e-5, 3e-6])
    field = np.broadcast_to(gvec[:, None, None, None], (3, 4, 5, 6)).copy()
    g = np.zeros(O.pop_shape(p))
    inv0 = O.invariants(p, g, np.zeros((0, 3)))
    for n in range(1, 4):
        g = O.run(p, g, *NO_ATOMS, field, 1)[0]
        inv = O.invariants(p, g, np.zeros((0, 3)))
        assert abs(inv[0] - inv0[0]) < 1e-12
        np.testing.assert_allclose(inv[1:4], n * 120 * gvec, rtol=1e-12)


def test_coupled_mass_and_momentum_ledger(O):
    """Atoms with LJ and friction in a 27-speed fluid: sum_x j + sum_a m v is conserved step by
    step, and mass always is."""
    from workloads import small_workload
    w = small_workload(12, 40, seed=3, gamma=0.15, k_tether=0.0, steps=0, velocity_set=27)
    p = O.params_from_workload(w)
    assert O.pop_shape(p)[0] == 27
    g = np.zeros(O.pop_shape(p))
    X, V = w.x0.astype(float), w.v0.astype(float)
    for _ in range(15):
        before = O.invariants(p, g, V)
        g, X, V = O.run(p, g, X, V, w.x0, w.bonds, None, 1)
        after = O.invariants(p, g, V)
        assert abs(after[0] - before[0]) < 1e-13 * before[0]
        tot0, tot1 = before[1:4] + before[4:7], after[1:4] + after[4:7]
        assert np.abs(tot1 - tot0).max() < 1e-15 + 1e-13 * np.abs(after[4:7]).max()
    assert np.abs(V).max() > 0


def test_unknown_sets_are_refused(O):
    with pytest.raises(ValueError):
        O.velocity_set(15)
    p = O.make_params(4, 0.8, velocity_set=15)
    with pytest.raises(RuntimeError):
        O.run(p, np.zeros((19, 4, 4, 4)), *NO_ATOMS, None, 1)


# ---------------------------------------------------------------- thermal noise on D3Q27

def test_mode_basis_orthogonal_in_exact_arithmetic(O):
    """The 27 modes: integer polynomials of c, orthogonal under the D3Q27 weights with norms
    n_a n_b n_c (n = 1, 1/3, 2 for the factors 1, c, 3c^2 - 1), density and momentum first,
    parity under c -> -c as published."""
    e, b, odd = O.mode_basis27()
    c, w = O.velocity_set(27)
    wf = [Fraction(x).limit_denominator(1000) for x in w]
    ei = np.rint(e).astype(int)
    assert np.array_equal(ei, e)
    assert (ei[0] == 1).all() and (ei[1:4] == c.T).all()
    norms = set()
    for k in range(27):
        for l in range(27):
            s = sum(wf[i] * int(ei[k, i]) * int(ei[l, i]) for i in range(27))
            if k != l:
                assert s == 0, (k, l)
            else:
                assert abs(float(s) - b[k]) < 1e-14 * float(s)
                norms.add(s)
        where = {tuple(int(v) for v in c[i]): i for i in range(27)}
        flipped = [where[tuple(-int(v) for v in c[i])] for i in range(27)]
        sign = -1 if odd[k] else 1
        assert (ei[k, flipped] == sign * ei[k]).all(), k
    # every norm is a product of three factors from {1, 1/3, 2}
    f = [Fraction(1), Fraction(1, 3), Fraction(2)]
    products = {a * bb * cc for a in f for bb in f for cc in f}
    assert norms <= products
    assert int(odd.sum()) == 13        # the modes with an odd number of c factors


def test_normal_stream_extends_the_d3q19_one(O):
    """D3Q27 draws six Philox calls per site and step; the first four are the D3Q19 draws."""
    z16 = O.site_normals(77, 12, 345)
    z24 = O.site_normals_n(77, 12, 345, 6)
    np.testing.assert_array_equal(z24[:16], z16)
    extra = np.concatenate([O.site_normals_n(5, 3, s, 6)[16:] for s in range(3000)])
    assert abs(extra.mean()) < 4.0 / np.sqrt(extra.size)
    assert abs(extra.var() - 1.0) < 4.0 * np.sqrt(2.0 / extra.size)


@pytest.mark.parametrize("magic", [0.0, 0.1875])
def test_noise_conserves_and_has_mode_variances(O, magic):
    e, b, odd = O.mode_basis27()
    c, w = O.velocity_set(27)
    kT, tau, rho = 2e-4, 0.7, 1.1
    xi = np.stack([O.site_noise(kT, tau, rho, 99, 5, s, trt_magic=magic, q=27) for s in range(4000)])
    scale = np.abs(xi).max()
    assert np.abs(xi.sum(1)).max() < 1e-15 * 27 * scale
    assert np.abs(xi @ c).max() < 1e-15 * 27 * scale
    m = xi @ e.T
    om_p = 1.0 / tau
    om_m = 1.0 / (0.5 + magic / (tau - 0.5)) if magic > 0 else om_p
    om = np.where(odd == 1, om_m, om_p)
    want = 3.0 * rho * kT * b * (1.0 - (1.0 - om) ** 2)
    var = (m ** 2).mean(0)
    assert np.all(var[:4] < 1e-25)
    rel = var[4:] / want[4:]
    tol = 4.0 * np.sqrt(2.0 / m.shape[0])
    assert np.all(np.abs(rel - 1.0) < tol), rel


def test_thermal_equipartition(O):
    """<u^2> per component = kT (1 - 1/S) and <(rho - rho0)^2> = 3 kT (1 - 1/S) on an 8^3
    lattice at kT = 1e-4, with mass and momentum exact."""
    L, tau, kT = 8, 0.8, 1e-4
    p = O.make_params(L, tau, kT=kT, seed=2027, velocity_set=27)
    S = L ** 3
    g = np.zeros(O.pop_shape(p))
    X = np.zeros((0, 3))
    u2, r2 = [], []
    step, burn, every, total = 0, 150, 3, 1350
    while step < total:
        p.step0 = step
        g, _, _ = O.run(p, g, X, X, X, np.zeros((0, 2), np.int32), None, every)
        step += every
        if step > burn:
            rho, u = O.observables(p, g)
            u2.append((u ** 2).mean())
            r2.append(((rho - 1.0) ** 2).mean())
    inv = O.invariants(p, g, X)
    assert abs(inv[0] - S) < 1e-11 * S
    assert np.abs(inv[1:4]).max() < 1e-13
    u2m, r2m = np.mean(u2), np.mean(r2)
    assert abs(u2m / (kT * (1 - 1 / S)) - 1.0) < 0.06, u2m
    assert abs(r2m / (3 * kT * (1 - 1 / S)) - 1.0) < 0.06, r2m
