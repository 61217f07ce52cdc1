"""Pins of the oracle's lattice part (Eq. 1-3 of the paper, Section 2.2) against facts that do
not come from the oracle itself: exact lattice identities, moment identities, conservation,
brute-force streaming, and closed-form hydrodynamics (shear-wave decay at nu = (tau - 1/2)/3,
forced Kolmogorov flow)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

RNG = np.random.default_rng(1234)


# ---------------------------------------------------------------- velocity set (D3Q19)

def test_velocity_set_exact_isotropy(O):
    c, w = O.velocity_set()
    assert c.shape == (19, 3)
    # the weights are the exact rationals 1/3, 1/18, 1/36 by speed class
    wf = []
    for i in range(19):
        n2 = int((c[i] ** 2).sum())
        want = {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}[n2]
        assert abs(w[i] - float(want)) < 1e-16
        wf.append(want)
    # 19 distinct vectors: rest, 6 faces, 12 edges
    assert len({tuple(v) for v in c}) == 19
    assert sorted(int((v ** 2).sum()) for v in c) == [0] + [1] * 6 + [2] * 12
    # opposite(i) = i+1 for odd i
    for i in range(1, 19, 2):
        assert (c[i] == -c[i + 1]).all()
    # moments in exact arithmetic
    d = lambda a, b: 1 if a == b else 0
    assert sum(wf) == 1
    for a in range(3):
        assert sum(wf[i] * int(c[i, a]) for i in range(19)) == 0
        for b in range(3):
            assert sum(wf[i] * int(c[i, a]) * int(c[i, b]) for i in range(19)) == Fraction(d(a, b), 3)
            for g in range(3):
                assert sum(wf[i] * int(c[i, a] * c[i, b] * c[i, g]) for i in range(19)) == 0
    for a, b, g, h in itertools.product(range(3), repeat=4):
        m4 = sum(wf[i] * int(c[i, a] * c[i, b] * c[i, g] * c[i, h]) for i in range(19))
        want = Fraction(d(a, b) * d(g, h) + d(a, g) * d(b, h) + d(a, h) * d(b, g), 9)
        assert m4 == want, (a, b, g, h)


# ---------------------------------------------------------------- equilibrium

@pytest.mark.parametrize("drho,u", [(0.0, (0.0, 0.0, 0.0)), (0.013, (0.02, -0.01, 0.005)),
                                    (-0.2, (0.1, 0.05, -0.07))])
def test_equilibrium_moments(O, drho, u):
    """f_eq = w rho0 + g_eq: sum f_eq = rho, sum c f_eq = rho u,
    sum c c f_eq = rho (u u + I/3) (the second-order truncated Maxwellian)."""
    c, w = O.velocity_set()
    rho0 = 1.0
    rho = rho0 + drho
    u = np.array(u)
    f = w * rho0 + O.equilibrium(rho0, drho, u)
    assert abs(f.sum() - rho) < 1e-14
    np.testing.assert_allclose(c.T @ f, rho * u, atol=1e-15)
    Pi = np.einsum("ia,ib,i->ab", c, c, f)
    np.testing.assert_allclose(Pi, rho * (np.outer(u, u) + np.eye(3) / 3.0), atol=1e-15)


# ---------------------------------------------------------------- collision (Eq. 1 + Guo)

@pytest.mark.parametrize("tau", [0.55, 0.8, 1.7])
def test_collision_conservation_and_guo_moments(O, tau):
    """Without force the collision conserves mass and momentum; with Guo forcing the
    post-collision momentum is j + F exactly and the second moment relaxes toward the
    forced equilibrium:  Pi* = Pi - (Pi - Pi_eq(u*))/tau + (1 - 1/(2 tau)) (u* F + F u*)."""
    c, w = O.velocity_set()
    rho0 = 1.0
    for trial in range(5):
        g = RNG.normal(0, 1e-3, 19)
        F = RNG.normal(0, 1e-3, 3) * (trial > 0)
        out = O.collide_node(tau, rho0, g, F)
        drho = g.sum()
        j = c.T @ g
        assert abs(out.sum() - drho) < 1e-17 * 19 + 1e-18
        np.testing.assert_allclose(c.T @ out, j + F, atol=1e-17)
        rho = rho0 + drho
        us = (j + 0.5 * F) / rho
        Pi = np.einsum("ia,ib,i->ab", c, c, g)
        Pi_eq = drho / 3.0 * np.eye(3) + rho * np.outer(us, us)
        want = Pi - (Pi - Pi_eq) / tau + (1 - 0.5 / tau) * (np.outer(us, F) + np.outer(F, us))
        np.testing.assert_allclose(np.einsum("ia,ib,i->ab", c, c, out), want, atol=1e-16)


def test_collision_fixed_point_is_equilibrium(O):
    """A node already at equilibrium and without force is left unchanged."""
    g = O.equilibrium(1.0, 0.01, np.array([0.03, -0.02, 0.01]))
    out = O.collide_node(0.7, 1.0, g, np.zeros(3))
    np.testing.assert_allclose(out, g, atol=1e-17)


def test_collision_relaxation_rate(O):
    """A pure non-equilibrium perturbation with zero mass and momentum (a shear-stress
    mode) is scaled by (1 - 1/tau) per collision: the sign of the relaxation term."""
    c, w = O.velocity_set()
    tau = 0.8
    # non-equilibrium part proportional to w_i (c_ix c_iy): zero density and momentum
    neq = 1e-4 * w * c[:, 0] * c[:, 1]
    assert abs(neq.sum()) < 1e-20 and np.abs(c.T @ neq).max() < 1e-20
    out = O.collide_node(tau, 1.0, neq, np.zeros(3))
    np.testing.assert_allclose(out, (1 - 1 / tau) * neq, atol=1e-20)


# ---------------------------------------------------------------- streaming

def test_streaming_brute_force(O):
    c, _ = O.velocity_set()
    L = (5, 4, 3)
    S = 60
    rng = np.random.default_rng(7)
    for i in range(19):
        post = np.zeros((19, L[2], L[1], L[0]))
        x, y, z = rng.integers(L[0]), rng.integers(L[1]), rng.integers(L[2])
        post[i, z, y, x] = 1.0
        pre = O.stream(L, post)
        xx, yy, zz = (x + c[i, 0]) % L[0], (y + c[i, 1]) % L[1], (z + c[i, 2]) % L[2]
        assert pre[i, zz, yy, xx] == 1.0
        assert pre.sum() == 1.0
    post = rng.normal(size=(19, L[2], L[1], L[0]))
    pre = O.stream(L, post)
    np.testing.assert_allclose(pre.sum(axis=(1, 2, 3)), post.sum(axis=(1, 2, 3)), rtol=1e-14)
    assert S == np.prod(L)


# ---------------------------------------------------------------- hydrodynamics

def _shear_wave_rate(O, Ly, tau, steps=(10, 100), U0=1e-4):
    """Decay rate per step of u_x = U0 sin(2 pi y / Ly) in a (2, Ly, 2) periodic box."""
    p = O.make_params((2, Ly, 2), tau)
    y = np.arange(Ly)
    g = np.zeros(O.pop_shape(p))
    for yy in y:
        ge = O.equilibrium(1.0, 0.0, np.array([U0 * np.sin(2 * np.pi * yy / Ly), 0.0, 0.0]))
        g[:, :, yy, :] = ge[:, None, None]
    amps = {}
    s = np.sin(2 * np.pi * y / Ly)
    g = O.run(p, g, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2)), None,
              steps[0])[0]
    _, u = O.observables(p, g)
    amps[steps[0]] = 2.0 / Ly * (u[0, 0, :, 0] * s).sum()
    g = O.run(p, g, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2)), None,
              steps[1] - steps[0])[0]
    _, u = O.observables(p, g)
    amps[steps[1]] = 2.0 / Ly * (u[0, 0, :, 0] * s).sum()
    return np.log(amps[steps[0]] / amps[steps[1]]) / (steps[1] - steps[0])


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.2])
def test_shear_wave_viscosity(O, tau):
    """Shear-wave amplitude decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3, i.e. the
    relation omega = 2/(6 nu + 1) of the paper; within 1% at Ly = 32."""
    Ly = 32
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / Ly
    rate = _shear_wave_rate(O, Ly, tau)
    assert rate > 0, "shear wave must decay"
    assert abs(rate / (nu * k * k) - 1) < 0.01, (rate, nu * k * k)


def test_shear_wave_converges_second_order(O):
    """The relative error of the decay rate shrinks ~4x per doubling of Ly."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    errs = []
    for Ly in (8, 16, 32):
        k = 2 * np.pi / Ly
        errs.append(abs(_shear_wave_rate(O, Ly, tau) / (nu * k * k) - 1))
    assert errs[2] < errs[1] < errs[0]
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_uniform_force_momentum_ledger(O):
    """A uniform force density g adds exactly g per node per step to sum_x j; mass is unchanged."""
    L = (6, 5, 4)
    p = O.make_params(L, 0.7, bf_kind=3)
    field = np.zeros((3, 4, 5, 6))
    gvec = np.array([1e-5, -2e-5, 3e-6])
    field[:] = gvec[:, None, None, None]
    g = np.zeros(O.pop_shape(p))
    S = 120
    inv0 = O.invariants(p, g, np.zeros((0, 3)))
    for n in range(1, 4):
        g = O.run(p, g, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2)),
                  field, 1)[0]
        inv = O.invariants(p, g, np.zeros((0, 3)))
        assert abs(inv[0] - inv0[0]) < 1e-12
        np.testing.assert_allclose(inv[1:4], n * S * gvec, rtol=1e-12)


def test_kolmogorov_transient(O):
    """From rest under g_x = g0 sin(2 pi y/Ly): the velocity amplitude follows
    A(t) = g0 / (rho0 nu k^2) (1 - exp(-nu k^2 t)) (within 1%)."""
    Ly, tau, g0 = 32, 0.6, 1e-6
    p = O.make_params((2, Ly, 2), tau, bf_kind=1, bf_amp=g0)
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / Ly
    g = np.zeros(O.pop_shape(p))
    y = np.arange(Ly)
    s = np.sin(2 * np.pi * y / Ly)
    t = 0
    for t_next in (100, 400):
        g = O.run(p, g, np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2)),
                  None, t_next - t)[0]
        t = t_next
        _, u = O.observables(p, g)
        A = 2.0 / Ly * (u[0, 0, :, 0] * s).sum()
        want = g0 / (nu * k * k) * (1 - np.exp(-nu * k * k * t))
        assert abs(A / want - 1) < 0.01, (t, A, want)
        # the flow stays a pure x-directed sine profile
        assert np.abs(u[1:]).max() < 1e-6 * abs(A)
