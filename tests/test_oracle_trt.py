"""Pins of the oracle's two-relaxation-time collision (the collision-variant extension):
the part of the non-equilibrium even under c -> -c relaxes at omega+ = 1/tau, the odd part at
omega-, with Lambda = (1/omega+ - 1/2)(1/omega- - 1/2) the "magic" parameter.

* Lambda = (tau - 1/2)^2 gives omega- = omega+: the BGK collision;
* mass and momentum: sum g* = sum g, sum c g* = j + F exactly, for any Lambda;
* each mode of the orthogonal moment basis relaxes by its own factor: 1 - omega- for the six
  modes odd under c -> -c beyond momentum (k = 10..15), 1 - omega+ for the even ones;
* the shear wave still decays as exp(-nu k^2 t) with nu = (1/omega+ - 1/2)/3 (within 1%);
* with thermal noise, equipartition holds with the odd modes' noise set by omega-.
"""
import numpy as np
import pytest


def _random_node(rng, amp=1e-3):
    return rng.normal(0, amp, 19), rng.normal(0, 1e-4, 3)


@pytest.mark.parametrize("tau", [0.55, 0.8, 1.3])
def test_trt_reduces_to_bgk(O, tau):
    rng = np.random.default_rng(1)
    for _ in range(20):
        g, F = _random_node(rng)
        a = O.collide_node(tau, 1.0, g, F)
        b = O.collide_node_trt(tau, (tau - 0.5) ** 2, 1.0, g, F)
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-17)


@pytest.mark.parametrize("magic", [1 / 12, 3 / 16, 1 / 4, 1.0])
def test_trt_conserves_mass_and_momentum(O, magic):
    c, w = O.velocity_set()
    rng = np.random.default_rng(2)
    for _ in range(20):
        g, F = _random_node(rng)
        out = O.collide_node_trt(0.7, magic, 1.0, g, F)
        assert abs(out.sum() - g.sum()) < 1e-17
        np.testing.assert_allclose(c.T @ out, c.T @ g + F, rtol=0, atol=1e-17)


@pytest.mark.parametrize("tau,magic", [(0.6, 1 / 4), (0.9, 3 / 16), (0.55, 1 / 12)])
def test_trt_mode_relaxation_rates(O, tau, magic):
    e, b = O.mode_basis()
    c, w = O.velocity_set()
    om_p = 1.0 / tau
    om_m = 1.0 / (0.5 + magic / (tau - 0.5))
    eps = 1e-4
    for k in range(4, 19):
        g = eps * w * e[k]                   # mode k alone, fluid at rest: g_eq = 0
        out = O.collide_node_trt(tau, magic, 1.0, g, np.zeros(3))
        want = (1.0 - (om_m if 10 <= k <= 15 else om_p)) * g
        np.testing.assert_allclose(out, want, rtol=0, atol=1e-18, err_msg="mode %d" % k)


def _trt_shear_rate(O, Ly, tau, magic, steps=(10, 100), U0=1e-4):
    p = O.make_params((2, Ly, 2), tau, trt_magic=magic)
    y = np.arange(Ly)
    g = np.zeros(O.pop_shape(p))
    for yy in y:
        g[:, :, yy, :] = O.equilibrium(1.0, 0.0, np.array([U0 * np.sin(2 * np.pi * yy / Ly), 0, 0]))[:, None, None]
    s = np.sin(2 * np.pi * y / Ly)
    E = np.zeros((0, 3))
    amps = []
    for n in (steps[0], steps[1] - steps[0]):
        g = O.run(p, g, E, E, E, np.zeros((0, 2)), None, n)[0]
        _, u = O.observables(p, g)
        amps.append(2.0 / Ly * (u[0, 0, :, 0] * s).sum())
    return np.log(amps[0] / amps[1]) / (steps[1] - steps[0])


@pytest.mark.parametrize("tau,magic", [(0.8, 1 / 4), (0.6, 3 / 16), (1.2, 1 / 12)])
def test_trt_shear_wave_viscosity(O, tau, magic):
    Ly = 32
    nu = (tau - 0.5) / 3.0
    k = 2 * np.pi / Ly
    rate = _trt_shear_rate(O, Ly, tau, magic)
    assert abs(rate / (nu * k * k) - 1) < 0.01, (rate, nu * k * k)


def test_trt_thermal_equipartition(O):
    L, tau, kT, magic = 8, 0.7, 1e-4, 3 / 16
    p = O.make_params(L, tau, kT=kT, seed=99, trt_magic=magic)
    S = L ** 3
    g = np.zeros(O.pop_shape(p))
    E = np.zeros((0, 3))
    u2, r2 = [], []
    step = 0
    while step < 1500:
        p.step0 = step
        g = O.run(p, g, E, E, E, np.zeros((0, 2), np.int32), None, 3)[0]
        step += 3
        if step > 150:
            rho, u = O.observables(p, g)
            u2.append((u ** 2).mean())
            r2.append(((rho - 1.0) ** 2).mean())
    assert abs(np.mean(u2) / (kT * (1 - 1 / S)) - 1) < 0.06
    assert abs(np.mean(r2) / (3 * kT * (1 - 1 / S)) - 1) < 0.06
