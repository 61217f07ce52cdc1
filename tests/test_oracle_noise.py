"""Pins of the oracle's thermal noise (fluctuating LB, the xi_i of Eq. 1's source term).

* Philox4x32-10 against its published known-answer vectors;
* the moment basis: exactly orthogonal under the D3Q19 weights (rational arithmetic), its
  first four modes the conserved mass and momentum;
* the normals: zero mean, unit variance, uncorrelated across sites and steps;
* the noise: no mass or momentum, and the variance mu b_k (1 - (1 - omega)^2) on each
  non-conserved mode, mu = 3 rho kT;
* equipartition in a thermal fluid at rest: <u_a^2> = kT/rho0 and <drho^2> = 3 rho0 kT per
  site (each reduced by the conserved global mode, a factor 1 - 1/S).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers(O):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = O.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10], (r, ["%08x" % x for x in out])


def test_mode_basis_exactly_orthogonal(O):
    e, b = O.mode_basis()
    c, w = O.velocity_set()
    assert np.array_equal(e, np.round(e))          # integer polynomials of c
    W = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    assert np.allclose([float(x) for x in W], w, rtol=0, atol=0)
    E = [[int(e[k, i]) for i in range(19)] for k in range(19)]
    for k in range(19):
        for l in range(19):
            g = sum(W[i] * E[k][i] * E[l][i] for i in range(19))
            if k == l:
                assert g > 0 and abs(float(g) - b[k]) < 1e-15
            else:
                assert g == 0, (k, l, g)
    # modes 0..3 are the conserved density and momentum
    assert np.array_equal(e[0], np.ones(19))
    assert np.array_equal(e[1:4], c.T)


def test_normals_statistics(O):
    z = np.concatenate([O.site_normals(12345, step, site) for step in range(4) for site in range(1024)])
    n = z.size
    assert abs(z.mean()) < 4.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4.0 * np.sqrt(2.0 / n)
    assert abs((z ** 4).mean() - 3.0) < 0.15               # Gaussian kurtosis
    a = np.stack([O.site_normals(12345, 0, s) for s in range(2048)])
    b = np.stack([O.site_normals(12345, 1, s) for s in range(2048)])
    c = np.stack([O.site_normals(54321, 0, s) for s in range(2048)])
    for x, y in ((a, b), (a, c), (a[:-1], a[1:])):
        r = np.corrcoef(x.ravel(), y.ravel())[0, 1]
        assert abs(r) < 4.0 / np.sqrt(x.size), r


def test_noise_conserves_and_has_mode_variances(O):
    e, b = O.mode_basis()
    c, w = O.velocity_set()
    kT, tau, rho = 2e-4, 0.7, 1.1
    xi = np.stack([O.site_noise(kT, tau, rho, 99, 5, s) for s in range(4000)])
    scale = np.abs(xi).max()
    assert np.abs(xi.sum(1)).max() < 1e-15 * 19 * scale
    assert np.abs(xi @ c).max() < 1e-15 * 19 * scale
    m = xi @ e.T                                           # modes of the noise
    om = 1.0 / tau
    want = 3.0 * rho * kT * b * (1.0 - (1.0 - om) ** 2)
    var = (m ** 2).mean(0)
    assert np.all(var[:4] < 1e-25)
    rel = var[4:] / want[4:]
    tol = 4.0 * np.sqrt(2.0 / m.shape[0])
    assert np.all(np.abs(rel - 1.0) < tol), rel


def test_thermal_equipartition(O):
    L, tau, kT = 8, 0.8, 1e-4
    p = O.make_params(L, tau, kT=kT, seed=2024)
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
    assert abs(inv[0] - S) < 1e-11 * S                     # mass exact
    assert np.abs(inv[1:4]).max() < 1e-13                  # momentum exact (zero)
    n_eff = len(u2)
    u2m, r2m = np.mean(u2), np.mean(r2)
    want_u2 = kT * (1.0 - 1.0 / S)
    want_r2 = 3.0 * kT * (1.0 - 1.0 / S)
    # samples every 3 steps are correlated; 6% covers the remaining statistical error
    assert abs(u2m / want_u2 - 1.0) < 0.06, (u2m, want_u2, n_eff)
    assert abs(r2m / want_r2 - 1.0) < 0.06, (r2m, want_r2, n_eff)
