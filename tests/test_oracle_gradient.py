"""The oracle's forward-mode (dual-number) derivative of the trajectory loss
L = (1/N) sum_a |X_a(T) - (X_a(0) + D)|^2 is pinned against central finite differences of the
float64 oracle (h = 1e-4 for gamma and tau, truncation error ~h^2), on the D3Q19 and the
D3Q27 lattice."""
import numpy as np
import pytest


@pytest.fixture(scope="module", params=[19, 27])
def small(O, request):
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, velocity_set=request.param)
    rng = np.random.default_rng(3)
    p = O.params_from_workload(w)
    p.bf_kind = 3
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    g = np.zeros(O.pop_shape(p))
    return p, w, g, field, D, rng


STEPS = 12


@pytest.mark.parametrize("wrt,name", [(0, "gamma"), (1, "tau")])
def test_dual_matches_central_difference_scalar(O, small, wrt, name):
    p, w, g, field, D, _ = small
    loss, dl = O.loss_derivative(p, g, w.x0, w.v0, w.bonds, field, D, STEPS, wrt)
    h = 1e-4
    base = getattr(p, name)
    setattr(p, name, base + h)
    lp = O.loss(p, g, w.x0, w.v0, w.bonds, field, D, STEPS)
    setattr(p, name, base - h)
    lm = O.loss(p, g, w.x0, w.v0, w.bonds, field, D, STEPS)
    setattr(p, name, base)
    l0 = O.loss(p, g, w.x0, w.v0, w.bonds, field, D, STEPS)
    assert abs(l0 - loss) < 1e-14 * abs(loss)
    fd = (lp - lm) / (2 * h)
    assert abs(dl) > 0
    assert abs(fd - dl) < 1e-6 * abs(dl), (name, fd, dl)


def test_dual_matches_central_difference_field_direction(O, small):
    p, w, g, field, D, rng = small
    dfield = rng.normal(0, 1.0, size=field.shape)
    loss, dl = O.loss_derivative(p, g, w.x0, w.v0, w.bonds, field, D, STEPS, 2, dfield)
    h = 1e-6
    lp = O.loss(p, g, w.x0, w.v0, w.bonds, field + h * dfield, D, STEPS)
    lm = O.loss(p, g, w.x0, w.v0, w.bonds, field - h * dfield, D, STEPS)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - dl) < 1e-5 * abs(dl) + 1e-12, (fd, dl)
