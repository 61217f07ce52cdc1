"""The two-relaxation-time collision variant on the GPU against the oracle: lattice, coupled
atoms, thermal noise (odd modes at omega-), the BGK special case, and the adjoint."""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


def _g0(O, w, seed, amp=1e-3):
    p = O.params_from_workload(w)
    return np.random.default_rng(seed).normal(0, amp, size=O.pop_shape(p)).astype(np.float32)


@pytest.mark.parametrize("tau,magic", [(0.55, 3 / 16), (0.8, 1 / 4), (1.1, 1 / 12)])
def test_trt_lattice_parity(O, tau, magic):
    from workloads import small_workload
    w = small_workload((18, 14, 11), 0, seed=1, tau=tau, steps=0, bf_kind=1, bf_amp=1e-5,
                       trt_magic=magic)
    g0 = _g0(O, w, 2)
    r = compare(gpu_run(w, 30, g0=g0), oracle_run(O, w, 30, g0=g0), w)
    say("TRT lattice tau %g magic %g:" % (tau, magic), r)
    assert max(r.values()) < 1e-5, r


def test_trt_coupled_and_thermal_parity(O):
    from workloads import small_workload
    w = small_workload((22, 20, 18), 200, seed=8, tau=0.7, gamma=0.1, k_tether=0.05, mass=8.0,
                       trt_magic=3 / 16, kT=1e-5, noise_seed=11)
    r = compare(gpu_run(w, 15), oracle_run(O, w, 15), w)
    say("TRT coupled thermal ball, 15 steps:", r)
    assert max(r.values()) < 1e-5, r


def test_trt_special_case_is_bgk(O):
    from workloads import small_workload
    tau = 0.8
    base = dict(seed=3, tau=tau, gamma=0.1, k_tether=0.05, mass=8.0)
    wb = small_workload((16, 14, 12), 100, **base)
    wt = small_workload((16, 14, 12), 100, trt_magic=(tau - 0.5) ** 2, **base)
    a, b = gpu_run(wb, 20), gpu_run(wt, 20)
    for k in ("u", "g", "d", "v"):
        e = np.linalg.norm(a[k] - b[k]) / max(np.linalg.norm(a[k]), 1e-300)
        assert e < 2e-6, (k, e)


@pytest.mark.parametrize("kT", [0.0, 1e-5])
def test_trt_adjoint(O, kT):
    from test_gpu_adjoint import _check, _dfields, _gpu_grads, _oracle_grads
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, trt_magic=3 / 16, kT=kT,
                         noise_seed=5)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 12, 5)
    _check(outs, _oracle_grads(O, w, field, D, 12, dfields), dfields, 1e-3)
