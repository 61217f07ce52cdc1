"""The fluctuating-LB noise on the GPU: the same Philox4x32-10 noise as the oracle (parity),
continuity across checkpoints, equipartition, and the adjoint with noise."""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


def test_thermal_fluid_parity(O):
    from workloads import small_workload
    w = small_workload((20, 16, 12), 0, seed=3, tau=0.8, steps=0, kT=1e-4, noise_seed=77)
    steps = 25
    r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
    say("thermal fluid, 25 steps:", r)
    assert r["g"] < 1e-5 and r["u"] < 1e-5 and r["rho"] < 1e-5, r


def test_thermal_coupled_parity(O):
    from workloads import small_workload
    w = small_workload((24, 20, 18), 200, seed=8, tau=0.8, gamma=0.1, k_tether=0.05, mass=8.0,
                       kT=1e-5, noise_seed=5)
    steps = 10
    r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
    say("thermal coupled ball, 10 steps:", r)
    assert max(r.values()) < 1e-5, r


def test_noise_continues_across_checkpoint():
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import small_workload
    w = small_workload((16, 16, 16), 60, seed=2, tau=0.7, gamma=0.1, mass=8.0, kT=1e-5, noise_seed=9)
    a = CoupledLB.from_workload(w)
    a.step(10)
    snap = a.save_state()
    a.step(10)
    ga = a.populations()
    a.load_state(snap)
    assert a.step_count == 10
    a.step(10)
    gb = a.populations()
    assert bool((ga == gb).all())
    a.close()


def test_equipartition_on_gpu():
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB, make_params
    L, kT = 32, 1e-4
    sim = CoupledLB(make_params(L, 0.8, kT=kT, seed=31))
    sim.step(400)
    u2, r2 = [], []
    for _ in range(150):
        sim.step(20)
        rho, u, _, _ = sim.read_fields()
        u2.append(float((u.double() ** 2).mean()))
        r2.append(float(((rho.double() - 1.0) ** 2).mean()))
    inv = sim.invariants()
    sim.close()
    S = L ** 3
    ru = np.mean(u2) / (kT * (1 - 1 / S))
    rr = np.mean(r2) / (3 * kT * (1 - 1 / S))
    say("GPU equipartition: <u^2>/(kT/rho0) = %.4f, <drho^2>/(3 rho0 kT) = %.4f" % (ru, rr))
    assert abs(ru - 1) < 0.02 and abs(rr - 1) < 0.02
    # exact in exact arithmetic (pinned in FP64 on the oracle); FP32 storage and collision at
    # populations of the noise's size (~1e-2) random-walk by ~20 ulp per site and step, about
    # 2e-4 over sqrt(S * steps) ~ 1e4 site-steps here
    say("mass drift %.3e, momentum %s" % (inv[0] - S, inv[1:4]))
    assert abs(inv[0] - S) < 1e-7 * S and max(abs(x) for x in inv[1:4]) < 1e-7 * S


def test_adjoint_with_noise(O):
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB, params_from_workload
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, kT=1e-5, noise_seed=123)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    steps = 12
    p = params_from_workload(w)
    p.bf_kind = A.LB_BF_FIELD
    sim = CoupledLB(p, w.x0, w.v0, w.bonds, field.astype(np.float32))
    ck = sim.run_checkpointed(steps, 5)
    d = sim.displacement().double().cpu().numpy()
    out = sim.backward(ck, torch.from_numpy((2.0 * (d - D) / w.n_atoms).astype(np.float32)))
    sim.close()
    po = O.params_from_workload(w)
    po.bf_kind = 3
    g0 = np.zeros(O.pop_shape(po))
    f64 = field.astype(np.float32).astype(np.float64)
    X0, V0 = w.x0.astype(np.float64), w.v0.astype(np.float64)
    _, dg = O.loss_derivative(po, g0, X0, V0, w.bonds, f64, D, steps, 0)
    _, dt = O.loss_derivative(po, g0, X0, V0, w.bonds, f64, D, steps, 1)
    df = rng.normal(0, 1.0, size=field.shape)
    _, db = O.loss_derivative(po, g0, X0, V0, w.bonds, f64, D, steps, 2, df)
    dbg = float((out["body_force"].double().cpu().numpy() * df).sum())
    errs = (abs(out["gamma"] - dg) / abs(dg), abs(out["tau"] - dt) / abs(dt), abs(dbg - db) / abs(db))
    say("adjoint with noise, rel errors (gamma, tau, db):", errs)
    assert max(errs) < 1e-3, errs
