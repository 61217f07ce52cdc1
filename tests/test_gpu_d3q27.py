"""D3Q27 (the higher-order velocity set of the paper's outlook, Section 4) on the GPU against
the oracle: the fused sweep from random states on ragged lattices (BGK and two relaxation
times, every body-force kind), a shear wave with Kolmogorov forcing over 100 steps, the
narrow storage formats' one-step bound, the population upload, coupled globules, one
full-size sampled step at 256^3 with 200,000 atoms in the benchmarked schedule, the adjoint
against the oracle's exact derivatives, and the thermal noise on the 27-mode basis (parity,
equipartition, adjoint)."""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, rel_l2, say

pytestmark = pytest.mark.gpu


def _random_state(O, p, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, amp, size=O.pop_shape(p))
    return g.astype(np.float32).astype(np.float64)


def _ball(L, n=0, **kw):
    from workloads import small_workload
    return small_workload(L, n, velocity_set=27, **kw)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_population_upload_roundtrip(O, storage):
    import torch
    w = _ball((9, 7, 5), seed=1, steps=0)
    p = O.params_from_workload(w)
    assert O.pop_shape(p)[0] == 27
    g0 = _random_state(O, p, seed=2)
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]
    gp = gpu_run(w, 0, storage=storage, g0=g0)
    assert gp["g"].shape[0] == 27
    assert np.array_equal(gp["g"], torch.tensor(g0).to(dt).double().numpy())


@pytest.mark.parametrize("L,bf,magic", [((13, 11, 9), 1, 0.0), ((16, 16, 16), 2, 0.1875),
                                        ((24, 10, 7), 3, 0.0), ((2, 3, 5), 1, 0.25)])
def test_sweep_from_random_state(O, L, bf, magic):
    """Ragged lattices (partial last tile), the smallest extents, every body-force kind, BGK
    and two relaxation times; 1 and 10 steps."""
    w = _ball(L, seed=1, tau=0.7, steps=0, bf_kind=bf, bf_amp=3e-5, trt_magic=magic)
    if bf == 3:
        rng = np.random.default_rng(11)
        w.body_force = rng.normal(0, 1e-5, size=(3, L[2], L[1], L[0])).astype(np.float32)
    p = O.params_from_workload(w)
    g0 = _random_state(O, p, seed=5)
    for steps in (1, 10):
        r = compare(gpu_run(w, steps, g0=g0), oracle_run(O, w, steps, g0=g0), w)
        say("d3q27", L, bf, magic, steps, r)
        assert r["g"] < 1e-6 and r["u"] < 1e-6 and r["rho"] < 1e-6, r


def test_shear_wave_and_kolmogorov_100_steps(O):
    w = _ball((8, 32, 8), seed=1, tau=0.6, steps=0, bf_kind=1, bf_amp=1e-6)
    p = O.params_from_workload(w)
    g0 = np.zeros(O.pop_shape(p))
    for y in range(32):
        g0[:, :, y, :] = O.equilibrium(1.0, 0.0, [1e-3 * np.sin(2 * np.pi * y / 32), 0, 0],
                                       q=27)[:, None, None]
    g0 = g0.astype(np.float32).astype(np.float64)
    r = compare(gpu_run(w, 100, g0=g0), oracle_run(O, w, 100, g0=g0), w)
    say("d3q27 shear+kolmogorov", r)
    assert r["u"] < 1e-5 and r["g"] < 1e-5, r


@pytest.mark.parametrize("storage,rel", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_narrow_storage_one_step(O, storage, rel):
    """Each stored value is the FP32 collision result rounded once to the format."""
    import torch
    w = _ball((12, 10, 9), seed=1, tau=0.7, steps=0, bf_kind=1, bf_amp=1e-5)
    p = O.params_from_workload(w)
    g0 = _random_state(O, p, seed=9)
    dt = torch.float16 if storage == "f16" else torch.bfloat16
    g0 = torch.tensor(g0).to(dt).double().numpy()
    gp = gpu_run(w, 1, storage=storage, g0=g0)
    orc = oracle_run(O, w, 1, g0=g0)
    err = np.abs(gp["g"] - orc["g"])
    tiny = 2.0 ** -24 if storage == "f16" else 0.0
    bound = rel * np.abs(orc["g"]) + tiny + 1e-9
    say("d3q27", storage, "max err/bound", float((err / bound).max()))
    assert (err <= bound).all()


@pytest.mark.parametrize("magic", [0.0, 0.1875])
def test_globule_short_horizon(O, magic):
    """A 1,500-atom globule (bonds, bonded-pair exclusion, LJ, Kolmogorov forcing) on a ragged
    lattice, BGK and two relaxation times."""
    from workloads import globule_workload
    w = globule_workload((40, 36, 30), 1, 1500, seed=6, tau=0.6, gamma=0.2, name="glob27",
                         bf_kind=1, bf_amp=1e-6, velocity_set=27, trt_magic=magic)
    for steps in (1, 10):
        r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
        say("d3q27 globule", magic, steps, r)
        assert max(r.values()) < 1e-5, r


def test_one_step_full_size_sampled(O):
    """256^3 with 200,000 atoms in ten globules, two streams: one step from a seeded random
    lattice state, compared on sampled sites (half of them on atom stencils) and atoms."""
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import make_workload
    w = make_workload(2)
    w.velocity_set = 27
    rng = np.random.default_rng(127)
    shape = (27, w.L[2], w.L[1], w.L[0])
    say("d3q27 full size: random lattice state", shape)
    g0 = rng.standard_normal(size=shape, dtype=np.float32)
    g0 *= np.float32(1e-4)
    L = np.array(w.L)
    rand = rng.integers(0, int(np.prod(L)), size=2000)
    a = rng.integers(0, w.n_atoms, size=2000)
    n = (np.floor(w.x0[a].astype(np.float64)).astype(np.int64) + rng.integers(0, 2, size=(2000, 3))) % L
    sites = np.unique(np.concatenate([rand, n[:, 0] + L[0] * (n[:, 1] + L[1] * n[:, 2])]))
    atoms = np.sort(rng.choice(w.n_atoms, size=300, replace=False)).astype(np.int32)
    say("d3q27 full size: GPU step")
    sim = CoupledLB.from_workload(w)
    sim.set_populations(g0)
    sim.step(1)
    g1 = sim.populations().reshape(27, -1)
    gs = g1[:, torch.from_numpy(sites).to(g1.device)].T.double().cpu().numpy()
    del g1
    idx = torch.from_numpy(atoms).long().to("cuda")
    d = sim.displacement()[idx].double().cpu().numpy()
    _, _, _, v = sim.read_fields()
    vs = v[idx].double().cpu().numpy()
    sim.close()
    torch.cuda.empty_cache()
    say("d3q27 full size: oracle sampled step,", len(sites), "sites,", len(atoms), "atoms")
    p = O.params_from_workload(w)
    g64 = g0.astype(np.float64)
    del g0
    go, Xo, Vo = O.step_sampled(p, g64, w.x0, w.v0, w.x0, w.bonds, w.body_force, sites, atoms)
    del g64
    errs = {"g": rel_l2(gs, go), "disp": rel_l2(d, Xo - w.x0[atoms].astype(np.float64)),
            "v": rel_l2(vs, Vo)}
    say("d3q27 full size: rel. L2 over samples:", errs)
    assert max(errs.values()) < 1e-5, errs


def test_adjoint_matches_oracle_derivatives(O):
    """The adjoint on 27 velocities (checkpoint-and-recompute, 12 steps in segments of 5)
    against the oracle's exact dual-number derivatives: dL/dgamma, dL/dtau and dL/dF_ext along
    seeded directions, 1e-3 relative (FP32 adjoint against FP64 derivatives)."""
    from test_gpu_adjoint import _check, _dfields, _gpu_grads, _oracle_grads
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, velocity_set=27)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 12, 5, reps=2)
    _check(outs, _oracle_grads(O, w, field, D, 12, dfields), dfields, 1e-3)


def test_adjoint_linear_ball_two_relaxation_times(O):
    """Tethers and friction without LJ (linear dynamics) on a ragged box, two relaxation
    times: 20 steps in segments of 7, 2e-4 relative."""
    from test_gpu_adjoint import _check, _dfields, _gpu_grads, _oracle_grads
    w = _ball((14, 12, 10), 40, seed=5, tau=0.8, gamma=0.1, k_tether=0.05, lj=False, mass=8.0,
              trt_magic=0.1875)
    rng = np.random.default_rng(9)
    field = rng.normal(0, 1e-5, size=(3, 10, 12, 14))
    D = np.array([0.0, 0.8, -0.6])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 20, 7)
    _check(outs, _oracle_grads(O, w, field, D, 20, dfields), dfields, 2e-4)


# ------------------------------------------------------------------ thermal noise on D3Q27

@pytest.mark.parametrize("magic", [0.0, 0.1875])
def test_thermal_fluid_parity(O, magic):
    """The same Philox noise on the 27-mode basis as the oracle (BGK and two relaxation
    times), 25 steps."""
    w = _ball((20, 16, 12), seed=3, tau=0.8, steps=0, kT=1e-4, noise_seed=77, trt_magic=magic)
    r = compare(gpu_run(w, 25), oracle_run(O, w, 25), w)
    say("d3q27 thermal fluid", magic, r)
    assert r["g"] < 1e-5 and r["u"] < 1e-5 and r["rho"] < 1e-5, r


def test_thermal_coupled_parity(O):
    w = _ball((24, 20, 18), 200, seed=8, tau=0.8, gamma=0.1, k_tether=0.05, mass=8.0, kT=1e-5,
              noise_seed=5)
    r = compare(gpu_run(w, 10), oracle_run(O, w, 10), w)
    say("d3q27 thermal coupled ball", r)
    assert max(r.values()) < 1e-5, r


def test_equipartition_on_gpu():
    """<u^2> = kT/rho0 per component and <(rho - rho0)^2> = 3 rho0 kT (times 1 - 1/S) on a
    32^3 thermal lattice, within 2%; mass and momentum to FP32 round-off."""
    from paper_2305_05025_amd.coupled import CoupledLB, make_params
    L, kT = 32, 1e-4
    sim = CoupledLB(make_params(L, 0.8, kT=kT, seed=31, velocity_set=27))
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
    say("d3q27 GPU equipartition: %.4f %.4f" % (ru, rr))
    assert abs(ru - 1) < 0.02 and abs(rr - 1) < 0.02
    assert abs(inv[0] - S) < 1e-7 * S and max(abs(x) for x in inv[1:4]) < 1e-7 * S


def test_adjoint_with_noise(O):
    from test_gpu_adjoint import _check, _dfields, _gpu_grads, _oracle_grads
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15, kT=1e-5, noise_seed=123,
                         velocity_set=27)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 12, 5)
    _check(outs, _oracle_grads(O, w, field, D, 12, dfields), dfields, 1e-3)
