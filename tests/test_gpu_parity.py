"""Parity of the HIP path (through the C interface) with the CPU oracle.

Tolerances (FP32 deviation storage, FP32 arithmetic, against the FP64 oracle):
  * lattice-only and non-chaotic coupled runs: rel. L2 <= 1e-5 on u, rho - rho0, populations,
    atom displacement and velocity, after 100 steps;
  * runs with Lennard-Jones: the atom trajectories are chaotic (a rounding-level difference
    doubles about every 9 steps, measured with the oracle itself in FP32 vs FP64), so the
    1e-5 gate applies up to 20 steps; at 100 steps the GPU must stay within the spread that
    an FP32-level perturbation of the initial velocities produces in the FP64 oracle.
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, rel_l2, say

pytestmark = pytest.mark.gpu


def _random_state(O, p, seed, amp=1e-3):
    rng = np.random.default_rng(seed)
    g = rng.normal(0.0, amp, size=O.pop_shape(p))
    return g.astype(np.float32).astype(np.float64)


# ------------------------------------------------------------------ lattice alone

@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_population_upload_roundtrip(O, storage):
    """lb_set_populations then lb_read_populations returns the state (rounded to the format)."""
    import torch
    from workloads import small_workload
    w = small_workload((9, 7, 5), 0, seed=1, steps=0)
    p = O.params_from_workload(w)
    g0 = _random_state(O, p, seed=2)
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[storage]
    want = torch.tensor(g0).to(dt).double().numpy()
    gp = gpu_run(w, 0, storage=storage, g0=g0)
    assert np.array_equal(gp["g"], want)

@pytest.mark.parametrize("L,bf", [((13, 11, 9), 1), ((16, 16, 16), 2), ((24, 10, 7), 3)])
def test_sweep_from_random_state(O, L, bf):
    """Random non-equilibrium state on ragged lattices (tiles with a partial tail), all three
    body-force kinds; 1 and 10 steps."""
    from workloads import small_workload
    w = small_workload(L, 0, seed=1, tau=0.7, steps=0, bf_kind=bf, bf_amp=3e-5)
    if bf == 3:
        rng = np.random.default_rng(11)
        w.body_force = rng.normal(0, 1e-5, size=(3, L[2], L[1], L[0])).astype(np.float32)
    p = O.params_from_workload(w)
    g0 = _random_state(O, p, seed=5)
    for steps in (1, 10):
        gp = gpu_run(w, steps, g0=g0)
        orc = oracle_run(O, w, steps, g0=g0)
        r = compare(gp, orc, w)
        say(L, bf, steps, r)
        assert r["g"] < 1e-6 and r["u"] < 1e-6 and r["rho"] < 1e-6, r


def test_shear_wave_and_kolmogorov_100_steps(O):
    from workloads import small_workload
    w = small_workload((8, 32, 8), 0, seed=1, tau=0.6, steps=0, bf_kind=1, bf_amp=1e-6)
    p = O.params_from_workload(w)
    g0 = np.zeros(O.pop_shape(p))
    for y in range(32):
        g0[:, :, y, :] = O.equilibrium(1.0, 0.0, [1e-3 * np.sin(2 * np.pi * y / 32), 0, 0])[:, None, None]
    g0 = g0.astype(np.float32).astype(np.float64)
    gp = gpu_run(w, 100, g0=g0)
    orc = oracle_run(O, w, 100, g0=g0)
    r = compare(gp, orc, w)
    say("shear+kolmogorov", r)
    assert r["u"] < 1e-5 and r["g"] < 1e-5, r


@pytest.mark.parametrize("storage,rel", [("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_narrow_storage_one_step(O, storage, rel):
    """One step from a state representable in the format: each stored value is the FP32
    collision result rounded once to the format (within half an ulp of the format)."""
    import torch
    from workloads import small_workload
    L = (12, 10, 9)
    w = small_workload(L, 0, seed=1, tau=0.7, steps=0, bf_kind=1, bf_amp=1e-5)
    p = O.params_from_workload(w)
    g0 = _random_state(O, p, seed=9)
    dt = torch.float16 if storage == "f16" else torch.bfloat16
    g0 = torch.tensor(g0).to(dt).double().numpy()
    gp = gpu_run(w, 1, storage=storage, g0=g0)
    orc = oracle_run(O, w, 1, g0=g0)
    err = np.abs(gp["g"] - orc["g"])
    tiny = 2.0 ** -24 if storage == "f16" else 0.0   # f16 subnormal spacing
    bound = rel * np.abs(orc["g"]) + tiny + 1e-9
    say(storage, "max err/bound", float((err / bound).max()))
    assert (err <= bound).all()


# ------------------------------------------------------------------ coupled: configuration 0

def _c0(lj=True):
    from workloads import make_workload
    w = make_workload(0)
    if not lj:
        w.lj_eps = 0.0
        w.name += "_nolj"
    return w


@pytest.mark.parametrize("steps", [1, 10, 20])
def test_config0_short_horizon(O, steps):
    w = _c0()
    r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
    say("c0", steps, r)
    assert max(r.values()) < 1e-5, r


def test_config0_without_lj_100_steps(O):
    """Tethers + friction only: linear, non-chaotic dynamics; the 1e-5 gate at 100 steps."""
    w = _c0(lj=False)
    r = compare(gpu_run(w, 100), oracle_run(O, w, 100), w)
    say("c0 no LJ 100", r)
    assert max(r.values()) < 1e-5, r


def test_config0_100_steps(O):
    """The ball workload (tethers, Lennard-Jones between all atoms) over 100 steps.  Its LJ
    dynamics amplify rounding: the spread of the FP64 scheme itself under a one-ulp (2^-24
    relative, random sign) change of the initial velocities is 2.1e-6 on v after 100 steps.
    Gates: u, rho, g and the displacement within 1e-5; the velocity within 6 times that
    spread (measured 9.9e-6, 4.7 times it; for seeds 10 and 11 of the same construction
    9.4e-6 and 1.2e-5, so a flat 1e-5 on v does not hold for every seed)."""
    w = _c0()
    orc = oracle_run(O, w, 100)
    rng = np.random.default_rng(17)
    wp = _c0()
    wp.v0 = (w.v0.astype(np.float64) * (1 + 2.0 ** -24 * rng.choice([-1, 1], size=w.v0.shape)))
    spread = compare(oracle_run(O, wp, 100), orc, w)
    r = compare(gpu_run(w, 100), orc, w)
    say("c0 100 gpu", r, "fp64 one-ulp spread", spread)
    for k in ("u", "rho", "g", "disp", "x"):
        assert r[k] < 1e-5, (k, r[k])
    assert r["v"] < 6.0 * spread["v"], (r["v"], spread["v"])


def test_paper_coupling_rate_tethered_ball(O):
    """The friction at the paper's own rate, gamma dt / m = 0.2 per step (unit mass; the
    benchmark workloads use m = 32 for their Lennard-Jones packings): 200 tethered atoms without
    Lennard-Jones, stable at m = 1, dragged by a Kolmogorov flow over 50 steps.  The atoms'
    initial velocities relax towards the fluid's within a few steps, so every atom velocity is
    set by the interpolated fluid velocity and the two-way coupling."""
    from workloads import small_workload
    w = small_workload((24, 22, 20), 200, seed=13, tau=0.7, gamma=0.2, k_tether=0.05, lj=False, mass=1.0,
                       bf_kind=1, bf_amp=1e-4)
    r = compare(gpu_run(w, 50), oracle_run(O, w, 50), w)
    say("gamma/m = 0.2, tethered ball, 50 steps", r)
    assert max(r.values()) < 1e-5, r


# ------------------------------------------------------------------ coupled: globules

def _globule(L=(40, 36, 30), n=1500, bf=1, seed=6):
    from workloads import globule_workload
    w = globule_workload(L, 1, n, seed=seed, tau=0.6, gamma=0.2, name="glob%d" % n,
                         bf_kind=bf, bf_amp=1e-6 if bf == 1 else 0.0)
    if bf == 3:
        rng = np.random.default_rng(seed)
        w.body_force = rng.normal(0, 1e-6, size=(3, L[2], L[1], L[0])).astype(np.float32)
    return w


@pytest.mark.parametrize("bf", [1, 3])
def test_globule_short_horizon(O, bf):
    """Bonds, bonded-pair LJ exclusion, body force, ragged lattice."""
    w = _globule(bf=bf)
    for steps in (1, 10):
        r = compare(gpu_run(w, steps), oracle_run(O, w, steps), w)
        say("globule", bf, steps, r)
        assert max(r.values()) < 1e-5, r


def test_momentum_and_mass_ledger_on_gpu(O):
    """No tethers, no net body force: total (fluid + atom) momentum and mass are conserved
    by the GPU step to rounding, measured by the library's FP64 sums."""
    w = _globule(bf=0, n=800, L=(24, 24, 24))
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    sim = CoupledLB.from_workload(w)
    inv0 = np.array(sim.invariants())
    orc0 = O.invariants(O.params_from_workload(w), np.zeros(O.pop_shape(O.params_from_workload(w))), w.v0)
    np.testing.assert_allclose(inv0, orc0, rtol=1e-7, atol=1e-12)
    # FP32 force sums and velocity updates round at 2^-24 of the atom momentum scale per step
    p_scale = float(w.mass * np.abs(w.v0.astype(np.float64)).sum())
    for k in range(1, 6):
        sim.step(10)
        inv = np.array(sim.invariants())
        _, _, _, v = sim.read_fields()
        p_scale = max(p_scale, float(w.mass * v.double().abs().sum()))
        say("ledger", inv)
        assert abs(inv[0] - inv0[0]) < 1e-9 * inv0[0]
        p_tot = inv[1:4] + inv[4:7]
        drift = np.abs(p_tot - (inv0[1:4] + inv0[4:7])).max()
        say("momentum drift", drift, "bound", 1.2e-7 * p_scale * 10 * k)
        assert drift < 1.2e-7 * p_scale * 10 * k
    sim.close()


def test_determinism_and_checkpoint(O):
    """Two runs are bitwise identical; save/continue equals load/continue bitwise."""
    from paper_2305_05025_amd.coupled import CoupledLB
    w = _globule(n=1000, L=(32, 32, 32))
    a = CoupledLB.from_workload(w)
    b = CoupledLB.from_workload(w)
    a.step(15)
    b.step(15)
    snap = a.save_state()
    a.step(15)
    b.step(15)
    ga, gb = a.populations(), b.populations()
    _, _, xa, va = a.read_fields()
    _, _, xb, vb = b.read_fields()
    assert (ga == gb).all() and (xa == xb).all() and (va == vb).all()
    a.load_state(snap)
    assert a.step_count == 15
    a.step(15)
    _, _, xc, vc = a.read_fields()
    assert (a.populations() == gb).all() and (xc == xb).all() and (vc == vb).all()
    assert a.step_count == 30
    a.close()
    b.close()


def test_call_chunking_is_bitwise_identical(O):
    """30 steps in one lb_couple_step call and the same 30 in calls of 1, 1, 1, 7 and 20 steps
    give identical bits (each call starts by binning its first step; within a call the next
    binning overlaps the sweep)."""
    from paper_2305_05025_amd.coupled import CoupledLB
    w = _globule(n=1000, L=(32, 30, 28))
    a = CoupledLB.from_workload(w)
    b = CoupledLB.from_workload(w)
    a.step(30)
    for n in (1, 1, 1, 7, 20):
        b.step(n)
    assert a.step_count == b.step_count == 30
    _, _, xa, va = a.read_fields()
    _, _, xb, vb = b.read_fields()
    assert (a.populations() == b.populations()).all() and (xa == xb).all() and (va == vb).all()
    a.close()
    b.close()


def test_single_stream_schedule_is_bitwise_identical(O):
    """The overlapped two-stream schedule, with the force field started early or after the
    coupling kernels (LBMD_LATE_FORCES), and the single-stream one give identical bits.  With
    4000 atoms (and more neighbour cells than that) the three launch the force field on
    different grids (768, 512 and 1000 workgroups)."""
    import os
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB
    w = _globule(n=4000, L=(48, 44, 40))
    outs = []
    for flags, late in ((0, False), (0, True), (A.LB_FLAG_SINGLE_STREAM, False)):
        if late:
            os.environ["LBMD_LATE_FORCES"] = "1"
        try:
            sim = CoupledLB.from_workload(w, flags=flags)
        finally:
            os.environ.pop("LBMD_LATE_FORCES", None)
        sim.step(12)
        g = sim.populations()
        _, _, x, v = sim.read_fields()
        outs.append((g, x, v))
        sim.close()
    for other in outs[1:]:
        for a, b in zip(outs[0], other):
            assert (a == b).all()


def test_small_lattice_one_stream_default_is_bitwise_identical(O):
    """A lattice of at most LB_ONE_STREAM_MAX_SITES sites (the 32^3 ball) runs on one stream by
    default; with LBMD_OVERLAP_SMALL it takes the two-stream schedule.  Both give identical
    bits, and the default matches the oracle."""
    import os
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB
    w = _c0()
    assert int(np.prod(w.L)) <= A.LB_ONE_STREAM_MAX_SITES
    outs = []
    for overlap in (False, True):
        if overlap:
            os.environ["LBMD_OVERLAP_SMALL"] = "1"
        try:
            sim = CoupledLB.from_workload(w)
        finally:
            os.environ.pop("LBMD_OVERLAP_SMALL", None)
        sim.step(12)
        g = sim.populations()
        _, _, x, v = sim.read_fields()
        outs.append((g, x, v))
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        assert (a == b).all()
    r = compare(gpu_run(w, 12), oracle_run(O, w, 12), w)
    say("c0 12 steps, one stream", r)
    assert max(r.values()) < 1e-5, r


def test_contexts_interleaved_on_their_own_streams():
    """Three contexts at once, each on a caller stream of its own, their calls interleaved with no
    synchronisation between them: two of the 48 x 44 x 40 globule (two-stream schedule, each
    with its own atom stream and events) and the 32^3 ball (one stream).  Each ends with the
    bits of the same steps run alone on the default stream."""
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    wa, wb = _globule(n=4000, L=(48, 44, 40)), _c0()

    def state(sim):
        g = sim.populations()
        _, _, x, v = sim.read_fields()
        return g, x, v

    def alone(w, n):
        sim = CoupledLB.from_workload(w)
        sim.step(n)
        out = state(sim)
        sim.close()
        return out

    sims = [CoupledLB.from_workload(w, stream=torch.cuda.Stream()) for w in (wa, wa, wb)]
    for calls in ((3, 2, 4), (5, 6, 2), (4, 4, 0)):
        for sim, n in zip(sims, calls):
            sim.step(n)
    outs = [state(sim) for sim in sims]
    for sim in sims:
        sim.close()
    ref_a, ref_b = alone(wa, 12), alone(wb, 6)
    for out, ref in zip(outs, (ref_a, ref_a, ref_b)):
        for a, b in zip(out, ref):
            assert (a == b).all()


def test_error_paths_on_device():
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB, make_params
    x = torch.tensor([[4.0, 4.0, 4.0], [float("nan"), 1.0, 1.0]])
    v = torch.zeros(2, 3)
    with pytest.raises(A.LBError) as e:
        CoupledLB(make_params(12, 0.8, n_atoms=2, mass=8.0), x, v)
    assert e.value.status == A.LB_EINVAL and "x0" in str(e.value)
    x = torch.tensor([[4.0, 4.0, 4.0], [5.0, 5.0, 5.0]])
    with pytest.raises(A.LBError) as e:
        CoupledLB(make_params(12, 0.8, n_atoms=2, mass=8.0, n_bonds=1), x, v,
                  bonds=torch.tensor([[0, 2]], dtype=torch.int32))
    assert e.value.status == A.LB_EINVAL and "bond" in str(e.value)
    # 60 atoms inside one neighbour-list cell: the capacity check latches an overflow
    rng = np.random.default_rng(0)
    # (12 / floor(12 / 2.5025) = 3-wide cells: [3.2, 5.8]^3 lies inside cell (1, 1, 1))
    xs = torch.tensor(3.2 + rng.uniform(0, 2.6, size=(60, 3)), dtype=torch.float32)
    sim = CoupledLB(make_params(12, 0.8, n_atoms=60, mass=8.0, lj_eps=1e-9), xs, torch.zeros(60, 3))
    sim.step(1)
    with pytest.raises(A.LBError) as e:
        sim.check()
    assert e.value.status == A.LB_EOVERFLOW
    sim.close()
    # a NaN population is reported after the next step
    sim = CoupledLB(make_params(8, 0.8))
    g = np.zeros((19, 8, 8, 8), np.float32)
    g[3, 2, 2, 2] = np.nan
    sim.set_populations(g)
    sim.step(1)
    with pytest.raises(A.LBError) as e:
        sim.check()
    assert e.value.status == A.LB_ENONFINITE
    sim.close()
