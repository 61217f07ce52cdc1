"""Parity at the full sizes of all five workloads (32^3 tethered ball, 128^3 globule with
Kolmogorov forcing, 256^3 with ten globules, 96^3 globule with a body-force field, 384^3 with
fifty globules and sign-shear forcing), in the launch configuration bench.py times (two
streams, one for the 32^3 ball, whose lattice is small enough to run on one; FP32 storage): one coupled step from a seeded random lattice state and the
workload's atoms, compared with the oracle on sampled outputs it computes one by one
(populations at sampled sites, half of them on atom stencils; positions and velocities of
sampled atoms).  Rel. L2 over the samples <= 1e-5, and element by element
max |GPU - oracle| / max |oracle| <= 1e-5.  The 256^3 workload is also checked with thermal
noise at the benchmark's kT = 1e-4, so that the noise generator's counter, keyed by site and
step, is compared at 16.7M sites."""
import numpy as np
import pytest

from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


def _sample_sites(rng, w, n_random, n_near):
    L = np.array(w.L)
    S = int(np.prod(L))
    rand = rng.integers(0, S, size=n_random)
    a = rng.integers(0, w.n_atoms, size=n_near)
    base = np.floor(w.x0[a].astype(np.float64)).astype(np.int64)
    off = rng.integers(0, 2, size=(n_near, 3))
    n = (base + off) % L
    near = n[:, 0] + L[0] * (n[:, 1] + L[1] * n[:, 2])
    return np.unique(np.concatenate([rand, near]))


@pytest.mark.parametrize("config", [0, 1, 2, 3, 4])
def test_one_step_full_size_sampled(O, config):
    from workloads import make_workload
    say("full-size sampled parity: building workload", config)
    _one_step_sampled(O, make_workload(config), 100 + config)


def test_one_step_full_size_sampled_thermal(O):
    """The 256^3 workload with the fluctuating lattice of the benchmark's thermal leg."""
    import dataclasses
    from workloads import make_workload
    say("full-size sampled parity, thermal: building workload 2")
    _one_step_sampled(O, dataclasses.replace(make_workload(2), kT=1e-4, noise_seed=7), 205)


def _one_step_sampled(O, w, seed):
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    rng = np.random.default_rng(seed)
    shape = (19, w.L[2], w.L[1], w.L[0])
    say("  random lattice state", shape)
    g0 = rng.standard_normal(size=shape, dtype=np.float32)
    g0 *= np.float32(1e-4)
    sites = _sample_sites(rng, w, 2000, 2000)
    atoms = np.sort(rng.choice(w.n_atoms, size=min(300, w.n_atoms), replace=False)).astype(np.int32)

    say("  GPU step", w.name)
    sim = CoupledLB.from_workload(w)
    sim.set_populations(g0)
    sim.step(1)
    g1 = sim.populations().reshape(19, -1)
    gs = g1[:, torch.from_numpy(sites).to(g1.device)].T.double().cpu().numpy()
    del g1
    d = sim.displacement()[torch.from_numpy(atoms).long().to("cuda")].double().cpu().numpy()
    _, _, _, v = sim.read_fields()
    vs = v[torch.from_numpy(atoms).long().to("cuda")].double().cpu().numpy()
    sim.close()
    torch.cuda.empty_cache()

    say("  oracle sampled step:", len(sites), "sites,", len(atoms), "atoms")
    p = O.params_from_workload(w)
    g64 = g0.astype(np.float64)
    del g0
    go, Xo, Vo = O.step_sampled(p, g64, w.x0, w.v0, w.x0, w.bonds, w.body_force, sites, atoms)
    del g64
    x0 = w.x0[atoms].astype(np.float64)
    errs = {"g": rel_l2(gs, go), "disp": rel_l2(d, Xo - x0), "v": rel_l2(vs, Vo)}
    say("  rel. L2 over samples:", errs)
    assert max(errs.values()) < 1e-5, errs
    # element by element: max |GPU - oracle| / max |oracle| over every sampled value, so that
    # a wrong value at a few nodes cannot hide in the norm
    ew = {"g": np.abs(gs - go).max() / np.abs(go).max(),
          "disp": np.abs(d - (Xo - x0)).max() / np.abs(Xo - x0).max(),
          "v": np.abs(vs - Vo).max() / np.abs(Vo).max()}
    say("  max |diff| / max |ref| over samples:", ew)
    assert max(ew.values()) < 1e-5, ew
