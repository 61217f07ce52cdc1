"""The fused coupled sweep against the unfused kernels, bit for bit.

Fused (LB_FLAG_FUSED_COUPLING): one workgroup per hot brick (16 x 4 x 4 sites touched by an
atom stencil) computes the coupling velocity on the brick and a one-node halo, the friction of
the atoms listed there and their spread force in LDS, then updates the brick's sites; a plain
sweep updates every other site beside it.  Unfused (the default): coupling velocity at the
flagged nodes, friction, spread, then one sweep over every site.  Both follow
the same arithmetic, so populations, positions and velocities must agree bit for bit, on
lattices that bricks do not divide, lattices narrower than a brick (where the halo wraps onto
the brick), with thermal noise, two relaxation times, D3Q27, 16-bit storage, the Coulomb term,
every body-force kind and the single-stream schedule."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _run(w, steps, chain, storage="f32", flags=0):
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB
    if not chain:
        flags |= A.LB_FLAG_FUSED_COUPLING
    sim = CoupledLB.from_workload(w, storage=storage, flags=flags)
    sim.step(steps)
    g = sim.populations()
    _, _, x, v = sim.read_fields()
    d = sim.displacement()
    sim.check()
    sim.close()
    torch.cuda.synchronize()
    return g, x, v, d


def _case(name):
    from workloads import globule_workload, seeded_charges, small_workload
    rng = np.random.default_rng(sum(map(ord, name)))
    if name == "globule_kolmogorov":
        return globule_workload((40, 36, 30), 1, 1500, seed=6, tau=0.6, gamma=0.2, bf_kind=1,
                                bf_amp=1e-5), "f32"
    if name == "ball_field_thermal":
        L = (26, 19, 18)
        w = small_workload(L, 300, seed=3, tau=0.7, bf_kind=3, kT=1e-4, noise_seed=9)
        w.body_force = rng.normal(0, 1e-5, size=(3, L[2], L[1], L[0])).astype(np.float32)
        return w, "f32"
    if name == "q27_trt_f16":
        return globule_workload((22, 20, 18), 1, 400, seed=4, tau=0.7, gamma=0.2, velocity_set=27,
                                trt_magic=0.1875, bf_kind=2, bf_amp=1e-5), "f16"
    if name == "narrow_box_bf16":
        # 10 < 16 sites along x (one brick, whose halo wraps onto it); 9 = 2 bricks + 1 row in z
        return small_workload((10, 8, 9), 40, seed=7, tau=0.75, gamma=0.15, radius=2.2), "bf16"
    if name == "charged_globule":
        w = globule_workload((34, 30, 33), 1, 900, seed=5, tau=0.65, gamma=0.2, coul_k=0.02)
        w.charges = seeded_charges(w.n_atoms, 3)
        return w, "f32"
    if name == "tiny_lattice":
        w = small_workload((3, 2, 5), 0, seed=1, tau=0.7, gamma=0.3, k_tether=0.05, lj=False,
                           mass=2.0)
        w.x0 = np.array([[0.3, 1.7, 4.6], [2.9, 0.2, 0.5], [1.5, 1.0, 2.0]], np.float32)
        w.v0 = rng.normal(0, 0.02, size=w.x0.shape).astype(np.float32)
        return w, "f32"
    raise ValueError(name)


@pytest.mark.parametrize("name", ["globule_kolmogorov", "ball_field_thermal", "q27_trt_f16",
                                  "narrow_box_bf16", "charged_globule", "tiny_lattice"])
def test_fused_equals_unfused_bitwise(name):
    w, storage = _case(name)
    say("fused vs unfused", name, w.L, "atoms", w.n_atoms, storage)
    steps = 9
    fused = _run(w, steps, chain=False, storage=storage)
    chain = _run(w, steps, chain=True, storage=storage)
    for a, b in zip(fused, chain):
        assert bool((a == b).all()), name


def test_fused_single_stream_equals_two_streams():
    from paper_2305_05025_amd import _abi as A
    w, storage = _case("globule_kolmogorov")
    a = _run(w, 11, chain=False)
    b = _run(w, 11, chain=False, flags=A.LB_FLAG_SINGLE_STREAM)
    for u, v in zip(a, b):
        assert bool((u == v).all())
