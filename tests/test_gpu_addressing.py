"""The lattice kernels address a population plane by a scalar base and a 32-bit lane byte
offset when every plane's sites span at most 4 GiB, and by 64-bit lane addresses otherwise
(lattices beyond 2^30 sites in FP32).  Setting LBMD_WIDE_OFFSETS when a context is created
forces the 64-bit form on a small lattice: both forms must give identical bits, forward (every
storage format, both velocity sets, noise, two relaxation times, coupled globules) and in the
adjoint."""
import os

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _create(wide, make):
    if wide:
        os.environ["LBMD_WIDE_OFFSETS"] = "1"
    try:
        return make()
    finally:
        os.environ.pop("LBMD_WIDE_OFFSETS", None)


@pytest.mark.parametrize("q,storage,kT,magic", [(19, "f32", 0.0, 0.0), (19, "f16", 0.0, 0.0),
                                                (19, "bf16", 1e-5, 0.1875),
                                                (27, "f32", 1e-5, 0.0), (27, "bf16", 0.0, 0.25)])
def test_wide_and_narrow_addressing_identical(q, storage, kT, magic):
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import globule_workload
    w = globule_workload((22, 20, 18), 1, 400, seed=4, tau=0.7, gamma=0.2, velocity_set=q,
                         kT=kT, noise_seed=9, trt_magic=magic, bf_kind=1, bf_amp=1e-6)
    say("addressing", q, storage, kT, magic)
    outs = []
    for wide in (False, True):
        sim = _create(wide, lambda: CoupledLB.from_workload(w, storage=storage))
        sim.step(15)
        g = sim.populations().cpu().numpy()
        rho, u, x, v = sim.read_fields()
        outs.append((g, rho.cpu().numpy(), u.cpu().numpy(), x.cpu().numpy(), v.cpu().numpy()))
        sim.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("q", [19, 27])
def test_wide_and_narrow_adjoint_identical(q):
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB, params_from_workload
    from workloads import globule_workload
    L = 12
    w = globule_workload(L, 1, 80, seed=21, tau=0.7, gamma=0.15, velocity_set=q)
    field = np.random.default_rng(3).normal(0, 1e-5, size=(3, L, L, L)).astype(np.float32)
    say("adjoint addressing", q)
    outs = []
    for wide in (False, True):
        p = params_from_workload(w, "f32")
        p.bf_kind = A.LB_BF_FIELD
        sim = _create(wide, lambda: CoupledLB(p, w.x0, w.v0, w.bonds, field, charges=w.charges))
        ck = sim.run_checkpointed(10, 4)
        d = sim.displacement().double().cpu().numpy()
        dLdX = torch.from_numpy((2.0 * d / w.n_atoms).astype(np.float32))
        outs.append(sim.backward(ck, dLdX))
        sim.close()
    a, b = outs
    assert a["gamma"] == b["gamma"] and a["tau"] == b["tau"]
    assert bool((a["body_force"] == b["body_force"]).all())
