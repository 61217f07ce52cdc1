"""lb_invariants_noalloc (the conserved sums with the reduction's partial sums in the library's
fixed device array, written asynchronously to caller device memory) against lb_invariants
(partials in the context's workspace), through the C interface: two calls in a row, the second
on a context with a smaller lattice and fewer atoms, each bit for bit equal to lb_invariants."""
import math

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _sum_noalloc(sim):
    import torch
    from paper_2305_05025_amd import _abi as A
    out = torch.full((7,), math.nan, dtype=torch.float64, device=sim.device)
    torch.cuda.synchronize(sim.device)
    A.lb_invariants_noalloc(sim.ctx, out.data_ptr())
    sim.stream.synchronize()
    return out.cpu().numpy()


def test_noalloc_invariants_equal_workspace_invariants():
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB
    from workloads import globule_workload, small_workload
    big = globule_workload((40, 36, 30), 1, 1500, seed=6, tau=0.6, gamma=0.2, bf_kind=1, bf_amp=1e-5)
    small = small_workload((12, 10, 9), 30, seed=2, tau=0.7, gamma=0.1, mass=8.0)
    results = []
    for w, steps in ((big, 9), (small, 5)):
        say("noalloc invariants", w.name, w.L, "atoms", w.n_atoms, "steps", steps)
        sim = CoupledLB.from_workload(w)
        sim.step(steps)
        got = _sum_noalloc(sim)
        ref = np.array(A.lb_invariants(sim.ctx))
        say("  noalloc", got.tolist(), "workspace", ref.tolist())
        assert np.array_equal(got, ref), (got, ref)
        # the momentum sums are not all zero: the comparison has something to compare
        assert np.abs(ref[1:]).max() > 0
        results.append(got)
        sim.close()
    assert not np.array_equal(results[0], results[1])
