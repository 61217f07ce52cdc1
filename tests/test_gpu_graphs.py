"""For a graph replay of the steady-state steps of the overlapped schedule.  Replays must give
the same bits as the eager launches: calls of different lengths, so that replays start in both
step parities with eager steps between them, and synchronisations and reads between the calls;
a globule with LJ and bonds, a ragged ball with a body-force field, D3Q27 with two relaxation
times and FP16 storage.

The library has no graph path at present (every step is launched eagerly): the test is skipped,
and un-skipped it fails at once rather than compare eager launches with themselves.  A graph
path would be switched on by a parameter flag named LB_FLAG_STEP_GRAPHS."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="the HIP-graph replay of the three-stream step (stream capture with the "
                            "force and atom streams forked from a private origin stream) ended the "
                            "process with SIGSEGV inside lb_couple_step at its first capture; no cause "
                            "was found in this code, so the graph path was taken out and the library "
                            "launches every step eagerly"),
]


def _graph_flag():
    from paper_2305_05025_amd import _abi as A
    flag = getattr(A, "LB_FLAG_STEP_GRAPHS", None)
    if flag is None:
        pytest.fail("the library has no graph path (no LB_FLAG_STEP_GRAPHS): nothing to compare")
    return flag


def _make(w, graphs, **kw):
    from paper_2305_05025_amd.coupled import CoupledLB
    return CoupledLB.from_workload(w, flags=_graph_flag() if graphs else 0, **kw)


def _workload(kind):
    from workloads import globule_workload, small_workload
    if kind == "globule":
        return globule_workload((40, 36, 30), 1, 1200, seed=6, tau=0.6, gamma=0.2, bf_kind=1,
                                bf_amp=1e-6), "f32"
    if kind == "ball_field":
        L = (24, 20, 18)
        w = small_workload(L, 300, seed=3, tau=0.7, bf_kind=3)
        w.body_force = np.random.default_rng(5).normal(0, 1e-6, size=(3, L[2], L[1], L[0])).astype(np.float32)
        return w, "f32"
    return globule_workload((22, 20, 18), 1, 400, seed=4, tau=0.7, gamma=0.2, velocity_set=27,
                            trt_magic=0.1875), "f16"


@pytest.mark.parametrize("kind", ["globule", "ball_field", "q27_trt_f16"])
def test_graph_replays_match_eager(kind):
    import torch
    w, storage = _workload(kind)
    calls = [3, 25, 10, 17, 40]
    outs = []
    for graphs in (True, False):
        say("graphs", kind, graphs, "calls", calls)
        sim = _make(w, graphs, storage=storage)
        res = []
        for n in calls:
            sim.step(n)
            torch.cuda.synchronize()
            g = sim.populations().cpu().numpy()
            _, _, x, v = sim.read_fields()
            res.append((g, x.cpu().numpy(), v.cpu().numpy()))
        assert sim.step_count == sum(calls)
        sim.check()
        sim.close()
        outs.append(res)
    for k, (a, b) in enumerate(zip(*outs)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), (kind, "after call", k)
