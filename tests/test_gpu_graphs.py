"""Graph replay of the step (LB_FLAG_STEP_GRAPHS) against the eager launches, bit for bit.

With the flag, a call of two or more steps replays a two-step graph captured once per
starting parity (a call's odd last step is launched eagerly, so the next call starts at the
other parity and uses the other graph).  The calls below have lengths 3, 25, 10, 17 and 40:
both graphs are built and replayed many times, with the eager odd steps, synchronisations and
reads of the populations and atoms between the calls, and the state after every call must
equal that of the same calls launched eagerly.  Cases: a globule with LJ and bonds on the
two-stream schedule and on one stream, a ragged ball with a body-force field, D3Q27 with two
relaxation times and FP16 storage, and a lattice without atoms.  Thermal noise (whose counter
is the step) and LB_FLAG_CHECK_FINITE take the eager path under the flag; that is checked too."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _graph_flag():
    from paper_2305_05025_amd import _abi as A
    flag = getattr(A, "LB_FLAG_STEP_GRAPHS", None)
    if flag is None:
        pytest.fail("the library has no graph path (no LB_FLAG_STEP_GRAPHS): nothing to compare")
    return flag


def _workload(kind):
    from workloads import globule_workload, small_workload
    if kind in ("globule", "globule_single_stream"):
        return globule_workload((40, 36, 30), 1, 1200, seed=6, tau=0.6, gamma=0.2, bf_kind=1,
                                bf_amp=1e-6), "f32"
    if kind == "ball_field":
        L = (24, 20, 18)
        w = small_workload(L, 300, seed=3, tau=0.7, bf_kind=3)
        w.body_force = np.random.default_rng(5).normal(0, 1e-6, size=(3, L[2], L[1], L[0])).astype(np.float32)
        return w, "f32"
    if kind == "lattice_only":
        return small_workload((20, 18, 22), 0, seed=2, tau=0.65, bf_kind=1, bf_amp=1e-5), "f32"
    if kind == "thermal_ball":
        w = small_workload((16, 14, 12), 100, seed=4, tau=0.7, kT=1e-4, noise_seed=3)
        return w, "f32"
    return globule_workload((22, 20, 18), 1, 400, seed=4, tau=0.7, gamma=0.2, velocity_set=27,
                            trt_magic=0.1875), "f16"


def _run(w, storage, flags, calls):
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    sim = CoupledLB.from_workload(w, storage=storage, flags=flags)
    res = []
    for n in calls:
        sim.step(n)
        torch.cuda.synchronize()
        g = sim.populations().cpu().numpy()
        if w.n_atoms:
            _, _, x, v = sim.read_fields()
            res.append((g, x.cpu().numpy(), v.cpu().numpy()))
        else:
            res.append((g,))
    assert sim.step_count == sum(calls)
    sim.check()
    sim.close()
    return res


@pytest.mark.parametrize("kind", ["globule", "globule_single_stream", "ball_field", "q27_trt_f16",
                                  "lattice_only"])
def test_graph_replays_match_eager(kind):
    from paper_2305_05025_amd import _abi as A
    w, storage = _workload(kind)
    calls = [3, 25, 10, 17, 40]
    base = A.LB_FLAG_SINGLE_STREAM if kind == "globule_single_stream" else 0
    say("graphs", kind, "calls", calls)
    graph = _run(w, storage, base | _graph_flag(), calls)
    eager = _run(w, storage, base, calls)
    for k, (a, b) in enumerate(zip(graph, eager)):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), (kind, "after call", k)


@pytest.mark.parametrize("extra", ["thermal", "check_finite"])
def test_graph_flag_falls_back_to_eager(extra):
    """Under the flag, thermal noise and the per-step finiteness check run eagerly: same bits."""
    from paper_2305_05025_amd import _abi as A
    if extra == "thermal":
        w, storage = _workload("thermal_ball")
        base = 0
    else:
        w, storage = _workload("ball_field")
        base = A.LB_FLAG_CHECK_FINITE
    calls = [4, 7]
    graph = _run(w, storage, base | _graph_flag(), calls)
    eager = _run(w, storage, base, calls)
    for a, b in zip(graph, eager):
        for u, v in zip(a, b):
            assert np.array_equal(u, v), extra
