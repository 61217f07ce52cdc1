"""GPU adjoint (lb_backward, checkpoint-and-recompute) against the oracle's exact
forward-mode derivatives of the same discrete scheme.

Loss (the differentiation workload's): L = (1/N) sum_a |X_a(T) - (X_a(0) + D)|^2.  The GPU gets
dL/dX(T) = 2 (X(T) - X(0) - D)/N from its own final displacement and returns dL/dgamma,
dL/dtau and dL/dF_ext; the oracle gives dL/dgamma, dL/dtau and the directional derivative
<dL/dF_ext, dF> along seeded directions, all in FP64.  Tolerance: 1e-3 relative (FP32
adjoint against FP64 exact derivatives), tighter where the dynamics are linear.
"""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def _gpu_grads(w, field, D, steps, k, storage="f32", reps=1):
    import torch
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB, params_from_workload
    say("adjoint", w.name, w.L, "atoms", w.n_atoms, "steps", steps, "k", k, storage)
    p = params_from_workload(w, storage)
    p.bf_kind = A.LB_BF_FIELD
    sim = CoupledLB(p, w.x0, w.v0, w.bonds, field.astype(np.float32), charges=w.charges)
    ck = sim.run_checkpointed(steps, k)
    d = sim.displacement().double().cpu().numpy()
    g_before = sim.populations().cpu().numpy()
    dLdX = 2.0 * (d - D[None, :]) / w.n_atoms
    outs = [sim.backward(ck, torch.from_numpy(dLdX.astype(np.float32))) for _ in range(reps)]
    g_after = sim.populations().cpu().numpy()
    assert sim.step_count == steps
    assert np.array_equal(g_before, g_after), "lb_backward must restore the context's state"
    sim.close()
    return outs, d


def _oracle_grads(O, w, field, D, steps, dfields):
    p = O.params_from_workload(w)
    p.bf_kind = 3
    g0 = np.zeros(O.pop_shape(p))
    X0 = w.x0.astype(np.float64)
    V0 = w.v0.astype(np.float64)
    f64 = field.astype(np.float32).astype(np.float64)
    _, dg = O.loss_derivative(p, g0, X0, V0, w.bonds, f64, D, steps, 0)
    _, dt = O.loss_derivative(p, g0, X0, V0, w.bonds, f64, D, steps, 1)
    dbs = [O.loss_derivative(p, g0, X0, V0, w.bonds, f64, D, steps, 2, df)[1] for df in dfields]
    return dg, dt, dbs


def _check(outs, orc, dfields, tol):
    dg, dt, dbs = orc
    out = outs[0]
    db = out["body_force"].double().cpu().numpy()
    errs = {"gamma": abs(out["gamma"] - dg) / abs(dg), "tau": abs(out["tau"] - dt) / abs(dt)}
    for q, (df, ref) in enumerate(zip(dfields, dbs)):
        errs["db%d" % q] = abs(float((db * df).sum()) - ref) / abs(ref)
    say("adjoint rel errors", errs, "oracle", dg, dt, dbs)
    for k, e in errs.items():
        assert e < tol, (k, e, errs)
    for o in outs[1:]:      # repeated backward passes are bitwise identical
        assert o["gamma"] == out["gamma"] and o["tau"] == out["tau"]
        assert bool((o["body_force"] == out["body_force"]).all())


def _dfields(rng, shape, n=2):
    return [rng.normal(0, 1.0, size=shape) for _ in range(n)]


def test_adjoint_side_stream_is_bitwise_identical():
    """In a two-stream context each adjoint step runs the force field's Hessian-vector product on
    the atom stream beside its lattice part; on one stream it runs in order.  Both give the same
    bits for every gradient (a 16^3 globule, whose default is one stream; LBMD_OVERLAP_SMALL
    gives it two)."""
    import os
    from workloads import globule_workload
    L = 16
    w = globule_workload(L, 1, 200, seed=8, tau=0.7, gamma=0.15)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-6, size=(3, L, L, L))
    D = rng.normal(size=3)
    D /= np.linalg.norm(D)
    outs = []
    for overlap in (False, True):
        if overlap:
            os.environ["LBMD_OVERLAP_SMALL"] = "1"
        try:
            o, _ = _gpu_grads(w, field, D, 12, 5)
        finally:
            os.environ.pop("LBMD_OVERLAP_SMALL", None)
        outs.append(o[0])
    a, b = outs
    assert a["gamma"] == b["gamma"] and a["tau"] == b["tau"], (a["gamma"], b["gamma"], a["tau"], b["tau"])
    for key in ("body_force", "x0", "v0"):
        assert bool((a[key] == b[key]).all()), key


def test_adjoint_globule_with_lj_and_bonds(O):
    """One 60-atom globule (bonds + LJ) in a 10^3 box with a random body-force field;
    12 steps in segments of 5 (three segments, the last one shorter)."""
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 12, 5, reps=2)
    _check(outs, _oracle_grads(O, w, field, D, 12, dfields), dfields, 1e-3)


def test_adjoint_tethered_ball_without_lj(O):
    """Linear dynamics (tethers + friction, no LJ) on a ragged 14 x 12 x 10 box: 20 steps in
    segments of 7."""
    from workloads import small_workload
    w = small_workload((14, 12, 10), 40, seed=5, tau=0.8, gamma=0.1, k_tether=0.05, lj=False,
                       mass=8.0)
    rng = np.random.default_rng(9)
    field = rng.normal(0, 1e-5, size=(3, 10, 12, 14))
    D = np.array([0.0, 0.8, -0.6])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 20, 7)
    _check(outs, _oracle_grads(O, w, field, D, 20, dfields), dfields, 2e-4)


def test_adjoint_segment_length_does_not_matter(O):
    """k = 1, 4 and n_steps give the same gradients (recompute is exact)."""
    from workloads import globule_workload
    L = 12
    w = globule_workload(L, 1, 80, seed=4, tau=0.75, gamma=0.2)
    rng = np.random.default_rng(1)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.36, 0.48, 0.8])
    res = [_gpu_grads(w, field, D, 9, k)[0][0] for k in (1, 4, 9)]
    for r in res[1:]:
        assert r["gamma"] == res[0]["gamma"] and r["tau"] == res[0]["tau"]
        assert bool((r["body_force"] == res[0]["body_force"]).all())


def test_autograd_function_matches_direct_call(O):
    """torch.autograd through paper_2305_05025_amd.autograd.trajectory gives the gradients of
    the direct lb_backward call, and they match the oracle."""
    import torch
    from paper_2305_05025_amd.autograd import trajectory
    from workloads import globule_workload
    L = 10
    w = globule_workload(L, 1, 60, seed=21, tau=0.7, gamma=0.15)
    rng = np.random.default_rng(3)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.6, -0.48, 0.64])
    dfields = _dfields(rng, field.shape)
    gamma = torch.tensor(0.15, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    b = torch.tensor(field.astype(np.float32), device="cuda", requires_grad=True)
    say("autograd trajectory", w.name)
    disp, v = trajectory(w, gamma, tau, b, 12, k=5)
    Dt = torch.tensor(D, dtype=torch.float32, device="cuda")
    loss = ((disp - Dt) ** 2).sum(1).mean()
    loss.backward()
    dg, dt, dbs = _oracle_grads(O, w, field, D, 12, dfields)
    assert abs(gamma.grad.item() - dg) < 1e-3 * abs(dg)
    assert abs(tau.grad.item() - dt) < 1e-3 * abs(dt)
    db = b.grad.double().cpu().numpy()
    for df, ref in zip(dfields, dbs):
        assert abs(float((db * df).sum()) - ref) < 1e-3 * abs(ref)


def _max_stencil_records(w):
    """Largest number of atom records in the 27 neighbour-list cells around an occupied cell
    (cells as wide as the cut-off allows, periodic)."""
    L = np.array(w.L)
    nc = np.floor(L / w.lj_rc).astype(int)
    x = np.mod(w.x0.astype(np.float64), L)
    c = np.minimum(np.floor(x / (L / nc)).astype(int), nc - 1)
    cnt = np.zeros(tuple(nc[::-1]), int)
    np.add.at(cnt, (c[:, 2], c[:, 1], c[:, 0]), 1)
    occ = np.argwhere(cnt > 0)
    tot = np.zeros(len(occ), int)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                tot += cnt[(occ[:, 0] + dz) % nc[2], (occ[:, 1] + dy) % nc[1], (occ[:, 2] + dx) % nc[0]]
    return int(tot.max())


def test_adjoint_dense_globule_two_staging_rounds(O):
    """A 700-atom globule in a 16^3 box: around its densest cells the 27 neighbour cells hold
    more than the 320 records one staging round takes, so the force field and its
    Hessian-vector product stage them in two rounds.  10 steps in segments of 4."""
    from workloads import globule_workload
    L = 16
    w = globule_workload(L, 1, 700, seed=8, tau=0.7, gamma=0.15)
    assert _max_stencil_records(w) > 320
    rng = np.random.default_rng(17)
    field = rng.normal(0, 1e-5, size=(3, L, L, L))
    D = np.array([0.48, 0.6, -0.64])
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 10, 4)
    _check(outs, _oracle_grads(O, w, field, D, 10, dfields), dfields, 1e-3)


def _gpu_loss(w, field, D, steps, gamma=None, tau=None):
    """The loss from the GPU forward alone (FP32 state, loss summed in FP64)."""
    from paper_2305_05025_amd import _abi as A
    from paper_2305_05025_amd.coupled import CoupledLB, params_from_workload
    p = params_from_workload(w, "f32")
    p.bf_kind = A.LB_BF_FIELD
    if gamma is not None:
        p.gamma = gamma
    if tau is not None:
        p.tau = tau
    sim = CoupledLB(p, w.x0, w.v0, w.bonds, field.astype(np.float32), charges=w.charges)
    sim.step(steps)
    d = sim.displacement().double().cpu().numpy()
    sim.close()
    return float(((d - D[None, :]) ** 2).sum(axis=1).mean())


def test_adjoint_matches_gpu_central_differences():
    """The adjoint's dL/dgamma, dL/dtau and two directional derivatives along dL/dF_ext
    against central differences of the GPU forward itself (tethered ball, linear dynamics,
    20 steps in segments of 7).  Each step h is set so that L changes by about 2e-4 L, far
    above the FP32 rounding of L, while the truncation error (order h^2) stays small: 2e-3
    relative (measured: 2e-5 for gamma, 3e-4 for tau, 1e-5 for the field directions)."""
    from workloads import small_workload
    w = small_workload((14, 12, 10), 40, seed=5, tau=0.8, gamma=0.1, k_tether=0.05, lj=False,
                       mass=8.0)
    rng = np.random.default_rng(19)
    field = rng.normal(0, 1e-5, size=(3, 10, 12, 14))
    D = np.array([0.0, 0.8, -0.6])
    dfields = [rng.normal(0, 1e-5, size=field.shape) for _ in range(2)]
    outs, _ = _gpu_grads(w, field, D, 20, 7)
    out = outs[0]
    L0 = _gpu_loss(w, field, D, 20)
    db = out["body_force"].double().cpu().numpy()
    errs = {}
    for name, g in (("gamma", out["gamma"]), ("tau", out["tau"])):
        base = w.gamma if name == "gamma" else w.tau
        h = min(1e-4 * L0 / abs(g), 1e-2 * base)
        lp = _gpu_loss(w, field, D, 20, **{name: base + h})
        lm = _gpu_loss(w, field, D, 20, **{name: base - h})
        fd = (lp - lm) / (2.0 * h)
        errs[name] = abs(g - fd) / abs(fd)
        say("FD", name, "h", h, "adjoint", g, "central difference", fd)
    for q, df in enumerate(dfields):
        g = float((db * df).sum())
        eps = 1e-4 * L0 / abs(g)
        fd = (_gpu_loss(w, field + eps * df, D, 20) - _gpu_loss(w, field - eps * df, D, 20)) / (2.0 * eps)
        errs["db%d" % q] = abs(g - fd) / abs(fd)
        say("FD body force direction", q, "eps", eps, "adjoint", g, "central difference", fd)
    say("adjoint vs GPU central differences, rel. errors", errs)
    assert max(errs.values()) < 2e-3, errs


_ORACLE_CACHE = {}


@pytest.mark.parametrize("k", [5, 20])
def test_adjoint_differentiation_workload_full_size(O, k):
    """The differentiation workload at its full size: 96^3 lattice, one 5,000-atom globule
    (bonds + Lennard-Jones), a seeded random body-force field, the workload's loss target;
    20 steps in segments of k = 5 (four segments) and k = 20 (one).  Gradients for gamma, tau
    and two directions of the body-force field against the oracle's dual numbers."""
    from workloads import make_workload
    w = make_workload(3)
    rng = np.random.default_rng(303)
    field = rng.normal(0, 1e-5, size=(3,) + tuple(w.L[::-1]))
    D = w.target_shift.astype(np.float64)
    dfields = _dfields(rng, field.shape)
    outs, _ = _gpu_grads(w, field, D, 20, k)
    if "c3" not in _ORACLE_CACHE:
        say("oracle dual-number derivatives, 96^3, 20 steps")
        _ORACLE_CACHE["c3"] = _oracle_grads(O, w, field, D, 20, dfields)
    _check(outs, _ORACLE_CACHE["c3"], dfields, 1e-3)
