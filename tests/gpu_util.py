"""Helpers shared by the GPU parity tests: run a workload through the HIP library (via the
C interface) and through the CPU oracle, and compare."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    """Print the case being run and flush, so a failing GPU step names itself."""
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu_run(w, steps, storage="f32", g0=None, chunks=None):
    """Run a workload on cuda:0; returns observables as float64 numpy arrays."""
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB
    say("gpu_run", w.name, w.L, "atoms", w.n_atoms, "steps", steps, storage)
    sim = CoupledLB.from_workload(w, storage=storage, device="cuda:0")
    if g0 is not None:
        sim.set_populations(np.asarray(g0, np.float32))
    for n in (chunks or [steps]):
        sim.step(n)
    rho, u, x, v = sim.read_fields()
    d = sim.displacement()
    g = sim.populations()
    inv = sim.invariants()
    torch.cuda.synchronize()
    out = dict(rho=rho.double().cpu().numpy(), u=u.double().cpu().numpy(),
               x=x.double().cpu().numpy(), v=v.double().cpu().numpy(),
               d=d.double().cpu().numpy(),
               g=g.double().cpu().numpy(), inv=np.array(inv), steps=sim.step_count)
    sim.close()
    return out


def oracle_run(O, w, steps, g0=None, precision="f64"):
    p = O.params_from_workload(w)
    g = np.zeros(O.pop_shape(p)) if g0 is None else np.asarray(g0, np.float64)
    field = w.body_force
    g1, X1, V1 = O.run(p, g, w.x0, w.v0, w.x0, w.bonds, field, steps, precision=precision)
    rho, u = O.observables(p, g1, field)
    return dict(rho=rho, u=u, x=X1, v=V1, g=g1, d=X1 - w.x0.astype(np.float64),
                inv=O.invariants(p, g1, V1))


def max_rel(a, b):
    """Element by element: max |a - b| over max |b| (a wrong value at a few sites or atoms
    shows here even where it would vanish in a norm over the whole field)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return float(np.abs(a - b).max() / (mb if mb > 0 else 1.0)) if b.size else 0.0


def compare(gp, orc, w):
    """rel. L2 errors, and element-by-element errors (keys ending in _max: max |GPU - oracle|
    over max |oracle|).  The density deviation is compared through the populations g (its
    exact carrier); rho itself comes back as FP32 absolute density, whose rounding near rho0
    (2^-24 relative) is compared as such.  Atom displacement is the library's integrated
    X - x0; the unwrapped FP32 positions are compared at their own resolution."""
    r = dict(u=rel_l2(gp["u"], orc["u"]),
             rho=rel_l2(gp["rho"], orc["rho"]),
             g=rel_l2(gp["g"], orc["g"]),
             u_max=max_rel(gp["u"], orc["u"]),
             g_max=max_rel(gp["g"], orc["g"]))
    if w.n_atoms:
        r["disp"] = rel_l2(gp["d"], orc["d"])
        r["v"] = rel_l2(gp["v"], orc["v"])
        r["x"] = rel_l2(gp["x"], orc["x"])
        r["disp_max"] = max_rel(gp["d"], orc["d"])
        r["v_max"] = max_rel(gp["v"], orc["v"])
    return r
