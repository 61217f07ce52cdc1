"""Error of each population storage format (FP32, FP16, BF16 deviations; collision in FP32)
against the FP64 oracle after many steps.

Two cases:
  * lattice only: a Kolmogorov flow from rest plus a shear wave, 48 x 48 x 16, 300 steps (no
    atoms, so no chaotic amplification: the errors are those of the storage format);
  * coupled: one 5,000-atom globule (bonds + Lennard-Jones) in a 48^3 box with the
    parameters of the 256^3 / 200,000-atom workload (tau 0.55, gamma 0.2), 200 steps.  The
    atom dynamics are chaotic, so the oracle's own FP32 run (same algorithm, float
    arithmetic) is measured beside it as the floor that rounding alone produces.
Each test prints its table (rel. L2 of u, rho - rho0, atom displacement and velocity).
"""
import numpy as np
import pytest

from gpu_util import compare, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


def _table(name, rows):
    keys = sorted({k for r in rows.values() for k in r})
    say("%s: rel. L2 against the FP64 oracle" % name)
    say("  %-12s" % "run" + "".join("%12s" % k for k in keys))
    for run, r in rows.items():
        say("  %-12s" % run + "".join("%12.3e" % r.get(k, float("nan")) for k in keys))


def test_storage_formats_lattice_only(O):
    from workloads import small_workload
    L = (48, 48, 16)
    steps = 300
    w = small_workload(L, 0, seed=7, tau=0.55, steps=0, bf_kind=1, bf_amp=1e-5)
    g0 = np.zeros(O.pop_shape(O.params_from_workload(w)))
    for y in range(L[1]):
        g0[:, :, y, :] = O.equilibrium(1.0, 0.0, [0.0, 0.0, 2e-3 * np.sin(2 * np.pi * y / L[1])])[:, None, None]
    orc = oracle_run(O, w, steps, g0=g0)
    rows = {"oracle-f32": compare(oracle_run(O, w, steps, g0=g0, precision="f32"), orc, w)}
    for fmt in ("f32", "f16", "bf16"):
        rows["gpu-" + fmt] = compare(gpu_run(w, steps, storage=fmt, g0=g0), orc, w)
    _table("lattice only, %s, %d steps" % (L, steps), rows)
    assert rows["gpu-f32"]["u"] < 1e-5
    assert rows["gpu-f16"]["u"] < 5e-3
    assert rows["gpu-bf16"]["u"] < 2e-2


def test_storage_formats_coupled_globule(O):
    from workloads import globule_workload
    steps = 200
    w = globule_workload(48, 1, 5000, seed=2, tau=0.55, gamma=0.2)
    orc = oracle_run(O, w, steps)
    rows = {"oracle-f32": compare(oracle_run(O, w, steps, precision="f32"), orc, w)}
    for fmt in ("f32", "f16", "bf16"):
        rows["gpu-" + fmt] = compare(gpu_run(w, steps, storage=fmt), orc, w)
    _table("one 5,000-atom globule in 48^3, tau 0.55, gamma 0.2, %d steps" % steps, rows)
    floor = rows["oracle-f32"]
    for k in ("u", "disp", "v"):
        assert rows["gpu-f32"][k] < max(50 * floor[k], 1e-5), (k, rows)
    assert rows["gpu-f16"]["u"] < 5e-2
    assert rows["gpu-bf16"]["u"] < 2e-1


def test_storage_formats_full_size_500_steps():
    """The 256^3 / 200,000-atom workload at its full size, read after 50 and after 500 steps.
    The oracle cannot run this (its Lennard-Jones term is O(N^2)), so the narrow formats are
    compared with the GPU's FP32 path, whose parity with the oracle is checked on smaller
    cases and on one full-size step.  An FP32 run whose initial velocities differ by one ulp
    gives the spread that the chaotic atom dynamics alone produce.  After 500 steps that
    spread is of order one and the formats' differences lie within it (gate: 1.3x the spread
    for FP16, 2x for BF16); after 50 steps the spread is still small and the formats' own
    error shows (gate: u within 1e-3 for FP16, 1e-2 for BF16; measured 2.4e-4 and 1.7e-3)."""
    import torch
    from paper_2305_05025_amd.coupled import CoupledLB, params_from_workload
    from workloads import make_workload
    w = make_workload(2)
    marks = (50, 500)

    def run(fmt, v0=None):
        say("full-size", fmt, marks, "(v0 + 1 ulp)" if v0 is not None else "")
        if v0 is None:
            sim = CoupledLB.from_workload(w, storage=fmt, device="cuda:0")
        else:
            sim = CoupledLB(params_from_workload(w, fmt), w.x0, v0, w.bonds, None, charges=w.charges)
        outs, done = {}, 0
        for m in marks:
            sim.step(m - done)
            done = m
            _, u, _, v = sim.read_fields()
            outs[m] = dict(u=u.double().cpu().numpy(), disp=sim.displacement().double().cpu().numpy(),
                           v=v.double().cpu().numpy())
        sim.close()
        torch.cuda.empty_cache()
        return outs

    rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
    ref = run("f32")
    runs = {"f32, v0 + 1 ulp": run("f32", v0=np.nextafter(w.v0.astype(np.float32), np.float32(np.inf)))}
    for fmt in ("f16", "bf16"):
        runs[fmt] = run(fmt)
    rows = {m: {k: {q: rel(r[m][q], ref[m][q]) for q in ("u", "disp", "v")} for k, r in runs.items()}
            for m in marks}
    for m in marks:
        say("256^3, 200,000 atoms, %d steps: rel. L2 against the GPU's FP32 run" % m)
        for k, r in rows[m].items():
            say("  %-16s" % k + "".join("  %s %.3e" % (q, r[q]) for q in ("u", "disp", "v")))
    spread = rows[500]["f32, v0 + 1 ulp"]
    for q in ("u", "disp", "v"):
        assert rows[500]["f16"][q] < 1.3 * spread[q] and rows[500]["bf16"][q] < 2.0 * spread[q], rows
    assert rows[50]["f16"]["u"] < 1e-3 and rows[50]["bf16"]["u"] < 1e-2, rows
