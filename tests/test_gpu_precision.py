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
