"""Conditioning of the differentiation workload's gradient (96^3 lattice, one 5,000-atom globule,
loss = mean squared distance of the atoms from the target displacement), measured with the
oracle's exact dual-number derivative dL/dgamma: how much it moves when the initial velocities
change by one FP32 ulp (the smallest change an FP32 input can carry).

Measured (dL/dgamma; relative change under v0 -> nextafter(v0, +inf)):
  20 steps 2.4e-8, 50 steps 2.8e-8, 100 steps 8.5e-9, 200 steps 4.7e-3.
So up to about 100 steps the gradient is a well-defined quantity, while over the workload's
full 200 steps the chaotic Lennard-Jones dynamics make dL/dgamma depend on the last bits of
the inputs at the half-percent level: an FP32 adjoint can match an FP64 reference there only
to about that level, and the GPU adjoint's parity is checked at 20 steps.  (With the pair
force cut off without the shift that makes it continuous at r_c, the 200-step change was
3.2e-2.)  The 200-step case takes a few minutes and runs only with LBMD_SLOW_TESTS=1.
"""
import os

import numpy as np
import pytest


def _dgamma(O, steps, bump):
    from workloads import make_workload
    w = make_workload(3)
    p = O.params_from_workload(w)
    p.bf_kind = 3
    field = np.zeros((3,) + tuple(w.L[::-1]))
    v0 = w.v0
    if bump:
        v0 = np.nextafter(v0.astype(np.float32), np.float32(np.inf))
    return O.loss_derivative(p, np.zeros(O.pop_shape(p)), w.x0.astype(np.float64),
                             v0.astype(np.float64), w.bonds, field,
                             w.target_shift.astype(np.float64), steps, 0)[1]


def test_gradient_well_conditioned_over_20_steps(O):
    a, b = _dgamma(O, 20, False), _dgamma(O, 20, True)
    rel = abs(b - a) / abs(a)
    print("20 steps: dL/dgamma %.10e, one-ulp change of v0: relative %.2e" % (a, rel))
    assert rel < 1e-6


@pytest.mark.skipif(not os.environ.get("LBMD_SLOW_TESTS"), reason="a few minutes on 8 cores; "
                    "set LBMD_SLOW_TESTS=1")
def test_gradient_ill_conditioned_over_200_steps(O):
    a, b = _dgamma(O, 200, False), _dgamma(O, 200, True)
    rel = abs(b - a) / abs(a)
    print("200 steps: dL/dgamma %.10e, one-ulp change of v0: relative %.2e" % (a, rel))
    assert rel > 1e-3
