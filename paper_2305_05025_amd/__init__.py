"""MI355X (gfx950) coupled lattice-Boltzmann / atom friction-coupling library.

The computation lives in ``liblbmd.so`` (HIP kernels behind the C interface of
include/lbmd.h); this package is its Python binding.  ``_abi`` mirrors the C entry points
one to one; ``coupled.CoupledLB`` manages a context with torch-provided memory and stream.
"""
from . import _abi  # noqa: F401
from ._abi import (  # noqa: F401
    LBError,
    lb_couple_step,
    lb_destroy,
    lb_init,
    lb_invariants,
    lb_last_error,
    lb_read_fields,
    lb_read_displacement,
    lb_read_populations,
    lb_set_populations,
    lb_state_bytes,
    lb_state_load,
    lb_state_save,
    lb_status_check,
    lb_step_count,
    lb_timing_begin,
    lb_timing_end,
    lb_velocity_set,
    lb_workspace_bytes,
    lb_params,
)


def CoupledLB(*args, **kwargs):  # noqa: N802 - lazily imports torch
    from .coupled import CoupledLB as _C
    return _C(*args, **kwargs)
