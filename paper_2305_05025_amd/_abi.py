"""ctypes binding of ``liblbmd.so`` (the C interface in include/lbmd.h).

Argument marshalling only: every function forwards to the entry point of the same name.
The library is loaded from this package directory; if it has not been built the import
fails loudly (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbmd.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_ESTATE, LB_ENONFINITE, LB_EOVERFLOW = range(7)
LB_STORE_F32, LB_STORE_F16, LB_STORE_BF16 = 0, 1, 2
LB_BF_NONE, LB_BF_KOLMOGOROV, LB_BF_SIGN_SHEAR, LB_BF_FIELD = 0, 1, 2, 3
LB_FLAG_CHECK_FINITE = 0x1
LB_FLAG_SINGLE_STREAM = 0x2
# lattices of at most this many sites always run on the caller's stream alone
LB_ONE_STREAM_MAX_SITES = 32768
LB_FLAG_FUSED_COUPLING = 0x4
LB_FLAG_STEP_GRAPHS = 0x8

STATUS_NAMES = {0: "LB_OK", 1: "LB_EINVAL", 2: "LB_ENOMEM", 3: "LB_EDEVICE", 4: "LB_ESTATE",
                5: "LB_ENONFINITE", 6: "LB_EOVERFLOW"}


class lb_params(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 3),
        ("tau", ctypes.c_float),
        ("rho0", ctypes.c_float),
        ("storage", ctypes.c_int32),
        ("n_atoms", ctypes.c_int32),
        ("mass", ctypes.c_float),
        ("gamma", ctypes.c_float),
        ("k_tether", ctypes.c_float),
        ("n_bonds", ctypes.c_int32),
        ("k_bond", ctypes.c_float),
        ("r0_bond", ctypes.c_float),
        ("lj_eps", ctypes.c_float),
        ("lj_sigma", ctypes.c_float),
        ("lj_rc", ctypes.c_float),
        ("lj_exclude_bonded", ctypes.c_int32),
        ("bf_kind", ctypes.c_int32),
        ("bf_amp", ctypes.c_float),
        ("flags", ctypes.c_uint32),
        ("kT", ctypes.c_float),
        ("seed", ctypes.c_uint32 * 2),
        ("coul_k", ctypes.c_float),
        ("trt_magic", ctypes.c_float),
        ("velocity_set", ctypes.c_int32),
    ]


class LBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None

# (name, restype, argtypes)
_SIGS = [
    ("lb_velocity_set", None, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_velocity_set_q", ctypes.c_int, [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_workspace_bytes", ctypes.c_size_t, [ctypes.POINTER(lb_params)]),
    ("lb_init", ctypes.c_int, [ctypes.POINTER(lb_params), ctypes.c_void_p, ctypes.c_size_t,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("lb_couple_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("lb_read_fields", ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    ("lb_read_displacement", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_read_populations", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_set_populations", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_set_charges", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_invariants", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("lb_invariants_noalloc", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_status_check", ctypes.c_int, [ctypes.c_void_p]),
    ("lb_step_count", ctypes.c_int64, [ctypes.c_void_p]),
    ("lb_state_bytes", ctypes.c_size_t, [ctypes.c_void_p]),
    ("lb_state_save", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_state_load", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_timing_begin", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    ("lb_timing_end", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    ("lb_adjoint_workspace_bytes", ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int32]),
    ("lb_backward", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("lb_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("lb_last_error", ctypes.c_char_p, [ctypes.c_void_p]),
]


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                "liblbmd.so is not built (expected at %s); run __graft_entry__.build() or "
                "python -m paper_2305_05025_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int, ctx=None):
    if status != LB_OK:
        raise LBError(status, lb_last_error(ctx))


def lb_last_error(ctx=None) -> str:
    msg = lib().lb_last_error(ctx)
    return msg.decode() if msg else ""


def lb_velocity_set():
    c = (ctypes.c_int8 * 57)()
    w = (ctypes.c_double * 19)()
    lib().lb_velocity_set(ctypes.addressof(c), ctypes.addressof(w))
    return [tuple(c[3 * i:3 * i + 3]) for i in range(19)], list(w)


def lb_velocity_set_q(q: int):
    c = (ctypes.c_int8 * (3 * 27))()
    w = (ctypes.c_double * 27)()
    st = lib().lb_velocity_set_q(int(q), ctypes.addressof(c), ctypes.addressof(w))
    if st != 0:
        raise LBError(st, lb_last_error())
    return [tuple(c[3 * i:3 * i + 3]) for i in range(q)], list(w)[:q]


def lb_workspace_bytes(p: lb_params) -> int:
    return int(lib().lb_workspace_bytes(ctypes.byref(p)))


def lb_init(p: lb_params, workspace: int, workspace_bytes: int, x0: int, v0: int, bonds: int,
            body_force: int, stream: int):
    """Pointers are integers (device addresses, 0 for NULL).  Returns the context handle."""
    out = ctypes.c_void_p()
    st = lib().lb_init(ctypes.byref(p), workspace or None, workspace_bytes, x0 or None, v0 or None,
                       bonds or None, body_force or None, stream or None, ctypes.byref(out))
    _check(st, None)
    return out


def lb_couple_step(ctx, n_steps: int):
    _check(lib().lb_couple_step(ctx, int(n_steps)), ctx)


def lb_read_fields(ctx, rho: int = 0, u: int = 0, x: int = 0, v: int = 0):
    _check(lib().lb_read_fields(ctx, rho or None, u or None, x or None, v or None), ctx)


def lb_read_displacement(ctx, d: int):
    _check(lib().lb_read_displacement(ctx, d or None), ctx)


def lb_read_populations(ctx, g: int):
    _check(lib().lb_read_populations(ctx, g or None), ctx)


def lb_set_populations(ctx, g: int):
    _check(lib().lb_set_populations(ctx, g or None), ctx)


def lb_set_charges(ctx, q: int):
    _check(lib().lb_set_charges(ctx, q or None), ctx)


def lb_invariants(ctx):
    out = (ctypes.c_double * 7)()
    _check(lib().lb_invariants(ctx, out), ctx)
    return list(out)


def lb_invariants_noalloc(ctx, out7: int):
    """Queue the 7 sums into the device buffer at out7 (FP64); asynchronous."""
    _check(lib().lb_invariants_noalloc(ctx, out7 or None), ctx)


def lb_status_check(ctx):
    _check(lib().lb_status_check(ctx), ctx)


def lb_step_count(ctx) -> int:
    return int(lib().lb_step_count(ctx))


def lb_state_bytes(ctx) -> int:
    return int(lib().lb_state_bytes(ctx))


def lb_state_save(ctx, dst: int):
    _check(lib().lb_state_save(ctx, dst or None), ctx)


def lb_state_load(ctx, src: int):
    _check(lib().lb_state_load(ctx, src or None), ctx)


def lb_timing_begin(ctx, max_steps: int):
    _check(lib().lb_timing_begin(ctx, int(max_steps)), ctx)


def lb_timing_end(ctx):
    """(sweep_ms, atom_ms, steps) summed over the timed steps."""
    out = (ctypes.c_double * 3)()
    _check(lib().lb_timing_end(ctx, out), ctx)
    return out[0], out[1], int(out[2])


def lb_adjoint_workspace_bytes(ctx, k: int) -> int:
    return int(lib().lb_adjoint_workspace_bytes(ctx, int(k)))


def lb_backward(ctx, ckpts: int, n_steps: int, k: int, adj_ws: int, adj_ws_bytes: int, dL_dX: int,
                dL_dv: int = 0, dL_db: int = 0, dL_dX0: int = 0, dL_dv0: int = 0):
    """(dL/dgamma, dL/dtau); the device outputs are written in place."""
    dg, dt = ctypes.c_double(), ctypes.c_double()
    _check(lib().lb_backward(ctx, ckpts or None, int(n_steps), int(k), adj_ws or None, int(adj_ws_bytes),
                             dL_dX or None, dL_dv or None, ctypes.byref(dg), ctypes.byref(dt),
                             dL_db or None, dL_dX0 or None, dL_dv0 or None), ctx)
    return dg.value, dt.value


def lb_destroy(ctx):
    _check(lib().lb_destroy(ctx), None)
