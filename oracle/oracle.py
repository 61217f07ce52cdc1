"""ctypes front-end of the plain CPU oracle (``lbmd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the benchmark's CPU
baseline leg, never by the product path.  It shares no code with the HIP library.

Arrays crossing this interface are float64 (int32 for bonds), C-contiguous:
populations [Q, nz, ny, nx] (Q = 19 or 27 velocities), fields [3, nz, ny, nx], atom arrays
[N, 3].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbmd_oracle.cpp")
# LBMD_ORACLE_LIB names another build of the same source (the sanitizer test's); it is used
# as it is, never rebuilt here
LIB_OVERRIDE = os.environ.get("LBMD_ORACLE_LIB")
LIB = LIB_OVERRIDE or os.path.join(HERE, "liblbmd_oracle.so")

# The oracle is compiled without target-specific flags so that the same binary runs on any
# x86-64 host, and without floating-point contraction so that it evaluates exactly the
# expressions as written.
CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
            # independent site and atom loops run on the host's cores (every value is computed
            # by the same expression whatever the thread count)
            "-fopenmp"]


def build(force: bool = True) -> str:
    if LIB_OVERRIDE:
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


# AddressSanitizer and UndefinedBehaviorSanitizer, every finding fatal
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                  "-fno-omit-frame-pointer", "-g"]


def build_sanitized(path: str) -> str:
    """The oracle built with the sanitizers at `path` (load it with the ASan runtime
    preloaded)."""
    subprocess.check_call(["g++", *CXXFLAGS, *SANITIZE_FLAGS, SRC, "-o", path])
    return path


class OrParams(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32 * 3),
        ("n_atoms", ctypes.c_int32),
        ("n_bonds", ctypes.c_int32),
        ("lj_exclude_bonded", ctypes.c_int32),
        ("bf_kind", ctypes.c_int32),
        ("pad", ctypes.c_int32),
        ("tau", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("k_tether", ctypes.c_double),
        ("k_bond", ctypes.c_double),
        ("r0_bond", ctypes.c_double),
        ("lj_eps", ctypes.c_double),
        ("lj_sigma", ctypes.c_double),
        ("lj_rc", ctypes.c_double),
        ("bf_amp", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("seed", ctypes.c_uint32 * 2),
        ("step0", ctypes.c_int64),
        ("coul_k", ctypes.c_double),
        ("charge", ctypes.POINTER(ctypes.c_double)),
        ("trt_magic", ctypes.c_double),
        ("velocity_set", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not LIB_OVERRIDE and (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC)):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        pp = ctypes.POINTER(OrParams)
        L.or_velocity_set.argtypes = [ip, dp]
        L.or_equilibrium.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_collide_node.argtypes = [ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.or_stream.argtypes = [ip, dp, dp]
        L.or_interpolate.argtypes = [ip, dp, ctypes.c_int32, dp, dp]
        L.or_spread.argtypes = [ip, ctypes.c_int32, dp, dp, dp]
        L.or_forces.argtypes = [pp, dp, dp, ip, dp]
        L.or_forces_by_atom.argtypes = [pp, dp, dp, ip, dp]
        L.or_energy.argtypes = [pp, dp, dp, ip]
        L.or_energy.restype = ctypes.c_double
        L.or_external_force.argtypes = [pp, dp, dp]
        L.or_observables.argtypes = [pp, dp, dp, dp, dp]
        L.or_invariants.argtypes = [pp, dp, dp, dp]
        for f in (L.or_run, L.or_run_f32):
            f.argtypes = [pp, dp, dp, dp, dp, ip, dp, ctypes.c_int32]
            f.restype = ctypes.c_int
        L.or_loss_derivative.argtypes = [pp, dp, dp, dp, dp, ip, dp, dp, ctypes.c_int32,
                                         ctypes.c_int32, dp, dp, dp]
        L.or_loss_derivative.restype = ctypes.c_int
        L.or_step_sampled.argtypes = [pp, dp, dp, dp, dp, ip, dp, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int64), dp, ctypes.c_int32, ip, dp, dp]
        L.or_step_sampled.restype = ctypes.c_int
        L.or_loss.argtypes = [pp, dp, dp, dp, dp, ip, dp, dp, ctypes.c_int32, dp]
        L.or_loss.restype = ctypes.c_int
        up = ctypes.POINTER(ctypes.c_uint32)
        L.or_philox4x32_10.argtypes = [up, up, up]
        L.or_site_normals.argtypes = [up, ctypes.c_int64, ctypes.c_int64, dp]
        L.or_mode_basis.argtypes = [dp, dp]
        L.or_site_noise.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, up,
                                    ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_double]
        L.or_collide_node_trt.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp, dp]
        L.or_velocity_set_q.argtypes = [ctypes.c_int32, ip, dp]
        L.or_velocity_set_q.restype = ctypes.c_int
        L.or_equilibrium_q.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_collide_node_q.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, dp, dp, dp]
        L.or_stream_q.argtypes = [ctypes.c_int32, ip, dp, dp]
        L.or_site_noise_q.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      up, ctypes.c_int64, ctypes.c_int64, dp, ctypes.c_double]
        L.or_site_normals_n.argtypes = [up, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, dp]
        L.or_mode_basis27.argtypes = [dp, dp, ip]
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    if a is None:
        return None
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def make_params(L, tau, rho0=1.0, gamma=0.0, mass=1.0, k_tether=0.0, k_bond=0.0, r0_bond=1.0,
                lj_eps=0.0, lj_sigma=1.0, lj_rc=2.5, lj_exclude_bonded=0, bf_kind=0, bf_amp=0.0,
                n_atoms=0, n_bonds=0, kT=0.0, seed=0, step0=0, coul_k=0.0, charges=None,
                trt_magic=0.0, velocity_set=19) -> OrParams:
    p = OrParams()
    Ls = (L, L, L) if np.isscalar(L) else tuple(L)
    for a in range(3):
        p.L[a] = int(Ls[a])
    p.n_atoms, p.n_bonds = int(n_atoms), int(n_bonds)
    p.lj_exclude_bonded, p.bf_kind = int(lj_exclude_bonded), int(bf_kind)
    p.tau, p.rho0, p.gamma, p.mass = float(tau), float(rho0), float(gamma), float(mass)
    p.k_tether, p.k_bond, p.r0_bond = float(k_tether), float(k_bond), float(r0_bond)
    p.lj_eps, p.lj_sigma, p.lj_rc, p.bf_amp = float(lj_eps), float(lj_sigma), float(lj_rc), float(bf_amp)
    p.kT = float(kT)
    p.seed[0], p.seed[1] = int(seed) & 0xffffffff, (int(seed) >> 32) & 0xffffffff
    p.step0 = int(step0)
    p.coul_k = float(coul_k)
    p.trt_magic = float(trt_magic)
    p.velocity_set = int(velocity_set)
    if charges is not None:
        q = f64(charges).reshape(-1)
        assert q.size == p.n_atoms
        p._charges = q           # kept alive with the parameters
        p.charge = _d(q)
    return p


def params_from_workload(w) -> OrParams:
    return make_params(w.L, w.tau, w.rho0, w.gamma, w.mass, w.k_tether, w.k_bond, w.r0_bond,
                       w.lj_eps, w.lj_sigma, w.lj_rc, w.lj_exclude_bonded, w.bf_kind, w.bf_amp,
                       n_atoms=w.n_atoms, n_bonds=len(w.bonds), kT=getattr(w, "kT", 0.0),
                       seed=getattr(w, "noise_seed", 0), coul_k=getattr(w, "coul_k", 0.0),
                       charges=getattr(w, "charges", None), trt_magic=getattr(w, "trt_magic", 0.0),
                       velocity_set=getattr(w, "velocity_set", 19))


def n_sites(p: OrParams) -> int:
    return int(p.L[0]) * int(p.L[1]) * int(p.L[2])


def n_velocities(p: OrParams) -> int:
    return 27 if int(p.velocity_set) == 27 else 19


def pop_shape(p: OrParams):
    return (n_velocities(p), int(p.L[2]), int(p.L[1]), int(p.L[0]))


def velocity_set(q=19):
    """(c [q, 3], w [q]) of the D3Q19 or D3Q27 set."""
    c = np.zeros((q, 3), np.int32)
    w = np.zeros(q, np.float64)
    if lib().or_velocity_set_q(int(q), _i(c), _d(w)) != 0:
        raise ValueError("velocity set must be 19 or 27")
    return c, w


def equilibrium(rho0, drho, u, q=19):
    out = np.zeros(q)
    lib().or_equilibrium_q(int(q), float(rho0), float(drho), _d(f64(u)), _d(out))
    return out


def collide_node(tau, rho0, g, F, q=19, magic=0.0):
    out = np.zeros(q)
    lib().or_collide_node_q(int(q), float(tau), float(magic), float(rho0), _d(f64(g)), _d(f64(F)),
                            _d(out))
    return out


def stream(L, post):
    """Streaming of a [Q, nz, ny, nx] array (Q = 19 or 27 from its first axis)."""
    post = f64(post)
    pre = np.zeros_like(post)
    lib().or_stream_q(int(post.shape[0]), _i(i32(L)), _d(post), _d(pre))
    return pre


def interpolate(L, field, X):
    X = f64(X)
    U = np.zeros_like(X)
    lib().or_interpolate(_i(i32(L)), _d(f64(field)), int(X.shape[0]), _d(X), _d(U))
    return U


def spread(L, X, F, field=None):
    X = f64(X)
    Ls = i32(L)
    if field is None:
        field = np.zeros((3, int(Ls[2]), int(Ls[1]), int(Ls[0])))
    field = f64(field).copy()
    lib().or_spread(_i(Ls), int(X.shape[0]), _d(X), _d(f64(F)), _d(field))
    return field


def forces(p: OrParams, X, X0, bonds):
    X = f64(X)
    F = np.zeros_like(X)
    lib().or_forces(ctypes.byref(p), _d(X), _d(f64(X0)), _i(i32(bonds).reshape(-1, 2)), _d(F))
    return F


def num_threads() -> int:
    """Threads of the oracle's parallel loops."""
    return int(lib().or_num_threads())


def forces_by_atom(p: OrParams, X, X0, bonds):
    """The force field evaluated atom by atom over cell-list candidates (the coupled step's
    form); equal to forces() bit for bit."""
    X = f64(X)
    F = np.zeros_like(X)
    lib().or_forces_by_atom(ctypes.byref(p), _d(X), _d(f64(X0)), _i(i32(bonds).reshape(-1, 2)), _d(F))
    return F


def energy(p: OrParams, X, X0, bonds):
    return lib().or_energy(ctypes.byref(p), _d(f64(X)), _d(f64(X0)), _i(i32(bonds).reshape(-1, 2)))


def external_force(p: OrParams, field=None):
    out = np.zeros((3,) + pop_shape(p)[1:])
    lib().or_external_force(ctypes.byref(p), _d(f64(field)) if field is not None else None, _d(out))
    return out


def observables(p: OrParams, g, field=None):
    g = f64(g)
    rho = np.zeros(pop_shape(p)[1:])
    u = np.zeros((3,) + pop_shape(p)[1:])
    lib().or_observables(ctypes.byref(p), _d(g), _d(f64(field)) if field is not None else None,
                         _d(rho), _d(u))
    return rho, u


def invariants(p: OrParams, g, V):
    out = np.zeros(7)
    lib().or_invariants(ctypes.byref(p), _d(f64(g)), _d(f64(V).reshape(-1, 3)), _d(out))
    return out


def run(p: OrParams, g, X, V, X0, bonds, field=None, n_steps=1, precision="f64"):
    """n_steps coupled steps; returns new (g, X, V) arrays (inputs are not modified)."""
    g = f64(g).copy()
    X = f64(X).copy()
    V = f64(V).copy()
    fn = lib().or_run if precision == "f64" else lib().or_run_f32
    rc = fn(ctypes.byref(p), _d(g), _d(X), _d(V), _d(f64(X0)), _i(i32(bonds).reshape(-1, 2)),
            _d(f64(field)) if field is not None else None, int(n_steps))
    if rc != 0:
        raise RuntimeError("oracle run failed (%d)" % rc)
    return g, X, V


def step_sampled(p: OrParams, g, X, V, X0, bonds, field, site_idx, atom_idx):
    """One step; returns (g' [n_sites, Q] at site_idx, X' [n, 3], V' [n, 3] of atom_idx)."""
    site_idx = np.ascontiguousarray(site_idx, dtype=np.int64)
    atom_idx = i32(atom_idx)
    gout = np.zeros((len(site_idx), n_velocities(p)))
    Xo = np.zeros((len(atom_idx), 3))
    Vo = np.zeros((len(atom_idx), 3))
    rc = lib().or_step_sampled(
        ctypes.byref(p), _d(f64(g)), _d(f64(X)), _d(f64(V)), _d(f64(X0)),
        _i(i32(bonds).reshape(-1, 2)), _d(f64(field)) if field is not None else None,
        len(site_idx), site_idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(gout),
        len(atom_idx), _i(atom_idx), _d(Xo), _d(Vo))
    if rc != 0:
        raise RuntimeError("oracle step_sampled failed (%d)" % rc)
    return gout, Xo, Vo


def loss_derivative(p: OrParams, g, X, V, bonds, field, D, n_steps, wrt, dfield=None):
    """(loss, d loss) along gamma (wrt=0), tau (wrt=1) or a body-force direction (wrt=2)."""
    loss = ctypes.c_double()
    dl = ctypes.c_double()
    X = f64(X)
    rc = lib().or_loss_derivative(
        ctypes.byref(p), _d(f64(g)), _d(X), _d(f64(V)), _d(X), _i(i32(bonds).reshape(-1, 2)),
        _d(f64(field)) if field is not None else None, _d(f64(D)), int(n_steps), int(wrt),
        _d(f64(dfield)) if dfield is not None else None, ctypes.byref(loss), ctypes.byref(dl))
    if rc != 0:
        raise RuntimeError("oracle loss_derivative failed (%d)" % rc)
    return loss.value, dl.value


def loss(p: OrParams, g, X, V, bonds, field, D, n_steps):
    out = ctypes.c_double()
    X = f64(X)
    rc = lib().or_loss(ctypes.byref(p), _d(f64(g)), _d(X), _d(f64(V)), _d(X),
                       _i(i32(bonds).reshape(-1, 2)),
                       _d(f64(field)) if field is not None else None, _d(f64(D)), int(n_steps),
                       ctypes.byref(out))
    if rc != 0:
        raise RuntimeError("oracle loss failed (%d)" % rc)
    return out.value


def _u32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter under a 2-word key (four uint32)."""
    c, cp = _u32(ctr)
    k, kp = _u32(key)
    out, op = _u32(np.zeros(4))
    lib().or_philox4x32_10(cp, kp, op)
    return out


def site_normals(seed, step, site):
    """The 16 standard normals of one site and step."""
    k, kp = _u32([seed & 0xffffffff, (seed >> 32) & 0xffffffff])
    z = np.zeros(16)
    lib().or_site_normals(kp, int(step), int(site), _d(z))
    return z


def mode_basis():
    """(e [19 modes, 19 velocities], b [19]) of the orthogonal moment basis."""
    e = np.zeros((19, 19))
    b = np.zeros(19)
    lib().or_mode_basis(_d(e), _d(b))
    return e, b


def site_noise(kT, tau, rho, seed, step, site, trt_magic=0.0, q=19):
    """The thermal noise xi [q] added after the collision at one site (q = 19 or 27)."""
    k, kp = _u32([seed & 0xffffffff, (seed >> 32) & 0xffffffff])
    xi = np.zeros(q)
    lib().or_site_noise_q(int(q), float(kT), float(tau), float(rho), kp, int(step), int(site), _d(xi),
                          float(trt_magic))
    return xi


def site_normals_n(seed, step, site, ncalls):
    """4 * ncalls standard normals of one site and step (ncalls = 4: D3Q19, 6: D3Q27)."""
    k, kp = _u32([seed & 0xffffffff, (seed >> 32) & 0xffffffff])
    z = np.zeros(4 * ncalls)
    lib().or_site_normals_n(kp, int(step), int(site), int(ncalls), _d(z))
    return z


def mode_basis27():
    """(e [27 modes, 27 velocities], b [27], odd [27]) of the D3Q27 tensor-product basis."""
    e = np.zeros((27, 27))
    b = np.zeros(27)
    odd = np.zeros(27, np.int32)
    lib().or_mode_basis27(_d(e), _d(b), _i(odd))
    return e, b, odd


def collide_node_trt(tau, magic, rho0, g, F):
    """The two-relaxation-time collision at one node (magic = 0: BGK)."""
    out = np.zeros(19)
    lib().or_collide_node_trt(float(tau), float(magic), float(rho0), _d(f64(g)), _d(f64(F)), _d(out))
    return out


def rest_state(p: OrParams):
    """Pre-collision deviation populations of fluid at rest (all zero)."""
    return np.zeros(pop_shape(p))
