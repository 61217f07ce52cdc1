"""PyTorch front-end of the coupled lattice-Boltzmann / atom library.

PyTorch supplies device memory (one uint8 workspace tensor, input/output tensors) and the
HIP stream (torch's current stream); every step of the computation runs in the library's
HIP kernels through the C interface.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _abi as A

STORAGE = {"f32": A.LB_STORE_F32, "f16": A.LB_STORE_F16, "bf16": A.LB_STORE_BF16}


def make_params(L, tau, rho0=1.0, storage="f32", n_atoms=0, mass=1.0, gamma=0.0, k_tether=0.0,
                n_bonds=0, k_bond=0.0, r0_bond=1.0, lj_eps=0.0, lj_sigma=1.0, lj_rc=2.5,
                lj_exclude_bonded=0, bf_kind=0, bf_amp=0.0, flags=0, kT=0.0, seed=0,
                coul_k=0.0, trt_magic=0.0, velocity_set=19) -> A.lb_params:
    p = A.lb_params()
    Ls = (L, L, L) if isinstance(L, int) else tuple(L)
    for k in range(3):
        p.L[k] = int(Ls[k])
    p.tau, p.rho0 = float(tau), float(rho0)
    p.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    p.n_atoms, p.mass, p.gamma, p.k_tether = int(n_atoms), float(mass), float(gamma), float(k_tether)
    p.n_bonds, p.k_bond, p.r0_bond = int(n_bonds), float(k_bond), float(r0_bond)
    p.lj_eps, p.lj_sigma, p.lj_rc = float(lj_eps), float(lj_sigma), float(lj_rc)
    p.lj_exclude_bonded, p.bf_kind, p.bf_amp = int(lj_exclude_bonded), int(bf_kind), float(bf_amp)
    p.flags = int(flags)
    p.kT = float(kT)
    p.seed[0], p.seed[1] = int(seed) & 0xffffffff, (int(seed) >> 32) & 0xffffffff
    p.coul_k = float(coul_k)
    p.trt_magic = float(trt_magic)
    p.velocity_set = int(velocity_set)
    return p


def params_from_workload(w, storage="f32", flags=0) -> A.lb_params:
    return make_params(w.L, w.tau, w.rho0, storage, w.n_atoms, w.mass, w.gamma, w.k_tether,
                       len(w.bonds), w.k_bond, w.r0_bond, w.lj_eps, w.lj_sigma, w.lj_rc,
                       w.lj_exclude_bonded, w.bf_kind, w.bf_amp, flags,
                       getattr(w, "kT", 0.0), getattr(w, "noise_seed", 0), getattr(w, "coul_k", 0.0),
                       getattr(w, "trt_magic", 0.0), getattr(w, "velocity_set", 19))


def _aligned_workspace(nbytes: int, device) -> tuple:
    raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    base = raw.data_ptr()
    off = (-base) % 256
    return raw, base + off


class CoupledLB:
    """One coupled lattice + atom system living on one GPU.

    x0, v0: [N, 3] float32 (unwrapped positions, velocities); bonds: [n_bonds, 2] int32;
    body_force: [3, nz, ny, nx] float32 when bf_kind is LB_BF_FIELD; charges: [N] float32 for
    the Coulomb term (zero when not given).
    """

    def __init__(self, params: A.lb_params, x0=None, v0=None, bonds=None, body_force=None,
                 device="cuda", stream: Optional[torch.cuda.Stream] = None, charges=None):
        self.device = torch.device(device)
        self.params = params
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.L = tuple(int(params.L[k]) for k in range(3))
        self.S = self.L[0] * self.L[1] * self.L[2]
        self.Q = 27 if int(params.velocity_set) == 27 else 19
        self.N = int(params.n_atoms)
        nbytes = A.lb_workspace_bytes(params)
        if nbytes == 0:
            # the validator's message comes from lb_init
            A.lb_init(params, 0, 0, 0, 0, 0, 0, 0)
        self._ws, ws_ptr = _aligned_workspace(nbytes, self.device)
        dev = self.device

        def t32(a, shape):
            if a is None:
                return None
            return torch.as_tensor(a, dtype=torch.float32).reshape(shape).contiguous().to(dev)

        x0t = t32(x0, (self.N, 3)) if self.N else None
        v0t = t32(v0, (self.N, 3)) if self.N else None
        bt = None
        if params.n_bonds:
            bt = torch.as_tensor(bonds, dtype=torch.int32).reshape(-1, 2).contiguous().to(dev)
        bft = t32(body_force, (3, self.S)) if params.bf_kind == A.LB_BF_FIELD else None
        ptr = lambda t: t.data_ptr() if t is not None else 0
        torch.cuda.synchronize(self.device)   # inputs were staged on torch's current stream
        with torch.cuda.stream(self.stream):
            self.ctx = A.lb_init(params, ws_ptr, nbytes, ptr(x0t), ptr(v0t), ptr(bt), ptr(bft),
                                 self.stream.cuda_stream)
        qt = None
        if charges is not None and self.N:
            qt = t32(charges, (self.N,))
            A.lb_set_charges(self.ctx, qt.data_ptr())
            self.stream.synchronize()
        self._inputs = (x0t, v0t, bt, bft, qt)   # kept alive until set-up copies are done

    @classmethod
    def from_workload(cls, w, storage="f32", device="cuda", flags=0, stream=None):
        return cls(params_from_workload(w, storage, flags), w.x0, w.v0, w.bonds, w.body_force,
                   device=device, stream=stream, charges=getattr(w, "charges", None))

    # -- stepping / observables ------------------------------------------------------------
    def step(self, n: int = 1):
        A.lb_couple_step(self.ctx, n)

    def read_fields(self):
        """(rho [nz,ny,nx], u [3,nz,ny,nx], x_unwrapped [N,3], v [N,3]) as device tensors."""
        nz, ny, nx = self.L[2], self.L[1], self.L[0]
        rho = torch.empty((nz, ny, nx), dtype=torch.float32, device=self.device)
        u = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=self.device)
        x = torch.empty((self.N, 3), dtype=torch.float32, device=self.device)
        v = torch.empty((self.N, 3), dtype=torch.float32, device=self.device)
        A.lb_read_fields(self.ctx, rho.data_ptr(), u.data_ptr(),
                         x.data_ptr() if self.N else 0, v.data_ptr() if self.N else 0)
        self.stream.synchronize()
        return rho, u, x, v

    def displacement(self):
        """X - x0 [N, 3] (the integrated displacement, full FP32 precision)."""
        d = torch.empty((self.N, 3), dtype=torch.float32, device=self.device)
        if self.N:
            A.lb_read_displacement(self.ctx, d.data_ptr())
            self.stream.synchronize()
        return d

    def populations(self):
        """Pre-collision deviations g [Q, nz, ny, nx] (float32, Q = 19 or 27)."""
        g = torch.empty((self.Q, self.L[2], self.L[1], self.L[0]), dtype=torch.float32, device=self.device)
        A.lb_read_populations(self.ctx, g.data_ptr())
        self.stream.synchronize()
        return g

    def set_populations(self, g):
        """Load pre-collision deviations g [Q, nz, ny, nx] as the current lattice state."""
        gt = torch.as_tensor(g, dtype=torch.float32).reshape(self.Q, self.S).contiguous().to(self.device)
        torch.cuda.synchronize(self.device)
        A.lb_set_populations(self.ctx, gt.data_ptr())
        self.stream.synchronize()

    def invariants(self):
        return A.lb_invariants(self.ctx)

    def check(self):
        A.lb_status_check(self.ctx)

    @property
    def step_count(self) -> int:
        return A.lb_step_count(self.ctx)

    # -- checkpoints -----------------------------------------------------------------------
    def save_state(self) -> torch.Tensor:
        n = A.lb_state_bytes(self.ctx)
        raw, ptr = _aligned_workspace(n, self.device)
        A.lb_state_save(self.ctx, ptr)
        return raw, ptr

    def load_state(self, snap):
        A.lb_state_load(self.ctx, snap[1])

    # -- gradients (checkpoint-and-recompute adjoint) --------------------------------------
    def run_checkpointed(self, n_steps: int, k: int) -> dict:
        """Advance n_steps, saving the state before every segment of k steps (the last segment
        may be shorter).  Returns the checkpoint record that backward() consumes."""
        if n_steps < 1 or k < 1:
            raise ValueError("n_steps and k must be >= 1")
        sb = A.lb_state_bytes(self.ctx)
        n_seg = -(-n_steps // k)
        raw, base = _aligned_workspace(sb * n_seg, self.device)
        for s in range(n_seg):
            A.lb_state_save(self.ctx, base + s * sb)
            A.lb_couple_step(self.ctx, min(k, n_steps - s * k))
        return {"raw": raw, "ptr": base, "n_steps": int(n_steps), "k": int(k)}

    def backward(self, ckpt: dict, dL_dX, dL_dv=None, want_body_force: bool = True,
                 want_initial: bool = True) -> dict:
        """Gradients of a loss L of the final atom state, given dL/dX and dL/dv [N, 3] there:
        dL/dgamma, dL/dtau (floats), dL/dF_ext [3, nz, ny, nx] and dL/dX, dL/dv at the first
        checkpoint (tensors, or None when not asked for)."""
        k = ckpt["k"]
        nb = A.lb_adjoint_workspace_bytes(self.ctx, k)
        if nb == 0:
            raise ValueError("backward needs atoms")
        raw, adj = _aligned_workspace(nb, self.device)
        f32 = lambda t: torch.as_tensor(t, dtype=torch.float32).reshape(self.N, 3).contiguous().to(self.device)
        dX = f32(dL_dX)
        dv = f32(dL_dv) if dL_dv is not None else None
        nz, ny, nx = self.L[2], self.L[1], self.L[0]
        db = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=self.device) if want_body_force else None
        dX0 = torch.empty((self.N, 3), dtype=torch.float32, device=self.device) if want_initial else None
        dv0 = torch.empty((self.N, 3), dtype=torch.float32, device=self.device) if want_initial else None
        ptr = lambda t: t.data_ptr() if t is not None else 0
        torch.cuda.synchronize(self.device)   # inputs were staged on torch's current stream
        dg, dt = A.lb_backward(self.ctx, ckpt["ptr"], ckpt["n_steps"], k, adj, nb, dX.data_ptr(),
                               ptr(dv), ptr(db), ptr(dX0), ptr(dv0))
        del raw
        return {"gamma": dg, "tau": dt, "body_force": db, "x0": dX0, "v0": dv0}

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            A.lb_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
