"""Initial-condition generators for the coupled LB/atom workloads.

Everything here is seeded (numpy PCG64) and quantised to float32 before it leaves, so
that the CPU oracle and the HIP path start from bit-identical inputs.

Workload families (lattice units, dx = dt = 1, atom mass ATOM_MASS):

* ``ball``: atoms uniform in a ball, placed by sequential rejection with a minimum pair
  separation, so that the Lennard-Jones repulsion at t = 0 stays bounded.
* ``globule``: compact chains.  Each globule is a self-avoiding walk on the unit simple
  cubic grid confined to a ball of radius R, grown depth-first with Warnsdorff's rule
  (step to the free neighbour that has the fewest free onward neighbours, random tie
  break) and backtracking.  Consecutive chain atoms are 1.0 apart and carry a harmonic
  bond; each globule gets one random sub-cell offset so that atoms do not sit on nodes.
  Globule centres are rejection-sampled at least 2R + r_c apart under periodic images.

The protein system of the paper (a 53k-atom glycosylated spike in a 19.2 nm box) is not
reproduced; these globules stand in for it with a protein-like compact density of about
0.6 atoms per lattice cell.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Atom mass in lattice units (rho0 * dx^3).  The configurations give none.  The explicit
# atom update is stable only while U''/m < 4 (dt = 1) along every mode; the Lennard-Jones
# curvature at contact is U''(sigma) = 456 eps / sigma^2 = 4.56, compact packings stack
# several contacts on one axis, and atoms kicked apart by compressed contacts at t = 0 can
# cross deep into the repulsive core within one step.  m = 1 diverges within a few steps;
# m = 8 still lost one 20,000-atom globule of ten at 256^3 within 20 steps; m = 16 and
# m = 32 ran every configuration (1000 / 500 / 200 steps) stably.  m = 32 (about 150 amu at
# dx = 2 Angstrom: a residue-sized coarse-grained bead) is used, for margin.
ATOM_MASS = 32.0

# Body-force kinds (integer codes shared with the C interface by convention).
BF_NONE = 0
BF_KOLMOGOROV = 1
BF_SIGN_SHEAR = 2
BF_FIELD = 3


@dataclasses.dataclass
class Workload:
    name: str
    L: tuple
    tau: float
    rho0: float
    gamma: float
    mass: float
    k_tether: float
    k_bond: float
    r0_bond: float
    lj_eps: float
    lj_sigma: float
    lj_rc: float
    lj_exclude_bonded: int
    bf_kind: int
    bf_amp: float
    steps: int
    x0: np.ndarray                      # [N, 3] float32, unwrapped positions
    v0: np.ndarray                      # [N, 3] float32
    bonds: np.ndarray                   # [n_bonds, 2] int32
    body_force: Optional[np.ndarray]    # [3, nz, ny, nx] float32 (BF_FIELD only)
    target_shift: Optional[np.ndarray]  # [3] float32: loss target displacement D
    seed: int
    kT: float = 0.0                     # thermal energy of the lattice noise (0: athermal)
    noise_seed: int = 0                 # key of the counter-based noise generator
    coul_k: float = 0.0                 # implicit-solvent Coulomb prefactor (0: off)
    charges: Optional[np.ndarray] = None  # [N] float32 atom charges
    trt_magic: float = 0.0              # two-relaxation-time collision parameter (0: BGK)
    velocity_set: int = 19              # lattice velocities: 19 (D3Q19) or 27 (D3Q27)

    @property
    def n_atoms(self) -> int:
        return int(self.x0.shape[0])

    @property
    def n_sites(self) -> int:
        return int(self.L[0]) * int(self.L[1]) * int(self.L[2])

    def params(self) -> dict:
        """Scalar parameters as a plain dict (no arrays)."""
        return {k: getattr(self, k) for k in (
            "L", "tau", "rho0", "gamma", "mass", "k_tether", "k_bond", "r0_bond",
            "lj_eps", "lj_sigma", "lj_rc", "lj_exclude_bonded", "bf_kind", "bf_amp", "kT",
            "noise_seed", "coul_k", "trt_magic", "velocity_set")}


# ---------------------------------------------------------------------------------------
# atom placement
# ---------------------------------------------------------------------------------------

def ball_atoms(n: int, radius: float, centre, d_min: float, rng: np.random.Generator,
               max_tries: int = 2_000_000) -> np.ndarray:
    """n points uniform in a ball, accepted one by one only if at least d_min from all
    previously accepted points (random sequential addition)."""
    centre = np.asarray(centre, dtype=np.float64)
    pts = np.empty((n, 3), dtype=np.float64)
    k = 0
    tries = 0
    d2min = d_min * d_min
    while k < n:
        # draw a batch of candidates uniformly in the ball
        cand = rng.uniform(-radius, radius, size=(256, 3))
        cand = cand[(cand * cand).sum(1) <= radius * radius]
        for c in cand:
            tries += 1
            if tries > max_tries:
                raise RuntimeError("ball_atoms: could not place %d atoms" % n)
            if k:
                dd = pts[:k] - c
                if (dd * dd).sum(1).min() < d2min:
                    continue
            pts[k] = c
            k += 1
            if k == n:
                break
    return pts + centre


_NB6 = ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1))


def confined_saw(n: int, radius: float, rng: np.random.Generator,
                 max_work: Optional[int] = None) -> np.ndarray:
    """Self-avoiding walk of n grid sites confined to |p| <= radius (integer offsets from
    the ball centre).  Depth-first growth with Warnsdorff's rule and backtracking."""
    r = int(np.ceil(radius)) + 1
    G = 2 * r + 1
    ax = np.arange(-r, r + 1)
    X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
    inside = (X * X + Y * Y + Z * Z) <= radius * radius
    if int(inside.sum()) < n:
        raise ValueError("confined_saw: ball of radius %g holds fewer than %d sites" % (radius, n))
    offs = [dx * G * G + dy * G + dz for dx, dy, dz in _NB6]
    max_work = max_work or 60 * n
    inside_flat = inside.ravel()
    inside_idx = np.flatnonzero(inside_flat)

    for _attempt in range(16):
        free = bytearray(inside_flat.astype(np.uint8).tobytes())
        start = int(inside_idx[rng.integers(len(inside_idx))])
        free[start] = 0
        path = [start]
        options = []   # per path entry: list of remaining candidate sites (best last)
        work = 0

        def candidates(site):
            cands = []
            for o in offs:
                s = site + o
                if free[s]:
                    onward = 0
                    for o2 in offs:
                        if free[s + o2]:
                            onward += 1
                    cands.append((onward, rng.random(), s))
            # best (fewest onward moves) last so that pop() takes it
            cands.sort(reverse=True)
            return [c[2] for c in cands]

        options.append(candidates(start))
        ok = False
        while work < max_work:
            work += 1
            if len(path) == n:
                ok = True
                break
            opts = options[-1]
            if opts:
                s = opts.pop()
                if not free[s]:
                    continue
                free[s] = 0
                path.append(s)
                options.append(candidates(s))
            else:
                # dead end: undo the last site
                s = path.pop()
                options.pop()
                free[s] = 1
                if not path:
                    break
        if ok:
            p = np.array(path, dtype=np.int64)
            i = p // (G * G)
            j = (p // G) % G
            k = p % G
            return np.stack([i - r, j - r, k - r], axis=1)
    raise RuntimeError("confined_saw: failed to grow a walk of %d sites in radius %g" % (n, radius))


def _periodic_dist(a, b, L):
    d = np.abs(a - b)
    d = np.minimum(d, L - d)
    return np.sqrt((d * d).sum(-1))


def globule_centres(n_glob: int, L, min_sep: float, rng: np.random.Generator,
                    first=None, max_tries: int = 200_000) -> np.ndarray:
    L = np.asarray(L, dtype=np.float64)
    cs = []
    if first is not None:
        cs.append(np.asarray(first, dtype=np.float64))
    tries = 0
    while len(cs) < n_glob:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("globule_centres: cannot place %d globules" % n_glob)
        c = rng.uniform(0.0, 1.0, size=3) * L
        if cs and _periodic_dist(np.array(cs), c, L).min() < min_sep:
            continue
        cs.append(c)
    return np.array(cs)


def globules(n_glob: int, n_per: int, radius: float, L, lj_rc: float,
             rng: np.random.Generator, first_centre=None):
    """Positions [n_glob*n_per, 3] (float64) and chain bonds [n_glob*(n_per-1), 2]."""
    centres = globule_centres(n_glob, L, 2.0 * radius + lj_rc, rng, first=first_centre)
    xs, bonds = [], []
    for g, c in enumerate(centres):
        walk = confined_saw(n_per, radius, rng).astype(np.float64)
        offset = rng.uniform(0.0, 1.0, size=3)
        xs.append(walk + c + offset - 0.5)
        base = g * n_per
        idx = np.arange(n_per - 1, dtype=np.int64) + base
        bonds.append(np.stack([idx, idx + 1], axis=1))
    return np.concatenate(xs), np.concatenate(bonds)


def _q32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


# ---------------------------------------------------------------------------------------
# the five benchmark configurations (lattice units)
# ---------------------------------------------------------------------------------------

def _base(name, L, tau, steps, seed, **kw):
    d = dict(name=name, L=(L, L, L), tau=tau, rho0=1.0, gamma=0.2, mass=ATOM_MASS,
             k_tether=0.0, k_bond=0.5, r0_bond=1.0, lj_eps=0.01, lj_sigma=1.0,
             lj_rc=2.5, lj_exclude_bonded=1, bf_kind=BF_NONE, bf_amp=0.0,
             steps=steps, seed=seed, body_force=None, target_shift=None)
    d.update(kw)
    return d


CONFIGS = {
    0: dict(desc="32^3 tau 0.8, 500 tethered atoms in a ball r=6, LJ all pairs, 100 steps"),
    1: dict(desc="128^3 tau 0.6, one 20k-atom globule, Kolmogorov forcing, 1000 steps"),
    2: dict(desc="256^3 tau 0.55, 10 x 20k-atom globules, 500 steps"),
    3: dict(desc="96^3 tau 0.7, one 5k-atom globule, body-force field, 200 steps"),
    4: dict(desc="384^3 tau 0.55, 50 x 20k-atom globules, sign-shear forcing, 200 steps"),
}


def globule_radius(n_per: int) -> float:
    """R = 20 for a 20k-atom globule, scaled as n^(1/3) otherwise."""
    return 20.0 * (n_per / 20000.0) ** (1.0 / 3.0)


def seeded_charges(n: int, seed: int, q0: float = 0.5) -> np.ndarray:
    """A neutral (for even n) set of charges +-q0 in seeded random order, float32."""
    q = np.where(np.arange(n) % 2 == 0, q0, -q0)
    np.random.default_rng(seed).shuffle(q)
    return q.astype(np.float32)


def make_workload(k: int, seed: Optional[int] = None) -> Workload:
    """Benchmark configuration k (0..4) with its recorded seed (= k unless overridden)."""
    seed = k if seed is None else seed
    rng = np.random.default_rng(seed)
    if k == 0:
        L = 32
        x = ball_atoms(500, 6.0, (16.0, 16.0, 16.0), 1.0, rng)
        v = rng.normal(0.0, 0.01, size=x.shape)
        d = _base("c0_32cube_ball500", L, 0.8, 100, seed, gamma=0.1, k_tether=0.05,
                  k_bond=0.0, lj_exclude_bonded=0)
        bonds = np.zeros((0, 2), np.int32)
    elif k in (1, 2, 3, 4):
        L, tau, steps, n_glob, n_per, gamma, name = {
            1: (128, 0.6, 1000, 1, 20000, 0.2, "c1_128cube_globule20k"),
            2: (256, 0.55, 500, 10, 20000, 0.2, "c2_256cube_globules200k"),
            3: (96, 0.7, 200, 1, 5000, 0.15, "c3_96cube_globule5k"),
            4: (384, 0.55, 200, 50, 20000, 0.2, "c4_384cube_globules1m"),
        }[k]
        R = globule_radius(n_per)
        first = (L / 2.0, L / 2.0, L / 2.0) if n_glob == 1 else None
        x, bonds = globules(n_glob, n_per, R, (L, L, L), 2.5, rng, first_centre=first)
        v = rng.normal(0.0, 0.01, size=x.shape)
        extra = {}
        if k == 1:
            extra = dict(bf_kind=BF_KOLMOGOROV, bf_amp=1e-6)
        elif k == 4:
            extra = dict(bf_kind=BF_SIGN_SHEAR, bf_amp=1e-6)
        elif k == 3:
            xi = rng.normal(0.0, 1.0, size=3)
            extra = dict(bf_kind=BF_FIELD, bf_amp=0.0,
                         body_force=np.zeros((3, L, L, L), np.float32),
                         target_shift=_q32(xi / np.linalg.norm(xi)))
        d = _base(name, L, tau, steps, seed, gamma=gamma, **extra)
    else:
        raise ValueError("unknown configuration %r" % (k,))
    return Workload(x0=_q32(x), v0=_q32(v), bonds=np.ascontiguousarray(bonds, np.int32), **d)


def globule_workload(L, n_glob: int, n_per: int, seed: int, tau: float = 0.6,
                     gamma: float = 0.2, steps: int = 10, name: str = "globules", **kw) -> Workload:
    """Globule workload of arbitrary size (the construction of configurations 1-4)."""
    rng = np.random.default_rng(seed)
    Ls = (L, L, L) if np.isscalar(L) else tuple(L)
    R = globule_radius(n_per)
    first = tuple(l / 2.0 for l in Ls) if n_glob == 1 else None
    x, bonds = globules(n_glob, n_per, R, Ls, 2.5, rng, first_centre=first)
    v = rng.normal(0.0, 0.01, size=x.shape)
    d = _base(name, Ls[0], tau, steps, seed, gamma=gamma)
    d["L"] = Ls
    body = kw.pop("body_force", None)
    tgt = kw.pop("target_shift", None)
    d.update(kw)
    return Workload(x0=_q32(x), v0=_q32(v), bonds=np.ascontiguousarray(bonds, np.int32),
                    body_force=body, target_shift=tgt, **{k: d[k] for k in d
                                                          if k not in ("body_force", "target_shift")})


def small_workload(L, n_atoms: int, seed: int, radius: Optional[float] = None, tau: float = 0.8,
                   gamma: float = 0.1, k_tether: float = 0.05, lj: bool = True,
                   steps: int = 10, name: str = "ball", **kw) -> Workload:
    """Ball workload of arbitrary size (the construction of configuration 0)."""
    rng = np.random.default_rng(seed)
    Ls = (L, L, L) if np.isscalar(L) else tuple(L)
    if radius is None:
        radius = (3.0 * n_atoms / (4.0 * np.pi * 0.55)) ** (1.0 / 3.0)
    centre = tuple(l / 2.0 for l in Ls)
    x = ball_atoms(n_atoms, radius, centre, 1.0, rng) if n_atoms else np.zeros((0, 3))
    v = rng.normal(0.0, 0.01, size=x.shape)
    d = _base(name, Ls[0], tau, steps, seed, gamma=gamma, k_tether=k_tether, k_bond=0.0,
              lj_exclude_bonded=0, lj_eps=0.01 if lj else 0.0)
    d["L"] = Ls
    body = kw.pop("body_force", None)
    tgt = kw.pop("target_shift", None)
    d.update(kw)
    return Workload(x0=_q32(x), v0=_q32(v), bonds=np.zeros((0, 2), np.int32),
                    body_force=body, target_shift=tgt, **{k: d[k] for k in d
                                                          if k not in ("body_force", "target_shift")})
