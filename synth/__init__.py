"""Seeded synthetic workloads for the beam-plasma PIC step.

This module only builds inputs: grid descriptions and FP64 initial particle
arrays.  It holds none of the PIC step's arithmetic and is shared by the
oracle-side tests and the GPU-side tests and benchmark; neither side is
imported from here.

The physical set-up follows the paper's problem statement and its 2D PIC
paragraph: an electron beam of density n_b drifting along z through plasma
electrons of density n_p = n0 - n_b whose return drift cancels the beam
current, on an immobile neutralising ion background, periodic box in the
plane transverse to the beam.  Sizes, drifts, temperatures and collision
rates of the five workloads are the synthetic stand-ins described in the
design notes (the paper prints its own parameters only for the 2D case).

Units: x in c/w_p, u = gamma v / c, densities in n0, charge e, mass m_e.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np

SEED = 0x08084078          # base seed of every workload; run r uses SEED + r


@dataclass(frozen=True)
class SpeciesCfg:
    name: str
    density: float           # n_s / n0
    ppc: int                 # macro-particles per cell
    drift_u: tuple           # (ux, uy, uz) drift, gamma*beta
    u_th: float              # Gaussian spread per component, m c
    q: float = -1.0
    m: float = 1.0
    nu: float = 0.0          # scattering rate off the ions, w_p (0 = collisionless)
    cancel_current_of: int = -1   # shift this species' u_z so the net J_z is zero
    coll_model: int = 0      # 0: isotropic scattering at rate nu; 1: Coulomb small-angle
    coll_vref: float = 0.0   # Coulomb model: speed (c) at which the momentum-transfer rate is nu
    binary: bool = False     # takes part in the binary (electron-electron) collisions of the workload

    @property
    def weight(self) -> float:
        return self.density / self.ppc


@dataclass(frozen=True)
class Workload:
    name: str
    ndim: int
    n: tuple                 # cells per axis (2 or 3 entries)
    d: tuple                 # cell size per axis, c/w_p
    dt: float                # 1/w_p
    steps: int
    species: tuple
    seed: int = SEED
    lattice: bool = False    # regular sub-lattice positions instead of random
    nu_ee: float = 0.0       # binary collisions among the `binary` species: rate at relative speed ee_vref
    ee_vref: float = 0.0

    @property
    def cells(self) -> int:
        return int(np.prod(self.n))

    @property
    def particles(self) -> int:
        return self.cells * sum(s.ppc for s in self.species)


GAMMA_BEAM = 3.0
U_BEAM = math.sqrt(GAMMA_BEAM ** 2 - 1.0)     # 2.8284271...


def beam_plasma(n, d=None, dt=0.1, steps=200, ppc=16, u_th_beam=0.1, u_th_plasma=0.01,
                nu=0.0, n_b=0.1, u_beam=U_BEAM, name="custom", seed=SEED, lattice=False,
                coll_model=0, coll_vref=0.0, nu_ee=0.0, ee_vref=0.0, binary=(True, True)) -> Workload:
    """Beam (index 0) along +z and return-current plasma (index 1); the plasma
    scatters off the ions at rate nu (coll_model 0: isotropic at a fixed
    rate; 1: Coulomb small-angle, rate nu at speed coll_vref).  nu_ee > 0:
    binary electron-electron collisions (rate nu_ee at relative speed
    ee_vref) among the species flagged in `binary` (beam, plasma)."""
    n = tuple(int(v) for v in n)
    ndim = len(n)
    if d is None:
        d = (0.2,) * ndim
    on = nu_ee > 0.0
    beam = SpeciesCfg("beam", n_b, ppc, (0.0, 0.0, u_beam), u_th_beam, binary=on and binary[0])
    plasma = SpeciesCfg("plasma", 1.0 - n_b, ppc, (0.0, 0.0, 0.0), u_th_plasma, nu=nu,
                        cancel_current_of=0, coll_model=coll_model, coll_vref=coll_vref, binary=on and binary[1])
    return Workload(name, ndim, n, tuple(d), dt, steps, (beam, plasma), seed, lattice, nu_ee, ee_vref)


# The five workloads: 2D 64^2 FP64 parity case; 2D 1024^2 64 ppc collisional
# (FP64 and mixed precision); 3D 256x256x512 8 ppc; batched 2D ensemble.
C1 = beam_plasma((64, 64), steps=200, ppc=16, u_th_beam=0.1, name="C1")
C2 = beam_plasma((1024, 1024), steps=1000, ppc=64, u_th_beam=0.3, nu=0.05, name="C2")
C3 = replace(C2, name="C3")
C4 = beam_plasma((256, 256, 512), steps=500, ppc=8, u_th_beam=0.1, name="C4")

C5_RUNS = 256
C5_SIDES = (64, 128, 256, 512)


def c5_members(nruns: int = C5_RUNS, seed: int = SEED) -> list[Workload]:
    """The ensemble: side from {64,128,256,512}, beam u_th ~ U[0.05,0.5],
    nu ~ U[0,0.1], one ppc ~ U{16..64} per run used by both species, 300
    steps; run r is seeded with seed + r."""
    rng = np.random.default_rng(seed ^ 0xC5C5)
    out = []
    for r in range(nruns):
        side = int(rng.choice(C5_SIDES))
        u_th = float(rng.uniform(0.05, 0.5))
        nu = float(rng.uniform(0.0, 0.1))
        ppc = int(rng.integers(16, 65))
        out.append(beam_plasma((side, side), steps=300, ppc=ppc, u_th_beam=u_th, nu=nu,
                               name=f"C5[{r}]", seed=seed + r))
    return out


# ---------------------------------------------------------------------------
@dataclass
class Particles:
    """FP64 particle arrays of one species: x (ndim, N) in c/w_p, u (3, N), id (N,)."""
    x: np.ndarray
    u: np.ndarray
    id: np.ndarray


def _positions(wl: Workload, sc: SpeciesCfg, rng) -> np.ndarray:
    ndim = wl.ndim
    n = wl.n
    cells = wl.cells
    # cell-major order: x fastest, then y, then z; ppc slots per cell
    idx = np.arange(cells, dtype=np.int64)
    coords = []
    rem = idx
    for a in range(ndim):
        coords.append(rem % n[a])
        rem = rem // n[a]
    x = np.empty((ndim, cells * sc.ppc))
    if wl.lattice:
        p = round(sc.ppc ** (1.0 / ndim))
        if p ** ndim != sc.ppc:
            raise ValueError("lattice load needs ppc = p^ndim")
        sub = np.stack(np.meshgrid(*([np.arange(p)] * ndim), indexing="ij"), axis=0)
        sub = sub.reshape(ndim, -1)[::-1]          # x fastest inside the cell
        frac = (sub + 0.5) / p                      # (ndim, ppc)
        for a in range(ndim):
            x[a] = ((coords[a][:, None] + frac[a][None, :]) * wl.d[a]).reshape(-1)
    else:
        for a in range(ndim):
            U = rng.random((cells, sc.ppc))
            x[a] = ((coords[a][:, None] + U) * wl.d[a]).reshape(-1)
    for a in range(ndim):
        L = n[a] * wl.d[a]
        x[a] = np.where(x[a] >= L, x[a] - L, x[a])
    return x


def net_current_z(parts: list[Particles], species) -> float:
    """sum_s q_s w_s sum_p u_z/gamma (in units of n0 e c per cell)."""
    tot = 0.0
    for p, sc in zip(parts, species):
        g = np.sqrt(1.0 + (p.u ** 2).sum(axis=0))
        tot += sc.q * sc.weight * float((p.u[2] / g).sum())
    return tot


def load(wl: Workload) -> list[Particles]:
    """Initial particles of every species.

    Each cell holds exactly ppc particles of each species with uniform
    in-cell positions (or a regular sub-lattice); each momentum component is
    drift + u_th * N(0,1); the sample mean of u_x and u_y is removed per
    species; the species named by cancel_current_of gets one common u_z
    shift, found by Newton iteration in FP64, that zeroes the realised net
    current sum q w u_z/gamma.  ids are unique across species.
    """
    rng = np.random.default_rng(wl.seed)
    parts = []
    next_id = 0
    for sc in wl.species:
        x = _positions(wl, sc, rng)
        N = x.shape[1]
        u = np.empty((3, N))
        for c in range(3):
            u[c] = sc.drift_u[c] + (sc.u_th * rng.standard_normal(N) if sc.u_th > 0 else 0.0)
        if N:
            for c in range(2):
                u[c] -= u[c].mean()
        ids = np.arange(next_id, next_id + N, dtype=np.uint64).astype(np.uint32)
        next_id += N
        parts.append(Particles(x, u, ids))
    for s, sc in enumerate(wl.species):
        if sc.cancel_current_of >= 0:
            _cancel_current(parts, wl.species, s)
    return parts


def _cancel_current(parts, species, s):
    """Newton on the common shift delta of species s's u_z."""
    sc = species[s]
    p = parts[s]
    other = 0.0
    for k, (pk, sk) in enumerate(zip(parts, species)):
        if k != s:
            g = np.sqrt(1.0 + (pk.u ** 2).sum(axis=0))
            other += sk.q * sk.weight * float((pk.u[2] / g).sum())
    u_perp2 = p.u[0] ** 2 + p.u[1] ** 2
    uz = p.u[2].copy()
    qw = sc.q * sc.weight
    # start from the cold-fluid estimate of the return drift
    n_tot = max(p.u.shape[1], 1)
    v_target = -other / (qw * n_tot)
    v_target = max(min(v_target, 0.99), -0.99)
    delta = v_target / math.sqrt(1.0 - v_target ** 2) - float(uz.mean())
    for _ in range(50):
        w = uz + delta
        g = np.sqrt(1.0 + u_perp2 + w * w)
        f = other + qw * float((w / g).sum())
        fp = qw * float(((1.0 + u_perp2) / g ** 3).sum())
        step = f / fp
        delta -= step
        if abs(step) <= 1e-16 * max(1.0, abs(delta)):
            break
    p.u[2] = uz + delta


def cold_return_drift(n_b: float = 0.1, u_beam: float = U_BEAM) -> float:
    """u_z of a cold return current that cancels a cold beam: n_b v_b + n_p v_p = 0."""
    v_b = u_beam / math.sqrt(1.0 + u_beam ** 2)
    v_p = -n_b * v_b / (1.0 - n_b)
    return v_p / math.sqrt(1.0 - v_p ** 2)


# ---------------------------------------------------------------------------
# The reduced quasi-neutral model (kinetic beam, fluid return current): its
# inputs are the beam alone; the plasma starts at rest relative to a = A_z
# (its return current is part of the model's initial solve).
@dataclass(frozen=True)
class HybridWorkload:
    name: str
    n: tuple                 # nodes per axis (nx, ny), powers of two
    d: tuple                 # node spacing, c/w_p
    dt: float                # 1/w_p
    steps: int
    n_b: float               # mean beam density / n0
    ppc: int                 # beam macro-particles per cell
    u_b: float               # beam u_z drift
    u_th: float              # Gaussian spread of each beam momentum component
    nu: float                # collision rate of the return-current plasma
    iters: int = 10          # fixed-point sweeps of the field solve per step
    seed: int = SEED
    lattice: bool = False    # regular sub-lattice (ppc must be a square)
    seed_mode: tuple = ()    # (m, xi): x -> x + xi sin(2 pi m x / L_x)

    @property
    def cells(self) -> int:
        return int(self.n[0] * self.n[1])

    @property
    def particles(self) -> int:
        return self.cells * self.ppc

    @property
    def weight(self) -> float:
        return self.n_b / self.ppc


def hybrid_load(wl: HybridWorkload):
    """Beam particles in cell-major order (x fastest), exactly ppc per cell:
    positions (2, N), transverse momenta (2, N) with the sample mean removed,
    and u_z (N,) = u_b + u_th N(0,1)."""
    rng = np.random.default_rng(wl.seed)
    nx, ny = wl.n
    dx, dy = wl.d
    cells = nx * ny
    ci = np.repeat(np.arange(cells, dtype=np.int64), wl.ppc)
    N = ci.size
    if wl.lattice:
        side = int(round(math.sqrt(wl.ppc)))
        if side * side != wl.ppc:
            raise ValueError("lattice loading needs a square ppc")
        k = np.tile(np.arange(wl.ppc), cells)
        off = np.stack([(k % side + 0.5) / side, (k // side + 0.5) / side])
    else:
        off = rng.uniform(0.0, 1.0, (2, N))
    x = np.stack([((ci % nx) + off[0]) * dx, ((ci // nx) + off[1]) * dy])
    if wl.seed_mode:
        m, xi = wl.seed_mode
        L = nx * dx
        x[0] = np.mod(x[0] + xi * np.sin(2 * math.pi * m * x[0] / L), L)
        x[0][x[0] >= L] = 0.0
    u = np.zeros((2, N))
    uz = np.full(N, float(wl.u_b))
    if wl.u_th > 0:
        u = wl.u_th * rng.standard_normal((2, N))
        u -= u.mean(axis=1, keepdims=True)
        uz = uz + wl.u_th * rng.standard_normal(N)
    return x, u, uz


# H1: the reduced-model parity case; H2: the benchmark size (the paper's
# collisional hot beam, Eqs. 1-7, on a 1024^2 grid).
H1 = HybridWorkload("H1", (64, 64), (0.2, 0.2), 0.1, 100, 0.1, 16, U_BEAM, 0.1, 0.05)
H2 = HybridWorkload("H2", (1024, 1024), (0.125, 0.125), 0.0625, 200, 0.1, 64, 0.9 / math.sqrt(1 - 0.81), 0.37, 0.15)
