"""FP64 CPU oracle for the beam-plasma PIC step (test infrastructure).

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark may load this package; the product library
never does.  The numerical work lives in ``pic_oracle.c`` (plain C, FP64,
no fast-math); this module only marshals numpy arrays into it.  The
oracle shares no code with the HIP path and imports nothing from it.

The scheme (gather, relativistic Boris push, Esirkepov charge-conserving
deposit, isotropic scattering of the return-current electrons, Yee update)
is described in the header of ``pic_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


_FLAGS = ["-O3", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP, no fast-math, no FMA
    contraction; portable code, since the library travels between hosts)."""
    if force or not os.path.exists(_LIB):
        subprocess.run(["gcc", *_FLAGS, "-o", _LIB + ".tmp", _SRC, "-lm"], check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def build_native() -> list:
    """Recompile the oracle for the host this process runs on (-march=native
    added; the arithmetic is unchanged: no contraction, no fast-math, and the
    summation order is fixed by the code) and load that build.  Used for the
    CPU timing baseline.  Returns the compiler flags."""
    global _lib
    flags = _FLAGS + ["-march=native"]
    out = _LIB.replace(".so", "_native.so")
    subprocess.run(["gcc", *flags, "-o", out + ".tmp", _SRC, "-lm"], check=True)
    os.replace(out + ".tmp", out)
    _lib = None
    lib(out)
    return flags


class _Grid(C.Structure):
    _fields_ = [("ndim", C.c_int), ("n", C.c_int * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("E", C.POINTER(C.c_double) * 3), ("B", C.POINTER(C.c_double) * 3),
                ("J", C.POINTER(C.c_double) * 3), ("nu_ee", C.c_double), ("ee_vref", C.c_double)]


class _Species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double), ("nu", C.c_double),
                ("n", C.c_int64), ("x", C.POINTER(C.c_double) * 3), ("u", C.POINTER(C.c_double) * 3),
                ("id", C.POINTER(C.c_uint32)), ("model", C.c_int), ("vref", C.c_double), ("ee", C.c_int)]


class _Diag(C.Structure):
    _fields_ = [("W", C.c_double * 6), ("kinetic", C.c_double * 8), ("p_particles", C.c_double * 3),
                ("p_species", (C.c_double * 3) * 8), ("p_field", C.c_double * 3), ("collisions", C.c_int64),
                ("ee_pairs", C.c_int64)]


_lib = None


def lib(path: str | None = None):
    global _lib
    if _lib is None:
        if path is None:
            if not os.path.exists(_LIB):
                build()
            path = _LIB
        L = C.CDLL(path)
        P = C.POINTER
        dp = P(C.c_double)
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_philox2x32_10.argtypes = [P(C.c_uint32), C.c_uint32, P(C.c_uint32)]
        L.orc_collision_key.argtypes = [C.c_uint64, C.c_uint32]
        L.orc_collision_key.restype = C.c_uint32
        L.orc_gather.argtypes = [P(_Grid), dp, dp, dp]
        L.orc_boris.argtypes = [dp, dp, dp, C.c_double]
        L.orc_deposit.argtypes = [P(_Grid), dp * 3, C.c_double, dp, dp, C.c_double]
        L.orc_collision_threshold.argtypes = [C.c_double, C.c_double]
        L.orc_collision_threshold.restype = C.c_uint32
        L.orc_collide.argtypes = [dp, C.c_uint32, C.c_int64, C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_collide.restype = C.c_int
        L.orc_coulomb.argtypes = [dp, C.c_uint32, C.c_int64, C.c_uint64, C.c_uint32, C.c_double, C.c_double,
                                  C.c_double]
        L.orc_coulomb.restype = C.c_int
        L.orc_yee_b.argtypes = [P(_Grid), C.c_double]
        L.orc_yee_e.argtypes = [P(_Grid)]
        L.orc_field_energy.argtypes = [P(_Grid), dp]
        L.orc_field_momentum.argtypes = [P(_Grid), P(C.c_double)]
        L.orc_rho.argtypes = [P(_Grid), P(_Species), C.c_int, dp]
        L.orc_divergence.argtypes = [P(_Grid), dp * 3, dp]
        L.orc_step.argtypes = [P(_Grid), P(_Species), C.c_int, C.c_int64, C.c_uint64, C.c_uint32, P(_Diag)]
        L.orc_step.restype = C.c_int
        L.orc_ee_pair.argtypes = [dp, C.c_double, C.c_double, C.c_uint32, dp, C.c_double, C.c_double, C.c_double,
                                  C.c_int64, C.c_uint64, C.c_uint32, C.c_double, C.c_double, C.c_double]
        L.orc_ee_pair.restype = C.c_int
        L.orc_ee_collide.argtypes = [P(_Grid), P(_Species), C.c_int, C.c_int64, C.c_uint64, C.c_uint32]
        L.orc_ee_collide.restype = C.c_int64
        L.orc_num_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def philox2x32_10(ctr, key) -> np.ndarray:
    """Philox2x32-10 block for a 2-word counter and 1-word key."""
    c = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in ctr])
    o = (C.c_uint32 * 2)()
    lib().orc_philox2x32_10(c, int(key) & 0xFFFFFFFF, o)
    return np.array(list(o), dtype=np.uint32)


def collision_key(seed: int, run: int) -> int:
    return int(lib().orc_collision_key(seed, run))


def collision_threshold(nu: float, dt: float) -> int:
    return int(lib().orc_collision_threshold(nu, dt))


def collide(u, pid: int, step: int, seed: int, run: int, thr: int):
    """Apply the scattering draw to one momentum; returns (u_new, scattered)."""
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    hit = lib().orc_collide(_dp(uu), pid, step, seed, run, thr)
    return uu, bool(hit)


def coulomb(u, pid: int, step: int, seed: int, run: int, nu: float, vref: float, dt: float):
    """Apply one step of Coulomb small-angle scattering off the ions to one
    momentum; returns (u_new, turned)."""
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    hit = lib().orc_coulomb(_dp(uu), pid, step, seed, run, nu, vref, dt)
    return uu, bool(hit)


def ee_pair(ua, ma, wa, ida, ub, mb, wb, f, step, seed, run, nu, vref, dt):
    """One binary collision of the pair (a, b) (a first in the pair): returns
    (u_a', u_b', scattered)."""
    a = np.ascontiguousarray(ua, dtype=np.float64).copy()
    b = np.ascontiguousarray(ub, dtype=np.float64).copy()
    hit = lib().orc_ee_pair(_dp(a), ma, wa, ida, _dp(b), mb, wb, f, step, seed, run, nu, vref, dt)
    return a, b, bool(hit)


def boris(u, E, B, qmdt2: float) -> np.ndarray:
    uu = np.ascontiguousarray(u, dtype=np.float64).copy()
    e = np.ascontiguousarray(E, dtype=np.float64)
    b = np.ascontiguousarray(B, dtype=np.float64)
    lib().orc_boris(_dp(uu), _dp(e), _dp(b), qmdt2)
    return uu


@dataclass
class SpeciesState:
    """One species: constants and FP64 particle arrays (positions in c/w_p)."""
    q: float
    m: float
    w: float
    nu: float
    x: np.ndarray          # (ndim, N)
    u: np.ndarray          # (3, N)
    id: np.ndarray         # (N,) uint32
    model: int = 0         # 0: isotropic scattering at rate nu; 1: Coulomb small-angle, nu at speed vref
    vref: float = 0.0
    ee: bool = False       # takes part in the binary (pairwise) collisions

    @property
    def n(self) -> int:
        return int(self.u.shape[1])


@dataclass
class Fields:
    ndim: int
    n: tuple
    d: tuple
    dt: float
    E: np.ndarray = field(default=None)   # (3, n2, n1, n0)
    B: np.ndarray = field(default=None)
    J: np.ndarray = field(default=None)

    def __post_init__(self):
        shp = (3, self.n[2], self.n[1], self.n[0])
        if self.E is None:
            self.E = np.zeros(shp)
        if self.B is None:
            self.B = np.zeros(shp)
        if self.J is None:
            self.J = np.zeros(shp)

    def cgrid(self) -> _Grid:
        g = _Grid()
        g.ndim = self.ndim
        for a in range(3):
            g.n[a] = int(self.n[a])
            g.d[a] = float(self.d[a])
        g.dt = float(self.dt)
        for c in range(3):
            g.E[c] = _dp(self.E[c])
            g.B[c] = _dp(self.B[c])
            g.J[c] = _dp(self.J[c])
        return g


def _cspecies(sp: list[SpeciesState], ndim: int):
    arr = (_Species * len(sp))()
    for i, s in enumerate(sp):
        assert s.x.shape[0] == ndim and s.x.flags.c_contiguous and s.u.flags.c_contiguous
        c = arr[i]
        c.q, c.m, c.w, c.nu = s.q, s.m, s.w, s.nu
        c.n = s.n
        for a in range(3):
            c.x[a] = _dp(s.x[a]) if a < ndim else C.POINTER(C.c_double)()
            c.u[a] = _dp(s.u[a])
        c.id = s.id.ctypes.data_as(C.POINTER(C.c_uint32))
        c.model = int(s.model)
        c.vref = float(s.vref)
        c.ee = 1 if s.ee else 0
    return arr


class OracleRun:
    """A periodic FP64 PIC run held in numpy arrays.

    ``step(n)`` advances n full steps.  With ``diag=True`` each step returns a
    record for the time level at its start: field energies W_i = sum F_i^2 dV
    of E^n, B^n, the time-centred kinetic energy dV sum w (gamma^n - 1) per
    species, the particle and field z momentum and the number of scattering
    events in the step.
    """

    def __init__(self, ndim, n, d, dt, species: list[SpeciesState], seed: int, run: int = 0,
                 nu_ee: float = 0.0, ee_vref: float = 0.0):
        n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        d = tuple(float(v) for v in d) + (1.0,) * (3 - len(d))
        self.f = Fields(ndim, n, d, float(dt))
        self.nu_ee, self.ee_vref = float(nu_ee), float(ee_vref)
        self.species = species
        for s in species:
            s.x = np.ascontiguousarray(s.x, dtype=np.float64)
            s.u = np.ascontiguousarray(s.u, dtype=np.float64)
            s.id = np.ascontiguousarray(s.id, dtype=np.uint32)
        self.seed = int(seed)
        self.run = int(run)
        self.step_index = 0
        self._g = self.f.cgrid()
        self._g.nu_ee = self.nu_ee
        self._g.ee_vref = self.ee_vref
        self._sp = _cspecies(species, ndim)

    @property
    def ndim(self):
        return self.f.ndim

    def step(self, nsteps: int = 1, diag: bool = False):
        L = lib()
        out = []
        for _ in range(nsteps):
            d = _Diag() if diag else None
            rc = L.orc_step(C.byref(self._g), self._sp, len(self.species), self.step_index,
                            self.seed, self.run, C.byref(d) if d is not None else None)
            if rc != 0:
                raise MemoryError("oracle step failed")
            if diag:
                out.append(dict(step=self.step_index, W=np.array(d.W[:]),
                                kinetic=np.array(d.kinetic[:len(self.species)]),
                                p_particles=np.array(d.p_particles[:]),
                                p_species=np.array([d.p_species[s][:] for s in range(len(self.species))]),
                                p_field=np.array(d.p_field[:]),
                                collisions=int(d.collisions), ee_pairs=int(d.ee_pairs)))
            self.step_index += 1
        return out

    def ee_collide(self, step: int | None = None) -> int:
        """The binary-collision stage alone, at the current positions, for time
        level `step` (default: the run's current step); returns the number
        of pairs that scattered."""
        st = self.step_index if step is None else int(step)
        n = lib().orc_ee_collide(C.byref(self._g), self._sp, len(self.species), st, self.seed, self.run)
        if n < 0:
            raise MemoryError("oracle binary collisions failed")
        return int(n)

    def field_energy(self) -> np.ndarray:
        W = np.zeros(6)
        lib().orc_field_energy(C.byref(self._g), _dp(W))
        return W

    def field_momentum(self) -> np.ndarray:
        p = np.zeros(3)
        lib().orc_field_momentum(C.byref(self._g), _dp(p))
        return p

    def rho(self) -> np.ndarray:
        r = np.zeros(self.f.E.shape[1:])
        lib().orc_rho(C.byref(self._g), self._sp, len(self.species), _dp(r))
        return r

    def divergence(self, F: np.ndarray) -> np.ndarray:
        F = np.ascontiguousarray(F, dtype=np.float64)
        out = np.zeros(F.shape[1:])
        arr = (C.POINTER(C.c_double) * 3)(_dp(F[0]), _dp(F[1]), _dp(F[2]))
        lib().orc_divergence(C.byref(self._g), arr, _dp(out))
        return out

    def gather(self, x) -> tuple[np.ndarray, np.ndarray]:
        xx = np.zeros(3)
        xx[: self.ndim] = x[: self.ndim]
        E = np.zeros(3)
        B = np.zeros(3)
        lib().orc_gather(C.byref(self._g), _dp(xx), _dp(E), _dp(B))
        return E, B

    def deposit(self, qw, x0, x1, vz, J: np.ndarray | None = None) -> np.ndarray:
        """Esirkepov deposit of one move into J (a fresh zero array if None)."""
        if J is None:
            J = np.zeros_like(self.f.J)
        a0 = np.zeros(3)
        a1 = np.zeros(3)
        a0[: self.ndim] = x0[: self.ndim]
        a1[: self.ndim] = x1[: self.ndim]
        arr = (C.POINTER(C.c_double) * 3)(_dp(J[0]), _dp(J[1]), _dp(J[2]))
        lib().orc_deposit(C.byref(self._g), arr, qw, _dp(a0), _dp(a1), vz)
        return J

    def yee_b(self, h=0.5):
        lib().orc_yee_b(C.byref(self._g), h)

    def yee_e(self):
        lib().orc_yee_e(C.byref(self._g))


def num_threads() -> int:
    return int(lib().orc_num_threads())
