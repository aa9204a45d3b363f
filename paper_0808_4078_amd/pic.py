"""Python binding of libpic.so (argument marshalling only).

Every step of the PIC path runs in the HIP kernels behind the C ABI in
``include/pic.h``; this module converts arguments, allocates the
caller-owned device buffers with PyTorch and passes the current HIP stream.
It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK = 0
PIC_E_INVALID_ARG = -1
PIC_E_UNSUPPORTED = -2
PIC_E_CFL = -3
PIC_E_BUFFER_TOO_SMALL = -4
PIC_E_HIP = -5
PIC_E_STATE = -6
PIC_E_CAPACITY = -7
PIC_PREC_FP64 = 0
PIC_PREC_MIXED = 1
PIC_COLL_ISOTROPIC = 0
PIC_COLL_COULOMB = 1
PIC_FLAG_FREEZE_FIELDS = 1
PIC_FLAG_NO_COLLIDE = 2
PIC_FLAG_LATTICE_LOAD = 4
PIC_FLAG_HOST_LOAD = 8
PIC_FLAG_NO_GRAPH = 16
PIC_FLAG_TRACK_IDS = 32
PIC_FLAG_GAUSS_RESIDUAL = 64
MAX_SPECIES = 8

STATUS = {0: "PIC_OK", -1: "PIC_E_INVALID_ARG", -2: "PIC_E_UNSUPPORTED", -3: "PIC_E_CFL",
          -4: "PIC_E_BUFFER_TOO_SMALL", -5: "PIC_E_HIP", -6: "PIC_E_STATE", -7: "PIC_E_CAPACITY"}


class GridDesc(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("d", C.c_double * 3), ("dt", C.c_double),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("run", C.c_uint32),
                ("tile", C.c_int32 * 3), ("diag_every", C.c_int32), ("flags", C.c_uint32),
                ("reserve", C.c_double), ("nu_ee", C.c_double), ("ee_vref", C.c_double), ("shape", C.c_int32)]


class SpeciesDesc(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("density", C.c_double), ("ppc", C.c_int32),
                ("drift_u", C.c_double * 3), ("u_th", C.c_double), ("cancel_current_of", C.c_int32),
                ("nu_coll", C.c_double), ("coll_model", C.c_int32), ("coll_vref", C.c_double),
                ("binary", C.c_int32)]


class Sizes(C.Structure):
    _fields_ = [("particle_bytes", C.c_size_t * MAX_SPECIES), ("field_bytes", C.c_size_t),
                ("scratch_bytes", C.c_size_t), ("diag_bytes", C.c_size_t)]


class Buffers(C.Structure):
    _fields_ = [("particles", C.c_void_p * MAX_SPECIES), ("fields", C.c_void_p),
                ("scratch", C.c_void_p), ("diag", C.c_void_p)]


class Diag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("W", C.c_double * 6),
                ("kinetic", C.c_double * MAX_SPECIES), ("p_species", (C.c_double * 3) * MAX_SPECIES),
                ("p_particles", C.c_double * 3), ("p_field", C.c_double * 3), ("collisions", C.c_int64),
                ("n_particles", C.c_int64 * MAX_SPECIES), ("rebins", C.c_int64), ("gauss_resid", C.c_double),
                ("rho_dev", C.c_double), ("continuity_resid", C.c_double), ("rho_step", C.c_double),
                ("ee_pairs", C.c_int64)]

    def as_dict(self, ns: int) -> dict:
        return dict(step=int(self.step), time=float(self.time), W=np.array(self.W[:]),
                    kinetic=np.array(self.kinetic[:ns]), p_particles=np.array(self.p_particles[:]),
                    p_species=np.array([self.p_species[s][:] for s in range(ns)]),
                    p_field=np.array(self.p_field[:]), collisions=int(self.collisions),
                    n_particles=np.array(self.n_particles[:ns]), rebins=int(self.rebins),
                    gauss_resid=float(self.gauss_resid), rho_dev=float(self.rho_dev),
                    continuity_resid=float(self.continuity_resid), rho_step=float(self.rho_step),
                    ee_pairs=int(self.ee_pairs))


class RunInfo(C.Structure):
    """pic_run_info: how a run or batch enqueues its steps."""
    _fields_ = [("graph", C.c_int32), ("static_scratch", C.c_int32), ("steps_enqueued", C.c_int64),
                ("graph_launches", C.c_int64), ("direct_steps", C.c_int64), ("scratch_bytes", C.c_size_t),
                ("shape", C.c_int32), ("block_threads", C.c_int32), ("inflight", C.c_int32)]

    def as_dict(self) -> dict:
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class PicError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} -> {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None

EXPORTS = ["pic_query", "pic_init", "pic_load_particles", "pic_step", "pic_step_profiled", "pic_sync", "pic_diagnostics",
           "pic_diag_history", "pic_read_fields", "pic_write_fields", "pic_read_particles", "pic_destroy",
           "pic_status_string", "pic_last_error", "pic_info", "pic_init_static_scratch", "pic_batch_query", "pic_batch_init", "pic_batch_step",
           "pic_batch_step_profiled", "pic_batch_sync", "pic_batch_info", "pic_batch_launch_info",
           "pic_batch_diagnostics",
           "pic_batch_destroy", "pic_tune_query",
           "pic_tune", "pic_tune_shape", "pic_copy_probe", "pic_checkpoint", "pic_restore", "pic_hyb_query", "pic_hyb_init", "pic_hyb_step",
           "pic_hyb_step_profiled", "pic_hyb_sync", "pic_hyb_read_grid", "pic_hyb_read_particles",
           "pic_hyb_diag_history", "pic_hyb_last_error", "pic_hyb_destroy"]


class HybDesc(C.Structure):
    """pic_hyb_desc: the reduced quasi-neutral model's run description."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dt", C.c_double), ("nu", C.c_double), ("n0", C.c_double), ("weight", C.c_double),
                ("nparticles", C.c_int64), ("iters", C.c_int32), ("diag_every", C.c_int32),
                ("sort_every", C.c_int32), ("flags", C.c_uint32)]


class HybDiag(C.Structure):
    _fields_ = [("step", C.c_int64), ("time", C.c_double), ("beam_energy", C.c_double), ("beam_a2", C.c_double),
                ("grad_energy", C.c_double), ("a2_energy", C.c_double), ("eq7", C.c_double),
                ("W_Bperp", C.c_double), ("W_Ez", C.c_double), ("beam_pz", C.c_double), ("mean_a", C.c_double),
                ("mean_psi", C.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


def lib():
    """The loaded libpic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0808_4078_amd.build` "
                               "(there is no fallback path)")
        # libpic.so needs libamdhip64.so.7.  PyTorch bundles a HIP runtime with
        # that soname; bringing torch's runtime up first makes the library bind
        # to it, so the process holds one HIP runtime and torch's buffers and
        # streams are valid in the library.
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        L.pic_query.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, P(Sizes)]
        L.pic_init.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, P(Buffers), vp, P(vp)]
        L.pic_init_static_scratch.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, P(Buffers), vp, P(vp)]
        L.pic_load_particles.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int64]
        L.pic_step.argtypes = [vp, C.c_int32]
        L.pic_step_profiled.argtypes = [vp, C.c_int32, P(C.c_double)]
        L.pic_sync.argtypes = [vp]
        L.pic_info.argtypes = [vp, P(RunInfo)]
        L.pic_diagnostics.argtypes = [vp, P(Diag)]
        L.pic_diag_history.argtypes = [vp, P(Diag), C.c_int64, P(C.c_int64)]
        L.pic_read_fields.argtypes = [vp, vp, vp, vp]
        L.pic_write_fields.argtypes = [vp, vp, vp]
        L.pic_read_particles.argtypes = [vp, C.c_int, vp, vp, vp, C.c_int64, P(C.c_int64)]
        L.pic_destroy.argtypes = [vp]
        L.pic_checkpoint.argtypes = [vp, C.c_char_p]
        L.pic_restore.argtypes = [vp, C.c_char_p]
        L.pic_status_string.argtypes = [C.c_int]
        L.pic_status_string.restype = C.c_char_p
        L.pic_last_error.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.pic_batch_query.argtypes = [C.c_int, P(vp), P(C.c_size_t)]
        L.pic_batch_init.argtypes = [C.c_int, P(vp), vp, C.c_size_t, C.c_int32, C.c_uint32, P(vp)]
        L.pic_batch_step.argtypes = [vp, C.c_int32]
        L.pic_batch_step_profiled.argtypes = [vp, C.c_int32, P(C.c_double)]
        L.pic_batch_sync.argtypes = [vp]
        L.pic_batch_info.argtypes = [vp, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
        L.pic_batch_launch_info.argtypes = [vp, P(RunInfo)]
        L.pic_batch_diagnostics.argtypes = [vp, C.c_int, P(Diag)]
        L.pic_batch_destroy.argtypes = [vp]
        L.pic_tune_query.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, C.c_int32, P(C.c_size_t)]
        L.pic_tune.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, C.c_int32, vp, C.c_size_t, vp, C.c_int32,
                               P(C.c_int32), P(C.c_double)]
        L.pic_tune_shape.argtypes = [P(GridDesc), P(SpeciesDesc), C.c_int, C.c_int32, vp, C.c_size_t, vp,
                                     C.c_int32, P(C.c_int32), P(C.c_double)]
        L.pic_copy_probe.argtypes = [P(vp), P(vp), C.c_int, C.c_int64, C.c_int64, vp]
        L.pic_hyb_query.argtypes = [P(HybDesc), P(C.c_size_t), P(C.c_size_t)]
        L.pic_hyb_init.argtypes = [P(HybDesc), vp, C.c_size_t, vp, C.c_size_t, vp, vp, vp, vp, vp, vp, P(vp)]
        L.pic_hyb_step.argtypes = [vp, C.c_int32]
        L.pic_hyb_step_profiled.argtypes = [vp, C.c_int32, P(C.c_double)]
        L.pic_hyb_sync.argtypes = [vp]
        L.pic_hyb_read_grid.argtypes = [vp, vp, vp]
        L.pic_hyb_read_particles.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.pic_hyb_diag_history.argtypes = [vp, P(HybDiag), C.c_int32, P(C.c_int32)]
        L.pic_hyb_last_error.argtypes = [vp, C.c_char_p, C.c_size_t]
        L.pic_hyb_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _last_error(handle) -> str:
    buf = C.create_string_buffer(1024)
    lib().pic_last_error(handle, buf, 1024)
    return buf.value.decode(errors="replace")


def _check(rc: int, what: str, handle=None):
    if rc != PIC_OK:
        raise PicError(rc, what, _last_error(handle))


def make_descs(ndim, n, d, dt, species, precision=PIC_PREC_MIXED, seed=0, run=0, tile=0,
               diag_every=0, flags=0, reserve=0.0, nu_ee=0.0, ee_vref=0.0, shape=0):
    """Descriptors from plain values.  species: list of dicts with keys
    charge, mass, density, ppc, drift_u, u_th, cancel_current_of, nu_coll
    (optional: coll_model, coll_vref, binary)."""
    g = GridDesc()
    g.ndim = ndim
    for a in range(3):
        g.n[a] = int(n[a]) if a < len(n) else 1
        g.d[a] = float(d[a]) if a < len(d) else 1.0
        g.tile[a] = int(tile) if a < ndim else 0
    g.dt = float(dt)
    g.precision = int(precision)
    g.seed = int(seed)
    g.run = int(run)
    g.diag_every = int(diag_every)
    g.flags = int(flags)
    g.reserve = float(reserve)
    g.nu_ee = float(nu_ee)
    g.ee_vref = float(ee_vref)
    g.shape = int(shape)
    arr = (SpeciesDesc * len(species))()
    for i, s in enumerate(species):
        arr[i].charge = float(s.get("charge", -1.0))
        arr[i].mass = float(s.get("mass", 1.0))
        arr[i].density = float(s["density"])
        arr[i].ppc = int(s["ppc"])
        du = s.get("drift_u", (0.0, 0.0, 0.0))
        for c in range(3):
            arr[i].drift_u[c] = float(du[c])
        arr[i].u_th = float(s.get("u_th", 0.0))
        arr[i].cancel_current_of = int(s.get("cancel_current_of", -1))
        arr[i].nu_coll = float(s.get("nu_coll", 0.0))
        arr[i].coll_model = int(s.get("coll_model", PIC_COLL_ISOTROPIC))
        arr[i].coll_vref = float(s.get("coll_vref", 0.0))
        arr[i].binary = 1 if s.get("binary", False) else 0
    return g, arr


def workload_descs(wl, precision=PIC_PREC_MIXED, tile=0, diag_every=0, flags=0, run=0, reserve=0.0, shape=0):
    """Descriptors of a synthetic workload object (attributes ndim, n, d, dt,
    seed, species[name, q, m, density, ppc, drift_u, u_th, nu, cancel_current_of, and
    optionally coll_model, coll_vref])."""
    sp = [dict(charge=s.q, mass=s.m, density=s.density, ppc=s.ppc, drift_u=s.drift_u, u_th=s.u_th,
               cancel_current_of=s.cancel_current_of, nu_coll=s.nu,
               coll_model=getattr(s, "coll_model", PIC_COLL_ISOTROPIC), coll_vref=getattr(s, "coll_vref", 0.0),
               binary=getattr(s, "binary", False))
          for s in wl.species]
    if getattr(wl, "lattice", False):
        flags |= PIC_FLAG_LATTICE_LOAD
    return make_descs(wl.ndim, wl.n, wl.d, wl.dt, sp, precision, wl.seed, run, tile, diag_every, flags, reserve,
                      getattr(wl, "nu_ee", 0.0), getattr(wl, "ee_vref", 0.0), shape)


def query(grid: GridDesc, species) -> Sizes:
    out = Sizes()
    _check(lib().pic_query(C.byref(grid), species, len(species), C.byref(out)), "pic_query")
    return out


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Run:
    """A PIC run on the current CUDA (HIP) device.  Buffers are torch
    tensors owned by this object; the stream is torch's current stream."""

    def __init__(self, grid: GridDesc, species, device=None, stream=None, static_scratch: bool = False):
        """static_scratch: initialise with pic_init_static_scratch (the run
        uses the library's own scratch on its device; no scratch tensor)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required for the PIC library")
        self.torch = torch
        self.grid = grid
        self.species = species
        self.ns = len(species)
        self.ndim = int(grid.ndim)
        self.n = tuple(int(grid.n[a]) for a in range(self.ndim))
        self.cells = int(np.prod(self.n))
        self.device = torch.device(device if device is not None else "cuda")
        sz = query(grid, species)
        self.sizes = sz
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)

        # The buffers belong to the run's stream in torch's caching allocator,
        # so their memory is not handed out again before that stream's work
        # (the run's steps) is done; pic_destroy also waits for the stream.
        def alloc(nbytes):
            with torch.cuda.stream(self.stream):
                return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)

        self._bufs = [alloc(sz.particle_bytes[s]) for s in range(self.ns)]
        self._fields = alloc(sz.field_bytes)
        self._scratch = None if static_scratch else alloc(sz.scratch_bytes)
        self._diag = alloc(sz.diag_bytes)
        b = Buffers()
        for s in range(self.ns):
            b.particles[s] = self._bufs[s].data_ptr()
        b.fields = self._fields.data_ptr()
        b.scratch = None if static_scratch else self._scratch.data_ptr()
        b.diag = self._diag.data_ptr()
        h = C.c_void_p()
        init = lib().pic_init_static_scratch if static_scratch else lib().pic_init
        _check(init(C.byref(grid), species, self.ns, C.byref(b), C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "pic_init_static_scratch" if static_scratch else "pic_init")
        self.h = h

    # ------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            _check(lib().pic_destroy(self.h), "pic_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def device_bytes(self) -> int:
        scratch = int(self._scratch.numel()) if self._scratch is not None else 0
        return sum(int(t.numel()) for t in self._bufs) + int(self._fields.numel() + self._diag.numel()) + scratch

    def load_particles(self, s: int, x: np.ndarray, u: np.ndarray, ids: np.ndarray):
        x = np.ascontiguousarray(x, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        n = u.shape[1]
        assert x.shape == (self.ndim, n) and u.shape == (3, n) and ids.shape == (n,)
        _check(lib().pic_load_particles(self.h, s, _ptr(x), _ptr(u), _ptr(ids), n), "pic_load_particles", self.h)

    def step(self, n: int = 1):
        _check(lib().pic_step(self.h, int(n)), "pic_step", self.h)

    GROUPS = ("field_diag", "particle", "relayout", "reduce_j", "yee", "advance")

    def step_profiled(self, n: int) -> dict:
        """n steps with HIP events around each kernel group; returns the
        summed milliseconds per group (synchronising)."""
        ms = (C.c_double * 6)()
        _check(lib().pic_step_profiled(self.h, int(n), ms), "pic_step_profiled", self.h)
        return dict(zip(self.GROUPS, list(ms)))

    def sync(self):
        _check(lib().pic_sync(self.h), "pic_sync", self.h)

    def info(self) -> dict:
        """pic_info: graph or kernel-by-kernel steps, and the step counts."""
        i = RunInfo()
        _check(lib().pic_info(self.h, C.byref(i)), "pic_info", self.h)
        return i.as_dict()

    def diagnostics(self) -> dict:
        d = Diag()
        _check(lib().pic_diagnostics(self.h, C.byref(d)), "pic_diagnostics", self.h)
        return d.as_dict(self.ns)

    def history(self, max_records: int = 4096) -> list:
        arr = (Diag * max_records)()
        n = C.c_int64()
        _check(lib().pic_diag_history(self.h, arr, max_records, C.byref(n)), "pic_diag_history", self.h)
        return [arr[i].as_dict(self.ns) for i in range(n.value)]

    @property
    def field_shape(self):
        """(3, nz, ny, nx), nz = 1 in 2D."""
        n3 = tuple(self.n) + (1,) * (3 - len(self.n))
        return (3, n3[2], n3[1], n3[0])

    def read_fields(self):
        shp = self.field_shape
        E = np.zeros(shp)
        B = np.zeros(shp)
        J = np.zeros(shp)
        _check(lib().pic_read_fields(self.h, _ptr(E), _ptr(B), _ptr(J)), "pic_read_fields", self.h)
        return E, B, J

    def write_fields(self, E=None, B=None):
        shp = self.field_shape
        Ep = np.ascontiguousarray(E, dtype=np.float64) if E is not None else None
        Bp = np.ascontiguousarray(B, dtype=np.float64) if B is not None else None
        for a in (Ep, Bp):
            if a is not None and a.shape != shp:
                raise ValueError(f"field array shape {a.shape}, expected {shp}")
        _check(lib().pic_write_fields(self.h, _ptr(Ep) if Ep is not None else None,
                                      _ptr(Bp) if Bp is not None else None), "pic_write_fields", self.h)

    def checkpoint(self, path: str):
        _check(lib().pic_checkpoint(self.h, os.fsencode(path)), "pic_checkpoint", self.h)

    def restore(self, path: str):
        _check(lib().pic_restore(self.h, os.fsencode(path)), "pic_restore", self.h)

    def read_particles(self, s: int):
        cnt = C.c_int64()
        rc = lib().pic_read_particles(self.h, s, None, None, None, 0, C.byref(cnt))
        if rc not in (PIC_OK, -4):
            _check(rc, "pic_read_particles", self.h)
        n = cnt.value
        x = np.zeros((self.ndim, max(n, 1)))
        u = np.zeros((3, max(n, 1)))
        ids = np.zeros(max(n, 1), dtype=np.uint32)
        _check(lib().pic_read_particles(self.h, s, _ptr(x), _ptr(u), _ptr(ids), max(n, 1), C.byref(cnt)),
               "pic_read_particles", self.h)
        return x[:, :n], u[:, :n], ids[:n]


class Batch:
    """Runs stepped together (pic_batch_*).  The runs must have been created
    on one stream; the batch keeps them alive and releases them on close()."""

    GROUPS = Run.GROUPS

    def __init__(self, runs, persistent_blocks: int = 0, graph: bool = True):
        import torch
        self.runs = list(runs)
        n = len(self.runs)
        arr = (C.c_void_p * n)(*[r.h for r in self.runs])
        self._arr = arr
        nbytes = C.c_size_t()
        _check(lib().pic_batch_query(n, arr, C.byref(nbytes)), "pic_batch_query")
        self._table = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.runs[0].device)
        h = C.c_void_p()
        _check(lib().pic_batch_init(n, arr, C.c_void_p(self._table.data_ptr()), int(self._table.numel()),
                                    int(persistent_blocks), 0 if graph else PIC_FLAG_NO_GRAPH, C.byref(h)),
               "pic_batch_init")
        self.h = h
        self.stream = self.runs[0].stream

    def step(self, n: int = 1):
        _check(lib().pic_batch_step(self.h, int(n)), "pic_batch_step")

    def step_profiled(self, n: int) -> dict:
        ms = (C.c_double * 6)()
        _check(lib().pic_batch_step_profiled(self.h, int(n), ms), "pic_batch_step_profiled")
        return dict(zip(self.GROUPS, list(ms)))

    def sync(self):
        _check(lib().pic_batch_sync(self.h), "pic_batch_sync")

    def info(self) -> dict:
        pb = (C.c_int32 * 3)()
        it = (C.c_int32 * 3)()
        sh = (C.c_int32 * 3)()
        _check(lib().pic_batch_info(self.h, pb, it, sh), "pic_batch_info")
        return {"persistent_blocks": list(pb), "items": list(it), "shapes": list(sh)}

    def launch_info(self) -> dict:
        """pic_batch_launch_info: graph or kernel-by-kernel steps, and the counts."""
        i = RunInfo()
        _check(lib().pic_batch_launch_info(self.h, C.byref(i)), "pic_batch_launch_info")
        return i.as_dict()

    def diagnostics(self, run: int) -> dict:
        """The latest record of member `run` (index in the list given)."""
        d = Diag()
        _check(lib().pic_batch_diagnostics(self.h, int(run), C.byref(d)), "pic_batch_diagnostics")
        return d.as_dict(self.runs[run].ns)

    def close(self):
        if getattr(self, "h", None):
            _check(lib().pic_batch_destroy(self.h), "pic_batch_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def tune(grid: GridDesc, species, nsteps: int = 10, copies: int = 1, stream=None):
    """pic_tune: (best tile edge, {edge: ms per step}) for this configuration
    (copies > 1: a batch of that many copies), timed on the current device
    inside a temporary torch workspace."""
    import torch
    nbytes = C.c_size_t()
    _check(lib().pic_tune_query(C.byref(grid), species, len(species), int(copies), C.byref(nbytes)),
           "pic_tune_query")
    ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    best = C.c_int32()
    ms = (C.c_double * 3)()
    _check(lib().pic_tune(C.byref(grid), species, len(species), int(copies), C.c_void_p(ws.data_ptr()),
                          int(ws.numel()), C.c_void_p(st.cuda_stream), int(nsteps), C.byref(best), ms), "pic_tune")
    del ws
    return int(best.value), {e: ms[k] for k, e in enumerate((8, 16, 32)) if ms[k] >= 0}


def copy_probe(src, dst, chunk: int = 256, stream=None):
    """pic_copy_probe: copy the 4-byte-word device tensors src[a] -> dst[a]
    (equal sizes, at most 8) in one launch, a workgroup per `chunk` words of
    every array (asynchronous on the stream)."""
    import torch
    n = len(src)
    if n != len(dst) or not 1 <= n <= 8:
        raise ValueError("copy_probe: 1..8 source and destination tensors")
    words = src[0].numel() * src[0].element_size() // 4
    for t in list(src) + list(dst):
        if not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() != words * 4:
            raise ValueError("copy_probe: contiguous device tensors of equal size")
    sa = (C.c_void_p * n)(*[t.data_ptr() for t in src])
    da = (C.c_void_p * n)(*[t.data_ptr() for t in dst])
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(lib().pic_copy_probe(sa, da, n, words, int(chunk), C.c_void_p(st.cuda_stream)), "pic_copy_probe")


# pic_particle shapes (PIC_PARTICLE_SHAPES): threads per workgroup, particles in flight per lane
SHAPES = {0: (256, 2), 1: (256, 1), 2: (256, 3), 3: (512, 2), 4: (128, 2)}
# a shape other than the default is taken only when it beats the default by
# more than this fraction (the tuner's run-to-run spread is about 1%)
SHAPE_MARGIN = 0.02


def pick_shape(ms: dict, margin: float = SHAPE_MARGIN) -> int:
    """The launch shape to use from tune_shape's timings: the fastest if it
    beats shape 0 by more than `margin`, else shape 0."""
    best = min(ms, key=lambda k: ms[k])
    return best if 0 not in ms or ms[best] < (1.0 - margin) * ms[0] else 0


def tune_shape(grid: GridDesc, species, nsteps: int = 10, copies: int = 1, stream=None):
    """pic_tune_shape: (best launch shape, {shape: ms per step}) at the
    grid's tile edge (copies > 1: a batch of that many copies)."""
    import torch
    nbytes = C.c_size_t()
    _check(lib().pic_tune_query(C.byref(grid), species, len(species), int(copies), C.byref(nbytes)),
           "pic_tune_query")
    ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device="cuda")
    st = stream if stream is not None else torch.cuda.current_stream()
    best = C.c_int32()
    ms = (C.c_double * len(SHAPES))()
    _check(lib().pic_tune_shape(C.byref(grid), species, len(species), int(copies), C.c_void_p(ws.data_ptr()),
                                int(ws.numel()), C.c_void_p(st.cuda_stream), int(nsteps), C.byref(best), ms),
           "pic_tune_shape")
    del ws
    return int(best.value), {k: ms[k] for k in SHAPES if ms[k] >= 0}


# ---------------------------------------------------------------------------
# The reduced quasi-neutral model (pic_hyb_*)
def _hyb_check(rc: int, what: str, handle=None):
    if rc != PIC_OK:
        buf = C.create_string_buffer(1024)
        lib().pic_hyb_last_error(handle, buf, 1024)
        raise PicError(rc, what, buf.value.decode(errors="replace"))


def hyb_desc(wl, nparticles: int, diag_every: int = 0, sort_every: int = 0, flags: int = 0, n0: float = 1.0):
    """pic_hyb_desc of a synth.HybridWorkload with `nparticles` beam particles."""
    return HybDesc(int(wl.n[0]), int(wl.n[1]), float(wl.d[0]), float(wl.d[1]), float(wl.dt), float(wl.nu),
                   float(n0), float(wl.weight), int(nparticles), int(wl.iters), int(diag_every), int(sort_every),
                   int(flags))


class HybridRun:
    """A run of the reduced model on the current CUDA (HIP) device: torch
    buffers owned by this object, torch's current stream.  x, y, ux, uy, uz
    are host FP64 arrays of the beam particles (ids follow their order)."""

    GROUPS = ("solve", "particle", "nodes", "sort_advance")

    def __init__(self, desc: HybDesc, x, y, ux, uy, uz, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a ROCm GPU is required for the PIC library")
        self.desc = desc
        self.n = int(desc.nparticles)
        self.shape = (int(desc.ny), int(desc.nx))
        pb, gb = C.c_size_t(), C.c_size_t()
        _hyb_check(lib().pic_hyb_query(C.byref(desc), C.byref(pb), C.byref(gb)), "pic_hyb_query")
        dev = torch.device(device if device is not None else "cuda")
        self._pbuf = torch.empty(int(pb.value), dtype=torch.uint8, device=dev)
        self._gbuf = torch.empty(int(gb.value), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, ux, uy, uz)]
        for a in arrs:
            if a.shape != (self.n,):
                raise ValueError(f"particle arrays must have shape ({self.n},)")
        h = C.c_void_p()
        _hyb_check(lib().pic_hyb_init(C.byref(desc), C.c_void_p(self._pbuf.data_ptr()), int(pb.value),
                                      C.c_void_p(self._gbuf.data_ptr()), int(gb.value),
                                      C.c_void_p(self.stream.cuda_stream), *[_ptr(a) for a in arrs], C.byref(h)),
                   "pic_hyb_init")
        self.h = h

    @property
    def device_bytes(self) -> int:
        return int(self._pbuf.numel() + self._gbuf.numel())

    def step(self, n: int = 1):
        _hyb_check(lib().pic_hyb_step(self.h, int(n)), "pic_hyb_step", self.h)

    def step_profiled(self, n: int) -> dict:
        g = (C.c_double * 4)()
        _hyb_check(lib().pic_hyb_step_profiled(self.h, int(n), g), "pic_hyb_step_profiled", self.h)
        return {k: g[i] for i, k in enumerate(self.GROUPS)}

    def sync(self):
        _hyb_check(lib().pic_hyb_sync(self.h), "pic_hyb_sync", self.h)

    def read_grid(self):
        a = np.empty(self.shape)
        psi = np.empty(self.shape)
        _hyb_check(lib().pic_hyb_read_grid(self.h, _ptr(a), _ptr(psi)), "pic_hyb_read_grid", self.h)
        return a, psi

    def read_particles(self):
        """(x (2, N), u_perp (2, N), p_z (N,), id (N,)) in storage order."""
        n = self.n
        x, y, ux, uy, pz = (np.empty(n) for _ in range(5))
        ids = np.empty(n, dtype=np.uint32)
        _hyb_check(lib().pic_hyb_read_particles(self.h, _ptr(x), _ptr(y), _ptr(ux), _ptr(uy), _ptr(pz),
                                                _ptr(ids)), "pic_hyb_read_particles", self.h)
        return np.stack([x, y]), np.stack([ux, uy]), pz, ids

    def history(self, max_records: int = 4096) -> list:
        out = (HybDiag * max_records)()
        n = C.c_int32()
        _hyb_check(lib().pic_hyb_diag_history(self.h, out, int(max_records), C.byref(n)), "pic_hyb_diag_history",
                   self.h)
        return [out[i].as_dict() for i in range(n.value)]

    def close(self):
        if getattr(self, "h", None):
            _hyb_check(lib().pic_hyb_destroy(self.h), "pic_hyb_destroy", self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
