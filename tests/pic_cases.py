"""Matched oracle / GPU runs built from the same seeded synthetic inputs
(test infrastructure)."""
from __future__ import annotations

import sys

import numpy as np

import oracle


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_species(wl, parts):
    return [oracle.SpeciesState(sc.q, sc.m, sc.weight, sc.nu, p.x.copy(), p.u.copy(), p.id.copy(),
                                sc.coll_model, sc.coll_vref, getattr(sc, "binary", False))
            for sc, p in zip(wl.species, parts)]


def oracle_run(wl, parts, run_index=0):
    return oracle.OracleRun(wl.ndim, wl.n, wl.d, wl.dt, oracle_species(wl, parts), wl.seed, run_index,
                            nu_ee=getattr(wl, "nu_ee", 0.0), ee_vref=getattr(wl, "ee_vref", 0.0))


def gpu_run(wl, parts, precision, tile=0, flags=0, diag_every=0, run_index=0):
    """A GPU run with the given particles loaded from the host (ids tracked)."""
    from paper_0808_4078_amd import pic
    g, sp = pic.workload_descs(wl, precision=precision, tile=tile, diag_every=diag_every,
                               flags=flags | pic.PIC_FLAG_HOST_LOAD | pic.PIC_FLAG_TRACK_IDS, run=run_index)
    r = pic.Run(g, sp)
    for s, p in enumerate(parts):
        r.load_particles(s, p.x, p.u, p.id)
    return r


def stack(E, B):
    return np.concatenate([np.asarray(E).ravel(), np.asarray(B).ravel()])


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, (a.shape, b.shape)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def by_id(x, u, ids):
    o = np.argsort(ids)
    return x[:, o], u[:, o], ids[o]


def periodic_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)
