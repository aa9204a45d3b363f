"""Tile-edge and launch-shape choice for ensembles of runs.

The tile edge fixes the particles one workgroup of the particle kernel owns
(ppc * edge^ndim) and its LDS footprint; the best edge depends on the grid
size (work items per run) and the particle load.  The timing itself is the
library's ``pic_tune`` (fresh device-loaded runs, graph-replayed steps); this
module groups the members of an ensemble into classes of equal grid and
similar load, tunes one representative per class, and keeps the answers in a
JSON cache keyed by the class.

Inside a large ensemble the device is full whatever one member's tile
count, so what decides is the cost per particle at saturation, not the
latency of a member alone (alone, a small grid prefers small tiles only
because they give more workgroups).  The representative is therefore timed
as a batch of enough copies to hold about SATURATION particles.

``choose_launch`` adds the particle kernel's launch shape (threads per
workgroup and particles in flight per lane, ``pic.SHAPES``): each class's
representative is timed in every shape at its chosen edge
(``pic_tune_shape``), and since the members of one tile edge share one
particle kernel in a batch, each edge takes the shape that wins for the
most members at that edge.  A class takes a shape other than the default
only when it beats the default by more than ``pic.SHAPE_MARGIN``.
"""
from __future__ import annotations

import json
import os

from . import pic

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_0808_4078_amd", "tiles.json")
SATURATION = 1 << 25          # particles that keep every compute unit busy
MAX_COPIES = 128


def load_band(ppc_total: int) -> int:
    """Particle-load band of a run: total particles per cell over species,
    rounded to bands of 32."""
    return max(1, (int(ppc_total) + 31) // 32)


def class_key(wl, precision: int, saturate: bool) -> str:
    ppc = sum(s.ppc for s in wl.species)
    mode = "sat" if saturate else "alone"
    return f"d{wl.ndim}-n{'x'.join(str(v) for v in wl.n[:wl.ndim])}-band{load_band(ppc)}-p{precision}-{mode}"


def copies_for(wl, saturate: bool) -> int:
    if not saturate:
        return 1
    return int(min(MAX_COPIES, max(1, -(-SATURATION // wl.particles))))


def _read(path):
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _write(path, data):
    if not path:
        return
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose_tiles(workloads, precision=pic.PIC_PREC_MIXED, nsteps: int = 10, cache_path=DEFAULT_CACHE,
                 log=None, saturate: bool = True):
    """Tile edge for every workload (saturate=True: for stepping them in one
    large batch; False: for stepping each alone).  Returns (tiles, report)
    where report maps each class key to {"tile", "ms", "copies",
    "representative", "members", "cached"}."""
    cache = _read(cache_path)
    classes = {}
    for i, wl in enumerate(workloads):
        classes.setdefault(class_key(wl, precision, saturate), []).append(i)
    report = {}
    dirty = False
    for key, idx in sorted(classes.items()):
        # representative: the member with the median particle load of the class
        idx_sorted = sorted(idx, key=lambda i: sum(s.ppc for s in workloads[i].species))
        rep = idx_sorted[len(idx_sorted) // 2]
        if key in cache and "tile" in cache[key]:
            ent = dict(cache[key])
            ent["cached"] = True
        else:
            g, sp = pic.workload_descs(workloads[rep], precision=precision)
            copies = copies_for(workloads[rep], saturate)
            best, ms = pic.tune(g, sp, nsteps=nsteps, copies=copies)
            ent = {"tile": best, "ms": {str(k): v for k, v in ms.items()}, "copies": copies, "cached": False}
            cache[key] = {"tile": best, "ms": ent["ms"], "copies": copies}
            dirty = True
            if log:
                log(f"autotune {key}: tile {best} over {copies} copies "
                    f"({', '.join(f'{k}: {v:.3f} ms' for k, v in ms.items())})")
        ent["representative"] = rep
        ent["members"] = len(idx)
        report[key] = ent
    if dirty:
        _write(cache_path, cache)
    tiles = [0] * len(workloads)
    for key, idx in classes.items():
        for i in idx:
            tiles[i] = int(report[key]["tile"])
    return tiles, report


def choose_launch(workloads, precision=pic.PIC_PREC_MIXED, nsteps: int = 10, cache_path=DEFAULT_CACHE,
                  log=None, saturate: bool = True):
    """Tile edge and launch shape for every workload.  Returns (tiles,
    shapes, report): report as choose_tiles, each class entry also holding
    "shape" (its own choice), "shape_ms" and "shape_cached", and
    report["_edges"] mapping each edge in use to the shape applied to it."""
    tiles, report = choose_tiles(workloads, precision, nsteps, cache_path, log, saturate)
    cache = _read(cache_path)
    classes = {}
    for i, wl in enumerate(workloads):
        classes.setdefault(class_key(wl, precision, saturate), []).append(i)
    dirty = False
    for key, idx in sorted(classes.items()):
        ent = report[key]
        skey = f"{key}-t{ent['tile']}-shape"
        if skey in cache and "shape" in cache[skey]:
            ent["shape"] = int(cache[skey]["shape"])
            ent["shape_ms"] = dict(cache[skey]["ms"])
            ent["shape_cached"] = True
            continue
        rep = ent["representative"]
        g, sp = pic.workload_descs(workloads[rep], precision=precision, tile=int(ent["tile"]))
        copies = copies_for(workloads[rep], saturate)
        _, ms = pic.tune_shape(g, sp, nsteps=nsteps, copies=copies)
        best = pic.pick_shape(ms)
        ent["shape"] = best
        ent["shape_ms"] = {str(k): v for k, v in ms.items()}
        ent["shape_cached"] = False
        cache[skey] = {"shape": best, "ms": ent["shape_ms"]}
        dirty = True
        if log:
            log(f"autotune {key}: shape {best} {pic.SHAPES[best]} at tile {ent['tile']} "
                f"({', '.join(f'{k}: {v:.3f} ms' for k, v in ms.items())})")
    if dirty:
        _write(cache_path, cache)
    # one shape per edge: the one whose classes hold the most members
    votes = {}
    for key, idx in classes.items():
        e = report[key]
        votes.setdefault(int(e["tile"]), {}).setdefault(int(e["shape"]), 0)
        votes[int(e["tile"])][int(e["shape"])] += len(idx)
    edge_shape = {t: max(sorted(v), key=lambda k: v[k]) for t, v in votes.items()}
    report["_edges"] = {str(t): sh for t, sh in sorted(edge_shape.items())}
    shapes = [edge_shape[t] for t in tiles]
    return tiles, shapes, report
