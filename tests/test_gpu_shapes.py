"""The particle kernel's launch shapes (threads per workgroup x particles in
flight per lane, pic_grid_desc.shape) and their tuner, through the C ABI.

A shape changes which lanes process which particles and in what order the
stayers are written back, never a particle's arithmetic, and the tile
current is an FP64 sum of FP32 terms (exact in any order, nearly always), so
every shape must step the same state: particles by id and the fields are
compared with the default shape's run, and, for a host-loaded run, with the
oracle."""
import numpy as np
import pytest

import synth
from pic_cases import by_id, log, oracle_run, rel_err, stack

pytestmark = pytest.mark.gpu

SHAPES = (1, 2, 3, 4)


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _run(pic, wl, shape, tile, coulomb=False):
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=tile, diag_every=5, shape=shape,
                               flags=pic.PIC_FLAG_TRACK_IDS)
    return pic.Run(g, sp)


def _same_state(a, b, ns, bar):
    Ea, Ba, Ja = a.read_fields()
    Eb, Bb, Jb = b.read_fields()
    ef = rel_err(stack(Ea, Ba), stack(Eb, Bb))
    worst = 0.0
    for s in range(ns):
        xa, ua, ia = by_id(*a.read_particles(s))
        xb, ub, ib = by_id(*b.read_particles(s))
        assert np.array_equal(ia, ib)
        worst = max(worst, float(np.max(np.abs(xa - xb))), float(np.max(np.abs(ua - ub))))
    ha, hb = a.history(), b.history()
    assert [r["step"] for r in ha] == [r["step"] for r in hb]
    for ra, rb in zip(ha, hb):
        assert ra["collisions"] == rb["collisions"]
        assert np.array_equal(ra["n_particles"], rb["n_particles"])
    assert ef < bar and worst < bar, (ef, worst)
    return ef, worst


@pytest.mark.parametrize("case", ["2d-t16", "2d-t8-coulomb", "2d-t32", "3d"])
def test_every_shape_steps_the_default_state(pic, case):
    """2D (tiles 8, 16, 32; isotropic and Coulomb scattering) and 3D: 25
    steps in every shape against shape 0, particles by id and fields."""
    log(f"case shapes {case}")
    if case == "3d":
        wl, tile = synth.beam_plasma((16, 16, 32), ppc=4, u_th_beam=0.2, nu=0.05, name="sh3d"), 8
    elif case == "2d-t8-coulomb":
        wl = synth.beam_plasma((64, 64), ppc=16, u_th_beam=0.3, nu=0.05, coll_model=pic.PIC_COLL_COULOMB,
                               coll_vref=0.1, name="sh2c")
        tile = 8
    else:
        tile = 16 if case == "2d-t16" else 32
        wl = synth.beam_plasma((64, 64), ppc=24, u_th_beam=0.3, nu=0.05, name="sh2")
    base = _run(pic, wl, 0, tile)
    base.step(25)
    base.sync()
    info = base.info()
    assert (info["shape"], info["block_threads"], info["inflight"]) == (0, 256, 2)
    for s in SHAPES:
        r = _run(pic, wl, s, tile)
        r.step(25)
        r.sync()
        info = r.info()
        assert (info["shape"], info["block_threads"], info["inflight"]) == (s, *pic.SHAPES[s])
        assert info["graph"] == 1 and info["graph_launches"] == 25
        ef, worst = _same_state(r, base, len(wl.species), 1e-5)
        log(f"  shape {s} {pic.SHAPES[s]}: fields {ef:.1e}, particles {worst:.1e}")
        r.close()
    base.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_shape_against_oracle(pic, shape):
    """A host-loaded mixed run in each shape against the FP64 oracle (C1
    parity bar of the mixed path, 1e-3; 60 steps)."""
    log(f"case shape {shape} vs oracle")
    wl = synth.beam_plasma((64, 64), ppc=16, u_th_beam=0.1, nu=0.05, name="sh-orc")
    parts = synth.load(wl)
    gp, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=16, shape=shape,
                                flags=pic.PIC_FLAG_HOST_LOAD | pic.PIC_FLAG_TRACK_IDS)
    r = pic.Run(gp, sp)
    for s, p in enumerate(parts):
        r.load_particles(s, p.x, p.u, p.id)
    orc = oracle_run(wl, parts)
    r.step(60)
    orc.step(60)
    r.sync()
    E, B, _ = r.read_fields()
    err = rel_err(stack(E, B), stack(orc.f.E, orc.f.B))
    log(f"  fields vs oracle {err:.2e}")
    assert err < 1e-3
    r.close()


def test_tune_shape(pic):
    """pic_tune_shape times every shape in mixed precision (shape 0 only in
    FP64) and returns the fastest."""
    log("case tune shape")
    wl = synth.beam_plasma((128, 128), ppc=16, name="tune-shape")
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=16)
    best, ms = pic.tune_shape(g, sp, nsteps=4)
    log("  " + ", ".join(f"{k}: {v:.3f} ms" for k, v in ms.items()) + f" -> {best}")
    assert set(ms) == set(pic.SHAPES) and all(v > 0 for v in ms.values())
    assert ms[best] == min(ms.values())
    best, ms = pic.tune_shape(g, sp, nsteps=3, copies=3)
    assert set(ms) == set(pic.SHAPES) and ms[best] == min(ms.values())
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_FP64, tile=16)
    best, ms = pic.tune_shape(g, sp, nsteps=3)
    assert best == 0 and set(ms) == {0}


def test_batch_groups_take_their_shapes(pic):
    """Members of tile edge 8 in shape 2 and of edge 16 in shape 3 in one
    batch, each against its twin stepped alone; members of one edge with
    different shapes are refused."""
    log("case batch shapes")
    cfg = [((32, 32), 8, 2), ((64, 64), 16, 3), ((64, 32), 8, 2), ((48, 48), 16, 3)]

    def runs():
        out = []
        for i, (n, t, s) in enumerate(cfg):
            wl = synth.beam_plasma(n, ppc=16, u_th_beam=0.2, nu=0.05, name=f"bs{i}", seed=synth.SEED + 400 + i)
            g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=t, diag_every=5, shape=s,
                                       flags=pic.PIC_FLAG_TRACK_IDS)
            out.append(pic.Run(g, sp))
        return out
    alone, members = runs(), runs()
    batch = pic.Batch(members)
    assert batch.info()["shapes"] == [2, 3, -1]
    batch.step(20)
    for r in alone:
        r.step(20)
    batch.sync()
    for r in alone:
        r.sync()
    for m, r in zip(members, alone):
        ef, worst = _same_state(m, r, 2, 1e-5)
        log(f"  member fields {ef:.1e}, particles {worst:.1e}")
    batch.close()
    for r in alone + members:
        r.close()
    wl = synth.beam_plasma((32, 32), ppc=8, name="bs-x")
    mixed = []
    for s in (0, 1):
        g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=8, shape=s)
        mixed.append(pic.Run(g, sp))
    with pytest.raises(pic.PicError) as e:
        pic.Batch(mixed)
    assert e.value.code == pic.PIC_E_INVALID_ARG
    for r in mixed:
        r.close()


def test_choose_launch_and_cache(pic, tmp_path):
    """autotune.choose_launch: a tile edge and a shape per member, one shape
    per edge, both kept in the cache."""
    log("case choose_launch")
    from paper_0808_4078_amd import autotune
    wls = [synth.beam_plasma((64, 64), ppc=16, name="a"), synth.beam_plasma((64, 64), ppc=12, name="b"),
           synth.beam_plasma((32, 32), ppc=16, name="c")]
    cache = str(tmp_path / "launch.json")
    assert pic.pick_shape({0: 1.0, 1: 0.99, 3: 0.995}) == 0 and pic.pick_shape({0: 1.0, 3: 0.9, 1: 0.95}) == 3
    tiles, shapes, rep = autotune.choose_launch(wls, nsteps=3, cache_path=cache)
    assert len(tiles) == len(shapes) == 3 and all(s in pic.SHAPES for s in shapes)
    edges = rep["_edges"]
    for t, s in zip(tiles, shapes):
        assert edges[str(t)] == s
    for k, v in rep.items():
        if not k.startswith("_"):
            assert not v["shape_cached"] and set(int(x) for x in v["shape_ms"]) == set(pic.SHAPES)
    tiles2, shapes2, rep2 = autotune.choose_launch(wls, nsteps=3, cache_path=cache)
    assert tiles2 == tiles and shapes2 == shapes
    assert all(v["shape_cached"] for k, v in rep2.items() if not k.startswith("_"))
