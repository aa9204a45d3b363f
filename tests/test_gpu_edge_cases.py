"""Edge cases of the HIP path against the FP64 oracle (through the C ABI):
an empty species, a ragged particle count that fills no whole wave, a grid of
one tile (every mover re-enters the tile it left), 3D grids of 1-3 tiles per
axis, a non-square grid, a
collision rate at which every draw below 2^32 - 1 scatters, and a species of
zero weight (pushed, but carrying no current)."""
import numpy as np
import pytest

import synth
from pic_cases import by_id, gpu_run, log, oracle_run, periodic_diff, rel_err, stack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _parity(pic, wl, parts, steps, tile=0, bar=1e-9):
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, pic.PIC_PREC_FP64, tile=tile, diag_every=1)
    orecs = orc.step(steps, diag=True)
    g.step(steps)
    hist = g.history()
    assert [h["collisions"] for h in hist] == [o["collisions"] for o in orecs]
    E, B, _ = g.read_fields()
    ref = stack(orc.f.E, orc.f.B)
    err = rel_err(stack(E, B), ref) if np.linalg.norm(ref) > 0 else float(np.linalg.norm(stack(E, B)))
    assert err < bar, err
    L = (np.array(wl.n) * np.array(wl.d))[:, None]
    for s, sp in enumerate(orc.species):
        x, u, ids = by_id(*g.read_particles(s))
        xo, uo, io = by_id(sp.x, sp.u, sp.id)
        assert np.array_equal(ids, io)
        assert hist[-1]["n_particles"][s] == io.size
        if io.size:
            assert np.max(np.abs(periodic_diff(x, xo, L))) < 1e-9
            assert np.max(np.abs(u - uo)) < 1e-9
    g.close()
    return err, orecs


def _random_particles(wl, s, n, rng, u_th=0.2):
    L = np.array(wl.n) * np.array(wl.d)
    x = rng.uniform(0, 1, (wl.ndim, n)) * L[:, None]
    u = u_th * rng.standard_normal((3, n))
    base = 0 if s == 0 else 1_000_000
    return synth.Particles(x, u, np.arange(base, base + n, dtype=np.uint32))


def test_empty_species(pic):
    log("case edge: empty species")
    wl = synth.beam_plasma((32, 32), ppc=8, u_th_beam=0.2, nu=0.05)
    parts = synth.load(wl)
    parts[1] = synth.Particles(np.zeros((2, 0)), np.zeros((3, 0)), np.zeros(0, dtype=np.uint32))
    _parity(pic, wl, parts, 20, tile=8)


def test_ragged_particle_count(pic):
    log("case edge: ragged count (1000 and 77 particles)")
    wl = synth.beam_plasma((32, 32), ppc=8, nu=0.05)
    rng = np.random.default_rng(7)
    parts = [_random_particles(wl, 0, 1000, rng), _random_particles(wl, 1, 77, rng, u_th=0.05)]
    _parity(pic, wl, parts, 30, tile=8)


def test_single_tile_grid(pic):
    log("case edge: one tile (8 x 8)")
    wl = synth.beam_plasma((8, 8), ppc=16, u_th_beam=0.3, nu=0.05)
    _parity(pic, wl, synth.load(wl), 30, tile=8)


@pytest.mark.parametrize("n", [(8, 8, 8), (8, 8, 16), (16, 8, 24)])
def test_3d_small_and_uneven_grids(pic, n):
    """3D grids of one tile, of one tile across x and y, and of 1-3 tiles per
    axis: the current reduction's neighbour tiles coincide with the node's
    own tile or wrap around, and every mover re-enters a neighbour that may
    be its own tile."""
    log(f"case edge: 3D grid {n}")
    wl = synth.beam_plasma(n, ppc=4, u_th_beam=0.3, nu=0.05)
    _parity(pic, wl, synth.load(wl), 20, tile=8)


def test_non_square_grid(pic):
    log("case edge: 64 x 16 grid")
    wl = synth.beam_plasma((64, 16), ppc=8, u_th_beam=0.3, nu=0.05)
    _parity(pic, wl, synth.load(wl), 30, tile=16)


def test_every_particle_scatters(pic):
    log("case edge: nu dt >> 1 (threshold clamped at 2^32 - 1)")
    wl = synth.beam_plasma((16, 16), ppc=8, nu=1e4)
    parts = synth.load(wl)
    _, orecs = _parity(pic, wl, parts, 10, tile=8)
    assert all(o["collisions"] == parts[1].id.size for o in orecs)


def test_zero_weight_species(pic):
    log("case edge: a species of zero density")
    wl = synth.beam_plasma((32, 32), ppc=8, u_th_beam=0.2)
    sp0, sp1 = wl.species
    from dataclasses import replace
    wl = replace(wl, species=(sp0, replace(sp1, density=0.0, cancel_current_of=-1)))
    parts = synth.load(wl)
    _parity(pic, wl, parts, 20, tile=8)
