"""The ensemble tuner's host logic (paper_0808_4078_amd/autotune.py) with the
library's timings replaced by fixed tables: classes, representatives, the
tile and launch-shape choice, the 2% margin before a non-default shape is
taken, one shape per tile edge by member majority, and the JSON cache."""
import json

import pytest

import synth
from paper_0808_4078_amd import autotune, pic


@pytest.fixture
def fake_timings(monkeypatch):
    calls = {"tune": [], "tune_shape": []}

    def tune(grid, species, nsteps=10, copies=1, stream=None):
        calls["tune"].append((tuple(grid.n[:2]), copies))
        n = grid.n[0]
        # small grids prefer tile 8, the others tile 16
        return (8, {8: 1.0, 16: 1.1, 32: 1.5}) if n <= 64 else (16, {8: 1.2, 16: 1.0, 32: 1.3})

    def tune_shape(grid, species, nsteps=10, copies=1, stream=None):
        calls["tune_shape"].append((tuple(grid.n[:2]), grid.tile[0]))
        n = grid.n[0]
        if n == 128:          # shape 3 clearly faster
            ms = {0: 1.0, 1: 1.01, 2: 1.0, 3: 0.9, 4: 1.2}
        elif n == 256:        # shape 1 faster, but within the margin
            ms = {0: 1.0, 1: 0.99, 2: 1.0, 3: 1.02, 4: 1.2}
        else:
            ms = {0: 1.0, 1: 1.05, 2: 1.04, 3: 1.1, 4: 1.3}
        return min(ms, key=ms.get), ms

    monkeypatch.setattr(pic, "tune", tune)
    monkeypatch.setattr(pic, "tune_shape", tune_shape)
    return calls


def _members():
    return ([synth.beam_plasma((128, 128), ppc=16, name=f"a{i}", seed=synth.SEED + i) for i in range(3)]
            + [synth.beam_plasma((256, 256), ppc=16, name="b")]
            + [synth.beam_plasma((64, 64), ppc=16, name=f"c{i}", seed=synth.SEED + 10 + i) for i in range(2)])


def test_pick_shape_margin():
    assert pic.pick_shape({0: 1.0, 1: 0.99, 3: 0.995}) == 0
    assert pic.pick_shape({0: 1.0, 3: 0.9, 1: 0.95}) == 3
    assert pic.pick_shape({0: 1.0}) == 0
    assert pic.pick_shape({0: 1.0, 2: 0.979}) == 2 and pic.pick_shape({0: 1.0, 2: 0.981}) == 0


def test_choose_launch_classes_edges_and_cache(fake_timings, tmp_path):
    cache = str(tmp_path / "c.json")
    wls = _members()
    tiles, shapes, rep = autotune.choose_launch(wls, nsteps=3, cache_path=cache)
    # 128^2 and 256^2 classes take tile 16, the 64^2 class tile 8
    assert tiles == [16, 16, 16, 16, 8, 8]
    # edge 16: the 128^2 class (3 members, shape 3) outvotes the 256^2 class (1 member, shape 0:
    # its shape 1 is within the margin); edge 8 keeps the default
    assert rep["_edges"] == {"8": 0, "16": 3}
    assert shapes == [3, 3, 3, 3, 0, 0]
    classes = {k: v for k, v in rep.items() if not k.startswith("_")}
    assert len(classes) == 3 and sum(v["members"] for v in classes.values()) == len(wls)
    assert all(not v["cached"] and not v["shape_cached"] for v in classes.values())
    assert len(fake_timings["tune"]) == 3 and len(fake_timings["tune_shape"]) == 3
    # the shape is timed at the class's own tile edge
    assert sorted(fake_timings["tune_shape"]) == [((64, 64), 8), ((128, 128), 16), ((256, 256), 16)]
    data = json.load(open(cache))
    assert len(data) == 6                         # a tile entry and a shape entry per class
    # a second call is answered from the cache, without timing
    tiles2, shapes2, rep2 = autotune.choose_launch(wls, nsteps=3, cache_path=cache)
    assert (tiles2, shapes2) == (tiles, shapes)
    assert len(fake_timings["tune"]) == 3 and len(fake_timings["tune_shape"]) == 3
    assert all(v["cached"] and v["shape_cached"] for k, v in rep2.items() if not k.startswith("_"))


def test_copies_fill_the_device_in_saturated_mode():
    wl = synth.beam_plasma((64, 64), ppc=16, name="s")
    assert autotune.copies_for(wl, saturate=False) == 1
    c = autotune.copies_for(wl, saturate=True)
    assert c * wl.particles >= autotune.SATURATION or c == autotune.MAX_COPIES
