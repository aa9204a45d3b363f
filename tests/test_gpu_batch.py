"""The ensemble path (pic_batch_*) and the tile autotuner, through the C ABI.

A batch member goes through the same kernels as the run stepped alone, so
each member is checked against its twin stepped alone (fields to rounding
of the order-dependent FP64 sums, scattering events and particle counts
exactly), and one host-loaded FP64 member directly against the oracle."""
import numpy as np
import pytest

import synth
from pic_cases import gpu_run, log, oracle_run, rel_err, stack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


# uneven members: (cells, tile edge, ppc, beam u_th, nu)
MEMBERS = [((32, 32), 8, 16, 0.1, 0.0),
           ((64, 64), 16, 24, 0.3, 0.05),
           ((64, 32), 32, 12, 0.5, 0.1),
           ((128, 128), 16, 8, 0.2, 0.02),
           ((48, 48), 16, 16, 0.05, 0.08)]


def _workloads():
    return [synth.beam_plasma(n, ppc=ppc, u_th_beam=uth, nu=nu, name=f"member{i}", seed=synth.SEED + 100 + i)
            for i, (n, _, ppc, uth, nu) in enumerate(MEMBERS)]


def _device_runs(pic, prec, diag_every=5):
    runs = []
    for wl, m in zip(_workloads(), MEMBERS):
        g, sp = pic.workload_descs(wl, precision=prec, tile=m[1], diag_every=diag_every)
        runs.append(pic.Run(g, sp))
    return runs


def _compare(pic, a, b, field_bar):
    Ea, Ba, Ja = a.read_fields()
    Eb, Bb, Jb = b.read_fields()
    err = rel_err(stack(Ea, Ba), stack(Eb, Bb))
    assert err < field_bar, err
    assert rel_err(Ja, Jb) < 100 * field_bar
    ha, hb = a.history(), b.history()
    assert len(ha) == len(hb) and len(ha) > 0
    for ra, rb in zip(ha, hb):
        assert ra["step"] == rb["step"]
        assert ra["collisions"] == rb["collisions"]
        assert np.array_equal(ra["n_particles"], rb["n_particles"])
    return err


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_batch_members_match_runs_stepped_alone(pic, prec, bar):
    log(f"case batch vs alone {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    alone = _device_runs(pic, p)
    members = _device_runs(pic, p)
    batch = pic.Batch(members)
    info = batch.info()
    assert info["items"] == [16, 16 + 64 + 9, 2]
    for _ in range(2):      # several graph replays with host reads in between
        batch.step(20)
        for r in alone:
            r.step(20)
        batch.sync()
        for r in alone:
            r.sync()
        errs = [_compare(pic, m, r, bar) for m, r in zip(members, alone)]
        log(f"  max member field error {max(errs):.3e}")
    # pic_batch_diagnostics: member i's latest record, as the run's own
    for i, (m, r) in enumerate(zip(members, alone)):
        db, dr = batch.diagnostics(i), r.diagnostics()
        assert db["step"] == dr["step"] and db["n_particles"].tolist() == dr["n_particles"].tolist()
        assert np.max(np.abs(db["W"] - dr["W"])) <= 1e3 * bar * max(1e-12, np.max(np.abs(dr["W"])))
    with pytest.raises(pic.PicError) as e:
        batch.diagnostics(len(members))
    assert e.value.code == pic.PIC_E_INVALID_ARG
    batch.close()
    for r in alone + members:
        r.close()


def test_batch_graph_and_queue_shapes_agree(pic):
    """Graph replay vs kernel-by-kernel launches, and a persistent grid of 3
    workgroups (each takes many items) vs the default grid."""
    log("case batch graph / persistent grid")
    p = pic.PIC_PREC_MIXED
    ra, rb, rc = _device_runs(pic, p), _device_runs(pic, p), _device_runs(pic, p)
    a = pic.Batch(ra)
    b = pic.Batch(rb, graph=False)
    c = pic.Batch(rc, persistent_blocks=3)
    assert c.info()["persistent_blocks"] == [3, 3, 3]
    for bt in (a, b, c):
        bt.step(15)
        bt.sync()
    for x, y, z in zip(ra, rb, rc):
        _compare(pic, x, y, 1e-5)
        _compare(pic, x, z, 1e-5)
    # a's and c's steps were graph replays, b's direct launches
    for bt, graph in ((a, 1), (b, 0), (c, 1)):
        li = bt.launch_info()
        assert li["graph"] == graph and li["steps_enqueued"] == 15
        assert li["graph_launches"] == (15 if graph else 0) and li["direct_steps"] == (0 if graph else 15)
    for bt in (a, b, c):
        bt.close()


def test_batch_member_against_oracle(pic):
    """A host-loaded FP64 member of a batch (next to device-loaded members)
    against the oracle on the same particles."""
    log("case batch member vs oracle")
    wl = synth.beam_plasma((32, 32), ppc=16, u_th_beam=0.1, nu=0.05, name="member-orc")
    parts = synth.load(wl)
    m = gpu_run(wl, parts, pic.PIC_PREC_FP64, tile=8)
    others = _device_runs(pic, pic.PIC_PREC_FP64)[1:]
    batch = pic.Batch([m] + others)
    orc = oracle_run(wl, parts)
    batch.step(30)
    orc.step(30)
    batch.sync()
    E, B, J = m.read_fields()
    err = rel_err(stack(E, B), stack(orc.f.E, orc.f.B))
    log(f"  fields vs oracle {err:.3e}")
    assert err < 1e-9
    batch.close()


def test_batch_profiled_step_and_member_states(pic):
    log("case batch profiled + member states")
    runs = _device_runs(pic, pic.PIC_PREC_MIXED, diag_every=0)
    batch = pic.Batch(runs)
    ms = batch.step_profiled(3)
    assert set(ms) == set(pic.Batch.GROUPS)
    assert ms["particle"] > 0 and all(v >= 0 for v in ms.values())
    with pytest.raises(pic.PicError) as e:
        runs[0].step(1)
    assert e.value.code == -6
    with pytest.raises(pic.PicError) as e:
        runs[1].close()
    assert e.value.code == -6
    with pytest.raises(pic.PicError) as e:
        pic.Batch(runs[:2])               # already members of a batch
    assert e.value.code == -6
    batch.close()
    runs[0].step(1)                       # released
    runs[0].sync()
    for r in runs:
        r.close()


def test_tuner_and_cache(pic, tmp_path):
    log("case tuner")
    from paper_0808_4078_amd import autotune
    wl = synth.beam_plasma((64, 64), ppc=16, name="tune")
    g, sp = pic.workload_descs(wl)
    for copies in (1, 6):
        best, ms = pic.tune(g, sp, nsteps=4, copies=copies)
        assert set(ms) == {8, 16, 32} and best in ms
        assert all(v > 0 for v in ms.values()) and ms[best] == min(ms.values())
    wls = [wl, synth.beam_plasma((64, 64), ppc=12, name="b"), synth.beam_plasma((32, 32), ppc=16, name="c")]
    cache = str(tmp_path / "tiles.json")
    tiles, rep = autotune.choose_tiles(wls, nsteps=3, cache_path=cache)
    assert all(v["copies"] > 1 for v in rep.values())
    assert len(rep) == 2 and tiles[0] == tiles[1] and tiles[2] in (8, 16, 32)
    assert not any(v["cached"] for v in rep.values())
    tiles2, rep2 = autotune.choose_tiles(wls, nsteps=3, cache_path=cache)
    assert tiles2 == tiles and all(v["cached"] for v in rep2.values())


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_batch_3d_members_match_runs_stepped_alone(pic, prec, bar):
    """3D3V members of uneven size (8^3 tiles) in one batch, against the same
    runs stepped alone."""
    log(f"case batch 3d vs alone {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    shapes = [((16, 16, 16), 4, 0.1), ((16, 16, 32), 2, 0.3), ((32, 16, 16), 4, 0.2)]

    def runs():
        out = []
        for i, (n, ppc, uth) in enumerate(shapes):
            wl = synth.beam_plasma(n, ppc=ppc, u_th_beam=uth, name=f"m3d{i}", seed=synth.SEED + 200 + i)
            g, sp = pic.workload_descs(wl, precision=p, tile=8, diag_every=5)
            out.append(pic.Run(g, sp))
        return out
    alone, members = runs(), runs()
    batch = pic.Batch(members)
    for _ in range(2):
        batch.step(15)
        for r in alone:
            r.step(15)
        batch.sync()
        for r in alone:
            r.sync()
        errs = [_compare(pic, m, r, bar) for m, r in zip(members, alone)]
        log(f"  max member field error {max(errs):.3e}")
    batch.close()
    for r in alone + members:
        r.close()


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-10), ("mixed", 1e-5)])
def test_batch_with_coulomb_members(pic, prec, bar):
    """A batch whose members mix the two scattering models (Coulomb
    small-angle and isotropic at a fixed rate) runs the kernel that carries
    the Coulomb branch; each member matches its twin stepped alone."""
    log(f"case batch coulomb {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    cfg = [((32, 32), 16, pic.PIC_COLL_COULOMB), ((64, 32), 12, 0), ((48, 48), 8, pic.PIC_COLL_COULOMB)]

    def runs():
        out = []
        for i, (n, ppc, model) in enumerate(cfg):
            wl = synth.beam_plasma(n, ppc=ppc, u_th_beam=0.2, nu=0.05, coll_model=model, coll_vref=0.1,
                                   name=f"mc{i}", seed=synth.SEED + 300 + i)
            g, sp = pic.workload_descs(wl, precision=p, tile=16, diag_every=5)
            out.append(pic.Run(g, sp))
        return out
    alone, members = runs(), runs()
    batch = pic.Batch(members)
    for _ in range(2):
        batch.step(15)
        for r in alone:
            r.step(15)
        batch.sync()
        for r in alone:
            r.sync()
        errs = [_compare(pic, m, r, bar) for m, r in zip(members, alone)]
        log(f"  max member field error {max(errs):.3e}")
    # the Coulomb members turn every plasma particle every step
    for m, (n, ppc, model) in zip(members, cfg):
        h = m.history()[-1]
        if model == pic.PIC_COLL_COULOMB:
            assert h["collisions"] == n[0] * n[1] * ppc
    batch.close()
    for r in alone + members:
        r.close()
