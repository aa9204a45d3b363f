"""Checkpoint / restore through the C ABI: a run restored from a checkpoint
continues exactly like the run that wrote it."""
import numpy as np
import pytest

import synth
from pic_cases import log, rel_err, stack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_restore_continues_the_run(pic, prec, tmp_path):
    log(f"case checkpoint {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    wl = synth.beam_plasma((64, 64), ppc=16, u_th_beam=0.2, nu=0.05, name="ckpt")
    g, sp = pic.workload_descs(wl, precision=p, diag_every=5)
    a = pic.Run(g, sp)
    a.step(15)
    path = str(tmp_path / "run.ckpt")
    a.checkpoint(path)
    a.step(15)
    Ea, Ba, Ja = a.read_fields()
    ha = a.history()
    # a fresh run that skips the loader, restored from the file
    g2, sp2 = pic.workload_descs(wl, precision=p, diag_every=5, flags=pic.PIC_FLAG_HOST_LOAD)
    b = pic.Run(g2, sp2)
    b.restore(path)
    b.step(15)
    Eb, Bb, Jb = b.read_fields()
    hb = b.history()
    err = rel_err(stack(Eb, Bb), stack(Ea, Ba))
    log(f"  restored vs original field error {err:.3e}")
    assert err < 1e-12
    assert [r["step"] for r in hb] == [r["step"] for r in ha]
    for ra, rb in zip(ha, hb):
        assert ra["collisions"] == rb["collisions"]
        assert np.array_equal(ra["n_particles"], rb["n_particles"])
    xa, ua, ia = a.read_particles(1)
    xb, ub, ib = b.read_particles(1)
    oa, ob = np.argsort(ia), np.argsort(ib)
    assert np.array_equal(ia[oa], ib[ob])
    assert np.max(np.abs(ua[:, oa] - ub[:, ob])) < 1e-12
    # a run with other descriptors refuses the file
    wl2 = synth.beam_plasma((64, 64), ppc=12, name="other")
    g3, sp3 = pic.workload_descs(wl2, precision=p, diag_every=5, flags=pic.PIC_FLAG_HOST_LOAD)
    c = pic.Run(g3, sp3)
    with pytest.raises(pic.PicError) as e:
        c.restore(path)
    assert e.value.code == -6
    for r in (a, b, c):
        r.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_restore_continues_a_3d_run(pic, prec, tmp_path):
    """The same for a 3D3V run (8^3 tiles), with the history continued."""
    log(f"case checkpoint 3d {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    wl = synth.beam_plasma((16, 16, 32), ppc=4, u_th_beam=0.2, name="ckpt3d")
    # ids stored for every species (collisionless ones keep none by default)
    g, sp = pic.workload_descs(wl, precision=p, diag_every=5, flags=pic.PIC_FLAG_TRACK_IDS)
    a = pic.Run(g, sp)
    a.step(10)
    path = str(tmp_path / "run3d.ckpt")
    a.checkpoint(path)
    a.step(10)
    Ea, Ba, _ = a.read_fields()
    g2, sp2 = pic.workload_descs(wl, precision=p, diag_every=5,
                                 flags=pic.PIC_FLAG_HOST_LOAD | pic.PIC_FLAG_TRACK_IDS)
    b = pic.Run(g2, sp2)
    b.restore(path)
    b.step(10)
    Eb, Bb, _ = b.read_fields()
    err = rel_err(stack(Eb, Bb), stack(Ea, Ba))
    log(f"  restored vs original field error {err:.3e}")
    assert err < 1e-12
    assert [r["step"] for r in b.history()] == [r["step"] for r in a.history()]
    for s in range(2):
        xa, ua, ia = a.read_particles(s)
        xb, ub, ib = b.read_particles(s)
        oa, ob = np.argsort(ia), np.argsort(ib)
        assert np.array_equal(ia[oa], ib[ob])
        assert np.max(np.abs(xa[:, oa] - xb[:, ob])) < 1e-12
    for r in (a, b):
        r.close()


def test_restore_ignores_descriptor_padding(pic, tmp_path):
    """The descriptors' padding bytes (after precision, run, ppc, ...) carry
    no data: a run whose descriptors were built over garbage bytes (as a C
    caller's uninitialised stack would leave them) writes a checkpoint that a
    run with zeroed descriptors restores."""
    import ctypes as C
    log("case checkpoint padding")
    wl = synth.beam_plasma((32, 32), ppc=8, u_th_beam=0.2, name="pad")
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, diag_every=5)
    g_dirty = pic.GridDesc()
    C.memset(C.byref(g_dirty), 0xAB, C.sizeof(g_dirty))
    sp_dirty = (pic.SpeciesDesc * len(sp))()
    C.memset(sp_dirty, 0xCD, C.sizeof(sp_dirty))
    for name, _ in pic.GridDesc._fields_:
        setattr(g_dirty, name, getattr(g, name))
    for i in range(len(sp)):
        for name, _ in pic.SpeciesDesc._fields_:
            setattr(sp_dirty[i], name, getattr(sp[i], name))
    assert bytes(g_dirty) != bytes(g)           # the padding differs
    a = pic.Run(g_dirty, sp_dirty)
    a.step(5)
    path = str(tmp_path / "pad.ckpt")
    a.checkpoint(path)
    g2, sp2 = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, diag_every=5, flags=pic.PIC_FLAG_HOST_LOAD)
    b = pic.Run(g2, sp2)
    b.restore(path)
    a.step(5)
    b.step(5)
    Ea, Ba, _ = a.read_fields()
    Eb, Bb, _ = b.read_fields()
    assert rel_err(stack(Eb, Bb), stack(Ea, Ba)) == 0.0
    for r in (a, b):
        r.close()
