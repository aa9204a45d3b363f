"""Host-side checks of the C ABI (no GPU): the library loads, exports every
entry point declared in include/pic.h, its ctypes mirrors match the C
struct sizes, and pic_query validates descriptors."""
import os
import re
import subprocess

import pytest

import synth
from paper_0808_4078_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pic.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(pic_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_entry_point():
    names = declared_functions()
    assert len(names) >= 13
    L = pic.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(pic.EXPORTS) == set(names)


def test_ctypes_structs_match_the_header(tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text('#include "pic.h"\n#include <stdio.h>\n#include <stddef.h>\nint main(void){'
                    'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(pic_grid_desc),'
                    'sizeof(pic_species_desc), sizeof(pic_sizes), sizeof(pic_buffers), sizeof(pic_diag),'
                    'offsetof(pic_grid_desc, flags), offsetof(pic_diag, rebins), sizeof(pic_hyb_desc),'
                    'offsetof(pic_hyb_desc, flags), sizeof(pic_hyb_diag), offsetof(pic_hyb_diag, mean_psi),'
                    'offsetof(pic_grid_desc, ee_vref), offsetof(pic_diag, ee_pairs), offsetof(pic_grid_desc, shape),'
                    'sizeof(pic_run_info), offsetof(pic_run_info, inflight));'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    import ctypes as C
    want = [C.sizeof(pic.GridDesc), C.sizeof(pic.SpeciesDesc), C.sizeof(pic.Sizes), C.sizeof(pic.Buffers),
            C.sizeof(pic.Diag), pic.GridDesc.flags.offset, pic.Diag.rebins.offset, C.sizeof(pic.HybDesc),
            pic.HybDesc.flags.offset, C.sizeof(pic.HybDiag), pic.HybDiag.mean_psi.offset,
            pic.GridDesc.ee_vref.offset, pic.Diag.ee_pairs.offset, pic.GridDesc.shape.offset,
            C.sizeof(pic.RunInfo), pic.RunInfo.inflight.offset]
    assert got == want


def test_status_strings():
    L = pic.lib()
    for code in range(-7, 1):
        assert L.pic_status_string(code)


def _descs(**kw):
    wl = synth.C1
    return pic.workload_descs(wl, **kw)


def test_query_sizes_c1_and_c3():
    g, sp = _descs(precision=pic.PIC_PREC_FP64)
    s64 = pic.query(g, sp)
    g, sp = _descs(precision=pic.PIC_PREC_MIXED)
    s32 = pic.query(g, sp)
    assert s64.field_bytes > s32.field_bytes > 0
    assert s64.particle_bytes[0] > s32.particle_bytes[0] > 0
    # C3: 1024^2, 64 ppc, 2 species -> each species store holds >= 64 M slots per set
    g, sp = pic.workload_descs(synth.C3, precision=pic.PIC_PREC_MIXED)
    s = pic.query(g, sp)
    assert s.particle_bytes[0] >= 2 * 64 * 1024 * 1024 * 28


@pytest.mark.parametrize("field,value,code", [
    ("dt", 0.2, -3),            # more than half a cell per step
    ("tile", 12, -2),           # not a supported tile
    ("tile", 32, 0),
])
def test_query_validation(field, value, code):
    wl = synth.C1
    if field == "dt":
        g, sp = pic.make_descs(2, wl.n, wl.d, value, [dict(density=1.0, ppc=4)])
    else:
        g, sp = pic.make_descs(2, wl.n, wl.d, wl.dt, [dict(density=1.0, ppc=4)], tile=value)
    out = pic.Sizes()
    import ctypes as C
    rc = pic.lib().pic_query(C.byref(g), sp, 1, C.byref(out))
    assert rc == code


def test_query_rejects_bad_species_and_grid():
    import ctypes as C
    out = pic.Sizes()
    g, sp = pic.make_descs(2, (64, 48), (0.2, 0.2), 0.1, [dict(density=1.0, ppc=0)])
    assert pic.lib().pic_query(C.byref(g), sp, 1, C.byref(out)) == -1
    g, sp = pic.make_descs(2, (64, 36), (0.2, 0.2), 0.1, [dict(density=1.0, ppc=4)])
    assert pic.lib().pic_query(C.byref(g), sp, 1, C.byref(out)) == -1      # 36 is not a multiple of 8
    g, sp = pic.make_descs(2, (64, 40), (0.2, 0.2), 0.1, [dict(density=1.0, ppc=4)])
    assert pic.lib().pic_query(C.byref(g), sp, 1, C.byref(out)) == 0       # common tile 8
    g, sp = pic.make_descs(2, (64, 64), (0.2, 0.2), 0.1, [dict(density=1.0, ppc=4)])
    assert pic.lib().pic_query(C.byref(g), sp, 0, C.byref(out)) == -1
    assert pic.lib().pic_query(C.byref(g), sp, 9, C.byref(out)) == -1


def test_batch_and_tuner_queries_validate_on_the_host():
    import ctypes as C
    L = pic.lib()
    nbytes = C.c_size_t(123)
    assert L.pic_batch_query(0, None, C.byref(nbytes)) == -1
    arr = (C.c_void_p * 2)(None, None)
    assert L.pic_batch_query(2, arr, C.byref(nbytes)) == -1          # NULL member
    out = C.c_void_p()
    assert L.pic_batch_init(0, None, None, 0, 0, 0, C.byref(out)) == -1
    # workspace of the tuner: the largest candidate's four buffers
    g, sp = pic.workload_descs(synth.C1, precision=pic.PIC_PREC_MIXED)
    assert L.pic_tune_query(C.byref(g), sp, len(sp), 1, C.byref(nbytes)) == 0
    biggest = 0
    for t in (8, 16, 32):
        gt, spt = pic.workload_descs(synth.C1, precision=pic.PIC_PREC_MIXED, tile=t)
        s = pic.query(gt, spt)
        biggest = max(biggest, sum(s.particle_bytes[:2]) + s.field_bytes + s.scratch_bytes + s.diag_bytes)
    assert biggest <= nbytes.value < biggest + 8 * 256
    one = nbytes.value
    assert L.pic_tune_query(C.byref(g), sp, len(sp), 3, C.byref(nbytes)) == 0       # 3 copies + batch table
    assert 3 * biggest < nbytes.value < 3 * one + 64 * 1024
    assert L.pic_tune_query(C.byref(g), sp, len(sp), 0, C.byref(nbytes)) == -1
    g, sp = pic.make_descs(2, (36, 36), (0.2, 0.2), 0.1, [dict(density=1.0, ppc=4)])
    assert L.pic_tune_query(C.byref(g), sp, 1, 1, C.byref(nbytes)) == -1  # no edge divides 36
    best = C.c_int32()
    ms = (C.c_double * 3)()
    g, sp = pic.workload_descs(synth.C1)
    assert L.pic_tune(C.byref(g), sp, len(sp), 1, None, 0, None, 4, C.byref(best), ms) == -1
    ms5 = (C.c_double * len(pic.SHAPES))()
    assert L.pic_tune_shape(C.byref(g), sp, len(sp), 1, None, 0, None, 4, C.byref(best), ms5) == -1


@pytest.mark.parametrize("prec,shape,code", [
    (pic.PIC_PREC_MIXED, 0, 0), (pic.PIC_PREC_MIXED, 4, 0), (pic.PIC_PREC_MIXED, 5, -1),
    (pic.PIC_PREC_MIXED, -1, -1), (pic.PIC_PREC_FP64, 0, 0), (pic.PIC_PREC_FP64, 3, -1)])
def test_query_validates_the_launch_shape(prec, shape, code):
    """Shapes 0..4 in mixed precision; FP64 runs take shape 0 only."""
    import ctypes as C
    g, sp = pic.workload_descs(synth.C1, precision=prec, shape=shape)
    out = pic.Sizes()
    assert pic.lib().pic_query(C.byref(g), sp, len(sp), C.byref(out)) == code


def test_shape_table_matches_the_header():
    src = open(HEADER).read()
    assert int(re.search(r"#define PIC_PARTICLE_SHAPES (\d+)", src).group(1)) == len(pic.SHAPES)
    for k, (blk, inflight) in pic.SHAPES.items():
        assert re.search(rf"\b{k}: {blk} / {inflight}\b", src), k


def test_checkpoint_entry_points_reject_null_handles(tmp_path):
    L = pic.lib()
    p = str(tmp_path / "x.ckpt").encode()
    assert L.pic_checkpoint(None, p) == -1
    assert L.pic_restore(None, p) == -1


def _hyb(**kw):
    d = dict(nx=64, ny=32, dx=0.2, dy=0.2, dt=0.1, nu=0.05, n0=1.0, weight=0.1 / 16, nparticles=64 * 32 * 16,
             iters=10, diag_every=1, sort_every=0, flags=0)
    d.update(kw)
    return pic.HybDesc(*[d[f] for f, _ in pic.HybDesc._fields_])


def test_reduced_model_query_sizes():
    """pic_hyb_query: two particle sets of 5 FP64 + 1 u32 arrays, and the node
    planes of the grid buffer."""
    import ctypes as C
    pb, gb = C.c_size_t(), C.c_size_t()
    assert pic.lib().pic_hyb_query(C.byref(_hyb()), C.byref(pb), C.byref(gb)) == pic.PIC_OK
    N, cells = 64 * 32 * 16, 64 * 32
    assert pb.value >= 2 * N * (5 * 8 + 4)
    assert pb.value < 2 * N * (5 * 8 + 4) + 12 * 256
    assert gb.value >= cells * (13 * 8 + 16)


@pytest.mark.parametrize("field,value,code", [
    ("nx", 48, pic.PIC_E_UNSUPPORTED), ("ny", 4, pic.PIC_E_UNSUPPORTED), ("nx", 8192, pic.PIC_E_UNSUPPORTED),
    ("dx", 0.0, pic.PIC_E_INVALID_ARG), ("dt", -1.0, pic.PIC_E_INVALID_ARG), ("nu", -0.1, pic.PIC_E_INVALID_ARG),
    ("n0", 0.0, pic.PIC_E_INVALID_ARG), ("iters", 0, pic.PIC_E_INVALID_ARG), ("iters", 65, pic.PIC_E_INVALID_ARG),
    ("nparticles", -1, pic.PIC_E_INVALID_ARG), ("sort_every", -2, pic.PIC_E_INVALID_ARG),
    ("flags", 1, pic.PIC_E_INVALID_ARG), ("weight", 1.0, pic.PIC_E_UNSUPPORTED)])
def test_reduced_model_query_validation(field, value, code):
    """Invalid descriptors are refused on the host (weight 1 at 16 per cell:
    mean beam density above n0, no plasma left for quasi-neutrality)."""
    import ctypes as C
    pb, gb = C.c_size_t(), C.c_size_t()
    assert pic.lib().pic_hyb_query(C.byref(_hyb(**{field: value})), C.byref(pb), C.byref(gb)) == code
    buf = C.create_string_buffer(256)
    pic.lib().pic_hyb_last_error(None, buf, 256)
    assert buf.value


def test_reduced_model_init_rejects_bad_arguments_on_the_host():
    """Null buffers, short buffers and particles outside the box are refused
    before any device work."""
    import ctypes as C
    import numpy as np
    d = _hyb(nparticles=4)
    h = C.c_void_p()
    z = np.zeros(4)
    p = z.ctypes.data_as(C.c_void_p)
    L = pic.lib()
    assert L.pic_hyb_init(C.byref(d), None, 0, None, 0, None, p, p, p, p, p, C.byref(h)) == pic.PIC_E_INVALID_ARG
    fake = C.c_void_p(1 << 40)
    assert L.pic_hyb_init(C.byref(d), fake, 16, fake, 16, None, p, p, p, p, p, C.byref(h)) == \
        pic.PIC_E_BUFFER_TOO_SMALL
    xs = np.array([0.0, 1.0, 64 * 0.2, 2.0])            # x = L_x is outside [0, L_x)
    big = 1 << 40
    assert L.pic_hyb_init(C.byref(d), fake, big, fake, big, None, xs.ctypes.data_as(C.c_void_p), p, p, p, p,
                          C.byref(h)) == pic.PIC_E_INVALID_ARG
    assert not h.value
    for fn in ("pic_hyb_step", "pic_hyb_sync"):
        args = (None, 1) if fn == "pic_hyb_step" else (None,)
        assert getattr(L, fn)(*args) == pic.PIC_E_INVALID_ARG
    assert L.pic_hyb_destroy(None) == pic.PIC_OK
