"""pic_init_static_scratch through the C ABI: a run on the library's own
scratch array steps exactly like the same run on a caller-owned scratch
buffer (pic_init), on two initialisations in a row on the device -- the
second on a smaller grid, over the contents the first one left behind."""
import numpy as np
import pytest

import synth
from pic_cases import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _twin_runs(pic, wl, prec, flags):
    g, sp = pic.workload_descs(wl, precision=prec, diag_every=5, flags=flags | pic.PIC_FLAG_NO_GRAPH)
    ref = pic.Run(g, sp)
    g2, sp2 = pic.workload_descs(wl, precision=prec, diag_every=5, flags=flags)
    st = pic.Run(g2, sp2, static_scratch=True)
    return ref, st


def _rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _compare(ref, st, steps, exact):
    """Fields, current and every record of the two runs.  Mixed precision
    is compared bit for bit (its FP32 terms add exactly in the FP64 tile
    accumulators); FP64 to 1e-12, since the order of the LDS current
    atomics changes the last bits from run to run.  Counts exactly."""
    ref.step(steps)
    st.step(steps)
    Er, Br, Jr = ref.read_fields()
    Es, Bs, Js = st.read_fields()
    bar = 0.0 if exact else 1e-12
    err = max(_rel(Es, Er), _rel(Bs, Br), _rel(Js, Jr))
    log(f"  fields and current: relative difference {err:.2e}")
    assert err <= bar
    hr, hs = ref.history(), st.history()
    assert len(hr) == len(hs) == steps // 5
    for a, b in zip(hr, hs):
        assert a["step"] == b["step"]
        assert _rel(b["W"], a["W"]) <= bar and _rel(b["kinetic"], a["kinetic"]) <= max(bar, 1e-14)
        assert a["collisions"] == b["collisions"] and np.array_equal(a["n_particles"], b["n_particles"])
        for k in ("continuity_resid", "gauss_resid", "rho_step", "rho_dev"):
            assert (a[k] < 0) == (b[k] < 0)
            assert abs(a[k] - b[k]) <= 1e-12 * max(abs(a["rho_step"]), abs(a["rho_dev"]), 1e-300) + 1e-15


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_static_scratch_matches_caller_scratch(pic, prec):
    p = pic.PIC_PREC_MIXED if prec == "mixed" else pic.PIC_PREC_FP64
    # first call: a 128^2 collisional run with the Gauss and continuity checks
    log(f"case static scratch {prec}: 128x128, 16 ppc, 40 steps")
    wl = synth.beam_plasma((128, 128), ppc=16, u_th_beam=0.3, nu=0.05, name="static-1")
    ref, st = _twin_runs(pic, wl, p, pic.PIC_FLAG_GAUSS_RESIDUAL)
    info = st.info()
    assert info["static_scratch"] == 1 and info["graph"] == 0
    # a second run on the same device is refused while the first holds the scratch
    g, sp = pic.workload_descs(synth.beam_plasma((32, 32), ppc=4), precision=p)
    with pytest.raises(pic.PicError) as e:
        pic.Run(g, sp, static_scratch=True)
    assert e.value.code == pic.PIC_E_STATE
    _compare(ref, st, 40, prec == "mixed")
    ref.close()
    st.close()
    # second call, smaller input: 64^2, no checks, over the first run's leftovers
    log(f"case static scratch {prec}: 64x64, 8 ppc, 30 steps")
    wl = synth.beam_plasma((64, 64), ppc=8, u_th_beam=0.1, nu=0.1, name="static-2")
    ref, st = _twin_runs(pic, wl, p, 0)
    _compare(ref, st, 30, prec == "mixed")
    ref.close()
    st.close()


def test_static_scratch_refuses_what_does_not_fit(pic):
    log("case static scratch limits")
    big = synth.beam_plasma((2048, 2048), ppc=1, name="too-big")
    g, sp = pic.workload_descs(big, precision=pic.PIC_PREC_FP64)
    assert pic.query(g, sp).scratch_bytes > 64 << 20
    with pytest.raises(pic.PicError) as e:
        pic.Run(g, sp, static_scratch=True)
    assert e.value.code == pic.PIC_E_BUFFER_TOO_SMALL
