"""The Gauss's-law diagnostic (PIC_FLAG_GAUSS_RESIDUAL) on the GPU, through
the C ABI: with the ions carrying -rho_0, div E^n - (rho^n - rho_0) stays at
its initial value because the deposit conserves charge and the Yee update
keeps div curl B = 0.  Checked at round-off in FP64 (2D and 3D), at FP32
accumulation level in mixed precision, and against a planted divergence:
fields written before step 0 give a residual equal to max |div E| of those
fields, computed here with the same discrete divergence, at every record."""
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


def _records(pic, wl, prec, steps, diag_every=10, E=None):
    g, sp = pic.workload_descs(wl, precision=prec, diag_every=diag_every, flags=pic.PIC_FLAG_GAUSS_RESIDUAL)
    r = pic.Run(g, sp)
    if E is not None:
        r.write_fields(E, None)
    r.step(steps)
    h = r.history()
    r.close()
    return h


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-11), ("mixed", 1e-4)])
def test_gauss_residual_2d(pic, prec, bar):
    log(f"case gauss 2d {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    h = _records(pic, synth.C1, p, 100)
    assert len(h) == 10 and h[0]["gauss_resid"] == 0.0 and h[0]["rho_dev"] == 0.0
    dev = max(x["rho_dev"] for x in h)
    worst = max(x["gauss_resid"] for x in h)
    log(f"  max |rho - rho_0| {dev:.3e}, worst residual {worst:.3e}")
    assert dev > 1e-3
    assert worst < bar * dev


def test_gauss_residual_3d_fp64(pic):
    log("case gauss 3d fp64")
    wl = synth.beam_plasma((16, 16, 32), ppc=4, u_th_beam=0.1, u_th_plasma=0.02, steps=30)
    h = _records(pic, wl, pic.PIC_PREC_FP64, 30, diag_every=5)
    dev = max(x["rho_dev"] for x in h)
    worst = max(x["gauss_resid"] for x in h)
    log(f"  max |rho - rho_0| {dev:.3e}, worst residual {worst:.3e}")
    assert dev > 1e-3 and worst < 1e-11 * dev


def test_gauss_residual_measures_a_planted_divergence(pic):
    """Random E written before step 0: every record's residual equals
    max |div E_0| (div E - (rho - rho_0) is conserved by the step)."""
    log("case gauss planted")
    wl = synth.beam_plasma((32, 32), ppc=8, u_th_beam=0.2, steps=30)
    rng = np.random.default_rng(4)
    E = 0.01 * rng.standard_normal((3, 1, 32, 32))
    d = wl.d
    div = (E[0, 0] - np.roll(E[0, 0], 1, axis=1)) / d[0] + (E[1, 0] - np.roll(E[1, 0], 1, axis=0)) / d[1]
    want = float(np.max(np.abs(div)))
    h = _records(pic, wl, pic.PIC_PREC_FP64, 30, diag_every=10, E=E)
    for x in h:
        assert abs(x["gauss_resid"] / want - 1) < 1e-9, (x["step"], x["gauss_resid"], want)


def test_gauss_flag_is_refused_in_a_batch(pic):
    log("case gauss batch refusal")
    wl = synth.beam_plasma((32, 32), ppc=4)
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, flags=pic.PIC_FLAG_GAUSS_RESIDUAL)
    r = pic.Run(g, sp)
    with pytest.raises(pic.PicError) as e:
        pic.Batch([r])
    assert e.value.code == pic.PIC_E_UNSUPPORTED
    r.close()
