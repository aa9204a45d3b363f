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


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-11), ("mixed", 1e-4)])
def test_continuity_residual_2d(pic, prec, bar):
    """The step's charge continuity rho^{n+1} - rho^n + dt div J^{n+1/2} = 0
    (the property of the Esirkepov deposit) on every node, recorded on the
    device: at round-off against max |rho^{n+1} - rho^n| in FP64 and at the
    FP32 level of the tile current in mixed precision."""
    log(f"case continuity 2d {prec}")
    p = pic.PIC_PREC_FP64 if prec == "fp64" else pic.PIC_PREC_MIXED
    h = _records(pic, synth.C1, p, 100)
    assert len(h) == 10
    step = min(x["rho_step"] for x in h)
    worst = max(x["continuity_resid"] for x in h)
    log(f"  min max|rho' - rho| {step:.3e}, worst continuity residual {worst:.3e}")
    assert step > 1e-4
    assert worst < bar * step


def test_continuity_residual_3d_fp64(pic):
    log("case continuity 3d fp64")
    wl = synth.beam_plasma((16, 16, 32), ppc=4, u_th_beam=0.1, u_th_plasma=0.02, steps=30)
    h = _records(pic, wl, pic.PIC_PREC_FP64, 30, diag_every=5)
    step = min(x["rho_step"] for x in h)
    worst = max(x["continuity_resid"] for x in h)
    log(f"  min max|rho' - rho| {step:.3e}, worst continuity residual {worst:.3e}")
    assert step > 1e-4 and worst < 1e-11 * step


@pytest.mark.parametrize("ndim", [2, 3])
def test_continuity_records_against_the_oracle(pic, ndim):
    """Every step's record against the oracle's charge on the nodes (orc_rho
    before and after the step) and its current (orc_divergence of J^{n+1/2}),
    host-loaded identical particles in FP64: max |rho^{n+1} - rho^n| agrees
    to 1e-10 (relative) and both continuity residuals sit at round-off."""
    from pic_cases import gpu_run, oracle_run
    log(f"case continuity vs oracle {ndim}d")
    n = (32, 32) if ndim == 2 else (8, 8, 16)
    wl = synth.beam_plasma(n, ppc=8 if ndim == 2 else 4, u_th_beam=0.2, u_th_plasma=0.05, steps=8)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    want_step, want_res = [], []
    for _ in range(wl.steps):
        r0 = orc.rho()
        orc.step(1)
        drho = orc.rho() - r0
        want_step.append(float(np.max(np.abs(drho))))
        want_res.append(float(np.max(np.abs(drho + wl.dt * orc.divergence(orc.f.J)))))
    g = gpu_run(wl, parts, pic.PIC_PREC_FP64, flags=pic.PIC_FLAG_GAUSS_RESIDUAL, diag_every=1)
    g.step(wl.steps)
    h = g.history()
    g.close()
    assert [x["step"] for x in h] == list(range(wl.steps))
    for x, ws, wr in zip(h, want_step, want_res):
        assert abs(x["rho_step"] / ws - 1) < 1e-10, (x["step"], x["rho_step"], ws)
        assert x["continuity_resid"] < 1e-11 * ws and wr < 1e-11 * ws
    log(f"  rho_step {h[-1]['rho_step']:.6e} (oracle {want_step[-1]:.6e}), residual gpu "
        f"{max(x['continuity_resid'] for x in h):.2e} oracle {max(want_res):.2e}")
