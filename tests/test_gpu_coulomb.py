"""The Coulomb small-angle scattering model (PIC_COLL_COULOMB) on the GPU,
through the C ABI: parity with the FP64 oracle in 2D and 3D (every particle
of the species turns every step, by a Philox draw on (id, step)), and, at a
size the oracle cannot step, the exact one-step drag law at two speeds in
test-particle mode (the v^-3 dependence of the momentum-transfer rate)."""
import math

import numpy as np
import pytest
from scipy.special import erfcx

import synth
from pic_cases import by_id, gpu_run, log, oracle_run, periodic_diff, rel_err, stack

pytestmark = pytest.mark.gpu

PRECS = {"fp64": 0, "mixed": 1}
COULOMB = 1


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


@pytest.mark.parametrize("prec,f_bar,u_bar", [("fp64", 1e-9, 1e-9), ("mixed", 1e-3, 1e-4)])
def test_coulomb_parity_2d(pic, prec, f_bar, u_bar):
    """64^2 beam-plasma, the return-current plasma scattering off the ions at
    nu = 0.05 at v = 0.05 (its thermal speed): fields every 10 steps, the
    per-step scattering count, and every particle by id after 60 steps."""
    log(f"case coulomb 2d {prec}")
    wl = synth.beam_plasma((64, 64), ppc=8, u_th_beam=0.1, u_th_plasma=0.05, nu=0.05, steps=60,
                           coll_model=COULOMB, coll_vref=0.05)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS[prec], diag_every=1)
    worst, orecs = 0.0, []
    for _ in range(wl.steps // 10):
        orecs += orc.step(10, diag=True)
        g.step(10)
        E, B, _ = g.read_fields()
        worst = max(worst, rel_err(stack(E, B), stack(orc.f.E, orc.f.B)))
    hist = g.history()
    log(f"  worst stacked field error {worst:.3e}")
    assert [h["collisions"] for h in hist] == [o["collisions"] for o in orecs]
    assert all(o["collisions"] == parts[1].id.size for o in orecs)
    assert worst < f_bar
    L = (np.array(wl.n) * np.array(wl.d))[:, None]
    for s, sp in enumerate(orc.species):
        x, u, ids = by_id(*g.read_particles(s))
        xo, uo, io = by_id(sp.x, sp.u, sp.id)
        assert np.array_equal(ids, io)
        assert np.max(np.abs(periodic_diff(x, xo, L))) < u_bar
        assert np.max(np.abs(u - uo)) < u_bar
    g.close()


@pytest.mark.parametrize("prec,f_bar,u_bar", [("fp64", 1e-9, 1e-9), ("mixed", 1e-3, 1e-4)])
def test_coulomb_parity_3d(pic, prec, f_bar, u_bar):
    log(f"case coulomb 3d {prec}")
    wl = synth.beam_plasma((16, 16, 16), ppc=4, u_th_beam=0.1, u_th_plasma=0.05, nu=0.05, steps=20,
                           coll_model=COULOMB, coll_vref=0.05)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS[prec], diag_every=1)
    orecs = orc.step(wl.steps, diag=True)
    g.step(wl.steps)
    assert [h["collisions"] for h in g.history()] == [o["collisions"] for o in orecs]
    E, B, _ = g.read_fields()
    err = rel_err(stack(E, B), stack(orc.f.E, orc.f.B))
    log(f"  field error {err:.2e}")
    assert err < f_bar
    L = (np.array(wl.n) * np.array(wl.d))[:, None]
    for s, sp in enumerate(orc.species):
        x, u, ids = by_id(*g.read_particles(s))
        xo, uo, io = by_id(sp.x, sp.u, sp.id)
        assert np.array_equal(ids, io)
        assert np.max(np.abs(periodic_diff(x, xo, L))) < u_bar
        assert np.max(np.abs(u - uo)) < u_bar
    g.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_coulomb_drag_law_at_scale(pic, prec):
    """Two cold species streaming along z at u = 0.1 and 0.2 in zero frozen
    fields, 2^20 particles each, 40 steps.  |u| is kept by every turn, so the
    speed and the per-step variance s^2 = nu (vref/v)^3 dt / 2 stay fixed and
    the mean u_z decays by exactly E[cos theta] = 2 E[1/(1+delta^2)] - 1 =
    sqrt(2 pi)/s erfcx(1/(sqrt(2) s)) - 1 per step; checked to 5 standard
    errors for each speed (their rates differ by the v^-3 law)."""
    log(f"case coulomb drag law {prec}")
    nu, vref, dt, steps = 0.05, 0.1, 0.1, 40
    sps = [synth.SpeciesCfg(f"s{i}", 0.5, 16, (0.0, 0.0, u0), 0.0, nu=nu, coll_model=COULOMB, coll_vref=vref)
           for i, u0 in enumerate((0.1, 0.2))]
    wl = synth.Workload("drag", 2, (256, 256), (0.2, 0.2), dt, steps, tuple(sps))
    g, sp = pic.workload_descs(wl, precision=PRECS[prec], diag_every=steps,
                               flags=pic.PIC_FLAG_FREEZE_FIELDS)
    r = pic.Run(g, sp)
    r.step(steps)
    r.sync()
    rates = []
    for s, u0 in enumerate((0.1, 0.2)):
        x, u, ids = r.read_particles(s)
        assert ids.size == wl.cells * 16
        U = np.linalg.norm(u, axis=0)
        assert np.max(np.abs(U / u0 - 1)) < (1e-12 if prec == "fp64" else 2e-5)
        v = u0 / math.sqrt(1 + u0 * u0)
        s_ = math.sqrt(0.5 * nu * dt * (vref / v) ** 3)
        c = math.sqrt(2 * math.pi) / s_ * erfcx(1 / (math.sqrt(2) * s_)) - 1
        want = u0 * c ** steps
        got = float(u[2].mean())
        se = float(u[2].std()) / math.sqrt(u.shape[1])
        log(f"  u0 {u0}: mean u_z {got:.6f}, exact {want:.6f} (se {se:.1e}), per-step loss {1 - c:.3e}")
        assert abs(got - want) < 5 * se
        assert abs(float(u[0].mean())) < 5 * float(u[0].std()) / math.sqrt(u.shape[1])
        rates.append(-math.log(c) / dt)
    # momentum-transfer rates at the two speeds follow (v1/v2)^3 to the
    # small-angle accuracy of the per-step law
    v1, v2 = (u0 / math.sqrt(1 + u0 * u0) for u0 in (0.1, 0.2))
    assert abs(rates[0] / rates[1] / (v2 / v1) ** 3 - 1) < 0.02
    r.close()
