"""The reduced quasi-neutral model on the GPU (pic_hyb_*, through the C ABI)
against its FP64 oracle (oracle/hybrid.py) on the same seeded inputs: the
potential, the plasma's canonical momentum, every particle by id and the
Eq. (7) record, with and without the cell sort; the seeded cold-beam growth
against the model's dispersion relation; and, at the benchmark size, one
step recomputed by the oracle (the solve over the whole grid, sampled
particles one by one)."""
import math
from dataclasses import replace

import numpy as np
import pytest

import synth
from oracle import theory
from oracle.hybrid import Hybrid
from pic_cases import log, periodic_diff, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _pair(pic, wl, diag_every=1, sort_every=0):
    x, u, uz = synth.hybrid_load(wl)
    orc = Hybrid(wl.n, wl.d, wl.dt, wl.nu, x, u, uz, wl.weight, iters=wl.iters)
    g = pic.HybridRun(pic.hyb_desc(wl, x.shape[1], diag_every=diag_every, sort_every=sort_every),
                      x[0], x[1], u[0], u[1], uz)
    return orc, g


def _compare(orc, g, wl, bar):
    a, psi = g.read_grid()
    ea = rel_err(a, orc.a_cur)
    ep = rel_err(psi, orc.psi)
    xg, ug, pzg, ids = g.read_particles()
    o = np.argsort(ids)
    assert np.array_equal(ids[o], np.arange(ids.size))
    L = (np.array(wl.n) * np.array(wl.d))[:, None]
    ex = float(np.max(np.abs(periodic_diff(xg[:, o], orc.x, L)))) if ids.size else 0.0
    eu = float(np.max(np.abs(ug[:, o] - orc.u))) if ids.size else 0.0
    epz = float(np.max(np.abs(pzg[o] - orc.P))) if ids.size else 0.0
    log(f"  a {ea:.2e} psi {ep:.2e} x {ex:.2e} u {eu:.2e} p_z {epz:.2e}")
    assert ea < bar and ep < bar and ex < bar and eu < bar and epz < bar


@pytest.mark.parametrize("sort_every", [0, 7])
def test_hybrid_parity_fp64(pic, sort_every):
    """H1 (64^2, 16 ppc, warm collisional beam): 60 steps, the state and
    every record of Eq. (7)'s terms, FP64 to 1e-9."""
    log(f"case hybrid parity sort_every={sort_every}")
    wl = replace(synth.H1, steps=60)
    orc, g = _pair(pic, wl, sort_every=sort_every)
    _compare(orc, g, wl, 1e-11)                       # after the initial solve
    orecs = orc.step(wl.steps, diag=True)
    g.step(wl.steps)
    _compare(orc, g, wl, 1e-9)
    grecs = g.history()
    assert [r["step"] for r in grecs] == [r["step"] for r in orecs]
    for k in ("beam_energy", "beam_a2", "grad_energy", "a2_energy", "eq7", "W_Ez", "beam_pz", "mean_a"):
        got = np.array([r[k] for r in grecs])
        want = np.array([r[k] for r in orecs])
        assert np.max(np.abs(got - want)) <= 1e-9 * max(1e-12, np.max(np.abs(want))), k
    g.close()


def test_hybrid_graph_matches_direct_launches(pic):
    log("case hybrid graph vs direct")
    wl = replace(synth.H1, steps=20)
    x, u, uz = synth.hybrid_load(wl)
    runs = [pic.HybridRun(pic.hyb_desc(wl, x.shape[1], sort_every=5, flags=f), x[0], x[1], u[0], u[1], uz)
            for f in (0, pic.PIC_FLAG_NO_GRAPH)]
    for _ in range(3):
        for r in runs:
            r.step(wl.steps)
            r.sync()
        (a0, p0), (a1, p1) = runs[0].read_grid(), runs[1].read_grid()
        assert rel_err(a0, a1) < 1e-12 and rel_err(p0, p1) < 1e-12
    for r in runs:
        r.close()


def test_hybrid_seeded_growth_on_gpu(pic):
    """A cold lattice beam with one seeded mode (64 x 8 nodes): the GPU's mode
    grows at the rate of the model's dispersion relation (grid factors
    included), to 1%."""
    log("case hybrid seeded growth")
    wl = synth.HybridWorkload("seeded", (64, 8), (0.2, 0.2), 0.1, 1500, 0.1, 4, synth.U_BEAM, 0.0, 0.0,
                              lattice=True, seed_mode=(1, 1e-5))
    x, u, uz = synth.hybrid_load(wl)
    g = pic.HybridRun(pic.hyb_desc(wl, x.shape[1]), x[0], x[1], u[0], u[1], uz)
    k = 2 * math.pi / (wl.n[0] * wl.d[0])
    xh = np.arange(wl.n[0]) * wl.d[0]
    ts, W = [], []
    for s in range(0, wl.steps, 5):
        a, _ = g.read_grid()
        W.append((abs(np.sum(a.mean(axis=0) * np.exp(-1j * k * xh))) * 2 / wl.n[0]) ** 2)
        ts.append(s * wl.dt)
        g.step(5)
    g.close()
    ts, W = np.array(ts), np.array(W)
    win = theory.fit_growth_window(ts, W, span=5)
    rate = theory.fit_growth_rate(ts, W, win)
    want = theory.hybrid_cold_growth(k, wl.n_b, wl.u_b, 0.0, dx=wl.d[0])
    log(f"  growth {rate:.5f} theory {want:.5f}")
    assert abs(rate / want - 1) < 0.01


def test_hybrid_full_size_step_recomputed(pic):
    """H2 (1024^2 nodes, 64 ppc: 67 108 864 particles; hot collisional beam;
    sort every 20 steps; graph replay), after 25 steps: the oracle rebuilds
    the deposit of every particle, solves Eq. (2) for the next a and compares
    the whole grid; then pushes 2048 sampled particles one by one with the
    GPU's own fields and compares them."""
    log("case hybrid full size H2")
    wl = synth.H2
    x, u, uz = synth.hybrid_load(wl)
    N = x.shape[1]
    g = pic.HybridRun(pic.hyb_desc(wl, N, sort_every=20), x[0], x[1], u[0], u[1], uz)
    del x, u, uz
    g.step(24)
    a2, _ = g.read_grid()                                   # a^23
    g.step(1)
    a1, psi = g.read_grid()                                 # a^24, psi^25
    xs, us, pz, ids = g.read_particles()                    # x^25, u^(24+1/2)
    g.step(1)
    a_new, _ = g.read_grid()                                # a^25
    x2, u2, _, ids2 = g.read_particles()
    g.close()
    assert np.array_equal(np.sort(ids), np.arange(N, dtype=np.uint32))
    orc = Hybrid.from_state(wl.n, wl.d, wl.dt, wl.nu, xs, us, pz, wl.weight, a1, a2, psi, iters=wl.iters)
    a_ref = orc.solve(orc.dep, orc.psi, 2.0 * a1 - a2)
    err = rel_err(a_new, a_ref)
    log(f"  solve over the grid: {err:.2e}")
    assert err < 1e-10
    rng = np.random.default_rng(11)
    pick = rng.choice(N, 2048, replace=False)
    sub = Hybrid.from_state(wl.n, wl.d, wl.dt, wl.nu, xs[:, pick], us[:, pick], pz[pick], wl.weight, a1, a2, psi,
                            iters=wl.iters)
    sub.c0 = orc.c0
    # push only: the particles' step with the GPU's a^25
    abar = sub.interp(a_new, sub.x)
    Gx, Gy = sub.grad_at(a_new, sub.x)
    bp = sub.interp(psi, sub.x) + abar
    uzp = sub.P + abar
    gm = np.sqrt(1 + sub.u[0] ** 2 + sub.u[1] ** 2 + uzp ** 2)
    f = -(uzp / gm - bp) * wl.dt
    un = sub.u + f * np.stack([Gx, Gy])
    gp = np.sqrt(1 + un[0] ** 2 + un[1] ** 2 + uzp ** 2)
    xn = sub.x + wl.dt * un / gp
    pos = {int(i): k for k, i in enumerate(ids2)}
    j = np.array([pos[int(ids[p])] for p in pick])
    L = (np.array(wl.n) * np.array(wl.d))[:, None]
    ex = float(np.max(np.abs(periodic_diff(x2[:, j], xn, L))))
    eu = float(np.max(np.abs(u2[:, j] - un)))
    log(f"  sampled particles: |dx| {ex:.2e} |du| {eu:.2e}")
    assert ex < 1e-10 and eu < 1e-10
