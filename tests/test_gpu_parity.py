"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the
same seeded inputs.  Bars: FP64 mode to round-off growth (fields 1e-5
relative over 200 steps), mixed mode 1e-3 relative; integer decisions
(collision events, particle counts) exactly."""
import math

import numpy as np
import pytest

import synth
from oracle import theory
from pic_cases import by_id, gpu_run, log, oracle_run, periodic_diff, rel_err, stack

pytestmark = pytest.mark.gpu

PRECS = {"fp64": 0, "mixed": 1}


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _random_fields(shape, rng, scale=0.05):
    return scale * rng.standard_normal(shape), scale * rng.standard_normal(shape)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_push_in_frozen_random_fields(pic, prec):
    """Gather + Boris + move of every particle in fixed random E, B over 20
    steps, compared particle by particle (by id) with the oracle."""
    log(f"case push_frozen {prec}")
    wl = synth.beam_plasma((32, 32), ppc=4, u_th_beam=0.3, u_th_plasma=0.05, steps=20)
    parts = synth.load(wl)
    rng = np.random.default_rng(7)
    E, B = _random_fields((3, 1, 32, 32), rng)
    orc = oracle_run(wl, parts)
    orc.f.E[:] = E
    orc.f.B[:] = B
    g = gpu_run(wl, parts, PRECS[prec], flags=pic.PIC_FLAG_FREEZE_FIELDS)
    g.write_fields(E, B)
    for _ in range(wl.steps):
        orc.step(1)
        orc.f.E[:] = E
        orc.f.B[:] = B
    g.step(wl.steps)
    L = np.array([wl.n[0] * wl.d[0], wl.n[1] * wl.d[1]])[:, None]
    tol_x, tol_u = (1e-12, 1e-12) if prec == "fp64" else (2e-5, 2e-5)
    for s in range(2):
        x, u, ids = by_id(*g.read_particles(s))
        sp = orc.species[s]
        xo, uo, io = by_id(sp.x, sp.u, sp.id)
        assert np.array_equal(ids, io)
        assert np.max(np.abs(periodic_diff(x, xo, L))) < tol_x * 20
        assert np.max(np.abs(u - uo)) < tol_u * max(1.0, np.abs(uo).max())
    # J of the last step from the frozen-field push
    _, _, J = g.read_fields()
    assert rel_err(J, orc.f.J) < (1e-12 if prec == "fp64" else 2e-5)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_first_step_current(pic, prec):
    """J^{1/2} of the 64^2 beam-plasma load from zero fields, node by node."""
    log(f"case first_step_current {prec}")
    wl = synth.C1
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    orc.step(1)
    g = gpu_run(wl, parts, PRECS[prec])
    g.step(1)
    E, B, J = g.read_fields()
    jmax = np.abs(orc.f.J).max()
    assert jmax > 0 and J.shape == orc.f.J.shape
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.max(np.abs(J - orc.f.J)) < tol * jmax
    assert rel_err(stack(E, B), stack(orc.f.E, orc.f.B)) < tol


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-5), ("mixed", 1e-3)])
def test_c1_fields_200_steps(pic, prec, bar):
    """The 64^2, 16 ppc beam-plasma case over 200 steps: stacked relative
    L2 error of (E, B) at every 10th step within the bar; diagnostic
    records (field energies, kinetic energies) agree."""
    log(f"case c1_200 {prec}")
    wl = synth.C1
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS[prec], diag_every=10)
    worst = 0.0
    orecs = []
    for blk in range(20):
        orecs += orc.step(10, diag=True)[:1]
        g.step(10)
        E, B, _ = g.read_fields()
        err = rel_err(stack(E, B), stack(orc.f.E, orc.f.B))
        worst = max(worst, err)
    log(f"  worst stacked field error {worst:.3e}")
    assert worst < bar
    hist = g.history()
    assert [h["step"] for h in hist] == list(range(0, 200, 10))
    for h, o in zip(hist[1:], orecs[1:]):
        assert np.allclose(h["W"], o["W"], rtol=10 * bar, atol=1e-12)
        assert np.allclose(h["kinetic"], o["kinetic"], rtol=1e-6 if prec == "mixed" else 1e-12)
        assert h["n_particles"].tolist() == [p.id.size for p in parts]


def test_collisional_return_current_parity(pic):
    """Scattering of the plasma electrons (nu = 0.05): the GPU makes exactly
    the oracle's collision decisions (integer compare of the same Philox
    draw) and the fields stay within the FP64 bar."""
    log("case collisional fp64")
    wl = synth.beam_plasma((64, 64), ppc=16, u_th_beam=0.1, nu=0.05, steps=100)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS["fp64"], diag_every=1)
    orecs = orc.step(wl.steps, diag=True)
    g.step(wl.steps)
    hist = g.history()
    assert [h["collisions"] for h in hist] == [o["collisions"] for o in orecs]
    assert sum(o["collisions"] for o in orecs) > 1000
    E, B, _ = g.read_fields()
    assert rel_err(stack(E, B), stack(orc.f.E, orc.f.B)) < 1e-5
    x, u, ids = by_id(*g.read_particles(1))
    sp = orc.species[1]
    xo, uo, io = by_id(sp.x, sp.u, sp.id)
    assert np.array_equal(ids, io)
    assert np.max(np.abs(u - uo)) < 1e-6


def test_overflow_and_relayout_path(pic):
    """A sheet of fast particles streams into empty tiles: incoming movers
    overflow the tiles' reserves, the store is re-laid out on the device,
    no particle is lost and the run still matches the oracle."""
    log("case rebin fp64")
    n, T = 32, 8
    sc = synth.SpeciesCfg("sheet", 1.0, 4, (0.0, 0.0, 0.0), 0.0)
    wl = synth.Workload("sheet", 2, (n, n), (0.2, 0.2), 0.1, 24, (sc,))
    rng = np.random.default_rng(3)
    N = n * n * 4
    x = np.empty((2, N))
    x[0] = rng.uniform(0, 8 * 0.2, N)          # all in the first tile column
    x[1] = rng.uniform(0, n * 0.2, N)
    u = np.zeros((3, N))
    u[0] = 7.0                                  # 0.49 cells per step along +x
    u[1] = 0.3 * rng.standard_normal(N)
    parts = [synth.Particles(x, u, np.arange(N, dtype=np.uint32))]
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS["fp64"], tile=T, diag_every=1)
    orc.step(wl.steps)
    g.step(wl.steps)
    rec = g.history()[-1]
    assert rec["rebins"] >= 1
    xg, ug, ig = by_id(*g.read_particles(0))
    assert ig.size == N and np.array_equal(ig, np.arange(N))
    sp = orc.species[0]
    xo, uo, io = by_id(sp.x, sp.u, sp.id)
    L = np.array([n * 0.2, n * 0.2])[:, None]
    assert np.max(np.abs(periodic_diff(xg, xo, L))) < 1e-9
    assert np.max(np.abs(ug - uo)) < 1e-9
    E, B, _ = g.read_fields()
    assert rel_err(stack(E, B), stack(orc.f.E, orc.f.B)) < 1e-9


def test_graph_replay_matches_direct_launches(pic):
    log("case graph vs direct")
    wl = synth.C1
    parts = synth.load(wl)
    a = gpu_run(wl, parts, PRECS["fp64"])
    b = gpu_run(wl, parts, PRECS["fp64"], flags=pic.PIC_FLAG_NO_GRAPH)
    for _ in range(3):       # several replays with host work in between
        a.step(10)
        b.step(10)
        a.sync()
        b.sync()
        Ea, Ba, Ja = a.read_fields()
        Eb, Bb, Jb = b.read_fields()
        assert rel_err(stack(Ea, Ba), stack(Eb, Bb)) < 1e-12
        assert rel_err(Ja, Jb) < 1e-12
    # every step of `a` was one graph replay, every step of `b` direct launches
    ia, ib = a.info(), b.info()
    assert ia["graph"] == 1 and ia["graph_launches"] == 30 and ia["direct_steps"] == 0
    assert ib["graph"] == 0 and ib["graph_launches"] == 0 and ib["direct_steps"] == 30
    assert ia["steps_enqueued"] == ib["steps_enqueued"] == 30 and ia["static_scratch"] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_device_loader(pic, prec):
    """The device loader: exactly ppc per cell, zero mean transverse
    momentum, zero net current, drift and spread as requested, unique ids."""
    log(f"case device loader {prec}")
    wl = synth.C1
    g, sp = pic.workload_descs(wl, precision=PRECS[prec], flags=pic.PIC_FLAG_TRACK_IDS)
    r = pic.Run(g, sp)
    parts = []
    for s, sc in enumerate(wl.species):
        x, u, ids = r.read_particles(s)
        assert x.shape[1] == wl.cells * sc.ppc
        ix = np.floor(x[0] / wl.d[0]).astype(int)
        iy = np.floor(x[1] / wl.d[1]).astype(int)
        assert np.all(np.bincount(iy * wl.n[0] + ix, minlength=wl.cells) == sc.ppc)
        assert abs(u[0].mean()) < 1e-6 and abs(u[1].mean()) < 1e-6
        N = u.shape[1]
        assert abs(u[2].mean() - sc.drift_u[2]) < 5 * sc.u_th / math.sqrt(N) + (0.2 if s == 1 else 0)
        assert abs(u[0].std() / sc.u_th - 1) < 0.05
        parts.append(synth.Particles(x, u, ids))
    ids = np.concatenate([p.id for p in parts])
    assert len(np.unique(ids)) == ids.size
    jz = synth.net_current_z(parts, wl.species)
    assert abs(jz) < (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cold_beam_weibel_rate_gpu(pic, prec):
    """Seeded single-mode cold-beam filamentation on the GPU grows at the
    cold-fluid rate (3%) and at the oracle's fitted rate (2%)."""
    log(f"case weibel {prec}")
    m, nx, ny = 4, 64, 8
    wl = synth.beam_plasma((nx, ny), ppc=4, u_th_beam=0.0, u_th_plasma=0.0, lattice=True, steps=660)
    parts = synth.load(wl)
    k = 2 * math.pi * m / (nx * 0.2)
    xh = (np.arange(nx) + 0.5) * 0.2
    B0 = np.zeros((3, 1, ny, nx))
    B0[1, 0] = 1e-6 * np.cos(k * xh)[None, :]
    g = gpu_run(wl, parts, PRECS[prec])
    g.write_fields(None, B0)
    orc = oracle_run(wl, parts)
    orc.f.B[:] = B0
    amps_g, amps_o = [], []
    for _ in range(wl.steps // 10):
        _, B, _ = g.read_fields()
        amps_g.append(abs(np.sum(B[1, 0].mean(axis=0) * np.exp(-1j * k * xh))) * 2 / nx)
        amps_o.append(abs(np.sum(orc.f.B[1, 0].mean(axis=0) * np.exp(-1j * k * xh))) * 2 / nx)
        g.step(10)
        orc.step(10)
    t = np.arange(len(amps_g)) * 10 * wl.dt
    Wo = np.array(amps_o) ** 2
    win = theory.fit_growth_window(t, Wo, span=5)
    go = theory.fit_growth_rate(t, Wo, win)
    gg = theory.fit_growth_rate(t, np.array(amps_g) ** 2, win)
    want = theory.weibel_cold_rate(k, theory.beam_plasma_species())
    log(f"  rates gpu {gg:.5f} oracle {go:.5f} theory {want:.5f} window {win}")
    assert abs(gg / go - 1) < 0.02
    assert abs(gg / want - 1) < 0.03


# --------------------------------------------------------------------------- 3D
@pytest.mark.parametrize("prec,bar,n", [("fp64", 1e-5, (16, 16, 32)), ("mixed", 1e-3, (16, 16, 32)),
                                         ("fp64", 1e-5, (32, 32, 64))])
def test_3d_fields_and_particles(pic, prec, bar, n):
    """3D3V (beam along z, collisionless, 8^3 tiles) on a 16x16x32 box and
    (FP64) on the reduced 32x32x64 grid: fields within the bar every 10 steps
    over 60 steps and particles by id at the end."""
    log(f"case 3d {prec} {n}")
    wl = synth.beam_plasma(n, ppc=4, u_th_beam=0.1, u_th_plasma=0.02, steps=60)
    parts = synth.load(wl)
    orc = oracle_run(wl, parts)
    g = gpu_run(wl, parts, PRECS[prec], diag_every=10)
    worst = 0.0
    for _ in range(wl.steps // 10):
        orc.step(10)
        g.step(10)
        E, B, J = g.read_fields()
        worst = max(worst, rel_err(stack(E, B), stack(orc.f.E, orc.f.B)))
    log(f"  worst stacked field error {worst:.3e}")
    assert worst < bar
    assert rel_err(J, orc.f.J) < 10 * bar
    L = np.array([n * 0.2 for n in wl.n])[:, None]
    for s in range(2):
        x, u, ids = by_id(*g.read_particles(s))
        sp = orc.species[s]
        xo, uo, io = by_id(sp.x, sp.u, sp.id)
        assert np.array_equal(ids, io)
        tol = 1e-9 if prec == "fp64" else 1e-4
        assert np.max(np.abs(periodic_diff(x, xo, L))) < tol
        assert np.max(np.abs(u - uo)) < tol * 10


def test_3d_device_loader_and_continuity(pic):
    """3D device load: exactly ppc per cell; after one step the current
    satisfies rho^1 - rho^0 + dt div J = 0 on every node (rho from the
    particles read back, by the oracle's CIC deposit)."""
    log("case 3d loader + continuity")
    import oracle
    wl = synth.beam_plasma((16, 16, 16), ppc=8, u_th_beam=0.3, u_th_plasma=0.05)
    g, sp = pic.workload_descs(wl, precision=PRECS["fp64"], flags=pic.PIC_FLAG_TRACK_IDS)
    r = pic.Run(g, sp)
    before = [r.read_particles(s) for s in range(2)]
    for (x, u, ids), sc in zip(before, wl.species):
        idx = [np.floor(x[a] / wl.d[a]).astype(int) for a in range(3)]
        flat = (idx[2] * wl.n[1] + idx[1]) * wl.n[0] + idx[0]
        assert np.all(np.bincount(flat, minlength=wl.cells) == sc.ppc)
    r.step(1)
    after = [r.read_particles(s) for s in range(2)]
    _, _, J = r.read_fields()

    def rho(parts):
        sps = [oracle.SpeciesState(sc.q, sc.m, sc.weight, 0.0, np.ascontiguousarray(x), np.ascontiguousarray(u),
                                   ids) for (x, u, ids), sc in zip(parts, wl.species)]
        return oracle.OracleRun(3, wl.n, wl.d, wl.dt, sps, 1).rho()
    o = oracle.OracleRun(3, wl.n, wl.d, wl.dt, [], 1)
    res = rho(after) - rho(before) + wl.dt * o.divergence(J)
    assert np.max(np.abs(res)) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_3d_face_crossings_current(pic, prec):
    """J^{1/2} node by node for crafted 3D moves from zero fields: every face
    crossed in both directions on each axis (single-face path), pairs and
    triples of faces (general window) and stayers, in cells on both sides of
    the 8^3 tile boundaries and inside the tiles."""
    log(f"case 3d face crossings {prec}")
    wl = synth.beam_plasma((16, 16, 16), ppc=2, u_th_beam=0.0, u_th_plasma=0.0, steps=1)
    rng = np.random.default_rng(7)
    cells = [0, 3, 7, 8, 15]
    xs, us = [], []
    for cx in cells:
        for cy in cells:
            for cz in cells:
                for kind in range(8):
                    # kind bit a: cross along axis a; the sign comes from the draw
                    off = rng.uniform(0.2, 0.8, 3)
                    u = rng.normal(0.0, 0.05, 3)
                    for a in range(3):
                        if kind >> a & 1:
                            up = rng.random() < 0.5
                            off[a] = rng.uniform(0.75, 0.95) if up else rng.uniform(0.05, 0.25)
                            u[a] = (1.0 if up else -1.0) * rng.uniform(1.5, 3.0)
                    xs.append((np.array([cx, cy, cz]) + off) * np.array(wl.d))
                    us.append(u)
    x = np.ascontiguousarray(np.array(xs).T)
    u = np.ascontiguousarray(np.array(us).T)
    parts = [synth.Particles(x, u, np.arange(x.shape[1], dtype=np.uint32)),
             synth.Particles(np.zeros((3, 0)), np.zeros((3, 0)), np.zeros(0, dtype=np.uint32))]
    orc = oracle_run(wl, parts)
    orc.step(1)
    g = gpu_run(wl, parts, PRECS[prec])
    g.step(1)
    _, _, J = g.read_fields()
    jmax = np.abs(orc.f.J).max()
    assert jmax > 0 and J.shape == orc.f.J.shape
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert np.max(np.abs(J - orc.f.J)) < tol * jmax
    xg, ug, ids = by_id(*g.read_particles(0))
    L = np.array([n * 0.2 for n in wl.n])[:, None]
    assert np.array_equal(ids, np.arange(x.shape[1]))
    assert np.max(np.abs(periodic_diff(xg, orc.species[0].x, L))) < (1e-12 if prec == "fp64" else 1e-5)
    g.close()


_TS_CACHE = {}


def _two_stream_oracle(wl, parts, k, zh):
    """E_z mode amplitudes and the final fields of the oracle run (cached:
    both precisions compare against the same FP64 run)."""
    if "amps" not in _TS_CACHE:
        orc = oracle_run(wl, parts)
        amps = []
        for _ in range(wl.steps):
            orc.step(1)
            amps.append(abs(np.sum(orc.f.E[2].mean(axis=(1, 2)) * np.exp(-1j * k * zh))) * 2 / len(zh))
        _TS_CACHE["amps"] = np.array(amps)
        _TS_CACHE["E"] = [e.copy() for e in orc.f.E]
    return _TS_CACHE["amps"], _TS_CACHE["E"]


@pytest.mark.parametrize("prec,bar", [("fp64", 1e-8), ("mixed", 0.1)])
def test_two_stream_growth_3d_gpu(pic, prec, bar):
    """3D longitudinal instability: the lattice-loaded cold beam (n_b = 0.1,
    gamma = 3) on its return current, velocity-seeded at mode 4 along the
    beam of an 8 x 8 x 128 box, 800 steps.  The GPU's E_z mode grows at the
    oracle's rate (2%) and at the cold-fluid two-stream rate (3%); at the end
    the mode amplitude matches the oracle's and so does E_z node by node
    (FP64: 1e-8; mixed: 3% on the mode, 10% node by node -- early on the
    beam's per-step u_z increments, ~1e-7, are below the FP32 spacing at
    u_z = 2.83, 2.4e-7, which shifts the uniform part of E_z by a few % of
    the mode's amplitude)."""
    log(f"case two-stream 3d {prec}")
    m, nz = 4, 128
    wl = synth.beam_plasma((8, 8, nz), ppc=8, u_th_beam=0.0, u_th_plasma=0.0, lattice=True, steps=800)
    parts = synth.load(wl)
    k = 2 * math.pi * m / (nz * 0.2)
    parts[0].u[2] += 1e-4 * np.sin(k * parts[0].x[2])
    zh = (np.arange(nz) + 0.5) * 0.2
    amps_o, E_o = _two_stream_oracle(wl, parts, k, zh)
    g = gpu_run(wl, parts, PRECS[prec])
    amps = []
    for _ in range(wl.steps):
        g.step(1)
        E, _, _ = g.read_fields()
        amps.append(abs(np.sum(np.asarray(E[2]).mean(axis=(1, 2)) * np.exp(-1j * k * zh))) * 2 / nz)
    t = (np.arange(wl.steps) + 1) * wl.dt
    win = theory.fit_growth_window(t, amps_o ** 2)
    assert win[1] - win[0] > 150
    go = theory.fit_growth_rate(t, amps_o ** 2, win)
    gg = theory.fit_growth_rate(t, np.array(amps) ** 2, win)
    want = theory.two_stream_cold_rate(k, theory.beam_plasma_species(0.1, math.sqrt(8.0)))
    log(f"  rates gpu {gg:.5f} oracle {go:.5f} theory {want:.5f} window {win}")
    assert abs(gg / go - 1) < 0.02
    assert abs(gg / want - 1) < 0.03
    assert abs(amps[-1] / amps_o[-1] - 1) < (1e-8 if prec == "fp64" else 3e-2)
    E, _, _ = g.read_fields()
    assert rel_err(np.asarray(E[2]), E_o[2]) < bar
    g.close()


_C3S_CACHE = {}


@pytest.mark.parametrize("prec,w_bar,k_bar", [("fp64", 1e-10, 1e-12), ("mixed", 1e-4, 1e-6)])
def test_c3_physics_energy_records(pic, prec, w_bar, k_bar):
    """The C3 workload's physics (beam u_th 0.3 with its return current
    scattering at nu = 0.05, 64 particles per cell per species) on a 128^2
    box the oracle can step, 300 steps: every diagnostic record's six field
    energies W_i and two kinetic energies against the FP64 oracle's -- the
    error of the mixed-precision path on this workload, stated per record."""
    log(f"case c3 physics energy records {prec}")
    wl = synth.beam_plasma((128, 128), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=300,
                           name="c3-128")
    parts = synth.load(wl)
    if "recs" not in _C3S_CACHE:
        orc = oracle_run(wl, parts)
        _C3S_CACHE["recs"] = orc.step(wl.steps, diag=True)[::10]
    ro = _C3S_CACHE["recs"]
    g = gpu_run(wl, parts, PRECS[prec], diag_every=10)
    g.step(wl.steps)
    hg = g.history()
    g.close()
    assert [h["step"] for h in hg] == [r["step"] for r in ro]
    Wg = np.array([h["W"] for h in hg])
    Wo = np.array([r["W"] for r in ro])
    kg = np.array([h["kinetic"][:2] for h in hg])
    ko = np.array([r["kinetic"][:2] for r in ro])
    w_err = float(np.max(np.abs(Wg - Wo)[1:] / np.abs(Wo)[1:]))
    k_err = float(np.max(np.abs(kg - ko) / ko))
    log(f"  worst per-record W_i error {w_err:.2e}, kinetic {k_err:.2e}")
    assert w_err < w_bar and k_err < k_bar
