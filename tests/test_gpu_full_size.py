"""Parity at the full benchmark size, in the launch configuration bench.py
times (C3 mixed / C2 FP64: 1024^2 cells, 64 particles per cell per species,
134 217 728 particles, tile 16, device loader, graph replay, diagnostics
every 10 steps).  The oracle cannot step this size in a test, so it checks
sampled outputs one by one: for random particles (by id) it recomputes one
step -- gather from the GPU's own E^n, B^n, Boris push, move, scattering draw
-- and compares position and momentum; integer outputs (scattering decisions,
particle counts) must match exactly."""
import math

import numpy as np
import pytest

import oracle
import synth
from pic_cases import log

pytestmark = pytest.mark.gpu

SAMPLE = 1536          # particles per species


@pytest.fixture(scope="module")
def pic():
    from paper_0808_4078_amd import pic as p
    p.lib()
    return p


def _node_currents(orc, wl, E_step, before, after, nodes):
    """J at the given nodes from an oracle deposit of every particle within
    reach of them (2.5 cells per axis, periodic), each pushed by the oracle
    from its state at the start of the step."""
    L = np.array(wl.n, dtype=float) * np.array(wl.d)
    Jacc = np.zeros_like(orc.f.J)
    for s, sc in enumerate(wl.species):
        x0, u0, _ = before[s]
        near = np.zeros(x0.shape[1], dtype=bool)
        for (i, j) in nodes:
            c = np.array([i * wl.d[0], j * wl.d[1]])[:, None]
            dd = x0 - c
            dd -= L[:, None] * np.round(dd / L[:, None])
            near |= (np.abs(dd[0]) < 2.5 * wl.d[0]) & (np.abs(dd[1]) < 2.5 * wl.d[1])
        qmdt2 = sc.q * wl.dt / (2.0 * sc.m)
        qw = sc.q * sc.weight
        for a in np.flatnonzero(near):
            x = x0[:, a]
            Eg, Bg = orc.gather(x)
            u = oracle.boris(u0[:, a], Eg, Bg, qmdt2)
            g_ = math.sqrt(1.0 + float(u @ u))
            orc.deposit(qw, x, x + wl.dt * u[:2] / g_, u[2] / g_, Jacc)
    return Jacc


def _sampled_step(pic, prec, warm, x_tol, u_tol, flags=0, j_nodes=0, shape=0):
    wl = synth.C3
    p = pic.PIC_PREC_MIXED if prec == "mixed" else pic.PIC_PREC_FP64
    g, sp = pic.workload_descs(wl, precision=p, tile=16, diag_every=10, flags=flags, shape=shape)
    tracked = [sc.nu > 0 or bool(flags & pic.PIC_FLAG_TRACK_IDS) for sc in wl.species]
    r = pic.Run(g, sp)
    r.step(warm)
    r.sync()
    E, B, _ = r.read_fields()                       # E^n, B^n of the step about to run
    before = [r.read_particles(s) for s in range(len(wl.species))]
    r.step(1)
    r.sync()
    after = [r.read_particles(s) for s in range(len(wl.species))]
    _, _, J_gpu = r.read_fields()
    d0 = r.history()[-1]
    n_expect = [wl.cells * sc.ppc for sc in wl.species]
    r.close()
    # a particle-free oracle grid holding the GPU's fields, for the gather
    orc = oracle.OracleRun(2, wl.n, wl.d, wl.dt, [oracle.SpeciesState(-1.0, 1.0, 1.0, 0.0, np.zeros((2, 0)),
                                                                      np.zeros((3, 0)),
                                                                      np.zeros(0, dtype=np.uint32))], wl.seed)
    orc.f.E[...] = E
    orc.f.B[...] = B
    L = np.array(wl.n, dtype=float) * np.array(wl.d)
    rng = np.random.default_rng(2024)
    step = warm                                       # index of the step just taken
    worst_x = worst_u = 0.0
    scattered = 0
    for s, sc in enumerate(wl.species):
        (x0, u0, i0), (x1, u1, i1) = before[s], after[s]
        assert x0.shape[1] == n_expect[s] and x1.shape[1] == n_expect[s]
        if not tracked[s]:
            continue          # no ids carried: particles cannot be followed across a step
        ids = rng.choice(i0, size=SAMPLE, replace=False)
        ids.sort()
        j0 = np.flatnonzero(np.isin(i0, ids))
        j1 = np.flatnonzero(np.isin(i1, ids))
        j0 = j0[np.argsort(i0[j0])]
        j1 = j1[np.argsort(i1[j1])]
        assert np.array_equal(i0[j0], ids) and np.array_equal(i1[j1], ids)
        thr = oracle.collision_threshold(sc.nu, wl.dt) if sc.nu > 0 else 0
        qmdt2 = sc.q * wl.dt / (2.0 * sc.m)
        for a, b in zip(j0, j1):
            x = x0[:, a]
            Eg, Bg = orc.gather(x)
            u = oracle.boris(u0[:, a], Eg, Bg, qmdt2)
            g_ = math.sqrt(1.0 + float(u @ u))
            xn = x + wl.dt * u[:2] / g_
            un, hit = (oracle.collide(u, int(i0[a]), step, wl.seed, 0, thr) if sc.nu > 0 else (u, False))
            scattered += int(hit)
            dx = xn - x1[:, b]
            dx -= L * np.round(dx / L)
            worst_x = max(worst_x, float(np.max(np.abs(dx) / np.array(wl.d))))
            worst_u = max(worst_u, float(np.max(np.abs(un - u1[:, b])) / (1.0 + float(np.max(np.abs(un))))))
    log(f"  {prec}: sampled {SAMPLE} particles of each tracked species, worst |dx|/d {worst_x:.2e}, "
        f"worst |du| {worst_u:.2e}, scattered {scattered}")
    if j_nodes:
        nodes = [tuple(int(v) for v in rng.integers(0, wl.n[0], 2)) for _ in range(j_nodes)]
        Jo = _node_currents(orc, wl, E, before, after, nodes)
        worst_j, scale = 0.0, 0.0
        for (i, j) in nodes:
            for c in range(3):
                worst_j = max(worst_j, abs(float(J_gpu[c, 0, j, i] - Jo[c, 0, j, i])))
                scale = max(scale, abs(float(Jo[c, 0, j, i])))
        log(f"  J at {j_nodes} nodes: worst |J_gpu - J_oracle| {worst_j:.2e} (largest |J| {scale:.2e})")
        assert worst_j < 1e-5 * max(scale, 1e-3)
    assert worst_x < x_tol and worst_u < u_tol
    assert 0 < scattered < SAMPLE // 20
    assert list(d0["n_particles"]) == n_expect
    return worst_x, worst_u


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_full_size_mixed_sampled_step(pic, shape):
    """In every launch shape of the particle kernel (bench.py takes the one
    pic_tune_shape finds fastest)."""
    log(f"case full size C3 mixed (sampled), shape {shape}")
    _sampled_step(pic, "mixed", 10, 2e-5, 2e-5, shape=shape)


def test_full_size_fp64_sampled_step(pic):
    log("case full size C2 fp64 (sampled)")
    _sampled_step(pic, "fp64", 10, 1e-10, 1e-10)


def test_full_size_mixed_both_species(pic):
    """The same with ids carried for the beam too (PIC_FLAG_TRACK_IDS), so both
    species are sampled, after 30 warm-up steps; and the current of the step
    at 8 random nodes (deposit + FP64 grid reduction) against an oracle
    deposit of every particle that reaches them."""
    log("case full size C3 mixed, ids tracked (sampled)")
    _sampled_step(pic, "mixed", 30, 2e-5, 2e-5, flags=pic.PIC_FLAG_TRACK_IDS, j_nodes=8)


@pytest.mark.parametrize("shape", [0, 1, 2, 3, 4])
def test_full_size_c4_gauss_and_counts(pic, shape):
    """C4 at its full size in the configuration bench.py times (256 x 256 x
    512 cells, 8 particles per cell per species, 536 870 912 particles, 8^3
    tiles, 200% store reserve): reading the particles back is out of reach,
    so the check is on properties that hold at any size -- Gauss's law kept
    to the FP32 level of the mixed deposit at every record, and every
    particle present; in every launch shape of the particle kernel."""
    log(f"case full size C4 mixed (Gauss residual, counts), shape {shape}")
    import bench
    wl = synth.C4
    g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=8, diag_every=10,
                               flags=pic.PIC_FLAG_GAUSS_RESIDUAL, reserve=bench.RESERVE_3D, shape=shape)
    r = pic.Run(g, sp)
    r.step(31)
    r.sync()
    h = r.history()
    r.close()
    n_expect = [wl.cells * sc.ppc for sc in wl.species]
    dev = max(x["rho_dev"] for x in h)
    worst = max(x["gauss_resid"] for x in h)
    log(f"  records {len(h)}, max |rho - rho_0| {dev:.3e}, worst residual {worst:.3e}")
    assert [x["step"] for x in h] == [0, 10, 20, 30]
    assert dev > 1e-3 and worst < 1e-4 * dev
    for x in h:
        assert list(x["n_particles"][:2]) == n_expect


def test_full_size_c5_counts_and_members(pic):
    """C5 at its full size (256 uneven 2D runs, 1.68e9 particles) as one
    batch, 20 steps: every member keeps all its particles, and three members
    of different sizes match their twins stepped alone exactly (mixed
    precision: the FP64 tile sums of FP32 terms do not depend on order)."""
    log("case full size C5 (counts, members vs alone)")
    members = synth.c5_members()

    def make(wl):
        g, sp = pic.workload_descs(wl, precision=pic.PIC_PREC_MIXED, tile=16, diag_every=10)
        return pic.Run(g, sp)
    runs = [make(wl) for wl in members]
    batch = pic.Batch(runs)
    batch.step(20)
    batch.sync()
    for r, wl in zip(runs, members):
        n = r.diagnostics()["n_particles"][:2].tolist()
        assert n == [wl.cells * sc.ppc for sc in wl.species], (wl.name, n)
    picks = sorted({0, len(members) // 2, len(members) - 1} |
                   {int(np.argmax([wl.cells for wl in members]))})
    for i in picks:
        alone = make(members[i])
        alone.step(20)
        alone.sync()
        Ea, Ba, _ = alone.read_fields()
        Eb, Bb, _ = runs[i].read_fields()
        log(f"  member {i} ({members[i].n[0]}^2): max |field difference| "
            f"{max(np.abs(Ea - Eb).max(), np.abs(Ba - Bb).max()):.1e}")
        assert np.array_equal(Ea, Eb) and np.array_equal(Ba, Bb)
        alone.close()
    batch.close()
    for r in runs:
        r.close()
