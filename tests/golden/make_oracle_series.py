"""Writes the oracle's long-run field-energy series into tests/golden/.

Test infrastructure: this script calls only the FP64 oracle (``oracle/``)
and the seeded input generator (``synth/``), never the GPU library.  The
series are too long for the GPU tests to recompute (minutes to tens of
minutes of host time), so the tests read them from here.

Families:

* ``c3phys``: the headline workload's physics (beam n_b = 0.1, u_z = sqrt(8),
  u_th = 0.3; return-current plasma u_th = 0.01 scattering off the ions at
  nu = 0.05; 64 particles per cell per species; dx = 0.2, dt = 0.1) on a
  256^2 box for 1000 steps: the growth of the transverse magnetic energy is
  the Weibel / resistive filamentation of the beam (theory part; field-energy
  diagnostic of the 2D PIC paragraph), against which the GPU's mixed and
  FP64 paths are compared.
* ``c3full``: the headline workload itself (C3: 1024^2 cells, 64 particles
  per cell per species, 134 217 728 particles) for 800 steps, through the
  linear filamentation (t ~ 25 to 65) into saturation: the full-size series
  the GPU's mixed and FP64 runs of the benchmark workload are compared with
  (about two hours of host time on 8 cores).
* ``c4phys``: the 3D workload's physics (C4: beam u_th = 0.1, 8 particles
  per cell per species, collisionless; dx = 0.2, dt = 0.1) on a 64 x 64 x
  128 box (8 388 608 particles) for 500 steps, through the 3D filamentation
  of the beam into saturation (about ten minutes of host time on 8 cores).
* ``c3coul``: C3's physics on 256^2 with the return-current plasma on the
  Coulomb small-angle model (nu = 0.05 at the reference speed 0.1, every
  plasma particle turned every step) for 600 steps (about five minutes).
* ``c3bin``: C3's physics on 256^2 with the binary electron-electron
  collisions on (beam-plasma and plasma-plasma pairs in every cell, nu_ee =
  0.05 at the reference speed 0.1) for 300 steps; the records add the
  number of scattered pairs (about 16 minutes of host time on 8 cores).
* ``hyb-d``: the paper's collisional hot-beam case (d) in its reduced
  quasi-neutral model (oracle/hybrid.py): 128^2 nodes over 20 x 20 c/w_p,
  64 beam particles per cell, v_b = 0.9 c, u_th = 0.37, nu = 0.15, dt =
  0.0625, to 20 plasma periods (2011 steps; about 35 minutes); records every
  10 steps of W_Bperp, the beam's energy and z momentum, W_Ez and Eq. (7).
* ``paper-a`` .. ``paper-d``: the four 2D cases of the paper at its own
  parameters (2D PIC paragraph; captions of Figs. 1-2): 160^2 cells of
  0.125 c/w_p, 64 particles per cell per species, v_b = 0.9 c, n_p/n_b = 9,
  cold (u_th 0.01) or hot (u_th 0.37) beam, nu = 0 or 0.15, run to 20 plasma
  periods with dt = 0.0625.

Every record is taken at the start of the step (time level n): W_i = sum
F_i^2 dV of the six components, the time-centred kinetic energy per species,
the z momentum of the particles and of the field, and the scattering count.
The paper cases also store, every 50 steps, the transverse magnetic energy
spectrum |B_x(k)|^2 + |B_y(k)|^2 summed over the rings |k| = m 2 pi / L,
m = 0..4 (the k-resolved growth of Eq. (12)).

Usage: python tests/golden/make_oracle_series.py [c3phys] [c3full] [c3coul] [c3bin] [c4phys] [hyb-d] [paper-a] ...
(no argument: all; ``annotate`` only rewrites the fit line of the c3phys
header from its stored data).  Set OMP_NUM_THREADS to share the host; the results do
not depend on the thread count.
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# The headline physics on a box the oracle can step through its linear phase.
C3PHYS = synth.beam_plasma((256, 256), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=1000,
                           name="c3phys-256")
C3PHYS_DIAG = 10

# The headline workload at its full size, through its linear phase.
C3FULL = synth.beam_plasma((1024, 1024), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=800,
                           name="c3-1024")

# The headline physics with the plasma on the Coulomb model (the benchmark's Coulomb line).
C3COUL = synth.beam_plasma((256, 256), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=600,
                           coll_model=1, coll_vref=0.1, name="c3coul-256")

# The headline physics with binary collisions (the values of the benchmark's binary line).
C3BIN = synth.beam_plasma((256, 256), ppc=64, u_th_beam=0.3, u_th_plasma=0.01, nu=0.05, steps=300,
                          nu_ee=0.05, ee_vref=0.1, name="c3bin-256")

# The 3D workload's physics on a box the oracle can step through its linear phase.
C4PHYS = synth.beam_plasma((64, 64, 128), steps=500, ppc=8, u_th_beam=0.1, name="c4phys-64x64x128")

# The paper's four 2D cases.
PAPER_N, PAPER_DX, PAPER_DT = 160, 0.125, 0.0625
PAPER_STEPS = int(round(20 * 2 * math.pi / PAPER_DT))
PAPER_VB = 0.9
PAPER_CASES = {"a": (0.01, 0.0), "b": (0.01, 0.15), "c": (0.37, 0.0), "d": (0.37, 0.15)}
PAPER_DIAG = 10
PAPER_MODE_EVERY = 50


def paper_workload(case: str):
    uth, nu = PAPER_CASES[case]
    u_b = PAPER_VB / math.sqrt(1.0 - PAPER_VB * PAPER_VB)
    return synth.beam_plasma((PAPER_N, PAPER_N), d=(PAPER_DX, PAPER_DX), dt=PAPER_DT, steps=PAPER_STEPS,
                             ppc=64, u_th_beam=uth, nu=nu, u_beam=u_b, name=f"paper-{case}")


def ring_spectrum(Bx: np.ndarray, By: np.ndarray, d: float, mmax: int = 4) -> np.ndarray:
    """|B_x(k)|^2 + |B_y(k)|^2 of a square 2D plane summed over the rings
    round(|k| L / 2 pi) = m, m = 0..mmax."""
    n = Bx.shape[-1]
    L = n * d
    kx = np.fft.fftfreq(n, d=d) * 2 * math.pi
    K = np.sqrt(kx[None, :] ** 2 + kx[:, None] ** 2)
    shell = np.rint(K / (2 * math.pi / L)).astype(int)
    P = np.abs(np.fft.fft2(Bx)) ** 2 + np.abs(np.fft.fft2(By)) ** 2
    return np.bincount(shell.ravel(), weights=P.ravel(), minlength=mmax + 1)[:mmax + 1]


def _species(wl, parts):
    return [oracle.SpeciesState(sc.q, sc.m, sc.weight, sc.nu, p.x.copy(), p.u.copy(), p.id.copy(),
                                sc.coll_model, sc.coll_vref, sc.binary and wl.nu_ee > 0.0)
            for sc, p in zip(wl.species, parts)]


def _header(wl, diag_every, extra=()):
    sp = wl.species
    lines = [f"# oracle series {wl.name}: written by tests/golden/make_oracle_series.py (FP64 oracle only)",
             f"# grid {'x'.join(map(str, wl.n))} d {wl.d[0]} dt {wl.dt} steps {wl.steps} seed {wl.seed:#x}",
             f"# beam n {sp[0].density} ppc {sp[0].ppc} u_z {sp[0].drift_u[2]!r} u_th {sp[0].u_th}",
             f"# plasma n {sp[1].density} ppc {sp[1].ppc} u_th {sp[1].u_th} nu {sp[1].nu} (return current, "
             f"Newton-cancelled)",
             f"# record every {diag_every} steps at time level n: step time W_Ex W_Ey W_Ez W_Bx W_By W_Bz "
             f"K_beam K_plasma p_z(particles) p_z(field) collisions"]
    return lines + [f"# {e}" for e in extra]


def _rec_line(r, dt):
    W = " ".join(f"{v:.17e}" for v in r["W"])
    K = " ".join(f"{v:.17e}" for v in r["kinetic"][:2])
    return (f"{r['step']} {r['step'] * dt:.10g} {W} {K} {r['p_particles'][2]:.17e} {r['p_field'][2]:.17e} "
            f"{r['collisions']}")


def run_c3phys(path, wl=C3PHYS):
    parts = synth.load(wl)
    orc = oracle.OracleRun(wl.ndim, wl.n, wl.d, wl.dt, _species(wl, parts), wl.seed, 0)
    extra = ((f"plasma scattering: Coulomb small-angle model, coll_vref {wl.species[1].coll_vref}",)
             if wl.species[1].coll_model == 1 else ())
    lines = _header(wl, C3PHYS_DIAG, extra)
    t0 = time.time()
    for s in range(wl.steps):
        recs = orc.step(1, diag=(s % C3PHYS_DIAG == 0))
        if recs:
            lines.append(_rec_line(recs[0], wl.dt))
            if s % 100 == 0:
                r = recs[0]
                print(f"{wl.name} step {s} W_Bperp {r['W'][3] + r['W'][4]:.4e} ({time.time() - t0:.0f} s)",
                      flush=True)
                with open(path + ".part", "w") as fh:          # progress, for runs of hours
                    fh.write("\n".join(lines) + "\n")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    if os.path.exists(path + ".part"):
        os.remove(path + ".part")


def run_c3bin(path, wl=C3BIN):
    """As run_c3phys, with the binary collisions on and the scattered pairs
    appended to every record."""
    parts = synth.load(wl)
    orc = oracle.OracleRun(wl.ndim, wl.n, wl.d, wl.dt, _species(wl, parts), wl.seed, 0,
                           nu_ee=wl.nu_ee, ee_vref=wl.ee_vref)
    lines = _header(wl, C3PHYS_DIAG, (f"binary collisions nu_ee {wl.nu_ee} ee_vref {wl.ee_vref} (all species); "
                                      "last column: scattered pairs",))
    t0 = time.time()
    for s in range(wl.steps):
        recs = orc.step(1, diag=(s % C3PHYS_DIAG == 0))
        if recs:
            lines.append(_rec_line(recs[0], wl.dt) + f" {recs[0]['ee_pairs']}")
            if s % 50 == 0:
                print(f"{wl.name} step {s} W_Bperp {recs[0]['W'][3] + recs[0]['W'][4]:.4e} "
                      f"({time.time() - t0:.0f} s)", flush=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


HYB_DIAG = 10


def hybrid_paper_d():
    u_b = PAPER_VB / math.sqrt(1.0 - PAPER_VB * PAPER_VB)
    n, L = 128, 20.0
    return synth.HybridWorkload("hyb-paper-d", (n, n), (L / n, L / n), PAPER_DT, PAPER_STEPS, 0.1, 64, u_b, 0.37,
                                0.15, seed=synth.SEED + 7)


def run_hybrid(path):
    from oracle.hybrid import Hybrid
    wl = hybrid_paper_d()
    x, u, uz = synth.hybrid_load(wl)
    orc = Hybrid(wl.n, wl.d, wl.dt, wl.nu, x, u, uz, wl.weight, iters=wl.iters)
    lines = [f"# oracle series {wl.name}: written by tests/golden/make_oracle_series.py (FP64 reduced-model "
             f"oracle only)",
             f"# grid {wl.n[0]}x{wl.n[1]} d {wl.d[0]} dt {wl.dt} steps {wl.steps} seed {wl.seed:#x} n_b {wl.n_b} "
             f"ppc {wl.ppc} u_z {wl.u_b!r} u_th {wl.u_th} nu {wl.nu} sweeps {wl.iters}",
             f"# record every {HYB_DIAG} steps: step time W_Bperp beam_energy beam_pz W_Ez eq7"]
    t0 = time.time()
    for s in range(wl.steps):
        recs = orc.step(1, diag=(s % HYB_DIAG == 0))
        if recs:
            r = recs[0]
            lines.append(f"{r['step']} {r['time']:.10g} {r['W_Bperp']:.17e} {r['beam_energy']:.17e} "
                         f"{r['beam_pz']:.17e} {r['W_Ez']:.17e} {r['eq7']:.17e}")
            if s % 200 == 0:
                print(f"{wl.name} step {s} W_Bperp {r['W_Bperp']:.4e} ({time.time() - t0:.0f} s)", flush=True)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def run_paper(case, path_w, path_m):
    wl = paper_workload(case)
    parts = synth.load(wl)
    orc = oracle.OracleRun(wl.ndim, wl.n, wl.d, wl.dt, _species(wl, parts), wl.seed, 0)
    lines = _header(wl, PAPER_DIAG)
    mlines = [f"# oracle ring spectra {wl.name}: written by tests/golden/make_oracle_series.py",
              f"# every {PAPER_MODE_EVERY} steps: step time then |Bx(k)|^2+|By(k)|^2 summed over rings "
              f"m = 0..4 (|k| = m 2 pi / L, L = {PAPER_N * PAPER_DX})"]
    t0 = time.time()
    for s in range(wl.steps):
        if s % PAPER_MODE_EVERY == 0:
            P = ring_spectrum(orc.f.B[0, 0], orc.f.B[1, 0], PAPER_DX)
            mlines.append(f"{s} {s * wl.dt:.10g} " + " ".join(f"{v:.17e}" for v in P))
        recs = orc.step(1, diag=(s % PAPER_DIAG == 0))
        if recs:
            lines.append(_rec_line(recs[0], wl.dt))
            if s % 200 == 0:
                r = recs[0]
                print(f"paper-{case} step {s} W_Bperp {r['W'][3] + r['W'][4]:.4e} ({time.time() - t0:.0f} s)",
                      flush=True)
    with open(path_w, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    with open(path_m, "w") as fh:
        fh.write("\n".join(mlines) + "\n")


def annotate_c3phys(path):
    """Adds the growth-rate fit of the stored oracle series to its header:
    the linear window of ln(W_Bx + W_By) (the longest run of centred local
    slopes within 10% of their mean, below 10% of the series maximum; the
    first record, W = 0, left out) and the oracle's rate over it."""
    from oracle import theory
    lines = [ln for ln in open(path).read().splitlines() if not ln.startswith("# fit:")]
    o = np.loadtxt(path)
    t, Wb = o[:, 1], o[:, 5] + o[:, 6]
    a, b = theory.fit_growth_window(t[1:], Wb[1:])
    a, b = a + 1, b + 1
    rate = theory.fit_growth_rate(t, Wb, (a, b))
    head = [i for i, ln in enumerate(lines) if ln.startswith("#")][-1] + 1
    lines.insert(head, f"# fit: window records {a} {b} (t = {t[a]:g} .. {t[b - 1]:g}), oracle growth rate "
                       f"{rate:.12f}")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main(argv):
    which = argv or ["c3phys"] + [f"paper-{c}" for c in PAPER_CASES] + ["c3full"]
    for w in which:
        if w == "c3phys":
            run_c3phys(os.path.join(HERE, "oracle_c3phys_256.txt"))
            annotate_c3phys(os.path.join(HERE, "oracle_c3phys_256.txt"))
        elif w == "annotate":
            annotate_c3phys(os.path.join(HERE, "oracle_c3phys_256.txt"))
        elif w == "hyb-d":
            run_hybrid(os.path.join(HERE, "oracle_hybrid_paper_d.txt"))
        elif w == "c3coul":
            run_c3phys(os.path.join(HERE, "oracle_c3coul_256.txt"), C3COUL)
            annotate_c3phys(os.path.join(HERE, "oracle_c3coul_256.txt"))
        elif w == "c3bin":
            run_c3bin(os.path.join(HERE, "oracle_c3bin_256.txt"))
        elif w == "c4phys":
            run_c3phys(os.path.join(HERE, "oracle_c4phys_64x64x128.txt"), C4PHYS)
            annotate_c3phys(os.path.join(HERE, "oracle_c4phys_64x64x128.txt"))
        elif w == "c3full":
            run_c3phys(os.path.join(HERE, "oracle_c3_1024.txt"), C3FULL)
            annotate_c3phys(os.path.join(HERE, "oracle_c3_1024.txt"))
        elif w.startswith("paper-"):
            c = w.split("-", 1)[1]
            run_paper(c, os.path.join(HERE, f"oracle_paper_{c}_energy.txt"),
                      os.path.join(HERE, f"oracle_paper_{c}_modes.txt"))
        else:
            raise SystemExit(f"unknown series {w}")


if __name__ == "__main__":
    main(sys.argv[1:])
