"""The paper's four 2D cases at its own parameters (the 2D PIC paragraph):
a 20 x 20 c/w_p box of 160^2 cells (dx = 0.125 c/w_p), 64 particles per
cell per species, n_p/n_b = 9, beam v_b = 0.9 c, hot beam u_th = 0.37 m c
(the text's ~70 keV), collision rate nu/w_p = 0.15, run to T = 20 (2 pi/w_p).

The Letter's figures are missing, so the check is against its text and its
dispersion relation, Eq. (12), and against the FP64 oracle run on the same
initial particles (tests/golden/oracle_paper_*_{energy,modes}.txt, written by
tests/golden/make_oracle_series.py, oracle only):
  (a) cold beam, collisionless: Weibel growth;
  (b) cold beam, collisional: growth;
  (c) hot beam, collisionless: no growth (thermal stabilisation);
  (d) hot beam, collisional: growth driven by the resistive return current,
      with the k-resolved rate of Eq. (12) at the box's fundamental mode.
dt = 0.0625/w_p is the largest step the deposit window allows (dt <= dx/2).
"""
import math
import os

import numpy as np
import pytest

import synth
from oracle import theory
from pic_cases import gpu_run, log

pytestmark = pytest.mark.gpu

N, DX, DT = 160, 0.125, 0.0625
L = N * DX
STEPS = int(round(20 * 2 * math.pi / DT))          # T = 20 plasma periods
V_B = 0.9
CASES = {"a": (0.01, 0.0), "b": (0.01, 0.15), "c": (0.37, 0.0), "d": (0.37, 0.15)}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MODE_EVERY = 50


def workload(case):
    uth, nu = CASES[case]
    u_b = V_B / math.sqrt(1.0 - V_B * V_B)
    return synth.beam_plasma((N, N), d=(DX, DX), dt=DT, steps=STEPS, ppc=64, u_th_beam=uth, nu=nu, u_beam=u_b,
                             name=f"paper-{case}")


def ring_spectrum(Bx, By):
    """|B_x(k)|^2 + |B_y(k)|^2 summed over the rings round(|k| L/2pi) = m, m = 0..4."""
    kx = np.fft.fftfreq(N, d=DX) * 2 * math.pi
    K = np.sqrt(kx[None, :] ** 2 + kx[:, None] ** 2)
    shell = np.rint(K / (2 * math.pi / L)).astype(int)
    P = np.abs(np.fft.fft2(Bx)) ** 2 + np.abs(np.fft.fft2(By)) ** 2
    return np.bincount(shell.ravel(), weights=P.ravel(), minlength=5)[:5]


def oracle_case(case):
    e = np.loadtxt(os.path.join(GOLDEN, f"oracle_paper_{case}_energy.txt"))
    m = np.loadtxt(os.path.join(GOLDEN, f"oracle_paper_{case}_modes.txt"))
    return dict(t=e[:, 1], W=e[:, 2:8], Wb=e[:, 5] + e[:, 6], ts=m[:, 1], modes=m[:, 2:7])


@pytest.fixture(scope="module")
def runs():
    """Per case and precision: the record series (every 10 steps) and the
    ring spectra every 50 steps, from the oracle's initial particles."""
    from paper_0808_4078_amd import pic
    pic.lib()
    out = {}
    for name in CASES:
        wl = workload(name)
        parts = synth.load(wl)
        for prec, p in (("mixed", pic.PIC_PREC_MIXED), ("fp64", pic.PIC_PREC_FP64)):
            log(f"case paper 2D ({name}) {prec}: u_th {CASES[name][0]} nu {CASES[name][1]}")
            r = gpu_run(wl, parts, p, diag_every=10)
            ts, modes = [], []
            for s0 in range(0, STEPS, MODE_EVERY):
                _, B, _ = r.read_fields()
                modes.append(ring_spectrum(B[0, 0], B[1, 0]))
                ts.append(s0 * DT)
                r.step(min(MODE_EVERY, STEPS - s0))
            h = r.history()
            r.close()
            W = np.array([x["W"] for x in h])
            out[name, prec] = dict(t=np.array([x["time"] for x in h]), W=W, Wb=W[:, 3] + W[:, 4],
                                   ts=np.array(ts), modes=np.array(modes))
    return out


def _rate(run, m, t0, t1):
    """Amplitude growth rate of box mode m between t0 and t1."""
    ts, e = run["ts"], run["modes"][:, m]
    i0, i1 = int(np.argmin(abs(ts - t0))), int(np.argmin(abs(ts - t1)))
    return 0.5 * math.log(e[i1] / e[i0]) / (ts[i1] - ts[i0])


def _window_rate(o, g):
    """Growth rates of W_Bperp fitted over the oracle's linear window
    (first record, W = 0, left out)."""
    a, b = theory.fit_growth_window(o["t"][1:], o["Wb"][1:])
    win = (a + 1, b + 1)
    return theory.fit_growth_rate(o["t"], o["Wb"], win), theory.fit_growth_rate(o["t"], g["Wb"], win), win


def test_hot_beam_needs_collisions_to_filament(runs):
    c, d = runs["c", "mixed"], runs["d", "mixed"]
    log(f"  W_Bperp end: (a) {runs['a', 'mixed']['Wb'][-1]:.3e} (b) {runs['b', 'mixed']['Wb'][-1]:.3e} "
        f"(c) {c['Wb'][-1]:.3e} (d) {d['Wb'][-1]:.3e}")
    assert c["Wb"].max() < 1e-2                      # (c) stays at the noise level
    assert d["Wb"][-1] > 30.0 * c["Wb"][-1]           # (d) grows far above it
    assert runs["a", "mixed"]["Wb"].max() > 1.0 and runs["b", "mixed"]["Wb"].max() > 1.0   # cold beams filament
    # the growth of (d) is exponential over the middle of the run
    i25, i100 = int(np.argmin(abs(d["t"] - 25))), int(np.argmin(abs(d["t"] - 100)))
    assert d["Wb"][i100] > 20.0 * d["Wb"][i25]


def test_collisional_growth_rate_against_eq12(runs):
    """Box mode 1 (k = 2 pi/L = 0.314 c/w_p, near the maximum of Eq. (12)):
    measured amplitude growth of (d) over t = 25..75 against Eq. (12) with the
    relativistic transverse inertia (theory.paper_case_parameters): the fluid
    closure of a kinetic beam, so a band, not a match (context)."""
    cs2, wb2b2 = theory.paper_case_parameters(v_b=V_B, n_b=0.1, u_th=0.37)
    k1 = 2 * math.pi / L
    g_th = theory.warm_beam_growth(k1, cs2, wb2b2, 0.15)
    g_pic = _rate(runs["d", "mixed"], 1, 25.0, 75.0)
    log(f"  (d) mode-1 growth: PIC {g_pic:.4f}, Eq. (12) {g_th:.4f}; collisionless Eq. (12) "
        f"{theory.warm_beam_growth(k1, cs2, wb2b2, 0.0):.4f}")
    assert theory.warm_beam_growth(k1, cs2, wb2b2, 0.0) == 0.0
    assert 0.6 * g_th < g_pic < 1.6 * g_th
    # Eq. (12) damps the shorter modes of (d); mode 3 grows much more slowly than mode 1
    assert _rate(runs["d", "mixed"], 3, 25.0, 75.0) < 0.5 * g_pic


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_paper_cases_against_the_oracle(runs, prec):
    """The four cases against the FP64 oracle run on the same particles:
    (d)'s mode-1 growth over t = 25..75 and the W_Bperp growth of (a) and (b)
    over the oracle's linear window agree to 2%; (c) stays at the noise level
    in both; the records' six field energies agree where a record's energy
    is above 1e-6 of the run's largest: FP64 over the whole run to 1e-6
    (measured 2.6e-8, in the cold collisionless case (a), whose filaments
    amplify round-off fastest; 1.5e-12 in (d)), mixed over the linear phase
    t <= 60 to the mixed path's 1e-3 field bar (the whole-run worst is
    logged: past the predictability horizon the cold beams' FP32 runs
    decorrelate from the oracle's pointwise, as any two runs of a chaotic
    system do, while their growth rates still agree)."""
    worst, worst_all = {}, {}
    for name in CASES:
        o, g = oracle_case(name), runs[name, prec]
        assert np.allclose(o["t"], g["t"]) and np.allclose(o["ts"], g["ts"])
        big = np.abs(o["W"]) > 1e-6 * np.abs(o["W"]).max()
        rel = np.where(big, np.abs(g["W"] - o["W"]) / np.where(big, np.abs(o["W"]), 1.0), 0.0)
        worst_all[name] = float(rel.max())
        worst[name] = worst_all[name] if prec == "fp64" else float(rel[o["t"] <= 60.0].max())
    ro, rg = _rate(oracle_case("d"), 1, 25.0, 75.0), _rate(runs["d", prec], 1, 25.0, 75.0)
    msg = f"  {prec}: worst record W_i error " + ", ".join(f"({k}) {v:.1e}" for k, v in worst.items())
    msg += " (whole run: " + ", ".join(f"({k}) {v:.1e}" for k, v in worst_all.items()) + ")"
    msg += f"; (d) mode-1 growth gpu {rg:.5f} oracle {ro:.5f}"
    rates = {}
    for name in ("a", "b"):
        rates[name] = _window_rate(oracle_case(name), runs[name, prec])
        msg += f"; ({name}) W_Bperp growth gpu {rates[name][1]:.5f} oracle {rates[name][0]:.5f}"
    log(msg)
    assert abs(rg / ro - 1) < 0.02
    for name in ("a", "b"):
        r_o, r_g, win = rates[name]
        assert win[1] - win[0] >= 10 and r_o > 0.05
        assert abs(r_g / r_o - 1) < 0.02
    assert oracle_case("c")["Wb"].max() < 1e-2 and runs["c", prec]["Wb"].max() < 1e-2
    bar = 1e-6 if prec == "fp64" else 1e-3
    assert max(worst.values()) < bar, worst
