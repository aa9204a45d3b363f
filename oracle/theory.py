"""Closed forms and fits used to pin the oracle and to compare runs.

Test infrastructure.  Nothing here calls the PIC step; these are the
independent references the oracle is checked against, plus the growth-rate
fit and the parity metrics that compare a run with the oracle.

Running this file writes ``tests/golden/weibel_cold_rates.txt`` from the
closed forms below (it calls nothing outside ``oracle/``).
"""
from __future__ import annotations

import math
import os

import numpy as np


# ---------------------------------------------------------------------------
# Cold-fluid filamentation (Weibel) rate of drifting cold electron species
# with immobile ions, k along x, drifts along z, full Maxwell equations.
# Linearising the relativistic cold-fluid equations with E = (E_x, 0, E_z),
# B = (0, B_y, 0) gives, with W = omega^2 and per-species alpha = n_s/n0,
#   A0 = sum alpha/gamma, A1 = sum alpha v/gamma, A2 = sum alpha v^2/gamma,
#   A3 = sum alpha/gamma^3,
#   (W^2 - (k^2 + A3) W - k^2 A2) (W - A0) = k^2 A1^2 .
# The growth rate is sqrt(-W) for the negative real root.  The paper's
# collisionless warm-beam theory (Eqs. 8-11) is the long-wavelength
# non-relativistic limit of the same physics; this is the cold, relativistic,
# all-k form used to pin the cold-beam run.
def weibel_cold_rate(k: float, species) -> float:
    """species: iterable of (alpha, u_z).  Returns the growth rate (1/w_p)."""
    A0 = A1 = A2 = A3 = 0.0
    for alpha, u in species:
        g = math.sqrt(1.0 + u * u)
        v = u / g
        A0 += alpha / g
        A1 += alpha * v / g
        A2 += alpha * v * v / g
        A3 += alpha / g ** 3
    k2 = k * k
    # expand: W^3 - (A0 + k2 + A3) W^2 + (A0 (k2 + A3) - k2 A2) W + k2 A2 A0 - k2 A1^2 = 0
    coeffs = [1.0, -(A0 + k2 + A3), A0 * (k2 + A3) - k2 * A2, k2 * A2 * A0 - k2 * A1 * A1]
    roots = np.roots(coeffs)
    neg = [r.real for r in roots if abs(r.imag) < 1e-12 * max(1.0, abs(r)) and r.real < 0.0]
    if not neg:
        return 0.0
    return math.sqrt(-min(neg))


# ---------------------------------------------------------------------------
# The paper's warm-beam filamentation dispersion with a resistive return
# current (Eq. 12), in units of w_p and c/w_p (so k_pe = 1 for the ambient
# plasma):
#   omega^2 = c_s^2 k^2 - wb2b2 k^2 / (k^2 + kpe2 / (1 + i nu / omega)),
# with c_s^2 the beam's sound speed squared and wb2b2 = omega_b^2 beta_0^2.
# Writing 1/(1 + i nu/omega) = omega/(omega + i nu) and multiplying by
# (omega + i nu)(k^2 + ...) gives the cubic
#   (omega^2 - c_s^2 k^2) ((k^2 + kpe2) omega + i nu k^2)
#       + wb2b2 k^2 (omega + i nu) = 0 .
# With nu = 0 its roots are omega = 0 and omega^2 = c_s^2 k^2 -
# wb2b2 k^2/(k^2 + kpe2); for a warm beam (c_s^2 > wb2b2/kpe2) none grows.
# For small nu and k^2 << kpe2 the growing root tends to Eq. (14),
#   omega = i nu wb2b2 / (kpe2 c_s^2 - wb2b2).
def warm_beam_roots(k: float, cs2: float, wb2b2: float, nu: float, kpe2: float = 1.0) -> np.ndarray:
    """The three roots omega (complex, 1/w_p) of the cubic form of Eq. (12)."""
    k2 = k * k
    s = cs2 * k2
    g = wb2b2 * k2
    a = k2 + kpe2
    b = 1j * nu * k2
    return np.roots([a, b, g - s * a, -s * b + 1j * g * nu])


def warm_beam_growth(k: float, cs2: float, wb2b2: float, nu: float, kpe2: float = 1.0) -> float:
    """Largest imaginary part of the roots of Eq. (12) (0 if none grows)."""
    return max(0.0, float(np.max(warm_beam_roots(k, cs2, wb2b2, nu, kpe2).imag)))


def warm_beam_growth_long_wave(cs2: float, wb2b2: float, nu: float, kpe2: float = 1.0) -> float:
    """Eq. (14): the collision-driven growth rate of a warm beam at long
    wavelength, nu wb2b2 / (kpe2 c_s^2 - wb2b2) (positive modified sound
    speed assumed)."""
    return nu * wb2b2 / (kpe2 * cs2 - wb2b2)


def hybrid_cold_roots(k: float, n_b: float, u_b: float, nu: float, n0: float = 1.0, dx: float = 0.0):
    """Linear filamentation of a cold beam (density n_b, u_z = u_b) in the
    reduced model with local quasi-neutrality, a mode k across the beam.
    Linearising Eqs. (2)-(4), (6) about the uniform state with the neutralising
    return current beta_p0 = -n_b beta_0/n_p, n_p = n0 - n_b:
      force on a beam electron   -(beta_0 - beta_p0) grad a  (transverse mass gamma),
      current of a density bump  (beta_0 - beta_p0) delta n_b  (the plasma gives way),
      the beam's own z response  chi = n_b/gamma^3 (Eq. 6: delta u_z = delta a),
      plasma response            n_p delta a omega/(omega + i nu)  (Eq. 3),
    give omega^2 (k^2 + chi + n_p omega/(omega + i nu)) = -A k^2 with
    A = (n_b/gamma)(beta_0 - beta_p0)^2: Eq. (12) with c_s = 0, k_pe^2 = n_p,
    omega_b^2 beta_0^2 = A, plus chi.  As a cubic:
      (k^2 + chi + n_p) w^3 + i nu (k^2 + chi) w^2 + A k^2 w + i nu A k^2 = 0.
    With dx > 0 the grid's own factors replace the continuum ones (mode along
    a grid axis): the 5-point Laplacian's (2/dx)^2 sin^2(k dx/2) for k^2, the
    staggered difference (2/dx) sin(k dx/2) for one k of the force, and the
    cloud-in-cell transfer S = (sin(k dx/2)/(k dx/2))^2 once for the gather
    and once for the deposit."""
    gamma = math.sqrt(1.0 + u_b * u_b)
    beta0 = u_b / gamma
    n_p = n0 - n_b
    bbar = beta0 + n_b * beta0 / n_p
    A = n_b / gamma * bbar * bbar
    chi = n_b / gamma ** 3
    if dx > 0:
        h = 0.5 * k * dx
        kg = 2.0 / dx * math.sin(h)
        S = (math.sin(h) / h) ** 2
        K2 = kg * kg
        Ak2 = A * k * kg * S * S
        chi = chi * S * S
    else:
        K2 = k * k
        Ak2 = A * k * k
    return np.roots([K2 + chi + n_p, 1j * nu * (K2 + chi), Ak2, 1j * nu * Ak2])


def hybrid_cold_growth(k, n_b, u_b, nu, n0=1.0, dx=0.0) -> float:
    return max(0.0, float(np.max(hybrid_cold_roots(k, n_b, u_b, nu, n0, dx).imag)))


def paper_case_parameters(v_b: float = 0.9, n_b: float = 0.1, u_th: float = 0.37):
    """(c_s^2, wb2b2) of the paper's 2D beam for Eq. (12), with the
    relativistic transverse inertia gamma_b m: the beam's transverse thermal
    velocity is u_th/gamma_b, c_s^2 = 3 (u_th/gamma_b)^2 (the text's
    c_s^2 = 3 v_th^2), omega_b^2 = n_b/(gamma_b n0) and beta_0 = v_b (the
    text's approximation of v_bz - v_pz)."""
    gamma_b = 1.0 / math.sqrt(1.0 - v_b * v_b)
    cs2 = 3.0 * (u_th / gamma_b) ** 2
    wb2b2 = n_b / gamma_b * v_b * v_b
    return cs2, wb2b2


def beam_plasma_species(n_b=0.1, u_beam=math.sqrt(8.0)):
    """Cold beam and the cold return current that cancels it."""
    v_b = u_beam / math.sqrt(1 + u_beam ** 2)
    v_p = -n_b * v_b / (1 - n_b)
    u_p = v_p / math.sqrt(1 - v_p ** 2)
    return [(n_b, u_beam), (1 - n_b, u_p)]


# ---------------------------------------------------------------------------
# Cold-fluid longitudinal (two-stream) dispersion of drifting cold electron
# species with immobile ions, k along the drifts: each species responds to
# E_z with the longitudinal mass gamma^3 m, so
#   1 = sum_s alpha_s / (gamma_s^3 (omega - k v_s)^2) .
# Clearing the denominators gives a polynomial of degree 2 x (number of
# species) in omega; the growth rate is the largest imaginary part of its
# roots.
def two_stream_cold_roots(k: float, species) -> np.ndarray:
    """species: iterable of (alpha, u_z).  All roots omega (1/w_p) at k."""
    terms = []
    for alpha, u in species:
        g = math.sqrt(1.0 + u * u)
        terms.append((alpha / g ** 3, k * u / g))
    full = np.poly1d([1.0])
    for _, kv in terms:
        full = full * np.poly1d([1.0, -kv]) ** 2
    rhs = np.poly1d([0.0])
    for i, (a, _) in enumerate(terms):
        others = np.poly1d([1.0])
        for j, (_, kv) in enumerate(terms):
            if j != i:
                others = others * np.poly1d([1.0, -kv]) ** 2
        rhs = rhs + a * others
    return np.roots((full - rhs).coeffs)


def two_stream_cold_rate(k: float, species) -> float:
    return max(0.0, float(np.max(two_stream_cold_roots(k, species).imag)))


def two_stream_cold_rate_weak(n_b, n_p, gamma_b):
    """Maximum growth rate of the weak cold beam-plasma two-stream
    instability (beam much thinner than the plasma), in w_pe of the plasma:
    (sqrt(3)/2^{4/3}) (n_b/n_p)^{1/3} / gamma_b."""
    return math.sqrt(3.0) / 2 ** (4.0 / 3.0) * (n_b / n_p) ** (1.0 / 3.0) / gamma_b


# ---------------------------------------------------------------------------
# Discrete closed forms of the time integrators.
def boris_gyration(u_perp: float, u_par: float, qB_over_m: float, dt: float):
    """Exact discrete orbit of the Boris rotation in a uniform B.

    With gamma = sqrt(1 + u_perp^2 + u_par^2), Omega = |q B|/(m gamma) and
    a = Omega dt / 2, each step turns u_perp by 2 atan(a) and keeps |u|; the
    positions lie on a circle of radius r_L sqrt(1 + a^2), r_L = u_perp/|qB/m|.
    Returns (angle per step, polygon radius)."""
    g = math.sqrt(1.0 + u_perp ** 2 + u_par ** 2)
    a = abs(qB_over_m) * dt / (2.0 * g)
    r_L = u_perp / abs(qB_over_m)
    return 2.0 * math.atan(a), r_L * math.sqrt(1.0 + a * a)


def yee_vacuum_omega(k, d, dt):
    """Discrete vacuum dispersion of the Yee scheme:
    sin^2(w dt/2)/dt^2 = sum_i sin^2(k_i d_i/2)/d_i^2."""
    s = sum(math.sin(ki * di / 2) ** 2 / di ** 2 for ki, di in zip(k, d))
    return 2.0 / dt * math.asin(dt * math.sqrt(s))


def leapfrog_plasma_omega(wp: float, dt: float) -> float:
    """Oscillation frequency of a cold plasma under leap-frog integration:
    sin(w dt/2) = wp dt / 2."""
    return 2.0 / dt * math.asin(wp * dt / 2.0)


# ---------------------------------------------------------------------------
# Growth-rate fit and parity metrics.
def fit_growth_window(t, W, span=21, tol=0.10, frac_max=0.10):
    """Window of linear growth of ln W(t): the longest contiguous range where
    the centred local slope (least squares over `span` samples) stays within
    +-tol of the range mean and W stays below frac_max of its running max at
    the end of the series.  Returns (i0, i1) inclusive-exclusive indices."""
    t = np.asarray(t, dtype=float)
    y = np.log(np.asarray(W, dtype=float))
    n = len(t)
    h = span // 2
    slope = np.full(n, np.nan)
    for i in range(h, n - h):
        tt = t[i - h:i + h + 1]
        yy = y[i - h:i + h + 1]
        slope[i] = np.polyfit(tt, yy, 1)[0]
    wmax = float(np.max(W))
    ok = (np.asarray(W) < frac_max * wmax) & np.isfinite(slope) & (slope > 0)
    best = (0, 0)
    i = 0
    while i < n:
        if not ok[i]:
            i += 1
            continue
        j = i
        while j < n and ok[j]:
            j += 1
        # shrink from the left until all slopes are within tol of the mean
        a, b = i, j
        while b - a > 2:
            m = float(np.mean(slope[a:b]))
            dev = np.abs(slope[a:b] - m) / abs(m)
            if np.all(dev <= tol):
                break
            worst = a + int(np.argmax(dev))
            if worst - a < b - 1 - worst:
                a = worst + 1
            else:
                b = worst
        if b - a > best[1] - best[0]:
            best = (a, b)
        i = j
    return best


def fit_growth_rate(t, W, window):
    """Growth rate of a field amplitude from an energy series:
    half the least-squares slope of ln W over the window."""
    i0, i1 = window
    t = np.asarray(t, dtype=float)[i0:i1]
    y = np.log(np.asarray(W, dtype=float)[i0:i1])
    return 0.5 * float(np.polyfit(t, y, 1)[0])


def stacked_rel_err(F, F_ref):
    """||F - F_ref||_2 / ||F_ref||_2 over all components stacked."""
    F = np.asarray(F, dtype=float)
    F_ref = np.asarray(F_ref, dtype=float)
    return float(np.linalg.norm((F - F_ref).ravel()) / np.linalg.norm(F_ref.ravel()))


def _write_golden(path):
    sp = beam_plasma_species(0.1, math.sqrt(8.0))
    L = 64 * 0.2
    lines = ["# Cold-fluid filamentation growth rate, beam n_b=0.1 gamma=3 (u=sqrt(8)) + cancelling",
             "# cold return current, immobile ions; written by oracle/theory.py from the",
             "# closed-form dispersion relation (W^2-(k^2+A3)W-k^2A2)(W-A0)=k^2A1^2.",
             "# columns: mode m on a box of side 12.8 c/w_p, k (w_p/c), rate (w_p)"]
    for m in (1, 2, 4, 8, 16):
        k = 2 * math.pi * m / L
        lines.append(f"{m} {k:.12f} {weibel_cold_rate(k, sp):.12f}")
    lines.append(f"inf inf {weibel_cold_rate(1e6, sp):.12f}")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    _write_golden(os.path.join(here, "..", "tests", "golden", "weibel_cold_rates.txt"))
