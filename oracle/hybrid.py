"""FP64 CPU oracle of the paper's reduced quasi-neutral beam-plasma model
(test infrastructure).

Test infrastructure only: the test suite, the smoke check and the CPU
baseline leg of the benchmark may use it; the product library never does.
It shares no code with the HIP path.  Plain numpy; the FFT (numpy.fft) and
the scatter-add (numpy.bincount) are the only library steps.

The model (the theory part of the paper, Eqs. 1-7), in the units of the PIC
path: t in 1/w_p, x in c/w_p, densities in n0, u = gamma v/c, and the
normalised potential a = e A_z/(m c^2).  Beam and plasma are electrons; the
sign of their charge is absorbed, so Eq. (2) reads
    lap a = n_b beta_bz + n_p beta_pz                          (Eq. 2)
with no displacement current.  The plasma is a cold fluid streaming along z,
    d_t beta_pz + nu beta_pz = d_t a                            (Eq. 3)
the beam is kinetic in the transverse plane,
    d(u_perp)/dt = -(beta_z - beta_pz) grad a                   (Eq. 4)
and its z momentum follows from the conserved canonical momentum,
    u_z = u_z0 + a - a_0                                        (Eq. 6)
The fields B_perp = -e_z x grad a, E_z = -d_t a and E_perp = -beta_pz grad a
(Eq. 1) are implied.  Without collisions,
    sum_j w_j (gamma_j - a_j^2/2) + int (|grad a|^2 + n0 a^2)/2  (Eq. 7)
is conserved.

Readings (where the paper leaves the model's closure or numerics open):
  * quasi-neutrality holds locally: n_p(x) = n0 - n_b(x), clipped at 0.
    This is what makes Eq. (7)'s second term exact and gives the linear
    theory's beta_0 = (v_bz - v_pz)/c (the remark after Eq. 9);
  * the plasma's canonical momentum psi = beta_pz - a obeys
    d_t psi = -nu (psi + a) (Eq. 3 rewritten) and starts at 0: the plasma
    then carries beta_pz = a, which at t = 0 is the return current that
    neutralises the beam;
  * grid: nodes at (i dx, j dy), periodic; the 5-point Laplacian; grad a by
    forward differences on the staggered points ((i+1/2) dx, j dy) and
    (i dx, (j+1/2) dy) (where B_y and B_x sit on a Yee grid); cloud-in-cell
    weights for the deposit and for every gather;
  * time: x and a at integer steps, u_perp at half steps.  a^n solves Eq. (2)
    with the beam current linearised about a* = 2 a^(n-1) - a^(n-2):
    beta_z(a) ~ beta_z(a*) + chi (a - a*), chi = d beta_z/d u_z
    = (1 + u_perp^2)/gamma^3, deposited per particle.  The variable
    coefficient is handled by a fixed number of fixed-point sweeps, each an
    FFT solve of the constant-coefficient operator lap - c0 with
    c0 = n0 - <n_b>;
  * the push takes beta_z = u_z^n/gamma^- with gamma^- from u_perp^(n-1/2),
    then moves with gamma^+ from u_perp^(n+1/2); psi advances by
    psi^(n+1) = psi^n - nu dt (psi^n + a^n): the drag acts on the plasma's
    velocity beta_pz = psi + a, which quasi-neutrality keeps nearly constant
    in the mean while psi and a drift together;
  * the Eq. (7) record takes gamma^n = (gamma^- + gamma^+)/2.
"""
from __future__ import annotations

import math

import numpy as np


class Hybrid:
    """One run of the reduced model.  x: (2, N) positions, u: (2, N)
    transverse momenta taken as u_perp^(-1/2), uz: (N,) initial u_z, w: the
    beam's density per macro-particle (n_b / particles per cell)."""

    def __init__(self, n, d, dt, nu, x, u, uz, w, n0=1.0, iters=10):
        self.nx, self.ny = int(n[0]), int(n[1])
        self.dx, self.dy = float(d[0]), float(d[1])
        self.dt, self.nu, self.n0, self.iters = float(dt), float(nu), float(n0), int(iters)
        self.w = float(w)
        self.x = np.array(x, dtype=np.float64)
        self.u = np.array(u, dtype=np.float64)
        self.dA = self.dx * self.dy
        self.L = np.array([self.nx * self.dx, self.ny * self.dy])
        npart = self.x.shape[1]
        self.c0 = self.n0 - self.w * npart / (self.nx * self.ny)
        kx = np.arange(self.nx)
        ky = np.arange(self.ny)
        self.symbol = (-(4.0 / self.dx ** 2) * np.sin(math.pi * kx / self.nx)[None, :] ** 2
                       - (4.0 / self.dy ** 2) * np.sin(math.pi * ky / self.ny)[:, None] ** 2 - self.c0)
        self.step_index = 0
        self.psi = np.zeros((self.ny, self.nx))
        # initial state: the exact beam current (u_z given), a^0, the canonical momenta
        uz = np.asarray(uz, dtype=np.float64)
        g = np.sqrt(1.0 + self.u[0] ** 2 + self.u[1] ** 2 + uz ** 2)
        zero = np.zeros(npart)
        dep = self._deposit(self.x, uz / g, zero, zero)
        a0 = self.solve(dep, self.psi, np.zeros((self.ny, self.nx)))
        self.P = uz - self.interp(a0, self.x)
        self.a_cur = a0
        self.a_prev = a0.copy()
        self.dep = self._deposit_linearised(self.x, self.u, self.predict(self.a_cur, self.a_prev))

    @classmethod
    def from_state(cls, n, d, dt, nu, x, u, P, w, a_cur, a_prev, psi, n0=1.0, iters=10):
        """A run continued from a given state: positions x^n, u_perp^(n-1/2),
        canonical momenta P, a^(n-1), a^(n-2), psi^n; the deposit at x^n is
        made here about a* = 2 a^(n-1) - a^(n-2)."""
        h = cls.__new__(cls)
        h.nx, h.ny = int(n[0]), int(n[1])
        h.dx, h.dy = float(d[0]), float(d[1])
        h.dt, h.nu, h.n0, h.iters = float(dt), float(nu), float(n0), int(iters)
        h.w = float(w)
        h.x = np.array(x, dtype=np.float64)
        h.u = np.array(u, dtype=np.float64)
        h.P = np.array(P, dtype=np.float64)
        h.dA = h.dx * h.dy
        h.L = np.array([h.nx * h.dx, h.ny * h.dy])
        h.c0 = h.n0 - h.w * h.x.shape[1] / (h.nx * h.ny)
        kx, ky = np.arange(h.nx), np.arange(h.ny)
        h.symbol = (-(4.0 / h.dx ** 2) * np.sin(math.pi * kx / h.nx)[None, :] ** 2
                    - (4.0 / h.dy ** 2) * np.sin(math.pi * ky / h.ny)[:, None] ** 2 - h.c0)
        h.step_index = 0
        h.psi = np.array(psi, dtype=np.float64)
        h.a_cur = np.array(a_cur, dtype=np.float64)
        h.a_prev = np.array(a_prev, dtype=np.float64)
        h.dep = h._deposit_linearised(h.x, h.u, h.predict(h.a_cur, h.a_prev))
        return h

    @staticmethod
    def predict(a1, a2):
        """The point a* about which the next step linearises the beam current:
        the linear extrapolation 2 a^(n-1) - a^(n-2) of the last two solutions.
        Since a^n - a* = O(dt^2), the linearisation leaves an error O(dt^4) per
        step against the self-consistent solution of Eqs. (2) and (6)."""
        return 2.0 * a1 - a2

    # ---- cloud-in-cell weights, gathers and deposit
    def _axis(self, xa, h, n, shift):
        f = xa / h - shift
        i = np.floor(f)
        o = f - i
        i0 = i.astype(np.int64) % n
        return i0, (i0 + 1) % n, o

    def interp(self, F, x):
        """F given on the nodes (i dx, j dy), at the points x."""
        i0, i1, ox = self._axis(x[0], self.dx, self.nx, 0.0)
        j0, j1, oy = self._axis(x[1], self.dy, self.ny, 0.0)
        return ((1 - ox) * (1 - oy) * F[j0, i0] + ox * (1 - oy) * F[j0, i1]
                + (1 - ox) * oy * F[j1, i0] + ox * oy * F[j1, i1])

    def gradients(self, a):
        """Forward differences: gx at ((i+1/2) dx, j dy), gy at (i dx, (j+1/2) dy)."""
        gx = (np.roll(a, -1, axis=1) - a) / self.dx
        gy = (np.roll(a, -1, axis=0) - a) / self.dy
        return gx, gy

    def grad_at(self, a, x):
        gx, gy = self.gradients(a)
        i0, i1, ox = self._axis(x[0], self.dx, self.nx, 0.5)
        j0, j1, oy = self._axis(x[1], self.dy, self.ny, 0.0)
        Gx = ((1 - ox) * (1 - oy) * gx[j0, i0] + ox * (1 - oy) * gx[j0, i1]
              + (1 - ox) * oy * gx[j1, i0] + ox * oy * gx[j1, i1])
        i0, i1, ox = self._axis(x[0], self.dx, self.nx, 0.0)
        j0, j1, oy = self._axis(x[1], self.dy, self.ny, 0.5)
        Gy = ((1 - ox) * (1 - oy) * gy[j0, i0] + ox * (1 - oy) * gy[j0, i1]
              + (1 - ox) * oy * gy[j1, i0] + ox * oy * gy[j1, i1])
        return Gx, Gy

    def deposit(self, x, q):
        """sum_j q_j W(node - x_j) on the nodes (CIC)."""
        i0, i1, ox = self._axis(x[0], self.dx, self.nx, 0.0)
        j0, j1, oy = self._axis(x[1], self.dy, self.ny, 0.0)
        idx = np.concatenate([j0 * self.nx + i0, j0 * self.nx + i1, j1 * self.nx + i0, j1 * self.nx + i1])
        wts = np.concatenate([q * (1 - ox) * (1 - oy), q * ox * (1 - oy), q * (1 - ox) * oy, q * ox * oy])
        return np.bincount(idx, weights=wts, minlength=self.nx * self.ny).reshape(self.ny, self.nx)

    def _deposit(self, x, beta, chi, abar):
        w = self.w
        return (self.deposit(x, np.full(x.shape[1], w)), self.deposit(x, w * beta),
                self.deposit(x, w * chi), self.deposit(x, w * chi * abar))

    def _deposit_linearised(self, x, u, astar):
        """n_b, the beam current at a*, and the linear response chi about it."""
        abar = self.interp(astar, x)
        uz = self.P + abar
        up2 = u[0] ** 2 + u[1] ** 2
        g = np.sqrt(1.0 + up2 + uz ** 2)
        return self._deposit(x, uz / g, (1.0 + up2) / g ** 3, abar)

    # ---- Eq. (2) with the local plasma density and the linearised beam current
    def solve(self, dep, psi, start):
        nb, J, X, Y = dep
        n_p = np.maximum(self.n0 - nb, 0.0)
        c = n_p + X
        R = J - Y + n_p * psi
        a = start
        for _ in range(self.iters):
            a = np.real(np.fft.ifft2(np.fft.fft2(R + (c - self.c0) * a) / self.symbol))
        return a

    # ---- one step
    def step(self, nsteps=1, diag=False):
        recs = []
        for _ in range(nsteps):
            recs.append(self._step(diag))
        return recs if diag else None

    def _step(self, diag):
        dt = self.dt
        a = self.solve(self.dep, self.psi, self.predict(self.a_cur, self.a_prev))
        x, u = self.x, self.u
        abar = self.interp(a, x)
        Gx, Gy = self.grad_at(a, x)
        bp = self.interp(self.psi, x) + abar          # beta_pz at the particle
        uz = self.P + abar                             # Eq. (6)
        g_minus = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + uz ** 2)
        f = -(uz / g_minus - bp) * dt                  # Eq. (4)
        u[0] += f * Gx
        u[1] += f * Gy
        g_plus = np.sqrt(1.0 + u[0] ** 2 + u[1] ** 2 + uz ** 2)
        x[0] = np.mod(x[0] + dt * u[0] / g_plus, self.L[0])
        x[1] = np.mod(x[1] + dt * u[1] / g_plus, self.L[1])
        x[0][x[0] >= self.L[0]] = 0.0
        x[1][x[1] >= self.L[1]] = 0.0
        rec = None
        if diag:
            gx, gy = self.gradients(a)
            g2 = float(np.sum(gx ** 2 + gy ** 2))
            rec = dict(step=self.step_index, time=self.step_index * dt,
                       beam_energy=self.dA * self.w * float(np.sum(0.5 * (g_minus + g_plus))),
                       beam_a2=self.dA * self.w * float(np.sum(0.5 * abar ** 2)),
                       grad_energy=0.5 * self.dA * g2,
                       a2_energy=0.5 * self.dA * self.n0 * float(np.sum(a ** 2)),
                       W_Bperp=self.dA * g2,
                       W_Ez=self.dA * float(np.sum(((a - self.a_cur) / dt) ** 2)),
                       beam_pz=self.dA * self.w * float(np.sum(uz)),
                       mean_a=float(np.mean(a)), mean_psi=float(np.mean(self.psi)))
            rec["eq7"] = rec["beam_energy"] - rec["beam_a2"] + rec["grad_energy"] + rec["a2_energy"]
        self.dep = self._deposit_linearised(x, u, self.predict(a, self.a_cur))
        self.psi = self.psi - self.nu * dt * (self.psi + a)         # Eq. (3): d_t psi = -nu beta_pz
        self.a_prev = self.a_cur
        self.a_cur = a
        self.step_index += 1
        return rec

    def uz(self):
        """u_z of every particle at the latest solved a (Eq. 6)."""
        return self.P + self.interp(self.a_cur, self.x)
