/*
 * pic_oracle.c -- plain FP64 particle-in-cell reference (test infrastructure).
 *
 * This file is the oracle that the GPU path is checked against.  It is test
 * infrastructure, not product code: only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it, and it shares no source,
 * header, table or helper with the HIP library.
 *
 * What it computes.  The paper (Karmakar, Kumar, Shvets, Polomarov, Pukhov,
 * arXiv:0808.4078) studies a relativistic electron beam and its return
 * current in a quasi-neutral plasma with immobile ions (problem statement,
 * opening of the theory part; PIC-simulation paragraph).  It runs PIC
 * simulations of that system but prints none of the numerics, so the scheme
 * below is the textbook electromagnetic PIC cycle, written from the original
 * method papers:
 *
 *   gather   : E, B at x^n, bilinear (trilinear) weights at each component's
 *              own Yee-staggered location;
 *   push     : relativistic Boris rotation (Boris 1970), u^{n-1/2} -> u^{n+1/2};
 *   move     : x^{n+1} = x^n + dt u^{n+1/2}/gamma^{n+1/2};
 *   deposit  : charge-conserving current of Esirkepov (2001) with the linear
 *              (cloud-in-cell) form factor, J^{n+1/2};
 *   collide  : elastic isotropic scattering of return-current electrons off
 *              the immobile ions with probability 1 - exp(-nu dt) per step,
 *              |u| kept; in the fluid limit this is the -nu v_pz drag of the
 *              plasma momentum equation, Eq. (3);
 *   fields   : Yee (1966) FDTD, B half step, E full step with -J, B half step.
 *
 * Normalised units: t in 1/w_p, x in c/w_p, u = gamma v / c, fields
 * eF/(m c w_p) (the paper's field normalisation in the field-energy
 * diagnostic), densities in n0 (w_p is built on n0), charge in e, mass in m_e.
 * Equations: du/dt = (q/m)(E + v x B), dB/dt = -curl E, dE/dt = curl B - J.
 * A macro-particle of weight w adds q w S to the charge density at a node,
 * where S is the form factor, so a uniform load of ppc particles per cell of
 * weight (n_s/n0)/ppc gives density q n_s/n0.
 *
 * Grid: planes are [n2][n1][n0] with x fastest.  A component located at a
 * half-integer index along an axis is stored at the lower integer index:
 * Ex(i+1/2,j,k) Ey(i,j+1/2,k) Ez(i,j,k+1/2) Bx(i,j+1/2,k+1/2)
 * By(i+1/2,j,k+1/2) Bz(i+1/2,j+1/2,k); J is co-located with E and the charge
 * density sits on integer nodes.  The 2D3V case (z ignorable, the paper's
 * transverse-plane geometry) is n2 = 1: every z difference then vanishes,
 * particles carry no z position, and J_z comes from v_z and the 2D Esirkepov
 * weight instead of the z running sum.  Boundaries are periodic.
 *
 * Random numbers: Philox2x32-10 and Philox4x32-10 (Salmon, Moraes, Dror,
 * Shaw, SC'11), written from their published definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int ndim;             /* 2 (2D3V) or 3 */
    int n[3];             /* cells per axis, n[2] = 1 in 2D */
    double d[3];          /* cell size per axis in c/w_p (d[2] unused in 2D) */
    double dt;            /* time step in 1/w_p */
    double *E[3], *B[3], *J[3];   /* caller-owned planes, n[0]*n[1]*n[2] each */
    double nu_ee;         /* electron-electron binary collisions: rate at relative speed ee_vref (0 = off) */
    double ee_vref;       /* reference relative speed of nu_ee, units of c */
} orc_grid;

typedef struct {
    double q, m, w;       /* charge, mass, weight (n_s/n0)/ppc */
    double nu;            /* collision frequency in w_p, 0 = collisionless */
    int64_t n;            /* number of particles */
    double *x[3];         /* positions in c/w_p (x[2] unused in 2D) */
    double *u[3];         /* momenta gamma v / c */
    const uint32_t *id;   /* particle identity, keys the collision draw */
    int model;            /* 0: isotropic scattering at the fixed rate nu;
                             1: Coulomb small-angle scattering, momentum-transfer
                                rate nu at speed vref, scaling as v^-3 */
    double vref;          /* reference speed of model 1, units of c */
    int ee;               /* takes part in the binary (pairwise) collisions */
} orc_species;

typedef struct {
    double W[6];          /* sum F_i^2 dV at time n, Ex Ey Ez Bx By Bz */
    double kinetic[8];    /* dV sum w (gamma^n - 1) per species */
    double p_particles[3];/* dV sum w u^n over all species */
    double p_species[8][3];/* dV sum w u^n per species */
    double p_field[3];    /* dV sum E x B (each product at the E component's point) */
    int64_t collisions;   /* number of scattering events in the step */
    int64_t ee_pairs;     /* binary-collision pairs that scattered in the step */
} orc_diag;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): a 4x32-bit counter and a 2x32-bit
 * key; each round multiplies words 0 and 2 by fixed odd constants, xors
 * the high halves with the other words and the key, permutes, and the key
 * is advanced by the Weyl increments between rounds.                     */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* Philox2x32-10 (same paper): a 2x32-bit counter and a 32-bit key; each
 * round multiplies word 0 by a fixed odd constant, xors the high half with
 * the key and word 1, and the key advances by a Weyl increment.          */
void orc_philox2x32_10(const uint32_t ctr[2], uint32_t key, uint32_t out[2])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], k = key;
    for (int r = 0; r < 10; ++r) {
        if (r > 0) k += 0x9E3779B9u;
        uint64_t p = (uint64_t)0xD256D193u * c0;
        uint32_t hi = (uint32_t)(p >> 32), lo = (uint32_t)p;
        c0 = hi ^ k ^ c1;
        c1 = lo;
    }
    out[0] = c0;
    out[1] = c1;
}

/* uniform in (0,1) from 32 random bits, exact in FP64 */
static double u01(uint32_t r) { return ((double)r + 0.5) * (1.0 / 4294967296.0); }

/* ------------------------------------------------------------------ */
static int wrapi(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }

static size_t cells(const orc_grid *g) { return (size_t)g->n[0] * g->n[1] * g->n[2]; }

static size_t at(const orc_grid *g, int i, int j, int k)
{
    return ((size_t)wrapi(k, g->n[2]) * g->n[1] + wrapi(j, g->n[1])) * g->n[0] + wrapi(i, g->n[0]);
}

/* Yee stagger of each component (in units of a cell), Ex Ey Ez Bx By Bz */
static const double STAG[6][3] = {
    {0.5, 0.0, 0.0}, {0.0, 0.5, 0.0}, {0.0, 0.0, 0.5},
    {0.0, 0.5, 0.5}, {0.5, 0.0, 0.5}, {0.5, 0.5, 0.0},
};

/* Field value at cell coordinates X of the component F with stagger s:
 * linear weights along every resolved axis; an unresolved z (2D) has one
 * node of weight 1.                                                      */
static double interp(const orc_grid *g, const double *F, const double X[3], const double s[3])
{
    int i0[3] = {0, 0, 0};
    double wl[3] = {1.0, 1.0, 1.0}, wh[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < g->ndim; ++a) {
        double xs = X[a] - s[a];
        double fl = floor(xs);
        i0[a] = (int)fl;
        wh[a] = xs - fl;
        wl[a] = 1.0 - wh[a];
    }
    int nk = g->ndim == 3 ? 2 : 1;
    double v = 0.0;
    for (int c = 0; c < nk; ++c)
        for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) {
                double wgt = (a ? wh[0] : wl[0]) * (b ? wh[1] : wl[1]) * (c ? wh[2] : wl[2]);
                v += wgt * F[at(g, i0[0] + a, i0[1] + b, i0[2] + c)];
            }
    return v;
}

void orc_gather(const orc_grid *g, const double x[3], double E[3], double B[3])
{
    double X[3] = {0, 0, 0};
    for (int a = 0; a < g->ndim; ++a) X[a] = x[a] / g->d[a];
    for (int c = 0; c < 3; ++c) {
        E[c] = interp(g, g->E[c], X, STAG[c]);
        B[c] = interp(g, g->B[c], X, STAG[3 + c]);
    }
}

/* Relativistic Boris push (Boris 1970): half electric kick, magnetic
 * rotation with t = (q dt / 2 m gamma^-) B and s = 2t/(1+t^2), half kick.
 * qmdt2 = q dt / (2 m).                                                  */
void orc_boris(double u[3], const double E[3], const double B[3], double qmdt2)
{
    double um[3], t[3], s[3], up[3], w[3];
    for (int i = 0; i < 3; ++i) um[i] = u[i] + qmdt2 * E[i];
    double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    for (int i = 0; i < 3; ++i) t[i] = qmdt2 * B[i] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int i = 0; i < 3; ++i) s[i] = 2.0 * t[i] / (1.0 + t2);
    w[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    w[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    w[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    up[0] = um[0] + (w[1] * s[2] - w[2] * s[1]);
    up[1] = um[1] + (w[2] * s[0] - w[0] * s[2]);
    up[2] = um[2] + (w[0] * s[1] - w[1] * s[0]);
    for (int i = 0; i < 3; ++i) u[i] = up[i] + qmdt2 * E[i];
}

/* Linear (cloud-in-cell) form factor of a particle at cell coordinate X,
 * seen from node i.                                                      */
static double cic(double X, int i)
{
    double r = fabs(X - (double)i);
    return r < 1.0 ? 1.0 - r : 0.0;
}

/* Esirkepov (2001) charge-conserving deposit of one particle moving from
 * x0 to x1 (unwrapped, |x1-x0| < one cell per axis) into J.  The window
 * along each resolved axis starts at floor(min(X0,X1)) and spans 3 nodes,
 * which holds both form factors.  DS = S1 - S0 and
 *   W_x = DS_x (S0_y S0_z + DS_y S0_z/2 + S0_y DS_z/2 + DS_y DS_z/3)
 * (cyclic for y, z); J_x(i+1/2) = J_x(i-1/2) - q w (dx/dt) W_x(i) as a
 * running sum from the window's low edge.  In 2D3V the out-of-plane
 * current is J_z = q w v_z W_z with
 *   W_z = S0_x S0_y + DS_x S0_y/2 + S0_x DS_y/2 + DS_x DS_y/3.          */
void orc_deposit(const orc_grid *g, double *const Jp[3], double qw,
                 const double x0[3], const double x1[3], double vz)
{
    int lo[3] = {0, 0, 0}, nw[3] = {1, 1, 1};
    double S0[3][3], DS[3][3];
    for (int a = 0; a < 3; ++a)
        for (int m = 0; m < 3; ++m) { S0[a][m] = (m == 0) ? 1.0 : 0.0; DS[a][m] = 0.0; }
    for (int a = 0; a < g->ndim; ++a) {
        double X0 = x0[a] / g->d[a], X1 = x1[a] / g->d[a];
        lo[a] = (int)floor(X0 < X1 ? X0 : X1);
        nw[a] = 3;
        for (int m = 0; m < 3; ++m) {
            S0[a][m] = cic(X0, lo[a] + m);
            DS[a][m] = cic(X1, lo[a] + m) - S0[a][m];
        }
    }
    const double third = 1.0 / 3.0;
    /* J_x: running sum along x */
    for (int c = 0; c < nw[2]; ++c)
        for (int b = 0; b < nw[1]; ++b) {
            double acc = 0.0;
            for (int a = 0; a < nw[0]; ++a) {
                double W = DS[0][a] * (S0[1][b] * S0[2][c] + 0.5 * DS[1][b] * S0[2][c]
                                       + 0.5 * S0[1][b] * DS[2][c] + third * DS[1][b] * DS[2][c]);
                acc -= qw * (g->d[0] / g->dt) * W;
                Jp[0][at(g, lo[0] + a, lo[1] + b, lo[2] + c)] += acc;
            }
        }
    /* J_y: running sum along y */
    for (int c = 0; c < nw[2]; ++c)
        for (int a = 0; a < nw[0]; ++a) {
            double acc = 0.0;
            for (int b = 0; b < nw[1]; ++b) {
                double W = DS[1][b] * (S0[0][a] * S0[2][c] + 0.5 * DS[0][a] * S0[2][c]
                                       + 0.5 * S0[0][a] * DS[2][c] + third * DS[0][a] * DS[2][c]);
                acc -= qw * (g->d[1] / g->dt) * W;
                Jp[1][at(g, lo[0] + a, lo[1] + b, lo[2] + c)] += acc;
            }
        }
    if (g->ndim == 3) {
        /* J_z: running sum along z */
        for (int b = 0; b < nw[1]; ++b)
            for (int a = 0; a < nw[0]; ++a) {
                double acc = 0.0;
                for (int c = 0; c < nw[2]; ++c) {
                    double W = DS[2][c] * (S0[0][a] * S0[1][b] + 0.5 * DS[0][a] * S0[1][b]
                                           + 0.5 * S0[0][a] * DS[1][b] + third * DS[0][a] * DS[1][b]);
                    acc -= qw * (g->d[2] / g->dt) * W;
                    Jp[2][at(g, lo[0] + a, lo[1] + b, lo[2] + c)] += acc;
                }
            }
    } else {
        for (int b = 0; b < nw[1]; ++b)
            for (int a = 0; a < nw[0]; ++a) {
                double W = S0[0][a] * S0[1][b] + 0.5 * DS[0][a] * S0[1][b]
                           + 0.5 * S0[0][a] * DS[1][b] + third * DS[0][a] * DS[1][b];
                Jp[2][at(g, lo[0] + a, lo[1] + b, 0)] += qw * vz * W;
            }
    }
}

/* Scattering off the immobile ions.  The decision draw is Philox2x32-10 on
 * counter (id, step) with key  seed_lo ^ (seed_hi * 0x9E3779B9) ^
 * (run * 0x85EBCA6B); the event happens when its word 0 is below
 * floor(P 2^32), P = 1 - exp(-nu dt), an integer decision.  A scattered
 * particle draws its new direction from Philox4x32-10 on counter
 * (id, step, 1, run), key (seed lo, seed hi): cos(theta) = 1 - 2 U(word 1),
 * phi = 2 pi U(word 2); the direction is isotropic and |u| is kept.
 * Returns 1 if the particle scattered.                                    */
uint32_t orc_collision_key(uint64_t seed, uint32_t run)
{
    return (uint32_t)seed ^ ((uint32_t)(seed >> 32) * 0x9E3779B9u) ^ (run * 0x85EBCA6Bu);
}
/* Coulomb small-angle scattering off the immobile ions (Takizuka & Abe
 * 1977, binary collision of an electron with an ion of infinite mass): in a
 * step every electron turns by theta with tan(theta/2) = delta, delta normal
 * with variance nu_m(v) dt / 2, where nu_m(v) = nu (vref/v)^3 is the
 * momentum-transfer rate at speed v = |u|/gamma; the azimuth phi is uniform
 * and |u| is kept.  The draw is Philox4x32-10 on counter (id, step, 3, run),
 * key (seed lo, seed hi): delta = sqrt(var) sqrt(-2 ln U0) cos(2 pi U1),
 * phi = 2 pi U2.  The new momentum follows Takizuka and Abe's rotation of u
 * about itself (u along z when its transverse part is zero).  Returns 1 if
 * the particle turned (u != 0).                                           */
int orc_coulomb(double u[3], uint32_t id, int64_t step, uint64_t seed, uint32_t run, double nu, double vref,
                double dt)
{
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!(u2 > 0.0) || !(nu > 0.0)) return 0;
    uint32_t ctr[4] = {id, (uint32_t)step, 3u, run};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    const double U = sqrt(u2);
    const double v = U / sqrt(1.0 + u2);
    const double var = 0.5 * nu * dt * (vref / v) * (vref / v) * (vref / v);
    const double delta = sqrt(var) * sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * M_PI * u01(r[1]));
    const double d2 = delta * delta;
    const double ct = (1.0 - d2) / (1.0 + d2), st = 2.0 * delta / (1.0 + d2);
    const double ph = 2.0 * M_PI * u01(r[2]);
    const double cp = cos(ph), sp = sin(ph);
    const double up = sqrt(u[0] * u[0] + u[1] * u[1]);
    double du[3];
    if (up > 0.0) {
        du[0] = (u[0] * u[2] / up) * st * cp - (u[1] * U / up) * st * sp - u[0] * (1.0 - ct);
        du[1] = (u[1] * u[2] / up) * st * cp + (u[0] * U / up) * st * sp - u[1] * (1.0 - ct);
        du[2] = -up * st * cp - u[2] * (1.0 - ct);
    } else {
        du[0] = U * st * cp;
        du[1] = U * st * sp;
        du[2] = -u[2] * (1.0 - ct);
    }
    for (int c = 0; c < 3; ++c) u[c] += du[c];
    return 1;
}

uint32_t orc_collision_threshold(double nu, double dt)
{
    double P = 1.0 - exp(-nu * dt);
    double t = floor(P * 4294967296.0);
    if (t < 0.0) t = 0.0;
    if (t > 4294967295.0) t = 4294967295.0;
    return (uint32_t)t;
}

int orc_collide(double u[3], uint32_t id, int64_t step, uint64_t seed, uint32_t run, uint32_t thr)
{
    uint32_t dctr[2] = {id, (uint32_t)step}, d[2];
    orc_philox2x32_10(dctr, orc_collision_key(seed, run), d);
    if (!(d[0] < thr)) return 0;
    uint32_t ctr[4] = {id, (uint32_t)step, 1u, run};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    double um = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double ct = 1.0 - 2.0 * u01(r[1]);
    double st = sqrt(fmax(0.0, 1.0 - ct * ct));
    double ph = 2.0 * M_PI * u01(r[2]);
    u[0] = um * st * cos(ph);
    u[1] = um * st * sin(ph);
    u[2] = um * ct;
    return 1;
}

/* ------------------------------------------------------------------ */
/* Binary collisions between the particles of the species that take part
 * (the paper's "binary collision module", velocity-dependent variant):
 * Takizuka & Abe (1977) pairing inside each cell, with the scattering done
 * in the pair's centre-of-momentum frame so that relativistic pairs (the
 * beam on the return current) keep their total four-momentum.
 *
 * Pairing (at the positions x^{n+1}, after the push, move, deposit and the
 * scattering off the ions): the participants of a cell are ordered by the
 * sort key word 0 of Philox4x32-10 on counter (id, step, 4, run), key
 * (seed lo, seed hi) -- a random permutation that does not depend on the
 * storage order -- with ties broken by id.  Pairs are (0,1), (2,3), ...;
 * with an odd count N >= 3 the first three form the pairs (0,1), (1,2),
 * (2,0), each at half the variance (Takizuka and Abe's rule), and the pairs
 * continue from the fourth.
 *
 * One pair (a, b), a the first of the two: draws from Philox4x32-10 on
 * counter (id_a, step, 5, run), key (seed lo, seed hi).  With the
 * lab-frame relative velocity v_rel = |u_a/gamma_a - u_b/gamma_b| the
 * deflection of the relative momentum in the centre-of-momentum frame is
 * tan(theta/2) = delta, delta = s sqrt(-2 ln U0) cos(2 pi U1),
 * s^2 = f (nu dt / 2) (vref / v_rel)^3 (f = 1, or 1/2 in the triple): the
 * rate nu at relative speed vref with Coulomb's v^-3 law; the azimuth is
 * phi = 2 pi U2.  The momentum p*_a of a in that frame is turned by
 * (theta, phi) about itself (the rotation of Takizuka and Abe), p*_b =
 * -p*_a, and both are boosted back.  Equal weights: both particles take the
 * new momenta, so the pair keeps its momentum and energy.  Unequal weights
 * (Nanbu and Yonemura 1998): the particle of smaller weight always takes its
 * new momentum, the other only if U3 < w_small / w_large, which keeps
 * momentum and energy in expectation.  A pair with v_rel = 0 is left alone.
 * Returns the number of pairs that scattered.                            */
typedef struct {
    int64_t cell;
    uint32_t key, id;
    int s;
    int64_t p;
} orc_ee_entry;

static int ee_cmp(const void *x, const void *y)
{
    const orc_ee_entry *a = (const orc_ee_entry *)x, *b = (const orc_ee_entry *)y;
    if (a->cell != b->cell) return a->cell < b->cell ? -1 : 1;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->id != b->id) return a->id < b->id ? -1 : 1;
    return 0;
}

/* Lorentz boost of a four-momentum (e, p) by velocity bv (|bv| < 1):
 * sign +1 to the frame moving with bv, -1 back from it. */
static void boost(const double bv[3], double gc, double sign, double *e, double p[3])
{
    const double b2 = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
    if (!(b2 > 0.0)) return;
    const double bp = bv[0] * p[0] + bv[1] * p[1] + bv[2] * p[2];
    const double c = (gc - 1.0) * bp / b2 - sign * gc * (*e);
    const double en = gc * ((*e) - sign * bp);
    for (int i = 0; i < 3; ++i) p[i] += c * bv[i];
    *e = en;
}

int orc_ee_pair(double ua[3], double ma, double wa, uint32_t ida, double ub[3], double mb, double wb,
                double f, int64_t step, uint64_t seed, uint32_t run, double nu, double vref, double dt)
{
    const double ga = sqrt(1.0 + ua[0] * ua[0] + ua[1] * ua[1] + ua[2] * ua[2]);
    const double gb = sqrt(1.0 + ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
    double dv[3];
    for (int i = 0; i < 3; ++i) dv[i] = ua[i] / ga - ub[i] / gb;
    const double vrel = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    if (!(vrel > 0.0)) return 0;
    uint32_t ctr[4] = {ida, (uint32_t)step, 5u, run};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    const double s2 = f * 0.5 * nu * dt * (vref / vrel) * (vref / vrel) * (vref / vrel);
    const double delta = sqrt(s2) * sqrt(-2.0 * log(u01(r[0]))) * cos(2.0 * M_PI * u01(r[1]));
    const double d2 = delta * delta;
    const double st = 2.0 * delta / (1.0 + d2), omc = 2.0 * d2 / (1.0 + d2);
    const double ph = 2.0 * M_PI * u01(r[2]);
    const double cp = cos(ph), sp = sin(ph);
    /* which of the two take the new momenta */
    int take_a = 1, take_b = 1;
    if (wa != wb) {
        const int a_heavy = wa > wb;
        const double ratio = a_heavy ? wb / wa : wa / wb;
        const int heavy_scatters = u01(r[3]) < ratio;
        if (a_heavy) take_a = heavy_scatters;
        else take_b = heavy_scatters;
    }
    /* centre-of-momentum frame */
    const double E = ma * ga + mb * gb;
    double P[3], bv[3];
    for (int i = 0; i < 3; ++i) {
        P[i] = ma * ua[i] + mb * ub[i];
        bv[i] = P[i] / E;
    }
    const double gc = E / sqrt(E * E - (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]));
    double ea = ma * ga, pa[3] = {ma * ua[0], ma * ua[1], ma * ua[2]};
    boost(bv, gc, 1.0, &ea, pa);
    /* turn p*_a by (theta, phi) about itself */
    const double pm = sqrt(pa[0] * pa[0] + pa[1] * pa[1] + pa[2] * pa[2]);
    const double pp = sqrt(pa[0] * pa[0] + pa[1] * pa[1]);
    double dp[3];
    if (pp > 0.0) {
        dp[0] = (pa[0] * pa[2] / pp) * st * cp - (pa[1] * pm / pp) * st * sp - pa[0] * omc;
        dp[1] = (pa[1] * pa[2] / pp) * st * cp + (pa[0] * pm / pp) * st * sp - pa[1] * omc;
        dp[2] = -pp * st * cp - pa[2] * omc;
    } else {
        dp[0] = pm * st * cp;
        dp[1] = pm * st * sp;
        dp[2] = -pa[2] * omc;
    }
    double qa[3], qb[3];
    for (int i = 0; i < 3; ++i) {
        qa[i] = pa[i] + dp[i];
        qb[i] = -qa[i];
    }
    const double eas = sqrt(ma * ma + qa[0] * qa[0] + qa[1] * qa[1] + qa[2] * qa[2]);
    const double ebs = sqrt(mb * mb + qb[0] * qb[0] + qb[1] * qb[1] + qb[2] * qb[2]);
    double e1 = eas;
    boost(bv, gc, -1.0, &e1, qa);
    if (take_a && take_b) {
        for (int i = 0; i < 3; ++i) {
            const double pb = P[i] - qa[i];
            ua[i] = qa[i] / ma;
            ub[i] = pb / mb;
        }
    } else if (take_a) {
        for (int i = 0; i < 3; ++i) ua[i] = qa[i] / ma;
    } else {
        double e2 = ebs;
        boost(bv, gc, -1.0, &e2, qb);
        for (int i = 0; i < 3; ++i) ub[i] = qb[i] / mb;
    }
    return 1;
}

int64_t orc_ee_collide(const orc_grid *g, orc_species *sp, int ns, int64_t step, uint64_t seed, uint32_t run)
{
    int64_t total = 0;
    for (int s = 0; s < ns; ++s)
        if (sp[s].ee) total += sp[s].n;
    if (total < 2 || !(g->nu_ee > 0.0)) return 0;
    orc_ee_entry *ent = (orc_ee_entry *)malloc((size_t)total * sizeof(orc_ee_entry));
    if (!ent) return -1;
    int64_t k = 0;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int s = 0; s < ns; ++s) {
        if (!sp[s].ee) continue;
        for (int64_t p = 0; p < sp[s].n; ++p) {
            int c[3] = {0, 0, 0};
            for (int a = 0; a < g->ndim; ++a) c[a] = wrapi((int)floor(sp[s].x[a][p] / g->d[a]), g->n[a]);
            uint32_t ctr[4] = {sp[s].id[p], (uint32_t)step, 4u, run}, r[4];
            orc_philox4x32_10(ctr, key, r);
            ent[k].cell = ((int64_t)c[2] * g->n[1] + c[1]) * g->n[0] + c[0];
            ent[k].key = r[0];
            ent[k].id = sp[s].id[p];
            ent[k].s = s;
            ent[k].p = p;
            ++k;
        }
    }
    qsort(ent, (size_t)total, sizeof(orc_ee_entry), ee_cmp);
    int64_t pairs = 0;
    for (int64_t i0 = 0; i0 < total;) {
        int64_t i1 = i0;
        while (i1 < total && ent[i1].cell == ent[i0].cell) ++i1;
        const int64_t N = i1 - i0;
        int64_t start = i0;
        if (N >= 3 && (N & 1)) {
            static const int tri[3][2] = {{0, 1}, {1, 2}, {2, 0}};
            for (int t = 0; t < 3; ++t) {
                const orc_ee_entry *A = &ent[i0 + tri[t][0]], *B = &ent[i0 + tri[t][1]];
                orc_species *SA = &sp[A->s], *SB = &sp[B->s];
                double ua[3] = {SA->u[0][A->p], SA->u[1][A->p], SA->u[2][A->p]};
                double ub[3] = {SB->u[0][B->p], SB->u[1][B->p], SB->u[2][B->p]};
                pairs += orc_ee_pair(ua, SA->m, SA->w, A->id, ub, SB->m, SB->w, 0.5, step, seed, run, g->nu_ee,
                                     g->ee_vref, g->dt);
                for (int c = 0; c < 3; ++c) {
                    SA->u[c][A->p] = ua[c];
                    SB->u[c][B->p] = ub[c];
                }
            }
            start = i0 + 3;
        }
        for (int64_t i = start; i + 1 < i1; i += 2) {
            const orc_ee_entry *A = &ent[i], *B = &ent[i + 1];
            orc_species *SA = &sp[A->s], *SB = &sp[B->s];
            double ua[3] = {SA->u[0][A->p], SA->u[1][A->p], SA->u[2][A->p]};
            double ub[3] = {SB->u[0][B->p], SB->u[1][B->p], SB->u[2][B->p]};
            pairs += orc_ee_pair(ua, SA->m, SA->w, A->id, ub, SB->m, SB->w, 1.0, step, seed, run, g->nu_ee,
                                 g->ee_vref, g->dt);
            for (int c = 0; c < 3; ++c) {
                SA->u[c][A->p] = ua[c];
                SB->u[c][B->p] = ub[c];
            }
        }
        i0 = i1;
    }
    free(ent);
    return pairs;
}

/* ------------------------------------------------------------------ */
/* Yee (1966) updates.  h = fraction of dt for the B half steps.         */
void orc_yee_b(const orc_grid *g, double h)
{
    const double cx = h * g->dt / g->d[0], cy = h * g->dt / g->d[1];
    const double cz = g->ndim == 3 ? h * g->dt / g->d[2] : 0.0;
    double *Ex = g->E[0], *Ey = g->E[1], *Ez = g->E[2];
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                size_t o = at(g, i, j, k);
                g->B[0][o] -= cy * (Ez[at(g, i, j + 1, k)] - Ez[o]) - cz * (Ey[at(g, i, j, k + 1)] - Ey[o]);
                g->B[1][o] -= cz * (Ex[at(g, i, j, k + 1)] - Ex[o]) - cx * (Ez[at(g, i + 1, j, k)] - Ez[o]);
                g->B[2][o] -= cx * (Ey[at(g, i + 1, j, k)] - Ey[o]) - cy * (Ex[at(g, i, j + 1, k)] - Ex[o]);
            }
}

void orc_yee_e(const orc_grid *g)
{
    const double dt = g->dt, cx = dt / g->d[0], cy = dt / g->d[1];
    const double cz = g->ndim == 3 ? dt / g->d[2] : 0.0;
    double *Bx = g->B[0], *By = g->B[1], *Bz = g->B[2];
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                size_t o = at(g, i, j, k);
                g->E[0][o] += cy * (Bz[o] - Bz[at(g, i, j - 1, k)]) - cz * (By[o] - By[at(g, i, j, k - 1)]) - dt * g->J[0][o];
                g->E[1][o] += cz * (Bx[o] - Bx[at(g, i, j, k - 1)]) - cx * (Bz[o] - Bz[at(g, i - 1, j, k)]) - dt * g->J[1][o];
                g->E[2][o] += cx * (By[o] - By[at(g, i - 1, j, k)]) - cy * (Bx[o] - Bx[at(g, i, j - 1, k)]) - dt * g->J[2][o];
            }
}

/* ------------------------------------------------------------------ */
/* Diagnostics.                                                         */
static double cell_volume(const orc_grid *g)
{
    return g->d[0] * g->d[1] * (g->ndim == 3 ? g->d[2] : 1.0);
}

/* W_i = sum over cells of F_i^2 dV: the per-component field energy that
 * the paper records (its field-energy diagnostic), without a factor 1/2. */
void orc_field_energy(const orc_grid *g, double W[6])
{
    size_t nc = cells(g);
    double dv = cell_volume(g);
    for (int c = 0; c < 6; ++c) {
        const double *F = c < 3 ? g->E[c] : g->B[c - 3];
        double s = 0.0;
        for (size_t o = 0; o < nc; ++o) s += F[o] * F[o];
        W[c] = s * dv;
    }
}

/* z component of the field momentum, dV sum (E_x B_y - E_y B_x); B_x, B_y
 * are averaged over their two z neighbours onto the E_x, E_y points (in
 * 2D the pairs are co-located and the average is the identity).         */
/* Field momentum sum E x B dV.  Each product E_a B_b is taken at E_a's
 * point; B_b is averaged over the two points around it along the axis in
 * which the staggers differ (Yee: E_x (i+1/2,j,k), B_y (i+1/2,j,k+1/2),
 * B_z (i+1/2,j+1/2,k) and cyclically).                                    */
void orc_field_momentum(const orc_grid *g, double p[3])
{
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                size_t o = at(g, i, j, k);
                size_t mi = at(g, i - 1, j, k), mj = at(g, i, j - 1, k), mk = at(g, i, j, k - 1);
                const double *E[3] = {g->E[0], g->E[1], g->E[2]}, *B[3] = {g->B[0], g->B[1], g->B[2]};
                s[0] += E[1][o] * 0.5 * (B[2][o] + B[2][mi]) - E[2][o] * 0.5 * (B[1][o] + B[1][mi]);
                s[1] += E[2][o] * 0.5 * (B[0][o] + B[0][mj]) - E[0][o] * 0.5 * (B[2][o] + B[2][mj]);
                s[2] += E[0][o] * 0.5 * (B[1][o] + B[1][mk]) - E[1][o] * 0.5 * (B[0][o] + B[0][mk]);
            }
    for (int c = 0; c < 3; ++c) p[c] = s[c] * cell_volume(g);
}

/* charge density on integer nodes, rho = sum q w S(x) (CIC) */
void orc_rho(const orc_grid *g, const orc_species *sp, int ns, double *rho)
{
    memset(rho, 0, cells(g) * sizeof(double));
    for (int s = 0; s < ns; ++s) {
        double qw = sp[s].q * sp[s].w;
        for (int64_t p = 0; p < sp[s].n; ++p) {
            int i0[3] = {0, 0, 0};
            double wl[3] = {1, 1, 1}, wh[3] = {0, 0, 0};
            for (int a = 0; a < g->ndim; ++a) {
                double X = sp[s].x[a][p] / g->d[a];
                double fl = floor(X);
                i0[a] = (int)fl;
                wh[a] = X - fl;
                wl[a] = 1.0 - wh[a];
            }
            int nk = g->ndim == 3 ? 2 : 1;
            for (int c = 0; c < nk; ++c)
                for (int b = 0; b < 2; ++b)
                    for (int a = 0; a < 2; ++a)
                        rho[at(g, i0[0] + a, i0[1] + b, i0[2] + c)] +=
                            qw * (a ? wh[0] : wl[0]) * (b ? wh[1] : wl[1]) * (c ? wh[2] : wl[2]);
        }
    }
}

/* divergence on integer nodes of a vector field co-located with E */
void orc_divergence(const orc_grid *g, double *const F[3], double *out)
{
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i) {
                size_t o = at(g, i, j, k);
                double v = (F[0][o] - F[0][at(g, i - 1, j, k)]) / g->d[0]
                         + (F[1][o] - F[1][at(g, i, j - 1, k)]) / g->d[1];
                if (g->ndim == 3) v += (F[2][o] - F[2][at(g, i, j, k - 1)]) / g->d[2];
                out[o] = v;
            }
}

/* ------------------------------------------------------------------ */
/* One full PIC step n -> n+1.                                          */
#define ORC_CHUNKS 16

static double wrap_pos(double x, double L)
{
    while (x < 0.0) x += L;
    while (x >= L) x -= L;
    return x;
}

int orc_step(const orc_grid *g, orc_species *sp, int ns, int64_t step,
             uint64_t seed, uint32_t run, orc_diag *diag)
{
    size_t nc = cells(g);
    double dv = cell_volume(g);
    double L[3] = {g->n[0] * g->d[0], g->n[1] * g->d[1], g->n[2] * g->d[2]};
    if (diag) {
        memset(diag, 0, sizeof(*diag));
        orc_field_energy(g, diag->W);
        orc_field_momentum(g, diag->p_field);
    }
    /* per-chunk current partials, summed in chunk order: the result does
     * not depend on the number of threads                                 */
    double *part = (double *)calloc((size_t)ORC_CHUNKS * 3 * nc, sizeof(double));
    if (!part) return -1;
    double ke[ORC_CHUNKS][8], pp[ORC_CHUNKS][8][3];
    int64_t ncoll[ORC_CHUNKS];
    memset(ke, 0, sizeof(ke)); memset(pp, 0, sizeof(pp)); memset(ncoll, 0, sizeof(ncoll));

    #pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
        double *Jp[3] = {part + ((size_t)ch * 3 + 0) * nc, part + ((size_t)ch * 3 + 1) * nc,
                         part + ((size_t)ch * 3 + 2) * nc};
        for (int s = 0; s < ns; ++s) {
            orc_species *S = &sp[s];
            const double qmdt2 = S->q * g->dt / (2.0 * S->m);
            const double qw = S->q * S->w;
            const uint32_t thr = (S->nu > 0.0 && S->model == 0) ? orc_collision_threshold(S->nu, g->dt) : 0u;
            const int coulomb = S->nu > 0.0 && S->model == 1;
            int64_t p0 = S->n * ch / ORC_CHUNKS, p1 = S->n * (ch + 1) / ORC_CHUNKS;
            for (int64_t p = p0; p < p1; ++p) {
                double x0[3] = {0, 0, 0}, x1[3] = {0, 0, 0}, E[3], B[3];
                double u[3] = {S->u[0][p], S->u[1][p], S->u[2][p]};
                for (int a = 0; a < g->ndim; ++a) x0[a] = S->x[a][p];
                double g_old = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                double u_old[3] = {u[0], u[1], u[2]};
                orc_gather(g, x0, E, B);
                orc_boris(u, E, B, qmdt2);
                double gam = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                for (int a = 0; a < g->ndim; ++a) x1[a] = x0[a] + g->dt * u[a] / gam;
                orc_deposit(g, Jp, qw, x0, x1, u[2] / gam);
                if (diag) {
                    ke[ch][s] += S->w * (0.5 * (g_old + gam) - 1.0);
                    for (int c = 0; c < 3; ++c) pp[ch][s < 8 ? s : 7][c] += S->w * 0.5 * (u_old[c] + u[c]);
                }
                if (thr && S->id) ncoll[ch] += orc_collide(u, S->id[p], step, seed, run, thr);
                if (coulomb && S->id) ncoll[ch] += orc_coulomb(u, S->id[p], step, seed, run, S->nu, S->vref, g->dt);
                for (int a = 0; a < g->ndim; ++a) S->x[a][p] = wrap_pos(x1[a], L[a]);
                S->u[0][p] = u[0]; S->u[1][p] = u[1]; S->u[2][p] = u[2];
            }
        }
    }
    for (int c = 0; c < 3; ++c) {
        double *J = g->J[c];
        for (size_t o = 0; o < nc; ++o) {
            double v = 0.0;
            for (int ch = 0; ch < ORC_CHUNKS; ++ch) v += part[((size_t)ch * 3 + c) * nc + o];
            J[o] = v;
        }
    }
    free(part);
    /* binary collisions at the new positions, after the scattering off the ions */
    const int64_t ee = orc_ee_collide(g, sp, ns, step, seed, run);
    if (ee < 0) return -1;
    if (diag) diag->ee_pairs = ee;
    if (diag) {
        for (int ch = 0; ch < ORC_CHUNKS; ++ch) {
            for (int s = 0; s < ns && s < 8; ++s) diag->kinetic[s] += ke[ch][s] * dv;
            for (int s = 0; s < ns && s < 8; ++s)
                for (int c = 0; c < 3; ++c) {
                    diag->p_species[s][c] += pp[ch][s][c] * dv;
                    diag->p_particles[c] += pp[ch][s][c] * dv;
                }
            diag->collisions += ncoll[ch];
        }
    } else {
        (void)ncoll;
    }
    orc_yee_b(g, 0.5);
    orc_yee_e(g);
    orc_yee_b(g, 0.5);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
