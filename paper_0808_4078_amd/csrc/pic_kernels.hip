// HIP kernels of the beam-plasma PIC step for gfx950 (MI355X).
//
// One step (gather -> Boris push -> move -> Esirkepov deposit -> scattering ->
// current reduction -> Yee update) is a fixed sequence of launches:
//   k_field_diag     FP64 field energies of E^n, B^n on diagnostic steps
//   k_particle       one workgroup per particle tile: E/B staged in LDS,
//                    per-particle gather, push, move, charge-conserving
//                    deposit into an LDS current tile, scattering, and
//                    binning of the particle into the next step's store
//   k_rebin_*        re-layout of the particle store (early exit unless an
//                    incoming-mover reserve overflowed during the step)
//   k_reduce_j       fixed-order FP64 sum of the overlapping tile currents
//   k_yee_b/k_yee_e  B half step, E full step with -J, B half step
//   k_rho/k_gauss    (only with PIC_FLAG_GAUSS_RESIDUAL, on diagnostic steps)
//                    CIC charge of the particles and max |div E - (rho - rho_0)|
//   k_rho/k_continuity (the same steps, after the current reduction) charge
//                    after the move and max |rho^{n+1} - rho^n + dt div J|
//   k_advance        diagnostic record, counter reset, step/parity update
//
// The numerical scheme is the relativistic Boris push (Boris 1970), the
// Esirkepov (2001) charge-conserving deposit with the linear form factor and
// the Yee (1966) FDTD update on the staggered grid
//   Ex(i+1/2,j) Ey(i,j+1/2) Ez(i,j) Bx(i,j+1/2) By(i+1/2,j) Bz(i+1/2,j+1/2),
// half-integer positions stored at the lower integer index, J with E.
// Collisions follow the fluid drag of Eq. (3): each step a collisional
// particle is scattered isotropically off the immobile ions with
// probability 1 - exp(-nu dt), |u| kept; or, per species, every particle is
// turned by a small Coulomb angle whose variance scales as v^-3
// (Takizuka-Abe), |u| kept.  Units: t in 1/w_p, x in c/w_p, u = gamma v/c,
// fields e F/(m c w_p).
#include <hip/hip_ext.h>
#include <algorithm>
#include <hip/hip_runtime.h>

#include "pic_internal.hpp"

namespace pic {

// Pointers read from the parameter block are generic to the compiler; the
// particle and field arrays are in global memory, and saying so gives global
// (not flat) loads, stores and atomics.
#define GLB __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLB T *gbl(T *p) { return (GLB T *)p; }
template <typename T> __device__ __forceinline__ const GLB T *gbl(const T *p) { return (const GLB T *)p; }
// Element access with a 32-bit byte offset from a scalar base (every
// particle array is smaller than 4 GiB; pic_query checks it), which maps to
// the base-register + 32-bit-offset form of global loads and stores.
template <typename T> __device__ __forceinline__ T ld(const GLB T *base, uint32_t i)
{
    return *(const GLB T *)((const GLB char *)base + i * (uint32_t)sizeof(T));
}
template <typename T> __device__ __forceinline__ void st(GLB T *base, uint32_t i, T v)
{
    *(GLB T *)((GLB char *)base + i * (uint32_t)sizeof(T)) = v;
}

// LDS current deposit.  Most particles do not cross a node line in a step, so
// many window weights are exactly zero; skipping them keeps those lanes off
// the LDS atomic unit.
template <typename A, typename R>
__device__ __forceinline__ void lds_add(A *p, R v)
{
    if (v != R(0)) atomicAdd(p, A(v));
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Philox2x32-10 (same paper): the per-step scatter decision needs one word.
__device__ __forceinline__ uint32_t philox2x32_10_w0(uint32_t c0, uint32_t c1, uint32_t k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p = (uint64_t)0xD256D193u * c0;
        const uint32_t hi = (uint32_t)(p >> 32), lo = (uint32_t)p;
        c0 = hi ^ k ^ c1;
        c1 = lo;
        k += 0x9E3779B9u;
    }
    return c0;
}

__device__ __forceinline__ double u01d(uint32_t r) { return ((double)r + 0.5) * 2.3283064365386963e-10; }

// uniform in (0,1) in FP32, exactly representable
__device__ __forceinline__ float u01f(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-8f + 2.98023223876953125e-8f; }

template <typename R> struct Arith;
template <> struct Arith<float> {
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ void sc(float a, float *s, float *c) { sincosf(a, s, c); }
    static __device__ __forceinline__ float ln(float x) { return logf(x); }
    static __device__ __forceinline__ float cs(float a) { return cosf(a); }
};
template <> struct Arith<double> {
    static __device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ void sc(double a, double *s, double *c) { sincos(a, s, c); }
    static __device__ __forceinline__ double ln(double x) { return log(x); }
    static __device__ __forceinline__ double cs(double a) { return cos(a); }
};

// Mixed precision: a particle in a bin keeps its cell within the tile (16
// bits, lx | ly << ts | lz << 2 ts with ts = log2 T; the tile follows from
// the bin, and a tile's origin is a multiple of T on every axis), the
// overflow list the global packed cell (ix | iy << csh[1] | iz << csh[2]).
__device__ __forceinline__ uint32_t local_of_global(const Geometry &g, uint32_t c)
{
    const int ts = g.tshift[0];
    const uint32_t m = (uint32_t)g.tile[0] - 1u;
    uint32_t l = 0;
    for (int a = 0; a < g.ndim; ++a) l |= (((c >> g.csh[a]) & g.cmask[a]) & m) << (a * ts);
    return l;
}

// The step counter and particle-set parity live in memory that kernels also
// update; reading them through readfirstlane tells the compiler they are
// uniform, so everything indexed by them stays in scalar registers.
template <typename KP>
__device__ __forceinline__ int64_t uniform_step(KP kp)
{
    const int64_t v = kp->state->step;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
// A value every lane of the wave holds (read from LDS or from memory at a
// uniform address) as a scalar.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
template <typename P>
__device__ __forceinline__ P *wave_uniform_ptr(P *p)
{
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P *)(((uint64_t)hi << 32) | lo);
}

template <typename KP>
__device__ __forceinline__ int uniform_par(KP kp)
{
    return __builtin_amdgcn_readfirstlane(kp->state->par);
}

template <typename KP>
__device__ __forceinline__ bool diag_step(KP kp, int64_t step)
{
    return kp->diag_every > 0 && (step % kp->diag_every) == 0;
}

// Block-wide FP64 sum of N values held per thread; result valid in thread 0.
// Fixed reduction order, so repeated runs give identical bits.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*sred)[N])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double x = v[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
        v[i] = x;
    }
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) sred[wave][i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double x = sred[0][i];
            for (int w = 1; w < nw; ++w) x += sred[w][i];
            v[i] = x;
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Field energies W_i = sum F_i^2 dV and z field momentum of E^n, B^n.
template <typename R>
__device__ __forceinline__ void field_diag_body(const KParams *__restrict__ kp, int bid, int nb)
{
    __shared__ double sred[4][9];
    const int64_t step = uniform_step(kp);
    if (!diag_step(kp, step)) return;
    const R *F = (const R *)kp->F;
    const int64_t cells = kp->g.cells;
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int64_t nxy = (int64_t)nx * ny;
    double a[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t o = (int64_t)bid * 256 + threadIdx.x; o < cells; o += (int64_t)nb * 256) {
        double v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            v[c] = (double)F[c * cells + o];
            a[c] += v[c] * v[c];
        }
        // E x B with each product at its E component's point: B averaged over
        // the two points around it along the axis where the staggers differ
        const int i = (int)(o % nx), j = (int)((o / nx) % ny);
        const int64_t mi = i ? o - 1 : o + nx - 1;                 // i-1
        const int64_t mj = j ? o - nx : o + nxy - nx;              // j-1
        const int64_t mk = o >= nxy ? o - nxy : o + cells - nxy;   // k-1 (2D: the same cell)
        const double bz_i = 0.5 * (v[5] + (double)F[5 * cells + mi]);
        const double by_i = 0.5 * (v[4] + (double)F[4 * cells + mi]);
        const double bx_j = 0.5 * (v[3] + (double)F[3 * cells + mj]);
        const double bz_j = 0.5 * (v[5] + (double)F[5 * cells + mj]);
        const double by_k = 0.5 * (v[4] + (double)F[4 * cells + mk]);
        const double bx_k = 0.5 * (v[3] + (double)F[3 * cells + mk]);
        a[6] += v[1] * bz_i - v[2] * by_i;
        a[7] += v[2] * bx_j - v[0] * bz_j;
        a[8] += v[0] * by_k - v[1] * bx_k;
    }
    block_sum<9>(a, sred);
    if (threadIdx.x == 0)
        for (int c = 0; c < 9; ++c) kp->field_diag[bid * kFieldDiag + c] = a[c];
}

// ---------------------------------------------------------------------------
// The particle kernel.  One workgroup per tile of T^D cells (D = 2: the
// 2D3V transverse plane, z ignorable; D = 3: 3D3V).
//
// LDS: E, B on the nodes [t0-1, t0+T] of every resolved axis ((T+2)^D per
// component) and the tile current on [t0-1, t0+T+1] ((T+3)^D per component),
// accumulated in type A.  A particle in cell i of the tile has local cell
// lc = i - t0 + 1 in both arrays.  Its 3-node deposit window per axis is
// anchored at the nearest node (i or i+1), which holds the form factor
// before and after a move of less than half a cell.
//
// Per particle: gather -> Boris -> move -> Esirkepov deposit -> scattering
// -> binning into the next step's store (stayers at the bin front through a
// wave-aggregated LDS counter; movers at the back of their new tile's bin,
// above the particles that tile held at the step start; overflow list when
// that room is used up).

// Field at local cell (b[0], b[1], b[2]) with per-axis weights (w0, w1):
// bilinear over 4 nodes (D = 2) or trilinear over 8 (D = 3).
template <typename R, int D, int NF>
__device__ __forceinline__ R interp(const R *F, int bx, int by, int bz, R x0, R x1, R y0, R y1, R z0, R z1)
{
    const int o = (D == 3 ? bz * NF * NF : 0) + by * NF + bx;
    R v = y0 * (x0 * F[o] + x1 * F[o + 1]) + y1 * (x0 * F[o + NF] + x1 * F[o + NF + 1]);
    if constexpr (D == 3) {
        const int q = o + NF * NF;
        v = z0 * v + z1 * (y0 * (x0 * F[q] + x1 * F[q + 1]) + y1 * (x0 * F[q + NF] + x1 * F[q + NF + 1]));
    }
    return v;
}

// Esirkepov deposit of one move into the LDS current tile.  Positions are
// in cell units relative to the particle's cell (local cell lc, whose lower
// node has local index lc): x0 at t^n (in [0,1)), x1 at t^{n+1}.  kd = q w
// d_a/dt per axis; kzv = q w v_z (2D out-of-plane current).
//
// Pair factors P_pq[m][l] = S0p S0q + DSp S0q/2 + S0p DSq/2 + DSp DSq/3 with
// DS = S1 - S0; W_x = DSx Pyz, W_y = DSy Pxz, W_z = DSz Pxy (3D) and each
// current is the running sum of -q w (d/dt) W along its own axis.  In 2D,
// J_z = q w v_z Pxy.

// General case: 3-node window per axis around the node nearest to x0, which
// holds the form factor before and after any move shorter than half a cell.
template <typename R, typename A, int D, int NJ>
__device__ __forceinline__ void deposit_window(A *sJx, A *sJy, A *sJz, const int (&lc)[3], const R (&x0)[3],
                                               const R (&x1)[3], const R (&kd)[3], R kzv)
{
    constexpr int SY = NJ, SZ = NJ * NJ;
    R S0[3][3], DS[3][3];
    int w0 = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const int ca = x0[a] >= R(0.5) ? 1 : 0;
        const R d0 = x0[a] - R(ca), d1 = x1[a] - R(ca);
        S0[a][0] = fmax(R(0), -d0);
        S0[a][1] = R(1) - fabs(d0);
        S0[a][2] = fmax(R(0), d0);
        DS[a][0] = fmax(R(0), -d1) - S0[a][0];
        DS[a][1] = R(1) - fabs(d1) - S0[a][1];
        DS[a][2] = fmax(R(0), d1) - S0[a][2];
        w0 += (lc[a] + ca - 1) * (a == 0 ? 1 : a == 1 ? SY : SZ);
    }
    if constexpr (D == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const R ry = S0[1][b] + R(0.5) * DS[1][b];
            const R qy = R(0.5) * S0[1][b] + R(1.0 / 3.0) * DS[1][b];
            const R j0 = -kd[0] * (DS[0][0] * ry);
            const R j1 = j0 - kd[0] * (DS[0][1] * ry);
            lds_add(&sJx[w0 + b * SY], j0);
            lds_add(&sJx[w0 + b * SY + 1], j1);
#pragma unroll
            for (int a = 0; a < 3; ++a) lds_add(&sJz[w0 + b * SY + a], kzv * (S0[0][a] * ry + DS[0][a] * qy));
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const R rx = S0[0][a] + R(0.5) * DS[0][a];
            const R j0 = -kd[1] * (DS[1][0] * rx);
            const R j1 = j0 - kd[1] * (DS[1][1] * rx);
            lds_add(&sJy[w0 + a], j0);
            lds_add(&sJy[w0 + SY + a], j1);
        }
    } else {
        auto P = [&](int p, int q, int m, int l) {
            return S0[p][m] * (S0[q][l] + R(0.5) * DS[q][l]) + DS[p][m] * (R(0.5) * S0[q][l] + R(1.0 / 3.0) * DS[q][l]);
        };
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const R pyz = P(1, 2, b, c);
                const R j0 = -kd[0] * (DS[0][0] * pyz);
                const R j1 = j0 - kd[0] * (DS[0][1] * pyz);
                const int o = w0 + c * SZ + b * SY;
                lds_add(&sJx[o], j0);
                lds_add(&sJx[o + 1], j1);
            }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R pxz = P(0, 2, a, c);
                const R j0 = -kd[1] * (DS[1][0] * pxz);
                const R j1 = j0 - kd[1] * (DS[1][1] * pxz);
                const int o = w0 + c * SZ + a;
                lds_add(&sJy[o], j0);
                lds_add(&sJy[o + SY], j1);
            }
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R pxy = P(0, 1, a, b);
                const R j0 = -kd[2] * (DS[2][0] * pxy);
                const R j1 = j0 - kd[2] * (DS[2][1] * pxy);
                const int o = w0 + b * SY + a;
                lds_add(&sJz[o], j0);
                lds_add(&sJz[o + SZ], j1);
            }
    }
}

// A particle that stays in its cell (x1 in [0,1) on every axis): the form
// factors live on the cell's two nodes per axis, S0 = (1-x0, x0) and
// DS = (-dx, dx), and the window's nonzero entries reduce to
//   J_x(i+1/2, j+b) = kd_x dx (S0y + DSy/2)[b]  (the y average over the move)
// and likewise for y (and z); in 2D J_z(i+a, j+b) = kzv (S0x[a] ry[b] + DSx[a] qy[b]).
template <typename R, typename A, int D, int NJ>
__device__ __forceinline__ void deposit_cell(A *sJx, A *sJy, A *sJz, const int (&lc)[3], const R (&x0)[3],
                                             const R (&x1)[3], const R (&kd)[3], R kzv)
{
    constexpr int SY = NJ, SZ = NJ * NJ;
    R dd[3], m[3], s0[3][2], ds[3][2], h[3][2], q[3][2];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        dd[a] = x1[a] - x0[a];
        m[a] = x0[a] + R(0.5) * dd[a];
        s0[a][0] = R(1) - x0[a];
        s0[a][1] = x0[a];
        ds[a][0] = -dd[a];
        ds[a][1] = dd[a];
        h[a][0] = R(1) - m[a];                                   // S0 + DS/2
        h[a][1] = m[a];
        q[a][0] = R(0.5) * s0[a][0] - R(1.0 / 3.0) * dd[a];     // S0/2 + DS/3
        q[a][1] = R(0.5) * s0[a][1] + R(1.0 / 3.0) * dd[a];
    }
    int o = lc[0] + lc[1] * SY;
    if constexpr (D == 3) o += lc[2] * SZ;
    if constexpr (D == 2) {
        const R jx = kd[0] * dd[0], jy = kd[1] * dd[1];
        atomicAdd(&sJx[o], A(jx * h[1][0]));
        atomicAdd(&sJx[o + SY], A(jx * h[1][1]));
        atomicAdd(&sJy[o], A(jy * h[0][0]));
        atomicAdd(&sJy[o + 1], A(jy * h[0][1]));
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                atomicAdd(&sJz[o + b * SY + a], A(kzv * (s0[0][a] * h[1][b] + ds[0][a] * q[1][b])));
    } else {
        auto P = [&](int p, int r, int i, int l) { return s0[p][i] * h[r][l] + ds[p][i] * q[r][l]; };
        const R jx = kd[0] * dd[0], jy = kd[1] * dd[1], jz = kd[2] * dd[2];
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                atomicAdd(&sJx[o + c * SZ + b * SY], A(jx * P(1, 2, b, c)));
                atomicAdd(&sJy[o + c * SZ + b], A(jy * P(0, 2, b, c)));
                atomicAdd(&sJz[o + c * SY + b], A(jz * P(0, 1, b, c)));
            }
    }
}

// A 3D move that crosses exactly one cell face, along axis w (per lane): on
// the two other axes u < v the form factors live on the cell's two nodes (as
// in deposit_cell); along w they span three nodes starting at nb, the cell's
// lower node for an upward crossing and the node below it for a downward one.
// Of the window's 54 entries only 20 can be nonzero: J_w on 2 edges x 2 x 2
// nodes, J_u and J_v on 1 edge x 2 x 3 nodes.  sJ holds the three components
// NJ^3 apart.
template <typename R, typename A, int NJ>
__device__ __forceinline__ void deposit_face(A *sJ, const int (&lc)[3], const R (&x0)[3], const R (&x1)[3],
                                             const R (&kd)[3])
{
    constexpr int ST[3] = {1, NJ, NJ * NJ};
    constexpr int NJ_D = NJ * NJ * NJ;
    auto off = [](R x) { return x < R(0) || x >= R(1); };
    const int w = off(x1[0]) ? 0 : off(x1[1]) ? 1 : 2;
    const int u = w == 0 ? 1 : 0, v = w == 2 ? 1 : 2;
    auto pick = [](const R (&a)[3], int i) { return i == 0 ? a[0] : i == 1 ? a[1] : a[2]; };
    const R xu0 = pick(x0, u), xv0 = pick(x0, v), xw0 = pick(x0, w);
    const R du = pick(x1, u) - xu0, dv = pick(x1, v) - xv0, xw1 = pick(x1, w);
    const int su = u == 0 ? ST[0] : ST[1], sv = v == 1 ? ST[1] : ST[2];
    const int sw = w == 0 ? ST[0] : w == 1 ? ST[1] : ST[2];
    // two-node factors on u and v: S0, DS = (-d, d), h = S0 + DS/2, q = S0/2 + DS/3
    const R s0u[2] = {R(1) - xu0, xu0}, s0v[2] = {R(1) - xv0, xv0};
    const R dsu[2] = {-du, du}, dsv[2] = {-dv, dv};
    const R hv[2] = {R(1) - (xv0 + R(0.5) * dv), xv0 + R(0.5) * dv};
    const R qv[2] = {R(0.5) * s0v[0] - R(1.0 / 3.0) * dv, R(0.5) * s0v[1] + R(1.0 / 3.0) * dv};
    // three-node factors on w
    const bool up = xw1 >= R(1);
    R S0w[3], DSw[3];
    if (up) {
        S0w[0] = R(1) - xw0; S0w[1] = xw0; S0w[2] = R(0);
        DSw[0] = -S0w[0]; DSw[1] = (R(2) - xw1) - xw0; DSw[2] = xw1 - R(1);
    } else {
        S0w[0] = R(0); S0w[1] = R(1) - xw0; S0w[2] = xw0;
        DSw[0] = -xw1; DSw[1] = (R(1) + xw1) - S0w[1]; DSw[2] = -xw0;
    }
    R hw[3], qw[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        hw[m] = S0w[m] + R(0.5) * DSw[m];
        qw[m] = R(0.5) * S0w[m] + R(1.0 / 3.0) * DSw[m];
    }
    const R kw = w == 0 ? kd[0] : w == 1 ? kd[1] : kd[2];
    const R ju = (u == 0 ? kd[0] : kd[1]) * du, jv = (v == 1 ? kd[1] : kd[2]) * dv;
    const int o = lc[0] + lc[1] * ST[1] + lc[2] * ST[2] - (up ? 0 : sw);
    A *Ju = sJ + u * NJ_D, *Jv = sJ + v * NJ_D, *Jw = sJ + w * NJ_D;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const R p = s0u[i] * hv[j] + dsu[i] * qv[j];
            const R j0 = -kw * (DSw[0] * p);
            const R j1 = j0 - kw * (DSw[1] * p);
            const int a = o + i * su + j * sv;
            atomicAdd(&Jw[a], A(j0));
            atomicAdd(&Jw[a + sw], A(j1));
        }
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            atomicAdd(&Ju[o + j * sv + m * sw], A(ju * (s0v[j] * hw[m] + dsv[j] * qw[m])));
            atomicAdd(&Jv[o + j * su + m * sw], A(jv * (s0u[j] * hw[m] + dsu[j] * qw[m])));
        }
}

// Crossing particles wait in per-wave LDS stacks and are deposited 64 at a
// time, with every lane busy: in 3D, single-face crossers (stack A, from the
// bottom) through deposit_face and the others (stack B, from the top) through
// deposit_window; in 2D all of them through deposit_window (stack B).  Each
// stack is drained when it holds 64 entries, so before an append each holds at
// most 63 and after it both together at most 190.
template <int D> constexpr int kQueue = D == 3 ? 192 : 128;
constexpr int kOrderBuckets = 64;
constexpr int kAdvanceThreads = 1024;    // workgroup size of the end-of-step kernel (one workgroup per run)
constexpr int kXcds = kBatchXcds;        // accelerator dies (XCDs), each with its own L2

// Movers staged per wave in mixed mode before they are written, grouped by
// destination tile (FP64 writes each mover at once: 1 entry).
template <typename R, int D>
constexpr int kMoverStage = sizeof(R) == 4 ? (D == 3 ? 24 : 64) : 1;

// KP: pointer to the run's parameters -- the kernel argument, or (batched
// runs) a constant-address-space pointer, which lets the parameter loads be
// scalar loads (the parameter blocks are never written by a kernel).
// CB: the kernel carries the Coulomb scattering branch (runs with a species on
// that model); without it the branch and its registers are compiled out.
// SH: launch shape (kBlock threads, kBatch particles in flight per lane).
// BS: the field stage issues all of a thread's loads before its LDS writes
// (one workgroup per tile); the persistent batched kernel keeps the plain
// loop, whose registers do not add to those it holds across work items.
template <typename R, typename A, int D, int T, bool CB, int SH, bool BS, typename KP>
__device__ __forceinline__ void particle_body(KP kp, int bid, int nb)
{
    constexpr int kBlock = kShapeBlock[SH];
    constexpr int kBatch = kShapeInflight[SH];
    constexpr int NF = T + 2;
    constexpr int NJ = T + 3;
    constexpr int NF_D = D == 3 ? NF * NF * NF : NF * NF;
    constexpr int NJ_D = D == 3 ? NJ * NJ * NJ : NJ * NJ;
    constexpr int SJ_Y = NJ, SJ_Z = NJ * NJ;        // LDS strides of the current tile
    constexpr int TS = T == 8 ? 3 : T == 16 ? 4 : 5; // log2 T: bit width of an in-tile cell coordinate
    __shared__ R sF[6 * NF_D];
    __shared__ A sJ[3 * NJ_D];
    constexpr int QC = kQueue<D>;
    constexpr int QV = D == 3 ? 2 * D : 2 * D + 1;       // x0, x1 (and q w v_z in 2D)
    __shared__ int sQc[kBlock / 64][QC];                 // crossing-particle stacks per wave
    __shared__ R sQv[kBlock / 64][QV][QC];
    // movers staged per wave (mixed mode): destination tile and stored words
    constexpr int MS = kMoverStage<R, D>;
    constexpr int MW = D + 5;                            // cell, offsets, momenta, id
    __shared__ int sMt[kBlock / 64][MS];
    __shared__ uint32_t sMw[kBlock / 64][MW][MS];
    __shared__ uint32_t s_front[kMaxSpecies];           // stayers written to the front of each species' bin
    __shared__ double sred[kBlock / 64][kTileDiag];

    const int tile = bid;
    (void)nb;
    const int ntx = kp->g.nt[0], nty = kp->g.nt[1];
    const int n[3] = {kp->g.n[0], kp->g.n[1], kp->g.n[2]};
    const int ntiles = kp->g.ntiles;
    int t0[3];
    t0[0] = (tile % ntx) * T;
    t0[1] = ((tile / ntx) % nty) * T;
    t0[2] = (tile / (ntx * nty)) * T;
    const int64_t step = uniform_step(kp);
    const int src = uniform_par(kp), dst = src ^ 1;
    const bool diag = diag_step(kp, step);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tsh = kp->g.tshift[0];
    uint32_t csh[3], cmask[3];
    for (int a = 0; a < 3; ++a) {
        csh[a] = (uint32_t)kp->g.csh[a];
        cmask[a] = kp->g.cmask[a];
    }
    const uint32_t seed0 = (uint32_t)kp->seed, seed1 = (uint32_t)(kp->seed >> 32);
    const uint32_t runid = kp->run;
    // key of the scatter-decision draw (Philox2x32-10 on (id, step))
    const uint32_t ckey = seed0 ^ (seed1 * 0x9E3779B9u) ^ (runid * 0x85EBCA6Bu);
    DevState *state = kp->state;

    {
        // Field stage: every load of the thread is issued before the first
        // LDS write, so the stage costs one memory round trip, not one per
        // value (6 (T+2)^D values over the workgroup: 24 per thread for 8^3
        // tiles).
        const GLB R *F = gbl((const R *)kp->F);
        const int64_t plane = kp->g.cells;
        constexpr int NS = 6 * NF_D;
        auto src_of = [&](int i) {
            const int c = i / NF_D, r = i - c * NF_D;
            const int lx = r % NF, ly = (r / NF) % NF, lz = D == 3 ? r / (NF * NF) : 0;
            int gx = t0[0] - 1 + lx, gy = t0[1] - 1 + ly, gz = D == 3 ? t0[2] - 1 + lz : 0;
            gx += gx < 0 ? n[0] : 0;
            gx -= gx >= n[0] ? n[0] : 0;
            gy += gy < 0 ? n[1] : 0;
            gy -= gy >= n[1] ? n[1] : 0;
            if constexpr (D == 3) {
                gz += gz < 0 ? n[2] : 0;
                gz -= gz >= n[2] ? n[2] : 0;
            }
            return c * plane + ((int64_t)gz * n[1] + gy) * n[0] + gx;
        };
        if constexpr (BS) {
            constexpr int NIT = (NS + kBlock - 1) / kBlock;
            R fv[NIT];
#pragma unroll
            for (int k = 0; k < NIT; ++k) {
                const int i = threadIdx.x + k * kBlock;
                fv[k] = R(0);
                if ((k + 1) * kBlock <= NS || i < NS) fv[k] = F[src_of(i)];
            }
            for (int i = threadIdx.x; i < 3 * NJ_D; i += kBlock) sJ[i] = A(0);
#pragma unroll
            for (int k = 0; k < NIT; ++k) {
                const int i = threadIdx.x + k * kBlock;
                if ((k + 1) * kBlock <= NS || i < NS) sF[i] = fv[k];
            }
        } else {
            for (int i = threadIdx.x; i < NS; i += kBlock) sF[i] = F[src_of(i)];
            for (int i = threadIdx.x; i < 3 * NJ_D; i += kBlock) sJ[i] = A(0);
        }
    }
    if (threadIdx.x < kMaxSpecies) s_front[threadIdx.x] = 0;
    __syncthreads();

    const R *sEx = sF, *sEy = sF + NF_D, *sEz = sF + 2 * NF_D;
    const R *sBx = sF + 3 * NF_D, *sBy = sF + 4 * NF_D, *sBz = sF + 5 * NF_D;
    A *sJx = sJ, *sJy = sJ + NJ_D, *sJz = sJ + 2 * NJ_D;

    R dtd[3];
    for (int a = 0; a < 3; ++a) dtd[a] = R(kp->g.dt / kp->g.d[a]);

    uint32_t load = 0;                                      // particles of the tile, all species
    for (int s = 0; s < kp->nspecies; ++s) {
        const auto &S = kp->sp[s];
        const int32_t bstart = S.start[tile], bcap = S.cap[tile];
        const uint32_t nf = S.cnt_front[src * ntiles + tile];
        const uint32_t nb = S.cnt_back[src * ntiles + tile];
        const uint32_t total = nf + nb;
        load += total;
        const R qm = R(S.qmdt2);
        R kd[3];                                            // q w d_a/dt
        for (int a = 0; a < 3; ++a) kd[a] = R(S.qw * kp->g.d[a] / kp->g.dt);
        const R qw = R(S.qw);
        const double wgt = S.w;
        const bool collide = S.collide != 0;
        const bool coulomb = CB && S.coll_model == PIC_COLL_COULOMB;
        const R csig2 = R(S.coll_sig2);
        const bool track = S.track_id != 0;
        const uint32_t thr = S.coll_thr;
        const GLB uint16_t *__restrict__ icell = gbl(S.cell[src]);
        const GLB R *__restrict__ ipos[3] = {gbl((const R *)S.pos[src][0]), gbl((const R *)S.pos[src][1]),
                                             gbl((const R *)S.pos[src][2])};
        const GLB R *__restrict__ iu0 = gbl((const R *)S.u[src][0]);
        const GLB R *__restrict__ iu1 = gbl((const R *)S.u[src][1]);
        const GLB R *__restrict__ iu2 = gbl((const R *)S.u[src][2]);
        const GLB uint32_t *__restrict__ iid = gbl(S.id[src]);
        const GLB int32_t *__restrict__ tstart = gbl(S.start);
        const GLB int32_t *__restrict__ tcap = gbl(S.cap);
        const GLB uint32_t *__restrict__ cf_src = gbl(S.cnt_front + src * ntiles);
        const GLB uint32_t *__restrict__ cb_src = gbl(S.cnt_back + src * ntiles);
        GLB uint32_t *cb_dst = gbl(S.cnt_back + dst * ntiles);

        GLB uint16_t *__restrict__ ocell = gbl(S.cell[dst]);
        GLB R *__restrict__ opos_a[3] = {gbl((R *)S.pos[dst][0]), gbl((R *)S.pos[dst][1]), gbl((R *)S.pos[dst][2])};
        GLB R *__restrict__ ou0 = gbl((R *)S.u[dst][0]);
        GLB R *__restrict__ ou1 = gbl((R *)S.u[dst][1]);
        GLB R *__restrict__ ou2 = gbl((R *)S.u[dst][2]);
        GLB uint32_t *__restrict__ oid = gbl(S.id[dst]);

        // Raw fields of one particle as stored.  Each lane holds the next
        // kBatch particles (k, k+256, ...): before processing the oldest it
        // issues the loads of the one kBatch steps ahead, so every lane keeps
        // kBatch particles' loads in flight while it computes.
        struct Raw {
            uint32_t c;
            R p[D];
            R u[3];
            uint32_t id;
        };
        auto fetch = [&](uint32_t k, Raw &r) {
            const uint32_t slot = k < nf ? (uint32_t)bstart + k : (uint32_t)(bstart + bcap) - nb + (k - nf);
            if constexpr (sizeof(R) == 4) r.c = (uint32_t)ld(icell, slot);
#pragma unroll
            for (int a = 0; a < D; ++a) r.p[a] = ld(ipos[a], slot);
            r.u[0] = ld(iu0, slot);
            r.u[1] = ld(iu1, slot);
            r.u[2] = ld(iu2, slot);
            r.id = track ? ld(iid, slot) : 0u;
        };
        double acc[kTileDiag] = {0, 0, 0, 0, 0, 0};
        uint32_t nqa = 0, nqb = 0;                           // wave-uniform stack heights
        auto drain = [&](uint32_t e, bool face) {
            const int pk = sQc[wave][e];
            const int qlc[3] = {pk & 0xff, (pk >> 8) & 0xff, (pk >> 16) & 0xff};
            R qx0[3] = {R(0), R(0), R(0)}, qx1[3] = {R(0), R(0), R(0)};
#pragma unroll
            for (int a = 0; a < D; ++a) {
                qx0[a] = sQv[wave][a][e];
                qx1[a] = sQv[wave][D + a][e];
            }
            if constexpr (D == 3) {
                if (face)
                    deposit_face<R, A, NJ>(sJ, qlc, qx0, qx1, kd);
                else
                    deposit_window<R, A, D, NJ>(sJx, sJy, sJz, qlc, qx0, qx1, kd, R(0));
            } else {
                deposit_window<R, A, D, NJ>(sJx, sJy, sJz, qlc, qx0, qx1, kd, sQv[wave][2 * D][e]);
            }
        };
        // A particle that leaves the tile (mover) is written at the back of
        // its new tile's bin, in a slot reserved with a global atomic above
        // that tile's start-of-step count.  In mixed mode the movers of a
        // wave are first staged in LDS; a flush groups them by destination,
        // takes one atomic per destination and writes each destination's
        // movers to consecutive slots, so their stores are contiguous runs
        // rather than scattered words, and the atomic round trip is paid
        // once per flush.  FP64 writes each mover at once (the stage would
        // cost occupancy).
        auto emit_mover = [&](uint32_t slot, int32_t room, int32_t top, const Raw &m) {
            if ((int64_t)slot < (int64_t)room) {
                const uint32_t o = (uint32_t)top - slot;
                if constexpr (sizeof(R) == 4) {
                    uint32_t lc = 0;                             // the cell within the new tile
#pragma unroll
                    for (int a = 0; a < D; ++a) lc |= (((m.c >> csh[a]) & cmask[a]) & (uint32_t)(T - 1)) << (a * TS);
                    st(ocell, o, (uint16_t)lc);
                }
#pragma unroll
                for (int a = 0; a < D; ++a) st(opos_a[a], o, m.p[a]);
                st(ou0, o, m.u[0]);
                st(ou1, o, m.u[1]);
                st(ou2, o, m.u[2]);
                if (track) st(oid, o, m.id);
            } else {
                // no room left in the new tile's bin: overflow list (set 2),
                // re-laid out at the end of the step
                const uint32_t oi = atomicAdd(&state->ovf_count[s], 1u);
                state->rebin = 1;
                if (oi < S.ovf_cap) {
                    if constexpr (sizeof(R) == 4) gbl(S.ovf_cell)[oi] = m.c;
                    for (int a = 0; a < D; ++a) gbl((R *)S.pos[2][a])[oi] = m.p[a];
                    gbl((R *)S.u[2][0])[oi] = m.u[0];
                    gbl((R *)S.u[2][1])[oi] = m.u[1];
                    gbl((R *)S.u[2][2])[oi] = m.u[2];
                    if (track) gbl(S.id[2])[oi] = m.id;
                } else {
                    atomicOr(&state->fatal, 1);
                }
            }
        };
        // reserve one slot in tile t and write m there (unstaged path)
        auto emit_now = [&](int t, const Raw &m) {
            const uint32_t slot = __hip_atomic_fetch_add(cb_dst + t, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            emit_mover(slot, tcap[t] - (int32_t)cf_src[t] - (int32_t)cb_src[t], tstart[t] + tcap[t] - 1, m);
        };
        uint32_t mv_n = 0;                                   // staged movers of this wave (uniform)
        auto flush_movers = [&]() {
            __builtin_amdgcn_wave_barrier();
            const bool valid = (uint32_t)lane < mv_n;
            const int td = valid ? sMt[wave][lane] : -1;
            uint64_t rem = __ballot(valid);
            int leader = 0;
            uint32_t rank = 0, lead_cnt = 0;
            while (rem) {                                    // one pass per distinct destination
                const int l = __ffsll((unsigned long long)rem) - 1;
                const int tl = __builtin_amdgcn_readlane(td, l);
                const bool mine = valid && td == tl;
                const uint64_t same = __ballot(mine);
                if (mine) {
                    leader = l;
                    rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(same >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)same, 0u));
                }
                if (lane == l) lead_cnt = (uint32_t)__popcll(same);
                rem &= ~same;
            }
            uint32_t b0 = 0;
            int32_t room = 0, top = 0;
            if (valid && lane == leader) {
                b0 = __hip_atomic_fetch_add(cb_dst + td, lead_cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                room = tcap[td] - (int32_t)cf_src[td] - (int32_t)cb_src[td];
                top = tstart[td] + tcap[td] - 1;
            }
            b0 = (uint32_t)__shfl((int)b0, leader, 64);
            room = __shfl(room, leader, 64);
            top = __shfl(top, leader, 64);
            if (valid) {
                Raw m;
                m.c = sMw[wave][0][lane];
#pragma unroll
                for (int a = 0; a < D; ++a) m.p[a] = __uint_as_float(sMw[wave][1 + a][lane]);
#pragma unroll
                for (int c = 0; c < 3; ++c) m.u[c] = __uint_as_float(sMw[wave][1 + D + c][lane]);
                m.id = sMw[wave][4 + D][lane];
                emit_mover(b0 + rank, room, top, m);
            }
            __builtin_amdgcn_wave_barrier();
            mv_n = 0;
        };
        Raw q[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t kk = u * kBlock + threadIdx.x;
            if (kk < total) fetch(kk, q[u]);
        }
#pragma unroll 1
        for (uint32_t base = 0; base < total; base += kBlock) {
            {
            const uint32_t k = base + threadIdx.x;
            const bool active = k < total;
            const Raw cur = q[0];
#pragma unroll
            for (int v = 0; v + 1 < kBatch; ++v) q[v] = q[v + 1];
            {
                const uint32_t kn = k + kBatch * kBlock;
                if (kn < total) fetch(kn, q[kBatch - 1]);
            }
            int ic1[D];
            R off1[D];
            int t1 = -1;
            R ux = R(0), uy = R(0), uz = R(0);
            uint32_t pid = 0;
            for (int a = 0; a < D; ++a) { ic1[a] = 0; off1[a] = R(0); }
            bool cross = false;                               // leaves its cell this step
            int ncross = 0;                                   // faces crossed
            int q_lc = 0;
            R q_x0[D], q_x1[D], q_kz = R(0);
            if (active) {
                int ic[3] = {0, 0, 0};
                R off[3] = {R(0), R(0), R(0)};
                if constexpr (sizeof(R) == 4) {
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        ic[a] = t0[a] + (int)((cur.c >> (a * TS)) & (uint32_t)(T - 1));
                        off[a] = cur.p[a];
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        const double X = cur.p[a];
                        ic[a] = (int)floor(X);
                        off[a] = X - ic[a];
                    }
                }
                ux = cur.u[0];
                uy = cur.u[1];
                uz = cur.u[2];
                pid = cur.id;
                const R uox = ux, uoy = uy, uoz = uz;

                // ---- gather: linear weights at each component's stagger
                int lc[3], lh[3];
                R a0[3], a1[3], b0[3], b1[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    lc[a] = ic[a] - t0[a] + 1;
                    const int h = off[a] < R(0.5) ? 1 : 0;
                    lh[a] = lc[a] - h;
                    a1[a] = off[a];                             // integer stagger
                    a0[a] = R(1) - off[a];
                    b1[a] = off[a] - R(0.5) + R(h);             // half stagger
                    b0[a] = R(1) - b1[a];
                }
                const R Ex = interp<R, D, NF>(sEx, lh[0], lc[1], lc[2], b0[0], b1[0], a0[1], a1[1], a0[2], a1[2]);
                const R Ey = interp<R, D, NF>(sEy, lc[0], lh[1], lc[2], a0[0], a1[0], b0[1], b1[1], a0[2], a1[2]);
                const R Ez = interp<R, D, NF>(sEz, lc[0], lc[1], lh[2], a0[0], a1[0], a0[1], a1[1], b0[2], b1[2]);
                const R Bx = interp<R, D, NF>(sBx, lc[0], lh[1], lh[2], a0[0], a1[0], b0[1], b1[1], b0[2], b1[2]);
                const R By = interp<R, D, NF>(sBy, lh[0], lc[1], lh[2], b0[0], b1[0], a0[1], a1[1], b0[2], b1[2]);
                const R Bz = interp<R, D, NF>(sBz, lh[0], lh[1], lc[2], b0[0], b1[0], b0[1], b1[1], a0[2], a1[2]);

                // ---- relativistic Boris push
                const R umx = ux + qm * Ex, umy = uy + qm * Ey, umz = uz + qm * Ez;
                const R ig = Arith<R>::rsq(R(1) + umx * umx + umy * umy + umz * umz);
                const R tx = qm * Bx * ig, ty = qm * By * ig, tz = qm * Bz * ig;
                const R sf = R(2) * Arith<R>::rcp(R(1) + tx * tx + ty * ty + tz * tz);
                const R sx = tx * sf, sy = ty * sf, sz = tz * sf;
                const R wx = umx + (umy * tz - umz * ty);
                const R wy = umy + (umz * tx - umx * tz);
                const R wz = umz + (umx * ty - umy * tx);
                ux = umx + (wy * sz - wz * sy) + qm * Ex;
                uy = umy + (wz * sx - wx * sz) + qm * Ey;
                uz = umz + (wx * sy - wy * sx) + qm * Ez;
                const R ig1 = Arith<R>::rsq(R(1) + ux * ux + uy * uy + uz * uz);
                const R v[3] = {ux * ig1, uy * ig1, uz * ig1};

                // ---- move in cell units, relative to the particle's cell
                R x1[3] = {R(0), R(0), R(0)};
                int kk[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    x1[a] = off[a] + v[a] * dtd[a];
                    kk[a] = (int)floor(x1[a]);
                    ncross += kk[a] != 0 ? 1 : 0;
                }
                cross = ncross != 0;

                // ---- Esirkepov deposit: particles that stay in their cell now,
                // the others through the per-wave queue below
                const R kzv = qw * v[2];
                if (!cross) {
                    deposit_cell<R, A, D, NJ>(sJx, sJy, sJz, lc, off, x1, kd, kzv);
                } else {
                    q_lc = lc[0] | (lc[1] << 8) | (D == 3 ? lc[2] << 16 : 0);
#pragma unroll
                    for (int a = 0; a < D; ++a) {
                        q_x0[a] = off[a];
                        q_x1[a] = x1[a];
                    }
                    q_kz = kzv;
                }

                if (diag) {
                    const double go = sqrt(1.0 + (double)uox * uox + (double)uoy * uoy + (double)uoz * uoz);
                    const double gn = sqrt(1.0 + (double)ux * ux + (double)uy * uy + (double)uz * uz);
                    acc[0] += wgt * (0.5 * (go + gn) - 1.0);
                    acc[1] += wgt * 0.5 * ((double)uox + (double)ux);
                    acc[2] += wgt * 0.5 * ((double)uoy + (double)uy);
                    acc[3] += wgt * 0.5 * ((double)uoz + (double)uz);
                    acc[4] += 1.0;
                }

                // ---- scattering off the ions (collisional species)
                if (collide && coulomb) {
                    // Coulomb small-angle scattering off the ions: turn by theta,
                    // tan(theta/2) ~ N(0, coll_sig2 / v^3), uniform azimuth,
                    // Takizuka-Abe rotation of u (|u| kept)
                    const R u2 = ux * ux + uy * uy + uz * uz;
                    if (u2 > R(0)) {
                        const uint4 r = philox10(make_uint4(pid, (uint32_t)step, kPurposeCoulomb, runid), seed0, seed1);
                        const R v2 = u2 / (R(1) + u2);
                        const R var = csig2 / (v2 * sqrt(v2));
                        const R delta = sqrt(R(-2) * var * Arith<R>::ln(R(u01d(r.x)))) *
                                        Arith<R>::cs(R(6.283185307179586) * R(u01d(r.y)));
                        const R d2 = delta * delta;
                        const R inv = R(1) / (R(1) + d2);
                        const R omc = R(2) * d2 * inv;                  // 1 - cos(theta)
                        const R st = R(2) * delta * inv;                // sin(theta)
                        R sp, cp;
                        Arith<R>::sc(R(6.283185307179586) * R(u01d(r.z)), &sp, &cp);
                        const R up2 = ux * ux + uy * uy;
                        if (up2 > R(0)) {
                            const R iup = Arith<R>::rsq(up2);
                            const R a = st * cp * iup, b = st * sp * sqrt(u2) * iup;
                            const R dz = -up2 * iup * st * cp - uz * omc;
                            const R dx = ux * uz * a - uy * b - ux * omc;
                            uy += uy * uz * a + ux * b - uy * omc;
                            ux += dx;
                            uz += dz;
                        } else {
                            const R U = sqrt(u2);
                            ux += U * st * cp;
                            uy += U * st * sp;
                            uz -= uz * omc;
                        }
                        if (diag) acc[5] += 1.0;
                    }
                } else if (collide) {
                    if (philox2x32_10_w0(pid, (uint32_t)step, ckey) < thr) {
                        const uint4 r = philox10(make_uint4(pid, (uint32_t)step, kPurposeCollide, runid), seed0, seed1);
                        const R um = sqrt(ux * ux + uy * uy + uz * uz);
                        const R ct = R(1) - R(2) * R(u01d(r.y));
                        const R st = sqrt(fmax(R(0), R(1) - ct * ct));
                        R sn, cs;
                        Arith<R>::sc(R(6.283185307179586) * R(u01d(r.z)), &sn, &cs);
                        ux = um * st * cs;
                        uy = um * st * sn;
                        uz = um * ct;
                        if (diag) acc[5] += 1.0;
                    }
                }

                // ---- new cell and offset, destination tile
                bool bad = false;
                t1 = 0;
#pragma unroll
                for (int a = D - 1; a >= 0; --a) {
                    int k1 = kk[a];
                    R o1 = x1[a] - R(k1);
                    if (o1 >= R(1)) { o1 = R(0); k1 += 1; }
                    int i1 = ic[a] + k1;
                    i1 += i1 < 0 ? n[a] : 0;
                    i1 -= i1 >= n[a] ? n[a] : 0;
                    if ((unsigned)i1 >= (unsigned)n[a]) { bad = true; i1 = 0; }
                    ic1[a] = i1;
                    off1[a] = o1;
                    t1 = t1 * kp->g.nt[a] + (i1 >> tsh);
                }
                if (bad) atomicOr(&state->fatal, 2);
            }

            // ---- crossing particles: push onto the wave's stacks, drain a
            // stack when it holds a full wave of entries
            {
                const bool fa = D == 3 && cross && ncross == 1;
                const bool fb = cross && !fa;
                const uint64_t am = __ballot(fa), bm = __ballot(fb);
                if (am | bm) {
                    if (cross) {
                        const uint64_t m = fa ? am : bm;
                        const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        const uint32_t e = fa ? nqa + r : (uint32_t)QC - 1u - (nqb + r);
                        sQc[wave][e] = q_lc;
#pragma unroll
                        for (int a = 0; a < D; ++a) {
                            sQv[wave][a][e] = q_x0[a];
                            sQv[wave][D + a][e] = q_x1[a];
                        }
                        if constexpr (D == 2) sQv[wave][2 * D][e] = q_kz;
                    }
                    nqa += (uint32_t)__popcll(am);
                    nqb += (uint32_t)__popcll(bm);
                    if (nqa >= 64) {
                        nqa -= 64;
                        drain(nqa + lane, true);
                    }
                    if (nqb >= 64) {
                        nqb -= 64;
                        drain((uint32_t)QC - 1u - (nqb + lane), false);
                    }
                }
            }

            // ---- binning
            const bool stay = active && t1 == tile;
            const uint64_t smask = __ballot(stay);
            uint32_t opos = 0;
            bool wr = false;
            if (smask) {
                const int leader = __ffsll((unsigned long long)smask) - 1;
                uint32_t bfront = 0;
                if (lane == leader) bfront = atomicAdd(&s_front[s], (uint32_t)__popcll(smask));
                bfront = __builtin_amdgcn_readlane(bfront, leader);
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(smask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)smask, 0u));
                if (stay) {
                    opos = (uint32_t)bstart + bfront + rank;
                    wr = true;
                }
            }
            uint32_t cpack = 0, lpack = 0;             // global (movers) and in-tile (stayers) cell
            if constexpr (sizeof(R) == 4) {
#pragma unroll
                for (int a = 0; a < D; ++a) {
                    cpack |= (uint32_t)ic1[a] << csh[a];
                    lpack |= ((uint32_t)ic1[a] & (uint32_t)(T - 1)) << (a * TS);
                }
            }
            {
                const bool mover = active && !stay;
                if constexpr (MS > 1) {
                    const uint64_t mm = __ballot(mover);
                    if (mm) {
                        const uint32_t inc = (uint32_t)__popcll(mm);
                        if (mv_n + inc > (uint32_t)MS) flush_movers();
                        if (inc <= (uint32_t)MS) {
                            if (mover) {
                                const uint32_t e = mv_n + __builtin_amdgcn_mbcnt_hi(
                                                              (uint32_t)(mm >> 32),
                                                              __builtin_amdgcn_mbcnt_lo((uint32_t)mm, 0u));
                                sMt[wave][e] = t1;
                                sMw[wave][0][e] = cpack;
#pragma unroll
                                for (int a = 0; a < D; ++a) sMw[wave][1 + a][e] = __float_as_uint((float)off1[a]);
                                sMw[wave][1 + D][e] = __float_as_uint((float)ux);
                                sMw[wave][2 + D][e] = __float_as_uint((float)uy);
                                sMw[wave][3 + D][e] = __float_as_uint((float)uz);
                                sMw[wave][4 + D][e] = pid;
                            }
                            mv_n += inc;
                        } else if (mover) {
                            // more movers than the stage holds (3D): unstaged
                            Raw m;
                            m.c = cpack;
#pragma unroll
                            for (int a = 0; a < D; ++a) m.p[a] = off1[a];
                            m.u[0] = ux;
                            m.u[1] = uy;
                            m.u[2] = uz;
                            m.id = pid;
                            emit_now(t1, m);
                        }
                    }
                } else if (mover) {
                    Raw m;
                    m.c = cpack;
#pragma unroll
                    for (int a = 0; a < D; ++a) m.p[a] = R((double)ic1[a] + off1[a]);
                    m.u[0] = ux;
                    m.u[1] = uy;
                    m.u[2] = uz;
                    m.id = pid;
                    emit_now(t1, m);
                }
            }
            if (wr) {
                if constexpr (sizeof(R) == 4) {
                    st(ocell, opos, (uint16_t)lpack);
#pragma unroll
                    for (int a = 0; a < D; ++a) st(opos_a[a], opos, off1[a]);
                } else {
#pragma unroll
                    for (int a = 0; a < D; ++a) st(opos_a[a], opos, R((double)ic1[a] + off1[a]));
                }
                st(ou0, opos, ux);
                st(ou1, opos, uy);
                st(ou2, opos, uz);
                if (track) st(oid, opos, pid);
            }
            }
        }
        if constexpr (MS > 1) {
            if (mv_n) flush_movers();
        }
        if ((uint32_t)lane < nqa) drain(lane, true);
        if ((uint32_t)lane < nqb) drain((uint32_t)QC - 1u - lane, false);
        // no barrier between species (each has its own front counter, the
        // stacks and stages are per wave): a wave goes on to the next
        // species while the others finish; diagnostic steps sum per species
        if (diag) {
            block_sum<kTileDiag>(acc, sred);
            if (threadIdx.x == 0)
                for (int v = 0; v < kTileDiag; ++v)
                    kp->tile_diag[((int64_t)tile * kp->nspecies + s) * kTileDiag + v] = acc[v];
        }
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)kp->nspecies) kp->sp[threadIdx.x].cnt_front[dst * ntiles + tile] = s_front[threadIdx.x];
    if (threadIdx.x == 0)
        kp->tile_bucket[tile] = (uint8_t)min(kOrderBuckets - 1, (int)((double)load * kp->order_scale + 0.5));
    GLB R *Jt = gbl((R *)kp->Jtile) + (int64_t)tile * 3 * NJ_D;
    for (int i = threadIdx.x; i < 3 * NJ_D; i += kBlock) Jt[i] = R(sJ[i]);
}

// ---------------------------------------------------------------------------
// Store re-layout after an overflow of some tile's incoming-mover reserve.
// Data of the step sits in set dst (bins) and set 2 (overflow list); it is
// rewritten into set src with capacities count + a uniform reserve, and the
// parity is kept so that the next step reads set src.
__device__ __forceinline__ void rebin_count_body(const KParams *__restrict__ kp, int bid, int nb)
{
    const DevState *st = kp->state;
    if (!st->rebin) return;
    const int ntiles = kp->g.ntiles;
    const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
    if (i >= (int64_t)kp->nspecies * ntiles) return;
    const int s = (int)(i / ntiles), t = (int)(i % ntiles);
    const SpeciesDev &S = kp->sp[s];
    const int src = st->par, dst = src ^ 1;
    const int64_t room = (int64_t)S.cap[t] - S.cnt_front[src * ntiles + t] - S.cnt_back[src * ntiles + t];
    const int64_t vb = min((int64_t)S.cnt_back[dst * ntiles + t], room);
    const int32_t c = (int32_t)(S.cnt_front[dst * ntiles + t] + vb);
    kp->rb_count[i] = c;
    kp->rb_fill[i] = c;
}

template <typename R>
__device__ __forceinline__ int tile_of(const KParams *kp, const SpeciesDev &S, int set, int64_t p)
{
    int t = 0;
    for (int a = kp->g.ndim - 1; a >= 0; --a) {
        int i;
        (void)set;   // the overflow list (set 2): global cells
        if constexpr (sizeof(R) == 4) i = (int)((S.ovf_cell[p] >> kp->g.csh[a]) & kp->g.cmask[a]);
        else i = (int)floor(((const double *)S.pos[2][a])[p]);
        i = min(max(i, 0), kp->g.n[a] - 1);
        t = t * kp->g.nt[a] + (i >> kp->g.tshift[a]);
    }
    return t;
}

// ---- Gauss's-law check (PIC_FLAG_GAUSS_RESIDUAL): at step 0 and on
// diagnostic steps, the CIC charge of the particles at the start of the
// step, one workgroup per tile into an LDS tile of (T+1)^D nodes (a tile's
// particles have their cells in the tile), written as the tile's partial;
// then per node: the partials' sum rho, div E of the fields at the start of
// the step, and the maxima of |div E - (rho - rho_0)| and |rho - rho_0|.
template <typename KP>
__device__ __forceinline__ bool gauss_step(KP kp, int64_t step)
{
    return (kp->flags & PIC_FLAG_GAUSS_RESIDUAL) && (step == 0 || diag_step(kp, step));
}

// CIC charge of the particles on the tile's nodes (per-tile partials).
// NEXT = false: the particles at the start of the step (x^n); NEXT = true:
// after the particle kernel and any re-layout (x^{n+1}), which sit in the
// other particle set, or, after a re-layout, back in the same one.
template <typename R, int D, int T, bool NEXT>
__global__ __launch_bounds__(256) void k_rho(const KParams *__restrict__ kp)
{
    constexpr int N1 = T + 1;
    constexpr int ND = D == 3 ? N1 * N1 * N1 : N1 * N1;
    __shared__ double srho[ND];
    const DevState *stp = kp->state;
    const int64_t step = stp->step;
    if (!gauss_step(kp, step)) return;
    if (NEXT && (stp->fatal & 4)) return;
    const int tile = blockIdx.x, ntiles = kp->g.ntiles;
    const int par = NEXT ? (stp->rebin ? stp->par : stp->par ^ 1) : stp->par;
    const int ntx = kp->g.nt[0], nty = kp->g.nt[1];
    const int t0[3] = {(tile % ntx) * T, ((tile / ntx) % nty) * T, (tile / (ntx * nty)) * T};
    for (int e = threadIdx.x; e < ND; e += blockDim.x) srho[e] = 0.0;
    __syncthreads();
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int64_t nf = S.cnt_front[par * ntiles + tile], nb = S.cnt_back[par * ntiles + tile];
        const int64_t b0 = S.start[tile], cap = S.cap[tile];
        const double qw = S.qw;
        for (int64_t k = threadIdx.x; k < nf + nb; k += blockDim.x) {
            const int64_t slot = k < nf ? b0 + k : b0 + cap - nb + (k - nf);
            int l[3] = {0, 0, 0};
            double o[3] = {0.0, 0.0, 0.0};
            bool inside = true;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                int ic;
                if constexpr (sizeof(R) == 4) {
                    ic = t0[a] + (int)(((uint32_t)S.cell[par][slot] >> (a * kp->g.tshift[0])) & (uint32_t)(T - 1));
                    o[a] = (double)((const float *)S.pos[par][a])[slot];
                } else {
                    const double X = ((const double *)S.pos[par][a])[slot];
                    ic = (int)floor(X);
                    o[a] = X - ic;
                }
                l[a] = ic - t0[a];
                inside = inside && l[a] >= 0 && l[a] < T;
            }
            if (!inside) {
                atomicOr(&kp->state->fatal, 8);
                continue;
            }
#pragma unroll
            for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
#pragma unroll
                for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                    for (int dx = 0; dx < 2; ++dx) {
                        double w = (dx ? o[0] : 1.0 - o[0]) * (dy ? o[1] : 1.0 - o[1]);
                        if (D == 3) w *= dz ? o[2] : 1.0 - o[2];
                        atomicAdd(&srho[((l[2] + dz) * N1 + l[1] + dy) * N1 + l[0] + dx], qw * w);
                    }
        }
    }
    __syncthreads();
    double *out = kp->rho_tile + (int64_t)tile * ND;
    for (int e = threadIdx.x; e < ND; e += blockDim.x) out[e] = srho[e];
}

// Charge on node o (grid indices idx) from the per-tile partials of k_rho:
// a node belongs to its own tile (local index i mod T) and, on a tile edge,
// to the tile below (local index T); the partials are summed in that order.
template <int D>
__device__ __forceinline__ double node_rho(const KParams *__restrict__ kp, const int (&idx)[3])
{
    const int T = kp->g.tile[0], N1 = T + 1;
    const int64_t ND = D == 3 ? (int64_t)N1 * N1 * N1 : (int64_t)N1 * N1;
    double rho = 0.0;
    for (int cz = 0; cz < (D == 3 ? 2 : 1); ++cz) {
        int tz = 0, lz = 0;
        if (D == 3) {
            tz = idx[2] / T;
            lz = idx[2] - tz * T;
            if (cz) {
                if (lz) continue;
                tz = tz ? tz - 1 : kp->g.nt[2] - 1;
                lz = T;
            }
        }
        for (int cy = 0; cy < 2; ++cy) {
            int ty = idx[1] / T, ly = idx[1] - (idx[1] / T) * T;
            if (cy) {
                if (ly) continue;
                ty = ty ? ty - 1 : kp->g.nt[1] - 1;
                ly = T;
            }
            for (int cx = 0; cx < 2; ++cx) {
                int tx = idx[0] / T, lx = idx[0] - (idx[0] / T) * T;
                if (cx) {
                    if (lx) continue;
                    tx = tx ? tx - 1 : kp->g.nt[0] - 1;
                    lx = T;
                }
                const int64_t t = ((int64_t)tz * kp->g.nt[1] + ty) * kp->g.nt[0] + tx;
                rho += kp->rho_tile[t * ND + ((int64_t)lz * N1 + ly) * N1 + lx];
            }
        }
    }
    return rho;
}

// Backward-difference divergence on node o of a vector field co-located with
// E (component a stored at the lower node of its half-integer point).
template <int D, typename V>
__device__ __forceinline__ double node_div(const KParams *__restrict__ kp, const V *F, int64_t o,
                                           const int (&idx)[3])
{
    const int n[3] = {kp->g.n[0], kp->g.n[1], kp->g.n[2]};
    const int64_t cells = kp->g.cells;
    double div = 0.0;
    for (int a = 0; a < D; ++a) {
        int im[3] = {idx[0], idx[1], idx[2]};
        im[a] = idx[a] ? idx[a] - 1 : n[a] - 1;
        const int64_t om = ((int64_t)im[2] * n[1] + im[1]) * n[0] + im[0];
        const V *Fa = F + (int64_t)a * cells;
        div += ((double)Fa[o] - (double)Fa[om]) / kp->g.d[a];
    }
    return div;
}

// Block maxima of two per-thread values into part[2 * block + i].
__device__ __forceinline__ void block_max2(double (&m)[2], double *part)
{
    __shared__ double sred[4][2];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        double x = m[i];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
        if (lane == 0) sred[wave][i] = x;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        double x = sred[0][threadIdx.x];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) x = fmax(x, sred[w][threadIdx.x]);
        part[2 * (int64_t)blockIdx.x + threadIdx.x] = x;
    }
}

// Gauss's law on every node: |div E - (rho - rho_0)| and |rho - rho_0|; keeps
// rho^n for the continuity check of the same step.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_gauss(const KParams *__restrict__ kp)
{
    const int64_t step = kp->state->step;
    if (!gauss_step(kp, step)) return;
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m[2] = {0.0, 0.0};
    if (o < cells) {
        const int n[3] = {kp->g.n[0], kp->g.n[1], kp->g.n[2]};
        const int idx[3] = {(int)(o % n[0]), (int)((o / n[0]) % n[1]), (int)(o / ((int64_t)n[0] * n[1]))};
        const double rho = node_rho<D>(kp, idx);
        if (step == 0) kp->rho0[o] = rho;
        kp->rho_n[o] = rho;
        const double dev = rho - kp->rho0[o];
        const double div = node_div<D>(kp, (const R *)kp->F, o, idx);
        m[0] = fabs(div - dev);
        m[1] = fabs(dev);
    }
    block_max2(m, kp->gauss_part);
}

// Charge continuity of the step on every node, from the charge of the
// particles before (rho^n, kept by k_gauss) and after it (rho^{n+1}, the
// partials of k_rho<NEXT>) and the grid current of the step:
// |rho^{n+1} - rho^n + dt div J^{n+1/2}| and |rho^{n+1} - rho^n|.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_continuity(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!gauss_step(kp, st->step) || (st->fatal & 4)) return;
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double m[2] = {0.0, 0.0};
    if (o < cells) {
        const int n[3] = {kp->g.n[0], kp->g.n[1], kp->g.n[2]};
        const int idx[3] = {(int)(o % n[0]), (int)((o / n[0]) % n[1]), (int)(o / ((int64_t)n[0] * n[1]))};
        const double drho = node_rho<D>(kp, idx) - kp->rho_n[o];
        m[0] = fabs(drho + kp->g.dt * node_div<D>(kp, kp->J, o, idx));
        m[1] = fabs(drho);
    }
    block_max2(m, kp->cont_part);
}

// ---------------------------------------------------------------------------
// Binary (pairwise) collisions among the species that take part, after the
// particles of the step have been binned (the paper's binary collision
// module between electrons).  In each cell the participants are ordered by
// a Philox key on (id, step) -- ties by id -- and paired (0,1), (2,3), ...;
// an odd count N >= 3 starts with the triple (0,1), (1,2), (2,0) at half the
// variance (Takizuka and Abe 1977).  A pair turns its relative momentum in
// its centre-of-momentum frame by theta, tan(theta/2) = delta ~ N(0, s^2),
// s^2 = f (nu dt/2)(vref/v_rel)^3, at a uniform azimuth, and is boosted back:
// equal weights keep the pair's four-momentum; with unequal weights the
// heavier particle takes its new momentum with probability w_small/w_large
// (Nanbu and Yonemura 1998).
//
// One workgroup per tile.  The tile's participants are counted per cell and
// put in cell order by a counting sort into a list in scratch memory (store
// slot and species of each), then handled in ranges of consecutive cells
// holding at most kBinCap of them: the range's entries go to LDS with the
// 64-bit key (Philox key << 32 | id), each entry's rank among its cell's
// entries in key order places it (a rank sort per cell: a cell holds a few
// hundred participants at most, and the lanes of a wave mostly share one
// cell, so they read the same keys), and the pairs (a triple counts as one
// unit, done by one thread in order) are spread over the threads; the
// momenta are read and written in the particle store in place.
constexpr int kBinCap = 2048;                       // 4096: 8% slower (LDS: 2 workgroups per CU, not 4)

template <typename R>
__device__ __forceinline__ void boost_frame(const R (&bv)[3], R b2, R gc, R sign, R &e, R (&p)[3])
{
    if (!(b2 > R(0))) return;
    const R bp = bv[0] * p[0] + bv[1] * p[1] + bv[2] * p[2];
    const R c = (gc - R(1)) * bp / b2 - sign * gc * e;
    const R en = gc * (e - sign * bp);
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] += c * bv[i];
    e = en;
}

// One pair (a first).  Returns true if the pair scattered; ua, ub hold the
// momenta (gamma v / c) of the particles that take their new momenta.
template <typename R>
__device__ bool binary_pair(R (&ua)[3], R ma, R wa, uint32_t ida, R (&ub)[3], R mb, R wb, R f, uint32_t step,
                            uint32_t seed0, uint32_t seed1, uint32_t run, R cee)
{
    const R ga = sqrt(R(1) + ua[0] * ua[0] + ua[1] * ua[1] + ua[2] * ua[2]);
    const R gb = sqrt(R(1) + ub[0] * ub[0] + ub[1] * ub[1] + ub[2] * ub[2]);
    R dv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dv[i] = ua[i] / ga - ub[i] / gb;
    const R vrel = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    if (!(vrel > R(0))) return false;
    const uint4 r = philox10(make_uint4(ida, step, kPurposeBinaryPair, run), seed0, seed1);
    const R iv = R(1) / vrel;
    const R s2 = f * cee * iv * iv * iv;
    R sn, cs;
    const R delta = sqrt(s2) * sqrt(R(-2) * Arith<R>::ln(R(u01d(r.x)))) *
                    Arith<R>::cs(R(6.283185307179586) * R(u01d(r.y)));
    const R d2 = delta * delta;
    const R st = R(2) * delta / (R(1) + d2), omc = R(2) * d2 / (R(1) + d2);
    Arith<R>::sc(R(6.283185307179586) * R(u01d(r.z)), &sn, &cs);
    bool take_a = true, take_b = true;
    if (wa != wb) {
        const bool a_heavy = wa > wb;
        const R ratio = a_heavy ? wb / wa : wa / wb;
        const bool heavy = R(u01d(r.w)) < ratio;
        if (a_heavy) take_a = heavy;
        else take_b = heavy;
    }
    const R E = ma * ga + mb * gb;
    R P[3], bv[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        P[i] = ma * ua[i] + mb * ub[i];
        bv[i] = P[i] / E;
    }
    const R b2 = bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
    const R gc = E / sqrt(E * E - (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]));
    R ea = ma * ga, pa[3] = {ma * ua[0], ma * ua[1], ma * ua[2]};
    boost_frame<R>(bv, b2, gc, R(1), ea, pa);
    const R pm = sqrt(pa[0] * pa[0] + pa[1] * pa[1] + pa[2] * pa[2]);
    const R pp = sqrt(pa[0] * pa[0] + pa[1] * pa[1]);
    R dp[3];
    if (pp > R(0)) {
        dp[0] = (pa[0] * pa[2] / pp) * st * cs - (pa[1] * pm / pp) * st * sn - pa[0] * omc;
        dp[1] = (pa[1] * pa[2] / pp) * st * cs + (pa[0] * pm / pp) * st * sn - pa[1] * omc;
        dp[2] = -pp * st * cs - pa[2] * omc;
    } else {
        dp[0] = pm * st * cs;
        dp[1] = pm * st * sn;
        dp[2] = -pa[2] * omc;
    }
    R qa[3], qb[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        qa[i] = pa[i] + dp[i];
        qb[i] = -qa[i];
    }
    R e1 = sqrt(ma * ma + qa[0] * qa[0] + qa[1] * qa[1] + qa[2] * qa[2]);
    boost_frame<R>(bv, b2, gc, R(-1), e1, qa);
    if (take_a && take_b) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const R pb = P[i] - qa[i];
            ua[i] = qa[i] / ma;
            ub[i] = pb / mb;
        }
    } else if (take_a) {
#pragma unroll
        for (int i = 0; i < 3; ++i) ua[i] = qa[i] / ma;
    } else {
        R e2 = sqrt(mb * mb + qb[0] * qb[0] + qb[1] * qb[1] + qb[2] * qb[2]);
        boost_frame<R>(bv, b2, gc, R(-1), e2, qb);
#pragma unroll
        for (int i = 0; i < 3; ++i) ub[i] = qb[i] / mb;
    }
    return true;
}

constexpr int kBinThreads = 512;

template <typename R, int D, int T>
__global__ __launch_bounds__(kBinThreads) void k_binary(const KParams *__restrict__ kp)
{
    constexpr int TC = D == 3 ? T * T * T : T * T;      // cells of the tile
    constexpr uint32_t kSlotMask = (1u << 29) - 1u;
    __shared__ uint32_t s_cnt[TC];                       // participants per cell, then fill cursors
    __shared__ uint32_t s_off[TC + 1];                   // tile-wide exclusive prefix of the counts
    __shared__ uint32_t s_unit[TC + 1];                  // prefix of the work units of the range's cells
    __shared__ uint64_t s_k64[kBinCap];                  // sort key of each entry: Philox key << 32 | id
    __shared__ uint32_t s_ent[kBinCap];                  // slot | species << 29 of each entry
    __shared__ uint16_t s_cell[kBinCap];                 // cell (in the range) of each entry
    __shared__ uint16_t s_idx[kBinCap];                  // entry at each sorted position
    __shared__ uint32_t s_range[2];
    __shared__ uint32_t s_pairs;
    const DevState *st = kp->state;
    DevState *stw = kp->state;
    if (st->fatal & 4) return;                           // the store was not re-laid out
    const uint32_t step = (uint32_t)st->step;
    const int par = st->rebin ? st->par : st->par ^ 1;   // where this step's particles now are
    const int tile = blockIdx.x, ntiles = kp->g.ntiles;
    const int ntx = kp->g.nt[0], nty = kp->g.nt[1];
    const int t0[3] = {(tile % ntx) * T, ((tile / ntx) % nty) * T, (tile / (ntx * nty)) * T};
    const uint32_t seed0 = (uint32_t)kp->seed, seed1 = (uint32_t)(kp->seed >> 32), run = kp->run;
    const R cee = R(0.5 * kp->nu_ee * kp->g.dt * kp->ee_vref * kp->ee_vref * kp->ee_vref);

    // local cell of a stored particle (-1 if outside the tile)
    auto local_cell = [&](const SpeciesDev &S, int64_t slot) {
        int l[3] = {0, 0, 0};
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            int ic;
            if constexpr (sizeof(R) == 4)
                ic = t0[a] + (int)(((uint32_t)S.cell[par][slot] >> (a * kp->g.tshift[0])) & (uint32_t)(T - 1));
            else
                ic = (int)floor(((const double *)S.pos[par][a])[slot]);
            l[a] = ic - t0[a];
            inside = inside && l[a] >= 0 && l[a] < T;
        }
        return inside ? (l[2] * T + l[1]) * T + l[0] : -1;
    };
    auto slot_of = [&](const SpeciesDev &S, int64_t k, int64_t nf, int64_t nb) {
        return k < nf ? (int64_t)S.start[tile] + k : (int64_t)S.start[tile] + S.cap[tile] - nb + (k - nf);
    };
    // the tile's list of participants: at the sum of the participating
    // species' bin starts (bins are laid out in tile order in every species,
    // so the lists of different tiles do not overlap)
    int64_t lbase = 0;
    for (int s = 0; s < kp->nspecies; ++s)
        if (kp->sp[s].binary) lbase += kp->sp[s].start[tile];
    uint32_t *list = kp->ee_ent + lbase;

    for (int c = threadIdx.x; c < TC; c += blockDim.x) s_cnt[c] = 0;
    if (threadIdx.x == 0) s_pairs = 0;
    __syncthreads();
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        if (!S.binary) continue;
        const int64_t nf = S.cnt_front[par * ntiles + tile], nb = S.cnt_back[par * ntiles + tile];
        for (int64_t k = threadIdx.x; k < nf + nb; k += blockDim.x) {
            const int lc = local_cell(S, slot_of(S, k, nf, nb));
            if (lc < 0) atomicOr(&stw->fatal, 8);
            else atomicAdd(&s_cnt[lc], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run_total = 0;
        for (int c = 0; c < TC; ++c) {
            s_off[c] = run_total;
            run_total += s_cnt[c];
        }
        s_off[TC] = run_total;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < TC; c += blockDim.x) s_cnt[c] = 0;
    __syncthreads();
    // counting sort of the participants by cell into the tile's list (the
    // order inside a cell is free: the rank sort below fixes it)
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        if (!S.binary) continue;
        const int64_t nf = S.cnt_front[par * ntiles + tile], nb = S.cnt_back[par * ntiles + tile];
        for (int64_t k = threadIdx.x; k < nf + nb; k += blockDim.x) {
            const int64_t slot = slot_of(S, k, nf, nb);
            const int lc = local_cell(S, slot);
            if (lc < 0) continue;
            const uint32_t pos = s_off[lc] + atomicAdd(&s_cnt[lc], 1u);
            list[pos] = (uint32_t)slot | ((uint32_t)s << 29);
        }
    }
    __syncthreads();                                     // the list is visible to the whole workgroup
    uint32_t my_pairs = 0;
    int c0 = 0;
    while (c0 < TC) {
        if (threadIdx.x == 0) {
            int c1 = c0;
            while (c1 < TC && s_off[c1 + 1] - s_off[c0] <= (uint32_t)kBinCap) ++c1;
            if (c1 == c0) {                                  // one cell above the limit: left alone
                atomicOr(&stw->fatal, 16);
                c1 = c0 + 1;
                s_range[1] = 1;
            } else {
                s_range[1] = 0;
            }
            s_range[0] = (uint32_t)c1;
        }
        __syncthreads();
        const int c1 = (int)s_range[0];
        const bool skip = s_range[1] != 0;
        const uint32_t base = s_off[c0], n_in = s_off[c1] - base;
        if (!skip && n_in >= 2) {
            // the range's entries with their sort keys and cells
            for (uint32_t i = threadIdx.x; i < n_in; i += blockDim.x) {
                const uint32_t e = list[base + i];
                const uint32_t slot = e & kSlotMask;
                const uint32_t id = kp->sp[e >> 29].id[par][slot];
                const uint32_t key = philox10(make_uint4(id, step, kPurposeBinaryKey, run), seed0, seed1).x;
                s_k64[i] = ((uint64_t)key << 32) | id;
                s_ent[i] = e;
                int lo = c0, hi = c1 - 1;                    // cell holding list position base + i
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= base + i) lo = mid;
                    else hi = mid - 1;
                }
                s_cell[i] = (uint16_t)(lo - c0);
            }
            __syncthreads();
            // rank of each entry among its cell's entries in (key, id) order
            // (ties, only possible with repeated ids, by list position)
            for (uint32_t i = threadIdx.x; i < n_in; i += blockDim.x) {
                const int c = c0 + s_cell[i];
                const uint32_t lo = s_off[c] - base, hi = s_off[c + 1] - base;
                const uint64_t k = s_k64[i];
                uint32_t r = 0;
                for (uint32_t j = lo; j < hi; ++j) {
                    const uint64_t kj = s_k64[j];
                    r += (kj < k || (kj == k && j < i)) ? 1u : 0u;
                }
                s_idx[lo + r] = (uint16_t)i;
            }
            // work units per cell: N/2 pairs, or the triple and (N-3)/2 pairs
            if (threadIdx.x == 0) {
                uint32_t u = 0;
                for (int c = c0; c < c1; ++c) {
                    s_unit[c - c0] = u;
                    const uint32_t N = s_off[c + 1] - s_off[c];
                    u += (N & 1u) ? (N >= 3 ? 1u + (N - 3) / 2 : 0u) : N / 2;
                }
                s_unit[c1 - c0] = u;
            }
            __syncthreads();
            const uint32_t units = s_unit[c1 - c0];
            for (uint32_t w = threadIdx.x; w < units; w += blockDim.x) {
                int lo = 0, hi = c1 - c0 - 1;                    // cell holding unit w
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_unit[mid] <= w) lo = mid;
                    else hi = mid - 1;
                }
                const int c = c0 + lo;
                const uint32_t N = s_off[c + 1] - s_off[c], seg = s_off[c] - base, ui = w - s_unit[lo];
                int np;
                uint32_t ea[3], eb[3];
                R fct;
                if ((N & 1u) && ui == 0) {                       // the triple
                    np = 3;
                    fct = R(0.5);
                    ea[0] = s_idx[seg]; eb[0] = s_idx[seg + 1];
                    ea[1] = s_idx[seg + 1]; eb[1] = s_idx[seg + 2];
                    ea[2] = s_idx[seg + 2]; eb[2] = s_idx[seg];
                } else {
                    np = 1;
                    fct = R(1);
                    const uint32_t k = (N & 1u) ? 3 + 2 * (ui - 1) : 2 * ui;
                    ea[0] = s_idx[seg + k];
                    eb[0] = s_idx[seg + k + 1];
                }
                for (int q = 0; q < np; ++q) {
                    const SpeciesDev &SA = kp->sp[s_ent[ea[q]] >> 29];
                    const SpeciesDev &SB = kp->sp[s_ent[eb[q]] >> 29];
                    const uint32_t sa = s_ent[ea[q]] & kSlotMask, sb = s_ent[eb[q]] & kSlotMask;
                    R ua[3], ub[3];
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        ua[i] = ((const R *)SA.u[par][i])[sa];
                        ub[i] = ((const R *)SB.u[par][i])[sb];
                    }
                    if (binary_pair<R>(ua, R(SA.m), R(SA.w), (uint32_t)s_k64[ea[q]], ub, R(SB.m), R(SB.w), fct,
                                       step, seed0, seed1, run, cee)) {
                        ++my_pairs;
#pragma unroll
                        for (int i = 0; i < 3; ++i) {
                            ((R *)SA.u[par][i])[sa] = ua[i];
                            ((R *)SB.u[par][i])[sb] = ub[i];
                        }
                    }
                }
            }
        }
        __syncthreads();                                     // the LDS lists are rebuilt for the next range
        c0 = c1;
    }
    atomicAdd(&s_pairs, my_pairs);
    __syncthreads();
    if (threadIdx.x == 0) kp->ee_tile[tile] = (int64_t)s_pairs;
}

template <typename R>
__device__ __forceinline__ void rebin_count_ovf_body(const KParams *__restrict__ kp, int bid, int nb)
{
    const DevState *st = kp->state;
    if (!st->rebin) return;
    const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int64_t n = min((int64_t)st->ovf_count[s], (int64_t)S.ovf_cap);
        for (int64_t p = i; p < n; p += (int64_t)nb * blockDim.x)
            atomicAdd(&kp->rb_count[(int64_t)s * kp->g.ntiles + tile_of<R>(kp, S, 2, p)], 1);
    }
}

// one block per species: capacities = count + uniform reserve, exclusive scan
__device__ __forceinline__ void rebin_scan_body(const KParams *__restrict__ kp, int bid, int nb)
{
    __shared__ int64_t spart[256];
    __shared__ int64_t s_total;
    DevState *st = kp->state;
    if (!st->rebin) return;
    const int s = bid;
    if (s >= kp->nspecies) return;
    const SpeciesDev &S = kp->sp[s];
    const int ntiles = kp->g.ntiles;
    const int32_t *cnt = kp->rb_count + (int64_t)s * ntiles;
    const int chunk = (ntiles + 255) / 256;
    const int t0 = threadIdx.x * chunk, t1 = min(t0 + chunk, ntiles);
    // pass 1: particle total
    int64_t local = 0;
    for (int t = t0; t < t1; ++t) local += cnt[t];
    spart[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        for (int i = 0; i < 256; ++i) tot += spart[i];
        s_total = tot;
    }
    __syncthreads();
    // reserve of tile t: m + floor(rest * count_t / total), which sums to at
    // most the free slots.  Half of the free slots are spread evenly (a tile
    // emptied by filamentation still takes the stream of movers from a dense
    // neighbour: in 3D about 6% of a tile's beam crosses into the next tile
    // along the drift every step) and half in proportion to the counts
    const int64_t total = s_total;
    const int64_t slack = S.ncap - total;
    if (slack < 0) {
        if (threadIdx.x == 0) atomicOr(&st->fatal, 4);
        return;
    }
    const int64_t m = slack / (2 * (int64_t)ntiles);
    const int64_t rest = slack - m * ntiles;
    auto reserve = [&](int64_t c) { return m + (total > 0 ? (rest * c) / total : rest / ntiles); };
    // capacity: count + reserve, rounded to a multiple of kBinAlign particles
    // (down, unless that would cut into the count) so that every bin starts
    // on a cache-line boundary of each particle array
    auto capacity = [&](int64_t c) {
        const int64_t v = c + reserve(c);
        return max((c + kBinAlign - 1) / kBinAlign * kBinAlign, v / kBinAlign * kBinAlign);
    };
    // pass 2: exclusive scan of the capacities
    local = 0;
    for (int t = t0; t < t1; ++t) local += capacity(cnt[t]);
    __syncthreads();
    spart[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 256; ++i) { const int64_t v = spart[i]; spart[i] = run; run += v; }
        if (run > S.ncap) atomicOr(&st->fatal, 4);     // rounding left no room (tiny reserve)
    }
    __syncthreads();
    int64_t off = spart[threadIdx.x];
    for (int t = t0; t < t1; ++t) {
        const int64_t c = capacity(cnt[t]);
        kp->rb_start[(int64_t)s * ntiles + t] = (int32_t)off;
        kp->rb_cap[(int64_t)s * ntiles + t] = (int32_t)c;
        off += c;
    }
}

// One particle's stored fields, for copies that load several particles
// before storing any (the loads are then in flight together).
template <typename R>
struct StoredParticle {
    uint32_t c;
    R p[3];
    R u[3];
    uint32_t id;
};
template <typename R>
__device__ __forceinline__ void load_stored(const SpeciesDev &S, int nd, int set, int64_t a, StoredParticle<R> &v)
{
    if constexpr (sizeof(R) == 4) v.c = set == 2 ? gbl(S.ovf_cell)[a] : (uint32_t)gbl(S.cell[set & 1])[a];
    for (int c = 0; c < 3; ++c)
        if (c < nd) v.p[c] = gbl((const R *)S.pos[set][c])[a];
    for (int c = 0; c < 3; ++c) v.u[c] = gbl((const R *)S.u[set][c])[a];
    v.id = S.track_id ? gbl(S.id[set])[a] : 0u;
}
template <typename R>
__device__ __forceinline__ void store_stored(const SpeciesDev &S, int nd, int set, int64_t b, const StoredParticle<R> &v)
{
    if constexpr (sizeof(R) == 4) gbl(S.cell[set & 1])[b] = (uint16_t)v.c;   // bins only (set 0 or 1)
    for (int c = 0; c < 3; ++c)
        if (c < nd) gbl((R *)S.pos[set][c])[b] = v.p[c];
    for (int c = 0; c < 3; ++c) gbl((R *)S.u[set][c])[b] = v.u[c];
    if (S.track_id) gbl(S.id[set])[b] = v.id;
}
constexpr int kCopyUnroll = 4;

// copy each tile's valid bin contents dst -> src (blocks stride over (tile, species))
template <typename R>
__device__ __forceinline__ void rebin_scatter_body(const KParams *__restrict__ kp, int bid, int nb)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int ntiles = kp->g.ntiles;
    const int src = st->par, dst = src ^ 1;
    for (int pair = bid; pair < ntiles * kp->nspecies; pair += nb) {
        const int s = pair / ntiles, t = pair - s * ntiles;
        const SpeciesDev &S = kp->sp[s];
        const int64_t room = (int64_t)S.cap[t] - S.cnt_front[src * ntiles + t] - S.cnt_back[src * ntiles + t];
        const int64_t nf = S.cnt_front[dst * ntiles + t];
        const int64_t vb = min((int64_t)S.cnt_back[dst * ntiles + t], room);
        const int64_t from0 = S.start[t], cap = S.cap[t];
        const int64_t to0 = kp->rb_start[(int64_t)s * ntiles + t];
        const int nd = kp->g.ndim;
        for (int64_t k0 = threadIdx.x; k0 < nf + vb; k0 += kCopyUnroll * (int64_t)blockDim.x) {
            StoredParticle<R> v[kCopyUnroll];
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) {
                const int64_t k = k0 + u * (int64_t)blockDim.x;
                if (k < nf + vb) load_stored<R>(S, nd, dst, k < nf ? from0 + k : from0 + cap - vb + (k - nf), v[u]);
            }
#pragma unroll
            for (int u = 0; u < kCopyUnroll; ++u) {
                const int64_t k = k0 + u * (int64_t)blockDim.x;
                if (k < nf + vb) store_stored<R>(S, nd, src, to0 + k, v[u]);
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ void rebin_scatter_ovf_body(const KParams *__restrict__ kp, int bid, int nb)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int src = st->par;
    const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int64_t n = min((int64_t)st->ovf_count[s], (int64_t)S.ovf_cap);
        for (int64_t p = i; p < n; p += (int64_t)nb * blockDim.x) {
            const int64_t idx = (int64_t)s * kp->g.ntiles + tile_of<R>(kp, S, 2, p);
            const int32_t slot = atomicAdd(&kp->rb_fill[idx], 1);
            StoredParticle<R> v;
            load_stored<R>(S, kp->g.ndim, 2, p, v);
            if constexpr (sizeof(R) == 4) v.c = local_of_global(kp->g, v.c);
            store_stored<R>(S, kp->g.ndim, src, (int64_t)kp->rb_start[idx] + slot, v);
        }
    }
}

__device__ __forceinline__ void rebin_finalize_body(const KParams *__restrict__ kp, int bid, int nb)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int ntiles = kp->g.ntiles;
    const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
    if (i >= (int64_t)kp->nspecies * ntiles) return;
    const int s = (int)(i / ntiles), t = (int)(i % ntiles);
    const SpeciesDev &S = kp->sp[s];
    const int src = st->par, dst = src ^ 1;
    S.start[t] = kp->rb_start[i];
    S.cap[t] = kp->rb_cap[i];
    S.cnt_front[src * ntiles + t] = (uint32_t)kp->rb_count[i];
    S.cnt_back[src * ntiles + t] = 0;
    S.cnt_back[dst * ntiles + t] = 0;
}

// ---------------------------------------------------------------------------
// Grid current: fixed-order FP64 sum of the tile partials covering each node.
// Along an axis, node i = a0*T + r is held by tile a0 (local r+1), by tile
// a0-1 when r <= 1 (local r+T+1) and by tile a0+1 when r = T-1 (local 0).
// In 3D consecutive threads take the nodes of one tile in its own x-y-z
// order, so that a wave reads 8 rows of one tile partial (nearly contiguous)
// instead of 64 nodes of a grid row spread over 64/T partials; the summation
// order per node is the same either way.  A workgroup's 256 nodes lie in
// one tile (512 nodes, tile edge 8), so the tiles below, at and above it on
// each axis are workgroup-uniform; per node and axis only the choice among
// them (and the local index) varies, and a partial's offset is the sum of
// one term per axis.
template <typename R>
__device__ __forceinline__ void reduce_j_tile3(const KParams *__restrict__ kp, int bid)
{
    constexpr int T = 8, NJ = T + 3, NJ_D = NJ * NJ * NJ;
    const int64_t cells = kp->g.cells;
    const int64_t q = (int64_t)bid * 256 + threadIdx.x;
    if (q >= cells) return;
    const int64_t t = (int64_t)bid >> 1;                  // 2 workgroups per tile
    const int r = (int)(q & 511);
    const int nt[3] = {kp->g.nt[0], kp->g.nt[1], kp->g.nt[2]};
    const int tc[3] = {(int)(t % nt[0]), (int)((t / nt[0]) % nt[1]), (int)(t / ((int64_t)nt[0] * nt[1]))};
    const int rr[3] = {r & 7, (r >> 3) & 7, r >> 6};
    const int64_t tstride[3] = {3 * (int64_t)NJ_D, 3 * (int64_t)NJ_D * nt[0], 3 * (int64_t)NJ_D * nt[0] * nt[1]};
    constexpr int lstride[3] = {1, NJ, NJ * NJ};
    int64_t off[3][2];
    int cn[3];
    int idx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int below = tc[a] == 0 ? nt[a] - 1 : tc[a] - 1;
        const int above = tc[a] + 1 == nt[a] ? 0 : tc[a] + 1;
        const int64_t own = (int64_t)tc[a] * tstride[a] + (rr[a] + 1) * lstride[a];
        if (rr[a] <= 1) {
            off[a][0] = (int64_t)below * tstride[a] + (rr[a] + 1 + T) * lstride[a];
            off[a][1] = own;
            cn[a] = 2;
        } else {
            off[a][0] = own;
            off[a][1] = (int64_t)above * tstride[a];
            cn[a] = rr[a] == T - 1 ? 2 : 1;
        }
        idx[a] = tc[a] * T + rr[a];
    }
    const GLB R *Jt = gbl((const R *)kp->Jtile);
    R vx[8], vy[8], vz[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int iz = k >> 2, iy = (k >> 1) & 1, ix = k & 1;
        vx[k] = vy[k] = vz[k] = R(0);
        if (iz < cn[2] && iy < cn[1] && ix < cn[0]) {
            const GLB R *p = Jt + (off[0][ix] + off[1][iy] + off[2][iz]);
            vx[k] = p[0];
            vy[k] = p[NJ_D];
            vz[k] = p[2 * NJ_D];
        }
    }
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        jx += (double)vx[k];
        jy += (double)vy[k];
        jz += (double)vz[k];
    }
    const int64_t o = ((int64_t)idx[2] * kp->g.n[1] + idx[1]) * kp->g.n[0] + idx[0];
    GLB double *J = gbl(kp->J);
    J[o] = jx;
    J[cells + o] = jy;
    J[2 * cells + o] = jz;
}

template <typename R, int D>
__device__ __forceinline__ void reduce_j_body(const KParams *__restrict__ kp, int bid, int nb)
{
    if constexpr (D == 3) {
        reduce_j_tile3<R>(kp, bid);
        return;
    }
    // 2D: one node per thread in grid row order
    const int64_t cells = kp->g.cells;
    const int64_t q = (int64_t)bid * blockDim.x + threadIdx.x;
    if (q >= cells) return;
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int T = kp->g.tile[0];
    int idx[3];
    const int64_t o = q;
    idx[0] = (int)(q % nx);
    idx[1] = (int)((q / nx) % ny);
    idx[2] = 0;
    const int NJ = kp->nj;
    const int64_t NJ_D = (int64_t)NJ * NJ;
    int tb[3], r[3];
    for (int a = 0; a < 3; ++a) {
        tb[a] = idx[a] / T;
        r[a] = idx[a] - tb[a] * T;
    }
    const GLB R *Jt = gbl((const R *)kp->Jtile);
    // Per axis the tiles holding the node, in increasing tile order: the one
    // below (local index r + 1 + T) when r <= 1, the node's own tile (r + 1),
    // the one above (local 0) when r = T - 1; tiles are at least 8 cells, so
    // at most two per axis.  All of a node's partials are loaded first and
    // then summed in that fixed order.
    int cn[3], ct[3][2], cl[3][2];
    for (int a = 0; a < 3; ++a) {
        cn[a] = 0;
        if (a < D) {
            const int ntile = kp->g.nt[a];
            if (r[a] <= 1) {
                ct[a][cn[a]] = tb[a] == 0 ? ntile - 1 : tb[a] - 1;
                cl[a][cn[a]++] = r[a] + 1 + T;
            }
            ct[a][cn[a]] = tb[a];
            cl[a][cn[a]++] = r[a] + 1;
            if (r[a] == T - 1 && cn[a] < 2) {
                ct[a][cn[a]] = tb[a] + 1 == ntile ? 0 : tb[a] + 1;
                cl[a][cn[a]++] = 0;
            }
        } else {
            ct[a][0] = 0;
            cl[a][0] = 0;
            cn[a] = 1;
        }
    }
    R vx[8], vy[8], vz[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int iz = k >> 2, iy = (k >> 1) & 1, ix = k & 1;
        vx[k] = vy[k] = vz[k] = R(0);
        if (iz < cn[2] && iy < cn[1] && ix < cn[0]) {
            const int64_t t = ((int64_t)ct[2][iz] * kp->g.nt[1] + ct[1][iy]) * kp->g.nt[0] + ct[0][ix];
            const GLB R *p = Jt + t * 3 * NJ_D + ((int64_t)cl[2][iz] * NJ + cl[1][iy]) * NJ + cl[0][ix];
            vx[k] = p[0];
            vy[k] = p[NJ_D];
            vz[k] = p[2 * NJ_D];
        }
    }
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        jx += (double)vx[k];
        jy += (double)vy[k];
        jz += (double)vz[k];
    }
    kp->J[o] = jx;
    kp->J[cells + o] = jy;
    kp->J[2 * cells + o] = jz;
}

// ---------------------------------------------------------------------------
// Yee updates (2D: n[2] == 1 and every z difference vanishes).
// Workgroup b of the single-run 3D current reduction runs on XCD b mod 8:
// each XCD takes a contiguous eighth of the node blocks, so the tile partials
// that neighbouring tiles share are read into one L2 (C4: 0.79 -> 0.72 ms).
// The Yee kernels keep the plain order, which measured faster for them.
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    return (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename R, int NDIM>
__device__ __forceinline__ void yee_b_body(const KParams *__restrict__ kp, int bid, int nb, double h)
{
    if (h == 0.0) return;
    const int nx = kp->g.n[0], ny = kp->g.n[1], nz = NDIM == 3 ? kp->g.n[2] : 1;
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)bid * blockDim.x + threadIdx.x;
    if (o >= cells) return;
    const int i = (int)(o % nx);
    const int j = (int)((o / nx) % ny);
    const int k = (int)(o / ((int64_t)nx * ny));
    const int64_t ip = i + 1 < nx ? o + 1 : o + 1 - nx;
    const int64_t jp = j + 1 < ny ? o + nx : o + nx - (int64_t)nx * ny;
    R *F = (R *)kp->F;
    const R *Ex = F, *Ey = F + cells, *Ez = F + 2 * cells;
    R *Bx = F + 3 * cells, *By = F + 4 * cells, *Bz = F + 5 * cells;
    const double hdt = h * kp->g.dt;
    const R cx = R(hdt / kp->g.d[0]), cy = R(hdt / kp->g.d[1]);
    const R ez = Ez[o], ey = Ey[o], ex = Ex[o];
    R bx = Bx[o] - cy * (Ez[jp] - ez);
    R by = By[o] + cx * (Ez[ip] - ez);
    R bz = Bz[o] - (cx * (Ey[ip] - ey) - cy * (Ex[jp] - ex));
    if constexpr (NDIM == 3) {
        const int64_t kp1 = k + 1 < nz ? o + (int64_t)nx * ny : o + (int64_t)nx * ny - cells;
        const R cz = R(hdt / kp->g.d[2]);
        bx += cz * (Ey[kp1] - ey);
        by -= cz * (Ex[kp1] - ex);
    }
    (void)k;
    Bx[o] = bx;
    By[o] = by;
    Bz[o] = bz;
}

template <typename R, int NDIM>
__device__ __forceinline__ void yee_e_body(const KParams *__restrict__ kp, int bid, int nb)
{
    if (kp->flags & PIC_FLAG_FREEZE_FIELDS) return;
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)bid * blockDim.x + threadIdx.x;
    if (o >= cells) return;
    const int i = (int)(o % nx);
    const int j = (int)((o / nx) % ny);
    const int64_t im = i > 0 ? o - 1 : o - 1 + nx;
    const int64_t jm = j > 0 ? o - nx : o - nx + (int64_t)nx * ny;
    R *F = (R *)kp->F;
    R *Ex = F, *Ey = F + cells, *Ez = F + 2 * cells;
    const R *Bx = F + 3 * cells, *By = F + 4 * cells, *Bz = F + 5 * cells;
    const double dt = kp->g.dt;
    const R cx = R(dt / kp->g.d[0]), cy = R(dt / kp->g.d[1]);
    const R rdt = R(dt);
    const R bz = Bz[o], by = By[o], bx = Bx[o];
    R ex = Ex[o] + cy * (bz - Bz[jm]) - rdt * R(kp->J[o]);
    R ey = Ey[o] - cx * (bz - Bz[im]) - rdt * R(kp->J[cells + o]);
    R ez = Ez[o] + cx * (by - By[im]) - cy * (bx - Bx[jm]) - rdt * R(kp->J[2 * cells + o]);
    if constexpr (NDIM == 3) {
        const int k = (int)(o / ((int64_t)nx * ny));
        const int64_t km = k > 0 ? o - (int64_t)nx * ny : o - (int64_t)nx * ny + cells;
        const R cz = R(dt / kp->g.d[2]);
        ex -= cz * (by - By[km]);
        ey += cz * (bx - Bx[km]);
    }
    Ex[o] = ex;
    Ey[o] = ey;
    Ez[o] = ez;
}

// ---------------------------------------------------------------------------
// End of step: diagnostic record, reset of the next destination's mover
// counters, step and parity update.  One workgroup.
__device__ __forceinline__ void advance_body(const KParams *__restrict__ kp, int bid, int nb)
{
    __shared__ double sred[kAdvanceThreads / 64][10];
    DevState *st = kp->state;
    const int64_t step = st->step;
    const int par = st->par;
    const int rebin = st->rebin;
    const int ntiles = kp->g.ntiles;
    const int ns = kp->nspecies;
    if (diag_step(kp, step)) {
        const double dv = kp->g.d[0] * kp->g.d[1] * (kp->g.ndim == 3 ? kp->g.d[2] : 1.0);
        double f[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = threadIdx.x; b < kp->fd_blocks; b += blockDim.x)
            for (int c = 0; c < 9; ++c) f[c] += kp->field_diag[b * kFieldDiag + c];
        block_sum<10>(f, sred);
        pic_diag rec;
        if (threadIdx.x == 0) {
            for (int c = 0; c < 6; ++c) rec.W[c] = f[c] * dv;
            for (int c = 0; c < 3; ++c) rec.p_field[c] = f[6 + c] * dv;
        }
        double coll_total = 0.0;
        double pp[3] = {0, 0, 0};
        for (int s = 0; s < ns; ++s) {
            double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
                for (int v = 0; v < kTileDiag; ++v) a[v] += kp->tile_diag[((int64_t)t * ns + s) * kTileDiag + v];
            block_sum<8>(a, (double(*)[8])sred);
            if (threadIdx.x == 0) {
                rec.kinetic[s] = a[0] * dv;
                for (int c = 0; c < 3; ++c) {
                    rec.p_species[s][c] = a[1 + c] * dv;
                    pp[c] += a[1 + c] * dv;
                }
                rec.n_particles[s] = (int64_t)a[4];
                coll_total += a[5];
            }
        }
        // residual maxima: Gauss's law (gm[0], gm[1]) and continuity (gm[2], gm[3])
        double gm[4] = {-1.0, -1.0, -1.0, -1.0};
        if (gauss_step(kp, step)) {
            const int64_t nbk = (kp->g.cells + 255) / 256;
            const bool cont = !(st->fatal & 4);
            for (int i = 0; i < 4; ++i) gm[i] = (i < 2 || cont) ? 0.0 : -1.0;
            for (int64_t b = threadIdx.x; b < nbk; b += blockDim.x) {
                gm[0] = fmax(gm[0], kp->gauss_part[2 * b]);
                gm[1] = fmax(gm[1], kp->gauss_part[2 * b + 1]);
                if (cont) {
                    gm[2] = fmax(gm[2], kp->cont_part[2 * b]);
                    gm[3] = fmax(gm[3], kp->cont_part[2 * b + 1]);
                }
            }
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
            for (int i = 0; i < 4; ++i) {
                double x = gm[i];
                for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_down(x, off, 64));
                if (lane == 0) sred[wave][i] = x;
            }
            __syncthreads();
            if (threadIdx.x == 0)
                for (int i = 0; i < 4; ++i) {
                    double x = sred[0][i];
                    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) x = fmax(x, sred[w][i]);
                    gm[i] = x;
                }
            __syncthreads();
        }
        double ee = 0.0;
        if (kp->binary) {
            double a[1] = {0.0};
            for (int t = threadIdx.x; t < ntiles; t += blockDim.x) a[0] += (double)kp->ee_tile[t];
            block_sum<1>(a, (double(*)[1])sred);
            ee = a[0];
        }
        if (threadIdx.x == 0) {
            rec.gauss_resid = gm[0];
            rec.rho_dev = gm[1];
            rec.continuity_resid = gm[2];
            rec.rho_step = gm[3];
            rec.ee_pairs = (int64_t)ee;
            for (int s = ns; s < kMaxSpecies; ++s) {
                rec.kinetic[s] = 0.0;
                rec.n_particles[s] = 0;
                for (int c = 0; c < 3; ++c) rec.p_species[s][c] = 0.0;
            }
            for (int c = 0; c < 3; ++c) rec.p_particles[c] = pp[c];
            rec.collisions = (int64_t)coll_total;
            rec.step = step;
            rec.time = (double)step * kp->g.dt;
            rec.rebins = st->rebins;
            kp->ring[st->ring_head % kRing] = rec;
        }
    }
    if (!rebin) {
        for (int64_t i = threadIdx.x; i < (int64_t)ns * ntiles; i += blockDim.x) {
            const int s = (int)(i / ntiles), t = (int)(i % ntiles);
            kp->sp[s].cnt_back[par * ntiles + t] = 0;
        }
    }
    // Work order of the next step.  Workgroup b of the particle launch runs
    // on XCD b mod 8 (round-robin dispatch) and takes tile order[b].  Tile t
    // keeps XCD class c = t mod 8 -- its y and z neighbours, the destinations
    // of most of its movers, share that XCD's L2 -- and within a class the
    // tiles go by decreasing load bucket (written by this step's particle
    // kernel from the tile's counts at the start of the step), so each XCD
    // starts its heaviest tiles first: order[8 r + c] is the r-th tile of
    // class c.  Class c holds exactly the positions b < ntiles with b mod 8
    // == c, so this is a permutation for any tile count.
    {
        __shared__ int s_hist[kXcds][kOrderBuckets];
        const uint8_t *bucket = kp->tile_bucket;
        for (int i = threadIdx.x; i < kXcds * kOrderBuckets; i += blockDim.x) (&s_hist[0][0])[i] = 0;
        __syncthreads();
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) atomicAdd(&s_hist[t % kXcds][bucket[t]], 1);
        __syncthreads();
        if (threadIdx.x < kXcds) {
            int run = 0;
            for (int b = kOrderBuckets - 1; b >= 0; --b) {
                const int c = s_hist[threadIdx.x][b];
                s_hist[threadIdx.x][b] = run;
                run += c;
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < ntiles; t += blockDim.x) {
            const int c = t % kXcds;
            const int r = atomicAdd(&s_hist[c][bucket[t]], 1);
            kp->order[kXcds * r + c] = t;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        if (diag_step(kp, step)) st->ring_head += 1;
        st->step = step + 1;
        if (rebin) {
            st->rebins += 1;
            st->rebin = 0;
            for (int s = 0; s < kMaxSpecies; ++s) st->ovf_count[s] = 0;
        } else {
            st->par = par ^ 1;
        }
    }
}

// ---------------------------------------------------------------------------
// Kernel entry points.  k_*: one run, the grid covers that run's blocks.
// kb_*: an ensemble; blockIdx.y picks the run, or a table maps each block to
// (run, block of that run), or (particle kernel) persistent workgroups take
// (run, tile) items from a queue, heaviest first.
template <typename R>
__global__ __launch_bounds__(256) void k_field_diag(const KParams *__restrict__ kp)
{
    field_diag_body<R>(kp, blockIdx.x, gridDim.x);
}
// each run writes exactly its own fd_blocks partial records
template <typename R>
__global__ __launch_bounds__(256) void kb_field_diag(const BatchTable *__restrict__ bt)
{
    const KParams *kp = bt->kp[blockIdx.y];
    const int nb = kp->fd_blocks;
    if ((int)blockIdx.x >= nb) return;
    field_diag_body<R>(kp, blockIdx.x, nb);
}

typedef __attribute__((address_space(4))) const KParams KParamsC;

// One workgroup per tile; workgroup b takes tile order[b] (see the work
// order built at the end of each step).
template <typename R, typename A, int D, int T, bool CB, int SH>
__global__ __launch_bounds__(kShapeBlock[SH]) void k_particle(const KParams *__restrict__ kp)
{
    const KParamsC *kc = (const KParamsC *)kp;
    particle_body<R, A, D, T, CB, SH, true>(kc, wave_uniform(kc->order[blockIdx.x]), 0);
}

// Persistent: workgroup w (on XCD w mod 8) takes the items of its XCD
// class from that class's queue -- a run's tile then runs on the XCD it has
// in a run stepped alone -- and, when its class is exhausted, the remaining
// items of the other classes.  The counters only grow, so every workgroup
// reaches the exit.
template <typename R, typename A, int D, int T, bool CB, int SH>
__global__ __launch_bounds__(kShapeBlock[SH]) void kb_particle(const BatchTable *__restrict__ bt)
{
    constexpr int g = T == 8 ? 0 : (T == 16 ? 1 : 2);
    __shared__ int s_item;
    const BatchGroup &G = bt->grp[g];
    const int c0 = blockIdx.x % kBatchXcds;
    for (int cc = 0; cc < kBatchXcds; ++cc) {
        const int c = (c0 + cc) % kBatchXcds;
        const int len = G.cls_len[c];
        const int2 *items = G.items + G.cls_start[c];
        for (;;) {
            if (threadIdx.x == 0) s_item = atomicAdd(&G.queue[c], 1);
            __syncthreads();
            const int i = wave_uniform(s_item);
            __syncthreads();
            if (i >= len) break;
            const int2 it = items[i];
            const KParamsC *kp = (const KParamsC *)wave_uniform_ptr(bt->kp[wave_uniform(it.x)]);
            particle_body<R, A, D, T, CB, SH, false>(kp, wave_uniform(kp->order[wave_uniform(it.y)]), 0);
        }
    }
}

#define PIC_RUN_KERNELS(NAME, BODY)                                                     \
    __global__ __launch_bounds__(256) void k_##NAME(const KParams *__restrict__ kp)    \
    {                                                                                   \
        BODY(kp, blockIdx.x, gridDim.x);                                                \
    }                                                                                   \
    __global__ __launch_bounds__(256) void kb_##NAME(const BatchTable *__restrict__ bt) \
    {                                                                                   \
        BODY(bt->kp[blockIdx.y], blockIdx.x, gridDim.x);                                \
    }
PIC_RUN_KERNELS(rebin_count, rebin_count_body)
PIC_RUN_KERNELS(rebin_scan, rebin_scan_body)
PIC_RUN_KERNELS(rebin_finalize, rebin_finalize_body)
#undef PIC_RUN_KERNELS

template <typename R>
__global__ __launch_bounds__(256) void k_rebin_count_ovf(const KParams *__restrict__ kp)
{
    rebin_count_ovf_body<R>(kp, blockIdx.x, gridDim.x);
}
template <typename R>
__global__ __launch_bounds__(256) void kb_rebin_count_ovf(const BatchTable *__restrict__ bt)
{
    rebin_count_ovf_body<R>(bt->kp[blockIdx.y], blockIdx.x, gridDim.x);
}
template <typename R>
__global__ __launch_bounds__(256) void k_rebin_scatter(const KParams *__restrict__ kp)
{
    rebin_scatter_body<R>(kp, blockIdx.x, gridDim.x);
}
template <typename R>
__global__ __launch_bounds__(256) void kb_rebin_scatter(const BatchTable *__restrict__ bt)
{
    rebin_scatter_body<R>(bt->kp[blockIdx.y], blockIdx.x, gridDim.x);
}
template <typename R>
__global__ __launch_bounds__(256) void k_rebin_scatter_ovf(const KParams *__restrict__ kp)
{
    rebin_scatter_ovf_body<R>(kp, blockIdx.x, gridDim.x);
}
template <typename R>
__global__ __launch_bounds__(256) void kb_rebin_scatter_ovf(const BatchTable *__restrict__ bt)
{
    rebin_scatter_ovf_body<R>(bt->kp[blockIdx.y], blockIdx.x, gridDim.x);
}

template <typename R, int D>
__global__ __launch_bounds__(256) void k_reduce_j(const KParams *__restrict__ kp)
{
    reduce_j_body<R, D>(kp, D == 3 ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x, gridDim.x);
}
template <typename R, int D>
__global__ __launch_bounds__(256) void kb_reduce_j(const BatchTable *__restrict__ bt)
{
    const int2 cb = bt->cell_blocks[blockIdx.x];
    reduce_j_body<R, D>(bt->kp[cb.x], cb.y, 0);
}
template <typename R, int D>
__global__ __launch_bounds__(256) void k_yee_b(const KParams *__restrict__ kp, double h)
{
    yee_b_body<R, D>(kp, blockIdx.x, gridDim.x, h);
}
template <typename R, int D>
__global__ __launch_bounds__(256) void kb_yee_b(const BatchTable *__restrict__ bt, double h)
{
    const int2 cb = bt->cell_blocks[blockIdx.x];
    const KParams *kp = bt->kp[cb.x];
    yee_b_body<R, D>(kp, cb.y, 0, (kp->flags & PIC_FLAG_FREEZE_FIELDS) ? 0.0 : h);
}
template <typename R, int D>
__global__ __launch_bounds__(256) void k_yee_e(const KParams *__restrict__ kp)
{
    yee_e_body<R, D>(kp, blockIdx.x, gridDim.x);
}
template <typename R, int D>
__global__ __launch_bounds__(256) void kb_yee_e(const BatchTable *__restrict__ bt)
{
    const int2 cb = bt->cell_blocks[blockIdx.x];
    yee_e_body<R, D>(bt->kp[cb.x], cb.y, 0);
}

__global__ __launch_bounds__(kAdvanceThreads) void k_advance(const KParams *__restrict__ kp)
{
    advance_body(kp, blockIdx.x, gridDim.x);
}
// one workgroup per run; the first also rewinds the particle-kernel queues
__global__ __launch_bounds__(kAdvanceThreads) void kb_advance(const BatchTable *__restrict__ bt)
{
    advance_body(bt->kp[blockIdx.x], 0, 1);
    if (blockIdx.x == 0 && threadIdx.x < kBatchGroups * kBatchXcds)
        bt->grp[threadIdx.x / kBatchXcds].queue[threadIdx.x % kBatchXcds] = 0;
}

// ---------------------------------------------------------------------------
// Device loader: exactly ppc particles per cell, bins laid out tile-major;
// inside a tile the k-th particle of every cell comes before the (k+1)-th of
// any cell, so the 64 lanes of a wave sit in 64 different cells and their
// current atomics hit different LDS words.  Uniform in-cell positions (or a
// regular sub-lattice) and Gaussian momenta come from Philox draws keyed by
// the particle id.
template <typename R, int D>
__global__ __launch_bounds__(256) void k_load(const KParams *__restrict__ kp, int s)
{
    const SpeciesDev &S = kp->sp[s];
    const int T = kp->g.tile[0];
    const int TD = D == 3 ? T * T * T : T * T;
    const int64_t per_tile = (int64_t)S.ppc * TD;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= per_tile * kp->g.ntiles) return;
    const int tile = (int)(p / per_tile);
    const int64_t q = p - tile * per_tile;
    const int slot = (int)(q / TD), cl = (int)(q - (int64_t)slot * TD);
    const int ntx = kp->g.nt[0], nty = kp->g.nt[1];
    int ic[3];
    ic[0] = (tile % ntx) * T + cl % T;
    ic[1] = ((tile / ntx) % nty) * T + (cl / T) % T;
    ic[2] = D == 3 ? (tile / (ntx * nty)) * T + cl / (T * T) : 0;
    const int64_t cell = ((int64_t)ic[2] * kp->g.n[1] + ic[1]) * kp->g.n[0] + ic[0];
    const uint32_t id = (uint32_t)(S.id_base + cell * S.ppc + slot);
    const uint32_t k0 = (uint32_t)kp->seed, k1 = (uint32_t)(kp->seed >> 32);
    const uint4 r0 = philox10(make_uint4(id, 0u, kPurposeLoad, kp->run), k0, k1);
    const uint4 r1 = philox10(make_uint4(id, 1u, kPurposeLoad, kp->run), k0, k1);
    const uint32_t rw[3] = {r0.x, r0.y, r0.z};
    double off[3];
    if (kp->flags & PIC_FLAG_LATTICE_LOAD) {
        const int m = (int)rint(pow((double)S.ppc, 1.0 / D));
        int rem = slot;
        for (int a = 0; a < D; ++a) {
            off[a] = (rem % m + 0.5) / m;
            rem /= m;
        }
    } else {
        for (int a = 0; a < D; ++a) off[a] = sizeof(R) == 4 ? (double)u01f(rw[a]) : u01d(rw[a]);
    }
    // Box-Muller on two pairs of uniforms
    const double ra = sqrt(-2.0 * log(u01d(r1.x))), pa = 6.283185307179586 * u01d(r1.y);
    const double rb = sqrt(-2.0 * log(u01d(r1.z))), pb = 6.283185307179586 * u01d(r1.w);
    const double z[3] = {ra * cos(pa), ra * sin(pa), rb * cos(pb)};
    const int64_t pos = (int64_t)S.start[tile] + q;
    if constexpr (sizeof(R) == 4) {
        uint32_t c = 0;
        for (int a = 0; a < D; ++a) {
            c |= ((uint32_t)ic[a] & (uint32_t)(kp->g.tile[0] - 1)) << (a * kp->g.tshift[0]);
            ((float *)S.pos[0][a])[pos] = (float)off[a];
        }
        S.cell[0][pos] = (uint16_t)c;
    } else {
        for (int a = 0; a < D; ++a) ((double *)S.pos[0][a])[pos] = (double)ic[a] + off[a];
    }
    for (int c = 0; c < 3; ++c) ((R *)S.u[0][c])[pos] = R(S.drift[c] + S.uth * z[c]);
    if (S.track_id) S.id[0][pos] = id;
}

// Visits every particle of species s in the current set: calls f(u, i, slot).
template <typename R, typename Fn>
__device__ __forceinline__ void for_each_particle(const KParams *kp, int s, Fn &&f)
{
    const SpeciesDev &S = kp->sp[s];
    const int ntiles = kp->g.ntiles;
    const int par = kp->state->par;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t nf = S.cnt_front[par * ntiles + t], nb = S.cnt_back[par * ntiles + t];
        const int64_t b0 = S.start[t], cap = S.cap[t];
        for (int64_t k = threadIdx.x; k < nf + nb; k += blockDim.x) {
            const int64_t slot = k < nf ? b0 + k : b0 + cap - nb + (k - nf);
            f(par, slot);
        }
    }
}

// Loader reductions (FP64): sum u_x, sum u_y, sum (u_z + delta)/gamma,
// sum (1 + u_perp^2)/gamma^3 (the derivative of the previous sum in delta),
// sum u_z/gamma, count.
template <typename R>
__global__ __launch_bounds__(256) void k_moments(const KParams *__restrict__ kp, int s, double delta)
{
    __shared__ double sred[4][kMomentVals];
    const SpeciesDev &S = kp->sp[s];
    double a[kMomentVals] = {0, 0, 0, 0, 0, 0};
    for_each_particle<R>(kp, s, [&](int set, int64_t slot) {
        const double ux = ((const R *)S.u[set][0])[slot];
        const double uy = ((const R *)S.u[set][1])[slot];
        const double uz = ((const R *)S.u[set][2])[slot];
        const double up2 = ux * ux + uy * uy;
        const double w = uz + delta;
        const double g = sqrt(1.0 + up2 + w * w);
        a[0] += ux;
        a[1] += uy;
        a[2] += w / g;
        a[3] += (1.0 + up2) / (g * g * g);
        a[4] += uz / sqrt(1.0 + up2 + uz * uz);
        a[5] += 1.0;
    });
    block_sum<kMomentVals>(a, sred);
    if (threadIdx.x == 0)
        for (int v = 0; v < kMomentVals; ++v) kp->moments[blockIdx.x * kMomentVals + v] = a[v];
}

template <typename R>
__global__ __launch_bounds__(256) void k_shift_u(const KParams *__restrict__ kp, int s, double dux,
                                                 double duy, double duz)
{
    const SpeciesDev &S = kp->sp[s];
    for_each_particle<R>(kp, s, [&](int set, int64_t slot) {
        R *u0 = (R *)S.u[set][0], *u1 = (R *)S.u[set][1], *u2 = (R *)S.u[set][2];
        u0[slot] = R((double)u0[slot] + dux);
        u1[slot] = R((double)u1[slot] + duy);
        u2[slot] = R((double)u2[slot] + duz);
    });
}

// ---------------------------------------------------------------------------
// Launches one kernel; with `ev` it is a hipExtLaunchKernelGGL whose start
// and stop events carry the dispatch's own timestamps (ev[2k], ev[2k+1] for
// the k-th kernel of the step).
struct Launcher {
    hipStream_t st;
    hipEvent_t *ev;
    int *groups = nullptr;   // if set: the kernel group of each launch is recorded here
    bool dry = false;        // record only, launch nothing
    int grp = 0;             // group of the next launches
    int k = 0;
    template <typename... KArgs, typename... A>
    void operator()(void (*kern)(KArgs...), dim3 g, dim3 b, A... args)
    {
        if (groups) groups[k] = grp;
        if (!dry) {
            if (ev) hipExtLaunchKernelGGL(kern, g, b, 0, st, ev[2 * k], ev[2 * k + 1], 0, args...);
            else hipLaunchKernelGGL(kern, g, b, 0, st, args...);
        }
        ++k;
    }
};

// The particle kernel of a run or batch group in launch shape `shape` (FP64
// kernels exist in shape 0 only; the runtime refuses others).
template <typename R, typename A, int D, int T, bool CB>
static auto particle_kernel(int shape)
{
    using F = void (*)(const KParams *);
    F f = k_particle<R, A, D, T, CB, 0>;
    if constexpr (sizeof(R) == 4) {
        switch (shape) {
        case 1: f = k_particle<R, A, D, T, CB, 1>; break;
        case 2: f = k_particle<R, A, D, T, CB, 2>; break;
        case 3: f = k_particle<R, A, D, T, CB, 3>; break;
        case 4: f = k_particle<R, A, D, T, CB, 4>; break;
        default: break;
        }
    }
    return f;
}
template <typename R, typename A, int D, int T, bool CB>
static auto batch_particle_kernel(int shape)
{
    using F = void (*)(const BatchTable *);
    F f = kb_particle<R, A, D, T, CB, 0>;
    if constexpr (sizeof(R) == 4) {
        switch (shape) {
        case 1: f = kb_particle<R, A, D, T, CB, 1>; break;
        case 2: f = kb_particle<R, A, D, T, CB, 2>; break;
        case 3: f = kb_particle<R, A, D, T, CB, 3>; break;
        case 4: f = kb_particle<R, A, D, T, CB, 4>; break;
        default: break;
        }
    }
    return f;
}
static int shape_block(int precision_is_mixed, int shape)
{
    return precision_is_mixed && shape > 0 && shape < kShapes ? kShapeBlock[shape] : kShapeBlock[0];
}

// Kernel order of a step (groups in brackets): [0 Gauss checks: charge,
// residual] | [0] field diag | [1] particle | [2] 6 x re-layout | [1] binary
// collisions (if any) | [3] J reduction | [0 continuity check: charge,
// residual] | [4] 3 x Yee | [5] advance.
template <typename R, typename A, int D, int T>
static hipError_t step_kernels(const KParams &hp, const KParams *dp, Launcher &L)
{
    const int ntiles = hp.g.ntiles;
    const int64_t cells = hp.g.cells;
    const unsigned cb = (unsigned)((cells + 255) / 256);
    const unsigned nst = (unsigned)((hp.nspecies * ntiles + 255) / 256);
    const bool gauss = (hp.flags & PIC_FLAG_GAUSS_RESIDUAL) != 0;
    if (gauss) {
        L.grp = 0;
        L(k_rho<R, D, T, false>, dim3(ntiles), dim3(256), dp);
        L(k_gauss<R, D>, dim3(cb), dim3(256), dp);
    }
    L.grp = 0;
    L(k_field_diag<R>, dim3(hp.fd_blocks), dim3(256), dp);
    L.grp = 1;
    const unsigned pbk = (unsigned)shape_block(sizeof(R) == 4, hp.shape);
    if (hp.coulomb) L(particle_kernel<R, A, D, T, true>(hp.shape), dim3(ntiles), dim3(pbk), dp);
    else L(particle_kernel<R, A, D, T, false>(hp.shape), dim3(ntiles), dim3(pbk), dp);
    L.grp = 2;
    L(k_rebin_count, dim3(nst), dim3(256), dp);
    L(k_rebin_count_ovf<R>, dim3(256), dim3(256), dp);
    L(k_rebin_scan, dim3(hp.nspecies), dim3(256), dp);
    // one workgroup per 8 (species, tile) bins, 1024 to 16384 (the copy
    // needs many workgroups in flight; an idle launch costs the same)
    const unsigned scb = (unsigned)std::min<int64_t>(16384, std::max<int64_t>(1024, (int64_t)ntiles * hp.nspecies / 8));
    L(k_rebin_scatter<R>, dim3(scb), dim3(256), dp);
    L(k_rebin_scatter_ovf<R>, dim3(256), dim3(256), dp);
    L(k_rebin_finalize, dim3(nst), dim3(256), dp);
    if (hp.binary) {
        L.grp = 1;
        L(k_binary<R, D, T>, dim3(ntiles), dim3(kBinThreads), dp);
    }
    L.grp = 3;
    L(k_reduce_j<R, D>, dim3(cb), dim3(256), dp);
    if (gauss) {
        L.grp = 0;
        L(k_rho<R, D, T, true>, dim3(ntiles), dim3(256), dp);
        L(k_continuity<R, D>, dim3(cb), dim3(256), dp);
    }
    // frozen fields: the Yee kernels still run (fixed launch shape) but exit
    const double h = (hp.flags & PIC_FLAG_FREEZE_FIELDS) ? 0.0 : 0.5;
    L.grp = 4;
    L(k_yee_b<R, D>, dim3(cb), dim3(256), dp, h);
    L(k_yee_e<R, D>, dim3(cb), dim3(256), dp);
    L(k_yee_b<R, D>, dim3(cb), dim3(256), dp, h);
    L.grp = 5;
    L(k_advance, dim3(1), dim3(kAdvanceThreads), dp);
    return L.dry ? hipSuccess : hipGetLastError();
}

// The tile current is accumulated in FP64 in LDS in both modes: on gfx950 an
// FP32 LDS atomic add (ds_add_f32) measured about 4x slower than the FP64
// one (ds_add_f64) in this kernel (C3: 6.1 ms against 1.6 ms per launch).  The
// partial written to HBM is in the run's precision (FP32 in mixed mode).
template <typename R>
static hipError_t step_prec(const KParams &hp, const KParams *dp, Launcher &L)
{
    using A = double;
    if (hp.g.ndim == 3) {
        if (hp.g.tile[0] == 8) return step_kernels<R, A, 3, 8>(hp, dp, L);
        return hipErrorInvalidValue;
    }
    switch (hp.g.tile[0]) {
    case 8: return step_kernels<R, A, 2, 8>(hp, dp, L);
    case 16: return step_kernels<R, A, 2, 16>(hp, dp, L);
    case 32: return step_kernels<R, A, 2, 32>(hp, dp, L);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const KParams &hp, const KParams *dp, hipStream_t st, hipEvent_t *ev)
{
    Launcher L{st, ev};
    return hp.precision == PIC_PREC_MIXED ? step_prec<float>(hp, dp, L) : step_prec<double>(hp, dp, L);
}

int step_kernel_groups(const KParams &hp, int *groups)
{
    Launcher L{nullptr, nullptr};
    L.groups = groups;
    L.dry = true;
    const hipError_t e = hp.precision == PIC_PREC_MIXED ? step_prec<float>(hp, nullptr, L)
                                                       : step_prec<double>(hp, nullptr, L);
    return e == hipSuccess ? L.k : -1;
}

// The same kernel sequence over a whole ensemble (kBatchKernels launches):
// field diag | particle, one per tile group | 6 x re-layout | J reduction |
// 3 x Yee | advance.
template <typename R, typename A, int D, int T>
static void batch_particle(Launcher &L, const BatchTable &ht, const BatchTable *dt, int pblocks)
{
    constexpr int g = T == 8 ? 0 : (T == 16 ? 1 : 2);
    const unsigned nb = ht.grp[g].n_items > 0 ? (unsigned)std::max(1, pblocks) : 1u;
    const int shape = ht.grp[g].shape;
    const unsigned pbk = (unsigned)shape_block(sizeof(R) == 4, shape);
    if (ht.coulomb) L(batch_particle_kernel<R, A, D, T, true>(shape), dim3(nb), dim3(pbk), dt);
    else L(batch_particle_kernel<R, A, D, T, false>(shape), dim3(nb), dim3(pbk), dt);
}

template <typename R, int D>
static hipError_t batch_kernels(const BatchTable &ht, const BatchTable *dt, const int *pb, hipStream_t st,
                                hipEvent_t *ev)
{
    using A = double;
    const unsigned nr = (unsigned)ht.nruns;
    Launcher L{st, ev};
    L(kb_field_diag<R>, dim3(ht.max_fd_blocks, nr), dim3(256), dt);
    if constexpr (D == 3) {
        batch_particle<R, A, 3, 8>(L, ht, dt, pb[0]);
        // fixed dispatch count: two one-workgroup launches that find the
        // queue of group 0 exhausted and exit (3D has one tile edge)
        batch_particle<R, A, 3, 8>(L, ht, dt, 0);
        batch_particle<R, A, 3, 8>(L, ht, dt, 0);
    } else {
        batch_particle<R, A, 2, 8>(L, ht, dt, pb[0]);
        batch_particle<R, A, 2, 16>(L, ht, dt, pb[1]);
        batch_particle<R, A, 2, 32>(L, ht, dt, pb[2]);
    }
    L(kb_rebin_count, dim3(ht.nst_blocks, nr), dim3(256), dt);
    L(kb_rebin_count_ovf<R>, dim3(kBatchRebinBlocks, nr), dim3(256), dt);
    L(kb_rebin_scan, dim3(ht.max_species, nr), dim3(256), dt);
    L(kb_rebin_scatter<R>, dim3(kBatchRebinBlocks, nr), dim3(256), dt);
    L(kb_rebin_scatter_ovf<R>, dim3(kBatchRebinBlocks, nr), dim3(256), dt);
    L(kb_rebin_finalize, dim3(ht.nst_blocks, nr), dim3(256), dt);
    L(kb_reduce_j<R, D>, dim3(ht.n_cell_blocks), dim3(256), dt);
    L(kb_yee_b<R, D>, dim3(ht.n_cell_blocks), dim3(256), dt, 0.5);
    L(kb_yee_e<R, D>, dim3(ht.n_cell_blocks), dim3(256), dt);
    L(kb_yee_b<R, D>, dim3(ht.n_cell_blocks), dim3(256), dt, 0.5);
    L(kb_advance, dim3(nr), dim3(kAdvanceThreads), dt);
    return hipGetLastError();
}

hipError_t launch_batch_step(int precision, int ndim, const BatchTable &ht, const BatchTable *dt,
                             const int pblocks[kBatchGroups], hipStream_t st, hipEvent_t *ev)
{
    if (ndim == 3) {
        if (ht.grp[1].n_items || ht.grp[2].n_items) return hipErrorInvalidValue;
        return precision == PIC_PREC_MIXED ? batch_kernels<float, 3>(ht, dt, pblocks, st, ev)
                                           : batch_kernels<double, 3>(ht, dt, pblocks, st, ev);
    }
    return precision == PIC_PREC_MIXED ? batch_kernels<float, 2>(ht, dt, pblocks, st, ev)
                                       : batch_kernels<double, 2>(ht, dt, pblocks, st, ev);
}

template <typename R, int D, int T>
static hipError_t occupancy(bool cb, int shape, int *n)
{
    const int bk = shape_block(sizeof(R) == 4, shape);
    return cb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(n, batch_particle_kernel<R, double, D, T, true>(shape), bk, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(n, batch_particle_kernel<R, double, D, T, false>(shape), bk, 0);
}

hipError_t batch_particle_occupancy(int precision, int ndim, int g, bool cb, int shape, int *n)
{
    const bool mx = precision == PIC_PREC_MIXED;
    if (ndim == 3) return mx ? occupancy<float, 3, 8>(cb, shape, n) : occupancy<double, 3, 8>(cb, shape, n);
    switch (g) {
    case 0: return mx ? occupancy<float, 2, 8>(cb, shape, n) : occupancy<double, 2, 8>(cb, shape, n);
    case 1: return mx ? occupancy<float, 2, 16>(cb, shape, n) : occupancy<double, 2, 16>(cb, shape, n);
    case 2: return mx ? occupancy<float, 2, 32>(cb, shape, n) : occupancy<double, 2, 32>(cb, shape, n);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_load_species(const KParams &hp, const KParams *dp, int s, hipStream_t st)
{
    const int T = hp.g.tile[0];
    const int64_t TD = hp.g.ndim == 3 ? (int64_t)T * T * T : (int64_t)T * T;
    const int64_t n = (int64_t)hp.sp[s].ppc * TD * hp.g.ntiles;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (hp.precision == PIC_PREC_MIXED) {
        if (hp.g.ndim == 3) hipLaunchKernelGGL((k_load<float, 3>), dim3(blocks), dim3(256), 0, st, dp, s);
        else hipLaunchKernelGGL((k_load<float, 2>), dim3(blocks), dim3(256), 0, st, dp, s);
    } else {
        if (hp.g.ndim == 3) hipLaunchKernelGGL((k_load<double, 3>), dim3(blocks), dim3(256), 0, st, dp, s);
        else hipLaunchKernelGGL((k_load<double, 2>), dim3(blocks), dim3(256), 0, st, dp, s);
    }
    return hipGetLastError();
}

hipError_t launch_moments(const KParams &hp, const KParams *dp, int s, double delta_uz, hipStream_t st)
{
    if (hp.precision == PIC_PREC_MIXED)
        hipLaunchKernelGGL(k_moments<float>, dim3(kMomentBlocks), dim3(256), 0, st, dp, s, delta_uz);
    else
        hipLaunchKernelGGL(k_moments<double>, dim3(kMomentBlocks), dim3(256), 0, st, dp, s, delta_uz);
    return hipGetLastError();
}

hipError_t launch_shift_u(const KParams &hp, const KParams *dp, int s, double dux, double duy, double duz,
                          hipStream_t st)
{
    if (hp.precision == PIC_PREC_MIXED)
        hipLaunchKernelGGL(k_shift_u<float>, dim3(kMomentBlocks), dim3(256), 0, st, dp, s, dux, duy, duz);
    else
        hipLaunchKernelGGL(k_shift_u<double>, dim3(kMomentBlocks), dim3(256), 0, st, dp, s, dux, duy, duz);
    return hipGetLastError();
}

}  // namespace pic
