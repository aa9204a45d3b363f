// HIP kernels of the beam-plasma PIC step for gfx950 (MI355X).
//
// One step (gather -> Boris push -> move -> Esirkepov deposit -> scattering ->
// current reduction -> Yee update) is a fixed sequence of launches:
//   k_field_diag     FP64 field energies of E^n, B^n on diagnostic steps
//   k_particle_2d    one workgroup per particle tile: E/B staged in LDS,
//                    per-particle gather, push, move, charge-conserving
//                    deposit into an LDS current tile, scattering, and
//                    binning of the particle into the next step's store
//   k_rebin_*        re-layout of the particle store (early exit unless an
//                    incoming-mover reserve overflowed during the step)
//   k_reduce_j_2d    fixed-order FP64 sum of the overlapping tile currents
//   k_yee_b/k_yee_e  B half step, E full step with -J, B half step
//   k_advance        diagnostic record, counter reset, step/parity update
//
// The numerical scheme is the relativistic Boris push (Boris 1970), the
// Esirkepov (2001) charge-conserving deposit with the linear form factor and
// the Yee (1966) FDTD update on the staggered grid
//   Ex(i+1/2,j) Ey(i,j+1/2) Ez(i,j) Bx(i,j+1/2) By(i+1/2,j) Bz(i+1/2,j+1/2),
// half-integer positions stored at the lower integer index, J with E.
// Collisions follow the fluid drag of Eq. (3): each step a collisional
// particle is scattered isotropically off the immobile ions with
// probability 1 - exp(-nu dt), |u| kept.  Units: t in 1/w_p, x in c/w_p,
// u = gamma v/c, fields e F/(m c w_p).
#include <hip/hip_runtime.h>

#include "pic_internal.hpp"

namespace pic {

// Pointers read from the parameter block are generic to the compiler; the
// particle and field arrays are in global memory, and saying so gives global
// (not flat) loads, stores and atomics.
#define GLB __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLB T *gbl(T *p) { return (GLB T *)p; }
template <typename T> __device__ __forceinline__ const GLB T *gbl(const T *p) { return (const GLB T *)p; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ double u01d(uint32_t r) { return ((double)r + 0.5) * 2.3283064365386963e-10; }

// uniform in (0,1) in FP32, exactly representable
__device__ __forceinline__ float u01f(uint32_t r) { return (float)(r >> 8) * 5.9604644775390625e-8f + 2.98023223876953125e-8f; }

template <typename R> struct Arith;
template <> struct Arith<float> {
    static __device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ void sc(float a, float *s, float *c) { sincosf(a, s, c); }
};
template <> struct Arith<double> {
    static __device__ __forceinline__ double rsq(double x) { return 1.0 / sqrt(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ void sc(double a, double *s, double *c) { sincos(a, s, c); }
};

__device__ __forceinline__ bool diag_step(const KParams *kp, int64_t step)
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
__global__ __launch_bounds__(256) void k_field_diag(const KParams *__restrict__ kp)
{
    __shared__ double sred[4][7];
    const int64_t step = kp->state->step;
    if (!diag_step(kp, step)) return;
    const R *F = (const R *)kp->F;
    const int64_t cells = kp->g.cells;
    const int64_t nxy = (int64_t)kp->g.n[0] * kp->g.n[1];
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x; o < cells; o += (int64_t)gridDim.x * 256) {
        double v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            v[c] = (double)F[c * cells + o];
            a[c] += v[c] * v[c];
        }
        int64_t om = o - nxy;
        if (om < 0) om += cells;                      // k-1 (in 2D: the same cell)
        const double by = 0.5 * (v[4] + (double)F[4 * cells + om]);
        const double bx = 0.5 * (v[3] + (double)F[3 * cells + om]);
        a[6] += v[0] * by - v[1] * bx;
    }
    block_sum<7>(a, sred);
    if (threadIdx.x == 0)
        for (int c = 0; c < 7; ++c) kp->field_diag[blockIdx.x * kFieldDiag + c] = a[c];
}

// ---------------------------------------------------------------------------
// The particle kernel (2D3V).  One workgroup per T x T tile.
//
// LDS: E,B on nodes [tx0-1, tx0+T] x [ty0-1, ty0+T] ((T+2)^2 per component)
// and the tile current on nodes [tx0-1, tx0+T+1]^2 ((T+3)^2 per component).
// A particle in cell ix of the tile has local cell lc = ix - tx0 + 1 in both
// arrays.  Its 3-node deposit window per axis is anchored at the nearest
// node (ix or ix+1), which holds the form factor before and after a move
// of less than half a cell.
template <typename R, int T>
__global__ __launch_bounds__(kBlock) void k_particle_2d(const KParams *__restrict__ kp)
{
    constexpr int NF = T + 2;
    constexpr int NJ = T + 3;
    __shared__ R sF[6 * NF * NF];
    __shared__ R sJ[3 * NJ * NJ];
    __shared__ uint32_t s_front;
    __shared__ double sred[kBlock / 64][kTileDiag];

    const int tile = blockIdx.x;
    const int ntx = kp->g.nt[0];
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int ntiles = kp->g.ntiles;
    const int tx0 = (tile % ntx) * T, ty0 = (tile / ntx) * T;
    const int64_t step = kp->state->step;
    const int src = kp->state->par, dst = src ^ 1;
    const bool diag = diag_step(kp, step);
    const int lane = threadIdx.x & 63;
    const uint32_t csh1 = (uint32_t)kp->g.csh[1];
    const uint32_t cmask0 = kp->g.cmask[0];
    const uint32_t seed0 = (uint32_t)kp->seed, seed1 = (uint32_t)(kp->seed >> 32);
    const uint32_t runid = kp->run;
    DevState *state = kp->state;

    {
        const GLB R *F = gbl((const R *)kp->F);
        const int64_t plane = kp->g.cells;
        for (int i = threadIdx.x; i < 6 * NF * NF; i += kBlock) {
            const int c = i / (NF * NF), r = i - c * (NF * NF);
            const int ly = r / NF, lx = r - ly * NF;
            int gx = tx0 - 1 + lx, gy = ty0 - 1 + ly;
            gx += gx < 0 ? nx : 0;
            gx -= gx >= nx ? nx : 0;
            gy += gy < 0 ? ny : 0;
            gy -= gy >= ny ? ny : 0;
            sF[i] = F[c * plane + (int64_t)gy * nx + gx];
        }
        for (int i = threadIdx.x; i < 3 * NJ * NJ; i += kBlock) sJ[i] = R(0);
    }
    __syncthreads();

    const R *sEx = sF, *sEy = sF + NF * NF, *sEz = sF + 2 * NF * NF;
    const R *sBx = sF + 3 * NF * NF, *sBy = sF + 4 * NF * NF, *sBz = sF + 5 * NF * NF;
    R *sJx = sJ, *sJy = sJ + NJ * NJ, *sJz = sJ + 2 * NJ * NJ;

    const R dtdx = R(kp->g.dt / kp->g.d[0]);
    const R dtdy = R(kp->g.dt / kp->g.d[1]);

    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int32_t bstart = S.start[tile], bcap = S.cap[tile];
        const uint32_t nf = S.cnt_front[src * ntiles + tile];
        const uint32_t nb = S.cnt_back[src * ntiles + tile];
        const uint32_t total = nf + nb;
        const R qm = R(S.qmdt2);
        const R kx = R(S.qw * kp->g.d[0] / kp->g.dt);   // q w dx/dt
        const R ky = R(S.qw * kp->g.d[1] / kp->g.dt);
        const R qw = R(S.qw);
        const double wgt = S.w;
        const bool collide = S.collide != 0;
        const bool track = S.track_id != 0;
        const uint32_t thr = S.coll_thr;
        const GLB uint32_t *__restrict__ icell = gbl(S.cell[src]);
        const GLB R *__restrict__ ip0 = gbl((const R *)S.pos[src][0]);
        const GLB R *__restrict__ ip1 = gbl((const R *)S.pos[src][1]);
        const GLB R *__restrict__ iu0 = gbl((const R *)S.u[src][0]);
        const GLB R *__restrict__ iu1 = gbl((const R *)S.u[src][1]);
        const GLB R *__restrict__ iu2 = gbl((const R *)S.u[src][2]);
        const GLB uint32_t *__restrict__ iid = gbl(S.id[src]);
        const GLB int32_t *__restrict__ tstart = gbl(S.start);
        const GLB int32_t *__restrict__ tcap = gbl(S.cap);
        const GLB uint32_t *__restrict__ cf_src = gbl(S.cnt_front + src * ntiles);
        const GLB uint32_t *__restrict__ cb_src = gbl(S.cnt_back + src * ntiles);
        GLB uint32_t *cb_dst = gbl(S.cnt_back + dst * ntiles);

        if (threadIdx.x == 0) s_front = 0;
        __syncthreads();

        double acc[kTileDiag] = {0, 0, 0, 0, 0, 0};
        for (uint32_t base = 0; base < total; base += kBlock) {
            const uint32_t k = base + threadIdx.x;
            const bool active = k < total;
            int ix1 = 0, iy1 = 0, t1 = -1;
            R ox1 = R(0), oy1 = R(0), ux = R(0), uy = R(0), uz = R(0);
            uint32_t pid = 0;
            if (active) {
                const int64_t slot = k < nf ? (int64_t)bstart + k : (int64_t)bstart + bcap - nb + (k - nf);
                int ix, iy;
                R ox, oy;
                if constexpr (sizeof(R) == 4) {
                    const uint32_t c = icell[slot];
                    ix = (int)(c & cmask0);
                    iy = (int)(c >> csh1);
                    ox = ip0[slot];
                    oy = ip1[slot];
                } else {
                    const double X = ip0[slot], Y = ip1[slot];
                    ix = (int)floor(X);
                    iy = (int)floor(Y);
                    ox = X - ix;
                    oy = Y - iy;
                }
                ux = iu0[slot];
                uy = iu1[slot];
                uz = iu2[slot];
                if (track) pid = iid[slot];
                const R uox = ux, uoy = uy, uoz = uz;

                // ---- gather: linear weights at each component's stagger
                const int lcx = ix - tx0 + 1, lcy = iy - ty0 + 1;
                const int hx = ox < R(0.5) ? 1 : 0, hy = oy < R(0.5) ? 1 : 0;
                const R ax1 = ox, ax0 = R(1) - ox;                     // integer x
                const R bx1 = ox - R(0.5) + R(hx), bx0 = R(1) - bx1;   // half x
                const R ay1 = oy, ay0 = R(1) - oy;
                const R by1 = oy - R(0.5) + R(hy), by0 = R(1) - by1;
                const int lhx = lcx - hx, lhy = lcy - hy;
                // (half x, int y): Ex, By
                const int o_hi = lcy * NF + lhx;
                // (int x, half y): Ey, Bx
                const int o_ih = lhy * NF + lcx;
                // (int, int): Ez
                const int o_ii = lcy * NF + lcx;
                // (half, half): Bz
                const int o_hh = lhy * NF + lhx;
                const R Ex = ay0 * (bx0 * sEx[o_hi] + bx1 * sEx[o_hi + 1]) + ay1 * (bx0 * sEx[o_hi + NF] + bx1 * sEx[o_hi + NF + 1]);
                const R By = ay0 * (bx0 * sBy[o_hi] + bx1 * sBy[o_hi + 1]) + ay1 * (bx0 * sBy[o_hi + NF] + bx1 * sBy[o_hi + NF + 1]);
                const R Ey = by0 * (ax0 * sEy[o_ih] + ax1 * sEy[o_ih + 1]) + by1 * (ax0 * sEy[o_ih + NF] + ax1 * sEy[o_ih + NF + 1]);
                const R Bx = by0 * (ax0 * sBx[o_ih] + ax1 * sBx[o_ih + 1]) + by1 * (ax0 * sBx[o_ih + NF] + ax1 * sBx[o_ih + NF + 1]);
                const R Ez = ay0 * (ax0 * sEz[o_ii] + ax1 * sEz[o_ii + 1]) + ay1 * (ax0 * sEz[o_ii + NF] + ax1 * sEz[o_ii + NF + 1]);
                const R Bz = by0 * (bx0 * sBz[o_hh] + bx1 * sBz[o_hh + 1]) + by1 * (bx0 * sBz[o_hh + NF] + bx1 * sBz[o_hh + NF + 1]);

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
                const R vz = uz * ig1;

                // ---- move in cell units, relative to the particle's cell
                const R x1 = ox + ux * ig1 * dtdx;
                const R y1 = oy + uy * ig1 * dtdy;

                // ---- Esirkepov deposit on the 3x3 window around the nearest node
                const int cxa = ox >= R(0.5) ? 1 : 0, cya = oy >= R(0.5) ? 1 : 0;
                const R d0x = ox - R(cxa), d1x = x1 - R(cxa);
                const R d0y = oy - R(cya), d1y = y1 - R(cya);
                const R S0x[3] = {fmax(R(0), -d0x), R(1) - fabs(d0x), fmax(R(0), d0x)};
                const R S0y[3] = {fmax(R(0), -d0y), R(1) - fabs(d0y), fmax(R(0), d0y)};
                const R DSx[3] = {fmax(R(0), -d1x) - S0x[0], R(1) - fabs(d1x) - S0x[1], fmax(R(0), d1x) - S0x[2]};
                const R DSy[3] = {fmax(R(0), -d1y) - S0y[0], R(1) - fabs(d1y) - S0y[1], fmax(R(0), d1y) - S0y[2]};
                const int w0 = (lcy + cya - 1) * NJ + (lcx + cxa - 1);
                const R kzv = qw * vz;
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const R ry = S0y[b] + R(0.5) * DSy[b];
                    const R qy = R(0.5) * S0y[b] + R(1.0 / 3.0) * DSy[b];
                    const R j0 = -kx * (DSx[0] * ry);
                    const R j1 = j0 - kx * (DSx[1] * ry);
                    atomicAdd(&sJx[w0 + b * NJ], j0);
                    atomicAdd(&sJx[w0 + b * NJ + 1], j1);
#pragma unroll
                    for (int a = 0; a < 3; ++a) atomicAdd(&sJz[w0 + b * NJ + a], kzv * (S0x[a] * ry + DSx[a] * qy));
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const R rx = S0x[a] + R(0.5) * DSx[a];
                    const R j0 = -ky * (DSy[0] * rx);
                    const R j1 = j0 - ky * (DSy[1] * rx);
                    atomicAdd(&sJy[w0 + a], j0);
                    atomicAdd(&sJy[w0 + NJ + a], j1);
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
                if (collide) {
                    const uint4 r = philox10(make_uint4(pid, (uint32_t)step, kPurposeCollide, runid), seed0, seed1);
                    if (r.x < thr) {
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

                // ---- new cell and offset
                int kx1 = (int)floor(x1), ky1 = (int)floor(y1);
                ox1 = x1 - R(kx1);
                oy1 = y1 - R(ky1);
                if (ox1 >= R(1)) { ox1 = R(0); kx1 += 1; }
                if (oy1 >= R(1)) { oy1 = R(0); ky1 += 1; }
                ix1 = ix + kx1;
                iy1 = iy + ky1;
                ix1 += ix1 < 0 ? nx : 0;
                ix1 -= ix1 >= nx ? nx : 0;
                iy1 += iy1 < 0 ? ny : 0;
                iy1 -= iy1 >= ny ? ny : 0;
                if ((unsigned)ix1 >= (unsigned)nx || (unsigned)iy1 >= (unsigned)ny) {
                    atomicOr(&state->fatal, 2);
                    ix1 = 0;
                    iy1 = 0;
                }
                t1 = (iy1 >> kp->g.tshift[1]) * ntx + (ix1 >> kp->g.tshift[0]);
            }

            // ---- binning: stayers fill the bin front (wave-aggregated LDS
            // counter), movers take slots from the back of their new tile's
            // bin, above the particles that tile held at the step start.
            const bool stay = active && t1 == tile;
            const uint64_t smask = __ballot(stay);
            int64_t opos = -1;
            if (smask) {
                const int leader = __ffsll((unsigned long long)smask) - 1;
                uint32_t b0 = 0;
                if (lane == leader) b0 = atomicAdd(&s_front, (uint32_t)__popcll(smask));
                b0 = __shfl(b0, leader, 64);
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(smask >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)smask, 0u));
                if (stay) opos = (int64_t)bstart + b0 + rank;
            }
            bool to_ovf = false;
            if (active && !stay) {
                const uint32_t b = __hip_atomic_fetch_add(cb_dst + t1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int64_t room = (int64_t)tcap[t1] - (int64_t)cf_src[t1] - (int64_t)cb_src[t1];
                if ((int64_t)b < room) opos = (int64_t)tstart[t1] + tcap[t1] - 1 - b;
                else to_ovf = true;
            }
            int set = dst;
            if (to_ovf) {
                const uint32_t oi = atomicAdd(&state->ovf_count[s], 1u);
                state->rebin = 1;
                if (oi < S.ovf_cap) { opos = oi; set = 2; }
                else atomicOr(&state->fatal, 1);
            }
            if (opos >= 0) {
                GLB R *op0 = gbl((R *)S.pos[set][0]), *op1 = gbl((R *)S.pos[set][1]);
                GLB R *ou0 = gbl((R *)S.u[set][0]), *ou1 = gbl((R *)S.u[set][1]), *ou2 = gbl((R *)S.u[set][2]);
                if constexpr (sizeof(R) == 4) {
                    gbl(S.cell[set])[opos] = (uint32_t)ix1 | ((uint32_t)iy1 << csh1);
                    op0[opos] = ox1;
                    op1[opos] = oy1;
                } else {
                    op0[opos] = (double)ix1 + ox1;
                    op1[opos] = (double)iy1 + oy1;
                }
                ou0[opos] = ux;
                ou1[opos] = uy;
                ou2[opos] = uz;
                if (track) gbl(S.id[set])[opos] = pid;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) S.cnt_front[dst * ntiles + tile] = s_front;
        if (diag) {
            block_sum<kTileDiag>(acc, sred);
            if (threadIdx.x == 0)
                for (int v = 0; v < kTileDiag; ++v)
                    kp->tile_diag[((int64_t)tile * kp->nspecies + s) * kTileDiag + v] = acc[v];
        }
    }
    __syncthreads();
    GLB R *Jt = gbl((R *)kp->Jtile) + (int64_t)tile * 3 * NJ * NJ;
    for (int i = threadIdx.x; i < 3 * NJ * NJ; i += kBlock) Jt[i] = sJ[i];
}

// ---------------------------------------------------------------------------
// Store re-layout after an overflow of some tile's incoming-mover reserve.
// Data of the step sits in set dst (bins) and set 2 (overflow list); it is
// rewritten into set src with capacities count + a uniform reserve, and the
// parity is kept so that the next step reads set src.
__global__ void k_rebin_count(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!st->rebin) return;
    const int ntiles = kp->g.ntiles;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    int ix, iy;
    if constexpr (sizeof(R) == 4) {
        const uint32_t c = S.cell[set][p];
        ix = (int)(c & kp->g.cmask[0]);
        iy = (int)(c >> kp->g.csh[1]);
    } else {
        ix = (int)floor(((const double *)S.pos[set][0])[p]);
        iy = (int)floor(((const double *)S.pos[set][1])[p]);
    }
    ix = min(max(ix, 0), kp->g.n[0] - 1);
    iy = min(max(iy, 0), kp->g.n[1] - 1);
    return (iy >> kp->g.tshift[1]) * kp->g.nt[0] + (ix >> kp->g.tshift[0]);
}

template <typename R>
__global__ void k_rebin_count_ovf(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!st->rebin) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int64_t n = min((int64_t)st->ovf_count[s], (int64_t)S.ovf_cap);
        for (int64_t p = i; p < n; p += (int64_t)gridDim.x * blockDim.x)
            atomicAdd(&kp->rb_count[(int64_t)s * kp->g.ntiles + tile_of<R>(kp, S, 2, p)], 1);
    }
}

// one block per species: capacities = count + uniform reserve, exclusive scan
__global__ __launch_bounds__(256) void k_rebin_scan(const KParams *__restrict__ kp)
{
    __shared__ int64_t spart[256];
    DevState *st = kp->state;
    if (!st->rebin) return;
    const int s = blockIdx.x;
    const SpeciesDev &S = kp->sp[s];
    const int ntiles = kp->g.ntiles;
    const int32_t *cnt = kp->rb_count + (int64_t)s * ntiles;
    const int chunk = (ntiles + 255) / 256;
    const int t0 = threadIdx.x * chunk, t1 = min(t0 + chunk, ntiles);
    int64_t local = 0;
    for (int t = t0; t < t1; ++t) local += cnt[t];
    spart[threadIdx.x] = local;
    __syncthreads();
    __shared__ int64_t s_total;
    if (threadIdx.x == 0) {
        int64_t run = 0;
        for (int i = 0; i < 256; ++i) { const int64_t v = spart[i]; spart[i] = run; run += v; }
        s_total = run;
    }
    __syncthreads();
    const int64_t reserve = (S.ncap - s_total) / ntiles;
    if (reserve < 0 && threadIdx.x == 0) atomicOr(&st->fatal, 4);
    const int64_t rv = reserve < 0 ? 0 : reserve;
    int64_t off = spart[threadIdx.x] + rv * t0;
    for (int t = t0; t < t1; ++t) {
        kp->rb_start[(int64_t)s * ntiles + t] = (int32_t)off;
        kp->rb_cap[(int64_t)s * ntiles + t] = (int32_t)(cnt[t] + rv);
        off += cnt[t] + rv;
    }
}

template <typename R>
__device__ __forceinline__ void copy_particle(const KParams *kp, const SpeciesDev &S, int from, int64_t a,
                                              int to, int64_t b)
{
    if constexpr (sizeof(R) == 4) S.cell[to][b] = S.cell[from][a];
    for (int c = 0; c < 2; ++c) ((R *)S.pos[to][c])[b] = ((const R *)S.pos[from][c])[a];
    for (int c = 0; c < 3; ++c) ((R *)S.u[to][c])[b] = ((const R *)S.u[from][c])[a];
    if (S.track_id) S.id[to][b] = S.id[from][a];
}

// copy each tile's valid bin contents dst -> src (blocks stride over (tile, species))
template <typename R>
__global__ __launch_bounds__(256) void k_rebin_scatter(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int ntiles = kp->g.ntiles;
    const int src = st->par, dst = src ^ 1;
    for (int pair = blockIdx.x; pair < ntiles * kp->nspecies; pair += gridDim.x) {
        const int s = pair / ntiles, t = pair - s * ntiles;
        const SpeciesDev &S = kp->sp[s];
        const int64_t room = (int64_t)S.cap[t] - S.cnt_front[src * ntiles + t] - S.cnt_back[src * ntiles + t];
        const int64_t nf = S.cnt_front[dst * ntiles + t];
        const int64_t vb = min((int64_t)S.cnt_back[dst * ntiles + t], room);
        const int64_t from0 = S.start[t], cap = S.cap[t];
        const int64_t to0 = kp->rb_start[(int64_t)s * ntiles + t];
        for (int64_t k = threadIdx.x; k < nf + vb; k += blockDim.x) {
            const int64_t a = k < nf ? from0 + k : from0 + cap - vb + (k - nf);
            copy_particle<R>(kp, S, dst, a, src, to0 + k);
        }
    }
}

template <typename R>
__global__ void k_rebin_scatter_ovf(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int src = st->par;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int s = 0; s < kp->nspecies; ++s) {
        const SpeciesDev &S = kp->sp[s];
        const int64_t n = min((int64_t)st->ovf_count[s], (int64_t)S.ovf_cap);
        for (int64_t p = i; p < n; p += (int64_t)gridDim.x * blockDim.x) {
            const int64_t idx = (int64_t)s * kp->g.ntiles + tile_of<R>(kp, S, 2, p);
            const int32_t slot = atomicAdd(&kp->rb_fill[idx], 1);
            copy_particle<R>(kp, S, 2, p, src, (int64_t)kp->rb_start[idx] + slot);
        }
    }
}

__global__ void k_rebin_finalize(const KParams *__restrict__ kp)
{
    const DevState *st = kp->state;
    if (!st->rebin || (st->fatal & 4)) return;
    const int ntiles = kp->g.ntiles;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
template <typename R>
__global__ __launch_bounds__(256) void k_reduce_j_2d(const KParams *__restrict__ kp)
{
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= (int64_t)nx * ny) return;
    const int i = (int)(o % nx), j = (int)(o / nx);
    const int T = kp->g.tile[0];
    const int NJ = kp->nj;
    const int ntx = kp->g.nt[0], nty = kp->g.nt[1];
    const int a0 = i / T, b0 = j / T, ri = i - a0 * T, rj = j - b0 * T;
    const R *Jt = (const R *)kp->Jtile;
    double jx = 0.0, jy = 0.0, jz = 0.0;
    for (int dy = -1; dy <= 1; ++dy) {
        const int ly = rj + 1 - dy * T;
        if (ly < 0 || ly >= NJ) continue;
        int tb = b0 + dy;
        tb += tb < 0 ? nty : 0;
        tb -= tb >= nty ? nty : 0;
        for (int dx = -1; dx <= 1; ++dx) {
            const int lx = ri + 1 - dx * T;
            if (lx < 0 || lx >= NJ) continue;
            int ta = a0 + dx;
            ta += ta < 0 ? ntx : 0;
            ta -= ta >= ntx ? ntx : 0;
            const R *p = Jt + (int64_t)(tb * ntx + ta) * 3 * NJ * NJ + ly * NJ + lx;
            jx += (double)p[0];
            jy += (double)p[NJ * NJ];
            jz += (double)p[2 * NJ * NJ];
        }
    }
    const int64_t cells = kp->g.cells;
    kp->J[o] = jx;
    kp->J[cells + o] = jy;
    kp->J[2 * cells + o] = jz;
}

// ---------------------------------------------------------------------------
// Yee updates (2D: n[2] == 1 and every z difference vanishes).
template <typename R, int NDIM>
__global__ __launch_bounds__(256) void k_yee_b(const KParams *__restrict__ kp, double h)
{
    const int nx = kp->g.n[0], ny = kp->g.n[1], nz = NDIM == 3 ? kp->g.n[2] : 1;
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ __launch_bounds__(256) void k_yee_e(const KParams *__restrict__ kp)
{
    const int nx = kp->g.n[0], ny = kp->g.n[1];
    const int64_t cells = kp->g.cells;
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
__global__ __launch_bounds__(256) void k_advance(const KParams *__restrict__ kp)
{
    __shared__ double sred[4][8];
    DevState *st = kp->state;
    const int64_t step = st->step;
    const int par = st->par;
    const int rebin = st->rebin;
    const int ntiles = kp->g.ntiles;
    const int ns = kp->nspecies;
    if (diag_step(kp, step)) {
        const double dv = kp->g.d[0] * kp->g.d[1] * (kp->g.ndim == 3 ? kp->g.d[2] : 1.0);
        double f[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int b = threadIdx.x; b < kFieldDiagBlocks; b += blockDim.x)
            for (int c = 0; c < 7; ++c) f[c] += kp->field_diag[b * kFieldDiag + c];
        block_sum<8>(f, sred);
        pic_diag rec;
        if (threadIdx.x == 0) {
            for (int c = 0; c < 6; ++c) rec.W[c] = f[c] * dv;
            rec.p_field_z = f[6] * dv;
        }
        double coll_total = 0.0;
        double pp[3] = {0, 0, 0};
        for (int s = 0; s < ns; ++s) {
            double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int t = threadIdx.x; t < ntiles; t += blockDim.x)
                for (int v = 0; v < kTileDiag; ++v) a[v] += kp->tile_diag[((int64_t)t * ns + s) * kTileDiag + v];
            block_sum<8>(a, sred);
            if (threadIdx.x == 0) {
                rec.kinetic[s] = a[0] * dv;
                for (int c = 0; c < 3; ++c) pp[c] += a[1 + c] * dv;
                rec.n_particles[s] = (int64_t)a[4];
                coll_total += a[5];
            }
        }
        if (threadIdx.x == 0) {
            for (int s = ns; s < kMaxSpecies; ++s) { rec.kinetic[s] = 0.0; rec.n_particles[s] = 0; }
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
// Device loader (2D): exactly ppc particles per cell, bins laid out
// tile-major; inside a tile the k-th particle of every cell comes before the
// (k+1)-th of any cell, so the 64 lanes of a wave sit in 64 different cells
// and their current atomics hit different LDS words.  Uniform in-cell
// positions (or a regular sub-lattice) and Gaussian momenta come from
// Philox draws keyed by the particle id.
template <typename R>
__global__ __launch_bounds__(256) void k_load_2d(const KParams *__restrict__ kp, int s)
{
    const SpeciesDev &S = kp->sp[s];
    const int T = kp->g.tile[0];
    const int64_t per_tile = (int64_t)S.ppc * T * T;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= per_tile * kp->g.ntiles) return;
    const int tile = (int)(p / per_tile);
    const int64_t q = p - tile * per_tile;
    const int slot = (int)(q / (T * T)), cl = (int)(q - (int64_t)slot * T * T);
    const int ix = (tile % kp->g.nt[0]) * T + cl % T;
    const int iy = (tile / kp->g.nt[0]) * T + cl / T;
    const uint32_t id = (uint32_t)(S.id_base + ((int64_t)iy * kp->g.n[0] + ix) * S.ppc + slot);
    const uint32_t k0 = (uint32_t)kp->seed, k1 = (uint32_t)(kp->seed >> 32);
    const uint4 r0 = philox10(make_uint4(id, 0u, kPurposeLoad, kp->run), k0, k1);
    const uint4 r1 = philox10(make_uint4(id, 1u, kPurposeLoad, kp->run), k0, k1);
    double ox, oy;
    if (kp->flags & PIC_FLAG_LATTICE_LOAD) {
        int m = (int)rint(sqrt((double)S.ppc));
        ox = (slot % m + 0.5) / m;
        oy = (slot / m + 0.5) / m;
    } else {
        ox = sizeof(R) == 4 ? (double)u01f(r0.x) : u01d(r0.x);
        oy = sizeof(R) == 4 ? (double)u01f(r0.y) : u01d(r0.y);
    }
    // Box-Muller on two pairs of uniforms
    const double ra = sqrt(-2.0 * log(u01d(r1.x))), pa = 6.283185307179586 * u01d(r1.y);
    const double rb = sqrt(-2.0 * log(u01d(r1.z))), pb = 6.283185307179586 * u01d(r1.w);
    const double z[3] = {ra * cos(pa), ra * sin(pa), rb * cos(pb)};
    const int64_t pos = (int64_t)S.start[tile] + q;
    if constexpr (sizeof(R) == 4) {
        S.cell[0][pos] = (uint32_t)ix | ((uint32_t)iy << kp->g.csh[1]);
        ((float *)S.pos[0][0])[pos] = (float)ox;
        ((float *)S.pos[0][1])[pos] = (float)oy;
    } else {
        ((double *)S.pos[0][0])[pos] = (double)ix + ox;
        ((double *)S.pos[0][1])[pos] = (double)iy + oy;
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
// ev (optional): kNumGroups + 1 events recorded at the group boundaries
// field-diag | particle | re-layout | current reduction | Yee | advance.
template <typename R, int T>
static hipError_t step_2d(const KParams &hp, const KParams *dp, hipStream_t st, hipEvent_t *ev)
{
    const int ntiles = hp.g.ntiles;
    const int64_t cells = hp.g.cells;
    const unsigned cb = (unsigned)((cells + 255) / 256);
    const unsigned nst = (unsigned)((hp.nspecies * ntiles + 255) / 256);
    if (ev) (void)hipEventRecord(ev[0], st);
    hipLaunchKernelGGL(k_field_diag<R>, dim3(kFieldDiagBlocks), dim3(256), 0, st, dp);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL((k_particle_2d<R, T>), dim3(ntiles), dim3(kBlock), 0, st, dp);
    if (ev) (void)hipEventRecord(ev[2], st);
    hipLaunchKernelGGL(k_rebin_count, dim3(nst), dim3(256), 0, st, dp);
    hipLaunchKernelGGL(k_rebin_count_ovf<R>, dim3(256), dim3(256), 0, st, dp);
    hipLaunchKernelGGL(k_rebin_scan, dim3(hp.nspecies), dim3(256), 0, st, dp);
    hipLaunchKernelGGL(k_rebin_scatter<R>, dim3(1024), dim3(256), 0, st, dp);
    hipLaunchKernelGGL(k_rebin_scatter_ovf<R>, dim3(256), dim3(256), 0, st, dp);
    hipLaunchKernelGGL(k_rebin_finalize, dim3(nst), dim3(256), 0, st, dp);
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL(k_reduce_j_2d<R>, dim3(cb), dim3(256), 0, st, dp);
    if (ev) (void)hipEventRecord(ev[4], st);
    if (!(hp.flags & PIC_FLAG_FREEZE_FIELDS)) {
        hipLaunchKernelGGL((k_yee_b<R, 2>), dim3(cb), dim3(256), 0, st, dp, 0.5);
        hipLaunchKernelGGL((k_yee_e<R, 2>), dim3(cb), dim3(256), 0, st, dp);
        hipLaunchKernelGGL((k_yee_b<R, 2>), dim3(cb), dim3(256), 0, st, dp, 0.5);
    }
    if (ev) (void)hipEventRecord(ev[5], st);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, st, dp);
    if (ev) (void)hipEventRecord(ev[6], st);
    return hipGetLastError();
}

template <typename R>
static hipError_t step_2d_tile(const KParams &hp, const KParams *dp, hipStream_t st, hipEvent_t *ev)
{
    switch (hp.g.tile[0]) {
    case 8: return step_2d<R, 8>(hp, dp, st, ev);
    case 16: return step_2d<R, 16>(hp, dp, st, ev);
    case 32: return step_2d<R, 32>(hp, dp, st, ev);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step(const KParams &hp, const KParams *dp, hipStream_t st, hipEvent_t *ev)
{
    if (hp.g.ndim != 2) return hipErrorInvalidValue;
    return hp.precision == PIC_PREC_MIXED ? step_2d_tile<float>(hp, dp, st, ev)
                                          : step_2d_tile<double>(hp, dp, st, ev);
}

hipError_t launch_load_species(const KParams &hp, const KParams *dp, int s, hipStream_t st)
{
    const int T = hp.g.tile[0];
    const int64_t n = (int64_t)hp.sp[s].ppc * T * T * hp.g.ntiles;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (hp.precision == PIC_PREC_MIXED)
        hipLaunchKernelGGL(k_load_2d<float>, dim3(blocks), dim3(256), 0, st, dp, s);
    else
        hipLaunchKernelGGL(k_load_2d<double>, dim3(blocks), dim3(256), 0, st, dp, s);
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
