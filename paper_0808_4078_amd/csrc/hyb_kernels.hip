// HIP kernels of the reduced quasi-neutral model (the theory part of the
// paper, Eqs. 1-7), FP64, for gfx950.
//
// A step (time level n): the Eq. (2) solve for a^n from the deposit made at
// x^n (a row transform, then per sweep: column transform + inverse symbol +
// inverse column transform, and the inverse row transform fused with the
// next sweep's row transform); the particle kernel (gather a^n, grad a^n and psi^n at
// x^n, Eq. (6) for u_z, Eq. (4) for u_perp, move, deposit at x^(n+1) with
// the current linearised about a* = 2 a^n - a^(n-1)); the node kernel
// (Eq. (3) for psi, a^n -> a^(n-1) -> a^(n-2), diagnostics, clears); the
// particle sort (every sort_every steps); the bookkeeping kernel.
#include <hip/hip_ext.h>
#include <math.h>

#include "hyb_internal.hpp"

namespace hyb {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) { return i & (n - 1); }   // n a power of two, i >= -n

__device__ __forceinline__ int brev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Sums of NV per-thread values over the workgroup, written to out[0..NV)
// in a fixed order (wave tree, then waves in order).
template <int NV>
__device__ void block_sums(const double *v, double *out)
{
    __shared__ double s[kThreads / 64][NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        const double t = wave_sum(v[k]);
        if (lane == 0) s[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += s[w][threadIdx.x];
        out[threadIdx.x] = t;
    }
}

// Exclusive prefix over the workgroup; *total receives the sum.
__device__ int block_scan_excl(int v, int *total)
{
    __shared__ int ws[kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) ws[wave] = inc;
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) off += ws[w];
        tot += ws[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// ---- cloud-in-cell weights and gathers
struct Cic {
    int i0, i1, j0, j1;
    double ox, oy;
};

// Weights of the point (x, y) on a lattice shifted by (shx, shy) cells.
__device__ __forceinline__ Cic cic(double x, double y, const Params &P, double shx, double shy)
{
    const double fx = x * P.inv_dx - shx, fy = y * P.inv_dy - shy;
    const double flx = floor(fx), fly = floor(fy);
    Cic c;
    c.ox = fx - flx;
    c.oy = fy - fly;
    c.i0 = wrapi((int)flx, P.nx);
    c.i1 = wrapi(c.i0 + 1, P.nx);
    c.j0 = wrapi((int)fly, P.ny);
    c.j1 = wrapi(c.j0 + 1, P.ny);
    return c;
}

// Node addressing of the gathers: the global grid, or a tile's field window
// in LDS (kFw nodes per axis from (wx, wy); node (i, j) of the grid at
// ((j - wy) mod ny) kFw + (i - wx) mod nx, valid for the nodes around a
// particle that lies inside the window).
struct GlobalNodes {
    int nx;
    __device__ __forceinline__ int operator()(int i, int j) const { return j * nx + i; }
};
struct WindowNodes {
    int wx, wy, mx, my;
    __device__ __forceinline__ int operator()(int i, int j) const
    {
        return ((j - wy) & my) * kFw + ((i - wx) & mx);
    }
};

template <typename N>
__device__ __forceinline__ double bilin(const double *__restrict__ F, const Cic &c, const N &at)
{
    return (1 - c.ox) * (1 - c.oy) * F[at(c.i0, c.j0)] + c.ox * (1 - c.oy) * F[at(c.i1, c.j0)] +
           (1 - c.ox) * c.oy * F[at(c.i0, c.j1)] + c.ox * c.oy * F[at(c.i1, c.j1)];
}

// d a/dx at ((i+1/2) dx, j dy), interpolated; c from the lattice shifted by half a cell in x.
template <typename N>
__device__ __forceinline__ double grad_x(const double *__restrict__ a, const Cic &c, const Params &P, const N &at)
{
    const int i0p = wrapi(c.i0 + 1, P.nx), i1p = wrapi(c.i1 + 1, P.nx);
    const double g00 = (a[at(i0p, c.j0)] - a[at(c.i0, c.j0)]) * P.inv_dx;
    const double g10 = (a[at(i1p, c.j0)] - a[at(c.i1, c.j0)]) * P.inv_dx;
    const double g01 = (a[at(i0p, c.j1)] - a[at(c.i0, c.j1)]) * P.inv_dx;
    const double g11 = (a[at(i1p, c.j1)] - a[at(c.i1, c.j1)]) * P.inv_dx;
    return (1 - c.ox) * (1 - c.oy) * g00 + c.ox * (1 - c.oy) * g10 + (1 - c.ox) * c.oy * g01 + c.ox * c.oy * g11;
}

// d a/dy at (i dx, (j+1/2) dy), interpolated; c from the lattice shifted by half a cell in y.
template <typename N>
__device__ __forceinline__ double grad_y(const double *__restrict__ a, const Cic &c, const Params &P, const N &at)
{
    const int j0p = wrapi(c.j0 + 1, P.ny), j1p = wrapi(c.j1 + 1, P.ny);
    const double g00 = (a[at(c.i0, j0p)] - a[at(c.i0, c.j0)]) * P.inv_dy;
    const double g10 = (a[at(c.i1, j0p)] - a[at(c.i1, c.j0)]) * P.inv_dy;
    const double g01 = (a[at(c.i0, j1p)] - a[at(c.i0, c.j1)]) * P.inv_dy;
    const double g11 = (a[at(c.i1, j1p)] - a[at(c.i1, c.j1)]) * P.inv_dy;
    return (1 - c.ox) * (1 - c.oy) * g00 + c.ox * (1 - c.oy) * g10 + (1 - c.ox) * c.oy * g01 + c.ox * c.oy * g11;
}

__device__ __forceinline__ double wrap_pos(double v, double L)
{
    if (v < 0.0) v += L;
    else if (v >= L) v -= L;
    if (v >= L) v = 0.0;
    return v;
}

__device__ __forceinline__ bool sort_step(const Params &P, int64_t step)
{
    return P.sort_every > 0 && step % P.sort_every == P.sort_every - 1;
}

// Sort key of cell (i, j): tile-major, then row and column inside the tile.
__device__ __forceinline__ int sort_key(int i, int j, const Params &P)
{
    const int lt = P.ltile, m = P.tile - 1;
    const int tile = (j >> lt) * P.tiles_x + (i >> lt);
    return (tile << (2 * lt)) + ((j & m) << lt) + (i & m);
}

// The deposit is accumulated in 64-bit fixed point (kDepScale units per
// unit of density or current): each particle's terms are rounded once, and
// every later sum -- in registers, across lanes, in LDS and in the grid --
// is an integer sum, exact in any order.  The deposit, and with it the whole
// run, therefore does not depend on the order in which particles are stored
// or atomics land.  |node value| < 2^15 (far above any density or current of
// this model), rounding 2^-49 per term.
//
// The rounding to an integer: for |x| < 2^51, x + 1.5 * 2^52 lies in
// [2^52, 2^53), where FP64 numbers are the integers, so the addition itself
// rounds x to the nearest integer (ties to even, as llrint) and the low
// mantissa bits hold it: one add and a 64-bit subtract instead of the
// general FP64 -> int64 conversion.  `big` is raised for a term outside
// that range (|v| >= 4; a particle's terms are far smaller), which the
// caller then converts the general way.
__device__ __forceinline__ Fix to_fix_fast(double v, bool &big)
{
    const double x = v * kDepScale;
    big |= !(fabs(x) < 2251799813685248.0);              // 2^51
    return __double_as_longlong(x + 6755399441055744.0) - 0x4338000000000000ll;
}
__device__ __forceinline__ Fix to_fix(double v) { return (Fix)llrint(v * kDepScale); }
__device__ __forceinline__ void fix_add(Fix *p, Fix v)
{
    if (v != 0) atomicAdd((unsigned long long *)p, (unsigned long long)v);
}

// Adds the four quantities acc[k][n] of one cell's run of particles (node n
// of cell (i0, j0)) into the tile's LDS window when the cell lies inside it
// (unconditionally: a run's sums are almost never exactly zero), else
// straight into the global deposit.
__device__ __forceinline__ void flush_run(Fix (*win)[kWin * kWin], Fix *const *dst, const Fix acc[4][4],
                                          int i0, int j0, int wx0, int wy0, const Params &P)
{
    const int di = wrapi(i0 - wx0, P.nx), dj = wrapi(j0 - wy0, P.ny);
    if (di <= kWin - 2 && dj <= kWin - 2) {
        const int e = dj * kWin + di;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            atomicAdd((unsigned long long *)&win[k][e], (unsigned long long)acc[k][0]);
            atomicAdd((unsigned long long *)&win[k][e + 1], (unsigned long long)acc[k][1]);
            atomicAdd((unsigned long long *)&win[k][e + kWin], (unsigned long long)acc[k][2]);
            atomicAdd((unsigned long long *)&win[k][e + kWin + 1], (unsigned long long)acc[k][3]);
        }
    } else {
        const int i1 = wrapi(i0 + 1, P.nx), j1 = wrapi(j0 + 1, P.ny);
        const int off[4] = {j0 * P.nx + i0, j0 * P.nx + i1, j1 * P.nx + i0, j1 * P.nx + i1};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int n = 0; n < 4; ++n) fix_add(dst[k] + off[n], acc[k][n]);
    }
}

// Sums of the 16 deposit terms v over each run of consecutive lanes with
// equal `key`; the last lane of each run (returned true) ends with the run's
// totals.  Segmented inclusive scan toward higher lanes with DPP lane moves
// (no LDS traffic): shifts by 1, 2, 4, 8 within each row of 16 lanes, then
// lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and
// 3.  At each step a lane adds the moved value only if its source lane is in
// the same run (same run index), so lane i ends with the sum over its run's
// lanes up to i.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_int(int v, int old)
{
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ void scan_step(Fix v[16], int sid)
{
    const bool same = dpp_int<CTRL, ROWS>(sid, -1) == sid;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const long long b = v[k];
        const int lo = dpp_int<CTRL, ROWS>((int)(b & 0xffffffffll), 0);
        const int hi = dpp_int<CTRL, ROWS>((int)(b >> 32), 0);
        const Fix o = ((long long)hi << 32) | (unsigned int)lo;
        if (same) v[k] += o;
        __builtin_amdgcn_sched_barrier(0);     // keep the moves of one value at a time live
    }
}

__device__ __forceinline__ bool segment_sums(Fix v[16], int key)
{
    constexpr int kRowShr = 0x110, kRowBcast15 = 0x142, kRowBcast31 = 0x143;
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || prev != key;
    const uint64_t heads = __ballot(head);
    const int sid = __popcll(heads & (~0ull >> (63 - lane)));     // run index of this lane
    scan_step<kRowShr + 1, 0xf>(v, sid);
    scan_step<kRowShr + 2, 0xf>(v, sid);
    scan_step<kRowShr + 4, 0xf>(v, sid);
    scan_step<kRowShr + 8, 0xf>(v, sid);
    scan_step<kRowBcast15, 0xa>(v, sid);
    scan_step<kRowBcast31, 0xc>(v, sid);
    return lane == 63 || ((heads >> (lane + 1)) & 1ull);
}

// Gather at x^n (a, psi at the nodes, grad a at the staggered points),
// Eq. (6) for u_z, Eq. (4) for u_perp, move.  The three stencils share
// nodes: bilinear a on the cell's 4 nodes, d a/dx on 3 columns x the cell's
// 2 rows, d a/dy on the cell's 2 columns x 3 rows -- 8 distinct nodes, each
// loaded once (the staggered lattices' first column / row is the cell's or
// the one before it).
template <typename N>
__device__ __forceinline__ void push_particle(const Params &P, const double *an, const double *ps, const N &at,
                                              double &x, double &y, double &ux, double &uy, double pz, bool diag,
                                              double dacc[kPDiag])
{
    const Cic c = cic(x, y, P, 0.0, 0.0);
    const Cic cx = cic(x, y, P, 0.5, 0.0);
    const Cic cy = cic(x, y, P, 0.0, 0.5);
    const int nx = P.nx, ny = P.ny;
    const double a00 = an[at(c.i0, c.j0)], a10 = an[at(c.i1, c.j0)];
    const double a01 = an[at(c.i0, c.j1)], a11 = an[at(c.i1, c.j1)];
    // x: the staggered lattice starts at the cell's column (hx) or the one before
    const bool hx = cx.i0 == c.i0;
    const int xe = hx ? wrapi(c.i0 + 2, nx) : cx.i0;
    const double e0 = an[at(xe, c.j0)], e1 = an[at(xe, c.j1)];
    const double gA0 = hx ? (a10 - a00) * P.inv_dx : (a00 - e0) * P.inv_dx;
    const double gB0 = hx ? (e0 - a10) * P.inv_dx : (a10 - a00) * P.inv_dx;
    const double gA1 = hx ? (a11 - a01) * P.inv_dx : (a01 - e1) * P.inv_dx;
    const double gB1 = hx ? (e1 - a11) * P.inv_dx : (a11 - a01) * P.inv_dx;
    const bool hy = cy.j0 == c.j0;
    const int ye = hy ? wrapi(c.j0 + 2, ny) : cy.j0;
    const double f0 = an[at(c.i0, ye)], f1 = an[at(c.i1, ye)];
    const double hA0 = hy ? (a01 - a00) * P.inv_dy : (a00 - f0) * P.inv_dy;
    const double hB0 = hy ? (f0 - a01) * P.inv_dy : (a01 - a00) * P.inv_dy;
    const double hA1 = hy ? (a11 - a10) * P.inv_dy : (a10 - f1) * P.inv_dy;
    const double hB1 = hy ? (f1 - a11) * P.inv_dy : (a11 - a10) * P.inv_dy;
    const double abar = (1 - c.ox) * (1 - c.oy) * a00 + c.ox * (1 - c.oy) * a10 + (1 - c.ox) * c.oy * a01 +
                        c.ox * c.oy * a11;
    const double psib = bilin(ps, c, at);
    const double Gx = (1 - cx.ox) * (1 - cx.oy) * gA0 + cx.ox * (1 - cx.oy) * gB0 + (1 - cx.ox) * cx.oy * gA1 +
                      cx.ox * cx.oy * gB1;
    const double Gy = (1 - cy.ox) * (1 - cy.oy) * hA0 + cy.ox * (1 - cy.oy) * hA1 + (1 - cy.ox) * cy.oy * hB0 +
                      cy.ox * cy.oy * hB1;
    const double uz = pz + abar;                                   // Eq. (6)
    const double gm = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    const double f = -(uz * (1.0 / gm) - (psib + abar)) * P.dt;    // Eq. (4)
    ux += f * Gx;
    uy += f * Gy;
    const double gp = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    const double vs = P.dt / gp;
    x = wrap_pos(x + ux * vs, P.Lx);
    y = wrap_pos(y + uy * vs, P.Ly);
    if (!(x >= 0.0 && x < P.Lx && y >= 0.0 && y < P.Ly)) {
        atomicOr(&P.state->fatal, 1);
        x = 0.0;
        y = 0.0;
    }
    if (diag) {
        dacc[0] += P.w * (0.5 * (gm + gp));
        dacc[1] += P.w * (0.5 * abar * abar);
        dacc[2] += P.w * uz;
    }
}

// a* = 2 a^n - a^(n-1) at a particle: from the staged a* plane (LDS window),
// or from the grid node by node (the same arithmetic).
struct StarWindow {
    const double *astar;
    WindowNodes at;
    __device__ __forceinline__ double operator()(const Cic &c) const { return bilin(astar, c, at); }
};
struct StarGrid {
    const double *an, *aold;
    GlobalNodes at;
    __device__ __forceinline__ double node(int i, int j) const { return 2.0 * an[at(i, j)] - aold[at(i, j)]; }
    __device__ __forceinline__ double operator()(const Cic &c) const
    {
        return (1 - c.ox) * (1 - c.oy) * node(c.i0, c.j0) + c.ox * (1 - c.oy) * node(c.i1, c.j0) +
               (1 - c.ox) * c.oy * node(c.i0, c.j1) + c.ox * c.oy * node(c.i1, c.j1);
    }
};

// Deposit terms of a particle at (x, y): n_b, the beam current at a* and its
// linear response (MODE 1: the exact current of u_z = pz; MODE 2 first sets
// p_z = u_z - a^0(x), where a* = a^0).
template <int MODE, typename S>
__device__ __forceinline__ void deposit_terms(const Params &P, const S &star, const Cic &c, double ux, double uy,
                                              double &pz, double v[16])
{
    double beta, chi = 0.0, as = 0.0;
    if (MODE == 1) {
        beta = pz / sqrt(1.0 + ux * ux + uy * uy + pz * pz);
    } else {
        as = star(c);                                                  // a* at the particle
        if (MODE == 2) pz = pz - as;
        const double uzs = pz + as;
        const double up2 = ux * ux + uy * uy;
        const double g = sqrt(1.0 + up2 + uzs * uzs);
        const double rg = 1.0 / g;
        beta = uzs * rg;
        chi = (1.0 + up2) * (rg * rg * rg);
    }
    const double q[4] = {P.w, P.w * beta, P.w * chi, P.w * chi * as};
    const double wt[4] = {(1 - c.ox) * (1 - c.oy), c.ox * (1 - c.oy), (1 - c.ox) * c.oy, c.ox * c.oy};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int n = 0; n < 4; ++n) v[4 * k + n] = q[k] * wt[n];
}

// One workgroup per particle tile: the particles that the last sort placed
// in tile b (they have drifted by less than kMargin cells since, in
// practice).  Thread t takes kRun consecutive particles at a time (a run;
// the lanes' runs are adjacent, so every load instruction of the wave reads
// one contiguous span).  a^n, a^(n-1) and psi on the tile's field window
// (kFw nodes per axis) are staged in LDS for the gathers (a particle outside
// the window gathers from the grid).  The particles are cell-sorted: a run's
// deposit terms are summed in registers while its cell stays the same, then
// summed across consecutive lanes of the same cell, and the last lane of
// each such group adds them to an LDS window of (tile + 2 margin + 1)^2
// nodes, which is added to the global deposit at the end (atomics:
// neighbouring windows overlap).
// MODE 0: one step (gather at x^n, Eqs. (6) and (4), move, deposit at
// x^(n+1)).  MODE 1 (init): deposit the exact current of the given u_z (held
// in the p_z array).  MODE 2 (init): p_z = u_z - a^0(x), then the
// linearised deposit about a^0.
// Two particles per run: longer runs sum more terms in registers but spread
// each load instruction over kRun x 8 bytes per lane (4: +14%, 8: x2.1 at
// the benchmark size); one per run leaves the lane scan to do all merging.
constexpr int kRun = 2;

// (Three waves per SIMD: the register budget that keeps the DPP scan's moves
// from pushing the step kernel to two.)
template <int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_particle(const Params *__restrict__ pp)
{
    __shared__ Fix win[4][kWin * kWin];
    __shared__ double fw[3][kFw * kFw];        // a^n, a* = 2 a^n - a^(n-1), psi on the field window
    const Params &P = *pp;
    const int64_t step = P.state->step;
    const int cur = P.state->cur;
    const bool diag = MODE == 0 && P.diag_every > 0 && step % P.diag_every == 0;
    const int nx = P.nx, ny = P.ny;
    const double *an = MODE == 0 ? P.it[(P.iters - 1) & 1] : P.a1;   // a^n
    const double *aold = MODE == 0 ? P.a1 : P.a2;                     // a^(n-1)
    Fix *const *dst = MODE == 0 ? P.dep[1 - (int)(step & 1)] : P.dep[0];
    double *X = P.x[cur], *Y = P.y[cur], *UX = P.ux[cur], *UY = P.uy[cur], *PZ = P.pz[cur];
    const int b = blockIdx.x;
    const int tx0 = (b % P.tiles_x) << P.ltile, ty0 = (b / P.tiles_x) << P.ltile;
    const int wx0 = tx0 - kMargin, wy0 = ty0 - kMargin;               // deposit window origin
    const int fx0 = tx0 - kMargin - 1, fy0 = ty0 - kMargin - 1;       // field window origin
    for (int e = threadIdx.x; e < 4 * kWin * kWin; e += kThreads) (&win[0][0])[e] = 0;
    if (MODE != 1) {
        for (int e = threadIdx.x; e < kFw * kFw; e += kThreads) {
            const int node = wrapi(fy0 + e / kFw, ny) * nx + wrapi(fx0 + e % kFw, nx);
            fw[0][e] = an[node];
            fw[1][e] = 2.0 * an[node] - aold[node];
            fw[2][e] = MODE == 0 ? P.psi[node] : 0.0;
        }
    }
    __syncthreads();
    const GlobalNodes gn{nx};
    const WindowNodes wn{fx0, fy0, nx - 1, ny - 1};
    const int s0 = P.tile_start[cur][b], s1 = P.tile_start[cur][b + 1];
    double dacc[kPDiag] = {0.0, 0.0, 0.0};
    for (int base = s0; base < s1; base += kThreads * kRun) {
        Fix v[16];
        int key = -1, ci0 = 0, cj0 = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = 0;
        // the next particle's loads are issued before the current one is
        // processed, so they overlap its arithmetic
        const int i0 = base + (int)threadIdx.x * kRun;
        double nx_ = 0.0, ny_ = 0.0, nux = 0.0, nuy = 0.0, npz = 0.0;
        if (i0 < s1) {
            nx_ = X[i0];
            ny_ = Y[i0];
            nux = UX[i0];
            nuy = UY[i0];
            npz = PZ[i0];
        }
#pragma unroll 1
        for (int r = 0; r < kRun; ++r) {
            const int idx = i0 + r;
            if (idx >= s1) break;
            double x = nx_, y = ny_, ux = nux, uy = nuy, pz = npz;
            if (r + 1 < kRun && idx + 1 < s1) {
                nx_ = X[idx + 1];
                ny_ = Y[idx + 1];
                nux = UX[idx + 1];
                nuy = UY[idx + 1];
                npz = PZ[idx + 1];
            }
            if (MODE == 0) {
                const int di = wrapi((int)floor(x * P.inv_dx) - fx0, nx), dj = wrapi((int)floor(y * P.inv_dy) - fy0, ny);
                if (di >= 1 && di <= kFw - 3 && dj >= 1 && dj <= kFw - 3)
                    push_particle(P, fw[0], fw[2], wn, x, y, ux, uy, pz, diag, dacc);
                else
                    push_particle(P, an, P.psi, gn, x, y, ux, uy, pz, diag, dacc);
                X[idx] = x;
                Y[idx] = y;
                UX[idx] = ux;
                UY[idx] = uy;
            }
            const Cic c = cic(x, y, P, 0.0, 0.0);
            double vv[16];
            if (MODE != 1 && wrapi(c.i0 - fx0, nx) <= kFw - 2 && wrapi(c.j0 - fy0, ny) <= kFw - 2)
                deposit_terms<MODE>(P, StarWindow{fw[1], wn}, c, ux, uy, pz, vv);
            else
                deposit_terms<MODE>(P, StarGrid{an, aold, gn}, c, ux, uy, pz, vv);
            if (MODE == 2) PZ[idx] = pz;
            const int k2 = c.j0 * nx + c.i0;
            if (k2 != key) {
                if (key >= 0) flush_run(win, dst, (const Fix(*)[4])v, ci0, cj0, wx0, wy0, P);
                key = k2;
                ci0 = c.i0;
                cj0 = c.j0;
#pragma unroll
                for (int k = 0; k < 16; ++k) v[k] = 0;
            }
            Fix fx[16];
            bool big = false;
#pragma unroll
            for (int k = 0; k < 16; ++k) fx[k] = to_fix_fast(vv[k], big);
            if (big) {
#pragma unroll
                for (int k = 0; k < 16; ++k) fx[k] = to_fix(vv[k]);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] += fx[k];
        }
        if (segment_sums(v, key) && key >= 0) flush_run(win, dst, (const Fix(*)[4])v, ci0, cj0, wx0, wy0, P);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kWin * kWin; e += kThreads) {
        const int node = wrapi(wy0 + e / kWin, ny) * nx + wrapi(wx0 + e % kWin, nx);
#pragma unroll
        for (int k = 0; k < 4; ++k) fix_add(dst[k] + node, win[k][e]);
    }
    if (diag) block_sums<kPDiag>(dacc, P.pdiag + (size_t)b * kPDiag);
}

// ---- Eq. (2): lap a - (n_p + X) a = J - Y + n_p psi, n_p = max(n0 - n_b, 0);
// each sweep solves (lap - c0) a_new = J - Y + n_p psi + (n_p + X - c0) a_old.

// In-place radix-2 decimation-in-time transforms of `batch` sequences of
// length 2^logn stored back to back in LDS, input in bit-reversed order,
// output in natural order; tw[t] = exp(-2 pi i t / 2^logn).
__device__ __forceinline__ double2 cmul(double2 w, double2 v)
{
    return make_double2(w.x * v.x - w.y * v.y, w.x * v.y + w.y * v.x);
}

__device__ __forceinline__ double2 twiddle(const double2 *__restrict__ tw, int t, bool inverse)
{
    double2 w = tw[t];
    if (inverse) w.y = -w.y;
    return w;
}

// Stages are taken two at a time: the four values that two consecutive
// radix-2 stages combine (i, i+h, i+2h, i+3h) are loaded once, both stages'
// butterflies are done in registers with the same arithmetic as one stage
// at a time, and they are stored once -- half the LDS round trips and
// barriers.  An odd stage count ends with one single stage.
__device__ void fft_lds(double2 *z, int logn, int batch, const double2 *__restrict__ tw, bool inverse)
{
    const int n = 1 << logn;
    int s = 1;
    for (; s + 1 <= logn; s += 2) {
        const int h = 1 << (s - 1);
        const int qn = n >> 2;
        const int total = batch * qn;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int b = e >> (logn - 2);
            const int k = e & (qn - 1);
            const int pos = k & (h - 1);
            const int i = ((k >> (s - 1)) << (s + 1)) + pos;
            double2 *zb = z + b * n;
            const double2 w1 = twiddle(tw, pos << (logn - s), inverse);
            const double2 w2 = twiddle(tw, pos << (logn - s - 1), inverse);
            const double2 w3 = twiddle(tw, (pos + h) << (logn - s - 1), inverse);
            const double2 a0 = zb[i], a1 = zb[i + h], a2 = zb[i + 2 * h], a3 = zb[i + 3 * h];
            // stage s: (i, i+h) and (i+2h, i+3h)
            const double2 t1 = cmul(w1, a1), t3 = cmul(w1, a3);
            const double2 b0 = make_double2(a0.x + t1.x, a0.y + t1.y), b1 = make_double2(a0.x - t1.x, a0.y - t1.y);
            const double2 b2 = make_double2(a2.x + t3.x, a2.y + t3.y), b3 = make_double2(a2.x - t3.x, a2.y - t3.y);
            // stage s+1: (i, i+2h) and (i+h, i+3h)
            const double2 u2 = cmul(w2, b2), u3 = cmul(w3, b3);
            zb[i] = make_double2(b0.x + u2.x, b0.y + u2.y);
            zb[i + 2 * h] = make_double2(b0.x - u2.x, b0.y - u2.y);
            zb[i + h] = make_double2(b1.x + u3.x, b1.y + u3.y);
            zb[i + 3 * h] = make_double2(b1.x - u3.x, b1.y - u3.y);
        }
        __syncthreads();
    }
    if (s == logn) {
        const int half = 1 << (s - 1);
        const int hn = n >> 1;
        const int total = batch * hn;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int b = e >> (logn - 1);
            const int k = e & (hn - 1);
            const int pos = k & (half - 1);
            const int i1 = ((k >> (s - 1)) << s) + pos;
            double2 *zb = z + b * n;
            const double2 w = twiddle(tw, pos << (logn - s), inverse);
            const double2 u = zb[i1], v = cmul(w, zb[i1 + half]);
            zb[i1] = make_double2(u.x + v.x, u.y + v.y);
            zb[i1 + half] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// First sweep's row transform (one workgroup per row): the step's
// coefficients R = J - Y + n_p psi and C = n_p + X - c0 are stored for the
// later sweeps, and the right-hand side R + C a^(0), a^(0) = 2 a^(n-1) -
// a^(n-2), is transformed along x.
__global__ __launch_bounds__(kThreads) void k_rows_first(const Params *__restrict__ pp)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int j = blockIdx.x, nx = P.nx;
    const int p = (int)(P.state->step & 1);
    const Fix *nb = P.dep[p][0], *J = P.dep[p][1], *Xc = P.dep[p][2], *Yc = P.dep[p][3];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const int64_t o = (int64_t)j * nx + i;
        const double ap = 2.0 * P.a1[o] - P.a2[o];
        const double n_p = fmax(P.n0 - (double)nb[o] * kDepUnit, 0.0);
        const double c = n_p + (double)Xc[o] * kDepUnit;
        const double R = (double)J[o] * kDepUnit - (double)Yc[o] * kDepUnit + n_p * P.psi[o];
        const double C = c - P.c0;
        P.rhsR[o] = R;
        P.rhsC[o] = C;
        z[brev(i, P.lx)] = make_double2(R + C * ap, 0.0);
    }
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, false);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) P.W[(int64_t)j * nx + i] = z[i];
}

// Between sweeps (one workgroup per row): the inverse row transform gives
// the sweep's result a, from which the next right-hand side R + C a is
// transformed along x, without a round trip of a through memory.
__global__ __launch_bounds__(kThreads) void k_rows_mid(const Params *__restrict__ pp)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int j = blockIdx.x, nx = P.nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) z[brev(i, P.lx)] = P.W[(int64_t)j * nx + i];
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, true);
    const double s = 1.0 / (double)P.cells;
    double v[kFftLds / kThreads];
    int m = 0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x, ++m) {
        const int64_t o = (int64_t)j * nx + i;
        v[m] = P.rhsR[o] + P.rhsC[o] * (z[i].x * s);
    }
    __syncthreads();
    m = 0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x, ++m) z[brev(i, P.lx)] = make_double2(v[m], 0.0);
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, false);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) P.W[(int64_t)j * nx + i] = z[i];
}

// Column transform, division by the symbol -(4/dx^2) sin^2 - (4/dy^2) sin^2 - c0,
// inverse column transform (cols_per_block columns per workgroup).
__global__ __launch_bounds__(kColThreads) void k_cols(const Params *__restrict__ pp)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int CB = P.cols_per_block, ny = P.ny, nx = P.nx, ly = P.ly;
    // Workgroups go to the 8 XCDs in turn, and a row's CB values fill only
    // part of a 128-byte line: consecutive workgroups on one XCD take
    // neighbouring column groups, so both halves of a line are fetched into
    // the same L2 (a bijection of the groups when the count divides by 8).
    const int nbk = (int)gridDim.x, bk = (int)blockIdx.x;
    const int grp = (nbk & 7) ? bk : (bk & 7) * (nbk >> 3) + (bk >> 3);
    const int c0 = grp * CB;
    for (int e = threadIdx.x; e < CB * ny; e += blockDim.x) {
        const int c = e & (CB - 1), j = e / CB;
        z[c * ny + brev(j, ly)] = P.W[(int64_t)j * nx + c0 + c];
    }
    __syncthreads();
    fft_lds(z, ly, CB, P.twy, false);
    // scale, writing each value to its bit-reversed slot for the inverse pass
    for (int e = threadIdx.x; e < CB * ny; e += blockDim.x) {
        const int c = e >> ly, k = e & (ny - 1);
        const int r = brev(k, ly);
        if (k <= r) {
            const double lxv = P.lapx[c0 + c];
            const double sk = 1.0 / (-(lxv + P.lapy[k]) - P.c0);
            const double sr = 1.0 / (-(lxv + P.lapy[r]) - P.c0);
            const double2 vk = z[c * ny + k], vr = z[c * ny + r];
            z[c * ny + r] = make_double2(vk.x * sk, vk.y * sk);
            z[c * ny + k] = make_double2(vr.x * sr, vr.y * sr);
        }
    }
    __syncthreads();
    fft_lds(z, ly, CB, P.twy, true);
    for (int e = threadIdx.x; e < CB * ny; e += blockDim.x) {
        const int c = e & (CB - 1), j = e / CB;
        P.W[(int64_t)j * nx + c0 + c] = z[c * ny + j];
    }
}

// Last sweep's inverse row transform; the real part / (nx ny) is a^n.
__global__ __launch_bounds__(kThreads) void k_rows_inv(const Params *__restrict__ pp)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int j = blockIdx.x, nx = P.nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) z[brev(i, P.lx)] = P.W[(int64_t)j * nx + i];
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, true);
    const double s = 1.0 / (double)P.cells;
    double *out = P.it[(P.iters - 1) & 1];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) out[(int64_t)j * nx + i] = z[i].x * s;
}

// ---- node update after the particle kernel: Eq. (3), a history, clears, diagnostics
__global__ __launch_bounds__(kThreads) void k_nodes(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    const int64_t step = P.state->step;
    const int p = (int)(step & 1);
    const bool diag = P.diag_every > 0 && step % P.diag_every == 0;
    const double *an = P.it[(P.iters - 1) & 1];
    double acc[kGDiag] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < P.cells; o += (int64_t)gridDim.x * kThreads) {
        const double a = an[o];
        const double ps = P.psi[o];
        const double a_old = P.a1[o];
        if (diag) {
            const int i = (int)(o & (P.nx - 1)), j = (int)(o >> P.lx);
            const double gx = (an[(int64_t)j * P.nx + wrapi(i + 1, P.nx)] - a) / P.dx;
            const double gy = (an[(int64_t)wrapi(j + 1, P.ny) * P.nx + i] - a) / P.dy;
            acc[0] += gx * gx + gy * gy;
            acc[1] += a * a;
            const double et = (a - a_old) / P.dt;
            acc[2] += et * et;
            acc[3] += a;
            acc[4] += ps;
        }
        P.psi[o] = ps - P.nu * P.dt * (ps + a);       // Eq. (3)
        P.a2[o] = a_old;
        P.a1[o] = a;
#pragma unroll
        for (int k = 0; k < 4; ++k) P.dep[p][k][o] = 0;
        P.cell_count[o] = 0;
    }
    if (diag) block_sums<kGDiag>(acc, P.gdiag + (size_t)blockIdx.x * kGDiag);
}

// a^(n-1) = a^(n-2) = the initial solve; clear the exact deposit.
__global__ __launch_bounds__(kThreads) void k_init_nodes(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    const double *an = P.it[(P.iters - 1) & 1];
    for (int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x; o < P.cells; o += (int64_t)gridDim.x * kThreads) {
        P.a1[o] = an[o];
        P.a2[o] = an[o];
#pragma unroll
        for (int k = 0; k < 4; ++k) P.dep[0][k][o] = 0;
    }
}

// ---- counting sort of the particles by sort key (tile-major cell order)
// into the other particle set.  Runs every sort_every steps (tile kernels
// below) and once at initialisation (`force`: the particles are in input
// order, so the count and scatter run over the whole array).
__device__ __forceinline__ bool sorting(const Params &P, int force)
{
    return force || sort_step(P, P.state->step);
}

__device__ __forceinline__ int key_of(double x, double y, const Params &P)
{
    return sort_key(wrapi((int)floor(x * P.inv_dx), P.nx), wrapi((int)floor(y * P.inv_dy), P.ny), P);
}

// Each valid lane adds 1 to ctr[key]; lanes of the wave with equal keys add
// together through one atomic by their leader (the particles are nearly in
// key order, so a wave holds few keys).  Returns the counter's value before
// the lane's own increment (its slot).
__device__ int wave_key_add(int *ctr, bool valid, int key)
{
    const int lane = threadIdx.x & 63;
    uint64_t pend = __ballot(valid);
    int slot = -1, rounds = 0;
    while (pend) {
        if (rounds == kWaveRounds) {
            if ((pend >> lane) & 1ull) slot = atomicAdd(ctr + key, 1);
            break;
        }
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int lk = __shfl(key, leader, 64);
        const uint64_t grp = __ballot(((pend >> lane) & 1ull) && key == lk);
        int base = 0;
        if (lane == leader) base = atomicAdd(ctr + lk, __popcll(grp));
        base = __shfl(base, leader, 64);
        if ((grp >> lane) & 1ull) slot = base + __popcll(grp & ((1ull << lane) - 1ull));
        pend &= ~grp;
        ++rounds;
    }
    return slot;
}

__global__ __launch_bounds__(kThreads) void k_sort_count(const Params *__restrict__ pp, int force)
{
    const Params &P = *pp;
    if (!sorting(P, force)) return;
    const int cur = P.state->cur;
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < P.np; base += (int64_t)gridDim.x * kThreads) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < P.np;
        const int key = valid ? key_of(P.x[cur][i], P.y[cur][i], P) : 0;
        (void)wave_key_add(P.cell_count, valid, key);
    }
}

__global__ __launch_bounds__(kThreads) void k_scan_chunks(const Params *__restrict__ pp, int force)
{
    const Params &P = *pp;
    if (!sorting(P, force)) return;
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    int s = 0;
    for (int k = threadIdx.x; k < kScanChunk; k += kThreads)
        if (b0 + k < P.cells) s += P.cell_count[b0 + k];
    int tot;
    (void)block_scan_excl(s, &tot);
    if (threadIdx.x == 0) P.scan_part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(const Params *__restrict__ pp, int nchunks, int force)
{
    const Params &P = *pp;
    if (!sorting(P, force)) return;
    const int per = (nchunks + kThreads - 1) / kThreads;
    const int b = threadIdx.x * per;
    int s = 0;
    for (int k = 0; k < per; ++k)
        if (b + k < nchunks) s += P.scan_part[b + k];
    int tot;
    int run = block_scan_excl(s, &tot);
    for (int k = 0; k < per; ++k)
        if (b + k < nchunks) {
            const int v = P.scan_part[b + k];
            P.scan_part[b + k] = run;
            run += v;
        }
    if (threadIdx.x == 0) P.tile_start[P.state->cur ^ 1][P.ntiles] = (int)P.np;
}

// Exclusive prefix of the counts: the scatter cursor of each key, and the
// first particle of each tile.
__global__ __launch_bounds__(kThreads) void k_scan_apply(const Params *__restrict__ pp, int force)
{
    const Params &P = *pp;
    if (!sorting(P, force)) return;
    constexpr int per = kScanChunk / kThreads;
    const int64_t b = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * per;
    const int tmask = (1 << (2 * P.ltile)) - 1;
    const int nxt = P.state->cur ^ 1;
    int v[per];
    int s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = b + k < P.cells ? P.cell_count[b + k] : 0;
        s += v[k];
    }
    int tot;
    int run = block_scan_excl(s, &tot) + P.scan_part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < per; ++k)
        if (b + k < P.cells) {
            P.cell_start[b + k] = run;
            if (((b + k) & tmask) == 0) P.tile_start[nxt][(b + k) >> (2 * P.ltile)] = run;
            run += v[k];
        }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const Params *__restrict__ pp, int force)
{
    const Params &P = *pp;
    if (!sorting(P, force)) return;
    const int s = P.state->cur, d = s ^ 1;
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < P.np; base += (int64_t)gridDim.x * kThreads) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < P.np;
        double x = 0.0, y = 0.0;
        int key = 0;
        if (valid) {
            x = P.x[s][i];
            y = P.y[s][i];
            key = key_of(x, y, P);
        }
        const int slot = wave_key_add(P.cell_start, valid, key);
        if (valid) {
            P.x[d][slot] = x;
            P.y[d][slot] = y;
            P.ux[d][slot] = P.ux[s][i];
            P.uy[d][slot] = P.uy[s][i];
            P.pz[d][slot] = P.pz[s][i];
            P.id[d][slot] = P.id[s][i];
        }
    }
}

// The regular sort, one workgroup per tile over the particles of the tile's
// current range (they lie within its kWinC^2-cell window, apart from rare
// stragglers).  Count: an LDS histogram of the window's cells, added to the
// global counts; the histogram is kept per tile for the scatter.
__device__ __forceinline__ int tile_bin(double x, double y, int wcx, int wcy, const Params &P, int *key)
{
    const int i = wrapi((int)floor(x * P.inv_dx), P.nx), j = wrapi((int)floor(y * P.inv_dy), P.ny);
    *key = sort_key(i, j, P);
    const int di = wrapi(i - wcx, P.nx), dj = wrapi(j - wcy, P.ny);
    return di < kWinC && dj < kWinC ? dj * kWinC + di : -1;
}

// Lanes with equal bins add together (one LDS atomic per bin per wave);
// returns the bin's count before the lane's own increment.
__device__ int wave_lds_add(int *cnt, bool valid, int bin)
{
    const int lane = threadIdx.x & 63;
    uint64_t pend = __ballot(valid);
    int slot = -1;
    while (pend) {
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int lb = __shfl(bin, leader, 64);
        const uint64_t grp = __ballot(((pend >> lane) & 1ull) && bin == lb);
        int base = 0;
        if (lane == leader) base = atomicAdd(cnt + lb, __popcll(grp));
        base = __shfl(base, leader, 64);
        if ((grp >> lane) & 1ull) slot = base + __popcll(grp & ((1ull << lane) - 1ull));
        pend &= ~grp;
    }
    return slot;
}

__global__ __launch_bounds__(kThreads) void k_sort_count_tiles(const Params *__restrict__ pp)
{
    __shared__ int hist[kWinC * kWinC];
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    const int cur = P.state->cur, b = blockIdx.x;
    const int wcx = ((b % P.tiles_x) << P.ltile) - kMargin, wcy = ((b / P.tiles_x) << P.ltile) - kMargin;
    for (int e = threadIdx.x; e < kWinC * kWinC; e += kThreads) hist[e] = 0;
    __syncthreads();
    const int s0 = P.tile_start[cur][b], s1 = P.tile_start[cur][b + 1];
    const double *X = P.x[cur], *Y = P.y[cur];
    // each thread's next particle is loaded while the current one is binned
    double nx_ = 0.0, ny_ = 0.0;
    if (s0 + (int)threadIdx.x < s1) {
        nx_ = X[s0 + threadIdx.x];
        ny_ = Y[s0 + threadIdx.x];
    }
    for (int base = s0; base < s1; base += kThreads) {
        const int i = base + (int)threadIdx.x;
        const bool valid = i < s1;
        const double x = nx_, y = ny_;
        if (i + kThreads < s1) {
            nx_ = X[i + kThreads];
            ny_ = Y[i + kThreads];
        }
        int key = 0, bin = -1;
        if (valid) bin = tile_bin(x, y, wcx, wcy, P, &key);
        if (valid && bin < 0) atomicAdd(P.cell_count + key, 1);
        (void)wave_lds_add(hist, valid && bin >= 0, bin);
    }
    __syncthreads();
    int *keep = P.bins + (size_t)b * kWinC * kWinC;
    for (int e = threadIdx.x; e < kWinC * kWinC; e += kThreads) {
        const int c = hist[e];
        keep[e] = c;
        if (c) atomicAdd(P.cell_count + sort_key(wrapi(wcx + e % kWinC, P.nx), wrapi(wcy + e / kWinC, P.ny), P), c);
    }
}

// Scatter: each non-empty bin reserves its range of its cell's slots with one
// atomic; particles take consecutive slots of their bin's range.
__global__ __launch_bounds__(kThreads) void k_sort_scatter_tiles(const Params *__restrict__ pp)
{
    __shared__ int hbase[kWinC * kWinC];
    __shared__ int hcur[kWinC * kWinC];
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    const int s = P.state->cur, d = s ^ 1, b = blockIdx.x;
    const int wcx = ((b % P.tiles_x) << P.ltile) - kMargin, wcy = ((b / P.tiles_x) << P.ltile) - kMargin;
    const int *keep = P.bins + (size_t)b * kWinC * kWinC;
    for (int e = threadIdx.x; e < kWinC * kWinC; e += kThreads) {
        const int c = keep[e];
        hbase[e] = c ? atomicAdd(P.cell_start + sort_key(wrapi(wcx + e % kWinC, P.nx), wrapi(wcy + e / kWinC, P.ny), P), c)
                     : 0;
        hcur[e] = 0;
    }
    __syncthreads();
    const int s0 = P.tile_start[s][b], s1 = P.tile_start[s][b + 1];
    const double *X = P.x[s], *Y = P.y[s], *UX = P.ux[s], *UY = P.uy[s], *PZ = P.pz[s];
    const uint32_t *ID = P.id[s];
    // each thread's next particle is loaded while the current one is placed
    struct Part {
        double x, y, ux, uy, pz;
        uint32_t id;
    };
    auto load = [&](int i) { return Part{X[i], Y[i], UX[i], UY[i], PZ[i], ID[i]}; };
    Part nxt{};
    if (s0 + (int)threadIdx.x < s1) nxt = load(s0 + (int)threadIdx.x);
    for (int base = s0; base < s1; base += kThreads) {
        const int i = base + (int)threadIdx.x;
        const bool valid = i < s1;
        const Part q = nxt;
        if (i + kThreads < s1) nxt = load(i + kThreads);
        int key = 0, bin = -1;
        if (valid) bin = tile_bin(q.x, q.y, wcx, wcy, P, &key);
        const int rank = wave_lds_add(hcur, valid && bin >= 0, bin);
        if (valid) {
            const int slot = bin >= 0 ? hbase[bin] + rank : atomicAdd(P.cell_start + key, 1);
            P.x[d][slot] = q.x;
            P.y[d][slot] = q.y;
            P.ux[d][slot] = q.ux;
            P.uy[d][slot] = q.uy;
            P.pz[d][slot] = q.pz;
            P.id[d][slot] = q.id;
        }
    }
}

// The sorted set becomes the current one.
__global__ void k_sort_finish(const Params *__restrict__ pp, int force)
{
    const Params &P = *pp;
    if (threadIdx.x == 0 && sorting(P, force)) P.state->cur ^= 1;
}

// ---- bookkeeping: the diagnostic record (fixed-order sums) and the step counter.
__global__ __launch_bounds__(kThreads) void k_advance(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    State *S = P.state;
    const int64_t step = S->step;
    const bool diag = P.diag_every > 0 && step % P.diag_every == 0;
    if (diag) {
        __shared__ double part[kThreads][kPDiag + kGDiag];
        double s[kPDiag + kGDiag] = {};
        for (int b = threadIdx.x; b < P.ntiles; b += kThreads)
            for (int k = 0; k < kPDiag; ++k) s[k] += P.pdiag[(size_t)b * kPDiag + k];
        for (int b = threadIdx.x; b < kGridBlocks; b += kThreads)
            for (int k = 0; k < kGDiag; ++k) s[kPDiag + k] += P.gdiag[(size_t)b * kGDiag + k];
        for (int k = 0; k < kPDiag + kGDiag; ++k) part[threadIdx.x][k] = s[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[kPDiag + kGDiag] = {};
            for (int i = 0; i < kThreads; ++i)
                for (int k = 0; k < kPDiag + kGDiag; ++k) t[k] += part[i][k];
            pic_hyb_diag r;
            r.step = step;
            r.time = (double)step * P.dt;
            r.beam_energy = P.dA * t[0];
            r.beam_a2 = P.dA * t[1];
            r.beam_pz = P.dA * t[2];
            r.grad_energy = 0.5 * P.dA * t[3];
            r.a2_energy = 0.5 * P.dA * P.n0 * t[4];
            r.W_Bperp = P.dA * t[3];
            r.W_Ez = P.dA * t[5];
            r.mean_a = t[6] / (double)P.cells;
            r.mean_psi = t[7] / (double)P.cells;
            r.eq7 = r.beam_energy - r.beam_a2 + r.grad_energy + r.a2_energy;
            P.ring[S->ring_head] = r;
            S->ring_head = (S->ring_head + 1) % kRing;
            S->ring_count = S->ring_count < kRing ? S->ring_count + 1 : kRing;
        }
    }
    if (threadIdx.x == 0) S->step = step + 1;
}

struct Launcher {
    hipStream_t st;
    hipEvent_t *ev;
    int *groups;
    int k = 0;
    template <typename... KArgs, typename... A>
    void operator()(int group, void (*kern)(KArgs...), dim3 g, dim3 b, size_t lds, A... args)
    {
        if (ev) hipExtLaunchKernelGGL(kern, g, b, lds, st, ev[2 * k], ev[2 * k + 1], 0, args...);
        else hipLaunchKernelGGL(kern, g, b, lds, st, args...);
        if (groups) groups[k] = group;
        ++k;
    }
};

void solve(Launcher &L, const Params &hp, const Params *dp)
{
    const size_t row_lds = sizeof(double2) * (size_t)hp.nx;
    const size_t col_lds = sizeof(double2) * (size_t)hp.cols_per_block * hp.ny;
    L(0, k_rows_first, dim3(hp.ny), dim3(kThreads), row_lds, dp);
    for (int it = 0; it < hp.iters; ++it) {
        L(0, k_cols, dim3(hp.nx / hp.cols_per_block), dim3(kColThreads), col_lds, dp);
        if (it + 1 < hp.iters) L(0, k_rows_mid, dim3(hp.ny), dim3(kThreads), row_lds, dp);
    }
    L(0, k_rows_inv, dim3(hp.ny), dim3(kThreads), row_lds, dp);
}

int scan_chunks(const Params &hp) { return (int)((hp.cells + kScanChunk - 1) / kScanChunk); }

void sort(Launcher &L, const Params &hp, const Params *dp, int force)
{
    const int nch = scan_chunks(hp);
    if (force) L(3, k_sort_count, dim3(kPartBlocks), dim3(kThreads), 0, dp, force);
    else L(3, k_sort_count_tiles, dim3(hp.ntiles), dim3(kThreads), 0, dp);
    L(3, k_scan_chunks, dim3(nch), dim3(kThreads), 0, dp, force);
    L(3, k_scan_top, dim3(1), dim3(kThreads), 0, dp, nch, force);
    L(3, k_scan_apply, dim3(nch), dim3(kThreads), 0, dp, force);
    if (force) L(3, k_sort_scatter, dim3(kPartBlocks), dim3(kThreads), 0, dp, force);
    else L(3, k_sort_scatter_tiles, dim3(hp.ntiles), dim3(kThreads), 0, dp);
    L(3, k_sort_finish, dim3(1), dim3(64), 0, dp, force);
}

}  // namespace

hipError_t launch_init(const Params &hp, const Params *dp, hipStream_t st)
{
    Launcher L{st, nullptr, nullptr};
    sort(L, hp, dp, 1);
    L(0, k_particle<1>, dim3(hp.ntiles), dim3(kThreads), 0, dp);
    solve(L, hp, dp);
    L(0, k_init_nodes, dim3(kGridBlocks), dim3(kThreads), 0, dp);
    L(0, k_particle<2>, dim3(hp.ntiles), dim3(kThreads), 0, dp);
    return hipGetLastError();
}

int step_launches(const Params &hp) { return 2 * hp.iters + 1 + 9; }

hipError_t launch_step(const Params &hp, const Params *dp, hipStream_t st, hipEvent_t *ev, int *groups, int *nlaunch)
{
    Launcher L{st, ev, groups};
    solve(L, hp, dp);
    L(1, k_particle<0>, dim3(hp.ntiles), dim3(kThreads), 0, dp);
    L(2, k_nodes, dim3(kGridBlocks), dim3(kThreads), 0, dp);
    sort(L, hp, dp, 0);
    L(3, k_advance, dim3(1), dim3(kThreads), 0, dp);
    if (nlaunch) *nlaunch = L.k;
    return hipGetLastError();
}

}  // namespace hyb
