// HIP kernels of the reduced quasi-neutral model (the theory part of the
// paper, Eqs. 1-7), FP64, for gfx950.
//
// A step (time level n): the Eq. (2) solve for a^n from the deposit made at
// x^n (iters x [row FFT, column FFT + inverse symbol + inverse column FFT,
// inverse row FFT]); the particle kernel (gather a^n, grad a^n and psi^n at
// x^n, Eq. (6) for u_z, Eq. (4) for u_perp, move, deposit at x^(n+1) with
// the current linearised about a* = 2 a^n - a^(n-1)); the node kernel
// (Eq. (3) for psi, a^n -> a^(n-1) -> a^(n-2), diagnostics, clears); the
// cell sort (every sort_every steps); the bookkeeping kernel.
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
    const double fx = x / P.dx - shx, fy = y / P.dy - shy;
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

__device__ __forceinline__ double bilin(const double *__restrict__ F, const Cic &c, int nx)
{
    return (1 - c.ox) * (1 - c.oy) * F[c.j0 * nx + c.i0] + c.ox * (1 - c.oy) * F[c.j0 * nx + c.i1] +
           (1 - c.ox) * c.oy * F[c.j1 * nx + c.i0] + c.ox * c.oy * F[c.j1 * nx + c.i1];
}

// d a/dx at ((i+1/2) dx, j dy), interpolated; c from the lattice shifted by half a cell in x.
__device__ __forceinline__ double grad_x(const double *__restrict__ a, const Cic &c, const Params &P)
{
    const int nx = P.nx;
    const int i0p = wrapi(c.i0 + 1, nx), i1p = wrapi(c.i1 + 1, nx);
    const double g00 = (a[c.j0 * nx + i0p] - a[c.j0 * nx + c.i0]) / P.dx;
    const double g10 = (a[c.j0 * nx + i1p] - a[c.j0 * nx + c.i1]) / P.dx;
    const double g01 = (a[c.j1 * nx + i0p] - a[c.j1 * nx + c.i0]) / P.dx;
    const double g11 = (a[c.j1 * nx + i1p] - a[c.j1 * nx + c.i1]) / P.dx;
    return (1 - c.ox) * (1 - c.oy) * g00 + c.ox * (1 - c.oy) * g10 + (1 - c.ox) * c.oy * g01 + c.ox * c.oy * g11;
}

// d a/dy at (i dx, (j+1/2) dy), interpolated; c from the lattice shifted by half a cell in y.
__device__ __forceinline__ double grad_y(const double *__restrict__ a, const Cic &c, const Params &P)
{
    const int nx = P.nx;
    const int j0p = wrapi(c.j0 + 1, P.ny), j1p = wrapi(c.j1 + 1, P.ny);
    const double g00 = (a[j0p * nx + c.i0] - a[c.j0 * nx + c.i0]) / P.dy;
    const double g10 = (a[j0p * nx + c.i1] - a[c.j0 * nx + c.i1]) / P.dy;
    const double g01 = (a[j1p * nx + c.i0] - a[c.j1 * nx + c.i0]) / P.dy;
    const double g11 = (a[j1p * nx + c.i1] - a[c.j1 * nx + c.i1]) / P.dy;
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

// Deposit of four quantities q[k] with CIC weights wt[n] on the four nodes
// off[n] of each lane's cell `key`.  Lanes of one cell are summed across
// the wave first (particles are kept in cell order, so a wave usually spans
// one or a few cells) and the leader adds the sums; after kWaveRounds cells
// the remaining lanes add their own terms.
__device__ void deposit_wave(double *const dst[4], bool valid, int key, const int off[4], const double q[4],
                             const double wt[4])
{
    const int lane = threadIdx.x & 63;
    uint64_t pend = __ballot(valid);
    int rounds = 0;
    while (pend) {
        if (rounds == kWaveRounds) {
            if ((pend >> lane) & 1ull) {
#pragma unroll
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int n = 0; n < 4; ++n) unsafeAtomicAdd(dst[k] + off[n], q[k] * wt[n]);
            }
            break;
        }
        const int leader = __ffsll((unsigned long long)pend) - 1;
        const int lk = __shfl(key, leader, 64);
        const bool mine = ((pend >> lane) & 1ull) && key == lk;
        const uint64_t grp = __ballot(mine);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const double s = wave_sum(mine ? q[k] * wt[n] : 0.0);
                if (lane == leader) unsafeAtomicAdd(dst[k] + off[n], s);
            }
        pend &= ~grp;
        ++rounds;
    }
}

// MODE 0: one step of every particle (push, move, deposit at the new
// position).  MODE 1 (init): deposit the exact current of the given u_z
// (held in the p_z array).  MODE 2 (init): p_z = u_z - a^0(x), then the
// linearised deposit about a^0.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_particle(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    const int64_t step = P.state->step;
    const int cur = P.state->cur;
    const bool diag = MODE == 0 && P.diag_every > 0 && step % P.diag_every == 0;
    const int nx = P.nx;
    const double *an = MODE == 0 ? P.it[(P.iters - 1) & 1] : P.a1;   // a^n
    const double *aold = MODE == 0 ? P.a1 : P.a2;                     // a^(n-1)
    double *const *dst = MODE == 0 ? P.dep[1 - (int)(step & 1)] : P.dep[0];
    double *X = P.x[cur], *Y = P.y[cur], *UX = P.ux[cur], *UY = P.uy[cur], *PZ = P.pz[cur];
    double acc[kPDiag] = {0.0, 0.0, 0.0};
    for (int64_t base = (int64_t)blockIdx.x * kThreads; base < P.np; base += (int64_t)gridDim.x * kThreads) {
        const int64_t idx = base + threadIdx.x;
        const bool valid = idx < P.np;
        double q[4] = {0.0, 0.0, 0.0, 0.0}, wt[4] = {0.0, 0.0, 0.0, 0.0};
        int key = 0, off[4] = {0, 0, 0, 0};
        if (valid) {
            double x = X[idx], y = Y[idx], ux = UX[idx], uy = UY[idx], pz = PZ[idx];
            if (MODE == 0) {
                // gather at x^n: a, psi (nodes), grad a (staggered)
                const Cic c = cic(x, y, P, 0.0, 0.0);
                const double abar = bilin(an, c, nx);
                const double psib = bilin(P.psi, c, nx);
                const double Gx = grad_x(an, cic(x, y, P, 0.5, 0.0), P);
                const double Gy = grad_y(an, cic(x, y, P, 0.0, 0.5), P);
                const double uz = pz + abar;                                   // Eq. (6)
                const double gm = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
                const double f = -(uz / gm - (psib + abar)) * P.dt;            // Eq. (4)
                ux += f * Gx;
                uy += f * Gy;
                const double gp = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
                x = wrap_pos(x + P.dt * ux / gp, P.Lx);
                y = wrap_pos(y + P.dt * uy / gp, P.Ly);
                if (!(x >= 0.0 && x < P.Lx && y >= 0.0 && y < P.Ly)) {
                    atomicOr(&P.state->fatal, 1);
                    x = 0.0;
                    y = 0.0;
                }
                if (diag) {
                    acc[0] += P.w * (0.5 * (gm + gp));
                    acc[1] += P.w * (0.5 * abar * abar);
                    acc[2] += P.w * uz;
                }
                X[idx] = x;
                Y[idx] = y;
                UX[idx] = ux;
                UY[idx] = uy;
            }
            const Cic c = cic(x, y, P, 0.0, 0.0);
            double beta, chi = 0.0, as = 0.0;
            if (MODE == 1) {
                beta = pz / sqrt(1.0 + ux * ux + uy * uy + pz * pz);
            } else {
                if (MODE == 2) {
                    pz = pz - bilin(an, c, nx);
                    PZ[idx] = pz;
                }
                as = 2.0 * bilin(an, c, nx) - bilin(aold, c, nx);              // a* at the particle
                const double uzs = pz + as;
                const double up2 = ux * ux + uy * uy;
                const double g = sqrt(1.0 + up2 + uzs * uzs);
                beta = uzs / g;
                chi = (1.0 + up2) / (g * g * g);
            }
            q[0] = P.w;
            q[1] = P.w * beta;
            q[2] = P.w * chi;
            q[3] = P.w * chi * as;
            wt[0] = (1 - c.ox) * (1 - c.oy);
            wt[1] = c.ox * (1 - c.oy);
            wt[2] = (1 - c.ox) * c.oy;
            wt[3] = c.ox * c.oy;
            key = c.j0 * nx + c.i0;
            off[0] = key;
            off[1] = c.j0 * nx + c.i1;
            off[2] = c.j1 * nx + c.i0;
            off[3] = c.j1 * nx + c.i1;
        }
        deposit_wave(dst, valid, key, off, q, wt);
    }
    if (diag) block_sums<kPDiag>(acc, P.pdiag + (size_t)blockIdx.x * kPDiag);
}

// ---- Eq. (2): lap a - (n_p + X) a = J - Y + n_p psi, n_p = max(n0 - n_b, 0);
// each sweep solves (lap - c0) a_new = J - Y + n_p psi + (n_p + X - c0) a_old.

// In-place radix-2 decimation-in-time transforms of `batch` sequences of
// length 2^logn stored back to back in LDS, input in bit-reversed order,
// output in natural order; tw[t] = exp(-2 pi i t / 2^logn).
__device__ void fft_lds(double2 *z, int logn, int batch, const double2 *__restrict__ tw, bool inverse)
{
    const int n = 1 << logn;
    const int hn = n >> 1;
    const int total = batch * hn;
    for (int s = 1; s <= logn; ++s) {
        const int half = 1 << (s - 1);
        const int tsh = logn - s;
        for (int e = threadIdx.x; e < total; e += blockDim.x) {
            const int b = e >> (logn - 1);
            const int k = e & (hn - 1);
            const int pos = k & (half - 1);
            const int i1 = ((k >> (s - 1)) << s) + pos;
            double2 w = tw[pos << tsh];
            if (inverse) w.y = -w.y;
            double2 *zb = z + b * n;
            const double2 u = zb[i1], v0 = zb[i1 + half];
            const double2 v = make_double2(w.x * v0.x - w.y * v0.y, w.x * v0.y + w.y * v0.x);
            zb[i1] = make_double2(u.x + v.x, u.y + v.y);
            zb[i1 + half] = make_double2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// Row transform of the sweep's right-hand side (one workgroup per row).
__global__ __launch_bounds__(kThreads) void k_rows_fwd(const Params *__restrict__ pp, int iter)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int j = blockIdx.x, nx = P.nx;
    const int p = (int)(P.state->step & 1);
    const double *nb = P.dep[p][0], *J = P.dep[p][1], *Xc = P.dep[p][2], *Yc = P.dep[p][3];
    const double *prev = P.it[(iter + 1) & 1];
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        const int64_t o = (int64_t)j * nx + i;
        const double ap = iter == 0 ? 2.0 * P.a1[o] - P.a2[o] : prev[o];
        const double n_p = fmax(P.n0 - nb[o], 0.0);
        const double c = n_p + Xc[o];
        const double R = J[o] - Yc[o] + n_p * P.psi[o];
        z[brev(i, P.lx)] = make_double2(R + (c - P.c0) * ap, 0.0);
    }
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, false);
    for (int i = threadIdx.x; i < nx; i += blockDim.x) P.W[(int64_t)j * nx + i] = z[i];
}

// Column transform, division by the symbol -(4/dx^2) sin^2 - (4/dy^2) sin^2 - c0,
// inverse column transform (cols_per_block columns per workgroup).
__global__ __launch_bounds__(kThreads) void k_cols(const Params *__restrict__ pp)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int CB = P.cols_per_block, ny = P.ny, nx = P.nx, ly = P.ly;
    const int c0 = blockIdx.x * CB;
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

// Inverse row transform; the real part / (nx ny) is the sweep's result.
__global__ __launch_bounds__(kThreads) void k_rows_inv(const Params *__restrict__ pp, int iter)
{
    extern __shared__ double2 z[];
    const Params &P = *pp;
    const int j = blockIdx.x, nx = P.nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) z[brev(i, P.lx)] = P.W[(int64_t)j * nx + i];
    __syncthreads();
    fft_lds(z, P.lx, 1, P.twx, true);
    const double s = 1.0 / (double)P.cells;
    double *out = P.it[iter & 1];
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
        for (int k = 0; k < 4; ++k) P.dep[p][k][o] = 0.0;
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
        for (int k = 0; k < 4; ++k) P.dep[0][k][o] = 0.0;
    }
}

// ---- cell sort (counting sort by cell into the other particle set)
__device__ __forceinline__ int cell_of(double x, double y, const Params &P)
{
    const int i = wrapi((int)floor(x / P.dx), P.nx);
    const int j = wrapi((int)floor(y / P.dy), P.ny);
    return j * P.nx + i;
}

__global__ __launch_bounds__(kThreads) void k_sort_count(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    const int cur = P.state->cur;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P.np; i += (int64_t)gridDim.x * kThreads)
        atomicAdd(&P.cell_count[cell_of(P.x[cur][i], P.y[cur][i], P)], 1);
}

__global__ __launch_bounds__(kThreads) void k_scan_chunks(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    const int64_t b0 = (int64_t)blockIdx.x * kScanChunk;
    int s = 0;
    for (int k = threadIdx.x; k < kScanChunk; k += kThreads)
        if (b0 + k < P.cells) s += P.cell_count[b0 + k];
    int tot;
    (void)block_scan_excl(s, &tot);
    if (threadIdx.x == 0) P.scan_part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_top(const Params *__restrict__ pp, int nchunks)
{
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
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
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    constexpr int per = kScanChunk / kThreads;
    const int64_t b = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * per;
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
            run += v[k];
        }
}

__global__ __launch_bounds__(kThreads) void k_sort_scatter(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    if (!sort_step(P, P.state->step)) return;
    const int s = P.state->cur, d = s ^ 1;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < P.np; i += (int64_t)gridDim.x * kThreads) {
        const double x = P.x[s][i], y = P.y[s][i];
        const int64_t slot = atomicAdd(&P.cell_start[cell_of(x, y, P)], 1);
        P.x[d][slot] = x;
        P.y[d][slot] = y;
        P.ux[d][slot] = P.ux[s][i];
        P.uy[d][slot] = P.uy[s][i];
        P.pz[d][slot] = P.pz[s][i];
        P.id[d][slot] = P.id[s][i];
    }
}

// ---- bookkeeping: the diagnostic record (fixed-order sums), the particle
// set after a sort, the step counter.
__global__ __launch_bounds__(kThreads) void k_advance(const Params *__restrict__ pp)
{
    const Params &P = *pp;
    State *S = P.state;
    const int64_t step = S->step;
    const bool diag = P.diag_every > 0 && step % P.diag_every == 0;
    if (diag) {
        __shared__ double part[kThreads][kPDiag + kGDiag];
        double s[kPDiag + kGDiag] = {};
        for (int b = threadIdx.x; b < kPartBlocks; b += kThreads)
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
    if (threadIdx.x == 0) {
        if (sort_step(P, step)) S->cur ^= 1;
        S->step = step + 1;
    }
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
    for (int it = 0; it < hp.iters; ++it) {
        L(0, k_rows_fwd, dim3(hp.ny), dim3(kThreads), row_lds, dp, it);
        L(0, k_cols, dim3(hp.nx / hp.cols_per_block), dim3(kThreads), col_lds, dp);
        L(0, k_rows_inv, dim3(hp.ny), dim3(kThreads), row_lds, dp, it);
    }
}

int scan_chunks(const Params &hp) { return (int)((hp.cells + kScanChunk - 1) / kScanChunk); }

}  // namespace

hipError_t launch_init(const Params &hp, const Params *dp, hipStream_t st)
{
    Launcher L{st, nullptr, nullptr};
    L(0, k_particle<1>, dim3(kPartBlocks), dim3(kThreads), 0, dp);
    solve(L, hp, dp);
    L(0, k_init_nodes, dim3(kGridBlocks), dim3(kThreads), 0, dp);
    L(0, k_particle<2>, dim3(kPartBlocks), dim3(kThreads), 0, dp);
    return hipGetLastError();
}

int step_launches(const Params &hp) { return 3 * hp.iters + 8; }

hipError_t launch_step(const Params &hp, const Params *dp, hipStream_t st, hipEvent_t *ev, int *groups, int *nlaunch)
{
    Launcher L{st, ev, groups};
    solve(L, hp, dp);
    L(1, k_particle<0>, dim3(kPartBlocks), dim3(kThreads), 0, dp);
    L(2, k_nodes, dim3(kGridBlocks), dim3(kThreads), 0, dp);
    const int nch = scan_chunks(hp);
    L(3, k_sort_count, dim3(kPartBlocks), dim3(kThreads), 0, dp);
    L(3, k_scan_chunks, dim3(nch), dim3(kThreads), 0, dp);
    L(3, k_scan_top, dim3(1), dim3(kThreads), 0, dp, nch);
    L(3, k_scan_apply, dim3(nch), dim3(kThreads), 0, dp);
    L(3, k_sort_scatter, dim3(kPartBlocks), dim3(kThreads), 0, dp);
    L(3, k_advance, dim3(1), dim3(kThreads), 0, dp);
    if (nlaunch) *nlaunch = L.k;
    return hipGetLastError();
}

}  // namespace hyb
