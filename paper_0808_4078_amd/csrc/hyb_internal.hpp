// Internal declarations of the reduced quasi-neutral model (kinetic beam,
// fluid return current, a = e A_z/(m c^2) from Ampere's law without
// displacement current): device parameter block, state and launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

namespace hyb {

constexpr int kThreads = 256;
constexpr int kPartBlocks = 2048;     // sort kernels: fixed grid, grid-stride loop
constexpr int kGridBlocks = 1024;     // node-wise kernels: fixed grid, grid-stride loop
constexpr int kRing = 4096;           // diagnostic records kept on the device
constexpr int kPDiag = 3;             // per-block particle sums: w gamma, w a^2/2, w u_z
constexpr int kGDiag = 5;             // per-block node sums: |grad a|^2, a^2, (d_t a)^2, a, psi
constexpr int kScanChunk = 2048;      // cells per block of the sort's prefix sum
constexpr int kMaxNodes = 4096;       // nodes per axis
constexpr int kFftLds = 4096;         // complex values per FFT workgroup (64 KiB of LDS)
constexpr int kColThreads = 1024;     // threads of a column-transform workgroup (few workgroups: latency hiding)
constexpr int kWaveRounds = 8;        // distinct sort keys merged per wave before plain atomics
constexpr int kMaxTile = 16;          // tile edge (cells) of the particle kernel
constexpr int kMargin = 2;            // cells of drift since the last sort that the tile's window absorbs
constexpr int kWin = kMaxTile + 2 * kMargin + 1;   // nodes per axis of a tile's deposit window
constexpr int kFw = kMaxTile + 2 * kMargin + 4;    // nodes per axis of a tile's field window (gathers)
constexpr int kWinC = kMaxTile + 2 * kMargin;      // cells per axis of a tile's sort bins

// Deposit planes hold 64-bit fixed point: kDepScale units per unit
// (integer sums are exact in any order; see the particle kernel).
using Fix = long long;
constexpr double kDepScale = 562949953421312.0;   // 2^49
constexpr double kDepUnit = 1.0 / kDepScale;

struct State {
    int64_t step;        // time level n of the next step
    int32_t cur;         // particle set in use (the cell sort alternates 0/1)
    int32_t ring_head;   // next ring slot
    int32_t ring_count;  // records written (saturates at kRing)
    int32_t fatal;       // 1: a particle left the box (non-finite momentum)
};

struct Params {
    int nx, ny, lx, ly;            // nodes per axis and their log2
    int iters, diag_every, sort_every, cols_per_block;
    int tile, ltile, tiles_x, ntiles;  // particle tiles: edge (cells) and its log2, tiles along x, count
    int64_t np;                    // beam macro-particles
    int64_t cells;                 // nx * ny
    double dx, dy, dt, nu, n0, w, c0, dA, Lx, Ly, inv_dx, inv_dy;
    // particles: two sets (the sort writes the other one)
    double *x[2], *y[2], *ux[2], *uy[2], *pz[2];
    uint32_t *id[2];
    // nodes
    double *a1;                    // a^(n-1): the last solved potential
    double *a2;                    // a^(n-2)
    double *psi;                   // plasma canonical momentum beta_pz - a
    double *it[2];                 // solve result (it[(iters-1) & 1] holds a^n after the solve)
    double *rhsR, *rhsC;           // per step: J - Y + n_p psi, and n_p + X - c0 (the sweeps' coefficients)
    Fix *dep[2][4];                // deposit sets (fixed point): n_b, J at a*, chi, chi a*
    double2 *W;                    // complex FFT plane [ny][nx]
    double2 *twx, *twy;            // exp(-2 pi i t / n), t < n/2
    double *lapx, *lapy;           // (4/d^2) sin^2(pi k / n)
    int32_t *cell_count;           // [cells] particles per sort key (tile-major cell index)
    int32_t *cell_start;           // [cells] exclusive prefix, then the scatter cursor
    int32_t *tile_start[2];        // [ntiles + 1] per particle set: first particle of each tile after the sort
    int32_t *bins;                 // [ntiles][kWinC^2] particles per cell of each tile's sort window
    int32_t *scan_part;            // [ceil(cells / kScanChunk)] chunk sums
    double *pdiag;                 // [ntiles][kPDiag]
    double *gdiag;                 // [kGridBlocks][kGDiag]
    State *state;
    pic_hyb_diag *ring;            // [kRing]
};

// Kernel groups of a step, for the profiled launch: solve | particle | grid | sort + bookkeeping.
constexpr int kGroups = 4;

// Enqueues the init sequence (exact deposit, solve, a^0, p_z and the first
// linearised deposit) on `st`.
hipError_t launch_init(const Params &hp, const Params *dp, hipStream_t st);
// Enqueues one step; with `ev` (2 events per launch) each launch is timed and
// `groups` receives the group of each launch; *nlaunch the launch count.
hipError_t launch_step(const Params &hp, const Params *dp, hipStream_t st, hipEvent_t *ev, int *groups,
                       int *nlaunch);
// Launches of one step (for sizing the event arrays).
int step_launches(const Params &hp);

}  // namespace hyb
