// Internal layout shared by the HIP kernels and the host runtime of libpic.
//
// Everything the kernels need lives in one device-resident KParams block
// written once at initialisation, so a step is a fixed sequence of launches
// with pointer-only arguments (replayable as a graph).  Per-step mutable
// state (step counter, particle-set parity, overflow flags) is in DevState,
// also in device memory, and is advanced by the last kernel of each step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pic.h"

namespace pic {

constexpr int kMaxSpecies = PIC_MAX_SPECIES;
// Launch shapes of the particle kernel: threads per workgroup and the
// particles each lane keeps in flight (their loads issued ahead of the one it
// processes).  Shape 0 is the default and the only one of the FP64 kernels;
// mixed-precision runs take any (pic_grid_desc.shape, chosen by the tuner).
constexpr int kShapes = PIC_PARTICLE_SHAPES;
constexpr int kShapeBlock[kShapes] = {256, 256, 256, 512, 128};
constexpr int kShapeInflight[kShapes] = {2, 1, 3, 2, 2};
constexpr int kBlock = kShapeBlock[0];
constexpr int kRing = 4096;          // diagnostic records kept on the device
constexpr int kTileDiag = 6;         // per tile and species: KE, px, py, pz, count, collisions
constexpr int kFieldDiag = 10;       // per block: W[6], p_field[3], unused
constexpr int kFieldDiagBlocks = 512;
constexpr int kBinAlign = 64;        // particle-store bins start at multiples of this many slots
constexpr int kMomentBlocks = 1024;  // loader reductions
constexpr int kMomentVals = 6;

// Philox counter word 2 tags the purpose of a draw.
constexpr uint32_t kPurposeCollide = 1u;
constexpr uint32_t kPurposeLoad = 2u;
constexpr uint32_t kPurposeCoulomb = 3u;
constexpr uint32_t kPurposeBinaryKey = 4u;     // pairing order of the binary collisions
constexpr uint32_t kPurposeBinaryPair = 5u;    // one pair's deflection

struct DevState {
    int64_t step;        // index n of the step about to run
    int32_t par;         // particle set holding the current particles (0/1)
    int32_t rebin;       // an incoming-mover reserve overflowed during this step
    int32_t fatal;       // sticky: 1 overflow list exhausted, 2 particle off the grid, 4 store reserve
                         // exhausted, 8 particle outside its bin, 16 binary collisions: a cell above the
                         // participant limit
    int32_t pad;
    int64_t rebins;      // re-layouts performed so far
    int64_t ring_head;   // diagnostic records written so far
    uint32_t ovf_count[kMaxSpecies];
};

// Particle arrays of one species.  Sets 0 and 1 alternate as source and
// destination from step to step; set 2 is the overflow list.
//  mixed: sets 0, 1: cell within the tile of the particle's bin, 16 bits
//         (lx | ly << ts | lz << 2 ts, ts = log2 T); set 2: global packed
//         cell (ix | iy << sh1 | iz << sh2); pos = FP32 in-cell offset
//  fp64 : no cell array, pos = absolute FP64 position in cell units
struct SpeciesDev {
    uint16_t *cell[2];
    uint32_t *ovf_cell;
    void *pos[3][3];     // [set][axis]
    void *u[3][3];       // [set][component]
    uint32_t *id[3];
    int32_t *start;      // [tiles] first slot of each tile's bin
    int32_t *cap;        // [tiles] bin capacity
    uint32_t *cnt_front; // [2][tiles] particles written from the bin's front
    uint32_t *cnt_back;  // [2][tiles] movers written from the bin's back
    int64_t ncap;        // slots per set
    int64_t nominal;     // ppc * cells
    uint32_t ovf_cap;
    uint32_t coll_thr;   // scatter when the 32-bit draw is below this (isotropic model)
    int32_t collide;
    int32_t coll_model;  // PIC_COLL_ISOTROPIC or PIC_COLL_COULOMB
    double coll_sig2;    // Coulomb model: variance of tan(theta/2) = coll_sig2 / v^3
    int32_t track_id;    // carry ids (collisional species, or all in test mode)
    double q, m, w;
    double qmdt2;        // q dt / (2 m)
    double qw;           // q w
    int32_t ppc;
    int32_t id_base;
    double drift[3];     // loader: mean momentum
    double uth;          // loader: Gaussian spread per component
    int32_t binary;      // takes part in the binary (pairwise) collisions
};

struct Geometry {
    int ndim;
    int n[3];
    double d[3];
    double dt;
    int tile[3];
    int nt[3];           // tiles per axis
    int ntiles;
    int tshift[3];       // log2(tile)
    int csh[3];          // cell packing shifts (mixed)
    uint32_t cmask[3];
    int64_t cells;
};

struct KParams {
    Geometry g;
    int nspecies;
    int precision;       // PIC_PREC_*
    int diag_every;
    unsigned flags;
    uint64_t seed;
    uint32_t run;
    SpeciesDev sp[kMaxSpecies];
    void *F;             // 6 planes Ex Ey Ez Bx By Bz (float or double)
    double *J;           // 3 planes
    void *Jtile;         // [tiles][3][nj^ndim] per-tile partial currents
    int nj;              // tile edge + 3
    double *tile_diag;   // [tiles][nspecies][kTileDiag]
    double *field_diag;  // [kFieldDiagBlocks][kFieldDiag]
    double *moments;     // [kMomentBlocks][kMomentVals]
    DevState *state;
    pic_diag *ring;      // [kRing]
    int32_t *rb_count;   // [nspecies][tiles]
    int32_t *rb_start;   // [nspecies][tiles]
    int32_t *rb_cap;     // [nspecies][tiles]
    int32_t *rb_fill;    // [nspecies][tiles]
    int fd_blocks;       // blocks (and partial records) of the field-diagnostic reduction
    int32_t *order;      // [tiles] particle-kernel work order (XCD class, then decreasing load)
    uint8_t *tile_bucket;   // [tiles] load bucket of each tile, written by the particle kernel
    double order_scale;  // bucket = round(particles in the tile * order_scale): 16 per nominal load
    int32_t coulomb;     // 1 if a species scatters with the Coulomb model (selects the particle kernel)
    int32_t shape;       // particle-kernel launch shape (index into kShapeBlock / kShapeInflight)
    double nu_ee;        // binary collisions: rate at relative speed ee_vref (0 = off)
    double ee_vref;
    int32_t binary;      // 1 if the binary-collision kernel runs (nu_ee > 0 and a species takes part)
    int64_t *ee_tile;    // [tiles] binary-collision pairs scattered in the tile this step
    uint32_t *ee_ent;    // binary collisions: each tile's participants in cell order (slot | species << 29),
                         // the tile's list at the sum over participating species of its bin starts
    // Gauss-law and continuity checks (PIC_FLAG_GAUSS_RESIDUAL only; null otherwise)
    double *rho_tile;    // [tiles][(T+1)^ndim] per-tile charge partials
    double *rho0;        // [cells] charge on the nodes at step 0
    double *rho_n;       // [cells] charge on the nodes at the start of the current check step
    double *gauss_part;  // [ceil(cells / 256)][2] per-block maxima of the residual and of |rho - rho0|
    double *cont_part;   // [ceil(cells / 256)][2] per-block maxima of the continuity residual and |rho' - rho|
};

// An ensemble of runs stepped together: every launch of a step covers all
// runs.  Runs share precision and dimension; in 2D each run has its own tile
// edge, and the particle kernel is launched once per edge (group g: edge
// 8 << g; 3D runs use group 0).  The work items (run, k) -- the k-th tile of
// the run's work order, whose tile index is k mod 8 -- are split by XCD
// class k mod 8 into one list and one queue per class.
constexpr int kBatchXcds = 8;
struct BatchGroup {
    int n_items;                   // work items of the runs with this edge
    const int2 *items;             // [n_items] (run, k), class-major; in a class,
                                   // runs with the most particles per tile first
    int cls_start[kBatchXcds];     // first item of each class
    int cls_len[kBatchXcds];       // items of each class
    int *queue;                    // [kBatchXcds] work counters of the persistent particle kernel
    int shape;                     // particle-kernel launch shape of the runs with this edge
};
constexpr int kBatchGroups = 3;
struct BatchTable {
    int nruns;
    int n_cell_blocks;    // 256-cell blocks over all runs
    int nst_blocks;       // max over runs of ceil(nspecies * tiles / 256)
    int max_species;
    int max_fd_blocks;    // max over runs of KParams::fd_blocks
    int coulomb;          // 1 if any run has a species on the Coulomb scattering model
    const KParams *const *kp;   // [nruns] device parameter blocks
    const int2 *cell_blocks;    // [n_cell_blocks] (run, block of that run)
    BatchGroup grp[kBatchGroups];
};
constexpr int kBatchRebinBlocks = 256;

// Host-callable launchers (defined in the .hip translation units).
// Kernels of one step and the group each belongs to: field-diag (0),
// particle (1), re-layout (2), current reduction (3), Yee (4), advance (5).
constexpr int kNumGroups = 6;
constexpr int kStepKernels = 13;
constexpr int kKernelGroup[kStepKernels] = {0, 1, 2, 2, 2, 2, 2, 2, 3, 4, 4, 4, 5};
// A single run's step is kStepKernels launches, plus four with
// PIC_FLAG_GAUSS_RESIDUAL (the charge deposits and residuals of the Gauss
// and continuity checks, group 0) and one with binary collisions (group 1).
// step_kernel_groups fills groups[] with each launch's group and returns the
// number of launches.
int step_kernel_groups(const KParams &hp, int *groups);
// ev: NULL, or 2 * kStepKernels events (start/stop of each dispatch)
hipError_t launch_step(const KParams &hp, const KParams *dp, hipStream_t s, hipEvent_t *ev = nullptr);
// Batch step: the particle kernel is one launch per tile group (empty groups
// launch one workgroup that exits), so a batch step has kBatchKernels
// dispatches; kBatchKernelGroup maps them to the groups above.
// pblocks[g]: persistent workgroups of group g's particle launch.
constexpr int kBatchKernels = kStepKernels + kBatchGroups - 1;
constexpr int kBatchKernelGroup[kBatchKernels] = {0, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 4, 4, 4, 5};
hipError_t launch_batch_step(int precision, int ndim, const BatchTable &ht, const BatchTable *dt,
                             const int pblocks[kBatchGroups], hipStream_t s, hipEvent_t *ev = nullptr);
// Workgroups of the batch particle kernel of tile group g that fit on one
// compute unit at once.
hipError_t batch_particle_occupancy(int precision, int ndim, int g, bool coulomb, int shape, int *blocks_per_cu);
// Initialisation shared by pic_init (static_device = -1, the caller's
// scratch) and pic_init_static_scratch (the library's scratch of that
// device, already claimed; pic_destroy releases it).
int init_run(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
             const pic_buffers *buffers, void *hip_stream, pic_run **out, int static_device);
// One run at a time per device may hold the library's scratch of that device.
constexpr int kMaxDevices = 64;
bool claim_static_scratch(int device);     // false if held
void release_static_scratch(int device);
// Records a message for pic_last_error(NULL, ...) and returns code.
int fail_global(int code, const char *fmt, ...);

hipError_t launch_load_species(const KParams &hp, const KParams *dp, int s, hipStream_t st);
hipError_t launch_moments(const KParams &hp, const KParams *dp, int s, double delta_uz, hipStream_t st);
hipError_t launch_shift_u(const KParams &hp, const KParams *dp, int s, double dux, double duy,
                          double duz, hipStream_t st);

}  // namespace pic
