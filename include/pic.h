/*
 * pic.h -- C ABI of the MI355X beam-plasma particle-in-cell library (libpic.so).
 *
 * The library advances the relativistic beam / return-current system of
 * Karmakar, Kumar, Shvets, Polomarov and Pukhov (arXiv:0808.4078): electron
 * species drifting along z through a quasi-neutral plasma with an immobile
 * neutralising ion background (problem statement at the start of the theory
 * part; the 2D and 3D PIC-simulation paragraphs).  One step is: field gather,
 * relativistic Boris push, charge-conserving (Esirkepov) current deposit,
 * scattering of collisional species off the ions (isotropic at a fixed rate,
 * whose fluid limit is the drag term of Eq. (3), or Coulomb small-angle),
 * optional binary electron-electron collisions within each cell, and a Yee
 * update of E and B.  The paper's reduced quasi-neutral model has its own
 * entry points (pic_hyb_*, at the end).
 *
 * Units are normalised: t in 1/w_p, x in c/w_p, u = gamma v/c, fields
 * eF/(m c w_p) (the normalisation of the paper's field-energy diagnostic),
 * densities in n0, charge in e, mass in m_e.
 *
 * Conventions for every entry point:
 *  - Return value: PIC_OK (0) or a negative PIC_E_* code.  No C++ exception
 *    crosses the ABI.  pic_last_error() gives a message for the last failure
 *    on a handle.
 *  - Device memory is owned by the caller.  pic_query() gives the four
 *    buffer sizes; the caller allocates them on the device that is current
 *    when pic_init() is called and keeps them alive until pic_destroy().
 *    The library never allocates or frees device memory.  It keeps small
 *    host-side state (descriptors, a captured graph) in the handle.
 *  - Streams are owned by the caller.  Work is enqueued on the stream given
 *    to pic_init(); entry points marked "synchronising" wait for it.
 *  - Device-side faults and capacity exhaustion surface as PIC_E_HIP /
 *    PIC_E_CAPACITY at the next synchronising call.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PIC_OK = 0,
    PIC_E_INVALID_ARG = -1,      /* bad descriptor, pointer or size */
    PIC_E_UNSUPPORTED = -2,      /* valid physics, configuration not built */
    PIC_E_CFL = -3,              /* Courant condition of the scheme violated */
    PIC_E_BUFFER_TOO_SMALL = -4, /* caller buffer smaller than pic_query's size */
    PIC_E_HIP = -5,              /* HIP runtime error (launch, copy, device fault) */
    PIC_E_STATE = -6,            /* call not valid in the handle's current state */
    PIC_E_CAPACITY = -7          /* particle store overflowed its reserve */
};

enum { PIC_PREC_FP64 = 0, PIC_PREC_MIXED = 1 };

/* Scattering models of a collisional species (pic_species_desc.coll_model). */
enum {
    PIC_COLL_ISOTROPIC = 0,  /* isotropic scattering at the fixed rate nu_coll (default) */
    PIC_COLL_COULOMB = 1     /* Coulomb small-angle scattering, rate nu_coll at speed coll_vref */
};

enum {
    PIC_FLAG_FREEZE_FIELDS = 1u,  /* skip current reduction and field update (test-particle mode) */
    PIC_FLAG_NO_COLLIDE = 2u,     /* ignore every species' collision rate */
    PIC_FLAG_LATTICE_LOAD = 4u,   /* device loader: regular sub-lattice positions */
    PIC_FLAG_HOST_LOAD = 8u,      /* do not load on the device; caller calls pic_load_particles */
    PIC_FLAG_NO_GRAPH = 16u,      /* launch kernels one by one instead of replaying a graph */
    PIC_FLAG_TRACK_IDS = 32u,     /* carry particle ids for every species (by default only
                                     collisional species, whose draws are keyed by id, do) */
    PIC_FLAG_GAUSS_RESIDUAL = 64u /* at step 0 and on diagnostic steps, deposit the particles'
                                     charge before and after the move and record the Gauss's-law
                                     and charge-continuity residuals (single runs only) */
};

#define PIC_MAX_SPECIES 8

/* Launch shapes of the particle kernel (pic_grid_desc.shape): threads per
 * workgroup / particles each lane keeps in flight (the loads of the next
 * ones issued before the current one is processed).
 *   0: 256 / 2 (default; the only shape of FP64 runs)   1: 256 / 1
 *   2: 256 / 3   3: 512 / 2   4: 128 / 2
 * The shape changes how the work is spread over the device, never the
 * arithmetic; pic_tune_shape times them. */
#define PIC_PARTICLE_SHAPES 5

/* Grid and run parameters.
 *   ndim      2 (2D3V: x,y resolved, z ignorable -- the paper's transverse plane)
 *             or 3 (3D3V).
 *   n[3]      cells per axis (n[2] ignored in 2D); periodic boundaries.
 *   d[3]      cell size per axis in c/w_p.
 *   dt        time step in 1/w_p.  Must satisfy dt <= d_i/2 on every resolved
 *             axis (a particle crosses at most half a cell per step), which
 *             also implies the Yee Courant condition.
 *   precision PIC_PREC_FP64: FP64 positions, momenta, fields and currents.
 *             PIC_PREC_MIXED: int32 cell index + FP32 in-cell offset, FP32
 *             momenta, FP32 push and per-tile FP32 current, FP64 grid-level
 *             current reduction and diagnostics, FP32 E and B.
 *   seed, run key of the counter-based random streams (Philox2x32-10 for the
 *             per-step scattering decision, Philox4x32-10 for the loader and
 *             the scattering direction) and the run index mixed into it.
 *   tile[3]   particle tile edge in cells, the same on every resolved axis
 *             (0 = library default: 16 or 8 in 2D, 8 in 3D); 2D supports 8, 16
 *             and 32, 3D supports 8; n must be a multiple of the tile.
 *   diag_every record diagnostics every diag_every steps (0 = never).
 *   flags     PIC_FLAG_* bits.
 *   reserve   spare particle-store capacity per tile, as a fraction of the
 *             tile's nominal particle count (0 = library default 1.0).  A
 *             tile whose population outgrows its spare capacity triggers a
 *             re-layout of the store at the end of the step; spare slots are
 *             never read, so a larger reserve costs device memory only.
 *             Must be in [0, 8].
 *   nu_ee, ee_vref  binary (pairwise) collisions among the particles of the
 *             species with pic_species_desc.binary set (the paper's binary
 *             collision module between electrons: beam-plasma and
 *             plasma-plasma).  Each step, after the push, move, deposit and
 *             the scattering off the ions, the participants of every cell
 *             (at x^{n+1}) are put in the order of word 0 of Philox4x32-10 on
 *             counter (id, step, 4, run), key (seed lo, seed hi), ties by id,
 *             and paired (0,1), (2,3), ...; an odd count N >= 3 starts with
 *             the triple (0,1), (1,2), (2,0) at half the variance (Takizuka
 *             and Abe 1977).  A pair (a, b) turns its relative momentum in its
 *             centre-of-momentum frame by theta, tan(theta/2) ~ N(0, s^2),
 *             s^2 = (nu_ee dt/2) (ee_vref / v_rel)^3 (v_rel = |v_a - v_b| in
 *             the lab; rate nu_ee at relative speed ee_vref, Coulomb's v^-3
 *             law), uniform azimuth (draws: Philox4x32-10 on (id_a, step, 5,
 *             run)); equal weights keep the pair's four-momentum, unequal
 *             weights keep it in expectation (the heavier particle takes its
 *             new momentum with probability w_small/w_large; Nanbu and
 *             Yonemura 1998).  nu_ee = 0: off.  With nu_ee > 0, ee_vref must
 *             be in (0, 1) and the participants need ids (they are tracked).
 *             Limit: 2048 participants in one cell (PIC_E_CAPACITY beyond);
 *             not available in ensembles.
 *   shape     particle-kernel launch shape, 0..PIC_PARTICLE_SHAPES-1 (0 for
 *             FP64 runs).  A launch choice, not part of the run's state:
 *             pic_restore accepts a checkpoint taken with another shape. */
typedef struct {
    int32_t ndim;
    int32_t n[3];
    double d[3];
    double dt;
    int32_t precision;
    uint64_t seed;
    uint32_t run;
    int32_t tile[3];
    int32_t diag_every;
    uint32_t flags;
    double reserve;
    double nu_ee;
    double ee_vref;
    int32_t shape;
} pic_grid_desc;

/* One particle species.
 *   charge, mass        in e and m_e (electrons: -1, 1).
 *   density             n_s / n0.
 *   ppc                 macro-particles per cell; weight = density / ppc.  The
 *                       store is sized for density*cells*ppc particles.
 *   drift_u, u_th       device loader: u = drift_u + u_th * N(0,1) per component
 *                       (mean of u_x, u_y removed afterwards).
 *   cancel_current_of   device loader: shift this species' u_z so the total
 *                       current sum q w u_z/gamma of all species is zero
 *                       (the return current neutralising the beam); -1 = no.
 *   nu_coll             scattering rate off the ions in w_p (0 = collisionless).
 *   coll_model          PIC_COLL_ISOTROPIC: with probability 1 - exp(-nu dt) per
 *                       step the particle takes an isotropic direction, |u| kept
 *                       (the drag term of Eq. (3) in the fluid limit).
 *                       PIC_COLL_COULOMB: binary Coulomb collisions with the
 *                       immobile ions (Takizuka-Abe small-angle form, ion mass
 *                       infinite): every step the particle turns by theta,
 *                       tan(theta/2) ~ N(0, nu_m(v) dt / 2), uniform azimuth, |u|
 *                       kept, with momentum-transfer rate nu_m(v) =
 *                       nu_coll (coll_vref / v)^3 (v = |u|/gamma).
 *   coll_vref           reference speed of PIC_COLL_COULOMB in c (> 0 when
 *                       nu_coll > 0); ignored otherwise.
 *   binary              1: the species takes part in the binary collisions
 *                       of pic_grid_desc.nu_ee; 0: not. */
typedef struct {
    double charge, mass, density;
    int32_t ppc;
    double drift_u[3];
    double u_th;
    int32_t cancel_current_of;
    double nu_coll;
    int32_t coll_model;
    double coll_vref;
    int32_t binary;
} pic_species_desc;

/* Sizes in bytes of the caller-owned device buffers. */
typedef struct {
    size_t particle_bytes[PIC_MAX_SPECIES];
    size_t field_bytes, scratch_bytes, diag_bytes;
} pic_sizes;

/* Device pointers (256-byte aligned) of the caller-owned buffers. */
typedef struct {
    void *particles[PIC_MAX_SPECIES];
    void *fields;
    void *scratch;
    void *diag;
} pic_buffers;

/* One diagnostic record for time level `step` (taken while that step runs):
 *   W[6]           sum over cells of F_i^2 dV for Ex,Ey,Ez,Bx,By,Bz at time step
 *                  (the paper's per-component field energy, no factor 1/2).
 *   kinetic[s]     dV sum w (gamma - 1), gamma time-centred at the step.
 *   p_species[s]   dV sum w u of species s, time-centred.
 *   p_particles[3] dV sum w u, time-centred, all species.
 *   p_field[3]     dV sum E x B, each product at its E component's point (B
 *                  averaged over the two points around it).
 *   collisions     scattering events off the ions during the step.
 *   ee_pairs       binary-collision pairs that scattered during the step.
 *   n_particles[s] particles of species s.
 *   rebins         particle-store re-layouts performed so far.
 *   gauss_resid    with PIC_FLAG_GAUSS_RESIDUAL: max over nodes of
 *                  |div E - (rho - rho_0)| at the step, rho the CIC charge
 *                  of the particles on the nodes, rho_0 that of step 0 (the
 *                  immobile ions carry -rho_0); -1 when not computed.
 *   rho_dev        with PIC_FLAG_GAUSS_RESIDUAL: max over nodes of
 *                  |rho - rho_0| (the scale of the residual); -1 otherwise.
 *   continuity_resid with PIC_FLAG_GAUSS_RESIDUAL: max over nodes of
 *                  |rho^{n+1} - rho^n + dt div J^{n+1/2}| for this step's
 *                  move (rho the CIC charge of the particles before and after
 *                  it, J the step's grid current, div the backward difference
 *                  onto the nodes): the charge conservation that the
 *                  Esirkepov deposit guarantees (Esirkepov 2001); -1 when not
 *                  computed.
 *   rho_step       with PIC_FLAG_GAUSS_RESIDUAL: max over nodes of
 *                  |rho^{n+1} - rho^n| (the scale of continuity_resid); -1
 *                  otherwise. */
typedef struct {
    int64_t step;
    double time;
    double W[6];
    double kinetic[PIC_MAX_SPECIES];
    double p_species[PIC_MAX_SPECIES][3];
    double p_particles[3];
    double p_field[3];
    int64_t collisions;
    int64_t n_particles[PIC_MAX_SPECIES];
    int64_t rebins;
    double gauss_resid;
    double rho_dev;
    double continuity_resid;
    double rho_step;
    int64_t ee_pairs;
} pic_diag;

typedef struct pic_run pic_run;

/* Host only (touches no device).  Validates the descriptors and returns the
 * buffer sizes.  Errors: INVALID_ARG (null pointer, nspecies out of 1..8,
 * n or ppc <= 0, n not a multiple of the tile), CFL, UNSUPPORTED. */
int pic_query(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
              pic_sizes *out);

/* Binds the caller's buffers (sizes checked against pic_query), zeroes the
 * fields, lays out the particle store and, unless PIC_FLAG_HOST_LOAD, loads
 * the species on the device (exactly ppc per cell, uniform in-cell positions,
 * Gaussian momenta, mean transverse momentum removed, net current cancelled by
 * a Newton shift in FP64).  Unless PIC_FLAG_NO_GRAPH, one step is captured as
 * a hipGraph; a failed capture fails the call with PIC_E_HIP.  `hip_stream`
 * is a hipStream_t (NULL = default stream).  Synchronising.  On success *out
 * owns host state only. */
int pic_init(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
             const pic_buffers *buffers, void *hip_stream, pic_run **out);

/* Test path: replaces species s with n host particles.  x is FP64 SoA
 * [ndim][n] in c/w_p (wrapped into the box), u is FP64 SoA [3][n], id is
 * [n] uint32 (keys the collision draw).  n must not exceed ppc * cells of
 * the species.  Synchronising. */
int pic_load_particles(pic_run *run, int species, const double *x, const double *u,
                       const uint32_t *id, int64_t n);

/* Enqueues nsteps full steps on the bound stream (asynchronous). */
int pic_step(pic_run *run, int32_t nsteps);

/* Measurement path: enqueues nsteps full steps exactly as pic_step but as
 * individual launches, each carrying start/stop HIP events that record the
 * dispatch's own execution interval on the bound stream; waits for them and
 * adds each kernel group's summed kernel milliseconds into group_ms[6]:
 * [0] field diagnostics, [1] particle kernel (gather, push, move, deposit,
 * scattering, binning), [2] store re-layout, [3] current reduction,
 * [4] Yee update, [5] end-of-step bookkeeping.  Synchronising. */
int pic_step_profiled(pic_run *run, int32_t nsteps, double *group_ms);

/* Waits for the bound stream; reports device-side capacity failures. */
int pic_sync(pic_run *run);

/* How a run (or a batch) enqueues its steps.
 *   graph           1 if a step is the replay of one captured hipGraph, 0 if
 *                   its kernels are launched one by one (PIC_FLAG_NO_GRAPH,
 *                   or a run on the library's scratch).
 *   static_scratch  1 if the run lives on the library's own scratch
 *                   (pic_init_static_scratch).
 *   steps_enqueued  steps enqueued so far (graph_launches + direct_steps,
 *                   plus the steps of a restored checkpoint).
 *   graph_launches  steps enqueued as one graph replay.
 *   direct_steps    steps enqueued kernel by kernel (including the
 *                   measurement path pic_step_profiled).
 *   scratch_bytes   scratch the run uses (pic_query's scratch_bytes).
 *   shape, block_threads, inflight  the particle kernel's launch shape and
 *                   its threads per workgroup and particles in flight per
 *                   lane. */
typedef struct {
    int32_t graph;
    int32_t static_scratch;
    int64_t steps_enqueued;
    int64_t graph_launches;
    int64_t direct_steps;
    size_t scratch_bytes;
    int32_t shape;
    int32_t block_threads;
    int32_t inflight;
} pic_run_info;

/* Host only.  Fills *out for the run.  Errors: INVALID_ARG (NULL). */
int pic_info(pic_run *run, pic_run_info *out);

/* Synchronising.  Copies the most recent diagnostic record; PIC_E_STATE if
 * none has been recorded yet. */
int pic_diagnostics(pic_run *run, pic_diag *out);

/* Synchronising.  Copies up to `max` of the most recent records, oldest first
 * (the device ring keeps the last 4096); *count receives the number copied. */
int pic_diag_history(pic_run *run, pic_diag *out, int64_t max, int64_t *count);

/* Synchronising.  FP64 host copies of the grid planes, each n0*n1*n2 values,
 * [n2][n1][n0] x fastest, half-integer positions stored at the lower index:
 * E and B: [3][cells] (Ex,Ey,Ez / Bx,By,Bz), J: [3][cells] of the last step.
 * Any pointer may be NULL. */
int pic_read_fields(pic_run *run, double *E, double *B, double *J);

/* Synchronising.  Overwrites E and B from FP64 host planes (layout as above;
 * either may be NULL). */
int pic_write_fields(pic_run *run, const double *E, const double *B);

/* Synchronising.  Copies species s out: x FP64 [ndim][cap] in c/w_p, u FP64
 * [3][cap], id [cap]; *count receives the particle number (PIC_E_BUFFER_TOO_SMALL
 * if it exceeds cap).  Order is the store's order, not id order. */
int pic_read_particles(pic_run *run, int species, double *x, double *u, uint32_t *id,
                       int64_t cap, int64_t *count);

/* Synchronising.  Writes the run's complete state -- particle store, fields,
 * current, scratch (step counter, parity, work order), diagnostic ring --
 * with its descriptors to the file `path` (overwritten).  The file holds the
 * raw buffers (sizes as pic_query gives), so it is as large as the device
 * state.  Errors: INVALID_ARG (null argument, file not writable),
 * CAPACITY / HIP (as pic_sync). */
int pic_checkpoint(pic_run *run, const char *path);

/* Synchronising.  Replaces the run's state by the checkpoint in `path`.  The
 * run must have been initialised with the same grid and species descriptors
 * (flags that only steer initialisation -- HOST_LOAD, NO_GRAPH, LATTICE_LOAD
 * -- may differ; pass PIC_FLAG_HOST_LOAD to skip the device loader of a run
 * that is about to be restored).  Stepping then continues exactly where the
 * checkpointed run stood.  Errors: INVALID_ARG (unreadable, foreign or
 * truncated file), STATE (descriptors differ), HIP. */
int pic_restore(pic_run *run, const char *path);

/* Waits for the run's stream (the caller may free the buffers once this
 * returns), then frees the handle's host state (not the caller's buffers)
 * and, for a run made by pic_init_static_scratch, releases the library's
 * scratch of its device.  Errors: STATE (the run is in a batch), HIP (the
 * wait failed; the handle is freed all the same). */
int pic_destroy(pic_run *run);

/* ---- Initialisation without a scratch allocation ---------------------------
 * For callers that cannot allocate device memory (code running under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): as
 * pic_init, but the scratch buffer is not the caller's -- buffers->scratch
 * must be NULL -- and the run uses a scratch array that the library holds on
 * each device (PIC_STATIC_SCRATCH_BYTES, reserved on every device the
 * library runs on until the process ends).  The caller still allocates the
 * particle, field and diagnostic buffers.  This call allocates no device
 * memory and creates no stream or graph: steps are launched kernel by
 * kernel (pic_info reports graph = 0), so a caller may capture pic_step
 * into a graph of its own.
 * The array is shared by every run on a device: at most one run per device
 * holds it at a time, from this call to pic_destroy; a second call on the
 * same device returns PIC_E_STATE until then (two runs on it would race).
 * Everything the step reads before writing it is cleared here, so the
 * contents a previous run left behind do not matter.
 * Errors: those of pic_init; INVALID_ARG (buffers->scratch not NULL);
 * BUFFER_TOO_SMALL (pic_query's scratch_bytes exceeds
 * PIC_STATIC_SCRATCH_BYTES: a grid of up to ~1M cells with 16^2 tiles fits);
 * STATE (the device's scratch is held by another run); UNSUPPORTED (device
 * index >= 64). */
#define PIC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int pic_init_static_scratch(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
                            const pic_buffers *buffers, void *hip_stream, pic_run **out);

/* Static string for a status code. */
const char *pic_status_string(int status);

/* Bandwidth probe (measurement only, no part of a step): copies `narrays`
 * (1..8) device arrays of n 4-byte words, src[a] -> dst[a], in one launch of
 * workgroups of 256 lanes, workgroup b copying words [b chunk, (b+1) chunk)
 * of every array, 256 consecutive words at a time -- the access pattern of
 * the particle kernel's state streams (a workgroup per tile's bin) without
 * its arithmetic, binning or LDS work -- so its rate is the practical copy
 * ceiling of that pattern at that chunk length (chunk = 256: one word of
 * each array per lane).  src and dst are host arrays of device pointers; the
 * arrays must not overlap.  Asynchronous on `hip_stream`.  Errors:
 * INVALID_ARG (NULL, narrays out of range, n < 0, chunk not a positive
 * multiple of 256), HIP. */
int pic_copy_probe(const void *const *src, void *const *dst, int narrays, int64_t n, int64_t chunk,
                   void *hip_stream);

/* Copies the last error message of the handle (or of the last failed
 * pic_init / pic_query when run is NULL) into buf. */
int pic_last_error(pic_run *run, char *buf, size_t n);

/* ---- Ensembles -----------------------------------------------------------
 * Many independent runs (the paper's parameter scans: beam temperature,
 * collision rate, box size) stepped together.  A batch step is one kernel
 * sequence over every member: the particle kernel is persistent -- its
 * workgroups take (run, tile) work items from a device queue, runs with the
 * most particles per tile first -- and is launched once per tile edge in use;
 * the re-layout, current-reduction and Yee kernels each cover every member's
 * cells in one launch.  Unless PIC_FLAG_NO_GRAPH is given, a step is the
 * replay of one captured graph.  Each member goes through the same kernels'
 * arithmetic as when stepped alone (tile by tile, the same workgroup code).
 *
 * Members are initialised runs (pic_init) sharing precision, ndim and the
 * bound stream; in 2D their tile edges may differ.  While a batch holds a
 * run, pic_step / pic_step_profiled / pic_destroy on it return PIC_E_STATE;
 * the read-out calls (pic_diagnostics, pic_read_fields, ...) work as usual.
 * Failures are described by pic_last_error(NULL, ...). */
typedef struct pic_batch pic_batch;

/* Host only.  Size of the device table of a batch of these runs.  Errors:
 * INVALID_ARG (nruns < 1, NULL or repeated run), UNSUPPORTED (mixed
 * precision or ndim). */
int pic_batch_query(int nruns, pic_run *const *runs, size_t *table_bytes);

/* Builds the batch: writes the work-item and block tables into the caller's
 * device buffer `table` (>= pic_batch_query's size, kept alive until
 * pic_batch_destroy) and captures the step graph (a failed capture fails the
 * call with PIC_E_HIP).  persistent_blocks:
 * workgroups of each particle launch (0 = as many as fit on the device at
 * once).  flags: PIC_FLAG_NO_GRAPH or 0.  Synchronising.  Errors as
 * pic_batch_query, plus BUFFER_TOO_SMALL, STATE (a run already in a batch),
 * INVALID_ARG (members on different streams). */
int pic_batch_init(int nruns, pic_run *const *runs, void *table, size_t table_bytes,
                   int32_t persistent_blocks, uint32_t flags, pic_batch **out);

/* Enqueues nsteps steps of every member on the shared stream (asynchronous). */
int pic_batch_step(pic_batch *batch, int32_t nsteps);

/* As pic_step_profiled, for the batch: group_ms[6] receives the summed
 * kernel milliseconds per kernel group over all members.  Synchronising. */
int pic_batch_step_profiled(pic_batch *batch, int32_t nsteps, double *group_ms);

/* Waits for the stream; returns the first member's failure, if any. */
int pic_batch_sync(pic_batch *batch);

/* Synchronising.  The most recent diagnostic record of member `run` (its
 * index in the runs given to pic_batch_init), as pic_diagnostics.  Errors:
 * INVALID_ARG (run out of range), STATE (no record yet). */
int pic_batch_diagnostics(pic_batch *batch, int run, pic_diag *out);

/* Host only.  For tile edges 8, 16, 32 (index 0..2): the particle kernel's
 * workgroups, work items (0 where no member uses the edge) and launch shape
 * (-1 where no member uses the edge).  The members of one edge share one
 * particle kernel, so pic_batch_init refuses members of one edge with
 * different shapes (PIC_E_INVALID_ARG).  Any pointer may be NULL. */
int pic_batch_info(pic_batch *batch, int32_t persistent_blocks[3], int32_t items[3], int32_t shapes[3]);

/* Host only.  How the batch enqueues its steps (pic_run_info; the fields
 * static_scratch, scratch_bytes and the shape fields are 0: the shapes are
 * per tile edge, see pic_batch_info). */
int pic_batch_launch_info(pic_batch *batch, pic_run_info *out);

/* Waits for the stream, releases the members and frees the host state. */
int pic_batch_destroy(pic_batch *batch);

/* ---- Tile autotuner --------------------------------------------------------
 * The tile edge sets the particles per workgroup (ppc * edge^ndim) and the
 * LDS footprint of the particle kernel.  pic_tune builds, inside the caller's
 * workspace, `copies` fresh device-loaded runs of the described configuration
 * (run indices grid->run + i) for every edge in {8, 16, 32} that divides each
 * resolved axis (3D: 8 only), times `nsteps` graph-replayed steps after
 * max(2, nsteps) warm-up steps -- of the run alone when copies == 1, of a batch of the
 * copies otherwise (enough copies fill the device, which is the situation of
 * a member of a large ensemble) -- and returns the fastest edge in
 * *best_tile and each candidate's milliseconds per step in ms[3] (edge 8,
 * 16, 32; -1 where not tried).  grid->tile and PIC_FLAG_HOST_LOAD are
 * ignored; every candidate runs in grid->shape.  Synchronising, on
 * `hip_stream`; the workspace may be reused once it returns.
 * pic_tune_query (host only) gives the workspace size, which also serves
 * pic_tune_shape.  Errors: INVALID_ARG (copies out of 1..4096, no edge
 * divides the grid, nsteps < 1), BUFFER_TOO_SMALL, and those of pic_init. */
int pic_tune_query(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
                   int32_t copies, size_t *workspace_bytes);
int pic_tune(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
             int32_t copies, void *workspace, size_t workspace_bytes, void *hip_stream,
             int32_t nsteps, int32_t *best_tile, double ms[3]);
/* The same measurement over the particle kernel's launch shapes at the
 * grid's tile edge (grid->tile, 0 = library default): ms[s] for shape s
 * (-1 where not tried: FP64 runs try shape 0 only), the fastest in
 * *best_shape.  grid->shape is ignored.  Errors as pic_tune, and
 * INVALID_ARG when the tile edge does not divide the grid. */
int pic_tune_shape(const pic_grid_desc *grid, const pic_species_desc *species, int nspecies,
                   int32_t copies, void *workspace, size_t workspace_bytes, void *hip_stream,
                   int32_t nsteps, int32_t *best_shape, double ms[PIC_PARTICLE_SHAPES]);

/* ---- The reduced quasi-neutral model ---------------------------------------
 * The paper's own model of the filamenting beam (the theory part, Eqs. 1-7):
 * the beam is kinetic in the transverse plane, the return-current plasma is
 * a cold fluid streaming along z with collisional drag, and the field is the
 * single potential a = e A_z/(m c^2) of Ampere's law without displacement
 * current.  In the units above, with local quasi-neutrality
 * n_p(x) = max(n0 - n_b(x), 0):
 *   lap a = n_b beta_bz + n_p beta_pz                         (Eq. 2)
 *   d_t psi = -nu beta_pz, psi = beta_pz - a                 (Eq. 3)
 *   d(u_perp)/dt = -(beta_z - beta_pz) grad a                 (Eq. 4)
 *   u_z = p_z + a, p_z the conserved canonical momentum       (Eq. 6)
 * so that B_perp = -e_z x grad a, E_z = -d_t a, E_perp = -beta_pz grad a
 * (Eq. 1), and Eq. (7) is conserved when nu = 0.  Numerics: nodes at
 * (i dx, j dy), periodic; cloud-in-cell deposit and gathers; grad a by
 * forward differences at ((i+1/2) dx, j dy) and (i dx, (j+1/2) dy); a^n from
 * Eq. (2) with the beam current linearised about a* = 2 a^(n-1) - a^(n-2)
 * (d beta_z/d u_z = (1 + u_perp^2)/gamma^3), solved by `iters` fixed-point
 * sweeps, each an FFT solve of lap - (n0 - <n_b>); leapfrog in time (x, a at
 * integer steps, u_perp at half steps).  Everything is FP64.
 *
 * Buffers (caller-owned device memory, sizes from pic_hyb_query):
 *  - particles: two copies (the cell sort alternates between them) of the
 *    SoA arrays x, y, u_x, u_y, p_z (FP64) and id (u32), each array on a
 *    256-byte boundary;
 *  - grid: a^(n-1), a^(n-2), psi, two solve iterates, two deposit sets
 *    (n_b, J at a*, chi, chi a*), one complex FFT plane, twiddle and
 *    Laplacian tables, counters, the sort's cell offsets, diagnostic
 *    partials and a ring of 4096 pic_hyb_diag records.
 * Errors are reported as for pic_run; pic_hyb_last_error describes them. */
typedef struct pic_hyb_desc {
    int32_t nx, ny;        /* nodes per axis: powers of two in 8..4096 */
    double dx, dy;         /* node spacing, c/w_p (> 0) */
    double dt;             /* time step, 1/w_p (> 0) */
    double nu;             /* collision rate of the return-current plasma (Eq. 3), w_p (>= 0) */
    double n0;             /* ion (background) density, n0 units: 1 in the paper's set-up (> 0) */
    double weight;         /* beam density carried by one macro-particle: n_b / ppc (>= 0) */
    int64_t nparticles;    /* beam macro-particles, 0..2^31 - 1 */
    int32_t iters;         /* fixed-point sweeps of the Eq. (2) solve per step, 1..64 */
    int32_t diag_every;    /* 0: no diagnostics; k: a record every k steps */
    int32_t sort_every;    /* 0: never; k: re-sort the particles by cell every k steps */
    uint32_t flags;        /* PIC_FLAG_NO_GRAPH or 0 */
} pic_hyb_desc;

/* One diagnostic record at time level n (energies per unit length in z, in
 * n0 m c^2 (c/w_p)^2): the terms of Eq. (7) and the field energies. */
typedef struct pic_hyb_diag {
    int64_t step;
    double time;
    double beam_energy;    /* dA sum_j w gamma_j^n, gamma^n = (gamma^- + gamma^+)/2 */
    double beam_a2;        /* dA sum_j w a(x_j)^2 / 2 */
    double grad_energy;    /* dA sum |grad a|^2 / 2 (staggered differences) */
    double a2_energy;      /* dA sum n0 a^2 / 2 */
    double eq7;            /* beam_energy - beam_a2 + grad_energy + a2_energy */
    double W_Bperp;        /* dA sum |B_perp|^2 = 2 grad_energy */
    double W_Ez;           /* dA sum ((a^n - a^(n-1))/dt)^2 */
    double beam_pz;        /* dA sum_j w u_z,j^n */
    double mean_a;         /* node mean of a^n */
    double mean_psi;       /* node mean of psi^n */
} pic_hyb_diag;

typedef struct pic_hyb pic_hyb;

/* Host only.  Validates the descriptor and gives the two buffer sizes.
 * Errors: INVALID_ARG (a field out of its range), UNSUPPORTED (a size that
 * is not a power of two in 8..4096). */
int pic_hyb_query(const pic_hyb_desc *desc, size_t *particle_bytes, size_t *grid_bytes);

/* Initialises a run on the current device and enqueues everything on
 * `hip_stream`: the host arrays (nparticles each; ids 0..N-1 follow this
 * order) are copied in, the beam current of the given u_z is deposited,
 * Eq. (2) is solved for a^0 (psi = 0: the plasma starts with the
 * neutralising return current beta_pz = a^0), and p_z = u_z - a^0(x) is
 * stored.  u_x, u_y are taken as u_perp^(-1/2).  Positions must lie in
 * [0, nx dx) x [0, ny dy).  Synchronising.  Errors: those of pic_hyb_query,
 * INVALID_ARG (NULL pointer, a position outside the box), BUFFER_TOO_SMALL,
 * HIP. */
int pic_hyb_init(const pic_hyb_desc *desc, void *particles, size_t particle_bytes, void *grid,
                 size_t grid_bytes, void *hip_stream, const double *x, const double *y, const double *ux,
                 const double *uy, const double *uz, pic_hyb **out);

/* Enqueues nsteps steps (one captured graph per step unless
 * PIC_FLAG_NO_GRAPH).  Asynchronous. */
int pic_hyb_step(pic_hyb *h, int32_t nsteps);

/* The same steps launched kernel by kernel with HIP events on each launch;
 * group_ms[4] receives the summed milliseconds of: the Eq. (2) solve, the
 * particle kernel, the grid update (psi, a, diagnostics), the cell sort and
 * step bookkeeping.  Synchronising. */
int pic_hyb_step_profiled(pic_hyb *h, int32_t nsteps, double *group_ms);

/* Waits for the stream; reports a device-side failure. */
int pic_hyb_sync(pic_hyb *h);

/* Synchronising.  Copies a^n of the last step (a^0 before the first) and
 * psi^(n+1) into host arrays of ny*nx doubles (row-major, x fastest); either
 * may be NULL. */
int pic_hyb_read_grid(pic_hyb *h, double *a, double *psi);

/* Synchronising.  Copies the particles (storage order; the cell sort
 * permutes them): x^(n+1), y^(n+1), u_perp^(n+1/2), p_z and the ids into
 * host arrays of nparticles entries; any pointer may be NULL. */
int pic_hyb_read_particles(pic_hyb *h, double *x, double *y, double *ux, double *uy, double *pz, uint32_t *id);

/* Synchronising.  Copies up to `max` of the most recent records, oldest
 * first; *n receives the count. */
int pic_hyb_diag_history(pic_hyb *h, pic_hyb_diag *out, int32_t max, int32_t *n);

/* Message of the last failure on h (h == NULL: of the last failed
 * pic_hyb_query / pic_hyb_init on this thread). */
int pic_hyb_last_error(pic_hyb *h, char *buf, size_t n);

/* Waits for the stream and frees the host state (not the caller's buffers). */
int pic_hyb_destroy(pic_hyb *h);

#ifdef __cplusplus
}
#endif
#endif /* PIC_H */
