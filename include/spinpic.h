/*
 * spinpic.h - C ABI of the spin-resolved particle-in-cell step for MI355X.
 *
 * One time step advances every macro-particle and the fields by dt:
 *   gather E, B at the particle from the staggered Yee grid (first order),
 *   relativistic Boris push of u = gamma*beta,
 *   Thomas-BMT spin precession ds/dt = -Omega x s with Omega of section 2
 *     Eq. 2 and the coefficients of Eq. 3 (a = the species' anomaly),
 *   position update, charge-conserving (Esirkepov) current deposition,
 *   Yee FDTD update of E and B.
 * The polarization of section 2 Eq. 4, P = (1/N) sum s_i over an ensemble
 * (a species within a kinetic-energy window), is reduced in FP64.
 *
 * Units: time 1/omega0, length c/omega0, u = p/(m c) of the species, fields
 * m_e c omega0 / e, densities (and particle weights) in n_c, J in e n_c c.
 * A species has charge Z (units of e), mass mu (units of m_e) and anomaly a.
 *
 * Conventions for every call:
 *   - Return value: PIC_OK (0) or a negative PIC_E* code; nothing throws or
 *     aborts.  pic_last_error() gives a human-readable reason.
 *   - Host pointers belong to the caller and are only read/written during
 *     the call.  Device memory belongs to the context; it comes from the
 *     caller's allocator when one is given, else from hipMalloc.
 *   - All GPU work is enqueued on the HIP stream given to pic_init.
 *     pic_step only enqueues (it does not wait for the GPU); every call that
 *     returns data to the host waits for the stream first.
 *   - A context is not thread-safe: one host thread at a time per context.
 */
#ifndef SPINPIC_H
#define SPINPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PIC_OK = 0,
    PIC_EINVAL = -1,      /* bad argument or configuration */
    PIC_ECFL = -2,        /* dt violates the Yee stability (Courant) limit */
    PIC_EHIP = -3,        /* a HIP runtime call failed */
    PIC_ECAPACITY = -4,   /* particle storage exhausted */
    PIC_ENONFINITE = -5,  /* a NaN or Inf was found in the state */
    PIC_ESTATE = -6,      /* call on a context that is NULL or unusable */
    PIC_ENOMEM = -7       /* device allocation failed */
};

enum { PIC_FP64 = 0, PIC_FP32_MIXED = 1 };

/* pic_config.deposit_acc */
enum { PIC_ACC_DEFAULT = 0, PIC_ACC_FP32 = 1, PIC_ACC_FP64 = 2 };

/* pic_config.flags */
enum {
    PIC_FLAG_TEST_PARTICLE = 1, /* fields frozen, no current deposit */
    /* Deterministic mode: bitwise-reproducible runs.  The current of a step is
     * summed as 64-bit fixed-point integers (units of 2^-S with S chosen at
     * pic_init so that the sum of |Z w| over all particles stays below 2^61
     * units: no node's current can pass it), inside each tile and across
     * tiles, and converted to FP64 before the field update; the polarization
     * of section 2 Eq. 4 is summed the same way (each spin component split in
     * two 31-bit integer parts).  Integer sums do not depend on the order of
     * the atomic additions, so two runs from the same state give bitwise
     * identical particles, fields and polarization, and so does a run started
     * again from pic_particles_cells and pic_fields (E, B) with
     * PIC_FLAG_CELL_ROWS.  The FP64 current then carries a rounding of 2^-S per
     * contribution instead of FP64 roundoff.  Not with pic_window and not in
     * batches (PIC_EINVAL). */
    PIC_FLAG_DETERMINISTIC = 2,
    /* The initial particle rows of pic_state are in cell form,
     * PIC_PARTICLE_CELL_COLS values: cell index along x, y, z (whole numbers,
     * 0 <= c < n; 0 on axes beyond ndim), in-cell offset along x, y, z (in
     * [0, 1); as pic_particles_cells returns them), ux uy uz, sx sy sz, w.
     * This is how a run is restarted exactly from its read-back. */
    PIC_FLAG_CELL_ROWS = 4
};

/* pic_fields mask bits; components are returned in this order */
enum {
    PIC_EX = 1u << 0, PIC_EY = 1u << 1, PIC_EZ = 1u << 2,
    PIC_BX = 1u << 3, PIC_BY = 1u << 4, PIC_BZ = 1u << 5,
    PIC_JX = 1u << 6, PIC_JY = 1u << 7, PIC_JZ = 1u << 8,
    PIC_RHO = 1u << 9
};

#define PIC_MAX_SPECIES 4
#define PIC_PARTICLE_IN_COLS 10   /* x y z ux uy uz sx sy sz w */
#define PIC_PARTICLE_OUT_COLS 11  /* id x y z ux uy uz sx sy sz w */
#define PIC_PARTICLE_CELL_COLS 13      /* cx cy cz ox oy oz ux uy uz sx sy sz w */
#define PIC_PARTICLE_CELL_OUT_COLS 14  /* id cx cy cz ox oy oz ux uy uz sx sy sz w */

typedef struct {
    double Z;   /* charge in units of e (electron: -1) */
    double mu;  /* mass in units of m_e (proton: 1836.15267343) */
    double a;   /* gyromagnetic anomaly of section 2 Eq. 3 */
} pic_species;

typedef struct {
    int32_t ndim;        /* 2 (x, y; d/dz = 0, three velocity components) or 3 */
    int32_t n[3];        /* cells per axis; n[2] is ignored in 2D.
                            2D: n[0], n[1] <= 65535; 3D: n[0], n[1] <= 2047, n[2] <= 1023 */
    double d[3];         /* cell size per axis (c/omega0) */
    double dt;           /* time step (1/omega0); dt^2 * sum 1/d^2 must be < 1 */
    int32_t precision;   /* PIC_FP64, or PIC_FP32_MIXED: particles stored and pushed
                            in FP32; E, B, J and the field update stay FP64, and so
                            do all reductions */
    int32_t nspecies;    /* 1 .. PIC_MAX_SPECIES */
    pic_species sp[PIC_MAX_SPECIES];
    int32_t tile[3];     /* tile edge in cells per axis; 0 selects the default
                            (16x16 in 2D, 12x6x6 in 3D FP32, 6x6x6 in 3D FP64) */
    double slack;        /* spare capacity per tile segment as a fraction of its
                            initial population (>= 0; 0 selects 0.25, or 1.0 for
                            3D FP64 with its smaller default tiles) */
    int32_t flags;       /* PIC_FLAG_* */
    int32_t deposit_acc; /* PIC_FP32_MIXED only: precision of the per-tile
                            shared-memory current sums that precede the one FP64
                            global add per node (PIC_ACC_*; PIC_ACC_DEFAULT is
                            FP64) */
} pic_config;

/* Initial state, all host memory in float64, copied during pic_init. */
typedef struct {
    int64_t count[PIC_MAX_SPECIES];           /* particles per species */
    const double* particles[PIC_MAX_SPECIES]; /* count[s] rows of PIC_PARTICLE_IN_COLS:
                                                 x y z (c/omega0; z ignored in 2D),
                                                 ux uy uz, sx sy sz (|s| = 1), w */
    const double* fields;  /* 6 components Ex Ey Ez Bx By Bz, each [nz][ny][nx] with
                              x fastest (nz = 1 in 2D), at their Yee positions;
                              NULL starts from zero fields */
} pic_state;

/* Optional device allocator; alloc returns NULL on failure.  A repack
 * allocates the new particle store (one array per particle field) before it
 * frees the old one; a store that must grow gets a quarter more slots than
 * it needs, and otherwise the size of the current one, so that a caching
 * allocator can serve each repack from the arrays the previous one freed. */
typedef struct {
    void* (*alloc)(void* user, size_t bytes);
    void (*free)(void* user, void* ptr);
    void* user;
} pic_allocator;

typedef struct pic_ctx pic_ctx;

/* Validate cfg, copy the initial state to the device sorted by tile, and
 * return a new context in *out.  Errors: PIC_EINVAL (bad sizes, species,
 * tile, precision, non-unit spin (| |s|^2 - 1 | above 1e-6, or 1e-4 with
 * PIC_FP32_MIXED, whose spins drift by that much over thousands of steps),
 * non-finite input, cell rows out of range), PIC_ECFL, PIC_ENOMEM,
 * PIC_EHIP.  alloc may be NULL; hip_stream may be NULL (the null stream). */
int pic_init(const pic_config* cfg, const pic_state* init, const pic_allocator* alloc,
             void* hip_stream, pic_ctx** out);

/* Enqueue nsteps >= 0 full time steps.  Returns PIC_ESTATE on a NULL or
 * failed context, PIC_EHIP when a launch fails, PIC_ECAPACITY when particle
 * storage is exhausted, PIC_ENONFINITE when the push has produced a NaN or
 * infinite momentum or spin: every push kernel probes its particles and sets
 * a device flag, which the host reads every 16 steps (every 4 while the
 * overflow store is large; it waits for the stream then anyway) and before
 * every read-back call. */
int pic_step(pic_ctx* ctx, int32_t nsteps);

/* Section 2 Eq. 4: mean spin of the particles of one species (species = -1:
 * all species) whose kinetic energy mu*(gamma-1)*0.51099895 MeV lies in
 * [ekin_min_mev, ekin_max_mev).  FP64.  Waits for the stream.  With no
 * particle selected, P_out is 0 and *N_out is 0. */
int pic_polarization(pic_ctx* ctx, int32_t species, double ekin_min_mev,
                     double ekin_max_mev, double P_out[3], int64_t* N_out);

#define PIC_MAX_RECORD_STEPS 65536

/* Per-step record of section 2 Eq. 4, summed by the push kernels while they
 * push (no pass over the particles of its own).  From this call on, every
 * step of pic_step records the mean spin and the count of the particles the
 * selection takes (species, or -1 for all; kinetic energy in
 * [ekin_min_mev, ekin_max_mev) MeV as for pic_polarization, infinite bounds
 * allowed) in the state the step leaves: what pic_polarization would return
 * after that step.  It differs from that only by the order of the FP64 sums,
 * and, with a moving window, the particles injected at the end of a step
 * enter from the next step on.  capacity (1 .. PIC_MAX_RECORD_STEPS): steps
 * the record holds; pic_step returns PIC_ECAPACITY, before enqueuing a step
 * that would not fit, until pic_polarization_history has emptied it.
 * capacity 0 stops recording and frees the record; another call starts a
 * new, empty one (after waiting for the stream).  Device memory: capacity x
 * 1 KiB, through the allocator.  Not in the deterministic mode (PIC_EINVAL). */
int pic_polarization_record(pic_ctx* ctx, int32_t species, double ekin_min_mev,
                            double ekin_max_mev, int32_t capacity);

/* The steps recorded since the record started or was last read, oldest
 * first: P_out[3 k .. 3 k + 2] the mean spin and N_out[k] the count of the
 * k-th (P 0 where the count is 0); *nsteps_out of them, 0 when no record is
 * kept.  cap: the entries N_out has room for (P_out: 3 cap); less than the
 * steps recorded is PIC_EINVAL.  Waits for the stream, then empties the
 * record.  PIC_ENONFINITE as pic_polarization. */
int pic_polarization_history(pic_ctx* ctx, double* P_out, int64_t* N_out, int32_t cap,
                             int32_t* nsteps_out);

/* Copy the masked components (PIC_EX ... PIC_RHO, in bit order) to host_out
 * as float64, each [nz][ny][nx] with x fastest.  J is the current of the last
 * step.  cap_doubles must hold popcount(mask)*cells values.  Waits. */
int pic_fields(pic_ctx* ctx, uint32_t mask, double* host_out, size_t cap_doubles);

/* Binned diagnostics (the energy spectra and polarization-versus-energy
 * plots of the paper's section 3).  All sums in FP64 on the device; all wait
 * for the stream.  Bins are equal over [lo, hi): a value v falls in bin
 * floor((v - lo) / (hi - lo) * nbins), capped at nbins - 1, and values outside
 * [lo, hi) are not counted.  Kinetic energy is mu*(sqrt(1 + u2) - 1)*0.51099895
 * MeV with u2 = (ux*ux + uy*uy) + uz*uz, summed in that order. */
#define PIC_MAX_SPECTRUM_BINS 1024

/* Energy spectrum of one species (species = -1: all) in nbins bins over
 * [emin, emax) MeV, 1 <= nbins <= PIC_MAX_SPECTRUM_BINS: count_out[b] number of
 * macro-particles, weight_out[b] sum of their weights, spin_out[3b + k] sum of
 * s_k, so that section 2 Eq. 4 for bin b is spin_out[3b + k] / count_out[b].
 * The three host arrays hold nbins, nbins and 3*nbins doubles.  Errors:
 * PIC_EINVAL for a bad species, nbins, range (need emin < emax, finite) or a
 * NULL array. */
int pic_spectrum(pic_ctx* ctx, int32_t species, double emin, double emax, int32_t nbins,
                 double* count_out, double* weight_out, double* spin_out);

/* pic_spectrum without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the bins are summed in a buffer the library holds
 * in static device memory, one per GPU (5 * PIC_MAX_SPECTRUM_BINS doubles,
 * 40 KiB, kept until the process ends), cleared by a kernel at the start of
 * every call and copied straight into the caller's arrays.  No hipMalloc,
 * hipFree, allocator callback or host allocation happens on this path.
 * Same arguments, results and errors as pic_spectrum; nbins above
 * PIC_MAX_SPECTRUM_BINS is PIC_EINVAL.  Calls that overlap on one GPU (from
 * several host threads, or on several streams) share the buffer and race:
 * keep them in sequence.  Waits for the stream. */
int pic_spectrum_noalloc(pic_ctx* ctx, int32_t species, double emin, double emax, int32_t nbins,
                         double* count_out, double* weight_out, double* spin_out);

/* Weighted position-momentum histogram of one species: position along axis
 * (0 .. ndim-1, in c/omega0, as pic_particles reports it) in nx bins over
 * [xmin, xmax), momentum mu*u_comp (comp 0 .. 2, in m_e c) in np bins over
 * [pmin, pmax); out[ix*np + ip] receives the sum of w (nx*np doubles,
 * nx*np <= 2^26).  Errors: PIC_EINVAL for bad arguments. */
int pic_phase_space(pic_ctx* ctx, int32_t species, int32_t axis, double xmin, double xmax,
                    int32_t nx, int32_t comp, double pmin, double pmax, int32_t np, double* out);

/* Number density of one species on the nodes: the cloud-in-cell sum of w
 * (the charge density of that species divided by Z), float64 [nz][ny][nx];
 * cap_doubles must hold the cell count. */
int pic_density(pic_ctx* ctx, int32_t species, double* out, size_t cap_doubles);

/* Copy the particles of one species, sorted by id (the row index in the
 * initial state), as rows of PIC_PARTICLE_OUT_COLS float64 values.  cap_doubles
 * must hold count*11 values; *n_out receives the count.  Waits. */
int pic_particles(pic_ctx* ctx, int32_t species, double* host_out, size_t cap_doubles,
                  int64_t* n_out);

/* As pic_particles, with each position as the particle's cell index and its
 * in-cell offset per axis, exactly as stored (rows of
 * PIC_PARTICLE_CELL_OUT_COLS: id, cx cy cz, ox oy oz, ux uy uz, sx sy sz, w;
 * 0 on axes beyond ndim).  Every value is the stored one converted to
 * float64 without rounding, so that pic_init with PIC_FLAG_CELL_ROWS (the
 * rows without the id column, in id order) restores the particles bit for
 * bit.  cap_doubles must hold count*14 values.  Waits. */
int pic_particles_cells(pic_ctx* ctx, int32_t species, double* host_out, size_t cap_doubles,
                        int64_t* n_out);

/* Test hook for the non-finite probe: overwrite u_x of one stored particle
 * of `species` (the first one of the first non-empty tile) with a NaN.  The
 * next pic_step's push then produces a non-finite state, which the probe in
 * the push kernel records: pic_step returns PIC_ENONFINITE at its next check
 * (every 16 steps at the latest) and the read-back calls return it at once.  Returns
 * PIC_EINVAL when the species has no particle in a tile.  Waits. */
int pic_test_poison(pic_ctx* ctx, int32_t species);

/* Diagnostics in FP64: out[0 .. nspecies-1] kinetic energy per species
 * (sum mu (gamma-1) w V), out[nspecies] field energy (sum (E^2+B^2)/2 V),
 * out[nspecies+1] max over nodes of |(div E - rho) - (div E - rho) at init|;
 * V is the cell volume.  cap must be >= nspecies + 2.  Waits. */
int pic_energy(pic_ctx* ctx, double* out, int32_t cap);

/* Counters since init: out[0] steps, out[1] particles that changed tile,
 * out[2] particles currently in the overflow store, out[3] repacks done,
 * out[4] particles in the box; with cap >= 8 also out[5 .. 7] the tile edge
 * in cells per axis in use (1 on axes beyond ndim); with cap >= 12 also
 * out[8 .. 11] the particles of each species in the box (what pic_particles
 * returns); with cap >= 13 also out[12] the moving window's shifts so far.
 * cap >= 5.  Waits. */
int pic_stats(pic_ctx* ctx, int64_t* out, int32_t cap);

/* ---------------------------------------------------------------------------
 * Co-moving window and open x faces (the co-moving frame of the paper's
 * runs, section 2).
 *
 * After pic_window the x axis is open: fields beyond the two x faces read as
 * zero for the gather, current deposited beyond them is lost, particles that
 * cross them leave the box, and the Yee update takes its ghost columns (E_y,
 * E_z beyond the high face, B_y, B_z beyond the low face) from Mur's
 * first-order absorbing condition: ghost(new) = inside(old) + k (inside(new)
 * - ghost(old)), k = (c dt - dx)/(c dt + dx), "inside" the column next to
 * the face.  It returns about 1e-5 of a normally incident pulse's energy and
 * 1 % at 30 degrees.  The Mur state starts from the first and last columns
 * at pic_window and again after every shift.  y and z stay periodic.
 *
 * The window moves along +x at `speed`: after step n it has travelled
 * n speed dt (n counted from the pic_window call), and whenever that reaches
 * another shift_cells cells the box shifts by shift_cells cells: fields and
 * the last step's current move shift_cells cells towards -x, the first
 * shift_cells columns of particles leave, and the last shift_cells columns
 * start with zero fields and cold plasma.  Injection puts ppc particles of
 * every species into each new cell whose centre (lab frame, x measured from
 * the box's position at pic_window) sees density
 *     n(x) = n0 min(1, max(0, (x - ramp_start) / ramp_len))   (ramp_len > 0)
 *     n(x) = n0 for x >= ramp_start, else 0                    (ramp_len = 0)
 * with n > 0, at in-cell offset (q + 1/2)/ppc along every axis (q = 0 ..
 * ppc-1), u = 0, spin s0 and weight n/ppc.  Particle q of column c (0 ..
 * shift_cells-1 from the first new column) in cell row (y, z) of a species
 * gets id next + ((z ny + y) shift_cells + c) ppc + q, where next starts at
 * the species' initial count and advances by nz ny shift_cells ppc per
 * shift.  Ids of the initial particles are their row indices; pic_particles
 * returns the particles in the box sorted by id, with positions in box
 * coordinates.
 * ------------------------------------------------------------------------- */
typedef struct {
    double speed;          /* window velocity along +x, units of c (0: a fixed box with open x faces) */
    int32_t shift_cells;   /* cells per shift: a multiple of the tile's x edge, below n[0] */
    int32_t ppc;           /* injected particles per cell and species, 0 .. 256 (0: none) */
    double n0;             /* injected density, n_c */
    double ramp_start;     /* lab-frame x (c/omega0) where the injected density starts */
    double ramp_len;       /* length of the linear ramp to n0 (c/omega0); 0: a step */
    double s0[3];          /* injected spin, |s0| = 1 (when ppc > 0) */
} pic_window_config;

/* Open the x faces and start the window (a later call replaces the
 * parameters and restarts the travel count).  The reference of the
 * div E - rho diagnostic is taken again with the open faces.  Errors:
 * PIC_EINVAL for parameters outside the ranges above, PIC_ECAPACITY when
 * the ids of injected particles would pass 2^31.  Waits. */
int pic_window(pic_ctx* ctx, const pic_window_config* w);

/* Per-kernel GPU timing with HIP events on the context's stream.
 * pic_timing(ctx, 1) starts (and resets) recording of every kernel class,
 * pic_timing(ctx, 2) of the push+deposit kernel only (no events between the
 * other kernels of a step, whose launches then follow each other without
 * them), 0 stops it; other values are PIC_EINVAL.
 * pic_timing_read fills ms_out[k] (total milliseconds) and launches_out[k]
 * for k = 0 push+deposit (including the compaction of the slots tile
 * leavers vacate), 1 overflow push, 2 insertion of tile leavers, 3 field
 * update (one fused Yee pass per step); cap >= 4.  Waits. */
int pic_timing(pic_ctx* ctx, int32_t enable);
int pic_timing_read(pic_ctx* ctx, double* ms_out, int64_t* launches_out, int32_t cap);

/* Reason for the last failure on ctx, or of the last failed pic_init on this
 * thread when ctx is NULL.  Owned by the library; valid until the next call. */
const char* pic_last_error(const pic_ctx* ctx);

/* Release every device buffer of ctx (through the allocator it was created
 * with) after waiting for its stream.  NULL is ignored. */
void pic_free(pic_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Batches: many independent 2D runs of uneven size stepped together.
 *
 * The runs share one particle store and concatenated field arrays; a step is
 * one persistent push over the tiles of every run (largest tiles first, the
 * workgroups taking tiles from a queue until none is left), one overflow
 * push, one leaver insertion and one field-update launch, whatever the
 * number of runs.  Each run is the step of pic_step on its own grid.
 * ------------------------------------------------------------------------- */
typedef struct pic_batch pic_batch;

/* nrun runs (1..65535) from cfgs[r], inits[r] (as for pic_init; host memory,
 * copied).  All runs must be 2D with the same precision, species, flags,
 * deposit_acc and slack; grids, cell sizes, time steps, tiles and particles
 * may differ.  Runs whose cfg tile is 0 x 0 get 16 x 16, or with
 * autotune != 0 a square tile of 8, 12, 16, 24 or 32 cells (clipped to the
 * grid) chosen by timing the batch: first every such run at each candidate
 * (the fastest push launch gives c*), then each run at the candidate not
 * larger than c* under which its tiles took the smallest share of the
 * launch; the per-run choice is kept only if its launch is faster than c*
 * for all.  (The largest tile of a batch sets how many workgroups of the
 * persistent push fit on a compute unit.)  Errors as pic_init, with the run
 * named in pic_batch_last_error. */
int pic_batch_init(int32_t nrun, const pic_config* cfgs, const pic_state* inits, int32_t autotune,
                   const pic_allocator* alloc, void* hip_stream, pic_batch** out);

/* Enqueue nsteps >= 0 steps of every run. */
int pic_batch_step(pic_batch* b, int32_t nsteps);

/* As pic_polarization, pic_fields (E, B, J only) and pic_particles, for run
 * `run`.  Wait. */
int pic_batch_polarization(pic_batch* b, int32_t run, int32_t species, double ekin_min_mev,
                           double ekin_max_mev, double P_out[3], int64_t* N_out);
int pic_batch_fields(pic_batch* b, int32_t run, uint32_t mask, double* host_out, size_t cap_doubles);
int pic_batch_particles(pic_batch* b, int32_t run, int32_t species, double* host_out,
                        size_t cap_doubles, int64_t* n_out);

/* Run `run`: out[0], out[1] its tile, out[2] its particles, out[3] its cells. */
int pic_batch_info(pic_batch* b, int32_t run, int64_t out[4]);

/* The autotuner's measurements: *ncand_out candidate tile edges into
 * cand_out (cap_cand >= *ncand_out); ns_out[r * ncand + c] the push time
 * per particle-step of run r under candidate c: the summed durations of its
 * tiles over the number of workgroups of the persistent push, which run side
 * by side (0 where not tried); kernel_ms_out[c] (ncand + 1 entries) the mean
 * push launch with the tunable runs at candidate c, and kernel_ms_out[ncand]
 * with the per-run choice (0 if every run chose c*).  *ncand_out is 0 when
 * nothing was tuned. */
int pic_batch_tuning(pic_batch* b, int32_t* cand_out, double* ns_out, double* kernel_ms_out,
                     int32_t cap_cand, int32_t* ncand_out);

/* As pic_stats (out[5] workgroups of the persistent push, out[6] tiles of
 * all runs when cap >= 7), pic_timing and pic_timing_read. */
int pic_batch_stats(pic_batch* b, int64_t* out, int32_t cap);
int pic_batch_timing(pic_batch* b, int32_t enable);
int pic_batch_timing_read(pic_batch* b, double* ms_out, int64_t* launches_out, int32_t cap);

const char* pic_batch_last_error(const pic_batch* b);
void pic_batch_free(pic_batch* b);

/* ---------------------------------------------------------------------------
 * Differentiable test-particle spin tracking.
 *
 * n independent particles of one species cross an analytic linear wake moving
 * at c along z; each step is the PIC step's Boris push and Thomas-BMT spin
 * rotation (section 2 Eq. 1-3) with the fields evaluated at the particle,
 * xi = z - t, S = sin(kp xi), C = cos(kp xi):
 *     E = (E0 kp x S / 2, E0 kp y S / 2, E0 C),  B = (-E0 kp y S / 4, E0 kp x S / 4, 0)
 * (E_z = E0 cos, radial E_r = E0 kp r / 2 sin, azimuthal B_phi = E_r / 2).
 * Positions sit at t = n dt, momenta u = gamma beta and spins half a step
 * earlier.  The forward pass returns P, the polarization of section 2 Eq. 4
 * over all n particles after the last step; the backward pass returns the
 * gradient of J = c . P with respect to E0, kp and every initial position,
 * momentum and spin, by the adjoint of the discrete map (not of the ODE),
 * recomputing K-step segments from states kept every K steps.
 * ------------------------------------------------------------------------- */
typedef struct {
    double Z, mu, a;       /* species: charge / e, mass / m_e, anomaly */
    double dt;             /* time step (1/omega0), > 0 */
    int32_t nsteps;        /* steps of a run, >= 0 */
    int32_t checkpoint;    /* K: the state is kept every K steps, 1 <= K */
    int32_t precision;     /* PIC_FP64, or PIC_FP32_MIXED: trajectory and adjoint
                              in FP32, sums over particles in FP64 */
} pic_track_config;

typedef struct pic_track pic_track;

/* Allocate the device buffers for n >= 1 particles (states, ceil(nsteps/K)
 * checkpoints and K scratch states, 9 values each per particle).  alloc and
 * hip_stream as for pic_init.  Errors: PIC_EINVAL, PIC_ENOMEM, PIC_EHIP. */
int pic_track_create(const pic_track_config* cfg, int64_t n, const pic_allocator* alloc,
                     void* hip_stream, pic_track** out);

/* Run the trajectories for field parameters (E0, kp) from x0, u0, s0 (host,
 * n rows of 3 float64 each, row-major).  P_out[3] receives the final
 * polarization; x_out, u_out, s_out (host, n x 3, each may be NULL) the final
 * state.  Keeps the checkpoints for pic_track_backward.  Waits.  Errors:
 * PIC_EINVAL (NULL input, non-finite value), PIC_EHIP. */
int pic_track_forward(pic_track* tr, double E0, double kp, const double* x0, const double* u0,
                      const double* s0, double P_out[3], double* x_out, double* u_out,
                      double* s_out);

/* Gradient of J = c . P for the last forward run: grad_theta[0] = dJ/dE0,
 * grad_theta[1] = dJ/dkp; grad_x0, grad_u0, grad_s0 (host, n x 3, each may be
 * NULL) dJ/d(initial state); grad_theta_each (host, n x 2, may be NULL) each
 * particle's share of the two parameter derivatives.  Waits.  Errors:
 * PIC_ESTATE without a forward run, PIC_EINVAL, PIC_EHIP. */
int pic_track_backward(pic_track* tr, const double c[3], double grad_theta[2], double* grad_x0,
                       double* grad_u0, double* grad_s0, double* grad_theta_each);

/* Kernel times of the last forward and backward runs in ms (HIP events on
 * the handle's stream): ms_out[0] forward, ms_out[1] backward. */
int pic_track_timing(pic_track* tr, double ms_out[2]);

/* Reason for the last failure on tr, or of the last failed pic_track_create
 * on this thread when tr is NULL. */
const char* pic_track_last_error(const pic_track* tr);

/* Release the handle and its device buffers.  NULL is ignored. */
void pic_track_free(pic_track* tr);

#ifdef __cplusplus
}
#endif

#endif /* SPINPIC_H */
