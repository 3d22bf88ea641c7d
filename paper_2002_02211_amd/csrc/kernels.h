// Host-side launchers of the HIP kernels (internal to libspinpic).
#pragma once

#include "common.h"

namespace spinpic {

using freal = double;   // grid fields E, B, J

template <typename real, typename acc_t>
size_t tile_lds_bytes(const Geom& g, int max_chunks);

// Per-step record of section 2 Eq. 4, summed by the push kernels while they
// push: the three spin sums and the count of the selected particles (one
// species, or -1 for all; with window set, kinetic energy in [emin, emax)
// MeV, evaluated as the on-demand reduction does), each workgroup adding its
// sums into slot (workgroup index mod kRecSlots) of acc, kRecStride doubles
// a slot; the host adds the slots up.
constexpr int kRecSlots = 32;
constexpr int kRecStride = 4;
struct RecArgs {
    double* acc;   // nullptr: no record
    int species;
    int window;
    double emin, emax;
    double mu[kMaxSpecies];
};

template <typename real, typename acc_t, int DIM>
hipError_t launch_push_tiles(const Geom& g, const Consts<real>& k, const PArrays<real>& p,
                             const Segs& seg, const PArrays<real>& lv, int32_t* ctr, int slot,
                             const Fields<freal>& f, int deposit, const RecArgs& rec, hipStream_t stream);

// 3D push marching along z over runs of R tiles of one tile column (field
// and current guard planes carried between the tiles of a run); T[2] >= 3.
template <typename real, typename acc_t>
hipError_t launch_push_march(const Geom& g, const Consts<real>& k, const PArrays<real>& p, const Segs& seg,
                             const PArrays<real>& lv, int32_t* ctr, int slot, const Fields<freal>& f, int deposit,
                             int R, int xcd_major, hipStream_t stream);

template <typename real, int DIM>
hipError_t launch_push_stash(const Geom& g, const Consts<real>& k, const PArrays<real>& st,
                             int32_t* ctr, const Fields<freal>& f, int deposit, const RecArgs& rec,
                             int blocks, hipStream_t stream);

template <typename real, int DIM>
hipError_t launch_insert(const Geom& g, const PArrays<real>& p, const Segs& seg,
                         const PArrays<real>& lv, const PArrays<real>& st, int32_t* ctr, int slot,
                         unsigned long long* moved, int blocks, hipStream_t stream);

template <typename real>
hipError_t launch_repack_segments(const PArrays<real>& from, const PArrays<real>& to,
                                  const int32_t* old_start, const int32_t* new_start,
                                  const int32_t* count, int nseg, int ndim, hipStream_t stream);

// ---- batches of independent 2D runs in shared stores
// Run r's fields start at cell cell_off of the concatenated field arrays, its
// segments at sid_base and its tiles at tile_base; its leavers and overflow
// particles carry r * kMaxSpecies + species in the species word.
template <typename real>
struct RunDesc {
    Geom g;
    Consts<real> k;      // particle constants (push precision)
    Consts<freal> kf;    // field-update constants
    long long cell_off;
    int sid_base;
    int tile_base;
    int yee_blk_base;    // first block of this run in the field-update launch
};

struct TileRef {
    int run;
    int t;   // tile index within the run
};

// The batched push's queues: the work list cut into 8 contiguous chunks,
// one per XCD (chunk x = items [start[x], start[x + 1])).
struct XcdQueues {
    int start[9];
};

// Persistent push: blocks workgroups (a multiple of 8) take tiles from the
// queue of their XCD, then from the others; run_ns (nruns counters, may be
// NULL) accumulates each run's tile time.
template <typename real, typename acc_t>
hipError_t launch_push_tiles_batch(const RunDesc<real>* runs, const TileRef* order, const XcdQueues& q, int blocks,
                                   size_t lds, const PArrays<real>& p, const Segs& seg, const PArrays<real>& lv,
                                   int32_t* ctr, int slot, const Fields<freal>& f, int deposit,
                                   unsigned long long* run_ns, hipStream_t stream);
// Workgroups of the batched push that fit on one CU with lds bytes of shared memory.
template <typename real, typename acc_t>
int push_batch_blocks_per_cu(size_t lds);
template <typename real>
hipError_t launch_push_stash_batch(const RunDesc<real>* runs, const PArrays<real>& st, int32_t* ctr,
                                   const Fields<freal>& f, int deposit, int blocks, hipStream_t stream);
template <typename real>
hipError_t launch_insert_batch(const RunDesc<real>* runs, const PArrays<real>& p, const Segs& seg,
                               const PArrays<real>& lv, const PArrays<real>& st, int32_t* ctr, int slot,
                               unsigned long long* moved, int blocks, hipStream_t stream);
// Field update of every run (fused Yee step, periodic): each run covered
// by its own blocks, yee_blocks(nx, ny) of them from runs[r].yee_blk_base
// on; blk_run[b] is the run of block b (nblocks in all).  Reads f, writes
// out (distinct arrays of the same size); zeroes jclear.
int yee_blocks(int nx, int ny);
template <typename real>
hipError_t launch_yee_fused_batch(const RunDesc<real>* runs, const int32_t* blk_run, int nblocks,
                                  const Fields<freal>& f, const Fields<freal>& out, freal* const* jclear,
                                  hipStream_t stream);

// Moving window.  A shift moves the box S cells along +x: every field array
// shifts S cells towards -x with zeros in the last S columns (dst must not
// alias src), the particles of the kept segments move S cells down in x,
// and cold plasma is injected into the last S columns.
struct InjectArgs {
    int S;                 // columns injected: the last S of the box
    int ppc;               // particles per cell and species
    long long origin;      // cells from the lab-frame origin to the box's first cell
    double dx;
    double n0, ramp_start, ramp_len;   // lab-frame density: n0 times a ramp (a step if ramp_len is 0)
    double s0[3];
    int32_t next_id[kMaxSpecies];      // id of the species' first particle of this shift
};
template <typename freal>
hipError_t launch_shift_x(const Geom& g, const freal* src, freal* dst, int S, hipStream_t stream);
template <typename real, int DIM>
hipError_t launch_shift_cells(const PArrays<real>& p, const Segs& seg, int S, int nseg, hipStream_t stream);
// The segment table rotated by k tile columns into `to` (no aliasing with
// `from`): segment d takes the start, capacity and count of the segment k
// columns further along x; the last k columns take the slots of the first k
// columns, with count 0.
hipError_t launch_rotate_segments(const Geom& g, const Segs& from, const Segs& to, int k, hipStream_t stream);
// Overflow-store particles moved S cells towards -x; those that thereby
// leave the box are marked dead.  The store's size is read on the device.
template <typename real, int DIM>
hipError_t launch_shift_stash(const PArrays<real>& st, const int32_t* ctr, int S, hipStream_t stream);
template <typename real, int DIM>
hipError_t launch_inject(const Geom& g, const PArrays<real>& p, const Segs& seg, const PArrays<real>& st,
                         int32_t* ctr, const InjectArgs& a, hipStream_t stream);

// The whole Yee step (B half step, E step with -dt J, B half step) in one
// pass: reads f.E, f.B, f.J, writes out.E and out.B (distinct arrays of the
// same size) and zeroes the three current arrays jclear (may be NULL).
// With open x faces (g.open_x) it reads the Mur state from f.mur and writes
// the advanced state to out.mur (distinct, MUR_COLUMNS x ny nz values each);
// hipErrorInvalidValue if either is missing.
template <typename real, int DIM>
hipError_t launch_yee_fused(const Geom& g, const Consts<real>& k, const Fields<real>& f, const Fields<real>& out,
                            real* const* jclear, hipStream_t stream);
// Mur state of open x faces (f.mur) started from the current fields.
template <typename real, int DIM>
hipError_t launch_mur_reset(const Geom& g, const Fields<real>& f, hipStream_t stream);

// FP64 reductions.  acc receives sums by atomic adds and must be zeroed first.
//   polarization: acc[0..2] += s, acc[3] += 1 over the selected particles.
//   kinetic:      acc[sp] += mu (gamma - 1) w.
//   rho:          rho (ncells doubles) += CIC charge Z w on the nodes (one
//                 species, or all with species = -1).
struct ReduceArgs {
    int run;                // overflow-store particles of this run only (0 outside batches)
    int species;            // -1 = all
    double emin, emax;      // MeV window [emin, emax)
    double mu[kMaxSpecies];
    double Z[kMaxSpecies];
};

// The particle reductions add workgroup w's sums into slot w mod kRedSlots of
// acc (kRedStride doubles a slot), so that the adds of tens of thousands of
// workgroups do not all go to the same few addresses; the caller clears
// kRedSlots * kRedStride doubles and adds the slots up.
constexpr int kRedSlots = 32;
constexpr int kRedStride = 8;

template <typename real, int DIM>
hipError_t launch_reduce_particles(int mode, const Geom& g, const PArrays<real>& p,
                                   const Segs& seg, const PArrays<real>& st, const int32_t* ctr,
                                   const ReduceArgs& ra, double* acc, double* rho,
                                   hipStream_t stream);
enum { RED_POLARIZATION = 0, RED_KINETIC = 1, RED_RHO = 2 };

// Binned diagnostics over all particles (tiles and overflow store).
//   spectrum: out[b] += 1, out[nbins + b] += w, out[2 nbins + 3 b + k] += s_k
//             for kinetic energy in bin b of [lo, hi) (species -1: all);
//   phase:    out[ix * np + ip] += w for position x_axis in bin ix of
//             [lo, hi) and mu u_comp in bin ip of [plo, phi) (one species).
struct BinArgs {
    int mode;
    int species;
    double lo, hi;
    int nbins;
    int axis, comp;
    double plo, phi;
    int np;
    double d[3];
    double mu[kMaxSpecies];
};
enum { BIN_SPECTRUM = 0, BIN_PHASE = 1 };

template <typename real, int DIM>
hipError_t launch_bin_particles(const Geom& g, const PArrays<real>& p, const Segs& seg,
                                const PArrays<real>& st, const int32_t* ctr, const BinArgs& ba,
                                double* out, hipStream_t stream);

// Field energy: acc[0] += sum (E^2 + B^2) / 2 over the cells.
template <typename real>
hipError_t launch_field_energy(const Geom& g, const Fields<real>& f, double* acc,
                               hipStream_t stream);

// div E - rho - ref at every node; per-block maxima of |.| into blockmax
// (blocks entries), and, when ref_out is non-NULL, the value itself.
struct Vec3d {
    double v[3];
};

template <typename real, int DIM>
hipError_t launch_div_residual(const Geom& g, const Vec3d& inv_d,
                               const Fields<real>& f, const double* rho, const double* ref,
                               double* ref_out, double* blockmax, int blocks, hipStream_t stream);

// Deterministic mode.  Section 2 Eq. 4 summed as integers: acc[k] += hi,
// acc[3 + k] += lo of each selected s_k (s_k = (hi + lo 2^-31) 2^-31), acc[6]
// += 1; acc must be zeroed first.  And the current's fixed-point words
// turned into their FP64 values in place (value = integer * inv_scale).
template <typename real, int DIM>
hipError_t launch_polarization_fixed(const Geom& g, const PArrays<real>& p, const Segs& seg, const PArrays<real>& st,
                                     const int32_t* ctr, const ReduceArgs& ra, unsigned long long* acc,
                                     hipStream_t stream);
hipError_t launch_fixed_to_double(double* const J[3], long long n, double inv_scale, hipStream_t stream);

// out[0 .. n) = 0 (a kernel, not a memset).
hipError_t launch_fill_zero(double* out, long long n, hipStream_t stream);

// Non-finite probe over particle momenta/spins and fields: flag[0] = 1 if any.
template <typename real>
hipError_t launch_nonfinite(const real* data, long long n, int32_t* flag, hipStream_t stream);

}  // namespace spinpic
