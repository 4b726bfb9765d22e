// Host-side context of the PIC-MCC library and the launchers each kernel
// file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "pic.h"
#include "pic_device.h"

// Forward pass of the warm-start network on the caller's stream with the
// input x of a D x H x W grid; *out receives the network's output buffer.
// False if the grid does not fit the network.
bool pic_unet_infer(pic_unet* u, const float* x, int D, int H, int W,
                    hipStream_t st, const float** out);
// The grid D x H x W is within the network's maximum.
bool pic_unet_fits(const pic_unet* u, int D, int H, int W);

namespace pic {

// One multigrid level: nx*ny*(nz+1) nodes with spacing 2^l dx.  Equations
// on level l are scaled by dx^2: (6u - sum of neighbours) = h2 * f with
// h2 = 4^l.
struct Level {
  int nx, ny, nz;
  long long nnodes;
  double h2;
  double *u, *f;       // FP64 unknowns and right-hand side
  float *uf, *ff;      // FP32 counterparts (mixed-precision V-cycles)
  double* us;          // spare FP64 / FP32 unknowns: target of the fused
  float* usf;          // pre-smoothing pass, source of the post-smoothing
};

// Largest coarse level the exact (spectral) solve takes: nodes per axis in
// x and y (powers of two by FFT up to kSpecMaxFFT, other even sizes by a
// direct transform up to kSpecMaxXY), unknown planes in z.
constexpr int kSpecMaxXY = 32, kSpecMaxFFT = 64, kSpecMaxPlanes = 256;
// Removed ions a step can list for the in-place removal (more: full binning).
constexpr int kDeadList = 4096;

struct QueueCall {
  int species;
  long long n, offset;
};

}  // namespace pic

struct pic_ctx {
  pic_config cfg;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  pic::GridC g;
  long long nnodes, ncells, ntiles;
  bool mixed;

  // Particles: two buffers per species (binning ping-pong).
  pic::Parts P[4][2];
  pic::PartsM PM[4][2];
  int cur[4];
  uint32_t* key[4];          // cell index of each particle, or kDead
  uint32_t* tsb[4][2];       // ntiles + 1 offsets of the binned order
  int tcur[4];               // which tsb buffer holds the current order
  uint32_t* tile_cursor;     // scatter cursors
  uint32_t* tcnt[2];         // destination-tile counts of the tile push (e, ion)
  bool tcounted;             // tcnt holds this step's counts
  uint32_t* scan_block;      // block sums of the tile scan
  long long n_binned[4];     // particles covered by the tile ranges
  uint2* chunks;             // (tile, piece) work list of the charged species
  uint32_t* cstart;          // ntiles + 1 chunk offsets
  long long nch_bound;       // host bound of the chunk count
  long long nch_cap;         // capacity of the chunk list
  // Neutrals are compacted in place between full binning passes.
  uint32_t* cmp_idx;         // holes then movers, capacity[1] each

  // Node fields.
  long long* acc;            // int64 charge units
  double* E;                 // FP64: 4 doubles per node; mixed: 4 floats
  int nlev;
  pic::Level lev[16];
  // Exact solve of one coarse level (DFT in x, y; tridiagonal in z per
  // mode), in the V-cycle's precision; spec_level < 0: none.
  int spec_level;
  int spec_modes, spec_planes;   // ny * (nx/2 + 1); unknown planes
  void* spec_s;                  // spectrum, planes x modes x (re, im)
  void* spec_m;                  // inverse pivots, planes x modes
  bool spec_ready;               // pivots computed
  double* partials;          // reduction partials
  double* part_n;            // neutral push partials (one per workgroup)
  int npartials;
  long long* qpartials;      // integer reduction partials

  // Collisions and ionisation matching.
  int* ncount;               // neutrals per cell
  bool ncount_valid;         // ncount counts the first n_start1 neutrals
  long long* acc_next;       // charge of the state the last advance left
  bool acc_next_valid;       // ... and it is the current particles'
  // Ions are binned again only when one left the domain, or when the
  // ions out of tile order (unbinned tail, binned ones that crossed a tile
  // face since the last pass) pass a bound; the decision reads this step's
  // counters while the electrons bin.
  long long ion_moved_accum;
  bool ions_binned;          // this step binned them
  pic::Counters* hmid;       // pinned copy of the counters for it
  uint32_t* dead1;           // indices of this step's removed neutrals
  uint32_t* dead2;           // indices of this step's removed ions
  uint2* rm_pairs;           // (hole, mover) slots of a listed removal
  hipEvent_t ev_mid;
  pic::Counters* hpin;       // pinned landing buffer of the counter readbacks
  hipEvent_t ev_sync;        // polled by stream_wait
  long long n_start1;        // neutrals at the start of the step's sources
  uint32_t* flag;            // cells holding ionisation events (one bit each)
  pic::CandRec* cand;        // null-collision candidates
  uint32_t* cand_cnt;        // candidates per tile
  uint32_t* el_cnt;          // elastic collisions per tile (+ tail)
  pic::Rec *ev, *nc, *ok;    // events, neutral candidates, matched events
  uint2* okp;                // (electron, neutral) index of a matched event
  pic::Rec* rec_tmp;         // merge buffer of the record sorts
  long long ev_cap_p2;       // power-of-two capacity of the record lists

  // Cathode-absorbed list: raw (unsorted) and sorted outputs.
  pic::Rec* ab_rec;
  double *ab_raw_pos, *ab_raw_vel;
  int32_t* ab_species;
  uint64_t* ab_id;
  double *ab_pos, *ab_vel;

  // Injection queue and Fowler-Nordheim scratch.
  double *q_pos, *q_vel;
  unsigned* fn_scan;         // nx*ny + 1

  // Cell grouping (buffers only with PIC_FLAG_CELL_GROUPS): counts per key
  // (cell for the ion processes, half tile for the Coulomb pass), their
  // offsets and scan block sums; the ion processes' records (scatter and
  // cell order) and list of crowded cells with its counter; the Coulomb
  // pass's index words of the charged particles by half tile.
  pic_coulomb coul;
  unsigned *cg_cnt, *cg_off, *cg_bsum, *cg_big, *cg_nbig;
  pic::Rec* cg_rec;
  pic::Rec* cg_srt;
  long long cg_work_cap;            // records: all particles' capacity
  unsigned* cg_idx;                 // index words binned by tile plane
  unsigned* cg_poff;                // tile planes' offsets into cg_idx
  unsigned* cg_hot;                 // planes of many records (ion processes)
  unsigned* cg_hpre;                // their sizes prefixed
  unsigned* cg_rest;                // planes whose small cells k_ip_small runs
  long long cg_big_cap;
  long long cg_nkeys;               // tile-major cell numbers (tiles x 512)
  // Recombination, Cu+ ionisation, charge exchange: settings and the listed
  // Cu+ ionisations (sort records, (electron, ion) index pairs).
  pic_ion_processes ionp;
  pic::Rec* ip_ev;
  uint2* ip_evp;

  // Debye-length check: per-block moments of electrons and ions, block
  // partials of its reductions and its four results.
  double* dbg_mom;
  long long* dbg_qpart;
  double* dbg_part;
  double* dbg_out;

  pic::Counters* dc;         // device counters
  pic::Counters hc;          // host copy after the last sync

  // Host mirrors (exact after each synchronising call).
  long long n[4];
  unsigned long long next_id;
  unsigned long long next_id_src;  // first id after the host-known sources
  long long step;
  pic_collisions coll;
  pic_sources src;
  std::vector<pic::QueueCall> queue;
  long long queue_used;
  int last_vcycles;
  pic_solve_info last_solve;

  // Warm start of the field solve (PIC_WS_*), the attached network and the
  // recorded (input, previous potential) of the last solve.
  int warm_mode;
  pic_unet* net;
  float* warm_x;             // (nz, ny, nx, 2) network input
  double* warm_prev;         // potential before the warm start, all nodes
  bool warm_recorded;
  double* phi_hist;          // potential of the step solve before the last
  bool u_solved;             // lev[0].u is the last step solve's result
  bool hist_valid;           // phi_hist is the step solve before that one
  std::string err;

  // Optional phase timing (HIP events on the context's stream).
  bool timing;
  bool ev_made;
  // Up to kTimeIv intervals per phase between two collections (one step).
  static constexpr int kTimeIv = 256;
  hipEvent_t tev[PIC_NPHASES][kTimeIv][2];
  int tn[PIC_NPHASES];
  double tms[PIC_NPHASES];
  long long tcalls[PIC_NPHASES];
};

namespace pic {

// Wait for everything queued on the context's stream by polling an event:
// a blocking wait wakes the host some ten microseconds after the GPU is
// done, and the GPU stays idle until the host queues more work.
inline hipError_t stream_wait(pic_ctx* c) {
  // A context without its event (the allocation-free solve) waits plainly.
  if (!c->ev_sync) return hipStreamSynchronize(c->stream);
  hipError_t e = hipEventRecord(c->ev_sync, c->stream);
  if (e != hipSuccess) return e;
  while ((e = hipEventQuery(c->ev_sync)) == hipErrorNotReady) {
  }
  return e;
}

// Record the start (begin = true) or end of a timed phase.
inline void tmark(pic_ctx* c, int ph, bool begin) {
  if (!c->timing) return;
  const int i = c->tn[ph];
  if (i >= pic_ctx::kTimeIv) return;
  hipEventRecord(c->tev[ph][i][begin ? 0 : 1], c->stream);
  if (!begin) c->tn[ph] = i + 1;
}

// ---- field (k_field.hip) ---------------------------------------------------
void field_rhs(pic_ctx* c, const double* rho_or_null);
void field_solve(pic_ctx* c, bool warm, pic_solve_info* info, int* status);
void field_efield(pic_ctx* c);
// Target (phi - phi_prev) / sigma of the last recorded solve, (nz, ny, nx).
void field_warm_target(pic_ctx* c, float* t);
void field_phi_to_level0(pic_ctx* c);
// Extrapolated start (phi = 2 phi - phi_hist, phi_hist = old phi) when the
// history is valid, else the history is just filled.
void field_extrapolate(pic_ctx* c);

// ---- particles (k_particles.hip) -------------------------------------------
// ---- diagnostics (k_debye.hip) ---------------------------------------------
// Doubles of the per-block moment records for ncells cells (block = 1).
long long debye_moment_doubles(long long ncells);
// Debye-length check over blocks of block^3 cells; lam_out (may be null):
// lambda_D per block; out (device, 4 doubles): checked, unresolved,
// lambda_min, ratio_max.
void parts_debye(pic_ctx* c, int block, double alpha_D, double* lam_out,
                 double* out);

// ---- Coulomb collisions (k_coulomb.hip) ----------------------------------
long long coulomb_scan_blocks(long long ncells);
void parts_coulomb(pic_ctx* c, double dt);
// ---- ion processes (k_ionproc.hip) ----------------------------------------
void parts_ion_processes(pic_ctx* c, double dt);
// Sort an event record list of at most max_events entries by (hi, lo).
void sort_event_records(pic_ctx* c, Rec* a, unsigned long long* count);

void parts_deposit(pic_ctx* c);
// The last step's cathode records of the species in mask, offset back along
// their velocity by 3 lattice_a, into SoA outputs of stride nout.
void parts_md_return(pic_ctx* c, double lattice_a, unsigned mask,
                     double* pos, double* vel, uint64_t* ids, int32_t* sp,
                     long long nout);
// One step's particle work: host-known sources (and the counter reset) and
// the neutral push need no field; the Fowler-Nordheim source, the charged
// pushes and the collisions do.
void parts_sources_host(pic_ctx* c);
void parts_push_neutral(pic_ctx* c, double dt);
void parts_sources_fn(pic_ctx* c, double dt);
void parts_push_collide(pic_ctx* c, double dt);
// Workgroups (and partial sums) of the neutral push for n neutrals.
long long neutral_push_blocks(long long n);
void parts_bin(pic_ctx* c);
void parts_bin_species(pic_ctx* c, int s);
void parts_chunks(pic_ctx* c, const long long hb[3]);
// Device arrays of species s (current buffer, native layout) and their
// element sizes; returns the number of arrays.
int parts_arrays(pic_ctx* c, int s, void** ptr, size_t* elem);
void parts_restore_keys(pic_ctx* c, int s, long long n);
void parts_load(pic_ctx* c, int s, long long n, const double* pos,
                const double* vel, const uint64_t* ids);
void parts_read(pic_ctx* c, int s, long long n, double* pos, double* vel,
                uint64_t* ids);
bool parts_validate(pic_ctx* c, const double* pos, const double* vel,
                    long long n);

}  // namespace pic
