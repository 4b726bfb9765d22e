/*
 * pic.h -- C ABI of the MI355X (gfx950) electrostatic PIC-MCC step.
 *
 * The library advances the plasma above a cathode as in the paper's plasma
 * model: superparticles (electrons, Cu neutrals, Cu+ ions) are injected as
 * emitted electrons and evaporated or sputtered neutrals, their charge
 * drives Poisson's equation (Eq. 1) with Dirichlet or Neumann conditions on
 * the z faces, they move under the electric force, electrons collide with
 * neutrals by Monte Carlo collisions whose probability per step is
 * P = 1 - exp(-u n sigma(E) dt) (Eq. 4, in null-collision form), and the
 * particles that reach the cathode are handed back to the surface model
 * (Appendix A: transfer of ions to MD).
 *
 * Conventions
 *   - Units are SI at the boundary (m, s, V, V/m, m/s, m^2, eV where named).
 *   - Grid: nx * ny * nz cells of edge dx; nodes i in [0,nx), j in [0,ny)
 *     periodic, k in [0,nz] from the cathode (z = 0) to the anode
 *     (z = nz*dx).  Node arrays hold nx*ny*(nz+1) values, x fastest, then y,
 *     then z (index (k*ny + j)*nx + i).
 *   - Particle arrays are structure-of-arrays: a "pos3n" buffer holds
 *     x[0..n), then y[0..n), then z[0..n); "vel3n" likewise.
 *   - Every pointer argument named *device* must be device memory visible
 *     to the stream given at pic_init; the library never allocates device
 *     memory: all state lives in the caller-provided workspace.
 *   - All work is enqueued on the context's stream.  Calls that return
 *     results to the host (pic_step, pic_advance, pic_field, poisson_solve,
 *     pic_read_*) synchronise that stream before returning.
 *   - A context is not thread-safe; use one per host thread and stream.
 *
 * Errors: every call returns a pic_status; no C++ exception crosses the
 * ABI.  Device-side conditions (capacity overflow, non-finite values) are
 * sticky flags read at the end of the step and returned by that call;
 * pic_last_error() gives a text description of the last failure.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_ABI_VERSION 5

typedef enum {
  PIC_OK = 0,
  PIC_ERR_ARG = -1,       /* invalid argument or configuration           */
  PIC_ERR_CAPACITY = -2,  /* a particle/event buffer would overflow       */
  PIC_ERR_NOCONV = -3,    /* Poisson solve did not reach rel_tol          */
  PIC_ERR_NONFINITE = -4, /* NaN/Inf found in particle or field data      */
  PIC_ERR_HIP = -5,       /* a HIP runtime call failed                    */
  PIC_ERR_STATE = -6      /* call not valid in the current state          */
} pic_status;

/* Species: electrons, Cu atoms, Cu+ and Cu2+ (the higher charge state made
 * by electron-impact ionisation of Cu+, see pic_set_ion_processes). */
enum { PIC_ELECTRON = 0, PIC_NEUTRAL = 1, PIC_ION = 2, PIC_ION2 = 3 };
#define PIC_NSPECIES 4
enum { PIC_BC_DIRICHLET = 0, PIC_BC_NEUMANN = 1 };
enum { PIC_FP64 = 0, PIC_MIXED = 1 };
enum { PIC_ION_LOTZ = 0, PIC_ION_CONST = 1 };
/* PIC_FLAG_CELL_GROUPS: reserve the workspace that groups the particles
 * by cell each step (36 bytes per particle of capacity of electrons, Cu
 * and Cu+ together, and about 8 per cell), needed by the Coulomb
 * collisions (pic_set_coulomb) and the ion processes
 * (pic_set_ion_processes); the grid must then have fewer than 2^30 cells
 * and those three capacities must sum to at most 0xFFFFFFF0 (else
 * PIC_ERR_ARG).
 * PIC_FLAG_PLAIN_SMOOTHER: smooth with one launch per colour and sweep
 * instead of the fused two-sweep pass (same arithmetic, same results).
 * PIC_FLAG_MG_ALL_LEVELS: run the V-cycle down to the coarsest level
 * instead of solving the first coarse level small enough exactly (at most
 * 64 x 64 nodes per plane if both are powers of two, else 32 x 32, and 256
 * unknown planes: 2-D DFT in x, y, tridiagonal solve in z per mode). */
enum { PIC_FLAG_PLAIN_SMOOTHER = 1, PIC_FLAG_MG_ALL_LEVELS = 2,
       PIC_FLAG_CELL_GROUPS = 4 };
enum { PIC_WARM_ZERO = 0, PIC_WARM_GIVEN = 1 };
/* Warm start of the field solve in pic_step / pic_field (and of
 * poisson_solve with PIC_WARM_GIVEN): the previous potential; the same
 * while recording the learned start's training pair; the learned start; or
 * the linear extrapolation of the two previous potentials. */
enum { PIC_WS_PREV = 0, PIC_WS_RECORD = 1, PIC_WS_UNET = 2, PIC_WS_EXTRAP = 3 };

typedef struct pic_ctx pic_ctx;

/* Grid, boundary conditions, solver and capacities (Eq. 1 and its
 * Dirichlet/Neumann boundary data). */
typedef struct {
  int32_t nx, ny, nz;      /* cells per axis; each must be >= 2 and even  */
  double dx;               /* cell edge, m                                 */
  int32_t bc_lo, bc_hi;    /* PIC_BC_* for the cathode / anode face        */
  double v_lo, v_hi;       /* Dirichlet: potential, V.  Neumann: dphi/dz
                              at the face, V/m.  Both Neumann is rejected
                              (singular with periodic x, y).              */
  int32_t precision;       /* PIC_FP64, or PIC_MIXED: FP32 particles and
                              FP32 smoothing with FP64 refinement          */
  int32_t field_solve;     /* 1: particle charge drives phi; 0: boundary
                              data only (test configurations)             */
  int32_t mg_levels;       /* multigrid levels, 0 = as deep as possible    */
  int32_t max_vcycles;     /* V-cycle limit per solve (PIC_ERR_NOCONV)     */
  int32_t nu_pre, nu_post; /* red-black Gauss-Seidel sweeps per level      */
  int32_t coarse_sweeps;   /* sweeps on a coarsest level wider than 1x1    */
  int32_t sort_every;      /* reserved, must be 1: particles are binned by
                              tile after every step                        */
  double rel_tol;          /* ||b - A phi||_2 / ||b||_2 target, e.g. 1e-10 */
  uint64_t seed;           /* Philox key                                   */
  uint32_t w_sp;           /* superparticle weight (all species), >= 1     */
  uint32_t flags;          /* PIC_FLAG_* (0 by default)                    */
  int64_t capacity[PIC_NSPECIES]; /* particles per species (electron, Cu,
                              Cu+, Cu2+)                                   */
  int64_t queue_capacity;  /* particles pic_inject may queue per step      */
  int64_t max_events;      /* ionisation events / cathode absorptions /
                              Fowler-Nordheim electrons per step           */
} pic_config;

/* Electron-neutral collision model (Eq. 4; ionisation and elastic). */
typedef struct {
  int32_t enabled;         /* 0 disables MCC                               */
  int32_t ion_model;       /* PIC_ION_LOTZ or PIC_ION_CONST                */
  double sigma_el;         /* elastic cross section, m^2                   */
  double lotz_a;           /* Lotz constant, m^2 eV^2 (4.5e-18 = 4.5e-14
                              cm^2 eV^2)                                   */
  double ion_I_eV;         /* ionisation threshold, eV (Cu: 7.73)          */
  double sigma_ion_const;  /* PIC_ION_CONST cross section above I, m^2     */
  double E_max_eV;         /* majorant energy of the null-collision method */
} pic_collisions;

/* Coulomb collisions by binary pairing within cells (the paper's Monte
 * Carlo collisions, after Takizuka & Abe), applied each step after the
 * electron-neutral collisions to the charged particles of every cell.  A
 * cell's electrons and its ions are each put in a random order (ascending
 * 53-bit Philox draw of (id, step), then id); consecutive particles pair,
 * an odd count N >= 3 starts with a triplet (0,1), (1,2), (2,0) of
 * half-variance collisions; then max(N_e, N_i) electron-ion collisions,
 * collision k between electron k mod N_e and ion k mod N_i in ascending k,
 * at the lower density.  Each collision turns the relative velocity u by
 * theta with tan(theta/2) normal of variance
 * e^4 n lnL dt / (8 pi eps0^2 m_r^2 |u|^3) and a uniform azimuth, keeping
 * momentum and energy.  Cells with more than 2048 charged particles set
 * the event error (PIC_ERR_CAPACITY).  Needs PIC_FLAG_CELL_GROUPS. */
typedef struct {
  int32_t enabled;         /* 0: off (default)                             */
  int32_t reserved;
  double ln_lambda;        /* Coulomb logarithm lnL, e.g. 10               */
} pic_coulomb;
pic_status pic_set_coulomb(pic_ctx* ctx, const pic_coulomb* c);

/* Recombination, electron-impact ionisation of Cu+ and resonant charge
 * exchange (the paper's Monte Carlo collisions include charge exchange and
 * recombination, and its ions reach several charge levels), applied each
 * step after the Coulomb collisions.  The paper gives no cross sections;
 * they are parameters:
 *   sigma_rec(E) = sigma_rec_1eV * (1 eV / max(E, 1e-3 eV)),
 *   sigma_ion2(E) = lotz_a2 ln(E / I2) / (E I2) for E > I2, else 0,
 *   sigma_cx(eps) = max(cx_a - cx_b ln(max(eps, 1e-6 eV) / 1 eV), 0)^2
 *     with eps = m_r u^2 / 2 of the Cu+ / Cu pair (eV).
 * Per cell, electrons, Cu+ and Cu each in a random order (53-bit Philox
 * draw of (id, step), then id): each electron collides with probability
 * 1 - exp(-n_i (sigma_rec + sigma_ion2) v dt) (Eq. 4, n_i the cell's Cu+
 * density), the r-th colliding one with the r-th Cu+ (none left:
 * starved); recombination leaves a Cu atom with the ion's position and id
 * and the pair's centre-of-mass velocity; ionisation shares the energy
 * above I2 uniformly between two isotropic electrons (the secondary at the
 * primary's position, ids next_id + rank by primary id) and makes the ion
 * a Cu2+.  Then each Cu+ left meets atom k mod N_n of the cell's atoms with
 * probability 1 - exp(-n_n sigma_cx u dt) (u the pair's relative speed):
 * the two records exchange position, velocity and id.  Crowded cells
 * (more than 2048 electrons and Cu+ together; any number of atoms) set the
 * event error.  Needs
 * PIC_FLAG_CELL_GROUPS (its records then cover electrons, Cu and Cu+). */
typedef struct {
  int32_t enabled;         /* 0: off (default)                             */
  int32_t reserved;
  double sigma_rec_1eV;    /* m^2                                          */
  double lotz_a2;          /* m^2 eV^2                                     */
  double ion2_I_eV;        /* Cu+ -> Cu2+ threshold, eV (20.29)            */
  double cx_a, cx_b;       /* m                                            */
} pic_ion_processes;
pic_status pic_set_ion_processes(pic_ctx* ctx, const pic_ion_processes* p);

/* Per-step particle sources at the cathode and in the gap, and the
 * nanoparticle as an electron sink. */
typedef struct {
  int32_t disk_on, fn_on, sphere_on;
  /* sph_absorb: the sphere (a nanoparticle) absorbs every electron whose
   * straight path in a step touches it, and tallies alpha_EH times the
   * electron's kinetic energy as the particle's heat (Appendix A, electron
   * heating of NPs); ions and neutrals pass through.  Independent of
   * sphere_on (the neutral source). */
  int32_t sph_absorb;
  /* Disk at z = 0: electrons with a flux-weighted half-Maxwellian normal
   * speed at kT_e, neutrals with a half-space Maxwellian at T_n. */
  double disk_cx, disk_cy, disk_radius;
  int64_t disk_n_e;
  double disk_kT_e_eV;
  int64_t disk_n_n;
  double disk_T_n_K;
  /* Fowler-Nordheim emission from the surface nodes inside a disk, driven
   * by the local field -E_z(z = 0) (elementary FN, work function phi_w). */
  double fn_cx, fn_cy, fn_radius, fn_phi_w_eV, fn_kT_e_eV;
  /* Sphere (e.g. an evaporating nanoparticle): neutrals from its surface,
   * Maxwellian at T with the inward normal component reflected. */
  double sph_cx, sph_cy, sph_cz, sph_radius;
  int64_t sph_n;
  double sph_T_K;
  double sph_alpha_eh;     /* energy fraction an absorbed electron leaves
                              as heat, 0..1 (the paper's estimate: 0.5)   */
} pic_sources;

typedef struct {
  int32_t vcycles;         /* V-cycles taken                               */
  int32_t converged;       /* 1 if rel_residual <= rel_tol                 */
  double rel_residual;     /* final ||b - A phi|| / ||b||                  */
  double b_norm;           /* ||b||_2 of the scaled system                 */
  double rel_residual0;    /* of the start the V-cycles began from         */
  double warm_ratio;       /* learned start: ||r(phi_0)|| / ||r(phi_prev)||
                              (1 when not used or rejected)                */
  int32_t warm_used;       /* the network ran in this solve                */
  int32_t warm_rejected;   /* ... and its start was rejected (non-finite,
                              or a larger residual than phi_prev's)        */
  int32_t refinements;     /* mixed form: refinement rounds (FP32 V-cycles
                              on the correction, then the FP64 residual);
                              0 in FP64                                    */
} pic_solve_info;

typedef struct {
  int64_t counts[PIC_NSPECIES];          /* live particles after the step             */
  int64_t emitted[PIC_NSPECIES];         /* particles added by queue and sources      */
  int64_t fn_emitted;         /* of which Fowler-Nordheim electrons        */
  int64_t cathode[PIC_NSPECIES];         /* absorbed at z = 0                         */
  int64_t anode[PIC_NSPECIES];           /* absorbed at z = nz*dx                     */
  int64_t candidates;         /* null-collision candidates                 */
  int64_t elastic;
  int64_t ionisations;        /* successful (matched) ionisations          */
  int64_t starved;            /* ionisations without a neutral left        */
  int64_t over_majorant;      /* candidates above E_max                    */
  int64_t near_threshold;     /* draws within 1e-6 of a threshold that
                                 involves a transcendental function        */
  int64_t total_charge_units; /* sum of node charges, 2^-39 w_sp e units   */
  double kinetic[PIC_NSPECIES]; /* kinetic energy after the push, J        */
  double field_energy;        /* 1/2 sum q phi over nodes, J               */
  pic_solve_info solve;
  int64_t step;               /* steps completed                           */
  uint64_t next_id;           /* next particle id to assign                */
  int64_t np_absorbed;        /* electrons absorbed by the nanoparticle    */
  double np_heat;             /* alpha_EH * sum of their energies, J       */
  int64_t coulomb_like;       /* Coulomb collisions of like pairs          */
  int64_t coulomb_ei;         /* ... and electron-ion                      */
  int64_t recombinations;     /* e + Cu+ -> Cu                             */
  int64_t ionisations2;       /* e + Cu+ -> 2e + Cu2+                      */
  int64_t charge_exchanges;   /* Cu+ + Cu -> Cu + Cu+                      */
  int64_t ion_starved;        /* electron-ion events without a Cu+ left    */
} pic_diag;

/* Particles absorbed at the cathode in the last step, sorted by
 * (species, id): the ions (and neutrals, electrons) the surface model takes
 * back.  Device pointers owned by the library, valid until the next
 * pic_step / pic_advance / pic_destroy. */
typedef struct {
  int64_t n;
  const int32_t* species;  /* device                                      */
  const uint64_t* id;      /* device                                      */
  const double* pos;       /* device, 3n SoA: crossing point, z = 0        */
  const double* vel;       /* device, 3n SoA: half-step velocity           */
} pic_absorbed;

/* Atoms handed back to MD from the last step's cathode list (Appendix A,
 * transfer of bombarding ions): each particle of a species selected by
 * species_mask (bit s for species s; the paper hands back the ions,
 * 1u << PIC_ION) is placed at its crossing point offset backwards along its
 * velocity by three lattice constants, x_MD = x_c - 3 a v / |v|, x and y
 * wrapped into the periodic box, so the atom starts above the surface and
 * clear of its atoms.  Outputs (caller-owned device buffers of at least cap
 * entries; species may be NULL) keep the list's (species, id) order:
 * pos3n and vel3n SoA (m, m/s), ids, species; *n receives the count.
 * PIC_ERR_CAPACITY (with *n set) if cap is too small; PIC_ERR_STATE before
 * the first step.  Synchronises the context's stream. */
pic_status pic_md_return(pic_ctx* ctx, double lattice_a, uint32_t species_mask,
                         int64_t cap, double* pos3n_device,
                         double* vel3n_device, uint64_t* ids_device,
                         int32_t* species_device, int64_t* n);

/* Resolution of the grid against the Debye length of the electrons and ions
 * (Appendix A: mesh criterion d_max = 3.4 lambda_D alpha_D, the paper uses
 * alpha_D = 0.5).  Per block of block^3 cells (block = 1, 2, 4 or 8,
 * dividing nx, ny, nz; blocks x fastest) and charged species with N >= 2
 * particles: n = N w_sp / (block dx)^3 and k T = m S / (3 (N - 1)), S the
 * sum of |v - mean v|^2 over the block's particles; 1 / lambda_D^2 = sum
 * over those species of n e^2 / (eps0 k T).  A block with no such species
 * has no Debye length (lambda = +inf).  The grid resolves a block when
 * dx <= d_max.  lambda_device (may be NULL): nx*ny*nz / block^3 values, m.
 * Moments are summed with atomics, so lambda_D is reproducible to rounding
 * (not bit for bit).  Synchronises the context's stream. */
typedef struct {
  int64_t blocks;          /* blocks of the grid                           */
  int64_t checked;         /* with a finite Debye length                   */
  int64_t unresolved;      /* of them with dx > d_max                      */
  double lambda_min;       /* smallest Debye length, m (inf: none)         */
  double ratio_max;        /* largest dx / d_max (0: none)                 */
} pic_debye_info;
pic_status pic_debye_check(pic_ctx* ctx, int32_t block, double alpha_D,
                           double* lambda_device, pic_debye_info* info);

/* The nanoparticle's electron energy-loss fraction (Appendix A):
 * (1 - R)(1 - exp(-d / ell))(1 - phi_w / E_e) for reflection probability R,
 * particle diameter d and inelastic mean free path ell (same length unit),
 * work function phi_w and electron energy E_e (eV).  The paper prints the
 * middle factor as exp(-d/ell) but evaluates it as 0.76 = 1 - exp(-1/0.7);
 * this follows the value (0.85 * 0.76 * 0.775 = 0.50). */
double pic_alpha_eh(double R, double d, double ell, double phi_w_eV,
                    double E_e_eV);

/* Workspace size for a configuration; the caller allocates it (e.g. with
 * torch) with at least 256-byte alignment. */
pic_status pic_workspace_bytes(const pic_config* cfg, size_t* bytes);

/* Validate cfg, carve the workspace, build the multigrid hierarchy and zero
 * the state.  hip_stream is a hipStream_t (NULL = default stream). */
pic_status pic_init(const pic_config* cfg, void* workspace_device,
                    size_t bytes, void* hip_stream, pic_ctx** out);
void pic_destroy(pic_ctx* ctx);

pic_status pic_set_collisions(pic_ctx* ctx, const pic_collisions* c);
pic_status pic_set_sources(pic_ctx* ctx, const pic_sources* s);

/* Queue n particles of one species (emitted electrons, evaporated or
 * sputtered neutrals, ...).  pos3n/vel3n are device buffers the caller keeps
 * alive until the stream passes this call.  Queued particles receive ids
 * next_id + rank (call order) at the next step and are pushed in it; their
 * velocity is taken as the half-step velocity. */
pic_status pic_inject(pic_ctx* ctx, int32_t species, int64_t n,
                      const double* pos3n_device, const double* vel3n_device);

/* One full step: deposit charge, solve Poisson (warm start: the previous
 * phi), compute E, add queued and source particles, push, collide, bin.
 * out (may be NULL) receives the cathode-absorbed list; diag (may be NULL)
 * the step's diagnostics. */
pic_status pic_step(pic_ctx* ctx, double dt, pic_absorbed* out,
                    pic_diag* diag);

/* rho (charge density at nodes, C/m^3) -> phi (V) with the context's grid
 * and boundary data.  phi is read as the initial guess when
 * warm == PIC_WARM_GIVEN.  Does not touch the particle state. */
pic_status poisson_solve(pic_ctx* ctx, const double* rho_device,
                         double* phi_device, int32_t warm,
                         pic_solve_info* info);

/* The three stages pic_step is made of, for tests and for callers that
 * supply their own field. */
pic_status pic_deposit(pic_ctx* ctx);                        /* -> charge  */
pic_status pic_field(pic_ctx* ctx, pic_solve_info* info);    /* -> phi, E  */
pic_status pic_set_phi(pic_ctx* ctx, const double* phi_device); /* -> E    */
pic_status pic_advance(pic_ctx* ctx, double dt, pic_absorbed* out,
                       pic_diag* diag);

/* State access.  pic_load_particles replaces a species' population with
 * caller data (ids included); positions must satisfy 0 <= z/dx < nz. */
pic_status pic_load_particles(pic_ctx* ctx, int32_t species, int64_t n,
                              const double* pos3n_device,
                              const double* vel3n_device,
                              const uint64_t* ids_device);
pic_status pic_count(pic_ctx* ctx, int32_t species, int64_t* n);
pic_status pic_read_particles(pic_ctx* ctx, int32_t species, int64_t cap,
                              double* pos3n_device, double* vel3n_device,
                              uint64_t* ids_device, int64_t* n);
/* Copies of the node fields; any pointer may be NULL.  acc: int64 charge
 * units; phi: V; E3: 3 arrays of node values (Ex block, Ey, Ez), V/m. */
pic_status pic_read_fields(pic_ctx* ctx, int64_t* acc_device,
                           double* phi_device, double* E3_device);
pic_status pic_set_clock(pic_ctx* ctx, int64_t step, uint64_t next_id);

/* Checkpoint and resume.  The checkpoint (host memory, caller-owned,
 * pic_checkpoint_bytes large) holds the grid, precision and seed, the
 * clock and id counter, the collision and source settings, every
 * particle in the context's native layout, the last potential (the next
 * solve's warm start) and the last solve's V-cycle count.  Every random
 * number is keyed by (id, step), so a context restored from it continues
 * exactly as the saved one would (particle storage order aside).
 * pic_checkpoint_save: PIC_ERR_STATE while injections are queued.
 * pic_checkpoint_load: the context must have the same grid, boundary
 * data, precision, seed and weight (PIC_ERR_ARG otherwise) and room for
 * the particles (PIC_ERR_CAPACITY); the warm-start mode is not part of
 * the checkpoint. */
pic_status pic_checkpoint_bytes(pic_ctx* ctx, size_t* bytes);
pic_status pic_checkpoint_save(pic_ctx* ctx, void* host, size_t bytes);
pic_status pic_checkpoint_load(pic_ctx* ctx, const void* host, size_t bytes);
pic_status pic_get_diag(pic_ctx* ctx, pic_diag* diag);

/* Per-phase GPU time, measured with HIP events recorded on the context's
 * stream around each phase of a step (off by default; at most 256 intervals
 * of a phase per step are timed).  ms[PIC_NPHASES] receives the time
 * accumulated since timing was enabled, calls[] (may be NULL) the number of
 * timed intervals of each phase. */
#define PIC_NPHASES 16
enum {
  PIC_PH_DEPOSIT = 0, PIC_PH_RHS, PIC_PH_POISSON, PIC_PH_EFIELD,
  PIC_PH_SOURCES, PIC_PH_PUSH_NEUTRAL, PIC_PH_PUSH_ION, PIC_PH_PUSH_ELECTRON,
  PIC_PH_COLLIDE, PIC_PH_ABSORBED, PIC_PH_BIN,
  PIC_PH_WARM,    /* warm-start stage of the solve (inside PIC_PH_POISSON) */
  PIC_PH_SMOOTH0, /* each finest-level smoothing launch (inside the solve;
                     calls counts launches)                               */
  PIC_PH_DEBYE,   /* pic_debye_check                                      */
  PIC_PH_COULOMB, /* Coulomb binary collisions (inside PIC_PH_COLLIDE)    */
  PIC_PH_ION_COLL /* ion-neutral and recombination collisions (inside
                     PIC_PH_COLLIDE)                                      */
};
pic_status pic_enable_timing(pic_ctx* ctx, int32_t on);
pic_status pic_phase_times(pic_ctx* ctx, double* ms, int64_t* calls);

/* ---- Learned Poisson warm start -------------------------------------------
 * A 3-D U-Net (levels of 16/32/64/128 channels, 3x3x3 convolutions with
 * bias and ReLU, 2^3 average pooling, nearest upsampling with
 * concatenation, 1x1x1 head) maps a normalised pair (residual of the warm
 * start r = b - A phi_prev, previous potential) to a normalised potential
 * correction; multigrid then finishes the solve to the same residual and
 * acts as fallback and judge.  BF16 weights and activations, FP32
 * accumulation on the matrix cores, FP32 master weights with Adam.
 * Grids are D x H x W voxels (z, y, x), each a multiple of 8; tensors are
 * channels-last FP32 at the boundary: input (D,H,W,2), target and output
 * (D,H,W).  Padding: circular in x, y, zero in z.
 * Parameter vector (pic_unet_param_count FP32 values): per convolution in
 * the order e0a e0b e1a e1b e2a e2b ba bb d2a d2b d1a d1b d0a d0b, the
 * weights W[co][tap][ci] (tap = (dz+1)*9 + (dy+1)*3 + (dx+1)) then the
 * bias[co]; then the head's 16 weights and its bias. */
typedef struct pic_unet pic_unet;
int64_t pic_unet_param_count(void);
pic_status pic_unet_workspace_bytes(int32_t D, int32_t H, int32_t W,
                                    size_t* bytes);
/* D, H, W: the largest grid the object will see. */
pic_status pic_unet_init(int32_t D, int32_t H, int32_t W,
                         void* workspace_device, size_t bytes,
                         void* hip_stream, pic_unet** out);
void pic_unet_destroy(pic_unet* u);
/* Set (resets the Adam moments) / get the FP32 parameters. */
pic_status pic_unet_set_params(pic_unet* u, const float* params_device);
pic_status pic_unet_get_params(pic_unet* u, float* params_device);
pic_status pic_unet_forward(pic_unet* u, const float* input_device,
                            int32_t D, int32_t H, int32_t W,
                            float* out_device);
/* Mean-squared-error loss of one sample and its parameter gradient
 * (grad_device may be NULL). */
pic_status pic_unet_gradients(pic_unet* u, const float* input_device,
                              const float* target_device, int32_t D,
                              int32_t H, int32_t W, float* grad_device,
                              double* loss);
/* Training loss.  PIC_UNET_LOSS_MSE (default): mean squared error of the
 * output against the target.  PIC_UNET_LOSS_RESIDUAL: sum over the unknown
 * planes z >= k0 of (A (out - target))^2 / V, with A the scaled 7-point
 * Poisson operator of the network grid (x, y periodic, zero beyond the top
 * plane; k0 = 1: Dirichlet bottom plane, k0 = 0: Neumann bottom, mirrored),
 * i.e. the squared residual of the warm start it produces over sigma^2.
 * PIC_ERR_ARG for another mode or k0. */
enum { PIC_UNET_LOSS_MSE = 0, PIC_UNET_LOSS_RESIDUAL = 1 };
pic_status pic_unet_set_loss(pic_unet* u, int32_t mode, int32_t k0);
/* One Adam step on one sample; loss is that sample's loss before it. */
pic_status pic_unet_train_step(pic_unet* u, const float* input_device,
                               const float* target_device, int32_t D,
                               int32_t H, int32_t W, float lr, float beta1,
                               float beta2, float eps, double* loss);
const char* pic_unet_last_error(const pic_unet* u);

/* Warm start of the context's field solve.  mode PIC_WS_PREV: the previous
 * potential.  PIC_WS_EXTRAP: 2 phi_{n-1} - phi_{n-2}, from the converged
 * potentials of the last two step solves (a classical start, not the
 * paper's); until two such solves follow one another (after pic_set_phi,
 * poisson_solve, an unconverged solve or a step in another mode) the
 * previous potential.  Checkpoints carry both.  PIC_WS_RECORD: the previous
 * potential, and each solve records the pair for pic_warm_pair.  PIC_WS_UNET: each solve also runs net (which must outlive
 * this use and must not be driven from another stream meanwhile) on the
 * context's stream: with r0 = b - A phi_prev on the unknowns, sigma its RMS
 * and V_ref the largest Dirichlet face potential (at least 1 V), the input
 * is (r0 / sigma, phi_prev / V_ref) on the nz planes k < nz, and
 * phi_0 = phi_prev + sigma * output on the unknowns of those planes.  phi_0
 * replaces phi_prev only if its residual is finite and not larger; the
 * V-cycles then finish the solve to rel_tol either way.  The grid
 * (D, H, W) = (nz, ny, nx) must be multiples of 8 within the net's maximum,
 * else PIC_ERR_ARG. */
pic_status pic_set_warm_start(pic_ctx* ctx, int32_t mode, pic_unet* net);

/* ---- Allocation-free Poisson solve ----------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * solve as poisson_solve (rho -> phi with cfg's grid, boundary data,
 * precision, multigrid settings and rel_tol; cfg's capacities are ignored)
 * without a context or a workspace: the multigrid state lives in a fixed
 * device buffer of the library, PIC_STATIC_SCRATCH_BYTES large, one per GPU
 * it runs on, held until the process ends.  Nothing is allocated: no
 * hipMalloc, hipFree or host allocation.  rho and phi are caller-owned
 * device arrays of nx*ny*(nz+1) FP64 values (x fastest); phi is read as the
 * initial guess when warm == PIC_WARM_GIVEN.  Enqueued on hip_stream (a
 * hipStream_t, NULL = default), which is synchronised before returning.
 * Every call on one GPU shares that GPU's buffer and clears it first:
 * calls that overlap on one GPU (several host threads or streams) race.
 * Errors: PIC_ERR_ARG (invalid cfg or arguments), PIC_ERR_CAPACITY (the
 * grid's multigrid state, about 27 bytes per node in FP64 plus the exact
 * coarse level, exceeds the buffer: roughly above 2 M nodes), PIC_ERR_HIP,
 * PIC_ERR_NOCONV. */
#define PIC_STATIC_SCRATCH_BYTES (64u << 20)
pic_status poisson_solve_static(const pic_config* cfg,
                                const double* rho_device, double* phi_device,
                                int32_t warm, pic_solve_info* info,
                                void* hip_stream);


/* The last recorded solve's network input (nz, ny, nx, 2) and target
 * (phi - phi_prev) / sigma (nz, ny, nx), FP32 device buffers: the learned
 * start's training pair.  PIC_ERR_STATE if no solve has been recorded. */
pic_status pic_warm_pair(pic_ctx* ctx, float* input_device,
                         float* target_device);

const char* pic_last_error(const pic_ctx* ctx);
int32_t pic_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
