// Device-side building blocks of the PIC-MCC kernels (gfx950).
//
// Everything here is written for 64-wide CDNA wavefronts.  Floating-point
// code must be compiled with -ffp-contract=off: the charge weights, the
// gather and the push are defined operation by operation (no fused
// multiply-add) so that their results are reproducible bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

// CODATA 2022.
constexpr double kE = 1.602176634e-19;       // elementary charge, C
constexpr double kMe = 9.1093837139e-31;     // electron mass, kg
constexpr double kEps0 = 8.8541878188e-12;   // vacuum permittivity, F/m
constexpr double kKB = 1.380649e-23;         // Boltzmann constant, J/K
constexpr double kAmu = 1.66053906892e-27;   // atomic mass constant, kg
constexpr double kH = 6.62607015e-34;        // Planck constant, J s
constexpr double kMcu = 63.546 * kAmu;       // Cu atom / Cu+ ion mass, kg
constexpr double kTwoPi = 6.283185307179586;
constexpr double kEuler = 2.718281828459045;
constexpr double kPi = 3.141592653589793;

// Cloud-in-cell weights are quantised to 13 bits per axis; a particle's
// three-axis weight product is an integer of at most 2^39.
constexpr int kQ = 8192;
constexpr double kQScale = 1.0 / 549755813888.0;  // 2^-39

constexpr uint32_t kDead = 0xFFFFFFFFu;           // key of a removed particle
constexpr int kTile = 8;                           // deposit tile edge, cells

// Philox tags (counter word 3) of the per-particle draws.
enum : uint32_t {
  kTagMcc0 = 0, kTagMcc1 = 1, kTagMcc2 = 2, kTagMcc3 = 3,
  kTagSrc0 = 8, kTagSrc1 = 9, kTagSrc2 = 10, kTagFn = 12
};

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// multiplications, key bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox10(uint32_t& c0, uint32_t& c1,
                                         uint32_t& c2, uint32_t& c3,
                                         uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // Each product as one 64-bit multiply (one v_mad_u64_u32 instead of a
    // low and a high multiply).
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c0 = n0; c1 = (uint32_t)p1; c2 = n2; c3 = (uint32_t)p0;
  }
}

// Two 53-bit uniforms in [0, 1) for (id, step, tag) under the run's seed.
__device__ __forceinline__ void uniform2(uint64_t id, uint32_t step,
                                         uint32_t tag, uint64_t seed,
                                         double& ua, double& ub) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32), c2 = step, c3 = tag;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = ((uint64_t)c0 << 21) ^ (uint64_t)(c1 >> 11);
  const uint64_t b = ((uint64_t)c2 << 21) ^ (uint64_t)(c3 >> 11);
  ua = (double)a * 0x1p-53;
  ub = (double)b * 0x1p-53;
}

// Cell index and quantised upper weight along one axis: g = x * inv_dx,
// i = floor(g), fq = floor((g - i) * 8192 + 0.5) in [0, 8192].
__device__ __forceinline__ void cic_axis(double x, double inv_dx, int& i,
                                         int& fq) {
  const double g = x * inv_dx;
  const double fl = floor(g);
  const double f = g - fl;
  i = (int)fl;
  fq = (int)floor(f * 8192.0 + 0.5);
}

__device__ __forceinline__ int wrap_index(int i, int n) {
  return i >= n ? i - n : (i < 0 ? i + n : i);
}

__device__ __forceinline__ double wrap_coord(double x, double len) {
  if (x < 0.0) x = x + len;
  if (x >= len) x = x - len;
  return x;
}

// Grid constants shared by the kernels (passed by value).
struct GridC {
  int nx, ny, nz;
  int tnx, tny, tnz;       // tiles per axis
  double dx, inv_dx, lx, ly;
  long long nxy;           // nodes per z plane
};

// Structure-of-arrays particle storage of one species, FP64 layout.
struct Parts {
  double *x, *y, *z, *vx, *vy, *vz;
  uint64_t* id;
};

// Structure-of-arrays particle storage, mixed layout: cell index plus FP32
// offsets inside the cell (cell units) and FP32 velocities (m/s).
struct PartsM {
  uint32_t* cell;
  float *ox, *oy, *oz, *vx, *vy, *vz;
  uint64_t* id;
};

// Layout accessors: every particle kernel except the pushes is written once
// against this interface and instantiated for both layouts.
template <class PT>
struct Acc;

template <>
struct Acc<Parts> {
  static __device__ __forceinline__ void pos(const Parts& p, long long i,
                                             const GridC&, double& x,
                                             double& y, double& z) {
    x = p.x[i]; y = p.y[i]; z = p.z[i];
  }
  static __device__ __forceinline__ void set_pos(const Parts& p, long long i,
                                                 const GridC&, double x,
                                                 double y, double z) {
    p.x[i] = x; p.y[i] = y; p.z[i] = z;
  }
  static __device__ __forceinline__ void vel(const Parts& p, long long i,
                                             double& vx, double& vy,
                                             double& vz) {
    vx = p.vx[i]; vy = p.vy[i]; vz = p.vz[i];
  }
  static __device__ __forceinline__ void set_vel(const Parts& p, long long i,
                                                 double vx, double vy,
                                                 double vz) {
    p.vx[i] = vx; p.vy[i] = vy; p.vz[i] = vz;
  }
  // Cell and quantised upper CIC weight per axis (x, y wrapped).
  static __device__ __forceinline__ void cic(const Parts& p, long long i,
                                             const GridC& g, int& ix, int& fx,
                                             int& iy, int& fy, int& iz,
                                             int& fz) {
    cic_axis(p.x[i], g.inv_dx, ix, fx);
    cic_axis(p.y[i], g.inv_dx, iy, fy);
    cic_axis(p.z[i], g.inv_dx, iz, fz);
    if (ix >= g.nx) ix -= g.nx;
    if (iy >= g.ny) iy -= g.ny;
  }
  static __device__ __forceinline__ void copy_pos(const Parts& s, long long i,
                                                  const Parts& d, long long j) {
    d.x[j] = s.x[i]; d.y[j] = s.y[i]; d.z[j] = s.z[i];
  }
  static __device__ __forceinline__ void copy(const Parts& s, long long i,
                                              const Parts& d, long long j) {
    d.x[j] = s.x[i]; d.y[j] = s.y[i]; d.z[j] = s.z[i];
    d.vx[j] = s.vx[i]; d.vy[j] = s.vy[i]; d.vz[j] = s.vz[i];
    d.id[j] = s.id[i];
  }
};

// Split a coordinate into cell and FP32 offset in [0, 1).
__device__ __forceinline__ void split_coord(double x, double inv_dx, int n,
                                            bool periodic, int& i, float& o) {
  const double gg = x * inv_dx;
  const double fl = floor(gg);
  i = (int)fl;
  o = (float)(gg - fl);
  if (o >= 1.0f) {
    o = 0.0f;
    i += 1;
  }
  if (periodic) {
    if (i >= n) i -= n;
  } else if (i >= n) {           // within rounding of the top face
    i = n - 1;
    o = 0x1.fffffep-1f;
  }
}

template <>
struct Acc<PartsM> {
  static __device__ __forceinline__ void decode(unsigned cell, const GridC& g,
                                                int& i, int& j, int& k) {
    i = (int)(cell % (unsigned)g.nx);
    const unsigned r = cell / (unsigned)g.nx;
    j = (int)(r % (unsigned)g.ny);
    k = (int)(r / (unsigned)g.ny);
  }
  static __device__ __forceinline__ void pos(const PartsM& p, long long i,
                                             const GridC& g, double& x,
                                             double& y, double& z) {
    int a, b, c;
    decode(p.cell[i], g, a, b, c);
    x = ((double)a + (double)p.ox[i]) * g.dx;
    y = ((double)b + (double)p.oy[i]) * g.dx;
    z = ((double)c + (double)p.oz[i]) * g.dx;
  }
  static __device__ __forceinline__ void set_pos(const PartsM& p, long long i,
                                                 const GridC& g, double x,
                                                 double y, double z) {
    int a, b, c;
    float ox, oy, oz;
    split_coord(x, g.inv_dx, g.nx, true, a, ox);
    split_coord(y, g.inv_dx, g.ny, true, b, oy);
    split_coord(z, g.inv_dx, g.nz, false, c, oz);
    p.cell[i] = ((unsigned)c * (unsigned)g.ny + (unsigned)b) * (unsigned)g.nx +
                (unsigned)a;
    p.ox[i] = ox; p.oy[i] = oy; p.oz[i] = oz;
  }
  static __device__ __forceinline__ void vel(const PartsM& p, long long i,
                                             double& vx, double& vy,
                                             double& vz) {
    vx = (double)p.vx[i]; vy = (double)p.vy[i]; vz = (double)p.vz[i];
  }
  static __device__ __forceinline__ void set_vel(const PartsM& p, long long i,
                                                 double vx, double vy,
                                                 double vz) {
    p.vx[i] = (float)vx; p.vy[i] = (float)vy; p.vz[i] = (float)vz;
  }
  static __device__ __forceinline__ void cic(const PartsM& p, long long i,
                                             const GridC& g, int& ix, int& fx,
                                             int& iy, int& fy, int& iz,
                                             int& fz) {
    decode(p.cell[i], g, ix, iy, iz);
    fx = (int)floorf(p.ox[i] * 8192.0f + 0.5f);
    fy = (int)floorf(p.oy[i] * 8192.0f + 0.5f);
    fz = (int)floorf(p.oz[i] * 8192.0f + 0.5f);
  }
  static __device__ __forceinline__ void copy_pos(const PartsM& s, long long i,
                                                  const PartsM& d, long long j) {
    d.cell[j] = s.cell[i];
    d.ox[j] = s.ox[i]; d.oy[j] = s.oy[i]; d.oz[j] = s.oz[i];
  }
  static __device__ __forceinline__ void copy(const PartsM& s, long long i,
                                              const PartsM& d, long long j) {
    d.cell[j] = s.cell[i];
    d.ox[j] = s.ox[i]; d.oy[j] = s.oy[i]; d.oz[j] = s.oz[i];
    d.vx[j] = s.vx[i]; d.vy[j] = s.vy[i]; d.vz[j] = s.vz[i];
    d.id[j] = s.id[i];
  }
};

// Device-resident counters of one step.  All are updated with atomics or by
// single-thread kernels and copied to the host once at the end of a step.
struct Counters {
  unsigned long long n[4];          // live particles
  unsigned long long next_id;
  unsigned long long fn_total;      // Fowler-Nordheim electrons this step
  unsigned long long cathode[4], anode[4];
  unsigned long long n_cand;        // null-collision candidates
  unsigned long long n_elastic;
  unsigned long long n_events;      // ionisation events before matching
  unsigned long long n_ok;          // matched ionisations
  unsigned long long n_over;        // candidates above E_max
  unsigned long long n_near;        // near-threshold draws
  unsigned long long n_ab;          // cathode-absorbed list length
  unsigned long long n_ncand;       // neutrals in cells with events
  unsigned long long n_tail_cand;   // candidates among unbinned electrons
  unsigned long long n_el_tail;     // elastic collisions among them
  unsigned long long ion_moved;     // binned ions pushed out of their tile
  unsigned long long n_dead1;       // neutrals removed this step (listed)
  unsigned long long n_dead2;       // ions removed this step (listed)
  unsigned long long n_pairs;       // (hole, mover) pairs of a listed removal
  unsigned long long sorted_n[4];   // counts after the binning pass
  unsigned long long n_dead;        // removed neutrals (compaction)
  unsigned long long n_holes;       // ... of them below the new count
  unsigned long long n_movers;      // live neutrals above it (= n_holes)
  unsigned long long np_hits;       // electrons absorbed by the nanoparticle
  unsigned long long coul_like;     // Coulomb collisions: like pairs
  unsigned long long coul_ei;       // ... electron-ion
  unsigned long long f3_rec;        // recombinations
  unsigned long long f3_ion2;       // ionisations of Cu+ (listed)
  unsigned long long f3_cx;         // charge exchanges
  unsigned long long f3_starved;    // electron-ion events without an ion
  long long total_charge;
  unsigned int err;                 // sticky error bits (kErr*)
  int vcycles;
  int done;                         // Poisson solve converged
  int refinements;                  // FP64 residuals of the mixed form's refinement
  double rel_res;
  double b_norm;
  double kinetic[4];
  double field_energy;
  double np_heat;                   // alpha_EH * their kinetic energy, J
  // Warm start of the field solve.
  double warm_r0;                   // ||r|| of the previous potential
  double sigma;                     // RMS of that residual over unknowns
  double warm_ratio;                // ||r(phi_0)|| / ||r(phi_prev)||
  double rel_res0;                  // relative residual before the V-cycles
  int warm_reject;                  // learned start rejected this solve
  int warm_pad;
};

enum : unsigned int {
  kErrCapacity = 1u, kErrNonFinite = 2u, kErrEvents = 4u, kErrQueue = 8u
};

// Small-list record sorted by (hi, lo): events (cell, electron id),
// neutral candidates (cell, neutral id), matched events (0, electron id) and
// the absorbed list (species, id); val is a payload index.
struct Rec {
  unsigned long long lo;
  unsigned int hi, val;
};

// A null-collision candidate as the push leaves it: the electron's index,
// id and kicked velocity, so the collision pass reads one contiguous record
// instead of gathering from the particle arrays.
struct CandRec {
  double vx, vy, vz;
  unsigned long long id;
  unsigned int i, pad;
};

__device__ __forceinline__ bool rec_less(const Rec& a, const Rec& b) {
  return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo);
}

// Blocks are dispatched round-robin over the 8 XCDs; remapping gives each
// XCD a contiguous range of work items so neighbouring tiles share an L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned per = nb / 8u;
  if (per == 0u || b >= per * 8u) return b;
  return (b % 8u) * per + b / 8u;
}

}  // namespace pic
