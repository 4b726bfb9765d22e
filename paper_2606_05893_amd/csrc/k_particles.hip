// Particle side of the PIC-MCC step on gfx950: sources, charge deposition,
// field gather + leapfrog push + absorbing/periodic boundaries, null-
// collision MCC (Eq. 4) with ionisation target matching, the cathode sink
// list, and binning of the particles by 8x8x8-cell tile (which is also the
// compaction that removes absorbed and consumed particles).
//
// Particles are structure-of-arrays, so every per-particle kernel reads and
// writes fully coalesced 64-lane streams; the only scattered traffic is the
// field gather (8 nodes, L2-resident because particles are binned by tile)
// and integer atomics.  Charge is accumulated in LDS per tile with 64-bit
// integer atomics and flushed once per node, so the sum is exact and
// independent of order.
#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kSmallLds = 2048;   // records sorted in LDS by k_sort_small
constexpr int kFixedBlocks = 2048;

inline unsigned nblk(long long n, int t = kT) {
  return (unsigned)((n + t - 1) / t);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long bcast64(unsigned long long v,
                                                      int src) {
  const unsigned lo = __shfl((unsigned)v, src);
  const unsigned hi = __shfl((unsigned)(v >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

// Wave-aggregated append: one atomic per wavefront.  Every lane of the wave
// must call it (pred may be false).  Returns the slot of a predicated lane.
__device__ __forceinline__ unsigned long long wave_append(
    bool pred, unsigned long long* counter) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return 0ull;
  const int lane = lane_id();
  const int leader = __ffsll((long long)mask) - 1;
  const unsigned long long below =
      lane ? (mask & (~0ull >> (64 - lane))) : 0ull;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  base = bcast64(base, leader);
  return base + (unsigned long long)__popcll(below);
}

// Run-length aggregated counter increment for keys that arrive grouped
// (binned particles): the first lane of each run of equal keys adds the run
// length.  Returns, per lane, its slot when 'fetch' is set (the counter's
// old value plus its rank in the run).  All lanes must call it.
__device__ __forceinline__ unsigned run_add(unsigned key, unsigned* counters,
                                            bool fetch) {
  const int lane = lane_id();
  const unsigned prev = __shfl_up(key, 1);
  const bool head = lane == 0 || key != prev;
  const unsigned long long hm = __ballot(head);
  const unsigned long long above = lane == 63 ? 0ull : (hm >> (lane + 1));
  const int len = above ? __ffsll((long long)above) : 64 - lane;
  // Head lane of this lane's run: highest set bit of hm at or below lane.
  const unsigned long long upto = hm & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
  const int head_lane = 63 - __clzll((long long)upto);
  unsigned base = 0;
  if (head && key != kDead) {
    if (fetch)
      base = atomicAdd(&counters[key], (unsigned)len);
    else
      atomicAdd(&counters[key], (unsigned)len);
  }
  if (!fetch) return 0;
  base = __shfl(base, head_lane);
  return base + (unsigned)(lane - head_lane);
}

__device__ __forceinline__ unsigned tile_of_cell(unsigned cell, const GridC& g) {
  const unsigned i = cell % (unsigned)g.nx;
  const unsigned r = cell / (unsigned)g.nx;
  const unsigned j = r % (unsigned)g.ny;
  const unsigned k = r / (unsigned)g.ny;
  return ((k / kTile) * (unsigned)g.tny + j / kTile) * (unsigned)g.tnx + i / kTile;
}

// Cell of an in-domain position (0 <= z/dx < nz): the one the MCC uses for
// the target density and the binning uses for tiles.
__device__ __forceinline__ unsigned cell_of(double x, double y, double z,
                                            const GridC& g) {
  int i = (int)floor(x * g.inv_dx);
  int j = (int)floor(y * g.inv_dx);
  const int k = (int)floor(z * g.inv_dx);
  if (i >= g.nx) i -= g.nx;
  if (j >= g.ny) j -= g.ny;
  return ((unsigned)k * (unsigned)g.ny + (unsigned)j) * (unsigned)g.nx + (unsigned)i;
}

// ---- step bookkeeping ---------------------------------------------------------
__global__ void k_begin(Counters* dc, unsigned long long n0,
                        unsigned long long n1, unsigned long long n2,
                        unsigned long long next_id) {
  dc->n[0] = n0; dc->n[1] = n1; dc->n[2] = n2;
  dc->next_id = next_id;
  dc->fn_total = 0;
  for (int s = 0; s < 3; ++s) {
    dc->cathode[s] = 0; dc->anode[s] = 0; dc->kinetic[s] = 0.0;
    dc->sorted_n[s] = 0;
  }
  dc->n_cand = dc->n_elastic = dc->n_events = dc->n_ok = 0;
  dc->n_over = dc->n_near = dc->n_ab = dc->n_ncand = 0;
}

// ---- sources ------------------------------------------------------------------
__global__ void k_append_queue(Parts p, long long dst, const double* __restrict__ qpos,
                               const double* __restrict__ qvel, long long n,
                               unsigned long long id0) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const long long d = dst + t;
  p.x[d] = qpos[t]; p.y[d] = qpos[n + t]; p.z[d] = qpos[2 * n + t];
  p.vx[d] = qvel[t]; p.vy[d] = qvel[n + t]; p.vz[d] = qvel[2 * n + t];
  p.id[d] = id0 + (unsigned long long)t;
}

__device__ __forceinline__ double flux_vz(double u, double vth2) {
  return sqrt((-2.0 * vth2) * log(1.0 - u));
}

// Disk at z = 0.  species 0: electrons (normal speed from a flux-weighted
// half-Maxwellian, no tangential velocity); species 1: neutrals (Gaussian
// tangential components, flux-weighted normal component).
__global__ void k_disk(Parts p, long long dst, long long n,
                       unsigned long long id0, int species, double cx,
                       double cy, double radius, double vth2, GridC g,
                       uint32_t step, uint64_t seed) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const unsigned long long id = id0 + (unsigned long long)t;
  double u1, u2, u3, u4;
  uniform2(id, step, kTagSrc0, seed, u1, u2);
  const double r = radius * sqrt(u1);
  const double th = kTwoPi * u2;
  const long long d = dst + t;
  p.x[d] = wrap_coord(cx + r * cos(th), g.lx);
  p.y[d] = wrap_coord(cy + r * sin(th), g.ly);
  p.z[d] = 0.0;
  p.id[d] = id;
  uniform2(id, step, kTagSrc1, seed, u3, u4);
  if (species == 0) {
    p.vx[d] = 0.0;
    p.vy[d] = 0.0;
    p.vz[d] = flux_vz(u3, vth2);
  } else {
    const double rr = sqrt((-2.0 * vth2) * log(1.0 - u3));
    const double ph = kTwoPi * u4;
    p.vx[d] = rr * cos(ph);
    p.vy[d] = rr * sin(ph);
    double u5, u6;
    uniform2(id, step, kTagSrc2, seed, u5, u6);
    p.vz[d] = flux_vz(u5, vth2);
  }
}

// Sphere surface source: uniform points on the sphere, Maxwellian velocity
// with the inward normal component reflected.
__global__ void k_sphere(Parts p, long long dst, long long n,
                         unsigned long long id0, double cx, double cy,
                         double cz, double radius, double sig, GridC g,
                         uint32_t step, uint64_t seed) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const unsigned long long id = id0 + (unsigned long long)t;
  double u1, u2, u3, u4, u5, u6;
  uniform2(id, step, kTagSrc0, seed, u1, u2);
  const double c = 1.0 - 2.0 * u1;
  const double s = sqrt(1.0 - c * c);
  const double ps = kTwoPi * u2;
  const double nx = s * cos(ps), ny = s * sin(ps), nz = c;
  const long long d = dst + t;
  p.x[d] = wrap_coord(cx + radius * nx, g.lx);
  p.y[d] = wrap_coord(cy + radius * ny, g.ly);
  p.z[d] = cz + radius * nz;
  p.id[d] = id;
  uniform2(id, step, kTagSrc1, seed, u3, u4);
  const double rr = sqrt(-2.0 * log(1.0 - u3));
  const double g1 = rr * cos(kTwoPi * u4), g2 = rr * sin(kTwoPi * u4);
  uniform2(id, step, kTagSrc2, seed, u5, u6);
  const double g3 = sqrt(-2.0 * log(1.0 - u5)) * cos(kTwoPi * u6);
  double vx = sig * g1, vy = sig * g2, vz = sig * g3;
  const double vn = (vx * nx + vy * ny) + vz * nz;
  if (vn < 0.0) {
    const double tt = 2.0 * vn;
    vx = vx - tt * nx;
    vy = vy - tt * ny;
    vz = vz - tt * nz;
  }
  p.vx[d] = vx; p.vy[d] = vy; p.vz[d] = vz;
}

// Fowler-Nordheim counts per surface node inside the emitting disk:
// J = (a/phi) F^2 exp(-b phi^1.5/F) with F = -E_z(z = 0); the expected
// number J dx^2 dt / e is rounded stochastically.
template <typename TE>
__global__ void k_fn_count(const TE* __restrict__ E, unsigned* __restrict__ cnt,
                           GridC g, double cx, double cy, double radius,
                           double a_phi, double b_phi, double c_fn,
                           uint32_t step, uint64_t seed, Counters* dc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= g.nxy) return;
  const int i = (int)(t % g.nx), j = (int)(t / g.nx);
  const double ddx = (double)i * g.dx - cx;
  const double ddy = (double)j * g.dx - cy;
  unsigned c = 0;
  if ((ddx * ddx + ddy * ddy) <= radius * radius) {
    const double F = -(double)E[4 * t + 2];
    double J = 0.0;
    if (F > 0.0) J = ((a_phi * F) * F) * exp(-(b_phi / F));
    const double mean = J * c_fn;
    const double fl = floor(mean);
    const double frac = mean - fl;
    double u, unused;
    uniform2((unsigned long long)t | (1ull << 63), step, kTagFn, seed, u, unused);
    if (fabs(u - frac) < 1e-6) atomicAdd(&dc->n_near, 1ull);
    c = (unsigned)fl + (u < frac ? 1u : 0u);
  }
  cnt[t] = c;
}

// Exclusive scan of n values in one workgroup (n <= 1024 * 256); writes
// out[0..n] with out[n] = total.
__global__ void k_scan1(const unsigned* __restrict__ in, unsigned* __restrict__ out,
                        long long n) {
  __shared__ unsigned s[1024];
  const int tid = threadIdx.x;
  const long long per = (n + 1023) / 1024;
  const long long b0 = tid * per;
  unsigned sum = 0;
  for (long long q = 0; q < per; ++q) {
    const long long i = b0 + q;
    if (i < n) sum += in[i];
  }
  s[tid] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned v = tid >= o ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += v;
    __syncthreads();
  }
  unsigned run = tid ? s[tid - 1] : 0u;
  for (long long q = 0; q < per; ++q) {
    const long long i = b0 + q;
    if (i < n) {
      const unsigned v = in[i];
      out[i] = run;
      run += v;
    }
  }
  if (tid == 1023) out[n] = s[1023];
}

template <typename TE>
__global__ void k_fn_spawn(Parts p, long long dst, long long cap,
                           const unsigned* __restrict__ scan, GridC g,
                           unsigned long long id0, double vth2, uint32_t step,
                           uint64_t seed, Counters* dc) {
  const unsigned total = scan[g.nxy];
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t == 0) {
    dc->fn_total = total;
    if ((long long)total > cap) atomicOr(&dc->err, kErrEvents);
  }
  if (t >= total || t >= cap) return;
  // Node: the last one whose scan value is <= t.
  long long lo = 0, hi = g.nxy - 1;
  while (lo < hi) {
    const long long mid = (lo + hi + 1) >> 1;
    if (scan[mid] <= (unsigned)t) lo = mid; else hi = mid - 1;
  }
  const int i = (int)(lo % g.nx), j = (int)(lo / g.nx);
  const unsigned long long id = id0 + (unsigned long long)t;
  double u1, u2, u3, u4;
  uniform2(id, step, kTagSrc0, seed, u1, u2);
  const long long d = dst + t;
  p.x[d] = wrap_coord((double)i * g.dx + (u1 - 0.5) * g.dx, g.lx);
  p.y[d] = wrap_coord((double)j * g.dx + (u2 - 0.5) * g.dx, g.ly);
  p.z[d] = 0.0;
  uniform2(id, step, kTagSrc1, seed, u3, u4);
  p.vx[d] = 0.0;
  p.vy[d] = 0.0;
  p.vz[d] = flux_vz(u3, vth2);
  p.id[d] = id;
}

__global__ void k_fn_commit(Counters* dc, long long cap) {
  unsigned long long t = dc->fn_total;
  if ((long long)t > cap) t = (unsigned long long)cap;
  dc->n[0] += t;
  dc->next_id += t;
}

// ---- deposition ---------------------------------------------------------------
// One workgroup per 8x8x8-cell tile: the tile's electrons and ions (binned
// order) add their quantised CIC weights into a 9x9x9 int64 LDS block with
// 64-bit LDS atomics; the block is then added to the node array with one
// global atomic per non-zero node.  Particles outside the tile (never, when
// the binning invariant holds) fall back to global atomics.
__global__ void __launch_bounds__(kT) k_deposit(
    Parts pe, Parts pi, const uint32_t* __restrict__ tse,
    const uint32_t* __restrict__ tsi, long long* __restrict__ acc, GridC g) {
  __shared__ unsigned long long s[9 * 9 * 9];
  const unsigned t = xcd_block(blockIdx.x, gridDim.x);
  const int tx = (int)(t % g.tnx);
  const int ty = (int)((t / g.tnx) % g.tny);
  const int tz = (int)(t / ((unsigned)g.tnx * g.tny));
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  for (int q = threadIdx.x; q < 729; q += blockDim.x) s[q] = 0ull;
  __syncthreads();
  for (int sp = 0; sp < 2; ++sp) {
    const Parts& p = sp ? pi : pe;
    const uint32_t* ts = sp ? tsi : tse;
    const long long sign = sp ? 1 : -1;
    const unsigned b = ts[t], e = ts[t + 1];
    for (unsigned q = b + threadIdx.x; q < e; q += blockDim.x) {
      int ix, fx, iy, fy, iz, fz;
      cic_axis(p.x[q], g.inv_dx, ix, fx);
      cic_axis(p.y[q], g.inv_dx, iy, fy);
      cic_axis(p.z[q], g.inv_dx, iz, fz);
      if (ix >= g.nx) ix -= g.nx;
      if (iy >= g.ny) iy -= g.ny;
      const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                      wz[2] = {kQ - fz, fz};
      const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
      const bool inside = lx >= 0 && lx < kTile && ly >= 0 && ly < kTile &&
                          lz >= 0 && lz < kTile;
      for (int c = 0; c < 2; ++c)
        for (int bb = 0; bb < 2; ++bb)
          for (int a = 0; a < 2; ++a) {
            const long long v = sign * (wx[a] * wy[bb] * wz[c]);
            if (inside) {
              atomicAdd(&s[((lz + c) * 9 + (ly + bb)) * 9 + (lx + a)],
                        (unsigned long long)v);
            } else {
              const long long node =
                  ((long long)(iz + c) * g.ny + wrap_index(iy + bb, g.ny)) * g.nx +
                  wrap_index(ix + a, g.nx);
              atomicAdd(reinterpret_cast<unsigned long long*>(&acc[node]),
                        (unsigned long long)v);
            }
          }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < 729; q += blockDim.x) {
    const unsigned long long v = s[q];
    if (!v) continue;
    const int a = q % 9, bb = (q / 9) % 9, c = q / 81;
    const int gk = z0 + c;
    if (gk > g.nz) continue;   // (cannot receive charge; partial tiles)
    const int gi = wrap_index(x0 + a, g.nx), gj = wrap_index(y0 + bb, g.ny);
    atomicAdd(reinterpret_cast<unsigned long long*>(
                  &acc[((long long)gk * g.ny + gj) * g.nx + gi]),
              v);
  }
}

// ---- push ---------------------------------------------------------------------
struct MccC {
  int enabled, ion_model;
  double c_coll;          // g_max dt w_sp / dx^3
  double inv_gmax, sigma_el, lotz_a, ion_I, sigma_const, E_max;
  double half_me, ratio;  // 0.5 m_e; 2 m_e / M
  double two_e_me;        // 2 e / m_e
};

// Field at a particle with the deposit's quantised weights, accumulated in
// the fixed order z-corner, y-corner, x-corner.
__device__ __forceinline__ void gather(const double* __restrict__ E,
                                       const GridC& g, double x, double y,
                                       double z, double& ex, double& ey,
                                       double& ez) {
  int ix, fx, iy, fy, iz, fz;
  cic_axis(x, g.inv_dx, ix, fx);
  cic_axis(y, g.inv_dx, iy, fy);
  cic_axis(z, g.inv_dx, iz, fz);
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  ex = 0.0; ey = 0.0; ez = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long row =
          ((long long)(iz + c) * g.ny + wrap_index(iy + b, g.ny)) * g.nx;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double w = (double)(wx[a] * wy[b] * wz[c]) * kQScale;
        const double4 e = *reinterpret_cast<const double4*>(
            E + 4 * (row + wrap_index(ix + a, g.nx)));
        ex = ex + w * e.x;
        ey = ey + w * e.y;
        ez = ez + w * e.z;
      }
    }
  }
}

// Push one species (SP: 0 electron, 1 neutral, 2 ion).  Per particle:
// gather + kick (charged), drift, cathode/anode absorption, x/y wrap, cell
// key; neutrals count themselves per cell; electrons take the null-
// collision candidate draw U1 < 1 - exp(-N_c c_coll) and append candidates.
template <int SP>
__global__ void __launch_bounds__(kT) k_push(
    Parts p, uint32_t* __restrict__ key, const double* __restrict__ E,
    GridC g, double qm_dt, double dt, double mass_half,
    int* __restrict__ ncount, uint32_t* __restrict__ cand, MccC m,
    uint32_t step, uint64_t seed, Rec* __restrict__ ab_rec,
    double* __restrict__ ab_pos, double* __restrict__ ab_vel, long long ab_cap,
    Counters* dc, double* __restrict__ part) {
  __shared__ double sk[kT];
  const long long n = (long long)dc->n[SP];
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const bool live = i < n;
  double ke = 0.0;
  bool cathode = false, is_cand = false;
  unsigned cell = kDead;
  double x = 0, y = 0, z = 0, vx = 0, vy = 0, vz = 0;
  unsigned long long id = 0;
  if (live) {
    x = p.x[i]; y = p.y[i]; z = p.z[i];
    vx = p.vx[i]; vy = p.vy[i]; vz = p.vz[i];
    if (SP != 1) {
      double ex, ey, ez;
      gather(E, g, x, y, z, ex, ey, ez);
      vx = vx + qm_dt * ex;
      vy = vy + qm_dt * ey;
      vz = vz + qm_dt * ez;
    }
    x = x + vx * dt;
    y = y + vy * dt;
    z = z + vz * dt;
    ke = (vx * vx + vy * vy) + vz * vz;
    const double gz = z * g.inv_dx;
    const double xw = wrap_coord(x, g.lx), yw = wrap_coord(y, g.ly);
    if (!(xw >= 0.0 && xw < g.lx && yw >= 0.0 && yw < g.ly) || !(gz == gz) ||
        !isfinite(vx) || !isfinite(vy) || !isfinite(vz)) {
      // Non-finite, or moved more than one period in a step: removed and
      // reported.
      atomicOr(&dc->err, kErrNonFinite);
    } else if (gz < 0.0) {
      cathode = true;
    } else if (gz >= (double)g.nz) {
      atomicAdd(&dc->anode[SP], 1ull);
    } else {
      x = xw;
      y = yw;
      cell = cell_of(x, y, z, g);
      p.x[i] = x; p.y[i] = y; p.z[i] = z;
      p.vx[i] = vx; p.vy[i] = vy; p.vz[i] = vz;
      if (SP == 1) atomicAdd(&ncount[cell], 1);
    }
    key[i] = cell;
    if (SP == 0 && cell != kDead && m.enabled) {
      const int nc = ncount[cell];
      if (nc > 0) {
        id = p.id[i];
        const double pstar = 1.0 - exp(-((double)nc * m.c_coll));
        double u1, u2;
        uniform2(id, step, kTagMcc0, seed, u1, u2);
        if (fabs(u1 - pstar) < 1e-6) atomicAdd(&dc->n_near, 1ull);
        is_cand = u1 < pstar;
      }
    }
  }
  // Cathode sink list (wave-aggregated).
  const unsigned long long slot = wave_append(cathode, &dc->n_ab);
  if (cathode) {
    atomicAdd(&dc->cathode[SP], 1ull);
    if ((long long)slot < ab_cap) {
      const double tc = -z / vz;
      const double xc = wrap_coord(x + vx * tc, g.lx);
      const double yc = wrap_coord(y + vy * tc, g.ly);
      Rec r;
      r.hi = SP; r.lo = p.id[i]; r.val = (unsigned)slot; r.pad = 0;
      ab_rec[slot] = r;
      ab_pos[3 * slot] = xc; ab_pos[3 * slot + 1] = yc; ab_pos[3 * slot + 2] = 0.0;
      ab_vel[3 * slot] = vx; ab_vel[3 * slot + 1] = vy; ab_vel[3 * slot + 2] = vz;
    } else {
      atomicOr(&dc->err, kErrEvents);
    }
  }
  if (SP == 0) {
    const unsigned long long cs = wave_append(is_cand, &dc->n_cand);
    if (is_cand) cand[cs] = (uint32_t)i;
  }
  // Kinetic energy partials (fixed tree per block).
  sk[threadIdx.x] = ke;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sk[threadIdx.x] = sk[threadIdx.x] + sk[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sk[0] * mass_half;
}

__global__ void k_sum_partials(const double* __restrict__ part, long long n,
                               double* out) {
  __shared__ double s[1024];
  double a = 0.0;
  for (long long q = threadIdx.x; q < n; q += blockDim.x) a = a + part[q];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// ---- collisions ---------------------------------------------------------------
__device__ __forceinline__ void isotropic(double uc, double up, double& nx,
                                          double& ny, double& nz) {
  const double c = 1.0 - 2.0 * uc;
  const double s = sqrt(1.0 - c * c);
  const double ps = kTwoPi * up;
  nx = s * cos(ps);
  ny = s * sin(ps);
  nz = c;
}

__device__ __forceinline__ double sigma_ion(const MccC& m, double E_eV) {
  if (!(E_eV > m.ion_I)) return 0.0;
  if (m.ion_model == PIC_ION_LOTZ)
    return (m.lotz_a * log(E_eV / m.ion_I)) / (E_eV * m.ion_I);
  return m.sigma_const;
}

// Candidates: second draw U2 against the cumulative process probabilities
// (ionisation, then elastic).  Elastic scattering is applied at once;
// ionisation events are recorded as (cell, electron id) for matching.
__global__ void k_mcc(Parts p, const uint32_t* __restrict__ key,
                      const uint32_t* __restrict__ cand, MccC m, uint32_t step,
                      uint64_t seed, Rec* __restrict__ ev, uint8_t* __restrict__ flag,
                      long long ev_cap, Counters* dc) {
  const long long nc = (long long)dc->n_cand;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < nc;
       t += (long long)gridDim.x * blockDim.x) {
    const uint32_t i = cand[t];
    const unsigned long long id = p.id[i];
    const double vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
    double u1, u2;
    uniform2(id, step, kTagMcc0, seed, u1, u2);
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    const double v = sqrt(v2);
    const double E_eV = (m.half_me * v2) / kE;
    if (E_eV > m.E_max) atomicAdd(&dc->n_over, 1ull);
    const double s_ion = sigma_ion(m, E_eV);
    const double p_ion = (s_ion * v) * m.inv_gmax;
    const double p_el = (m.sigma_el * v) * m.inv_gmax;
    const double p_tot = p_ion + p_el;
    if ((p_ion > 0.0 && fabs(u2 - p_ion) < 1e-6) || fabs(u2 - p_tot) < 1e-6)
      atomicAdd(&dc->n_near, 1ull);
    if (u2 < p_ion) {
      const unsigned long long s = atomicAdd(&dc->n_events, 1ull);
      const uint32_t cell = key[i];
      if ((long long)s < ev_cap) {
        Rec r;
        r.hi = cell; r.lo = id; r.val = i; r.pad = 0;
        ev[s] = r;
        flag[cell] = 1;
      } else {
        atomicOr(&dc->err, kErrEvents);
      }
    } else if (u2 < p_tot) {
      atomicAdd(&dc->n_elastic, 1ull);
      double u3, u4, nx, ny, nz;
      uniform2(id, step, kTagMcc1, seed, u3, u4);
      isotropic(u3, u4, nx, ny, nz);
      const double cosx = ((vx * nx + vy * ny) + vz * nz) / v;
      const double fac = sqrt(1.0 - m.ratio * (1.0 - cosx));
      const double sp = v * fac;
      p.vx[i] = sp * nx;
      p.vy[i] = sp * ny;
      p.vz[i] = sp * nz;
    }
  }
}

// Bitonic sort of a small record list by (hi, lo) in one workgroup: in LDS
// when it fits, otherwise in place in global memory.  At most cap records
// are valid; the buffer holds the next power of two above cap.
__global__ void __launch_bounds__(1024) k_sort_small(
    Rec* __restrict__ a, const unsigned long long* __restrict__ count,
    long long cap) {
  __shared__ Rec s[kSmallLds];
  long long n = (long long)*count;
  if (n > cap) n = cap;
  if (n <= 1) return;
  long long P = 1;
  while (P < n) P <<= 1;
  const Rec maxr = {~0ull, ~0ull, 0u, 0u};
  if (P <= kSmallLds) {
    for (long long q = threadIdx.x; q < P; q += blockDim.x) s[q] = q < n ? a[q] : maxr;
    __syncthreads();
    for (long long k = 2; k <= P; k <<= 1)
      for (long long j = k >> 1; j > 0; j >>= 1) {
        for (long long q = threadIdx.x; q < P; q += blockDim.x) {
          const long long o = q ^ j;
          if (o > q) {
            const bool up = (q & k) == 0;
            const Rec x = s[q], y = s[o];
            if (up ? rec_less(y, x) : rec_less(x, y)) { s[q] = y; s[o] = x; }
          }
        }
        __syncthreads();
      }
    for (long long q = threadIdx.x; q < n; q += blockDim.x) a[q] = s[q];
    return;
  }
  for (long long q = n + threadIdx.x; q < P; q += blockDim.x) a[q] = maxr;
  __syncthreads();
  for (long long k = 2; k <= P; k <<= 1)
    for (long long j = k >> 1; j > 0; j >>= 1) {
      for (long long q = threadIdx.x; q < P; q += blockDim.x) {
        const long long o = q ^ j;
        if (o > q) {
          const bool up = (q & k) == 0;
          const Rec x = a[q], y = a[o];
          if (up ? rec_less(y, x) : rec_less(x, y)) { a[q] = y; a[o] = x; }
        }
      }
      __syncthreads();
    }
}

// Neutrals in cells that hold ionisation events.
__global__ void k_neutral_cands(Parts p, const uint32_t* __restrict__ key,
                                const uint8_t* __restrict__ flag,
                                Rec* __restrict__ nc, long long cap,
                                Counters* dc) {
  if (dc->n_events == 0) return;
  const long long n = (long long)dc->n[1];
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  bool hit = false;
  unsigned cell = kDead;
  if (i < n) {
    cell = key[i];
    hit = cell != kDead && flag[cell];
  }
  const unsigned long long s = wave_append(hit, &dc->n_ncand);
  if (hit) {
    if ((long long)s < cap) {
      Rec r;
      r.hi = cell; r.lo = p.id[i]; r.val = (unsigned)i; r.pad = 0;
      nc[s] = r;
    } else {
      atomicOr(&dc->err, kErrEvents);
    }
  }
}

// Events (sorted by cell, id): the r-th event of a cell takes the cell's
// r-th neutral (sorted by id) if there is one.
__global__ void k_match(const Rec* __restrict__ ev, const Rec* __restrict__ nc,
                        Rec* __restrict__ ok, long long cap, Counters* dc) {
  long long ne = (long long)dc->n_events;
  if (ne > cap) ne = cap;
  long long nn = (long long)dc->n_ncand;
  if (nn > cap) nn = cap;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < ne;
       e += (long long)gridDim.x * blockDim.x) {
    const unsigned long long cell = ev[e].hi;
    long long r = 0;
    while (e - r - 1 >= 0 && ev[e - r - 1].hi == cell) ++r;
    long long lo = 0, hi = nn;
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (nc[mid].hi < cell) lo = mid + 1; else hi = mid;
    }
    long long end = lo;
    while (end < nn && nc[end].hi == cell) ++end;
    if (lo + r < end) {
      const unsigned long long s = atomicAdd(&dc->n_ok, 1ull);
      Rec o;
      o.hi = 0; o.lo = ev[e].lo; o.val = ev[e].val; o.pad = nc[lo + r].val;
      ok[s] = o;
    }
  }
}

// Matched events in primary-id order: secondary ids next_id + rank; energy
// above threshold shared uniformly, both electrons isotropic; the neutral
// becomes the Cu+ ion (same position, velocity, id).
__global__ void k_ionise(Parts pe, Parts pn, Parts pi, uint32_t* __restrict__ ke,
                         uint32_t* __restrict__ kn, uint32_t* __restrict__ ki,
                         const Rec* __restrict__ ok, MccC m, uint32_t step,
                         uint64_t seed, long long cap_e, long long cap_i,
                         Counters* dc) {
  const long long nok = (long long)dc->n_ok;
  const long long ne0 = (long long)dc->n[0], ni0 = (long long)dc->n[2];
  const unsigned long long id0 = dc->next_id;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < nok;
       r += (long long)gridDim.x * blockDim.x) {
    const uint32_t ie = ok[r].val, in = ok[r].pad;
    const unsigned long long pid = ok[r].lo;
    double u3, u4, u5, u6, u7, u8;
    uniform2(pid, step, kTagMcc1, seed, u3, u4);
    uniform2(pid, step, kTagMcc2, seed, u5, u6);
    uniform2(pid, step, kTagMcc3, seed, u7, u8);
    const double vx = pe.vx[ie], vy = pe.vy[ie], vz = pe.vz[ie];
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    const double E_eV = (m.half_me * v2) / kE;
    const double avail = E_eV - m.ion_I;
    const double Es = u3 * avail;
    const double Ep = avail - Es;
    const double vp = sqrt(Ep * m.two_e_me);
    const double vs = sqrt(Es * m.two_e_me);
    double px, py, pz, sx, sy, sz;
    isotropic(u4, u5, px, py, pz);
    isotropic(u6, u7, sx, sy, sz);
    pe.vx[ie] = vp * px; pe.vy[ie] = vp * py; pe.vz[ie] = vp * pz;
    const long long de = ne0 + r, di = ni0 + r;
    if (de < cap_e && di < cap_i) {
      pe.x[de] = pe.x[ie]; pe.y[de] = pe.y[ie]; pe.z[de] = pe.z[ie];
      pe.vx[de] = vs * sx; pe.vy[de] = vs * sy; pe.vz[de] = vs * sz;
      pe.id[de] = id0 + (unsigned long long)r;
      ke[de] = ke[ie];
      pi.x[di] = pn.x[in]; pi.y[di] = pn.y[in]; pi.z[di] = pn.z[in];
      pi.vx[di] = pn.vx[in]; pi.vy[di] = pn.vy[in]; pi.vz[di] = pn.vz[in];
      pi.id[di] = pn.id[in];
      ki[di] = kn[in];
    } else {
      atomicOr(&dc->err, kErrCapacity);
    }
    kn[in] = kDead;
  }
}

__global__ void k_ionise_commit(Counters* dc, const Rec* __restrict__ ev,
                                uint8_t* __restrict__ flag, long long cap,
                                long long cap_e, long long cap_i) {
  long long ne = (long long)dc->n_events;
  if (ne > cap) ne = cap;
  for (long long e = threadIdx.x; e < ne; e += blockDim.x) flag[ev[e].hi] = 0;
  __syncthreads();
  if (threadIdx.x) return;
  long long ok = (long long)dc->n_ok;
  long long add = ok;
  if ((long long)dc->n[0] + add > cap_e) add = cap_e - (long long)dc->n[0];
  if ((long long)dc->n[2] + add > cap_i) add = cap_i - (long long)dc->n[2];
  if (add < 0) add = 0;
  dc->n[0] += add;
  dc->n[2] += add;
  dc->next_id += ok;
}

// Sorted cathode list -> output arrays (SoA, stride n).
__global__ void k_ab_gather(const Rec* __restrict__ rec,
                            const double* __restrict__ rpos,
                            const double* __restrict__ rvel,
                            int32_t* __restrict__ sp, uint64_t* __restrict__ id,
                            double* __restrict__ pos, double* __restrict__ vel,
                            long long cap, Counters* dc) {
  long long n = (long long)dc->n_ab;
  if (n > cap) n = cap;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x) {
    const unsigned s = rec[r].val;
    sp[r] = (int32_t)rec[r].hi;
    id[r] = rec[r].lo;
    for (int d = 0; d < 3; ++d) {
      pos[d * n + r] = rpos[3 * s + d];
      vel[d * n + r] = rvel[3 * s + d];
    }
  }
}

// ---- binning ------------------------------------------------------------------
__global__ void k_tile_hist(const uint32_t* __restrict__ key, unsigned* __restrict__ cnt,
                            GridC g, const unsigned long long* __restrict__ np) {
  const long long n = (long long)*np;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  unsigned t = kDead;
  if (i < n) {
    const uint32_t k = key[i];
    if (k != kDead) t = tile_of_cell(k, g);
  }
  run_add(t, cnt, false);
}

// Multi-block exclusive scan of the tile counts: per-block sums, a scan of
// the block sums, then the per-block scans with their offsets.
constexpr int kScanPer = 1024;  // elements per block (256 threads x 4)

__global__ void k_scan_blocks(const unsigned* __restrict__ in, long long n,
                              unsigned* __restrict__ bsum) {
  __shared__ unsigned s[kT];
  const long long b0 = (long long)blockIdx.x * kScanPer;
  unsigned a = 0;
  for (int q = 0; q < 4; ++q) {
    const long long i = b0 + threadIdx.x * 4 + q;
    if (i < n) a += in[i];
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

__global__ void k_scan_apply(const unsigned* __restrict__ in, long long n,
                             const unsigned* __restrict__ bscan,
                             unsigned* __restrict__ out,
                             unsigned* __restrict__ cursor) {
  __shared__ unsigned s[kT];
  const long long b0 = (long long)blockIdx.x * kScanPer;
  unsigned v[4];
  unsigned a = 0;
  for (int q = 0; q < 4; ++q) {
    const long long i = b0 + threadIdx.x * 4 + q;
    v[q] = i < n ? in[i] : 0u;
    a += v[q];
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 1; o < kT; o <<= 1) {
    const unsigned t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  unsigned run = bscan[blockIdx.x] + (threadIdx.x ? s[threadIdx.x - 1] : 0u);
  for (int q = 0; q < 4; ++q) {
    const long long i = b0 + threadIdx.x * 4 + q;
    if (i < n) {
      out[i] = run;
      cursor[i] = run;
    }
    if (i == n) out[n] = run;
    run += v[q];
  }
}

// Move each live particle to its tile's range in the other buffer.  The
// keys are not carried along: the next push rewrites them.
__global__ void __launch_bounds__(kT) k_scatter(
    Parts src, Parts dst, const uint32_t* __restrict__ key,
    unsigned* __restrict__ cursor, GridC g,
    const unsigned long long* __restrict__ np) {
  const long long n = (long long)*np;
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  unsigned t = kDead;
  uint32_t k = kDead;
  if (i < n) {
    k = key[i];
    if (k != kDead) t = tile_of_cell(k, g);
  }
  const unsigned d = run_add(t, cursor, true);
  if (t == kDead) return;
  dst.x[d] = src.x[i]; dst.y[d] = src.y[i]; dst.z[d] = src.z[i];
  dst.vx[d] = src.vx[i]; dst.vy[d] = src.vy[i]; dst.vz[d] = src.vz[i];
  dst.id[d] = src.id[i];
}

__global__ void k_set_count(Counters* dc, int s, const unsigned* __restrict__ ts,
                            long long ntiles) {
  dc->n[s] = ts[ntiles];
  dc->sorted_n[s] = ts[ntiles];
}

// Cell keys of loaded particles; flags out-of-domain or non-finite input.
__global__ void k_keys(Parts p, uint32_t* __restrict__ key, long long n,
                       GridC g, Counters* dc) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = p.x[i], y = p.y[i], z = p.z[i];
  const double gz = z * g.inv_dx;
  const bool ok = x >= 0.0 && x < g.lx && y >= 0.0 && y < g.ly && gz >= 0.0 &&
                  gz < (double)g.nz && isfinite(p.vx[i]) && isfinite(p.vy[i]) &&
                  isfinite(p.vz[i]);
  if (!ok) {
    atomicOr(&dc->err, kErrNonFinite);
    key[i] = kDead;
    return;
  }
  key[i] = cell_of(x, y, z, g);
}

// Count injected particles outside the domain (or non-finite).
__global__ void k_validate(const double* __restrict__ pos,
                           const double* __restrict__ vel, long long n,
                           GridC g, unsigned long long* bad) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = pos[t], y = pos[n + t], z = pos[2 * n + t];
  const double gz = z * g.inv_dx;
  const bool ok = x >= 0.0 && x < g.lx && y >= 0.0 && y < g.ly && gz >= 0.0 &&
                  gz < (double)g.nz && isfinite(vel[t]) &&
                  isfinite(vel[n + t]) && isfinite(vel[2 * n + t]);
  if (!ok) atomicAdd(bad, 1ull);
}

__global__ void k_load(Parts p, const double* __restrict__ pos,
                       const double* __restrict__ vel,
                       const uint64_t* __restrict__ ids, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  p.x[t] = pos[t]; p.y[t] = pos[n + t]; p.z[t] = pos[2 * n + t];
  p.vx[t] = vel[t]; p.vy[t] = vel[n + t]; p.vz[t] = vel[2 * n + t];
  p.id[t] = ids[t];
}

__global__ void k_read(Parts p, double* __restrict__ pos, double* __restrict__ vel,
                       uint64_t* __restrict__ ids, long long n) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  pos[t] = p.x[t]; pos[n + t] = p.y[t]; pos[2 * n + t] = p.z[t];
  vel[t] = p.vx[t]; vel[n + t] = p.vy[t]; vel[2 * n + t] = p.vz[t];
  ids[t] = p.id[t];
}

MccC mcc_constants(const pic_ctx* c, double dt) {
  MccC m;
  const pic_collisions& k = c->coll;
  m.enabled = k.enabled;
  m.ion_model = k.ion_model;
  m.sigma_el = k.sigma_el;
  m.lotz_a = k.lotz_a;
  m.ion_I = k.ion_I_eV;
  m.sigma_const = k.sigma_ion_const;
  m.E_max = k.E_max_eV;
  const double sig_max = k.ion_model == PIC_ION_LOTZ
                             ? k.lotz_a / (kEuler * k.ion_I_eV * k.ion_I_eV)
                             : k.sigma_ion_const;
  const double v_max = sqrt((2.0 * (k.E_max_eV * kE)) / kMe);
  const double g_max = (k.sigma_el + sig_max) * v_max;
  m.inv_gmax = g_max > 0.0 ? 1.0 / g_max : 0.0;
  if (!(g_max > 0.0)) m.enabled = 0;
  const double inv_dx = c->g.inv_dx;
  const double inv_dx3 = (inv_dx * inv_dx) * inv_dx;
  m.c_coll = ((g_max * dt) * (double)c->cfg.w_sp) * inv_dx3;
  m.half_me = 0.5 * kMe;
  m.ratio = (2.0 * kMe) / kMcu;
  m.two_e_me = (2.0 * kE) / kMe;
  return m;
}

// Launch bound of a species: the host's upper bound of the device count,
// never above the capacity (kernels read the exact count on the device).
long long bound(const pic_ctx* c, int s) {
  long long n = c->n[s];
  if (n > c->cfg.capacity[s]) n = c->cfg.capacity[s];
  return n > 0 ? n : 1;
}

double qm_dt(int s, double dt) {
  const double q = s == 0 ? -kE : (s == 2 ? kE : 0.0);
  const double mass = s == 0 ? kMe : kMcu;
  return (q / mass) * dt;
}

}  // namespace

void parts_begin_step(pic_ctx* c) {
  (void)c;
}

void parts_deposit(pic_ctx* c) {
  hipMemsetAsync(c->acc, 0, c->nnodes * sizeof(long long), c->stream);
  k_deposit<<<(unsigned)c->ntiles, kT, 0, c->stream>>>(
      c->P[0][c->cur[0]], c->P[2][c->cur[2]], c->tile_start[0],
      c->tile_start[2], c->acc, c->g);
}

// Queue, disk, sphere and Fowler-Nordheim particles, ids in that order.
void parts_sources(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  long long n[3] = {c->n[0], c->n[1], c->n[2]};
  unsigned long long nid = c->next_id;
  for (const QueueCall& q : c->queue) {
    if (q.n <= 0) continue;
    k_append_queue<<<nblk(q.n), kT, 0, st>>>(
        c->P[q.species][c->cur[q.species]], n[q.species], c->q_pos + 3 * q.offset,
        c->q_vel + 3 * q.offset, q.n, nid);
    n[q.species] += q.n;
    nid += q.n;
  }
  c->queue.clear();
  c->queue_used = 0;
  const pic_sources& s = c->src;
  if (s.disk_on) {
    if (s.disk_n_e > 0) {
      const double vth2 = (s.disk_kT_e_eV * kE) / kMe;
      k_disk<<<nblk(s.disk_n_e), kT, 0, st>>>(
          c->P[0][c->cur[0]], n[0], s.disk_n_e, nid, 0, s.disk_cx, s.disk_cy,
          s.disk_radius, vth2, c->g, step, seed);
      n[0] += s.disk_n_e;
      nid += s.disk_n_e;
    }
    if (s.disk_n_n > 0) {
      const double vth2 = (kKB * s.disk_T_n_K) / kMcu;
      k_disk<<<nblk(s.disk_n_n), kT, 0, st>>>(
          c->P[1][c->cur[1]], n[1], s.disk_n_n, nid, 1, s.disk_cx, s.disk_cy,
          s.disk_radius, vth2, c->g, step, seed);
      n[1] += s.disk_n_n;
      nid += s.disk_n_n;
    }
  }
  if (s.sphere_on && s.sph_n > 0) {
    const double sig = sqrt((kKB * s.sph_T_K) / kMcu);
    k_sphere<<<nblk(s.sph_n), kT, 0, st>>>(
        c->P[1][c->cur[1]], n[1], s.sph_n, nid, s.sph_cx, s.sph_cy, s.sph_cz,
        s.sph_radius, sig, c->g, step, seed);
    n[1] += s.sph_n;
    nid += s.sph_n;
  }
  k_begin<<<1, 1, 0, st>>>(c->dc, n[0], n[1], n[2], nid);
  if (s.fn_on) {
    const double phi_j = s.fn_phi_w_eV * kE;
    const double a_fn = pow(kE, 3.0) / (8.0 * kPi * kH);
    const double b_fn = (8.0 * kPi * sqrt(2.0 * kMe)) / (3.0 * kE * kH);
    const double a_phi = a_fn / phi_j;
    const double b_phi = b_fn * phi_j * sqrt(phi_j);
    const double c_fn = ((c->g.dx * c->g.dx) * dt) / kE;
    if (c->mixed)
      k_fn_count<float><<<nblk(c->g.nxy), kT, 0, st>>>(
          reinterpret_cast<const float*>(c->E), c->fn_scan + c->g.nxy + 1, c->g,
          s.fn_cx, s.fn_cy, s.fn_radius, a_phi, b_phi, c_fn, step, seed, c->dc);
    else
      k_fn_count<double><<<nblk(c->g.nxy), kT, 0, st>>>(
          c->E, c->fn_scan + c->g.nxy + 1, c->g, s.fn_cx, s.fn_cy, s.fn_radius,
          a_phi, b_phi, c_fn, step, seed, c->dc);
    k_scan1<<<1, 1024, 0, st>>>(c->fn_scan + c->g.nxy + 1, c->fn_scan, c->g.nxy);
    long long cap = c->cfg.max_events;
    if (n[0] + cap > c->cfg.capacity[0]) cap = c->cfg.capacity[0] - n[0];
    if (cap < 0) cap = 0;
    const double vth2 = (s.fn_kT_e_eV * kE) / kMe;
    k_fn_spawn<double><<<nblk(c->cfg.max_events > 0 ? c->cfg.max_events : 1), kT, 0, st>>>(
        c->P[0][c->cur[0]], n[0], cap, c->fn_scan, c->g, nid, vth2, step, seed,
        c->dc);
    k_fn_commit<<<1, 1, 0, st>>>(c->dc, cap);
  }
  // Upper bounds of the counts for the launches that follow.
  c->n[0] = n[0] + (s.fn_on ? c->cfg.max_events : 0);
  c->n[1] = n[1];
  c->n[2] = n[2];
}

void parts_push_collide(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  MccC m = mcc_constants(c, dt);
  hipMemsetAsync(c->ncount, 0, c->ncells * sizeof(int), st);
  const long long ab_cap = c->cfg.max_events;
  double* kpart = c->partials;
  // Neutrals first: their per-cell counts are the MCC target densities.
  const int order[3] = {1, 2, 0};
  for (int oi = 0; oi < 3; ++oi) {
    const int s = order[oi];
    const long long nb = nblk(bound(c, s));
    Parts p = c->P[s][c->cur[s]];
    const double mh = 0.5 * (s == 0 ? kMe : kMcu);
    if (s == 1)
      k_push<1><<<nb, kT, 0, st>>>(p, c->key[1], c->E, c->g, 0.0, dt, mh,
                                   c->ncount, c->cand, m, step, seed, c->ab_rec,
                                   c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc,
                                   kpart);
    else if (s == 2)
      k_push<2><<<nb, kT, 0, st>>>(p, c->key[2], c->E, c->g, qm_dt(2, dt), dt,
                                   mh, c->ncount, c->cand, m, step, seed,
                                   c->ab_rec, c->ab_raw_pos, c->ab_raw_vel,
                                   ab_cap, c->dc, kpart);
    else
      k_push<0><<<nb, kT, 0, st>>>(p, c->key[0], c->E, c->g, qm_dt(0, dt), dt,
                                   mh, c->ncount, c->cand, m, step, seed,
                                   c->ab_rec, c->ab_raw_pos, c->ab_raw_vel,
                                   ab_cap, c->dc, kpart);
    k_sum_partials<<<1, 1024, 0, st>>>(kpart, nb, &c->dc->kinetic[s]);
  }
  // Record lists hold max_events entries (buffers are padded to a power of
  // two for the bitonic sort).
  const long long cap = c->cfg.max_events;
  if (m.enabled) {
    k_mcc<<<kFixedBlocks, kT, 0, st>>>(c->P[0][c->cur[0]], c->key[0], c->cand,
                                       m, step, seed, c->ev, c->flag, cap, c->dc);
    k_sort_small<<<1, 1024, 0, st>>>(c->ev, &c->dc->n_events, cap);
    k_neutral_cands<<<nblk(bound(c, 1)), kT, 0, st>>>(
        c->P[1][c->cur[1]], c->key[1], c->flag, c->nc, cap, c->dc);
    k_sort_small<<<1, 1024, 0, st>>>(c->nc, &c->dc->n_ncand, cap);
    k_match<<<64, kT, 0, st>>>(c->ev, c->nc, c->ok, cap, c->dc);
    k_sort_small<<<1, 1024, 0, st>>>(c->ok, &c->dc->n_ok, cap);
    k_ionise<<<64, kT, 0, st>>>(c->P[0][c->cur[0]], c->P[1][c->cur[1]],
                                c->P[2][c->cur[2]], c->key[0], c->key[1],
                                c->key[2], c->ok, m, step, seed,
                                c->cfg.capacity[0], c->cfg.capacity[2], c->dc);
    k_ionise_commit<<<1, 1024, 0, st>>>(c->dc, c->ev, c->flag, cap,
                                        c->cfg.capacity[0], c->cfg.capacity[2]);
    c->n[0] += cap;  // bound: secondaries
    c->n[2] += cap;
  }
  // Cathode list sorted by (species, id).
  k_sort_small<<<1, 1024, 0, st>>>(c->ab_rec, &c->dc->n_ab, cap);
  k_ab_gather<<<64, kT, 0, st>>>(c->ab_rec, c->ab_raw_pos, c->ab_raw_vel,
                                 c->ab_species, c->ab_id, c->ab_pos, c->ab_vel,
                                 cap, c->dc);
}

void parts_bin_species(pic_ctx* c, int s) {
  hipStream_t st = c->stream;
  const long long nb = nblk(bound(c, s));
  hipMemsetAsync(c->tile_cursor, 0, (c->ntiles + 1) * sizeof(unsigned), st);
  k_tile_hist<<<nb, kT, 0, st>>>(c->key[s], c->tile_cursor, c->g, &c->dc->n[s]);
  const long long nsb = (c->ntiles + 1 + kScanPer - 1) / kScanPer;
  k_scan_blocks<<<(unsigned)nsb, kT, 0, st>>>(c->tile_cursor, c->ntiles,
                                              c->scan_block);
  k_scan1<<<1, 1024, 0, st>>>(c->scan_block, c->scan_block + nsb + 1, nsb);
  k_scan_apply<<<(unsigned)nsb, kT, 0, st>>>(c->tile_cursor, c->ntiles,
                                             c->scan_block + nsb + 1,
                                             c->tile_start[s], c->tile_cursor);
  const int o = c->cur[s] ^ 1;
  k_scatter<<<nb, kT, 0, st>>>(c->P[s][c->cur[s]], c->P[s][o], c->key[s],
                               c->tile_cursor, c->g, &c->dc->n[s]);
  k_set_count<<<1, 1, 0, st>>>(c->dc, s, c->tile_start[s], c->ntiles);
  c->cur[s] = o;
}

void parts_bin(pic_ctx* c) {
  for (int s = 0; s < 3; ++s) parts_bin_species(c, s);
}

void parts_finish_step(pic_ctx* c) { (void)c; }

void parts_load(pic_ctx* c, int s, long long n, const double* pos,
                const double* vel, const uint64_t* ids) {
  hipStream_t st = c->stream;
  Parts p = c->P[s][c->cur[s]];
  if (n > 0) {
    k_load<<<nblk(n), kT, 0, st>>>(p, pos, vel, ids, n);
    k_keys<<<nblk(n), kT, 0, st>>>(p, c->key[s], n, c->g, c->dc);
  }
}

bool parts_validate(pic_ctx* c, const double* pos, const double* vel,
                    long long n) {
  if (n <= 0) return true;
  hipMemsetAsync(&c->dc->n_ncand, 0, sizeof(unsigned long long), c->stream);
  k_validate<<<nblk(n), kT, 0, c->stream>>>(pos, vel, n, c->g, &c->dc->n_ncand);
  unsigned long long bad = 0;
  hipMemcpyAsync(&bad, &c->dc->n_ncand, sizeof(bad), hipMemcpyDeviceToHost,
                 c->stream);
  hipStreamSynchronize(c->stream);
  return bad == 0;
}

void parts_keys(pic_ctx* c, int s) {
  const long long n = c->n[s];
  if (n > 0)
    k_keys<<<nblk(n), kT, 0, c->stream>>>(c->P[s][c->cur[s]], c->key[s], n,
                                          c->g, c->dc);
}

void parts_read(pic_ctx* c, int s, long long n, double* pos, double* vel,
                uint64_t* ids) {
  if (n > 0)
    k_read<<<nblk(n), kT, 0, c->stream>>>(c->P[s][c->cur[s]], pos, vel, ids, n);
}

}  // namespace pic
