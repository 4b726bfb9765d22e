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
#include <algorithm>

#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
// Records per LDS-sorted chunk and the workgroup that sorts it.  The
// bitonic pass is bound by LDS bandwidth (16-byte records): small chunks
// spread a list over many CUs, at the cost of two more merge rounds.
constexpr int kSortChunk = 256;
constexpr int kSortT = kSortChunk / 2;  // one compare-exchange per thread and stage
// Segment whose merge rounds run in LDS, in one launch (64 KB of records),
// and its workgroup (four records per thread).
constexpr int kMergeSeg = 4096;
constexpr int kMergeT = 1024;
static_assert(kMergeSeg % kSortChunk == 0 && kMergeSeg == 4 * kMergeT, "");
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

// Lanes below this one whose bit is set in mask.
__device__ __forceinline__ unsigned lanes_below(unsigned long long mask) {
  const int lane = lane_id();
  return lane ? (unsigned)__popcll(mask & (~0ull >> (64 - lane))) : 0u;
}

// Wave-aggregated count: the lanes with pred add one each to *counter
// (one atomic per wave).  All lanes must call it.
__device__ __forceinline__ void wave_count(bool pred,
                                           unsigned long long* counter) {
  const unsigned long long mask = __ballot(pred);
  if (!mask) return;
  if (lane_id() == __ffsll((long long)mask) - 1)
    atomicAdd(counter, (unsigned long long)__popcll(mask));
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

// Tile (u) of a cell and its slot among the 27 tiles around the source tile
// (tx, ty, tz), x and y periodic, or -1 when it lies further away.  One
// decode of the cell (two divisions); tile coordinates are shifts.
__device__ __forceinline__ int dest_slot(unsigned cell, int tx, int ty, int tz,
                                         const GridC& g, unsigned& u) {
  const unsigned i = cell % (unsigned)g.nx;
  const unsigned r = cell / (unsigned)g.nx;
  const unsigned j = r % (unsigned)g.ny;
  const unsigned k = r / (unsigned)g.ny;
  const int ux = (int)(i / kTile), uy = (int)(j / kTile), uz = (int)(k / kTile);
  u = ((unsigned)uz * (unsigned)g.tny + (unsigned)uy) * (unsigned)g.tnx + (unsigned)ux;
  int ox = ux - tx, oy = uy - ty;
  const int oz = uz - tz;
  if (ox > 1) ox -= g.tnx;
  if (ox < -1) ox += g.tnx;
  if (oy > 1) oy -= g.tny;
  if (oy < -1) oy += g.tny;
  if (ox < -1 || ox > 1 || oy < -1 || oy > 1 || oz < -1 || oz > 1) return -1;
  return ((oz + 1) * 3 + (oy + 1)) * 3 + (ox + 1);
}

// Count a pushed particle's destination tile for the binning pass: per
// neighbouring tile in LDS (sc, sd), else straight into the global counts.
// Returns the slot (13: its own tile; -1: farther; -2: removed).
constexpr int kSlotSelf = 13;
__device__ __forceinline__ int count_dest(unsigned cell, int tx, int ty,
                                          int tz, const GridC& g,
                                          unsigned* sc, unsigned* sd,
                                          unsigned* __restrict__ cnt) {
  if (cell == kDead) return -2;
  unsigned u;
  const int d = dest_slot(cell, tx, ty, tz, g, u);
  if (d >= 0) {
    atomicAdd(&sc[d], 1u);
    sd[d] = u;
  } else {
    atomicAdd(&cnt[u], 1u);
  }
  return d;
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

// ---- chunk work lists ----------------------------------------------------------
// A tile's binned particles of a species are split into pieces of at most
// kChunk, so a crowded tile (e.g. the neutrals above an evaporating disk)
// spreads over several workgroups.  A chunk (tile, piece) serves every
// species of its list: piece k of a tile covers [ts[t] + k kChunk, ...).
constexpr unsigned kChunk = 2048;

__device__ __forceinline__ void piece(const uint32_t* __restrict__ ts,
                                      unsigned t, unsigned k, unsigned& b,
                                      unsigned& e) {
  const unsigned tb = ts[t], te = ts[t + 1];
  b = tb + k * kChunk;
  if (b > te) b = te;
  e = te - b > kChunk ? b + kChunk : te;
}

__global__ void k_chunk_count(const uint32_t* __restrict__ ta,
                              const uint32_t* __restrict__ tb, long long nt,
                              unsigned* __restrict__ cnt) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const unsigned na = ta[t + 1] - ta[t];
  const unsigned nb = tb ? tb[t + 1] - tb[t] : 0u;
  const unsigned ca = (na + kChunk - 1) / kChunk, cb = (nb + kChunk - 1) / kChunk;
  cnt[t] = ca > cb ? ca : cb;
}

__global__ void k_chunk_fill(const unsigned* __restrict__ cstart, long long nt,
                             uint2* __restrict__ chunks) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nt) return;
  const unsigned b = cstart[t], e = cstart[t + 1];
  for (unsigned k = 0; b + k < e; ++k) chunks[b + k] = make_uint2((unsigned)t, k);
}

// ---- step bookkeeping ---------------------------------------------------------
__global__ void k_begin(Counters* dc, unsigned long long n0,
                        unsigned long long n1, unsigned long long n2,
                        unsigned long long n3, unsigned long long next_id) {
  dc->n[0] = n0; dc->n[1] = n1; dc->n[2] = n2; dc->n[3] = n3;
  dc->next_id = next_id;
  dc->fn_total = 0;
  for (int s = 0; s < 4; ++s) {
    dc->cathode[s] = 0; dc->anode[s] = 0; dc->kinetic[s] = 0.0;
    dc->sorted_n[s] = 0;
  }
  dc->n_dead = dc->n_holes = dc->n_movers = 0;
  dc->n_cand = dc->n_elastic = dc->n_events = dc->n_ok = 0;
  dc->n_over = dc->n_near = dc->n_ab = dc->n_ncand = 0;
  dc->n_tail_cand = dc->n_el_tail = 0;
  dc->ion_moved = dc->n_dead1 = dc->n_dead2 = 0;
  dc->np_hits = 0;
  dc->np_heat = 0.0;
  dc->coul_like = dc->coul_ei = 0;
  dc->f3_rec = dc->f3_ion2 = dc->f3_cx = dc->f3_starved = 0;
}

// ---- sources ------------------------------------------------------------------
template <class PT>
__global__ void k_append_queue(PT p, long long dst, const double* __restrict__ qpos,
                               const double* __restrict__ qvel, long long n,
                               unsigned long long id0, GridC g) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const long long d = dst + t;
  Acc<PT>::set_pos(p, d, g, qpos[t], qpos[n + t], qpos[2 * n + t]);
  Acc<PT>::set_vel(p, d, qvel[t], qvel[n + t], qvel[2 * n + t]);
  p.id[d] = id0 + (unsigned long long)t;
}

__device__ __forceinline__ double flux_vz(double u, double vth2) {
  return sqrt((-2.0 * vth2) * log(1.0 - u));
}

// Disk at z = 0.  species 0: electrons (normal speed from a flux-weighted
// half-Maxwellian, no tangential velocity); species 1: neutrals (Gaussian
// tangential components, flux-weighted normal component).
template <class PT>
__global__ void k_disk(PT p, long long dst, long long n,
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
  Acc<PT>::set_pos(p, d, g, wrap_coord(cx + r * cos(th), g.lx),
                   wrap_coord(cy + r * sin(th), g.ly), 0.0);
  p.id[d] = id;
  uniform2(id, step, kTagSrc1, seed, u3, u4);
  if (species == 0) {
    Acc<PT>::set_vel(p, d, 0.0, 0.0, flux_vz(u3, vth2));
  } else {
    const double rr = sqrt((-2.0 * vth2) * log(1.0 - u3));
    const double ph = kTwoPi * u4;
    double u5, u6;
    uniform2(id, step, kTagSrc2, seed, u5, u6);
    Acc<PT>::set_vel(p, d, rr * cos(ph), rr * sin(ph), flux_vz(u5, vth2));
  }
}

// Sphere surface source: uniform points on the sphere, Maxwellian velocity
// with the inward normal component reflected.
template <class PT>
__global__ void k_sphere(PT p, long long dst, long long n,
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
  Acc<PT>::set_pos(p, d, g, wrap_coord(cx + radius * nx, g.lx),
                   wrap_coord(cy + radius * ny, g.ly), cz + radius * nz);
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
  Acc<PT>::set_vel(p, d, vx, vy, vz);
}

// Fowler-Nordheim counts per surface node inside the emitting disk:
// J = (a/phi) F^2 exp(-b phi^1.5/F) with F = -E_z(z = 0); the expected
// number J dx^2 dt / e is rounded stochastically.
template <typename TE>
__global__ void k_fn_count(const TE* __restrict__ Ez, unsigned* __restrict__ cnt,
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
    const double F = -(double)Ez[t];
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

// Exclusive scan of n values in one workgroup of 1024 threads; writes
// out[0..n] with out[n] = total.  Wave w takes the values [w * span,
// (w + 1) * span), span a multiple of 64: a first pass sums them, the
// waves' totals give each wave its offset, and a second pass scans them
// 64 at a time (shuffles) with a running carry.  Every access is
// coalesced, and the loads of each pass go out kScanB at a time (clamped
// to a valid index), not as a chain.
constexpr int kScanB = 16;
__device__ __forceinline__ unsigned wave_incl_scan(unsigned v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const unsigned u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

__global__ void __launch_bounds__(1024) k_scan1(const unsigned* __restrict__ in,
                                                unsigned* __restrict__ out,
                                                long long n) {
  __shared__ unsigned wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const long long span = ((n + 15) / 16 + 63) / 64 * 64;
  const long long w0 = w * span < n ? w * span : n;
  const long long w1 = w0 + span < n ? w0 + span : n;
  unsigned tot = 0;
  for (long long q0 = w0; q0 < w1; q0 += 64 * kScanB) {
    unsigned v[kScanB];
#pragma unroll
    for (int k = 0; k < kScanB; ++k) {
      const long long q = q0 + 64 * k + lane;
      v[k] = in[q < w1 ? q : w1 - 1];
    }
#pragma unroll
    for (int k = 0; k < kScanB; ++k)
      tot += q0 + 64 * k + lane < w1 ? v[k] : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  if (lane == 0) wsum[w] = tot;
  __syncthreads();
  unsigned carry = 0, all = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    carry += k < w ? wsum[k] : 0u;
    all += wsum[k];
  }
  for (long long q0 = w0; q0 < w1; q0 += 64 * kScanB) {
    unsigned v[kScanB];
#pragma unroll
    for (int k = 0; k < kScanB; ++k) {
      const long long q = q0 + 64 * k + lane;
      v[k] = in[q < w1 ? q : w1 - 1];
    }
#pragma unroll
    for (int k = 0; k < kScanB; ++k) {
      if (q0 + 64 * k >= w1) break;  // (wave-uniform)
      const long long q = q0 + 64 * k + lane;
      const unsigned x = q < w1 ? v[k] : 0u;
      const unsigned incl = wave_incl_scan(x, lane);
      if (q < w1) out[q] = carry + incl - x;
      carry += __shfl(incl, 63, 64);
    }
  }
  if (tid == 0) out[n] = all;
}

template <class PT>
__global__ void k_fn_spawn(PT p, long long dst, long long cap,
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
  Acc<PT>::set_pos(p, d, g, wrap_coord((double)i * g.dx + (u1 - 0.5) * g.dx, g.lx),
                   wrap_coord((double)j * g.dx + (u2 - 0.5) * g.dx, g.ly), 0.0);
  uniform2(id, step, kTagSrc1, seed, u3, u4);
  Acc<PT>::set_vel(p, d, 0.0, 0.0, flux_vz(u3, vth2));
  p.id[d] = id;
}

__global__ void k_fn_commit(Counters* dc, long long cap) {
  unsigned long long t = dc->fn_total;
  if ((long long)t > cap) t = (unsigned long long)cap;
  dc->n[0] += t;
  dc->next_id += t;
}

// ---- deposition ---------------------------------------------------------------
// One workgroup per chunk of an 8x8x8-cell tile: the chunk's electrons and
// ions (binned order) add their quantised CIC weights into a 9x9x9 int64
// LDS block with 64-bit LDS atomics; the block is then added to the node
// array with one global atomic per non-zero node.  Particles outside the tile (never, when
// the binning invariant holds) fall back to global atomics.
template <class PT>
__global__ void __launch_bounds__(kT) k_deposit(
    PT pe, PT pi, const uint32_t* __restrict__ tse,
    const uint32_t* __restrict__ tsi, const uint2* __restrict__ chunks,
    const unsigned* __restrict__ nchunks, long long* __restrict__ acc,
    GridC g) {
  __shared__ unsigned long long s[9 * 9 * 9];
  const unsigned nchk = *nchunks;
  if (blockIdx.x >= nchk) return;
  const unsigned cb = xcd_block(blockIdx.x, nchk);
  const unsigned t = chunks[cb].x, kp = chunks[cb].y;
  const int tx = (int)(t % g.tnx);
  const int ty = (int)((t / g.tnx) % g.tny);
  const int tz = (int)(t / ((unsigned)g.tnx * g.tny));
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  for (int q = threadIdx.x; q < 729; q += blockDim.x) s[q] = 0ull;
  __syncthreads();
  for (int sp = 0; sp < 2; ++sp) {
    const PT& p = sp ? pi : pe;
    const uint32_t* ts = sp ? tsi : tse;
    const long long sign = sp ? 1 : -1;
    unsigned b, e;
    piece(ts, t, kp, b, e);
    for (unsigned q = b + threadIdx.x; q < e; q += blockDim.x) {
      int ix, fx, iy, fy, iz, fz;
      Acc<PT>::cic(p, q, g, ix, fx, iy, fy, iz, fz);
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

// Charge of the state a step leaves, taken in its push: a pushed charged
// particle adds its quantised CIC weights at the new position, as the
// deposit pass would from the stored position, into an 11^3 LDS block of
// the nodes around its tile (x0 - 1 .. x0 + 9 per axis), flushed with one
// global atomic per non-zero node; a particle outside that block, and the
// unbinned ones, add with global atomics.  The sums are integers, so their
// order does not matter.
constexpr int kDepW = kTile + 3;
constexpr int kDepN = kDepW * kDepW * kDepW;

__device__ __forceinline__ void dep_global(long long* __restrict__ acc,
                                           const GridC& g, int ix, int fx,
                                           int iy, int fy, int iz, int fz,
                                           long long sign) {
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  for (int c = 0; c < 2; ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a) {
        const long long node =
            ((long long)(iz + c) * g.ny + wrap_index(iy + bb, g.ny)) * g.nx +
            wrap_index(ix + a, g.nx);
        atomicAdd(reinterpret_cast<unsigned long long*>(&acc[node]),
                  (unsigned long long)(sign * (wx[a] * wy[bb] * wz[c])));
      }
}

__device__ __forceinline__ void dep_tile(unsigned long long* sq,
                                         long long* __restrict__ acc,
                                         const GridC& g, int x0, int y0,
                                         int z0, int ix, int fx, int iy,
                                         int fy, int iz, int fz,
                                         long long sign) {
  const int lx = ix - x0 + 1, ly = iy - y0 + 1, lz = iz - z0 + 1;
  if (lx < 0 || lx > kDepW - 2 || ly < 0 || ly > kDepW - 2 || lz < 0 ||
      lz > kDepW - 2) {
    dep_global(acc, g, ix, fx, iy, fy, iz, fz, sign);
    return;
  }
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  for (int c = 0; c < 2; ++c)
    for (int bb = 0; bb < 2; ++bb)
      for (int a = 0; a < 2; ++a)
        atomicAdd(&sq[((lz + c) * kDepW + (ly + bb)) * kDepW + (lx + a)],
                  (unsigned long long)(sign * (wx[a] * wy[bb] * wz[c])));
}

__device__ __forceinline__ void dep_flush(const unsigned long long* sq,
                                          long long* __restrict__ acc,
                                          const GridC& g, int x0, int y0,
                                          int z0) {
  for (int q = threadIdx.x; q < kDepN; q += blockDim.x) {
    const unsigned long long v = sq[q];
    if (!v) continue;
    const int a = q % kDepW, bb = (q / kDepW) % kDepW, c = q / (kDepW * kDepW);
    const int gk = z0 - 1 + c;
    if (gk < 0 || gk > g.nz) continue;   // (receives no charge)
    const int gi = wrap_index(x0 - 1 + a, g.nx), gj = wrap_index(y0 - 1 + bb, g.ny);
    atomicAdd(reinterpret_cast<unsigned long long*>(
                  &acc[((long long)gk * g.ny + gj) * g.nx + gi]),
              v);
  }
}

// Deposit of the particles after the tile ranges, with global atomics.
template <class PT>
__global__ void __launch_bounds__(kT) k_deposit_tail(
    PT p, long long first, const unsigned long long* __restrict__ np,
    long long* __restrict__ acc, GridC g, long long sign) {
  const long long i = first + blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= (long long)*np) return;
  int ix, fx, iy, fy, iz, fz;
  Acc<PT>::cic(p, i, g, ix, fx, iy, fy, iz, fz);
  dep_global(acc, g, ix, fx, iy, fy, iz, fz, sign);
}

// ---- push ---------------------------------------------------------------------
struct MccC {
  int enabled, ion_model;
  double c_coll;          // g_max dt w_sp / dx^3
  double inv_gmax, sigma_el, lotz_a, ion_I, sigma_const, E_max;
  double half_me, ratio;  // 0.5 m_e; 2 m_e / M
  double two_e_me;        // 2 e / m_e
  // Electron-absorbing nanoparticle (sph_on = 0: none).
  int sph_on;
  double sph_cx, sph_cy, sph_cz, sph_r2, sph_alpha, dt;
};

// Does the straight path (x0, y0, z0) + v t, 0 <= t <= dt, touch the closed
// ball of the nanoparticle (x, y: nearest periodic image of its centre)?
// With d = x0 - c and s = v dt the path is d + tau s, tau in [0, 1]: it
// touches the ball if it starts inside, or moves towards the centre with
// the smaller root of |d + tau s|^2 = R^2 at most 1.
__device__ __forceinline__ bool sphere_hit(const MccC& m, const GridC& g,
                                           double x0, double y0, double z0,
                                           double vx, double vy, double vz) {
  double dxx = x0 - m.sph_cx, dyy = y0 - m.sph_cy;
  const double hx = 0.5 * g.lx, hy = 0.5 * g.ly;
  if (dxx > hx) dxx = dxx - g.lx; else if (dxx < -hx) dxx = dxx + g.lx;
  if (dyy > hy) dyy = dyy - g.ly; else if (dyy < -hy) dyy = dyy + g.ly;
  const double dzz = z0 - m.sph_cz;
  const double sx = vx * m.dt, sy = vy * m.dt, sz = vz * m.dt;
  const double c0 = ((dxx * dxx + dyy * dyy) + dzz * dzz) - m.sph_r2;
  if (c0 <= 0.0) return true;
  const double b = (dxx * sx + dyy * sy) + dzz * sz;
  const double a = (sx * sx + sy * sy) + sz * sz;
  const double disc = b * b - a * c0;
  if (!(b < 0.0) || !(disc >= 0.0) || !(a > 0.0)) return false;
  return (-b - sqrt(disc)) / a <= 1.0;
}

// An electron absorbed by the nanoparticle: counted, and alpha_EH times its
// kinetic energy (|v|^2 = ke) added to the particle's heat.
__device__ __forceinline__ void np_absorb(const MccC& m, double ke,
                                          Counters* dc) {
  atomicAdd(&dc->np_hits, 1ull);
  atomicAdd(&dc->np_heat, m.sph_alpha * (m.half_me * ke));
}

// Field at a particle from the node arrays (Ex, Ey, Ez blocks of nn nodes),
// with the deposit's quantised weights, accumulated in the fixed order
// z-corner, y-corner, x-corner.
__device__ __forceinline__ void gather_global(const double* __restrict__ E,
                                              long long nn, const GridC& g,
                                              double x, double y, double z,
                                              double& ex, double& ey,
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
        const long long node = row + wrap_index(ix + a, g.nx);
        ex = ex + w * E[node];
        ey = ey + w * E[nn + node];
        ez = ez + w * E[2 * nn + node];
      }
    }
  }
}

// The same from a tile's 9x9x9 nodes staged in LDS; (lx, ly, lz) is the
// particle's cell inside the tile.
__device__ __forceinline__ void gather_lds(const double* sx, const double* sy,
                                           const double* sz, int lx, int ly,
                                           int lz, int fx, int fy, int fz,
                                           double& ex, double& ey, double& ez) {
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  ex = 0.0; ey = 0.0; ez = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int row = ((lz + c) * 9 + (ly + b)) * 9 + lx;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double w = (double)(wx[a] * wy[b] * wz[c]) * kQScale;
        ex = ex + w * sx[row + a];
        ey = ey + w * sy[row + a];
        ez = ez + w * sz[row + a];
      }
    }
  }
}

// Result of one particle's push.
struct PushOut {
  bool cathode, anode, cand;
  unsigned cell;
  double ke;           // |v|^2 after the kick
  double x, y, z, vx, vy, vz;
  float oxf, oyf, ozf; // mixed layout: the stored in-cell offsets
  unsigned long long id;  // electron candidates: the id of the draw
};

// CIC cell and quantised weights of a pushed particle's stored position
// (FP64: wrapped coordinates; mixed: cell and FP32 offsets), as the
// deposit computes them from memory.
__device__ __forceinline__ void cic_stored(const Parts&, const PushOut& o,
                                           const GridC& g, int& ix, int& fx,
                                           int& iy, int& fy, int& iz, int& fz) {
  cic_axis(o.x, g.inv_dx, ix, fx);
  cic_axis(o.y, g.inv_dx, iy, fy);
  cic_axis(o.z, g.inv_dx, iz, fz);
  if (ix >= g.nx) ix -= g.nx;
  if (iy >= g.ny) iy -= g.ny;
}

__device__ __forceinline__ void cic_stored(const PartsM&, const PushOut& o,
                                           const GridC& g, int& ix, int& fx,
                                           int& iy, int& fy, int& iz, int& fz) {
  Acc<PartsM>::decode(o.cell, g, ix, iy, iz);
  fx = (int)floorf(o.oxf * 8192.0f + 0.5f);
  fy = (int)floorf(o.oyf * 8192.0f + 0.5f);
  fz = (int)floorf(o.ozf * 8192.0f + 0.5f);
}

// Drift, boundaries, write-back and (electrons) the null-collision
// candidate draw U1 < 1 - exp(-N_c c_coll); velocities already kicked.
template <int SP>
__device__ __forceinline__ void finish_push(Parts& p, long long i, double x,
                                            double y, double z, double vx,
                                            double vy, double vz, double dt,
                                            const GridC& g, uint32_t* key,
                                            int* ncount, const MccC& m,
                                            uint32_t step, uint64_t seed,
                                            Counters* dc, PushOut& o,
                                            uint64_t idv) {
  const bool np = SP == 0 && m.sph_on && sphere_hit(m, g, x, y, z, vx, vy, vz);
  x = x + vx * dt;
  y = y + vy * dt;
  z = z + vz * dt;
  o.ke = (vx * vx + vy * vy) + vz * vz;
  o.cathode = false;
  o.anode = false;
  o.cand = false;
  o.cell = kDead;
  const double gz = z * g.inv_dx;
  const double xw = wrap_coord(x, g.lx), yw = wrap_coord(y, g.ly);
  if (!(xw >= 0.0 && xw < g.lx && yw >= 0.0 && yw < g.ly) || !(gz == gz) ||
      !isfinite(vx) || !isfinite(vy) || !isfinite(vz)) {
    // Non-finite, or moved more than one period in a step: removed and
    // reported.
    atomicOr(&dc->err, kErrNonFinite);
  } else if (np) {
    // Absorbed by the nanoparticle (which lies inside the domain, so a
    // path that leaves through a face cannot reach it afterwards).
    np_absorb(m, o.ke, dc);
  } else if (gz < 0.0) {
    o.cathode = true;
  } else if (gz >= (double)g.nz) {
    o.anode = true;
  } else {
    x = xw;
    y = yw;
    o.cell = cell_of(x, y, z, g);
    p.x[i] = x; p.y[i] = y; p.z[i] = z;
    // A neutral's velocity does not change; its cell count is added by the
    // caller (aggregated in LDS).
    if (SP != 1) {
      p.vx[i] = vx; p.vy[i] = vy; p.vz[i] = vz;
    }
  }
  key[i] = o.cell;
  if (SP == 0 && o.cell != kDead && m.enabled) {
    const int nc = ncount[o.cell];
    if (nc > 0) {
      const double pstar = 1.0 - exp(-((double)nc * m.c_coll));
      double u1, u2;
      uniform2(idv, step, kTagMcc0, seed, u1, u2);
      if (fabs(u1 - pstar) < 1e-6) atomicAdd(&dc->n_near, 1ull);
      o.cand = u1 < pstar;
      o.id = idv;
    }
  }
  o.x = x; o.y = y; o.z = z; o.vx = vx; o.vy = vy; o.vz = vz;
}

__device__ __forceinline__ CandRec cand_rec(const PushOut& o, long long i) {
  CandRec r;
  r.vx = o.vx; r.vy = o.vy; r.vz = o.vz;
  r.id = o.id;
  r.i = (unsigned)i;
  r.pad = 0u;
  return r;
}

// Index of a removed particle into the step's list of its species
// (wave-aggregated slot; entries past kDeadList are counted, not stored).
// All lanes must call it.
__device__ __forceinline__ void list_dead(bool dead, long long i,
                                          uint32_t* __restrict__ list,
                                          unsigned long long* count) {
  const unsigned long long slot = wave_append(dead, count);
  if (dead && slot < (unsigned long long)kDeadList) list[slot] = (uint32_t)i;
}

// Cathode sink record (wave-aggregated slot).  All lanes must call it.
template <int SP>
__device__ __forceinline__ void sink(const Parts& p, long long i,
                                     const PushOut& o, const GridC& g,
                                     Rec* ab_rec, double* ab_pos,
                                     double* ab_vel, long long ab_cap,
                                     Counters* dc) {
  wave_count(o.anode, &dc->anode[SP]);
  wave_count(o.cathode, &dc->cathode[SP]);
  const unsigned long long slot = wave_append(o.cathode, &dc->n_ab);
  if (!o.cathode) return;
  if ((long long)slot < ab_cap) {
    const double tc = -o.z / o.vz;
    const double xc = wrap_coord(o.x + o.vx * tc, g.lx);
    const double yc = wrap_coord(o.y + o.vy * tc, g.ly);
    Rec r;
    r.hi = SP; r.lo = p.id[i]; r.val = (unsigned)slot;
    ab_rec[slot] = r;
    ab_pos[3 * slot] = xc; ab_pos[3 * slot + 1] = yc; ab_pos[3 * slot + 2] = 0.0;
    ab_vel[3 * slot] = o.vx; ab_vel[3 * slot + 1] = o.vy;
    ab_vel[3 * slot + 2] = o.vz;
  } else {
    atomicOr(&dc->err, kErrEvents);
  }
}

__device__ __forceinline__ double block_sum(double v, double* sk) {
  sk[threadIdx.x] = v;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sk[threadIdx.x] = sk[threadIdx.x] + sk[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sk[0];
  __syncthreads();
  return r;
}

// Charged species, one workgroup per 8x8x8-cell tile: the tile's 9x9x9 E
// nodes are staged in LDS once and serve both the ions and the electrons
// binned in the tile.  Electron candidates are written to the tile's own
// segment of the candidate list (no global counter).
struct TileArgs {
  Parts pe, pi;
  const uint32_t *tse, *tsi;
  const uint2* chunks;
  const unsigned* nchunks;
  uint32_t *keye, *keyi;
  double qm_e, qm_i, dt;
  int* ncount;
  CandRec* cand;
  uint32_t* cand_cnt;
  Rec* ab_rec;
  double *ab_pos, *ab_vel;
  long long ab_cap;
  double *part_e, *part_i;
  unsigned *cnt_e, *cnt_i;   // destination-tile counts for the binning
  long long* dep;            // charge of the pushed state (int64 units)
  uint32_t* dead2;           // removed ions' indices
};

__global__ void __launch_bounds__(kT) k_push_tile(
    TileArgs A, const double* __restrict__ E, long long nn, GridC g, MccC m,
    uint32_t step, uint64_t seed, Counters* dc) {
  __shared__ double sx[729], sy[729], sz[729];
  __shared__ unsigned long long sq[kDepN];
  __shared__ double sk[kT];
  __shared__ unsigned s_cand;
  __shared__ unsigned s_nc[2][27], s_nd[2][27];  // destinations: e, ions
  const unsigned nchk = *A.nchunks;
  if (blockIdx.x >= nchk) return;
  const unsigned cb = xcd_block(blockIdx.x, nchk);
  const unsigned t = A.chunks[cb].x, kp = A.chunks[cb].y;
  unsigned be, ee, bi, ei;
  piece(A.tse, t, kp, be, ee);
  piece(A.tsi, t, kp, bi, ei);
  if (be == ee && bi == ei) {
    if (threadIdx.x == 0) {
      A.part_e[cb] = 0.0;
      A.part_i[cb] = 0.0;
      A.cand_cnt[cb] = 0;
    }
    return;
  }
  const int tx = (int)(t % g.tnx);
  const int ty = (int)((t / g.tnx) % g.tny);
  const int tz = (int)(t / ((unsigned)g.tnx * g.tny));
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  for (int q = threadIdx.x; q < 729; q += blockDim.x) {
    const int a = q % 9, b = (q / 9) % 9, c = q / 81;
    const int gk = z0 + c;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    if (gk <= g.nz) {
      const long long node = ((long long)gk * g.ny + wrap_index(y0 + b, g.ny)) *
                                 g.nx + wrap_index(x0 + a, g.nx);
      vx = E[node]; vy = E[nn + node]; vz = E[2 * nn + node];
    }
    sx[q] = vx; sy[q] = vy; sz[q] = vz;
  }
  for (int q = threadIdx.x; q < kDepN; q += blockDim.x) sq[q] = 0ull;
  if (threadIdx.x == 0) s_cand = 0;
  if (threadIdx.x < 54) (&s_nc[0][0])[threadIdx.x] = 0u;
  __syncthreads();
  double ke_i = 0.0, ke_e = 0.0;
  // Ions.
  for (unsigned base = bi; base < ei; base += blockDim.x) {
    const long long i = base + threadIdx.x;
    const bool live = i < ei;
    PushOut o;
    o.cathode = false;
    o.anode = false;
    bool moved = false;
    if (live) {
      const double x = A.pi.x[i], y = A.pi.y[i], z = A.pi.z[i];
      int ix, fx, iy, fy, iz, fz;
      cic_axis(x, g.inv_dx, ix, fx);
      cic_axis(y, g.inv_dx, iy, fy);
      cic_axis(z, g.inv_dx, iz, fz);
      if (ix >= g.nx) ix -= g.nx;
      if (iy >= g.ny) iy -= g.ny;
      const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
      double ex, ey, ez;
      if (lx >= 0 && lx < kTile && ly >= 0 && ly < kTile && lz >= 0 && lz < kTile)
        gather_lds(sx, sy, sz, lx, ly, lz, fx, fy, fz, ex, ey, ez);
      else
        gather_global(E, nn, g, x, y, z, ex, ey, ez);
      const double vx = A.pi.vx[i] + A.qm_i * ex;
      const double vy = A.pi.vy[i] + A.qm_i * ey;
      const double vz = A.pi.vz[i] + A.qm_i * ez;
      finish_push<2>(A.pi, i, x, y, z, vx, vy, vz, A.dt, g, A.keyi, A.ncount, m,
                     step, seed, dc, o, 0ull);
      ke_i = ke_i + o.ke;
      moved = count_dest(o.cell, tx, ty, tz, g, s_nc[1], s_nd[1], A.cnt_i) != kSlotSelf &&
              o.cell != kDead;
      if (o.cell != kDead) {
        int dx_, fx_, dy_, fy_, dz_, fz_;
        cic_stored(Parts(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
        dep_tile(sq, A.dep, g, x0, y0, z0, dx_, fx_, dy_, fy_, dz_, fz_, 1);
      }
    }
    sink<2>(A.pi, i, o, g, A.ab_rec, A.ab_pos, A.ab_vel, A.ab_cap, dc);
    wave_count(moved, &dc->ion_moved);
    list_dead(live && o.cell == kDead, i, A.dead2, &dc->n_dead2);
  }
  // Electrons.
  for (unsigned base = be; base < ee; base += blockDim.x) {
    const long long i = base + threadIdx.x;
    const bool live = i < ee;
    PushOut o;
    o.cathode = false;
    o.anode = false;
    o.cand = false;
    if (live) {
      const double x = A.pe.x[i], y = A.pe.y[i], z = A.pe.z[i];
      int ix, fx, iy, fy, iz, fz;
      cic_axis(x, g.inv_dx, ix, fx);
      cic_axis(y, g.inv_dx, iy, fy);
      cic_axis(z, g.inv_dx, iz, fz);
      if (ix >= g.nx) ix -= g.nx;
      if (iy >= g.ny) iy -= g.ny;
      const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
      double ex, ey, ez;
      if (lx >= 0 && lx < kTile && ly >= 0 && ly < kTile && lz >= 0 && lz < kTile)
        gather_lds(sx, sy, sz, lx, ly, lz, fx, fy, fz, ex, ey, ez);
      else
        gather_global(E, nn, g, x, y, z, ex, ey, ez);
      const double vx = A.pe.vx[i] + A.qm_e * ex;
      const double vy = A.pe.vy[i] + A.qm_e * ey;
      const double vz = A.pe.vz[i] + A.qm_e * ez;
      finish_push<0>(A.pe, i, x, y, z, vx, vy, vz, A.dt, g, A.keye, A.ncount, m,
                     step, seed, dc, o, A.pe.id[i]);
      ke_e = ke_e + o.ke;
      count_dest(o.cell, tx, ty, tz, g, s_nc[0], s_nd[0], A.cnt_e);
      if (o.cell != kDead) {
        int dx_, fx_, dy_, fy_, dz_, fz_;
        cic_stored(Parts(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
        dep_tile(sq, A.dep, g, x0, y0, z0, dx_, fx_, dy_, fy_, dz_, fz_, -1);
      }
      if (o.cand) A.cand[be + atomicAdd(&s_cand, 1u)] = cand_rec(o, i);
    }
    sink<0>(A.pe, i, o, g, A.ab_rec, A.ab_pos, A.ab_vel, A.ab_cap, dc);
  }
  const double si = block_sum(ke_i, sk);
  const double se = block_sum(ke_e, sk);
  if (threadIdx.x == 0) {
    A.part_i[cb] = si;
    A.part_e[cb] = se;
    A.cand_cnt[cb] = s_cand;
  }
  // The destination counts are complete (block_sum synchronised).
  if (threadIdx.x < 54) {
    const int sp = threadIdx.x / 27, d = threadIdx.x % 27;
    const unsigned n = s_nc[sp][d];
    if (n) atomicAdd(&(sp ? A.cnt_i : A.cnt_e)[s_nd[sp][d]], n);
  }
  dep_flush(sq, A.dep, g, x0, y0, z0);
}

// Particles not covered by tile ranges (sources and queue appended this
// step; all neutrals): one thread per particle, field from global memory.
template <int SP>
__global__ void __launch_bounds__(kT) k_push_list(
    Parts p, long long first, uint32_t* __restrict__ key,
    const double* __restrict__ E, long long nn, GridC g, double qm_dt,
    double dt, int* __restrict__ ncount, CandRec* __restrict__ cand, MccC m,
    uint32_t step, uint64_t seed, Rec* __restrict__ ab_rec,
    double* __restrict__ ab_pos, double* __restrict__ ab_vel, long long ab_cap,
    Counters* dc, double* __restrict__ part, long long* __restrict__ dep,
    uint32_t* __restrict__ dead2) {
  __shared__ double sk[kT];
  const long long n = (long long)dc->n[SP];
  const long long i = first + blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const bool live = i < n;
  PushOut o;
  o.cathode = false;
  o.anode = false;
  o.cand = false;
  o.ke = 0.0;
  if (live) {
    const double x = p.x[i], y = p.y[i], z = p.z[i];
    double vx = p.vx[i], vy = p.vy[i], vz = p.vz[i];
    if (SP != 1) {
      double ex, ey, ez;
      gather_global(E, nn, g, x, y, z, ex, ey, ez);
      vx = vx + qm_dt * ex;
      vy = vy + qm_dt * ey;
      vz = vz + qm_dt * ez;
    }
    finish_push<SP>(p, i, x, y, z, vx, vy, vz, dt, g, key, ncount, m, step,
                    seed, dc, o, SP == 0 ? p.id[i] : 0ull);
    if (SP != 1 && o.cell != kDead) {
      int dx_, fx_, dy_, fy_, dz_, fz_;
      cic_stored(Parts(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
      dep_global(dep, g, dx_, fx_, dy_, fy_, dz_, fz_,
                 SP == 0 ? -1 : (SP == 3 ? 2 : 1));
    }
  }
  sink<SP>(p, i, o, g, ab_rec, ab_pos, ab_vel, ab_cap, dc);
  if (SP == 2) list_dead(live && o.cell == kDead, i, dead2, &dc->n_dead2);
  if (SP == 0) {
    const unsigned long long cs = wave_append(o.cand, &dc->n_tail_cand);
    if (o.cand) cand[first + cs] = cand_rec(o, i);
  }
  const double s = block_sum(live ? o.ke : 0.0, sk);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---- mixed-precision push ---------------------------------------------------------
// Particles as cell index + FP32 offsets in [0, 1) + FP32 velocities; the
// field is gathered from FP32 node arrays and the kick and drift run in
// FP32 (the FP32 offset keeps slow neutrals moving, which an FP32 absolute
// coordinate would freeze).  Cell keys, charge and energies stay exact or
// FP64.
struct PushM {
  float ox, oy, oz, vx, vy, vz;
  int ix, iy, iz;        // cell after the drift (x, y wrapped)
};

// Drift in cell units and carry into the cell index; returns the cell key
// or kDead, and fills the FP64 PushOut (absolute position before the x, y
// wrap for the cathode crossing point).
template <int SP>
__device__ __forceinline__ void finish_push_m(PartsM& p, long long i, PushM q,
                                              float dtdx, const GridC& g,
                                              uint32_t* key, int* ncount,
                                              const MccC& m, uint32_t step,
                                              uint64_t seed, Counters* dc,
                                              PushOut& o) {
  bool np = false;
  if (SP == 0 && m.sph_on)
    np = sphere_hit(m, g, ((double)q.ix + (double)q.ox) * g.dx,
                    ((double)q.iy + (double)q.oy) * g.dx,
                    ((double)q.iz + (double)q.oz) * g.dx, (double)q.vx,
                    (double)q.vy, (double)q.vz);
  q.ox = q.ox + q.vx * dtdx;
  q.oy = q.oy + q.vy * dtdx;
  q.oz = q.oz + q.vz * dtdx;
  const float cx = floorf(q.ox), cy = floorf(q.oy), cz = floorf(q.oz);
  q.ox = q.ox - cx; q.oy = q.oy - cy; q.oz = q.oz - cz;
  int ix = q.ix + (int)cx, iy = q.iy + (int)cy, iz = q.iz + (int)cz;
  if (q.ox >= 1.0f) { q.ox = 0.0f; ix += 1; }
  if (q.oy >= 1.0f) { q.oy = 0.0f; iy += 1; }
  if (q.oz >= 1.0f) { q.oz = 0.0f; iz += 1; }
  o.vx = (double)q.vx; o.vy = (double)q.vy; o.vz = (double)q.vz;
  o.x = ((double)ix + (double)q.ox) * g.dx;
  o.y = ((double)iy + (double)q.oy) * g.dx;
  o.z = ((double)iz + (double)q.oz) * g.dx;
  o.ke = (o.vx * o.vx + o.vy * o.vy) + o.vz * o.vz;
  o.cathode = false;
  o.anode = false;
  o.cand = false;
  o.cell = kDead;
  const int jx = ix >= g.nx ? ix - g.nx : (ix < 0 ? ix + g.nx : ix);
  const int jy = iy >= g.ny ? iy - g.ny : (iy < 0 ? iy + g.ny : iy);
  if (jx < 0 || jx >= g.nx || jy < 0 || jy >= g.ny || !(q.ox == q.ox) ||
      !(q.oy == q.oy) || !(q.oz == q.oz) || !isfinite(q.vx) ||
      !isfinite(q.vy) || !isfinite(q.vz)) {
    atomicOr(&dc->err, kErrNonFinite);
  } else if (np) {
    np_absorb(m, o.ke, dc);
  } else if (iz < 0) {
    o.cathode = true;
  } else if (iz >= g.nz) {
    o.anode = true;
  } else {
    o.cell = ((unsigned)iz * (unsigned)g.ny + (unsigned)jy) * (unsigned)g.nx +
             (unsigned)jx;
    p.cell[i] = o.cell;
    p.ox[i] = q.ox; p.oy[i] = q.oy; p.oz[i] = q.oz;
    o.oxf = q.ox; o.oyf = q.oy; o.ozf = q.oz;
    if (SP != 1) {
      p.vx[i] = q.vx; p.vy[i] = q.vy; p.vz[i] = q.vz;
    }
  }
  key[i] = o.cell;
  if (SP == 0 && o.cell != kDead && m.enabled) {
    const int nc = ncount[o.cell];
    if (nc > 0) {
      const double pstar = 1.0 - exp(-((double)nc * m.c_coll));
      double u1, u2;
      const unsigned long long idv = p.id[i];
      uniform2(idv, step, kTagMcc0, seed, u1, u2);
      o.id = idv;
      if (fabs(u1 - pstar) < 1e-6) atomicAdd(&dc->n_near, 1ull);
      o.cand = u1 < pstar;
    }
  }
}

// FP32 CIC gather with the quantised weights; E nodes from LDS (tile) or
// from the global FP32 arrays.
__device__ __forceinline__ void gather_m(const float* sx, const float* sy,
                                         const float* sz, int lrow, int rs,
                                         int ps, int fx, int fy, int fz,
                                         float& ex, float& ey, float& ez) {
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  ex = 0.0f; ey = 0.0f; ez = 0.0f;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float w = (float)(wx[a] * wy[b] * wz[c]) * 0x1p-39f;
        const int q = lrow + c * ps + b * rs + a;
        ex = ex + w * sx[q];
        ey = ey + w * sy[q];
        ez = ez + w * sz[q];
      }
}

__device__ __forceinline__ void gather_m_global(const float* __restrict__ E,
                                                long long nn, const GridC& g,
                                                int ix, int iy, int iz, int fx,
                                                int fy, int fz, float& ex,
                                                float& ey, float& ez) {
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  ex = 0.0f; ey = 0.0f; ez = 0.0f;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const long long row =
          ((long long)(iz + c) * g.ny + wrap_index(iy + b, g.ny)) * g.nx;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const float w = (float)(wx[a] * wy[b] * wz[c]) * 0x1p-39f;
        const long long node = row + wrap_index(ix + a, g.nx);
        ex = ex + w * E[node];
        ey = ey + w * E[nn + node];
        ez = ez + w * E[2 * nn + node];
      }
    }
}

struct TileArgsM {
  PartsM pe, pi;
  const uint32_t *tse, *tsi;
  const uint2* chunks;
  const unsigned* nchunks;
  uint32_t *keye, *keyi;
  float qm_e, qm_i, dtdx;
  int* ncount;
  CandRec* cand;
  uint32_t* cand_cnt;
  Rec* ab_rec;
  double *ab_pos, *ab_vel;
  long long ab_cap;
  double *part_e, *part_i;
  unsigned *cnt_e, *cnt_i;   // destination-tile counts for the binning
  long long* dep;            // charge of the pushed state (int64 units)
  uint32_t* dead2;           // removed ions' indices
};

template <int SP>
__device__ __forceinline__ void push_one_m(PartsM& p, long long i,
                                           const float* sx, const float* sy,
                                           const float* sz, int x0, int y0,
                                           int z0, const float* __restrict__ E,
                                           long long nn, const GridC& g,
                                           float qm, float dtdx, uint32_t* key,
                                           int* ncount, const MccC& m,
                                           uint32_t step, uint64_t seed,
                                           Counters* dc, PushOut& o) {
  PushM q;
  Acc<PartsM>::decode(p.cell[i], g, q.ix, q.iy, q.iz);
  q.ox = p.ox[i]; q.oy = p.oy[i]; q.oz = p.oz[i];
  q.vx = p.vx[i]; q.vy = p.vy[i]; q.vz = p.vz[i];
  if (SP != 1) {
    const int fx = (int)floorf(q.ox * 8192.0f + 0.5f);
    const int fy = (int)floorf(q.oy * 8192.0f + 0.5f);
    const int fz = (int)floorf(q.oz * 8192.0f + 0.5f);
    const int lx = q.ix - x0, ly = q.iy - y0, lz = q.iz - z0;
    float ex, ey, ez;
    if (sx && lx >= 0 && lx < kTile && ly >= 0 && ly < kTile && lz >= 0 &&
        lz < kTile)
      gather_m(sx, sy, sz, (lz * 9 + ly) * 9 + lx, 9, 81, fx, fy, fz, ex, ey, ez);
    else
      gather_m_global(E, nn, g, q.ix, q.iy, q.iz, fx, fy, fz, ex, ey, ez);
    q.vx = q.vx + qm * ex;
    q.vy = q.vy + qm * ey;
    q.vz = q.vz + qm * ez;
  }
  finish_push_m<SP>(p, i, q, dtdx, g, key, ncount, m, step, seed, dc, o);
}

// Sink record from an FP64 PushOut, shared with the FP64 layout.
__device__ __forceinline__ void sink_m(const PartsM& p, long long i, int sp,
                                       const PushOut& o, const GridC& g,
                                       Rec* ab_rec, double* ab_pos,
                                       double* ab_vel, long long ab_cap,
                                       Counters* dc) {
  wave_count(o.anode, &dc->anode[sp]);
  wave_count(o.cathode, &dc->cathode[sp]);
  const unsigned long long slot = wave_append(o.cathode, &dc->n_ab);
  if (!o.cathode) return;
  if ((long long)slot < ab_cap) {
    const double tc = -o.z / o.vz;
    Rec r;
    r.hi = sp; r.lo = p.id[i]; r.val = (unsigned)slot;
    ab_rec[slot] = r;
    ab_pos[3 * slot] = wrap_coord(o.x + o.vx * tc, g.lx);
    ab_pos[3 * slot + 1] = wrap_coord(o.y + o.vy * tc, g.ly);
    ab_pos[3 * slot + 2] = 0.0;
    ab_vel[3 * slot] = o.vx; ab_vel[3 * slot + 1] = o.vy;
    ab_vel[3 * slot + 2] = o.vz;
  } else {
    atomicOr(&dc->err, kErrEvents);
  }
}

__global__ void __launch_bounds__(kT) k_push_tile_m(
    TileArgsM A, const float* __restrict__ E, long long nn, GridC g, MccC m,
    uint32_t step, uint64_t seed, Counters* dc) {
  __shared__ float sx[729], sy[729], sz[729];
  __shared__ unsigned long long sq[kDepN];
  __shared__ double sk[kT];
  __shared__ unsigned s_cand;
  __shared__ unsigned s_nc[2][27], s_nd[2][27];  // destinations: e, ions
  const unsigned nchk = *A.nchunks;
  if (blockIdx.x >= nchk) return;
  const unsigned cb = xcd_block(blockIdx.x, nchk);
  const unsigned t = A.chunks[cb].x, kp = A.chunks[cb].y;
  unsigned be, ee, bi, ei;
  piece(A.tse, t, kp, be, ee);
  piece(A.tsi, t, kp, bi, ei);
  if (be == ee && bi == ei) {
    if (threadIdx.x == 0) {
      A.part_e[cb] = 0.0;
      A.part_i[cb] = 0.0;
      A.cand_cnt[cb] = 0;
    }
    return;
  }
  const int tx = (int)(t % g.tnx);
  const int ty = (int)((t / g.tnx) % g.tny);
  const int tz = (int)(t / ((unsigned)g.tnx * g.tny));
  const int x0 = tx * kTile, y0 = ty * kTile, z0 = tz * kTile;
  for (int q = threadIdx.x; q < 729; q += blockDim.x) {
    const int a = q % 9, b = (q / 9) % 9, c = q / 81;
    const int gk = z0 + c;
    float vx = 0.0f, vy = 0.0f, vz = 0.0f;
    if (gk <= g.nz) {
      const long long node = ((long long)gk * g.ny + wrap_index(y0 + b, g.ny)) *
                                 g.nx + wrap_index(x0 + a, g.nx);
      vx = E[node]; vy = E[nn + node]; vz = E[2 * nn + node];
    }
    sx[q] = vx; sy[q] = vy; sz[q] = vz;
  }
  for (int q = threadIdx.x; q < kDepN; q += blockDim.x) sq[q] = 0ull;
  if (threadIdx.x == 0) s_cand = 0;
  if (threadIdx.x < 54) (&s_nc[0][0])[threadIdx.x] = 0u;
  __syncthreads();
  double ke_i = 0.0, ke_e = 0.0;
  for (unsigned base = bi; base < ei; base += blockDim.x) {
    const long long i = base + threadIdx.x;
    PushOut o;
    o.cathode = false;
    o.anode = false;
    bool moved = false;
    if (i < ei) {
      push_one_m<2>(A.pi, i, sx, sy, sz, x0, y0, z0, E, nn, g, A.qm_i, A.dtdx,
                    A.keyi, A.ncount, m, step, seed, dc, o);
      ke_i = ke_i + o.ke;
      moved = count_dest(o.cell, tx, ty, tz, g, s_nc[1], s_nd[1], A.cnt_i) != kSlotSelf &&
              o.cell != kDead;
      if (o.cell != kDead) {
        int dx_, fx_, dy_, fy_, dz_, fz_;
        cic_stored(PartsM(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
        dep_tile(sq, A.dep, g, x0, y0, z0, dx_, fx_, dy_, fy_, dz_, fz_, 1);
      }
    }
    sink_m(A.pi, i, 2, o, g, A.ab_rec, A.ab_pos, A.ab_vel, A.ab_cap, dc);
    wave_count(moved, &dc->ion_moved);
    list_dead(i < ei && o.cell == kDead, i, A.dead2, &dc->n_dead2);
  }
  for (unsigned base = be; base < ee; base += blockDim.x) {
    const long long i = base + threadIdx.x;
    PushOut o;
    o.cathode = false;
    o.anode = false;
    o.cand = false;
    if (i < ee) {
      push_one_m<0>(A.pe, i, sx, sy, sz, x0, y0, z0, E, nn, g, A.qm_e, A.dtdx,
                    A.keye, A.ncount, m, step, seed, dc, o);
      ke_e = ke_e + o.ke;
      count_dest(o.cell, tx, ty, tz, g, s_nc[0], s_nd[0], A.cnt_e);
      if (o.cell != kDead) {
        int dx_, fx_, dy_, fy_, dz_, fz_;
        cic_stored(PartsM(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
        dep_tile(sq, A.dep, g, x0, y0, z0, dx_, fx_, dy_, fy_, dz_, fz_, -1);
      }
      if (o.cand) A.cand[be + atomicAdd(&s_cand, 1u)] = cand_rec(o, i);
    }
    sink_m(A.pe, i, 0, o, g, A.ab_rec, A.ab_pos, A.ab_vel, A.ab_cap, dc);
  }
  const double si = block_sum(ke_i, sk);
  const double se = block_sum(ke_e, sk);
  if (threadIdx.x == 0) {
    A.part_i[cb] = si;
    A.part_e[cb] = se;
    A.cand_cnt[cb] = s_cand;
  }
  // The destination counts are complete (block_sum synchronised).
  if (threadIdx.x < 54) {
    const int sp = threadIdx.x / 27, d = threadIdx.x % 27;
    const unsigned n = s_nc[sp][d];
    if (n) atomicAdd(&(sp ? A.cnt_i : A.cnt_e)[s_nd[sp][d]], n);
  }
  dep_flush(sq, A.dep, g, x0, y0, z0);
}

template <int SP>
__global__ void __launch_bounds__(kT) k_push_list_m(
    PartsM p, long long first, uint32_t* __restrict__ key,
    const float* __restrict__ E, long long nn, GridC g, float qm, float dtdx,
    int* __restrict__ ncount, CandRec* __restrict__ cand, MccC m,
    uint32_t step, uint64_t seed, Rec* __restrict__ ab_rec,
    double* __restrict__ ab_pos, double* __restrict__ ab_vel, long long ab_cap,
    Counters* dc, double* __restrict__ part, long long* __restrict__ dep,
    uint32_t* __restrict__ dead2) {
  __shared__ double sk[kT];
  const long long n = (long long)dc->n[SP];
  const long long i = first + blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const bool live = i < n;
  PushOut o;
  o.cathode = false;
  o.anode = false;
  o.cand = false;
  o.ke = 0.0;
  if (live) {
    push_one_m<SP>(p, i, nullptr, nullptr, nullptr, 0, 0, 0, E, nn, g, qm,
                   dtdx, key, ncount, m, step, seed, dc, o);
    if (SP != 1 && o.cell != kDead) {
      int dx_, fx_, dy_, fy_, dz_, fz_;
      cic_stored(PartsM(), o, g, dx_, fx_, dy_, fy_, dz_, fz_);
      dep_global(dep, g, dx_, fx_, dy_, fy_, dz_, fz_,
                 SP == 0 ? -1 : (SP == 3 ? 2 : 1));
    }
  }
  sink_m(p, i, SP, o, g, ab_rec, ab_pos, ab_vel, ab_cap, dc);
  if (SP == 2) list_dead(live && o.cell == kDead, i, dead2, &dc->n_dead2);
  if (SP == 0) {
    const unsigned long long cs = wave_append(o.cand, &dc->n_tail_cand);
    if (o.cand) cand[first + cs] = cand_rec(o, i);
  }
  const double s = block_sum(live ? o.ke : 0.0, sk);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---- neutral push ---------------------------------------------------------
// Neutrals drift (no field), cross the boundaries and are counted per cell
// for the collisions.  The evaporation sources pile up neutrals in a few
// hundred cells above the cathode, so a global atomic per new neutral would
// serialise on those cells: a workgroup takes chunks of kNChunk neutrals
// and aggregates the new neutrals' cell counts in an LDS hash table first
// (one global atomic per distinct cell and chunk; probes that find no slot
// fall back to the global atomic).
constexpr int kNChunk = 4096;
constexpr int kHist = 2048;
constexpr unsigned kHistEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ void hist_clear(unsigned* hk, int* hc) {
  for (int s = threadIdx.x; s < kHist; s += blockDim.x) {
    hk[s] = kHistEmpty;
    hc[s] = 0;
  }
}

__device__ __forceinline__ void hist_add(unsigned* hk, int* hc, unsigned cell,
                                         int* __restrict__ ncount) {
  const unsigned h = (cell * 2654435761u) >> 21;
#pragma unroll 1
  for (int probe = 0; probe < 8; ++probe) {
    const unsigned s = (h + probe) & (kHist - 1);
    unsigned k = hk[s];
    if (k == kHistEmpty) k = atomicCAS(&hk[s], kHistEmpty, cell);
    if (k == kHistEmpty || k == cell) {
      atomicAdd(&hc[s], 1);
      return;
    }
  }
  atomicAdd(&ncount[cell], 1);
}

__device__ __forceinline__ void hist_flush(unsigned* hk, int* hc,
                                           int* __restrict__ ncount) {
  for (int s = threadIdx.x; s < kHist; s += blockDim.x)
    if (hk[s] != kHistEmpty) atomicAdd(&ncount[hk[s]], hc[s]);
}

// Neutrals per cell are kept up to date across steps: the first n_old
// neutrals (those at the start of the step, all counted) change the count
// only when their cell changes or they leave the domain, and the ones
// appended since are added.  A neutral's previous cell is that of its
// stored position, the value the previous step counted.
__global__ void __launch_bounds__(kT) k_push_neutral(
    Parts p, uint32_t* __restrict__ key, GridC g, double dt,
    int* __restrict__ ncount, long long n_old, MccC m, uint32_t step,
    uint64_t seed, Rec* __restrict__ ab_rec, double* __restrict__ ab_pos,
    double* __restrict__ ab_vel, long long ab_cap, Counters* dc,
    double* __restrict__ part, uint32_t* __restrict__ dead1) {
  __shared__ unsigned hk[kHist];
  __shared__ int hc[kHist];
  __shared__ double sk[kT];
  const long long n = (long long)dc->n[1];
  const long long nchunk = (n + kNChunk - 1) / kNChunk;
  double ke = 0.0;
  for (long long cb = blockIdx.x; cb < nchunk; cb += gridDim.x) {
    const long long b0 = cb * kNChunk;
    const bool fresh = b0 + kNChunk > n_old;  // holds appended neutrals
    if (fresh) {
      hist_clear(hk, hc);
      __syncthreads();
    }
    for (int r = 0; r < kNChunk; r += kT) {
      const long long i = b0 + r + threadIdx.x;
      PushOut o;
      o.cathode = false;
      o.anode = false;
      o.cand = false;
      if (i < n) {
        const double x = p.x[i], y = p.y[i], z = p.z[i];
        const unsigned prev = i < n_old ? cell_of(x, y, z, g) : kDead;
        finish_push<1>(p, i, x, y, z, p.vx[i], p.vy[i], p.vz[i], dt, g, key,
                       ncount, m, step, seed, dc, o, 0ull);
        if (o.cell != prev) {
          if (prev != kDead) atomicSub(&ncount[prev], 1);
          if (o.cell != kDead) {
            if (i >= n_old)
              hist_add(hk, hc, o.cell, ncount);
            else
              atomicAdd(&ncount[o.cell], 1);
          }
        }
        ke = ke + o.ke;
      }
      sink<1>(p, i, o, g, ab_rec, ab_pos, ab_vel, ab_cap, dc);
      list_dead(i < n && o.cell == kDead, i, dead1, &dc->n_dead1);
    }
    if (fresh) {
      __syncthreads();
      hist_flush(hk, hc, ncount);
      __syncthreads();
    }
  }
  const double s = block_sum(ke, sk);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kT) k_push_neutral_m(
    PartsM p, uint32_t* __restrict__ key, GridC g, float dtdx,
    int* __restrict__ ncount, long long n_old, MccC m, uint32_t step,
    uint64_t seed, Rec* __restrict__ ab_rec, double* __restrict__ ab_pos,
    double* __restrict__ ab_vel, long long ab_cap, Counters* dc,
    double* __restrict__ part, uint32_t* __restrict__ dead1) {
  __shared__ unsigned hk[kHist];
  __shared__ int hc[kHist];
  __shared__ double sk[kT];
  const long long n = (long long)dc->n[1];
  const long long nchunk = (n + kNChunk - 1) / kNChunk;
  double ke = 0.0;
  for (long long cb = blockIdx.x; cb < nchunk; cb += gridDim.x) {
    const long long b0 = cb * kNChunk;
    const bool fresh = b0 + kNChunk > n_old;  // holds appended neutrals
    if (fresh) {
      hist_clear(hk, hc);
      __syncthreads();
    }
    for (int r = 0; r < kNChunk; r += kT) {
      const long long i = b0 + r + threadIdx.x;
      PushOut o;
      o.cathode = false;
      o.anode = false;
      o.cand = false;
      if (i < n) {
        const unsigned prev = i < n_old ? p.cell[i] : kDead;
        push_one_m<1>(p, i, nullptr, nullptr, nullptr, 0, 0, 0, nullptr, 0, g,
                      0.0f, dtdx, key, ncount, m, step, seed, dc, o);
        if (o.cell != prev) {
          if (prev != kDead) atomicSub(&ncount[prev], 1);
          if (o.cell != kDead) {
            if (i >= n_old)
              hist_add(hk, hc, o.cell, ncount);
            else
              atomicAdd(&ncount[o.cell], 1);
          }
        }
        ke = ke + o.ke;
      }
      sink_m(p, i, 1, o, g, ab_rec, ab_pos, ab_vel, ab_cap, dc);
      list_dead(i < n && o.cell == kDead, i, dead1, &dc->n_dead1);
    }
    if (fresh) {
      __syncthreads();
      hist_flush(hk, hc, ncount);
      __syncthreads();
    }
  }
  const double s = block_sum(ke, sk);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Sum of two partial arrays (fixed order), times a factor; the first holds
// *na_dev entries when na_dev is given (chunk partials), else na.  Thread t
// adds entries t, t + 1024, ... in that order; the loads go out kScanB at a
// time (clamped to a valid entry), so they are not a chain.
__device__ __forceinline__ double strided_sum(const double* __restrict__ a,
                                              long long n, double acc) {
  for (long long q0 = threadIdx.x; q0 < n; q0 += (long long)kScanB * 1024) {
    double v[kScanB];
#pragma unroll
    for (int k = 0; k < kScanB; ++k) {
      const long long q = q0 + (long long)k * 1024;
      v[k] = a[q < n ? q : n - 1];
    }
#pragma unroll
    for (int k = 0; k < kScanB; ++k)
      if (q0 + (long long)k * 1024 < n) acc = acc + v[k];
  }
  return acc;
}

// Integer counterpart: thread t's share of the sum of n counts.
__device__ __forceinline__ unsigned long long strided_count(
    const uint32_t* __restrict__ a, long long n) {
  unsigned long long acc = 0;
  for (long long q0 = threadIdx.x; q0 < n; q0 += (long long)kScanB * 1024) {
    uint32_t v[kScanB];
#pragma unroll
    for (int k = 0; k < kScanB; ++k) {
      const long long q = q0 + (long long)k * 1024;
      v[k] = a[q < n ? q : n - 1];
    }
#pragma unroll
    for (int k = 0; k < kScanB; ++k)
      acc += q0 + (long long)k * 1024 < n ? v[k] : 0u;
  }
  return acc;
}

__global__ void __launch_bounds__(1024) k_sum_partials(
    const double* __restrict__ a, long long na,
    const unsigned* __restrict__ na_dev, const double* __restrict__ b,
    long long nb, double factor, double* out) {
  __shared__ double s[1024];
  if (na_dev) na = *na_dev;
  double acc = strided_sum(a, na, 0.0);
  acc = strided_sum(b, nb, acc);
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0] * factor;
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

// Null-collision candidates: second draw U2 against the cumulative process
// probabilities (ionisation, then elastic).  Elastic scattering is applied
// at once; ionisation events are recorded as (cell, electron id) for
// matching.  A wave takes kMccChunks consecutive chunks of binned electrons
// and walks their candidates (each chunk's sit in its own segment of the
// candidate list) as one list; then waves of kMccPiece candidates cover the
// unbinned electrons' ones.
constexpr int kMccPiece = 512;
constexpr int kMccChunks = 8;

template <class PT>
__global__ void __launch_bounds__(kT) k_mcc(
    PT p, const uint32_t* __restrict__ key, const CandRec* __restrict__ cand,
    const uint32_t* __restrict__ tse, const uint32_t* __restrict__ cand_cnt,
    const uint2* __restrict__ chunks, const unsigned* __restrict__ nchunks,
    long long tail_first, MccC m, uint32_t step,
    uint64_t seed, Rec* __restrict__ ev, uint32_t* __restrict__ flag,
    long long ev_cap, uint32_t* __restrict__ el_cnt, Counters* dc) {
  const long long nch = *nchunks;
  const long long ngrp = (nch + kMccChunks - 1) / kMccChunks;
  const long long w = blockIdx.x * (long long)(kT / 64) + threadIdx.x / 64;
  // Binned: the candidate segments of chunks t0 .. t0 + kMccChunks - 1
  // (segment k starts at sb[k] and holds pre[k + 1] - pre[k] candidates).
  // Unbinned: one piece of the tail's candidate list.
  long long t0 = 0, sb[kMccChunks];
  unsigned pre[kMccChunks + 1];
  long long b, e;
  const bool binned = w < ngrp;
  pre[0] = 0;
  if (binned) {
    t0 = w * kMccChunks;
#pragma unroll
    for (int k = 0; k < kMccChunks; ++k) {
      const long long t = t0 + k;
      unsigned c = 0, pb = 0, pe = 0;
      if (t < nch) {
        piece(tse, chunks[t].x, chunks[t].y, pb, pe);
        c = cand_cnt[t];
      }
      sb[k] = pb;
      pre[k + 1] = pre[k] + c;
    }
    b = 0;
    e = pre[kMccChunks];
  } else {
    const long long te = tail_first + (long long)dc->n_tail_cand;
    b = tail_first + (w - ngrp) * kMccPiece;
    e = b + kMccPiece < te ? b + kMccPiece : te;
    if (b >= e) return;  // whole wave
  }
  const int lane = lane_id();
  unsigned n_el = 0;  // wave-uniform
  for (long long base = b; base < e; base += 64) {
    long long q = base + lane;
    bool event = false, elastic = false;
    uint32_t i = 0;
    unsigned long long id = 0;
    if (q < e) {
      if (binned) {
        // Combined index -> (chunk segment, offset).
        long long at = sb[0] + q;
#pragma unroll
        for (int k = 1; k < kMccChunks; ++k)
          if ((unsigned)q >= pre[k]) at = sb[k] + (q - pre[k]);
        q = at;
      }
      const CandRec cr = cand[q];
      i = cr.i;
      id = cr.id;
      const double vx = cr.vx, vy = cr.vy, vz = cr.vz;
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
        event = true;
      } else if (u2 < p_tot) {
        elastic = true;
        double u3, u4, nx, ny, nz;
        uniform2(id, step, kTagMcc1, seed, u3, u4);
        isotropic(u3, u4, nx, ny, nz);
        const double cosx = ((vx * nx + vy * ny) + vz * nz) / v;
        const double fac = sqrt(1.0 - m.ratio * (1.0 - cosx));
        const double sp = v * fac;
        Acc<PT>::set_vel(p, i, sp * nx, sp * ny, sp * nz);
      }
    }
    n_el += (unsigned)__popcll(__ballot(elastic));
    const unsigned long long s = wave_append(event, &dc->n_events);
    if (event) {
      const uint32_t cell = key[i];
      if ((long long)s < ev_cap) {
        Rec r;
        r.hi = cell; r.lo = id; r.val = i;
        ev[s] = r;
        atomicOr(&flag[cell >> 5], 1u << (cell & 31u));
      } else {
        atomicOr(&dc->err, kErrEvents);
      }
    }
  }
  if (lane == 0) {
    if (binned) {
      // The group's count in its first chunk's slot (only the sum is used).
      for (int k = 0; k < kMccChunks; ++k)
        if (t0 + k < nch) el_cnt[t0 + k] = k ? 0u : n_el;
    } else if (n_el) {
      atomicAdd(&dc->n_el_tail, (unsigned long long)n_el);
    }
  }
}

// Sort of a record list by (hi, lo) (keys are unique): every kSortChunk
// chunk is sorted in LDS by its own workgroup (bitonic), then rounds of
// pairwise merges place each record at its rank in its own run plus the
// number of smaller keys in the partner run (binary search).  The rounds
// up to kMergeSeg run in LDS, one workgroup per segment, in one launch
// (the short lists end there); the host launches the wider rounds for the
// list's capacity, those whose run width reaches the list's length do
// nothing, and a last pass brings the result back into the first buffer
// when an odd number of them ran.
__global__ void __launch_bounds__(kSortT) k_sort_chunks(
    Rec* __restrict__ a, Rec* __restrict__ tmp,
    const unsigned long long* __restrict__ count, long long cap) {
  __shared__ Rec s[kSortChunk];
  long long n = (long long)*count;
  if (n > cap) n = cap;
  if (n <= 1) return;
  Rec maxr;
  maxr.lo = ~0ull; maxr.hi = ~0u; maxr.val = 0u;
  const int tid = threadIdx.x;
  // Chunks strided over the grid, which the host bounds (its launch
  // covers the capacity, not the device count).
  for (long long base = (long long)blockIdx.x * kSortChunk; base < n;
       base += (long long)gridDim.x * kSortChunk) {
  const int m = (int)(n - base < kSortChunk ? n - base : kSortChunk);
  // A short chunk is padded with the largest key, so the network is fixed.
  const Rec r0 = tid < m ? a[base + tid] : maxr;
  const Rec r1 = tid + kSortT < m ? a[base + tid + kSortT] : maxr;
  s[tid] = r0;
  s[tid + kSortT] = r1;
  __syncthreads();
  // Bitonic network: each stage compares the kSortChunk / 2 pairs (q, q | j)
  // with bit j of q clear, in the direction of bit k of q; thread t takes
  // the t-th pair.
#pragma unroll
  for (int k = 2; k <= kSortChunk; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int q = ((tid & ~(j - 1)) << 1) | (tid & (j - 1));
      const int o = q | j;
      const bool up = (q & k) == 0;
      const Rec x = s[q], y = s[o];
      if (up ? rec_less(y, x) : rec_less(x, y)) { s[q] = y; s[o] = x; }
      __syncthreads();
    }
  if (tid < m) a[base + tid] = s[tid];
  if (tid + kSortT < m) a[base + tid + kSortT] = s[tid + kSortT];
  __syncthreads();
  }
}

// Record i of a merge round: runs of width w (sorted) pairwise into runs
// of 2w; its position is its rank in its own run plus the number of smaller
// keys in the partner run (binary search).
__device__ __forceinline__ void merge_one(const Rec* __restrict__ src,
                                          Rec* __restrict__ dst, long long n,
                                          long long w, long long i) {
  const long long pair = i / (2 * w);
  const long long a0 = pair * 2 * w;
  const long long a1 = a0 + w < n ? a0 + w : n;      // run A = [a0, a1)
  const long long b1 = a1 + w < n ? a1 + w : n;      // run B = [a1, b1)
  const Rec x = src[i];
  long long pos;
  if (i < a1) {
    long long lo = a1, hi = b1;                        // count of B < x
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (rec_less(src[mid], x)) lo = mid + 1; else hi = mid;
    }
    pos = a0 + (i - a0) + (lo - a1);
  } else {
    long long lo = a0, hi = a1;                        // count of A < x
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (rec_less(src[mid], x)) lo = mid + 1; else hi = mid;
    }
    pos = a0 + (i - a1) + (lo - a0);
  }
  dst[pos] = x;
}

// The merge rounds of widths kSortChunk .. kMergeSeg / 2 of one segment,
// in LDS: each round reads every record and its new place (merge_one's
// rule), then, after a barrier, writes them back.
__global__ void __launch_bounds__(kMergeT) k_merge_lds(
    Rec* __restrict__ a, const unsigned long long* __restrict__ count,
    long long cap) {
  __shared__ Rec s[kMergeSeg];
  long long n = (long long)*count;
  if (n > cap) n = cap;
  // Segments strided over the grid (bounded by the host, as above).
  for (long long base = (long long)blockIdx.x * kMergeSeg;
       base + kSortChunk < n; base += (long long)gridDim.x * kMergeSeg) {
  const int m = (int)(n - base < kMergeSeg ? n - base : kMergeSeg);
  const int tid = threadIdx.x;
  constexpr int kPer = kMergeSeg / kMergeT;
  Rec r[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid + k * kMergeT;
    if (i < m) r[k] = a[base + i];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid + k * kMergeT;
    if (i < m) s[i] = r[k];
  }
  __syncthreads();
  for (int w = kSortChunk; w < m; w *= 2) {
    int pos[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int i = tid + k * kMergeT;
      pos[k] = 0;
      if (i >= m) continue;
      const int a0 = i / (2 * w) * (2 * w);
      const int a1 = a0 + w < m ? a0 + w : m;
      const int b1 = a1 + w < m ? a1 + w : m;
      const Rec x = s[i];
      r[k] = x;
      int lo, hi, own;
      if (i < a1) { lo = a1; hi = b1; own = i - a0; }
      else        { lo = a0; hi = a1; own = i - a1; }
      const int first = lo;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rec_less(s[mid], x)) lo = mid + 1; else hi = mid;
      }
      pos[k] = a0 + own + (lo - first);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if (tid + k * kMergeT < m) s[pos[k]] = r[k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int i = tid + k * kMergeT;
    if (i < m) a[base + i] = s[i];
  }
  __syncthreads();
  }
}

__global__ void k_merge_round(const Rec* __restrict__ src, Rec* __restrict__ dst,
                              const unsigned long long* __restrict__ count,
                              long long cap, long long w) {
  long long n = (long long)*count;
  if (n > cap) n = cap;
  if (w >= n) return;   // one run already
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    merge_one(src, dst, n, w, i);
}

// The sorted list back into the first buffer when the merge rounds that
// ran (those with run width below the length) were odd in number.
__global__ void k_copy_recs(const Rec* __restrict__ src, Rec* __restrict__ dst,
                            const unsigned long long* __restrict__ count,
                            long long cap) {
  long long n = (long long)*count;
  if (n > cap) n = cap;
  int rounds = 0;
  for (long long w = kMergeSeg; w < n; w *= 2) ++rounds;
  if ((rounds & 1) == 0) return;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// Neutrals in cells that hold ionisation events.  A workgroup scans
// kNCPer x kT neutrals (coalesced) and reserves its slots in the list with
// one atomic; the list order is free (it is sorted next).
constexpr int kNCPer = 16;
constexpr int kNCChunk = kNCPer * kT;

template <class PT>
__global__ void __launch_bounds__(kT) k_neutral_cands(
    PT p, const uint32_t* __restrict__ key, const uint32_t* __restrict__ flag,
    Rec* __restrict__ nc, long long cap, Counters* dc) {
  __shared__ unsigned sw[kT / 64];
  __shared__ unsigned long long sbase;
  if (dc->n_events == 0) return;
  const long long n = (long long)dc->n[1];
  const long long b0 = blockIdx.x * (long long)kNCChunk;
  if (b0 >= n) return;
  uint32_t cell[kNCPer];
  unsigned long long mk[kNCPer];
  unsigned cnt = 0;  // wave-uniform
#pragma unroll
  for (int r = 0; r < kNCPer; ++r) {
    const long long i = b0 + r * kT + threadIdx.x;
    cell[r] = i < n ? key[i] : kDead;
  }
#pragma unroll
  for (int r = 0; r < kNCPer; ++r) {
    const bool hit = cell[r] != kDead && ((flag[cell[r] >> 5] >> (cell[r] & 31u)) & 1u);
    mk[r] = __ballot(hit);
    cnt += (unsigned)__popcll(mk[r]);
  }
  const int w = threadIdx.x / 64;
  if (lane_id() == 0) sw[w] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned tot = 0;
    for (int q = 0; q < kT / 64; ++q) {
      const unsigned c = sw[q];
      sw[q] = tot;
      tot += c;
    }
    sbase = tot ? atomicAdd(&dc->n_ncand, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  unsigned long long s = sbase + sw[w];
#pragma unroll
  for (int r = 0; r < kNCPer; ++r) {
    if ((mk[r] >> lane_id()) & 1ull) {
      const unsigned long long slot = s + lanes_below(mk[r]);
      const long long i = b0 + r * kT + threadIdx.x;
      if ((long long)slot < cap) {
        Rec rec;
        rec.hi = cell[r]; rec.lo = p.id[i]; rec.val = (unsigned)i;
        nc[slot] = rec;
      } else {
        atomicOr(&dc->err, kErrEvents);
      }
    }
    s += (unsigned long long)__popcll(mk[r]);
  }
}

// Events (sorted by cell, id): the r-th event of a cell takes the cell's
// r-th neutral (sorted by id) if there is one.
__global__ void k_match(const Rec* __restrict__ ev, const Rec* __restrict__ nc,
                        Rec* __restrict__ ok, uint2* __restrict__ okp,
                        long long cap, Counters* dc) {
  long long ne = (long long)dc->n_events;
  if (ne > cap) ne = cap;
  long long nn = (long long)dc->n_ncand;
  if (nn > cap) nn = cap;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  bool hit = false;
  unsigned nidx = 0;
  if (e < ne) {
    const unsigned cell = ev[e].hi;
    long long r = 0;
    while (e - r - 1 >= 0 && ev[e - r - 1].hi == cell) ++r;
    long long lo = 0, hi = nn;
    while (lo < hi) {
      const long long mid = (lo + hi) >> 1;
      if (nc[mid].hi < cell) lo = mid + 1; else hi = mid;
    }
    if (lo + r < nn && nc[lo + r].hi == cell) {
      hit = true;
      nidx = nc[lo + r].val;
    }
  }
  const unsigned long long s = wave_append(hit, &dc->n_ok);
  if (hit) {
    Rec o;
    o.hi = 0; o.lo = ev[e].lo; o.val = (unsigned)s;
    ok[s] = o;
    okp[s] = make_uint2(ev[e].val, nidx);
  }
}

// Matched events in primary-id order: secondary ids next_id + rank; energy
// above threshold shared uniformly, both electrons isotropic; the neutral
// becomes the Cu+ ion (same position, velocity, id).
template <class PT>
__global__ void __launch_bounds__(kT) k_ionise(PT pe, PT pn, PT pi, uint32_t* __restrict__ ke,
                         uint32_t* __restrict__ kn, uint32_t* __restrict__ ki,
                         const Rec* __restrict__ ok, const uint2* __restrict__ okp,
                         MccC m, uint32_t step, uint64_t seed, long long cap_e,
                         long long cap_i, int* __restrict__ ncount,
                         long long* __restrict__ dep, GridC g,
                         uint32_t* __restrict__ dead1, Counters* dc) {
  const long long nok = (long long)dc->n_ok;
  const long long ne0 = (long long)dc->n[0], ni0 = (long long)dc->n[2];
  const unsigned long long id0 = dc->next_id;
  // Every lane of a wave takes the same number of rounds (the list of
  // consumed neutrals is filled per wave).
  for (long long r0 = blockIdx.x * (long long)blockDim.x; r0 < nok;
       r0 += (long long)gridDim.x * blockDim.x) {
    const long long r = r0 + threadIdx.x;
    const bool act = r < nok;
    uint32_t in = 0;
    if (act) {
    const uint2 pr = okp[ok[r].val];
    const uint32_t ie = pr.x;
    in = pr.y;
    const unsigned long long pid = ok[r].lo;
    // Charge of the new pair (the secondary at the primary's position, the
    // ion at the neutral's), taken before this event's stores.
    int cex, cfx, cey, cfy, cez, cfz, cix, cgx, ciy, cgy, ciz, cgz;
    Acc<PT>::cic(pe, ie, g, cex, cfx, cey, cfy, cez, cfz);
    Acc<PT>::cic(pn, in, g, cix, cgx, ciy, cgy, ciz, cgz);
    double u3, u4, u5, u6, u7, u8;
    uniform2(pid, step, kTagMcc1, seed, u3, u4);
    uniform2(pid, step, kTagMcc2, seed, u5, u6);
    uniform2(pid, step, kTagMcc3, seed, u7, u8);
    double vx, vy, vz;
    Acc<PT>::vel(pe, ie, vx, vy, vz);
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
    Acc<PT>::set_vel(pe, ie, vp * px, vp * py, vp * pz);
    const long long de = ne0 + r, di = ni0 + r;
    if (de < cap_e && di < cap_i) {
      Acc<PT>::copy_pos(pe, ie, pe, de);
      Acc<PT>::set_vel(pe, de, vs * sx, vs * sy, vs * sz);
      pe.id[de] = id0 + (unsigned long long)r;
      ke[de] = ke[ie];
      Acc<PT>::copy(pn, in, pi, di);
      ki[di] = kn[in];
      dep_global(dep, g, cex, cfx, cey, cfy, cez, cfz, -1);
      dep_global(dep, g, cix, cgx, ciy, cgy, ciz, cgz, 1);
    } else {
      atomicOr(&dc->err, kErrCapacity);
    }
    // The neutral leaves the per-cell counts of the next step.
    atomicSub(&ncount[kn[in]], 1);
    kn[in] = kDead;
    }
    list_dead(act, in, dead1, &dc->n_dead1);
  }
}

// Clears the event-cell flags, adds the matched ionisations to the counts
// and sums the per-tile elastic counts.
__global__ void __launch_bounds__(1024) k_ionise_commit(Counters* dc, const Rec* __restrict__ ev,
                                uint32_t* __restrict__ flag, long long cap,
                                long long cap_e, long long cap_i,
                                const uint32_t* __restrict__ el_cnt,
                                const uint32_t* __restrict__ cand_cnt,
                                const unsigned* __restrict__ nchunks) {
  const long long ntiles = *nchunks;
  __shared__ unsigned long long s[1024], s2[1024];
  long long ne = (long long)dc->n_events;
  if (ne > cap) ne = cap;
  for (long long e = threadIdx.x; e < ne; e += blockDim.x) flag[ev[e].hi >> 5] = 0u;
  const unsigned long long a = strided_count(el_cnt, ntiles);
  const unsigned long long b = strided_count(cand_cnt, ntiles);
  s[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s[threadIdx.x] += s[threadIdx.x + o];
      s2[threadIdx.x] += s2[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x) return;
  dc->n_elastic = s[0] + dc->n_el_tail;
  dc->n_cand = s2[0] + dc->n_tail_cand;
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

// Atoms handed back to MD: records [first, first + n) of the sorted cathode
// list to outputs [out0, out0 + n) of SoA arrays of stride nout, each
// crossing point offset backwards along the velocity by off = 3 a.
__global__ void k_md_return(const int32_t* __restrict__ sp,
                            const uint64_t* __restrict__ id,
                            const double* __restrict__ pos,
                            const double* __restrict__ vel, long long nab,
                            long long first, long long n, double off3a,
                            GridC g, double* __restrict__ opos,
                            double* __restrict__ ovel,
                            uint64_t* __restrict__ oid,
                            int32_t* __restrict__ osp, long long out0,
                            long long nout) {
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < n;
       r += (long long)gridDim.x * blockDim.x) {
    const long long q = first + r, o = out0 + r;
    const double vx = vel[q], vy = vel[nab + q], vz = vel[2 * nab + q];
    const double inv = 1.0 / sqrt((vx * vx + vy * vy) + vz * vz);
    const double off = off3a * inv;
    opos[o] = wrap_coord(pos[q] - off * vx, g.lx);
    opos[nout + o] = wrap_coord(pos[nab + q] - off * vy, g.ly);
    opos[2 * nout + o] = pos[2 * nab + q] - off * vz;
    ovel[o] = vx; ovel[nout + o] = vy; ovel[2 * nout + o] = vz;
    oid[o] = id[q];
    if (osp) osp[o] = sp[q];
  }
}

// ---- binning ------------------------------------------------------------------
// Particles of a binned tile move at most one tile per axis per step, so a
// tile's particles go to one of its 27 neighbours (slot d of dest_slot);
// counting per (tile, slot) in LDS needs one global atomic per non-empty
// slot (the rare farther moves take a global atomic each).

// Count the destination tiles of a tile's binned particles.
__global__ void __launch_bounds__(kT) k_bin_hist_tile(
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ ts,
    const uint2* __restrict__ chunks, const unsigned* __restrict__ nchunks,
    unsigned* __restrict__ cnt, GridC g) {
  __shared__ unsigned sc[27];
  __shared__ unsigned sdst[27];
  const unsigned nchk = *nchunks;
  if (blockIdx.x >= nchk) return;
  const unsigned cb = xcd_block(blockIdx.x, nchk);
  const unsigned t = chunks[cb].x;
  unsigned b, e;
  piece(ts, t, chunks[cb].y, b, e);
  if (b == e) return;
  if (threadIdx.x < 27) sc[threadIdx.x] = 0;
  __syncthreads();
  const int tx = (int)(t % g.tnx), ty = (int)((t / g.tnx) % g.tny),
            tz = (int)(t / ((unsigned)g.tnx * g.tny));
  for (unsigned q = b + threadIdx.x; q < e; q += blockDim.x)
    count_dest(key[q], tx, ty, tz, g, sc, sdst, cnt);
  __syncthreads();
  if (threadIdx.x < 27 && sc[threadIdx.x]) atomicAdd(&cnt[sdst[threadIdx.x]], sc[threadIdx.x]);
}

// Slot of key in the LDS hash table (inserted if absent), or -1 when the
// probes find no room.
__device__ __forceinline__ int hist_slot(unsigned* hk, unsigned key) {
  const unsigned h = (key * 2654435761u) >> 21;
#pragma unroll 1
  for (int probe = 0; probe < 8; ++probe) {
    const unsigned s = (h + probe) & (kHist - 1);
    unsigned k = hk[s];
    if (k == kHistEmpty) k = atomicCAS(&hk[s], kHistEmpty, key);
    if (k == kHistEmpty || k == key) return (int)s;
  }
  return -1;
}

// Unbinned tail (particles appended this step, e.g. a source's neutrals
// piling into a few tiles, or a whole population after a load): per chunk
// of kLChunk, tile counts aggregated in an LDS hash table, one global
// atomic per distinct tile.  The chunk is small so that a tail of ~1e5
// particles still spreads over all CUs.
constexpr int kLChunk = 1024;

__global__ void __launch_bounds__(kT) k_bin_hist_list(
    const uint32_t* __restrict__ key, unsigned* __restrict__ cnt, GridC g,
    long long first, const unsigned long long* __restrict__ np) {
  __shared__ unsigned hk[kHist];
  __shared__ int hc[kHist];
  hist_clear(hk, hc);
  __syncthreads();
  const long long n = (long long)*np;
  const long long b0 = first + blockIdx.x * (long long)kLChunk;
  for (int r = 0; r < kLChunk; r += kT) {
    const long long i = b0 + r + threadIdx.x;
    if (i >= n) break;
    const uint32_t k = key[i];
    if (k == kDead) continue;
    hist_add(hk, hc, tile_of_cell(k, g), reinterpret_cast<int*>(cnt));
  }
  __syncthreads();
  hist_flush(hk, hc, reinterpret_cast<int*>(cnt));
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


// Move a tile's live particles to their destination ranges in the other
// buffer: per slot, one global atomic reserves the block's range; ranks
// within it come from LDS counters.
template <class PT>
__global__ void __launch_bounds__(kT) k_bin_scatter_tile(
    PT src, PT dst, const uint32_t* __restrict__ key,
    const uint32_t* __restrict__ ts, const uint2* __restrict__ chunks,
    const unsigned* __restrict__ nchunks, unsigned* __restrict__ cursor,
    GridC g) {
  __shared__ unsigned sc[27], sbase[27], srank[27];
  __shared__ unsigned sdst[27];
  const unsigned nchk = *nchunks;
  if (blockIdx.x >= nchk) return;
  const unsigned cb = xcd_block(blockIdx.x, nchk);
  const unsigned t = chunks[cb].x;
  unsigned b, e;
  piece(ts, t, chunks[cb].y, b, e);
  if (b == e) return;
  if (threadIdx.x < 27) {
    sc[threadIdx.x] = 0;
    srank[threadIdx.x] = 0;
  }
  __syncthreads();
  const int tx = (int)(t % g.tnx), ty = (int)((t / g.tnx) % g.tny),
            tz = (int)(t / ((unsigned)g.tnx * g.tny));
  for (unsigned q = b + threadIdx.x; q < e; q += blockDim.x) {
    const uint32_t k = key[q];
    if (k == kDead) continue;
    unsigned u;
    const int d = dest_slot(k, tx, ty, tz, g, u);
    if (d >= 0) {
      atomicAdd(&sc[d], 1u);
      sdst[d] = u;
    }
  }
  __syncthreads();
  if (threadIdx.x < 27 && sc[threadIdx.x])
    sbase[threadIdx.x] = atomicAdd(&cursor[sdst[threadIdx.x]], sc[threadIdx.x]);
  __syncthreads();
  for (unsigned q = b + threadIdx.x; q < e; q += blockDim.x) {
    const uint32_t k = key[q];
    if (k == kDead) continue;
    unsigned u;
    const int d = dest_slot(k, tx, ty, tz, g, u);
    const unsigned pos = d >= 0 ? sbase[d] + atomicAdd(&srank[d], 1u)
                                : atomicAdd(&cursor[u], 1u);
    Acc<PT>::copy(src, q, dst, pos);
  }
}

// The tail's scatter: per chunk, the tile counts in LDS reserve one range
// per distinct tile with a single global atomic, and each particle takes
// the next rank in its tile's range (particles whose tile found no hash
// slot take a global slot directly).
constexpr int kPerThread = kLChunk / kT;

template <class PT>
__global__ void __launch_bounds__(kT) k_bin_scatter_list(
    PT src, PT dst, const uint32_t* __restrict__ key,
    unsigned* __restrict__ cursor, GridC g, long long first,
    const unsigned long long* __restrict__ np) {
  __shared__ unsigned hk[kHist];
  __shared__ int hc[kHist];
  __shared__ unsigned hb[kHist];
  hist_clear(hk, hc);
  __syncthreads();
  const long long n = (long long)*np;
  const long long b0 = first + blockIdx.x * (long long)kLChunk;
  int sl[kPerThread];
  unsigned pos[kPerThread];
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    sl[r] = -2;  // no particle
    const long long i = b0 + r * kT + threadIdx.x;
    if (i < n) {
      const uint32_t k = key[i];
      if (k != kDead) {
        const unsigned t = tile_of_cell(k, g);
        sl[r] = hist_slot(hk, t);
        if (sl[r] >= 0)
          atomicAdd(&hc[sl[r]], 1);
        else
          pos[r] = atomicAdd(&cursor[t], 1u);
      }
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < kHist; q += kT) {
    if (hk[q] != kHistEmpty) hb[q] = atomicAdd(&cursor[hk[q]], (unsigned)hc[q]);
    hc[q] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kPerThread; ++r) {
    if (sl[r] == -2) continue;
    const long long i = b0 + r * kT + threadIdx.x;
    const unsigned d = sl[r] >= 0 ? hb[sl[r]] + (unsigned)atomicAdd(&hc[sl[r]], 1) : pos[r];
    Acc<PT>::copy(src, i, dst, d);
  }
}

__global__ void k_set_count(Counters* dc, int s, const unsigned* __restrict__ ts,
                            long long ntiles) {
  dc->n[s] = ts[ntiles];
  dc->sorted_n[s] = ts[ntiles];
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

__device__ __forceinline__ uint32_t load_key(const Parts&, long long, double x,
                                             double y, double z,
                                             const GridC& g) {
  return cell_of(x, y, z, g);
}
__device__ __forceinline__ uint32_t load_key(const PartsM& p, long long t,
                                             double, double, double,
                                             const GridC&) {
  return p.cell[t];
}

// Load caller particles (FP64 SoA) and their cell keys; out-of-domain or
// non-finite input is flagged and keyed dead (dropped by the binning).
template <class PT>
__global__ void k_load(PT p, const double* __restrict__ pos,
                       const double* __restrict__ vel,
                       const uint64_t* __restrict__ ids,
                       uint32_t* __restrict__ key, long long n, GridC g,
                       Counters* dc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = pos[t], y = pos[n + t], z = pos[2 * n + t];
  const double vx = vel[t], vy = vel[n + t], vz = vel[2 * n + t];
  p.id[t] = ids[t];
  const double gz = z * g.inv_dx;
  const bool ok = x >= 0.0 && x < g.lx && y >= 0.0 && y < g.ly && gz >= 0.0 &&
                  gz < (double)g.nz && isfinite(vx) && isfinite(vy) &&
                  isfinite(vz);
  if (!ok) {
    atomicOr(&dc->err, kErrNonFinite);
    key[t] = kDead;
    return;
  }
  Acc<PT>::set_pos(p, t, g, x, y, z);
  Acc<PT>::set_vel(p, t, vx, vy, vz);
  key[t] = load_key(p, t, x, y, z, g);
}

// Cell keys of a population restored in its native layout.
__global__ void k_restore_keys(Parts p, uint32_t* __restrict__ key, long long n,
                               GridC g, Counters* dc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double x = p.x[t], y = p.y[t], z = p.z[t];
  const double gz = z * g.inv_dx;
  const bool ok = x >= 0.0 && x < g.lx && y >= 0.0 && y < g.ly && gz >= 0.0 &&
                  gz < (double)g.nz;
  if (!ok) atomicOr(&dc->err, kErrNonFinite);
  key[t] = ok ? cell_of(x, y, z, g) : kDead;
}
__global__ void k_restore_keys(PartsM p, uint32_t* __restrict__ key,
                               long long n, GridC g, Counters* dc) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  const uint32_t cell = p.cell[t];
  const bool ok = cell < (uint32_t)((long long)g.nxy * g.nz);
  if (!ok) atomicOr(&dc->err, kErrNonFinite);
  key[t] = ok ? cell : kDead;
}

template <class PT>
__global__ void k_read(PT p, double* __restrict__ pos, double* __restrict__ vel,
                       uint64_t* __restrict__ ids, long long n, GridC g) {
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= n) return;
  double x, y, z, vx, vy, vz;
  Acc<PT>::pos(p, t, g, x, y, z);
  Acc<PT>::vel(p, t, vx, vy, vz);
  pos[t] = x; pos[n + t] = y; pos[2 * n + t] = z;
  vel[t] = vx; vel[n + t] = vy; vel[2 * n + t] = vz;
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
  const pic_sources& s = c->src;
  m.sph_on = s.sph_absorb ? 1 : 0;
  m.sph_cx = s.sph_cx;
  m.sph_cy = s.sph_cy;
  m.sph_cz = s.sph_cz;
  m.sph_r2 = s.sph_radius * s.sph_radius;
  m.sph_alpha = s.sph_alpha_eh;
  m.dt = dt;
  return m;
}

// Launch bound of a species: the host's upper bound of the device count,
// never above the capacity (kernels read the exact count on the device).
long long bound(const pic_ctx* c, int s) {
  long long n = c->n[s];
  if (n > c->cfg.capacity[s]) n = c->cfg.capacity[s];
  return n > 0 ? n : 1;
}

uint32_t* ts_cur(pic_ctx* c, int s) { return c->tsb[s][c->tcur[s]]; }

// Sort a record list of at most cap entries (device count); tmp holds as
// many.  The result ends in a.
void sort_records(pic_ctx* c, Rec* a, Rec* tmp,
                  const unsigned long long* count, long long cap) {
  hipStream_t st = c->stream;
  // Grids bounded so that a short list in a large capacity costs little:
  // the kernels stride over the device count.
  const long long nchunk = std::min<long long>((cap + kSortChunk - 1) / kSortChunk, 4096);
  k_sort_chunks<<<(unsigned)nchunk, kSortT, 0, st>>>(a, tmp, count, cap);
  if (cap > kSortChunk)
    k_merge_lds<<<(unsigned)std::min<long long>((cap + kMergeSeg - 1) / kMergeSeg, 1024),
                  kMergeT, 0, st>>>(a, count, cap);
  Rec* src = a;
  Rec* dst = tmp;
  const unsigned nround = std::min<unsigned>(nblk(cap), kFixedBlocks);
  for (long long w = kMergeSeg; w < cap; w *= 2) {
    k_merge_round<<<nround, kT, 0, st>>>(src, dst, count, cap, w);
    Rec* t = src; src = dst; dst = t;
  }
  if (cap > kMergeSeg) k_copy_recs<<<256, kT, 0, st>>>(tmp, a, count, cap);
}

double qm_dt(int s, double dt) {
  const double q = s == 0 ? -kE : (s == 2 ? kE : (s == 3 ? 2.0 * kE : 0.0));
  const double mass = s == 0 ? kMe : kMcu;
  return (q / mass) * dt;
}

// Particle buffers of a layout.
template <class PT>
PT buf(pic_ctx* c, int s, int b);
template <>
Parts buf<Parts>(pic_ctx* c, int s, int b) { return c->P[s][b]; }
template <>
PartsM buf<PartsM>(pic_ctx* c, int s, int b) { return c->PM[s][b]; }

template <class PT>
PT cur(pic_ctx* c, int s) { return buf<PT>(c, s, c->cur[s]); }

template <class PT>
void deposit_t(pic_ctx* c) {
  k_deposit<PT><<<(unsigned)c->nch_bound, kT, 0, c->stream>>>(
      cur<PT>(c, 0), cur<PT>(c, 2), ts_cur(c, 0), ts_cur(c, 2), c->chunks,
      c->cstart + c->ntiles, c->acc, c->g);
  // Particles outside the tile ranges (ions left unbinned between passes).
  for (int s = 0; s < 3; s += 2) {
    const long long tail = std::max(0ll, bound(c, s) - c->n_binned[s]);
    if (tail > 0)
      k_deposit_tail<PT><<<nblk(tail), kT, 0, c->stream>>>(
          cur<PT>(c, s), c->n_binned[s], &c->dc->n[s], c->acc, c->g,
          s ? 1 : -1);
  }
  // Cu2+ (a list species, two charges each).
  const long long n3 = bound(c, 3);
  if (n3 > 0)
    k_deposit_tail<PT><<<nblk(n3), kT, 0, c->stream>>>(
        cur<PT>(c, 3), 0, &c->dc->n[3], c->acc, c->g, 2);
}

// Queue, disk, sphere and Fowler-Nordheim particles, ids in that order.
// The first part (counts known on the host, no field) also resets the
// step's counters; the Fowler-Nordheim part reads the cathode field.
template <class PT>
void sources_host_t(pic_ctx* c) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  long long n[4] = {c->n[0], c->n[1], c->n[2], c->n[3]};
  c->n_start1 = c->n[1];
  unsigned long long nid = c->next_id;
  for (const QueueCall& q : c->queue) {
    if (q.n <= 0) continue;
    k_append_queue<PT><<<nblk(q.n), kT, 0, st>>>(
        cur<PT>(c, q.species), n[q.species], c->q_pos + 3 * q.offset,
        c->q_vel + 3 * q.offset, q.n, nid, c->g);
    n[q.species] += q.n;
    nid += q.n;
  }
  c->queue.clear();
  c->queue_used = 0;
  const pic_sources& s = c->src;
  if (s.disk_on) {
    if (s.disk_n_e > 0) {
      const double vth2 = (s.disk_kT_e_eV * kE) / kMe;
      k_disk<PT><<<nblk(s.disk_n_e), kT, 0, st>>>(
          cur<PT>(c, 0), n[0], s.disk_n_e, nid, 0, s.disk_cx, s.disk_cy,
          s.disk_radius, vth2, c->g, step, seed);
      n[0] += s.disk_n_e;
      nid += s.disk_n_e;
    }
    if (s.disk_n_n > 0) {
      const double vth2 = (kKB * s.disk_T_n_K) / kMcu;
      k_disk<PT><<<nblk(s.disk_n_n), kT, 0, st>>>(
          cur<PT>(c, 1), n[1], s.disk_n_n, nid, 1, s.disk_cx, s.disk_cy,
          s.disk_radius, vth2, c->g, step, seed);
      n[1] += s.disk_n_n;
      nid += s.disk_n_n;
    }
  }
  if (s.sphere_on && s.sph_n > 0) {
    const double sig = sqrt((kKB * s.sph_T_K) / kMcu);
    k_sphere<PT><<<nblk(s.sph_n), kT, 0, st>>>(
        cur<PT>(c, 1), n[1], s.sph_n, nid, s.sph_cx, s.sph_cy, s.sph_cz,
        s.sph_radius, sig, c->g, step, seed);
    n[1] += s.sph_n;
    nid += s.sph_n;
  }
  k_begin<<<1, 1, 0, st>>>(c->dc, n[0], n[1], n[2], n[3], nid);
  for (int k = 0; k < 4; ++k) c->n[k] = n[k];
  c->next_id_src = nid;
}

template <class PT>
void sources_fn_t(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  const pic_sources& s = c->src;
  const long long n0 = c->n[0];
  const unsigned long long nid = c->next_id_src;
  if (s.fn_on) {
    const double phi_j = s.fn_phi_w_eV * kE;
    const double a_fn = pow(kE, 3.0) / (8.0 * kPi * kH);
    const double b_fn = (8.0 * kPi * sqrt(2.0 * kMe)) / (3.0 * kE * kH);
    const double a_phi = a_fn / phi_j;
    const double b_phi = b_fn * phi_j * sqrt(phi_j);
    const double c_fn = ((c->g.dx * c->g.dx) * dt) / kE;
    if (c->mixed)
      k_fn_count<float><<<nblk(c->g.nxy), kT, 0, st>>>(
          reinterpret_cast<const float*>(c->E) + 2 * c->nnodes,
          c->fn_scan + c->g.nxy + 1, c->g, s.fn_cx, s.fn_cy, s.fn_radius, a_phi,
          b_phi, c_fn, step, seed, c->dc);
    else
      k_fn_count<double><<<nblk(c->g.nxy), kT, 0, st>>>(
          c->E + 2 * c->nnodes, c->fn_scan + c->g.nxy + 1, c->g, s.fn_cx,
          s.fn_cy, s.fn_radius, a_phi, b_phi, c_fn, step, seed, c->dc);
    k_scan1<<<1, 1024, 0, st>>>(c->fn_scan + c->g.nxy + 1, c->fn_scan, c->g.nxy);
    long long cap = c->cfg.max_events;
    if (n0 + cap > c->cfg.capacity[0]) cap = c->cfg.capacity[0] - n0;
    if (cap < 0) cap = 0;
    const double vth2 = (s.fn_kT_e_eV * kE) / kMe;
    k_fn_spawn<PT><<<nblk(c->cfg.max_events > 0 ? c->cfg.max_events : 1), kT, 0, st>>>(
        cur<PT>(c, 0), n0, cap, c->fn_scan, c->g, nid, vth2, step, seed, c->dc);
    k_fn_commit<<<1, 1, 0, st>>>(c->dc, cap);
    // Upper bound of the electron count for the launches that follow.
    c->n[0] = n0 + c->cfg.max_events;
  }
}

// Neutral push (no field): cell counts for the collisions, boundary
// crossings, kinetic energy (partial sums in a region of its own).
template <class PT>
void push_neutral_t(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  const MccC m = mcc_constants(c, dt);
  const long long ab_cap = c->cfg.max_events;
  // Neutrals per cell: updated from the counts of the step before, or
  // counted afresh after the population was replaced.
  const long long n_old = c->ncount_valid ? c->n_start1 : 0;
  if (!c->ncount_valid) hipMemsetAsync(c->ncount, 0, c->ncells * sizeof(int), st);
  tmark(c, PIC_PH_PUSH_NEUTRAL, true);
  const long long nb = neutral_push_blocks(bound(c, 1));
  if (c->mixed)
    k_push_neutral_m<<<nb, kT, 0, st>>>(
        cur<PartsM>(c, 1), c->key[1], c->g, (float)(dt * c->g.inv_dx),
        c->ncount, n_old, m, step, seed, c->ab_rec, c->ab_raw_pos,
        c->ab_raw_vel, ab_cap, c->dc, c->part_n, c->dead1);
  else
    k_push_neutral<<<nb, kT, 0, st>>>(
        cur<Parts>(c, 1), c->key[1], c->g, dt, c->ncount, n_old, m, step,
        seed, c->ab_rec, c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc,
        c->part_n, c->dead1);
  c->ncount_valid = true;
  tmark(c, PIC_PH_PUSH_NEUTRAL, false);
  k_sum_partials<<<1, 1024, 0, st>>>(c->part_n, nb, nullptr, c->part_n, 0,
                                     0.5 * kMcu, &c->dc->kinetic[1]);
}

// Pushes of the FP64 layout.
void push_fp64(pic_ctx* c, double dt, const MccC& m, double* part_e,
               double* part_i, double* part_l, long long& nbi, long long& nbe,
               long long& nb3) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  const long long nn = c->nnodes;
  const long long nt = c->ntiles;
  const long long ab_cap = c->cfg.max_events;
  tmark(c, PIC_PH_PUSH_ELECTRON, true);
  TileArgs A;
  A.pe = cur<Parts>(c, 0);
  A.pi = cur<Parts>(c, 2);
  A.tse = ts_cur(c, 0);
  A.tsi = ts_cur(c, 2);
  A.chunks = c->chunks;
  A.nchunks = c->cstart + nt;
  A.keye = c->key[0];
  A.keyi = c->key[2];
  A.qm_e = qm_dt(0, dt);
  A.qm_i = qm_dt(2, dt);
  A.dt = dt;
  A.ncount = c->ncount;
  A.cand = c->cand;
  A.cand_cnt = c->cand_cnt;
  A.ab_rec = c->ab_rec;
  A.ab_pos = c->ab_raw_pos;
  A.ab_vel = c->ab_raw_vel;
  A.ab_cap = ab_cap;
  A.part_e = part_e;
  A.part_i = part_i;
  A.cnt_e = c->tcnt[0];
  A.cnt_i = c->tcnt[1];
  A.dep = c->acc_next;
  A.dead2 = c->dead2;
  k_push_tile<<<(unsigned)c->nch_bound, kT, 0, st>>>(A, c->E, nn, c->g, m,
                                                         step, seed, c->dc);
  tmark(c, PIC_PH_PUSH_ELECTRON, false);
  tmark(c, PIC_PH_PUSH_ION, true);
  const long long tail_i = std::max(0ll, bound(c, 2) - c->n_binned[2]);
  nbi = nblk(tail_i > 0 ? tail_i : 1);
  k_push_list<2><<<nbi, kT, 0, st>>>(
      cur<Parts>(c, 2), c->n_binned[2], c->key[2], c->E, nn, c->g,
      qm_dt(2, dt), dt, c->ncount, c->cand, m, step, seed, c->ab_rec,
      c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc, part_l, c->acc_next, c->dead2);
  const long long tail_e = std::max(0ll, bound(c, 0) - c->n_binned[0]);
  nbe = nblk(tail_e > 0 ? tail_e : 1);
  k_push_list<0><<<nbe, kT, 0, st>>>(
      cur<Parts>(c, 0), c->n_binned[0], c->key[0], c->E, nn, c->g,
      qm_dt(0, dt), dt, c->ncount, c->cand, m, step, seed, c->ab_rec,
      c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc, part_l + nbi, c->acc_next, c->dead2);
  // Cu2+: the whole list, field from global memory.
  const long long n3 = bound(c, 3);
  nb3 = n3 > 0 ? nblk(n3) : 0;
  if (n3 > 0)
    k_push_list<3><<<nb3, kT, 0, st>>>(
        cur<Parts>(c, 3), 0, c->key[3], c->E, nn, c->g, qm_dt(3, dt), dt,
        c->ncount, c->cand, m, step, seed, c->ab_rec, c->ab_raw_pos,
        c->ab_raw_vel, ab_cap, c->dc, part_l + nbi + nbe, c->acc_next,
        c->dead2);
  tmark(c, PIC_PH_PUSH_ION, false);
}

// Pushes of the mixed layout (FP32 field, kick and drift).
void push_mixed(pic_ctx* c, double dt, const MccC& m, double* part_e,
                double* part_i, double* part_l, long long& nbi, long long& nbe,
                long long& nb3) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  const long long nn = c->nnodes;
  const long long nt = c->ntiles;
  const long long ab_cap = c->cfg.max_events;
  const float* E = reinterpret_cast<const float*>(c->E);
  const float dtdx = (float)(dt * c->g.inv_dx);
  tmark(c, PIC_PH_PUSH_ELECTRON, true);
  TileArgsM A;
  A.pe = cur<PartsM>(c, 0);
  A.pi = cur<PartsM>(c, 2);
  A.tse = ts_cur(c, 0);
  A.tsi = ts_cur(c, 2);
  A.chunks = c->chunks;
  A.nchunks = c->cstart + nt;
  A.keye = c->key[0];
  A.keyi = c->key[2];
  A.qm_e = (float)qm_dt(0, dt);
  A.qm_i = (float)qm_dt(2, dt);
  A.dtdx = dtdx;
  A.ncount = c->ncount;
  A.cand = c->cand;
  A.cand_cnt = c->cand_cnt;
  A.ab_rec = c->ab_rec;
  A.ab_pos = c->ab_raw_pos;
  A.ab_vel = c->ab_raw_vel;
  A.ab_cap = ab_cap;
  A.part_e = part_e;
  A.part_i = part_i;
  A.cnt_e = c->tcnt[0];
  A.cnt_i = c->tcnt[1];
  A.dep = c->acc_next;
  A.dead2 = c->dead2;
  k_push_tile_m<<<(unsigned)c->nch_bound, kT, 0, st>>>(A, E, nn, c->g, m,
                                                           step, seed, c->dc);
  tmark(c, PIC_PH_PUSH_ELECTRON, false);
  tmark(c, PIC_PH_PUSH_ION, true);
  const long long tail_i = std::max(0ll, bound(c, 2) - c->n_binned[2]);
  nbi = nblk(tail_i > 0 ? tail_i : 1);
  k_push_list_m<2><<<nbi, kT, 0, st>>>(
      cur<PartsM>(c, 2), c->n_binned[2], c->key[2], E, nn, c->g,
      (float)qm_dt(2, dt), dtdx, c->ncount, c->cand, m, step, seed, c->ab_rec,
      c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc, part_l, c->acc_next, c->dead2);
  const long long tail_e = std::max(0ll, bound(c, 0) - c->n_binned[0]);
  nbe = nblk(tail_e > 0 ? tail_e : 1);
  k_push_list_m<0><<<nbe, kT, 0, st>>>(
      cur<PartsM>(c, 0), c->n_binned[0], c->key[0], E, nn, c->g,
      (float)qm_dt(0, dt), dtdx, c->ncount, c->cand, m, step, seed, c->ab_rec,
      c->ab_raw_pos, c->ab_raw_vel, ab_cap, c->dc, part_l + nbi, c->acc_next, c->dead2);
  const long long n3 = bound(c, 3);
  nb3 = n3 > 0 ? nblk(n3) : 0;
  if (n3 > 0)
    k_push_list_m<3><<<nb3, kT, 0, st>>>(
        cur<PartsM>(c, 3), 0, c->key[3], E, nn, c->g, (float)qm_dt(3, dt),
        dtdx, c->ncount, c->cand, m, step, seed, c->ab_rec, c->ab_raw_pos,
        c->ab_raw_vel, ab_cap, c->dc, part_l + nbi + nbe, c->acc_next,
        c->dead2);
  tmark(c, PIC_PH_PUSH_ION, false);
}

template <class PT>
void push_collide_t(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const uint32_t step = (uint32_t)c->step;
  const uint64_t seed = c->cfg.seed;
  const MccC m = mcc_constants(c, dt);
  const long long nt = c->ntiles;
  // The tile push counts the binned particles' destination tiles.
  hipMemsetAsync(c->tcnt[0], 0, 2 * (nt + 1) * sizeof(unsigned), st);
  c->tcounted = true;
  // Partial-sum regions: electron chunks, ion chunks, per-particle blocks.
  double* part_e = c->partials;
  double* part_i = c->partials + c->nch_cap;
  double* part_l = c->partials + 2 * c->nch_cap;
  long long nbi = 1, nbe = 1, nb3 = 0;
  // The pushes and the ionisations add the charge of the state this step
  // leaves; the next deposit takes it instead of a pass of its own.
  hipMemsetAsync(c->acc_next, 0, c->nnodes * sizeof(long long), st);
  if (c->mixed)
    push_mixed(c, dt, m, part_e, part_i, part_l, nbi, nbe, nb3);
  else
    push_fp64(c, dt, m, part_e, part_i, part_l, nbi, nbe, nb3);
  const long long nch = c->nch_bound;
  k_sum_partials<<<1, 1024, 0, st>>>(part_i, nch, c->cstart + nt, part_l,
                                     nbi, 0.5 * kMcu, &c->dc->kinetic[2]);
  k_sum_partials<<<1, 1024, 0, st>>>(part_e, nch, c->cstart + nt,
                                     part_l + nbi, nbe, 0.5 * kMe,
                                     &c->dc->kinetic[0]);
  if (nb3 > 0)
    k_sum_partials<<<1, 1024, 0, st>>>(part_l + nbi + nbe, nb3, nullptr,
                                       part_l + nbi + nbe, 0, 0.5 * kMcu,
                                       &c->dc->kinetic[3]);
  const long long cap = c->cfg.max_events;
  tmark(c, PIC_PH_COLLIDE, true);
  if (m.enabled) {
    // Waves: one per chunk, then the unbinned electrons' candidates (at
    // most one per electron appended this step) in pieces.
    const long long tail = std::max(0ll, bound(c, 0) - c->n_binned[0]);
    const long long waves = (nch + kMccChunks - 1) / kMccChunks +
                            std::max(1ll, (tail + kMccPiece - 1) / kMccPiece);
    k_mcc<PT><<<(unsigned)((waves + kT / 64 - 1) / (kT / 64)), kT, 0, st>>>(
        cur<PT>(c, 0), c->key[0], c->cand, ts_cur(c, 0), c->cand_cnt,
        c->chunks, c->cstart + nt, c->n_binned[0], m, step, seed, c->ev,
        c->flag, cap, c->el_cnt, c->dc);
    sort_records(c, c->ev, c->rec_tmp, &c->dc->n_events, cap);
    k_neutral_cands<PT><<<(unsigned)((bound(c, 1) + kNCChunk - 1) / kNCChunk), kT, 0, st>>>(
        cur<PT>(c, 1), c->key[1], c->flag, c->nc, cap, c->dc);
    sort_records(c, c->nc, c->rec_tmp, &c->dc->n_ncand, cap);
    k_match<<<nblk(cap), kT, 0, st>>>(c->ev, c->nc, c->ok, c->okp, cap, c->dc);
    sort_records(c, c->ok, c->rec_tmp, &c->dc->n_ok, cap);
    k_ionise<PT><<<64, kT, 0, st>>>(cur<PT>(c, 0), cur<PT>(c, 1), cur<PT>(c, 2),
                                    c->key[0], c->key[1], c->key[2], c->ok,
                                    c->okp, m, step, seed, c->cfg.capacity[0],
                                    c->cfg.capacity[2], c->ncount, c->acc_next,
                                    c->g, c->dead1, c->dc);
    k_ionise_commit<<<1, 1024, 0, st>>>(c->dc, c->ev, c->flag, cap,
                                        c->cfg.capacity[0], c->cfg.capacity[2],
                                        c->el_cnt, c->cand_cnt,
                                        c->cstart + nt);
    c->n[0] += cap;  // bound: secondaries
    c->n[2] += cap;
  }
  if (c->coul.enabled) {
    // Coulomb collisions of the charged particles the step leaves.
    tmark(c, PIC_PH_COULOMB, true);
    parts_coulomb(c, dt);
    tmark(c, PIC_PH_COULOMB, false);
  }
  if (c->ionp.enabled) {
    // Recombination, ionisation of Cu+ and charge exchange.
    tmark(c, PIC_PH_ION_COLL, true);
    parts_ion_processes(c, dt);
    tmark(c, PIC_PH_ION_COLL, false);
    c->n[0] += cap;  // bounds: secondaries, atoms, Cu2+
    c->n[1] += cap;
    c->n[3] += cap;
  }
  tmark(c, PIC_PH_COLLIDE, false);
  // Cathode list sorted by (species, id).
  tmark(c, PIC_PH_ABSORBED, true);
  sort_records(c, c->ab_rec, c->rec_tmp, &c->dc->n_ab, cap);
  k_ab_gather<<<64, kT, 0, st>>>(c->ab_rec, c->ab_raw_pos, c->ab_raw_vel,
                                 c->ab_species, c->ab_id, c->ab_pos, c->ab_vel,
                                 cap, c->dc);
  tmark(c, PIC_PH_ABSORBED, false);
}

// Bin one species by tile into the other buffer (removing dead particles):
// destination counts from the binned ranges (per chunk) and the appended
// tail (per particle), an exclusive scan, then the scatter.  The neutrals
// keep no tile ranges between passes (they are compacted in place), so all
// of them bin as one tail.
template <class PT>
void bin_species_t(pic_ctx* c, int s) {
  hipStream_t st = c->stream;
  const long long nt = c->ntiles;
  // Electrons and Cu+ keep tile ranges; Cu atoms and Cu2+ bin as one list.
  const bool tiled = s == 0 || s == 2;
  uint32_t* ts_old = ts_cur(c, s);
  uint32_t* ts_new = c->tsb[s][c->tcur[s] ^ 1];
  const long long first = tiled ? c->n_binned[s] : 0;
  // Destination counts of the binned ranges: taken by the tile push of this
  // step, else (after a load or a restore) from the keys.
  unsigned* cursor = c->tile_cursor;
  if (tiled && c->tcounted) {
    cursor = c->tcnt[s == 0 ? 0 : 1];
  } else {
    hipMemsetAsync(cursor, 0, (nt + 1) * sizeof(unsigned), st);
    if (tiled)
      k_bin_hist_tile<<<(unsigned)c->nch_bound, kT, 0, st>>>(
          c->key[s], ts_old, c->chunks, c->cstart + nt, cursor, c->g);
  }
  const long long tail = std::max(0ll, bound(c, s) - first);
  if (tail > 0)
    k_bin_hist_list<<<(unsigned)((tail + kLChunk - 1) / kLChunk), kT, 0, st>>>(
        c->key[s], cursor, c->g, first, &c->dc->n[s]);
  const long long nsb = (nt + 1 + kScanPer - 1) / kScanPer;
  k_scan_blocks<<<(unsigned)nsb, kT, 0, st>>>(cursor, nt, c->scan_block);
  k_scan1<<<1, 1024, 0, st>>>(c->scan_block, c->scan_block + nsb + 1, nsb);
  k_scan_apply<<<(unsigned)nsb, kT, 0, st>>>(cursor, nt,
                                             c->scan_block + nsb + 1, ts_new,
                                             cursor);
  const int o = c->cur[s] ^ 1;
  if (tiled)
    k_bin_scatter_tile<PT><<<(unsigned)c->nch_bound, kT, 0, st>>>(
        cur<PT>(c, s), buf<PT>(c, s, o), c->key[s], ts_old, c->chunks,
        c->cstart + nt, cursor, c->g);
  if (tail > 0)
    k_bin_scatter_list<PT><<<(unsigned)((tail + kLChunk - 1) / kLChunk), kT, 0, st>>>(
        cur<PT>(c, s), buf<PT>(c, s, o), c->key[s], cursor, c->g,
        first, &c->dc->n[s]);
  k_set_count<<<1, 1, 0, st>>>(c->dc, s, ts_new, nt);
  c->cur[s] = o;
  c->tcur[s] ^= 1;
}

// In-place removal of the dead neutrals (key kDead: ionised or absorbed).
// With n entries of which D are dead, the dead ones below n - D (holes) and
// the live ones at or above it (movers) are equally many; the j-th mover in
// list order fills the j-th hole.  Three light passes over the keys and a
// copy of the movers replace the full scatter of a binning pass.
// Each workgroup scans kCChunk keys (kCPer per thread, coalesced); the
// counts are aggregated per workgroup so that the shared counters take one
// atomic per workgroup, not one per wave.
constexpr int kCPer = 16;
constexpr int kCChunk = kCPer * kT;

__global__ void __launch_bounds__(kT) k_count_dead(
    const uint32_t* __restrict__ key, Counters* dc) {
  __shared__ unsigned sw[kT / 64];
  const long long n = (long long)dc->n[1];
  const long long b0 = blockIdx.x * (long long)kCChunk;
  if (b0 >= n) return;
  unsigned d = 0;  // wave-uniform
#pragma unroll
  for (int r = 0; r < kCPer; ++r) {
    const long long i = b0 + r * kT + threadIdx.x;
    const uint32_t k = key[i < n ? i : n - 1];
    d += (unsigned)__popcll(__ballot(i < n && k == kDead));
  }
  if (lane_id() == 0) sw[threadIdx.x / 64] = d;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned t = 0;
    for (int w = 0; w < kT / 64; ++w) t += sw[w];
    if (t) atomicAdd(&dc->n_dead, (unsigned long long)t);
  }
}

__global__ void __launch_bounds__(kT) k_compact_lists(
    const uint32_t* __restrict__ key, uint32_t* __restrict__ holes,
    uint32_t* __restrict__ movers, Counters* dc) {
  __shared__ unsigned sh[kT / 64], sm[kT / 64];
  __shared__ unsigned long long base[2];
  const long long n = (long long)dc->n[1];
  const long long keep = n - (long long)dc->n_dead;
  const long long b0 = blockIdx.x * (long long)kCChunk;
  if (b0 >= n || keep == n) return;
  unsigned long long mh[kCPer], mm[kCPer];
  unsigned th = 0, tm = 0;  // wave-uniform
#pragma unroll
  for (int r = 0; r < kCPer; ++r) {
    const long long i = b0 + r * kT + threadIdx.x;
    const bool dead = key[i < n ? i : n - 1] == kDead;
    mh[r] = __ballot(i < n && dead && i < keep);
    mm[r] = __ballot(i < n && !dead && i >= keep);
    th += (unsigned)__popcll(mh[r]);
    tm += (unsigned)__popcll(mm[r]);
  }
  const int w = threadIdx.x / 64;
  if (lane_id() == 0) {
    sh[w] = th;
    sm[w] = tm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned h = 0, m = 0;
    for (int q = 0; q < kT / 64; ++q) {
      const unsigned a = sh[q], b = sm[q];
      sh[q] = h;
      sm[q] = m;
      h += a;
      m += b;
    }
    base[0] = h ? atomicAdd(&dc->n_holes, (unsigned long long)h) : 0ull;
    base[1] = m ? atomicAdd(&dc->n_movers, (unsigned long long)m) : 0ull;
  }
  __syncthreads();
  unsigned long long oh = base[0] + sh[w], om = base[1] + sm[w];
#pragma unroll
  for (int r = 0; r < kCPer; ++r) {
    const uint32_t i = (uint32_t)(b0 + r * kT + threadIdx.x);
    if ((mh[r] >> lane_id()) & 1ull) holes[oh + lanes_below(mh[r])] = i;
    if ((mm[r] >> lane_id()) & 1ull) movers[om + lanes_below(mm[r])] = i;
    oh += (unsigned)__popcll(mh[r]);
    om += (unsigned)__popcll(mm[r]);
  }
}

template <class PT>
__global__ void k_compact_move(PT p, uint32_t* __restrict__ key,
                               const uint32_t* __restrict__ holes,
                               const uint32_t* __restrict__ movers,
                               Counters* dc) {
  // The two lists are equally long; the minimum only guards the reads.
  const long long h = (long long)min(dc->n_holes, dc->n_movers);
  for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < h;
       j += (long long)gridDim.x * blockDim.x) {
    const uint32_t from = movers[j], to = holes[j];
    Acc<PT>::copy(p, from, p, to);
    key[to] = key[from];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const unsigned long long k = dc->n[1] - dc->n_dead;
    dc->n[1] = k;
    dc->sorted_n[1] = k;
  }
}

template <class PT>
void compact_neutrals_t(pic_ctx* c) {
  hipStream_t st = c->stream;
  const long long nb = (bound(c, 1) + kCChunk - 1) / kCChunk;
  uint32_t* holes = c->cmp_idx;
  uint32_t* movers = c->cmp_idx + c->cfg.capacity[1];
  k_count_dead<<<(unsigned)nb, kT, 0, st>>>(c->key[1], c->dc);
  k_compact_lists<<<(unsigned)nb, kT, 0, st>>>(c->key[1], holes, movers, c->dc);
  k_compact_move<PT><<<1024, kT, 0, st>>>(
      cur<PT>(c, 1), c->key[1], holes, movers, c->dc);
}

}  // namespace

void sort_event_records(pic_ctx* c, Rec* a, unsigned long long* count) {
  sort_records(c, a, c->rec_tmp, count, c->cfg.max_events);
}

void parts_md_return(pic_ctx* c, double lattice_a, unsigned mask,
                     double* pos, double* vel, uint64_t* ids, int32_t* sp,
                     long long nout) {
  long long nab = (long long)c->hc.n_ab;
  if (nab > c->cfg.max_events) nab = c->cfg.max_events;
  const double off3a = 3.0 * lattice_a;
  long long first = 0, out0 = 0;
  for (int s = 0; s < 4; ++s) {
    const long long n = (long long)c->hc.cathode[s];
    if ((mask >> s) & 1u) {
      if (n > 0)
        k_md_return<<<(unsigned)std::min<long long>((n + kT - 1) / kT, 1024),
                      kT, 0, c->stream>>>(c->ab_species, c->ab_id, c->ab_pos,
                                          c->ab_vel, nab, first, n, off3a,
                                          c->g, pos, vel, ids, sp, out0, nout);
      out0 += n;
    }
    first += n;
  }
}

void parts_deposit(pic_ctx* c) {
  tmark(c, PIC_PH_DEPOSIT, true);
  if (c->acc_next_valid) {
    // The last advance pushed the current particles and added their charge.
    std::swap(c->acc, c->acc_next);
    c->acc_next_valid = false;
  } else {
    hipMemsetAsync(c->acc, 0, c->nnodes * sizeof(long long), c->stream);
    if (c->mixed)
      deposit_t<PartsM>(c);
    else
      deposit_t<Parts>(c);
  }
  tmark(c, PIC_PH_DEPOSIT, false);
}

void parts_sources_host(pic_ctx* c) {
  tmark(c, PIC_PH_SOURCES, true);
  if (c->mixed)
    sources_host_t<PartsM>(c);
  else
    sources_host_t<Parts>(c);
  tmark(c, PIC_PH_SOURCES, false);
}

void parts_sources_fn(pic_ctx* c, double dt) {
  tmark(c, PIC_PH_SOURCES, true);
  if (c->mixed)
    sources_fn_t<PartsM>(c, dt);
  else
    sources_fn_t<Parts>(c, dt);
  tmark(c, PIC_PH_SOURCES, false);
}

long long neutral_push_blocks(long long n) {
  return (n > 0 ? n : 1) / kNChunk + 1;
}

void parts_push_neutral(pic_ctx* c, double dt) {
  if (c->mixed)
    push_neutral_t<PartsM>(c, dt);
  else
    push_neutral_t<Parts>(c, dt);
}

void parts_push_collide(pic_ctx* c, double dt) {
  if (c->mixed)
    push_collide_t<PartsM>(c, dt);
  else
    push_collide_t<Parts>(c, dt);
}

void parts_bin_species(pic_ctx* c, int s) {
  if (c->mixed)
    bin_species_t<PartsM>(c, s);
  else
    bin_species_t<Parts>(c, s);
}

// Chunk list of the current tile ranges of electrons and ions (one chunk
// covers up to kChunk of each).  hb: host bound of the particles the ranges
// cover (for the launch bounds).
void parts_chunks(pic_ctx* c, const long long hb[3]) {
  hipStream_t st = c->stream;
  const long long nt = c->ntiles;
  const long long nsb = (nt + 1 + kScanPer - 1) / kScanPer;
  k_chunk_count<<<nblk(nt), kT, 0, st>>>(ts_cur(c, 0), ts_cur(c, 2), nt,
                                         c->tile_cursor);
  k_scan_blocks<<<(unsigned)nsb, kT, 0, st>>>(c->tile_cursor, nt, c->scan_block);
  k_scan1<<<1, 1024, 0, st>>>(c->scan_block, c->scan_block + nsb + 1, nsb);
  k_scan_apply<<<(unsigned)nsb, kT, 0, st>>>(c->tile_cursor, nt,
                                             c->scan_block + nsb + 1, c->cstart,
                                             c->cstart);
  k_chunk_fill<<<nblk(nt), kT, 0, st>>>(c->cstart, nt, c->chunks);
  c->nch_bound = std::min<long long>(nt + (hb[0] + hb[2]) / kChunk + 2, c->nch_cap);
}

// In-place removal of a step's few removed particles of species s (listed
// as they were removed): with n particles of which D are removed, each
// listed index below n - D is filled by one of the live particles at or
// above it (equally many), and the tile ranges ts, if given, are cut at
// n - D.  A filled slot may hold a particle of another tile; the pushes and
// the deposit treat such particles correctly.  One workgroup pairs the
// holes with the movers; the copies are k_remove_pairs'.
__global__ void __launch_bounds__(1024) k_remove_listed(
    const uint32_t* __restrict__ key, const uint32_t* __restrict__ list,
    const unsigned long long* __restrict__ ndead, int s,
    uint32_t* __restrict__ ts, long long nt, uint2* __restrict__ pairs,
    Counters* dc) {
  __shared__ uint32_t holes[kDeadList], movers[kDeadList];
  __shared__ unsigned nh, nm;
  const long long n = (long long)dc->n[s];
  const long long D = (long long)*ndead;
  if (D > kDeadList || D > n) {   // (the caller bins instead)
    if (threadIdx.x == 0) dc->n_pairs = 0;
    return;
  }
  const long long keep = n - D;
  if (threadIdx.x == 0) nh = nm = 0;
  __syncthreads();
  for (long long j = threadIdx.x; j < D; j += blockDim.x) {
    const uint32_t q = list[j];
    if ((long long)q < keep) holes[atomicAdd(&nh, 1u)] = q;
  }
  for (long long q = keep + threadIdx.x; q < n; q += blockDim.x)
    if (key[q] != kDead) movers[atomicAdd(&nm, 1u)] = (uint32_t)q;
  __syncthreads();
  // The copies run in k_remove_pairs, spread over the GPU.
  const unsigned np = nh < nm ? nh : nm;
  for (unsigned j = threadIdx.x; j < np; j += blockDim.x)
    pairs[j] = make_uint2(holes[j], movers[j]);
  if (ts)
    for (long long t = threadIdx.x; t <= nt; t += blockDim.x)
      if ((long long)ts[t] > keep) ts[t] = (uint32_t)keep;
  if (threadIdx.x == 0) {
    if (nh != nm) atomicOr(&dc->err, kErrCapacity);  // (cannot happen)
    dc->n[s] = (unsigned long long)keep;
    dc->sorted_n[s] = (unsigned long long)keep;
    dc->n_pairs = np;
  }
}

// Mover j into hole j.  Holes lie below the new count and movers at or
// above it: no copy reads a slot another writes.
template <class PT>
__global__ void k_remove_pairs(PT p, uint32_t* __restrict__ key,
                               const uint2* __restrict__ pairs,
                               const Counters* __restrict__ dc) {
  const unsigned j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= dc->n_pairs) return;
  const uint2 hm = pairs[j];
  Acc<PT>::copy(p, hm.y, p, hm.x);
  key[hm.x] = key[hm.y];
}

template <class PT>
void remove_listed_t(pic_ctx* c, int s, uint32_t* list,
                     const unsigned long long* ndead, uint32_t* ts) {
  k_remove_listed<<<1, 1024, 0, c->stream>>>(c->key[s], list, ndead, s, ts,
                                             c->ntiles, c->rm_pairs, c->dc);
  k_remove_pairs<PT><<<kDeadList / 64, 64, 0, c->stream>>>(
      cur<PT>(c, s), c->key[s], c->rm_pairs, c->dc);
}

// Ions move about 1e-5 cells per step: binning them every step would copy
// ten million records to file a few thousand new ones.  The ions that left
// the domain this step (a few) are removed in place instead, and the ions
// are binned again only when the ions out of tile order (the unbinned tail
// of new ions, those moved into removed ones' slots, and every binned ion
// that has crossed a tile face since the last pass) exceed kIonLazy plus
// 1/1024 of them, or when more than kDeadList left at once.  The pushes
// handle ions out of tile order correctly, only more slowly: the unbinned
// tail costs about 0.7 ns per ion and step, so with a few thousand new ions
// per step a bound of a few ten thousand balances its growth against one
// binning pass.  The decision reads this step's counters, copied as soon as
// the collisions are done, while the electrons bin.
constexpr long long kIonLazy = 1 << 15;

void parts_bin(pic_ctx* c) {
  hipStream_t st = c->stream;
  tmark(c, PIC_PH_BIN, true);
  hipMemcpyAsync(c->hmid, c->dc, sizeof(Counters), hipMemcpyDeviceToHost, st);
  hipEventRecord(c->ev_mid, st);
  parts_bin_species(c, 0);
  bool bin_ions = true, listed1 = false;
  if (hipEventSynchronize(c->ev_mid) == hipSuccess) {
    listed1 = c->hmid->err == 0 && c->hmid->n_dead1 <= (unsigned long long)kDeadList;
    const Counters& h = *c->hmid;
    const long long n2 = (long long)h.n[2];
    const long long tail = n2 - c->n_binned[2];
    c->ion_moved_accum += (long long)h.ion_moved;
    const long long dead = (long long)h.n_dead2;
    const long long bound2 = kIonLazy + c->n_binned[2] / 1024;
    bin_ions = h.err != 0 || tail < 0 || dead > kDeadList ||
               c->ion_moved_accum + tail + dead > bound2;
    if (!bin_ions) {
      if (dead > 0) {
        if (c->mixed)
          remove_listed_t<PartsM>(c, 2, c->dead2, &c->dc->n_dead2, ts_cur(c, 2));
        else
          remove_listed_t<Parts>(c, 2, c->dead2, &c->dc->n_dead2, ts_cur(c, 2));
        c->ion_moved_accum += dead;
      }
      // Exact: nothing else changes the ions until the next step.
      c->n[2] = n2 - dead;
      c->n_binned[2] = std::min(c->n_binned[2], c->n[2]);
    }
  }
  c->ions_binned = bin_ions;
  if (bin_ions) {
    parts_bin_species(c, 2);
    c->ion_moved_accum = 0;
  }
  // Cu2+ (few): binned as one list every step, which drops the removed.
  if (bound(c, 3) > 0) parts_bin_species(c, 3);
  c->tcounted = false;
  // Nothing reads the neutrals by tile (their push streams them, their
  // cell counts are kept from step to step, the event cells are a bit mask
  // in L2), so they are only compacted: a full binning pass of five
  // million records through the unbinned-list path cost 2.3 ms.  The few
  // thousand removed this step (ionised, absorbed) are listed, so one
  // workgroup fills their slots; with more, the scans over all keys do.
  if (listed1) {
    if (c->mixed)
      remove_listed_t<PartsM>(c, 1, c->dead1, &c->dc->n_dead1, nullptr);
    else
      remove_listed_t<Parts>(c, 1, c->dead1, &c->dc->n_dead1, nullptr);
  } else if (c->mixed) {
    compact_neutrals_t<PartsM>(c);
  } else {
    compact_neutrals_t<Parts>(c);
  }
  long long hb[3];
  for (int s = 0; s < 3; ++s) hb[s] = bound(c, s);
  parts_chunks(c, hb);
  tmark(c, PIC_PH_BIN, false);
}

void parts_load(pic_ctx* c, int s, long long n, const double* pos,
                const double* vel, const uint64_t* ids) {
  if (n <= 0) return;
  if (c->mixed)
    k_load<PartsM><<<nblk(n), kT, 0, c->stream>>>(cur<PartsM>(c, s), pos, vel,
                                                   ids, c->key[s], n, c->g,
                                                   c->dc);
  else
    k_load<Parts><<<nblk(n), kT, 0, c->stream>>>(cur<Parts>(c, s), pos, vel,
                                                 ids, c->key[s], n, c->g,
                                                 c->dc);
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

int parts_arrays(pic_ctx* c, int s, void** ptr, size_t* elem) {
  if (c->mixed) {
    PartsM p = cur<PartsM>(c, s);
    void* a[8] = {p.cell, p.ox, p.oy, p.oz, p.vx, p.vy, p.vz, p.id};
    const size_t e[8] = {4, 4, 4, 4, 4, 4, 4, 8};
    for (int k = 0; k < 8; ++k) { ptr[k] = a[k]; elem[k] = e[k]; }
    return 8;
  }
  Parts p = cur<Parts>(c, s);
  void* a[7] = {p.x, p.y, p.z, p.vx, p.vy, p.vz, p.id};
  for (int k = 0; k < 7; ++k) { ptr[k] = a[k]; elem[k] = 8; }
  return 7;
}

void parts_restore_keys(pic_ctx* c, int s, long long n) {
  if (n <= 0) return;
  if (c->mixed)
    k_restore_keys<<<nblk(n), kT, 0, c->stream>>>(cur<PartsM>(c, s), c->key[s], n,
                                                  c->g, c->dc);
  else
    k_restore_keys<<<nblk(n), kT, 0, c->stream>>>(cur<Parts>(c, s), c->key[s], n,
                                                  c->g, c->dc);
}

void parts_read(pic_ctx* c, int s, long long n, double* pos, double* vel,
                uint64_t* ids) {
  if (n <= 0) return;
  if (c->mixed)
    k_read<PartsM><<<nblk(n), kT, 0, c->stream>>>(cur<PartsM>(c, s), pos, vel,
                                                   ids, n, c->g);
  else
    k_read<Parts><<<nblk(n), kT, 0, c->stream>>>(cur<Parts>(c, s), pos, vel,
                                                 ids, n, c->g);
}

}  // namespace pic
