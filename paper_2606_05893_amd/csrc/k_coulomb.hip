// Coulomb collisions by binary pairing within cells (Takizuka & Abe), the
// collision model the paper cites for its Monte Carlo collisions.
//
// The charged particles are grouped by cell: a count per cell (one pass over
// the keys), an exclusive scan, and a scatter of one 16-byte record per
// particle (species in the top bit of the sort key, below it the 53-bit
// order draw of (id, step)) into its cell's segment.  Cells are numbered
// tile by tile, so that the cells of a tile, whose particles share one range
// of the tile-binned arrays, are served together.  A cell's records are then
// put in (key, id) order, which gives each species a random order that
// does not depend on where the particles sit in memory; consecutive
// particles of a species pair, an odd count leaves a triplet of half-weight
// collisions, and the electrons and ions of the cell collide in a sequence
// of max(N_e, N_i) collisions.
//
// Most cells hold a few charged particles.  The scatter copies each
// particle's velocity and id beside its record; a thread per record then
// finds the record's rank in its cell's order (by comparison with the
// others of the segment) and writes the copy, with the work it leads (a
// like pair or triplet, or an electron-ion chain), to its sorted place.
// The work is gathered into one list by class (pairs, triplets, chains of
// one, two, more collisions), the like collisions run a thread per pair on
// the copies, then the electron-ion collisions a thread per chain (the t-th
// particle of the smaller group with the larger group's t-th, (t+m)-th, ...
// particles; the chains share no particle, so they equal the sequence of
// the definition), and the copies go back to the particle arrays in the
// particles' order.  Crowded cells (more than kSmallCell records) go to a
// list served by one workgroup each: an LDS sort, the like pairs in
// parallel, and the electron-ion sequence in rounds of min(N_e, N_i)
// collisions, each round touching every particle at most once.
#include <cmath>

#include "cell_groups.h"
#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kSmallCell = 16;
constexpr int kBigT = 256;
constexpr int kCoulBigCell = 2048;    // records a crowded cell may hold
constexpr unsigned long long kSpBit = 1ull << 63;
constexpr int kScanB = 1024;          // cells per scan block
constexpr int kNC = 5;                // classes of the work list
constexpr int kCB = 2048;             // places per work-counting block
constexpr unsigned kNoCopy = 0xFFFFFFFFu;  // sorted place without a copy

enum : uint32_t {
  kTagOrder = 20, kTagDelta = 21, kTagPhi = 22, kTagDeltaEI = 23, kTagPhiEI = 24
};

// Pair types: 0 electron-electron, 1 ion-ion, 2 electron-ion.
struct CoulC {
  double w_dx3;
  double cvar[3];     // e^4 lnL dt / (8 pi eps0^2 m_r^2): <delta^2> = cvar n / u^3
  double a1[3], a2[3];  // m_r / m1, m_r / m2
  unsigned step;
  unsigned long long seed;
};

// 53-bit integer of the order draw of (id, step).
__device__ __forceinline__ unsigned long long order_key(unsigned long long id,
                                                        unsigned step,
                                                        unsigned long long seed) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32), c2 = step,
           c3 = kTagOrder;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((unsigned long long)c0 << 21) ^ (unsigned long long)(c1 >> 11);
}

template <class PT>
struct Sp2 {
  PT p[2];                             // electrons, ions
};

template <class PT>
__device__ __forceinline__ void get_v(const Sp2<PT>& S, int s, unsigned i,
                                      double& vx, double& vy, double& vz) {
  Acc<PT>::vel(S.p[s], i, vx, vy, vz);
}

template <class PT>
__device__ __forceinline__ void set_v(const Sp2<PT>& S, int s, unsigned i,
                                      double vx, double vy, double vz) {
  Acc<PT>::set_vel(S.p[s], i, vx, vy, vz);
}

// One binary collision of a pair of type ty on the velocities v1 and v2, in
// place: delta normal with the stated variance (halved in a triplet), phi
// uniform; the relative velocity turns by theta = 2 atan(delta) about
// itself.  Returns false (nothing changed) for zero relative speed.
__device__ bool pair_kick(double* v1, double* v2, int ty, double n, bool half,
                          unsigned long long id_c, uint32_t tag_d,
                          uint32_t tag_p, const CoulC& k) {
  const double ux = v1[0] - v2[0], uy = v1[1] - v2[1], uz = v1[2] - v2[2];
  const double u = sqrt((ux * ux + uy * uy) + uz * uz);
  if (!(u > 0.0)) return false;
  double var = (k.cvar[ty] * n) / ((u * u) * u);
  if (half) var = 0.5 * var;
  double u1, u2, u3, u4;
  uniform2(id_c, k.step, tag_d, k.seed, u1, u2);
  uniform2(id_c, k.step, tag_p, k.seed, u3, u4);
  const double g = sqrt(-2.0 * log(1.0 - u1)) * cospi(2.0 * u2);
  const double delta = sqrt(var) * g;
  const double uperp = sqrt(ux * ux + uy * uy);
  const double d2 = delta * delta;
  const double inv = 1.0 / (1.0 + d2);
  const double s = (2.0 * delta) * inv;
  const double omc = (2.0 * d2) * inv;
  double sp, cp;
  sincospi(2.0 * u3, &sp, &cp);
  double dux, duy, duz;
  if (uperp > 0.0) {
    const double iu = 1.0 / uperp;
    dux = ((((ux * iu) * uz) * s) * cp - (((uy * iu) * u) * s) * sp) - ux * omc;
    duy = ((((uy * iu) * uz) * s) * cp + (((ux * iu) * u) * s) * sp) - uy * omc;
    duz = (-(uperp * s)) * cp - uz * omc;
  } else {
    dux = (u * s) * cp;
    duy = (u * s) * sp;
    duz = -(uz * omc);
  }
  const double a1 = k.a1[ty], a2 = k.a2[ty];
  v1[0] = v1[0] + a1 * dux;
  v1[1] = v1[1] + a1 * duy;
  v1[2] = v1[2] + a1 * duz;
  v2[0] = v2[0] - a2 * dux;
  v2[1] = v2[1] - a2 * duy;
  v2[2] = v2[2] - a2 * duz;
  return true;
}

// The same collision on particle a (species sa) and b (sb) in their arrays.
template <class PT>
__device__ void collide(const Sp2<PT>& S, int sa, unsigned a, int sb,
                        unsigned b, double n, bool half,
                        unsigned long long id_c, uint32_t tag_d,
                        uint32_t tag_p, const CoulC& k) {
  double v1[3], v2[3];
  get_v(S, sa, a, v1[0], v1[1], v1[2]);
  get_v(S, sb, b, v2[0], v2[1], v2[2]);
  if (pair_kick(v1, v2, sa == sb ? sa : 2, n, half, id_c, tag_d, tag_p, k)) {
    set_v(S, sa, a, v1[0], v1[1], v1[2]);
    set_v(S, sb, b, v2[0], v2[1], v2[2]);
  }
}

// A particle's velocity and id, copied into its cell-sorted place.
struct PV {
  double v[3];
  unsigned long long id;
};

// The collision on two such copies.
__device__ __forceinline__ void collide_pv(PV* __restrict__ pv, unsigned a,
                                           unsigned b, int ty,
                                           double n, bool half,
                                           unsigned long long id_c,
                                           uint32_t tag_d, uint32_t tag_p,
                                           const CoulC& k) {
  double v1[3] = {pv[a].v[0], pv[a].v[1], pv[a].v[2]};
  double v2[3] = {pv[b].v[0], pv[b].v[1], pv[b].v[2]};
  if (pair_kick(v1, v2, ty, n, half, id_c, tag_d, tag_p, k)) {
    pv[a].v[0] = v1[0]; pv[a].v[1] = v1[1]; pv[a].v[2] = v1[2];
    pv[b].v[0] = v2[0]; pv[b].v[1] = v2[1]; pv[b].v[2] = v2[2];
  }
}

// A record's hi word holds its cell above two species bits.
__device__ __forceinline__ unsigned rec_sp(const Rec& r) { return r.hi & 3u; }
__device__ __forceinline__ unsigned rec_cell(const Rec& r) { return r.hi >> 2; }

template <class PT>
__device__ __forceinline__ unsigned long long rec_id(const Sp2<PT>& S,
                                                     const Rec& r) {
  return S.p[rec_sp(r)].id[r.val];
}

template <class PT>
__device__ __forceinline__ bool rec_before(const Sp2<PT>& S, const Rec& a,
                                           const Rec& b) {
  return a.lo < b.lo || (a.lo == b.lo && rec_id(S, a) < rec_id(S, b));
}

// ---- grouping ----------------------------------------------------------------
__global__ void k_cg_count(const uint32_t* __restrict__ ke,
                           const uint32_t* __restrict__ ki,
                           const Counters* dc, GridC g,
                           unsigned* __restrict__ cnt) {
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  long long lo, hi;
  block_range(ne + ni, lo, hi);
  for (long long t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const uint32_t c = t < ne ? ke[t] : ki[t - ne];
    if (c != kDead) atomicAdd(&cnt[tile_major(c, g)], 1u);
  }
}

// Inclusive scan of each block of kScanB counts, block totals to bsum.
__global__ void __launch_bounds__(kScanB) k_cg_scan_blocks(
    const unsigned* __restrict__ cnt, long long n, unsigned* __restrict__ off,
    unsigned* __restrict__ bsum) {
  __shared__ unsigned s[kScanB];
  const long long i = (long long)blockIdx.x * kScanB + threadIdx.x;
  s[threadIdx.x] = i < n ? cnt[i] : 0u;
  __syncthreads();
  for (int o = 1; o < kScanB; o <<= 1) {
    const unsigned v = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  if (i < n) off[i + 1] = s[threadIdx.x];
  if (threadIdx.x == kScanB - 1) bsum[blockIdx.x] = s[kScanB - 1];
}

// Exclusive scan of the block totals (one workgroup).
__global__ void __launch_bounds__(1024) k_cg_scan_sums(unsigned* __restrict__ bsum,
                                                        int nb) {
  __shared__ unsigned s[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  unsigned tot = 0;
  for (int q = 0; q < per && b0 + q < nb; ++q) tot += bsum[b0 + q];
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned v = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned run = s[threadIdx.x] - tot;
  for (int q = 0; q < per && b0 + q < nb; ++q) {
    const unsigned v = bsum[b0 + q];
    bsum[b0 + q] = run;
    run += v;
  }
}

__global__ void __launch_bounds__(kScanB) k_cg_scan_apply(
    unsigned* __restrict__ off, long long n, const unsigned* __restrict__ bsum) {
  const long long i = (long long)blockIdx.x * kScanB + threadIdx.x;
  if (i == 0) off[0] = 0u;
  if (i < n) off[i + 1] += bsum[blockIdx.x];
}

// One record per live charged particle into its cell's segment (order
// inside the segment arbitrary; the cell pass sorts it), with a copy of the
// particle's velocity and id beside it; each particle notes its slot.
template <class PT>
__global__ void k_cg_scatter(Sp2<PT> S, const uint32_t* __restrict__ ke,
                             const uint32_t* __restrict__ ki,
                             const Counters* dc, GridC g,
                             const unsigned* __restrict__ off,
                             unsigned* __restrict__ cnt, Rec* __restrict__ rec,
                             PV* __restrict__ pvu, unsigned* __restrict__ slot_of,
                             unsigned step, unsigned long long seed) {
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  long long lo, hi;
  block_range(ne + ni, lo, hi);
  for (long long t = lo + threadIdx.x; t < hi; t += blockDim.x) {
    const int s = t < ne ? 0 : 1;
    const unsigned i = (unsigned)(s ? t - ne : t);
    const uint32_t c0 = s ? ki[i] : ke[i];
    if (c0 == kDead) {
      slot_of[t] = kNoCopy;
      continue;
    }
    const unsigned c = tile_major(c0, g);
    const unsigned slot = off[c] + atomicSub(&cnt[c], 1u) - 1u;
    const unsigned long long id = S.p[s].id[i];
    Rec r;
    r.lo = (s ? kSpBit : 0ull) | order_key(id, step, seed);
    r.hi = (c << 2) | (unsigned)s;
    r.val = i;
    rec[slot] = r;
    PV x;
    get_v(S, s, i, x.v[0], x.v[1], x.v[2]);
    x.id = id;
    pvu[slot] = x;
    slot_of[t] = slot;
  }
}

// Cells of at most kSmallCell records, one thread per record: the record's
// rank in its cell's (key, id) order places it in the sorted array, and at
// that place goes the work it leads, if any.  Like collisions: the first of
// each consecutive pair of its species (after a leading triplet when the
// species count is odd; the triplet's first leads it).  Electron-ion
// collisions: K = max(N_e, N_i) in sequence, collision j between electron
// j mod N_e and ion j mod N_i.  Every particle of the larger group takes
// part once, the t-th of the smaller group (m of them) in collisions t,
// t + m, ...: m independent chains, each led by its smaller-group record.
// Every place of the sorted array gets its two work words (zero: none); the
// first record of a crowded cell lists the cell for the workgroup pass.
__global__ void __launch_bounds__(kT) k_cg_rank(
    const unsigned* __restrict__ off, long long ncells,
    const Rec* __restrict__ rec, const PV* __restrict__ pvu,
    PV* __restrict__ pv, unsigned* __restrict__ place_at,
    unsigned* __restrict__ big, long long big_cap, unsigned* __restrict__ nbig,
    uint2* __restrict__ like_w, uint2* __restrict__ ei_w) {
  long long lo, hi;
  block_range((long long)off[ncells], lo, hi);
  for (long long p = lo + threadIdx.x; p < hi; p += kT) {
    const Rec r = rec[p];
    const unsigned c = rec_cell(r);
    const unsigned b = off[c];
    const int n = (int)(off[c + 1] - b);
    uint2 li = make_uint2(0u, 0u), eit = make_uint2(0u, 0u);
    long long place = p;
    unsigned pl = kNoCopy;
    if (n > kSmallCell) {
      if ((unsigned)p == b) {
        const unsigned slot = atomicAdd(nbig, 1u);
        if ((long long)slot < big_cap) big[slot] = c;
      }
    } else if (n >= 2) {
      const PV me = pvu[p];
      int rank = 0, ne = 0;
      for (int j = 0; j < n; ++j) {
        const Rec x = rec[b + j];
        ne += rec_sp(x) == 0u;
        rank += (b + (unsigned)j != (unsigned)p) &&
                (x.lo < r.lo || (x.lo == r.lo && pvu[b + j].id < me.id));
      }
      place = (long long)b + rank;
      pv[place] = me;
      pl = (unsigned)place;
      const unsigned s = rec_sp(r);
      const int ni = n - ne;
      const int q = s ? rank - ne : rank;           // rank within the species
      const int N = s ? ni : ne;
      const int start = (N & 1) ? 3 : 0;
      const bool trip = (N & 1) && q == 0;
      const bool lead =
          N >= 2 && (trip || (q >= start && ((q - start) & 1) == 0 && q + 1 < N));
      const bool chain = ne > 0 && ni > 0 && s == (ne <= ni ? 0u : 1u);
      // Both words by selection, not by a branch around the assignment: the
      // branch form of this code was compiled to a wrong first word.
      li.x = lead ? (unsigned)place : 0u;
      li.y = lead ? ((unsigned)N | (trip ? 1u << 30 : 0u) | (s << 31)) : 0u;
      eit.x = chain ? b : 0u;
      eit.y = chain ? ((unsigned)q | ((unsigned)ne << 8) | ((unsigned)ni << 16)) : 0u;
    }
    place_at[p] = pl;
    like_w[place] = li;
    ei_w[place] = eit;
  }
}

// The copies of the small cells' particles back into their arrays, in the
// particles' order.
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_writeback(
    Sp2<PT> S, const Counters* dc, const unsigned* __restrict__ slot_of,
    const unsigned* __restrict__ place_at, const PV* __restrict__ pv) {
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  long long lo, hi;
  block_range(ne + ni, lo, hi);
  for (long long t = lo + threadIdx.x; t < hi; t += kT) {
    const unsigned slot = slot_of[t];
    if (slot == kNoCopy) continue;
    const unsigned pl = place_at[slot];
    if (pl == kNoCopy) continue;
    const int s = t < ne ? 0 : 1;
    const unsigned i = (unsigned)(s ? t - ne : t);
    set_v(S, s, i, pv[pl].v[0], pv[pl].v[1], pv[pl].v[2]);
  }
}

// ---- work lists ----------------------------------------------------------
// The work words are gathered into one list ordered by class, so that a
// wavefront runs one kind of work: like pairs, like triplets, then electron-
// ion chains of one, two, and three or more collisions.  A count per block
// of kCB places, an exclusive scan of the class-major counts, and a scatter
// in place order (ballots within each wavefront): deterministic, without
// contended atomics.
__device__ __forceinline__ int like_class(uint2 w) {
  return w.y == 0u ? -1 : (((w.y >> 30) & 1u) ? 1 : 0);
}

__device__ __forceinline__ int ei_class(uint2 w) {
  if (w.y == 0u) return -1;
  const int t = (int)(w.y & 0xFFu), ne = (int)((w.y >> 8) & 0xFFu),
            ni = (int)(w.y >> 16);
  const int K = ne > ni ? ne : ni, m = ne < ni ? ne : ni;
  const int len = (K - t + m - 1) / m;
  return len == 1 ? 2 : (len == 2 ? 3 : 4);
}

__global__ void __launch_bounds__(kT) k_cg_wcount(
    const unsigned* __restrict__ off, long long ncells,
    const uint2* __restrict__ like_w, const uint2* __restrict__ ei_w,
    unsigned* __restrict__ bcnt, int G) {
  __shared__ unsigned sc[kNC];
  if (threadIdx.x < kNC) sc[threadIdx.x] = 0u;
  __syncthreads();
  const long long nrec = (long long)off[ncells];
  const long long p0 = (long long)blockIdx.x * kCB;
  for (int i = 0; i < kCB / kT; ++i) {
    const long long p = p0 + i * kT + threadIdx.x;
    if (p >= nrec) break;
    const int lc = like_class(like_w[p]), ec = ei_class(ei_w[p]);
    if (lc >= 0) atomicAdd(&sc[lc], 1u);
    if (ec >= 0) atomicAdd(&sc[ec], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kNC) bcnt[threadIdx.x * G + blockIdx.x] = sc[threadIdx.x];
}

__global__ void __launch_bounds__(kT) k_cg_wscatter(
    const unsigned* __restrict__ off, long long ncells,
    const uint2* __restrict__ like_w, const uint2* __restrict__ ei_w,
    const unsigned* __restrict__ loff, int G, uint2* __restrict__ list) {
  constexpr int kW = kT / 64;
  __shared__ unsigned base[kNC];
  __shared__ unsigned wsum[kW][kNC];
  if (threadIdx.x < kNC) base[threadIdx.x] = loff[threadIdx.x * G + blockIdx.x];
  __syncthreads();
  const long long nrec = (long long)off[ncells];
  const long long p0 = (long long)blockIdx.x * kCB;
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int i = 0; i < kCB / kT; ++i) {
    const long long p = p0 + i * kT + threadIdx.x;
    uint2 lw = make_uint2(0u, 0u), ew = make_uint2(0u, 0u);
    if (p < nrec) {
      lw = like_w[p];
      ew = ei_w[p];
    }
    const int lc = like_class(lw), ec = ei_class(ew);
    int rl = 0, re = 0;
    for (int c = 0; c < kNC; ++c) {
      const unsigned long long m = __ballot(lc == c || ec == c);
      if (lane == 0) wsum[wv][c] = (unsigned)__popcll(m);
      const int r = __popcll(m & below);
      if (lc == c) rl = r;
      if (ec == c) re = r;
    }
    __syncthreads();
    if (lc >= 0) {
      unsigned o = base[lc];
      for (int w = 0; w < wv; ++w) o += wsum[w][lc];
      list[o + (unsigned)rl] = lw;
    }
    if (ec >= 0) {
      unsigned o = base[ec];
      for (int w = 0; w < wv; ++w) o += wsum[w][ec];
      list[o + (unsigned)re] = ew;
    }
    __syncthreads();
    if (threadIdx.x < kNC) {
      unsigned t = 0;
      for (int w = 0; w < kW; ++w) t += wsum[w][threadIdx.x];
      base[threadIdx.x] += t;
    }
    __syncthreads();
  }
}

// Like collisions of the small cells, one thread per pair or triplet (the
// triplet's three in order).
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_like(PV* __restrict__ pv,
                                                const unsigned* __restrict__ loff,
                                                int G,
                                                const uint2* __restrict__ list,
                                                CoulC k, Counters* dc) {
  const long long w0 = (long long)loff[0];
  long long lo, hi;
  block_range((long long)loff[2 * G] - w0, lo, hi);
  unsigned long long nl = 0;
  for (long long w = w0 + lo + threadIdx.x; w < w0 + hi; w += kT) {
    const uint2 it = list[w];
    const int s = (int)(it.y >> 31);
    const bool trip = (it.y >> 30) & 1u;
    const int N = (int)(it.y & 0x3FFFFFFFu);
    const double dens = (double)N * k.w_dx3;
    const unsigned a = it.x;
    const int nc = trip ? 3 : 1;
    for (int r = 0; r < nc; ++r) {
      const unsigned x = a + (unsigned)r;
      const unsigned y = r == 2 ? a : x + 1u;
      collide_pv(pv, x, y, s, dens, trip, pv[x].id, kTagDelta, kTagPhi, k);
    }
    nl += (unsigned long long)nc;
  }
  if (nl) atomicAdd(&dc->coul_like, nl);
}

// Electron-ion chains of the small cells, one thread per chain.
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_ei(PV* __restrict__ pv,
                                              const unsigned* __restrict__ loff,
                                              int G,
                                              const uint2* __restrict__ list,
                                              CoulC k, Counters* dc) {
  const long long w0 = (long long)loff[2 * G];
  long long lo, hi;
  block_range((long long)loff[kNC * G] - w0, lo, hi);
  unsigned long long nei = 0;
  for (long long w = w0 + lo + threadIdx.x; w < w0 + hi; w += kT) {
    const uint2 it = list[w];
    const unsigned b = it.x;
    const int t = (int)(it.y & 0xFFu), ne = (int)((it.y >> 8) & 0xFFu),
              ni = (int)(it.y >> 16);
    const int K = ne > ni ? ne : ni, m = ne < ni ? ne : ni;
    const double dens = (double)m * k.w_dx3;
    for (int j = t; j < K; j += m) {
      const unsigned a = b + (unsigned)(j % ne), bi = b + (unsigned)(ne + j % ni);
      const unsigned long long idc = ne >= ni ? pv[a].id : pv[bi].id;
      collide_pv(pv, a, bi, 2, dens, false, idc, kTagDeltaEI, kTagPhiEI, k);
      nei += 1;
    }
  }
  if (nei) atomicAdd(&dc->coul_ei, nei);
}

// Crowded cells: one workgroup each (grid-stride over the list).
template <class PT>
__global__ void __launch_bounds__(kBigT) k_cg_big(Sp2<PT> S,
                                                  const unsigned* __restrict__ off,
                                                  const Rec* __restrict__ rec,
                                                  const unsigned* __restrict__ big,
                                                  const unsigned* __restrict__ nbig,
                                                  long long big_cap, CoulC k,
                                                  Counters* dc) {
  __shared__ unsigned long long sk[kCoulBigCell];
  __shared__ unsigned sv[kCoulBigCell];
  __shared__ unsigned char ss[kCoulBigCell];
  __shared__ int s_ne;
  long long nlist = (long long)*nbig;
  if (nlist > big_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&dc->err, kErrEvents);
    nlist = big_cap;
  }
  unsigned long long nl = 0, nei = 0;
  for (long long q = blockIdx.x; q < nlist; q += gridDim.x) {
    const unsigned c = big[q];
    const unsigned b = off[c];
    const int n = (int)(off[c + 1] - b);
    if (n > kCoulBigCell) {
      if (threadIdx.x == 0) atomicOr(&dc->err, kErrEvents);
      continue;
    }
    int np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (int j = threadIdx.x; j < np2; j += kBigT) {
      if (j < n) {
        const Rec r = rec[b + j];
        sk[j] = r.lo;
        sv[j] = r.val;
        ss[j] = (unsigned char)rec_sp(r);
      } else {
        sk[j] = ~0ull;
        sv[j] = 0u;
        ss[j] = 1;
      }
    }
    __syncthreads();
    // Bitonic sort by key.
    for (int size = 2; size <= np2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int j = threadIdx.x; j < np2; j += kBigT) {
          const int p = j ^ stride;
          if (p > j) {
            const bool up = (j & size) == 0;
            const bool swap = up ? sk[j] > sk[p] : sk[j] < sk[p];
            if (swap) {
              const unsigned long long tk = sk[j]; sk[j] = sk[p]; sk[p] = tk;
              const unsigned tv = sv[j]; sv[j] = sv[p]; sv[p] = tv;
              const unsigned char ts = ss[j]; ss[j] = ss[p]; ss[p] = ts;
            }
          }
        }
        __syncthreads();
      }
    }
    if (threadIdx.x == 0) {
      // Equal keys (practically never) in id order, and the species split.
      for (int j = 1; j < n; ++j) {
        int m = j;
        while (m > 0 && sk[m] == sk[m - 1] &&
               S.p[ss[m]].id[sv[m]] < S.p[ss[m - 1]].id[sv[m - 1]]) {
          const unsigned tv = sv[m]; sv[m] = sv[m - 1]; sv[m - 1] = tv;
          const unsigned char ts = ss[m]; ss[m] = ss[m - 1]; ss[m - 1] = ts;
          --m;
        }
      }
      int ne = 0;
      while (ne < n && ss[ne] == 0) ++ne;
      s_ne = ne;
    }
    __syncthreads();
    const int ne = s_ne, ni = n - ne;
    // Like pairs: disjoint, in parallel (a triplet by one thread).
    for (int s = 0; s < 2; ++s) {
      const int base = s ? ne : 0;
      const int N = s ? ni : ne;
      if (N < 2) continue;
      const double dens = (double)N * k.w_dx3;
      const int start = (N & 1) ? 3 : 0;
      if (start && threadIdx.x == 0) {
        const unsigned a = sv[base], bb = sv[base + 1], cc = sv[base + 2];
        const PT& P = S.p[s];
        collide(S, s, a, s, bb, dens, true, P.id[a], kTagDelta, kTagPhi, k);
        collide(S, s, bb, s, cc, dens, true, P.id[bb], kTagDelta, kTagPhi, k);
        collide(S, s, cc, s, a, dens, true, P.id[cc], kTagDelta, kTagPhi, k);
        nl += 3;
      }
      for (int j = start + 2 * (int)threadIdx.x; j + 1 < N; j += 2 * kBigT) {
        const unsigned a = sv[base + j], bb = sv[base + j + 1];
        collide(S, s, a, s, bb, dens, false, S.p[s].id[a], kTagDelta, kTagPhi, k);
        nl += 1;
      }
    }
    __syncthreads();
    if (ne > 0 && ni > 0) {
      const int K = ne > ni ? ne : ni, Ns = ne < ni ? ne : ni;
      const double dens = (double)Ns * k.w_dx3;
      for (int r0 = 0; r0 < K; r0 += Ns) {
        const int r1 = r0 + Ns < K ? r0 + Ns : K;
        for (int j = r0 + (int)threadIdx.x; j < r1; j += kBigT) {
          const unsigned a = sv[j % ne], bb = sv[ne + j % ni];
          const unsigned long long idc =
              ne >= ni ? S.p[0].id[a] : S.p[1].id[bb];
          collide(S, 0, a, 1, bb, dens, false, idc, kTagDeltaEI, kTagPhiEI, k);
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) nei += (unsigned long long)K;
    }
    __syncthreads();
  }
  if (nl) atomicAdd(&dc->coul_like, nl);
  if (nei) atomicAdd(&dc->coul_ei, nei);
}

template <class PT>
Sp2<PT> sp2(pic_ctx* c);
template <>
Sp2<Parts> sp2<Parts>(pic_ctx* c) {
  return Sp2<Parts>{{c->P[0][c->cur[0]], c->P[2][c->cur[2]]}};
}
template <>
Sp2<PartsM> sp2<PartsM>(pic_ctx* c) {
  return Sp2<PartsM>{{c->PM[0][c->cur[0]], c->PM[2][c->cur[2]]}};
}

template <class PT>
void coulomb_t(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const long long nc = c->cg_nkeys;          // tile-major cell numbers
  CoulC k;
  const double e2 = kE * kE;
  const double den = (8.0 * kPi) * (kEps0 * kEps0);
  const double ms[2] = {kMe, kMcu};
  for (int ty = 0; ty < 3; ++ty) {
    const double m1 = ms[ty == 2 ? 0 : ty], m2 = ms[ty == 2 ? 1 : ty];
    const double mr = (m1 * m2) / (m1 + m2);
    k.cvar[ty] = (((e2 * e2) * c->coul.ln_lambda) * dt) / (den * (mr * mr));
    k.a1[ty] = mr / m1;
    k.a2[ty] = mr / m2;
  }
  const double inv = c->g.inv_dx;
  k.w_dx3 = (double)c->cfg.w_sp * ((inv * inv) * inv);
  k.step = (unsigned)c->step;
  k.seed = c->cfg.seed;
  const Sp2<PT> S = sp2<PT>(c);
  hipMemsetAsync(c->cg_cnt, 0, nc * sizeof(unsigned), st);
  hipMemsetAsync(c->cg_nbig, 0, sizeof(unsigned), st);
  const unsigned nblk = 4096;
  PV* pv = reinterpret_cast<PV*>(c->cg_pv);
  PV* pvu = reinterpret_cast<PV*>(c->cg_pvu);
  k_cg_count<<<nblk, kT, 0, st>>>(c->key[0], c->key[2], c->dc, c->g,
                                  c->cg_cnt);
  const long long nb = (nc + kScanB - 1) / kScanB;
  k_cg_scan_blocks<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_cnt, nc, c->cg_off,
                                                   c->cg_bsum);
  k_cg_scan_sums<<<1, 1024, 0, st>>>(c->cg_bsum, (int)nb);
  k_cg_scan_apply<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_off, nc, c->cg_bsum);
  k_cg_scatter<PT><<<nblk, kT, 0, st>>>(S, c->key[0], c->key[2], c->dc, c->g,
                                        c->cg_off, c->cg_cnt, c->cg_rec, pvu,
                                        c->cg_slot, k.step, k.seed);
  // Grids of a multiple of 8 workgroups (see xcd_block).
  k_cg_rank<<<8192, kT, 0, st>>>(c->cg_off, nc, c->cg_rec, pvu, pv,
                                 c->cg_place, c->cg_big, c->cg_big_cap,
                                 c->cg_nbig,
                                     c->cg_work, c->cg_work + c->cg_work_cap);
  const int G = c->cg_wblocks;
  const long long nw = (long long)kNC * G;
  const long long nwb = (nw + kScanB - 1) / kScanB;
  k_cg_wcount<<<G, kT, 0, st>>>(c->cg_off, nc, c->cg_work,
                                c->cg_work + c->cg_work_cap, c->cg_wcnt, G);
  k_cg_scan_blocks<<<(unsigned)nwb, kScanB, 0, st>>>(c->cg_wcnt, nw,
                                                    c->cg_woff, c->cg_wbsum);
  k_cg_scan_sums<<<1, 1024, 0, st>>>(c->cg_wbsum, (int)nwb);
  k_cg_scan_apply<<<(unsigned)nwb, kScanB, 0, st>>>(c->cg_woff, nw, c->cg_wbsum);
  k_cg_wscatter<<<G, kT, 0, st>>>(c->cg_off, nc, c->cg_work,
                                  c->cg_work + c->cg_work_cap, c->cg_woff, G,
                                  c->cg_list);
  k_cg_like<PT><<<8192, kT, 0, st>>>(pv, c->cg_woff, G, c->cg_list, k, c->dc);
  k_cg_ei<PT><<<8192, kT, 0, st>>>(pv, c->cg_woff, G, c->cg_list, k, c->dc);
  k_cg_writeback<PT><<<8192, kT, 0, st>>>(S, c->dc, c->cg_slot, c->cg_place,
                                          pv);
  k_cg_big<PT><<<512, kBigT, 0, st>>>(S, c->cg_off, c->cg_rec, c->cg_big,
                                      c->cg_nbig, c->cg_big_cap, k, c->dc);
}

}  // namespace

long long coulomb_scan_blocks(long long ncells) {
  return (ncells + kScanB - 1) / kScanB;
}

long long coulomb_work_blocks(long long records) {
  return (records + kCB - 1) / kCB;
}

long long coulomb_work_counts(long long records) {
  return (long long)kNC * coulomb_work_blocks(records);
}

void parts_coulomb(pic_ctx* c, double dt) {
  if (c->mixed)
    coulomb_t<PartsM>(c, dt);
  else
    coulomb_t<Parts>(c, dt);
}

}  // namespace pic
