// Coulomb collisions by binary pairing within cells (Takizuka & Abe), the
// collision model the paper cites for its Monte Carlo collisions.
//
// Within a cell the charged particles are put in (key, id) order, the key
// being the species (top bit) above the 53-bit order draw of (id, step):
// each species then takes a random order that does not depend on where the
// particles sit in memory.  Consecutive particles of a species pair (an odd
// count leaves a leading triplet of half-weight collisions), and then the
// electrons and ions of the cell collide in a sequence of max(N_e, N_i)
// collisions, collision j between electron j mod N_e and ion j mod N_i.
//
// The particle arrays are binned by tile (8x8x8 cells) and move little
// between binning passes, so the work is grouped by tile plane (one z layer
// of a tile, 64 cells): the index words of the plane's electrons and ions
// are binned (a count and a scatter per chunk of particles, aggregated by
// plane in LDS, so that a chunk, nearly all of one tile, takes a few global
// atomics), and one wavefront serves a plane at a time.  It counts the
// plane's particles by cell as it loads them (id, velocity) into LDS, puts
// the slots in cell order, ranks each particle in its cell by comparison
// with the others, lists the work by class (like pairs, like triplets,
// electron-ion chains of one, two, three or more collisions, so that a
// wavefront runs one kind), runs the like collisions of all cells (disjoint
// pairs, in parallel), then the electron-ion collisions as chains (the t-th
// particle of the smaller group meets the larger group's t-th, (t+m)-th,
// ... particles; the chains share no particle, so they equal the sequence
// of the definition), and writes the velocities back once.  A plane holding
// more particles than one LDS batch is served in batches of whole cells; a
// cell holding more than a batch is listed for a workgroup that sorts its
// keys in LDS (bitonic) and collides on the particle arrays, the
// electron-ion sequence in rounds of min(N_e, N_i) collisions that touch
// every particle at most once.
#include <cmath>

#include "cell_groups.h"
#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kCoulBigCell = 2048;    // particles a crowded cell may hold
constexpr unsigned long long kSpBit = 1ull << 63;
constexpr int kScanB = 1024;          // counts per scan block
constexpr int kCap = 184;             // particles of one LDS batch

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

// The random part of one collision, which does not depend on the
// velocities: the standard normal variate of (id_c, tag_d) and the cosine
// and sine of the azimuth drawn from (id_c, tag_p).
struct Draw {
  double g, c, s;
};

__device__ __forceinline__ Draw coll_draw(unsigned long long id_c,
                                          uint32_t tag_d, uint32_t tag_p,
                                          const CoulC& k) {
  double u1, u2, u3, u4;
  uniform2(id_c, k.step, tag_d, k.seed, u1, u2);
  uniform2(id_c, k.step, tag_p, k.seed, u3, u4);
  Draw d;
  d.g = sqrt(-2.0 * log(1.0 - u1)) * cospi(2.0 * u2);
  sincospi(2.0 * u3, &d.s, &d.c);
  return d;
}

// One binary collision of a pair of type ty on the velocities v1 and v2, in
// place, with its draw: delta normal with the stated variance (halved in a
// triplet), phi uniform; the relative velocity turns by theta =
// 2 atan(delta) about itself.  Returns false (nothing changed) for zero
// relative speed.
__device__ bool kick(double* v1, double* v2, int ty, double n, bool half,
                     const Draw& d, const CoulC& k) {
  const double ux = v1[0] - v2[0], uy = v1[1] - v2[1], uz = v1[2] - v2[2];
  const double u = sqrt((ux * ux + uy * uy) + uz * uz);
  if (!(u > 0.0)) return false;
  double var = (k.cvar[ty] * n) / ((u * u) * u);
  if (half) var = 0.5 * var;
  const double delta = sqrt(var) * d.g;
  const double uperp = sqrt(ux * ux + uy * uy);
  const double d2 = delta * delta;
  const double inv = 1.0 / (1.0 + d2);
  const double s = (2.0 * delta) * inv;
  const double omc = (2.0 * d2) * inv;
  const double sp = d.s, cp = d.c;
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

__device__ __forceinline__ bool pair_kick(double* v1, double* v2, int ty,
                                          double n, bool half,
                                          unsigned long long id_c,
                                          uint32_t tag_d, uint32_t tag_p,
                                          const CoulC& k) {
  return kick(v1, v2, ty, n, half, coll_draw(id_c, tag_d, tag_p, k), k);
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

// ---- binning of the charged particles' indices by plane ---------------------
// Charged particle t of the joint range (electrons, then ions): its key, and
// its index word t.
__device__ __forceinline__ uint32_t charged_key(const uint32_t* __restrict__ ke,
                                                const uint32_t* __restrict__ ki,
                                                long long ne, long long t,
                                                unsigned& gi) {
  gi = (unsigned)t;
  return t < ne ? ke[t] : ki[t - ne];
}

// Live charged particles per plane.
__global__ void __launch_bounds__(kT) k_cu_count(
    const uint32_t* __restrict__ ke, const uint32_t* __restrict__ ki,
    const Counters* dc, GridC g, unsigned* __restrict__ cnt) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  long long lo, hi;
  block_range(ne + ni, lo, hi);
  for (long long b = lo; b < hi; b += kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kPChunk < hi ? b + kPChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = charged_key(ke, ki, ne, t, gi);
      if (c == kDead) continue;
      const unsigned u = plane_of(c, g);
      const int q = plane_slot(hk, u);
      if (q >= 0)
        atomicAdd(&hc[q], 1u);
      else
        atomicAdd(&cnt[u], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPHash; q += kT)
      if (hk[q] != kGEmpty) atomicAdd(&cnt[hk[q]], hc[q]);
    __syncthreads();
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

// Each live charged particle's index word into its plane's range (order
// inside the range arbitrary: the cell pass sorts).  Per chunk the planes
// are counted in LDS, one range per distinct plane reserved with one global
// atomic, then each particle placed at the next slot of its plane's range.
__global__ void __launch_bounds__(kT) k_cu_scatter(
    const uint32_t* __restrict__ ke, const uint32_t* __restrict__ ki,
    const Counters* dc, GridC g, const unsigned* __restrict__ off,
    unsigned* __restrict__ cnt, unsigned* __restrict__ idx) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  __shared__ unsigned hb[kPHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  long long lo, hi;
  block_range(ne + ni, lo, hi);
  for (long long b = lo; b < hi; b += kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kPChunk < hi ? b + kPChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = charged_key(ke, ki, ne, t, gi);
      if (c == kDead) continue;
      const int q = plane_slot(hk, plane_of(c, g));
      if (q >= 0) atomicAdd(&hc[q], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      const unsigned u = hk[q];
      if (u != kGEmpty) {
        const unsigned m = hc[q];
        hb[q] = off[u] + atomicSub(&cnt[u], m) - m;
        hc[q] = 0u;
      }
    }
    __syncthreads();
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = charged_key(ke, ki, ne, t, gi);
      if (c == kDead) continue;
      const unsigned u = plane_of(c, g);
      // The table is unchanged since the count: a plane found there then is
      // found again, one that found no room finds none again.
      const int q = plane_slot(hk, u);
      const unsigned slot = q >= 0 ? hb[q] + atomicAdd(&hc[q], 1u)
                                   : off[u] + atomicSub(&cnt[u], 1u) - 1u;
      idx[slot] = gi;
    }
    __syncthreads();
  }
}

// ---- the cell pass -------------------------------------------------------------
// One wavefront per plane: a workgroup of one wavefront never waits at a
// barrier for others, so a plane's serial stretches (the longest electron-ion
// chain) leave the SIMD to the other planes' wavefronts.
constexpr int kCT = 64;

// LDS of a batch of whole cells.  Particles sit in load order (slots); the
// cell order is a permutation of the slots, and each cell's part of it is
// then ranked by (key, id).
struct BatchLds {
  unsigned long long key[kCap];   // species bit above the order draw
  unsigned long long id[kCap];
  double v[3][kCap];
  unsigned gi[kCap];              // index word (joint range)
  unsigned short cell[kCap];      // cell in the plane
  unsigned short perm[kCap];      // sorted place -> slot
  unsigned short work[kCap];      // cell order -> slot, then the work items
};

// Work classes, so that a wavefront runs one kind: like pairs, like
// triplets, electron-ion chains of one, two, and three or more collisions.
constexpr int kNCls = 5;

struct PlaneLdsC {
  unsigned off[kPlaneCells + 1];   // cell offsets in the plane's particles
  unsigned cur[kPlaneCells];
  unsigned short ne[kPlaneCells];  // electrons per cell
  unsigned cls[kNCls + 1];        // class offsets in the work list
  unsigned ccur[kNCls];
  int nslot, hi;
};

// The collision on two slots of the batch.
__device__ __forceinline__ void collide_lds(BatchLds& L, int a, int b, int ty,
                                            double n, bool half,
                                            unsigned long long id_c,
                                            uint32_t tag_d, uint32_t tag_p,
                                            const CoulC& k) {
  double v1[3] = {L.v[0][a], L.v[1][a], L.v[2][a]};
  double v2[3] = {L.v[0][b], L.v[1][b], L.v[2][b]};
  if (pair_kick(v1, v2, ty, n, half, id_c, tag_d, tag_p, k)) {
    L.v[0][a] = v1[0]; L.v[1][a] = v1[1]; L.v[2][a] = v1[2];
    L.v[0][b] = v2[0]; L.v[1][b] = v2[1]; L.v[2][b] = v2[2];
  }
}

// One particle of the plane into slot p of the batch (not yet its key).
template <class PT>
__device__ __forceinline__ void load_slot(const Sp2<PT>& S, const JointIx& J,
                                          BatchLds& L, int p, unsigned gi,
                                          int lc) {
  const int s = (int)J.sp(gi);
  const unsigned i = J.ix(gi);
  double vx, vy, vz;
  get_v(S, s, i, vx, vy, vz);
  L.id[p] = S.p[s].id[i];
  L.v[0][p] = vx;
  L.v[1][p] = vy;
  L.v[2][p] = vz;
  L.gi[p] = gi;
  L.cell[p] = (unsigned short)lc;
}

// The work a sorted place leads: its like class (0 pair, 1 triplet, -1
// none) and electron-ion chain class (2, 3, 4 for one, two, three or more
// collisions, -1 none).
__device__ __forceinline__ void place_work(const BatchLds& L, const PlaneLdsC& U,
                                           unsigned ob, int r, int& lcl,
                                           int& ecl) {
  lcl = ecl = -1;
  const int p = L.perm[r];
  const int lc = L.cell[p];
  const int m = (int)(U.off[lc + 1] - U.off[lc]);
  if (m < 2) return;
  const int b = (int)(U.off[lc] - ob);
  const int ne = U.ne[lc], ni = m - ne;
  const int s = (int)(L.key[p] >> 63);
  const int q = s ? r - b - ne : r - b;    // rank within the species
  const int N = s ? ni : ne;
  const int start = (N & 1) ? 3 : 0;
  const bool trip = (N & 1) && q == 0;
  if (N >= 2 && (trip || (q >= start && ((q - start) & 1) == 0 && q + 1 < N)))
    lcl = trip ? 1 : 0;
  if (ne > 0 && ni > 0 && s == (ne <= ni ? 0 : 1)) {
    const int K = ne > ni ? ne : ni, mm = ne < ni ? ne : ni;
    const int len = (K - q + mm - 1) / mm;
    ecl = len >= 3 ? 4 : len + 1;
  }
}

// The cells [c_lo, c_hi) of the plane, nb particles loaded in slots
// [0, nb): cell order, ranks, work lists, the collisions, the velocities
// back to the particle arrays.
template <class PT>
__device__ void batch_collide(const Sp2<PT>& S, const JointIx& J, int c_lo,
                              int c_hi, int nb,
                              BatchLds& L, PlaneLdsC& U, const CoulC& k,
                              unsigned long long& nl,
                              unsigned long long& nei) {
  const int tid = (int)threadIdx.x;
  const unsigned ob = U.off[c_lo];
  for (int c = c_lo + tid; c < c_hi; c += kCT) U.cur[c] = U.off[c] - ob;
  if (tid < kNCls) U.ccur[tid] = 0u;
  __syncthreads();
  // Cell order, and the keys of the particles that have a partner.
  for (int p = tid; p < nb; p += kCT) {
    const int lc = L.cell[p];
    L.work[atomicAdd(&U.cur[lc], 1u)] = (unsigned short)p;
    if (U.off[lc + 1] - U.off[lc] >= 2u) {
      const unsigned gi = L.gi[p];
      L.key[p] = (J.sp(gi) ? kSpBit : 0ull) | order_key(L.id[p], k.step, k.seed);
    }
  }
  __syncthreads();
  // Rank of each particle in its cell's (key, id) order.
  for (int x = tid; x < nb; x += kCT) {
    const int p = L.work[x];
    const int lc = L.cell[p];
    const int b = (int)(U.off[lc] - ob), m = (int)(U.off[lc + 1] - U.off[lc]);
    if (m < 2) {
      L.perm[b] = (unsigned short)p;
      continue;
    }
    const unsigned long long kp = L.key[p], ip = L.id[p];
    int rank = 0, ne = 0;
    for (int q = b; q < b + m; ++q) {
      const int o = L.work[q];
      const unsigned long long kq = L.key[o];
      ne += kq < kSpBit;
      rank += kq < kp || (kq == kp && L.id[o] < ip);
    }
    L.perm[b + rank] = (unsigned short)p;
    if (rank == 0) U.ne[lc] = (unsigned short)ne;
  }
  __syncthreads();
  // Work items by class: count, class offsets, placement (the list takes
  // the cell-order array's place).
  for (int r = tid; r < nb; r += kCT) {
    int lcl, ecl;
    place_work(L, U, ob, r, lcl, ecl);
    if (lcl >= 0) atomicAdd(&U.ccur[lcl], 1u);
    if (ecl >= 0) atomicAdd(&U.ccur[ecl], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    unsigned t = 0;
    for (int c = 0; c < kNCls; ++c) {
      U.cls[c] = t;
      t += U.ccur[c];
      U.ccur[c] = U.cls[c];
    }
    U.cls[kNCls] = t;
  }
  __syncthreads();
  for (int r = tid; r < nb; r += kCT) {
    int lcl, ecl;
    place_work(L, U, ob, r, lcl, ecl);
    if (lcl >= 0) L.work[atomicAdd(&U.ccur[lcl], 1u)] = (unsigned short)r;
    if (ecl >= 0) L.work[atomicAdd(&U.ccur[ecl], 1u)] = (unsigned short)r;
  }
  __syncthreads();
  // Like collisions: pairs, then leading triplets (three in order).
  const int n_like = (int)U.cls[2], n_pair = (int)U.cls[1];
  for (int w = tid; w < n_like; w += kCT) {
    const int r = L.work[w];
    const int p = L.perm[r];
    const int lc = L.cell[p];
    const int m = (int)(U.off[lc + 1] - U.off[lc]);
    const int ne = U.ne[lc];
    const int s = (int)J.sp(L.gi[p]);
    const int N = s ? m - ne : ne;
    const bool trip = w >= n_pair;
    const double dens = (double)N * k.w_dx3;
    const int nc = trip ? 3 : 1;
    for (int rr = 0; rr < nc; ++rr) {
      const int x = r + rr, y = rr == 2 ? r : x + 1;
      const int px = L.perm[x];
      collide_lds(L, px, L.perm[y], s, dens, trip, L.id[px], kTagDelta, kTagPhi, k);
    }
    nl += (unsigned long long)nc;
  }
  __syncthreads();
  // Electron-ion chains, shortest first.
  const int n_all = (int)U.cls[kNCls];
  for (int w = n_like + tid; w < n_all; w += kCT) {
    const int r = L.work[w];
    const int p = L.perm[r];
    const int lc = L.cell[p];
    const int b = (int)(U.off[lc] - ob), m = (int)(U.off[lc + 1] - U.off[lc]);
    const int ne = U.ne[lc], ni = m - ne;
    const int s = (int)J.sp(L.gi[p]);
    const int t = s ? r - b - ne : r - b;
    const int K = ne > ni ? ne : ni, mm = ne < ni ? ne : ni;
    const double dens = (double)mm * k.w_dx3;
    // Collision j pairs electron j mod N_e with ion j mod N_i; along the
    // chain (j = t, t + m, ...) the smaller group's index is t and the
    // larger group's is j itself (j < K).
    const bool e_small = ne <= ni;
    for (int j = t; j < K; j += mm) {
      const int pa = L.perm[b + (e_small ? t : j)];
      const int pb = L.perm[b + ne + (e_small ? j : t)];
      const unsigned long long idc = ne >= ni ? L.id[pa] : L.id[pb];
      collide_lds(L, pa, pb, 2, dens, false, idc, kTagDeltaEI, kTagPhiEI, k);
      nei += 1;
    }
  }
  __syncthreads();
  for (int p = tid; p < nb; p += kCT) {
    const int lc = L.cell[p];
    if (U.off[lc + 1] - U.off[lc] < 2u) continue;
    const unsigned gi = L.gi[p];
    set_v(S, (int)J.sp(gi), J.ix(gi), L.v[0][p], L.v[1][p], L.v[2][p]);
  }
  __syncthreads();
}

// Planes in turn (plane_first: a tile's eight planes at once on one XCD).
// A plane of at most kCap particles is loaded in one pass,
// counted by cell as it loads; a larger one is counted first and loaded in
// batches of whole cells; a cell of more than kCap particles is listed for
// the crowded-cell pass.
template <class PT>
__global__ void __launch_bounds__(kCT, 4) k_cu_cells(
    Sp2<PT> S, const uint32_t* __restrict__ ke, const uint32_t* __restrict__ ki,
    GridC g, const unsigned* __restrict__ uoff, long long nplanes,
    const unsigned* __restrict__ uidx, unsigned* __restrict__ crowd,
    long long crowd_cap, unsigned* __restrict__ ncrowd, CoulC k, Counters* dc) {
  __shared__ BatchLds L;
  __shared__ PlaneLdsC U;
  const int tid = (int)threadIdx.x;
  const JointIx J = joint_ix(dc);
  unsigned long long nl = 0, nei = 0;
  for (long long u = plane_first(); u < nplanes; u += gridDim.x) {
    const unsigned base = uoff[u];
    const int n = (int)(uoff[u + 1] - base);
    if (n < 2) continue;
    for (int c = tid; c < kPlaneCells; c += kCT) U.cur[c] = 0u;
    __syncthreads();
    const bool one = n <= kCap;
    for (int j = tid; j < n; j += kCT) {
      const unsigned gi = uidx[base + j];
      const uint32_t c0 = J.sp(gi) ? ki[J.ix(gi)] : ke[gi];
      const int lc = (int)(tile_major(c0, g) & (kPlaneCells - 1));
      atomicAdd(&U.cur[lc], 1u);
      if (one) load_slot(S, J, L, j, gi, lc);
    }
    __syncthreads();
    {
      // Exclusive scan of the plane's cell counts (one per lane).
      const unsigned t = U.cur[tid];
      unsigned incl = t;
      for (int o = 1; o < kCT; o <<= 1) {
        const unsigned y = __shfl_up(incl, o);
        if (tid >= o) incl += y;
      }
      U.off[tid] = incl - t;
      if (tid == kCT - 1) U.off[kPlaneCells] = incl;
    }
    __syncthreads();
    if (one) {
      batch_collide(S, J, 0, kPlaneCells, n, L, U, k, nl, nei);
      continue;
    }
    // Batches of whole cells of at most kCap particles.
    for (int c_lo = 0; c_lo < kPlaneCells;) {
      if (tid == 0) {
        int c_hi = c_lo + 1;
        if (U.off[c_lo + 1] - U.off[c_lo] <= (unsigned)kCap)
          while (c_hi < kPlaneCells && U.off[c_hi + 1] - U.off[c_lo] <= (unsigned)kCap)
            ++c_hi;
        U.hi = c_hi;
        U.nslot = 0;
      }
      __syncthreads();
      const int c_hi = U.hi;
      const int nb = (int)(U.off[c_hi] - U.off[c_lo]);
      if (nb > kCap) {
        if (tid == 0) {
          const unsigned q = atomicAdd(ncrowd, 1u);
          if ((long long)q < crowd_cap)
            crowd[q] = ((unsigned)u << kPlaneShift) | (unsigned)c_lo;
          else
            atomicOr(&dc->err, kErrEvents);
        }
      } else if (nb >= 2) {
        for (int j = tid; j < n; j += kCT) {
          const unsigned gi = uidx[base + j];
          const uint32_t c0 = J.sp(gi) ? ki[J.ix(gi)] : ke[gi];
          const int lc = (int)(tile_major(c0, g) & (kPlaneCells - 1));
          if (lc >= c_lo && lc < c_hi) load_slot(S, J, L, atomicAdd(&U.nslot, 1), gi, lc);
        }
        __syncthreads();
        batch_collide(S, J, c_lo, c_hi, nb, L, U, k, nl, nei);
      }
      __syncthreads();
      c_lo = c_hi;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    nl += __shfl_xor(nl, o);
    nei += __shfl_xor(nei, o);
  }
  if (tid == 0) {
    if (nl) atomicAdd(&dc->coul_like, nl);
    if (nei) atomicAdd(&dc->coul_ei, nei);
  }
}

// ---- crowded cells ---------------------------------------------------------------
// One workgroup per listed cell: its particles gathered from the plane's
// index words, their keys sorted in LDS (bitonic), the collisions on the
// particle arrays, the electron-ion sequence in rounds of min(N_e, N_i)
// collisions that touch every particle at most once.
template <class PT>
__global__ void __launch_bounds__(kT) k_cu_crowd(
    Sp2<PT> S, const uint32_t* __restrict__ ke, const uint32_t* __restrict__ ki,
    GridC g, const unsigned* __restrict__ uoff,
    const unsigned* __restrict__ uidx, const unsigned* __restrict__ crowd,
    long long crowd_cap, const unsigned* __restrict__ ncrowd, CoulC k,
    Counters* dc) {
  __shared__ unsigned long long skey[kCoulBigCell];
  __shared__ unsigned sgi[kCoulBigCell];
  __shared__ int s_m, s_ne;
  const int tid = (int)threadIdx.x;
  const JointIx J = joint_ix(dc);
  long long nlist = (long long)*ncrowd;
  if (nlist > crowd_cap) nlist = crowd_cap;
  unsigned long long nl = 0, nei = 0;
  for (long long q = blockIdx.x; q < nlist; q += gridDim.x) {
    const unsigned w = crowd[q];
    const unsigned u = w >> kPlaneShift;
    const int lc = (int)(w & (kPlaneCells - 1));
    const unsigned base = uoff[u];
    const int n = (int)(uoff[u + 1] - base);
    if (tid == 0) s_m = 0;
    __syncthreads();
    for (int j = tid; j < n; j += kT) {
      const unsigned gi = uidx[base + j];
      const int s = (int)J.sp(gi);
      const unsigned i = J.ix(gi);
      const uint32_t c0 = s ? ki[i] : ke[i];
      if ((int)(tile_major(c0, g) & (kPlaneCells - 1)) != lc) continue;
      const int p = atomicAdd(&s_m, 1);
      if (p < kCoulBigCell) {
        skey[p] = (s ? kSpBit : 0ull) | order_key(S.p[s].id[i], k.step, k.seed);
        sgi[p] = gi;
      }
    }
    __syncthreads();
    const int m = s_m;
    if (m > kCoulBigCell) {
      if (tid == 0) atomicOr(&dc->err, kErrEvents);
      __syncthreads();
      continue;
    }
    int np2 = 1;
    while (np2 < m) np2 <<= 1;
    for (int j = m + tid; j < np2; j += kT) {
      skey[j] = ~0ull;
      sgi[j] = 0u;
    }
    __syncthreads();
    // Bitonic sort by key.
    for (int size = 2; size <= np2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int j = tid; j < np2; j += kT) {
          const int p = j ^ stride;
          if (p > j) {
            const bool up = (j & size) == 0;
            const bool swap = up ? skey[j] > skey[p] : skey[j] < skey[p];
            if (swap) {
              const unsigned long long tk = skey[j]; skey[j] = skey[p]; skey[p] = tk;
              const unsigned tv = sgi[j]; sgi[j] = sgi[p]; sgi[p] = tv;
            }
          }
        }
        __syncthreads();
      }
    }
    if (tid == 0) {
      // Equal keys (practically never) in id order, and the species split.
      auto id_of = [&](unsigned gi) { return S.p[J.sp(gi)].id[J.ix(gi)]; };
      for (int j = 1; j < m; ++j) {
        int x = j;
        while (x > 0 && skey[x] == skey[x - 1] && id_of(sgi[x]) < id_of(sgi[x - 1])) {
          const unsigned tv = sgi[x]; sgi[x] = sgi[x - 1]; sgi[x - 1] = tv;
          --x;
        }
      }
      int ne = 0;
      while (ne < m && skey[ne] < kSpBit) ++ne;
      s_ne = ne;
    }
    __syncthreads();
    const int ne = s_ne, ni = m - ne;
    // Like pairs: disjoint, in parallel (a triplet by one thread).
    for (int s = 0; s < 2; ++s) {
      const int b0 = s ? ne : 0;
      const int N = s ? ni : ne;
      if (N < 2) continue;
      const double dens = (double)N * k.w_dx3;
      const int start = (N & 1) ? 3 : 0;
      const PT& P = S.p[s];
      if (start && tid == 0) {
        const unsigned a = J.ix(sgi[b0]), bb = J.ix(sgi[b0 + 1]),
                       cc = J.ix(sgi[b0 + 2]);
        collide(S, s, a, s, bb, dens, true, P.id[a], kTagDelta, kTagPhi, k);
        collide(S, s, bb, s, cc, dens, true, P.id[bb], kTagDelta, kTagPhi, k);
        collide(S, s, cc, s, a, dens, true, P.id[cc], kTagDelta, kTagPhi, k);
        nl += 3;
      }
      for (int j = start + 2 * tid; j + 1 < N; j += 2 * kT) {
        const unsigned a = J.ix(sgi[b0 + j]), bb = J.ix(sgi[b0 + j + 1]);
        collide(S, s, a, s, bb, dens, false, P.id[a], kTagDelta, kTagPhi, k);
        nl += 1;
      }
    }
    __syncthreads();
    // Electron-ion sequence in rounds of min(N_e, N_i) collisions.
    if (ne > 0 && ni > 0) {
      const int K = ne > ni ? ne : ni, Ns = ne < ni ? ne : ni;
      const double dens = (double)Ns * k.w_dx3;
      for (int r0 = 0; r0 < K; r0 += Ns) {
        const int r1 = r0 + Ns < K ? r0 + Ns : K;
        for (int j = r0 + tid; j < r1; j += kT) {
          const unsigned a = J.ix(sgi[j % ne]), bb = J.ix(sgi[ne + j % ni]);
          const unsigned long long idc = ne >= ni ? S.p[0].id[a] : S.p[1].id[bb];
          collide(S, 0, a, 1, bb, dens, false, idc, kTagDeltaEI, kTagPhiEI, k);
        }
        __syncthreads();
      }
      if (tid == 0) nei += (unsigned long long)K;
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
  const long long nu = c->cg_nkeys >> kPlaneShift;   // tile planes
  hipMemsetAsync(c->cg_cnt, 0, nu * sizeof(unsigned), st);
  // Grids of a multiple of 8 workgroups (see xcd_block).
  k_cu_count<<<4096, kT, 0, st>>>(c->key[0], c->key[2], c->dc, c->g,
                                  c->cg_cnt);
  const long long nb = (nu + kScanB - 1) / kScanB;
  k_cg_scan_blocks<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_cnt, nu, c->cg_poff,
                                                   c->cg_bsum);
  k_cg_scan_sums<<<1, 1024, 0, st>>>(c->cg_bsum, (int)nb);
  k_cg_scan_apply<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_poff, nu, c->cg_bsum);
  k_cu_scatter<<<4096, kT, 0, st>>>(c->key[0], c->key[2], c->dc, c->g,
                                    c->cg_poff, c->cg_cnt, c->cg_idx);
  hipMemsetAsync(c->cg_nbig, 0, sizeof(unsigned), st);
  k_cu_cells<PT><<<8192, kCT, 0, st>>>(S, c->key[0], c->key[2], c->g,
                                       c->cg_poff, nu, c->cg_idx, c->cg_big,
                                       c->cg_big_cap, c->cg_nbig, k, c->dc);
  k_cu_crowd<PT><<<256, kT, 0, st>>>(S, c->key[0], c->key[2], c->g, c->cg_poff,
                                     c->cg_idx, c->cg_big, c->cg_big_cap,
                                     c->cg_nbig, k, c->dc);
}

}  // namespace

long long coulomb_scan_blocks(long long ncells) {
  return (ncells + kScanB - 1) / kScanB;
}

void parts_coulomb(pic_ctx* c, double dt) {
  if (c->mixed)
    coulomb_t<PartsM>(c, dt);
  else
    coulomb_t<Parts>(c, dt);
}

}  // namespace pic
