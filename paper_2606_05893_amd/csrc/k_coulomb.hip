// Coulomb collisions by binary pairing within cells (Takizuka & Abe), the
// collision model the paper cites for its Monte Carlo collisions.
//
// The charged particles are grouped by cell: a count per cell (one pass over
// the keys), an exclusive scan, and a scatter of one 16-byte record per
// particle into its cell's segment (species in the top bit of the sort key,
// below it the 53-bit order draw of (id, step)).  A cell's records are then
// put in (key, id) order, which gives each species a random order that
// does not depend on where the particles sit in memory; consecutive
// particles of a species pair, an odd count leaves a triplet of half-weight
// collisions, and the electrons and ions of the cell collide in a sequence
// of max(N_e, N_i) collisions.
//
// Most cells hold a few charged particles.  There a thread per record
// finds the record's rank in its cell's order (by comparison with the
// others of the segment), and writes it, with the work it leads (a like
// pair or triplet, or an electron-ion chain), to its sorted place.  The
// like collisions then run a thread per pair, and after them the electron-
// ion collisions a thread per chain (the t-th particle of the smaller group
// with the larger group's t-th, (t+m)-th, ... particles; the chains share
// no particle, so they equal the sequence of the definition).  Crowded
// cells (more than kSmallCell records) go to a list served by one
// workgroup each: an LDS sort, the like pairs in parallel, and the
// electron-ion sequence in rounds of min(N_e, N_i) collisions, each round
// touching every particle at most once.
#include <cmath>

#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kSmallCell = 16;
constexpr int kBigT = 256;
constexpr int kCoulBigCell = 2048;    // records a crowded cell may hold
constexpr unsigned long long kSpBit = 1ull << 63;
constexpr int kScanB = 1024;          // cells per scan block

enum : uint32_t {
  kTagOrder = 20, kTagDelta = 21, kTagPhi = 22, kTagDeltaEI = 23, kTagPhiEI = 24
};

struct CoulC {
  double lnl, dt, q4, w_dx3, den;      // den = 8 pi eps0^2
  double m[2];                         // electron, Cu+ ion
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

// One binary collision of particle a (species sa) with particle b (sb):
// delta normal with the stated variance (halved in a triplet), phi uniform;
// the relative velocity turns by theta = 2 atan(delta) about itself.
template <class PT>
__device__ void collide(const Sp2<PT>& S, int sa, unsigned a, int sb,
                        unsigned b, double n, bool half,
                        unsigned long long id_c, uint32_t tag_d,
                        uint32_t tag_p, const CoulC& k) {
  double v1x, v1y, v1z, v2x, v2y, v2z;
  get_v(S, sa, a, v1x, v1y, v1z);
  get_v(S, sb, b, v2x, v2y, v2z);
  const double ux = v1x - v2x, uy = v1y - v2y, uz = v1z - v2z;
  const double u = sqrt((ux * ux + uy * uy) + uz * uz);
  if (!(u > 0.0)) return;
  const double m1 = k.m[sa], m2 = k.m[sb];
  const double mr = (m1 * m2) / (m1 + m2);
  double var = (((k.q4 * n) * k.lnl) * k.dt) / (k.den * ((mr * mr) * ((u * u) * u)));
  if (half) var = 0.5 * var;
  double u1, u2, u3, u4;
  uniform2(id_c, k.step, tag_d, k.seed, u1, u2);
  uniform2(id_c, k.step, tag_p, k.seed, u3, u4);
  const double g = sqrt(-2.0 * log(1.0 - u1)) * cos(kTwoPi * u2);
  const double phi = kTwoPi * u3;
  const double delta = sqrt(var) * g;
  const double uperp = sqrt(ux * ux + uy * uy);
  const double d2 = delta * delta;
  const double s = (2.0 * delta) / (1.0 + d2);
  const double omc = (2.0 * d2) / (1.0 + d2);
  const double cp = cos(phi), sp = sin(phi);
  double dux, duy, duz;
  if (uperp > 0.0) {
    dux = ((((ux / uperp) * uz) * s) * cp - (((uy / uperp) * u) * s) * sp) - ux * omc;
    duy = ((((uy / uperp) * uz) * s) * cp + (((ux / uperp) * u) * s) * sp) - uy * omc;
    duz = (-(uperp * s)) * cp - uz * omc;
  } else {
    dux = (u * s) * cp;
    duy = (u * s) * sp;
    duz = -(uz * omc);
  }
  const double a1 = mr / m1, a2 = mr / m2;
  set_v(S, sa, a, v1x + a1 * dux, v1y + a1 * duy, v1z + a1 * duz);
  set_v(S, sb, b, v2x - a2 * dux, v2y - a2 * duy, v2z - a2 * duz);
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
                           const Counters* dc, unsigned* __restrict__ cnt) {
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       t < ne + ni; t += stride) {
    const uint32_t c = t < ne ? ke[t] : ki[t - ne];
    if (c != kDead) atomicAdd(&cnt[c], 1u);
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
// inside the segment arbitrary; the cell pass sorts it).
template <class PT>
__global__ void k_cg_scatter(Sp2<PT> S, const uint32_t* __restrict__ ke,
                             const uint32_t* __restrict__ ki,
                             const Counters* dc,
                             const unsigned* __restrict__ off,
                             unsigned* __restrict__ cnt, Rec* __restrict__ rec,
                             unsigned step, unsigned long long seed) {
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       t < ne + ni; t += stride) {
    const int s = t < ne ? 0 : 1;
    const unsigned i = (unsigned)(s ? t - ne : t);
    const uint32_t c = s ? ki[i] : ke[i];
    if (c == kDead) continue;
    const unsigned slot = off[c] + atomicSub(&cnt[c], 1u) - 1u;
    Rec r;
    r.lo = (s ? kSpBit : 0ull) | order_key(S.p[s].id[i], step, seed);
    r.hi = (c << 2) | (unsigned)s;
    r.val = i;
    rec[slot] = r;
  }
}

// Workgroups are dispatched to the eight XCDs in turn; this numbering gives
// each XCD a contiguous run of them (grid a multiple of 8), so that a range
// of cells, and the particles of their tiles, stays in one XCD's L2.
__device__ __forceinline__ long long xcd_block() {
  return (long long)(blockIdx.x % 8u) * (gridDim.x / 8u) + blockIdx.x / 8u;
}

// The contiguous range [lo, hi) of n items this workgroup serves.
__device__ __forceinline__ void block_range(long long n, long long& lo,
                                            long long& hi) {
  const long long per = (n + gridDim.x - 1) / gridDim.x;
  lo = xcd_block() * per;
  hi = lo + per < n ? lo + per : n;
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
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_rank(
    Sp2<PT> S, const unsigned* __restrict__ off, long long ncells,
    const Rec* __restrict__ rec, Rec* __restrict__ srt,
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
    if (n > kSmallCell) {
      if ((unsigned)p == b) {
        const unsigned slot = atomicAdd(nbig, 1u);
        if ((long long)slot < big_cap) big[slot] = c;
      }
    } else if (n >= 2) {
      int rank = 0, ne = 0;
      for (int j = 0; j < n; ++j) {
        const Rec x = rec[b + j];
        ne += rec_sp(x) == 0u;
        rank += rec_before(S, x, r);
      }
      place = (long long)b + rank;
      srt[place] = r;
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
    like_w[place] = li;
    ei_w[place] = eit;
  }
}

// Like collisions of the small cells, one thread per pair or triplet.
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_like(Sp2<PT> S,
                                                const Rec* __restrict__ srt,
                                                const unsigned* __restrict__ off,
                                                long long ncells,
                                                const uint2* __restrict__ work,
                                                CoulC k, Counters* dc) {
  long long lo, hi;
  block_range((long long)off[ncells], lo, hi);
  unsigned long long nl = 0;
  for (long long w = lo + threadIdx.x; w < hi; w += kT) {
    const uint2 it = work[w];
    if (it.y == 0u) continue;
    const int s = (int)(it.y >> 31);
    const bool trip = (it.y >> 30) & 1u;
    const int N = (int)(it.y & 0x3FFFFFFFu);
    const double dens = (double)N * k.w_dx3;
    const PT& P = S.p[s];
    const unsigned a = srt[it.x].val, b = srt[it.x + 1].val;
    if (trip) {
      const unsigned c = srt[it.x + 2].val;
      collide(S, s, a, s, b, dens, true, P.id[a], kTagDelta, kTagPhi, k);
      collide(S, s, b, s, c, dens, true, P.id[b], kTagDelta, kTagPhi, k);
      collide(S, s, c, s, a, dens, true, P.id[c], kTagDelta, kTagPhi, k);
      nl += 3;
    } else {
      collide(S, s, a, s, b, dens, false, P.id[a], kTagDelta, kTagPhi, k);
      nl += 1;
    }
  }
  if (nl) atomicAdd(&dc->coul_like, nl);
}

// Electron-ion chains of the small cells, one thread per chain.
template <class PT>
__global__ void __launch_bounds__(kT) k_cg_ei(Sp2<PT> S,
                                              const Rec* __restrict__ srt,
                                              const unsigned* __restrict__ off,
                                              long long ncells,
                                              const uint2* __restrict__ work,
                                              CoulC k, Counters* dc) {
  long long lo, hi;
  block_range((long long)off[ncells], lo, hi);
  unsigned long long nei = 0;
  for (long long w = lo + threadIdx.x; w < hi; w += kT) {
    const uint2 it = work[w];
    if (it.y == 0u) continue;
    const unsigned b = it.x;
    const int t = (int)(it.y & 0xFFu), ne = (int)((it.y >> 8) & 0xFFu),
              ni = (int)(it.y >> 16);
    const int K = ne > ni ? ne : ni, m = ne < ni ? ne : ni;
    const double dens = (double)m * k.w_dx3;
    for (int j = t; j < K; j += m) {
      const unsigned a = srt[b + j % ne].val, bi = srt[b + ne + j % ni].val;
      const unsigned long long idc = ne >= ni ? S.p[0].id[a] : S.p[1].id[bi];
      collide(S, 0, a, 1, bi, dens, false, idc, kTagDeltaEI, kTagPhiEI, k);
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
  const long long nc = c->ncells;
  CoulC k;
  k.lnl = c->coul.ln_lambda;
  k.dt = dt;
  const double e2 = kE * kE;
  k.q4 = e2 * e2;
  const double inv = c->g.inv_dx;
  k.w_dx3 = (double)c->cfg.w_sp * ((inv * inv) * inv);
  k.den = (8.0 * kPi) * (kEps0 * kEps0);
  k.m[0] = kMe;
  k.m[1] = kMcu;
  k.step = (unsigned)c->step;
  k.seed = c->cfg.seed;
  const Sp2<PT> S = sp2<PT>(c);
  hipMemsetAsync(c->cg_cnt, 0, nc * sizeof(unsigned), st);
  hipMemsetAsync(c->cg_nbig, 0, sizeof(unsigned), st);
  const unsigned nblk = 4096;
  k_cg_count<<<nblk, kT, 0, st>>>(c->key[0], c->key[2], c->dc, c->cg_cnt);
  const long long nb = (nc + kScanB - 1) / kScanB;
  k_cg_scan_blocks<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_cnt, nc, c->cg_off,
                                                   c->cg_bsum);
  k_cg_scan_sums<<<1, 1024, 0, st>>>(c->cg_bsum, (int)nb);
  k_cg_scan_apply<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_off, nc, c->cg_bsum);
  k_cg_scatter<PT><<<nblk, kT, 0, st>>>(S, c->key[0], c->key[2], c->dc,
                                        c->cg_off, c->cg_cnt, c->cg_rec,
                                        k.step, k.seed);
  // Grids of a multiple of 8 workgroups (see xcd_block).
  k_cg_rank<PT><<<8192, kT, 0, st>>>(S, c->cg_off, nc, c->cg_rec, c->cg_srt,
                                     c->cg_big, c->cg_big_cap, c->cg_nbig,
                                     c->cg_work, c->cg_work + c->cg_work_cap);
  k_cg_like<PT><<<8192, kT, 0, st>>>(S, c->cg_srt, c->cg_off, nc, c->cg_work,
                                     k, c->dc);
  k_cg_ei<PT><<<8192, kT, 0, st>>>(S, c->cg_srt, c->cg_off, nc,
                                   c->cg_work + c->cg_work_cap, k, c->dc);
  k_cg_big<PT><<<512, kBigT, 0, st>>>(S, c->cg_off, c->cg_rec, c->cg_big,
                                      c->cg_nbig, c->cg_big_cap, k, c->dc);
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
