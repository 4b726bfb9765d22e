// Recombination (e + Cu+ -> Cu), electron-impact ionisation of Cu+
// (e + Cu+ -> 2e + Cu2+) and resonant charge exchange (Cu+ + Cu -> Cu + Cu+):
// the paper's remaining Monte Carlo collision processes and the higher
// charge state they lead to.
//
// Electrons, Cu+ and Cu atoms are grouped by cell as for the Coulomb
// collisions (count, scan, scatter of 16-byte records keyed by species and
// a random order draw, then a sort inside each cell).  Every cell is then
// processed in sequence by one thread (a workgroup sorts the crowded ones,
// their atoms a window at a time): first each electron in turn against the
// cell's Cu+ (Eq. 4 evaluated per electron; the r-th colliding electron
// takes the r-th ion), then the Cu+ left against the cell's atoms (ion k with atom k mod N_n,
// the real relative speed).  Recombinations and charge exchanges are applied
// in place (records swapped, atoms appended, the charge of the pushed state
// corrected); Cu+ ionisations are listed, sorted by primary id and
// committed in that order, which fixes the secondaries' ids.
#include <cmath>

#include "cell_groups.h"
#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kSmall = 32;
constexpr int kBigCell = 2048;        // charged records of a crowded cell
constexpr int kWin = 1024;            // atoms per selection window
constexpr unsigned long long kOrdMask = (1ull << 53) - 1ull;
constexpr int kScanB = 1024;
constexpr double kNear = 1e-6;

enum : uint32_t {
  kTagOrd = 25, kTagEI0 = 26, kTagEI1 = 27, kTagEI2 = 28, kTagEI3 = 29,
  kTagCX = 30
};

struct IonC {
  double s_rec, a2, I2, cx_a, cx_b;
  double w_dx3, dt, half_me, two_e_me;
  unsigned step;
  unsigned long long seed;
  long long cap_n;                  // atom capacity (recombinations)
  long long max_ev;                 // listed ionisations
  // The tile push counted every binned electron and Cu+ it left alive into
  // its destination tile; one removed here gives its slot back.
  long long nb_e, nb_i;             // binned ranges
  unsigned *tcnt_e, *tcnt_i;        // destination-tile counts
};

__device__ __forceinline__ unsigned tile_of(unsigned cell, const GridC& g) {
  const unsigned i = cell % (unsigned)g.nx;
  const unsigned r = cell / (unsigned)g.nx;
  const unsigned j = r % (unsigned)g.ny;
  const unsigned k = r / (unsigned)g.ny;
  return ((k / kTile) * (unsigned)g.tny + j / kTile) * (unsigned)g.tnx + i / kTile;
}

template <class PT>
struct Sp3 {
  PT e, i, n;                        // electrons, Cu+, Cu
  uint32_t *ke, *ki, *kn;            // their keys
};

// A record's hi word holds its tile-major cell number above two species
// bits (0 electron, 1 Cu+, 2 Cu).
__device__ __forceinline__ unsigned ip_sp(const Rec& r) { return r.hi & 3u; }

template <class PT>
__device__ __forceinline__ unsigned long long rid(const Sp3<PT>& S,
                                                  const Rec& r) {
  const unsigned s = ip_sp(r);
  return s == 0 ? S.e.id[r.val] : (s == 1 ? S.i.id[r.val] : S.n.id[r.val]);
}

__device__ __forceinline__ unsigned long long ord_key(unsigned long long id,
                                                      unsigned step,
                                                      unsigned long long seed) {
  uint32_t c0 = (uint32_t)id, c1 = (uint32_t)(id >> 32), c2 = step, c3 = kTagOrd;
  philox10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
  return ((unsigned long long)c0 << 21) ^ (unsigned long long)(c1 >> 11);
}

// CIC charge of one particle added to the pushed state's int64 node charge.
template <class PT>
__device__ void dep_add(const PT& p, unsigned i, const GridC& g,
                        long long* __restrict__ acc, long long w) {
  int ix, fx, iy, fy, iz, fz;
  Acc<PT>::cic(p, i, g, ix, fx, iy, fy, iz, fz);
  const long long wx[2] = {kQ - fx, fx}, wy[2] = {kQ - fy, fy},
                  wz[2] = {kQ - fz, fz};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const long long node =
            ((long long)(iz + c) * g.ny + wrap_index(iy + b, g.ny)) * g.nx +
            wrap_index(ix + a, g.nx);
        atomicAdd(reinterpret_cast<unsigned long long*>(&acc[node]),
                  (unsigned long long)(w * (wx[a] * wy[b] * wz[c])));
      }
}

__device__ __forceinline__ double sigma_rec(const IonC& k, double E) {
  return k.s_rec * (1.0 / (E > 1e-3 ? E : 1e-3));
}

__device__ __forceinline__ double sigma_ion2(const IonC& k, double E) {
  if (!(E > k.I2)) return 0.0;
  return (k.a2 * log(E / k.I2)) / (E * k.I2);
}

__device__ __forceinline__ double sigma_cx(const IonC& k, double eps) {
  double t = k.cx_a - k.cx_b * log(eps > 1e-6 ? eps : 1e-6);
  t = t > 0.0 ? t : 0.0;
  return t * t;
}

// Exchange two particle records (position, velocity, id) of one layout.
template <class PT>
__device__ void swap_records(const PT& a, unsigned i, const PT& b, unsigned j);

template <>
__device__ void swap_records<Parts>(const Parts& a, unsigned i, const Parts& b,
                                    unsigned j) {
  double t;
  t = a.x[i]; a.x[i] = b.x[j]; b.x[j] = t;
  t = a.y[i]; a.y[i] = b.y[j]; b.y[j] = t;
  t = a.z[i]; a.z[i] = b.z[j]; b.z[j] = t;
  t = a.vx[i]; a.vx[i] = b.vx[j]; b.vx[j] = t;
  t = a.vy[i]; a.vy[i] = b.vy[j]; b.vy[j] = t;
  t = a.vz[i]; a.vz[i] = b.vz[j]; b.vz[j] = t;
  const unsigned long long u = a.id[i];
  a.id[i] = b.id[j];
  b.id[j] = u;
}

template <>
__device__ void swap_records<PartsM>(const PartsM& a, unsigned i,
                                     const PartsM& b, unsigned j) {
  float t;
  const unsigned c = a.cell[i];
  a.cell[i] = b.cell[j]; b.cell[j] = c;
  t = a.ox[i]; a.ox[i] = b.ox[j]; b.ox[j] = t;
  t = a.oy[i]; a.oy[i] = b.oy[j]; b.oy[j] = t;
  t = a.oz[i]; a.oz[i] = b.oz[j]; b.oz[j] = t;
  t = a.vx[i]; a.vx[i] = b.vx[j]; b.vx[j] = t;
  t = a.vy[i]; a.vy[i] = b.vy[j]; b.vy[j] = t;
  t = a.vz[i]; a.vz[i] = b.vz[j]; b.vz[j] = t;
  const unsigned long long u = a.id[i];
  a.id[i] = b.id[j];
  b.id[j] = u;
}

// ---- grouping ----------------------------------------------------------------
__global__ void __launch_bounds__(kT) k_ig_count(const uint32_t* __restrict__ ke,
                                                  const uint32_t* __restrict__ ki,
                                                  const uint32_t* __restrict__ kn,
                                                  const Counters* dc, GridC g,
                                                  unsigned* __restrict__ cnt) {
  __shared__ unsigned hk[kGHash];
  __shared__ unsigned hc[kGHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2],
                  nn = (long long)dc->n[1];
  long long lo, hi;
  block_range(ne + ni + nn, lo, hi);
  for (long long b = lo; b < hi; b += kGChunk) {
    for (int q = threadIdx.x; q < kGHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kGChunk < hi ? b + kGChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      const uint32_t c = t < ne ? ke[t] : (t < ne + ni ? ki[t - ne] : kn[t - ne - ni]);
      if (c == kDead) continue;
      const unsigned u = tile_major(c, g);
      const int q = ghash_slot(hk, u);
      if (q >= 0)
        atomicAdd(&hc[q], 1u);
      else
        atomicAdd(&cnt[u], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kGHash; q += kT)
      if (hk[q] != kGEmpty) atomicAdd(&cnt[hk[q]], hc[q]);
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanB) k_ig_scan_blocks(
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

__global__ void __launch_bounds__(1024) k_ig_scan_sums(unsigned* __restrict__ bsum,
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

__global__ void __launch_bounds__(kScanB) k_ig_scan_apply(
    unsigned* __restrict__ off, long long n, const unsigned* __restrict__ bsum) {
  const long long i = (long long)blockIdx.x * kScanB + threadIdx.x;
  if (i == 0) off[0] = 0u;
  if (i < n) off[i + 1] += bsum[blockIdx.x];
}

template <class PT>
__global__ void __launch_bounds__(kT) k_ig_scatter(
    Sp3<PT> S, const Counters* dc, GridC g, const unsigned* __restrict__ off,
    unsigned* __restrict__ cnt, Rec* __restrict__ rec, unsigned step,
    unsigned long long seed) {
  // Per chunk: the records' cells counted in LDS, one range per distinct
  // cell reserved with one global atomic, then each record placed at the
  // next slot of its cell's range (the order inside a cell is set later by
  // the rank pass).
  __shared__ unsigned hk[kGHash];
  __shared__ unsigned hc[kGHash];
  __shared__ unsigned hb[kGHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2],
                  nn = (long long)dc->n[1];
  long long lo, hi;
  block_range(ne + ni + nn, lo, hi);
  auto cell_of = [&](long long t, unsigned& s, unsigned& i) {
    s = t < ne ? 0u : (t < ne + ni ? 1u : 2u);
    i = (unsigned)(s == 0 ? t : (s == 1 ? t - ne : t - ne - ni));
    return s == 0 ? S.ke[i] : (s == 1 ? S.ki[i] : S.kn[i]);
  };
  for (long long b = lo; b < hi; b += kGChunk) {
    for (int q = threadIdx.x; q < kGHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kGChunk < hi ? b + kGChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned s, i;
      const uint32_t c0 = cell_of(t, s, i);
      if (c0 == kDead) continue;
      const int q = ghash_slot(hk, tile_major(c0, g));
      if (q >= 0) atomicAdd(&hc[q], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kGHash; q += kT) {
      const unsigned k = hk[q];
      if (k != kGEmpty) {
        const unsigned m = hc[q];
        hb[q] = off[k] + atomicSub(&cnt[k], m) - m;
        hc[q] = 0u;
      }
    }
    __syncthreads();
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned s, i;
      const uint32_t c0 = cell_of(t, s, i);
      if (c0 == kDead) continue;
      const unsigned c = tile_major(c0, g);
      // The table is unchanged since the count: a key found there then is
      // found again, one that found no room finds none again.
      const int q = ghash_slot(hk, c);
      const unsigned slot = q >= 0 ? hb[q] + atomicAdd(&hc[q], 1u)
                                   : off[c] + atomicSub(&cnt[c], 1u) - 1u;
      const unsigned long long id = s == 0 ? S.e.id[i] : (s == 1 ? S.i.id[i] : S.n.id[i]);
      Rec r;
      r.lo = ((unsigned long long)s << 62) | ord_key(id, step, seed);
      r.hi = (c << 2) | s;
      r.val = i;
      rec[slot] = r;
    }
    __syncthreads();
  }
}

// Cells of at most kSmall records, one thread per record: its rank in the
// cell's (key, id) order places it in the sorted array.  The first record
// of a crowded cell lists the cell for the workgroup pass.
template <class PT>
__global__ void __launch_bounds__(kT) k_ig_rank(
    Sp3<PT> S, const unsigned* __restrict__ off, long long nkeys,
    const Rec* __restrict__ rec, Rec* __restrict__ srt,
    unsigned* __restrict__ big, unsigned* __restrict__ nbig, long long big_cap) {
  long long lo, hi;
  block_range((long long)off[nkeys], lo, hi);
  for (long long p = lo + threadIdx.x; p < hi; p += kT) {
    const Rec r = rec[p];
    const unsigned c = r.hi >> 2;
    const unsigned b = off[c];
    const int n = (int)(off[c + 1] - b);
    if (n > kSmall) {
      if ((unsigned)p == b) {
        const unsigned slot = atomicAdd(nbig, 1u);
        if ((long long)slot < big_cap) big[slot] = c;
      }
    } else if (n >= 2) {
      int rank = 0;
      for (int j = 0; j < n; ++j) {
        const Rec x = rec[b + j];
        rank += (b + (unsigned)j != (unsigned)p) &&
                (x.lo < r.lo || (x.lo == r.lo && rid(S, x) < rid(S, r)));
      }
      srt[b + rank] = r;
    }
  }
}

struct Tally {
  unsigned long long rec = 0, cx = 0, starved = 0, near = 0;
};

// Electrons re[0..ne) against the cell's Cu+ ri[0..ni), both in their
// random order; returns the number of Cu+ taken.
template <class PT>
__device__ int ip_electrons(const Sp3<PT>& S, const Rec* re, int ne,
                            const Rec* ri, int ni, unsigned cell,
                            const IonC& k, const GridC& g,
                            int* __restrict__ ncount,
                            long long* __restrict__ acc,
                            uint32_t* __restrict__ dead2, Rec* __restrict__ ev,
                            uint2* __restrict__ evp, Counters* dc, Tally& t) {
  int used = 0;                                     // Cu+ taken by electrons
  if (ni > 0) {
    const double dens = (double)ni * k.w_dx3;
    for (int a = 0; a < ne; ++a) {
      const unsigned e = re[a].val;
      double vx, vy, vz;
      Acc<PT>::vel(S.e, e, vx, vy, vz);
      const double v2 = (vx * vx + vy * vy) + vz * vz;
      const double v = sqrt(v2);
      const double E = (k.half_me * v2) / kE;
      const double sr = sigma_rec(k, E), si = sigma_ion2(k, E);
      const double st = sr + si;
      const double P = 1.0 - exp(-(((dens * st) * v) * k.dt));
      const unsigned long long eid = S.e.id[e];
      double u1, u2;
      uniform2(eid, k.step, kTagEI0, k.seed, u1, u2);
      const double frac = sr / st;
      if (fabs(u1 - P) < kNear) t.near += 1;
      if (!(u1 < P)) continue;
      if (used >= ni) {
        t.starved += 1;
        continue;
      }
      if (fabs(u2 - frac) < kNear) t.near += 1;
      const unsigned ion = ri[used].val;
      ++used;
      S.ki[ion] = kDead;
      if ((long long)ion < k.nb_i) atomicSub(&k.tcnt_i[tile_of(cell, g)], 1u);
      const unsigned long long d2 = atomicAdd(&dc->n_dead2, 1ull);
      if (d2 < (unsigned long long)kDeadList) dead2[d2] = ion;
      if (u2 < frac) {
        // Recombination: a Cu atom with the ion's position and id and the
        // pair's centre-of-mass velocity; the electron and the ion leave.
        const unsigned long long slot = atomicAdd(&dc->n[1], 1ull);
        if ((long long)slot >= k.cap_n) {
          atomicOr(&dc->err, kErrCapacity);
        } else {
          double ivx, ivy, ivz;
          Acc<PT>::vel(S.i, ion, ivx, ivy, ivz);
          const double den = kMcu + kMe;
          Acc<PT>::copy_pos(S.i, ion, S.n, (long long)slot);
          Acc<PT>::set_vel(S.n, (long long)slot, (kMcu * ivx + kMe * vx) / den,
                           (kMcu * ivy + kMe * vy) / den,
                           (kMcu * ivz + kMe * vz) / den);
          S.n.id[slot] = S.i.id[ion];
          S.kn[slot] = cell;
          atomicAdd(&ncount[cell], 1);
        }
        S.ke[e] = kDead;
        if ((long long)e < k.nb_e) atomicSub(&k.tcnt_e[tile_of(cell, g)], 1u);
        dep_add(S.e, e, g, acc, 1);
        dep_add(S.i, ion, g, acc, -1);
        t.rec += 1;
      } else {
        const unsigned long long q = atomicAdd(&dc->f3_ion2, 1ull);
        if ((long long)q < k.max_ev) {
          Rec x;
          x.lo = eid;
          x.hi = 0u;
          x.val = (unsigned)q;
          ev[q] = x;
          evp[q] = make_uint2(e, ion);
        } else {
          atomicOr(&dc->err, kErrEvents);
        }
      }
    }
  }
  return used;
}

// Charge exchange trial of one Cu+ with one atom of its cell (nn atoms).
template <class PT>
__device__ void cx_pair(const Sp3<PT>& S, unsigned ion, unsigned at, int nn,
                        const IonC& k, const GridC& g,
                        long long* __restrict__ acc, Tally& t) {
  const double dens = (double)nn * k.w_dx3;
  const double mr = 0.5 * kMcu;
  double ix, iy, iz, nx, ny, nz;
  Acc<PT>::vel(S.i, ion, ix, iy, iz);
  Acc<PT>::vel(S.n, at, nx, ny, nz);
  const double ux = ix - nx, uy = iy - ny, uz = iz - nz;
  const double u2 = (ux * ux + uy * uy) + uz * uz;
  const double u = sqrt(u2);
  const double eps = ((0.5 * mr) * u2) / kE;
  const double P = 1.0 - exp(-(((dens * sigma_cx(k, eps)) * u) * k.dt));
  double u1, u1b;
  uniform2(S.i.id[ion], k.step, kTagCX, k.seed, u1, u1b);
  if (fabs(u1 - P) < kNear) t.near += 1;
  if (u1 < P) {
    dep_add(S.i, ion, g, acc, -1);
    swap_records(S.i, ion, S.n, at);
    dep_add(S.i, ion, g, acc, 1);
    t.cx += 1;
  }
}

// One small cell's processes on records r[0..n) in (key, id) order:
// electrons, then Cu+, then atoms.
template <class PT>
__device__ void ip_cell(const Sp3<PT>& S, const Rec* r, int n, unsigned cell,
                        const IonC& k, const GridC& g, int* __restrict__ ncount,
                        long long* __restrict__ acc, uint32_t* __restrict__ dead2,
                        Rec* __restrict__ ev, uint2* __restrict__ evp,
                        Counters* dc, Tally& t) {
  int ne = 0, ni = 0;
  while (ne < n && ip_sp(r[ne]) == 0u) ++ne;
  while (ne + ni < n && ip_sp(r[ne + ni]) == 1u) ++ni;
  const int nn = n - ne - ni;
  const Rec* ri = r + ne;
  const Rec* rn = r + ne + ni;
  int used = 0;
  if (ni > 0)
    used = ip_electrons(S, r, ne, ri, ni, cell, k, g, ncount, acc, dead2, ev,
                        evp, dc, t);
  // Charge exchange of the Cu+ left with the cell's atoms.
  if (nn > 0)
    for (int a = used; a < ni; ++a)
      cx_pair(S, ri[a].val, rn[(a - used) % nn].val, nn, k, g, acc, t);
}

template <class PT>
__device__ void flush_tally(const Tally& t, Counters* dc) {
  if (t.rec) atomicAdd(&dc->f3_rec, t.rec);
  if (t.cx) atomicAdd(&dc->f3_cx, t.cx);
  if (t.starved) atomicAdd(&dc->f3_starved, t.starved);
  if (t.near) atomicAdd(&dc->n_near, t.near);
}

// Small cells with a Cu+, one thread each, on the sorted records.
template <class PT>
__global__ void __launch_bounds__(kT) k_ip_small(
    Sp3<PT> S, const unsigned* __restrict__ off, long long nkeys,
    const Rec* __restrict__ srt, IonC k, GridC g,
    int* __restrict__ ncount, long long* __restrict__ acc,
    uint32_t* __restrict__ dead2, Rec* __restrict__ ev,
    uint2* __restrict__ evp, Counters* dc) {
  Tally t;
  long long lo, hi;
  block_range(nkeys, lo, hi);
  for (long long c = lo + threadIdx.x; c < hi; c += kT) {
    const unsigned b = off[c], e = off[c + 1];
    const int n = (int)(e - b);
    if (n < 2 || n > kSmall) continue;
    const Rec* r = srt + b;
    // Nothing to do without a Cu+.
    bool has_ion = false;
    for (int j = 0; j < n; ++j) has_ion = has_ion || ip_sp(r[j]) == 1u;
    if (has_ion)
      ip_cell(S, r, n, cell_of_tile_major((unsigned)c, g), k, g, ncount, acc,
              dead2, ev, evp, dc, t);
  }
  flush_tally<PT>(t, dc);
}

// Block-wide sort of s[0..n) (n <= cap, cap a power of two) by key, then
// equal keys by id.  Called by every thread of the workgroup.
template <class PT>
__device__ void wg_sort(const Sp3<PT>& S, Rec* s, int n) {
  int np2 = 1;
  while (np2 < n) np2 <<= 1;
  for (int j = n + threadIdx.x; j < np2; j += kT) {
    Rec x;
    x.lo = ~0ull;
    x.hi = 3u;
    x.val = 0u;
    s[j] = x;
  }
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = threadIdx.x; j < np2; j += kT) {
        const int p = j ^ stride;
        if (p > j) {
          const bool up = (j & size) == 0;
          const bool sw = up ? s[j].lo > s[p].lo : s[j].lo < s[p].lo;
          if (sw) {
            const Rec x = s[j];
            s[j] = s[p];
            s[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    for (int j = 1; j < n; ++j) {
      int m = j;
      while (m > 0 && s[m].lo == s[m - 1].lo && rid(S, s[m]) < rid(S, s[m - 1])) {
        const Rec x = s[m];
        s[m] = s[m - 1];
        s[m - 1] = x;
        --m;
      }
    }
  }
  __syncthreads();
}

struct Sel {
  unsigned long long T;              // inclusive upper bound of the window
  int state;                         // 0 refine, 1 done, 2 too many equal keys
  int chosen, below;
};

// The next window of a crowded cell's atoms in their random order: those
// whose order draw lies in (lb, T], with T the smallest bound that holds
// `want` of them, found by radix selection over the 53-bit draw (8 bits a
// pass), relaxed to the end of a digit bin while the window fits kWin.
// Called by every thread; the result is left in *sel (state 2: error).
__device__ void select_window(const Rec* __restrict__ r, int n, long long lb,
                              int want, unsigned* hist, Sel* sel) {
  unsigned long long pv = 0, pm = 0;
  int below = 0;
  for (int sh = 45;; sh = sh >= 8 ? sh - 8 : 0) {
    for (int i = threadIdx.x; i < 256; i += kT) hist[i] = 0u;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kT) {
      const Rec x = r[j];
      if (ip_sp(x) != 2u) continue;
      const unsigned long long o = x.lo & kOrdMask;
      if ((long long)o <= lb || (o & pm) != pv) continue;
      atomicAdd(&hist[(o >> sh) & 0xFFu], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int cum = below, chosen = -1;
      for (int b = 0; b < 256; ++b) {
        if (cum + (int)hist[b] >= want) {
          chosen = b;
          break;
        }
        cum += (int)hist[b];
      }
      Sel d;
      d.chosen = chosen;
      d.below = cum;
      if (chosen < 0) {                  // fewer than want left: take them all
        d.state = 1;
        d.T = kOrdMask;
      } else {
        const int through = cum + (int)hist[chosen];
        d.T = pv | ((unsigned long long)chosen << sh) | ((1ull << sh) - 1ull);
        d.state = through <= kWin ? 1 : (sh == 0 ? 2 : 0);
      }
      *sel = d;
    }
    __syncthreads();
    const Sel d = *sel;
    if (d.state != 0) return;
    pv |= (unsigned long long)d.chosen << sh;
    pm |= 0xFFull << sh;
    below = d.below;
  }
}

// Crowded cells, one workgroup each.  The charged records are gathered and
// sorted in LDS and the electrons run against the Cu+ by the first thread
// (sequential by definition).  The atoms, however many, are never sorted as
// a whole: the live Cu+ take them window by window of the atoms' random
// order, each window selected by radix selection and sorted in LDS, the
// order starting again from the first atom when the ions outnumber them.
template <class PT>
__global__ void __launch_bounds__(kT) k_ip_big(
    Sp3<PT> S, const unsigned* __restrict__ off, const Rec* __restrict__ rec,
    const unsigned* __restrict__ big, const unsigned* __restrict__ nbig,
    long long big_cap, IonC k, GridC g, int* __restrict__ ncount,
    long long* __restrict__ acc, uint32_t* __restrict__ dead2,
    Rec* __restrict__ ev, uint2* __restrict__ evp, Counters* dc) {
  __shared__ Rec sr[kBigCell];
  __shared__ Rec sn[kWin];
  __shared__ unsigned hist[256];
  __shared__ Sel sel;
  __shared__ int s_nc, s_ni, s_w, s_used;
  long long nlist = (long long)*nbig;
  if (nlist > big_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&dc->err, kErrEvents);
    nlist = big_cap;
  }
  Tally t;
  for (long long q = blockIdx.x; q < nlist; q += gridDim.x) {
    const unsigned key = big[q];
    const unsigned c = cell_of_tile_major(key, g);
    const unsigned b = off[key];
    const int n = (int)(off[key + 1] - b);
    const Rec* r = rec + b;
    __syncthreads();
    if (threadIdx.x == 0) {
      s_nc = 0;
      s_ni = 0;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += kT) {
      const Rec x = r[j];
      if (ip_sp(x) >= 2u) continue;
      const int slot = atomicAdd(&s_nc, 1);
      if (slot < kBigCell) sr[slot] = x;
      if (ip_sp(x) == 1u) atomicAdd(&s_ni, 1);
    }
    __syncthreads();
    const int nc = s_nc, ni = s_ni, nn = n - nc, ne = nc - ni;
    if (ni == 0) continue;
    if (nc > kBigCell) {
      if (threadIdx.x == 0) atomicOr(&dc->err, kErrEvents);
      continue;
    }
    wg_sort(S, sr, nc);
    if (threadIdx.x == 0)
      s_used = ip_electrons(S, sr, ne, sr + ne, ni, c, k, g, ncount, acc, dead2,
                            ev, evp, dc, t);
    __syncthreads();
    const int used = s_used;
    const int live = ni - used;
    const Rec* ri = sr + ne + used;
    int m = 0, rank = 0;
    long long lb = -1;
    while (nn > 0 && m < live) {
      const int want = min(min(nn - rank, live - m), kWin);
      select_window(r, n, lb, want, hist, &sel);
      const Sel d = sel;
      if (d.state == 2) {
        if (threadIdx.x == 0) atomicOr(&dc->err, kErrEvents);
        break;
      }
      if (threadIdx.x == 0) s_w = 0;
      __syncthreads();
      for (int j = threadIdx.x; j < n; j += kT) {
        const Rec x = r[j];
        if (ip_sp(x) != 2u) continue;
        const unsigned long long o = x.lo & kOrdMask;
        if ((long long)o <= lb || o > d.T) continue;
        const int slot = atomicAdd(&s_w, 1);
        if (slot < kWin) sn[slot] = x;
      }
      __syncthreads();
      const int w = min(s_w, kWin);
      wg_sort(S, sn, w);
      const int take = min(w, live - m);
      if (threadIdx.x == 0)
        for (int a = 0; a < take; ++a)
          cx_pair(S, ri[m + a].val, sn[a].val, nn, k, g, acc, t);
      m += take;
      rank += w;
      lb = (long long)d.T;
      if (rank >= nn) {                  // every atom met: the order restarts
        rank = 0;
        lb = -1;
      }
      __syncthreads();
    }
  }
  flush_tally<PT>(t, dc);
}

// Listed Cu+ ionisations in primary-id order: kinematics, the secondary
// (id next_id + rank) and the Cu2+.
template <class PT>
__global__ void k_ip_commit(Sp3<PT> S, PT p3, uint32_t* __restrict__ k3,
                            const Rec* __restrict__ ev,
                            const uint2* __restrict__ evp, IonC k, GridC g,
                            long long cap_e, long long cap_3,
                            long long* __restrict__ acc, Counters* dc) {
  long long nev = (long long)dc->f3_ion2;
  if (nev > k.max_ev) nev = k.max_ev;
  const long long ne0 = (long long)dc->n[0], n30 = (long long)dc->n[3];
  const unsigned long long id0 = dc->next_id;
  for (long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x; r < nev;
       r += (long long)gridDim.x * blockDim.x) {
    const uint2 pr = evp[ev[r].val];
    const unsigned e = pr.x, ion = pr.y;
    const unsigned long long pid = ev[r].lo;
    double vx, vy, vz;
    Acc<PT>::vel(S.e, e, vx, vy, vz);
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    const double E = (k.half_me * v2) / kE;
    double u3, u4, u5, u6, u7, u8;
    uniform2(pid, k.step, kTagEI1, k.seed, u3, u4);
    uniform2(pid, k.step, kTagEI2, k.seed, u5, u6);
    uniform2(pid, k.step, kTagEI3, k.seed, u7, u8);
    const double avail = E - k.I2;
    const double Es = u3 * avail;
    const double Ep = avail - Es;
    const double vp = sqrt(Ep * k.two_e_me);
    const double vs = sqrt(Es * k.two_e_me);
    double c, s, ps;
    c = 1.0 - 2.0 * u4; s = sqrt(1.0 - c * c); ps = kTwoPi * u5;
    const double px = s * cos(ps), py = s * sin(ps), pz = c;
    c = 1.0 - 2.0 * u6; s = sqrt(1.0 - c * c); ps = kTwoPi * u7;
    const double sx = s * cos(ps), sy = s * sin(ps), sz = c;
    const long long de = ne0 + r, d3 = n30 + r;
    if (de >= cap_e || d3 >= cap_3) {
      atomicOr(&dc->err, kErrCapacity);
      continue;
    }
    Acc<PT>::set_vel(S.e, e, vp * px, vp * py, vp * pz);
    Acc<PT>::copy_pos(S.e, e, S.e, de);
    Acc<PT>::set_vel(S.e, de, vs * sx, vs * sy, vs * sz);
    S.e.id[de] = id0 + (unsigned long long)r;
    S.ke[de] = S.ke[e];
    Acc<PT>::copy(S.i, ion, p3, d3);
    k3[d3] = S.ke[e];
    // One more charge on the ion, one more electron.
    dep_add(S.i, ion, g, acc, 1);
    dep_add(S.e, e, g, acc, -1);
  }
}

__global__ void k_ip_counts(Counters* dc, long long max_ev, long long cap_e,
                            long long cap_3, long long cap_n) {
  long long nev = (long long)dc->f3_ion2;
  if (nev > max_ev) nev = max_ev;
  unsigned long long ne = dc->n[0] + (unsigned long long)nev;
  unsigned long long n3 = dc->n[3] + (unsigned long long)nev;
  dc->n[0] = ne > (unsigned long long)cap_e ? (unsigned long long)cap_e : ne;
  dc->n[3] = n3 > (unsigned long long)cap_3 ? (unsigned long long)cap_3 : n3;
  dc->next_id += (unsigned long long)nev;
  // Atom appends past the capacity were dropped (and flagged): keep the
  // count within it.
  if (dc->n[1] > (unsigned long long)cap_n) dc->n[1] = (unsigned long long)cap_n;
}

template <class PT>
Sp3<PT> sp3(pic_ctx* c);
template <>
Sp3<Parts> sp3<Parts>(pic_ctx* c) {
  return Sp3<Parts>{c->P[0][c->cur[0]], c->P[2][c->cur[2]], c->P[1][c->cur[1]],
                    c->key[0], c->key[2], c->key[1]};
}
template <>
Sp3<PartsM> sp3<PartsM>(pic_ctx* c) {
  return Sp3<PartsM>{c->PM[0][c->cur[0]], c->PM[2][c->cur[2]],
                     c->PM[1][c->cur[1]], c->key[0], c->key[2], c->key[1]};
}
template <class PT>
PT sp_cur(pic_ctx* c, int s);
template <>
Parts sp_cur<Parts>(pic_ctx* c, int s) { return c->P[s][c->cur[s]]; }
template <>
PartsM sp_cur<PartsM>(pic_ctx* c, int s) { return c->PM[s][c->cur[s]]; }

template <class PT>
void ionproc_t(pic_ctx* c, double dt) {
  hipStream_t st = c->stream;
  const long long nc = c->cg_nkeys;          // tile-major cell numbers
  const pic_ion_processes& q = c->ionp;
  IonC k;
  k.s_rec = q.sigma_rec_1eV;
  k.a2 = q.lotz_a2;
  k.I2 = q.ion2_I_eV;
  k.cx_a = q.cx_a;
  k.cx_b = q.cx_b;
  const double inv = c->g.inv_dx;
  k.w_dx3 = (double)c->cfg.w_sp * ((inv * inv) * inv);
  k.dt = dt;
  k.half_me = 0.5 * kMe;
  k.two_e_me = (2.0 * kE) / kMe;
  k.step = (unsigned)c->step;
  k.seed = c->cfg.seed;
  k.cap_n = c->cfg.capacity[1];
  k.max_ev = c->cfg.max_events;
  k.nb_e = c->tcounted ? c->n_binned[0] : 0;
  k.nb_i = c->tcounted ? c->n_binned[2] : 0;
  k.tcnt_e = c->tcnt[0];
  k.tcnt_i = c->tcnt[1];
  const Sp3<PT> S = sp3<PT>(c);
  hipMemsetAsync(c->cg_cnt, 0, nc * sizeof(unsigned), st);
  hipMemsetAsync(c->cg_nbig, 0, sizeof(unsigned), st);
  // Grids of a multiple of 8 workgroups (see xcd_block).
  k_ig_count<<<4096, kT, 0, st>>>(c->key[0], c->key[2], c->key[1], c->dc, c->g,
                                  c->cg_cnt);
  const long long nb = (nc + kScanB - 1) / kScanB;
  k_ig_scan_blocks<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_cnt, nc, c->cg_off,
                                                   c->cg_bsum);
  k_ig_scan_sums<<<1, 1024, 0, st>>>(c->cg_bsum, (int)nb);
  k_ig_scan_apply<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_off, nc, c->cg_bsum);
  k_ig_scatter<PT><<<4096, kT, 0, st>>>(S, c->dc, c->g, c->cg_off, c->cg_cnt,
                                        c->cg_rec, k.step, k.seed);
  k_ig_rank<PT><<<8192, kT, 0, st>>>(S, c->cg_off, nc, c->cg_rec, c->cg_srt,
                                     c->cg_big, c->cg_nbig, c->cg_big_cap);
  k_ip_small<PT><<<8192, kT, 0, st>>>(S, c->cg_off, nc, c->cg_srt, k, c->g,
                                      c->ncount, c->acc_next, c->dead2,
                                      c->ip_ev, c->ip_evp, c->dc);
  k_ip_big<PT><<<512, kT, 0, st>>>(S, c->cg_off, c->cg_rec, c->cg_big,
                                   c->cg_nbig, c->cg_big_cap, k, c->g,
                                   c->ncount, c->acc_next, c->dead2, c->ip_ev,
                                   c->ip_evp, c->dc);
  sort_event_records(c, c->ip_ev, &c->dc->f3_ion2);
  k_ip_commit<PT><<<64, kT, 0, st>>>(S, sp_cur<PT>(c, 3), c->key[3], c->ip_ev,
                                     c->ip_evp, k, c->g, c->cfg.capacity[0],
                                     c->cfg.capacity[3], c->acc_next, c->dc);
  k_ip_counts<<<1, 1, 0, st>>>(c->dc, k.max_ev, c->cfg.capacity[0],
                               c->cfg.capacity[3], c->cfg.capacity[1]);
}

}  // namespace

void parts_ion_processes(pic_ctx* c, double dt) {
  if (c->mixed)
    ionproc_t<PartsM>(c, dt);
  else
    ionproc_t<Parts>(c, dt);
}

}  // namespace pic
