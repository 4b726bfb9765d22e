// Recombination (e + Cu+ -> Cu), electron-impact ionisation of Cu+
// (e + Cu+ -> 2e + Cu2+) and resonant charge exchange (Cu+ + Cu -> Cu + Cu+):
// the paper's remaining Monte Carlo collision processes and the higher
// charge state they lead to.
//
// Electrons, Cu+ and Cu atoms are grouped by cell: their index words are
// binned by tile plane as for the Coulomb collisions, then one wavefront a
// plane writes the cells' offsets and, in each cell's segment, 16-byte
// records keyed by species and a random order draw: sorted by (key, id) in
// cells of at most kSmall, unsorted in the crowded ones (the few planes of
// many records, the atoms piled above an evaporating spot, are grouped by
// cell over the whole GPU instead).  Every cell is then processed in
// sequence by one thread (a workgroup sorts the crowded ones, their atoms a
// window at a time): first each electron in turn against the
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

// A cell's records in (key, id) order as a plane pass holds them in LDS:
// the keys and index words by slot, the sorted places' slots in perm.
struct LdsRecs {
  const unsigned long long* key;    // species in the top two bits
  const unsigned* ix;               // array indices
  const unsigned short* perm;
  int b;                            // the cell's first place
  unsigned cell;                    // its tile-major number
  __device__ Rec operator[](int j) const {
    const int p = perm[b + j];
    Rec r;
    r.lo = key[p];
    r.hi = (cell << 2) | (unsigned)(key[p] >> 62);
    r.val = ix[p];
    return r;
  }
  __device__ LdsRecs operator+(int d) const {
    LdsRecs x = *this;
    x.b += d;
    return x;
  }
};

struct Tally {
  unsigned long long rec = 0, cx = 0, starved = 0, near = 0;
};

// Electrons re[0..ne) against the cell's Cu+ ri[0..ni), both in their
// random order; returns the number of Cu+ taken.
template <class PT, class RV>
__device__ int ip_electrons(const Sp3<PT>& S, RV re, int ne,
                            RV ri, int ni, unsigned cell,
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
template <class PT, class RV>
__device__ void ip_cell(const Sp3<PT>& S, RV r, int n, unsigned cell,
                        const IonC& k, const GridC& g, int* __restrict__ ncount,
                        long long* __restrict__ acc, uint32_t* __restrict__ dead2,
                        Rec* __restrict__ ev, uint2* __restrict__ evp,
                        Counters* dc, Tally& t) {
  int ne = 0, ni = 0;
  while (ne < n && ip_sp(r[ne]) == 0u) ++ne;
  while (ne + ni < n && ip_sp(r[ne + ni]) == 1u) ++ni;
  const int nn = n - ne - ni;
  const RV ri = r + ne;
  const RV rn = r + ne + ni;
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

// ---- grouping ----------------------------------------------------------------
// Particle t of the joint range (electrons, Cu+, atoms): its key and its
// index word t.

template <class PT>
__device__ __forceinline__ uint32_t joint_key(const Sp3<PT>& S, long long ne,
                                              long long ni, long long t,
                                              unsigned& gi) {
  gi = (unsigned)t;
  if (t < ne) return S.ke[t];
  if (t < ne + ni) return S.ki[t - ne];
  return S.kn[t - ne - ni];
}

template <class PT>
__device__ __forceinline__ uint32_t key_of(const Sp3<PT>& S, const JointIx& J,
                                           unsigned gi) {
  const unsigned s = J.sp(gi), i = J.ix(gi);
  return s == 0 ? S.ke[i] : (s == 1 ? S.ki[i] : S.kn[i]);
}

// The sort record of a particle: species above its order draw; its
// tile-major cell above the species; its index.
template <class PT>
__device__ __forceinline__ Rec make_rec(const Sp3<PT>& S, const JointIx& J,
                                        unsigned gi, unsigned cell,
                                        unsigned step, unsigned long long seed) {
  const unsigned s = J.sp(gi), i = J.ix(gi);
  const unsigned long long id = s == 0 ? S.e.id[i] : (s == 1 ? S.i.id[i] : S.n.id[i]);
  Rec r;
  r.lo = ((unsigned long long)s << 62) | ord_key(id, step, seed);
  r.hi = (cell << 2) | s;
  r.val = i;
  return r;
}

// The id of a particle given its sort key (species in the top two bits)
// and its array index.
template <class PT>
__device__ __forceinline__ unsigned long long key_id(const Sp3<PT>& S,
                                                     unsigned long long key,
                                                     unsigned i) {
  const unsigned s = (unsigned)(key >> 62);
  return s == 0 ? S.e.id[i] : (s == 1 ? S.i.id[i] : S.n.id[i]);
}

// Live particles per plane.
template <class PT>
__global__ void __launch_bounds__(kT) k_pg_count(Sp3<PT> S, const Counters* dc,
                                                 GridC g,
                                                 unsigned* __restrict__ cnt) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2],
                  nn = (long long)dc->n[1];
  long long lo, hi;
  block_range(ne + ni + nn, lo, hi);
  for (long long b = lo; b < hi; b += kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kPChunk < hi ? b + kPChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = joint_key(S, ne, ni, t, gi);
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

// Each live particle's index word into its plane's range (order inside the
// range arbitrary); per chunk one range per distinct plane is reserved with
// one global atomic.
template <class PT>
__global__ void __launch_bounds__(kT) k_pg_scatter(
    Sp3<PT> S, const Counters* dc, GridC g, const unsigned* __restrict__ poff,
    unsigned* __restrict__ cnt, unsigned* __restrict__ pidx) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  __shared__ unsigned hb[kPHash];
  const long long ne = (long long)dc->n[0], ni = (long long)dc->n[2],
                  nn = (long long)dc->n[1];
  long long lo, hi;
  block_range(ne + ni + nn, lo, hi);
  for (long long b = lo; b < hi; b += kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const long long e = b + kPChunk < hi ? b + kPChunk : hi;
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = joint_key(S, ne, ni, t, gi);
      if (c == kDead) continue;
      const int q = plane_slot(hk, plane_of(c, g));
      if (q >= 0) atomicAdd(&hc[q], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      const unsigned u = hk[q];
      if (u != kGEmpty) {
        const unsigned m = hc[q];
        hb[q] = poff[u] + atomicSub(&cnt[u], m) - m;
        hc[q] = 0u;
      }
    }
    __syncthreads();
    for (long long t = b + threadIdx.x; t < e; t += kT) {
      unsigned gi;
      const uint32_t c = joint_key(S, ne, ni, t, gi);
      if (c == kDead) continue;
      const unsigned u = plane_of(c, g);
      // The table is unchanged since the count (see k_cu_scatter).
      const int q = plane_slot(hk, u);
      const unsigned slot = q >= 0 ? hb[q] + atomicAdd(&hc[q], 1u)
                                   : poff[u] + atomicSub(&cnt[u], 1u) - 1u;
      pidx[slot] = gi;
    }
    __syncthreads();
  }
}

// Per plane, one wavefront: its cells' offsets into off (a global prefix
// over the tile-major cells), the records of its crowded cells (more than
// kSmall) into rec unsorted, those cells listed for the workgroup pass.
// A plane of at most kPCap records is read once; its small cells (2 to
// kSmall records) are ranked in LDS and their processes run right there, a
// cell per lane, on the sorted records in LDS.  A larger plane ranks its
// small cells in batches into srt and is listed for k_ip_small; a plane of
// more than kHot records is listed for the hot-plane passes (and
// k_ip_small).  Four wavefronts per SIMD (128 registers, seven spilled):
// 1.11 ms against 1.25 at three, at the 128x128x512 workload.
constexpr int kPCap = 512;
constexpr int kHot = 4096;

struct PlaneLds {
  unsigned long long key[kPCap];
  unsigned gi[kPCap];             // array indices (the species is in key)
  unsigned char cell[kPCap];
  unsigned short ord[kPCap];      // one-pass plane: cell order -> slot
  unsigned short perm[kPCap];     // one-pass plane: sorted place -> slot
  unsigned cnt[kPlaneCells];
  unsigned off[kPlaneCells + 1];
  unsigned start[kPlaneCells];    // batch-local first slot of a small cell
  unsigned cur[kPlaneCells];
  int hi, nb;
};

__device__ __forceinline__ bool small_cell(unsigned m) {
  return m >= 2u && m <= (unsigned)kSmall;
}

template <class PT>
__global__ void __launch_bounds__(kPlaneCells, 4) k_pg_cells(
    Sp3<PT> S, GridC g, const unsigned* __restrict__ poff, long long nplanes,
    const unsigned* __restrict__ pidx, unsigned* __restrict__ off,
    Rec* __restrict__ rec, Rec* __restrict__ srt, unsigned* __restrict__ big,
    unsigned* __restrict__ nbig, long long big_cap, unsigned* __restrict__ hot,
    unsigned* __restrict__ nhot, unsigned* __restrict__ rest,
    unsigned* __restrict__ nrest, IonC k, int* __restrict__ ncount,
    long long* __restrict__ acc, uint32_t* __restrict__ dead2,
    Rec* __restrict__ ev, uint2* __restrict__ evp, Counters* dc) {
  __shared__ PlaneLds L;
  const int tid = (int)threadIdx.x;
  const unsigned step = k.step;
  const unsigned long long seed = k.seed;
  Tally t;

  for (long long u = plane_first(); u < nplanes; u += gridDim.x) {
    const unsigned base = poff[u];
    const int n = (int)(poff[u + 1] - base);
    const unsigned c0 = (unsigned)u << kPlaneShift;
    // (Read per plane, so that it is not held through the processes.)
    const JointIx J = joint_ix(dc);
    if (n > kHot) {
      if (tid == 0) {
        hot[atomicAdd(nhot, 1u)] = (unsigned)u;
        rest[atomicAdd(nrest, 1u)] = (unsigned)u;
      }
      continue;
    }
    L.cnt[tid] = 0u;
    __syncthreads();
    // A plane of at most kPCap records is read once: its records are made
    // as it is counted and kept in LDS in load order.
    const bool one = n <= kPCap;
    for (int j = tid; j < n; j += kPlaneCells) {
      const unsigned gi = pidx[base + j];
      const unsigned c = tile_major(key_of(S, J, gi), g);
      const int lc = (int)(c & (kPlaneCells - 1));
      atomicAdd(&L.cnt[lc], 1u);
      if (one) {
        L.key[j] = make_rec(S, J, gi, c, step, seed).lo;
        L.gi[j] = J.ix(gi);
        L.cell[j] = (unsigned char)lc;
      }
    }
    __syncthreads();
    const unsigned m = L.cnt[tid];
    {
      unsigned incl = m;
      for (int o = 1; o < kPlaneCells; o <<= 1) {
        const unsigned y = __shfl_up(incl, o);
        if (tid >= o) incl += y;
      }
      L.off[tid] = incl - m;
      off[c0 + tid] = base + incl - m;
      if (tid == kPlaneCells - 1) {
        L.off[kPlaneCells] = incl;
        if (u == nplanes - 1) off[c0 + kPlaneCells] = base + incl;
      }
    }
    __syncthreads();
    if (one) {
      // Crowded cells' records from LDS into their segments; the small
      // cells' slots in cell order, ranked by (key, id) into srt.
      L.cur[tid] = L.off[tid];
      if (m > (unsigned)kSmall) {
        const unsigned q = atomicAdd(nbig, 1u);
        if ((long long)q < big_cap) big[q] = c0 + tid;
      }
      __syncthreads();
      for (int j = tid; j < n; j += kPlaneCells) {
        const int lc = L.cell[j];
        const unsigned mc = L.cnt[lc];
        const unsigned x = atomicAdd(&L.cur[lc], 1u);
        L.ord[x] = (unsigned short)j;
        if (mc > (unsigned)kSmall) {
          Rec r;
          r.lo = L.key[j];
          r.hi = ((c0 + (unsigned)lc) << 2) | (unsigned)(L.key[j] >> 62);
          r.val = L.gi[j];
          rec[base + x] = r;
        }
      }
      __syncthreads();
      for (int x = tid; x < n; x += kPlaneCells) {
        const int j = L.ord[x];
        const int lc = L.cell[j];
        if (!small_cell(L.cnt[lc])) continue;
        const int b = (int)L.off[lc], mc = (int)L.cnt[lc];
        const unsigned long long kp = L.key[j];
        int rank = 0;
        for (int y = b; y < b + mc; ++y) {
          const int o = L.ord[y];
          const unsigned long long ky = L.key[o];
          if (ky < kp) {
            ++rank;
          } else if (ky == kp && o != j) {
            rank += key_id(S, L.key[o], L.gi[o]) < key_id(S, kp, L.gi[j]);
          }
        }
        L.perm[b + rank] = (unsigned short)j;
      }
      __syncthreads();
      // The processes of the plane's small cells with a Cu+, a cell per
      // lane, on the sorted records in LDS.
      const unsigned mc = L.cnt[tid];
      if (small_cell(mc)) {
        LdsRecs r{L.key, L.gi, L.perm, (int)L.off[tid], c0 + tid};
        bool has_ion = false;
        for (int j = 0; j < (int)mc; ++j) has_ion = has_ion || ip_sp(r[j]) == 1u;
        if (has_ion)
          ip_cell(S, r, (int)mc, cell_of_tile_major(c0 + tid, g), k, g, ncount,
                  acc, dead2, ev, evp, dc, t);
      }
      __syncthreads();
      continue;
    }
    // A larger plane: its small cells' records go to srt and k_ip_small
    // runs them.
    if (tid == 0) rest[atomicAdd(nrest, 1u)] = (unsigned)u;
    // Crowded cells: records straight into their segments, unsorted.
    if (__ballot(m > (unsigned)kSmall)) {
      L.cur[tid] = L.off[tid];
      if (m > (unsigned)kSmall) {
        const unsigned q = atomicAdd(nbig, 1u);
        if ((long long)q < big_cap) big[q] = c0 + tid;
      }
      __syncthreads();
      for (int j = tid; j < n; j += kPlaneCells) {
        const unsigned gi = pidx[base + j];
        const unsigned c = tile_major(key_of(S, J, gi), g);
        const int lc = (int)(c & (kPlaneCells - 1));
        if (L.cnt[lc] > (unsigned)kSmall)
          rec[base + atomicAdd(&L.cur[lc], 1u)] = make_rec(S, J, gi, c, step, seed);
      }
      __syncthreads();
    }
    // Small cells in batches.
    for (int c_lo = 0; c_lo < kPlaneCells;) {
      if (tid == 0) {
        int c_hi = c_lo, nb = 0;
        while (c_hi < kPlaneCells) {
          const unsigned mc = L.cnt[c_hi];
          const int add = small_cell(mc) ? (int)mc : 0;
          if (nb + add > kPCap) break;
          L.start[c_hi] = (unsigned)nb;
          L.cur[c_hi] = (unsigned)nb;
          nb += add;
          ++c_hi;
        }
        L.hi = c_hi;
        L.nb = nb;
      }
      __syncthreads();
      const int c_hi = L.hi, nb = L.nb;
      if (nb > 0) {
        for (int j = tid; j < n; j += kPlaneCells) {
          const unsigned gi = pidx[base + j];
          const uint32_t kc = key_of(S, J, gi);
          const int lc = (int)(tile_major(kc, g) & (kPlaneCells - 1));
          if (lc < c_lo || lc >= c_hi || !small_cell(L.cnt[lc])) continue;
          const int p = (int)atomicAdd(&L.cur[lc], 1u);
          const Rec r = make_rec(S, J, gi, c0 + lc, step, seed);
          L.key[p] = r.lo;
          L.gi[p] = J.ix(gi);
          L.cell[p] = (unsigned char)lc;
        }
        __syncthreads();
        for (int p = tid; p < nb; p += kPlaneCells) {
          const int lc = L.cell[p];
          const int b = (int)L.start[lc], mc = (int)L.cnt[lc];
          const unsigned long long kp = L.key[p];
          int rank = 0;
          for (int q = b; q < b + mc; ++q) {
            const unsigned long long kq = L.key[q];
            if (kq < kp) {
              ++rank;
            } else if (kq == kp && q != p) {
              // Equal draws (practically never): id order.
              rank += key_id(S, kq, L.gi[q]) < key_id(S, kp, L.gi[p]);
            }
          }
          Rec r;
          r.lo = kp;
          r.hi = ((c0 + (unsigned)lc) << 2) | (unsigned)(kp >> 62);
          r.val = L.gi[p];
          srt[base + L.off[lc] + rank] = r;
        }
      }
      __syncthreads();
      c_lo = c_hi;
    }
  }
  // The tallies, summed over the wavefront.
  for (int o = 32; o > 0; o >>= 1) {
    t.rec += __shfl_xor(t.rec, o);
    t.cx += __shfl_xor(t.cx, o);
    t.starved += __shfl_xor(t.starved, o);
    t.near += __shfl_xor(t.near, o);
  }
  if (tid == 0) flush_tally<PT>(t, dc);
}

// Planes of more than kHot records (the atoms piled above an evaporating
// spot): their records, taken together as one range (the planes' sizes
// prefixed), are grouped by cell over the whole GPU: a count per cell
// aggregated per chunk in LDS, each plane's cell offsets, a scatter into
// the cells' segments with one reservation per chunk and cell, and the few
// small cells' records ranked from there.  Per-cell counters of hot plane h
// are hcnt[64 h + cell].
__global__ void __launch_bounds__(1024) k_ph_prep(
    const unsigned* __restrict__ poff, const unsigned* __restrict__ hot,
    const unsigned* __restrict__ nhot, unsigned* __restrict__ hpre,
    unsigned* __restrict__ hcnt) {
  __shared__ unsigned s[1024];
  const int nh = (int)*nhot;
  const int per = (nh + 1023) / 1024;
  const int h0 = threadIdx.x * per;
  unsigned tot = 0;
  for (int q = 0; q < per && h0 + q < nh; ++q) {
    const unsigned u = hot[h0 + q];
    tot += poff[u + 1] - poff[u];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const unsigned v = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  unsigned run = s[threadIdx.x] - tot;
  for (int q = 0; q < per && h0 + q < nh; ++q) {
    const unsigned u = hot[h0 + q];
    hpre[h0 + q] = run;
    run += poff[u + 1] - poff[u];
  }
  if (threadIdx.x == 1023) hpre[nh] = s[1023];
  for (long long j = threadIdx.x; j < (long long)nh * kPlaneCells; j += 1024)
    hcnt[j] = 0u;
}

// The hot plane holding record t of the joint range (binary search).
__device__ __forceinline__ int hot_plane(const unsigned* __restrict__ hpre,
                                         int nh, unsigned t) {
  int lo = 0, hi = nh - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (hpre[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Record t of the hot range: its index word and its cell in the plane.
template <class PT>
__device__ __forceinline__ void hot_rec(const Sp3<PT>& S, const JointIx& J,
                                        const GridC& g,
                                        const unsigned* __restrict__ poff,
                                        const unsigned* __restrict__ hot,
                                        const unsigned* __restrict__ hpre,
                                        const unsigned* __restrict__ pidx,
                                        int nh, unsigned t, int& h,
                                        unsigned& gi, unsigned& c) {
  h = hot_plane(hpre, nh, t);
  gi = pidx[poff[hot[h]] + (t - hpre[h])];
  c = tile_major(key_of(S, J, gi), g);
}

template <class PT>
__global__ void __launch_bounds__(kT) k_ph_count(
    Sp3<PT> S, GridC g, const unsigned* __restrict__ poff,
    const unsigned* __restrict__ hot, const unsigned* __restrict__ nhot,
    const unsigned* __restrict__ hpre, const unsigned* __restrict__ pidx,
    unsigned* __restrict__ hcnt, const Counters* dc) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  const JointIx J = joint_ix(dc);
  const int nh = (int)*nhot;
  if (nh == 0) return;
  const unsigned tot = hpre[nh];
  for (unsigned b = blockIdx.x * (unsigned)kPChunk; b < tot;
       b += gridDim.x * (unsigned)kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const unsigned e = b + kPChunk < tot ? b + kPChunk : tot;
    for (unsigned t = b + threadIdx.x; t < e; t += kT) {
      int h;
      unsigned gi, c;
      hot_rec(S, J, g, poff, hot, hpre, pidx, nh, t, h, gi, c);
      const unsigned key = (unsigned)h * kPlaneCells + (c & (kPlaneCells - 1));
      const int q = plane_slot(hk, key);
      if (q >= 0)
        atomicAdd(&hc[q], 1u);
      else
        atomicAdd(&hcnt[key], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPHash; q += kT)
      if (hk[q] != kGEmpty) atomicAdd(&hcnt[hk[q]], hc[q]);
    __syncthreads();
  }
}

// Per hot plane (a wavefront each): its cells' offsets, the crowded cells
// listed, the counters turned into the cells' plane-local cursors.
__global__ void __launch_bounds__(kPlaneCells) k_ph_off(
    const unsigned* __restrict__ poff, long long nplanes,
    const unsigned* __restrict__ hot, const unsigned* __restrict__ nhot,
    unsigned* __restrict__ hcnt, unsigned* __restrict__ off,
    unsigned* __restrict__ big, unsigned* __restrict__ nbig,
    long long big_cap) {
  const int nh = (int)*nhot;
  const int lane = (int)threadIdx.x;
  for (int h = blockIdx.x; h < nh; h += gridDim.x) {
    const unsigned u = hot[h];
    const unsigned base = poff[u], c0 = u << kPlaneShift;
    const unsigned m = hcnt[h * kPlaneCells + lane];
    unsigned incl = m;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    off[c0 + lane] = base + incl - m;
    if (lane == 63 && (long long)u == nplanes - 1) off[c0 + kPlaneCells] = base + incl;
    if (m > (unsigned)kSmall) {
      const unsigned s = atomicAdd(nbig, 1u);
      if ((long long)s < big_cap) big[s] = c0 + lane;
    }
    hcnt[h * kPlaneCells + lane] = incl - m;
  }
}

template <class PT>
__global__ void __launch_bounds__(kT) k_ph_scatter(
    Sp3<PT> S, GridC g, const unsigned* __restrict__ poff,
    const unsigned* __restrict__ hot, const unsigned* __restrict__ nhot,
    const unsigned* __restrict__ hpre, const unsigned* __restrict__ pidx,
    unsigned* __restrict__ hcnt, Rec* __restrict__ rec, unsigned step,
    unsigned long long seed, const Counters* dc) {
  __shared__ unsigned hk[kPHash];
  __shared__ unsigned hc[kPHash];
  __shared__ unsigned hb[kPHash];
  const JointIx J = joint_ix(dc);
  const int nh = (int)*nhot;
  if (nh == 0) return;
  const unsigned tot = hpre[nh];
  for (unsigned b = blockIdx.x * (unsigned)kPChunk; b < tot;
       b += gridDim.x * (unsigned)kPChunk) {
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      hk[q] = kGEmpty;
      hc[q] = 0u;
    }
    __syncthreads();
    const unsigned e = b + kPChunk < tot ? b + kPChunk : tot;
    for (unsigned t = b + threadIdx.x; t < e; t += kT) {
      int h;
      unsigned gi, c;
      hot_rec(S, J, g, poff, hot, hpre, pidx, nh, t, h, gi, c);
      const int q = plane_slot(hk, (unsigned)h * kPlaneCells + (c & (kPlaneCells - 1)));
      if (q >= 0) atomicAdd(&hc[q], 1u);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kPHash; q += kT) {
      const unsigned key = hk[q];
      if (key != kGEmpty) {
        hb[q] = poff[hot[key >> kPlaneShift]] + atomicAdd(&hcnt[key], hc[q]);
        hc[q] = 0u;
      }
    }
    __syncthreads();
    for (unsigned t = b + threadIdx.x; t < e; t += kT) {
      int h;
      unsigned gi, c;
      hot_rec(S, J, g, poff, hot, hpre, pidx, nh, t, h, gi, c);
      const unsigned key = (unsigned)h * kPlaneCells + (c & (kPlaneCells - 1));
      // The table is unchanged since the count (see k_cu_scatter).
      const int q = plane_slot(hk, key);
      const unsigned slot = q >= 0 ? hb[q] + atomicAdd(&hc[q], 1u)
                                   : poff[hot[h]] + atomicAdd(&hcnt[key], 1u);
      rec[slot] = make_rec(S, J, gi, c, step, seed);
    }
    __syncthreads();
  }
}

// The small cells of the hot planes, a thread per (cell, record): rank in
// the cell's (key, id) order from the scattered records.
template <class PT>
__global__ void __launch_bounds__(kT) k_ph_rank(
    Sp3<PT> S, const unsigned* __restrict__ hot,
    const unsigned* __restrict__ nhot, const unsigned* __restrict__ off,
    const Rec* __restrict__ rec, Rec* __restrict__ srt) {
  const long long nt = (long long)*nhot * kPlaneCells * kSmall;
  for (long long t = blockIdx.x * (long long)kT + threadIdx.x; t < nt;
       t += (long long)gridDim.x * kT) {
    const int r = (int)(t % kSmall);
    const long long hc = t / kSmall;
    const unsigned c = (hot[hc / kPlaneCells] << kPlaneShift) + (unsigned)(hc % kPlaneCells);
    const unsigned b = off[c];
    const int m = (int)(off[c + 1] - b);
    if (!small_cell((unsigned)m) || r >= m) continue;
    const Rec x = rec[b + r];
    int rank = 0;
    for (int j = 0; j < m; ++j) {
      const Rec y = rec[b + j];
      rank += j != r && (y.lo < x.lo || (y.lo == x.lo && rid(S, y) < rid(S, x)));
    }
    srt[b + rank] = x;
  }
}

// Small cells with a Cu+ of the planes the plane pass did not run (more
// than kPCap records, or hot), one thread each, on the sorted records.  Four
// wavefronts per SIMD (128 registers, two spilled on rare paths): a chain of
// gathers per cell wants occupancy, 1039 -> 935 us at the 128x128x512
// workload; five (30 spilled) ran 1413 us.
template <class PT>
__global__ void __launch_bounds__(kT, 4) k_ip_small(
    Sp3<PT> S, const unsigned* __restrict__ off,
    const unsigned* __restrict__ rest, const unsigned* __restrict__ nrest,
    const Rec* __restrict__ srt, IonC k, GridC g,
    int* __restrict__ ncount, long long* __restrict__ acc,
    uint32_t* __restrict__ dead2, Rec* __restrict__ ev,
    uint2* __restrict__ evp, Counters* dc) {
  Tally t;
  const long long nt = (long long)*nrest * kPlaneCells;
  for (long long q = blockIdx.x * (long long)kT + threadIdx.x; q < nt;
       q += (long long)gridDim.x * kT) {
    const unsigned c = (rest[q / kPlaneCells] << kPlaneShift) + (unsigned)(q % kPlaneCells);
    const unsigned b = off[c], e = off[c + 1];
    const int n = (int)(e - b);
    if (n < 2 || n > kSmall) continue;
    const Rec* r = srt + b;
    // Nothing to do without a Cu+.
    bool has_ion = false;
    for (int j = 0; j < n; ++j) has_ion = has_ion || ip_sp(r[j]) == 1u;
    if (has_ion)
      ip_cell(S, r, n, cell_of_tile_major(c, g), k, g, ncount, acc, dead2, ev,
              evp, dc, t);
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
  const long long np = nc >> kPlaneShift;      // tile planes
  hipMemsetAsync(c->cg_cnt, 0, np * sizeof(unsigned), st);
  hipMemsetAsync(c->cg_nbig, 0, 3 * sizeof(unsigned), st);
  // Grids of a multiple of 8 workgroups (see xcd_block).
  k_pg_count<PT><<<4096, kT, 0, st>>>(S, c->dc, c->g, c->cg_cnt);
  const long long nb = (np + kScanB - 1) / kScanB;
  k_ig_scan_blocks<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_cnt, np, c->cg_poff,
                                                   c->cg_bsum);
  k_ig_scan_sums<<<1, 1024, 0, st>>>(c->cg_bsum, (int)nb);
  k_ig_scan_apply<<<(unsigned)nb, kScanB, 0, st>>>(c->cg_poff, np, c->cg_bsum);
  k_pg_scatter<PT><<<4096, kT, 0, st>>>(S, c->dc, c->g, c->cg_poff, c->cg_cnt,
                                        c->cg_idx);
  // Counters: crowded cells, hot planes, planes left to k_ip_small.
  k_pg_cells<PT><<<8192, kPlaneCells, 0, st>>>(
      S, c->g, c->cg_poff, np, c->cg_idx, c->cg_off, c->cg_rec, c->cg_srt,
      c->cg_big, c->cg_nbig, c->cg_big_cap, c->cg_hot, c->cg_nbig + 1,
      c->cg_rest, c->cg_nbig + 2, k, c->ncount, c->acc_next, c->dead2,
      c->ip_ev, c->ip_evp, c->dc);
  unsigned* nhot = c->cg_nbig + 1;
  k_ph_prep<<<1, 1024, 0, st>>>(c->cg_poff, c->cg_hot, nhot, c->cg_hpre,
                                c->cg_cnt);
  k_ph_count<PT><<<1024, kT, 0, st>>>(S, c->g, c->cg_poff, c->cg_hot, nhot,
                                      c->cg_hpre, c->cg_idx, c->cg_cnt, c->dc);
  k_ph_off<<<512, kPlaneCells, 0, st>>>(c->cg_poff, np, c->cg_hot, nhot,
                                        c->cg_cnt, c->cg_off, c->cg_big,
                                        c->cg_nbig, c->cg_big_cap);
  k_ph_scatter<PT><<<1024, kT, 0, st>>>(S, c->g, c->cg_poff, c->cg_hot, nhot,
                                        c->cg_hpre, c->cg_idx, c->cg_cnt,
                                        c->cg_rec, k.step, k.seed, c->dc);
  k_ph_rank<PT><<<512, kT, 0, st>>>(S, c->cg_hot, nhot, c->cg_off, c->cg_rec,
                                    c->cg_srt);
  k_ip_small<PT><<<512, kT, 0, st>>>(S, c->cg_off, c->cg_rest, c->cg_nbig + 2,
                                     c->cg_srt, k, c->g, c->ncount,
                                     c->acc_next, c->dead2, c->ip_ev,
                                     c->ip_evp, c->dc);
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
