// Resolution check of the grid against the Debye length of the electrons and
// ions (the mesh criterion of the paper's appendix: d_max = 3.4 lambda_D
// alpha_D), per block of b^3 cells.
//
// Pass 1 streams the charged particles once (positions for the block,
// velocities for the moments): HBM-bound.  Each workgroup takes 2048
// consecutive particles of one species, which the binning keeps in tile
// order, so they fall into few blocks: the moments (count, sum of v, sum of
// |v|^2) are summed per block in an LDS hash table and flushed with one
// global atomic per block and moment.  Pass 2 turns each block's moments
// into lambda_D and reduces the counts, the smallest lambda_D and the
// largest dx / d_max over a fixed grid (deterministic).
#include <cmath>

#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kT = 256;
constexpr int kPer = 8;                 // particles per thread
constexpr int kDChunk = kT * kPer;      // particles per workgroup
constexpr int kHash = 1024;             // LDS table entries
constexpr int kMom = 5;                 // count, sum vx, vy, vz, sum |v|^2
constexpr unsigned kEmpty = 0xFFFFFFFFu;
constexpr int kFinBlocks = 1024;

struct BlockGeo {
  int b, bx, by;                        // block edge (cells), blocks per axis
};

__device__ __forceinline__ unsigned block_of(int i, int j, int k,
                                             const BlockGeo& q) {
  return ((unsigned)(k / q.b) * (unsigned)q.by + (unsigned)(j / q.b)) *
             (unsigned)q.bx + (unsigned)(i / q.b);
}

__device__ __forceinline__ void cell_ijk(const Parts& p, long long n,
                                         const GridC& g, int& i, int& j,
                                         int& k) {
  i = (int)floor(p.x[n] * g.inv_dx);
  j = (int)floor(p.y[n] * g.inv_dx);
  k = (int)floor(p.z[n] * g.inv_dx);
  if (i >= g.nx) i -= g.nx;
  if (j >= g.ny) j -= g.ny;
}

__device__ __forceinline__ void cell_ijk(const PartsM& p, long long n,
                                         const GridC& g, int& i, int& j,
                                         int& k) {
  Acc<PartsM>::decode(p.cell[n], g, i, j, k);
}

// Moments of one species (slot sidx of the block record) summed per block.
template <class PT>
__global__ void __launch_bounds__(kT) k_debye_acc(PT p, long long n, int sidx,
                                                  GridC g, BlockGeo q,
                                                  double* __restrict__ mom) {
  __shared__ unsigned hk[kHash];
  __shared__ double hv[kMom][kHash];
  const long long base = (long long)blockIdx.x * kDChunk;
  if (base >= n) return;
  for (int t = threadIdx.x; t < kHash; t += kT) {
    hk[t] = kEmpty;
#pragma unroll
    for (int m = 0; m < kMom; ++m) hv[m][t] = 0.0;
  }
  __syncthreads();
  for (int r = 0; r < kPer; ++r) {
    const long long idx = base + (long long)r * kT + threadIdx.x;
    if (idx >= n) break;
    int i, j, k;
    cell_ijk(p, idx, g, i, j, k);
    double vx, vy, vz;
    Acc<PT>::vel(p, idx, vx, vy, vz);
    const unsigned key = block_of(i, j, k, q);
    const double v2 = (vx * vx + vy * vy) + vz * vz;
    unsigned h = (key * 2654435761u) & (kHash - 1);
    int slot = -1;
    for (int probe = 0; probe < 32; ++probe) {
      const unsigned old = atomicCAS(&hk[h], kEmpty, key);
      if (old == kEmpty || old == key) {
        slot = (int)h;
        break;
      }
      h = (h + 1) & (kHash - 1);
    }
    if (slot >= 0) {
      atomicAdd(&hv[0][slot], 1.0);
      atomicAdd(&hv[1][slot], vx);
      atomicAdd(&hv[2][slot], vy);
      atomicAdd(&hv[3][slot], vz);
      atomicAdd(&hv[4][slot], v2);
    } else {
      // Table crowded: straight to the global record.
      double* rec = mom + (size_t)key * (2 * kMom) + sidx * kMom;
      atomicAdd(rec + 0, 1.0);
      atomicAdd(rec + 1, vx);
      atomicAdd(rec + 2, vy);
      atomicAdd(rec + 3, vz);
      atomicAdd(rec + 4, v2);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < kHash; t += kT) {
    const unsigned key = hk[t];
    if (key == kEmpty) continue;
    double* rec = mom + (size_t)key * (2 * kMom) + sidx * kMom;
#pragma unroll
    for (int m = 0; m < kMom; ++m) atomicAdd(rec + m, hv[m][t]);
  }
}

__global__ void k_debye_zero(double* __restrict__ mom, long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += stride)
    mom[i] = 0.0;
}

struct DebyeC {
  double mass[2];        // electron, Cu+ ion
  double w, vol;         // superparticle weight, block volume (b dx)^3
  double e2, eps0, dx, dmax_per_lambda;
};

// lambda_D per block; block partials of (checked, unresolved) counts, the
// smallest lambda_D and the largest dx / d_max.
__global__ void __launch_bounds__(kT) k_debye_final(
    const double* __restrict__ mom, long long nb, DebyeC d,
    double* __restrict__ lam_out, long long* __restrict__ qpart,
    double* __restrict__ part) {
  __shared__ long long sc[kT], su[kT];
  __shared__ double smin[kT], smax[kT];
  long long checked = 0, unres = 0;
  double lmin = INFINITY, rmax = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < nb;
       b += stride) {
    double inv_l2 = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const double* r = mom + (size_t)b * (2 * kMom) + s * kMom;
      const double N = r[0];
      if (!(N >= 2.0)) continue;
      const double sx = r[1], sy = r[2], sz = r[3];
      const double ss = r[4] - ((sx * sx + sy * sy) + sz * sz) / N;
      const double kT_s = (d.mass[s] * ss) / (3.0 * (N - 1.0));
      if (!(kT_s > 0.0)) continue;
      const double n = (N * d.w) / d.vol;
      inv_l2 = inv_l2 + (n * d.e2) / (d.eps0 * kT_s);
    }
    double lam = INFINITY;
    if (inv_l2 > 0.0) {
      lam = 1.0 / sqrt(inv_l2);
      const double ratio = d.dx / (d.dmax_per_lambda * lam);
      checked += 1;
      if (ratio > 1.0) unres += 1;
      lmin = fmin(lmin, lam);
      rmax = fmax(rmax, ratio);
    }
    if (lam_out) lam_out[b] = lam;
  }
  sc[threadIdx.x] = checked;
  su[threadIdx.x] = unres;
  smin[threadIdx.x] = lmin;
  smax[threadIdx.x] = rmax;
  __syncthreads();
  for (int o = kT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sc[threadIdx.x] += sc[threadIdx.x + o];
      su[threadIdx.x] += su[threadIdx.x + o];
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    qpart[2 * blockIdx.x] = sc[0];
    qpart[2 * blockIdx.x + 1] = su[0];
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

// Fixed-order sum / min / max of the block partials into out[0..3]:
// checked, unresolved (as doubles, exact below 2^53), lambda_min, ratio_max.
__global__ void __launch_bounds__(1024) k_debye_reduce(
    const long long* __restrict__ qpart, const double* __restrict__ part,
    int nblk, double* __restrict__ out) {
  __shared__ long long sc[1024], su[1024];
  __shared__ double smin[1024], smax[1024];
  long long c = 0, u = 0;
  double lmin = INFINITY, rmax = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) {
    c += qpart[2 * i];
    u += qpart[2 * i + 1];
    lmin = fmin(lmin, part[2 * i]);
    rmax = fmax(rmax, part[2 * i + 1]);
  }
  sc[threadIdx.x] = c;
  su[threadIdx.x] = u;
  smin[threadIdx.x] = lmin;
  smax[threadIdx.x] = rmax;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sc[threadIdx.x] += sc[threadIdx.x + o];
      su[threadIdx.x] += su[threadIdx.x + o];
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + o]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = (double)sc[0];
    out[1] = (double)su[0];
    out[2] = smin[0];
    out[3] = smax[0];
  }
}

template <class PT>
PT species_arrays(pic_ctx* c, int s);
template <>
Parts species_arrays<Parts>(pic_ctx* c, int s) { return c->P[s][c->cur[s]]; }
template <>
PartsM species_arrays<PartsM>(pic_ctx* c, int s) { return c->PM[s][c->cur[s]]; }

template <class PT>
void accumulate(pic_ctx* c, const BlockGeo& q) {
  const int sp[2] = {0, 2};
  for (int k = 0; k < 2; ++k) {
    const int s = sp[k];
    const long long n = c->n[s];
    if (n <= 0) continue;
    const unsigned nblk = (unsigned)((n + kDChunk - 1) / kDChunk);
    k_debye_acc<PT><<<nblk, kT, 0, c->stream>>>(species_arrays<PT>(c, s), n,
                                                 k, c->g, q, c->dbg_mom);
  }
}

}  // namespace

long long debye_moment_doubles(long long ncells) { return 2 * kMom * ncells; }

// Moments, lambda_D and the criterion; out[0..3] (device) receives checked,
// unresolved, lambda_min, ratio_max.
void parts_debye(pic_ctx* c, int block, double alpha_D, double* lam_out,
                 double* out) {
  BlockGeo q;
  q.b = block;
  q.bx = c->cfg.nx / block;
  q.by = c->cfg.ny / block;
  const long long nb = (long long)q.bx * q.by * (c->cfg.nz / block);
  k_debye_zero<<<1024, kT, 0, c->stream>>>(c->dbg_mom, 2 * kMom * nb);
  if (c->mixed)
    accumulate<PartsM>(c, q);
  else
    accumulate<Parts>(c, q);
  DebyeC d;
  d.mass[0] = kMe;
  d.mass[1] = kMcu;
  const double side = (double)block * c->g.dx;
  d.w = (double)c->cfg.w_sp;
  d.vol = (side * side) * side;
  d.e2 = kE * kE;
  d.eps0 = kEps0;
  d.dx = c->g.dx;
  d.dmax_per_lambda = 3.4 * alpha_D;
  k_debye_final<<<kFinBlocks, kT, 0, c->stream>>>(
      c->dbg_mom, nb, d, lam_out, c->dbg_qpart, c->dbg_part);
  k_debye_reduce<<<1, 1024, 0, c->stream>>>(c->dbg_qpart, c->dbg_part,
                                            kFinBlocks, out);
}

}  // namespace pic
