// Field solve of the PIC step: right-hand side from the int64 node charge,
// vertex-centred geometric multigrid for the 7-point discretisation of
// Poisson's equation (Eq. 1) with Dirichlet or Neumann z faces and periodic
// x, y, and E = -grad(phi) at the nodes.
//
// All these kernels stream node arrays: they are HBM-bound (a few FLOP per
// byte), so they are written for coalesced 64-lane access along x and use no
// matrix cores.  The red-black Gauss-Seidel smoother is generic in the
// precision (FP64, or FP32 for the correction solve of the mixed form).
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "pic_ctx.h"

namespace pic {
namespace {

constexpr int kRedBlocks = 1024;  // fixed reduction grid: deterministic sums
constexpr int kThreads = 256;

struct LevelC {
  int nx, ny, nz, k0, k1, bc_lo, bc_hi;
  long long nxy;
  double h2;
};

LevelC level_c(const pic_ctx* c, int l) {
  const Level& L = c->lev[l];
  LevelC r;
  r.nx = L.nx; r.ny = L.ny; r.nz = L.nz;
  r.bc_lo = c->cfg.bc_lo; r.bc_hi = c->cfg.bc_hi;
  r.k0 = r.bc_lo == PIC_BC_DIRICHLET ? 1 : 0;
  r.k1 = r.bc_hi == PIC_BC_DIRICHLET ? L.nz - 1 : L.nz;
  r.nxy = (long long)L.nx * L.ny;
  r.h2 = L.h2;
  return r;
}

// Sum of the six neighbours of node (i, j, k) with the mirror ghost on a
// Neumann face.
template <typename T>
__device__ __forceinline__ T nb_sum(const T* u, const LevelC& L, int i, int j,
                                    int k) {
  const long long row = ((long long)k * L.ny + j) * L.nx;
  const int im = i ? i - 1 : L.nx - 1, ip = i + 1 < L.nx ? i + 1 : 0;
  const int jm = j ? j - 1 : L.ny - 1, jp = j + 1 < L.ny ? j + 1 : 0;
  const long long rjm = ((long long)k * L.ny + jm) * L.nx;
  const long long rjp = ((long long)k * L.ny + jp) * L.nx;
  T s = u[row + im] + u[row + ip];
  s = s + (u[rjm + i] + u[rjp + i]);
  T zs;
  if (k == 0)
    zs = T(2) * u[row + L.nxy + i];
  else if (k == L.nz)
    zs = T(2) * u[row - L.nxy + i];
  else
    zs = u[row - L.nxy + i] + u[row + L.nxy + i];
  return s + zs;
}

// ---- right-hand side --------------------------------------------------------
// b = acc * c_rho (a Neumann face node owns half a cell: x2) or
// b = rho * dx^2/eps0 (caller density), plus the Neumann data of the z
// faces; phi gets the Dirichlet face values.  Block partials of sum(b^2)
// and of the integer charge.
__global__ void k_rhs(const long long* __restrict__ acc,
                      const double* __restrict__ rho, double* __restrict__ b,
                      double* __restrict__ phi, LevelC L, double dx,
                      double scale, int from_rho, int field_solve, double v_lo,
                      double v_hi, double* __restrict__ part,
                      long long* __restrict__ qpart) {
  __shared__ double sb[kThreads];
  __shared__ long long sq[kThreads];
  double s2 = 0.0;
  long long sqs = 0;
  const long long n = L.nxy * (L.nz + 1);
  const long long stride = (long long)gridDim.x * blockDim.x;
  // Node indices fit 32 bits: the plane index by 32-bit division.
  const unsigned nxy = (unsigned)L.nxy;
  // Four nodes per round, their loads issued together (clamped), then
  // processed in index order as a plain strided loop would.
  constexpr int kU = 4;
  for (long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       i0 < n; i0 += kU * stride) {
    long long av[kU];
    double rv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      long long q = i0 + u * stride;
      q = q < n ? q : n - 1;
      if (from_rho) rv[u] = rho[q]; else av[u] = acc[q];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const long long idx = i0 + u * stride;
      if (idx >= n) break;
      const int k = (int)((unsigned)idx / nxy);
      double v = 0.0;
      if (from_rho) {
        v = rv[u] * scale;
      } else {
        const long long a = av[u];
        sqs += a;
        if (field_solve) v = (double)a * scale;
      }
      bool unknown = true;
      if (k == 0) {
        if (L.bc_lo == PIC_BC_DIRICHLET) {
          unknown = false;
          phi[idx] = v_lo;
        } else {
          if (!from_rho) v = v * 2.0;
          v = v - (2.0 * dx) * v_lo;
        }
      }
      if (k == L.nz) {
        if (L.bc_hi == PIC_BC_DIRICHLET) {
          unknown = false;
          phi[idx] = v_hi;
        } else {
          if (!from_rho) v = v * 2.0;
          v = v + (2.0 * dx) * v_hi;
        }
      }
      if (!unknown) v = 0.0;
      // The Dirichlet face values sit in phi's face planes, where the stencil
      // reads them, so they stay out of the stored right-hand side; ||b|| is
      // the norm of the system with them moved to the right (the relative
      // residual's denominator).
      b[idx] = v;
      double vb = v;
      if (k == 1 && L.bc_lo == PIC_BC_DIRICHLET) vb = vb + v_lo;
      if (k == L.nz - 1 && L.bc_hi == PIC_BC_DIRICHLET) vb = vb + v_hi;
      s2 = s2 + vb * vb;
    }
  }
  sb[threadIdx.x] = s2;
  sq[threadIdx.x] = sqs;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      sb[threadIdx.x] = sb[threadIdx.x] + sb[threadIdx.x + o];
      sq[threadIdx.x] += sq[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = sb[0];
    qpart[blockIdx.x] = sq[0];
  }
}

// Fixed-tree sum of the block partials.  mode 0: ||b|| (and the integer
// charge); mode 1: residual check after a V-cycle (counts the cycle, sets
// done when converged); mode 2: initial residual check of the warm start;
// mode 3: field energy; mode 4: as mode 1, after a refinement round of the
// mixed form (also counts the round).  Modes 1 and 4 count 'cycles' V-cycles
// (those run since the last check).
__global__ void k_final(const double* __restrict__ part,
                        const long long* __restrict__ qpart, int n,
                        Counters* dc, int mode, double tol, int cycles = 1) {
  __shared__ double s[1024];
  __shared__ long long q[1024];
  if ((mode == 1 || mode == 4) && dc->done) return;
  double a = 0.0;
  long long qa = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    a = a + part[i];
    if (mode == 0) qa += qpart[i];
  }
  s[threadIdx.x] = a;
  q[threadIdx.x] = qa;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + o];
      q[threadIdx.x] += q[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x) return;
  if (mode == 0) {
    dc->b_norm = sqrt(s[0]);
    dc->total_charge = q[0];
    dc->done = 0;
    dc->vcycles = 0;
    dc->rel_res = 1.0;
    dc->refinements = 0;
  } else if (mode == 1 || mode == 2 || mode == 4) {
    if (mode == 1 || mode == 4) dc->vcycles += cycles;
    if (mode == 4) dc->refinements += 1;
    const double bn = dc->b_norm;
    const double rr = bn > 0.0 ? sqrt(s[0]) / bn : 0.0;
    dc->rel_res = rr;
    if (mode == 2) dc->rel_res0 = rr;
    if (!(rr == rr)) {
      dc->err |= kErrNonFinite;
      dc->done = 1;
    } else if (rr <= tol) {
      dc->done = 1;
    }
  } else if (mode == 3) {
    dc->field_energy = 0.5 * s[0];
  }
}


// Residual r = f - A u / h2 on level 0 (FP64): block partials of sum(r^2).
// With rf != nullptr (mixed form) also writes r in FP32 as the right-hand
// side of the correction solve, and with ef != nullptr zeroes the FP32
// correction (the start of the next correction solve, unless its first
// smoothing pass starts from zero by itself).
__global__ void k_residual(const double* __restrict__ u,
                           const double* __restrict__ f, LevelC L,
                           double* __restrict__ part, const Counters* dc,
                           float* __restrict__ rf, float* __restrict__ ef) {
  __shared__ double sb[kThreads];
  if (dc->done) return;
  // Work item: an x-pair (i0, i0 + 1) of one row over a segment of the
  // unknown planes, marched up z with the pair's z neighbours in registers
  // (five loads per plane and pair: u above, the y-neighbour pairs, the
  // two outer x neighbours, f).  nx is even (the configuration requires
  // it), so a pair is one aligned
  // 16-byte word.  The items are spread over the fixed grid in a fixed
  // order, so the partial sums are deterministic.
  const int hx = L.nx / 2;
  const long long npair = (long long)hx * L.ny;
  const int nplane = L.k1 - L.k0 + 1;
  const long long nthr = (long long)gridDim.x * blockDim.x;
  int nseg = (int)(nthr / npair);
  nseg = nseg < 1 ? 1 : (nseg > nplane ? nplane : nseg);
  const int len = (nplane + nseg - 1) / nseg;
  const long long items = npair * nseg;
  const int nxy = (int)L.nxy;
  double s2 = 0.0;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < items;
       t += nthr) {
    const int pr = (int)(t % npair), sg = (int)(t / npair);
    const int px = pr % hx, j = pr / hx;
    const int i0 = 2 * px;
    const int ka = L.k0 + sg * len;
    const int kb = ka + len < L.k1 + 1 ? ka + len : L.k1 + 1;
    if (ka >= kb) continue;
    const int im = i0 ? i0 - 1 : L.nx - 1, ip = i0 + 2 < L.nx ? i0 + 2 : 0;
    const int jm = j ? j - 1 : L.ny - 1, jp = j + 1 < L.ny ? j + 1 : 0;
    const int r0 = j * L.nx, rm = jm * L.nx, rp = jp * L.nx;
    auto pair = [&](int k, int row) {
      return *reinterpret_cast<const double2*>(u + (long long)k * nxy + row + i0);
    };
    double2 cur = pair(ka, r0);
    double2 dn = pair(ka > 0 ? ka - 1 : 0, r0);
    for (int k = ka; k < kb; ++k) {
      const long long base = (long long)k * nxy;
      const double2 up = pair(k < L.nz ? k + 1 : k, r0);
      const double2 ym = pair(k, rm), yp = pair(k, rp);
      const double xl = u[base + r0 + im], xr = u[base + r0 + ip];
      const double2 fv = *reinterpret_cast<const double2*>(f + base + r0 + i0);
      double z0, z1;
      if (k == 0) {
        z0 = 2.0 * up.x;
        z1 = 2.0 * up.y;
      } else if (k == L.nz) {
        z0 = 2.0 * dn.x;
        z1 = 2.0 * dn.y;
      } else {
        z0 = dn.x + up.x;
        z1 = dn.y + up.y;
      }
      // As the stencil sum of one node: x pair, then y pair, then z pair.
      double n0 = xl + cur.y;
      n0 = n0 + (ym.x + yp.x);
      double n1 = cur.x + xr;
      n1 = n1 + (ym.y + yp.y);
      const double res0 = fv.x - (6.0 * cur.x - (n0 + z0));
      const double res1 = fv.y - (6.0 * cur.y - (n1 + z1));
      s2 = s2 + res0 * res0;
      s2 = s2 + res1 * res1;
      if (rf) {
        float2 rv;
        rv.x = (float)res0;
        rv.y = (float)res1;
        *reinterpret_cast<float2*>(rf + base + r0 + i0) = rv;
      }
      if (ef) *reinterpret_cast<float2*>(ef + base + r0 + i0) = make_float2(0.0f, 0.0f);
      dn = cur;
      cur = up;
    }
  }
  sb[threadIdx.x] = s2;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sb[threadIdx.x] = sb[threadIdx.x] + sb[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sb[0];
}

// ---- warm start of the solve --------------------------------------------
// The learned start works on the normalised residual of the previous
// potential: with r0 = b - A phi_prev and sigma its RMS over the unknowns,
// the network maps (r0 / sigma, phi_prev / V_ref) on the nz planes k < nz to
// a correction c, and phi_0 = phi_prev + sigma * c.  The exact correction
// A^-1 r0 is linear in r0, so the normalised map does not depend on the
// charge's magnitude or the grid spacing.

// Stage 0 (after the residual partials of phi_prev): ||r0|| and sigma.
// Stage 1 (after those of phi_0): accept or reject phi_0.
__global__ void k_warm_final(const double* __restrict__ part, int n,
                             Counters* dc, int stage, double n_unknown) {
  __shared__ double s[1024];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a = a + part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] = s[threadIdx.x] + s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x) return;
  const double r = sqrt(s[0]);
  if (stage == 0) {
    dc->warm_r0 = r;
    dc->sigma = r / sqrt(n_unknown);
    dc->warm_ratio = 1.0;
    dc->warm_reject = 0;
  } else {
    const double r0 = dc->warm_r0;
    // Non-finite output, or a start worse than the previous potential:
    // keep phi_prev.
    const bool bad = !(r == r) || r > r0;
    dc->warm_reject = bad ? 1 : 0;
    dc->warm_ratio = bad ? 1.0 : (r0 > 0.0 ? r / r0 : 1.0);
  }
}

// Network input and the saved previous potential.
__global__ void k_warm_input(const double* __restrict__ u,
                             const double* __restrict__ f, LevelC L,
                             const Counters* dc, double inv_vref,
                             float* __restrict__ x,
                             double* __restrict__ uprev) {
  const double sg = dc->sigma;
  const double inv_s = sg > 0.0 ? 1.0 / sg : 0.0;
  const long long n = L.nxy * (L.nz + 1);
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       idx < n; idx += (long long)gridDim.x * blockDim.x) {
    const double uv = u[idx];
    uprev[idx] = uv;
    const int k = (int)(idx / L.nxy);
    if (k >= L.nz) continue;
    double r = 0.0;
    if (k >= L.k0 && k <= L.k1) {
      const long long rem = idx - (long long)k * L.nxy;
      const int j = (int)(rem / L.nx), i = (int)(rem % L.nx);
      r = f[idx] - (6.0 * uv - nb_sum(u, L, i, j, k));
    }
    float2 v;
    v.x = (float)(r * inv_s);
    v.y = (float)(uv * inv_vref);
    reinterpret_cast<float2*>(x)[idx] = v;
  }
}

// phi_0 = phi_prev + sigma * c on the unknowns of the planes k < nz.
__global__ void k_warm_apply(double* __restrict__ u,
                             const double* __restrict__ uprev,
                             const float* __restrict__ c, LevelC L,
                             const Counters* dc) {
  const double sg = dc->sigma;
  const int k1 = L.k1 < L.nz - 1 ? L.k1 : L.nz - 1;
  const long long lo = (long long)L.k0 * L.nxy, hi = (long long)(k1 + 1) * L.nxy;
  for (long long idx = lo + blockIdx.x * (long long)blockDim.x + threadIdx.x;
       idx < hi; idx += (long long)gridDim.x * blockDim.x)
    u[idx] = uprev[idx] + sg * (double)c[idx];
}

__global__ void k_warm_revert(double* __restrict__ u,
                              const double* __restrict__ uprev, LevelC L,
                              const Counters* dc) {
  if (!dc->warm_reject) return;
  const long long lo = (long long)L.k0 * L.nxy, hi = (long long)(L.k1 + 1) * L.nxy;
  for (long long idx = lo + blockIdx.x * (long long)blockDim.x + threadIdx.x;
       idx < hi; idx += (long long)gridDim.x * blockDim.x)
    u[idx] = uprev[idx];
}

// Training target (phi - phi_prev) / sigma on the planes k < nz.
__global__ void k_warm_target(const double* __restrict__ u,
                              const double* __restrict__ uprev, LevelC L,
                              const Counters* dc, float* __restrict__ t) {
  const double sg = dc->sigma;
  const double inv_s = sg > 0.0 ? 1.0 / sg : 0.0;
  const long long n = L.nxy * L.nz;
  for (long long idx = blockIdx.x * (long long)blockDim.x + threadIdx.x;
       idx < n; idx += (long long)gridDim.x * blockDim.x)
    t[idx] = (float)((u[idx] - uprev[idx]) * inv_s);
}

// Over-relaxation of the red-black Gauss-Seidel update: u + w (gs - u)
// (w = 1: the plain update, computed as gs itself).
#ifndef PIC_SOR_OMEGA
#define PIC_SOR_OMEGA 1.25
#endif
template <typename T>
__device__ __forceinline__ T relax(T u, T gs) {
  if (PIC_SOR_OMEGA == 1.0) return gs;
  return u + T(PIC_SOR_OMEGA) * (gs - u);
}

// ---- multigrid node operations ---------------------------------------------
// Each is written for one work item t so that the same code serves the
// grid-wide kernels of the fine levels and the single-workgroup kernel that
// runs all the small coarse levels in one launch.

// Nodes of one colour of a red-black Gauss-Seidel sweep: (i + j + k) % 2 ==
// color get u = (neighbours + h2 f) / 6.
template <typename T>
__device__ __forceinline__ long long rbgs_count(const LevelC& L) {
  return (long long)(L.nx >> 1) * L.ny * (L.k1 - L.k0 + 1);
}
template <typename T>
__device__ __forceinline__ void rbgs_node(T* __restrict__ u,
                                          const T* __restrict__ f,
                                          const LevelC& L, int color,
                                          long long t) {
  const unsigned half = (unsigned)(L.nx >> 1), tt = (unsigned)t;
  const int m = (int)(tt % half);
  const unsigned r = tt / half;
  const int j = (int)(r % (unsigned)L.ny);
  const int k = L.k0 + (int)(r / (unsigned)L.ny);
  const int i = 2 * m + ((color + j + k) & 1);
  const long long idx = ((long long)k * L.ny + j) * L.nx + i;
  const T h2 = (T)L.h2;
  const T gs = (nb_sum(u, L, i, j, k) + h2 * f[idx]) * (T(1) / T(6));
  u[idx] = relax(u[idx], gs);
}

// Full-weighting restriction of the fine residual to coarse node t (the
// coarse correction starts at zero).
template <typename T>
__device__ __forceinline__ void restrict_node(const T* __restrict__ uf,
                                              const T* __restrict__ ff,
                                              T* __restrict__ uc,
                                              T* __restrict__ fc,
                                              const LevelC& F, const LevelC& Cc,
                                              long long t) {
  const unsigned tt = (unsigned)t;
  const int ic = (int)(tt % (unsigned)Cc.nx);
  const unsigned r = tt / (unsigned)Cc.nx;
  const int jc = (int)(r % (unsigned)Cc.ny);
  const int kc = (int)(r / (unsigned)Cc.ny);
  uc[t] = T(0);
  if (kc < Cc.k0 || kc > Cc.k1) {
    fc[t] = T(0);
    return;
  }
  const T inv_h2 = T(1) / (T)F.h2;
  T acc = T(0);
  for (int dk = -1; dk <= 1; ++dk) {
    int kf = 2 * kc + dk;
    if (kf < 0) kf = 1;                 // Neumann mirror
    if (kf > F.nz) kf = F.nz - 1;
    const T wz = dk ? T(1) : T(2);
    for (int dj = -1; dj <= 1; ++dj) {
      const int jf = wrap_index(2 * jc + dj, F.ny);
      const T wy = dj ? T(1) : T(2);
      for (int di = -1; di <= 1; ++di) {
        const int i_f = wrap_index(2 * ic + di, F.nx);
        const T wx = di ? T(1) : T(2);
        const long long fi = ((long long)kf * F.ny + jf) * F.nx + i_f;
        const T res = ff[fi] - (T(6) * uf[fi] - nb_sum(uf, F, i_f, jf, kf)) * inv_h2;
        acc = acc + (wx * wy * wz) * res;
      }
    }
  }
  fc[t] = acc * T(1.0 / 64.0);
}

// Trilinear prolongation of the coarse correction, added to fine unknown t.
template <typename T>
__device__ __forceinline__ void prolong_node(T* __restrict__ uf,
                                             const T* __restrict__ uc,
                                             const LevelC& F, const LevelC& Cc,
                                             long long t) {
  // Node indices fit 32 bits: 32-bit division is much cheaper than 64.
  const unsigned tt = (unsigned)t;
  const int i = (int)(tt % (unsigned)F.nx);
  const unsigned r = tt / (unsigned)F.nx;
  const int j = (int)(r % (unsigned)F.ny);
  const int k = F.k0 + (int)(r / (unsigned)F.ny);
  int ia[2], ja[2], ka[2];
  T wa[2], wb[2], wc[2];
  int na, nb, nc;
  if (i & 1) { ia[0] = i >> 1; ia[1] = wrap_index((i >> 1) + 1, Cc.nx); wa[0] = wa[1] = T(0.5); na = 2; }
  else { ia[0] = i >> 1; wa[0] = T(1); na = 1; }
  if (j & 1) { ja[0] = j >> 1; ja[1] = wrap_index((j >> 1) + 1, Cc.ny); wb[0] = wb[1] = T(0.5); nb = 2; }
  else { ja[0] = j >> 1; wb[0] = T(1); nb = 1; }
  if (k & 1) { ka[0] = k >> 1; ka[1] = (k >> 1) + 1; wc[0] = wc[1] = T(0.5); nc = 2; }
  else { ka[0] = k >> 1; wc[0] = T(1); nc = 1; }
  T s = T(0);
  for (int c3 = 0; c3 < nc; ++c3)
    for (int b3 = 0; b3 < nb; ++b3)
      for (int a3 = 0; a3 < na; ++a3)
        s = s + (wa[a3] * wb[b3] * wc[c3]) *
                    uc[((long long)ka[c3] * Cc.ny + ja[b3]) * Cc.nx + ia[a3]];
  const long long idx = ((long long)k * F.ny + j) * F.nx + i;
  uf[idx] = uf[idx] + s;
}

// Exact solve of a 1x1xN coarsest level (the x, y neighbours are the node
// itself): tridiagonal 2u - u_{k-1} - u_{k+1} = h2 f, Thomas algorithm,
// one thread.
template <typename T>
__device__ void line_solve(T* __restrict__ u, const T* __restrict__ f,
                           const LevelC& L, T* __restrict__ w) {
  const int m = L.k1 - L.k0 + 1;
  T* cp = w;
  T* dp = w + m;
  for (int r = 0; r < m; ++r) {
    const int k = L.k0 + r;
    T rhs = (T)L.h2 * f[k];
    T lo = (k == 0 || r == 0) ? T(0) : T(-1);
    T up = (k == L.nz || r == m - 1) ? T(0) : T(-1);
    if (k == 0) up = T(-2);
    if (k == L.nz) lo = T(-2);
    if (r == 0 && k > 0) rhs = rhs + u[k - 1];        // Dirichlet data
    if (r == m - 1 && k < L.nz) rhs = rhs + u[k + 1];
    if (r == 0) {
      cp[0] = up / T(2);
      dp[0] = rhs / T(2);
    } else {
      const T den = T(2) - lo * cp[r - 1];
      cp[r] = up / den;
      dp[r] = (rhs - lo * dp[r - 1]) / den;
    }
  }
  T x = dp[m - 1];
  u[L.k0 + m - 1] = x;
  for (int r = m - 2; r >= 0; --r) {
    x = dp[r] - cp[r] * x;
    u[L.k0 + r] = x;
  }
}

template <typename T>
__global__ void k_rbgs(T* __restrict__ u, const T* __restrict__ f, LevelC L,
                       int color, const Counters* dc) {
  if (dc->done) return;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= rbgs_count<T>(L)) return;
  rbgs_node(u, f, L, color, t);
}

template <typename T>
__global__ void k_restrict(const T* __restrict__ uf, const T* __restrict__ ff,
                           T* __restrict__ uc, T* __restrict__ fc, LevelC F,
                           LevelC Cc, const Counters* dc) {
  if (dc->done) return;
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= Cc.nxy * (Cc.nz + 1)) return;
  restrict_node(uf, ff, uc, fc, F, Cc, t);
}

// Prolongation with correction by fine x-pairs: the nodes 2i and 2i+1 of a
// fine row share their coarse nodes i, i+1, so one thread reads and writes
// the pair with one vector access each.  A wave covers 64 pairs of one row,
// so the y and z parities (how many coarse rows and planes contribute) are
// uniform across it.  Per node the sum runs in the same order as
// prolong_node (z, then y, then x), so the results are the same.
template <typename T>
struct Pair2;
template <>
struct Pair2<double> { using type = double2; };
template <>
struct Pair2<float> { using type = float2; };

template <typename T>
__global__ void __launch_bounds__(256) k_prolong_pairs(
    T* __restrict__ uf, const T* __restrict__ uc, LevelC F, LevelC Cc,
    int nbx, const Counters* dc) {
  if (dc->done) return;
  const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
  const int bx = blk % nbx, by = blk / nbx;
  const int ic = bx * 64 + (int)(threadIdx.x & 63);
  const int row = by * 4 + (int)(threadIdx.x >> 6);
  const int nrows = F.ny * (F.k1 - F.k0 + 1);
  if (ic >= (F.nx >> 1) || row >= nrows) return;
  const int j = row % F.ny;
  const int k = F.k0 + row / F.ny;
  const int ic1 = wrap_index(ic + 1, Cc.nx);
  int ja[2], ka[2];
  T wb[2], wc[2];
  int nb = 1, nc = 1;
  ja[0] = j >> 1;
  wb[0] = T(1);
  if (j & 1) {
    ja[1] = wrap_index((j >> 1) + 1, Cc.ny);
    wb[0] = wb[1] = T(0.5);
    nb = 2;
  }
  ka[0] = k >> 1;
  wc[0] = T(1);
  if (k & 1) {
    ka[1] = (k >> 1) + 1;
    wc[0] = wc[1] = T(0.5);
    nc = 2;
  }
  T s0 = T(0), s1 = T(0);
  for (int c3 = 0; c3 < nc; ++c3)
    for (int b3 = 0; b3 < nb; ++b3) {
      const T* cr = uc + ((long long)ka[c3] * Cc.ny + ja[b3]) * Cc.nx;
      const T a = cr[ic], b = cr[ic1];
      s0 = s0 + ((T(1) * wb[b3]) * wc[c3]) * a;
      const T w = (T(0.5) * wb[b3]) * wc[c3];
      s1 = s1 + w * a;
      s1 = s1 + w * b;
    }
  using V = typename Pair2<T>::type;
  V* p = reinterpret_cast<V*>(uf + ((long long)k * F.ny + j) * F.nx + 2 * ic);
  V v = *p;
  v.x = v.x + s0;
  v.y = v.y + s1;
  *p = v;
}

// Restriction with the fine residual staged in LDS: a workgroup takes an
// RX x RY x RZ block of coarse nodes, one per thread.  It stages the
// (2RX+3)(2RY+3)(2RZ+3) fine u nodes the block's residuals read (coalesced,
// each node once), computes the residual of the (2RX+1)(2RY+1)(2RZ+1) fine
// nodes under the block from LDS (same stencil and order as nb_sum), then
// applies the 27-point full weighting from LDS.  FP64 takes 8x8x4 blocks
// (31.8 KB of LDS); FP32 16x8x4 on 512 threads (29.3 KB), which stages 1.79
// fine nodes per owned one against 1.94 and halves the blocks, the pass
// being bound by its load and LDS instructions rather than by bytes.
template <typename T>
struct RTile {
  static constexpr int RX = 8, RY = 8, RZ = 4;
};
template <>
struct RTile<float> {
  static constexpr int RX = 16, RY = 8, RZ = 4;
};
template <typename T>
__host__ __device__ constexpr int restrict_threads() {
  return RTile<T>::RX * RTile<T>::RY * RTile<T>::RZ;
}

template <typename T>
__global__ void __launch_bounds__(restrict_threads<T>()) k_restrict_tiled(
    const T* __restrict__ uf, const T* __restrict__ ff, T* __restrict__ uc,
    T* __restrict__ fc, LevelC F, LevelC Cc, const Counters* dc) {
  constexpr int kRX = RTile<T>::RX, kRY = RTile<T>::RY, kRZ = RTile<T>::RZ;
  constexpr int kNT = restrict_threads<T>();
  constexpr int kFX = 2 * kRX + 1, kFY = 2 * kRY + 1, kFZ = 2 * kRZ + 1;
  constexpr int kUX = kFX + 2, kUY = kFY + 2, kUZ = kFZ + 2;
  constexpr int kUXY = kUX * kUY;
  // The staged u block, then (reused) the residuals.
  __shared__ T su[kUZ * kUXY];
  static_assert(kFZ * kFY * kFX <= kUZ * kUXY, "residuals reuse the u block");
  constexpr int kRPer = (kFZ * kFY * kFX + kNT - 1) / kNT;
  if (dc->done) return;
  const int tnx = (Cc.nx + kRX - 1) / kRX, tny = (Cc.ny + kRY - 1) / kRY;
  // Neighbouring tiles share halo nodes: keep them on one XCD's L2.
  const unsigned blk = xcd_block(blockIdx.x, gridDim.x);
  const int bx = blk % tnx, by = (blk / tnx) % tny, bz = blk / (tnx * tny);
  // The blocks cover the unknown coarse planes k0..k1 (the face planes of a
  // Dirichlet level are zeroed by the blocks next to them): with 2^m + 1
  // planes a level has 2^m - 1 unknown ones, so the blocks fill whole
  // rounds of resident workgroups instead of leaving a round for one plane.
  const int cx0 = bx * kRX, cy0 = by * kRY, cz0 = Cc.k0 + bz * kRZ;
  const T inv_h2 = T(1) / (T)F.h2;
  // Staged node (sx, sy, sz) is fine node (2cx0 - 2 + sx, 2cy0 - 2 + sy,
  // 2cz0 - 2 + sz), x and y wrapped; planes outside [0, nz] are loaded
  // clamped and never read.  The fine level is at least 16 nodes wide, so
  // one wrap suffices.
  const int nxy = (int)F.nxy;
  // Every global load of the block is issued before the first use (clamped
  // to a valid node where the slot is unused), so they are all in flight
  // together: the u block, then the f values of this thread's residuals.
  constexpr int kSPer = (kUZ * kUXY + kNT - 1) / kNT;
  T uv[kSPer];
#pragma unroll
  for (int m = 0; m < kSPer; ++m) {
    int q = threadIdx.x + kNT * m;
    q = q < kUZ * kUXY ? q : kUZ * kUXY - 1;
    const int sx = q % kUX, sy = (q / kUX) % kUY, sz = q / kUXY;
    const int i = wrap_index(2 * cx0 - 2 + sx, F.nx);
    const int j = wrap_index(2 * cy0 - 2 + sy, F.ny);
    int k = 2 * cz0 - 2 + sz;
    k = k < 0 ? 0 : (k > F.nz ? F.nz : k);
    uv[m] = uf[k * nxy + j * F.nx + i];
  }
  T fv[kRPer];
  int rk[kRPer], rc[kRPer];
#pragma unroll
  for (int m = 0; m < kRPer; ++m) {
    int q = threadIdx.x + kNT * m;
    q = q < kFZ * kFY * kFX ? q : kFZ * kFY * kFX - 1;
    const int lx = q % kFX, ly = (q / kFX) % kFY, lz = q / (kFX * kFY);
    int k = 2 * cz0 - 1 + lz;
    if (k < 0) k = 1;                    // Neumann mirror
    if (k > F.nz) k = F.nz - 1;
    const int i = wrap_index(2 * cx0 - 1 + lx, F.nx);
    const int j = wrap_index(2 * cy0 - 1 + ly, F.ny);
    rk[m] = k;
    // Plane k sits at sz = k - (2cz0 - 2), in 1..9, so k +- 1 are staged.
    rc[m] = ((k - 2 * cz0 + 2) * kUY + ly + 1) * kUX + lx + 1;
    fv[m] = ff[k * nxy + j * F.nx + i];
  }
#pragma unroll
  for (int m = 0; m < kSPer; ++m) {
    const int q = threadIdx.x + kNT * m;
    if (q < kUZ * kUXY) su[q] = uv[m];
  }
  __syncthreads();
  T rv[kRPer];
#pragma unroll
  for (int m = 0; m < kRPer; ++m) {
    const int k = rk[m], c = rc[m];
    T res = T(0);
    if (threadIdx.x + kNT * m < kFZ * kFY * kFX && k >= F.k0 && k <= F.k1) {
      T sn = su[c - 1] + su[c + 1];
      sn = sn + (su[c - kUX] + su[c + kUX]);
      T zs;
      if (k == 0)
        zs = T(2) * su[c + kUXY];
      else if (k == F.nz)
        zs = T(2) * su[c - kUXY];
      else
        zs = su[c - kUXY] + su[c + kUXY];
      res = fv[m] - (T(6) * su[c] - (sn + zs)) * inv_h2;
    }
    rv[m] = res;
  }
  __syncthreads();
  T* r = su;
#pragma unroll
  for (int m = 0; m < kRPer; ++m) {
    const int q = threadIdx.x + kNT * m;
    if (q < kFZ * kFY * kFX) r[q] = rv[m];
  }
  __syncthreads();
  const int tx = threadIdx.x % kRX, ty = (threadIdx.x / kRX) % kRY,
            tz = threadIdx.x / (kRX * kRY);
  const int ic = cx0 + tx, jc = cy0 + ty, kc = cz0 + tz;
  if (ic >= Cc.nx || jc >= Cc.ny || kc > Cc.nz) return;
  const long long t = ((long long)kc * Cc.ny + jc) * Cc.nx + ic;
  uc[t] = T(0);
  if (kc < Cc.k0 || kc > Cc.k1) {
    fc[t] = T(0);
    return;
  }
  if (kc == Cc.k0 && Cc.k0 > 0) {
    uc[t - Cc.nxy] = T(0);
    fc[t - Cc.nxy] = T(0);
  }
  if (kc == Cc.k1 && Cc.k1 < Cc.nz) {
    uc[t + Cc.nxy] = T(0);
    fc[t + Cc.nxy] = T(0);
  }
  T acc = T(0);
  for (int dk = 0; dk < 3; ++dk) {
    const T wz = dk == 1 ? T(2) : T(1);
    for (int dj = 0; dj < 3; ++dj) {
      const T wy = dj == 1 ? T(2) : T(1);
      const int row = ((2 * tz + dk) * kFY + (2 * ty + dj)) * kFX + 2 * tx;
      for (int di = 0; di < 3; ++di) {
        const T wx = di == 1 ? T(2) : T(1);
        acc = acc + (wx * wy * wz) * r[row + di];
      }
    }
  }
  fc[t] = acc * T(1.0 / 64.0);
}

// The levels from 'first' down, in one workgroup with every level's u and f
// held in LDS: the lower part of a V-cycle whose levels are too small to
// fill the GPU (one launch instead of several per level).  f of the first
// level is read from and u written back to global memory.
constexpr int kTailLdsBytes = 48 * 1024;

struct TailLevels {
  void* u0;
  const void* f0;
  LevelC L[16];
  long long off[16];     // offset of each level's u in LDS (elements)
  int first, last, nu_pre, nu_post, coarse_sweeps;
  long long total;       // elements of u (and of f) over the levels
};

template <typename T>
__global__ void __launch_bounds__(1024) k_mg_tail(TailLevels A,
                                                  const Counters* dc) {
  __shared__ __attribute__((aligned(16))) char lds[kTailLdsBytes];
  if (dc->done) return;
  T* su = reinterpret_cast<T*>(lds);
  T* sf = su + A.total;
  const long long tid = threadIdx.x, nth = blockDim.x;
  {
    const LevelC& L0 = A.L[A.first];
    const long long n0 = L0.nxy * (L0.nz + 1);
    const T* gu = reinterpret_cast<const T*>(A.u0);
    const T* gf = reinterpret_cast<const T*>(A.f0);
    for (long long t = tid; t < n0; t += nth) {
      su[t] = gu[t];
      sf[t] = gf[t];
    }
  }
  __syncthreads();
  for (int l = A.first; l < A.last; ++l) {
    T* u = su + A.off[l];
    const T* f = sf + A.off[l];
    const LevelC& L = A.L[l];
    const long long nr = rbgs_count<T>(L);
    for (int s = 0; s < A.nu_pre; ++s)
      for (int color = 0; color < 2; ++color) {
        for (long long t = tid; t < nr; t += nth) rbgs_node(u, f, L, color, t);
        __syncthreads();
      }
    const LevelC& C = A.L[l + 1];
    const long long ncn = C.nxy * (C.nz + 1);
    for (long long t = tid; t < ncn; t += nth)
      restrict_node(u, f, su + A.off[l + 1], sf + A.off[l + 1], L, C, t);
    __syncthreads();
  }
  {
    const int l = A.last;
    T* u = su + A.off[l];
    const T* f = sf + A.off[l];
    const LevelC& L = A.L[l];
    if (L.nx == 1 && L.ny == 1) {
      // Thomas scratch after the f arrays.
      if (tid == 0) line_solve(u, f, L, sf + A.total);
    } else {
      const long long nr = rbgs_count<T>(L);
      for (int s = 0; s < A.coarse_sweeps; ++s)
        for (int color = 0; color < 2; ++color) {
          for (long long t = tid; t < nr; t += nth) rbgs_node(u, f, L, color, t);
          __syncthreads();
        }
    }
    __syncthreads();
  }
  for (int l = A.last - 1; l >= A.first; --l) {
    T* u = su + A.off[l];
    const T* f = sf + A.off[l];
    const LevelC& L = A.L[l];
    const LevelC& C = A.L[l + 1];
    const long long nf = L.nxy * (L.k1 - L.k0 + 1);
    for (long long t = tid; t < nf; t += nth)
      prolong_node(u, su + A.off[l + 1], L, C, t);
    __syncthreads();
    const long long nr = rbgs_count<T>(L);
    for (int s = 0; s < A.nu_post; ++s)
      for (int color = 0; color < 2; ++color) {
        for (long long t = tid; t < nr; t += nth) rbgs_node(u, f, L, color, t);
        __syncthreads();
      }
  }
  {
    const LevelC& L0 = A.L[A.first];
    const long long n0 = L0.nxy * (L0.nz + 1);
    T* gu = reinterpret_cast<T*>(A.u0);
    for (long long t = tid; t < n0; t += nth) gu[t] = su[t];
  }
}

// Extrapolated start of a step solve: phi_0 = 2 phi_{n-1} - phi_{n-2} at
// every node (the Dirichlet face values are the same in both, so they stay),
// and the history becomes phi_{n-1}.  Without a valid history the history
// is only filled.
// hist <- 2 u - hist, the extrapolated start; the host then swaps the two
// buffers, so the old potential becomes the history (two arrays read and
// one written, where updating both in place writes two).
__global__ void k_extrap(const double* __restrict__ u, double* __restrict__ hist,
                         long long n) {
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < n;
       t += (long long)gridDim.x * blockDim.x)
    hist[t] = 2.0 * u[t] - hist[t];
}

// u += e on the level-0 unknowns (mixed form: FP64 correction accumulation).
__global__ void k_correct(double* __restrict__ u, const float* __restrict__ e,
                          LevelC L, const Counters* dc) {
  if (dc->done) return;
  const long long nu = L.nxy * (L.k1 - L.k0 + 1);
  const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (t >= nu) return;
  const long long idx = t + (long long)L.k0 * L.nxy;
  u[idx] = u[idx] + (double)e[idx];
}

// E = -grad(phi): central differences in x, y and inside z; second-order
// one-sided on the z faces.  Stored as three node arrays (Ex, Ey, Ez): the
// push stages a tile's nodes in LDS, reading whole rows.  Block partials of
// sum(q phi) for the field energy.
template <typename TE>
__global__ void k_efield(const double* __restrict__ phi,
                         const long long* __restrict__ acc,
                         TE* __restrict__ E, LevelC L, double h,
                         double q_unit, double* __restrict__ part) {
  using E2 = typename Pair2<TE>::type;
  __shared__ double sb[kThreads];
  double s = 0.0;
  const long long n = L.nxy * (L.nz + 1);
  // Work item: an x-pair of one row over a segment of the planes, marched
  // up z with the pair's z neighbours in registers (nx is even); the face
  // planes load the second plane their one-sided difference needs.  Items
  // are spread over the fixed grid in a fixed order: deterministic sums.
  const int hx = L.nx / 2;
  const long long npair = (long long)hx * L.ny;
  const int nplane = L.nz + 1;
  const long long nthr = (long long)gridDim.x * blockDim.x;
  int nseg = (int)(nthr / npair);
  nseg = nseg < 1 ? 1 : (nseg > nplane ? nplane : nseg);
  const int len = (nplane + nseg - 1) / nseg;
  const long long items = npair * nseg;
  const int nxy = (int)L.nxy;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < items;
       t += nthr) {
    const int pr = (int)(t % npair), sg = (int)(t / npair);
    const int px = pr % hx, j = pr / hx;
    const int i0 = 2 * px;
    const int ka = sg * len;
    const int kb = ka + len < nplane ? ka + len : nplane;
    if (ka >= kb) continue;
    const int im = i0 ? i0 - 1 : L.nx - 1, ip = i0 + 2 < L.nx ? i0 + 2 : 0;
    const int jm = j ? j - 1 : L.ny - 1, jp = j + 1 < L.ny ? j + 1 : 0;
    const int r0 = j * L.nx, rm = jm * L.nx, rp = jp * L.nx;
    auto pair = [&](int k, int row) {
      return *reinterpret_cast<const double2*>(phi + (long long)k * nxy + row + i0);
    };
    double2 cur = pair(ka, r0);
    double2 dn = pair(ka > 0 ? ka - 1 : 0, r0);
    for (int k = ka; k < kb; ++k) {
      const long long idx = (long long)k * nxy + r0 + i0;
      const double2 up = pair(k < L.nz ? k + 1 : k, r0);
      const double2 ym = pair(k, rm), yp = pair(k, rp);
      const double xl = phi[(long long)k * nxy + r0 + im];
      const double xr = phi[(long long)k * nxy + r0 + ip];
      const longlong2 ac = *reinterpret_cast<const longlong2*>(acc + idx);
      E2 ex, ey, ez;
      ex.x = (TE)((xl - cur.y) * h);
      ex.y = (TE)((cur.x - xr) * h);
      ey.x = (TE)((ym.x - yp.x) * h);
      ey.y = (TE)((ym.y - yp.y) * h);
      if (k == 0) {
        const double2 u2 = pair(2, r0);
        ez.x = (TE)(((3.0 * cur.x - 4.0 * up.x) + u2.x) * h);
        ez.y = (TE)(((3.0 * cur.y - 4.0 * up.y) + u2.y) * h);
      } else if (k == L.nz) {
        const double2 d2 = pair(k - 2, r0);
        ez.x = (TE)(((-3.0 * cur.x + 4.0 * dn.x) - d2.x) * h);
        ez.y = (TE)(((-3.0 * cur.y + 4.0 * dn.y) - d2.y) * h);
      } else {
        ez.x = (TE)((dn.x - up.x) * h);
        ez.y = (TE)((dn.y - up.y) * h);
      }
      *reinterpret_cast<E2*>(E + idx) = ex;
      *reinterpret_cast<E2*>(E + n + idx) = ey;
      *reinterpret_cast<E2*>(E + 2 * n + idx) = ez;
      s = s + ((double)ac.x * q_unit) * cur.x;
      s = s + ((double)ac.y * q_unit) * cur.y;
      dn = cur;
      cur = up;
    }
  }
  sb[threadIdx.x] = s;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sb[threadIdx.x] = sb[threadIdx.x] + sb[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sb[0];
}

inline unsigned nblocks(long long n, int t = kThreads) {
  return (unsigned)((n + t - 1) / t);
}

// ---- fused smoothing ------------------------------------------------------
// Two red-black Gauss-Seidel sweeps (red, black, red, black) in one pass over
// the level, from uin to uout.  A workgroup owns an SX x SY column of nodes
// and a segment of z planes and marches up z: at step p it applies
// half-sweep h to plane p-h (h = 0..3), so every half-sweep sees the other
// colour's values of the previous half-sweep on the three planes it reads.
// Half-sweep h updates the column widened by 3-h nodes in x, y and z (the
// halo it leaves valid for h+1), so the final values of the owned nodes are
// exactly those of four grid-wide colour launches; the widened nodes are
// recomputed by the neighbouring workgroups from the same old values.
//
// Each thread owns one x-pair (2k, 2k+1) of one row of the widened column
// for the whole march, and keeps the pair's values on the six planes in
// flight in registers.  At step p every half-sweep updates the pair's node
// of parity (row + p) on its own plane: its centre, its pair partner (one x
// neighbour) and its z neighbours are the thread's registers; only the
// other x neighbour and the two y neighbours are read from LDS, where each
// updated value is also stored.  A plane slot in LDS holds the even-x nodes
// of every row, then the odd-x ones, so a wave's reads are consecutive
// words.  The half-sweeps of one step read only values written in earlier
// steps (the z neighbours they share are one thread's registers), so one
// barrier per step suffices.  The u pair of plane p+4 and the f pair of
// plane p+2 (kept in registers for the four half-sweeps that use it) are
// loaded while step p computes.  HBM traffic per pass: u and f
// read and u written once, against about four times that for separate
// launches.
//
// The owned column is SX x SY nodes and the widened one (SX + 8) x (SY + 8),
// so a workgroup recomputes (SX + 8)(SY + 8) / (SX SY) nodes per owned node:
// 2.5 at 32 x 8, 1.69 at 64 x 16.  The march is bound by instruction issue,
// so the larger column pays; FP64 takes 64 x 16 (864 threads, 83 KB of
// LDS ring), FP32 32 x 16 (480 threads), which measured faster than 64 x 16
// in FP32 (more resident workgroups per CU for the latency of the march).
template <typename T>
struct SmoothTile;
template <>
struct SmoothTile<double> {
  static constexpr int SX = 64, SY = 16;
};
template <>
struct SmoothTile<float> {
  static constexpr int SX = 32, SY = 16;
};
constexpr int kSH = 4;
constexpr int kSR = 6;
// One x-pair of the widened column per thread.
template <typename T>
__host__ __device__ constexpr int smooth_threads() {
  return (SmoothTile<T>::SX + 2 * kSH) / 2 * (SmoothTile<T>::SY + 2 * kSH);
}
static_assert((kSH & 1) == 0, "x-pairs need even x");

__device__ __forceinline__ int wrap_n(int v, int n) {
  v = v < 0 ? v + n : v;
  return v >= n ? v - n : v;
}

template <int N>
using IC = std::integral_constant<int, N>;

static_assert(kSR == 6, "the march below is unrolled by the ring length");
// Ring index at step j (mod kSR) of the plane p + d.
__host__ __device__ constexpr int ring_slot(int j, int d) {
  return ((1 + j + d) % kSR + kSR) % kSR;
}

// Level-0 pass modes of the mixed form's FP32 correction solve: the first
// pass of a refinement round starts from a zero correction without reading
// one (kSmZeroIn); the last adds its correction to the FP64 potential u64 on
// the unknown planes instead of storing it (kSmAcc64: u64 + (double)e, the
// FP64 accumulation of the refinement).
enum : int { kSmPlain = 0, kSmZeroIn = 1, kSmAcc64 = 2 };

// NEU: a z face of the level holds unknowns (Neumann condition), so face
// planes are updated; with Dirichlet faces they never are.
template <typename T, bool NEU, int MODE>
__global__ void __launch_bounds__(smooth_threads<T>()) k_smooth2(
    const T* __restrict__ uin, T* __restrict__ uout, const T* __restrict__ f,
    LevelC L, int seg, const Counters* dc, double* __restrict__ u64) {
  static_assert(MODE == kSmPlain || std::is_same<T, float>::value,
                "pass modes of the FP32 correction solve");
  using P2 = typename Pair2<T>::type;
  constexpr int kSX = SmoothTile<T>::SX, kSY = SmoothTile<T>::SY;
  constexpr int kSPX = kSX + 2 * kSH, kSPY = kSY + 2 * kSH;
  constexpr int kSP = kSPX * kSPY;  // nodes per plane slot
  constexpr int kHX = kSPX / 2, kHP = kHX * kSPY;
  static_assert((kSX & 1) == 0 && kHX * kSPY == smooth_threads<T>(), "tile");
  __shared__ T ring[kSR][kSP];
  if (dc->done) return;
  const int tiles_x = (L.nx + kSX - 1) / kSX;
  const int tiles_y = (L.ny + kSY - 1) / kSY;
  // Neighbouring columns share halo nodes: keep them on one XCD's L2.
  int bi = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = bi % tiles_x;
  bi /= tiles_x;
  const int ty = bi % tiles_y;
  const int za = (bi / tiles_y) * seg;
  const int zb = za + seg < L.nz + 1 ? za + seg : L.nz + 1;
  const int x0 = tx * kSX - kSH, y0 = ty * kSY - kSH;
  const T h2 = (T)L.h2;
  const T sixth = T(1) / T(6);

  const int pk = threadIdx.x % kHX, ly = threadIdx.x / kHX;
  const int lx0 = 2 * pk;
  // x0, nx and ny are even, so the pair is one aligned 16-byte (8-byte)
  // word of a row in memory, and the local indices carry the colour.
  const int gy = wrap_n(wrap_n(y0 + ly, L.ny), L.ny);
  const int gx0 = wrap_n(wrap_n(x0 + lx0, L.nx), L.nx);
  const int goff = gy * L.nx + gx0;
  const int s0 = ly * kHX + pk;  // even node; the odd one at s0 + kHP
  // Bit h of inr[d]: node d of the pair lies in half-sweep h's region
  // (widened by e = 3 - h).  Bit masks, not an array indexed by the node,
  // which would live in scratch memory.
  unsigned inr0 = 0u, inr1 = 0u;
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int e = 3 - h;
    const bool yin = ly >= kSH - e && ly < kSH + kSY + e;
    if (yin && lx0 >= kSH - e && lx0 < kSH + kSX + e) inr0 |= 1u << h;
    if (yin && lx0 + 1 >= kSH - e && lx0 + 1 < kSH + kSX + e) inr1 |= 1u << h;
  }
  const bool owned = ly >= kSH && ly < kSH + kSY && lx0 >= kSH &&
                     lx0 < kSH + kSX && x0 + lx0 < L.nx && y0 + ly < L.ny;

  // Plane q takes half-sweep h when it holds unknowns and lies in h's
  // widened z range [za - e, zb - 1 + e], e = 3 - h; at step p that plane is
  // q = p - h, so the test is p - h - lo in [0, hi - lo] (one unsigned
  // compare).
  int lo[4];
  unsigned span[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    lo[h] = max(L.k0, za - (3 - h)) + h;
    const int hi = min(L.k1, zb - 1 + (3 - h)) + h;
    span[h] = hi >= lo[h] ? (unsigned)(hi - lo[h]) : 0u;
    if (hi < lo[h]) lo[h] = 0x3FFFFFFF;  // never: p - lo wraps above 0
  }
  auto active = [&](int h, int p) { return (unsigned)(p - lo[h]) <= span[h]; };
  auto clampz = [&](int z) { return z < 0 ? 0 : (z > L.nz ? L.nz : z); };
  // Node offsets fit in 32 bits (at most 2^31 - 1 nodes per level).
  const int nxy = (int)L.nxy;

  // The pair on the planes in flight: plane p + d at step j in slot
  // ring_slot(j, d), as in LDS.
  T v0[kSR], v1[kSR];
  T f0[kSR], f1[kSR];  // f of the pair, same slots (loaded two steps ahead)
  P2 pu[2];        // pairs loaded for later steps
  // A plane outside the level (z < 0 or z > nz) is committed too, from the
  // clamped loads: it is only read as the missing neighbour of a face
  // plane, which the face update never uses.
  auto fetch_u = [&](auto U, int z) {
    constexpr int iu = decltype(U)::value;
    if constexpr ((MODE & kSmZeroIn) != 0) {
      pu[iu].x = T(0);
      pu[iu].y = T(0);
    } else {
      pu[iu] = *reinterpret_cast<const P2*>(uin + clampz(z) * nxy + goff);
    }
  };
  // kSmAcc64: the FP64 pair of the plane stored two steps later, loaded
  // into slot (step & 1) once that slot's previous pair is stored.
  double2 pa[2];
  auto fetch_acc = [&](auto A, int z) {
    if constexpr ((MODE & kSmAcc64) != 0) {
      constexpr int ia = decltype(A)::value;
      pa[ia] = *reinterpret_cast<const double2*>(u64 + (long long)clampz(z) * nxy + goff);
    }
  };
  auto commit_u = [&](auto U, auto S) {
    constexpr int iu = decltype(U)::value, sl = decltype(S)::value;
    v0[sl] = pu[iu].x;
    v1[sl] = pu[iu].y;
    ring[sl][s0] = pu[iu].x;
    ring[sl][s0 + kHP] = pu[iu].y;
  };
  // f pair of plane z into ring slot S (read from two steps later on).
  auto fetch_f = [&](auto S, int z) {
    constexpr int sl = decltype(S)::value;
    const P2 w = *reinterpret_cast<const P2*>(f + clampz(z) * nxy + goff);
    f0[sl] = w.x;
    f1[sl] = w.y;
  };
  // Half-sweep h at step j (plane q = p - h) on the node of parity d.
  auto update = [&](auto H, auto J, int p, int d, unsigned inr) {
    constexpr int h = decltype(H)::value, j = decltype(J)::value;
    constexpr int sc = ring_slot(j, -h), sd = ring_slot(j, -h - 1),
                  su = ring_slot(j, 1 - h);
    if (!(active(h, p) && ((inr >> h) & 1u))) return;
    const int q = p - h;
    const T* pl = ring[sc];
    const int sn_i = s0 + d * kHP;
    // The x neighbour outside the pair: lx0 - 1 (odd half, pair pk - 1)
    // for the even node, lx0 + 2 (even half, pair pk + 1) for the odd one.
    const T xo = pl[d ? s0 + 1 : s0 + kHP - 1];
    const T xp = d ? v0[sc] : v1[sc];
    T sn = xo + xp;
    sn = sn + (pl[sn_i - kHX] + pl[sn_i + kHX]);
    const T a = d ? v1[sd] : v0[sd], b = d ? v1[su] : v0[su];
    // On a Neumann face the mirror node stands in for the missing one
    // (up + up on the cathode face, dn + dn on the anode face).
    const T zs = NEU ? (q == 0 ? b : a) + (q == L.nz ? a : b) : a + b;
    const T cu = d ? v1[sc] : v0[sc];
    const T fv = d ? f1[sc] : f0[sc];
    const T nv = relax(cu, ((sn + zs) + h2 * fv) * sixth);
    if (d) v1[sc] = nv; else v0[sc] = nv;
    ring[sc][sn_i] = nv;
  };
  // Step p (= p0 + j modulo kSR): the four half-sweeps (plane p-h), the
  // finished plane p-3 out, the pair of plane p+2 into the ring, the loads
  // of later steps issued, then the one barrier.
  const int d0 = (ly + za - 3) & 1;  // parity of the updated node at p0
  auto step = [&](auto J, int p) {
    constexpr int j = decltype(J)::value, jf = j & 1;
    const int d = d0 ^ jf;
    const unsigned inr = d ? inr1 : inr0;
    update(IC<0>(), J, p, d, inr);
    update(IC<1>(), J, p, d, inr);
    update(IC<2>(), J, p, d, inr);
    update(IC<3>(), J, p, d, inr);
    const int q = p - 3;
    if (owned && q >= za && q < zb) {
      constexpr int so = ring_slot(j, -3);
      if constexpr ((MODE & kSmAcc64) != 0) {
        if (q >= L.k0 && q <= L.k1) {
          double2 w = pa[jf];
          w.x = w.x + (double)v0[so];
          w.y = w.y + (double)v1[so];
          *reinterpret_cast<double2*>(u64 + (long long)q * L.nxy + goff) = w;
        }
      } else {
        P2 w;
        w.x = v0[so];
        w.y = v1[so];
        *reinterpret_cast<P2*>(uout + (long long)q * L.nxy + goff) = w;
      }
    }
    fetch_acc(IC<jf>(), p - 1);
    commit_u(IC<jf>(), IC<ring_slot(j, 2)>());
    fetch_u(IC<jf>(), p + 4);
    fetch_f(IC<ring_slot(j, 2)>(), p + 2);
    __syncthreads();
  };

  // Plane z lives in slot (z - p0 + 1) mod kSR; the march is unrolled by
  // kSR, so every slot index is a constant (and the two register sets
  // alternate with period 2, which divides kSR).
  const int p0 = za - 3, p1 = zb + 2;
  fetch_u(IC<0>(), p0 - 1);
  commit_u(IC<0>(), IC<0>());
  fetch_u(IC<0>(), p0);
  commit_u(IC<0>(), IC<1>());
  fetch_u(IC<0>(), p0 + 1);
  commit_u(IC<0>(), IC<2>());
  fetch_u(IC<0>(), p0 + 2);
  fetch_u(IC<1>(), p0 + 3);
  // f of planes p0 - 3 .. p0 + 1 (slots of d = -3 .. 1 at step 0).
  fetch_f(IC<ring_slot(0, -3)>(), p0 - 3);
  fetch_f(IC<ring_slot(0, -2)>(), p0 - 2);
  fetch_f(IC<ring_slot(0, -1)>(), p0 - 1);
  fetch_f(IC<ring_slot(0, 0)>(), p0);
  fetch_f(IC<ring_slot(0, 1)>(), p0 + 1);
  fetch_acc(IC<0>(), p0 - 3);
  fetch_acc(IC<1>(), p0 - 2);
  __syncthreads();
  for (int p = p0;; p += kSR) {
    step(IC<0>(), p);
    if (p + 1 > p1) break;
    step(IC<1>(), p + 1);
    if (p + 2 > p1) break;
    step(IC<2>(), p + 2);
    if (p + 3 > p1) break;
    step(IC<3>(), p + 3);
    if (p + 4 > p1) break;
    step(IC<4>(), p + 4);
    if (p + 5 > p1) break;
    step(IC<5>(), p + 5);
    if (p + 6 > p1) break;
  }
}

template <typename T>
T* lev_u(Level& L);
template <>
double* lev_u<double>(Level& L) { return L.u; }
template <>
float* lev_u<float>(Level& L) { return L.uf; }
template <typename T>
T* lev_s(Level& L);
template <>
double* lev_s<double>(Level& L) { return L.us; }
template <>
float* lev_s<float>(Level& L) { return L.usf; }
template <typename T>
T* lev_f(Level& L);
template <>
double* lev_f<double>(Level& L) { return L.f; }
template <>
float* lev_f<float>(Level& L) { return L.ff; }

// Coarsest level too large for LDS: exact line solve or red-black sweeps in
// one workgroup, in global memory.
template <typename T>
__global__ void k_coarse_global(T* __restrict__ u, const T* __restrict__ f,
                                LevelC L, int sweeps, const Counters* dc,
                                T* __restrict__ w) {
  if (dc->done) return;
  if (L.nx == 1 && L.ny == 1) {
    if (threadIdx.x == 0) line_solve(u, f, L, w);
    return;
  }
  const long long nr = rbgs_count<T>(L);
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (long long t = threadIdx.x; t < nr; t += blockDim.x)
        rbgs_node(u, f, L, color, t);
      __syncthreads();
    }
}

// First level from which all coarser levels fit in the tail kernel's LDS
// (u and f of every level, plus the coarse line solver's scratch); nlev if
// not even the coarsest does.
template <typename T>
int tail_first(const pic_ctx* c) {
  int l = c->nlev;
  long long tot = 0;
  for (int q = c->nlev - 1; q >= 0; --q) {
    const long long add = c->lev[q].nnodes;
    const long long bytes = (2 * (tot + add) + 2 * (c->lev[c->nlev - 1].nz + 2)) *
                            (long long)sizeof(T);
    if (bytes > kTailLdsBytes) break;
    tot += add;
    l = q;
  }
  return l;
}

// ---- exact solve of one coarse level -----------------------------------------
// With x and y periodic, the 7-point operator acts on the 2-D Fourier modes
// of a plane one by one: mode (kx, ky) has 6 - 2cos(2 pi kx/nx) -
// 2cos(2 pi ky/ny) on the diagonal and the z neighbours off it, so the level
// equation 6u - sum(neighbours) = h2 f becomes one tridiagonal system in z
// per mode over the unknown planes (a Neumann face row takes its inner
// neighbour twice; a Dirichlet face's correction is zero).  A real plane
// needs the modes kx = 0..nx/2 only.  Spectrum layout: [plane][mode][re,im],
// mode = ky (nx/2 + 1) + kx.

__device__ __forceinline__ int ilog2_pow2(int n) { return 31 - __clz(n); }

// Block-wide copy of n values, dst(q) <- src(q), with NB loads per thread in
// flight: the loads take clamped indices (always in range) and only the
// stores are guarded, so no load waits for the one before it.
constexpr int kSpecThreads = 256;
template <int NB, typename T, typename Ld, typename St>
__device__ __forceinline__ void batch_copy(int n, Ld ld, St st) {
  for (int q0 = threadIdx.x; q0 < n; q0 += NB * kSpecThreads) {
    T v[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int q = q0 + u * kSpecThreads;
      v[u] = ld(q < n ? q : n - 1);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const int q = q0 + u * kSpecThreads;
      if (q < n) st(q, v[u]);
    }
  }
}

// Elimination factors per mode, which depend on the grid only: the inverse
// pivots, plane by plane (layout [plane][mode]); the eliminated upper
// coefficient of plane p is up_p times its pivot's inverse.
template <typename T>
__global__ void k_spec_factor(LevelC L, T* __restrict__ mi, int nm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nm) return;
  const int nxh = L.nx / 2 + 1;
  const int kx = m % nxh, ky = m / nxh;
  const double d = 6.0 - 2.0 * cospi(2.0 * kx / L.nx) - 2.0 * cospi(2.0 * ky / L.ny);
  const int np = L.k1 - L.k0 + 1;
  double cprev = 0.0;
  for (int p = 0; p < np; ++p) {
    const int k = L.k0 + p;
    const double lo = p == 0 ? 0.0 : (k == L.nz ? -2.0 : -1.0);
    const double up = p == np - 1 ? 0.0 : (k == 0 ? -2.0 : -1.0);
    const double inv = 1.0 / (d - lo * cprev);
    cprev = up * inv;
    mi[(long long)p * nm + m] = (T)inv;
  }
}

// Twiddles e^{2 pi i q / n} = (cos, sin), q = 0..n-1.
template <typename T>
__device__ __forceinline__ void fill_twiddles(T* tw, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * q / n, &sn, &cs);
    tw[2 * q] = (T)cs;
    tw[2 * q + 1] = (T)sn;
  }
}

// Forward: h2 f of one unknown plane -> its spectrum (row DFTs of the real
// plane, then column DFTs of the half spectrum).
template <typename T>
__global__ void __launch_bounds__(kSpecThreads) k_spec_fwd(LevelC L,
                                                  const T* __restrict__ f,
                                                  T* __restrict__ s, int nm,
                                                  const Counters* dc) {
  __shared__ T fp[kSpecMaxXY * kSpecMaxXY];
  __shared__ T rr[kSpecMaxXY * (kSpecMaxXY / 2 + 1) * 2];
  __shared__ T twx[2 * kSpecMaxXY], twy[2 * kSpecMaxXY];
  if (dc->done) return;
  const int nx = L.nx, ny = L.ny, nxh = nx / 2 + 1;
  const int p = blockIdx.x;
  const T* src = f + (long long)(L.k0 + p) * L.nxy;
  batch_copy<4, T>(nx * ny, [&](int q) { return src[q]; },
                   [&](int q, T v) { fp[q] = v; });
  fill_twiddles(twx, nx);
  fill_twiddles(twy, ny);
  __syncthreads();
  // R(j, kx) = sum_i f(i, j) e^{-2 pi i kx i / nx}
  for (int q = threadIdx.x; q < ny * nxh; q += blockDim.x) {
    const int j = q / nxh, kx = q % nxh;
    T re = T(0), im = T(0);
    int w = 0;  // kx * i mod nx
#pragma unroll 8
    for (int i = 0; i < nx; ++i) {
      const T v = fp[j * nx + i];
      re = re + v * twx[2 * w];
      im = im - v * twx[2 * w + 1];
      w += kx;
      if (w >= nx) w -= nx;
    }
    rr[2 * q] = re;
    rr[2 * q + 1] = im;
  }
  __syncthreads();
  // F(ky, kx) = sum_j R(j, kx) e^{-2 pi i ky j / ny}, times h2.
  const T h2 = (T)L.h2;
  T* out = s + (long long)p * 2 * nm;
  for (int q = threadIdx.x; q < nm; q += blockDim.x) {
    const int ky = q / nxh, kx = q % nxh;
    T re = T(0), im = T(0);
    int w = 0;
#pragma unroll 8
    for (int j = 0; j < ny; ++j) {
      const T a = rr[2 * (j * nxh + kx)], b = rr[2 * (j * nxh + kx) + 1];
      const T c = twy[2 * w], sn = twy[2 * w + 1];
      re = re + (a * c + b * sn);
      im = im + (b * c - a * sn);
      w += ky;
      if (w >= ny) w -= ny;
    }
    out[2 * q] = h2 * re;
    out[2 * q + 1] = h2 * im;
  }
}

// The tridiagonal systems, one per (mode, real or imaginary part).  Both
// sweeps are first-order linear recurrences with coefficients that depend on
// the grid only: the elimination y_p = mi_p b_p + al_p y_{p-1}, al_p =
// -lo_p mi_p, and the back substitution x_p = y_p + be_p x_{p+1}, be_p =
// -up_p mi_p (up_p in {0, -1, -2}, so be_p is exact in either precision).
// Each lane runs one segment of kSeg planes of one column from a zero start,
// carrying the product of the coefficients along it; the segment ends are
// joined through LDS, and every plane is then corrected by its carried
// product times the joined value.  A workgroup holds 2^lgw columns (half as
// many modes) and kSpecThreads / 2^lgw segments; the plane data goes from
// HBM to registers and back once.
constexpr int kSeg = 16;

template <typename T>
__global__ void __launch_bounds__(kSpecThreads) k_spec_tri(
    LevelC L, T* __restrict__ s, const T* __restrict__ mi, int nm, int lgw,
    const Counters* dc) {
  __shared__ T jz[kSpecThreads], ja[kSpecThreads];
  if (dc->done) return;
  const int np = L.k1 - L.k0 + 1;
  const int w = 1 << lgw;
  const int t = threadIdx.x;
  const int c = t & (w - 1), sg = t >> lgw;
  const int m0 = blockIdx.x * (w >> 1);
  const int m = m0 + (c >> 1);
  const bool mok = m < nm;
  const int cc = mok ? c : (c & 1);  // a valid column, not stored
  const int mc = mok ? m : m0;
  const int p0 = sg * kSeg;
  T b[kSeg], f[kSeg], a[kSeg];
#pragma unroll
  for (int u = 0; u < kSeg; ++u) {
    const int p = p0 + u < np ? p0 + u : np - 1;
    b[u] = s[(long long)p * 2 * nm + 2 * m0 + cc];
    f[u] = mi[(long long)p * nm + mc];
  }
  // Elimination, segment-local.
  T z = T(0), A = T(1);
#pragma unroll
  for (int u = 0; u < kSeg; ++u) {
    const int p = p0 + u, k = L.k0 + p;
    if (p < np) {
      const T al = p == 0 ? T(0) : (k == L.nz ? T(2) : T(1)) * f[u];
      z = f[u] * b[u] + al * z;
      A = al * A;
    }
    b[u] = z;
    a[u] = A;
  }
  jz[t] = z;
  ja[t] = A;
  __syncthreads();
  T y = T(0);  // y at the plane before this segment
  for (int q = 0; q < sg; ++q) y = jz[(q << lgw) + c] + ja[(q << lgw) + c] * y;
#pragma unroll
  for (int u = 0; u < kSeg; ++u) b[u] = b[u] + a[u] * y;
  // Back substitution, segment-local from its last plane.
  T x = T(0), B = T(1);
#pragma unroll
  for (int u = kSeg - 1; u >= 0; --u) {
    const int p = p0 + u, k = L.k0 + p;
    if (p < np) {
      const T be = p == np - 1 ? T(0) : (k == 0 ? T(2) : T(1)) * f[u];
      x = b[u] + be * x;
      B = be * B;
    }
    b[u] = x;
    a[u] = B;
  }
  __syncthreads();
  jz[t] = x;
  ja[t] = B;
  __syncthreads();
  const int nsg = kSpecThreads >> lgw;
  T xn = T(0);  // x at the plane after this segment
  for (int q = nsg - 1; q > sg; --q)
    xn = jz[(q << lgw) + c] + ja[(q << lgw) + c] * xn;
  if (mok) {
#pragma unroll
    for (int u = 0; u < kSeg; ++u)
      if (p0 + u < np)
        s[(long long)(p0 + u) * 2 * nm + 2 * m0 + c] = b[u] + a[u] * xn;
  }
}

// Columns per workgroup of k_spec_tri (log2): enough segments of kSeg
// planes for np, at most 128 columns.
inline int spec_tri_lgw(int np) {
  const int segs = (np + kSeg - 1) / kSeg;
  int lgw = 7;
  while (lgw > 1 && (kSpecThreads >> lgw) < segs) --lgw;
  return lgw;
}

// Inverse: the solved spectrum of one plane -> u (column inverse DFTs,
// then the real row inverse DFT: kx = 0 and nx/2 once, the others twice).
template <typename T>
__global__ void __launch_bounds__(kSpecThreads) k_spec_inv(LevelC L,
                                                  const T* __restrict__ s,
                                                  T* __restrict__ u, int nm,
                                                  const Counters* dc) {
  __shared__ T sp[kSpecMaxXY * (kSpecMaxXY / 2 + 1) * 2];
  __shared__ T gg[kSpecMaxXY * (kSpecMaxXY / 2 + 1) * 2];
  __shared__ T twx[2 * kSpecMaxXY], twy[2 * kSpecMaxXY];
  if (dc->done) return;
  const int nx = L.nx, ny = L.ny, nxh = nx / 2 + 1;
  const int p = blockIdx.x;
  const T* in = s + (long long)p * 2 * nm;
  batch_copy<4, T>(2 * nm, [&](int q) { return in[q]; },
                   [&](int q, T v) { sp[q] = v; });
  fill_twiddles(twx, nx);
  fill_twiddles(twy, ny);
  __syncthreads();
  // G(j, kx) = sum_ky S(ky, kx) e^{+2 pi i ky j / ny}
  for (int q = threadIdx.x; q < ny * nxh; q += blockDim.x) {
    const int j = q / nxh, kx = q % nxh;
    T re = T(0), im = T(0);
    int w = 0;
#pragma unroll 8
    for (int ky = 0; ky < ny; ++ky) {
      const T a = sp[2 * (ky * nxh + kx)], b = sp[2 * (ky * nxh + kx) + 1];
      const T c = twy[2 * w], sn = twy[2 * w + 1];
      re = re + (a * c - b * sn);
      im = im + (a * sn + b * c);
      w += j;
      if (w >= ny) w -= ny;
    }
    gg[2 * q] = re;
    gg[2 * q + 1] = im;
  }
  __syncthreads();
  const T inv_n = T(1) / (T)(nx * ny);
  T* dst = u + (long long)(L.k0 + p) * L.nxy;
  const int kn = nx / 2;
  for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) {
    const int j = q / nx, i = q % nx;
    const T* g = gg + 2 * j * nxh;
    T acc = g[0] + ((i & 1) ? -g[2 * kn] : g[2 * kn]);
    T two = T(0);
    int w = i;  // kx * i mod nx
#pragma unroll 8
    for (int kx = 1; kx < kn; ++kx) {
      two = two + (g[2 * kx] * twx[2 * w] - g[2 * kx + 1] * twx[2 * w + 1]);
      w += i;
      if (w >= nx) w -= nx;
    }
    dst[q] = (acc + T(2) * two) * inv_n;
  }
}

// FFTs of planes whose nx and ny are powers of two (2 to kSpecMaxFFT), by
// the four-step split n = n1 n2 (n1 = min(n, 8)): per line, n2 register
// DFTs of length n1 over stride-n2 elements, the twiddles e^{+-2 pi i j2 k1
// / n}, then n1 register DFTs of length n2; output k1 + n1 k2.  Each axis
// costs two LDS exchanges.  Two real rows travel as one complex row z =
// row(2jp) + i row(2jp + 1) and are separated with the conjugate-symmetric
// halves of its transform (forward), or assembled from their half spectra
// (inverse).  One task per thread and phase: kFftThreads covers the largest
// phase (33 columns x 8).
constexpr int kFftThreads = 320;
constexpr int kFftSlots = 2304;  // complex LDS slots, largest layout at 64 x 64

// Complex DFT of length R in {1, 2, 4, 8} on registers 0..R-1, in place and
// in natural order; sg = -1: e^{-2 pi i j k / R}, +1: e^{+...}.
template <typename T>
__device__ __forceinline__ void dft4r(T& r0, T& i0, T& r1, T& i1, T& r2, T& i2,
                                      T& r3, T& i3, T sg) {
  const T ar = r0 + r2, ai = i0 + i2, br = r0 - r2, bi = i0 - i2;
  const T cr = r1 + r3, ci = i1 + i3;
  // (r1 - r3 + i (i1 - i3)) times e^{sg i pi / 2} = sg i
  const T dr = -sg * (i1 - i3), di = sg * (r1 - r3);
  r0 = ar + cr; i0 = ai + ci;
  r2 = ar - cr; i2 = ai - ci;
  r1 = br + dr; i1 = bi + di;
  r3 = br - dr; i3 = bi - di;
}

template <typename T>
__device__ __forceinline__ void dft_reg(T (&xr)[8], T (&xi)[8], int R, T sg) {
  if (R == 8) {
    // Even and odd halves, then the radix-2 merge with e^{sg 2 pi i k / 8}.
    dft4r(xr[0], xi[0], xr[2], xi[2], xr[4], xi[4], xr[6], xi[6], sg);
    dft4r(xr[1], xi[1], xr[3], xi[3], xr[5], xi[5], xr[7], xi[7], sg);
    const T h = T(0.70710678118654752440);
    const T o1r = h * (xr[3] - sg * xi[3]), o1i = h * (sg * xr[3] + xi[3]);
    const T o2r = -sg * xi[5], o2i = sg * xr[5];
    const T o3r = -h * (xr[7] + sg * xi[7]), o3i = h * (sg * xr[7] - xi[7]);
    const T e0r = xr[0], e0i = xi[0], e1r = xr[2], e1i = xi[2];
    const T e2r = xr[4], e2i = xi[4], e3r = xr[6], e3i = xi[6];
    const T o0r = xr[1], o0i = xi[1];
    xr[0] = e0r + o0r; xi[0] = e0i + o0i;
    xr[4] = e0r - o0r; xi[4] = e0i - o0i;
    xr[1] = e1r + o1r; xi[1] = e1i + o1i;
    xr[5] = e1r - o1r; xi[5] = e1i - o1i;
    xr[2] = e2r + o2r; xi[2] = e2i + o2i;
    xr[6] = e2r - o2r; xi[6] = e2i - o2i;
    xr[3] = e3r + o3r; xi[3] = e3i + o3i;
    xr[7] = e3r - o3r; xi[7] = e3i - o3i;
  } else if (R == 4) {
    dft4r(xr[0], xi[0], xr[1], xi[1], xr[2], xi[2], xr[3], xi[3], sg);
  } else if (R == 2) {
    const T ar = xr[0], ai = xi[0];
    xr[0] = ar + xr[1]; xi[0] = ai + xi[1];
    xr[1] = ar - xr[1]; xi[1] = ai - xi[1];
  }
}

// Twiddle table (cos, sin)(2 pi q / n), q < n.
template <typename C2>
__device__ __forceinline__ void fill_fft_tw(C2* tw, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * q / n, &sn, &cs);
    tw[q].x = cs;
    tw[q].y = sn;
  }
}

// x_k1 *= e^{sg 2 pi i j2 k1 / n}, k1 < R.
template <typename T, typename C2>
__device__ __forceinline__ void twiddle(T (&xr)[8], T (&xi)[8], int R,
                                        const C2* tw, int n, int j2, T sg) {
#pragma unroll
  for (int k1 = 1; k1 < 8; ++k1) {
    if (k1 < R) {
      const C2 w = tw[(j2 * k1) & (n - 1)];
      const T wi = sg * w.y;
      const T r = xr[k1] * w.x - xi[k1] * wi;
      xi[k1] = xr[k1] * wi + xi[k1] * w.x;
      xr[k1] = r;
    }
  }
}

// Forward: h2 f of one unknown plane -> its half spectrum (kx <= nx/2).
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_spec_fwd_fft(
    LevelC L, const T* __restrict__ f, T* __restrict__ s, int nm,
    const Counters* dc) {
  using C2 = typename Pair2<T>::type;
  __shared__ C2 buf[kFftSlots];
  __shared__ C2 twx[kSpecMaxFFT], twy[kSpecMaxFFT];
  if (dc->done) return;
  const int nx = L.nx, ny = L.ny, nxh = nx / 2 + 1, nyp = ny / 2;
  const int n1x = nx < 8 ? nx : 8, n2x = nx / n1x;
  const int n1y = ny < 8 ? ny : 8, n2y = ny / n1y;
  const int lg1x = ilog2_pow2(n1x), lg2x = ilog2_pow2(n2x);
  const int rs1 = n1x * (n2x + 1);  // row stride of the x scratch
  const int rz = nx + 8;            // row stride of the x spectra
  const int t = threadIdx.x;
  const T* src = f + (long long)(L.k0 + blockIdx.x) * L.nxy;
  fill_fft_tw(twx, nx);
  fill_fft_tw(twy, ny);
  T xr[8], xi[8];
  // Rows: task (jp, j2), j2 fastest.
  const bool tx1 = t < (nyp << lg2x);
  const int jp1 = t >> lg2x, j21 = t & (n2x - 1);
  if (tx1) {
#pragma unroll
    for (int j1 = 0; j1 < 8; ++j1) {
      if (j1 < n1x) {
        const int i = (j1 << lg2x) + j21;
        xr[j1] = src[(2 * jp1) * nx + i];
        xi[j1] = src[(2 * jp1 + 1) * nx + i];
      }
    }
  }
  __syncthreads();
  if (tx1) {
    dft_reg(xr, xi, n1x, T(-1));
    twiddle(xr, xi, n1x, twx, nx, j21, T(-1));
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
      if (k1 < n1x) {
        C2 v;
        v.x = xr[k1];
        v.y = xi[k1];
        buf[jp1 * rs1 + k1 * (n2x + 1) + j21] = v;
      }
  }
  __syncthreads();
  const bool tx2 = t < (nyp << lg1x);
  const int jp2 = t >> lg1x, k12 = t & (n1x - 1);
  if (tx2) {
#pragma unroll
    for (int j2 = 0; j2 < 8; ++j2)
      if (j2 < n2x) {
        const C2 v = buf[jp2 * rs1 + k12 * (n2x + 1) + j2];
        xr[j2] = v.x;
        xi[j2] = v.y;
      }
    dft_reg(xr, xi, n2x, T(-1));
  }
  __syncthreads();
  if (tx2) {
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2)
      if (k2 < n2x) {
        C2 v;
        v.x = xr[k2];
        v.y = xi[k2];
        buf[jp2 * rz + k12 + (k2 << lg1x)] = v;
      }
  }
  __syncthreads();
  // Columns kx <= nx/2: task (kx, j2), kx fastest; row j of the real
  // transform is (Z(kx) + conj Z(-kx)) / 2 (j even) or (Z(kx) - conj
  // Z(-kx)) / 2i (j odd) of its packed row; the 1/2 joins h2 at the end.
  const bool ty1 = t < nxh * n2y;
  const int kx1 = t % nxh, j2y = t / nxh;
  if (ty1) {
    const int km = (nx - kx1) & (nx - 1);
#pragma unroll
    for (int j1 = 0; j1 < 8; ++j1)
      if (j1 < n1y) {
        const int j = n2y * j1 + j2y;
        const C2 za = buf[(j >> 1) * rz + kx1], zb = buf[(j >> 1) * rz + km];
        const bool odd = j & 1;
        xr[j1] = odd ? za.y + zb.y : za.x + zb.x;
        xi[j1] = odd ? zb.x - za.x : za.y - zb.y;
      }
    dft_reg(xr, xi, n1y, T(-1));
    twiddle(xr, xi, n1y, twy, ny, j2y, T(-1));
  }
  __syncthreads();
  if (ty1) {
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
      if (k1 < n1y) {
        C2 v;
        v.x = xr[k1];
        v.y = xi[k1];
        buf[(k1 * n2y + j2y) * nxh + kx1] = v;
      }
  }
  __syncthreads();
  const bool ty2 = t < nxh * n1y;
  const int kx2 = t % nxh, k1y = t / nxh;
  if (ty2) {
#pragma unroll
    for (int j2 = 0; j2 < 8; ++j2)
      if (j2 < n2y) {
        const C2 v = buf[(k1y * n2y + j2) * nxh + kx2];
        xr[j2] = v.x;
        xi[j2] = v.y;
      }
    dft_reg(xr, xi, n2y, T(-1));
    const T sc = T(0.5) * (T)L.h2;
    C2* out = reinterpret_cast<C2*>(s + (long long)blockIdx.x * 2 * nm);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2)
      if (k2 < n2y) {
        C2 v;
        v.x = sc * xr[k2];
        v.y = sc * xi[k2];
        out[(k1y + n1y * k2) * nxh + kx2] = v;
      }
  }
}

// Inverse: the solved half spectrum of one plane -> u (columns first, then
// two rows at a time as one complex row whose halves are the Hermitian
// extensions of the two; the imaginary parts at kx = 0 and nx/2 are those
// of a real row's transform, zero).
template <typename T>
__global__ void __launch_bounds__(kFftThreads) k_spec_inv_fft(
    LevelC L, const T* __restrict__ s, T* __restrict__ u, int nm,
    const Counters* dc) {
  using C2 = typename Pair2<T>::type;
  __shared__ C2 buf[kFftSlots];
  __shared__ C2 twx[kSpecMaxFFT], twy[kSpecMaxFFT];
  if (dc->done) return;
  const int nx = L.nx, ny = L.ny, nxh = nx / 2 + 1, nyp = ny / 2;
  const int n1x = nx < 8 ? nx : 8, n2x = nx / n1x;
  const int n1y = ny < 8 ? ny : 8, n2y = ny / n1y;
  const int lg1x = ilog2_pow2(n1x), lg2x = ilog2_pow2(n2x);
  const int rs1 = n1x * (n2x + 1);
  const int rg = nxh + 3;  // row stride of the column-transformed spectrum
  const int t = threadIdx.x;
  const C2* in = reinterpret_cast<const C2*>(s + (long long)blockIdx.x * 2 * nm);
  fill_fft_tw(twx, nx);
  fill_fft_tw(twy, ny);
  T xr[8], xi[8];
  const bool ty1 = t < nxh * n2y;
  const int kx1 = t % nxh, j2y = t / nxh;
  if (ty1) {
#pragma unroll
    for (int j1 = 0; j1 < 8; ++j1)
      if (j1 < n1y) {
        const C2 v = in[(n2y * j1 + j2y) * nxh + kx1];
        xr[j1] = v.x;
        xi[j1] = v.y;
      }
  }
  __syncthreads();
  if (ty1) {
    dft_reg(xr, xi, n1y, T(1));
    twiddle(xr, xi, n1y, twy, ny, j2y, T(1));
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
      if (k1 < n1y) {
        C2 v;
        v.x = xr[k1];
        v.y = xi[k1];
        buf[(k1 * n2y + j2y) * nxh + kx1] = v;
      }
  }
  __syncthreads();
  const bool ty2 = t < nxh * n1y;
  const int kx2 = t % nxh, k1y = t / nxh;
  if (ty2) {
#pragma unroll
    for (int j2 = 0; j2 < 8; ++j2)
      if (j2 < n2y) {
        const C2 v = buf[(k1y * n2y + j2) * nxh + kx2];
        xr[j2] = v.x;
        xi[j2] = v.y;
      }
    dft_reg(xr, xi, n2y, T(1));
  }
  __syncthreads();
  if (ty2) {
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2)
      if (k2 < n2y) {
        C2 v;
        v.x = xr[k2];
        v.y = xi[k2];
        buf[(k1y + n1y * k2) * rg + kx2] = v;
      }
  }
  __syncthreads();
  // Rows: task (jp, j2), j2 fastest; z(kx) = Ga(kx) + i Gb(kx) with
  // G(nx - kx) = conj G(kx).
  const bool tx1 = t < (nyp << lg2x);
  const int jp1 = t >> lg2x, j21 = t & (n2x - 1);
  const int nh = nx / 2;
  if (tx1) {
#pragma unroll
    for (int j1 = 0; j1 < 8; ++j1)
      if (j1 < n1x) {
        const int kx = (j1 << lg2x) + j21;
        const bool hi = kx > nh;
        const int kk = hi ? nx - kx : kx;
        const C2 ga = buf[(2 * jp1) * rg + kk], gb = buf[(2 * jp1 + 1) * rg + kk];
        const bool edge = kk == 0 || kk == nh;
        const T gai = edge ? T(0) : (hi ? -ga.y : ga.y);
        const T gbi = edge ? T(0) : (hi ? -gb.y : gb.y);
        xr[j1] = ga.x - gbi;
        xi[j1] = gai + gb.x;
      }
    dft_reg(xr, xi, n1x, T(1));
    twiddle(xr, xi, n1x, twx, nx, j21, T(1));
  }
  __syncthreads();
  if (tx1) {
#pragma unroll
    for (int k1 = 0; k1 < 8; ++k1)
      if (k1 < n1x) {
        C2 v;
        v.x = xr[k1];
        v.y = xi[k1];
        buf[jp1 * rs1 + k1 * (n2x + 1) + j21] = v;
      }
  }
  __syncthreads();
  const bool tx2 = t < (nyp << lg1x);
  const int jp2 = t >> lg1x, k12 = t & (n1x - 1);
  if (tx2) {
#pragma unroll
    for (int j2 = 0; j2 < 8; ++j2)
      if (j2 < n2x) {
        const C2 v = buf[jp2 * rs1 + k12 * (n2x + 1) + j2];
        xr[j2] = v.x;
        xi[j2] = v.y;
      }
    dft_reg(xr, xi, n2x, T(1));
    const T sc = T(1) / (T)(nx * ny);
    T* dst = u + (long long)(L.k0 + blockIdx.x) * L.nxy;
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2)
      if (k2 < n2x) {
        const int i = k12 + (k2 << lg1x);
        dst[(2 * jp2) * nx + i] = sc * xr[k2];
        dst[(2 * jp2 + 1) * nx + i] = sc * xi[k2];
      }
  }
}

__host__ __device__ constexpr bool is_pow2(int n) { return n > 0 && !(n & (n - 1)); }

template <typename T>
void spectral_solve(pic_ctx* c, int l) {
  hipStream_t st = c->stream;
  Level& L = c->lev[l];
  const LevelC Lc = level_c(c, l);
  const int nm = c->spec_modes, np = c->spec_planes;
  T* s = reinterpret_cast<T*>(c->spec_s);
  T* mi = reinterpret_cast<T*>(c->spec_m);
  if (!c->spec_ready) {
    k_spec_factor<T><<<nblocks(nm), kThreads, 0, st>>>(Lc, mi, nm);
    c->spec_ready = true;
  }
  const bool fft = is_pow2(L.nx) && is_pow2(L.ny) && L.nx <= kSpecMaxFFT &&
                   L.ny <= kSpecMaxFFT;
  if (fft)
    k_spec_fwd_fft<T><<<(unsigned)np, kFftThreads, 0, st>>>(Lc, lev_f<T>(L), s, nm, c->dc);
  else
    k_spec_fwd<T><<<(unsigned)np, kSpecThreads, 0, st>>>(Lc, lev_f<T>(L), s, nm, c->dc);
  const int lgw = spec_tri_lgw(np);
  const int mpb = 1 << (lgw - 1);  // modes per workgroup
  k_spec_tri<T><<<(unsigned)((nm + mpb - 1) / mpb), kSpecThreads, 0, st>>>(
      Lc, s, mi, nm, lgw, c->dc);
  if (fft)
    k_spec_inv_fft<T><<<(unsigned)np, kFftThreads, 0, st>>>(Lc, s, lev_u<T>(L), nm, c->dc);
  else
    k_spec_inv<T><<<(unsigned)np, kSpecThreads, 0, st>>>(Lc, s, lev_u<T>(L), nm, c->dc);
}

// Workgroups of k_smooth2<T, *> the current device runs at once.
template <typename T>
long long smooth_slots() {
  static long long cached[64] = {0};
  int dev = 0;
  hipGetDevice(&dev);
  if (dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_smooth2<T, false, kSmPlain>,
                                                     smooth_threads<T>(), 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    // FP32 resident workgroups are many (small LDS ring, few registers):
    // half of them, in segments twice as long, spend fewer steps on the
    // segment ends and measured faster.
    cached[dev] = std::max(1LL, (long long)per_cu * cus / (sizeof(T) == 4 ? 2 : 1));
  }
  return cached[dev];
}

// Level l is smoothed by the fused two-sweep pass (it is neither the exact
// coarse level, the coarsest, nor in the single-workgroup tail).
template <typename T>
bool level_fused(pic_ctx* c, int l) {
  if (l == c->spec_level || l >= c->nlev - 1 || l >= tail_first<T>(c)) return false;
  const Level& L = c->lev[l];
  return lev_s<T>(c->lev[l]) && !(c->cfg.flags & PIC_FLAG_PLAIN_SMOOTHER) &&
         c->cfg.nu_pre == 2 && c->cfg.nu_post == 2 && L.nx >= SmoothTile<T>::SX &&
         L.ny >= SmoothTile<T>::SY;
}

template <typename T, bool NEU>
void launch_smooth(unsigned grid, hipStream_t st, const T* in, T* out,
                   const T* f, LevelC L, int seg, const Counters* dc, int mode,
                   double* u64) {
  constexpr int nt = smooth_threads<T>();
  if constexpr (std::is_same<T, float>::value) {
    switch (mode) {
      case kSmZeroIn:
        k_smooth2<T, NEU, kSmZeroIn><<<grid, nt, 0, st>>>(in, out, f, L, seg, dc, u64);
        return;
      case kSmAcc64:
        k_smooth2<T, NEU, kSmAcc64><<<grid, nt, 0, st>>>(in, out, f, L, seg, dc, u64);
        return;
      case kSmZeroIn | kSmAcc64:
        k_smooth2<T, NEU, kSmZeroIn | kSmAcc64><<<grid, nt, 0, st>>>(in, out, f, L, seg, dc, u64);
        return;
      default:
        break;
    }
  }
  k_smooth2<T, NEU, kSmPlain><<<grid, nt, 0, st>>>(in, out, f, L, seg, dc, u64);
}

// One V(nu_pre, nu_post) cycle from level l down.  Level 0 of an FP32
// cycle is the correction equation of the mixed form; l0_mode gives the
// pass modes of its fused smoothing (kSmZeroIn for the pre-smoothing pass,
// kSmAcc64 for the post-smoothing one).
template <typename T>
void vcycle(pic_ctx* c, int l, int l0_mode = kSmPlain) {
  hipStream_t st = c->stream;
  if (l == c->spec_level) {
    spectral_solve<T>(c, l);
    return;
  }
  const int tf = tail_first<T>(c);
  if (l == c->nlev - 1 && tf == c->nlev) {
    k_coarse_global<T><<<1, 1024, 0, st>>>(lev_u<T>(c->lev[l]),
                                           lev_f<T>(c->lev[l]), level_c(c, l),
                                           c->cfg.coarse_sweeps, c->dc,
                                           reinterpret_cast<T*>(c->partials));
    return;
  }
  {
    if (l >= tf) {
      TailLevels A;
      long long off = 0;
      for (int q = l; q < c->nlev; ++q) {
        A.L[q] = level_c(c, q);
        A.off[q] = off;
        off += c->lev[q].nnodes;
      }
      A.u0 = lev_u<T>(c->lev[l]);
      A.f0 = lev_f<T>(c->lev[l]);
      A.total = off;
      A.first = l;
      A.last = c->nlev - 1;
      A.nu_pre = c->cfg.nu_pre;
      A.nu_post = c->cfg.nu_post;
      A.coarse_sweeps = c->cfg.coarse_sweeps;
      k_mg_tail<T><<<1, 1024, 0, st>>>(A, c->dc);
      return;
    }
  }
  Level& L = c->lev[l];
  LevelC Lc = level_c(c, l);
  T* u = lev_u<T>(L);
  T* f = lev_f<T>(L);
  const long long nhalf = (long long)(L.nx / 2) * L.ny * (Lc.k1 - Lc.k0 + 1);
  // Fused pass (two sweeps each way): u -> spare before the restriction,
  // the coarse correction is added to the spare, spare -> u after.
  T* sp = lev_s<T>(L);
  const bool fused = level_fused<T>(c, l);
  unsigned fgrid = 0;
  int seg = 0;
  if (fused) {
    // One round of workgroups: as many z segments as the device keeps
    // resident, since each segment's march is a latency-bound chain.
    constexpr int kSX = SmoothTile<T>::SX, kSY = SmoothTile<T>::SY;
    const long long nxy_t = (long long)((L.nx + kSX - 1) / kSX) * ((L.ny + kSY - 1) / kSY);
    const long long slots = smooth_slots<T>();
    seg = (int)(((long long)(L.nz + 1) * nxy_t + slots - 1) / slots);
    // A segment of seg planes takes seg + 6 steps: below 4 the start-up
    // steps dominate.
    seg = seg < 4 ? 4 : seg;
    fgrid = (unsigned)(nxy_t * ((L.nz + 1 + seg - 1) / seg));
  }
  auto smooth_plain = [&](int sweeps) {
    for (int s = 0; s < sweeps; ++s)
      for (int color = 0; color < 2; ++color) {
        if (l == 0) tmark(c, PIC_PH_SMOOTH0, true);
        k_rbgs<T><<<nblocks(nhalf), kThreads, 0, st>>>(u, f, Lc, color, c->dc);
        if (l == 0) tmark(c, PIC_PH_SMOOTH0, false);
      }
  };
  auto smooth_fused = [&](const T* in, T* out, int mode) {
    if (l == 0) tmark(c, PIC_PH_SMOOTH0, true);
    if (Lc.k0 == 0 || Lc.k1 == Lc.nz)
      launch_smooth<T, true>(fgrid, st, in, out, f, Lc, seg, c->dc, mode, c->lev[0].u);
    else
      launch_smooth<T, false>(fgrid, st, in, out, f, Lc, seg, c->dc, mode, c->lev[0].u);
    if (l == 0) tmark(c, PIC_PH_SMOOTH0, false);
  };
  const int pre_mode = l == 0 ? (l0_mode & kSmZeroIn) : kSmPlain;
  const int post_mode = l == 0 ? (l0_mode & kSmAcc64) : kSmPlain;
  T* uc = u;  // fine values the restriction reads and the prolongation corrects
  if (fused) {
    smooth_fused(u, sp, pre_mode);
    uc = sp;
  } else {
    smooth_plain(c->cfg.nu_pre);
  }
  Level& N = c->lev[l + 1];
  LevelC Nc = level_c(c, l + 1);
  constexpr int kRX = RTile<T>::RX, kRY = RTile<T>::RY, kRZ = RTile<T>::RZ;
  if (N.nx >= kRX && N.ny >= kRY) {
    const long long nb = (long long)((N.nx + kRX - 1) / kRX) *
                         ((N.ny + kRY - 1) / kRY) * ((Nc.k1 - Nc.k0 + kRZ) / kRZ);
    k_restrict_tiled<T><<<(unsigned)nb, restrict_threads<T>(), 0, st>>>(
        uc, f, lev_u<T>(N), lev_f<T>(N), Lc, Nc, c->dc);
  } else {
    k_restrict<T><<<nblocks(N.nnodes), kThreads, 0, st>>>(
        uc, f, lev_u<T>(N), lev_f<T>(N), Lc, Nc, c->dc);
  }
  vcycle<T>(c, l + 1);
  {
    const int nbx = (Lc.nx / 2 + 63) / 64;
    const long long nby = ((long long)Lc.ny * (Lc.k1 - Lc.k0 + 1) + 3) / 4;
    k_prolong_pairs<T><<<(unsigned)(nbx * nby), 256, 0, st>>>(
        uc, lev_u<T>(N), Lc, Nc, nbx, c->dc);
  }
  if (fused)
    smooth_fused(sp, u, post_mode);
  else
    smooth_plain(c->cfg.nu_post);
}

}  // namespace

void field_rhs(pic_ctx* c, const double* rho) {
  LevelC L0 = level_c(c, 0);
  const double dx = c->g.dx;
  double scale;
  if (rho) {
    scale = (dx * dx) / kEps0;
  } else {
    scale = (((double)c->cfg.w_sp * kE) * kQScale) / (kEps0 * dx);
  }
  k_rhs<<<kRedBlocks, kThreads, 0, c->stream>>>(
      c->acc, rho, c->lev[0].f, c->lev[0].u, L0, dx, scale, rho ? 1 : 0,
      c->cfg.field_solve, c->cfg.v_lo, c->cfg.v_hi, c->partials,
      c->qpartials);
  k_final<<<1, 1024, 0, c->stream>>>(c->partials, c->qpartials, kRedBlocks,
                                     c->dc, 0, c->cfg.rel_tol);
}

// Solve A phi = b on level 0 (phi holds the warm start, or zero).  One
// synchronisation per batch of V-cycles; the batch size follows the last
// solve so a warm-started step normally syncs once.
void field_solve(pic_ctx* c, bool warm, pic_solve_info* info, int* status) {
  hipStream_t st = c->stream;
  Level& L0 = c->lev[0];
  LevelC Lc = level_c(c, 0);
  if (!warm) {
    const long long nu = Lc.nxy * (Lc.k1 - Lc.k0 + 1);
    hipMemsetAsync(L0.u + (long long)Lc.k0 * Lc.nxy, 0, nu * sizeof(double),
                   st);
  }
  const long long nu = Lc.nxy * (Lc.k1 - Lc.k0 + 1);
  // Mixed form: with a fused level-0 pass the correction solve starts from
  // zero and ends in the FP64 potential by itself; otherwise the FP32
  // correction is zeroed with each residual and added by k_correct.
  const bool mixed_fused = c->mixed && level_fused<float>(c, 0);
  float* rf = c->mixed ? L0.ff : nullptr;
  float* ef = c->mixed && !mixed_fused ? L0.uf : nullptr;
  bool used_net = false;
  if (warm && (c->warm_mode == PIC_WS_RECORD || c->warm_mode == PIC_WS_UNET)) {
    tmark(c, PIC_PH_WARM, true);
    // Record the normalised residual of the previous potential (the
    // network's input, and with the solution the training target).
    double vref = 1.0;
    if (c->cfg.bc_lo == PIC_BC_DIRICHLET && fabs(c->cfg.v_lo) > vref) vref = fabs(c->cfg.v_lo);
    if (c->cfg.bc_hi == PIC_BC_DIRICHLET && fabs(c->cfg.v_hi) > vref) vref = fabs(c->cfg.v_hi);
    k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                                c->dc, nullptr, nullptr);
    k_warm_final<<<1, 1024, 0, st>>>(c->partials, kRedBlocks, c->dc, 0,
                                     (double)nu);
    k_warm_input<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->dc,
                                                  1.0 / vref, c->warm_x,
                                                  c->warm_prev);
    c->warm_recorded = true;
    const float* out = nullptr;
    if (c->warm_mode == PIC_WS_UNET && c->net &&
        pic_unet_infer(c->net, c->warm_x, Lc.nz, Lc.ny, Lc.nx, st, &out)) {
      used_net = true;
      k_warm_apply<<<kRedBlocks, kThreads, 0, st>>>(L0.u, c->warm_prev, out,
                                                    Lc, c->dc);
      k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                                  c->dc, nullptr, nullptr);
      k_warm_final<<<1, 1024, 0, st>>>(c->partials, kRedBlocks, c->dc, 1,
                                       (double)nu);
      k_warm_revert<<<kRedBlocks, kThreads, 0, st>>>(L0.u, c->warm_prev, Lc,
                                                     c->dc);
    }
    tmark(c, PIC_PH_WARM, false);
  }
  // Initial check of the warm start.
  k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                              c->dc, rf, ef);
  k_final<<<1, 1024, 0, st>>>(c->partials, c->qpartials, kRedBlocks, c->dc, 2,
                              c->cfg.rel_tol);
  int launched = 0;
  // FP64: a V-cycle needs no residual, since the check only decides when to
  // stop, so the cycles the last solve says will not suffice run unchecked
  // (a solve that converges sooner just ends more accurate).  Mixed:
  // refinement rounds of kInner FP32 V-cycles on the correction equation
  // A e = r (r the FP64 residual rounded to FP32; two over-relaxed cycles cut
  // its error about 10^4-fold, to near FP32 accuracy), the correction added
  // to phi in FP64, then the FP64 residual: the convergence check and the
  // next round's right-hand side.  Batches count cycles in FP64 and rounds
  // in the mixed form.
  constexpr int kInner = 2;
  const int last = c->last_vcycles > 0 ? c->last_vcycles : 4;
  int batch = c->mixed ? (last + kInner - 1) / kInner : last;
  const int unchecked = c->mixed ? 0 : std::max(0, batch - 2);
  int pending = 0;  // FP64 cycles run since the last check
  *status = PIC_OK;
  while (true) {
    for (int b = 0; b < batch && launched < c->cfg.max_vcycles; ++b) {
      if (c->mixed) {
        const int n_in = std::min(kInner, c->cfg.max_vcycles - launched);
        for (int i = 0; i < n_in; ++i, ++launched) {
          int mode = kSmPlain;
          if (mixed_fused && i == 0) mode |= kSmZeroIn;
          if (mixed_fused && i == n_in - 1) mode |= kSmAcc64;
          vcycle<float>(c, 0, mode);
        }
        if (!mixed_fused)
          k_correct<<<nblocks(nu), kThreads, 0, st>>>(L0.u, L0.uf, Lc, c->dc);
        k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                                    c->dc, rf, ef);
        k_final<<<1, 1024, 0, st>>>(c->partials, c->qpartials, kRedBlocks,
                                    c->dc, 4, c->cfg.rel_tol, n_in);
        continue;
      }
      vcycle<double>(c, 0);
      ++pending;
      if (launched++ < unchecked) continue;
      k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                                  c->dc, rf, ef);
      k_final<<<1, 1024, 0, st>>>(c->partials, c->qpartials, kRedBlocks,
                                  c->dc, 1, c->cfg.rel_tol, pending);
      pending = 0;
    }
    if (pending) {  // the cycle limit ended the batch before its check
      k_residual<<<kRedBlocks, kThreads, 0, st>>>(L0.u, L0.f, Lc, c->partials,
                                                  c->dc, rf, ef);
      k_final<<<1, 1024, 0, st>>>(c->partials, c->qpartials, kRedBlocks,
                                  c->dc, 1, c->cfg.rel_tol, pending);
      pending = 0;
    }
    constexpr size_t kOff = offsetof(Counters, vcycles);
    hipMemcpyAsync(reinterpret_cast<char*>(c->hpin) + kOff,
                   reinterpret_cast<const char*>(c->dc) + kOff,
                   sizeof(Counters) - kOff, hipMemcpyDeviceToHost, st);
    stream_wait(c);
    std::memcpy(reinterpret_cast<char*>(&c->hc) + kOff,
                reinterpret_cast<const char*>(c->hpin) + kOff,
                sizeof(Counters) - kOff);
    if (c->hc.done || launched >= c->cfg.max_vcycles) break;
    batch = 1;
  }
  info->vcycles = c->hc.vcycles;
  info->converged = c->hc.done && !(c->hc.err & kErrNonFinite) ? 1 : 0;
  info->rel_residual = c->hc.rel_res;
  info->b_norm = c->hc.b_norm;
  info->rel_residual0 = c->hc.rel_res0;
  info->warm_used = used_net ? 1 : 0;
  info->warm_rejected = used_net ? c->hc.warm_reject : 0;
  info->warm_ratio = used_net ? c->hc.warm_ratio : 1.0;
  info->refinements = c->hc.refinements;
  c->last_vcycles = c->hc.vcycles > 0 ? c->hc.vcycles : 1;
  if (!info->converged) *status = PIC_ERR_NOCONV;
}

void field_extrapolate(pic_ctx* c) {
  if (c->hist_valid) {
    k_extrap<<<kRedBlocks, kThreads, 0, c->stream>>>(c->lev[0].u, c->phi_hist,
                                                     c->nnodes);
    std::swap(c->lev[0].u, c->phi_hist);
  } else {
    hipMemcpyAsync(c->phi_hist, c->lev[0].u, c->nnodes * sizeof(double),
                   hipMemcpyDeviceToDevice, c->stream);
  }
}

void field_warm_target(pic_ctx* c, float* t) {
  k_warm_target<<<kRedBlocks, kThreads, 0, c->stream>>>(
      c->lev[0].u, c->warm_prev, level_c(c, 0), c->dc, t);
}

void field_efield(pic_ctx* c) {
  LevelC L0 = level_c(c, 0);
  const double h = 0.5 * c->g.inv_dx;
  const double q_unit = ((double)c->cfg.w_sp * kE) * kQScale;
  if (c->mixed)
    k_efield<float><<<kRedBlocks, kThreads, 0, c->stream>>>(
        c->lev[0].u, c->acc, reinterpret_cast<float*>(c->E), L0, h, q_unit,
        c->partials);
  else
    k_efield<double><<<kRedBlocks, kThreads, 0, c->stream>>>(
        c->lev[0].u, c->acc, c->E, L0, h, q_unit, c->partials);
  k_final<<<1, 1024, 0, c->stream>>>(c->partials, c->qpartials, kRedBlocks,
                                     c->dc, 3, 0.0);
}

}  // namespace pic
