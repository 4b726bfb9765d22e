// Learned Poisson warm start: a 3-D U-Net (levels of 16/32/64/128
// channels, 3x3x3 convolutions, average pooling down, nearest upsampling
// and concatenation up, 1x1x1 head) with BF16 activations and weights and
// FP32 accumulation on the CDNA4 matrix cores, plus its backward pass and
// an Adam optimiser with FP32 master weights.
//
// Tensors are channels-last (D, H, W, C) BF16; padding is circular in x, y
// and zero in z.  The 3x3x3 convolution is an implicit GEMM: M = voxels,
// N = output channels, K = 27 * C_in flattened as (tap, channel) and walked
// in chunks of 32 by v_mfma_f32_16x16x32_bf16 (lane l holds row l % 16 and
// k = 8 (l / 16) .. +7 of A and B; D rows 4 (l / 16) .. +3, column l % 16).
// The input tile of a workgroup is staged in LDS per slice of 16 channels.
// The backward-data convolution is the same kernel with the kernel flipped
// and the channel roles swapped; the weight gradient is a second GEMM whose
// reduction runs over voxels, staged through LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "pic.h"
#include "pic_ctx.h"
#include "pic_device.h"

struct pic_unet;

namespace pic {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16;  // storage

__device__ __forceinline__ float bf2f(bf16 h) {
  return __uint_as_float((unsigned)h << 16);
}
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
// Round to nearest even (the CDNA4 conversion instruction, two at a time).
__device__ __forceinline__ unsigned f2bf2(float lo, float hi) {
  const bf16x2v h = __builtin_convertvector((f2v){lo, hi}, bf16x2v);
  unsigned r;
  __builtin_memcpy(&r, &h, 4);
  return r;
}
__device__ __forceinline__ bf16 f2bf(float x) {
  return (bf16)(f2bf2(x, 0.0f) & 0xffffu);
}

__device__ __forceinline__ bf16x8 load8(const bf16* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}
__device__ __forceinline__ bf16x8 zero8() {
  const uint4 v = make_uint4(0, 0, 0, 0);
  bf16x8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}

struct Dims {
  int D, H, W;
  long long V;
};

// Vectors of 8 BF16 channels (16 B) for the data-movement kernels; voxel
// indices fit 32 bits for every supported grid.
__device__ __forceinline__ uint4 ld16(const bf16* p) {
  return *reinterpret_cast<const uint4*>(p);
}
__device__ __forceinline__ void st16(bf16* p, uint4 v) {
  *reinterpret_cast<uint4*>(p) = v;
}
__device__ __forceinline__ void unpack8(uint4 v, float* f) {
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    f[2 * q] = __uint_as_float(w[q] << 16);
    f[2 * q + 1] = __uint_as_float(w[q] & 0xffff0000u);
  }
}
__device__ __forceinline__ void voxel_xyz(unsigned v, const Dims& d, int& x,
                                          int& y, int& z) {
  x = (int)(v % (unsigned)d.W);
  const unsigned r = v / (unsigned)d.W;
  y = (int)(r % (unsigned)d.H);
  z = (int)(r / (unsigned)d.H);
}

__device__ __forceinline__ long long nb_voxel(const Dims& d, int z, int y,
                                              int x, int tap) {
  const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
  const int zz = z + dz;
  if (zz < 0 || zz >= d.D) return -1;
  int yy = y + dy, xx = x + dx;
  if (yy < 0) yy += d.H;
  if (yy >= d.H) yy -= d.H;
  if (xx < 0) xx += d.W;
  if (xx >= d.W) xx -= d.W;
  return ((long long)zz * d.H + yy) * d.W + xx;
}

constexpr int KP(int cin) { return (27 * cin + 63) / 64 * 64; }

// Stage the halo of a tile for one slice of 16 input channels into LDS:
// HV voxels of 32 B as two planes of 16-byte halves (x and y periodic, z
// zero-padded).  The slice is channels c0 .. c0 + 15 of a tensor of C
// channels per voxel: at the tile's dims, or (UP) at half of them, read as
// its nearest upsampling (fine voxel (z, y, x) takes coarse (z/2, y/2,
// x/2)).  Every global load of a thread is issued before the first LDS
// store, so they are all in flight together.  ONE: the level is at least a
// halo wide, so one wrap brings every coordinate into range.
template <int HX, int HY, int HZ, int NTH, bool ONE, bool UP>
__device__ __forceinline__ void stage_halo_w(uint4* lds, const bf16* __restrict__ in,
                                             int C, int c0, const Dims& d, int x0,
                                             int y0, int z0) {
  constexpr int HV = HX * HY * HZ;
  constexpr int PER = (2 * HV + NTH - 1) / NTH;
  uint4 val[PER];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int q = (int)threadIdx.x + m * NTH;
    const int hv = q >> 1, hh = q & 1;
    const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
    const int gz = z0 + hz - 1;
    val[m] = make_uint4(0, 0, 0, 0);
    if (q < 2 * HV && gz >= 0 && gz < d.D) {
      int gy = y0 + hy - 1, gx = x0 + hx - 1;
      if constexpr (ONE) {
        gy = gy < 0 ? gy + d.H : (gy >= d.H ? gy - d.H : gy);
        gx = gx < 0 ? gx + d.W : (gx >= d.W ? gx - d.W : gx);
      } else {
        gy = (gy + d.H) % d.H;
        gx = (gx + d.W) % d.W;
      }
      size_t gv;
      if constexpr (UP)
        gv = ((size_t)(gz >> 1) * (d.H >> 1) + (gy >> 1)) * (d.W >> 1) + (gx >> 1);
      else
        gv = ((size_t)gz * d.H + gy) * d.W + gx;
      val[m] = ld16(in + gv * C + c0 + hh * 8);
    }
  }
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int q = (int)threadIdx.x + m * NTH;
    if (q < 2 * HV) lds[(q & 1) * HV + (q >> 1)] = val[m];
  }
}

// The same halo held in registers between its loads and its LDS stores
// (halo_load / halo_store), so that the loads of the next slice can be in
// flight while the current one is computed.
template <int HX, int HY, int HZ, int NTH>
struct HaloRegs {
  static constexpr int HV = HX * HY * HZ;
  static constexpr int PER = (2 * HV + NTH - 1) / NTH;
  uint4 v[PER];
};

template <int HX, int HY, int HZ, int NTH, bool UP>
__device__ __forceinline__ void halo_load_c(HaloRegs<HX, HY, HZ, NTH>& r,
                                            const bf16* __restrict__ in, int C, int c0,
                                            const Dims& d, int x0, int y0, int z0) {
  constexpr int HV = HX * HY * HZ;
  const bool one = d.H >= HY && d.W >= HX;
#pragma unroll
  for (int m = 0; m < r.PER; ++m) {
    const int q = (int)threadIdx.x + m * NTH;
    const int hv = q >> 1, hh = q & 1;
    const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
    const int gz = z0 + hz - 1;
    r.v[m] = make_uint4(0, 0, 0, 0);
    if (q < 2 * HV && gz >= 0 && gz < d.D) {
      int gy = y0 + hy - 1, gx = x0 + hx - 1;
      if (one) {
        gy = gy < 0 ? gy + d.H : (gy >= d.H ? gy - d.H : gy);
        gx = gx < 0 ? gx + d.W : (gx >= d.W ? gx - d.W : gx);
      } else {
        gy = (gy + d.H) % d.H;
        gx = (gx + d.W) % d.W;
      }
      size_t gv;
      if constexpr (UP)
        gv = ((size_t)(gz >> 1) * (d.H >> 1) + (gy >> 1)) * (d.W >> 1) + (gx >> 1);
      else
        gv = ((size_t)gz * d.H + gy) * d.W + gx;
      r.v[m] = ld16(in + gv * C + c0 + hh * 8);
    }
  }
}

template <int HX, int HY, int HZ, int NTH>
__device__ __forceinline__ void halo_load(HaloRegs<HX, HY, HZ, NTH>& r,
                                          const bf16* __restrict__ in, int C,
                                          const Dims& d, int x0, int y0, int z0,
                                          int sl) {
  halo_load_c<HX, HY, HZ, NTH, false>(r, in, C, sl * 16, d, x0, y0, z0);
}

// Slice sl of 'in' (CIN channels), or with CU > 0 of the concatenation
// [up(in) (CU channels, half dims), skip (CIN - CU)].
template <int CIN, int CU, int HX, int HY, int HZ, int NTH>
__device__ __forceinline__ void halo_load_cat(HaloRegs<HX, HY, HZ, NTH>& r,
                                              const bf16* __restrict__ in,
                                              const bf16* __restrict__ skip,
                                              const Dims& d, int x0, int y0, int z0,
                                              int sl) {
  if (CU > 0 && sl * 16 < CU)
    halo_load_c<HX, HY, HZ, NTH, true>(r, in, CU, sl * 16, d, x0, y0, z0);
  else if (CU > 0)
    halo_load_c<HX, HY, HZ, NTH, false>(r, skip, CIN - CU, sl * 16 - CU, d, x0, y0, z0);
  else
    halo_load_c<HX, HY, HZ, NTH, false>(r, in, CIN, sl * 16, d, x0, y0, z0);
}

template <int HX, int HY, int HZ, int NTH>
__device__ __forceinline__ void halo_store(uint4* lds, const HaloRegs<HX, HY, HZ, NTH>& r) {
  constexpr int HV = HX * HY * HZ;
#pragma unroll
  for (int m = 0; m < r.PER; ++m) {
    const int q = (int)threadIdx.x + m * NTH;
    if (q < 2 * HV) lds[(q & 1) * HV + (q >> 1)] = r.v[m];
  }
}

// Slice sl of the input: of 'in' (CIN channels), or with CU > 0 of the
// concatenation [up(in) (CU channels, half dims), skip (CIN - CU)].
template <int CIN, int CU, int HX, int HY, int HZ, int NTH>
__device__ __forceinline__ void stage_halo(uint4* lds, const bf16* __restrict__ in,
                                           const bf16* __restrict__ skip,
                                           const Dims& d, int x0, int y0, int z0,
                                           int sl) {
  const bool one = d.H >= HY && d.W >= HX;
  if (CU > 0 && sl * 16 < CU) {
    if (one)
      stage_halo_w<HX, HY, HZ, NTH, true, true>(lds, in, CU, sl * 16, d, x0, y0, z0);
    else
      stage_halo_w<HX, HY, HZ, NTH, false, true>(lds, in, CU, sl * 16, d, x0, y0, z0);
    return;
  }
  const bf16* src = CU > 0 ? skip : in;
  const int C = CU > 0 ? CIN - CU : CIN, c0 = sl * 16 - CU;
  if (one)
    stage_halo_w<HX, HY, HZ, NTH, true, false>(lds, src, C, c0, d, x0, y0, z0);
  else
    stage_halo_w<HX, HY, HZ, NTH, false, false>(lds, src, C, c0, d, x0, y0, z0);
}


// out = act(conv(in) + bias), LDS-tiled.  A workgroup owns an output tile
// of 16 (x) x TY x TZ voxels; per slice of 16 input channels it stages the
// tile's halo (18 x (TY+2) x (TZ+2) voxels, 32 B each, x and y periodic, z
// zero-padded) in LDS, so an input voxel is read from memory about twice
// per layer instead of once per tap; the two 8-channel halves of a voxel sit
// in separate LDS planes so that 16 lanes reading consecutive voxels touch
// 256 contiguous bytes.  A K-chunk of 32 is two taps x 16
// channels (lane group g = lane / 16: tap 2c + g / 2, channels 8 (g % 2) ..
// +7); the A operand comes from LDS, the B operand (weights) from the
// cache.  Each wave owns MT rows of 16 voxels and all COUT / 16 column
// tiles, with MT * COUT / 16 <= 16 accumulator tiles.
template <int CIN, int COUT, int TY, int TZ>
__global__ void __launch_bounds__(256) k_conv3t(const bf16* __restrict__ in,
                                                const bf16* __restrict__ Wk,
                                                const float* __restrict__ bias,
                                                bf16* __restrict__ out, Dims d,
                                                int relu) {
  constexpr int NT = COUT / 16;
  constexpr int TX = 16;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  constexpr int HV = HX * HY * HZ;
  constexpr int MT = TY * TZ / 4;
  constexpr int KPAD = KP(CIN);
  constexpr int NS = CIN / 16;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel multiples of 16");
  static_assert(MT >= 1 && MT * NT <= 16, "accumulator budget");
  __shared__ uint4 lds[HV * 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ntx = (d.W + TX - 1) / TX, nty = (d.H + TY - 1) / TY;
  // Neighbouring tiles share halo voxels: keep them on one XCD's L2.
  int bi = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = bi % ntx;
  bi /= ntx;
  const int ty = bi % nty, tz = bi / nty;
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int kg = lane >> 4, rl = lane & 15;
  const int half = kg & 1;
  f4 acc[MT][NT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
  for (int sl = 0; sl < NS; ++sl) {
    stage_halo<CIN, 0, HX, HY, HZ, 256>(lds, in, nullptr, d, x0, y0, z0, sl);
    __syncthreads();
    // Chunks 0..12 hold two taps; chunk 13 holds tap 26 and padding.
    auto chunk = [&](int ch, bool last) {
      const int tap = 2 * ch + (kg >> 1);
      const bool tv = !last || tap < 27;
      const int oz = tap / 9, oy = (tap / 3) % 3, ox = tap % 3;
      bf16x8 b[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = tv ? load8(Wk + (size_t)(nt * 16 + rl) * KPAD + tap * CIN + sl * 16 + half * 8)
                   : zero8();
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        const int r = wave * MT + mt;
        const int ly = r % TY, lz = r / TY;
        const int hv = ((lz + oz) * HY + (ly + oy)) * HX + rl + ox;
        bf16x8 a = zero8();
        if (tv) {
          const uint4 w = lds[half * HV + hv];
          __builtin_memcpy(&a, &w, 16);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[nt], acc[mt][nt], 0, 0, 0);
      }
    };
#pragma unroll 1
    for (int ch = 0; ch < 13; ++ch) chunk(ch, false);
    chunk(13, true);
    __syncthreads();
  }
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
    const int r = wave * MT + mt;
    const int gy = y0 + r % TY, gz = z0 + r / TY;
    if (gy >= d.H || gz >= d.D) continue;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + rl;
      const float bv = bias ? bias[co] : 0.0f;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int x = x0 + 4 * kg + j;
        if (x >= d.W) continue;
        float v = acc[mt][nt][j] + bv;
        if (relu) v = v > 0.0f ? v : 0.0f;
        out[(((size_t)gz * d.H + gy) * d.W + x) * COUT + co] = f2bf(v);
      }
    }
  }
}

// out = act(conv(in) + bias), register-blocked over output rows.  A
// workgroup owns an output tile of 16 (x) x 4WY x 4WZ voxels and stages its
// halo per slice of 16 input channels in LDS as k_conv3t does.  Each wave
// owns one 16-channel tile of C_out and a block of 4 x 4 output rows (y, z)
// of 16 voxels.  An input row of the halo is one MFMA operand whose K of 32
// is two x-offsets of the row (x offsets 0 and 1, or 2 and a slot whose
// weights are zero), so one LDS read of an input row serves every output
// row it reaches, up to nine (three z by three y offsets), and the wave's
// 18 weight fragments of the slice (3 z x 3 y offsets x 2 x-pairs) stay in
// registers: per slice a wave reads 6 x 6 x 2 input fragments for 288
// MFMAs (a quarter of the second pair's products are with zero weights),
// against one read per MFMA when the operand is formed per tap.  The
// product is taken as W X (rows: output channels, columns: voxels), so a
// lane ends with four consecutive channels of one voxel, stored as one
// 8-byte word.
//
// With CU > 0 the input is the decoder's concatenation [up(in), skip]
// formed in the staging (in: CU channels at half the dims; skip: CIN - CU
// channels), so the concatenated tensor is never written.
template <int CIN, int COUT, int WY, int WZ, int CU = 0>
__global__ void __launch_bounds__(64 * (COUT / 16) * WY * WZ) k_conv3r(
    const bf16* __restrict__ in, const bf16* __restrict__ skip,
    const bf16* __restrict__ Wk, const float* __restrict__ bias,
    bf16* __restrict__ out, Dims d, int relu) {
  static_assert(CU % 16 == 0 && CU < CIN, "concatenation split on slices");
  constexpr int NTC = COUT / 16, RY = 4, RZ = 4;
  constexpr int TX = 16, TY = WY * RY, TZ = WZ * RZ;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  constexpr int HV = HX * HY * HZ;
  constexpr int NTH = 64 * NTC * WY * WZ;
  constexpr int KPAD = KP(CIN);
  constexpr int NS = CIN / 16;
  static_assert(CIN % 16 == 0 && COUT % 16 == 0, "channel multiples of 16");
  __shared__ uint4 lds[HV * 2];
  // The wave index is uniform: scalar, so the per-row tests are scalar.
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nt = wave % NTC, sp = wave / NTC;
  const int wy = sp % WY, wz = sp / WY;
  const int ntx = (d.W + TX - 1) / TX, nty = (d.H + TY - 1) / TY;
  int bi = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = bi % ntx;
  bi /= ntx;
  const int ty = bi % nty, tz = bi / nty;
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int kg = lane >> 4, rl = lane & 15;
  const int half = kg & 1, slot = kg >> 1;
  const bf16* wrow = Wk + (size_t)(nt * 16 + rl) * KPAD + half * 8;
  f4 acc[RZ][RY];
#pragma unroll
  for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
    for (int yo = 0; yo < RY; ++yo) acc[zo][yo] = f4{0.f, 0.f, 0.f, 0.f};
  // PF: the next slice's halo loads are issued before the current slice is
  // computed and stored to LDS once it is done, holding the halo share in
  // registers through the MFMAs.  That paid where the kernel still fits two
  // waves per SIMD (32 and 64 output channels) and lost elsewhere.
  constexpr bool PF = CU == 0 && (COUT == 32 || COUT == 64) && NS > 1;
  if constexpr (PF) {
    HaloRegs<HX, HY, HZ, NTH> hr;
    halo_load(hr, in, CIN, d, x0, y0, z0, 0);
    halo_store(lds, hr);
    for (int sl = 0; sl < NS; ++sl) {
      if (sl + 1 < NS) halo_load(hr, in, CIN, d, x0, y0, z0, sl + 1);
      // Weight fragments of the slice: tap (oz, oy, ox) with ox = slot in the
      // first x-pair and ox = 2 (slot 0 only; zero in slot 1) in the second.
      bf16x8 wa[3][3], wb[3][3];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
          const int t0 = oz * 9 + oy * 3;
          wa[oz][oy] = load8(wrow + (t0 + slot) * CIN + sl * 16);
          const bf16x8 w2 = load8(wrow + (t0 + 2) * CIN + sl * 16);
          wb[oz][oy] = slot == 0 ? w2 : zero8();
        }
      __syncthreads();
      const uint4* lh = lds + half * HV + rl;
#pragma unroll
      for (int iz = 0; iz < RZ + 2; ++iz)
#pragma unroll
        for (int iy = 0; iy < RY + 2; ++iy) {
          const int hv = ((wz * RZ + iz) * HY + (wy * RY + iy)) * HX;
          // Slot 1 of the second pair reads the x + 2 voxel too (its weights
          // are zero): no divergent load.
          bf16x8 fa, fb;
          {
            const uint4 w0 = lh[hv + slot], w1 = lh[hv + 2];
            __builtin_memcpy(&fa, &w0, 16);
            __builtin_memcpy(&fb, &w1, 16);
          }
          // The products of one fragment go to distinct accumulators, so the
          // MFMAs of a pass are independent.
#pragma unroll
          for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
              const int zo = iz - oz, yo = iy - oy;
              if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
                acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[oz][oy], fa, acc[zo][yo], 0, 0, 0);
            }
#pragma unroll
          for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
              const int zo = iz - oz, yo = iy - oy;
              if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
                acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[oz][oy], fb, acc[zo][yo], 0, 0, 0);
            }
        }
      if (sl + 1 < NS) {
        __syncthreads();
        halo_store(lds, hr);
      }
    }
  } else {
    for (int sl = 0; sl < NS; ++sl) {
      stage_halo<CIN, CU, HX, HY, HZ, NTH>(lds, in, skip, d, x0, y0, z0, sl);
      // Weight fragments of the slice: tap (oz, oy, ox) with ox = slot in the
      // first x-pair and ox = 2 (slot 0 only; zero in slot 1) in the second.
      bf16x8 wa[3][3], wb[3][3];
#pragma unroll
      for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
          const int t0 = oz * 9 + oy * 3;
          wa[oz][oy] = load8(wrow + (t0 + slot) * CIN + sl * 16);
          const bf16x8 w2 = load8(wrow + (t0 + 2) * CIN + sl * 16);
          wb[oz][oy] = slot == 0 ? w2 : zero8();
        }
      __syncthreads();
      const uint4* lh = lds + half * HV + rl;
#pragma unroll
      for (int iz = 0; iz < RZ + 2; ++iz)
#pragma unroll
        for (int iy = 0; iy < RY + 2; ++iy) {
          const int hv = ((wz * RZ + iz) * HY + (wy * RY + iy)) * HX;
          // Slot 1 of the second pair reads the x + 2 voxel too (its weights
          // are zero): no divergent load.
          bf16x8 fa, fb;
          {
            const uint4 w0 = lh[hv + slot], w1 = lh[hv + 2];
            __builtin_memcpy(&fa, &w0, 16);
            __builtin_memcpy(&fb, &w1, 16);
          }
          // The products of one fragment go to distinct accumulators, so the
          // MFMAs of a pass are independent.
#pragma unroll
          for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
              const int zo = iz - oz, yo = iy - oy;
              if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
                acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[oz][oy], fa, acc[zo][yo], 0, 0, 0);
            }
#pragma unroll
          for (int oz = 0; oz < 3; ++oz)
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
              const int zo = iz - oz, yo = iy - oy;
              if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
                acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[oz][oy], fb, acc[zo][yo], 0, 0, 0);
            }
        }
      __syncthreads();
    }
  }
  // Lane: voxel x0 + rl, channels nt * 16 + 4 kg .. +3.
  const int x = x0 + rl;
  const int c0 = nt * 16 + 4 * kg;
  float bv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bv[j] = bias ? bias[c0 + j] : 0.0f;
  if (x < d.W) {
#pragma unroll
    for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
      for (int yo = 0; yo < RY; ++yo) {
        const int gy = y0 + wy * RY + yo, gz = z0 + wz * RZ + zo;
        if (gy >= d.H || gz >= d.D) continue;
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          v[j] = acc[zo][yo][j] + bv[j];
          if (relu) v[j] = fmaxf(v[j], 0.0f);
        }
        uint2 w;
        w.x = f2bf2(v[0], v[1]);
        w.y = f2bf2(v[2], v[3]);
        *reinterpret_cast<uint2*>(out + (((size_t)gz * d.H + gy) * d.W + x) * COUT + c0) = w;
      }
  }
}

// k_conv3r for 16 output channels as a persistent kernel: as many
// workgroups as the GPU holds at once, each taking a contiguous run of
// tiles (of one XCD's range, so that neighbouring tiles share its L2), its
// (tile, slice) items in turn.  The halo loads of the next item are issued
// before the current item is computed and stored to LDS after it, and with
// one slice the weight fragments are loaded once per workgroup; a one-shot
// workgroup otherwise waits on its halo loads with nothing to compute.
template <int CIN, int CU = 0>
__global__ void __launch_bounds__(256) k_conv3p(
    const bf16* __restrict__ in, const bf16* __restrict__ skip,
    const bf16* __restrict__ Wk, const float* __restrict__ bias,
    bf16* __restrict__ out, Dims d, int relu) {
  static_assert(CU % 16 == 0 && CU < CIN && CIN % 16 == 0, "channel slices");
  constexpr int RY = 4, RZ = 4, WY = 2;
  constexpr int TX = 16, TY = 8, TZ = 8;
  constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  constexpr int HV = HX * HY * HZ;
  constexpr int NTH = 256;
  constexpr int KPAD = KP(CIN);
  constexpr int NS = CIN / 16;
  __shared__ uint4 lds[HV * 2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int wy = wave % WY, wz = wave / WY;
  const int ntx = (d.W + TX - 1) / TX, nty = (d.H + TY - 1) / TY;
  const int ntiles = ntx * nty * ((d.D + TZ - 1) / TZ);
  const int per = (ntiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int lo = (int)xcd_block(blockIdx.x, gridDim.x) * per;
  const int hi = lo + per < ntiles ? lo + per : ntiles;
  if (lo >= hi) return;
  const int nitems = (hi - lo) * NS;
  const int kg = lane >> 4, rl = lane & 15;
  const int half = kg & 1, slot = kg >> 1;
  const bf16* wrow = Wk + (size_t)rl * KPAD + half * 8;
  const int c0 = 4 * kg;
  float bv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) bv[j] = bias ? bias[c0 + j] : 0.0f;
  auto origin = [&](int t, int& x0, int& y0, int& z0) {
    x0 = (t % ntx) * TX;
    y0 = ((t / ntx) % nty) * TY;
    z0 = (t / (ntx * nty)) * TZ;
  };
  f4 acc[RZ][RY];
#pragma unroll
  for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
    for (int yo = 0; yo < RY; ++yo) acc[zo][yo] = f4{0.f, 0.f, 0.f, 0.f};
  bf16x8 wa[3][3], wb[3][3];
  auto load_w = [&](int sl) {
#pragma unroll
    for (int oz = 0; oz < 3; ++oz)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy) {
        const int t0 = oz * 9 + oy * 3;
        wa[oz][oy] = load8(wrow + (t0 + slot) * CIN + sl * 16);
        const bf16x8 w2 = load8(wrow + (t0 + 2) * CIN + sl * 16);
        wb[oz][oy] = slot == 0 ? w2 : zero8();
      }
  };
  if (NS == 1) load_w(0);
  HaloRegs<HX, HY, HZ, NTH> hr;
  {
    int x0, y0, z0;
    origin(lo, x0, y0, z0);
    halo_load_cat<CIN, CU>(hr, in, skip, d, x0, y0, z0, 0);
    halo_store(lds, hr);
  }
  for (int j = 0; j < nitems; ++j) {
    const int t = lo + j / NS, sl = j % NS;
    if (j + 1 < nitems) {
      int x0, y0, z0;
      origin(lo + (j + 1) / NS, x0, y0, z0);
      halo_load_cat<CIN, CU>(hr, in, skip, d, x0, y0, z0, (j + 1) % NS);
    }
    if (NS > 1) load_w(sl);
    __syncthreads();
    const uint4* lh = lds + half * HV + rl + (wz * RZ * HY + wy * RY) * HX;
    // The input rows in a ring of three, each read two rows ahead of its
    // MFMAs so that the LDS latency is covered.
    constexpr int NP = (RZ + 2) * (RY + 2);
    uint4 ring[3][2];
    auto fetch = [&](int p, uint4 (&r)[2]) {
      const int hv = ((p / (RY + 2)) * HY + p % (RY + 2)) * HX;
      r[0] = lh[hv + slot];
      r[1] = lh[hv + 2];
    };
    fetch(0, ring[0]);
    fetch(1, ring[1]);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int iz = p / (RY + 2), iy = p % (RY + 2);
      if (p + 2 < NP) fetch(p + 2, ring[(p + 2) % 3]);
      {
        bf16x8 fa, fb;
        __builtin_memcpy(&fa, &ring[p % 3][0], 16);
        __builtin_memcpy(&fb, &ring[p % 3][1], 16);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
          for (int oy = 0; oy < 3; ++oy) {
            const int zo = iz - oz, yo = iy - oy;
            if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
              acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[oz][oy], fa, acc[zo][yo], 0, 0, 0);
          }
#pragma unroll
        for (int oz = 0; oz < 3; ++oz)
#pragma unroll
          for (int oy = 0; oy < 3; ++oy) {
            const int zo = iz - oz, yo = iy - oy;
            if (zo >= 0 && zo < RZ && yo >= 0 && yo < RY)
              acc[zo][yo] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wb[oz][oy], fb, acc[zo][yo], 0, 0, 0);
          }
      }
    }
    if (sl == NS - 1) {
      int x0, y0, z0;
      origin(t, x0, y0, z0);
      const int x = x0 + rl;
#pragma unroll
      for (int zo = 0; zo < RZ; ++zo)
#pragma unroll
        for (int yo = 0; yo < RY; ++yo) {
          const int gy = y0 + wy * RY + yo, gz = z0 + wz * RZ + zo;
          if (x < d.W && gy < d.H && gz < d.D) {
            float v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              v[q] = acc[zo][yo][q] + bv[q];
              if (relu) v[q] = fmaxf(v[q], 0.0f);
            }
            uint2 w;
            w.x = f2bf2(v[0], v[1]);
            w.y = f2bf2(v[2], v[3]);
            *reinterpret_cast<uint2*>(out + (((size_t)gz * d.H + gy) * d.W + x) * 16 + c0) = w;
          }
          acc[zo][yo] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (j + 1 < nitems) {
      __syncthreads();
      halo_store(lds, hr);
    }
  }
}

// Weight gradient dW[co][k] += sum_v g[v][co] x[v + tap(k)][ci(k)] over a
// chunk of voxels (dW unpadded: row stride 27 CIN); a workgroup owns 64 columns of k, each wave 16 of them
// for all COUT rows.  32-voxel slices of g and x are staged in LDS.
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_wgrad3(const bf16* __restrict__ x,
                                                const bf16* __restrict__ g,
                                                float* __restrict__ dW, Dims d,
                                                long long chunk) {
  constexpr int MT = COUT / 16;
  __shared__ __attribute__((aligned(16))) bf16 gs[32][COUT];
  __shared__ __attribute__((aligned(16))) bf16 xs[32][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int kbase = blockIdx.x * 64;
  const long long v0 = (long long)blockIdx.y * chunk;
  long long v1 = v0 + chunk;
  if (v1 > d.V) v1 = d.V;
  f4 acc[MT];
  for (int m = 0; m < MT; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
  for (long long vs = v0; vs < v1; vs += 32) {
    // Stage g (32 x COUT) and x (32 x 64 columns).
    for (int q = threadIdx.x; q < 32 * COUT / 8; q += 256) {
      const int vr = q / (COUT / 8), c8 = (q % (COUT / 8)) * 8;
      const long long v = vs + vr;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (v < v1) val = *reinterpret_cast<const uint4*>(g + v * COUT + c8);
      *reinterpret_cast<uint4*>(&gs[vr][c8]) = val;
    }
    {
      const int q = threadIdx.x;            // 32 voxels x 8 groups of 8
      const int vr = q >> 3, kg = (q & 7) * 8;
      const long long v = vs + vr;
      const int k = kbase + kg;
      const int tap = k / CIN, c = k - tap * CIN;
      uint4 val = make_uint4(0, 0, 0, 0);
      if (v < v1 && tap < 27) {
        const int xq = (int)(v % d.W), yq = (int)((v / d.W) % d.H),
                  zq = (int)(v / ((long long)d.W * d.H));
        const long long nv = nb_voxel(d, zq, yq, xq, tap);
        if (nv >= 0) val = *reinterpret_cast<const uint4*>(x + nv * CIN + c);
      }
      *reinterpret_cast<uint4*>(&xs[vr][kg]) = val;
    }
    __syncthreads();
    bf16x8 b;
    {
      bf16 tmp[8];
      for (int j = 0; j < 8; ++j) tmp[j] = xs[8 * (lane >> 4) + j][wave * 16 + (lane & 15)];
      __builtin_memcpy(&b, tmp, 16);
    }
    for (int m = 0; m < MT; ++m) {
      bf16 tmp[8];
      for (int j = 0; j < 8; ++j) tmp[j] = gs[8 * (lane >> 4) + j][m * 16 + (lane & 15)];
      bf16x8 a;
      __builtin_memcpy(&a, tmp, 16);
      acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[m], 0, 0, 0);
    }
    __syncthreads();
  }
  const int k = kbase + wave * 16 + (lane & 15);
  if (k >= 27 * CIN) return;
  for (int m = 0; m < MT; ++m)
    for (int j = 0; j < 4; ++j) {
      const int co = m * 16 + 4 * (lane >> 4) + j;
      atomicAdd(&dW[(long long)co * (27 * CIN) + k], acc[m][j]);
    }
}

// First layer (2 input channels): FP32 arithmetic, 16 outputs per voxel.
// The weights are indexed uniformly across the wave, so they come through
// the scalar cache as operands of the vector FMAs.
__global__ void __launch_bounds__(256) k_conv_first(
    const float* __restrict__ in, const float* __restrict__ W,  // [16][27][2]
    const float* __restrict__ b, bf16* __restrict__ out, Dims d) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (unsigned long long)d.V) return;
  int x, y, z;
  voxel_xyz(v, d, x, y, z);
  float acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = b[c];
#pragma unroll 3
  for (int tap = 0; tap < 27; ++tap) {
    const int zz = z + tap / 9 - 1;
    int yy = y + (tap / 3) % 3 - 1, xx = x + tap % 3 - 1;
    yy = yy < 0 ? yy + d.H : (yy >= d.H ? yy - d.H : yy);
    xx = xx < 0 ? xx + d.W : (xx >= d.W ? xx - d.W : xx);
    float2 i2 = make_float2(0.f, 0.f);
    if (zz >= 0 && zz < d.D)
      i2 = reinterpret_cast<const float2*>(in)[((unsigned)zz * d.H + yy) * d.W + xx];
#pragma unroll
    for (int c = 0; c < 16; ++c)
      acc[c] = fmaf(W[c * 54 + tap * 2 + 1], i2.y, fmaf(W[c * 54 + tap * 2], i2.x, acc[c]));
  }
  unsigned w[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const float a0 = acc[2 * q] > 0.f ? acc[2 * q] : 0.f;
    const float a1 = acc[2 * q + 1] > 0.f ? acc[2 * q + 1] : 0.f;
    w[q] = (unsigned)f2bf(a0) | ((unsigned)f2bf(a1) << 16);
  }
  st16(out + (size_t)v * 16, make_uint4(w[0], w[1], w[2], w[3]));
  st16(out + (size_t)v * 16 + 8, make_uint4(w[4], w[5], w[6], w[7]));
}

// dW of the first layer: a workgroup takes one tap and a chunk of voxels;
// each thread sums the 16 x 2 products g[v][co] x[v + tap][ci] of its
// voxels in registers, the wave reduces them with cross-lane shuffles, and
// the workgroup adds its 32 sums to dW[co][tap][ci] (16 x 27 x 2).
__global__ void __launch_bounds__(256) k_wgrad_first(
    const float* __restrict__ in, const bf16* __restrict__ g,
    float* __restrict__ dW, Dims d, unsigned chunk) {
  __shared__ float red[4][32];
  const int tap = blockIdx.y;
  const int oz = tap / 9 - 1, oy = (tap / 3) % 3 - 1, ox = tap % 3 - 1;
  const unsigned v0 = blockIdx.x * chunk;
  const unsigned long long vend = (unsigned long long)v0 + chunk;
  const unsigned v1 = vend < (unsigned long long)d.V ? (unsigned)vend : (unsigned)d.V;
  float acc[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) acc[e] = 0.f;
  for (unsigned v = v0 + threadIdx.x; v < v1; v += 256) {
    int x, y, z;
    voxel_xyz(v, d, x, y, z);
    const int zz = z + oz;
    if (zz < 0 || zz >= d.D) continue;
    int yy = y + oy, xx = x + ox;
    yy = yy < 0 ? yy + d.H : (yy >= d.H ? yy - d.H : yy);
    xx = xx < 0 ? xx + d.W : (xx >= d.W ? xx - d.W : xx);
    const float2 xi = reinterpret_cast<const float2*>(in)[((unsigned)zz * d.H + yy) * d.W + xx];
    float gf[16];
    unpack8(ld16(g + (size_t)v * 16), gf);
    unpack8(ld16(g + (size_t)v * 16 + 8), gf + 8);
#pragma unroll
    for (int co = 0; co < 16; ++co) {
      acc[2 * co] = fmaf(gf[co], xi.x, acc[2 * co]);
      acc[2 * co + 1] = fmaf(gf[co], xi.y, acc[2 * co + 1]);
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < 32; ++e) {
    float t = acc[e];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o);
    acc[e] = t;
  }
  if (lane == 0)
#pragma unroll
    for (int e = 0; e < 32; ++e) red[wave][e] = acc[e];
  __syncthreads();
  if (threadIdx.x < 32) {
    const float t = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                    (red[2][threadIdx.x] + red[3][threadIdx.x]);
    atomicAdd(&dW[(threadIdx.x >> 1) * 54 + tap * 2 + (threadIdx.x & 1)], t);
  }
}

// Bias gradient: sum over voxels per channel.  A thread adds 8 channels of
// its voxels; the workgroup reduces in LDS and adds one value per channel.
__global__ void __launch_bounds__(256) k_bias_grad(const bf16* __restrict__ g,
                                                   int C, Dims d,
                                                   float* __restrict__ db) {
  __shared__ float s[256][8];
  const unsigned G = (unsigned)C / 8;
  const unsigned rows = 256 / G;
  const unsigned r = threadIdx.x / G, cg = threadIdx.x % G;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (r < rows) {
    for (unsigned long long v = (unsigned long long)blockIdx.x * rows + r;
         v < (unsigned long long)d.V; v += (unsigned long long)gridDim.x * rows) {
      float f[8];
      unpack8(ld16(g + (size_t)v * C + 8 * cg), f);
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] += f[q];
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) s[threadIdx.x][q] = r < rows ? a[q] : 0.f;
  __syncthreads();
  if (threadIdx.x < (unsigned)C) {
    const unsigned c8 = threadIdx.x / 8, q = threadIdx.x % 8;
    float t = 0.f;
    for (unsigned rr = 0; rr < rows; ++rr) t += s[rr * G + c8][q];
    atomicAdd(&db[threadIdx.x], t);
  }
}

// gpre = gy * (y > 0), 8 values a thread.
__global__ void k_relu_bwd(const bf16* __restrict__ gy, const bf16* __restrict__ y,
                           bf16* __restrict__ gpre, long long n) {
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if ((unsigned long long)t * 8 >= (unsigned long long)n) return;
  const uint4 gv = ld16(gy + (size_t)t * 8), yv = ld16(y + (size_t)t * 8);
  const unsigned gw[4] = {gv.x, gv.y, gv.z, gv.w}, yw[4] = {yv.x, yv.y, yv.z, yv.w};
  unsigned o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const unsigned lo = (__uint_as_float(yw[q] << 16) > 0.f) ? (gw[q] & 0xffffu) : 0u;
    const unsigned hi = (__uint_as_float(yw[q] & 0xffff0000u) > 0.f) ? (gw[q] & 0xffff0000u) : 0u;
    o[q] = lo | hi;
  }
  st16(gpre + (size_t)t * 8, make_uint4(o[0], o[1], o[2], o[3]));
}

// Average pooling 2^3 (out dims d = input dims / 2), 8 channels a thread.
__global__ void k_pool(const bf16* __restrict__ in, bf16* __restrict__ out,
                       Dims d, int C) {
  const unsigned G = (unsigned)C / 8;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned long long)d.V * G) return;
  const unsigned v = t / G, g = t % G;
  int x, y, z;
  voxel_xyz(v, d, x, y, z);
  const unsigned W2 = 2 * d.W, H2 = 2 * d.H;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e) {
        float f[8];
        unpack8(ld16(in + ((size_t)((2 * z + a) * H2 + 2 * y + b) * W2 + 2 * x + e) * C + 8 * g), f);
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] = s[q] + f[q];
      }
  unsigned w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w[q] = (unsigned)f2bf(s[2 * q] * 0.125f) | ((unsigned)f2bf(s[2 * q + 1] * 0.125f) << 16);
  st16(out + (size_t)v * C + 8 * g, make_uint4(w[0], w[1], w[2], w[3]));
}

// Gradient through pooling added to an existing fine gradient:
// gfine[child] = gfine[child] + gcoarse[parent] / 8 (fine dims d), 8
// channels a thread.
__global__ void k_pool_bwd_add(const bf16* __restrict__ gc, bf16* __restrict__ gf,
                               Dims d, int C) {
  const unsigned G = (unsigned)C / 8;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned long long)d.V * G) return;
  const unsigned v = t / G, g = t % G;
  int x, y, z;
  voxel_xyz(v, d, x, y, z);
  const unsigned p = ((unsigned)(z / 2) * (d.H / 2) + y / 2) * (d.W / 2) + x / 2;
  float a[8], b[8];
  unpack8(ld16(gf + (size_t)v * C + 8 * g), a);
  unpack8(ld16(gc + (size_t)p * C + 8 * g), b);
  unsigned w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w[q] = (unsigned)f2bf(a[2 * q] + b[2 * q] * 0.125f) |
           ((unsigned)f2bf(a[2 * q + 1] + b[2 * q + 1] * 0.125f) << 16);
  st16(gf + (size_t)v * C + 8 * g, make_uint4(w[0], w[1], w[2], w[3]));
}

// Concatenation [up(coarse) (Cu channels), skip (Cs)] at fine dims d, 8
// channels a thread.
__global__ void k_up_cat(const bf16* __restrict__ coarse, int Cu,
                         const bf16* __restrict__ skip, int Cs,
                         bf16* __restrict__ out, Dims d) {
  const unsigned C = Cu + Cs, G = C / 8, Gu = (unsigned)Cu / 8;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned long long)d.V * G) return;
  const unsigned v = t / G, g = t % G;
  uint4 val;
  if (g < Gu) {
    int x, y, z;
    voxel_xyz(v, d, x, y, z);
    const unsigned p = ((unsigned)(z / 2) * (d.H / 2) + y / 2) * (d.W / 2) + x / 2;
    val = ld16(coarse + (size_t)p * Cu + 8 * g);
  } else {
    val = ld16(skip + (size_t)v * Cs + 8 * (g - Gu));
  }
  st16(out + (size_t)v * C + 8 * g, val);
}

// Split the concatenation's gradient: coarse part summed over the 8
// children (coarse dims dc), skip part copied (fine dims); 8 channels a
// thread.
__global__ void k_split_up(const bf16* __restrict__ gcat, int Cu, int Cs,
                           bf16* __restrict__ gcoarse, Dims dc) {
  const unsigned G = (unsigned)Cu / 8;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned long long)dc.V * G) return;
  const unsigned p = t / G, g = t % G;
  int x, y, z;
  voxel_xyz(p, dc, x, y, z);
  const unsigned W2 = 2 * dc.W, H2 = 2 * dc.H, C = Cu + Cs;
  float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int e = 0; e < 2; ++e) {
        float f[8];
        unpack8(ld16(gcat + ((size_t)((2 * z + a) * H2 + 2 * y + b) * W2 + 2 * x + e) * C + 8 * g), f);
#pragma unroll
        for (int q = 0; q < 8; ++q) s[q] = s[q] + f[q];
      }
  unsigned w[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    w[q] = (unsigned)f2bf(s[2 * q]) | ((unsigned)f2bf(s[2 * q + 1]) << 16);
  st16(gcoarse + (size_t)p * Cu + 8 * g, make_uint4(w[0], w[1], w[2], w[3]));
}
__global__ void k_split_skip(const bf16* __restrict__ gcat, int Cu, int Cs,
                             bf16* __restrict__ gskip, Dims d) {
  const unsigned G = (unsigned)Cs / 8;
  const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (unsigned long long)d.V * G) return;
  const unsigned v = t / G, g = t % G;
  st16(gskip + (size_t)v * Cs + 8 * g, ld16(gcat + (size_t)v * (Cu + Cs) + Cu + 8 * g));
}

// Head: out[v] = sum_c w[c] y[v][c] + b, FP32 output.
__global__ void k_head(const bf16* __restrict__ y, const float* __restrict__ w,
                       float* __restrict__ out, long long V) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (unsigned long long)V) return;
  float f[16];
  unpack8(ld16(y + (size_t)v * 16), f);
  unpack8(ld16(y + (size_t)v * 16 + 8), f + 8);
  float s = w[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) s = s + w[c] * f[c];
  out[v] = s;
}

// Loss (mean squared error) partials and the output gradient.
__global__ void k_mse(const float* __restrict__ out, const float* __restrict__ t,
                      float* __restrict__ gout, long long V,
                      double* __restrict__ part) {
  __shared__ double s[256];
  double a = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < V;
       v += (long long)gridDim.x * blockDim.x) {
    const float df = out[v] - t[v];
    a += (double)df * df;
    gout[v] = 2.0f * df / (float)V;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// Residual loss: q = A e on the unknown planes (z >= k0), e = c - t there
// and zero below k0 and beyond the top plane; A is the scaled 7-point
// operator (x, y periodic; a Neumann bottom, k0 = 0, mirrors plane 1).
// Block partials of sum q^2.
__device__ __forceinline__ float res_e(const float* c, const float* t, int z,
                                       unsigned row, int k0, int D) {
  return (z >= k0 && z < D) ? c[row] - t[row] : 0.0f;
}

__global__ void k_res_q(const float* __restrict__ c, const float* __restrict__ t,
                        float* __restrict__ q, Dims d, int k0,
                        double* __restrict__ part) {
  __shared__ double s[256];
  double a = 0.0;
  const unsigned plane = (unsigned)d.H * d.W;
  for (unsigned long long vv = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
       vv < (unsigned long long)d.V; vv += (unsigned long long)gridDim.x * blockDim.x) {
    const unsigned v = (unsigned)vv;
    int x, y, z;
    voxel_xyz(v, d, x, y, z);
    float r = 0.0f;
    if (z >= k0) {
      const unsigned base = (unsigned)z * plane;
      const int xm = x ? x - 1 : d.W - 1, xp = x + 1 < d.W ? x + 1 : 0;
      const int ym = y ? y - 1 : d.H - 1, yp = y + 1 < d.H ? y + 1 : 0;
      const float e0 = c[v] - t[v];
      float xy = res_e(c, t, z, base + y * d.W + xm, k0, d.D) +
                 res_e(c, t, z, base + y * d.W + xp, k0, d.D);
      xy = xy + (res_e(c, t, z, base + ym * d.W + x, k0, d.D) +
                 res_e(c, t, z, base + yp * d.W + x, k0, d.D));
      float zz;
      if (z == 0)
        zz = 2.0f * res_e(c, t, 1, v + plane, k0, d.D);
      else
        zz = res_e(c, t, z - 1, v - plane, k0, d.D) +
             res_e(c, t, z + 1, v + plane, k0, d.D);
      r = 6.0f * e0 - xy - zz;
    }
    q[v] = r;
    a += (double)r * r;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// gout = (2 / V) A^T q on the unknown planes (row z-1 = 0 of a Neumann
// bottom reaches plane 1 with coefficient 2).
__global__ void k_res_g(const float* __restrict__ q, float* __restrict__ gout,
                        Dims d, int k0, float scale) {
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= (unsigned long long)d.V) return;
  int x, y, z;
  voxel_xyz(v, d, x, y, z);
  float g = 0.0f;
  if (z >= k0) {
    const unsigned plane = (unsigned)d.H * d.W, base = (unsigned)z * plane;
    const int xm = x ? x - 1 : d.W - 1, xp = x + 1 < d.W ? x + 1 : 0;
    const int ym = y ? y - 1 : d.H - 1, yp = y + 1 < d.H ? y + 1 : 0;
    float xy = q[base + y * d.W + xm] + q[base + y * d.W + xp];
    xy = xy + (q[base + ym * d.W + x] + q[base + yp * d.W + x]);
    float zz = 0.0f;
    if (z - 1 >= k0) zz = (z - 1 == 0 ? 2.0f : 1.0f) * q[v - plane];
    if (z + 1 < d.D) zz = zz + q[v + plane];
    g = (6.0f * q[v] - xy - zz) * scale;
  }
  gout[v] = g;
}

// Head backward: gy[v][c] = gout[v] w[c]; dw[c] += sum gout y; db += sum.
__global__ void __launch_bounds__(256) k_head_bwd(
    const float* __restrict__ gout, const bf16* __restrict__ y,
    const float* __restrict__ w, bf16* __restrict__ gy, float* __restrict__ dw,
    long long V) {
  __shared__ float s[17][256];
  float acc[17];
#pragma unroll
  for (int c = 0; c < 17; ++c) acc[c] = 0.f;
  for (unsigned long long v = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x;
       v < (unsigned long long)V; v += (unsigned long long)gridDim.x * blockDim.x) {
    const float go = gout[v];
    float f[16];
    unpack8(ld16(y + (size_t)v * 16), f);
    unpack8(ld16(y + (size_t)v * 16 + 8), f + 8);
    unsigned o[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      o[q] = (unsigned)f2bf(go * w[2 * q]) | ((unsigned)f2bf(go * w[2 * q + 1]) << 16);
    st16(gy + (size_t)v * 16, make_uint4(o[0], o[1], o[2], o[3]));
    st16(gy + (size_t)v * 16 + 8, make_uint4(o[4], o[5], o[6], o[7]));
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = acc[c] + go * f[c];
    acc[16] = acc[16] + go;
  }
#pragma unroll
  for (int c = 0; c < 17; ++c) s[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int c = 0; c < 17; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 17) atomicAdd(&dw[threadIdx.x], s[threadIdx.x][0]);
}

__global__ void k_sum_d(const double* __restrict__ part, int n, double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// Adam with FP32 master weights (Kingma & Ba): bias-corrected moments.
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m,
                       float* __restrict__ v, const float* __restrict__ g,
                       long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 copies of a layer's weights: forward Wk[co][k = tap*ci_n + ci] and
// backward-data Wd[ci][k' = tap'*co_n + co] = W[co][26 - tap'][ci].
__global__ void k_pack_w(const float* __restrict__ W, int ci_n, int co_n,
                         bf16* __restrict__ Wk, int kpf, bf16* __restrict__ Wd,
                         int kpd) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long n = (long long)co_n * 27 * ci_n;
  if (i >= n) return;
  const int co = (int)(i / (27 * ci_n));
  const int r = (int)(i % (27 * ci_n));
  const int tap = r / ci_n, ci = r % ci_n;
  const bf16 h = f2bf(W[i]);
  Wk[(long long)co * kpf + tap * ci_n + ci] = h;
  if (Wd) Wd[(long long)ci * kpd + (26 - tap) * co_n + co] = h;
}

__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b,
                             long long n) {
  const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

}  // namespace
}  // namespace pic

// ============================================================================
// Host side.
// ============================================================================
namespace {

using pic::bf16;
using pic::Dims;

struct LayerSpec {
  int ci, co;
};
constexpr int kNL = 14;
constexpr LayerSpec kLayers[kNL] = {
    {2, 16},   {16, 16},  {16, 32}, {32, 32}, {32, 64},  {64, 64},  {64, 128},
    {128, 128}, {192, 64}, {64, 64}, {96, 32}, {32, 32},  {48, 16},  {16, 16}};
enum { E0A, E0B, E1A, E1B, E2A, E2B, BA, BB, D2A, D2B, D1A, D1B, D0A, D0B };
// Level of each layer's voxels.
constexpr int kLevel[kNL] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0};

long long param_count() {
  long long n = 0;
  for (int l = 0; l < kNL; ++l) n += (long long)kLayers[l].co * 27 * kLayers[l].ci + kLayers[l].co;
  return n + 17;
}

constexpr int kpad(int cin) { return (27 * cin + 63) / 64 * 64; }

}  // namespace

struct pic_unet {
  hipStream_t stream;
  int D, H, W;                 // maximum grid
  char* ws;
  size_t bytes;
  long long np;                // parameters
  float *p, *m, *v, *g;        // master, moments, gradient
  long long woff[kNL], boff[kNL], hoff;
  bf16 *wk[kNL], *wd[kNL];     // BF16 forward / backward-data weights
  // Activations (BF16, channels-last).
  float* x_in;                 // (V0, 2) FP32 input
  bf16 *y[kNL];                // layer outputs
  bf16 *p0, *p1, *p2;          // pooled
  bf16 *c2, *c1, *c0;          // concatenations
  float *out, *gout, *target;
  // Gradient scratch per level (two buffers of the level's widest tensor)
  // and a pre-activation buffer.
  bf16 *ga[4], *gb[4], *gp[4], *gs[4];
  float* dscratch;             // double partials (as float storage)
  double* dpart;
  int t;                       // Adam step
  int loss_mode, loss_k0;      // PIC_UNET_LOSS_*, first unknown plane
  float* q;                    // residual of the error (residual loss)
  std::string err;
};

namespace {

struct Carve {
  char* base;
  size_t off;
  template <typename T>
  T* take(long long n) {
    off = (off + 255) / 256 * 256;
    T* r = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (size_t)(n > 0 ? n : 1) * sizeof(T);
    return r;
  }
};

size_t unet_carve(pic_unet* u, char* base) {
  Carve cv{base, 0};
  const long long V0 = (long long)u->D * u->H * u->W;
  long long Vl[4];
  for (int l = 0; l < 4; ++l) Vl[l] = V0 >> (3 * l);
  u->np = param_count();
  u->p = cv.take<float>(u->np);
  u->m = cv.take<float>(u->np);
  u->v = cv.take<float>(u->np);
  u->g = cv.take<float>(u->np);
  long long off = 0;
  for (int l = 0; l < kNL; ++l) {
    u->woff[l] = off;
    off += (long long)kLayers[l].co * 27 * kLayers[l].ci;
    u->boff[l] = off;
    off += kLayers[l].co;
    u->wk[l] = cv.take<bf16>((long long)kLayers[l].co * kpad(kLayers[l].ci));
    u->wd[l] = cv.take<bf16>((long long)kLayers[l].ci * kpad(kLayers[l].co));
  }
  u->hoff = off;
  u->x_in = cv.take<float>(2 * V0);
  for (int l = 0; l < kNL; ++l) u->y[l] = cv.take<bf16>(Vl[kLevel[l]] * kLayers[l].co);
  u->p0 = cv.take<bf16>(Vl[1] * 16);
  u->p1 = cv.take<bf16>(Vl[2] * 32);
  u->p2 = cv.take<bf16>(Vl[3] * 64);
  u->c2 = cv.take<bf16>(Vl[2] * 192);
  u->c1 = cv.take<bf16>(Vl[1] * 96);
  u->c0 = cv.take<bf16>(Vl[0] * 48);
  u->out = cv.take<float>(V0);
  u->gout = cv.take<float>(V0);
  u->target = cv.take<float>(V0);
  const int widest[4] = {48, 96, 192, 128};
  for (int l = 0; l < 4; ++l) {
    u->ga[l] = cv.take<bf16>(Vl[l] * widest[l]);
    u->gb[l] = cv.take<bf16>(Vl[l] * widest[l]);
    u->gp[l] = cv.take<bf16>(Vl[l] * widest[l]);
    u->gs[l] = cv.take<bf16>(Vl[l] * widest[l]);
  }
  u->dpart = cv.take<double>(1024);
  u->q = cv.take<float>(V0);
  return cv.off + 256;
}

inline unsigned nb(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

Dims dims_at(const pic_unet* u, int D, int H, int W, int level) {
  Dims d;
  d.D = D >> level;
  d.H = H >> level;
  d.W = W >> level;
  d.V = (long long)d.D * d.H * d.W;
  return d;
}

// Workgroups of k_conv3p<CIN, CU> the current device holds at once.
template <int CIN, int CU>
unsigned conv3p_slots() {
  static unsigned cached[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  if (!cached[dev]) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, pic::k_conv3p<CIN, CU>, 256, 0) !=
            hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    cached[dev] = (unsigned)(per_cu * cus);
  }
  return cached[dev];
}

template <int CIN, int CU>
void conv3p_launch(hipStream_t st, const bf16* in, const bf16* skip, const bf16* Wk,
                   const float* b, bf16* out, Dims d, int relu) {
  const long long ntiles = (long long)((d.W + 15) / 16) * ((d.H + 7) / 8) * ((d.D + 7) / 8);
  const unsigned slots = conv3p_slots<CIN, CU>();
  const unsigned grid = ntiles < (long long)slots ? (unsigned)ntiles : slots;
  pic::k_conv3p<CIN, CU><<<grid, 256, 0, st>>>(in, skip, Wk, b, out, d, relu);
}

// Tile of k_conv3t for a column count: MT * COUT / 16 <= 16; the
// register-blocked k_conv3r for 32 to 128 output channels, its persistent
// form k_conv3p for 16.
template <int CIN, int COUT>
void conv_launch(hipStream_t st, const bf16* in, const bf16* Wk, const float* b,
                 bf16* out, Dims d, int relu) {
  if constexpr (COUT == 16) {
    conv3p_launch<CIN, 0>(st, in, nullptr, Wk, b, out, d, relu);
  } else if constexpr (COUT == 32 || COUT == 64 || COUT == 128) {
    constexpr int WY = COUT == 16 ? 2 : 1, WZ = COUT >= 64 ? 1 : 2;
    constexpr int TY = 4 * WY, TZ = 4 * WZ;
    const long long nbk = (long long)((d.W + 15) / 16) * ((d.H + TY - 1) / TY) *
                          ((d.D + TZ - 1) / TZ);
    pic::k_conv3r<CIN, COUT, WY, WZ><<<(unsigned)nbk, 64 * (COUT / 16) * WY * WZ, 0, st>>>(
        in, nullptr, Wk, b, out, d, relu);
  } else {
    constexpr int NT = COUT / 16;
    constexpr int TY = NT <= 2 ? 8 : (NT <= 8 ? 4 : 2);
    constexpr int TZ = NT <= 4 ? 4 : 2;
    const long long nbk = (long long)((d.W + 15) / 16) * ((d.H + TY - 1) / TY) *
                          ((d.D + TZ - 1) / TZ);
    pic::k_conv3t<CIN, COUT, TY, TZ><<<(unsigned)nbk, 256, 0, st>>>(in, Wk, b, out, d, relu);
  }
}

// Dispatch of the (C_in, C_out) pairs the network and its backward use.
bool conv(hipStream_t st, int cin, int cout, const bf16* in, const bf16* Wk,
          const float* b, bf16* out, Dims d, int relu) {
#define PIC_CONV(CI, CO)                                                   \
  if (cin == CI && cout == CO) {                                           \
    conv_launch<CI, CO>(st, in, Wk, b, out, d, relu);                      \
    return true;                                                           \
  }
  PIC_CONV(16, 16) PIC_CONV(16, 32) PIC_CONV(32, 32) PIC_CONV(32, 64)
  PIC_CONV(64, 64) PIC_CONV(64, 128) PIC_CONV(128, 128) PIC_CONV(192, 64)
  PIC_CONV(96, 32) PIC_CONV(48, 16)
  // backward-data shapes (channels swapped)
  PIC_CONV(32, 16) PIC_CONV(64, 32) PIC_CONV(128, 64) PIC_CONV(64, 192)
  PIC_CONV(32, 96) PIC_CONV(16, 48)
#undef PIC_CONV
  return false;
}

// Decoder convolution of [up(coarse) (CU channels), skip] without the
// concatenated tensor (inference).
template <int CIN, int COUT, int CU>
void conv_upcat_launch(hipStream_t st, const bf16* coarse, const bf16* skip,
                       const bf16* Wk, const float* b, bf16* out, Dims d) {
  if constexpr (COUT == 16) {
    conv3p_launch<CIN, CU>(st, coarse, skip, Wk, b, out, d, 1);
    return;
  }
  constexpr int WY = COUT == 16 ? 2 : 1, WZ = COUT == 64 ? 1 : 2;
  constexpr int TY = 4 * WY, TZ = 4 * WZ;
  const long long nbk = (long long)((d.W + 15) / 16) * ((d.H + TY - 1) / TY) *
                        ((d.D + TZ - 1) / TZ);
  pic::k_conv3r<CIN, COUT, WY, WZ, CU><<<(unsigned)nbk, 64 * (COUT / 16) * WY * WZ, 0, st>>>(
      coarse, skip, Wk, b, out, d, 1);
}

template <int CIN, int COUT>
void wgrad_launch(hipStream_t st, const bf16* x, const bf16* g, float* dW,
                  Dims d) {
  long long chunk = d.V / 256;
  if (chunk < 2048) chunk = 2048;
  chunk = (chunk + 31) / 32 * 32;
  dim3 grid(kpad(CIN) / 64, (unsigned)((d.V + chunk - 1) / chunk));
  pic::k_wgrad3<CIN, COUT><<<grid, 256, 0, st>>>(x, g, dW, d, chunk);
}

bool wgrad(hipStream_t st, int cin, int cout, const bf16* x, const bf16* g,
           float* dW, Dims d) {
#define PIC_WG(CI, CO)                                                     \
  if (cin == CI && cout == CO) {                                           \
    wgrad_launch<CI, CO>(st, x, g, dW, d);                                 \
    return true;                                                           \
  }
  PIC_WG(16, 16) PIC_WG(16, 32) PIC_WG(32, 32) PIC_WG(32, 64) PIC_WG(64, 64)
  PIC_WG(64, 128) PIC_WG(128, 128) PIC_WG(192, 64) PIC_WG(96, 32)
  PIC_WG(48, 16)
#undef PIC_WG
  return false;
}

void pack_weights(pic_unet* u) {
  for (int l = 0; l < kNL; ++l) {
    const LayerSpec& s = kLayers[l];
    if (l == E0A) continue;  // FP32 first layer
    pic::k_pack_w<<<nb((long long)s.co * 27 * s.ci), 256, 0, u->stream>>>(
        u->p + u->woff[l], s.ci, s.co, u->wk[l], kpad(s.ci), u->wd[l],
        kpad(s.co));
  }
}

// Forward pass of a D x H x W grid (input already in x_in); out -> u->out.
// keep: write the decoder's concatenations (the backward pass reads them);
// without it the decoders form them in their staging.
bool unet_forward(pic_unet* u, int D, int H, int W, bool keep = true) {
  hipStream_t st = u->stream;
  Dims d0 = dims_at(u, D, H, W, 0), d1 = dims_at(u, D, H, W, 1),
       d2 = dims_at(u, D, H, W, 2), d3 = dims_at(u, D, H, W, 3);
  const float* P = u->p;
  pic::k_conv_first<<<nb(d0.V), 256, 0, st>>>(u->x_in, P + u->woff[E0A],
                                             P + u->boff[E0A], u->y[E0A], d0);
  bool ok = true;
  auto L = [&](int l, const bf16* in, Dims d) {
    ok = ok && conv(st, kLayers[l].ci, kLayers[l].co, in, u->wk[l],
                    P + u->boff[l], u->y[l], d, 1);
  };
  L(E0B, u->y[E0A], d0);
  pic::k_pool<<<nb(d1.V * 2), 256, 0, st>>>(u->y[E0B], u->p0, d1, 16);
  L(E1A, u->p0, d1);
  L(E1B, u->y[E1A], d1);
  pic::k_pool<<<nb(d2.V * 4), 256, 0, st>>>(u->y[E1B], u->p1, d2, 32);
  L(E2A, u->p1, d2);
  L(E2B, u->y[E2A], d2);
  pic::k_pool<<<nb(d3.V * 8), 256, 0, st>>>(u->y[E2B], u->p2, d3, 64);
  L(BA, u->p2, d3);
  L(BB, u->y[BA], d3);
  if (keep) {
    pic::k_up_cat<<<nb(d2.V * 24), 256, 0, st>>>(u->y[BB], 128, u->y[E2B], 64, u->c2, d2);
    L(D2A, u->c2, d2);
  } else {
    conv_upcat_launch<192, 64, 128>(st, u->y[BB], u->y[E2B], u->wk[D2A], P + u->boff[D2A],
                                    u->y[D2A], d2);
  }
  L(D2B, u->y[D2A], d2);
  if (keep) {
    pic::k_up_cat<<<nb(d1.V * 12), 256, 0, st>>>(u->y[D2B], 64, u->y[E1B], 32, u->c1, d1);
    L(D1A, u->c1, d1);
  } else {
    conv_upcat_launch<96, 32, 64>(st, u->y[D2B], u->y[E1B], u->wk[D1A], P + u->boff[D1A],
                                  u->y[D1A], d1);
  }
  L(D1B, u->y[D1A], d1);
  if (keep) {
    pic::k_up_cat<<<nb(d0.V * 6), 256, 0, st>>>(u->y[D1B], 32, u->y[E0B], 16, u->c0, d0);
    L(D0A, u->c0, d0);
  } else {
    conv_upcat_launch<48, 16, 32>(st, u->y[D1B], u->y[E0B], u->wk[D0A], P + u->boff[D0A],
                                  u->y[D0A], d0);
  }
  L(D0B, u->y[D0A], d0);
  pic::k_head<<<nb(d0.V), 256, 0, st>>>(u->y[D0B], P + u->hoff, u->out, d0.V);
  return ok;
}

// Backward pass from u->gout into u->g (zeroed here).
bool unet_backward(pic_unet* u, int D, int H, int W) {
  hipStream_t st = u->stream;
  Dims d[4];
  for (int l = 0; l < 4; ++l) d[l] = dims_at(u, D, H, W, l);
  hipMemsetAsync(u->g, 0, u->np * sizeof(float), st);
  float* G = u->g;
  bool ok = true;
  // Head.
  pic::k_head_bwd<<<512, 256, 0, st>>>(u->gout, u->y[D0B], u->p + u->hoff,
                                       u->ga[0], G + u->hoff, d[0].V);
  // Layer backward: gy (post-activation gradient) -> gpre -> dW, db and
  // (if gx) the input gradient.
  auto back = [&](int l, const bf16* gy, const bf16* in, bf16* gpre, bf16* gx) {
    const LayerSpec& s = kLayers[l];
    const Dims& dd = d[kLevel[l]];
    pic::k_relu_bwd<<<nb(dd.V * s.co / 8), 256, 0, st>>>(gy, u->y[l], gpre, dd.V * s.co);
    ok = ok && wgrad(st, s.ci, s.co, in, gpre, G + u->woff[l], dd);
    pic::k_bias_grad<<<256, 256, 0, st>>>(gpre, s.co, dd, G + u->boff[l]);
    if (gx) ok = ok && conv(st, s.co, s.ci, gpre, u->wd[l], nullptr, gx, dd, 0);
  };
  // Level 0 decoder.
  back(D0B, u->ga[0], u->y[D0A], u->gp[0], u->gb[0]);
  back(D0A, u->gb[0], u->c0, u->gp[0], u->ga[0]);        // ga0: grad of c0 (48)
  pic::k_split_skip<<<nb(d[0].V * 2), 256, 0, st>>>(u->ga[0], 32, 16, u->gs[0], d[0]);
  pic::k_split_up<<<nb(d[1].V * 4), 256, 0, st>>>(u->ga[0], 32, 16, u->ga[1], d[1]);
  // Level 1 decoder.
  back(D1B, u->ga[1], u->y[D1A], u->gp[1], u->gb[1]);
  back(D1A, u->gb[1], u->c1, u->gp[1], u->ga[1]);        // grad of c1 (96)
  pic::k_split_skip<<<nb(d[1].V * 4), 256, 0, st>>>(u->ga[1], 64, 32, u->gs[1], d[1]);
  pic::k_split_up<<<nb(d[2].V * 8), 256, 0, st>>>(u->ga[1], 64, 32, u->ga[2], d[2]);
  // Level 2 decoder.
  back(D2B, u->ga[2], u->y[D2A], u->gp[2], u->gb[2]);
  back(D2A, u->gb[2], u->c2, u->gp[2], u->ga[2]);        // grad of c2 (192)
  pic::k_split_skip<<<nb(d[2].V * 8), 256, 0, st>>>(u->ga[2], 128, 64, u->gs[2], d[2]);
  pic::k_split_up<<<nb(d[3].V * 16), 256, 0, st>>>(u->ga[2], 128, 64, u->ga[3], d[3]);
  // Bottom.
  back(BB, u->ga[3], u->y[BA], u->gp[3], u->gb[3]);
  back(BA, u->gb[3], u->p2, u->gp[3], u->ga[3]);         // grad of p2 (64)
  // Encoder level 2: skip gradient + pooled gradient.
  pic::k_pool_bwd_add<<<nb(d[2].V * 8), 256, 0, st>>>(u->ga[3], u->gs[2], d[2], 64);
  back(E2B, u->gs[2], u->y[E2A], u->gp[2], u->gb[2]);
  back(E2A, u->gb[2], u->p1, u->gp[2], u->ga[2]);        // grad of p1 (32)
  pic::k_pool_bwd_add<<<nb(d[1].V * 4), 256, 0, st>>>(u->ga[2], u->gs[1], d[1], 32);
  back(E1B, u->gs[1], u->y[E1A], u->gp[1], u->gb[1]);
  back(E1A, u->gb[1], u->p0, u->gp[1], u->ga[1]);        // grad of p0 (16)
  pic::k_pool_bwd_add<<<nb(d[0].V * 2), 256, 0, st>>>(u->ga[1], u->gs[0], d[0], 16);
  back(E0B, u->gs[0], u->y[E0A], u->gp[0], u->gb[0]);    // grad of e0a (16)
  // First layer: weights only.
  pic::k_relu_bwd<<<nb(d[0].V * 2), 256, 0, st>>>(u->gb[0], u->y[E0A], u->gp[0], d[0].V * 16);
  const unsigned chunk = 8192;
  pic::k_wgrad_first<<<dim3((unsigned)((d[0].V + chunk - 1) / chunk), 27), 256, 0, st>>>(
      u->x_in, u->gp[0], G + u->woff[E0A], d[0], chunk);
  pic::k_bias_grad<<<256, 256, 0, st>>>(u->gp[0], 16, d[0], G + u->boff[E0A]);
  return ok;
}

pic_status unet_check(pic_unet* u, int D, int H, int W) {
  if (!u) return PIC_ERR_ARG;
  if (D < 8 || H < 8 || W < 8 || (D & 7) || (H & 7) || (W & 7) || D > u->D ||
      H > u->H || W > u->W || (long long)D * H * W > (long long)u->D * u->H * u->W)
    return PIC_ERR_ARG;
  return PIC_OK;
}

}  // namespace

bool pic_unet_fits(const pic_unet* u, int D, int H, int W) {
  return unet_check(const_cast<pic_unet*>(u), D, H, W) == PIC_OK;
}

// Inference for the solve's warm start: the network reads x in place and
// runs on the solver's stream.
bool pic_unet_infer(pic_unet* u, const float* x, int D, int H, int W,
                    hipStream_t st, const float** out) {
  if (unet_check(u, D, H, W) != PIC_OK) return false;
  float* keep_x = u->x_in;
  hipStream_t keep_st = u->stream;
  u->x_in = const_cast<float*>(x);
  u->stream = st;
  const bool ok = unet_forward(u, D, H, W, false);
  u->x_in = keep_x;
  u->stream = keep_st;
  *out = u->out;
  return ok;
}

extern "C" {

int64_t pic_unet_param_count(void) { return param_count(); }

pic_status pic_unet_workspace_bytes(int32_t D, int32_t H, int32_t W,
                                    size_t* bytes) {
  if (!bytes || D < 8 || H < 8 || W < 8 || (D & 7) || (H & 7) || (W & 7))
    return PIC_ERR_ARG;
  pic_unet u;
  u.D = D; u.H = H; u.W = W;
  *bytes = unet_carve(&u, nullptr);
  return PIC_OK;
}

pic_status pic_unet_init(int32_t D, int32_t H, int32_t W, void* ws,
                         size_t bytes, void* stream, pic_unet** out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  size_t need = 0;
  if (pic_unet_workspace_bytes(D, H, W, &need) != PIC_OK || !ws || bytes < need)
    return PIC_ERR_ARG;
  pic_unet* u = new (std::nothrow) pic_unet();
  if (!u) return PIC_ERR_STATE;
  u->D = D; u->H = H; u->W = W;
  u->stream = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(ws) + 255) / 256 * 256);
  u->ws = reinterpret_cast<char*>(ws);
  u->bytes = bytes;
  unet_carve(u, base);
  u->t = 0;
  u->loss_mode = PIC_UNET_LOSS_MSE;
  u->loss_k0 = 1;
  if (hipMemsetAsync(ws, 0, bytes, u->stream) != hipSuccess ||
      hipStreamSynchronize(u->stream) != hipSuccess) {
    delete u;
    return PIC_ERR_HIP;
  }
  *out = u;
  return PIC_OK;
}

void pic_unet_destroy(pic_unet* u) { delete u; }

pic_status pic_unet_set_loss(pic_unet* u, int32_t mode, int32_t k0) {
  if (!u || (mode != PIC_UNET_LOSS_MSE && mode != PIC_UNET_LOSS_RESIDUAL) ||
      (k0 != 0 && k0 != 1))
    return PIC_ERR_ARG;
  u->loss_mode = mode;
  u->loss_k0 = k0;
  return PIC_OK;
}

const char* pic_unet_last_error(const pic_unet* u) {
  return u ? u->err.c_str() : "null U-Net";
}

pic_status pic_unet_set_params(pic_unet* u, const float* params) {
  if (!u || !params) return PIC_ERR_ARG;
  if (hipMemcpyAsync(u->p, params, u->np * sizeof(float), hipMemcpyDeviceToDevice,
                     u->stream) != hipSuccess)
    return PIC_ERR_HIP;
  hipMemsetAsync(u->m, 0, u->np * sizeof(float), u->stream);
  hipMemsetAsync(u->v, 0, u->np * sizeof(float), u->stream);
  u->t = 0;
  pack_weights(u);
  return hipStreamSynchronize(u->stream) == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

pic_status pic_unet_get_params(pic_unet* u, float* params) {
  if (!u || !params) return PIC_ERR_ARG;
  if (hipMemcpyAsync(params, u->p, u->np * sizeof(float), hipMemcpyDeviceToDevice,
                     u->stream) != hipSuccess ||
      hipStreamSynchronize(u->stream) != hipSuccess)
    return PIC_ERR_HIP;
  return PIC_OK;
}

pic_status pic_unet_forward(pic_unet* u, const float* input, int32_t D,
                            int32_t H, int32_t W, float* out) {
  const pic_status c = unet_check(u, D, H, W);
  if (c != PIC_OK) return c;
  if (!input || !out) return PIC_ERR_ARG;
  const long long V = (long long)D * H * W;
  hipMemcpyAsync(u->x_in, input, 2 * V * sizeof(float), hipMemcpyDeviceToDevice,
                 u->stream);
  if (!unet_forward(u, D, H, W, false)) return PIC_ERR_STATE;
  hipMemcpyAsync(out, u->out, V * sizeof(float), hipMemcpyDeviceToDevice, u->stream);
  return hipStreamSynchronize(u->stream) == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

// Loss and parameter gradient of one sample (no update).
pic_status pic_unet_gradients(pic_unet* u, const float* input,
                              const float* target, int32_t D, int32_t H,
                              int32_t W, float* grad, double* loss) {
  const pic_status c = unet_check(u, D, H, W);
  if (c != PIC_OK) return c;
  if (!input || !target) return PIC_ERR_ARG;
  const long long V = (long long)D * H * W;
  hipStream_t st = u->stream;
  hipMemcpyAsync(u->x_in, input, 2 * V * sizeof(float), hipMemcpyDeviceToDevice, st);
  hipMemcpyAsync(u->target, target, V * sizeof(float), hipMemcpyDeviceToDevice, st);
  if (!unet_forward(u, D, H, W)) return PIC_ERR_STATE;
  if (u->loss_mode == PIC_UNET_LOSS_RESIDUAL) {
    const Dims d0 = dims_at(u, D, H, W, 0);
    pic::k_res_q<<<256, 256, 0, st>>>(u->out, u->target, u->q, d0, u->loss_k0, u->dpart);
    pic::k_res_g<<<nb(V), 256, 0, st>>>(u->q, u->gout, d0, u->loss_k0, 2.0f / (float)V);
  } else {
    pic::k_mse<<<256, 256, 0, st>>>(u->out, u->target, u->gout, V, u->dpart);
  }
  pic::k_sum_d<<<1, 256, 0, st>>>(u->dpart, 256, u->dpart + 512);
  if (!unet_backward(u, D, H, W)) return PIC_ERR_STATE;
  if (grad)
    hipMemcpyAsync(grad, u->g, u->np * sizeof(float), hipMemcpyDeviceToDevice, st);
  double l = 0.0;
  hipMemcpyAsync(&l, u->dpart + 512, sizeof(double), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) return PIC_ERR_HIP;
  if (loss) *loss = l / (double)V;
  return PIC_OK;
}

// One Adam step on one sample; returns the sample's loss before the step.
pic_status pic_unet_train_step(pic_unet* u, const float* input,
                               const float* target, int32_t D, int32_t H,
                               int32_t W, float lr, float beta1, float beta2,
                               float eps, double* loss) {
  const pic_status s = pic_unet_gradients(u, input, target, D, H, W, nullptr, loss);
  if (s != PIC_OK) return s;
  u->t += 1;
  const float c1 = 1.f - powf(beta1, (float)u->t);
  const float c2 = 1.f - powf(beta2, (float)u->t);
  pic::k_adam<<<nb(u->np), 256, 0, u->stream>>>(u->p, u->m, u->v, u->g, u->np,
                                                 lr, beta1, beta2, eps, c1, c2);
  pack_weights(u);
  return hipStreamSynchronize(u->stream) == hipSuccess ? PIC_OK : PIC_ERR_HIP;
}

}  // extern "C"
