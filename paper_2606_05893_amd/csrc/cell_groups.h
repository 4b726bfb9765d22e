// Helpers shared by the passes that group particles by cell (Coulomb
// collisions, ion processes): the XCD-aware split of a range over the
// workgroups and the tile-major numbering of cells.
#pragma once

#include "pic_device.h"

namespace pic {

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

// Cells are numbered tile by tile (512 to a tile, x fastest inside), so that
// the cells of one tile, whose particles share one range of the tile-binned
// arrays, are served together.
__device__ __forceinline__ unsigned tile_major(unsigned c, const GridC& g) {
  const unsigned i = c % (unsigned)g.nx;
  const unsigned r = c / (unsigned)g.nx;
  const unsigned j = r % (unsigned)g.ny;
  const unsigned k = r / (unsigned)g.ny;
  const unsigned t = ((k / kTile) * (unsigned)g.tny + j / kTile) * (unsigned)g.tnx + i / kTile;
  return (t * kTile + k % kTile) * (kTile * kTile) + (j % kTile) * kTile + i % kTile;
}

// The cell (x fastest, then y, then z) of a tile-major number.
__device__ __forceinline__ unsigned cell_of_tile_major(unsigned key,
                                                       const GridC& g) {
  const unsigned t = key / (kTile * kTile * kTile);
  const unsigned w = key % (kTile * kTile * kTile);
  const unsigned ti = t % (unsigned)g.tnx;
  const unsigned tr = t / (unsigned)g.tnx;
  const unsigned tj = tr % (unsigned)g.tny;
  const unsigned tk = tr / (unsigned)g.tny;
  const unsigned i = ti * kTile + w % kTile;
  const unsigned j = tj * kTile + (w / kTile) % kTile;
  const unsigned k = tk * kTile + w / (kTile * kTile);
  return (k * (unsigned)g.ny + j) * (unsigned)g.nx + i;
}

// Per-chunk LDS tables that aggregate the records of a chunk by cell, so
// that a cell many records share (the atoms piled above an evaporating spot)
// takes one global atomic per chunk instead of one per record.  A key whose
// probes find no room goes to the global counter directly; either way the
// counts and reservations are exact.
constexpr int kGHash = 4096;
constexpr int kGChunk = 4096;
constexpr unsigned kGEmpty = 0xFFFFFFFFu;

// Slot of key in the table (inserted if absent), or -1 when its two probes
// find no room.  Keys are cell numbers below 2^30.  Two probes suffice for
// the keys that repeat within a chunk (they claim a slot early); scattered
// keys mostly go to the global counter, as they would without the table,
// and long probe chains would only slow them.
__device__ __forceinline__ int ghash_slot(unsigned* hk, unsigned key) {
  const unsigned h = (key * 2654435761u) >> 20;
#pragma unroll
  for (int probe = 0; probe < 2; ++probe) {
    const unsigned s = (h + probe) & (kGHash - 1);
    unsigned k = hk[s];
    if (k == kGEmpty) k = atomicCAS(&hk[s], kGEmpty, key);
    if (k == kGEmpty || k == key) return (int)s;
  }
  return -1;
}

// Index words of the grouping passes: a particle's position in the range of
// the grouped species taken one after another (electrons, then Cu+, then Cu
// atoms), read back with the species counts at grouping time, which the
// passes leave unchanged until their commits.
struct JointIx {
  unsigned n0, n1;                  // electrons, Cu+
  __device__ __forceinline__ unsigned sp(unsigned t) const {
    return t < n0 ? 0u : (t - n0 < n1 ? 1u : 2u);
  }
  __device__ __forceinline__ unsigned ix(unsigned t) const {
    return t < n0 ? t : (t - n0 < n1 ? t - n0 : t - n0 - n1);
  }
};

__device__ __forceinline__ JointIx joint_ix(const Counters* dc) {
  return JointIx{(unsigned)dc->n[0], (unsigned)dc->n[2]};
}

// Binning by plane: a plane is one z layer of a tile (8x8 cells, 64
// consecutive tile-major numbers).  Particles binned by tile fall into few
// planes per chunk, so a chunk's planes are counted in a small LDS table and
// each distinct plane takes one global atomic per chunk; a plane whose two
// probes find no room (the unbinned tail's chunks, with many planes) takes
// the global counter per particle.
constexpr int kPlaneShift = 6;
constexpr int kPlaneCells = 1 << kPlaneShift;
static_assert(kPlaneCells == kTile * kTile, "a plane is one z layer of a tile");
constexpr int kPHash = 256;
constexpr int kPChunk = 4096;

__device__ __forceinline__ unsigned plane_of(unsigned c, const GridC& g) {
  return tile_major(c, g) >> kPlaneShift;
}

// The planes a workgroup of a per-plane pass serves: plane xcd_block() +
// k * gridDim.x, k = 0, 1, ...  The arrays are binned by tile, not by
// plane, so a plane's particles are spread over its tile's range; with this
// order the eight planes of a tile are served at the same time by eight
// workgroups on one XCD, which share the tile's cache lines in its L2.
// (The grid is a multiple of 8.)
__device__ __forceinline__ long long plane_first() { return xcd_block(); }

// Slot of a plane in the chunk's table (inserted if absent), or -1.
__device__ __forceinline__ int plane_slot(unsigned* hk, unsigned key) {
  const unsigned h = (key * 2654435761u) >> 24;
#pragma unroll
  for (int probe = 0; probe < 2; ++probe) {
    const unsigned s = (h + probe) & (kPHash - 1);
    unsigned k = hk[s];
    if (k == kGEmpty) k = atomicCAS(&hk[s], kGEmpty, key);
    if (k == kGEmpty || k == key) return (int)s;
  }
  return -1;
}

}  // namespace pic
