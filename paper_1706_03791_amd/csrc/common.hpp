// Internal definitions shared by the HIP kernels and the host runtime of the
// MI355X compressor (arXiv 1706.03791, SZ-1.4): container layout, the
// device-resident plan that carries data-dependent values between kernels,
// and launch geometry.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/szhip.h"
#include "container.hpp"

namespace szh {


// ------------------------------------------------------------- container
// The format and its constants are in container.hpp.

// Steps per synchronisation group in the wavefront sweep; also the element
// count of the aligned chunks staged through LDS rings.
constexpr int kG = 16;
constexpr int kRing = 32;

// ------------------------------------------------------------------ plan
// Device-resident values produced and consumed by the kernels of one call,
// so that a whole compression can be enqueued (and graph-captured) without
// host round trips.
struct DevPlan {
  int32_t status;        // first error seen by any kernel, 0 = ok
  uint32_t m;            // bits per code in use
  uint32_t rerun;        // adaptive m: second sweep required
  uint32_t m_suggested;
  uint64_t ebT_bits;     // element-type bit patterns of eb, 2eb, 1/(2eb)
  uint64_t twoeb_bits;
  uint64_t inv2eb_bits;
  double vmin, vmax, eb;
  uint32_t minmax_bits[4];  // ordered-integer min/max reduction scratch (f32: [0],[1]; f64: pairs)
  uint64_t minmax64[2];
  uint32_t nonfinite;
  uint32_t n_used;       // codebook entries
  uint64_t n_unpred, huff_bits, tail_bits;
  uint64_t off_cb, off_ch, off_bs, off_hd, off_tl, total;
  uint32_t raw;
  uint32_t xorc;         // unpredictable values XOR-coded (container flag bit 1)
  uint32_t max_len;
  uint64_t out_cap;
  uint32_t epoch;        // launches on this plan so far (kept across inits): tags exchange records
};

// --------------------------------------------------------------- geometry
// Fields are handled as padded 3-D arrays (Z, Y, X), X contiguous.  A "row"
// is one (z, y) line along X inside one independent block.
struct Geom {
  int64_t dims[3];
  int64_t blk[3];
  int32_t nblk[3];
  int32_t tz_per_blk, ty_per_blk;  // tiles per block (sweep kernels)
  int32_t ntiles;
  int32_t ndim;
  int64_t n;
};

// Tile claimed with a ticket of a single-field sweep.  Tickets are taken in
// a dependence order of the tiles, so every predecessor of a tile (the tiles
// before it along z and y in its block) holds a smaller ticket.  Order 0 is
// the tile numbering itself (blocks in order; z-tiles outer, y-tiles inner);
// order 1 numbers the tiles of a block y-tiles outer, another dependence
// order; order 2 also takes the blocks, which are independent, in reverse.
// All orders give the same bytes (the schedule-invariance check of the tests).
__device__ __forceinline__ int claim_tile(int ticket, uint32_t order, int tz_per_blk, int ty_per_blk, int ntiles) {
  if (order == 0) return ticket;
  const int per = tz_per_blk * ty_per_blk;
  int bi = ticket / per;
  const int q = ticket % per;
  if (order == 2) bi = ntiles / per - 1 - bi;
  const int tyt = q / tz_per_blk, tzt = q % tz_per_blk;
  return bi * per + tzt * ty_per_blk + tyt;
}

}  // namespace szh
