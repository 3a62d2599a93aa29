// Internal definitions shared by the HIP kernels and the host runtime of the
// MI355X compressor (arXiv 1706.03791, SZ-1.4): container layout, the
// device-resident plan that carries data-dependent values between kernels,
// and launch geometry.  Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/szhip.h"

namespace szh {


// ------------------------------------------------------------- container
// Byte layout (little endian), 192-byte header then 64-byte aligned sections:
//   0 u32 magic "SZH1"        4 u16 version      6 u16 flags (bit0 raw copy)
//   8 u8 dtype  9 u8 ndim  10 u8 layers  11 u8 m (bits per code in use)
//  12 u8 eb_mode  13 u8 m requested (0 adaptive)  14 u16 reserved
//  16 u64 dims[3]   40 u64 block[3]   64 f64 eb_abs   72 f64 eb_rel
//  80 u64 bit pattern of the element-type bound   88 u64 points
//  96 u64 unpredictable points  104 u64 Huffman bits  112 u64 tail bits
// 120 u32 symbols per chunk    124 u32 codebook entries  128 u64 chunks
// 136..176 u64 offsets: codebook, chunk table, bitstream, heads, tails, total
// Sections: codebook (u16 symbol, u8 length) sorted by symbol; chunk table
// (u32 bits per chunk); Huffman bitstream; heads (sign+exponent, 9 or 12
// bits each); tails (kept mantissa bits).  Bit streams are MSB-first in
// little-endian u32 words.
constexpr uint32_t kMagic = 0x31485A53u;
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHdr = 192;
constexpr uint32_t kAlign = 64;
constexpr uint32_t kDefaultChunk = 1024;
constexpr uint32_t kMaxChunk = 4096;
constexpr uint32_t kDefaultBlock1D = 2048;
constexpr int kLmax = 27;

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
  uint32_t max_len;
  uint64_t out_cap;
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

}  // namespace szh
