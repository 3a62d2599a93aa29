// Container format of the compressor and its host-side validation.  This
// header is plain C++ (no HIP): the kernels take the constants from it, the
// host runtime parses and checks headers with it, and it builds on its own
// with a host compiler (the sanitizer build of the header checks does so).
//
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
// (u32 bits per chunk, then u16 bits of each chunk's first half of symbols,
// where a second decoder of the chunk starts); Huffman bitstream; heads (sign+exponent, 9 or 12
// bits each); tails (kept mantissa bits).  Bit streams are MSB-first in
// little-endian u32 words.  A raw container (flag bit 0) is the header
// followed by the field itself.  With flag bit 1 the unpredictable values
// are XOR-coded: the heads section holds one u32 per chunk (the bits of the
// chunk's records) and the tails section the records.
#pragma once

#include <stdint.h>
#include <string.h>

#include "../../include/szhip.h"

namespace szh {

constexpr uint32_t kMagic = 0x31485A53u;
constexpr uint32_t kVersion = 2;
constexpr uint32_t kHdr = 192;
constexpr uint32_t kAlign = 64;
constexpr uint32_t kDefaultChunk = 1024;
constexpr uint32_t kMaxChunk = 4096;
constexpr uint32_t kDefaultBlock1D = 2048;
constexpr int kLmax = 27;

struct Hdr {
  uint32_t flags, dtype, ndim, layers, m, eb_mode, m_req;
  uint64_t dims[3], block[3];
  double eb_abs, eb_rel;
  uint64_t ebT_bits, n, n_unpred, huff_bits, tail_bits;
  uint32_t chunk, n_used;
  uint64_t n_chunks, off_cb, off_ch, off_bs, off_hd, off_tl, total;
};

inline uint64_t hdr_u64(const uint8_t* b) {
  uint64_t v = 0;
  for (int i = 7; i >= 0; i--) v = (v << 8) | b[i];
  return v;
}
inline uint32_t hdr_u32(const uint8_t* b) {
  return (uint32_t)b[0] | ((uint32_t)b[1] << 8) | ((uint32_t)b[2] << 16) | ((uint32_t)b[3] << 24);
}
inline uint64_t hdr_align64(uint64_t v) { return (v + (kAlign - 1)) & ~(uint64_t)(kAlign - 1); }

// Decode the header fields of a container whose first `size` bytes are at b.
// With check_total the stored total must fit in `size`.  Field values are
// checked by check_sections.
inline int parse_header(const uint8_t* b, size_t size, Hdr& h, bool check_total = true) {
  if (!b || size < kHdr) return SZ_ECORRUPT;
  if (hdr_u32(b) != kMagic || (uint32_t)(b[4] | (b[5] << 8)) != kVersion) return SZ_ECORRUPT;
  h.flags = (uint32_t)(b[6] | (b[7] << 8));
  h.dtype = b[8];
  h.ndim = b[9];
  h.layers = b[10];
  h.m = b[11];
  h.eb_mode = b[12];
  h.m_req = b[13];
  for (int d = 0; d < 3; d++) h.dims[d] = hdr_u64(b + 16 + 8 * d);
  for (int d = 0; d < 3; d++) h.block[d] = hdr_u64(b + 40 + 8 * d);
  uint64_t u = hdr_u64(b + 64);
  memcpy(&h.eb_abs, &u, 8);
  u = hdr_u64(b + 72);
  memcpy(&h.eb_rel, &u, 8);
  h.ebT_bits = hdr_u64(b + 80);
  h.n = hdr_u64(b + 88);
  h.n_unpred = hdr_u64(b + 96);
  h.huff_bits = hdr_u64(b + 104);
  h.tail_bits = hdr_u64(b + 112);
  h.chunk = hdr_u32(b + 120);
  h.n_used = hdr_u32(b + 124);
  h.n_chunks = hdr_u64(b + 128);
  h.off_cb = hdr_u64(b + 136);
  h.off_ch = hdr_u64(b + 144);
  h.off_bs = hdr_u64(b + 152);
  h.off_hd = hdr_u64(b + 160);
  h.off_tl = hdr_u64(b + 168);
  h.total = hdr_u64(b + 176);
  if (h.dtype > 1 || h.ndim < 1 || h.ndim > 3 || h.layers < 1 || h.layers > 4) return SZ_ECORRUPT;
  if (check_total && h.total > size) return SZ_ECORRUPT;
  return SZ_OK;
}

// Check a parsed header for internal consistency: every count within the
// bounds its definition allows, and every section offset and the total equal
// to the layout the compressor writes (sections in order, each 64-byte
// aligned).  Every count is bounded before it enters a sum, so no sum can
// wrap around: an offset field holding a huge value is rejected rather than
// turned into a small one.
inline int check_sections(const Hdr& h) {
  if (h.eb_mode > 2 || h.flags > 2) return SZ_ECORRUPT;
  uint64_t n = 1;
  for (uint32_t d = 0; d < 3; d++) {
    if (d >= h.ndim) {
      if (h.dims[d] != 0 && h.dims[d] != 1) return SZ_ECORRUPT;
      continue;
    }
    // n stays below 2^40; the test comes before the product, which cannot wrap
    if (h.dims[d] == 0 || h.dims[d] >= (1ull << 31) || n > ((1ull << 40) - 1) / h.dims[d]) return SZ_ECORRUPT;
    n *= h.dims[d];
    if (h.block[d] == 0 || h.block[d] > h.dims[d]) return SZ_ECORRUPT;
  }
  if (h.n != n) return SZ_ECORRUPT;
  const uint64_t ts = h.dtype ? 8 : 4;
  const uint64_t raw_total = kHdr + n * ts;  // < 2^44
  if (h.flags & 1) {
    // a raw copy: every section empty and placed right after the header
    const bool empty = h.n_unpred == 0 && h.huff_bits == 0 && h.tail_bits == 0 && h.n_used == 0 &&
                       h.n_chunks == 0 && h.off_cb == kHdr && h.off_ch == kHdr && h.off_bs == kHdr &&
                       h.off_hd == kHdr && h.off_tl == kHdr;
    return empty && h.total == raw_total ? SZ_OK : SZ_ECORRUPT;
  }
  if (h.m < 1 || h.m > 16 || (h.m_req != 0 && h.m_req != h.m)) return SZ_ECORRUPT;
  if (h.chunk < 256 || h.chunk > kMaxChunk || h.chunk % 256) return SZ_ECORRUPT;
  if (h.n_chunks != (n + h.chunk - 1) / h.chunk) return SZ_ECORRUPT;
  if (h.n_used < 1 || h.n_used > (1u << h.m)) return SZ_ECORRUPT;
  const bool xorc = (h.flags & 2) != 0;
  // bits per unpredictable value in the tails section at most: the kept
  // mantissa bits, or a whole XOR record (count of leading bytes + value)
  const uint64_t max_tail = xorc ? (h.dtype ? 3 + 64 : 2 + 32) : (h.dtype ? 52 : 23);
  const uint64_t head_bits = xorc ? 32ull * h.n_chunks : h.n_unpred * (h.dtype ? 12 : 9);
  if (h.n_unpred > n || h.huff_bits > n * (uint64_t)kLmax || h.huff_bits < n ||
      h.tail_bits > h.n_unpred * max_tail)
    return SZ_ECORRUPT;
  // each term below is < 2^46, so none of the sums can wrap
  const uint64_t off_cb = kHdr;
  const uint64_t off_ch = hdr_align64(off_cb + 3ull * h.n_used);
  const uint64_t off_bs = hdr_align64(off_ch + 6ull * h.n_chunks);
  const uint64_t off_hd = hdr_align64(off_bs + 4ull * ((h.huff_bits + 31) / 32));
  const uint64_t off_tl = hdr_align64(off_hd + 4ull * ((head_bits + 31) / 32));
  const uint64_t total = off_tl + 4ull * ((h.tail_bits + 31) / 32);
  if (h.off_cb != off_cb || h.off_ch != off_ch || h.off_bs != off_bs || h.off_hd != off_hd ||
      h.off_tl != off_tl || h.total != total)
    return SZ_ECORRUPT;
  // a container at least as large as the raw field is stored raw instead
  if (total >= raw_total) return SZ_ECORRUPT;
  return SZ_OK;
}

}  // namespace szh
