// Wave-tiled wavefront sweep for 3D fields with the 1-layer predictor
// (arXiv 1706.03791, Sec. III-A Eq. predmodel with n = 1, the 3D Lorenzo
// stencil; quantization of Sec. IV-A; the per-point loop of Algorithm 1).
//
// A workgroup of NW waves owns a tile of (NW * AZ) z-rows by 64 y-rows
// (a row runs along the contiguous X axis).  Lane ly of wave w owns the 64
// rows y0 + ly of the AZ z-rows z0 + AZ * w + a, and processes point x of
// sub-row a at step x + AZ * w + a + ly.  With this skew every neighbour of
// a point was produced one, two or three steps earlier:
//   * along x by the same lane (registers),
//   * along y by lane ly - 1 (a wave_shr:1 DPP move of that lane's output;
//     lane 0 takes the value published by the tile before it along y),
//   * along z by the same lane's sub-row a - 1 (registers), by the last
//     sub-row of wave w - 1 (passed through LDS once per step), or, for
//     wave 0, by the tile before it along z (published per group).
// The dependence chain inside a workgroup therefore costs one step per row
// and needs no LDS traffic along y.  Tiles are claimed through an atomic
// ticket in dependence order and publish their boundary rows every kWG
// steps as device-coherent records tagged with the launch (sweep_tag); the
// next tile polls the records themselves, so no store is ever waited for.
//
// Input values (compress) and decompressed values (decompress) stream
// through per-row LDS rings of two aligned chunks; codes stream through
// registers.  The arithmetic of one point is the fixed sequence of IEEE
// operations of the format (the library is built with -ffp-contract=off).
#pragma once

#include <type_traits>

#include "sweep.hpp"

namespace szh {

constexpr int kWG = 8;       // steps per group (also the chunk length in elements)
constexpr int kWRing = 16;   // ring slots per row: two chunks
constexpr int kWLanes = 64;  // y-rows per tile
struct WArgs {
  int64_t dims[3];   // Z, Y, X
  int64_t blk[3];
  int32_t nblk[3];
  int32_t tz_per_blk, ty_per_blk, ntiles;
  uint32_t nsp;      // steps stored per exchange row (multiple of kWG)
  const void* x;     // compress: input field
  void* codes;       // compress: output codes; decompress: input codes
  void* xo;          // compress (debug): every recorded value; decompress: output field
  void* xy;          // exchange towards the next tile along y: [tile][wave][step] tagged records
  void* xz;          // exchange towards the next tile along z: [tile][out | y-moved][group][piece][lane]
  const void* uvals; // decompress: unpredictable values in raster order
  const uint64_t* useg;
  uint64_t n_unpred;
  uint64_t codes_cap;  // elements in the code workspace
  uint64_t n;
  uint32_t* ticket;
  DevPlan* plan;
  uint32_t pass2;
  uint32_t export_all;
  uint32_t claim = 0;  // tile claim order of the single-field launch (claim_tile)
};

// Lane l takes lane l-1's value; lane 0 takes `old` (wave_shr:1).
template <typename T>
__device__ __forceinline__ T wave_shr1(T src, T old) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                             __builtin_bit_cast(int, src), 0x138, 0xF, 0xF, false));
  } else {
    const uint64_t s = __builtin_bit_cast(uint64_t, src), o = __builtin_bit_cast(uint64_t, old);
    const uint32_t lo =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)s, 0x138, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(s >> 32),
                                                              0x138, 0xF, 0xF, false);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}
template <typename T>
__device__ __forceinline__ T read_lane(T v, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
  }
}
// acc with lane `lane` replaced by the wave-uniform value v.
template <typename T>
__device__ __forceinline__ T write_lane(T acc, T v, int lane, int my_lane) {
  return my_lane == lane ? v : acc;
}

// One chunk of kWG codes as an integer (u8: 64 bits, u16: 128 bits), code i
// in bits [i * SB, (i + 1) * SB).
template <typename CT>
using CWord = typename std::conditional<sizeof(CT) == 1, uint64_t, unsigned __int128>::type;

template <typename CT>
__device__ __forceinline__ CWord<CT> load_code_chunk(__amdgpu_buffer_rsrc_t r, int64_t q) {
  // q may be negative or past the end: the offset then falls outside the
  // descriptor and the load returns zero
  const int64_t bo = q * (int64_t)(kWG * sizeof(CT));
  const int off = (bo < 0 || bo > 0x7FFFFF00ll) ? 0x7FFFFF00 : (int)bo;
  if constexpr (sizeof(CT) == 1) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    return ((uint64_t)v[1] << 32) | v[0];
  } else {
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return ((unsigned __int128)(((uint64_t)v[3] << 32) | v[2]) << 64) | (((uint64_t)v[1] << 32) | v[0]);
  }
}

// Codes of the window that starts o codes into chunk c0 (o in [0, kWG)).
template <typename CT>
__device__ __forceinline__ CWord<CT> code_window(CWord<CT> c0, CWord<CT> c1, int o) {
  constexpr int SB = 8 * sizeof(CT);
  constexpr int BITS = kWG * SB;
  if (o == 0) return c0;
  return (c0 >> (SB * o)) | (c1 << (BITS - SB * o));
}

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// The AZ values of one step as an 8-byte y-exchange record (a single f32
// value takes the low word).
template <typename T, int AZ>
__device__ __forceinline__ u32x2 pack_rec(const T (&v)[AZ]) {
  static_assert(AZ * sizeof(T) <= 8, "one 8-byte exchange record per step");
  if constexpr (sizeof(T) == 4) {
    return u32x2{__builtin_bit_cast(uint32_t, v[0]), AZ > 1 ? __builtin_bit_cast(uint32_t, v[AZ - 1]) : 0u};
  } else {
    const uint64_t a0 = __builtin_bit_cast(uint64_t, v[0]);
    return u32x2{(uint32_t)a0, (uint32_t)(a0 >> 32)};
  }
}

// Reduced binary representation of an unpredictable value (same result as
// truncate_unpred) computed with bit masks only, so the step stays one
// basic block: keep the value when the bound is not normal or the value is
// Inf/NaN or no mantissa bit can go; a signed zero when its exponent is 0 or
// below the bound's; else clear the low MANT - (e - e_eb) mantissa bits.
template <typename T>
__device__ __forceinline__ typename FTr<T>::U trunc_masked(typename FTr<T>::U u, int e_eb) {
  using U = typename FTr<T>::U;
  constexpr int MANT = FTr<T>::MANT, EXPB = FTr<T>::EXPB, EMAX = FTr<T>::EMAX;
  const int e = (int)((u >> MANT) & (U)EMAX);
  const int r = e - e_eb;
  const U keep = (U)0 - (U)((e_eb == 0) | (e == EMAX) | (r >= MANT));
  const U zero = (U)0 - (U)((e == 0) | (r < 0));
  const int rc = r < 0 ? 0 : (r > MANT - 1 ? MANT - 1 : r);
  const U mant = ~((((U)1) << (MANT - rc)) - 1);
  const U sign = ((U)1) << (MANT + EXPB);
  const U m = keep | (~keep & ((zero & sign) | (~zero & mant)));
  return u & m;
}

// A 16-byte store marked non-temporal: codes and reconstructed values are
// written once and not read again by the sweep, so their partly written
// lines should not take L2 capacity from the input lines still being read.
__device__ __forceinline__ void st_nt(void* p, uint4 v) {
  __builtin_nontemporal_store(u32x4{v.x, v.y, v.z, v.w}, (u32x4*)p);
}
__device__ __forceinline__ void st_nt(void* p, uint64_t v) {
  __builtin_nontemporal_store(v, (uint64_t*)p);
}

// Element a of an 8-byte exchange record.
template <typename T>
__device__ __forceinline__ T rec_elem(u32x2 v, int a) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, (uint32_t)v[a]);
  else
    return __builtin_bit_cast(T, ((uint64_t)v[1] << 32) | v[0]);
}

// Exchange records carry the launch's tag in every 8-byte unit: a 32-bit
// payload and the tag.  An aligned 8-byte access is a single unit, so a
// reader that finds the tag has this launch's payload, whatever the order in
// which the units of a record or of a group become visible; every record slot
// is written once per launch, slots of earlier launches hold older tags, and
// cleared memory holds none.  The tag sets bit 31, so it is never zero.
__device__ __forceinline__ uint32_t sweep_tag(const DevPlan* P, uint32_t pass2) {
  return 0x80000000u | (P->epoch << 1) | (pass2 & 1u);
}
// A 16-byte piece of z-records: two f32 values, or one f64 value.
template <typename T>
__device__ __forceinline__ u32x4 tag_piece(const T* v, uint32_t tag) {
  if constexpr (sizeof(T) == 4) {
    return u32x4{__builtin_bit_cast(uint32_t, v[0]), tag, __builtin_bit_cast(uint32_t, v[1]), tag};
  } else {
    const uint64_t b = __builtin_bit_cast(uint64_t, v[0]);
    return u32x4{(uint32_t)b, tag, (uint32_t)(b >> 32), tag};
  }
}
// Value e of a tagged piece (e < 2 for f32, 0 for f64).
template <typename T>
__device__ __forceinline__ T piece_value(u32x4 p, int e) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, (uint32_t)p[2 * e]);
  else
    return __builtin_bit_cast(T, ((uint64_t)p[2] << 32) | p[0]);
}

// LDS of one workgroup of the wave-tiled sweep (dynamic allocation).
// The z-exchange between waves is a ring of one entry per step of a group:
// entry e, slot s holds the value of a step e (mod kWG) of the row below
// wave s, that is wave s - 1's last sub-row, or for s = 0 the tile's
// z-halo, which wave 0 writes for a whole group at the end of the group
// before.  Every wave thus reads the row below at the same offsets.
template <typename T, int NW, int AZ>
struct WSweepLds {
  static constexpr size_t OFF_RING = 0;
  static constexpr size_t OFF_XW = OFF_RING + sizeof(T) * NW * AZ * kWRing * 64;
  static constexpr size_t OFF_YIN = OFF_XW + sizeof(T) * kWG * (NW + 1) * 2 * 64;
  static constexpr size_t BYTES = OFF_YIN + 8 * NW * kWG;
};

// One tile of the wave-tiled sweep, run by a workgroup of NW waves; `lds` is
// WSweepLds::BYTES of dynamic LDS; pass2 marks the second sweep of an
// adaptive compression.
template <typename T, typename CT, bool COMP, int NW, int AZ, bool DBG>
__device__ __forceinline__ void wsweep_body(const WArgs& A, const int tile_in, uint8_t* lds, const uint32_t pass2) {
  // the tile is the same for every lane: keep everything derived from it in
  // scalar registers
  const int tile = __builtin_amdgcn_readfirstlane(tile_in);
  using U = typename FTr<T>::U;
  using CW = CWord<CT>;
  constexpr int G = kWG;
  constexpr int TZ = NW * AZ;
  constexpr int SB = 8 * sizeof(CT);
  constexpr int XPC = (G * (int)sizeof(T)) / 16;  // 16-byte pieces per chunk of values
  constexpr int EPP = 16 / (int)sizeof(T);        // values per piece
  static_assert(AZ * sizeof(T) <= 8, "one 8-byte y-exchange record per step");

  using LD = WSweepLds<T, NW, AZ>;
  // per-row input (compress) or output (decompress) rings
  auto& s_ring = *reinterpret_cast<T (*)[NW][AZ][kWRing][64]>(lds + LD::OFF_RING);
  // the row below each wave: [step mod G][wave + 1 | 0 for the z-halo][out | moved][lane]
  auto& s_xw = *reinterpret_cast<T (*)[G][NW + 1][2][64]>(lds + LD::OFF_XW);
  auto& s_yin = *reinterpret_cast<u32x2 (*)[NW][kWG]>(lds + LD::OFF_YIN);   // y-halo records, one per step

  DevPlan* P = A.plan;
  if (P->status != 0) return;
  if (pass2 && !P->rerun) return;

  const int tid = threadIdx.x;
  const int w = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane(tid >> 6), ly = tid & 63;
  for (int i = tid; i < G * (NW + 1) * 2 * 64; i += NW * 64) (&s_xw[0][0][0][0])[i] = T(0);
  __syncthreads();

  // ---- tile geometry
  const int per_blk = A.tz_per_blk * A.ty_per_blk;
  const int bi = tile / per_blk, brem = tile % per_blk;
  const int tzt = brem / A.ty_per_blk, tyt = brem % A.ty_per_blk;
  const int bz = bi / (A.nblk[1] * A.nblk[2]), by = (bi / A.nblk[2]) % A.nblk[1], bx = bi % A.nblk[2];
  const int64_t Yd = A.dims[1], Xd = A.dims[2];
  const int64_t zb0 = (int64_t)bz * A.blk[0], zb1 = min(zb0 + A.blk[0], A.dims[0]);
  const int64_t yb0 = (int64_t)by * A.blk[1], yb1 = min(yb0 + A.blk[1], Yd);
  const int64_t xb0 = (int64_t)bx * A.blk[2], xb1 = min(xb0 + A.blk[2], Xd);
  const int64_t z0 = zb0 + (int64_t)tzt * TZ, y0 = yb0 + (int64_t)tyt * kWLanes;
  const int pred_z = tzt > 0 ? tile - A.ty_per_blk : -1;
  const int pred_y = tyt > 0 ? tile - 1 : -1;
  const bool succ_z = tzt + 1 < A.tz_per_blk && z0 + TZ < zb1;
  const bool succ_y = tyt + 1 < A.ty_per_blk && y0 + kWLanes < yb1;
  const int BX = (int)(xb1 - xb0);
  const int nsteps = BX + (TZ - 1) + (kWLanes - 1);
  const int ngroups = (nsteps + G - 1) / G;
  // groups run in pairs (the buffer sets alternate): an odd count gets one
  // more group, in which no point is active
  const int ngr = (ngroups + 1) & ~1;
  const int64_t yr = y0 + ly;

  int64_t rb[AZ];   // raster index of the row's first element
  int64_t wlo[AZ];  // raster index of the first element of group 0's window
  bool rv[AZ];
  int sk[AZ];
  int xlen[AZ];  // BX for a valid row, 0 for rows past the block edge
#pragma unroll
  for (int a = 0; a < AZ; a++) {
    const int64_t zr = z0 + AZ * w + a;
    rv[a] = zr < zb1 && yr < yb1;
    rb[a] = (zr * Yd + yr) * Xd + xb0;
    sk[a] = AZ * w + a + ly;
    wlo[a] = rb[a] - sk[a];
    xlen[a] = rv[a] ? (int)(xb1 - xb0) : 0;
  }

  const uint32_t m = P->m;
  const int32_t half = 1 << (m - 1);
  const T halfT = T(half), halfm1T = T(half - 1);
  const T ebT = bits_to<T>((U)P->ebT_bits);
  const T twoeb = bits_to<T>((U)P->twoeb_bits);
  const T inv2eb = bits_to<T>((U)P->inv2eb_bits);
  const int e_eb = (int)(((U)P->ebT_bits >> FTr<T>::MANT) & (U)FTr<T>::EMAX);

  // ---- exchange descriptors (one each for all tiles; offsets < 2 GiB)
  const uint32_t tag = sweep_tag(P, pass2);
  const uint64_t nsp = A.nsp;
  constexpr int VPP = sizeof(T) == 4 ? 2 : 1;  // values per tagged 16-byte piece
  constexpr int ZP = G / VPP;                  // pieces per group of z-records
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(A.xy, (uint64_t)A.ntiles * NW * nsp * 16);
  // (no z-exchange when a block holds one tile along z: its loads read zero)
  const __amdgpu_buffer_rsrc_t rz =
      make_rsrc(A.xz, A.tz_per_blk > 1 ? (uint64_t)A.ntiles * 2 * 64 * nsp * (2 * sizeof(T)) : 0);
  auto y_off = [&](int t, int step) -> int {  // 16-byte record of (tile t, wave w, step)
    return (int)((((int64_t)t * NW + w) * (int64_t)nsp + step) * 16);
  };
  // z records: [tile][out | y-moved][group][piece][lane] of tagged pieces, so
  // one wave's access to a piece of a group is 1 KiB of whole cache lines
  auto z_piece = [&](int t, int kind, int grp, int j) -> int {  // piece j of group grp of lane ly
    return (int)((((((int64_t)t * 2 + kind) * (int64_t)(nsp / G) + grp) * ZP + j) * 64 + ly) * 16);
  };
  auto z_unit = [&](int t, int kind, int idx) -> int {  // the tagged unit(s) of element idx (lane ly)
    return z_piece(t, kind, idx / G, (idx % G) / VPP) + (idx % VPP) * 8;
  };
  constexpr int kOut = 0x7FFFFF00;  // offset past every descriptor: loads read zero

  // ---- input descriptor (values for compress, codes for decompress), based
  // at the tile's first chunk so offsets stay small
  const int64_t tile_lo = ((z0 * Yd + y0) * Xd + xb0) - (TZ + kWLanes + G);
  // chunk index of the descriptor base, never before the buffer: chunks
  // below it (negative indices near the array start) fall outside and read 0
  const int64_t cbase = max((int64_t)0, tile_lo >> 3);
  const int64_t ebase = cbase * G;     // element index of the descriptor base
  const __amdgpu_buffer_rsrc_t rin =
      COMP ? make_rsrc((const T*)A.x + ebase, (uint64_t)max((int64_t)0, (int64_t)A.n - ebase) * sizeof(T))
           : make_rsrc((const CT*)A.codes + ebase, (uint64_t)max((int64_t)0, (int64_t)A.codes_cap - ebase) *
                                                       sizeof(CT));

  // ---- halo records of group gr
  // A predecessor writes its records of steps [0, ngr * G) along y and of
  // indices [0, ngr * G] along z (index k holds step k - 1); later records
  // are never needed by an active step and never waited for.  A missing
  // predecessor is a descriptor of zero records (its loads read zero and
  // touch no memory), chosen per tile in scalar registers.  Each wave loads
  // its own y-records; the z-halo's ZP pieces per kind are shared out among
  // the waves, piece j to wave j mod NW (wave 0 owns piece 0, the values read
  // at the first step of a group, before any barrier of that group).
  const bool wave0 = w == 0;  // uniform: scalar selects below
  constexpr bool kZX = NW > 1;                           // z-exchange compiled in (a 2D field has none)
  constexpr int ZPW = kZX ? (ZP + NW - 1) / NW : 1;      // z pieces per wave and kind
  // A predecessor stores records only for a successor with rows in the block
  // (a tile past the block's edge waits for none: its points are inactive).
  const bool need_y = pred_y >= 0 && y0 < yb1, need_z = kZX && pred_z >= 0 && z0 < zb1;
  const __amdgpu_buffer_rsrc_t ry_in = need_y ? ry : make_rsrc(A.xy, 0);
  const __amdgpu_buffer_rsrc_t rz_in = need_z ? rz : make_rsrc(A.xz, 0);
  const int pred_y0 = pred_y >= 0 ? pred_y : 0, pred_z0 = pred_z >= 0 ? pred_z : 0;
  const int last_rec = ngr * G;  // y-steps below it and z-indices up to it are written
  // y: lanes l and l + G hold the record of the values lane 0 needs at step gr*G + (l mod G)
  auto load_yh = [&](int gr) -> u32x4 {
    return __builtin_amdgcn_raw_buffer_load_b128(ry_in, y_off(pred_y0, gr * G + kWLanes + (ly & (G - 1))), 0,
                                                 kCoherent);
  };
  // The halo of one group as loaded: the wave's y-record and its z pieces
  // (the moved and unmoved values of the row below at steps gr*G - 1 + i,
  // records of indices gr*G + TZ + i; TZ is a multiple of VPP, so they form
  // whole pieces).  A piece past ZP is loaded through a descriptor of zero
  // records, so every wave issues the same loads on every path.
  struct Halo {
    u32x4 yh;
    u32x4 zo[ZPW], zy[ZPW];
  };
  auto zpiece_of = [&](int k) -> int { return w + NW * k; };
  auto load_h = [&](int gr, Halo& h) {
    h.yh = load_yh(gr);
    if constexpr (kZX) {
#pragma unroll
      for (int k = 0; k < ZPW; k++) {
        const int j = zpiece_of(k);
        const __amdgpu_buffer_rsrc_t r = j < ZP ? rz_in : make_rsrc(A.xz, 0);
        h.zo[k] = __builtin_amdgcn_raw_buffer_load_b128(r, z_unit(pred_z0, 0, gr * G + TZ + VPP * j), 0, kCoherent);
        h.zy[k] = __builtin_amdgcn_raw_buffer_load_b128(r, z_unit(pred_z0, 1, gr * G + TZ + VPP * j), 0, kCoherent);
      }
    }
  };
  // Whether the wave's part of the halo of group gr holds this launch's
  // records (wave-uniform).
  auto halo_ok = [&](int gr, const Halo& h) -> bool {
    const int ys = gr * G + kWLanes + (ly & (G - 1));
    bool ok = !need_y || ys >= last_rec || (h.yh[1] == tag && h.yh[3] == tag);
    if constexpr (kZX) {
      if (need_z) {
#pragma unroll
        for (int k = 0; k < ZPW; k++) {
          const int j = zpiece_of(k);
          const int k0 = gr * G + TZ + VPP * j, k1 = k0 + VPP - 1;  // indices of the piece's units
          ok &= j >= ZP || k0 > last_rec || (h.zo[k][1] == tag && h.zy[k][1] == tag);
          ok &= j >= ZP || k1 > last_rec || (h.zo[k][3] == tag && h.zy[k][3] == tag);
        }
      }
    }
    return __builtin_amdgcn_ballot_w64(!ok) == 0;
  };
  // Reload the halo of group gr until it holds this launch's records (the
  // predecessor is still writing it), or until the launch has failed.
  auto poll_halo = [&](int gr, Halo& h) {
    uint32_t spins = 0;
    while (!halo_ok(gr, h)) {
      if (__hip_atomic_load(&P->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spins > kSpinLimit) {
        if (ly == 0) atomicCAS(&P->status, 0, kStatusStalled);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      load_h(gr, h);
    }
  };

  // ---- input chunks: chunk q of sub-row a (raster elements [8q, 8q + 8))
  auto chunk_off = [&](int64_t q) -> int {
    const int64_t bo = (q - cbase) * (int64_t)(G * (COMP ? sizeof(T) : sizeof(CT)));
    return (bo < 0 || bo > 0x7FFFFF00ll) ? kOut : (int)bo;
  };
  auto load_x_chunk = [&](int64_t q, uint4 (&dst)[XPC]) {
    const int off = chunk_off(q);
#pragma unroll
    for (int j = 0; j < XPC; j++)
      dst[j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rin, off == kOut ? kOut : off + 16 * j,
                                                                               0, 0));
  };
  auto ring_put = [&](int a, int64_t q, const uint4 (&src)[XPC]) {
#pragma unroll
    for (int e = 0; e < G; e++) s_ring[w][a][(int)((q * G + e) & (kWRing - 1))][ly] = piece_elem<T>(src, e);
  };
  // Compression refills the rings cooperatively: each 16-byte load of the
  // wave takes XPC lanes per row (piece ly % XPC of row ly / XPC + h * 64 /
  // XPC), so it touches 64 / XPC cache lines rather than 64, and the pieces
  // go to their rows' ring columns.  Row r's window of group gr starts at
  // element rbase + r * X - (AZ w + a + r).
  constexpr int RPI = 64 / XPC;  // rows per load instruction
  int64_t rbase[AZ];
#pragma unroll
  for (int a = 0; a < AZ; a++) rbase[a] = rb[a] - (int64_t)ly * Xd;
  auto coop_chunk = [&](int a, int h, int gr) -> int64_t {  // chunk after row r's first chunk of group gr
    const int r = ly / XPC + RPI * h;
    const int64_t wl = rbase[a] + (int64_t)r * Xd - (int64_t)(AZ * w + a + r);
    return ((wl + (int64_t)gr * G) >> 3) + 1;
  };
  // Each group moves a row's window by one chunk, so the byte offset of a
  // lane's piece grows by one chunk per group and its ring slot flips bit 3
  // (slots are taken mod 16 and a chunk is 8 elements): both are computed
  // once per tile.
  int cb0[AZ][XPC];         // input byte offset of the lane's chunk for group 0 (< 0: before the buffer)
  uint32_t cput0[AZ][XPC];  // s_ring byte offset of the lane's piece for group 0
  if constexpr (COMP) {
#pragma unroll
    for (int a = 0; a < AZ; a++)
#pragma unroll
      for (int h = 0; h < XPC; h++) {
        const int r = ly / XPC + RPI * h, pc = ly % XPC;
        const int64_t q = coop_chunk(a, h, 0);
        cb0[a][h] = (int)((q - cbase) * (int64_t)(G * sizeof(T)));
        const uint32_t slot = (uint32_t)((q * G + pc * EPP) & (kWRing - 1));
        cput0[a][h] = ((((uint32_t)w * AZ + a) * kWRing + slot) * 64 + (uint32_t)r) * (uint32_t)sizeof(T);
      }
  }
  auto coop_load = [&](int a, int gr, uint4 (&dst)[XPC]) {
#pragma unroll
    for (int h = 0; h < XPC; h++) {
      const int bo = cb0[a][h] + gr * (int)(G * sizeof(T));
      dst[h] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                             rin, bo < 0 ? kOut : bo + 16 * (ly % XPC), 0, 0));
    }
  };
  // Decompression flushes the same way: lane ly stores piece ly % XPC of the
  // chunk row r completed in group gr, reading the values from r's column.
  auto coop_flush = [&](int a, int gr) {
    T* xg = (T*)A.xo;
    const int64_t zr = z0 + AZ * w + a;
#pragma unroll
    for (int h = 0; h < XPC; h++) {
      const int r = ly / XPC + RPI * h, pc = ly % XPC;
      if (!(zr < zb1 && y0 + r < yb1)) continue;
      const int64_t lo = rbase[a] + (int64_t)r * Xd, hi = lo + BX;
      const int64_t wl = lo - (int64_t)(AZ * w + a + r);
      const int64_t e0 = ((wl + (int64_t)gr * G) >> 3) * G + pc * EPP;  // first element of the piece
      if (e0 + EPP <= lo || e0 >= hi) continue;
      T v[EPP];
#pragma unroll
      for (int e = 0; e < EPP; e++) v[e] = s_ring[w][a][(int)((e0 + e) & (kWRing - 1))][r];
      if (e0 >= lo && e0 + EPP <= hi) {
        st_nt(xg + e0, pack_piece<T>(v, 0));
      } else {
#pragma unroll
        for (int e = 0; e < EPP; e++)
          if (e0 + e >= lo && e0 + e < hi) xg[e0 + e] = v[e];
      }
    }
  };
  auto coop_put = [&](int a, int gr, const uint4 (&src)[XPC]) {
    const uint32_t flip = (uint32_t)(gr & 1) * (8u * 64u * (uint32_t)sizeof(T));
#pragma unroll
    for (int h = 0; h < XPC; h++) {
      T* p = (T*)((uint8_t*)&s_ring[0][0][0][0] + (cput0[a][h] ^ flip));
#pragma unroll
      for (int e = 0; e < EPP; e++) p[e * 64] = piece_elem<T>(&src[h], e);
    }
  };

  // Output chunk q of sub-row a: only the elements of this row are written.
  auto store_codes = [&](int a, int64_t q, CW word) {
    if (!rv[a]) return;
    const int64_t e0 = q * G, lo = rb[a], hi = rb[a] + BX;
    if (e0 + G <= lo || e0 >= hi) return;
    CT* cg = (CT*)A.codes;
    if (e0 >= lo && e0 + G <= hi) {
      if constexpr (sizeof(CT) == 1) {
        st_nt(cg + e0, (uint64_t)word);
      } else {
        const uint64_t w0 = (uint64_t)word, w1 = (uint64_t)(word >> 64);
        st_nt(cg + e0, make_uint4((uint32_t)w0, (uint32_t)(w0 >> 32), (uint32_t)w1, (uint32_t)(w1 >> 32)));
      }
    } else {
#pragma unroll
      for (int j = 0; j < G; j++) {
        const int64_t e = e0 + j;
        if (e >= lo && e < hi) cg[e] = (CT)(word >> (SB * j));
      }
    }
  };
  // Chunks 2k and 2k + 1 of a row leave as one aligned store when both lie
  // inside the row (half the store instructions and cache-line writes);
  // otherwise each chunk is stored on its own.
  auto store_pair = [&](int a, int64_t qe, CW w0, CW w1) {
    if (!rv[a]) return;
    const int64_t e0 = qe * G, lo = rb[a], hi = rb[a] + BX;
    if (e0 >= lo && e0 + 2 * G <= hi) {
      CT* cg = (CT*)A.codes;
      if constexpr (sizeof(CT) == 1) {
        const uint64_t a0 = (uint64_t)w0, a1 = (uint64_t)w1;
        st_nt(cg + e0, make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32)));
      } else {
        const uint64_t a0 = (uint64_t)w0, a1 = (uint64_t)(w0 >> 64), b0 = (uint64_t)w1, b1 = (uint64_t)(w1 >> 64);
        st_nt(cg + e0, make_uint4((uint32_t)a0, (uint32_t)(a0 >> 32), (uint32_t)a1, (uint32_t)(a1 >> 32)));
        st_nt(cg + e0 + G, make_uint4((uint32_t)b0, (uint32_t)(b0 >> 32), (uint32_t)b1, (uint32_t)(b1 >> 32)));
      }
    } else {
      store_codes(a, qe, w0);
      store_codes(a, qe + 1, w1);
    }
  };
  auto flush_values = [&](int a, int64_t q) {
    if (!rv[a]) return;
    const int64_t e0 = q * G, lo = rb[a], hi = rb[a] + BX;
    if (e0 + G <= lo || e0 >= hi) return;
    T* xg = (T*)A.xo;
    T v[G];
#pragma unroll
    for (int j = 0; j < G; j++) v[j] = s_ring[w][a][(int)((e0 + j) & (kWRing - 1))][ly];
    if (e0 >= lo && e0 + G <= hi) {
#pragma unroll
      for (int j = 0; j < XPC; j++) st_nt(xg + e0 + EPP * j, pack_piece<T>(v, j));
    } else {
#pragma unroll
      for (int j = 0; j < G; j++) {
        const int64_t e = e0 + j;
        if (e >= lo && e < hi) xg[e] = v[j];
      }
    }
  };

  // ---- state
  T O1[AZ], O2[AZ], Y1[AZ], Y2[AZ], Y3[AZ];
#pragma unroll
  for (int a = 0; a < AZ; a++) O1[a] = O2[a] = Y1[a] = Y2[a] = Y3[a] = T(0);
  T VO1 = T(0), VO2 = T(0), VY1 = T(0), VY2 = T(0), VY3 = T(0);  // row below sub-row 0

  // halo records of the next group, loaded during this one (a halo loaded
  // two groups ahead hides more of the loads' latency but adds a group to
  // the lag between dependent tiles, which costs more)
  Halo hnx;
  hnx.yh = u32x4{0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < ZPW; k++) hnx.zo[k] = hnx.zy[k] = u32x4{0, 0, 0, 0};
  T ezo[G], ezy[G];  // last wave: records of indices g*G + i (index k = value of step k - 1)
#pragma unroll
  for (int i = 0; i < G; i++) ezo[i] = ezy[i] = T(0);
  T co = T(0), cy = T(0);  // value of the group's last step: record 0 of the next group

  // compress: input chunks of groups g + 1 (entry 0) and g + 2 (entry 1)
  uint4 xq2[2][AZ][COMP ? XPC : 1];
#pragma unroll
  for (int k = 0; k < 2; k++)
#pragma unroll
    for (int a = 0; a < AZ; a++)
#pragma unroll
      for (int h = 0; h < (COMP ? XPC : 1); h++) xq2[k][a][h] = make_uint4(0, 0, 0, 0);
  // decompress: code chunks of this window, the three after it, and the one
  // being loaded
  CW c0[AZ], c1[AZ], c2[AZ], c3[AZ], cpre[AZ];
  CW cacc[AZ], cprv[AZ];           // compress: codes of this and the previous group's window
  CW chold[AZ];                    // compress: an even chunk waiting for its partner
  int64_t qhold[AZ];               // its index, -1 for none
  uint32_t cpk[AZ][2];             // compress, 1-byte codes: the group's codes, four per word
  // Groups whose odd chunk q completes a pair (q - 1, q) that lies wholly
  // inside the row: [gpa, gpb] (the chunk of group g is (wlo >> 3) + g).
  int gpa[AZ], gpb[AZ];
  // Decompress: the unpredictable values a group consumes, in a register
  // window loaded during the group before (values uidx .. uidx + zc - 1 of
  // the row's raster-ordered stream), so that no step waits for memory
  // while other waves of the workgroup could run.  A one-wave tile is
  // latency-bound instead: it loads each value when the one before it is
  // consumed (`unext`), which costs fewer instructions per step.
  constexpr bool UWIN = !COMP && NW > 1;
  constexpr int UW = UWIN ? G : 1;
  T uw[AZ][UW], uw_nxt[AZ][UW];
  T unext[AZ];
  int64_t uidx[AZ];  // stream index of the first value this group consumes (next value: one-wave tiles)
  int zc[AZ];        // values this group consumes
#pragma unroll
  for (int a = 0; a < AZ; a++) {
    c0[a] = c1[a] = c2[a] = c3[a] = cpre[a] = cacc[a] = cprv[a] = chold[a] = (CW)0;
    qhold[a] = -1;
    cpk[a][0] = cpk[a][1] = 0;
    const int64_t q0 = wlo[a] >> 3;
    gpa[a] = (int)(((rb[a] + G - 1) >> 3) + 1 - q0);
    gpb[a] = rv[a] ? (int)(((rb[a] + BX) >> 3) - 1 - q0) : -1;
    uidx[a] = 0;
    zc[a] = 0;
    unext[a] = T(0);
#pragma unroll
    for (int j = 0; j < UW; j++) uw[a][j] = uw_nxt[a][j] = T(0);
  }
  // unpredictable values from the tile's first row on: offsets stay below 2 GiB
  const int64_t ubase =
      !UWIN ? 0 : (int64_t)A.useg[((z0 * Yd + y0) * (int64_t)A.nblk[2]) + bx];
  const __amdgpu_buffer_rsrc_t ru =
      make_rsrc(!UWIN ? nullptr : (const T*)A.uvals + ubase,
                !UWIN ? 0 : (uint64_t)max((int64_t)0, (int64_t)A.n_unpred - ubase) * sizeof(T));
  // Zero codes among the active steps of group gr's window `win` of sub-row
  // a: an exact zero-field mask (high bit of each SB-bit field set iff the
  // field is 0), restricted to the active steps [i0, i1), then a popcount.
  auto zeros_in = [&](CW win, int gr, int a) -> int {
    const int i0 = min(max(sk[a] - gr * G, 0), G);
    const int i1 = min(max(sk[a] + xlen[a] - gr * G, 0), G);
    if constexpr (sizeof(CT) == 1) {
      const uint64_t lo7 = 0x7F7F7F7F7F7F7F7Full;
      const uint64_t zm = ~(((win & lo7) + lo7) | win | lo7);
      const uint64_t am = (i1 > i0) ? (((i1 - i0) == 8 ? ~0ull : ((1ull << (8 * (i1 - i0))) - 1)) << (8 * i0)) : 0ull;
      return __builtin_popcountll(zm & am);
    } else {
      const uint64_t lo15 = 0x7FFF7FFF7FFF7FFFull;
      int z = 0;
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const uint64_t x = (uint64_t)(win >> (64 * h));
        const uint64_t zm = ~(((x & lo15) + lo15) | x | lo15);
        const int b0 = min(max(i0 - 4 * h, 0), 4), b1 = min(max(i1 - 4 * h, 0), 4);
        const uint64_t am = (b1 > b0) ? (((b1 - b0) == 4 ? ~0ull : ((1ull << (16 * (b1 - b0))) - 1)) << (16 * b0)) : 0ull;
        z += __builtin_popcountll(zm & am);
      }
      return z;
    }
  };
  // The z values from stream index u on into dst, entries [j0, j1) of the
  // window.  Lanes with z > j0 load them all (entries past z, or past the
  // stream, go unused); other lanes load from an offset past the descriptor.
  auto load_uw = [&](int64_t u, int z, T (&dst)[UW], int j0, int j1) {
    const int base = z > j0 ? (int)((u - ubase) * (int64_t)sizeof(T)) : kOut;
#pragma unroll
    for (int j = j0; j < j1; j++) {
      if constexpr (sizeof(T) == 4) {
        dst[j] = __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(ru, base + 4 * j, 0, 0));
      } else {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(ru, base + 8 * j, 0, 0);
        dst[j] = __builtin_bit_cast(T, ((uint64_t)v[1] << 32) | v[0]);
      }
    }
  };

  // The halo of a group into LDS: the y-records into s_yin, and the z-halo
  // into slot 0 of the exchange ring, the value of step gr*G + i - 1 at entry
  // (i - 1) mod G, where wave 0 reads it at step gr*G + i.  A wave writes the
  // pieces it owns; only wave 0's piece 0 is read before the next barrier.
  // Pieces past ZP go to slot NW, which nobody reads: every path that loads
  // a register then reads it, so the compiler's count of loads in flight
  // stays exact and it adds no waits of its own.
  auto put_halo = [&](const Halo& h) {
    s_yin[w][ly & (G - 1)] = u32x2{h.yh[0], h.yh[2]};  // lanes l and l + G hold the same record
    if constexpr (kZX) {
#pragma unroll
      for (int k = 0; k < ZPW; k++) {
        const int j = zpiece_of(k);
        const int slot = j < ZP ? 0 : NW;
#pragma unroll
        for (int u = 0; u < VPP; u++) {
          const int e = (VPP * j + u + G - 1) & (G - 1);
          s_xw[e][slot][0][ly] = piece_value<T>(h.zo[k], u);
          s_xw[e][slot][1][ly] = piece_value<T>(h.zy[k], u);
        }
      }
    }
    // lanes 0..G-1 wrote the records every lane of the wave reads next;
    // keep the compiler from moving the reads above the writes
    __builtin_amdgcn_wave_barrier();
  };
  // Load, check and write the halo of group gr until it holds this launch's
  // records (after a failed check).
  auto repoll_halo = [&](int gr) {
    Halo h;
    uint32_t spins = 0;
    do {
      if (__hip_atomic_load(&P->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (++spins > kSpinLimit) {
        if (ly == 0) atomicCAS(&P->status, 0, kStatusStalled);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      load_h(gr, h);
    } while (!halo_ok(gr, h));
    put_halo(h);
  };
  // One 16-byte piece of the cooperative input load of group gr.
  auto coop_load1 = [&](int a, int h, int gr) -> uint4 {
    const int bo = cb0[a][h] + gr * (int)(G * sizeof(T));
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rin, bo < 0 ? kOut : bo + 16 * (ly % XPC),
                                                                           0, 0));
  };
  // Input load instructions of a group (compress: one per step from step 0).
  constexpr int kInLoads = AZ * XPC;
  static_assert(!COMP || kInLoads <= G, "one input load per step");

  // ---- prologue: halo and input of the first group
  {
    Halo h0;
    load_h(0, h0);
    poll_halo(0, h0);
    put_halo(h0);
    if (wave0) {
      // Rows before lane 0 run ahead of it: the y-halo row (skew -1) already
      // produced x = 0 at step -1, and the corner row (z-1, y-1; skew -2) at
      // step -2.  Their values enter the histories before step 0 (polled for
      // like the halo: records become visible in no particular order).
      const bool sy = need_y, sz = need_z;
      const int ez = (TZ - 1) % VPP;  // unit of the z value in its piece
      u32x4 ry1 = {0, 0, 0, 0}, rz1 = {0, 0, 0, 0};
      uint32_t spins = 0;
      for (;;) {
        ry1 = __builtin_amdgcn_raw_buffer_load_b128(ry_in, y_off(pred_y0, kWLanes - 1), 0, kCoherent);
        rz1 = __builtin_amdgcn_raw_buffer_load_b128(need_z ? rz : rz_in, z_unit(pred_z0, 1, TZ - 1) & ~15, 0,
                                                    kCoherent);
        const bool ok = (!sy || (ry1[1] == tag && ry1[3] == tag)) &&
                        (!sz || (rz1[2 * ez + 1] == tag && rz1[VPP == 1 ? 3 : 2 * ez + 1] == tag));
        if (__builtin_amdgcn_ballot_w64(!ok) == 0) break;
        if (__hip_atomic_load(&P->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
        if (++spins > kSpinLimit) {
          if (ly == 0) atomicCAS(&P->status, 0, kStatusStalled);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
      if (sy) Y1[0] = ly == 0 ? rec_elem<T>(u32x2{ry1[0], ry1[2]}, 0) : T(0);
      if (sz) VY1 = piece_value<T>(rz1, ez);
    }
  }
  // Step -1 of each wave's last sub-row, read by the next wave at step 0
  // (nonzero only for the seeded y-halo value above when AZ == 1).
  if (w + 1 < NW) {
    s_xw[G - 1][w + 1][0][ly] = O1[AZ - 1];
    s_xw[G - 1][w + 1][1][ly] = Y1[AZ - 1];
  }
#pragma unroll
  for (int a = 0; a < AZ; a++) {
    const int64_t q0 = wlo[a] >> 3;
    if constexpr (COMP) {
      uint4 t0[XPC], t1[XPC];
      load_x_chunk(q0, t0);
      load_x_chunk(q0 + 1, t1);
      wait_vm();
      ring_put(a, q0, t0);
      ring_put(a, q0 + 1, t1);
      coop_load(a, 1, xq2[0][a]);
    } else {
      __amdgpu_buffer_rsrc_t r = rin;
      c0[a] = load_code_chunk<CT>(r, q0 - cbase);
      c1[a] = load_code_chunk<CT>(r, q0 + 1 - cbase);
      c2[a] = load_code_chunk<CT>(r, q0 + 2 - cbase);
      c3[a] = load_code_chunk<CT>(r, q0 + 3 - cbase);
      if (rv[a]) {
        const int64_t seg = ((z0 + AZ * w + a) * Yd + yr) * A.nblk[2] + bx;
        uidx[a] = (int64_t)A.useg[seg];
        if constexpr (!UWIN) unext[a] = ((uint64_t)uidx[a] < A.n_unpred) ? ((const T*)A.uvals)[uidx[a]] : T(0);
      }
    }
  }
  wait_vm();
  if constexpr (UWIN) {
    // group 0's window of unpredictable values
#pragma unroll
    for (int a = 0; a < AZ; a++) {
      const int o = (int)(wlo[a] & (G - 1));
      zc[a] = zeros_in(code_window<CT>(c0[a], c1[a], o), 0, a);
      load_uw(uidx[a], zc[a], uw[a], 0, UW);
    }
    wait_vm();
  }
  __syncthreads();

  // One group.  Compression loads the input of group g + 2 into X1 while it
  // puts that of group g + 1 (X0) into the rings; the loop alternates the
  // two buffers, so no register that a load may still be writing is ever
  // copied (a copy would wait for the load).  Every load of a group is
  // issued on every group, also the last (its records and chunks lie inside
  // the buffers or past them and go unused), so that no branch joins their
  // registers before they are used.
  using XB = uint4[AZ][COMP ? XPC : 1];
  auto group = [&](const int g, XB& X0, XB& X1) __attribute__((always_inline)) {
      const bool more = g + 1 < ngr;
      int zn[AZ];  // decompress: values the next group consumes
#pragma unroll
      for (int a = 0; a < AZ; a++) {
        const int64_t q = (wlo[a] + (int64_t)(g + 1) * G) >> 3;  // first chunk of the next window
        zn[a] = 0;
        if constexpr (!COMP) {
          cpre[a] = load_code_chunk<CT>(rin, q + 3 - cbase);
          if constexpr (UWIN) {
            zn[a] = zeros_in(code_window<CT>(c1[a], c2[a], (int)(wlo[a] & (G - 1))), g + 1, a);
            load_uw(uidx[a] + zc[a], zn[a], uw_nxt[a], 0, 2);
          }
        } else {
          (void)q;
        }
      }
      if constexpr (UWIN) {
        // Most windows hold at most two unpredictable values: two loads per
        // sub-row go out above.  Only when a lane of the wave needs more does
        // the wave load the rest of its window.
        bool several = false;
#pragma unroll
        for (int a = 0; a < AZ; a++) several |= zn[a] > 2;
        if (__builtin_amdgcn_ballot_w64(several) != 0) {
#pragma unroll
          for (int a = 0; a < AZ; a++) load_uw(uidx[a] + zc[a], zn[a], uw_nxt[a], 2, UW);
        }
      }
      // per-group window of each sub-row and its inputs
      int bslot[AZ];
      CW cwin[AZ];
#pragma unroll
      for (int a = 0; a < AZ; a++) {
        const int64_t lo = wlo[a] + (int64_t)g * G;
        bslot[a] = (int)(lo & (kWRing - 1));
        if constexpr (!COMP) cwin[a] = code_window<CT>(c0[a], c1[a], (int)(lo & (G - 1)));
      }
      T xin[AZ][COMP ? G : 1];
      T yk[G][AZ];  // this group's values; lane 63's are the y-successor's halo
      if constexpr (COMP) {
#pragma unroll
        for (int a = 0; a < AZ; a++)
#pragma unroll
          for (int i = 0; i < G; i++) xin[a][i] = s_ring[w][a][(bslot[a] + i) & (kWRing - 1)][ly];
      }

#pragma unroll
      for (int i = 0; i < G; i++) {
        const int sig = g * G + i;
        // the row below sub-row 0 at step sig - 1: the last sub-row of the
        // wave below, or the z-halo for wave 0 (ring slot w)
        const T vn_o = s_xw[(i + G - 1) & (G - 1)][w][0][ly];
        const T vn_y = s_xw[(i + G - 1) & (G - 1)][w][1][ly];
        const u32x2 yrec = s_yin[w][i];  // the y-halo values lane 0 takes at this step
        VO2 = VO1;
        VO1 = vn_o;
        VY3 = VY2;
        VY2 = VY1;
        VY1 = vn_y;
        // The AZ sub-rows are independent within a step (each reads only
        // values of earlier steps); every statement below runs across all of
        // them so their dependence chains interleave.
        T l1[AZ], l2[AZ], ly2[AZ], ly3[AZ], p[AZ], xq[AZ];
        bool act[AZ];
#pragma unroll
        for (int a = 0; a < AZ; a++) {
          l1[a] = a > 0 ? O1[a > 0 ? a - 1 : 0] : VO1;
          l2[a] = a > 0 ? O2[a > 0 ? a - 1 : 0] : VO2;
          ly2[a] = a > 0 ? Y2[a > 0 ? a - 1 : 0] : VY2;
          ly3[a] = a > 0 ? Y3[a > 0 ? a - 1 : 0] : VY3;
          act[a] = (unsigned)(sig - sk[a]) < (unsigned)xlen[a];
        }
        // Eq. predmodel, n = 1, terms in lexicographic order of (kz, ky, kx)
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = T(0) + O1[a];  // (0,0,1) +1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] + Y1[a];  // (0,1,0) +1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] - Y2[a];  // (0,1,1) -1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] + l1[a];  // (1,0,0) +1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] - l2[a];  // (1,0,1) -1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] - ly2[a];  // (1,1,0) -1
#pragma unroll
        for (int a = 0; a < AZ; a++) p[a] = p[a] + ly3[a];  // (1,1,1) +1
        if constexpr (COMP) {
          T t[AZ], rk[AZ], xqq[AZ];
          bool ok[AZ];
#pragma unroll
          for (int a = 0; a < AZ; a++) t[a] = (xin[a][i] - p[a]) * inv2eb;
#pragma unroll
          for (int a = 0; a < AZ; a++) rk[a] = rint(t[a]);
#pragma unroll
          for (int a = 0; a < AZ; a++) xqq[a] = p[a] + rk[a] * twoeb;
          // |rk| <= half - 1 implies |t| < half (rint moves t by at most 1/2),
          // so the format's test |t| < half needs no instruction of its own
#pragma unroll
          for (int a = 0; a < AZ; a++) ok[a] = (fabs(rk[a]) <= halfm1T) & (fabs(xin[a][i] - xqq[a]) < ebT);
          U xb[AZ];
          bool bad = false;
#pragma unroll
          for (int a = 0; a < AZ; a++) {
            xb[a] = to_bits<T>(xqq[a]);
            bad |= !ok[a];
          }
          // Unpredictable points are rare: the reduced representation is
          // computed only in steps where a lane of the wave has one (a
          // wave-uniform branch).
          if (__builtin_amdgcn_ballot_w64(bad) != 0) {
#pragma unroll
            for (int a = 0; a < AZ; a++) {
              const U okm = (U)0 - (U)ok[a];
              xb[a] = (xb[a] & okm) | (trunc_masked<T>(to_bits<T>(xin[a][i]), e_eb) & ~okm);
            }
          }
#pragma unroll
          for (int a = 0; a < AZ; a++) {
            const U am = (U)0 - (U)act[a];
            xq[a] = bits_to<T>(xb[a] & am);
            if constexpr (sizeof(CT) == 1) {
              // the code as a float (an exact integer below 256) packed into
              // byte i % 4 of word i / 4
              const float cf = ok[a] ? (float)(rk[a] + halfT) : 0.0f;
              cpk[a][i >> 2] = __builtin_amdgcn_cvt_pk_u8_f32(cf, (uint32_t)(i & 3), cpk[a][i >> 2]);
            } else {
              const uint32_t code = ok[a] ? (uint32_t)((int)rk[a] + half) : 0u;
              cacc[a] |= (CW)code << (SB * i);
            }
            if constexpr (DBG)
              if (act[a]) ((T*)A.xo)[rb[a] + (sig - sk[a])] = xq[a];
          }
        } else {
          bool took[AZ], any_took = false;
#pragma unroll
          for (int a = 0; a < AZ; a++) {
            const uint32_t code = (uint32_t)(cwin[a] >> (SB * i)) & ((1u << SB) - 1);
            const T v1 = p[a] + T((int32_t)code - half) * twoeb;
            if constexpr (UWIN) {
              xq[a] = act[a] ? (code != 0 ? v1 : uw[a][0]) : T(0);
              took[a] = act[a] && code == 0;
              any_took |= took[a];
            } else {
              xq[a] = act[a] ? (code != 0 ? v1 : unext[a]) : T(0);
              if (act[a] && code == 0) {
                uidx[a]++;
                unext[a] = ((uint64_t)uidx[a] < A.n_unpred) ? ((const T*)A.uvals)[uidx[a]] : T(0);
              }
            }
            s_ring[w][a][(bslot[a] + i) & (kWRing - 1)][ly] = xq[a];
          }
          if constexpr (UWIN) {
            // A consumed value leaves the window (at most G - 1 - i values
            // remain for the rest of the group).  Unpredictable points are
            // rare: the shift runs only in steps where a lane of the wave took
            // one (a wave-uniform branch).
            if (__builtin_amdgcn_ballot_w64(any_took) != 0) {
#pragma unroll
              for (int a = 0; a < AZ; a++)
#pragma unroll
                for (int j = 0; j + 1 < UW - i; j++) uw[a][j] = took[a] ? uw[a][j + 1] : uw[a][j];
            }
          }
        }
        // y-moved values: lane 0 takes the last row of the tile before along y
        T ynew[AZ];
#pragma unroll
        for (int a = 0; a < AZ; a++) ynew[a] = wave_shr1<T>(xq[a], rec_elem<T>(yrec, a));
#pragma unroll
        for (int a = 0; a < AZ; a++) {
          O2[a] = O1[a];
          O1[a] = xq[a];
          Y3[a] = Y2[a];
          Y2[a] = Y1[a];
          Y1[a] = ynew[a];
          yk[i][a] = xq[a];
        }
        // the wave above reads this wave's last sub-row at the next step
        if (w + 1 < NW) {
          s_xw[i][w + 1][0][ly] = xq[AZ - 1];
          s_xw[i][w + 1][1][ly] = ynew[AZ - 1];
        }
        if (i + 1 < G) {
          ezo[i + 1] = xq[AZ - 1];
          ezy[i + 1] = ynew[AZ - 1];
        } else {
          co = xq[AZ - 1];
          cy = ynew[AZ - 1];
        }
        // compression: one load of the input of group g + 2 per step
        if constexpr (COMP) {
          if (i < kInLoads) X1[i / XPC][i % XPC] = coop_load1(i / XPC, i % XPC, g + 2);
        }
        // the step's exchange between waves; a single wave needs no barrier
        // (its own LDS accesses complete in order)
        if constexpr (NW > 1) __syncthreads();
        // the next group's halo, checked at the end of this one
        if (i == 0) load_h(g + 1, hnx);
      }


      // ---- group end.  First the check of the next group's halo (loaded
      // after step 0): vector memory operations retire in order, so the wait
      // for its loads here includes none of this group's stores.
      const bool halo_in = halo_ok(g + 1, hnx);
      // ---- the boundary records, stored and never waited for
      if (succ_y) {
        // lane 63's G records move to lanes 64 - G .. 63 (one record each)
        // and leave with one store
        u32x2 rec = {0, 0};
#pragma unroll
        for (int i = 0; i < G; i++) {
          const u32x2 r = pack_rec<T, AZ>(yk[i]);
          const u32x2 r63 = {(uint32_t)__builtin_amdgcn_readlane((int)r[0], kWLanes - 1),
                             (uint32_t)__builtin_amdgcn_readlane((int)r[1], kWLanes - 1)};
          if (ly == kWLanes - G + i) rec = r63;
        }
        if (ly >= kWLanes - G)
          __builtin_amdgcn_raw_buffer_store_b128(u32x4{rec[0], tag, rec[1], tag}, ry,
                                                 y_off(tile, g * G + ly - (kWLanes - G)), 0, kCoherent);
      }
      if (succ_z && w == NW - 1) {
#pragma unroll
        for (int j = 0; j < ZP; j++) {
          __builtin_amdgcn_raw_buffer_store_b128(tag_piece<T>(ezo + VPP * j, tag), rz, z_piece(tile, 0, g, j), 0,
                                                 kCoherent);
          __builtin_amdgcn_raw_buffer_store_b128(tag_piece<T>(ezy + VPP * j, tag), rz, z_piece(tile, 1, g, j), 0,
                                                 kCoherent);
        }
        if (!more) {
          // the last step's value lives in record (g + 1) * G, past this group
          if constexpr (sizeof(T) == 4) {
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{__builtin_bit_cast(uint32_t, co), tag}, rz,
                                                  z_unit(tile, 0, (g + 1) * G), 0, kCoherent);
            __builtin_amdgcn_raw_buffer_store_b64(u32x2{__builtin_bit_cast(uint32_t, cy), tag}, rz,
                                                  z_unit(tile, 1, (g + 1) * G), 0, kCoherent);
          } else {
            __builtin_amdgcn_raw_buffer_store_b128(tag_piece<T>(&co, tag), rz, z_unit(tile, 0, (g + 1) * G), 0,
                                                   kCoherent);
            __builtin_amdgcn_raw_buffer_store_b128(tag_piece<T>(&cy, tag), rz, z_unit(tile, 1, (g + 1) * G), 0,
                                                   kCoherent);
          }
        }
      }
      ezo[0] = co;
      ezy[0] = cy;
      // ---- completed chunk of each row, input refill, register rotation.
      // None of it depends on the records just stored.
#pragma unroll
      for (int a = 0; a < AZ; a++) {
        const int64_t lo = wlo[a] + (int64_t)g * G;
        const int64_t q = lo >> 3;
        const int o = (int)(lo & (G - 1));
        if constexpr (COMP) {
          if constexpr (sizeof(CT) == 1) cacc[a] = ((CW)cpk[a][1] << 32) | cpk[a][0];
          const CW word = o ? ((cprv[a] >> (SB * (G - o))) | (cacc[a] << (SB * o))) : cacc[a];
          const bool qodd = (q & 1) != 0;
          // An even chunk waits for its partner; an odd one completes the pair:
          // one aligned store when the pair lies inside the row (all groups but
          // those at the row's ends), else chunk by chunk in a branch that the
          // wave takes only when one of its lanes needs it.
          const bool pair_ok = qodd && g >= gpa[a] && g <= gpb[a];
          if (pair_ok) {
            CT* cg = (CT*)A.codes + (q - 1) * G;
            if constexpr (sizeof(CT) == 1) {
              st_nt(cg, make_uint4((uint32_t)chold[a], (uint32_t)(chold[a] >> 32), (uint32_t)word,
                                   (uint32_t)(word >> 32)));
            } else {
              store_pair(a, q - 1, chold[a], word);
            }
          }
          const bool edge = qodd && !pair_ok && rv[a];
          if (__builtin_amdgcn_ballot_w64(edge) != 0) {
            if (edge) {
              if (qhold[a] == q - 1) store_codes(a, q - 1, chold[a]);
              store_codes(a, q, word);
            }
          }
          if (!qodd) chold[a] = word;
          qhold[a] = qodd ? -1 : q;
          cprv[a] = cacc[a];
          cacc[a] = (CW)0;
          // the chunk of group g + 1, loaded during group g - 1
          coop_put(a, g + 1, X0[a]);  // (past the last group: unread)
        } else {
          (void)q;
          coop_flush(a, g);
          c0[a] = c1[a];
          c1[a] = c2[a];
          c2[a] = c3[a];
          c3[a] = cpre[a];
          if constexpr (UWIN) {
            uidx[a] += zc[a];
            zc[a] = zn[a];
#pragma unroll
            for (int j = 0; j < UW; j++) uw[a][j] = uw_nxt[a][j];
          }
        }
      }
      // ---- the halo of group g + 1 into LDS.  Wave 0 read the entries of
      // group g's halo before the barrier of the step that read them (the
      // last at step G - 1), which every wave has passed, and its own reads
      // complete in order.  If the check found a record still missing, the
      // wave polls its part again, in registers of its own, and writes it
      // again.  (Past the last group the records are not waited for: see
      // last_rec.)
      put_halo(hnx);
      if (!halo_in) repoll_halo(g + 1);
  };
  for (int g = 0; g < ngr; g += 2) {
    group(g, xq2[0], xq2[1]);
    group(g + 1, xq2[1], xq2[0]);
  }
  // ---- the chunk after the last window (its head was produced in the last group)
#pragma unroll
  for (int a = 0; a < AZ; a++) {
    const int64_t lo = wlo[a] + (int64_t)(ngr - 1) * G;
    const int64_t q = (lo >> 3) + 1;
    const int o = (int)(lo & (G - 1));
    if constexpr (COMP) {
      if (o != 0) {
        const CW word = cprv[a] >> (SB * (G - o));
        if (qhold[a] == q - 1 && (q & 1)) {
          store_pair(a, q - 1, chold[a], word);
          qhold[a] = -1;
        } else {
          store_codes(a, q, word);
        }
      }
      if (qhold[a] >= 0) store_codes(a, qhold[a], chold[a]);
    } else {
      if (o != 0) flush_values(a, q);
    }
  }
}

// Single-field launch: tiles are claimed through the field's ticket in
// dependence order.
template <typename T, typename CT, bool COMP, int NW, int AZ, bool DBG>
__global__ void __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu((NW + 3) / 4, (NW + 3) / 4)))
wsweep_kernel(WArgs A) {
  extern __shared__ __align__(16) uint8_t sz_lds[];
  __shared__ int s_tile;
  if (A.plan->status != 0 || (A.pass2 && !A.plan->rerun)) return;
  if (threadIdx.x == 0) s_tile = claim_tile((int)atomicAdd(A.ticket, 1u), A.claim, A.tz_per_blk, A.ty_per_blk, A.ntiles);
  __syncthreads();
  wsweep_body<T, CT, COMP, NW, AZ, DBG>(A, s_tile, sz_lds, A.pass2);
}

}  // namespace szh
