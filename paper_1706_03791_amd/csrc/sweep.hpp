// Wavefront sweep of the multilayer predictor (arXiv 1706.03791, Sec. III-A,
// Eq. predmodel) with error-controlled quantization (Sec. IV-A) and the
// per-point loop of Algorithm 1, for gfx950.
//
// Every point is predicted from already *decompressed* neighbours, so the
// loop carries a dependence along every axis.  The sweep keeps the exact
// sequential result by processing point (z, y, x) at step x + s(z, y): a
// workgroup owns a tile of RZ x RY rows (a row is one (z, y) line along the
// contiguous X axis) and row (rz, ry) of the tile lags by s = rz + ry steps,
// so all neighbours (z-a, y-b, x-c) were produced at strictly earlier steps.
// Decompressed values live in an LDS ring of R slots along X; rows owned by
// the neighbouring tiles ("halo rows") are copied into the same ring from a
// global array that those tiles publish group by group behind progress
// flags.  The flags are relaxed agent-scope atomics; the ordering comes from
// the data accesses themselves: the publishing tile writes its rows with
// device-coherent stores (kCoherent: written through to the coherence point
// of all XCDs), waits for every one of them to complete (vmcnt 0) and meets
// its workgroup barrier before the flag store is issued; the waiting tile
// reads the flag, meets a workgroup barrier (which the compiler does not
// move memory accesses across) and only then issues its halo loads, also
// device-coherent, so no cached copy can answer them.  Tiles are claimed
// through an atomic ticket in dependence order, so every tile a workgroup
// waits on is already running.
//
// Input and output rows stream through per-row LDS rings in aligned chunks of
// kG elements, loaded and stored cooperatively (several lanes per row) so a
// wave instruction touches few cache lines.  The arithmetic of one point is
// the sequence of IEEE operations fixed by the format (no contraction: the
// library is compiled with -ffp-contract=off).
#pragma once

#include "common.hpp"

namespace szh {

template <typename T> struct FTr;
template <> struct FTr<float> {
  using U = uint32_t;
  static constexpr int MANT = 23, EXPB = 8, EMAX = 255;
};
template <> struct FTr<double> {
  using U = uint64_t;
  static constexpr int MANT = 52, EXPB = 11, EMAX = 2047;
};

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; i++) r *= b;
  return r;
}
constexpr int binom(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

// Offsets k = (a, b, c) along (z, y, x) and coefficients
// -prod_j (-1)^{k_j} C(n, k_j) of Eq. predmodel, in lexicographic order of k
// with the slowest dimension most significant.
template <int DIM, int NL>
struct Terms {
  static constexpr int N = ipow(NL + 1, DIM) - 1;
  int a[N], b[N], c[N], coef[N];
  constexpr Terms() : a(), b(), c(), coef() {
    int t = 0;
    for (int idx = 1; idx < ipow(NL + 1, DIM); idx++) {
      int k[3] = {0, 0, 0};
      int rem = idx;
      for (int d = 2; d >= 3 - DIM; d--) {
        k[d] = rem % (NL + 1);
        rem /= (NL + 1);
      }
      int prod = 1;
      for (int d = 3 - DIM; d < 3; d++) {
        int bn = binom(NL, k[d]);
        prod *= (k[d] & 1) ? -bn : bn;
      }
      a[t] = k[0];
      b[t] = k[1];
      c[t] = k[2];
      coef[t] = -prod;
      t++;
    }
  }
};

template <typename T>
__device__ __forceinline__ T bits_to(typename FTr<T>::U u) {
  return __builtin_bit_cast(T, u);
}
template <typename T>
__device__ __forceinline__ typename FTr<T>::U to_bits(T v) {
  return __builtin_bit_cast(typename FTr<T>::U, v);
}

// Reduced binary representation of an unpredictable value: sign, exponent
// and the top e(x) - e(eb) mantissa bits (zero when the value's exponent is
// below the bound's; everything when the bound is zero or subnormal, or the
// value is Inf/NaN).
template <typename T>
__device__ __forceinline__ T truncate_unpred(T x, typename FTr<T>::U ebT_bits) {
  using U = typename FTr<T>::U;
  constexpr int MANT = FTr<T>::MANT, EXPB = FTr<T>::EXPB, EMAX = FTr<T>::EMAX;
  const U u = to_bits<T>(x);
  const int e = (int)((u >> MANT) & (U)EMAX);
  const int e_eb = (int)((ebT_bits >> MANT) & (U)EMAX);
  if (e_eb == 0 || e == EMAX) return x;
  if (e == 0 || e < e_eb) return bits_to<T>((u >> (MANT + EXPB)) << (MANT + EXPB));
  int r = e - e_eb;
  if (r >= MANT) return x;
  const U mask = ~((((U)1) << (MANT - r)) - 1);
  return bits_to<T>(u & mask);
}

// The same truncation without branches (selects only), for the sweep's
// inner loop; returns the bit pattern.
template <typename T>
__device__ __forceinline__ typename FTr<T>::U truncate_bits(typename FTr<T>::U u, int e_eb) {
  using U = typename FTr<T>::U;
  constexpr int MANT = FTr<T>::MANT, EXPB = FTr<T>::EXPB, EMAX = FTr<T>::EMAX;
  const int e = (int)((u >> MANT) & (U)EMAX);
  const int r = e - e_eb;
  const bool keep = (e_eb == 0) | (e == EMAX) | (r >= MANT);
  const bool zero = (e == 0) | (r < 0);
  const int rc = r < 0 ? 0 : (r > MANT - 1 ? MANT - 1 : r);
  const U mask = ~((((U)1) << (MANT - rc)) - 1);
  const U sign = (u >> (MANT + EXPB)) << (MANT + EXPB);
  return keep ? u : (zero ? sign : (u & mask));
}

struct SweepArgs {
  Geom g;
  const void* x;          // compress: input field
  void* codes;            // compress: output codes; decompress: input codes
  void* xo;               // compress: optional copy of every recorded value; decompress: output field
  void* xchg;             // boundary rows published to successor tiles: [tile][row][step]
  uint32_t ne;            // exporter rows per tile
  uint32_t nsp;           // steps stored per exporter row (multiple of kG)
  const void* uvals;      // decompress: unpredictable values, raster order
  const uint64_t* useg;   // decompress: first unpredictable index of each row segment
  uint64_t n_unpred;
  uint64_t codes_cap;     // decompress: elements in the code workspace
  uint32_t* hist;         // compress: 2^m bins
  uint32_t* progress;     // per tile: completed steps
  uint32_t* ticket;
  DevPlan* plan;
  uint32_t pass2;         // adaptive-m second sweep: skip unless plan->rerun
  uint32_t export_all;    // compress debug: store every recorded value to xo
  uint32_t claim = 0;     // tile claim order of the single-field launch (claim_tile)
};

constexpr uint32_t kDone = 0xFFFFFFFFu;
// About 2^21 polls of a progress flag (each a device-scope load plus a short
// sleep) before a wait is declared stalled.
constexpr uint32_t kSpinLimit = 1u << 21;
constexpr int32_t kStatusStalled = -7;
constexpr int kHistWin = 1024;
// Cache policy of exchange traffic: sc0|sc1 = device-coherent (bypasses the
// per-CU cache and is coherent across the L2s of all XCDs), so a relaxed
// flag store after s_waitcnt publishes the data without L2 writeback or
// invalidation.
constexpr int kCoherent = 17;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima), issued as
// the builtin so the compiler's own wait tracking knows the loads are done.
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint64_t bytes) {
  const uint64_t cap = 0x7FFFFFF0ull;
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)(bytes < cap ? bytes : cap), 0x00020000);
}

// Element i of a register array of 16-byte pieces, and the reverse packing.
template <typename T>
__device__ __forceinline__ T piece_elem(const uint4* a, int i) {
  if constexpr (sizeof(T) == 4) {
    const uint4 v = a[i >> 2];
    const uint32_t w = (i & 3) == 0 ? v.x : (i & 3) == 1 ? v.y : (i & 3) == 2 ? v.z : v.w;
    return __builtin_bit_cast(T, w);
  } else {
    const uint4 v = a[i >> 1];
    const uint64_t w = (i & 1) ? (((uint64_t)v.w << 32) | v.z) : (((uint64_t)v.y << 32) | v.x);
    return __builtin_bit_cast(T, w);
  }
}
template <typename T>
__device__ __forceinline__ uint4 pack_piece(const T* e, int j) {
  if constexpr (sizeof(T) == 4) {
    return make_uint4(__builtin_bit_cast(uint32_t, e[4 * j]), __builtin_bit_cast(uint32_t, e[4 * j + 1]),
                      __builtin_bit_cast(uint32_t, e[4 * j + 2]), __builtin_bit_cast(uint32_t, e[4 * j + 3]));
  } else {
    const uint64_t a = __builtin_bit_cast(uint64_t, e[2 * j]), b = __builtin_bit_cast(uint64_t, e[2 * j + 1]);
    return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
  }
}
template <typename T>
__device__ __forceinline__ T load_coherent(__amdgpu_buffer_rsrc_t r, int byte_off) {
  if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 17));
  else
    return __builtin_bit_cast(T, (uint64_t)__builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 17));
}

template <int NL>
constexpr int ring_slots() {
  return (3 * NL + 1 <= 4) ? 4 : ((3 * NL + 1 <= 8) ? 8 : 16);
}

// Rows of a tile that successor tiles read (last NL rows along z and y).
template <int DIM, int NL, int RZ, int RY>
struct Exporters {
  static constexpr int NE = (DIM == 3) ? NL * RY + (RZ - NL) * NL : ((DIM == 2) ? NL : 0);
  static __device__ __forceinline__ int row(int rz, int ry) {
    if (DIM == 3) {
      if (rz >= RZ - NL) return (rz - (RZ - NL)) * RY + ry;
      if (ry >= RY - NL) return NL * RY + rz * NL + (ry - (RY - NL));
      return -1;
    }
    if (DIM == 2) return ry >= RY - NL ? ry - (RY - NL) : -1;
    return -1;
  }
};

// LDS of one workgroup of the sweep (taken from the dynamic allocation, so
// that a batched kernel holding several sweep bodies needs only the largest).
template <typename T, typename CT, int DIM, int NL, bool COMP, int RZ, int RY>
struct SweepLds {
  static constexpr int NT = RZ * RY;
  static constexpr int R = ring_slots<NL>();
  static constexpr int XZ = RZ + ((DIM == 3) ? NL : 0), XY = RY + ((DIM >= 2) ? NL : 0);
  static constexpr size_t a16(size_t v) { return (v + 15) & ~(size_t)15; }
  static constexpr size_t OFF_X = 0;
  static constexpr size_t OFF_V = a16(OFF_X + sizeof(T) * R * XZ * XY);
  static constexpr size_t OFF_C = a16(OFF_V + sizeof(T) * NT * kRing);
  static constexpr size_t OFF_H = a16(OFF_C + sizeof(CT) * NT * kRing);
  static constexpr size_t BYTES = a16(OFF_H + 4 * (COMP ? kHistWin : 1));
};

// One tile of the sweep, run by a workgroup of RZ * RY threads; `lds` is
// SweepLds::BYTES of dynamic LDS.
template <typename T, typename CT, int DIM, int NL, bool COMP, int RZ, int RY>
__device__ __forceinline__ void sweep_body(const SweepArgs& A, const int tile, uint8_t* lds) {
  using U = typename FTr<T>::U;
  constexpr int NT = RZ * RY;
  constexpr int R = ring_slots<NL>();
  constexpr int HZ = (DIM == 3) ? NL : 0;
  constexpr int HY = (DIM >= 2) ? NL : 0;
  constexpr int XZ = RZ + HZ, XY = RY + HY;
  constexpr Terms<DIM, NL> TT{};
  constexpr int NTERM = Terms<DIM, NL>::N;
  using EX = Exporters<DIM, NL, RZ, RY>;
  constexpr int NE = EX::NE;
  // halo rows: z-halo NL x (RY + NL), y-halo RZ x NL
  constexpr int H = (DIM == 3) ? (NL * (RY + NL) + RZ * NL) : ((DIM == 2) ? NL : 0);
  static_assert(H <= NT, "halo rows exceed threads");
  constexpr int XLPR = (kG * (int)sizeof(T)) / 16;   // 16-byte pieces per x / x' chunk
  constexpr int CLPR = (kG * (int)sizeof(CT)) / 16;  // 16-byte pieces per code chunk
  constexpr int XEPL = 16 / (int)sizeof(T);
  constexpr int CEPL = 16 / (int)sizeof(CT);

  using LD = SweepLds<T, CT, DIM, NL, COMP, RZ, RY>;
  auto& xring = *reinterpret_cast<T (*)[R][XZ][XY]>(lds + LD::OFF_X);
  auto& vring = *reinterpret_cast<T (*)[NT][kRing]>(lds + LD::OFF_V);   // compress: input x; decompress: output x'
  auto& cring = *reinterpret_cast<CT (*)[NT][kRing]>(lds + LD::OFF_C);  // codes (out for compress, in for decompress)
  auto& hl = *reinterpret_cast<uint32_t (*)[COMP ? kHistWin : 1]>(lds + LD::OFF_H);

  DevPlan* P = A.plan;
  if (P->status != 0) return;
  if (A.pass2 && !P->rerun) return;

  const int tid = threadIdx.x;
  const int rz = (DIM == 3) ? tid / RY : 0;
  const int ry = (DIM == 3) ? tid % RY : tid;
  const int s = (DIM == 1) ? 0 : rz + ry;
  const Geom& g = A.g;

  for (int i = tid; i < R * XZ * XY; i += NT) (&xring[0][0][0])[i] = T(0);
  if (COMP)
    for (int i = tid; i < kHistWin; i += NT) hl[i] = 0;
  __syncthreads();

  // ---- tile geometry
  int64_t zb0 = 0, zb1 = 1, yb0 = 0, yb1 = 1, xb0 = 0, xb1 = 0, z0 = 0, y0 = 0;
  int pred_z = -1, pred_y = -1, pred_zy = -1;
  if (DIM >= 2) {
    const int per_blk = g.tz_per_blk * g.ty_per_blk;
    const int bi = tile / per_blk;
    const int rem = tile % per_blk;
    const int tzt = rem / g.ty_per_blk, tyt = rem % g.ty_per_blk;
    const int b0 = bi / (g.nblk[1] * g.nblk[2]);
    const int b1 = (bi / g.nblk[2]) % g.nblk[1];
    const int b2 = bi % g.nblk[2];
    zb0 = (int64_t)b0 * g.blk[0];
    zb1 = min(zb0 + g.blk[0], g.dims[0]);
    yb0 = (int64_t)b1 * g.blk[1];
    yb1 = min(yb0 + g.blk[1], g.dims[1]);
    xb0 = (int64_t)b2 * g.blk[2];
    xb1 = min(xb0 + g.blk[2], g.dims[2]);
    z0 = zb0 + (int64_t)tzt * RZ;
    y0 = yb0 + (int64_t)tyt * RY;
    if (DIM == 3 && tzt > 0) pred_z = tile - g.ty_per_blk;
    if (tyt > 0) pred_y = tile - 1;
    if (DIM == 3 && tzt > 0 && tyt > 0) pred_zy = tile - g.ty_per_blk - 1;
    if (z0 >= zb1 || y0 >= yb1) {  // empty tile past a ragged block edge
      if (tid == 0) __hip_atomic_store(&A.progress[tile], kDone, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  const int64_t Xd = g.dims[2], Yd = g.dims[1];

  // per-row geometry (for any row index r of the tile)
  auto row_info = [&](int r, int64_t& base, int64_t& xlen, int& sk, bool& ok) {
    if (DIM == 1) {
      const int64_t id = (int64_t)tile * NT + r;
      const int64_t nb = (g.n + g.blk[2] - 1) / g.blk[2];
      ok = id < nb;
      base = id * g.blk[2];
      xlen = ok ? min(g.blk[2], g.n - base) : 0;
      sk = 0;
    } else {
      const int rrz = (DIM == 3) ? r / RY : 0;
      const int rry = (DIM == 3) ? r % RY : r;
      const int64_t zr = (DIM == 3) ? z0 + rrz : 0;
      const int64_t yr = y0 + rry;
      ok = zr < zb1 && yr < yb1;
      base = (zr * Yd + yr) * Xd + xb0;
      xlen = xb1 - xb0;
      sk = rrz + rry;
    }
  };

  int64_t base, xlen;
  int sk_unused;
  bool row_ok;
  row_info(tid, base, xlen, sk_unused, row_ok);
  const int64_t xlen_tile = (DIM == 1) ? g.blk[2] : (xb1 - xb0);
  const int span = (DIM == 1) ? 0 : (RZ - 1) + (RY - 1);
  const int nsteps = (int)xlen_tile + span;
  const int ngroups = (nsteps + kG - 1) / kG;

  const uint32_t m = P->m;
  const int32_t half = 1 << (m - 1);
  const T ebT = bits_to<T>((U)P->ebT_bits);
  const T twoeb = bits_to<T>((U)P->twoeb_bits);
  const T inv2eb = bits_to<T>((U)P->inv2eb_bits);
  const U ebT_bits = (U)P->ebT_bits;

  const T* __restrict__ xin = (const T*)A.x;
  CT* __restrict__ cglob = (CT*)A.codes;
  T* __restrict__ xo = (T*)A.xo;
  const int64_t ntot = g.n;

  // ---- exchange buffer: one descriptor for all tiles (wave-uniform)
  const __amdgpu_buffer_rsrc_t xr =
      make_rsrc(A.xchg, (uint64_t)g.ntiles * (uint64_t)(NE > 0 ? NE : 1) * A.nsp * sizeof(T));
  const int my_erow = EX::row(rz, ry);

  // ---- halo ownership: virtual row (hrz, hry) of this tile, read from a
  // predecessor's exporter row at a step offset d.
  bool h_own = false, h_in = false;
  int hrz = 0, hry = 0, hs = 0;
  int64_t h_elem = 0;  // element offset of the predecessor row's step 0 in xchg
  int hd = 0;
  if (DIM >= 2 && tid < H) {
    h_own = true;
    int ptile, prz, pry;
    if (DIM == 3) {
      if (tid < NL * (RY + NL)) {
        hrz = -(1 + tid / (RY + NL));
        hry = tid % (RY + NL) - NL;
        if (hry >= 0) {
          ptile = pred_z;
          prz = RZ + hrz;
          pry = hry;
          hd = RZ;
        } else {
          ptile = pred_zy;
          prz = RZ + hrz;
          pry = RY + hry;
          hd = RZ + RY;
        }
      } else {
        const int q = tid - NL * (RY + NL);
        hrz = q / NL;
        hry = -(1 + q % NL);
        ptile = pred_y;
        prz = hrz;
        pry = RY + hry;
        hd = RY;
      }
    } else {
      hrz = 0;
      hry = -(1 + tid);
      ptile = pred_y;
      prz = 0;
      pry = RY + hry;
      hd = RY;
    }
    hs = hrz + hry;
    h_in = ptile >= 0;
    if (h_in) h_elem = ((int64_t)ptile * NE + EX::row(prz, pry)) * (int64_t)A.nsp;
  }

  constexpr int HL = (kG * (int)sizeof(T)) / 16;  // 16-byte pieces per halo window
  uint4 hraw[HL], hnext[HL];
#pragma unroll
  for (int j = 0; j < HL; j++) hraw[j] = hnext[j] = make_uint4(0, 0, 0, 0);

  auto wait_preds = [&](int grp) {
    // halo values of group grp need z-pred steps + RZ and y-pred steps + RY
    if (DIM == 1) return;
    // Bounded wait: a tile only waits on tiles with smaller tickets, which
    // are already resident, so the wait always ends; the spin limit turns a
    // broken invariant into an error status instead of a hang (every tile
    // then runs to completion and publishes, so all waiters drain).
    if (tid == 0) {
      const uint32_t last = (uint32_t)(grp * kG + kG);
      const int preds[2] = {pred_z, pred_y};
      const uint32_t needs[2] = {last + RZ, last + RY};
      for (int q = 0; q < 2; q++) {
        if (preds[q] < 0) continue;
        uint32_t spins = 0;
        while (__hip_atomic_load(&A.progress[preds[q]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < needs[q]) {
          if (__hip_atomic_load(&P->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
          if (++spins > kSpinLimit) {
            atomicCAS(&P->status, 0, kStatusStalled);
            break;
          }
          __builtin_amdgcn_s_sleep(2);
        }
      }
    }
    __syncthreads();
  };

  // Halo window of group grp: predecessor steps [grp*kG + hd, +kG).
  auto load_halo = [&](int grp, uint4 (&dst)[HL]) {
    if (!h_own) return;
    const int64_t e0 = h_in ? h_elem + (int64_t)grp * kG + hd : 0;
#pragma unroll
    for (int j = 0; j < HL; j++) {
      const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(xr, (int)(e0 * sizeof(T)) + 16 * j, 0, kCoherent);
      dst[j] = __builtin_bit_cast(uint4, v);
    }
  };

  // ---- streamed chunks: register staging for the next group's input chunk
  constexpr int LPR_IN = COMP ? XLPR : CLPR;
  constexpr int EPL_IN = COMP ? XEPL : CEPL;
  uint4 pre[LPR_IN];
  bool pre_ok[LPR_IN];
  int64_t pre_pos[LPR_IN];
  int64_t row0_base, tmp_l;
  int tmp_s;
  bool tmp_ok;
  row_info(0, row0_base, tmp_l, tmp_s, tmp_ok);
  const int64_t xdesc_base = row0_base & ~(int64_t)(kG - 1);
  const __amdgpu_buffer_rsrc_t xrs =
      make_rsrc(COMP ? (const void*)(xin + xdesc_base) : nullptr,
                COMP ? (uint64_t)(ntot - xdesc_base) * sizeof(T) : 0);

  // Issue loads of the chunk holding the last element a job's row touches in
  // group grp (job j = i * NT + tid); loads are unconditional (out-of-range
  // input reads return zero, code reads are clamped into the padded
  // workspace) so no wait is placed before the group's steps.
  auto load_chunk_regs = [&](int grp) {
#pragma unroll
    for (int i = 0; i < LPR_IN; i++) {
      const int j = i * NT + tid;
      const int r = j / LPR_IN, part = j % LPR_IN;
      int64_t rb, rl;
      int rs;
      bool rok;
      row_info(r, rb, rl, rs, rok);
      const int64_t hi = rb + (int64_t)grp * kG + (kG - 1) - rs;
      const int64_t c0 = (hi >> 4) * kG;  // kG == 16
      pre_ok[i] = rok && (c0 + kG > rb) && (c0 < rb + rl);
      pre_pos[i] = c0 + part * EPL_IN;
      if (COMP) {
        const int off = (int)((c0 + part * EPL_IN - xdesc_base) * (int64_t)sizeof(T));
        pre[i] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(xrs, off, 0, 0));
      } else {
        int64_t e0 = c0 + part * EPL_IN;
        e0 = e0 < 0 ? 0 : (e0 > (int64_t)A.codes_cap - CEPL ? (int64_t)A.codes_cap - CEPL : e0);
        pre[i] = *(const uint4*)(cglob + e0);
      }
    }
  };
  auto store_chunk_ring = [&]() {
#pragma unroll
    for (int i = 0; i < LPR_IN; i++) {
      if (!pre_ok[i]) continue;
      const int j = i * NT + tid;
      const int r = j / LPR_IN;
      const int pos = (int)(pre_pos[i] & (kRing - 1));
      if (COMP)
        *(uint4*)&vring[r][pos] = pre[i];
      else
        *(uint4*)&cring[r][pos] = pre[i];
    }
  };

  // Flush of completed output chunks (codes for compress, x' for decompress).
  constexpr int LPR_OUT = COMP ? CLPR : XLPR;
  constexpr int EPL_OUT = COMP ? CEPL : XEPL;
  auto flush = [&](int grp, bool final_pass) {
#pragma unroll
    for (int i = 0; i < LPR_OUT; i++) {
      const int j = i * NT + tid;
      const int r = j / LPR_OUT, part = j % LPR_OUT;
      int64_t rb, rl;
      int rs;
      bool rok;
      row_info(r, rb, rl, rs, rok);
      if (!rok) continue;
      const int64_t hi = rb + (int64_t)grp * kG + (kG - 1) - rs;  // last raster index processed
      int64_t q;
      if (!final_pass) {
        q = ((hi + 1) >> 4) - 1;
      } else {
        // the chunk holding the row's last element, unless already complete
        const int64_t last = rb + rl - 1;
        q = last >> 4;
        const int64_t qdone = ((hi + 1) >> 4) - 1;
        if (q <= qdone) continue;
      }
      const int64_t c0 = q * kG;
      const int64_t lo_ok = rb, hi_ok = rb + rl;  // valid raster range of the row
      if (c0 + kG <= lo_ok || c0 >= hi_ok) continue;
      const int64_t e0 = c0 + part * EPL_OUT;
      const int pos = (int)(e0 & (kRing - 1));
      if (e0 >= lo_ok && e0 + EPL_OUT <= hi_ok) {
        if (COMP)
          *(uint4*)(cglob + e0) = *(const uint4*)&cring[r][pos];
        else
          *(uint4*)(xo + e0) = *(const uint4*)&vring[r][pos];
      } else {
        for (int e = 0; e < EPL_OUT; e++) {
          const int64_t ix = e0 + e;
          if (ix < lo_ok || ix >= hi_ok) continue;
          if (COMP)
            cglob[ix] = cring[r][(pos + e) & (kRing - 1)];
          else
            xo[ix] = vring[r][(pos + e) & (kRing - 1)];
        }
      }
    }
  };

  // ---- decompress: queue of this row's unpredictable values
  uint64_t uidx = 0;
  T unext = T(0);
  if (!COMP && row_ok) {
    int64_t seg;
    if (DIM == 1) {
      seg = (int64_t)tile * NT + tid;
    } else {
      const int64_t zr = (DIM == 3) ? z0 + rz : 0;
      const int64_t yr = y0 + ry;
      seg = (zr * Yd + yr) * g.nblk[2] + xb0 / g.blk[2];
    }
    uidx = A.useg[seg];
    unext = (uidx < A.n_unpred) ? ((const T*)A.uvals)[uidx] : T(0);
  }

  uint32_t cnt_center = 0, cnt_zero = 0;
  const int xlen_row = row_ok ? (int)xlen : 0;
  const int base_lo = (int)(base & (kRing - 1));
  const int e_eb = (int)((ebT_bits >> FTr<T>::MANT) & (U)FTr<T>::EMAX);
  const int32_t wbase = (COMP && (1 << m) > kHistWin) ? half - kHistWin / 2 : 0;
  T ev[kG];  // this row's values of the current group, published if it is an exporter

  // ---- prologue: group 0 halo and the two chunks group 0 may touch
  wait_preds(0);
  load_halo(0, hraw);
  // Halo rows with negative skew start before step 0: their first -hs cells
  // belong to steps that never run, so they are written here.
  if (DIM >= 2 && h_own && hs < 0) {
    for (int xl = 0; xl < -hs; xl++) {
      const int64_t e = h_in ? h_elem + (xl + hs) + hd : 0;
      const T v = load_coherent<T>(xr, (int)(e * sizeof(T)));
      xring[xl & (R - 1)][hrz + HZ][hry + HY] = (h_in && xl < xlen_tile) ? v : T(0);
    }
  }
  load_chunk_regs(-1);
  store_chunk_ring();
  load_chunk_regs(0);
  store_chunk_ring();
  // Nothing may still be in flight when the loop starts, or the compiler's
  // wait tracking (merging this path with the loop's back edge) would stall
  // every group's prefetch on it.
  wait_vm();
  __syncthreads();

  for (int grp = 0; grp < ngroups; grp++) {
    const bool more = grp + 1 < ngroups;
    if (more) {
      wait_preds(grp + 1);
      load_halo(grp + 1, hnext);
      load_chunk_regs(grp + 1);
    }
#pragma unroll
    for (int i = 0; i < kG; i++) {
      const int sigma = grp * kG + i;
      const int xl = sigma - s;
      const bool act = (unsigned)xl < (unsigned)xlen_row;
      if (DIM >= 2 && h_own) {
        const int hx = sigma - hs;
        const bool hv_ok = h_in && (unsigned)hx < (unsigned)xlen_tile;
        xring[hx & (R - 1)][hrz + HZ][hry + HY] = hv_ok ? piece_elem<T>(hraw, i) : T(0);
      }
      T p = T(0);
#pragma unroll
      for (int t = 0; t < NTERM; t++) {
        const T v = xring[(xl - TT.c[t]) & (R - 1)][rz - TT.a[t] + HZ][ry - TT.b[t] + HY];
        p = p + T(TT.coef[t]) * v;
      }
      const int rpos = (base_lo + xl) & (kRing - 1);
      T xq;
      if (COMP) {
        // Quantization of one point (same IEEE operations as the format
        // defines: t = (x - p) * (1/2eb), k = rint(t), x_q = p + k * 2eb,
        // predictable iff |t| < 2^(m-1), |k| <= 2^(m-1) - 1, |x - x_q| < eb).
        const T x = vring[tid][rpos];
        const T t = (x - p) * inv2eb;
        const bool inr = fabs(t) < T(half);
        const int k = inr ? (int)rint(t) : 0;
        const bool kin = (k <= half - 1) & (k >= -(half - 1));
        const T xqq = p + T(k) * twoeb;
        const bool ok = inr & kin & (fabs(x - xqq) < ebT);
        const T xt = bits_to<T>(truncate_bits<T>(to_bits<T>(x), e_eb));
        xq = act ? (ok ? xqq : xt) : T(0);
        const uint32_t code = ok ? (uint32_t)(k + half) : 0u;
        cnt_center += (act & ok & (k == 0)) ? 1u : 0u;
        cnt_zero += (act & !ok) ? 1u : 0u;
        if (act & ok & (k != 0)) {
          const uint32_t w = code - (uint32_t)wbase;
          if (w < (uint32_t)kHistWin)
            atomicAdd(&hl[w], 1u);
          else
            atomicAdd(&A.hist[code], 1u);
        }
        if (act) cring[tid][rpos] = (CT)code;
        if (A.export_all && act) xo[base + xl] = xq;
      } else {
        const int32_t code = (int32_t)cring[tid][rpos];
        const T v1 = p + T(code - half) * twoeb;
        const bool zc = act & (code == 0);
        xq = act ? (code != 0 ? v1 : unext) : T(0);
        if (zc) {
          uidx++;
          unext = (uidx < A.n_unpred) ? ((const T*)A.uvals)[uidx] : T(0);
        }
        if (act) vring[tid][rpos] = xq;
      }
      ev[i] = xq;
      xring[xl & (R - 1)][rz + HZ][ry + HY] = xq;
      if (DIM >= 2) __syncthreads();
    }
    // Group end.  Exporter rows publish their 16 values with coherent vector
    // stores; once every wave's stores are complete the progress flag moves.
    // The next input chunk replaces the ring half that this group finished
    // reading; completed output chunks are flushed after the flag so their
    // stores never delay a successor tile.
    if (DIM >= 2 && my_erow >= 0) {
      const int64_t e0 = ((int64_t)tile * NE + my_erow) * (int64_t)A.nsp + (int64_t)grp * kG;
#pragma unroll
      for (int j = 0; j < HL; j++) {
        const uint4 v = pack_piece<T>(ev, j);
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), xr, (int)(e0 * sizeof(T)) + 16 * j, 0,
                                               kCoherent);
      }
    }
    if (DIM == 1) __syncthreads();
    wait_vm();
    if (more) store_chunk_ring();
#pragma unroll
    for (int j = 0; j < HL; j++) hraw[j] = hnext[j];
    __syncthreads();
    if (DIM >= 2 && tid == 0) {
      const uint32_t done = more ? (uint32_t)((grp + 1) * kG) : kDone;
      __hip_atomic_store(&A.progress[tile], done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    flush(grp, false);
    if (!more) flush(grp, true);
  }

  if (COMP) {
    if (cnt_zero) {
      if (0 - wbase >= 0 && 0 - wbase < kHistWin)
        atomicAdd(&hl[0 - wbase], cnt_zero);
      else
        atomicAdd(&A.hist[0], cnt_zero);
    }
    if (cnt_center) atomicAdd(&hl[half - wbase], cnt_center);
    __syncthreads();
    const int nb = min(kHistWin, 1 << m);
    for (int i = tid; i < nb; i += NT)
      if (hl[i]) atomicAdd(&A.hist[wbase + i], hl[i]);
  }
}

// Single-field launch: tiles are claimed through the field's ticket in
// dependence order.
template <typename T, typename CT, int DIM, int NL, bool COMP, int RZ, int RY>
__global__ void __launch_bounds__(RZ * RY) sweep_kernel(SweepArgs A) {
  extern __shared__ __align__(16) uint8_t sz_lds[];
  __shared__ int s_tile;
  if (A.plan->status != 0 || (A.pass2 && !A.plan->rerun)) return;
  if (threadIdx.x == 0)
    s_tile = claim_tile((int)atomicAdd(A.ticket, 1u), A.claim, A.g.tz_per_blk, A.g.ty_per_blk, A.g.ntiles);
  __syncthreads();
  sweep_body<T, CT, DIM, NL, COMP, RZ, RY>(A, s_tile, sz_lds);
}

}  // namespace szh
