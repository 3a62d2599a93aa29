// Kernels around the wavefront sweep: value range and error bound
// (Metric 1), adaptive interval count (Sec. IV-B), Huffman codebook,
// encoding and decoding (Sec. IV-A), storage of unpredictable values
// (Sec. IV-B, Algorithm 1) and the container writer/reader.
#pragma once

#include "common.hpp"
#include "sweep.hpp"

namespace szh {
// Internal linkage: every translation unit that launches these kernels
// carries its own copy.
namespace {

// ------------------------------------------------------------ wave peers
// The lanes (among the `ok` ones) whose B-bit key equals this lane's, from
// B ballots.  Counting a key once per group, by the group's highest lane,
// replaces same-address LDS atomics, which serialise over the lanes.
template <int B>
__device__ __forceinline__ uint64_t wave_peers(bool ok, uint32_t key) {
  uint64_t peers = __ballot(ok);
#pragma unroll
  for (int b = 0; b < B; b++) {
    const uint64_t bb = __ballot(ok && ((key >> b) & 1u));
    peers &= ((key >> b) & 1u) ? bb : ~bb;
  }
  return peers;
}
__device__ __forceinline__ bool peers_last(uint64_t peers) {
  return (peers >> (threadIdx.x & 63)) == 1ull;
}

// ------------------------------------------------------------ block scans
// Exclusive scan over a workgroup of NT threads (NT a multiple of 64).
template <int NT, typename V>
__device__ __forceinline__ V block_exscan(V v, V* lds, V* total) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  V x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    V y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  if (wid == 0) {
    V w = (lane < NT / 64) ? lds[lane] : V(0);
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      V y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < NT / 64) lds[lane] = w;
  }
  __syncthreads();
  const V off = wid ? lds[wid - 1] : V(0);
  const V tot = lds[NT / 64 - 1];
  __syncthreads();
  if (total) *total = tot;
  return off + x - v;
}

template <int NT, typename V>
__device__ __forceinline__ V block_sum(V v, V* lds) {
  V tot;
  block_exscan<NT, V>(v, lds, &tot);
  return tot;
}

__device__ __forceinline__ void set_status(DevPlan* P, int code) {
  atomicCAS(&P->status, 0, code);
}

// ------------------------------------------------------------- utilities
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
// Two arrays zeroed by one launch.
__global__ void zero2_u32_kernel(uint32_t* p, uint64_t n, uint32_t* q, uint64_t m) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m;
       i += (uint64_t)gridDim.x * blockDim.x) {
    if (i < n)
      p[i] = 0;
    else
      q[i - n] = 0;
  }
}

// Zero the first plan->total bytes of the container (sections are written
// with OR operations and padding must read as zero).
__device__ __forceinline__ void zero_container_kernel_dev(uint32_t* out, const DevPlan* P) {
  if (P->status || P->raw) return;
  const uint64_t nw = (P->total + 3) / 4;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nw;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = 0;
}
// Zero n 16-byte words.
__global__ void zero16_kernel(uint4* p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}
__global__ void zero_container_kernel(uint32_t* out, const DevPlan* P) {
  zero_container_kernel_dev(out, P);
}


struct PlanInit {
  uint32_t m;        // 16 for the first adaptive sweep
  uint32_t eb_mode;
  double eb_abs, eb_rel;
  uint32_t dtype;
  uint64_t cap;
  uint32_t xorc;
};

__device__ __forceinline__ void plan_init_kernel_dev(DevPlan* P, PlanInit I) {
  if (threadIdx.x == 0) {
    DevPlan z = {};
    z.m = I.m;
    z.minmax_bits[0] = 0xFFFFFFFFu;
    z.minmax_bits[1] = 0;
    z.minmax64[0] = ~0ull;
    z.minmax64[1] = 0;
    z.out_cap = I.cap;
    z.xorc = I.xorc;
    z.epoch = P->epoch + 1;  // a new tag for this launch's exchange records
    *P = z;
  }
}
__global__ void plan_init_kernel(DevPlan* P, PlanInit I) {
  plan_init_kernel_dev(P, I);
}


// Order-preserving integer images of floating-point values.
__device__ __forceinline__ uint32_t ord32(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __builtin_bit_cast(float, u);
}
__device__ __forceinline__ uint64_t ord64(double f) {
  uint64_t u = __builtin_bit_cast(uint64_t, f);
  return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double unord64(uint64_t o) {
  uint64_t u = (o >> 63) ? (o & ~(1ull << 63)) : ~o;
  return __builtin_bit_cast(double, u);
}

// ----------------------------------------------------- K1: value range
// Min and max in T (only finite data uses the range: REL and BOTH modes
// reject non-finite input, flagged here), four 16-byte loads in flight per
// thread, combined across the grid as order-preserving integer keys.
template <typename T>
__device__ __forceinline__ void mm_update(T f, T& mn, T& mx, uint32_t& nf) {
  nf |= !isfinite(f);
  mn = f < mn ? f : mn;
  mx = f > mx ? f : mx;
}

template <typename T>
__device__ __forceinline__ void minmax_kernel_dev(const T* __restrict__ x, uint64_t n, DevPlan* P) {
  __shared__ uint64_t lmin[4], lmax[4];
  __shared__ uint32_t lnf;
  if (threadIdx.x == 0) lnf = 0;
  T mn = (T)__builtin_huge_val(), mx = -(T)__builtin_huge_val();
  uint32_t nf = 0;
  constexpr int V = 16 / sizeof(T);
  const uint64_t nv = n / V;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint4* xv = (const uint4*)x;
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    uint4 raw[4];
#pragma unroll
    for (int u = 0; u < 4; u++) raw[u] = xv[i + u * stride];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const T* v = (const T*)&raw[u];
#pragma unroll
      for (int e = 0; e < V; e++) mm_update<T>(v[e], mn, mx, nf);
    }
  }
  for (; i < nv; i += stride) {
    const uint4 raw = xv[i];
    const T* v = (const T*)&raw;
#pragma unroll
    for (int e = 0; e < V; e++) mm_update<T>(v[e], mn, mx, nf);
  }
  for (uint64_t k = nv * V + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
    mm_update<T>(x[k], mn, mx, nf);
  uint64_t omn = (sizeof(T) == 4) ? (uint64_t)ord32((float)mn) : ord64((double)mn);
  uint64_t omx = (sizeof(T) == 4) ? (uint64_t)ord32((float)mx) : ord64((double)mx);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint64_t a = __shfl_xor(omn, o, 64), b = __shfl_xor(omx, o, 64);
    omn = a < omn ? a : omn;
    omx = b > omx ? b : omx;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (nf) atomicOr(&lnf, 1u);
  if (lane == 0) {
    lmin[wid] = omn;
    lmax[wid] = omx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; w++) {
      omn = lmin[w] < omn ? lmin[w] : omn;
      omx = lmax[w] > omx ? lmax[w] : omx;
    }
    if (sizeof(T) == 4) {
      atomicMin(&P->minmax_bits[0], (uint32_t)omn);
      atomicMax(&P->minmax_bits[1], (uint32_t)omx);
    } else {
      atomicMin((unsigned long long*)&P->minmax64[0], (unsigned long long)omn);
      atomicMax((unsigned long long*)&P->minmax64[1], (unsigned long long)omx);
    }
    if (lnf) atomicOr(&P->nonfinite, 1u);
  }
}
template <typename T>
__global__ void __launch_bounds__(256) minmax_kernel(const T* __restrict__ x, uint64_t n, DevPlan* P) {
  minmax_kernel_dev<T>(x, n, P);
}


// Error bound in the element type: eb (double) rounded toward zero into T,
// 2eb = eb + eb and 1/(2eb), each one IEEE operation in T (Metric 1).
template <typename T>
__device__ __forceinline__ void eb_resolve_kernel_dev(DevPlan* P, PlanInit I) {
  using U = typename FTr<T>::U;
  if (threadIdx.x != 0 || P->status) return;
  double eb = I.eb_abs;
  if (I.eb_mode != SZ_EB_ABS) {
    if (P->nonfinite) {
      P->status = SZ_ENONFINITE;
      return;
    }
    double lo, hi;
    if (sizeof(T) == 4) {
      lo = (double)unord32(P->minmax_bits[0]);
      hi = (double)unord32(P->minmax_bits[1]);
    } else {
      lo = unord64(P->minmax64[0]);
      hi = unord64(P->minmax64[1]);
    }
    P->vmin = lo;
    P->vmax = hi;
    const double range = hi - lo;
    const double rel = I.eb_rel * range;
    eb = (I.eb_mode == SZ_EB_REL) ? rel : (I.eb_abs < rel ? I.eb_abs : rel);
  }
  const double tmax = (sizeof(T) == 4) ? 3.4028234663852886e38 : 1.7976931348623157e308;
  if (!(eb <= tmax / 4)) {
    P->status = SZ_EINVAL;
    return;
  }
  T e = (T)eb;
  if ((double)e > eb) e = bits_to<T>(to_bits<T>(e) - 1);
  const T two = e + e;
  const T inv = T(1) / two;
  P->eb = (double)e;
  P->ebT_bits = (uint64_t)to_bits<T>(e);
  P->twoeb_bits = (uint64_t)to_bits<T>(two);
  P->inv2eb_bits = (uint64_t)to_bits<T>(inv);
}
template <typename T>
__global__ void eb_resolve_kernel(DevPlan* P, PlanInit I) {
  eb_resolve_kernel_dev<T>(P, I);
}


// Adaptive interval count (Sec. IV-B): from the 2^16-code histogram, the
// smallest m whose intervals |k| <= 2^(m-1) - 1 hold theta * N points.
__device__ __forceinline__ void pick_m_kernel_dev(uint32_t* hist, DevPlan* P, uint64_t n, double theta) {
  __shared__ unsigned long long bucket[17];
  if (P->status) return;
  if (threadIdx.x < 17) bucket[threadIdx.x] = 0;
  __syncthreads();
  for (int i = threadIdx.x + 1; i < 65536; i += blockDim.x) {
    const uint32_t h = hist[i];
    if (!h) continue;
    const int k = i - 32768;
    const uint32_t a = (uint32_t)(k < 0 ? -k : k) + 1u;  // |k| + 1
    // smallest m with a <= 2^(m-1)
    int mk = 1;
    while ((1u << (mk - 1)) < a) mk++;
    atomicAdd(&bucket[mk], (unsigned long long)h);
  }
  __syncthreads();
  __shared__ uint32_t s_m;
  if (threadIdx.x == 0) {
    uint32_t mstar = 16;
    unsigned long long cov = 0;
    for (int m = 1; m <= 16; m++) {
      cov += bucket[m];
      if ((double)cov >= theta * (double)n) {
        mstar = m;
        break;
      }
    }
    s_m = mstar;
    P->m = mstar;
    P->rerun = mstar < 16;
  }
  __syncthreads();
  if (s_m < 16)
    for (int i = threadIdx.x; i < 65536; i += blockDim.x) hist[i] = 0;
}
__global__ void __launch_bounds__(1024) pick_m_kernel(uint32_t* hist, DevPlan* P, uint64_t n, double theta) {
  pick_m_kernel_dev(hist, P, n, theta);
}


// ------------------------------------------------------------ sorting
// Bitonic sort of n (power of two) 64-bit keys held at `k` (LDS or global)
// by one workgroup.
template <int NT>
__device__ void bitonic_sort(uint64_t* k, uint32_t n) {
  for (uint32_t size = 2; size <= n; size <<= 1) {
    for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (uint32_t t = threadIdx.x; t < n / 2; t += NT) {
        const uint32_t lo = 2 * t - (t & (stride - 1));
        const uint32_t hi = lo + stride;
        const bool up = ((lo & size) == 0);
        const uint64_t a = k[lo], b = k[hi];
        if ((a > b) == up) {
          k[lo] = b;
          k[hi] = a;
        }
      }
      __syncthreads();
    }
  }
}

// The same network for n keys in global memory (n a power of two), run by one
// workgroup: the passes whose stride stays inside an aligned chunk of CH keys
// run on that chunk in LDS (`buf`, CH keys), the wider ones as global passes
// that load 8 pairs per thread before comparing.  Directions follow the
// global index, so the result is that of bitonic_sort.
template <int NT>
__device__ void bitonic_sort_big(uint64_t* k, uint32_t n, uint64_t* buf, uint32_t CH) {
  if (n <= CH) {
    for (uint32_t e = threadIdx.x; e < n; e += NT) buf[e] = k[e];
    __syncthreads();
    bitonic_sort<NT>(buf, n);
    for (uint32_t e = threadIdx.x; e < n; e += NT) k[e] = buf[e];
    __syncthreads();
    return;
  }
  // strides size_lo .. 1 of sizes size_lo * 2 .. size_hi, chunk by chunk in LDS
  auto chunks = [&](uint32_t size_first, uint32_t size_last, uint32_t first_stride) {
    for (uint32_t c0 = 0; c0 < n; c0 += CH) {
      for (uint32_t e = threadIdx.x; e < CH; e += NT) buf[e] = k[c0 + e];
      __syncthreads();
      for (uint32_t size = size_first; size <= size_last; size <<= 1) {
        for (uint32_t stride = min(size >> 1, first_stride); stride > 0; stride >>= 1) {
          for (uint32_t t = threadIdx.x; t < CH / 2; t += NT) {
            const uint32_t lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
            const bool up = (((c0 + lo) & size) == 0);
            const uint64_t a = buf[lo], b = buf[hi];
            if ((a > b) == up) {
              buf[lo] = b;
              buf[hi] = a;
            }
          }
          __syncthreads();
        }
      }
      for (uint32_t e = threadIdx.x; e < CH; e += NT) k[c0 + e] = buf[e];
      __syncthreads();
    }
  };
  chunks(2, CH, CH);
  for (uint32_t size = 2 * CH; size <= n; size <<= 1) {
    for (uint32_t stride = size >> 1; stride >= CH; stride >>= 1) {
      constexpr int B = 8;
      for (uint32_t t0 = threadIdx.x; t0 < n / 2; t0 += NT * B) {
        uint64_t a[B], b[B];
        uint32_t lo[B];
#pragma unroll
        for (int u = 0; u < B; u++) {
          const uint32_t t = t0 + u * NT;
          lo[u] = 2 * t - (t & (stride - 1));
          a[u] = t < n / 2 ? k[lo[u]] : 0;
          b[u] = t < n / 2 ? k[lo[u] + stride] : 0;
        }
#pragma unroll
        for (int u = 0; u < B; u++) {
          const uint32_t t = t0 + u * NT;
          const bool up = ((lo[u] & size) == 0);
          if (t < n / 2 && (a[u] > b[u]) == up) {
            k[lo[u]] = b[u];
            k[lo[u] + stride] = a[u];
          }
        }
      }
      __syncthreads();
    }
    chunks(size, size, CH >> 1);
  }
}

constexpr int kCbNT = 1024;
constexpr int kCbNW = kCbNT / 64;
constexpr uint32_t kCbLdsSyms = 2048;
// Rounds of the parallel construction: the lightest available weight at
// least doubles per round and all weights sum to N < 2^40, so 41 suffice.
constexpr int kCbMaxRounds = 96;
constexpr int kCbBatch = 8;  // key loads a sort thread keeps in flight

// Entries of the nondecreasing sequence get(lo .. hi-1) below x (LE: not
// above x), by binary search.
template <bool LE, typename G>
__device__ __forceinline__ uint32_t cb_count(const G& get, uint32_t lo, uint32_t hi, uint64_t x) {
  uint32_t l = lo, h = hi;
  while (l < h) {
    const uint32_t mid = (l + h) >> 1;
    const uint64_t v = get(mid);
    if (LE ? (v <= x) : (v < x))
      l = mid + 1;
    else
      h = mid;
  }
  return l - lo;
}

// Stable LSD radix sort, by the frequency field, of n keys (frequency << 16
// | symbol) given in symbol order, so they end in (frequency, symbol) order
// in k.  One workgroup, 8-bit digits, as many passes as the largest
// frequency needs.  Each wave owns a contiguous segment of the keys and
// places them in order: a key's rank among the keys of its 64-key batch
// with the same digit comes from eight ballots, and the last of them moves
// the wave's offset for that digit on, so every pass keeps the order of
// equal digits.
__device__ void cb_radix_sort(uint64_t* k, uint64_t* tmp, uint32_t n, uint32_t* cnt, uint32_t* off,
                              uint32_t* red, uint32_t* s_max, uint32_t mx) {
  // mx: the largest frequency among the keys this thread wrote
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int o = 32; o >= 1; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
  if (tid == 0) *s_max = 0;
  __syncthreads();
  if (lane == 0) atomicMax(s_max, mx);
  __syncthreads();
  const int nbits = 32 - __clz(*s_max | 1u);
  const uint32_t seg = (n + kCbNW - 1) / kCbNW;
  const uint32_t s0 = min(n, (uint32_t)w * seg), s1 = min(n, s0 + seg);
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  uint64_t* src = k;
  uint64_t* dst = tmp;
  for (int shift = 16; shift < 16 + nbits; shift += 8) {
    for (int e = tid; e < kCbNW * 256; e += kCbNT) cnt[e] = 0;
    __syncthreads();
    for (uint32_t i0 = s0; i0 < s1; i0 += 64 * kCbBatch) {
      uint64_t kb[kCbBatch];
#pragma unroll
      for (int u = 0; u < kCbBatch; u++) kb[u] = i0 + 64 * u + lane < s1 ? src[i0 + 64 * u + lane] : 0ull;
#pragma unroll
      for (int u = 0; u < kCbBatch; u++) {
        const bool ok = i0 + 64 * u + lane < s1;
        const uint32_t d = (uint32_t)((kb[u] >> shift) & 255);
        // the high digits of small frequencies are all 0: a batch of one
        // digit is one add, not 64 adds to one address
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const uint64_t okm = __ballot(ok);  // (a ballot inside the lane-0 branch would see lane 0 only)
        if (__ballot(ok && d != d0) == 0) {
          if (lane == 0 && ok) atomicAdd(&cnt[w * 256 + d0], (uint32_t)__popcll(okm));
        } else if (ok) {
          atomicAdd(&cnt[w * 256 + d], 1u);
        }
      }
    }
    __syncthreads();
    // exclusive scan in (digit, wave) order: element e = digit * kCbNW + wave
    static_assert(kCbNW * 256 == 4 * kCbNT, "four scan elements per thread");
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = 4 * tid + q;
      v[q] = cnt[(e % kCbNW) * 256 + e / kCbNW];
      sum += v[q];
    }
    uint32_t base = block_exscan<kCbNT, uint32_t>(sum, red, nullptr);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = 4 * tid + q;
      off[(e % kCbNW) * 256 + e / kCbNW] = base;
      base += v[q];
    }
    __syncthreads();
    uint64_t kb[kCbBatch];
    for (uint32_t i0 = s0; i0 < s1; i0 += 64) {
      const uint32_t i = i0 + lane;
      const bool ok = i < s1;
      // the next kCbBatch batches are loaded together (src and dst differ)
      const uint32_t u = ((i0 - s0) / 64) % kCbBatch;
      if (u == 0) {
#pragma unroll
        for (int q = 0; q < kCbBatch; q++) kb[q] = i + 64 * q < s1 ? src[i + 64 * q] : 0ull;
      }
      uint64_t key = kb[0];
#pragma unroll
      for (int q = 1; q < kCbBatch; q++) key = u == (uint32_t)q ? kb[q] : key;
      const uint32_t d = (uint32_t)((key >> shift) & 255);
      uint64_t peers = __ballot(ok);
#pragma unroll
      for (int b = 0; b < 8; b++) {
        const uint64_t bb = __ballot(ok && ((d >> b) & 1u));
        peers &= ((d >> b) & 1u) ? bb : ~bb;
      }
      if (ok) {
        const uint32_t pos = off[w * 256 + d] + (uint32_t)__popcll(peers & below);
        dst[pos] = key;
        // the highest lane of each digit group moves the offset on
        if ((peers >> lane) == 1ull) off[w * 256 + d] = pos + 1;
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    uint64_t* t = src;
    src = dst;
    dst = t;
  }
  if (src != k) {
    for (uint32_t i = tid; i < n; i += kCbNT) k[i] = src[i];
    __syncthreads();
  }
}

// Stable counting of items 0..n-1 by a code length (1..27; 0 = no item):
// emit(i, base[len] + the number of earlier items of the same length).  One
// workgroup of NT threads; each wave takes a contiguous segment of the
// items, counts its lengths, and after a prefix over the waves ranks the
// items of each 64-item batch among their equal lengths with five ballots.
// `lc` is NT/64 x 32 words of LDS.
template <int NT, typename G, typename E>
__device__ __forceinline__ void rank_by_length(uint32_t n, const G& get_len, const uint32_t* base,
                                               uint32_t (*lc)[32], const E& emit) {
  constexpr int NWV = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < NWV * 32; e += NT) (&lc[0][0])[e] = 0;
  __syncthreads();
  const uint32_t sg = (n + NWV - 1) / NWV;
  const uint32_t g0 = min(n, (uint32_t)wv * sg), g1 = min(n, g0 + sg);
  for (uint32_t q0 = g0; q0 < g1; q0 += 64) {
    // a few lengths take most items: each length present is added once
    const uint32_t q = q0 + lane;
    const uint32_t l = q < g1 ? get_len(q) : 0u;
    const uint64_t peers = wave_peers<5>(l != 0, l);
    if (l && peers_last(peers)) lc[wv][l] += (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  if (tid >= 1 && tid < 32) {
    uint32_t c0 = base[tid];
    for (int ww = 0; ww < NWV; ww++) {
      const uint32_t cl = lc[ww][tid];
      lc[ww][tid] = c0;
      c0 += cl;
    }
  }
  __syncthreads();
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (uint32_t q0 = g0; q0 < g1; q0 += 64) {
    const uint32_t q = q0 + lane;
    const uint32_t l = q < g1 ? get_len(q) : 0u;
    uint64_t peers = __ballot(l != 0);
#pragma unroll
    for (int b = 0; b < 5; b++) {
      const uint64_t bb = __ballot(l != 0 && ((l >> b) & 1u));
      peers &= ((l >> b) & 1u) ? bb : ~bb;
    }
    if (l) {
      const uint32_t r = lc[wv][l] + (uint32_t)__popcll(peers & below);
      emit(q, r);
      if ((peers >> lane) == 1ull) lc[wv][l] = r + 1;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
}

// --------------------------------------------------- K4: Huffman codebook
struct CodebookArgs {
  const uint32_t* hist;
  uint8_t* len;        // 2^m
  uint32_t* cw;        // 2^m
  uint64_t* gkeys;     // 65536 (leaves)
  uint64_t* gw;        // 131072 (sort buffer, then internal-node weights)
  uint32_t* gpar;      // 131072 (parent of every node)
  uint32_t* ganc;      // 262144 (merge-order weights of a round, as 131072 u64)
  uint32_t* gdep;      // 262144 (merge-order node ids of a round; node depths)
  DevPlan* plan;
  uint64_t n;
  double theta;
};

// Code lengths of the two-queue construction over the leaves sorted by
// (frequency, symbol), the leaf queue winning ties (the oracle's definition),
// computed in rounds rather than one merge at a time.  Both queues are
// sorted and an internal node outweighs what it joins, so the order in
// which the construction consumes nodes is the merge of the two queues, and
// internal node c joins the nodes at places 2c and 2c + 1 of that order.
// A round starts from the two lightest available nodes, whose sum t is the
// weight of the next internal node; every node made from then on weighs at
// least t and every available internal node weighs at most t, so all
// available internal nodes and all leaves not heavier than t are consumed
// first, in merge order (a leaf before an internal node of equal weight, an
// older internal node before a newer one).  The round places those K nodes
// by binary searches in the other queue, joins them pairwise into new
// internal nodes and, when K is odd, joins the last with the first new node.
// Depths follow top-down, round by round in reverse.  Lengths above 27 are
// repaired by halving every frequency (keeping it >= 1) and rebuilding, as
// the oracle does.  Canonical codes follow in (length, symbol) order.
__device__ __forceinline__ void codebook_kernel_dev(CodebookArgs A) {
  DevPlan* P = A.plan;
  if (P->status) return;
  __shared__ uint64_t s_keys[kCbLdsSyms];
  __shared__ uint64_t s_w[2 * kCbLdsSyms];
  __shared__ uint32_t s_par[2 * kCbLdsSyms];
  __shared__ uint32_t s_dep[2 * kCbLdsSyms];
  __shared__ uint32_t s_mid[2 * kCbLdsSyms];
  __shared__ uint32_t s_red[64];
  __shared__ uint32_t s_rs[kCbMaxRounds + 1];
  __shared__ uint32_t s_lc[kCbNW][32];
  __shared__ uint64_t s_t;
  __shared__ uint32_t s_a, s_b, s_c, s_nr, s_maxd, s_first[32];

  const uint32_t m = P->m;
  const uint32_t nsym = 1u << m;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // used symbols, in symbol order
  const uint32_t per = (nsym + kCbNT - 1) / kCbNT;
  const uint32_t lo = min(nsym, tid * per), hi = min(nsym, lo + per);
  uint32_t cnt = 0;
  for (uint32_t q = lo; q < hi; q++) cnt += A.hist[q] != 0;
  uint32_t total;
  const uint32_t pos0 = block_exscan<kCbNT, uint32_t>(cnt, s_red, &total);
  const uint32_t s = total;
  for (uint32_t q = lo; q < hi; q++) A.len[q] = 0;

  if (s == 1) {
    __syncthreads();
    for (uint32_t q = lo; q < hi; q++)
      if (A.hist[q]) {
        A.len[q] = 1;
        A.cw[q] = 1u << 27;
      }
    if (tid == 0) {
      P->n_used = 1;
      P->max_len = 1;
    }
  } else if (s > 1) {
    // The construction takes its arrays as arguments so that, called with
    // the LDS arrays, every access compiles to LDS instructions.
    auto build = [&](uint64_t* K, uint64_t* IW, uint64_t* MW, uint32_t* MID, uint32_t* PAR, uint32_t* DEP,
                     bool lds) {
      uint32_t np2 = 1;
      while (np2 < s) np2 <<= 1;
      uint32_t kmax = 0;  // this thread's largest leaf frequency
      for (int halvings = 0; halvings < 64; halvings++) {
        // leaves with frequencies max(1, f >> halvings), in symbol order
        {
          uint32_t pos = pos0;
          kmax = 0;
          for (uint32_t q = lo; q < hi; q++) {
            const uint32_t f = A.hist[q];
            const uint32_t fh = max(1u, f >> min(halvings, 31));
            if (f) K[pos++] = ((uint64_t)fh << 16) | q;
            if (f) kmax = max(kmax, fh);
          }
          if (lds)
            for (uint32_t i = s + tid; i < np2; i += kCbNT) K[i] = ~0ull;
          __syncthreads();
        }
        if (lds)
          bitonic_sort<kCbNT>(K, np2);
        else
          cb_radix_sort(K, IW, s, s_mid, s_dep, s_red, &s_maxd, kmax);
        // rounds
        if (tid == 0) {
          s_a = 0;
          s_b = 0;
          s_c = 0;
          s_nr = 0;
        }
        __syncthreads();
        for (;;) {
          const uint32_t a = s_a, b = s_b, c = s_c, nr = s_nr;
          if ((s - a) + (c - b) <= 1 || nr >= (uint32_t)kCbMaxRounds) break;
          if (tid == 0) {
            // the two lightest available nodes, in merge order
            uint32_t i = a, j = b;
            uint64_t t = 0;
            for (int q = 0; q < 2; q++) {
              if (i < s && (j >= c || (K[i] >> 16) <= IW[j]))
                t += K[i++] >> 16;
              else
                t += IW[j++];
            }
            s_t = t;
            s_rs[nr] = c;
          }
          __syncthreads();
          const uint64_t t = s_t;
          // leaves of weight <= t (a prefix of the remaining leaves)
          uint32_t kl = 0;
          for (uint32_t base = a; base < s; base += kCbNT) {
            const uint32_t i = base + tid;
            const int cntc = __syncthreads_count(i < s && (K[i] >> 16) <= t);
            kl += (uint32_t)cntc;
            if (cntc < kCbNT) break;
          }
          const uint32_t kk = kl + (c - b);
          // merge places: a leaf after the internal nodes lighter than it; an
          // internal node after the leaves not heavier than it
          for (uint32_t i = a + tid; i < a + kl; i += kCbNT) {
            const uint64_t f = K[i] >> 16;
            const uint32_t p = (i - a) + cb_count<false>([&](uint32_t x) { return IW[x]; }, b, c, f);
            MW[p] = f;
            MID[p] = i;
          }
          for (uint32_t j = b + tid; j < c; j += kCbNT) {
            const uint64_t wj = IW[j];
            const uint32_t p = (j - b) + cb_count<true>([&](uint32_t x) { return K[x] >> 16; }, a, a + kl, wj);
            MW[p] = wj;
            MID[p] = s + j;
          }
          __syncthreads();
          const uint32_t npair = kk / 2;
          for (uint32_t q = tid; q < npair; q += kCbNT) {
            IW[c + q] = MW[2 * q] + MW[2 * q + 1];
            PAR[MID[2 * q]] = s + c + q;
            PAR[MID[2 * q + 1]] = s + c + q;
          }
          if ((kk & 1) && tid == 0) {
            // the last node joins the first new one, the lightest left
            IW[c + npair] = MW[kk - 1] + (MW[0] + MW[1]);
            PAR[MID[kk - 1]] = s + c + npair;
            PAR[s + c] = s + c + npair;
          }
          __syncthreads();
          if (tid == 0) {
            s_a = a + kl;
            s_b = c + (kk & 1);
            s_c = c + npair + (kk & 1);
            s_nr = nr + 1;
          }
          __syncthreads();
        }
        const uint32_t nr = s_nr, cend = s_c;
        if (nr >= (uint32_t)kCbMaxRounds) {
          if (tid == 0) set_status(P, SZ_EINVAL);
          return;
        }
        // depths, top-down: the root, then the rounds in reverse; within a
        // round only its first node can hang below its last
        if (tid == 0) {
          s_rs[nr] = cend;
          DEP[s + cend - 1] = 0;
        }
        __syncthreads();
        for (int r = (int)nr - 1; r >= 0; r--) {
          const uint32_t r0 = s_rs[r], r1 = s_rs[r + 1];
          if (tid == 0 && r1 - 1 != cend - 1) DEP[s + r1 - 1] = DEP[PAR[s + r1 - 1]] + 1;
          __syncthreads();
          if (lds) {
            for (uint32_t v = r0 + tid; v + 1 < r1; v += kCbNT) DEP[s + v] = DEP[PAR[s + v]] + 1;
          } else {
            for (uint32_t v0 = r0 + tid; v0 + 1 < r1; v0 += kCbNT * kCbBatch) {
              // a round's nodes hang below later rounds only (its last node,
              // the one its first may hang below, is set above), so the
              // parents of kCbBatch nodes are loaded together
              uint32_t pa[kCbBatch], dd[kCbBatch];
#pragma unroll
              for (int u = 0; u < kCbBatch; u++) pa[u] = v0 + u * kCbNT + 1 < r1 ? PAR[s + v0 + u * kCbNT] : 0u;
#pragma unroll
              for (int u = 0; u < kCbBatch; u++) dd[u] = v0 + u * kCbNT + 1 < r1 ? DEP[pa[u]] + 1 : 0u;
#pragma unroll
              for (int u = 0; u < kCbBatch; u++)
                if (v0 + u * kCbNT + 1 < r1) DEP[s + v0 + u * kCbNT] = dd[u];
            }
          }
          __syncthreads();
        }
        uint32_t md = 0;
        if (lds) {
          for (uint32_t i = tid; i < s; i += kCbNT) {
            const uint32_t d = DEP[PAR[i]] + 1;
            DEP[i] = d;
            md = max(md, d);
          }
        } else {
          for (uint32_t i0 = tid; i0 < s; i0 += kCbNT * kCbBatch) {
            // leaves read internal depths only: kCbBatch parents loaded together
            uint32_t pa[kCbBatch], dd[kCbBatch];
#pragma unroll
            for (int u = 0; u < kCbBatch; u++) pa[u] = i0 + u * kCbNT < s ? PAR[i0 + u * kCbNT] : 0u;
#pragma unroll
            for (int u = 0; u < kCbBatch; u++) dd[u] = i0 + u * kCbNT < s ? DEP[pa[u]] + 1 : 0u;
#pragma unroll
            for (int u = 0; u < kCbBatch; u++)
              if (i0 + u * kCbNT < s) {
                DEP[i0 + u * kCbNT] = dd[u];
                md = max(md, dd[u]);
              }
          }
        }
        for (int o = 32; o >= 1; o >>= 1) md = max(md, (uint32_t)__shfl_xor(md, o, 64));
        if (tid == 0) s_maxd = 0;
        __syncthreads();
        if (lane == 0) atomicMax(&s_maxd, md);
        __syncthreads();
        const uint32_t maxd = s_maxd;
        if (maxd <= (uint32_t)kLmax) {
          for (uint32_t i = tid; i < s; i += kCbNT) A.len[K[i] & 0xFFFF] = (uint8_t)DEP[i];
          if (tid == 0) {
            P->n_used = s;
            P->max_len = maxd;
          }
          break;
        }
        __syncthreads();
      }
    };
    if (s <= kCbLdsSyms)
      build(s_keys, s_w, s_w + kCbLdsSyms, s_mid, s_par, s_dep, true);
    else
      build(A.gkeys, A.gw, (uint64_t*)A.ganc, A.gdep, A.gpar, A.gdep + 131072, false);
    __syncthreads();
    // canonical codes in (length, symbol) order: the first code of each
    // length, then each symbol's rank among the symbols of its length
    if (tid < 32) s_first[tid] = 0;
    __syncthreads();
    for (uint32_t q = tid; q < nsym; q += kCbNT) {
      const uint32_t l = A.len[q];
      if (l) atomicAdd(&s_first[l], 1u);
    }
    __syncthreads();
    if (tid == 0) {
      uint32_t code = 0;
      for (int l = 1; l <= kLmax; l++) {
        const uint32_t cl = s_first[l];
        s_first[l] = code;
        code = (code + cl) << 1;
      }
    }
    __syncthreads();
    rank_by_length<kCbNT>(
        nsym, [&](uint32_t q) { return (uint32_t)A.len[q]; }, s_first, s_lc,
        [&](uint32_t q, uint32_t code) { A.cw[q] = ((uint32_t)A.len[q] << 27) | code; });
  }
  if (tid == 0) {
    const double hr = 1.0 - (double)A.hist[0] / (double)A.n;
    P->m_suggested = (hr < A.theta && m < 16) ? m + 1 : m;
  }
}
__global__ void __launch_bounds__(kCbNT) codebook_kernel(CodebookArgs A) {
  codebook_kernel_dev(A);
}


// ---------------------------------------------------------- bit helpers
// Stream bit b sits in word b/32 at bit 31 - b%32 (MSB first).
__device__ __forceinline__ void or_bits(uint32_t* words, uint64_t pos, uint64_t val, int nb) {
  // nb <= 57
  while (nb > 0) {
    const uint64_t w = pos >> 5;
    const int off = (int)(pos & 31);
    const int take = min(nb, 32 - off);
    const uint32_t chunk = (uint32_t)((val >> (nb - take)) & ((1ull << take) - 1));
    atomicOr(&words[w], chunk << (32 - off - take));
    pos += take;
    nb -= take;
  }
}

__device__ __forceinline__ uint64_t read_bits(const uint32_t* words, uint64_t nwords, uint64_t pos, int nb) {
  uint64_t v = 0;
  while (nb > 0) {
    const uint64_t w = pos >> 5;
    const int off = (int)(pos & 31);
    const int take = min(nb, 32 - off);
    const uint32_t word = (w < nwords) ? words[w] : 0u;
    v = (v << take) | ((word >> (32 - off - take)) & (uint32_t)((1ull << take) - 1));
    pos += take;
    nb -= take;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ int kept_bits(T x, typename FTr<T>::U ebT_bits) {
  using U = typename FTr<T>::U;
  constexpr int MANT = FTr<T>::MANT, EMAX = FTr<T>::EMAX;
  const int e = (int)((to_bits<T>(x) >> MANT) & (U)EMAX);
  const int e_eb = (int)((ebT_bits >> MANT) & (U)EMAX);
  if (e_eb == 0 || e == EMAX) return MANT;
  if (e == 0 || e < e_eb) return 0;
  return min(e - e_eb, MANT);
}

// ------------------------------------------------- K5a: per-chunk totals
// One wave per chunk of C symbols (C a multiple of 256): lane l takes the
// C/64 consecutive symbols starting at l*C/64, loaded as 16-byte vectors.
// Wave-wide sums and scans of u32 by DPP lane moves: row shifts by 1, 2, 4
// and 8 give the inclusive scan of each 16-lane row (lanes shifted in from
// outside the row read 0), then row broadcasts of lanes 15 and 31 carry the
// row totals into the later rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_move(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}
__device__ __forceinline__ uint32_t wave_inscan(uint32_t v) {
  v += dpp_move<0x111, 0xF>(v);  // row_shr:1
  v += dpp_move<0x112, 0xF>(v);  // row_shr:2
  v += dpp_move<0x114, 0xF>(v);  // row_shr:4
  v += dpp_move<0x118, 0xF>(v);  // row_shr:8
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readlane((int)wave_inscan(v), 63);
}
__device__ __forceinline__ uint32_t wave_exscan(uint32_t v) { return wave_inscan(v) - v; }

// ------------------------------------------------ K3: code histogram
// Histogram of the codes of a sweep (the wave-tiled sweep writes codes
// only).  With 1-byte codes (m <= 8) every bin lives in LDS, in 32 copies
// (one per lane pair of a wave, rows padded to 257 words so the copies of
// one bin sit in different banks), and every code is one LDS add without a
// branch: the codes at and next to the centre are the frequent ones, and
// lanes that add to one bin in one copy would serialise.  With 2-byte codes
// the centre and zero codes, the most frequent ones, are counted in
// registers.  With 2-byte codes a window of up to 16384 bins around the
// centre lives in LDS and codes outside it go straight to global atomics.
// A block's counts reach the histogram by atomics, or, with 1-byte codes and
// a partials array `hpart` (kHistBlocks rows of 256 bins), by plain stores
// of its row that hist_reduce_kernel then adds up in a fixed order: the
// atomics of every block onto the same few cache lines would serialise.
constexpr uint32_t kHistLds = 16384;
constexpr uint32_t kHistCopies = 32, kHistRow = 257;
constexpr uint32_t kHistBlocks = 512;  // grid of the 1-byte path with partials

template <typename CT>
__device__ __forceinline__ void hist_kernel_dev(const CT* __restrict__ codes, uint64_t n, uint32_t* hist,
                                                    const DevPlan* P, uint32_t pass2, uint32_t* hpart) {
  __shared__ uint32_t h[sizeof(CT) == 1 ? kHistCopies * kHistRow : kHistLds];
  if (P->status) return;
  if (pass2 && !P->rerun) return;
  const uint32_t m = P->m;
  const uint32_t nb = 1u << m, half = 1u << (m - 1);
  constexpr bool kCopies = sizeof(CT) == 1;  // nb <= 256
  const uint32_t W = kCopies ? nb : (nb < kHistLds ? nb : kHistLds);
  const uint32_t wbase = (!kCopies && nb > W) ? half - W / 2 : 0;
  const uint32_t clear = kCopies ? kHistCopies * kHistRow : W;
  for (uint32_t i = threadIdx.x; i < clear; i += 1024) h[i] = 0;
  __syncthreads();
  uint32_t* hc = kCopies ? h + (threadIdx.x & (kHistCopies - 1)) * kHistRow : h;  // this lane's copy
  uint32_t c_center = 0, c_zero = 0;
  auto count = [&](uint32_t code) {
    if constexpr (kCopies) {
      atomicAdd(&hc[code], 1u);  // every 1-byte code has a bin in the row
    } else if (code == half) {
      c_center++;
    } else if (code == 0) {
      c_zero++;
    } else {
      const uint32_t w = code - wbase;
      if (w < W)
        atomicAdd(&hc[w], 1u);
      else
        atomicAdd(&hist[code], 1u);
    }
  };
  constexpr int E = 16 / sizeof(CT);
  constexpr int U = 4;  // 16-byte loads in flight per thread
  const uint64_t nv = n / E;
  const uint64_t stride = (uint64_t)gridDim.x * 1024;
  auto count_vec = [&](const uint4 raw) {
    const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
    for (int e = 0; e < E; e++) {
      const uint32_t word = wd[e / (E / 4)];
      const int sh = (e % (E / 4)) * 8 * (int)sizeof(CT);
      count((word >> sh) & ((sizeof(CT) == 1) ? 0xFFu : 0xFFFFu));
    }
  };
  uint64_t v = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
  for (; v + (U - 1) * stride < nv; v += U * stride) {
    uint4 raw[U];
#pragma unroll
    for (int u = 0; u < U; u++) raw[u] = ((const uint4*)codes)[v + u * stride];
#pragma unroll
    for (int u = 0; u < U; u++) count_vec(raw[u]);
  }
  for (; v < nv; v += stride) count_vec(((const uint4*)codes)[v]);
  for (uint64_t i = nv * E + (uint64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += stride) count(codes[i]);
  c_center = wave_sum(c_center);
  c_zero = wave_sum(c_zero);
  const bool rows = kCopies && hpart != nullptr;
  if ((threadIdx.x & 63) == 0) {
    if (c_center) atomicAdd(&h[half - wbase], c_center);
    if (c_zero) {
      if (rows)
        atomicAdd(&h[0], c_zero);
      else
        atomicAdd(&hist[0], c_zero);
    }
  }
  __syncthreads();
  if (rows) {
    for (uint32_t i = threadIdx.x; i < 256; i += 1024) {
      uint32_t t = 0;
      if (i < W)
        for (uint32_t c = 0; c < kHistCopies; c++) t += h[c * kHistRow + i];
      hpart[(size_t)blockIdx.x * 256 + i] = t;
    }
    return;
  }
  for (uint32_t i = threadIdx.x; i < W; i += 1024) {
    uint32_t t = h[i];
    if constexpr (kCopies)
      for (uint32_t c = 1; c < kHistCopies; c++) t += h[c * kHistRow + i];
    if (t) atomicAdd(&hist[wbase + i], t);
  }
}

// Bins of the 1-byte histogram from the per-block rows: one block per bin,
// thread t adding rows t, t + 256, ... in order, then a fixed tree.
__global__ void __launch_bounds__(256) hist_reduce_kernel(const uint32_t* __restrict__ hpart, uint32_t rows,
                                                          uint32_t* hist, const DevPlan* P, uint32_t pass2) {
  __shared__ uint32_t red[4];
  if (P->status) return;
  if (pass2 && !P->rerun) return;
  const uint32_t bin = blockIdx.x;
  uint32_t t = 0;
  for (uint32_t r = threadIdx.x; r < rows; r += 256) t += hpart[(size_t)r * 256 + bin];
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) hist[bin] = red[0] + red[1] + red[2] + red[3];
}
template <typename CT>
__global__ void __launch_bounds__(1024) hist_kernel(const CT* __restrict__ codes, uint64_t n, uint32_t* hist,
                                                    const DevPlan* P, uint32_t pass2, uint32_t* hpart) {
  hist_kernel_dev<CT>(codes, n, hist, P, pass2, hpart);
}


// Histogram of 2-byte codes (m > 8) without global atomics: the bins are
// split into two halves of 32768, and each half is counted by blocks of its
// own (blockIdx.y) holding the whole half in LDS (128 KiB, dynamic), so
// every code lands in an LDS bin of exactly one block.  The zero and centre
// codes, the most frequent ones, are counted in registers.  Each block
// stores its row of counts with plain stores; hist2_reduce_kernel adds the
// rows of every bin in a fixed order.
constexpr uint32_t kHist2Half = 32768;
constexpr uint32_t kHist2MaxBlocks = 256;  // blocks per half
__host__ __device__ constexpr uint32_t hist2_blocks(uint64_t n) {
  return (uint32_t)(n / 65536 + 1 < kHist2MaxBlocks ? n / 65536 + 1 : kHist2MaxBlocks);
}
__global__ void __launch_bounds__(1024) hist2_kernel(const uint16_t* __restrict__ codes, uint64_t n,
                                                     uint32_t* __restrict__ hpart, const DevPlan* P,
                                                     uint32_t pass2) {
  extern __shared__ uint32_t h2[];
  if (P->status) return;
  if (pass2 && !P->rerun) return;
  const uint32_t m = P->m;
  const uint32_t nb = 1u << m, center = 1u << (m - 1);
  const uint32_t lo = blockIdx.y * kHist2Half;
  const uint32_t W = nb > lo ? min(nb - lo, kHist2Half) : 0u;
  uint32_t* row = hpart + ((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kHist2Half;
  if (W == 0) return;  // this half holds no bins at this m
  for (uint32_t i = threadIdx.x; i < W; i += 1024) h2[i] = 0;
  __syncthreads();
  uint32_t c_center = 0, c_zero = 0;
  auto count = [&](uint32_t code) {
    if (code == center) {
      c_center++;
    } else if (code == 0) {
      c_zero++;
    } else {
      const uint32_t w = code - lo;
      if (w < W) atomicAdd(&h2[w], 1u);
    }
  };
  auto count_vec = [&](const uint4 raw) {
    const uint32_t wd[4] = {raw.x, raw.y, raw.z, raw.w};
#pragma unroll
    for (int e = 0; e < 4; e++) {
      count(wd[e] & 0xFFFFu);
      count(wd[e] >> 16);
    }
  };
  constexpr int U = 4;  // 16-byte loads in flight per thread
  const uint64_t nv = n / 8;
  const uint64_t stride = (uint64_t)gridDim.x * 1024;
  uint64_t v = (uint64_t)blockIdx.x * 1024 + threadIdx.x;
  for (; v + (U - 1) * stride < nv; v += U * stride) {
    uint4 raw[U];
#pragma unroll
    for (int u = 0; u < U; u++) raw[u] = ((const uint4*)codes)[v + u * stride];
#pragma unroll
    for (int u = 0; u < U; u++) count_vec(raw[u]);
  }
  for (; v < nv; v += stride) count_vec(((const uint4*)codes)[v]);
  for (uint64_t i = nv * 8 + (uint64_t)blockIdx.x * 1024 + threadIdx.x; i < n; i += stride) count(codes[i]);
  c_center = wave_sum(c_center);
  c_zero = wave_sum(c_zero);
  if ((threadIdx.x & 63) == 0) {
    if (c_center && center - lo < W) atomicAdd(&h2[center - lo], c_center);
    if (c_zero && lo == 0) atomicAdd(&h2[0], c_zero);
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < W; i += 1024) row[i] = h2[i];
}
// Bin b of the 2-byte histogram: the rows of its half added up (integer
// sums: exact in any order).  A block of 1024 threads takes 256 bins, four
// threads per bin over every fourth row, eight loads in flight each.
__global__ void __launch_bounds__(1024) hist2_reduce_kernel(const uint32_t* __restrict__ hpart, uint32_t rows,
                                                            uint32_t* hist, const DevPlan* P, uint32_t pass2) {
  __shared__ uint32_t part[4][256];
  if (P->status) return;
  if (pass2 && !P->rerun) return;
  const uint32_t nb = 1u << P->m;
  const uint32_t q = threadIdx.x >> 8, bl = threadIdx.x & 255;
  const uint32_t b = blockIdx.x * 256 + bl;
  uint32_t t = 0;
  if (b < nb) {
    const uint32_t half = b / kHist2Half, w = b % kHist2Half;
    const uint32_t* col = hpart + (size_t)half * rows * kHist2Half + w;
    uint32_t r = q;
    for (; r + 28 < rows; r += 32) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; u++) v[u] = col[(size_t)(r + 4 * u) * kHist2Half];
#pragma unroll
      for (int u = 0; u < 8; u++) t += v[u];
    }
    for (; r < rows; r += 4) t += col[(size_t)r * kHist2Half];
  }
  part[q][bl] = t;
  __syncthreads();
  if (q == 0 && b < 65536) hist[b] = b < nb ? part[0][bl] + part[1][bl] + part[2][bl] + part[3][bl] : 0u;
}

// Four consecutive codes starting at i (a multiple of 4), as one 4- or
// 8-byte load; codes at or past n read as 0.
template <typename CT>
__device__ __forceinline__ void load4(const CT* __restrict__ codes, uint64_t i, uint64_t n, uint32_t (&o)[4]) {
  if (i + 4 <= n) {
    if constexpr (sizeof(CT) == 1) {
      const uint32_t w = *(const uint32_t*)(codes + i);
      o[0] = w & 0xFF;
      o[1] = (w >> 8) & 0xFF;
      o[2] = (w >> 16) & 0xFF;
      o[3] = w >> 24;
    } else {
      const uint2 w = *(const uint2*)(codes + i);
      o[0] = w.x & 0xFFFF;
      o[1] = w.x >> 16;
      o[2] = w.y & 0xFFFF;
      o[3] = w.y >> 16;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++) o[k] = (i + k < n) ? (uint32_t)codes[i + k] : 0u;
  }
}

// Code lengths (and codewords) live in LDS when the alphabet is small.
constexpr uint32_t kTabLds = 4096;

// Stage chunk c's codes into the wave's LDS buffer with 16-byte coalesced
// loads (codes past n read as 0); returns the number of real codes.
template <typename CT>
__device__ __forceinline__ uint32_t stage_codes(const CT* __restrict__ codes, uint64_t n, uint64_t c, uint32_t C,
                                                CT* sc, int lane) {
  const uint64_t i0 = c * C;
  const uint32_t cnt = (uint32_t)min((uint64_t)C, n - i0);
  constexpr uint32_t E = 16 / sizeof(CT);
  if (cnt == C) {
    // C is a multiple of 256 and codes are 16-byte aligned, so the chunk is
    // whole 16-byte vectors
    const uint4* src = (const uint4*)(codes + i0);
    uint4* dst = (uint4*)sc;
    const uint32_t nv = C / E;
#pragma unroll 4
    for (uint32_t v = lane; v < nv; v += 64) dst[v] = src[v];
  } else {
    for (uint32_t k = lane; k < C; k += 64) sc[k] = (k < cnt) ? codes[i0 + k] : (CT)0;
  }
  __builtin_amdgcn_wave_barrier();
  return cnt;
}

// Four codes from LDS starting at k (a multiple of 4).
template <typename CT>
__device__ __forceinline__ void lds_code4(const CT* sc, uint32_t k, uint32_t (&o)[4]) {
  if constexpr (sizeof(CT) == 1) {
    const uint32_t w = *(const uint32_t*)(sc + k);
    o[0] = w & 0xFF;
    o[1] = (w >> 8) & 0xFF;
    o[2] = (w >> 16) & 0xFF;
    o[3] = w >> 24;
  } else {
    const uint2 w = *(const uint2*)(sc + k);
    o[0] = w.x & 0xFFFF;
    o[1] = w.x >> 16;
    o[2] = w.y & 0xFFFF;
    o[3] = w.y >> 16;
  }
}

// Code length of symbol s: from the LDS table (len << 27 | code) when LT,
// else from the global length array.
template <bool LT>
__device__ __forceinline__ uint32_t code_entry(uint32_t s, const uint32_t* s_tab, const uint8_t* len,
                                               const uint32_t* cw, uint32_t tlo) {
  if constexpr (LT) {
    return s_tab[s];
  } else {
    // an alphabet larger than the LDS table: the table holds the window
    // [tlo, tlo + kTabLds) around the centre code, where most codes fall,
    // then at kTabLds the entry of code 0 (every unpredictable value)
    const uint32_t r = s - tlo;
    const uint32_t k = r < kTabLds ? r : (s == 0 ? kTabLds : kTabLds + 1);
    if (k <= kTabLds) return s_tab[k];
    return cw ? cw[s] : ((uint32_t)len[s] << 27);  // cw holds len << 27 | code
  }
}
// Code length of symbol s for the chunk totals: MODE 1 the whole table in
// LDS, MODE 0 its window (as code_entry), MODE 2 one byte per symbol in LDS.
template <int MODE>
__device__ __forceinline__ uint32_t code_len(uint32_t s, const uint32_t* s_tab, const uint8_t* s_len8,
                                             const uint8_t* len, uint32_t tlo) {
  if constexpr (MODE == 2)
    return s_len8[s];
  else
    return code_entry<MODE == 1>(s, s_tab, len, nullptr, tlo) >> 27;
}
// First symbol of the LDS window of a 2^m-symbol table (0 when it all fits).
__host__ __device__ constexpr uint32_t tab_window(uint32_t m) {
  return (1u << m) > kTabLds ? (1u << (m - 1)) - kTabLds / 2 : 0u;
}

// Bit fields appended MSB-first to a stream from bit `pos` on, gathered in a
// 64-bit register: words wholly inside the writer's range get plain stores;
// its first and last words, which it may share with the neighbouring ranges,
// are ORed in (the stream starts zeroed).
struct BitWriter {
  uint32_t* words;
  uint64_t aw, w_first;
  int used;
  bool any;  // a field was put: a writer that wrote nothing touches no word
  uint64_t acc;
  __device__ __forceinline__ BitWriter(uint32_t* w, uint64_t pos)
      : words(w), aw(pos >> 5), w_first(pos >> 5), used((int)(pos & 31)), any(false), acc(0) {}
  // nb <= 32 bits of val
  __device__ __forceinline__ void put(uint32_t val, int nb) {
    if (nb <= 0) return;
    any = true;
    acc |= (uint64_t)val << (64 - used - nb);  // used < 32, nb <= 32: inside 64 bits
    used += nb;
    if (used >= 32) {
      const uint32_t word = (uint32_t)(acc >> 32);
      if (aw == w_first)
        atomicOr(&words[aw], word);
      else
        words[aw] = word;
      aw++;
      acc <<= 32;
      used -= 32;
    }
  }
  __device__ __forceinline__ void finish() {
    if (any && used > 0) atomicOr(&words[aw], (uint32_t)(acc >> 32));
  }
};

// Four consecutive values x[i .. i+3] (i a multiple of 4: 16-byte aligned);
// at the end of the field (i + 4 > n) only the values below n are read.
template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ x, uint64_t i, uint64_t n, T (&v)[4]) {
  if (i + 4 > n) {
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = i + k < n ? x[i + k] : T(0);
  } else if constexpr (sizeof(T) == 4) {
    const uint4 u = *(const uint4*)(x + i);
    v[0] = __builtin_bit_cast(float, u.x);
    v[1] = __builtin_bit_cast(float, u.y);
    v[2] = __builtin_bit_cast(float, u.z);
    v[3] = __builtin_bit_cast(float, u.w);
  } else {
    const uint4 a = *(const uint4*)(x + i), b = *(const uint4*)(x + i + 2);
    v[0] = __builtin_bit_cast(double, ((uint64_t)a.y << 32) | a.x);
    v[1] = __builtin_bit_cast(double, ((uint64_t)a.w << 32) | a.z);
    v[2] = __builtin_bit_cast(double, ((uint64_t)b.y << 32) | b.x);
    v[3] = __builtin_bit_cast(double, ((uint64_t)b.w << 32) | b.z);
  }
}

// ------------------------------ XOR coding of unpredictable values (flag 1)
// Each unpredictable value's reduced pattern u (sign, exponent and kept
// mantissa bits, q = 1 + EXPB + r significant bits) is coded against the
// previous one of its chunk (0 for the first): a count of the leading zero
// bytes of u ^ prev (at most W/8 - 1, in LZB bits), then the significant
// bits of u after those bytes.
template <typename T>
struct XorRec {
  using U = typename FTr<T>::U;
  static constexpr int W = 8 * (int)sizeof(U);
  static constexpr int BMAX = W / 8 - 1;
  static constexpr int LZB = W == 32 ? 2 : 3;
  static constexpr int HB = 1 + FTr<T>::EXPB;
  __device__ static __forceinline__ int lead_bytes(U d) {
    int lz;
    if constexpr (sizeof(U) == 4)
      lz = d ? __clz((int)d) : W;
    else
      lz = d ? __clzll((long long)d) : W;
    return min(lz >> 3, BMAX);
  }
  // record bits of u after prev; q = significant bits of u
  __device__ static __forceinline__ int bits(U u, U prev, int q) {
    const int nb = q - 8 * lead_bytes(u ^ prev);
    return LZB + (nb > 0 ? nb : 0);
  }
};

// The pattern of the last unpredictable value in the lanes before this one
// (0 if none): a wave scan of (has, pattern) keeping the latest present.
template <typename U>
__device__ __forceinline__ U wave_prev_present(bool has, U last) {
  const int lane = threadIdx.x & 63;
  int h = has ? 1 : 0;
  uint64_t v = (uint64_t)last;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int hu = __shfl_up(h, o, 64);
    const uint64_t vu = __shfl_up(v, o, 64);
    if (lane >= o && !h) {
      h = hu;
      v = vu;
    }
  }
  // exclusive: the inclusive result of the lane before
  const int hp = __shfl_up(h, 1, 64);
  const uint64_t vp = __shfl_up(v, 1, 64);
  return (U)((lane > 0 && hp) ? vp : 0ull);
}

template <typename T, typename CT, int MODE>
__device__ __forceinline__ void chunk_stats_body(const CT* __restrict__ codes, const T* __restrict__ x,
                                                 const uint8_t* __restrict__ len, const uint32_t* s_tab,
                                                 const uint8_t* s_len8, CT* sc, uint64_t n, uint32_t C, uint32_t* cbits, uint32_t* cu,
                                                 uint32_t* ctb, typename FTr<T>::U ebb, uint32_t tlo) {
  const uint64_t n_chunks = (n + C - 1) / C;
  const int lane = threadIdx.x & 63;
  const uint32_t per = C / 64;
  for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < n_chunks; c += (uint64_t)gridDim.x * 4) {
    const uint32_t k0 = (uint32_t)lane * per;
    uint32_t b = 0, z = 0, tb = 0;
    if (sizeof(CT) == 1 && per == 16 && (c + 1) * C <= n) {
      // a whole chunk of 1-byte codes: the lane's 16 codes are one aligned
      // 16-byte vector, read straight into registers
      const uint4 v = ((const uint4*)(codes + c * C))[lane];
      const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int g = 0; g < 4; g++) {
        bool anyz = false;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const uint32_t sym = (wv[g] >> (8 * k)) & 0xFFu;
          b += code_len<MODE>(sym, s_tab, s_len8, len, tlo);
          anyz |= sym == 0;
        }
        if (anyz) {
          // unpredictable values come four at a time (16-byte aligned loads)
          T xv[4];
          load4<T>(x, c * C + k0 + 4 * g, n, xv);
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (((wv[g] >> (8 * k)) & 0xFFu) == 0) {
              z++;
              tb += (uint32_t)kept_bits<T>(xv[k], ebb);
            }
        }
      }
    } else {
      const uint32_t cnt = stage_codes<CT>(codes, n, c, C, sc, lane);
      for (uint32_t j = 0; j < per; j += 4) {
        uint32_t sym[4];
        lds_code4<CT>(sc, k0 + j, sym);
        bool anyz = false;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const bool real = k0 + j + k < cnt;
          b += real ? code_len<MODE>(sym[k], s_tab, s_len8, len, tlo) : 0u;
          anyz |= real && sym[k] == 0;
        }
        if (anyz) {
          T xv[4];
          load4<T>(x, c * C + k0 + j, n, xv);
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (k0 + j + k < cnt && sym[k] == 0) {
              z++;
              tb += (uint32_t)kept_bits<T>(xv[k], ebb);
            }
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    b = wave_sum(b);
    z = wave_sum(z);
    tb = wave_sum(tb);
    if (lane == 0) {
      cbits[c] = b;
      cu[c] = z;
      ctb[c] = tb;
    }
  }
}

// Per-chunk totals with XOR-coded unpredictable values: the bits of the
// chunk's records instead of its tail bits.  Two passes over each lane's
// codes: the first finds the lane's last unpredictable pattern (its
// successor lanes' starting point), the second sizes the records.
template <typename T, typename CT, int MODE>
__device__ __forceinline__ void chunk_stats_xor_body(const CT* __restrict__ codes, const T* __restrict__ x,
                                                     const uint8_t* __restrict__ len, const uint32_t* s_tab,
                                                     const uint8_t* s_len8, CT* sc, uint64_t n, uint32_t C, uint32_t* cbits, uint32_t* cu,
                                                     uint32_t* ctb, typename FTr<T>::U ebb, uint32_t tlo) {
  using U = typename FTr<T>::U;
  using XR = XorRec<T>;
  const uint64_t n_chunks = (n + C - 1) / C;
  const int lane = threadIdx.x & 63;
  const uint32_t per = C / 64;
  for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < n_chunks; c += (uint64_t)gridDim.x * 4) {
    const uint32_t cnt = stage_codes<CT>(codes, n, c, C, sc, lane);
    const uint32_t k0 = (uint32_t)lane * per;
    const uint64_t i0 = c * C + k0;
    uint32_t b = 0, z = 0, tb = 0;
    bool has = false;
    U last = 0;
    for (uint32_t j = 0; j < per; j += 4) {
      uint32_t sym[4];
      lds_code4<CT>(sc, k0 + j, sym);
      bool anyz = false;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const bool real = k0 + j + k < cnt;
        b += real ? code_len<MODE>(sym[k], s_tab, s_len8, len, tlo) : 0u;
        anyz |= real && sym[k] == 0;
      }
      if (anyz) {
        T xv[4];
        load4<T>(x, i0 + j, n, xv);
#pragma unroll
        for (int k = 0; k < 4; k++)
          if (k0 + j + k < cnt && sym[k] == 0) {
            z++;
            has = true;
            last = to_bits<T>(truncate_unpred<T>(xv[k], ebb));
          }
      }
    }
    U prev = wave_prev_present<U>(has, last);
    if (z) {
      for (uint32_t j = 0; j < per; j += 4) {
        uint32_t sym[4];
        lds_code4<CT>(sc, k0 + j, sym);
        bool anyz = false;
#pragma unroll
        for (int k = 0; k < 4; k++) anyz |= k0 + j + k < cnt && sym[k] == 0;
        if (!anyz) continue;
        T xv[4];
        load4<T>(x, i0 + j, n, xv);
#pragma unroll
        for (int k = 0; k < 4; k++)
          if (k0 + j + k < cnt && sym[k] == 0) {
            const U u = to_bits<T>(truncate_unpred<T>(xv[k], ebb));
            tb += (uint32_t)XR::bits(u, prev, XR::HB + kept_bits<T>(xv[k], ebb));
            prev = u;
          }
      }
    }
    __builtin_amdgcn_wave_barrier();
    b = wave_sum(b);
    z = wave_sum(z);
    tb = wave_sum(tb);
    if (lane == 0) {
      cbits[c] = b;
      cu[c] = z;
      ctb[c] = tb;
    }
  }
}

// L8 (2-byte codes with alphabets that may outgrow the LDS table): the code
// lengths as one byte per symbol in dynamic LDS after the codes, so that
// every length comes from LDS (65,536 bytes at m = 16).
template <typename T, typename CT, bool L8 = false>
__device__ __forceinline__ void chunk_stats_kernel_dev(const CT* __restrict__ codes, const T* __restrict__ x,
                                                          const uint8_t* __restrict__ len, uint64_t n,
                                                          uint32_t C, uint32_t* cbits, uint32_t* cu,
                                                          uint32_t* ctb, const DevPlan* P) {
  extern __shared__ uint4 s_dyn[];  // [4][C] codes, one slice per wave (then the L8 lengths)
  __shared__ uint32_t s_tab[L8 ? 1 : kTabLds + 1];
  if (P->status) return;
  const uint32_t nsym = 1u << P->m;
  const bool lt = nsym <= kTabLds;
  const uint32_t tlo = tab_window(P->m);
  uint8_t* s_len8 = (uint8_t*)((CT*)s_dyn + 4 * (size_t)C);
  if constexpr (L8) {
    for (uint32_t i = threadIdx.x; i < (nsym + 3) / 4; i += 256) ((uint32_t*)s_len8)[i] = ((const uint32_t*)len)[i];
  } else {
    for (uint32_t i = threadIdx.x; i < min(nsym, kTabLds); i += 256) s_tab[i] = (uint32_t)len[tlo + i] << 27;
    if (!lt && threadIdx.x == 0) s_tab[kTabLds] = (uint32_t)len[0] << 27;
  }
  __syncthreads();
  CT* sc = (CT*)s_dyn + (size_t)(threadIdx.x >> 6) * C;
  const auto ebb = (typename FTr<T>::U)P->ebT_bits;
  constexpr int MW = L8 ? 2 : 0;  // the mode when the alphabet outgrows the table
  if (P->xorc) {
    if (!L8 && (sizeof(CT) == 1 || lt))
      chunk_stats_xor_body<T, CT, 1>(codes, x, len, s_tab, s_len8, sc, n, C, cbits, cu, ctb, ebb, tlo);
    else
      chunk_stats_xor_body<T, CT, MW>(codes, x, len, s_tab, s_len8, sc, n, C, cbits, cu, ctb, ebb, tlo);
  } else if (!L8 && (sizeof(CT) == 1 || lt)) {
    chunk_stats_body<T, CT, 1>(codes, x, len, s_tab, s_len8, sc, n, C, cbits, cu, ctb, ebb, tlo);
  } else {
    chunk_stats_body<T, CT, MW>(codes, x, len, s_tab, s_len8, sc, n, C, cbits, cu, ctb, ebb, tlo);
  }
}
template <typename T, typename CT, bool L8 = false>
__global__ void __launch_bounds__(256) chunk_stats_kernel(const CT* __restrict__ codes, const T* __restrict__ x,
                                                          const uint8_t* __restrict__ len, uint64_t n,
                                                          uint32_t C, uint32_t* cbits, uint32_t* cu,
                                                          uint32_t* ctb, const DevPlan* P) {
  chunk_stats_kernel_dev<T, CT, L8>(codes, x, len, n, C, cbits, cu, ctb, P);
}


// ------------------------------------------ device-wide exclusive scans
// Phase 1: per-workgroup sums of 4096-element tiles.
__device__ __forceinline__ void scan_tile_sums_dev(const uint32_t* __restrict__ in, uint64_t n, uint64_t* tsum) {
  __shared__ uint64_t red[16];
  const uint64_t t0 = (uint64_t)blockIdx.x * 4096;
  uint64_t s = 0;
  for (int k = 0; k < 4; k++) {
    const uint64_t i = t0 + (uint64_t)k * 1024 + threadIdx.x;
    if (i < n) s += in[i];
  }
  s = block_sum<1024, uint64_t>(s, red);
  if (threadIdx.x == 0) tsum[blockIdx.x] = s;
}
__global__ void __launch_bounds__(1024) scan_tile_sums(const uint32_t* __restrict__ in, uint64_t n, uint64_t* tsum) {
  scan_tile_sums_dev(in, n, tsum);
}

// Phase 2: one workgroup scans the tile sums in place; total to *total.
__device__ __forceinline__ void scan_tile_offsets_dev(uint64_t* tsum, uint64_t ntiles, uint64_t* total) {
  __shared__ uint64_t red[16];
  const uint64_t per = (ntiles + 1023) / 1024;
  const uint64_t lo = min(ntiles, (uint64_t)threadIdx.x * per), hi = min(ntiles, lo + per);
  uint64_t s = 0;
  for (uint64_t i = lo; i < hi; i++) s += tsum[i];
  uint64_t tot;
  uint64_t off = block_exscan<1024, uint64_t>(s, red, &tot);
  for (uint64_t i = lo; i < hi; i++) {
    const uint64_t v = tsum[i];
    tsum[i] = off;
    off += v;
  }
  if (threadIdx.x == 0 && total) *total = tot;
}
__global__ void __launch_bounds__(1024) scan_tile_offsets(uint64_t* tsum, uint64_t ntiles, uint64_t* total) {
  scan_tile_offsets_dev(tsum, ntiles, total);
}
// Phase 2 of a scan whose total must equal `want` (else the container is
// corrupt).
__global__ void __launch_bounds__(1024) scan_tile_offsets_check(uint64_t* tsum, uint64_t ntiles, uint64_t* total,
                                                                uint64_t want, DevPlan* P) {
  scan_tile_offsets_dev(tsum, ntiles, total);
  if (threadIdx.x == 0 && *total != want) set_status(P, SZ_ECORRUPT);
}

// Phase 3: exclusive prefix of every element.
__device__ __forceinline__ void scan_apply_dev(const uint32_t* __restrict__ in, uint64_t n, const uint64_t* tsum,
                                                   uint64_t* out) {
  __shared__ uint64_t red[16];
  const uint64_t t0 = (uint64_t)blockIdx.x * 4096;
  uint64_t base = tsum[blockIdx.x];
  for (int k = 0; k < 4; k++) {
    const uint64_t i = t0 + (uint64_t)k * 1024 + threadIdx.x;
    const uint64_t v = (i < n) ? in[i] : 0;
    uint64_t tot;
    const uint64_t ex = block_exscan<1024, uint64_t>(v, red, &tot);
    if (i < n) out[i] = base + ex;
    base += tot;
  }
}
__global__ void __launch_bounds__(1024) scan_apply(const uint32_t* __restrict__ in, uint64_t n, const uint64_t* tsum,
                                                   uint64_t* out) {
  scan_apply_dev(in, n, tsum, out);
}

// Three scans of n elements each in one launch per phase (blockIdx.y picks
// the array): the same per-array work as scan_tile_sums, scan_tile_offsets
// and scan_apply.
struct Scan3 {
  const uint32_t* in[3];
  uint64_t* out[3];
  uint64_t* tsum[3];
  uint64_t* total[3];
};
__global__ void __launch_bounds__(1024) scan3_tile_sums(Scan3 S, uint64_t n) {
  scan_tile_sums_dev(S.in[blockIdx.y], n, S.tsum[blockIdx.y]);
}
__global__ void __launch_bounds__(1024) scan3_tile_offsets(Scan3 S, uint64_t ntiles) {
  scan_tile_offsets_dev(S.tsum[blockIdx.y], ntiles, S.total[blockIdx.y]);
}
__global__ void __launch_bounds__(1024) scan3_apply(Scan3 S, uint64_t n) {
  scan_apply_dev(S.in[blockIdx.y], n, S.tsum[blockIdx.y], S.out[blockIdx.y]);
}


// --------------------------------------- container layout (after scans)
struct LayoutArgs {
  DevPlan* plan;
  const uint64_t* tot_bits;
  const uint64_t* tot_u;
  const uint64_t* tot_tb;
  uint64_t n_chunks;
  uint64_t raw_size;  // header + S
  uint32_t head_bits;
  uint32_t xorc;      // heads section = one u32 record-bit count per chunk
};
__device__ __forceinline__ uint64_t align64(uint64_t v) { return (v + 63) & ~63ull; }

__device__ __forceinline__ void layout_kernel_dev(LayoutArgs A) {
  DevPlan* P = A.plan;
  if (threadIdx.x || P->status) return;
  P->huff_bits = *A.tot_bits;
  P->n_unpred = *A.tot_u;
  P->tail_bits = *A.tot_tb;
  P->off_cb = kHdr;
  P->off_ch = align64(kHdr + 3ull * P->n_used);
  P->off_bs = align64(P->off_ch + 6ull * A.n_chunks);
  P->off_hd = align64(P->off_bs + 4ull * ((P->huff_bits + 31) / 32));
  P->off_tl = align64(P->off_hd + (A.xorc ? 4ull * A.n_chunks : 4ull * ((P->n_unpred * A.head_bits + 31) / 32)));
  P->total = P->off_tl + 4ull * ((P->tail_bits + 31) / 32);
  P->raw = P->total >= A.raw_size;
  if (P->raw) P->total = A.raw_size;
  if (P->total > P->out_cap) P->status = SZ_ECAPACITY;
}
__global__ void layout_kernel(LayoutArgs A) {
  layout_kernel_dev(A);
}


// ------------------------------------------------------- K5c: encoding
// One wave per chunk: the chunk's codes are staged in LDS, lane offsets come
// from a wave scan of code lengths, bits are ORed into the wave's LDS words
// and then written out (words shared with the neighbouring chunks with an
// atomic OR, the rest with plain stores).  The (length, codeword) table sits
// in LDS as (len << 27) | code when 2^m <= 4096.
constexpr int kEncNT = 256;
// Unpredictable values per chunk above which their heads and tails are
// staged in LDS (below it, per-lane bit writers to memory cost less).
constexpr uint32_t kEncStageMin = 64;
// LDS words per wave for the chunk's largest stream: its codes (at most kLmax
// bits each), heads (9 or 12 bits each) or tails (kept mantissa bits, or
// XOR records of at most 2 + 32 or 3 + 64 bits)
__host__ __device__ constexpr uint32_t enc_words_per_wave(uint32_t C, uint32_t value_bytes, bool xorc) {
  const uint32_t huff = C * kLmax / 32 + 2;
  const uint32_t tail = C * (xorc ? (value_bytes == 8 ? 67u : 34u) : (value_bytes == 8 ? 52u : 23u)) / 32 + 2;
  const uint32_t head = C * (value_bytes == 8 ? 12u : 9u) / 32 + 2;
  return huff > tail ? (huff > head ? huff : head) : (tail > head ? tail : head);
}
// dynamic LDS of the encoder: per wave, the bit words then C codes of CT
__host__ __device__ constexpr uint32_t enc_lds_bytes(uint32_t C, uint32_t code_bytes, uint32_t value_bytes,
                                                     bool xorc) {
  return 4u * (enc_words_per_wave(C, value_bytes, xorc) * 4u + C * code_bytes);
}

template <typename T, typename CT, bool LT, bool XORC, int PR>
__device__ __forceinline__ void encode_body(const CT* __restrict__ codes, const T* __restrict__ x,
                                            const uint8_t* __restrict__ len, const uint32_t* __restrict__ cw,
                                            const uint32_t* s_tab, uint32_t* words, CT* sc, uint64_t n,
                                            uint32_t C, const uint32_t* cbits, const uint64_t* boff,
                                            const uint64_t* uoff, const uint64_t* toff, uint8_t* out,
                                            const DevPlan* P, uint32_t tlo) {
  using U = typename FTr<T>::U;
  constexpr int MANT = FTr<T>::MANT;
  constexpr int HB = 1 + FTr<T>::EXPB;
  const uint64_t n_chunks = (n + C - 1) / C;
  const int lane = threadIdx.x & 63;
  const uint32_t per = C / 64;
  uint32_t* bs = (uint32_t*)(out + P->off_bs);
  uint32_t* hd = (uint32_t*)(out + P->off_hd);
  uint32_t* tl = (uint32_t*)(out + P->off_tl);
  uint32_t* ch = (uint32_t*)(out + P->off_ch);
  const U ebb = (U)P->ebT_bits;
  for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < n_chunks; c += (uint64_t)gridDim.x * 4) {
    const uint32_t nb = cbits[c];
    const uint64_t b0 = boff[c];
    const uint32_t nw = (uint32_t)((((b0 & 31) + nb) + 31) / 32);
    for (uint32_t w = lane; w < nw; w += 64) words[w] = 0;
    const uint32_t cnt = stage_codes<CT>(codes, n, c, C, sc, lane);
    const uint32_t k0 = (uint32_t)lane * per;
    const uint64_t i0 = c * C + k0;  // a multiple of 4
    uint32_t mybits = 0, myz = 0, mytb = 0;
    // PR > 0 (a lane holds at most PR codes): the lane's unpredictable
    // values are loaded once, with every load in flight together, and kept
    // in registers for the passes below; otherwise each pass loads them.
    T xr[PR > 0 ? PR / 4 : 1][4];
    uint32_t zmask = 0;  // PR > 0: bit q set when the lane's code q is 0
    // PR != 0: the code entries (len << 27 | code) as well, for the bitstream
    // pass (0 past the chunk: a field of no bits); PR < 0 keeps the -PR
    // entries of a lane but loads the values in every pass
    constexpr int NE = PR < 0 ? -PR : PR;
    uint32_t ent[NE > 0 ? NE : 1];
    if constexpr (PR > 0) {
#pragma unroll
      for (int g = 0; g < PR / 4; g++) {
#pragma unroll
        for (int k = 0; k < 4; k++) ent[4 * g + k] = 0u;
        if ((uint32_t)(4 * g) < per) {
          uint32_t sym[4];
          lds_code4<CT>(sc, k0 + 4 * g, sym);
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const bool real = k0 + 4 * g + k < cnt;
            ent[4 * g + k] = real ? code_entry<LT>(sym[k], s_tab, len, cw, tlo) : 0u;
            mybits += ent[4 * g + k] >> 27;
            zmask |= (real && sym[k] == 0) ? 1u << (4 * g + k) : 0u;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < PR / 4; g++)
        if ((zmask >> (4 * g)) & 15u) load4<T>(x, i0 + 4 * g, n, xr[g]);
    }
    // The lane's unpredictable values, in order, as (reduced pattern, kept
    // mantissa bits); `emit` takes each one.
    auto each_unpred = [&](auto&& emit) {
      if constexpr (PR > 0) {
#pragma unroll
        for (int q = 0; q < PR; q++)
          if ((zmask >> q) & 1u)
            emit(to_bits<T>(truncate_unpred<T>(xr[q / 4][q % 4], ebb)), kept_bits<T>(xr[q / 4][q % 4], ebb));
      } else {
        for (uint32_t j = 0; j < per; j += 4) {
          uint32_t sym[4];
          lds_code4<CT>(sc, k0 + j, sym);
          bool anyz = false;
#pragma unroll
          for (int k = 0; k < 4; k++) anyz |= k0 + j + k < cnt && sym[k] == 0;
          if (!anyz) continue;
          // unpredictable values come four at a time (16-byte aligned loads)
          T xv[4];
          load4<T>(x, i0 + j, n, xv);
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (k0 + j + k < cnt && sym[k] == 0)
              emit(to_bits<T>(truncate_unpred<T>(xv[k], ebb)), kept_bits<T>(xv[k], ebb));
        }
      }
    };
    bool has = false;
    U last = 0;
    auto count_unpred = [&](U ub, int r) {
      myz++;
      if constexpr (XORC) {
        has = true;
        last = ub;
      } else {
        mytb += (uint32_t)r;
      }
    };
    if constexpr (PR > 0) {
      each_unpred(count_unpred);
    } else if constexpr (PR < 0) {
      // code entries and the unpredictable values in one pass
#pragma unroll
      for (int g = 0; g < NE / 4; g++) {
#pragma unroll
        for (int k = 0; k < 4; k++) ent[4 * g + k] = 0u;
        if ((uint32_t)(4 * g) < per) {
          const uint32_t j = 4 * g;
          uint32_t sym[4];
          lds_code4<CT>(sc, k0 + j, sym);
          bool anyz = false;
#pragma unroll
          for (int k = 0; k < 4; k++) {
            const bool real = k0 + j + k < cnt;
            ent[4 * g + k] = real ? code_entry<LT>(sym[k], s_tab, len, cw, tlo) : 0u;
            mybits += ent[4 * g + k] >> 27;
            anyz |= real && sym[k] == 0;
          }
          if (anyz) {
            T xv[4];
            load4<T>(x, i0 + j, n, xv);
#pragma unroll
            for (int k = 0; k < 4; k++)
              if (k0 + j + k < cnt && sym[k] == 0)
                count_unpred(to_bits<T>(truncate_unpred<T>(xv[k], ebb)), kept_bits<T>(xv[k], ebb));
          }
        }
      }
    } else {
      // code lengths and the unpredictable values in one pass
      for (uint32_t j = 0; j < per; j += 4) {
        uint32_t sym[4];
        lds_code4<CT>(sc, k0 + j, sym);
        bool anyz = false;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const bool real = k0 + j + k < cnt;
          mybits += real ? (code_entry<LT>(sym[k], s_tab, len, cw, tlo) >> 27) : 0u;
          anyz |= real && sym[k] == 0;
        }
        if (anyz) {
          T xv[4];
          load4<T>(x, i0 + j, n, xv);
#pragma unroll
          for (int k = 0; k < 4; k++)
            if (k0 + j + k < cnt && sym[k] == 0)
              count_unpred(to_bits<T>(truncate_unpred<T>(xv[k], ebb)), kept_bits<T>(xv[k], ebb));
        }
      }
    }
    // XOR coding: the chunk's previous pattern before the lane's first value
    // (the last of the lanes before it), then the sizes of the lane's records
    U prev0 = 0;
    if constexpr (XORC) {
      using XR = XorRec<T>;
      prev0 = wave_prev_present<U>(has, last);
      U prev = prev0;
      if (myz)
        each_unpred([&](U u, int r) {
          mytb += (uint32_t)XR::bits(u, prev, XR::HB + r);
          prev = u;
        });
      // the chunk's entry of the table of record bits (the heads section)
      const uint32_t tot = wave_sum(mytb);
      if (lane == 0) hd[c] = tot;
    }
    const uint64_t bpos = (b0 & 31) + wave_exscan(mybits);
    // the bits of the chunk's first half (lanes 0..31 hold its first C/2
    // codes): where a second decoder of the chunk starts
    if (lane == 32) ((uint16_t*)(ch + n_chunks))[c] = (uint16_t)(bpos - (b0 & 31));
    const uint64_t zex = wave_exscan(myz), tex = wave_exscan(mytb);
    const uint32_t zch = wave_sum(myz), tch = wave_sum(mytb);  // the chunk's values and tail bits
    __builtin_amdgcn_wave_barrier();
    // Three streams leave through the wave's LDS words in turn (codes, then
    // heads, then tails): each is written bit by bit in LDS and then copied
    // out in whole words, the words shared with the neighbouring chunks with
    // an atomic OR; bit writers straight to memory would make every wave
    // store touch a line per lane.
    auto copy_out = [&](uint32_t* dst, uint64_t bit0, uint64_t nbits) {
      const uint32_t nwo = (uint32_t)((((bit0 & 31) + nbits) + 31) / 32);
      const uint64_t gw0 = bit0 >> 5, bend = bit0 + nbits;
      __builtin_amdgcn_wave_barrier();
      for (uint32_t w = lane; w < nwo; w += 64) {
        const uint64_t gw = gw0 + w;
        const bool full = (gw * 32 >= bit0) && (gw * 32 + 32 <= bend);
        if (full)
          dst[gw] = words[w];
        else if (words[w])
          atomicOr(&dst[gw], words[w]);
      }
      __builtin_amdgcn_wave_barrier();
    };
    auto clear_words = [&](uint64_t bit0, uint64_t nbits) {
      const uint32_t nwo = (uint32_t)((((bit0 & 31) + nbits) + 31) / 32);
      for (uint32_t w = lane; w < nwo; w += 64) words[w] = 0;
      __builtin_amdgcn_wave_barrier();
    };
    {
      BitWriter wb(words, bpos);
      if constexpr (NE > 0) {
#pragma unroll
        for (int q = 0; q < NE; q++) wb.put(ent[q] & 0x07FFFFFFu, (int)(ent[q] >> 27));
      } else {
        for (uint32_t j = 0; j < per; j += 4) {
          uint32_t sym[4];
          lds_code4<CT>(sc, k0 + j, sym);
#pragma unroll
          for (int k = 0; k < 4; k++) {
            if (k0 + j + k >= cnt) break;
            const uint32_t e = code_entry<LT>(sym[k], s_tab, len, cw, tlo);
            wb.put(e & 0x07FFFFFFu, (int)(e >> 27));
          }
        }
      }
      wb.finish();
      copy_out(bs, b0, nb);
    }
    if (lane == 0) ch[c] = nb;
    if (zch) {
      // tails: the kept mantissa bits, or the XOR records
      U prev = prev0;
      auto put_tail = [&](BitWriter& wt, U ub, int r) {
        if constexpr (XORC) {
          // leading-byte count, then the significant bits after those bytes
          using XR = XorRec<T>;
          const int q = XR::HB + r;
          const int lzb = XR::lead_bytes(ub ^ prev);
          wt.put((uint32_t)lzb, XR::LZB);
          const int nbq = q - 8 * lzb;
          if (nbq > 0) {
            const U v = (ub >> (XR::W - q)) & ((((U)1) << (nbq - 1) << 1) - 1);
            if (nbq > 32) {
              wt.put((uint32_t)((uint64_t)v >> 32), nbq - 32);
              wt.put((uint32_t)v, 32);
            } else {
              wt.put((uint32_t)v, nbq);
            }
          }
          prev = ub;
        } else {
          const U tail = (ub & ((((U)1) << MANT) - 1)) >> (MANT - r);  // the top r mantissa bits
          if (r > 32) {
            wt.put((uint32_t)((uint64_t)tail >> 32), r - 32);
            wt.put((uint32_t)tail, 32);
          } else {
            wt.put((uint32_t)tail, r);
          }
        }
      };
      if (zch <= kEncStageMin) {
        // few values: their heads and tails go straight to memory
        BitWriter wh(hd, (uoff[c] + zex) * HB), wt(tl, toff[c] + tex);
        each_unpred([&](U ub, int r) {
          if constexpr (!XORC) wh.put((uint32_t)(ub >> MANT), HB);
          put_tail(wt, ub, r);
        });
        wh.finish();
        wt.finish();
      } else {
        if constexpr (!XORC) {
          // heads: sign and exponent of each value
          const uint64_t hb0 = uoff[c] * HB;
          clear_words(hb0, (uint64_t)zch * HB);
          BitWriter wh(words, (hb0 & 31) + zex * HB);
          each_unpred([&](U ub, int) { wh.put((uint32_t)(ub >> MANT), HB); });
          wh.finish();
          copy_out(hd, hb0, (uint64_t)zch * HB);
        }
        const uint64_t tb0 = toff[c];
        clear_words(tb0, tch);
        BitWriter wt(words, (tb0 & 31) + tex);
        each_unpred([&](U ub, int r) { put_tail(wt, ub, r); });
        wt.finish();
        copy_out(tl, tb0, tch);
      }
    }
  }
}

// PR: 0; 16 for chunks of at most 1024 codes (the unpredictable values and
// code entries of each lane held in registers; more registers, fewer loads);
// -16 for such chunks with the code entries only in registers.
template <typename T, typename CT, int PR = 0>
__device__ __forceinline__ void encode_kernel_dev(const CT* __restrict__ codes, const T* __restrict__ x,
                                                        const uint8_t* __restrict__ len,
                                                        const uint32_t* __restrict__ cw, uint64_t n, uint32_t C,
                                                        const uint32_t* cbits, const uint64_t* boff,
                                                        const uint64_t* uoff, const uint64_t* toff,
                                                        uint8_t* out, const DevPlan* P) {
  extern __shared__ uint4 s_dyn[];  // [4][words] then [4][C] codes
  // 1-byte codes have at most 256 symbols: a table that small leaves room
  // for a second workgroup per CU
  constexpr uint32_t kTab = sizeof(CT) == 1 ? 256 : kTabLds;
  __shared__ uint32_t s_tab[kTab + 1];
  if (P->status || P->raw) return;
  const uint32_t nsym = 1u << P->m;
  const bool lt = nsym <= kTab;
  const uint32_t tlo = tab_window(P->m);
  for (uint32_t i = threadIdx.x; i < min(nsym, kTab); i += kEncNT) s_tab[i] = cw[tlo + i];  // len << 27 | code
  if (!lt && threadIdx.x == 0) s_tab[kTab] = cw[0];  // code 0 beside the window
  __syncthreads();
  const int wv = threadIdx.x >> 6;
  const uint32_t wpw = enc_words_per_wave(C, sizeof(T), P->xorc != 0);
  uint32_t* words = (uint32_t*)s_dyn + (size_t)wv * wpw;
  CT* sc = (CT*)((uint32_t*)s_dyn + 4 * (size_t)wpw) + (size_t)wv * C;
  if (P->xorc) {
    if (sizeof(CT) == 1 || lt)
      encode_body<T, CT, true, true, PR>(codes, x, len, cw, s_tab, words, sc, n, C, cbits, boff, uoff, toff, out, P,
                                         tlo);
    else
      encode_body<T, CT, false, true, PR>(codes, x, len, cw, s_tab, words, sc, n, C, cbits, boff, uoff, toff, out, P,
                                          tlo);
  } else if (sizeof(CT) == 1 || lt) {
    encode_body<T, CT, true, false, PR>(codes, x, len, cw, s_tab, words, sc, n, C, cbits, boff, uoff, toff, out, P,
                                        tlo);
  } else {
    encode_body<T, CT, false, false, PR>(codes, x, len, cw, s_tab, words, sc, n, C, cbits, boff, uoff, toff, out, P,
                                         tlo);
  }
}
template <typename T, typename CT, int PR>
__global__ void __launch_bounds__(kEncNT) encode_kernel(const CT* __restrict__ codes, const T* __restrict__ x,
                                                        const uint8_t* __restrict__ len,
                                                        const uint32_t* __restrict__ cw, uint64_t n, uint32_t C,
                                                        const uint32_t* cbits, const uint64_t* boff,
                                                        const uint64_t* uoff, const uint64_t* toff,
                                                        uint8_t* out, const DevPlan* P, uint32_t by_share) {
  // by_share: both forms are launched and only one runs, the register form
  // when more than one value in 16 is unpredictable (its extra registers
  // cost occupancy that only such fields win back)
  if (by_share && ((P->n_unpred * 16 > n) != (PR > 0))) return;
  encode_kernel_dev<T, CT, PR>(codes, x, len, cw, n, C, cbits, boff, uoff, toff, out, P);
}


// -------------------------------------------------- K7: header + codebook
struct HeaderArgs {
  uint8_t* out;
  const uint8_t* len;
  const DevPlan* plan;
  uint32_t dtype, ndim, layers, eb_mode, m_req, chunk;
  uint64_t dims[3], block[3];
  double eb_abs, eb_rel;
  uint64_t n, n_chunks;
};

__device__ __forceinline__ void put64(uint8_t* b, uint64_t v) {
  for (int i = 0; i < 8; i++) b[i] = (uint8_t)(v >> (8 * i));
}

__device__ __forceinline__ void header_kernel_dev(HeaderArgs A) {
  __shared__ uint8_t h[kHdr];
  __shared__ uint32_t red[8];
  const DevPlan* P = A.plan;
  if (P->status) return;
  const int tid = threadIdx.x;
  if (tid < (int)kHdr) h[tid] = 0;
  __syncthreads();
  if (tid == 0) {
    const bool raw = P->raw;
    const uint64_t flags = raw ? 1 : (P->xorc ? 2 : 0);  // raw copy; XOR-coded unpredictable values
    put64(h + 0, kMagic | ((uint64_t)kVersion << 32) | (flags << 48));
    h[8] = (uint8_t)A.dtype;
    h[9] = (uint8_t)A.ndim;
    h[10] = (uint8_t)A.layers;
    h[11] = (uint8_t)P->m;
    h[12] = (uint8_t)A.eb_mode;
    h[13] = (uint8_t)A.m_req;
    for (int d = 0; d < 3; d++) put64(h + 16 + 8 * d, A.dims[d]);
    for (int d = 0; d < 3; d++) put64(h + 40 + 8 * d, A.block[d]);
    put64(h + 64, __builtin_bit_cast(uint64_t, A.eb_abs));
    put64(h + 72, __builtin_bit_cast(uint64_t, A.eb_rel));
    put64(h + 80, P->ebT_bits);
    put64(h + 88, A.n);
    put64(h + 96, raw ? 0 : P->n_unpred);
    put64(h + 104, raw ? 0 : P->huff_bits);
    put64(h + 112, raw ? 0 : P->tail_bits);
    put64(h + 120, (uint64_t)A.chunk | ((uint64_t)(raw ? 0 : P->n_used) << 32));
    put64(h + 128, raw ? 0 : A.n_chunks);
    put64(h + 136, raw ? kHdr : P->off_cb);
    put64(h + 144, raw ? kHdr : P->off_ch);
    put64(h + 152, raw ? kHdr : P->off_bs);
    put64(h + 160, raw ? kHdr : P->off_hd);
    put64(h + 168, raw ? kHdr : P->off_tl);
    put64(h + 176, P->total);
  }
  __syncthreads();
  if (tid < (int)kHdr / 4) ((uint32_t*)A.out)[tid] = ((uint32_t*)h)[tid];
  if (P->raw) return;
  // codebook section: (u16 symbol, u8 length) sorted by symbol
  const uint32_t nsym = 1u << P->m;
  const uint32_t per = (nsym + 255) / 256;
  const uint32_t lo = min(nsym, tid * per), hi = min(nsym, lo + per);
  uint8_t* cb = A.out + P->off_cb;
  auto put = [&](uint32_t q, uint32_t l, uint32_t& pos) {
    cb[3 * pos + 0] = (uint8_t)(q & 0xFF);
    cb[3 * pos + 1] = (uint8_t)(q >> 8);
    cb[3 * pos + 2] = (uint8_t)l;
    pos++;
  };
  if (per % 16 == 0) {
    // 16 lengths per load (the length array is 256-byte aligned), four
    // loads in flight: a thread's 256 lengths at m = 16 are 16 loads, not 256
    const uint4* L4 = (const uint4*)(A.len + lo);
    const uint32_t nv = per / 16;
    auto nz = [](uint32_t w) {
      return (uint32_t)((w & 0xFFu) != 0) + ((w & 0xFF00u) != 0) + ((w & 0xFF0000u) != 0) + ((w >> 24) != 0);
    };
    uint32_t cnt = 0;
    for (uint32_t v0 = 0; v0 < nv; v0 += 4) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) v[u] = v0 + u < nv ? L4[v0 + u] : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 4; u++) cnt += nz(v[u].x) + nz(v[u].y) + nz(v[u].z) + nz(v[u].w);
    }
    uint32_t pos = block_exscan<256, uint32_t>(cnt, red, nullptr);
    for (uint32_t v0 = 0; v0 < nv; v0 += 4) {
      uint4 v[4];
#pragma unroll
      for (int u = 0; u < 4; u++) v[u] = v0 + u < nv ? L4[v0 + u] : make_uint4(0, 0, 0, 0);
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t w[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int e = 0; e < 16; e++) {
          const uint32_t l = (w[e / 4] >> (8 * (e % 4))) & 0xFFu;
          if (l) put(lo + 16 * (v0 + u) + e, l, pos);
        }
      }
    }
  } else {
    uint32_t cnt = 0;
    for (uint32_t q = lo; q < hi; q++) cnt += A.len[q] != 0;
    uint32_t pos = block_exscan<256, uint32_t>(cnt, red, nullptr);
    for (uint32_t q = lo; q < hi; q++) {
      const uint8_t l = A.len[q];
      if (l) put(q, l, pos);
    }
  }
}
__global__ void __launch_bounds__(256) header_kernel(HeaderArgs A) {
  header_kernel_dev(A);
}


template <typename T>
__device__ __forceinline__ void raw_copy_kernel_dev(const T* __restrict__ x, uint8_t* out, uint64_t n, const DevPlan* P) {
  if (P->status || !P->raw) return;
  const uint64_t bytes = n * sizeof(T);
  uint8_t* dst = out + kHdr;
  const uint8_t* src = (const uint8_t*)x;
  const uint64_t nv = bytes / 16;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (uint64_t)gridDim.x * blockDim.x)
    ((uint4*)dst)[i] = ((const uint4*)src)[i];
  for (uint64_t i = nv * 16 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
       i += (uint64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}
template <typename T>
__global__ void raw_copy_kernel(const T* __restrict__ x, uint8_t* out, uint64_t n, const DevPlan* P) {
  raw_copy_kernel_dev<T>(x, out, n, P);
}
// The container's body before the encoder fills it: zeroed (the encoder ORs
// its bits in) or, for a raw container, the field itself; one launch for both.
template <typename T>
__global__ void container_prep_kernel(const T* __restrict__ x, uint8_t* out, uint64_t n, const DevPlan* P) {
  zero_container_kernel_dev((uint32_t*)out, P);
  raw_copy_kernel_dev<T>(x, out, n, P);
}


// Final status/size words for the asynchronous entry point.
__device__ __forceinline__ void finish_kernel_dev(const DevPlan* P, uint64_t* d_size, int32_t* d_status) {
  if (threadIdx.x) return;
  if (d_status) *d_status = P->status;
  if (d_size) *d_size = P->status ? 0 : P->total;
}
__global__ void finish_kernel(const DevPlan* P, uint64_t* d_size, int32_t* d_status) {
  finish_kernel_dev(P, d_size, d_status);
}


// =================================================================== decode
struct DecTables {
  uint32_t lut[4096];       // (len << 16) | sym for codes of length <= 12, 0 if longer
  // 1-byte codes (m <= 8): the codes that lie wholly inside a 12-bit window,
  // up to four: symbols in bytes 0..3 (first lowest), count in bits 32..35,
  // their total length in bits 36..39, how many are 0 in bits 40..42
  uint64_t mlut[4096];
  // 1-byte codes with at most kLut2Max 12-bit prefixes of longer codes: the
  // codes of 13..16 bits, (len << 16) | sym, at (prefix - lut2_p0) * 16 plus
  // the next 4 bits; 0 for longer codes.  lut2_n = 0 when not built.
  uint32_t lut2[128 * 16];
  uint32_t lut2_p0, lut2_n;
  uint32_t first[32], count[32], start[32];
  // lim[l]: (first[l] + count[l]) << (27 - l), the first 27-bit left-aligned
  // value past the codes of length <= l (non-decreasing in l)
  uint32_t lim[32];
  uint32_t nsorted;
};
constexpr int kLutBits = 12;
constexpr uint32_t kLut2Max = 128;

// Decode tables from the codebook section; checks symbols strictly
// increasing and the Kraft condition of the canonical code.
__global__ void __launch_bounds__(1024) dectab_kernel(const uint8_t* comp, uint64_t off_cb, uint32_t n_used,
                                                      uint32_t m, DecTables* D, uint64_t* gkeys,
                                                      uint32_t* sorted_syms, DevPlan* P) {
  __shared__ uint64_t s_keys[4096];
  __shared__ uint32_t s_lut[4096];  // the single-code table, built here and copied out once
  __shared__ uint32_t s_cnt[32], s_first[32], s_start[32];
  __shared__ uint32_t s_lc[16][32];
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) s_bad = 0;
  if (tid < 32) s_cnt[tid] = 0;
  for (int i = tid; i < 4096; i += 1024) s_lut[i] = 0;
  __syncthreads();
  const uint32_t nsym = 1u << m;
  if (n_used == 0 || n_used > nsym) {
    if (tid == 0) set_status(P, SZ_ECORRUPT);
    return;
  }
  uint32_t np2 = 1;
  while (np2 < n_used) np2 <<= 1;
  // The rest takes the key array as an argument so that, called with the LDS
  // array, its accesses compile to LDS instructions (a pointer that may
  // address LDS or global memory compiles to slower generic ones).
  auto build = [&](uint64_t* K, bool lds) {
    for (uint32_t e = tid; e < np2; e += 1024) {
      uint32_t l = 0;
      if (e < n_used) {
        const uint8_t* b = comp + off_cb + 3ull * e;
        const uint32_t sym = b[0] | (b[1] << 8);
        l = b[2];
        if (sym >= nsym || l == 0 || l > kLmax) s_bad = 1;
        if (e > 0) {
          const uint8_t* pb = b - 3;
          if ((uint32_t)(pb[0] | (pb[1] << 8)) >= sym) s_bad = 1;
        }
      }
      // one atomic per length present in the wave
      const bool okl = l >= 1 && l <= kLmax;
      const uint64_t peers = wave_peers<5>(okl, l);
      if (okl && peers_last(peers)) atomicAdd(&s_cnt[l], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t code = 0;
      uint32_t start = 0;
      for (int l = 1; l <= kLmax; l++) {
        s_first[l] = (uint32_t)code;
        s_start[l] = start;
        if (code + s_cnt[l] > (1ull << l)) s_bad = 1;
        code = (code + s_cnt[l]) << 1;
        start += s_cnt[l];
      }
      for (int l = 0; l < 32; l++) {
        const bool in = l >= 1 && l <= kLmax;
        D->first[l] = in ? s_first[l] : 0;
        D->count[l] = s_cnt[l];
        D->start[l] = in ? s_start[l] : 0;
        // Kraft-valid lengths keep first + count <= 2^l, so lim <= 2^27
        D->lim[l] = in ? (uint32_t)(((uint64_t)s_first[l] + s_cnt[l]) << (kLmax - l)) : (l ? (1u << kLmax) : 0u);
      }
      D->nsorted = n_used;
    }
    __syncthreads();
    if (s_bad) {
      if (tid == 0) set_status(P, SZ_ECORRUPT);
      return;
    }
    // the used symbols in (length, symbol) order: the section is in symbol
    // order, so each goes to the start of its length plus its rank there
    rank_by_length<1024>(
        n_used, [&](uint32_t e) { return (uint32_t)comp[off_cb + 3ull * e + 2]; }, s_start, s_lc,
        [&](uint32_t e, uint32_t pos) {
          const uint8_t* b = comp + off_cb + 3ull * e;
          const uint32_t sym = b[0] | (b[1] << 8);
          K[pos] = ((uint64_t)b[2] << 16) | sym;
          sorted_syms[pos] = sym;
        });
    // Codes of length l <= kLutBits own the windows [end_{l-1}, end_l), with
    // end_l = (first_l + count_l) << (kLutBits - l): a canonical code's ranges
    // follow each other as l grows.  Each window takes the smallest l whose
    // range ends past it and the symbol of rank (window >> (kLutBits - l)) -
    // first_l among the codes of that length; windows past end_kLutBits start
    // longer codes and stay 0.
    for (uint32_t q = tid; q < (1u << kLutBits); q += 1024) {
      uint32_t L = 0;
#pragma unroll
      for (int l = kLutBits; l >= 1; l--)
        if (q < ((s_first[l] + s_cnt[l]) << (kLutBits - l))) L = (uint32_t)l;
      uint32_t e = 0;
      if (L) {
        const uint32_t v = s_start[L] + (q >> (kLutBits - L)) - s_first[L];
        e = (L << 16) | (uint32_t)(K[v] & 0xFFFF);
      }
      s_lut[q] = e;
      D->lut[q] = e;
    }
    __syncthreads();  // the single-code table is complete
    if (nsym > 256) return;
    // greedy decode of each 12-bit window: the codes after the first are read
    // from the window shifted left, and one that reaches past bit 12 ends it
    for (uint32_t q = tid; q < (1u << kLutBits); q += 1024) {
      uint64_t syms = 0;
      uint32_t k = 0, used = 0, nz = 0;
      while (k < 4) {
        const uint32_t e = s_lut[(q << used) & ((1u << kLutBits) - 1)];
        const uint32_t l = e >> 16;
        if (!e || used + l > (uint32_t)kLutBits) break;
        const uint32_t sym = e & 0xFFFF;
        syms |= (uint64_t)sym << (8 * k);
        nz += sym == 0 ? 1u : 0u;
        used += l;
        k++;
      }
      D->mlut[q] = syms | ((uint64_t)k << 32) | ((uint64_t)used << 36) | ((uint64_t)nz << 40);
    }
    // Codes longer than 12 bits fill the code space after the short ones, so
    // their 12-bit prefixes are [p0, 4096) with p0 the space the short codes
    // take (the code is complete).
    uint32_t p0 = 0;
    for (int l = 1; l <= kLutBits; l++) p0 += s_cnt[l] << (kLutBits - l);
    const uint32_t nlong = (1u << kLutBits) - p0;
    if (nlong > kLut2Max) {
      if (tid == 0) D->lut2_n = 0;
      return;
    }
    for (uint32_t q = tid; q < kLut2Max * 16; q += 1024) D->lut2[q] = 0;
    __syncthreads();
    for (uint32_t v = tid; v < n_used; v += 1024) {
      const uint32_t sym = (uint32_t)(K[v] & 0xFFFF);
      const uint32_t l = (uint32_t)(K[v] >> 16);
      if (l > (uint32_t)kLutBits && l <= 16) {
        const uint32_t code = s_first[l] + (v - s_start[l]);
        const uint32_t a = code << (16 - l), b = (code + 1) << (16 - l);
        for (uint32_t x = a; x < b; x++) {
          const uint32_t r = (x >> 4) - p0;
          if (r < kLut2Max) D->lut2[r * 16 + (x & 15)] = (l << 16) | sym;
        }
      }
    }
    if (tid == 0) {
      D->lut2_p0 = p0;
      D->lut2_n = nlong;
    }
  };
  if (np2 <= 4096)
    build(s_keys, true);
  else
    build(gkeys, false);
}

// K8: one lane per chunk decodes its symbols sequentially from the chunk's
// bit offset.  A 12-bit table in LDS resolves short codes; a longer code's
// length is the count of per-length limits its 27-bit window reaches (the
// canonical code orders codes by length), and its symbol comes from the
// length-sorted symbol list (in LDS when it has at most 4096 entries).  The
// bitstream is read in 16-byte groups one group ahead of use, the decoded
// codes leave in 16-byte stores, and unpredictable codes are counted per
// row segment (block row) with the segment tracked incrementally.
// 2-byte codes: the decoder runs one 1024-thread workgroup per CU, so its LDS
// can hold the symbols of all but the longest 4096 codes (tables 16 KiB,
// bitstream windows 16 KiB, symbols 120 KiB).
constexpr uint32_t kSymLds = 61440;
constexpr int kDecRing = 16;    // words of bitstream per lane in LDS (1-byte codes)
constexpr int kDecPeriod = 8;   // iterations between the reloads of all lanes
// Decoder lanes: two lanes per chunk (one per half, the second from the
// chunk's stored half offset) in 1024-thread workgroups, so one copy of the
// decode tables serves four waves per SIMD.
template <typename CT> struct DecShape {
  static constexpr int NT = 1024;  // threads per workgroup
  static constexpr int LPC = 2;    // lanes per chunk
};

__device__ __forceinline__ uint4 load_words4(const uint32_t* words, uint64_t nwords, uint64_t w) {
  if (w + 4 <= nwords) return *(const uint4*)(words + w);
  uint4 r;
  r.x = (w + 0 < nwords) ? words[w + 0] : 0u;
  r.y = (w + 1 < nwords) ? words[w + 1] : 0u;
  r.z = (w + 2 < nwords) ? words[w + 2] : 0u;
  r.w = (w + 3 < nwords) ? words[w + 3] : 0u;
  return r;
}
__device__ __forceinline__ uint32_t pick4(const uint4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

template <typename CT>
__global__ void __launch_bounds__(DecShape<CT>::NT) decode_kernel(const uint8_t* __restrict__ comp, uint64_t off_bs,
                                                     uint64_t nwords, uint64_t n, uint32_t C, uint64_t n_chunks,
                                                     const uint32_t* cbits, const uint64_t* boff,
                                                     const DecTables* D, const uint32_t* sorted_syms,
                                                     CT* codes, uint32_t* segcnt, int64_t X, int64_t Bx,
                                                     int32_t nbx, DevPlan* P) {
  constexpr int NT = DecShape<CT>::NT, LPC = DecShape<CT>::LPC;
  __shared__ uint32_t lut[4096];
  __shared__ uint32_t s_first[32], s_start[32], s_lim[32];
  constexpr uint32_t kSyms = sizeof(CT) == 1 ? 256 : kSymLds;
  __shared__ uint16_t s_syms[kSyms];
  __shared__ uint32_t s_win[sizeof(CT) == 1 ? 1 : 4][sizeof(CT) == 1 ? 1 : NT];  // each lane's current 16-byte group
  __shared__ uint32_t s_lut2[sizeof(CT) == 1 ? kLut2Max * 16 : 1];
  __shared__ uint2 s_mlut[sizeof(CT) == 1 ? 4096 : 1];
  __shared__ uint32_t s_ring[sizeof(CT) == 1 ? kDecRing : 1][sizeof(CT) == 1 ? NT : 1];  // 1-byte codes: per-lane bitstream ring
  const uint32_t nsorted = D->nsorted;
  const uint32_t nsl = min(nsorted, kSyms);  // symbols held in LDS (the shortest codes')
  const uint32_t n2 = sizeof(CT) == 1 ? D->lut2_n : 0u, p02 = sizeof(CT) == 1 ? D->lut2_p0 : 0u;
  if constexpr (sizeof(CT) == 1)
    if (n2)
      for (uint32_t i = threadIdx.x; i < kLut2Max * 16; i += NT) s_lut2[i] = D->lut2[i];
  for (int i = threadIdx.x; i < 4096; i += NT) lut[i] = D->lut[i];
  if constexpr (sizeof(CT) == 1)
    for (int i = threadIdx.x; i < 4096; i += NT) {
      const uint64_t e = D->mlut[i];
      s_mlut[i] = make_uint2((uint32_t)e, (uint32_t)(e >> 32));
    }
  for (uint32_t i = threadIdx.x; i < nsl; i += NT) s_syms[i] = (uint16_t)sorted_syms[i];
  if (threadIdx.x < 32) {
    s_first[threadIdx.x] = D->first[threadIdx.x];
    s_start[threadIdx.x] = D->start[threadIdx.x];
    s_lim[threadIdx.x] = D->lim[threadIdx.x];
  }
  __syncthreads();
  if (P->status) return;
  const uint64_t gl = (uint64_t)blockIdx.x * NT + threadIdx.x;
  const uint64_t c = gl / LPC;
  if (c >= n_chunks) return;
  const uint32_t hf = (uint32_t)(gl % LPC);  // half of the chunk (two lanes per chunk)
  const int t = threadIdx.x;
  // The bitstream is read in 16-byte aligned groups of 4 words: the group in
  // use sits in this lane's LDS slot, the next one is in flight in registers
  // (never copied, so its load is waited for only when it is needed).
  const uint32_t* words = (const uint32_t*)(comp + off_bs);  // 64-byte aligned section
  // The lane's span of the chunk: the whole chunk, or with two lanes per
  // chunk its first or second half, split at the stored half offset (the
  // u16 table after the chunk bit counts).
  uint64_t pos = boff[c];
  uint64_t end = pos + cbits[c];
  uint64_t i0 = c * C, i1 = min(n, i0 + C);
  if constexpr (LPC == 2) {
    const uint32_t mid = ((const uint16_t*)(cbits + n_chunks))[c];
    if (mid > cbits[c]) {
      set_status(P, SZ_ECORRUPT);
      return;
    }
    if (hf == 0) {
      end = pos + mid;
      i1 = min(i1, i0 + C / 2);
    } else {
      pos += mid;
      i0 = min(i1, i0 + C / 2);
    }
  }
  uint64_t wg = (pos >> 5) & ~3ull;
  uint4 pend = make_uint4(0, 0, 0, 0);
  int wi = 0;
  uint64_t buf = 0;
  int nb = 0;
  if constexpr (sizeof(CT) != 1) {
    const uint4 g0 = load_words4(words, nwords, wg);
    s_win[0][t] = g0.x;
    s_win[1][t] = g0.y;
    s_win[2][t] = g0.z;
    s_win[3][t] = g0.w;
    pend = load_words4(words, nwords, wg + 4);
    wi = (int)((pos >> 5) - wg);  // index of the next word to take from the slot
    buf = ((uint64_t)s_win[wi][t] << 32) << (pos & 31);
    nb = 32 - (int)(pos & 31);
    wi++;
  }
  // row segment of i0: seg = row * nbx + col / Bx, rem = elements left in it
  const uint64_t row0 = i0 / (uint64_t)X, col0 = i0 - row0 * (uint64_t)X;
  int64_t bx = (int64_t)(col0 / (uint64_t)Bx);
  uint64_t seg = row0 * (uint64_t)nbx + (uint64_t)bx;
  int64_t rem = min(X, (bx + 1) * Bx) - (int64_t)col0;
  uint32_t zc = 0;
  constexpr int SB = 8 * sizeof(CT);  // bits per code
  constexpr int PER = 128 / SB;       // codes per 16-byte store
  bool bad = false;
  if constexpr (sizeof(CT) == 1) {
    // Up to four codes per table read: a window whose codes all fit in 12
    // bits, lie inside the chunk and inside the row segment is taken whole;
    // otherwise one code is decoded as below.  Codes leave in aligned 8-byte
    // stores from a byte accumulator (first code lowest).
    // The bitstream reaches each lane through a ring of kDecRing words in
    // LDS, refilled 8 words at a time with loads issued every kDecPeriod
    // iterations and landed at the next period: the waits for them (which
    // also wait for the code stores before them) then come once per period
    // for the whole wave rather than whenever one lane runs out.  A lane
    // that still runs out loads its next word directly (rare).
    // Every counter in the loop is a 32-bit offset from the lane's first
    // code, first word or first bit (a lane spans at most one chunk).
    const uint32_t ni = (uint32_t)(i1 - i0);  // codes of this lane
    CT* const cbase = codes + i0;
    const uint64_t w0 = pos >> 5;
    const uint32_t* const wbase = words + w0;
    // words readable from w0 on (a lane reads fewer than 2^30)
    const uint32_t rnw = w0 < nwords ? (uint32_t)min(nwords - w0, (uint64_t)1 << 30) : 0u;
    auto ld4 = [&](uint32_t r) -> uint4 {
      if (r + 4 <= rnw) return *(const uint4*)(wbase + r);
      uint4 v;
      v.x = (r + 0 < rnw) ? wbase[r + 0] : 0u;
      v.y = (r + 1 < rnw) ? wbase[r + 1] : 0u;
      v.z = (r + 2 < rnw) ? wbase[r + 2] : 0u;
      v.w = (r + 3 < rnw) ? wbase[r + 3] : 0u;
      return v;
    };
    // the end of the current row segment, and the end of what one table
    // read may take (the segment's end or the lane's, whichever is first)
    uint32_t send = (uint32_t)min(rem, (int64_t)ni + 1);
    uint32_t lim = min(send, ni);
    uint64_t acc8 = 0;
    int nab = 0;      // codes pending in acc8 (< 8)
    uint32_t rg = 0;  // offset of the first pending code, a multiple of 8
    uint32_t ri = 0;  // codes decoded
    uint32_t rb = 0;  // bits consumed
#pragma unroll
    for (int q = 0; q < kDecRing / 4; q++) {
      const uint4 g = ld4(4 * q);
      s_ring[4 * q + 0][t] = g.x;
      s_ring[4 * q + 1][t] = g.y;
      s_ring[4 * q + 2][t] = g.z;
      s_ring[4 * q + 3][t] = g.w;
    }
    // word offsets: landed in the ring [fland - kDecRing, fland), requested
    // up to fiss, next to take into buf rword; word r sits in slot r % kDecRing
    uint32_t fland = kDecRing, fiss = kDecRing, rword = 1;
    uint4 p0 = make_uint4(0, 0, 0, 0), p1 = p0;  // in-flight words [fland, fland + 8)
    buf = ((uint64_t)s_ring[0][t] << 32) << (pos & 31);
    nb = 32 - (int)(pos & 31);
    uint32_t it = 0;
    while (ri < ni) {
      if ((it++ & (kDecPeriod - 1)) == 0) {
        if (fiss > fland) {
          const uint32_t wv[8] = {p0.x, p0.y, p0.z, p0.w, p1.x, p1.y, p1.z, p1.w};
#pragma unroll
          for (int q = 0; q < 8; q++) s_ring[(fland + q) & (kDecRing - 1)][t] = wv[q];
          fland += 8;
        }
        if (fland - rword <= (uint32_t)(kDecRing - 8)) {
          p0 = ld4(fland);
          p1 = ld4(fland + 4);
          fiss = fland + 8;
        }
      }
      if (nb < 32 && rword >= fland) {
        // ran out: take the next word directly into its slot
        s_ring[rword & (kDecRing - 1)][t] = rword < rnw ? wbase[rword] : 0u;
        __asm__ volatile("" ::: "memory");
      }
      {
        const bool rf = nb < 32;
        const uint32_t wd = s_ring[rword & (kDecRing - 1)][t];
        buf |= rf ? ((uint64_t)wd << (32 - nb)) : 0ull;
        nb += rf ? 32 : 0;
        rword += rf ? 1 : 0;
      }
      // both tables are read; selects pick the window or its first code, so
      // lanes that take either stay on one path
      const uint32_t w12 = (uint32_t)(buf >> (64 - kLutBits));
      const uint2 me = s_mlut[w12];
      const uint32_t e = lut[w12];
      const uint32_t k = me.y & 0xF;
      const bool fast = k != 0 && ri + k <= lim;
      uint32_t sym = e & 0xFFFF, l1 = e >> 16;
      uint32_t e2 = 0;
      if (e == 0) {
        // (one branch for both rare cases: the common path passes a single test)
        if (n2) {
          // a code of 13..16 bits: the second table, by prefix and next 4 bits
          e2 = s_lut2[(w12 - p02) * 16 + (uint32_t)((buf >> (64 - 16)) & 15)];
          sym = e2 & 0xFFFF;
          l1 = e2 >> 16;
        }
        if (e2 == 0) {
          // a code longer than the tables: its length is the count of limits
          // its 27-bit window reaches
          const uint32_t v27 = (uint32_t)(buf >> (64 - kLmax));
          l1 = kLutBits + 1;
#pragma unroll
          for (int q = kLutBits + 1; q < kLmax; q++) l1 += (v27 >= s_lim[q]) ? 1u : 0u;
          if (v27 >= s_lim[kLmax]) {
            bad = true;
            break;
          }
          const uint32_t idx = s_start[l1] + ((v27 >> (kLmax - l1)) - s_first[l1]);
          if (idx < nsl) {
            sym = s_syms[idx];
          } else {
            sym = sorted_syms[idx];
            __builtin_amdgcn_s_waitcnt(0x0F70);
          }
        }
      }
      const uint32_t syms = fast ? me.x : sym;
      const uint32_t l = fast ? ((me.y >> 4) & 0xF) : l1;
      const uint32_t nz = fast ? ((me.y >> 8) & 0x7) : (sym == 0 ? 1u : 0u);
      const uint32_t kk = fast ? k : 1u;
      buf <<= l;
      nb -= (int)l;
      rb += l;
      zc += nz;
      acc8 |= (uint64_t)syms << (8 * nab);
      if (nab + (int)kk >= 8) {
        *(uint64_t*)(cbase + rg) = acc8;
        acc8 = (nab + (int)kk > 8) ? ((uint64_t)syms >> (8 * (8 - nab))) : 0ull;
        nab = nab + (int)kk - 8;
        rg += 8;
      } else {
        nab += (int)kk;
      }
      ri += kk;
      if (ri == send) {
        if (zc) atomicAdd(&segcnt[seg], zc);
        zc = 0;
        seg++;
        if (++bx == nbx) bx = 0;
        const int64_t seglen = min(X, (bx + 1) * Bx) - bx * Bx;
        send = (uint32_t)min((int64_t)send + seglen, (int64_t)ni + 1);
        lim = min(send, ni);
      }
    }
    if (zc && !bad) atomicAdd(&segcnt[seg], zc);
    if (!bad)
      for (int q = 0; q < nab; q++) cbase[rg + q] = (CT)(acc8 >> (8 * q));
    if (bad || (uint64_t)rb != end - pos) set_status(P, SZ_ECORRUPT);
  } else {
  uint64_t acc_lo = 0, acc_hi = 0;
  int nacc = 0;
  for (uint64_t i = i0; i < i1; i++) {
    if (nb < 32) {
      if (wi == 4) {
        s_win[0][t] = pend.x;
        s_win[1][t] = pend.y;
        s_win[2][t] = pend.z;
        s_win[3][t] = pend.w;
        // re-read the slot from LDS rather than forward pend's registers,
        // which the next load is about to reuse
        __asm__ volatile("" ::: "memory");
        wg += 4;
        pend = load_words4(words, nwords, wg + 4);
        wi = 0;
      }
      buf |= (uint64_t)s_win[wi][t] << (32 - nb);
      nb += 32;
      wi++;
    }
    const uint32_t e = lut[(uint32_t)(buf >> (64 - kLutBits))];
    uint32_t sym, l;
    if (e) {
      sym = e & 0xFFFF;
      l = e >> 16;
    } else {
      const uint32_t v27 = (uint32_t)(buf >> (64 - kLmax));
      l = kLutBits + 1;
#pragma unroll
      for (int q = kLutBits + 1; q < kLmax; q++) l += (v27 >= s_lim[q]) ? 1u : 0u;
      if (v27 >= s_lim[kLmax]) {
        bad = true;
        break;
      }
      const uint32_t idx = s_start[l] + ((v27 >> (kLmax - l)) - s_first[l]);
      if (idx < nsl) {
        sym = s_syms[idx];
      } else {
        sym = sorted_syms[idx];
        // keep the load's register out of the other paths' wait analysis
        __builtin_amdgcn_s_waitcnt(0x0F70);
      }
    }
    buf <<= l;
    nb -= (int)l;
    pos += l;
    // shift the code into a 128-bit accumulator (first code lowest)
    acc_lo = (acc_lo >> SB) | (acc_hi << (64 - SB));
    acc_hi = (acc_hi >> SB) | ((uint64_t)sym << (64 - SB));
    if (++nacc == PER) {
      *(uint4*)(codes + (i + 1 - PER)) =
          make_uint4((uint32_t)acc_lo, (uint32_t)(acc_lo >> 32), (uint32_t)acc_hi, (uint32_t)(acc_hi >> 32));
      nacc = 0;
    }
    zc += (sym == 0) ? 1u : 0u;
    if (--rem == 0) {
      if (zc) atomicAdd(&segcnt[seg], zc);
      zc = 0;
      seg++;
      if (++bx == nbx) bx = 0;
      rem = min(X, (bx + 1) * Bx) - bx * Bx;
    }
  }
  if (zc && !bad) atomicAdd(&segcnt[seg], zc);
  if (!bad && nacc) {
    // ragged end of the array: the last nacc codes sit in the top of the accumulator
    for (int q = 0; q < nacc; q++) {
      const int slot = PER - nacc + q;  // position inside the 128-bit value
      const uint64_t word = slot * SB < 64 ? acc_lo : acc_hi;
      const int sh = (slot * SB) % 64;
      codes[i1 - nacc + q] = (CT)((word >> sh) & ((1ull << SB) - 1));
    }
  }
  if (bad || pos != end) set_status(P, SZ_ECORRUPT);
  }
}

// K9a: kept-bit count of every unpredictable value, summed per group of 1024.
// MSB-first bits of a stream read in order through a 64-bit buffer.
struct SeqBits {
  const uint32_t* w;
  uint64_t nw, next, buf;
  int have;
  __device__ __forceinline__ SeqBits(const uint32_t* words, uint64_t nwords, uint64_t pos)
      : w(words), nw(nwords), next(pos >> 5), buf(0), have(0) {
    refill();
    const int off = (int)(pos & 31);
    buf <<= off;
    have -= off;
  }
  __device__ __forceinline__ void refill() {
    const uint32_t word = next < nw ? w[next] : 0u;
    next++;
    buf |= (uint64_t)word << (32 - have);
    have += 32;
  }
  // 1 <= nb <= 32
  __device__ __forceinline__ uint32_t get(int nb) {
    if (have < nb) refill();
    const uint32_t v = (uint32_t)(buf >> (64 - nb));
    buf <<= nb;
    have -= nb;
    return v;
  }
  __device__ __forceinline__ uint64_t get64(int nb) {  // 0 <= nb <= 64
    if (nb <= 0) return 0;
    if (nb <= 32) return get(nb);
    const uint64_t hi = get(nb - 32);
    return (hi << 32) | get(32);
  }
};

template <typename T>
__device__ __forceinline__ int unpred_kept_bits(uint32_t head, uint64_t ebT_bits) {
  constexpr int MANT = FTr<T>::MANT, EMAX = FTr<T>::EMAX;
  const int e = (int)(head & EMAX);
  const int e_eb = (int)((ebT_bits >> MANT) & (uint64_t)EMAX);
  if (e_eb == 0 || e == EMAX) return MANT;
  if (e == 0 || e < e_eb) return 0;
  return min(e - e_eb, MANT);
}

// Unpredictable values per thread of the two kernels below (at most kUpt,
// `upt` of a launch): each thread reads its values' heads (and then tails)
// in order through a bit buffer, so with many values a block of 256 threads
// covers 4096 of them with one scan; few values run one per thread.
constexpr int kUpt = 16;
inline uint32_t unpred_per_thread(uint64_t U) { return U >= (1u << 20) ? (uint32_t)kUpt : 1u; }

template <typename T>
__global__ void __launch_bounds__(256) unpred_sums_kernel(const uint8_t* comp, uint64_t off_hd, uint64_t hd_words,
                                                          uint64_t U, uint64_t ebT_bits, uint32_t upt,
                                                          uint32_t* rsum, const DevPlan* P) {
  constexpr int HB = 1 + FTr<T>::EXPB;
  __shared__ uint32_t red[4];
  if (P->status) return;
  const uint64_t j0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * upt;
  uint32_t r = 0;
  if (j0 < U) {
    SeqBits hb((const uint32_t*)(comp + off_hd), hd_words, j0 * HB);
    const int cnt = (int)min((uint64_t)upt, U - j0);
    for (int k = 0; k < cnt; k++) r += (uint32_t)unpred_kept_bits<T>(hb.get(HB), ebT_bits);
  }
  r = block_sum<256, uint32_t>(r, red);
  if (threadIdx.x == 0) rsum[blockIdx.x] = r;
}

// K9b: rebuild each unpredictable value from its head and kept tail bits.
template <typename T>
__global__ void __launch_bounds__(256) unpred_values_kernel(const uint8_t* comp, uint64_t off_hd, uint64_t hd_words,
                                                            uint64_t off_tl, uint64_t tl_words, uint64_t U,
                                                            uint64_t ebT_bits, uint32_t upt, const uint64_t* roff,
                                                            uint64_t tail_bits, T* vals, DevPlan* P) {
  using UT = typename FTr<T>::U;
  constexpr int HB = 1 + FTr<T>::EXPB, MANT = FTr<T>::MANT;
  __shared__ uint64_t red[4];
  if (P->status) return;
  const uint64_t j0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * upt;
  const int cnt = j0 < U ? (int)min((uint64_t)upt, U - j0) : 0;
  uint32_t head[kUpt];
  uint64_t r_tot = 0;
  {
    SeqBits hb((const uint32_t*)(comp + off_hd), hd_words, cnt ? j0 * HB : 0);
#pragma unroll
    for (int k = 0; k < kUpt; k++) {
      head[k] = k < cnt ? hb.get(HB) : 0u;
      r_tot += k < cnt ? (uint64_t)unpred_kept_bits<T>(head[k], ebT_bits) : 0ull;
    }
  }
  uint64_t tot;
  const uint64_t pos = roff[blockIdx.x] + block_exscan<256, uint64_t>(r_tot, red, &tot);
  if (!cnt) return;
  SeqBits tb((const uint32_t*)(comp + off_tl), tl_words, pos);
  UT u[kUpt];
#pragma unroll
  for (int k = 0; k < kUpt; k++) {
    const int r = k < cnt ? unpred_kept_bits<T>(head[k], ebT_bits) : 0;
    const uint64_t tail = tb.get64(r);
    u[k] = ((UT)head[k] << MANT) | (r ? (UT)tail << (MANT - r) : (UT)0);
  }
  if (cnt == kUpt) {
    // 16 values from a multiple of 16: aligned 16-byte stores
    constexpr int E = 16 / (int)sizeof(T);
#pragma unroll
    for (int q = 0; q < kUpt / E; q++) {
      uint4 v;
      if constexpr (sizeof(T) == 4)
        v = make_uint4((uint32_t)u[E * q], (uint32_t)u[E * q + 1], (uint32_t)u[E * q + 2], (uint32_t)u[E * q + 3]);
      else
        v = make_uint4((uint32_t)u[E * q], (uint32_t)((uint64_t)u[E * q] >> 32), (uint32_t)u[E * q + 1],
                       (uint32_t)((uint64_t)u[E * q + 1] >> 32));
      *(uint4*)(vals + j0 + E * q) = v;
    }
  } else {
    for (int k = 0; k < cnt; k++) vals[j0 + k] = bits_to<T>(u[k]);
  }
  if (j0 + cnt == U && pos + r_tot != tail_bits) set_status(P, SZ_ECORRUPT);
}

// ------------------------- XOR-coded unpredictable values (flag bit 1)
// Zero codes of each chunk of the decoded code array (one wave per chunk).
template <typename CT>
__global__ void __launch_bounds__(256) chunk_zeros_kernel(const CT* __restrict__ codes, uint64_t n, uint32_t C,
                                                          uint32_t* cz, const DevPlan* P) {
  if (P->status) return;
  const uint64_t n_chunks = (n + C - 1) / C;
  const int lane = threadIdx.x & 63;
  for (uint64_t c = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6); c < n_chunks; c += (uint64_t)gridDim.x * 4) {
    const uint64_t i0 = c * C, i1 = min(n, i0 + C);
    uint32_t z = 0;
    for (uint64_t i = i0 + lane; i < i1; i += 64) z += codes[i] == 0;
    z = wave_sum(z);
    if (lane == 0) cz[c] = z;
  }
}


// One thread per chunk parses the chunk's records in order: the leading
// bytes come from the previous value of the chunk, sign and exponent are
// completed from the stream, the exponent gives the kept bits and so the
// rest of the record.  A chunk whose records do not end where its table
// entry says marks the container corrupt.
template <typename T>
__global__ void __launch_bounds__(256) unpred_xor_kernel(const uint8_t* comp, uint64_t off_tl, uint64_t tl_words,
                                                         const uint32_t* __restrict__ table,
                                                         const uint64_t* __restrict__ roff,
                                                         const uint32_t* __restrict__ cz,
                                                         const uint64_t* __restrict__ uoff, uint64_t n_chunks,
                                                         uint64_t ebT_bits, T* vals, DevPlan* P) {
  using U = typename FTr<T>::U;
  using XR = XorRec<T>;
  constexpr int MANT = FTr<T>::MANT, EMAX = FTr<T>::EMAX;
  if (P->status) return;
  const uint64_t c = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n_chunks) return;
  const int e_eb = (int)((ebT_bits >> MANT) & (uint64_t)EMAX);
  const uint64_t start = roff[c];
  SeqBits br((const uint32_t*)(comp + off_tl), tl_words, start);
  uint64_t consumed = 0;
  U prev = 0;
  T* out = vals + uoff[c];
  const uint32_t cnt = cz[c];
  for (uint32_t k = 0; k < cnt; k++) {
    const int lzb = (int)br.get(XR::LZB);
    if (lzb > XR::BMAX) {
      set_status(P, SZ_ECORRUPT);
      return;
    }
    U u = lzb ? (prev & ~((((U)1) << (XR::W - 8 * lzb)) - 1)) : (U)0;
    const int kk = max(0, XR::HB - 8 * lzb);  // sign and exponent bits still to read
    if (kk) u |= (U)br.get(kk) << (XR::W - 8 * lzb - kk);
    const int e = (int)((u >> MANT) & (U)EMAX);
    int r;
    if (e_eb == 0 || e == EMAX) r = MANT;
    else if (e == 0) r = 0;
    else r = min(max(e - e_eb, 0), MANT);
    const int q = XR::HB + r;
    const int rest = q - 8 * lzb - kk;
    if (rest > 0) u |= (U)br.get64(rest) << (XR::W - q);
    out[k] = bits_to<T>(u);
    prev = u;
    consumed += (uint64_t)XR::LZB + (uint64_t)kk + (uint64_t)(rest > 0 ? rest : 0);
  }
  if (consumed != table[c]) set_status(P, SZ_ECORRUPT);
}

__global__ void check_total_kernel(const uint64_t* got, uint64_t want, DevPlan* P) {
  if (threadIdx.x == 0 && *got != want) set_status(P, SZ_ECORRUPT);
}

}  // namespace
}  // namespace szh
