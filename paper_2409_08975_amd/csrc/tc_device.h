// Device helpers for gfx950 (wave64): counter-based RNG, exact range
// reduction, branch-light binary searches, 128-bit accumulation and
// wavefront reductions/scans.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/tc.h"

namespace tc {

constexpr int kWave = 64;
constexpr int kMaxAttempts = 1024;

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) -------------------
// Ten rounds of two 32x32->64 multiplies (multipliers 0xD2511F53 and
// 0xCD9E8D57) with the Weyl key schedule (0x9E3779B9, 0xBB67AE85).
struct Words4 {
  uint32_t x0, x1, x2, x3;
};

__host__ __device__ __forceinline__ Words4 philox_block(uint64_t seed, uint32_t stream,
                                                        uint64_t i, uint32_t attempt) {
  uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = attempt, c3 = stream;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Words4{c0, c1, c2, c3};
}

// ---- Lemire range reduction with rejection ---------------------------------
// floor(x * s / 2^64); the draw is rejected iff the low 64 bits of x * s are
// below (2^64 - s) mod s.  The modulo is only needed when low < s.
__device__ __forceinline__ bool range64(uint64_t x, uint64_t s, uint64_t* out) {
  uint64_t lo = x * s;
  uint64_t hi = __umul64hi(x, s);
  if (lo < s) {
    uint64_t thresh = (0ull - s) % s;
    if (lo < thresh) return false;
  }
  *out = hi;
  return true;
}

__device__ __forceinline__ bool range32(uint32_t x, uint32_t s, uint32_t* out) {
  uint64_t p = (uint64_t)x * (uint64_t)s;
  uint32_t lo = (uint32_t)p;
  if (lo < s) {
    uint32_t thresh = (0u - s) % s;
    if (lo < thresh) return false;
  }
  *out = (uint32_t)(p >> 32);
  return true;
}

// Wave-uniform values as scalars.  Wavefront-cooperative kernels
// branch and loop on per-item values (item index, list bounds, maxima,
// carries) that every lane holds identically after a broadcast or a
// butterfly; reading them through v_readfirstlane makes that uniformity
// visible to the compiler, so those branches are scalar and the wavefront is
// never split around them (a split would let lanes run a broadcast from a
// lane that is masked off).
__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
  return ((uint64_t)uni((uint32_t)(v >> 32)) << 32) | uni((uint32_t)v);
}
__device__ __forceinline__ int64_t uni64s(int64_t v) { return (int64_t)uni64((uint64_t)v); }

// ---- searches over sorted device arrays ------------------------------------
// first index in [lo, hi) with a[idx] >= key
template <typename T>
__device__ __forceinline__ uint32_t lower_bound(const T* __restrict__ a, uint32_t lo, uint32_t hi,
                                                T key) {
  uint32_t n = hi - lo;
  while (n > 0) {
    uint32_t half = n >> 1;
    uint32_t mid = lo + half;
    bool go_right = a[mid] < key;
    lo = go_right ? mid + 1 : lo;
    n = go_right ? n - half - 1 : half;
  }
  return lo;
}

// first index in [lo, hi) with a[idx] > key
template <typename T>
__device__ __forceinline__ uint32_t upper_bound(const T* __restrict__ a, uint32_t lo, uint32_t hi,
                                                T key) {
  uint32_t n = hi - lo;
  while (n > 0) {
    uint32_t half = n >> 1;
    uint32_t mid = lo + half;
    bool go_right = !(key < a[mid]);
    lo = go_right ? mid + 1 : lo;
    n = go_right ? n - half - 1 : half;
  }
  return lo;
}

// ---- 128-bit unsigned accumulation ----------------------------------------
struct U128 {
  uint64_t lo, hi;
};

__device__ __forceinline__ U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
  return r;
}

__device__ __forceinline__ U128 shfl_xor128(U128 v, int mask) {
  U128 r;
  r.lo = __shfl_xor(v.lo, mask, kWave);
  r.hi = __shfl_xor(v.hi, mask, kWave);
  return r;
}

__device__ __forceinline__ U128 wave_sum128(U128 v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = add128(v, shfl_xor128(v, off));
  return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// inclusive scan across the wave (lane order)
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v) {
  const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    T o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

// ---- wavefront collectives without LDS traffic -------------------------------
// For code where all 64 lanes are active.  A lane's value moves to another
// lane through DPP (data-parallel primitives: an operand modifier of the
// vector ALU) instead of ds_bpermute, which goes through the LDS crossbar.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  // bound_ctrl: a lane whose source is outside its row reads 0; lanes of
  // rows outside ROW_MASK keep the old value 0
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, true);
}

// Inclusive prefix sum over the wavefront in lane order: shifts by 1, 2, 4
// and 8 lanes inside each row of 16, then lane 15 of rows 0 and 2 added into
// rows 1 and 3, then lane 31 into rows 2 and 3.
__device__ __forceinline__ uint32_t scan_dpp(uint32_t v) {
  v += dpp_u32<0x111, 0xF>(v);
  v += dpp_u32<0x112, 0xF>(v);
  v += dpp_u32<0x114, 0xF>(v);
  v += dpp_u32<0x118, 0xF>(v);
  v += dpp_u32<0x142, 0xA>(v);
  v += dpp_u32<0x143, 0xC>(v);
  return v;
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = dpp_u32<CTRL, ROW_MASK>((uint32_t)v);
  const uint32_t hi = dpp_u32<CTRL, ROW_MASK>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t scan_dpp(uint64_t v) {
  v += dpp_u64<0x111, 0xF>(v);
  v += dpp_u64<0x112, 0xF>(v);
  v += dpp_u64<0x114, 0xF>(v);
  v += dpp_u64<0x118, 0xF>(v);
  v += dpp_u64<0x142, 0xA>(v);
  v += dpp_u64<0x143, 0xC>(v);
  return v;
}

// The value of a lane given by a wave-uniform index, as a scalar.
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int lane) {
  return ((uint64_t)lane_u32((uint32_t)(v >> 32), lane) << 32) | lane_u32((uint32_t)v, lane);
}

// Sum of the 64 lanes' u64 values as 128 bits (exact), uniform.
__device__ __forceinline__ U128 wave_sum128_dpp(uint64_t c) {
  const uint64_t lo = lane_u64(scan_dpp((uint64_t)(uint32_t)c), 63);
  const uint64_t hi = lane_u64(scan_dpp(c >> 32), 63);
  const uint64_t r = lo + (hi << 32);
  return U128{r, (hi >> 32) + (r < lo ? 1ull : 0ull)};
}

// Correctly rounded (round-to-nearest-even) conversion of a 128-bit unsigned
// integer to binary64.  The top 64 significant bits are converted with the
// lowest bit forced to 1 when any lower bit is set (a sticky bit below the
// rounding position keeps the single rounding exact), then scaled exactly.
__device__ __forceinline__ double u128_to_double(uint64_t lo, uint64_t hi) {
  if (hi == 0) return (double)lo;
  int lz = __clzll(hi);
  int shift = 64 - lz;  // bits beyond 64, 1..64
  uint64_t top, rest;
  if (shift == 64) {
    top = hi;
    rest = lo;
  } else {
    top = (hi << (64 - shift)) | (lo >> shift);
    rest = lo << (64 - shift);
  }
  if (rest != 0) top |= 1ull;
  return ldexp((double)top, shift);
}

// ---- pair-run hash table ----------------------------------------------------
struct __align__(16) PairSlot {
  uint64_t key;    // src << 32 | dst, or kPairEmpty
  uint32_t start;  // first position of the run in the pair index
  uint32_t end;    // one past the last
};
constexpr uint64_t kPairEmpty = ~0ull;

__host__ __device__ __forceinline__ uint64_t pair_key(uint32_t a, uint32_t b) {
  return ((uint64_t)a << 32) | (uint64_t)b;
}

__host__ __device__ __forceinline__ uint64_t pair_hash(uint64_t key, int log2cap) {
  return (key * 0x9E3779B97F4A7C15ull) >> (64 - log2cap);
}

// Entries of sampled level k (pair_t[16^k i]) of a pair index of m entries.
__host__ __device__ __forceinline__ int64_t skip_level_len(int64_t m, int k) {
  return (m + ((int64_t)1 << (4 * k)) - 1) >> (4 * k);
}

// Two bisections over the same sorted array, one step of each per round so
// that their loads are in flight together.  On return lo_x is the first
// index in [lo_x, lo_x + n_x) whose value exceeds k_x (or lo_x + n_x).  A
// finished search probes the other's index and ignores the value, so every
// load stays inside a range the caller searches.
__device__ __forceinline__ void upper_bound_pair(const int64_t* __restrict__ a, uint32_t& lo_a,
                                                 uint32_t n_a, int64_t k_a, uint32_t& lo_b,
                                                 uint32_t n_b, int64_t k_b) {
  while ((n_a | n_b) != 0u) {
    const uint32_t h_a = n_a >> 1, h_b = n_b >> 1;
    const uint32_t m_a = lo_a + h_a, m_b = lo_b + h_b;
    const int64_t v_a = a[n_a ? m_a : m_b];
    const int64_t v_b = a[n_b ? m_b : m_a];
    const bool go_a = n_a != 0u && !(k_a < v_a);
    const bool go_b = n_b != 0u && !(k_b < v_b);
    lo_a = go_a ? m_a + 1 : lo_a;
    lo_b = go_b ? m_b + 1 : lo_b;
    n_a = n_a == 0u ? 0u : (go_a ? n_a - h_a - 1 : h_a);
    n_b = n_b == 0u ? 0u : (go_b ? n_b - h_b - 1 : h_b);
  }
}

// Both ends of a window inside the run [r0, r1) of the pair index (times
// sorted): *ra = first position with time > t_a and *rb = first position
// with time > t_b (at least *ra).  For each end, from the coarsest sampled
// level down, a bisection over the samples pair_t[16^k i] inside its range
// cuts the range to the gap between two neighbouring samples; the last step
// bisects at most 16 consecutive times (one or two cache lines).  The probes
// of a long run thus fall mostly on the small sampled levels, which stay in
// cache.  The two ends are searched in lockstep, so a window costs one chain
// of dependent reads instead of two.
__device__ __forceinline__ void run_window(const int64_t* __restrict__ pair_t,
                                           const int64_t* __restrict__ skip, int64_t m,
                                           uint32_t r0, uint32_t r1, int64_t t_a, int64_t t_b,
                                           uint32_t* ra, uint32_t* rb) {
  const int64_t n1 = skip_level_len(m, 1), n2 = skip_level_len(m, 2);
  uint32_t lo_a = r0, hi_a = r1, lo_b = r0, hi_b = r1;
  for (int k = 3; k >= 1; --k) {
    const int sh = 4 * k;
    const uint32_t i0_a = (uint32_t)(((uint64_t)lo_a + ((uint64_t)1 << sh) - 1) >> sh);
    const uint32_t i1_a = hi_a > lo_a ? (hi_a - 1) >> sh : 0u;
    const uint32_t i0_b = (uint32_t)(((uint64_t)lo_b + ((uint64_t)1 << sh) - 1) >> sh);
    const uint32_t i1_b = hi_b > lo_b ? (hi_b - 1) >> sh : 0u;
    // samples i0..i1 lie in [lo, hi); a range of 16 or fewer is left to the
    // last step
    const uint32_t c_a = (hi_a - lo_a > 16u && i1_a >= i0_a) ? i1_a - i0_a + 1 : 0u;
    const uint32_t c_b = (hi_b - lo_b > 16u && i1_b >= i0_b) ? i1_b - i0_b + 1 : 0u;
    if ((c_a | c_b) == 0u) continue;
    const int64_t* C = skip + (k == 1 ? 0 : (k == 2 ? n1 : n1 + n2));
    uint32_t j_a = i0_a, j_b = i0_b;
    upper_bound_pair(C, j_a, c_a, t_a, j_b, c_b, t_b);
    const uint32_t le_a = j_a - i0_a, le_b = j_b - i0_b;  // samples with time <= t
    if (c_a) {
      if (le_a > 0) lo_a = ((i0_a + le_a - 1) << sh) + 1;
      if (le_a < c_a) hi_a = (i0_a + le_a) << sh;
    }
    if (c_b) {
      if (le_b > 0) lo_b = ((i0_b + le_b - 1) << sh) + 1;
      if (le_b < c_b) hi_b = (i0_b + le_b) << sh;
    }
  }
  upper_bound_pair(pair_t, lo_a, hi_a - lo_a, t_a, lo_b, hi_b - lo_b, t_b);
  *ra = lo_a;
  *rb = lo_b > lo_a ? lo_b : lo_a;
}

// [start, end) of the run of edges a -> b in the pair index (empty if none)
__device__ __forceinline__ void pair_run(const PairSlot* __restrict__ tab, int log2cap, int32_t a,
                                         int32_t b, uint32_t* start, uint32_t* end) {
  const uint64_t key = pair_key((uint32_t)a, (uint32_t)b);
  *start = 0;
  *end = 0;
  const uint64_t mask = (1ull << log2cap) - 1;
  uint64_t h = pair_hash(key, log2cap);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const PairSlot sl = tab[h];
    if (sl.key == key) {
      *start = sl.start;
      *end = sl.end;
      return;
    }
    if (sl.key == kPairEmpty) return;
    h = (h + 1) & mask;
  }
}

__device__ __forceinline__ void set_status(uint32_t* status, uint32_t bits) {
  atomicOr(status, bits);
}

}  // namespace tc
