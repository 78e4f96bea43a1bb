// Sample + CheckMotif + ListCount + reduction (Algorithms Sample,
// CheckMotif, ListCount and the last line of Estimate).
//
// The k samples are processed in chunks.  Per chunk:
//   k_paths          one thread per sample: a Philox4x32-10 block keyed by
//                    (seed, stream) at counter (i, attempt); r uniform in
//                    [0, W) by Lemire reduction of a 64-bit draw; p with
//                    S[p] <= r < S[p+1] by binary search of the exact CDF;
//                    j1, j3 uniform inside the two windows; gathers give
//                    e1 = (x, u, t1), e2 = (u, v, t2), e3 = (v, y, t3).
//                    CheckMotif rejects unless x, u, v, y are distinct,
//                    t1 < t2 < t3 and t3 - t1 <= delta.  For an accepted path
//                    the window (t3, t1 + delta] of every distinct pair used
//                    by the batch's lists is found once (a hash lookup of the
//                    pair's run, then two binary searches on time) and stored
//                    per sample.  A motif with no list counts 1, with one list
//                    counts its length, with an empty list counts 0; every
//                    other (sample, motif) is appended to a work queue.
//   k_listcount_wave one wavefront per queued item, items handed out by an
//                    atomic counter.  ListCount level by level:
//                      c_1[i] = #{j : L_0[j] < L_1[i]},
//                      c_r[i] = P_{r-1}[#{j : L_{r-1}[j] < L_r[i]}],
//                    where P_r is the exclusive prefix sum of c_r (so that
//                    P_r[q] counts the chains ending among the first q entries
//                    of L_r), and X = sum_i c_{l-1}[i].  The 64 lanes take 64
//                    entries of L_r at a time: a binary search in L_{r-1}, a
//                    lookup of P_{r-1} in LDS and a wavefront prefix scan
//                    that writes P_r back to LDS.  Each level's total is also
//                    summed in 128 bits, which flags a total >= 2^64.
//                    A first pass stages the keys in LDS (lists up to 1,024
//                    entries); a second, narrow pass searches the pair index
//                    in memory (lists up to 65,536 entries).
//   k_listcount_big  items with a longer list: one thread per item runs the
//                    same count as a merged sweep over the lists in time
//                    order.
// Per-thread sums are 64-bit with carries sent straight to the high word, so
// cnt is an exact 128-bit integer whatever the launch shape or item order.
#include <hip/hip_runtime.h>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kSBlock = 256;
constexpr uint64_t kMaxChunk = 1ull << 22;
constexpr int kKeyCap = 1024;      // longest list of the LDS-staged wavefront ListCount
constexpr int kFastWaves = 5120;   // its wavefronts (one prefix-sum scratch slice each)
constexpr int kWideCap = 65536;    // longest list of the global-memory wavefront ListCount
constexpr int kWideWaves = 64;     // its wavefronts

struct SampleArgs {
  // graph
  const uint32_t* out_off;
  const int32_t* out_src;
  const int32_t* out_dst;
  const int32_t* out_eid;
  const int64_t* out_t;
  const int32_t* in_src;
  const int32_t* in_eid;
  const int64_t* in_t;
  const int32_t* pair_dst;
  const int64_t* pair_t;
  const PairSlot* pair_hash;
  int32_t pair_hash_log2;
  // weights
  const uint32_t* lo_in;
  const uint32_t* a;
  const uint32_t* lo_out;
  const uint32_t* b;
  const uint64_t* S;
  const uint64_t* tree;  // levels 1.. of the search tree over S
  uint64_t tree_off[kMaxTreeLevels];
  int32_t tree_levels;
  const uint32_t* wstatus;
  int64_t m;
  int64_t delta;
  // sampling
  uint64_t k;
  uint64_t seed;
  uint64_t i0;
  uint32_t stream_id;
  uint64_t c0;     // first sample (0-based, relative to i0) of this chunk
  uint32_t clen;   // samples in this chunk
  uint32_t chunk;  // stride of the per-sample window arrays
  // outputs
  uint64_t* cnt;
  uint64_t* hits;
  uint32_t* status;
  int32_t* e1;
  int32_t* e2;
  int32_t* e3;
  uint64_t* X;
  // per-chunk scratch
  uint32_t* win_lo;   // [n_pairs][chunk]
  uint32_t* win_len;  // [n_pairs][chunk]
  uint32_t* item_code;  // (local sample index) | (motif << 24)
  uint32_t* item_count;
  uint32_t* item_next;  // work counter of the fast wavefront ListCount
  uint32_t* mid_code;   // items with a list longer than the register ListCount holds
  uint32_t* mid_count;
  uint32_t* wide_code;  // items with a list longer than kKeyCap
  uint32_t* wide_count;
  uint32_t* wide_next;
  uint32_t* big_code;   // items with a list longer than kWideCap
  uint32_t* big_count;
  uint64_t* fast_p;     // [kFastWaves][2][kKeyCap + 1]
  uint64_t* wide_p;     // [kWideWaves][2][kWideCap + 1]
  uint32_t item_cap;
  MotifPlan plan;
};

// [lo, hi) positions in the pair index of edges va -> vb with time in (t_lo, t_hi]
__device__ __forceinline__ void pair_window(const SampleArgs& A, int32_t va, int32_t vb,
                                            int64_t t_lo, int64_t t_hi, uint32_t* lo,
                                            uint32_t* hi) {
  uint32_t r0, r1;
  pair_run(A.pair_hash, A.pair_hash_log2, va, vb, &r0, &r1);
  const uint32_t l = upper_bound<int64_t>(A.pair_t, r0, r1, t_lo);
  const uint32_t h = upper_bound<int64_t>(A.pair_t, l, r1, t_hi);
  *lo = l;
  *hi = h;
}

__device__ __forceinline__ int32_t slot_vertex(int s, int32_t x, int32_t u, int32_t v, int32_t y) {
  return s == 0 ? x : (s == 1 ? u : (s == 2 ? v : y));
}

__device__ __forceinline__ void accumulate(uint64_t* s_acc, uint32_t* s_hit, const SampleArgs& A,
                                           int j, int tid, uint64_t X) {
  const uint64_t old = s_acc[j * kSBlock + tid];
  const uint64_t nv = old + X;
  if (nv < old) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], 1ull);
  s_acc[j * kSBlock + tid] = nv;
  s_hit[j * kSBlock + tid] += (X != 0);
}

// block reduction of the per-thread sums, then one set of atomics per block
__device__ void flush_block(const uint64_t* s_acc, const uint32_t* s_hit, uint64_t* s_red,
                            const SampleArgs& A, int nm, uint32_t st_bits) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int nw = kSBlock / kWave;
  for (int j = 0; j < nm; ++j) {
    const U128 s = wave_sum128(U128{s_acc[j * kSBlock + tid], 0});
    const uint64_t h = wave_sum64((uint64_t)s_hit[j * kSBlock + tid]);
    if (lane == 0) {
      s_red[(j * nw + wave) * 3 + 0] = s.lo;
      s_red[(j * nw + wave) * 3 + 1] = s.hi;
      s_red[(j * nw + wave) * 3 + 2] = h;
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) st_bits |= __shfl_xor(st_bits, off, kWave);
  if (lane == 0 && st_bits) atomicOr(A.status, st_bits);
  __syncthreads();
  if (tid < nm) {
    const int j = tid;
    U128 s{0, 0};
    uint64_t h = 0;
    for (int w = 0; w < nw; ++w) {
      s = add128(s, U128{s_red[(j * nw + w) * 3 + 0], s_red[(j * nw + w) * 3 + 1]});
      h += s_red[(j * nw + w) * 3 + 2];
    }
    if (s.lo | s.hi) {
      const uint64_t old = atomicAdd((unsigned long long*)&A.cnt[2 * j], (unsigned long long)s.lo);
      const uint64_t carry = (old + s.lo < old) ? 1ull : 0ull;
      if (s.hi + carry) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], s.hi + carry);
    }
    if (h) atomicAdd((unsigned long long*)&A.hits[j], (unsigned long long)h);
  }
}

// upper_bound(S, r) - 1 through the 16-ary tree: one 128-byte node per level
__device__ __forceinline__ uint32_t tree_search(const SampleArgs& A, uint64_t r) {
  uint64_t i = 0;
  for (int L = A.tree_levels; L >= 0; --L) {
    const uint64_t* lvl = (L == 0) ? A.S : A.tree + A.tree_off[L];
    const uint64_t node = (L == A.tree_levels) ? 0 : i;
    const ulonglong2* nd = reinterpret_cast<const ulonglong2*>(lvl + 16 * node);
    uint32_t cnt = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const ulonglong2 v = nd[q];
      cnt += (v.x <= r) + (v.y <= r);
    }
    i = 16 * node + cnt - 1;
  }
  return (uint32_t)i;
}

struct PathRec {
  int32_t x, u, v, y;
  int64_t t1, t3;
  uint32_t li;
};

template <int NM>
__global__ __launch_bounds__(kSBlock) void k_paths(SampleArgs A) {
  constexpr int nw = kSBlock / kWave;
  __shared__ uint64_t s_red[NM * nw * 3];
  __shared__ PathRec s_path[kSBlock];
  __shared__ uint32_t s_nvalid;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int nm = A.plan.n_motifs;
  const int np = A.plan.n_pairs;
  const uint64_t W = A.S[A.m];
  const int wave = tid >> 6;
  if (tid == 0) s_nvalid = 0;
  __syncthreads();
  uint32_t st_bits = 0;
  const uint32_t li = blockIdx.x * kSBlock + tid;  // sample index inside the chunk
  const bool active = li < A.clen && *A.wstatus == 0;
  const uint64_t ii = A.c0 + li;                    // output index
  bool valid = false;
  int32_t x = 0, u = 0, v = 0, y = 0;
  int64_t t1 = 0, t3 = 0;
  if (active) {
    if (W == 0) {
      if (A.e1) {
        A.e1[ii] = -1;
        A.e2[ii] = -1;
        A.e3[ii] = -1;
      }
      if (A.X)
        for (int j = 0; j < nm; ++j) A.X[(uint64_t)j * A.k + ii] = 0;
    } else {
      const uint64_t i = A.i0 + ii;  // counter of the random stream
      const Words4 blk0 = philox_block(A.seed, A.stream_id, i, 0);
      uint64_t r;
      bool ok = range64((uint64_t)blk0.x0 | ((uint64_t)blk0.x1 << 32), W, &r);
      for (uint32_t att = 1; !ok && att < kMaxAttempts; ++att) {
        const Words4 bk = philox_block(A.seed, A.stream_id, i, att);
        ok = range64((uint64_t)bk.x0 | ((uint64_t)bk.x1 << 32), W, &r);
      }
      if (!ok) {
        st_bits |= TC_F_RNG;
        r = 0;
      }
      // p with S[p] <= r < S[p+1]
      const uint32_t p = tree_search(A, r);
      const uint32_t ap = A.a[p], bp = A.b[p];
      uint32_t j1, j3;
      ok = range32(blk0.x2, ap, &j1);
      for (uint32_t att = 1; !ok && att < kMaxAttempts; ++att)
        ok = range32(philox_block(A.seed, A.stream_id, i, att).x2, ap, &j1);
      if (!ok) {
        st_bits |= TC_F_RNG;
        j1 = 0;
      }
      ok = range32(blk0.x3, bp, &j3);
      for (uint32_t att = 1; !ok && att < kMaxAttempts; ++att)
        ok = range32(philox_block(A.seed, A.stream_id, i, att).x3, bp, &j3);
      if (!ok) {
        st_bits |= TC_F_RNG;
        j3 = 0;
      }
      u = A.out_src[p];
      v = A.out_dst[p];
      const int64_t t2 = A.out_t[p];
      const uint32_t q1 = A.lo_in[p] + j1;
      const uint32_t q3 = A.lo_out[p] + j3;
      x = A.in_src[q1];
      t1 = A.in_t[q1];
      y = A.out_dst[q3];
      t3 = A.out_t[q3];
      if (A.e1) {
        A.e1[ii] = A.in_eid[q1];
        A.e2[ii] = A.out_eid[p];
        A.e3[ii] = A.out_eid[q3];
      }
      valid = x != u && x != v && x != y && u != v && u != y && v != y && t1 < t2 && t2 < t3 &&
              (t3 - t1) <= A.delta;
    }
  }
  // compact the accepted paths of the block into LDS
  {
    const uint64_t mask = __ballot(valid);
    uint32_t base = 0;
    if (lane == 0 && mask) base = atomicAdd(&s_nvalid, (uint32_t)__popcll(mask));
    base = __shfl(base, 0, kWave);
    if (valid) s_path[base + __popcll(mask & lt_mask)] = PathRec{x, u, v, y, t1, t3, li};
  }
  __syncthreads();
  // one (path, pair) window per task, spread over the block
  const uint32_t nvalid = s_nvalid;
  for (uint32_t task = tid; task < nvalid * (uint32_t)np; task += kSBlock) {
    const uint32_t q = task / nvalid, sidx = task - q * nvalid;
    const PathRec P = s_path[sidx];
    uint32_t lo, hi;
    pair_window(A, slot_vertex(A.plan.pair_a[q], P.x, P.u, P.v, P.y),
                slot_vertex(A.plan.pair_b[q], P.x, P.u, P.v, P.y), P.t3, P.t1 + A.delta, &lo,
                &hi);
    A.win_lo[(uint64_t)q * A.chunk + P.li] = lo;
    A.win_len[(uint64_t)q * A.chunk + P.li] = hi - lo;
  }
  __threadfence_block();
  __syncthreads();
  {
    for (int j = 0; j < nm; ++j) {
      const int l = A.plan.n_lists[j];
      uint64_t X = 0;
      bool defer = false;
      if (valid) {
        if (l == 0) {
          X = 1;
        } else if (l == 1) {
          X = A.win_len[(uint64_t)A.plan.list_pair[j][0] * A.chunk + li];
        } else {
          // an empty list gives 0 unless the lists before it could already
          // hold 2^64 chains (then the count must run to flag it)
          uint64_t prod = 1;
          bool empty = false, big = false;
          for (int r = 0; r < l; ++r) {
            const uint32_t len = A.win_len[(uint64_t)A.plan.list_pair[j][r] * A.chunk + li];
            if (len == 0) empty = true;
            if (!empty && __builtin_mul_overflow(prod, (uint64_t)len, &prod)) big = true;
          }
          if (!empty || big) defer = true;
        }
      }
      // one queue reservation per wave
      const uint64_t mask = __ballot(defer);
      if (mask) {
        const int leader = __ffsll((long long)mask) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(A.item_count, (uint32_t)__popcll(mask));
        base = __shfl(base, leader, kWave);
        if (defer) {
          const uint32_t slot = base + (uint32_t)__popcll(mask & lt_mask);
          A.item_code[slot] = li | ((uint32_t)j << 24);
        }
      }
      if (active && W != 0 && !defer && A.X) A.X[(uint64_t)j * A.k + ii] = X;
      // this sample's resolved count goes straight into the block sums
      const U128 sx = wave_sum128(U128{defer ? 0ull : X, 0});
      const uint64_t h = wave_sum64((!defer && X != 0) ? 1ull : 0ull);
      if (lane == 0) {
        s_red[(j * nw + wave) * 3 + 0] = sx.lo;
        s_red[(j * nw + wave) * 3 + 1] = sx.hi;
        s_red[(j * nw + wave) * 3 + 2] = h;
      }
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) st_bits |= __shfl_xor(st_bits, off, kWave);
  if (lane == 0 && st_bits) atomicOr(A.status, st_bits);
  __syncthreads();
  if (tid < nm) {
    const int j = tid;
    U128 sum{0, 0};
    uint64_t hh = 0;
    for (int w = 0; w < nw; ++w) {
      sum = add128(sum, U128{s_red[(j * nw + w) * 3 + 0], s_red[(j * nw + w) * 3 + 1]});
      hh += s_red[(j * nw + w) * 3 + 2];
    }
    if (sum.lo | sum.hi) {
      const uint64_t old = atomicAdd((unsigned long long*)&A.cnt[2 * j], (unsigned long long)sum.lo);
      const uint64_t carry = (old + sum.lo < old) ? 1ull : 0ull;
      if (sum.hi + carry) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], sum.hi + carry);
    }
    if (hh) atomicAdd((unsigned long long*)&A.hits[j], (unsigned long long)hh);
  }
}

// Number of strictly increasing chains through lists 0..l-1 (pair-index
// ranges [ptr, end)), by the merged sweep described at the top.
template <int ML, bool CHECKED>
__device__ uint64_t sweep(const int64_t* __restrict__ pair_t, uint32_t (&ptr)[ML],
                          const uint32_t (&end)[ML], int l, bool* overflow) {
  // head[r] is the first unconsumed time of list r and nxt[r] the one after
  // it, loaded one step ahead so the sweep rarely waits on memory.
  const int64_t kNone = INT64_MAX;
  int64_t head[ML], nxt[ML];
  uint64_t f[ML];
#pragma unroll
  for (int r = 0; r < ML; ++r) {
    f[r] = 0;
    head[r] = (r < l && ptr[r] < end[r]) ? pair_t[ptr[r]] : kNone;
    nxt[r] = (r < l && ptr[r] + 1 < end[r]) ? pair_t[ptr[r] + 1] : kNone;
  }
  while (true) {
    int64_t tmin = head[0];
#pragma unroll
    for (int r = 1; r < ML; ++r) tmin = head[r] < tmin ? head[r] : tmin;
    if (tmin == kNone) break;
#pragma unroll
    for (int r = ML - 1; r >= 0; --r) {
      if (r < l && head[r] == tmin) {
        uint64_t c = 0;
        do {
          ++c;
          ++ptr[r];
          head[r] = nxt[r];
          nxt[r] = (ptr[r] + 1 < end[r]) ? pair_t[ptr[r] + 1] : kNone;
        } while (head[r] == tmin);
        const uint64_t prev = (r == 0) ? 1ull : f[r - 1];
        if (CHECKED) {
          uint64_t add;
          if (__builtin_mul_overflow(c, prev, &add)) *overflow = true;
          if (__builtin_add_overflow(f[r], add, &f[r])) *overflow = true;
        } else {
          f[r] += c * prev;
        }
      }
    }
  }
  uint64_t X = 0;
#pragma unroll
  for (int r = 0; r < ML; ++r)
    if (r == l - 1) X = f[r];
  return X;
}

// Register-resident ListCount, one wavefront per item (64-thread blocks),
// for items whose lists all have at most 64 * CH entries and whose window is
// shorter than 2^32.  All keys are staged once in LDS as 32-bit offsets from
// the smallest head; lane q of chunk h holds entry 64 h + q of the current
// level.  Per level: the LDS binary search gives pos = #{L_{r-1} < key}, the
// value P_{r-1}[pos] is fetched from the lane that holds prefix entry pos - 1
// (ds_bpermute), and a wavefront scan with a carry across chunks gives P_r.
// Items are taken in a fixed stride; others go to the next queue.
constexpr int kRegKeys = 2048;  // keys staged per item by the register ListCount
template <int NM, int CH>
__global__ __launch_bounds__(kWave) void k_listcount_reg(SampleArgs A,
                                                         const uint32_t* __restrict__ in_code,
                                                         const uint32_t* __restrict__ in_count,
                                                         uint32_t* fwd_code, uint32_t* fwd_count) {
  __shared__ uint32_t s_key[kRegKeys];
  __shared__ uint64_t s_acc[NM];
  __shared__ uint64_t s_hits[NM];
  const int lane = threadIdx.x;
  const int nm = A.plan.n_motifs;
  if (lane < NM) {
    s_acc[lane] = 0;
    s_hits[lane] = 0;
  }
  uint32_t st_bits = 0;
  const uint32_t n_items = *in_count;
  const bool narrow_window = A.delta < ((int64_t)1 << 32);
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const uint32_t code = in_code[it];
    const uint32_t li = code & 0xFFFFFFu;
    const int j = (int)(code >> 24);
    const int l = A.plan.n_lists[j];
    uint32_t my_lo = 0, my_len = 0;
    int64_t my_first = INT64_MAX;
    if (lane < l) {
      const uint64_t q = A.plan.list_pair[j][lane];
      my_lo = A.win_lo[q * A.chunk + li];
      my_len = A.win_len[q * A.chunk + li];
      if (my_len) my_first = A.pair_t[my_lo];
    }
    uint32_t maxlen = my_len;
    int64_t base = my_first;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = __shfl_xor(maxlen, off, kWave);
      maxlen = o > maxlen ? o : maxlen;
      const int64_t b = __shfl_xor(base, off, kWave);
      base = b < base ? b : base;
    }
    // list r's keys start at my_off of lane r (exclusive prefix of the lengths)
    const uint32_t incl = wave_inclusive_scan(my_len);
    const uint32_t my_off = incl - my_len;
    const uint32_t total_keys = __shfl(incl, kWave - 1, kWave);
    if (maxlen > (uint32_t)(kWave * CH) || total_keys > (uint32_t)kRegKeys || !narrow_window) {
      if (lane == 0) fwd_code[atomicAdd(fwd_count, 1u)] = code;
      continue;
    }
    for (int r = 0; r < l; ++r) {
      const uint32_t lo = __shfl(my_lo, r, kWave), len = __shfl(my_len, r, kWave);
      const uint32_t off = __shfl(my_off, r, kWave);
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const uint32_t i = h * kWave + lane;
        if (i < len) s_key[off + i] = (uint32_t)(A.pair_t[lo + i] - base);
      }
    }
    __threadfence_block();
    uint64_t P[CH];  // P[h] on lane q: inclusive prefix through entry 64 h + q
#pragma unroll
    for (int h = 0; h < CH; ++h) P[h] = (uint64_t)(h * kWave + lane + 1);  // level 0: all ones
    U128 total{0, 0};
    for (int r = 1; r < l; ++r) {
      const uint32_t prev_len = __shfl(my_len, r - 1, kWave);
      const uint32_t len = __shfl(my_len, r, kWave);
      const uint32_t* kprev = s_key + __shfl(my_off, r - 1, kWave);
      const uint32_t* kcur = s_key + __shfl(my_off, r, kWave);
      uint64_t Pn[CH];
      uint64_t carry = 0;
      total = U128{0, 0};
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const uint32_t i = h * kWave + lane;
        const bool act = i < len;
        uint32_t pos = 0;
        if (act) pos = lower_bound<uint32_t>(kprev, 0u, prev_len, kcur[i]);
        // P_{r-1}[pos] lives on lane (pos - 1) & 63 of chunk (pos - 1) >> 6
        const uint32_t q = pos - 1;
        const int src = (int)(q & 63u);
        const uint32_t hsrc = q >> 6;
        uint64_t c = 0;
#pragma unroll
        for (int g = 0; g < CH; ++g) {
          const uint32_t lo32 = (uint32_t)__shfl((uint32_t)P[g], src, kWave);
          const uint32_t hi32 = (uint32_t)__shfl((uint32_t)(P[g] >> 32), src, kWave);
          if (hsrc == (uint32_t)g) c = ((uint64_t)hi32 << 32) | lo32;
        }
        if (!act || pos == 0) c = 0;
        const uint64_t inc = wave_inclusive_scan(c);
        Pn[h] = carry + inc;
        total = add128(total, wave_sum128(U128{c, 0}));
        carry += __shfl(inc, kWave - 1, kWave);
      }
      if (total.hi != 0) st_bits |= TC_F_OVERFLOW;
#pragma unroll
      for (int h = 0; h < CH; ++h) P[h] = Pn[h];
    }
    const uint64_t X = total.lo;
    if (lane == 0) {
      if (A.X) A.X[(uint64_t)j * A.k + A.c0 + li] = X;
      const uint64_t old = s_acc[j];
      const uint64_t nv = old + X;
      if (nv < old) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], 1ull);
      s_acc[j] = nv;
      s_hits[j] += (X != 0);
    }
    __threadfence_block();
  }
  if (lane == 0) {
    for (int j = 0; j < nm; ++j) {
      if (s_acc[j]) atomicAdd((unsigned long long*)&A.cnt[2 * j], (unsigned long long)s_acc[j]);
      if (s_hits[j]) atomicAdd((unsigned long long*)&A.hits[j], (unsigned long long)s_hits[j]);
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) st_bits |= __shfl_xor(st_bits, off, kWave);
  if (lane == 0 && st_bits) atomicOr(A.status, st_bits);
}

// One wavefront per item (64-thread blocks).  FAST keeps the keys of the
// previous and the current list in LDS as 32-bit offsets from the smallest
// head, so the searches are LDS probes (lists up to kKeyCap entries, window
// length below 2^32); otherwise the searches read the pair index directly
// (lists up to kWideCap).  Items over the limit go to the next queue.
template <int NM, bool FAST>
__global__ __launch_bounds__(kWave) void k_listcount_wave(SampleArgs A,
                                                          const uint32_t* __restrict__ in_code,
                                                          const uint32_t* __restrict__ in_count,
                                                          uint32_t* in_next, uint32_t* fwd_code,
                                                          uint32_t* fwd_count, uint64_t* pscratch,
                                                          uint32_t cap) {
  __shared__ uint32_t s_key[2][FAST ? kKeyCap : 1];
  __shared__ uint64_t s_acc[NM];
  __shared__ uint64_t s_hits[NM];
  // this wavefront's two prefix-sum buffers (L2-resident; written then read
  // by the same wavefront, ordered by a workgroup fence between levels)
  uint64_t* s_p[2] = {pscratch + (uint64_t)blockIdx.x * 2 * (cap + 1),
                      pscratch + ((uint64_t)blockIdx.x * 2 + 1) * (cap + 1)};
  const int lane = threadIdx.x;
  const int nm = A.plan.n_motifs;
  if (lane < NM) {
    s_acc[lane] = 0;
    s_hits[lane] = 0;
  }
  uint32_t st_bits = 0;
  const uint32_t n_items = *in_count;
  const bool narrow_window = A.delta < ((int64_t)1 << 32);
  while (true) {
    uint32_t it = 0;
    if (lane == 0) it = atomicAdd(in_next, 1u);
    it = __shfl(it, 0, kWave);
    if (it >= n_items) break;
    const uint32_t code = in_code[it];
    const uint32_t li = code & 0xFFFFFFu;
    const int j = (int)(code >> 24);
    const int l = A.plan.n_lists[j];
    // lane r < l holds list r's window and its first time
    uint32_t my_lo = 0, my_len = 0;
    int64_t my_first = INT64_MAX;
    if (lane < l) {
      const uint64_t q = A.plan.list_pair[j][lane];
      my_lo = A.win_lo[q * A.chunk + li];
      my_len = A.win_len[q * A.chunk + li];
      if (FAST && my_len) my_first = A.pair_t[my_lo];
    }
    uint32_t maxlen = my_len;
    int64_t base = my_first;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = __shfl_xor(maxlen, off, kWave);
      maxlen = o > maxlen ? o : maxlen;
      const int64_t b = __shfl_xor(base, off, kWave);
      base = b < base ? b : base;
    }
    if (maxlen > cap || (FAST && !narrow_window)) {
      if (lane == 0) fwd_code[atomicAdd(fwd_count, 1u)] = code;
      continue;
    }
    if (FAST) {
      // keys of list 0
      const uint32_t lo0 = __shfl(my_lo, 0, kWave), len0 = __shfl(my_len, 0, kWave);
      for (uint32_t i = lane; i < len0; i += kWave)
        s_key[0][i] = (uint32_t)(A.pair_t[lo0 + i] - base);
      __threadfence_block();
    }
    U128 total{0, 0};
    int pb = 0;
    for (int r = 1; r < l; ++r) {
      const uint32_t prev_lo = __shfl(my_lo, r - 1, kWave);
      const uint32_t prev_len = __shfl(my_len, r - 1, kWave);
      const uint32_t lo = __shfl(my_lo, r, kWave);
      const uint32_t len = __shfl(my_len, r, kWave);
      const uint32_t* kprev = s_key[(r - 1) & 1];
      uint32_t* kcur = s_key[r & 1];
      const uint64_t* Pprev = s_p[pb ^ 1];
      uint64_t* Pcur = s_p[pb];
      total = U128{0, 0};
      uint64_t carry = 0;
      if (lane == 0) Pcur[0] = 0;
      for (uint32_t c0 = 0; c0 < len; c0 += kWave) {
        const uint32_t i = c0 + lane;
        const bool act = i < len;
        uint64_t c = 0;
        if (act) {
          const int64_t t = A.pair_t[lo + i];
          uint32_t pos;  // entries of L_{r-1} strictly before t
          if (FAST) {
            const uint32_t key = (uint32_t)(t - base);
            kcur[i] = key;
            pos = lower_bound<uint32_t>(kprev, 0u, prev_len, key);
          } else {
            pos = lower_bound<int64_t>(A.pair_t, prev_lo, prev_lo + prev_len, t) - prev_lo;
          }
          c = (r == 1) ? (uint64_t)pos : Pprev[pos];
        }
        const uint64_t inc = wave_inclusive_scan(c);
        if (act) Pcur[i + 1] = carry + inc;
        total = add128(total, wave_sum128(U128{c, 0}));
        carry += __shfl(inc, kWave - 1, kWave);
      }
      if (total.hi != 0) st_bits |= TC_F_OVERFLOW;
      pb ^= 1;
      __threadfence_block();
    }
    const uint64_t X = total.lo;
    if (lane == 0) {
      if (A.X) A.X[(uint64_t)j * A.k + A.c0 + li] = X;
      const uint64_t old = s_acc[j];
      const uint64_t nv = old + X;
      if (nv < old) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], 1ull);
      s_acc[j] = nv;
      s_hits[j] += (X != 0);
    }
  }
  if (lane == 0) {
    for (int j = 0; j < nm; ++j) {
      if (s_acc[j]) atomicAdd((unsigned long long*)&A.cnt[2 * j], (unsigned long long)s_acc[j]);
      if (s_hits[j]) atomicAdd((unsigned long long*)&A.hits[j], (unsigned long long)s_hits[j]);
    }
  }
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) st_bits |= __shfl_xor(st_bits, off, kWave);
  if (lane == 0 && st_bits) atomicOr(A.status, st_bits);
}

// Items with a list longer than kWideCap: one thread per item.
template <int NM>
__global__ __launch_bounds__(kSBlock) void k_listcount_big(SampleArgs A) {
  __shared__ uint64_t s_acc[NM * kSBlock];
  __shared__ uint32_t s_hit[NM * kSBlock];
  __shared__ uint64_t s_red[NM * (kSBlock / kWave) * 3];
  const int tid = threadIdx.x;
  const int nm = A.plan.n_motifs;
  for (int j = 0; j < NM; ++j) {
    s_acc[j * kSBlock + tid] = 0;
    s_hit[j * kSBlock + tid] = 0;
  }
  uint32_t st_bits = 0;
  const uint32_t n_items = *A.big_count;
  for (uint32_t it = blockIdx.x * kSBlock + tid; it < n_items; it += gridDim.x * kSBlock) {
    const uint32_t code = A.big_code[it];
    const uint32_t li = code & 0xFFFFFFu;
    const int j = (int)(code >> 24);
    const int l = A.plan.n_lists[j];
    uint32_t ptr[kMaxLists], end[kMaxLists];
    uint64_t prod = 1;
    bool big = false;
#pragma unroll
    for (int r = 0; r < kMaxLists; ++r) {
      ptr[r] = 0;
      end[r] = 0;
      if (r < l) {
        const uint64_t q = A.plan.list_pair[j][r];
        ptr[r] = A.win_lo[q * A.chunk + li];
        const uint32_t len = A.win_len[q * A.chunk + li];
        end[r] = ptr[r] + len;
        if (__builtin_mul_overflow(prod, (uint64_t)len, &prod)) big = true;
      }
    }
    bool ovf = false;
    const uint64_t X = big ? sweep<kMaxLists, true>(A.pair_t, ptr, end, l, &ovf)
                           : sweep<kMaxLists, false>(A.pair_t, ptr, end, l, &ovf);
    if (ovf) st_bits |= TC_F_OVERFLOW;
    if (A.X) A.X[(uint64_t)j * A.k + A.c0 + li] = X;
    accumulate(s_acc, s_hit, A, j, tid, X);
  }
  flush_block(s_acc, s_hit, s_red, A, nm, st_bits);
}

__global__ void k_zero_result(uint64_t* cnt, uint64_t* hits, uint32_t* status, int nm) {
  const int j = threadIdx.x;
  if (j < nm) {
    cnt[2 * j] = 0;
    cnt[2 * j + 1] = 0;
    hits[j] = 0;
  }
  if (j == 0) *status = 0;
}

__global__ void k_zero_counters(uint32_t* p) {
  // item_count, item_next, wide_count, wide_next, big_count, mid_count
  if (threadIdx.x < 6) p[threadIdx.x] = 0;
}

// C_hat_j = (cnt_j / k) * W, each integer rounded to nearest-even binary64
__global__ void k_finalize(const uint64_t* cnt, const uint64_t* S, int64_t m,
                           const uint32_t* wstatus, uint64_t k, double* est, uint32_t* status,
                           int nm) {
  const int j = threadIdx.x;
  const uint64_t W = S[m];
  if (j < nm) {
    const double c = u128_to_double(cnt[2 * j], cnt[2 * j + 1]);
    est[j] = (W == 0) ? 0.0 : (c / (double)k) * (double)W;
  }
  if (j == 0 && *wstatus) atomicOr(status, *wstatus);
}

// ------------------------------------------------------------ workspace ----
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

uint64_t sample_chunk(uint64_t k) {
  uint64_t c = k < kMaxChunk ? k : kMaxChunk;
  return c < 1 ? 1 : c;
}

struct SampleLayout {
  size_t win_lo, win_len, code, mid, wide, big, counters, fast_p, wide_p, total;
  uint64_t chunk, cap;
};

static SampleLayout sample_layout(uint64_t k, int32_t n_motifs) {
  SampleLayout L;
  L.chunk = sample_chunk(k);
  L.cap = L.chunk * (uint64_t)n_motifs;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  L.win_lo = take((size_t)kMaxPairs * L.chunk * 4);
  L.win_len = take((size_t)kMaxPairs * L.chunk * 4);
  L.code = take(L.cap * 4);
  L.mid = take(L.cap * 4);
  L.wide = take(L.cap * 4);
  L.big = take(L.cap * 4);
  L.counters = take(32);
  L.fast_p = take((size_t)kFastWaves * 2 * (kKeyCap + 1) * 8);
  L.wide_p = take((size_t)kWideWaves * 2 * (kWideCap + 1) * 8);
  L.total = o;
  return L;
}

size_t sample_workspace_bytes(uint64_t k, int32_t n_motifs) {
  return sample_layout(k, n_motifs).total;
}

template <int NM>
static void launch_chunk(const SampleArgs& A, hipStream_t st) {
  const unsigned blocks = (unsigned)((A.clen + kSBlock - 1) / kSBlock);
  hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, A.item_count);
  {
    TimedLaunch tl("k_paths", st);
    hipLaunchKernelGGL(k_paths<NM>, dim3(blocks), dim3(kSBlock), 0, st, A);
  }
  // enough wavefronts to fill the chip; each pulls items until the queue is empty
  {
    TimedLaunch tl("k_listcount_reg", st);
    hipLaunchKernelGGL((k_listcount_reg<NM, 4>), dim3(kFastWaves), dim3(kWave), 0, st, A,
                       (const uint32_t*)A.item_code, (const uint32_t*)A.item_count, A.mid_code,
                       A.mid_count);
  }
  hipLaunchKernelGGL((k_listcount_wave<NM, true>), dim3(kFastWaves), dim3(kWave), 0, st, A,
                     (const uint32_t*)A.mid_code, (const uint32_t*)A.mid_count, A.item_next,
                     A.wide_code, A.wide_count, A.fast_p, (uint32_t)kKeyCap);
  hipLaunchKernelGGL((k_listcount_wave<NM, false>), dim3(kWideWaves), dim3(kWave), 0, st, A,
                     (const uint32_t*)A.wide_code, (const uint32_t*)A.wide_count, A.wide_next,
                     A.big_code, A.big_count, A.wide_p, (uint32_t)kWideCap);
  hipLaunchKernelGGL(k_listcount_big<NM>, dim3(64), dim3(kSBlock), 0, st, A);
}

tc_status sample_estimate(const tc_graph* g, const tc_weights* w, const MotifPlan& plan,
                          uint64_t k, uint64_t seed, uint32_t stream_id, uint64_t i0,
                          tc_result* out, void* ws, size_t ws_bytes, hipStream_t st) {
  const SampleLayout L = sample_layout(k, plan.n_motifs);
  if (!ws || ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  SampleArgs A;
  A.out_off = g->out_off;
  A.out_src = g->out_src;
  A.out_dst = g->out_dst;
  A.out_eid = g->out_eid;
  A.out_t = g->out_t;
  A.in_src = g->in_src;
  A.in_eid = g->in_eid;
  A.in_t = g->in_t;
  A.pair_dst = g->pair_dst;
  A.pair_t = g->pair_t;
  A.pair_hash = (const PairSlot*)g->pair_hash;
  A.pair_hash_log2 = g->pair_hash_log2;
  A.lo_in = w->lo_in;
  A.a = w->a;
  A.lo_out = w->lo_out;
  A.b = w->b;
  A.S = w->S;
  A.tree = (const uint64_t*)w->scratch;
  {
    const STree T = stree_layout(g->m);
    A.tree_levels = T.levels;
    for (int L = 0; L < kMaxTreeLevels; ++L) A.tree_off[L] = L <= T.levels ? T.offset[L] : 0;
  }
  A.wstatus = w->status;
  A.m = g->m;
  A.delta = w->delta;
  A.k = k;
  A.seed = seed;
  A.i0 = i0;
  A.stream_id = stream_id;
  A.chunk = (uint32_t)L.chunk;
  A.cnt = out->cnt;
  A.hits = out->hits;
  A.status = out->status;
  A.e1 = out->e1;
  A.e2 = out->e2;
  A.e3 = out->e3;
  A.X = out->X;
  A.win_lo = (uint32_t*)(base + L.win_lo);
  A.win_len = (uint32_t*)(base + L.win_len);
  A.item_code = (uint32_t*)(base + L.code);
  A.wide_code = (uint32_t*)(base + L.wide);
  A.big_code = (uint32_t*)(base + L.big);
  A.item_count = (uint32_t*)(base + L.counters);
  A.item_next = A.item_count + 1;
  A.wide_count = A.item_count + 2;
  A.wide_next = A.item_count + 3;
  A.big_count = A.item_count + 4;
  A.mid_code = (uint32_t*)(base + L.mid);
  A.mid_count = A.item_count + 5;
  A.fast_p = (uint64_t*)(base + L.fast_p);
  A.wide_p = (uint64_t*)(base + L.wide_p);
  A.item_cap = (uint32_t)L.cap;
  A.plan = plan;
  const int nm = plan.n_motifs;
  hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, st, out->cnt, out->hits, out->status,
                     nm);
  for (uint64_t c0 = 0; c0 < k; c0 += L.chunk) {
    A.c0 = c0;
    A.clen = (uint32_t)((k - c0) < L.chunk ? (k - c0) : L.chunk);
    if (nm == 1)
      launch_chunk<1>(A, st);
    else if (nm <= 8)
      launch_chunk<8>(A, st);
    else
      launch_chunk<16>(A, st);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, (const uint64_t*)out->cnt,
                     (const uint64_t*)w->S, g->m, (const uint32_t*)w->status, k, out->estimate,
                     out->status, nm);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
