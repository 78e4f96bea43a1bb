// Sample + CheckMotif + reduction (Algorithms Sample, CheckMotif, ListCount
// and the final line of Estimate).
//
// One thread per sample (grid-stride).  Per sample: a Philox4x32-10 block
// keyed by (seed, stream) at counter (i, attempt); r uniform in [0, W) by
// Lemire reduction of a 64-bit draw; p with S[p] <= r < S[p+1] by binary
// search of the exact CDF; j1, j3 uniform inside the two windows; three
// gathers build e1 = (x, u, t1), e2 = (u, v, t2), e3 = (v, y, t3).
// CheckMotif rejects unless x, u, v, y are distinct, t1 < t2 < t3 and
// t3 - t1 <= delta.  Each later motif edge r becomes the list of times of the
// pair (phi(src_r), phi(dst_r)) inside (t3, t1 + delta], found by three
// binary searches in the pair index.  The number of strictly increasing
// chains through the lists is computed by one merged sweep in time order:
// f[r] counts chains ending in list r at times seen so far; a group of c
// equal timestamps in list r adds c * f[r-1] (f[-1] = 1), applied from the
// last list to the first so equal times never chain.  With one list the
// count is just its length.
//
// Per-thread sums are 64-bit with carries sent straight to the high word, so
// cnt is an exact 128-bit integer whatever the launch shape.
#include <hip/hip_runtime.h>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kSBlock = 256;

struct SampleArgs {
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
  const uint32_t* lo_in;
  const uint32_t* a;
  const uint32_t* lo_out;
  const uint32_t* b;
  const uint64_t* S;
  const uint32_t* wstatus;
  int64_t m;
  int64_t delta;
  uint64_t k;
  uint64_t seed;
  uint64_t i0;
  uint32_t stream_id;
  uint64_t* cnt;
  uint64_t* hits;
  uint32_t* status;
  int32_t* e1;
  int32_t* e2;
  int32_t* e3;
  uint64_t* X;
  MotifPlan plan;
};

// [lo, hi) positions in the pair index of edges va -> vb with time in (t_lo, t_hi]
__device__ __forceinline__ void pair_window(const SampleArgs& A, int32_t va, int32_t vb,
                                            int64_t t_lo, int64_t t_hi, uint32_t* lo,
                                            uint32_t* hi) {
  const uint32_t s0 = A.out_off[va], s1 = A.out_off[va + 1];
  const uint32_t r0 = lower_bound<int32_t>(A.pair_dst, s0, s1, vb);
  const uint32_t r1 = upper_bound<int32_t>(A.pair_dst, r0, s1, vb);
  const uint32_t l = upper_bound<int64_t>(A.pair_t, r0, r1, t_lo);
  const uint32_t h = upper_bound<int64_t>(A.pair_t, l, r1, t_hi);
  *lo = l;
  *hi = h;
}

__device__ __forceinline__ int32_t slot_vertex(int s, int32_t x, int32_t u, int32_t v, int32_t y) {
  return s == 0 ? x : (s == 1 ? u : (s == 2 ? v : y));
}

// X for motif j of the plan (the path already passed the anchor checks)
__device__ uint64_t closure_count(const SampleArgs& A, int j, int32_t x, int32_t u, int32_t v,
                                  int32_t y, int64_t t1, int64_t t3, bool* overflow) {
  const int l = A.plan.n_lists[j];
  if (l == 0) return 1;
  const int64_t t_hi = t1 + A.delta;
  if (l == 1) {
    uint32_t lo, hi;
    pair_window(A, slot_vertex(A.plan.a_slot[j][0], x, u, v, y),
                slot_vertex(A.plan.b_slot[j][0], x, u, v, y), t3, t_hi, &lo, &hi);
    return (uint64_t)(hi - lo);
  }
  uint32_t ptr[kMaxLists], end[kMaxLists];
  uint64_t f[kMaxLists];
#pragma unroll
  for (int r = 0; r < kMaxLists; ++r) {
    ptr[r] = 0;
    end[r] = 0;
    f[r] = 0;
    if (r < l)
      pair_window(A, slot_vertex(A.plan.a_slot[j][r], x, u, v, y),
                  slot_vertex(A.plan.b_slot[j][r], x, u, v, y), t3, t_hi, &ptr[r], &end[r]);
  }
  // An empty list makes X = 0.  The partial totals of the lists before it are
  // bounded by the product of their sizes, so unless that product reaches
  // 2^64 no overflow can be flagged either and the sweep is skipped.
  {
    int first_empty = -1;
#pragma unroll
    for (int r = kMaxLists - 1; r >= 0; --r)
      if (r < l && ptr[r] == end[r]) first_empty = r;
    if (first_empty >= 0) {
      uint64_t prod = 1;
      bool big = false;
#pragma unroll
      for (int r = 0; r < kMaxLists; ++r)
        if (r < first_empty && __builtin_mul_overflow(prod, (uint64_t)(end[r] - ptr[r]), &prod))
          big = true;
      if (!big) return 0;
    }
  }
  const int64_t kNone = INT64_MAX;
  while (true) {
    int64_t tmin = kNone;
#pragma unroll
    for (int r = 0; r < kMaxLists; ++r)
      if (r < l && ptr[r] < end[r]) {
        const int64_t h = A.pair_t[ptr[r]];
        tmin = h < tmin ? h : tmin;
      }
    if (tmin == kNone) break;
#pragma unroll
    for (int r = kMaxLists - 1; r >= 0; --r) {
      if (r < l) {
        uint64_t c = 0;
        while (ptr[r] < end[r] && A.pair_t[ptr[r]] == tmin) {
          ++c;
          ++ptr[r];
        }
        if (c) {
          const uint64_t prev = (r == 0) ? 1ull : f[r - 1];
          uint64_t add;
          if (__builtin_mul_overflow(c, prev, &add)) *overflow = true;
          if (__builtin_add_overflow(f[r], add, &f[r])) *overflow = true;
        }
      }
    }
  }
  return f[l - 1];
}

template <int NM>
__global__ __launch_bounds__(kSBlock) void k_sample(SampleArgs A) {
  // per-thread accumulators live in this thread's own LDS column, so the
  // motif loop can index them at run time without private-memory spills
  __shared__ uint64_t s_acc[NM][kSBlock];
  __shared__ uint32_t s_hit[NM][kSBlock];
  __shared__ uint64_t s_lo[NM][kSBlock / kWave];
  __shared__ uint64_t s_hi[NM][kSBlock / kWave];
  __shared__ uint64_t s_hits[NM][kSBlock / kWave];
  const int tid = threadIdx.x;
  const int nm = A.plan.n_motifs;
  const uint64_t W = A.S[A.m];
  const bool skip = (*A.wstatus != 0) || (W == 0 && !A.e1 && !A.X);
  for (int j = 0; j < NM; ++j) {
    s_acc[j][tid] = 0;
    s_hit[j][tid] = 0;
  }
  uint32_t st_bits = 0;
  const uint64_t stride = (uint64_t)gridDim.x * kSBlock;
  for (uint64_t ii = (uint64_t)blockIdx.x * kSBlock + tid; ii < A.k && !skip; ii += stride) {
    if (W == 0) {
      if (A.e1) {
        A.e1[ii] = -1;
        A.e2[ii] = -1;
        A.e3[ii] = -1;
      }
      if (A.X)
        for (int j = 0; j < nm; ++j) A.X[(uint64_t)j * A.k + ii] = 0;
      continue;
    }
    const uint64_t i = A.i0 + ii;
    const Words4 blk0 = philox_block(A.seed, A.stream_id, i, 0);
    // r uniform in [0, W)
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
    const uint32_t p = upper_bound<uint64_t>(A.S, 0u, (uint32_t)(A.m + 1), r) - 1u;
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
    const int32_t u = A.out_src[p], v = A.out_dst[p];
    const int64_t t2 = A.out_t[p];
    const uint32_t q1 = A.lo_in[p] + j1;
    const uint32_t q3 = A.lo_out[p] + j3;
    const int32_t x = A.in_src[q1];
    const int64_t t1 = A.in_t[q1];
    const int32_t y = A.out_dst[q3];
    const int64_t t3 = A.out_t[q3];
    if (A.e1) {
      A.e1[ii] = A.in_eid[q1];
      A.e2[ii] = A.out_eid[p];
      A.e3[ii] = A.out_eid[q3];
    }
    const bool valid = x != u && x != v && x != y && u != v && u != y && v != y && t1 < t2 &&
                       t2 < t3 && (t3 - t1) <= A.delta;
    bool ovf = false;
#pragma unroll 1
    for (int j = 0; j < nm; ++j) {
      const uint64_t X = valid ? closure_count(A, j, x, u, v, y, t1, t3, &ovf) : 0ull;
      if (A.X) A.X[(uint64_t)j * A.k + ii] = X;
      const uint64_t old = s_acc[j][tid];
      const uint64_t nv = old + X;
      if (nv < old) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], 1ull);
      s_acc[j][tid] = nv;
      s_hit[j][tid] += (X != 0);
    }
    if (ovf) st_bits |= TC_F_OVERFLOW;
  }
  // block reduction of the per-thread sums, then one set of atomics per block
  const int lane = tid & 63, wave = tid >> 6;
  for (int j = 0; j < nm; ++j) {
    const U128 s = wave_sum128(U128{s_acc[j][tid], 0});
    const uint64_t h = wave_sum64((uint64_t)s_hit[j][tid]);
    if (lane == 0) {
      s_lo[j][wave] = s.lo;
      s_hi[j][wave] = s.hi;
      s_hits[j][wave] = h;
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
    for (int w = 0; w < kSBlock / kWave; ++w) {
      s = add128(s, U128{s_lo[j][w], s_hi[j][w]});
      h += s_hits[j][w];
    }
    if (s.lo | s.hi) {
      const uint64_t old = atomicAdd((unsigned long long*)&A.cnt[2 * j], (unsigned long long)s.lo);
      const uint64_t carry = (old + s.lo < old) ? 1ull : 0ull;
      if (s.hi + carry) atomicAdd((unsigned long long*)&A.cnt[2 * j + 1], s.hi + carry);
    }
    if (h) atomicAdd((unsigned long long*)&A.hits[j], (unsigned long long)h);
  }
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

tc_status sample_estimate(const tc_graph* g, const tc_weights* w, const MotifPlan& plan,
                          uint64_t k, uint64_t seed, uint32_t stream_id, uint64_t i0,
                          tc_result* out, hipStream_t st) {
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
  A.lo_in = w->lo_in;
  A.a = w->a;
  A.lo_out = w->lo_out;
  A.b = w->b;
  A.S = w->S;
  A.wstatus = w->status;
  A.m = g->m;
  A.delta = w->delta;
  A.k = k;
  A.seed = seed;
  A.i0 = i0;
  A.stream_id = stream_id;
  A.cnt = out->cnt;
  A.hits = out->hits;
  A.status = out->status;
  A.e1 = out->e1;
  A.e2 = out->e2;
  A.e3 = out->e3;
  A.X = out->X;
  A.plan = plan;
  const int nm = plan.n_motifs;
  hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(64), 0, st, out->cnt, out->hits, out->status,
                     nm);
  uint64_t blocks = (k + kSBlock - 1) / kSBlock;
  if (blocks > 8192) blocks = 8192;
  if (nm == 1)
    hipLaunchKernelGGL(k_sample<1>, dim3((unsigned)blocks), dim3(kSBlock), 0, st, A);
  else if (nm <= 8)
    hipLaunchKernelGGL(k_sample<8>, dim3((unsigned)blocks), dim3(kSBlock), 0, st, A);
  else
    hipLaunchKernelGGL(k_sample<16>, dim3((unsigned)blocks), dim3(kSBlock), 0, st, A);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, (const uint64_t*)out->cnt,
                     (const uint64_t*)w->S, g->m, (const uint32_t*)w->status, k, out->estimate,
                     out->status, nm);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
