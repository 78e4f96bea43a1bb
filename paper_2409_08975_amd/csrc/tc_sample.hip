// Sample + CheckMotif + ListCount + reduction (Algorithms Sample,
// CheckMotif, ListCount and the last line of Estimate), for one or several
// values of delta at once (each delta with its own weights, all motifs
// sharing the anchor's class and rank order, sample i of every delta drawn
// from the same counter).
//
// The samples are processed in chunks of `chunk` samples per delta.  Per chunk:
//   k_paths          persistent: each block takes (delta, 256-sample tile)
//                    work units.  Per sample: a Philox4x32-10 block keyed by
//                    (seed, stream) at counter (i, attempt); r uniform in
//                    [0, W) by Lemire reduction of a 64-bit draw (or, in the
//                    exhaustive mode, r = the sample's CDF rank); p with
//                    S[p] <= r < S[p+1] through the 16-ary search tree over S;
//                    j1, j3 uniform inside the two side windows; gathers give
//                    the centre e2 = (u, v, t2) and the side edges e1 at u and
//                    e3 at v (either may be absent: a wedge), phi = (x, u, v, y).
//                    CheckMotif rejects unless the anchor's vertices are
//                    distinct, its times strictly increase in rank order and
//                    its span is at most delta.  The accepted anchors of the
//                    tile are compacted in LDS and the window of every
//                    distinct list key (a vertex pair of phi and a segment
//                    between anchor times; for the spine motifs the pair's
//                    times in (t3, t1 + delta]) is found once per anchor
//                    (hash lookup of the pair's run, two binary searches on
//                    time), spread over the block.  A motif with no list
//                    counts 1, with one list its length, with an empty list
//                    0; every other (sample, motif) is queued.
//   k_listcount_reg  one wavefront per queued item, lists up to 256 entries.
//                    ListCount level by level:
//                      c_1[i] = #{j : L_0[j] < L_1[i]},
//                      c_r[i] = P_{r-1}[#{j : L_{r-1}[j] < L_r[i]}],
//                    with P_r the prefix sums of c_r and X = sum_i c_{l-1}[i];
//                    keys staged in LDS, prefix sums held in registers across
//                    the lanes, gathered with ds_bpermute.
//   k_listcount_lds  one wavefront per item, lists up to 1,024 entries: the
//                    same recursion with keys in LDS and prefix sums in
//                    per-wavefront scratch.
//   k_listcount_wide one 128-thread block per item, lists up to 65,536
//                    entries: each level as a merge of L_{r-1} and L_r in
//                    LDS tiles, prefix sums in per-block scratch.
//   k_listcount_w128 items whose level total reached 2^64 in one of the
//                    passes above: the merged pass in 128-bit arithmetic.
//   k_listcount_big  lists longer than 65,536 entries: one thread per item,
//                    merged time sweep in 128-bit counts.
// Block sums are 128-bit and reach the outputs with one set of atomics per
// block, so cnt is exact whatever the launch shape, the item order or the
// tuning.
#include <hip/hip_runtime.h>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kSBlock = 256;
constexpr int kSWaves = kSBlock / kWave;
constexpr int kLiBits = 25;  // local sample index bits of an item code (then 4 motif, 3 delta bits)
static_assert(kLiBits + 4 + 3 <= 32 && kMaxDeltas <= 8, "item code: sample, motif, delta");
constexpr int kKeyCap = 1024;
constexpr int kWideCap = 65536;
constexpr int kMaxFastWaves = 8192;

struct DeltaArgs {
  const uint4* prec;  // [2 m]: {lo_in, a, lo_out, b}, {u, v, t lo, t hi}
  const uint64_t* S;
  const uint64_t* tree;  // levels 1.. of the search tree over S
  const uint32_t* wstatus;
  int64_t delta;
  uint64_t* cnt;
  uint64_t* hits;
  uint32_t* status;
  int32_t* e1;
  int32_t* e2;
  int32_t* e3;
  uint64_t* X;
  const uint32_t* h;  // proposal factors (importance sampling) or null
  const uint64_t* ps1;  // window proposal: prefix sums of side 1's entry factors, or null
  const uint64_t* ps3;  // ... of side 3's
  int32_t is;           // importance sampling (h, ps1 or ps3 set)
  uint32_t* P;
  double* m2;
  uint64_t* xmax;
};

struct SampleArgs {
  // graph
  const uint4* out_rec;  // {dst, eid, t lo, t hi} in out-CSR order
  const uint4* in_rec;   // {src, eid, t lo, t hi} in in-CSR order
  const int32_t* out_eid;
  const int64_t* pair_t;
  const PairSlot* pair_hash;
  int32_t pair_hash_log2;
  const int64_t* pair_skip;
  int64_t m;
  uint64_t tree_off[kMaxTreeLevels];
  int32_t tree_levels;
  // the top levels of every delta's tree (levels tree_cache_lo..tree_levels,
  // the last tree_cache_words words of the tree) are searched from LDS
  int32_t tree_cache_lo;
  uint32_t tree_cache_words;
  uint64_t tree_cache_base;  // word offset of level tree_cache_lo
  // deltas
  int32_t nd;
  DeltaArgs D[kMaxDeltas];
  // sampling
  uint64_t k;
  uint64_t seed;
  uint64_t i0;       // first counter, or (exhaustive) first CDF rank
  uint32_t stream_id;
  int32_t exhaustive;  // anchors of CDF ranks i0 .. i0 + k - 1 instead of random draws
  uint64_t c0;     // first sample (0-based, relative to i0) of this chunk
  uint32_t clen;   // samples per delta in this chunk
  uint32_t chunk;  // stride of the per-sample window arrays
  uint32_t tiles_per_delta;
  // per-chunk scratch
  uint32_t* win_lo;   // [nd][kMaxPairs][chunk]
  uint32_t* win_len;  // [nd][kMaxPairs][chunk]
  uint32_t* item_code;  // local sample | motif << 25 | delta << 29
  uint32_t* item_count;
  uint32_t* mid_code;
  uint32_t* mid_count;
  uint32_t* wide_code;
  uint32_t* wide_count;
  uint32_t* wide_next;
  uint32_t* big_code;
  uint32_t* big_count;
  uint32_t* w128_code;  // items whose count reached 2^64, lists up to kWideCap
  uint32_t* w128_count;
  uint32_t* w128_next;
  uint32_t* samp_h;  // [nd][chunk] proposal factor of each accepted sample
  uint64_t* fast_p;  // [fast waves][2][kKeyCap + 1]
  uint64_t* wide_p;  // [wide blocks][2][kWideCap + 1]
  uint32_t lds_cap;  // longest list of the LDS-key pass (at most kKeyCap)
  struct SpreadSums* spread;  // [kSpread][nd][n_motifs]
  MotifPlan plan;
};

__device__ __forceinline__ uint64_t win_index(const SampleArgs& A, int d, int q, uint32_t li) {
  return ((uint64_t)d * kMaxPairs + q) * A.chunk + li;
}

__device__ __forceinline__ void decode(uint32_t code, uint32_t* li, int* j, int* d) {
  *li = code & ((1u << kLiBits) - 1);
  *j = (int)((code >> kLiBits) & 15u);
  *d = (int)(code >> (kLiBits + 4));
}

// [lo, hi) positions in the pair index of edges va -> vb with time in (t_lo, t_hi]
__device__ __forceinline__ void pair_window(const SampleArgs& A, int32_t va, int32_t vb,
                                            int64_t t_lo, int64_t t_hi, uint32_t* lo,
                                            uint32_t* hi) {
  uint32_t r0, r1;
  pair_run(A.pair_hash, A.pair_hash_log2, va, vb, &r0, &r1);
  run_window(A.pair_t, A.pair_skip, A.m, r0, r1, t_lo, t_hi, lo, hi);
}

__device__ __forceinline__ int32_t slot_vertex(int s, int32_t x, int32_t u, int32_t v, int32_t y) {
  return s == 0 ? x : (s == 1 ? u : (s == 2 ? v : y));
}

// upper_bound(S, r) - 1 through the 16-ary tree: one 128-byte node per
// level, bisected (four 8-byte probes inside one cache line rather than the
// whole node, which keeps the vector-memory traffic of a lane per level low)
// Entries <= r of a sorted 16-entry node (upper_bound over it) in two
// rounds: the three quarter boundaries, then the four entries of the
// quarter, instead of four dependent probes.
__device__ __forceinline__ uint32_t node_count16(const uint64_t* __restrict__ node, uint64_t r) {
  const uint32_t q = (node[3] <= r ? 1u : 0u) + (node[7] <= r ? 1u : 0u) +
                     (node[11] <= r ? 1u : 0u);
  const uint64_t* e = node + 4 * q;
  return 4 * q + (e[0] <= r ? 1u : 0u) + (e[1] <= r ? 1u : 0u) + (e[2] <= r ? 1u : 0u) +
         (e[3] <= r ? 1u : 0u);
}

// s_tree holds the cached top levels of D's tree (see SampleArgs)
__device__ __forceinline__ uint32_t tree_search(const SampleArgs& A, const DeltaArgs& D,
                                                const uint64_t* s_tree, uint64_t r) {
  uint64_t i = 0;
  int L = A.tree_levels;
  for (; L >= 1 && L >= A.tree_cache_lo; --L) {  // uniform bounds
    const uint64_t* lvl = s_tree + (A.tree_off[L] - A.tree_cache_base);
    const uint64_t node = (L == A.tree_levels) ? 0 : i;
    i = 16 * node + node_count16(lvl + 16 * node, r) - 1;  // entries <= r, minus one
  }
  for (; L >= 0; --L) {
    const uint64_t* lvl = (L == 0) ? D.S : D.tree + A.tree_off[L];
    const uint64_t node = (L == A.tree_levels) ? 0 : i;
    i = 16 * node + node_count16(lvl + 16 * node, r) - 1;  // entries <= r, minus one
  }
  return (uint32_t)i;
}

// ---- per-block sums of (delta, motif) and their flush -------------------------
// Dynamic LDS: slot (w, d, j) at w * nd * nm + d * nm + j for NW wavefronts.
struct BlockSums {
  uint64_t lo, hi, hits, xmax;
  double m2;
  uint32_t ovf;
};
extern __shared__ BlockSums s_dyn_sums[];

__host__ __device__ inline size_t sums_bytes(int nw, int nd, int nm) {
  return (size_t)nw * nd * nm * sizeof(BlockSums);
}

__device__ __forceinline__ BlockSums* sums_slot(const SampleArgs& A, int w, int d, int j) {
  const int nm = A.plan.n_motifs;
  return &s_dyn_sums[(w * A.nd + d) * nm + j];
}

template <int NW>
__device__ __forceinline__ void sums_clear(const SampleArgs& A) {
  for (int i = threadIdx.x; i < NW * A.nd * A.plan.n_motifs; i += blockDim.x)
    s_dyn_sums[i] = BlockSums{0, 0, 0, 0, 0.0, 0u};
}

// 128-bit add that reports a carry out (a total >= 2^128)
__device__ __forceinline__ U128 add128c(U128 a, U128 b, bool* ovf) {
  const U128 r = add128(a, b);
  if (r.hi < a.hi || (r.hi == a.hi && r.lo < a.lo)) *ovf = true;
  return r;
}

__device__ __forceinline__ U128 wave_sum128c(U128 v, bool* ovf) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
    v = add128c(v, U128{__shfl_xor(v.lo, off, kWave), __shfl_xor(v.hi, off, kWave)}, ovf);
  return v;
}

__device__ __forceinline__ double wave_sumf64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ void sums_add(BlockSums* p, U128 v, uint64_t h, double sq, bool ovf,
                                         uint64_t xm) {
  bool o = ovf;
  const U128 r = add128c(U128{p->lo, p->hi}, v, &o);
  p->lo = r.lo;
  p->hi = r.hi;
  p->hits += h;
  p->m2 += sq;
  p->xmax = xm > p->xmax ? xm : p->xmax;
  if (o) p->ovf = 1u;
}

// Contribution of one sample to cnt: X for the method's weights; with a
// proposal factor hp, floor(X * 2^64 / hp) by long division in 32-bit limbs.
__device__ __forceinline__ U128 contribution(uint64_t X, bool is, uint32_t hp) {
  if (!is) return U128{X, 0};
  if (X == 0) return U128{0, 0};
  const uint32_t limb[4] = {(uint32_t)(X >> 32), (uint32_t)X, 0u, 0u};
  uint32_t q[4];
  uint64_t rem = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint64_t cur = (rem << 32) | limb[i];
    q[i] = (uint32_t)(cur / hp);
    rem = cur % hp;
  }
  return U128{((uint64_t)q[2] << 32) | q[3], ((uint64_t)q[0] << 32) | q[1]};
}

// (X / hp)^2 in binary64 (no contraction into a later sum)
__device__ __forceinline__ double square_term(uint64_t X, uint32_t hp) {
  if (X == 0) return 0.0;
  const double v = __ddiv_rn((double)X, (double)hp);
  return __dmul_rn(v, v);
}

// Blocks add their sums into one of kSpread copies of the (delta, motif)
// totals (copy blockIdx mod kSpread), so that thousands of blocks do not
// serialise on the same few words in L2; k_finalize reduces the copies in
// a fixed order.
constexpr int kSpread = 64;
struct SpreadSums {
  uint64_t lo, hi, hits, xmax;
  double m2;
};

__device__ __forceinline__ SpreadSums* spread_slot(const SampleArgs& A, int s, int d, int j) {
  return &A.spread[(s * A.nd + d) * A.plan.n_motifs + j];
}

// after a barrier: thread (d, j) adds the slots of all wavefronts to the
// block's copy of the totals
template <int NW>
__device__ void sums_flush(const SampleArgs& A) {
  const int nm = A.plan.n_motifs;
  for (int i = threadIdx.x; i < A.nd * nm; i += blockDim.x) {
    const int d = i / nm, j = i - d * nm;
    U128 sum{0, 0};
    uint64_t h = 0, xm = 0;
    double sq = 0.0;
    bool ovf = false;
    for (int w = 0; w < NW; ++w) {
      const BlockSums* p = sums_slot(A, w, d, j);
      sum = add128c(sum, U128{p->lo, p->hi}, &ovf);
      h += p->hits;
      sq += p->m2;
      xm = p->xmax > xm ? p->xmax : xm;
      if (p->ovf) ovf = true;
    }
    SpreadSums* t = spread_slot(A, (int)(blockIdx.x % kSpread), d, j);
    if (sum.lo | sum.hi) {
      const uint64_t old = atomicAdd((unsigned long long*)&t->lo, (unsigned long long)sum.lo);
      const uint64_t carry = (old + sum.lo < old) ? 1ull : 0ull;
      const uint64_t add_hi = sum.hi + carry;
      if (add_hi < sum.hi) ovf = true;
      if (add_hi) {
        const uint64_t old_hi = atomicAdd((unsigned long long*)&t->hi, (unsigned long long)add_hi);
        if (old_hi + add_hi < old_hi) ovf = true;
      }
    }
    if (h) atomicAdd((unsigned long long*)&t->hits, (unsigned long long)h);
    if (xm) atomicMax((unsigned long long*)&t->xmax, (unsigned long long)xm);
    if (A.D[d].m2 && sq != 0.0) atomicAdd(&t->m2, sq);
    if (ovf) atomicOr(A.D[d].status, TC_F_OVERFLOW | TC_F_MOTIF(j));
  }
}

__device__ __forceinline__ void flag_status(const SampleArgs& A, int d, uint32_t bits) {
  if (bits) atomicOr(A.D[d].status, bits);
}

// ---- paths ------------------------------------------------------------------
// Words of the search tree's top levels kept in LDS by the path kernel (the
// levels above the first one that would not fit; 16 + 32 + 320 words for
// m = 2*10^7), and their place after the gate window lengths.
constexpr int kTreeCache = 384;
__host__ __device__ inline size_t tree_cache_at(int n_gates) {
  return ((size_t)n_gates * kSBlock * 4 + 15) & ~(size_t)15;
}
// An accepted anchor: phi = (x, u, v, y) (x or y is -1 for a wedge's absent
// side) and its times by increasing rank T[0] < T[1] (< T[2]).
struct PathRec {
  int32_t x, u, v, y;
  int64_t T[3];
  uint32_t li;
};

// Window of list key q of an accepted anchor: the pair's times after the
// anchor time of its segment and before the next anchor time, or up to the
// first anchor time + delta after the last one (integer times, so "before
// T" is "at most T - 1").
template <bool GENERAL>
__device__ __forceinline__ void key_window(const SampleArgs& A, const PathRec& P, int q,
                                           int64_t delta, int64_t* lo, int64_t* hi) {
  if (!GENERAL) {  // the spine's lists all come after t3: (t3, t1 + delta]
    *lo = P.T[2];
    *hi = P.T[0] + delta;
    return;
  }
  const int sg = A.plan.pair_seg[q];
  *lo = P.T[sg];
  *hi = sg + 1 < A.plan.n_anchor ? P.T[sg + 1] - 1 : P.T[0] + delta;
}

// Five wavefronts per SIMD (at most 102 VGPRs, no spills in the spine form):
// the kernel waits on L2 and HBM round trips; with chunks of 2^25 samples
// this measured 1.5% faster than seven (72 VGPRs and spills), with 2^22
// chunks seven had been fastest.
// GENERAL = false is the form for the <-,+,<,>> class with the anchor ranks
// in path order (e1, centre, e3) and random draws, with those choices fixed
// at compile time (fewer live registers); GENERAL = true reads them from the
// plan (any class, wedges, the exhaustive mode).
// An edge of a side's window: a uniform position among its `len`, or with
// window factors (prefix sums `ps` over the side's CSR) position j with
// probability (ps[lo+j+1] - ps[lo+j]) / (ps[lo+len] - ps[lo]): a uniform
// integer u below that sum, then the position whose prefix interval holds u
// (bisection).  *g is the chosen position's factor (1 when uniform).  The
// draw takes word `w3` (x3) or x2 of the first attempt passing Lemire's test.
__device__ __forceinline__ uint32_t pick_side(const SampleArgs& A, uint64_t i, const Words4& blk0,
                                              bool w3, const uint64_t* __restrict__ ps,
                                              uint32_t lo, uint32_t len, uint64_t* g,
                                              uint32_t* st) {
  uint64_t base = 0, span = len;
  if (ps) {
    base = ps[lo];
    span = ps[lo + len] - base;
    if (span > 0xFFFFFFFFull) {  // the weight set is flagged too
      *st |= TC_F_OVERFLOW;
      span = 0xFFFFFFFFull;
    }
  }
  uint32_t u = 0;
  bool ok = range32(w3 ? blk0.x3 : blk0.x2, (uint32_t)span, &u);
  for (uint32_t att = 1; !ok && att < kMaxAttempts; ++att) {
    const Words4 bk = philox_block(A.seed, A.stream_id, i, att);
    ok = range32(w3 ? bk.x3 : bk.x2, (uint32_t)span, &u);
  }
  if (!ok) {
    *st |= TC_F_RNG;
    u = 0;
  }
  *g = 1;
  if (!ps) return u;
  // ps[lo + j] - base <= u < ps[lo + j + 1] - base
  uint32_t L = 0, H = len;
  while (H - L > 1) {
    const uint32_t mid = L + ((H - L) >> 1);
    if (ps[lo + mid] - base <= (uint64_t)u)
      L = mid;
    else
      H = mid;
  }
  *g = ps[lo + L + 1] - ps[lo + L];
  return L;
}

template <bool GENERAL>
__global__ __launch_bounds__(kSBlock, 5) void k_paths(SampleArgs A) {
  __shared__ PathRec s_path[kSBlock];
  __shared__ uint32_t s_nvalid;
  __shared__ uint32_t s_mask[kSBlock];     // pairs still needed by each accepted path
  __shared__ uint32_t s_off[kSBlock + 1];  // exclusive prefix of their counts
  __shared__ uint32_t s_wsum[kSWaves];
  __shared__ uint32_t s_qcnt[kSWaves];
  __shared__ uint32_t s_qbase;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int nm = A.plan.n_motifs;
  const int np = A.plan.n_pairs;
  // gate window length per (gate, accepted path), after the block sums in
  // dynamic LDS (sized for the plan's gates only)
  uint32_t* s_glen = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(s_dyn_sums) +
                                                 sums_bytes(kSWaves, A.nd, nm));
  // then the cached top levels of the current delta's tree
  uint64_t* s_tree = reinterpret_cast<uint64_t*>(
      reinterpret_cast<char*>(s_glen) + tree_cache_at(A.plan.n_gates));
  int cached_d = -1;
  sums_clear<kSWaves>(A);
  const uint32_t n_units = A.tiles_per_delta * (uint32_t)A.nd;
  for (uint32_t unit = blockIdx.x; unit < n_units; unit += gridDim.x) {
    const int d = (int)(unit / A.tiles_per_delta);
    const uint32_t tile = unit - (uint32_t)d * A.tiles_per_delta;
    const DeltaArgs& D = A.D[d];
    const uint64_t W = D.S[A.m];
    __syncthreads();  // the previous unit's LDS use is over
    if (tid == 0) s_nvalid = 0;
    if (d != cached_d) {  // uniform over the block
      for (uint32_t k = tid; k < A.tree_cache_words; k += kSBlock)
        s_tree[k] = D.tree[A.tree_cache_base + k];
      cached_d = d;
    }
    __syncthreads();
    uint32_t st_bits = 0;
    const uint32_t li = tile * kSBlock + tid;  // sample index inside the chunk
    const bool active = li < A.clen && *D.wstatus == 0;
    const uint64_t ii = A.c0 + li;  // output index
    bool valid = false;
    int32_t x = -1, u = 0, v = 0, y = -1;
    int64_t Tk[3] = {0, 0, 0};
    uint32_t hp = 1;
    // in exhaustive mode the sample is the anchor of CDF rank i0 + ii
    const uint64_t rank = A.i0 + ii;
    const bool exh = GENERAL && A.exhaustive;
    const bool none = W == 0 || (exh && rank >= W);
    if (active) {
      if (none) {
        if (D.P) D.P[ii] = 0xFFFFFFFFu;
        if (D.e1) {
          D.e1[ii] = -1;
          D.e2[ii] = -1;
          D.e3[ii] = -1;
        }
        if (D.X)
          for (int j = 0; j < nm; ++j) D.X[(uint64_t)j * A.k + ii] = 0;
      } else {
        uint64_t r;
        Words4 blk0{0, 0, 0, 0};
        const uint64_t i = A.i0 + ii;  // counter of the random stream
        if (exh) {
          r = rank;
        } else {
          blk0 = philox_block(A.seed, A.stream_id, i, 0);
          bool ok = range64((uint64_t)blk0.x0 | ((uint64_t)blk0.x1 << 32), W, &r);
          for (uint32_t att = 1; !ok && att < kMaxAttempts; ++att) {
            const Words4 bk = philox_block(A.seed, A.stream_id, i, att);
            ok = range64((uint64_t)bk.x0 | ((uint64_t)bk.x1 << 32), W, &r);
          }
          if (!ok) {
            st_bits |= TC_F_RNG;
            r = 0;
          }
        }
        const uint32_t p = tree_search(A, D, s_tree, r);  // S[p] <= r < S[p+1]
        const uint4 pr0 = D.prec[2 * (uint64_t)p], pr1 = D.prec[2 * (uint64_t)p + 1];
        const uint32_t ap = pr0.y, bp = pr0.w;
        uint32_t j1, j3;
        uint64_t g1 = 1, g3 = 1;  // window factors of the picks
        if (exh) {
          // rank r - S[p] = j1 * b + j3 (b >= 1: w_p = a * b > 0 here)
          const uint64_t jj = r - D.S[p];
          j1 = (uint32_t)(jj / bp);
          j3 = (uint32_t)(jj - (uint64_t)j1 * bp);
        } else {
          j1 = pick_side(A, i, blk0, false, D.ps1, pr0.x, ap, &g1, &st_bits);
          j3 = pick_side(A, i, blk0, true, D.ps3, pr0.z, bp, &g3, &st_bits);
        }
        u = (int32_t)pr1.x;
        v = (int32_t)pr1.y;
        const int64_t t2 = (int64_t)(((uint64_t)pr1.w << 32) | pr1.z);
        // the side edges: a record {other end, eid, t} of the in- or out-CSR
        const int m1 = GENERAL ? (int)A.plan.cls.mode1 : TC_SIDE_IN;
        const int m3 = GENERAL ? (int)A.plan.cls.mode3 : TC_SIDE_OUT;
        int64_t ts[3] = {0, t2, 0};
        int32_t eid1 = -1, eid3 = -1;
        if (m1 != TC_SIDE_NONE) {
          const uint4 er1 = (m1 == TC_SIDE_IN ? A.in_rec : A.out_rec)[pr0.x + j1];
          x = (int32_t)er1.x;
          eid1 = (int32_t)er1.y;
          ts[0] = (int64_t)(((uint64_t)er1.w << 32) | er1.z);
        }
        if (m3 != TC_SIDE_NONE) {
          const uint4 er3 = (m3 == TC_SIDE_IN ? A.in_rec : A.out_rec)[pr0.z + j3];
          y = (int32_t)er3.x;
          eid3 = (int32_t)er3.y;
          ts[2] = (int64_t)(((uint64_t)er3.w << 32) | er3.z);
        }
        if (D.e1) {
          D.e1[ii] = eid1;
          D.e2[ii] = A.out_eid[p];
          D.e3[ii] = eid3;
        }
        if (D.P) D.P[ii] = p;
        // CheckMotif: distinct vertices, times strictly increasing in rank
        // order, all within delta of the first
        const bool has1 = m1 != TC_SIDE_NONE, has3 = m3 != TC_SIDE_NONE;
        valid = u != v && (!has1 || (x != u && x != v)) && (!has3 || (y != u && y != v)) &&
                (!(has1 && has3) || x != y);
        const int na = GENERAL ? A.plan.n_anchor : 3;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
          Tk[kk] = kk < na ? ts[GENERAL ? A.plan.order[kk] : kk] : 0;
        for (int kk = 1; kk < na; ++kk) valid = valid && Tk[kk - 1] < Tk[kk];
        valid = valid && (Tk[na - 1] - Tk[0]) <= D.delta;
        if (D.is && valid) {
          // the path's proposal factor h_p g1 g3 (below 2^32, else flagged)
          const uint64_t hc = D.h ? (uint64_t)D.h[p] : 1ull;
          uint64_t hw = hc * g1;
          if (hw > 0xFFFFFFFFull || (hw *= g3) > 0xFFFFFFFFull) {
            st_bits |= TC_F_OVERFLOW;
            hw = 0xFFFFFFFFull;
          }
          hp = (uint32_t)hw;
          A.samp_h[(uint64_t)d * A.chunk + li] = hp;
        }
      }
    }
    // compact the accepted paths of the tile into LDS
    uint32_t my_sidx = 0;  // this sample's slot among them (if accepted)
    {
      const uint64_t mask = __ballot(valid);
      uint32_t base = 0;
      if (lane == 0 && mask) base = atomicAdd(&s_nvalid, (uint32_t)__popcll(mask));
      base = __shfl(base, 0, kWave);
      my_sidx = base + (uint32_t)__popcll(mask & lt_mask);
      if (valid) s_path[my_sidx] = PathRec{x, u, v, y, {Tk[0], Tk[1], Tk[2]}, li};
    }
    __syncthreads();
    // phase A: the gate pairs of every accepted path, one (path, pair)
    // window per task, spread over the block
    const uint32_t nvalid = s_nvalid;
    const uint32_t ng = (uint32_t)A.plan.n_gates;
    for (uint32_t task = tid; task < nvalid * ng; task += kSBlock) {
      const uint32_t gi = task / nvalid, sidx = task - gi * nvalid;
      const uint32_t q = A.plan.gate_pair[gi];
      const PathRec P = s_path[sidx];
      int64_t tlo, thi;
      key_window<GENERAL>(A, P, (int)q, D.delta, &tlo, &thi);
      uint32_t lo, hi;
      pair_window(A, slot_vertex(A.plan.pair_a[q], P.x, P.u, P.v, P.y),
                  slot_vertex(A.plan.pair_b[q], P.x, P.u, P.v, P.y), tlo, thi, &lo, &hi);
      A.win_lo[win_index(A, d, q, P.li)] = lo;
      A.win_len[win_index(A, d, q, P.li)] = hi - lo;
      s_glen[gi * kSBlock + sidx] = hi - lo;
    }
    __threadfence_block();
    __syncthreads();
    // phase B: the other pairs, only for motifs whose gate window is non-empty
    if ((uint32_t)np > ng) {
      uint32_t mask = 0;
      if (tid < nvalid) {
        for (int j = 0; j < nm; ++j)
          if (A.plan.n_lists[j] >= 2 &&
              s_glen[A.plan.gate_index[A.plan.list_pair[j][0]] * kSBlock + tid] != 0)
            mask |= A.plan.rest_mask[j];
      }
      const uint32_t cnt = (uint32_t)__popc(mask);
      const uint32_t inc = wave_inclusive_scan(cnt);
      if (lane == 63) s_wsum[wave] = inc;
      __syncthreads();
      uint32_t pre = 0;
      for (int w2 = 0; w2 < wave; ++w2) pre += s_wsum[w2];
      s_mask[tid] = mask;
      s_off[tid] = pre + inc - cnt;
      if (tid == kSBlock - 1) s_off[kSBlock] = pre + inc;
      __syncthreads();
      const uint32_t total = s_off[kSBlock];
      for (uint32_t task = tid; task < total; task += kSBlock) {
        // the accepted path of this task: last sidx with s_off[sidx] <= task
        uint32_t lo2 = 0, hi2 = nvalid;
        while (hi2 - lo2 > 1) {
          const uint32_t mid = (lo2 + hi2) >> 1;
          if (s_off[mid] <= task) lo2 = mid; else hi2 = mid;
        }
        const uint32_t sidx = lo2;
        uint32_t mk = s_mask[sidx];
        for (uint32_t skip = task - s_off[sidx]; skip > 0; --skip) mk &= mk - 1;
        const uint32_t q = (uint32_t)__ffs(mk) - 1;
        const PathRec P = s_path[sidx];
        int64_t tlo, thi;
        key_window<GENERAL>(A, P, (int)q, D.delta, &tlo, &thi);
        uint32_t lo, hi;
        pair_window(A, slot_vertex(A.plan.pair_a[q], P.x, P.u, P.v, P.y),
                    slot_vertex(A.plan.pair_b[q], P.x, P.u, P.v, P.y), tlo, thi, &lo, &hi);
        A.win_lo[win_index(A, d, q, P.li)] = lo;
        A.win_len[win_index(A, d, q, P.li)] = hi - lo;
      }
      __threadfence_block();
      __syncthreads();
    }
    uint32_t dmask = 0;
    uint32_t wdefer = 0;
    for (int j = 0; j < nm; ++j) {
      const int l = A.plan.n_lists[j];
      uint64_t X = 0;
      bool defer = false;
      if (valid) {
        if (l == 0) {
          X = 1;
        } else if (l == 1) {
          X = s_glen[A.plan.gate_index[A.plan.list_pair[j][0]] * kSBlock + my_sidx];
        } else {
          // an empty list gives 0 unless the lists before it could already
          // hold 2^64 chains (then the count must run to flag it)
          uint64_t prod = 1;
          bool empty = false, big = false;
          // lists after the first empty one were not searched (gating)
          for (int r = 0; r < l; ++r) {
            const uint32_t q = A.plan.list_pair[j][r];
            const uint32_t gi = A.plan.gate_index[q];
            const uint32_t len =
                gi != 0xFFu ? s_glen[gi * kSBlock + my_sidx] : A.win_len[win_index(A, d, (int)q, li)];
            if (len == 0) {
              empty = true;
              break;
            }
            if (__builtin_mul_overflow(prod, (uint64_t)len, &prod)) big = true;
          }
          if (!empty || big) defer = true;
        }
      }
      if (defer) dmask |= 1u << j;
      wdefer += (uint32_t)__popcll(__ballot(defer));
      if (active && !none && !defer && D.X) D.X[(uint64_t)j * A.k + ii] = X;
      const uint64_t Xc = defer ? 0ull : X;
      // most wavefronts close no path of a motif: their sums are all zero
      const uint64_t nz = __ballot(Xc != 0);
      if (nz) {
        bool ovf = false;
        const U128 sx = wave_sum128c(contribution(Xc, D.is != 0, hp), &ovf);
        const double sq = D.m2 ? wave_sumf64(square_term(Xc, hp)) : 0.0;
        uint64_t xm = Xc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          const uint64_t o = __shfl_xor(xm, off, kWave);
          xm = o > xm ? o : xm;
        }
        if (lane == 0)
          sums_add(sums_slot(A, wave, d, j), sx, (uint64_t)__popcll(nz), sq, ovf, xm);
      }
    }
    // queue the deferred (sample, motif) items of the unit with one
    // reservation for the whole block
    if (lane == 0) s_qcnt[wave] = wdefer;
    __syncthreads();
    if (tid == 0) {
      uint32_t tot = 0;
      for (int w = 0; w < kSWaves; ++w) tot += s_qcnt[w];
      s_qbase = tot ? atomicAdd(A.item_count, tot) : 0u;
    }
    __syncthreads();
    if (uni(wdefer) != 0) {
      uint32_t wbase = s_qbase;
      for (int w = 0; w < wave; ++w) wbase += s_qcnt[w];
      for (int j = 0; j < nm; ++j) {
        const bool dj = (dmask >> j) & 1u;
        const uint64_t mask = __ballot(dj);
        if (dj)
          A.item_code[wbase + (uint32_t)__popcll(mask & lt_mask)] =
              li | ((uint32_t)j << kLiBits) | ((uint32_t)d << (kLiBits + 4));
        wbase += (uint32_t)__popcll(mask);
      }
    }
    __syncthreads();  // s_qcnt and s_qbase are reused by the next unit
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) st_bits |= __shfl_xor(st_bits, off, kWave);
    if (lane == 0) flag_status(A, d, st_bits);
  }
  __syncthreads();
  sums_flush<kSWaves>(A);
}

// ---- ListCount ----------------------------------------------------------------
// Number of strictly increasing chains through lists 0..l-1 (pair-index
// ranges [ptr, end)) by a merged sweep in time order: f[r] counts chains
// ending in list r at times seen so far; a group of c equal times at the head
// of list r adds c * f[r-1] (f[-1] = 1), lists taken last to first so equal
// times never chain.  Counts are 128-bit; *overflow is set when one reaches
// 2^128.  This is the pass for the longest lists and for the items whose
// count reaches 2^64.
__device__ __forceinline__ U128 mul_u64_u128(uint64_t c, U128 f, bool* overflow) {
  // c * f modulo 2^128, flagging a product of 2^128 or more
  const uint64_t lo = c * f.lo;
  const uint64_t carry = __umul64hi(c, f.lo);
  const uint64_t hi_lo = c * f.hi;
  if (__umul64hi(c, f.hi) != 0) *overflow = true;
  const uint64_t hi = hi_lo + carry;
  if (hi < hi_lo) *overflow = true;
  return U128{lo, hi};
}

template <int ML>
__device__ U128 sweep128(const int64_t* __restrict__ pair_t, uint32_t (&ptr)[ML],
                         const uint32_t (&end)[ML], int l, bool* overflow) {
  const int64_t kNone = INT64_MAX;
  int64_t head[ML], nxt[ML];
  U128 f[ML];
#pragma unroll
  for (int r = 0; r < ML; ++r) {
    f[r] = U128{0, 0};
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
        const U128 prev = (r == 0) ? U128{1, 0} : f[r - 1];
        const U128 add = mul_u64_u128(c, prev, overflow);
        const U128 sum = add128(f[r], add);
        if (sum.hi < f[r].hi || (sum.hi == f[r].hi && sum.lo < f[r].lo)) *overflow = true;
        f[r] = sum;
      }
    }
  }
  U128 X{0, 0};
#pragma unroll
  for (int r = 0; r < ML; ++r)
    if (r == l - 1) X = f[r];
  return X;
}

// Items a one-wavefront pass hands on to a later pass.  Lane i holds the
// i-th, and they are queued with one reservation per 64 items (or at the end
// of the pass), instead of one atomic per item on the shared counter.  Call
// with the whole wavefront active; n is uniform.
struct FwdBuf {
  uint32_t code;  // this lane's held item
  uint32_t n;     // items held
};

__device__ __forceinline__ void fwd_flush(FwdBuf& f, uint32_t* count, uint32_t* queue) {
  if (f.n == 0) return;
  const int lane = threadIdx.x & 63;
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(count, f.n);
  base = (uint32_t)__builtin_amdgcn_readfirstlane(base);
  if ((uint32_t)lane < f.n) queue[base + lane] = f.code;
  f.n = 0;
}

__device__ __forceinline__ void fwd_push(FwdBuf& f, uint32_t code, uint32_t* count,
                                         uint32_t* queue) {
  if ((uint32_t)(threadIdx.x & 63) == f.n) f.code = code;
  if (++f.n == (uint32_t)kWave) fwd_flush(f, count, queue);
}

// record one item's count (lane 0 of a one-wavefront block)
__device__ __forceinline__ void item_done(const SampleArgs& A, int d, int j, uint32_t li,
                                          uint64_t X) {
  const DeltaArgs& D = A.D[d];
  if (D.X) D.X[(uint64_t)j * A.k + A.c0 + li] = X;
  const uint32_t hp = D.is ? A.samp_h[(uint64_t)d * A.chunk + li] : 1u;
  sums_add(sums_slot(A, 0, d, j), contribution(X, D.is != 0, hp), X != 0 ? 1ull : 0ull,
           D.m2 ? square_term(X, hp) : 0.0, false, X);
}

// Register-resident wavefront ListCount (64-thread blocks) for items whose
// lists all have at most 64 * CH entries and whose window is shorter than
// 2^32.  Keys are staged once in LDS as 32-bit offsets from the smallest
// head; lane q of chunk h holds entry 64 h + q of the current level.  Per
// level: an LDS binary search gives pos = #{L_{r-1} < key}, P_{r-1}[pos] comes
// from the lane holding prefix entry pos - 1, and a wavefront scan with a
// carry across chunks gives P_r.
// 1,024 keys (4 KB of LDS per one-wavefront block) keep the pass at the 7
// wavefronts per SIMD its registers allow; 2,048 keys capped it at 5.
constexpr int kRegKeys = 1024;
template <int CH>
__global__ __launch_bounds__(kWave) void k_listcount_reg(SampleArgs A) {
  __shared__ uint32_t s_key[kRegKeys];
  const int lane = threadIdx.x;
  sums_clear<1>(A);
  FwdBuf fb{0u, 0u};  // items for the LDS-key pass

  const uint32_t n_items = *A.item_count;
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const uint32_t code = A.item_code[it];
    uint32_t li;
    int j, d;
    decode(code, &li, &j, &d);
    const int l = A.plan.n_lists[j];
    uint32_t my_lo = 0, my_len = 0;
    int64_t my_first = INT64_MAX;
    if (lane < l) {
      const uint64_t wi = win_index(A, d, A.plan.list_pair[j][lane], li);
      my_lo = A.win_lo[wi];
      my_len = A.win_len[wi];
      if (my_len) my_first = A.pair_t[my_lo];
    }
    // longest list and smallest head time, read lane by lane as scalars
    uint32_t maxlen = 0;
    int64_t base = INT64_MAX;
    for (int r = 0; r < l; ++r) {
      const uint32_t len_r = lane_u32(my_len, r);
      const int64_t first_r = (int64_t)lane_u64((uint64_t)my_first, r);
      maxlen = len_r > maxlen ? len_r : maxlen;
      base = first_r < base ? first_r : base;
    }
    // list r's keys start at my_off of lane r (exclusive prefix of the lengths)
    const uint32_t incl = scan_dpp(my_len);
    const uint32_t my_off = incl - my_len;
    const uint32_t total_keys = lane_u32(incl, kWave - 1);
    if (maxlen > (uint32_t)(kWave * CH) || total_keys > (uint32_t)kRegKeys ||
        A.D[d].delta >= ((int64_t)1 << 32)) {
      fwd_push(fb, code, A.mid_count, A.mid_code);
      continue;
    }
    for (int r = 0; r < l; ++r) {
      const uint32_t lo = lane_u32(my_lo, r), len = lane_u32(my_len, r);
      const uint32_t off = lane_u32(my_off, r);
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        const uint32_t i = h * kWave + lane;
        if (i < len) s_key[off + i] = (uint32_t)(A.pair_t[lo + i] - base);
      }
    }
    __threadfence_block();
    uint64_t P[CH];  // P[h] on lane q: prefix through entry 64 h + q
#pragma unroll
    for (int h = 0; h < CH; ++h) P[h] = (uint64_t)(h * kWave + lane + 1);  // level 0: all ones
    // Level totals: T_0 = |L_0| and T_r <= |L_r| T_{r-1}.  While that bound
    // stays below 2^64 the running 64-bit carry is the exact total; only
    // otherwise are the 128-bit level sums formed (to detect overflow).
    uint64_t t_prev = lane_u32(my_len, 0);
    bool sat = false;  // a level total reached 2^64 (results undefined)
    for (int r = 1; r < l; ++r) {
      const uint32_t prev_len = lane_u32(my_len, r - 1);
      const uint32_t len = lane_u32(my_len, r);
      const uint32_t* kprev = s_key + lane_u32(my_off, r - 1);
      const uint32_t* kcur = s_key + lane_u32(my_off, r);
      const uint32_t nch = (len + kWave - 1) / kWave;       // chunks of this level
      const uint32_t pch = (prev_len + kWave - 1) / kWave;  // chunks of the previous one
      uint64_t bound;
      const bool exact64 = !sat && !__builtin_mul_overflow((uint64_t)len, t_prev, &bound);
      uint64_t Pn[CH];
      if (exact64 && bound < (1ull << 32)) {
        // Every prefix of the previous level is at most T_{r-1} and every
        // prefix of this one at most |L_r| T_{r-1} < 2^32: the level runs in
        // 32 bits (one lane exchange per gathered value, a 32-bit scan).
        uint32_t carry32 = 0;
#pragma unroll
        for (int h = 0; h < CH; ++h) {
          Pn[h] = 0;
          if ((uint32_t)h < nch) {  // uniform over the wavefront
            const uint32_t i = h * kWave + lane;
            const bool act = i < len;
            uint32_t pos = 0;
            if (act) pos = lower_bound<uint32_t>(kprev, 0u, prev_len, kcur[i]);
            const uint32_t q = pos - 1;
            const int src = (int)(q & 63u);
            const uint32_t hsrc = q >> 6;
            uint32_t c = 0;
#pragma unroll
            for (int g = 0; g < CH; ++g) {
              if ((uint32_t)g < pch) {
                const uint32_t v32 = (uint32_t)__shfl((uint32_t)P[g], src, kWave);
                if (hsrc == (uint32_t)g) c = v32;
              }
            }
            if (!act || pos == 0) c = 0;
            const uint32_t inc = scan_dpp(c);
            Pn[h] = (uint64_t)(carry32 + inc);
            carry32 += lane_u32(inc, kWave - 1);
          }
        }
        t_prev = carry32;
#pragma unroll
        for (int h = 0; h < CH; ++h) P[h] = Pn[h];
        continue;
      }
      uint64_t carry = 0;
      U128 total{0, 0};
#pragma unroll
      for (int h = 0; h < CH; ++h) {
        Pn[h] = 0;
        if ((uint32_t)h < nch) {  // uniform over the wavefront
          const uint32_t i = h * kWave + lane;
          const bool act = i < len;
          uint32_t pos = 0;
          if (act) pos = lower_bound<uint32_t>(kprev, 0u, prev_len, kcur[i]);
          const uint32_t q = pos - 1;  // prefix entry pos - 1: lane q & 63 of chunk q >> 6
          const int src = (int)(q & 63u);
          const uint32_t hsrc = q >> 6;
          uint64_t c = 0;
#pragma unroll
          for (int g = 0; g < CH; ++g) {
            if ((uint32_t)g < pch) {
              const uint32_t lo32 = (uint32_t)__shfl((uint32_t)P[g], src, kWave);
              const uint32_t hi32 = (uint32_t)__shfl((uint32_t)(P[g] >> 32), src, kWave);
              if (hsrc == (uint32_t)g) c = ((uint64_t)hi32 << 32) | lo32;
            }
          }
          if (!act || pos == 0) c = 0;
          const uint64_t inc = scan_dpp(c);
          Pn[h] = carry + inc;
          if (!exact64) total = add128(total, wave_sum128_dpp(c));
          carry += lane_u64(inc, kWave - 1);
        }
      }
      if (exact64) {
        t_prev = carry;
      } else {
        const uint64_t thi = uni64(total.hi), tlo = uni64(total.lo);
        if (thi != 0) sat = true;
        t_prev = thi ? ~0ull : tlo;
      }
#pragma unroll
      for (int h = 0; h < CH; ++h) P[h] = Pn[h];
    }
    // a level total of 2^64 or more: the 128-bit pass counts the item
    if (sat) {
      if (lane == 0) A.w128_code[atomicAdd(A.w128_count, 1u)] = code;
    } else if (lane == 0) {
      item_done(A, d, j, li, t_prev);
    }
    __threadfence_block();
  }
  fwd_flush(fb, A.mid_count, A.mid_code);
  __syncthreads();
  sums_flush<1>(A);
}

// Wavefront-per-item ListCount (64-thread blocks) for lists up to kKeyCap
// entries in a window shorter than 2^32: the keys of the previous and the
// current list sit in LDS as 32-bit offsets from the smallest head, the
// prefix sums in per-wavefront scratch.  Longer lists or wider windows go to
// the merged block-per-item pass.
// CAP (512 or 1,024, at least the lds_list_cap knob) sizes the key tiles:
// at 512 a wavefront takes 4 KB of LDS and eight fit per SIMD, at 1,024
// five.
template <int CAP>
__global__ __launch_bounds__(kWave) void k_listcount_lds(SampleArgs A, uint64_t* pscratch) {
  __shared__ uint32_t s_key[2][CAP];
  uint64_t* s_p[2] = {pscratch + (uint64_t)blockIdx.x * 2 * (kKeyCap + 1),
                      pscratch + ((uint64_t)blockIdx.x * 2 + 1) * (kKeyCap + 1)};
  const int lane = threadIdx.x;
  sums_clear<1>(A);
  FwdBuf fb{0u, 0u};  // items for the merged pass
  const uint32_t n_items = *A.mid_count;
  // items are dealt round robin (the loop index is uniform over the
  // wavefront; no shared counter is contended)
  for (uint32_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const uint32_t code = A.mid_code[it];
    uint32_t li;
    int j, d;
    decode(code, &li, &j, &d);
    const int l = A.plan.n_lists[j];
    uint32_t my_lo = 0, my_len = 0;
    int64_t my_first = INT64_MAX;
    if (lane < l) {
      const uint64_t wi = win_index(A, d, A.plan.list_pair[j][lane], li);
      my_lo = A.win_lo[wi];
      my_len = A.win_len[wi];
      if (my_len) my_first = A.pair_t[my_lo];
    }
    // longest list and smallest head time, read lane by lane as scalars
    uint32_t maxlen = 0;
    int64_t base = INT64_MAX;
    for (int r = 0; r < l; ++r) {
      const uint32_t len_r = lane_u32(my_len, r);
      const int64_t first_r = (int64_t)lane_u64((uint64_t)my_first, r);
      maxlen = len_r > maxlen ? len_r : maxlen;
      base = first_r < base ? first_r : base;
    }
    const bool fwd = maxlen > A.lds_cap || A.D[d].delta >= ((int64_t)1 << 32);
    U128 total{0, 0};
    bool sat = false;  // a level total reached 2^64
    if (!fwd) {
      const uint32_t lo0 = lane_u32(my_lo, 0), len0 = lane_u32(my_len, 0);
      for (uint32_t i = lane; i < len0; i += kWave)
        s_key[0][i] = (uint32_t)(A.pair_t[lo0 + i] - base);
      __threadfence_block();
      int pb = 0;
      // Level totals: T_0 = |L_0| and T_r <= |L_r| T_{r-1}.  While that bound
      // is below 2^64 the running 64-bit carry is the exact total (no 128-bit
      // sums); below 2^32 the level's prefix sums are kept as 32-bit words.
      uint64_t t_prev = lane_u32(my_len, 0);
      bool prev32 = false;
      for (int r = 1; r < l; ++r) {
        const uint32_t prev_len = lane_u32(my_len, r - 1);
        const uint32_t lo = lane_u32(my_lo, r);
        const uint32_t len = lane_u32(my_len, r);
        const uint32_t* kprev = s_key[(r - 1) & 1];
        uint32_t* kcur = s_key[r & 1];
        const uint64_t* Pprev = s_p[pb ^ 1];
        uint64_t* Pcur = s_p[pb];
        uint64_t bound;
        const bool exact64 = !sat && !__builtin_mul_overflow((uint64_t)len, t_prev, &bound);
        const bool cur32 = exact64 && bound < (1ull << 32);
        total = U128{0, 0};
        uint64_t carry = 0;
        if (lane == 0) {
          if (cur32)
            reinterpret_cast<uint32_t*>(Pcur)[0] = 0u;
          else
            Pcur[0] = 0;
        }
        for (uint32_t c0 = 0; c0 < len; c0 += kWave) {
          const uint32_t i = c0 + lane;
          const bool act = i < len;
          uint64_t c = 0;
          if (act) {
            const uint32_t key = (uint32_t)(A.pair_t[lo + i] - base);
            kcur[i] = key;
            const uint32_t pos = lower_bound<uint32_t>(kprev, 0u, prev_len, key);
            c = (r == 1) ? (uint64_t)pos
                         : (prev32 ? (uint64_t)reinterpret_cast<const uint32_t*>(Pprev)[pos]
                                   : Pprev[pos]);
          }
          const uint64_t inc = scan_dpp(c);
          if (act) {
            if (cur32)
              reinterpret_cast<uint32_t*>(Pcur)[i + 1] = (uint32_t)(carry + inc);
            else
              Pcur[i + 1] = carry + inc;
          }
          if (!exact64) total = add128(total, wave_sum128_dpp(c));
          carry += lane_u64(inc, kWave - 1);
        }
        if (exact64) {
          t_prev = carry;
        } else {
          total = U128{uni64(total.lo), uni64(total.hi)};
          if (total.hi != 0) sat = true;  // the 128-bit pass takes the item
          t_prev = total.hi ? ~0ull : total.lo;
        }
        prev32 = cur32;
        pb ^= 1;
        __threadfence_block();
      }
      total = U128{t_prev, 0};
    }
    if (fwd)
      fwd_push(fb, code, A.wide_count, A.wide_code);
    else if (sat) {
      if (lane == 0) A.w128_code[atomicAdd(A.w128_count, 1u)] = code;
    } else if (lane == 0)
      item_done(A, d, j, li, total.lo);
  }
  fwd_flush(fb, A.wide_count, A.wide_code);
  __syncthreads();
  sums_flush<1>(A);
}

// Block-per-item ListCount for lists up to kWideCap entries (128 threads).
// Level r is a merge of the sorted times of L_{r-1} (A) and L_r (B): a step
// stages a tile of A's times and of P_{r-1} in LDS and gives every thread four
// consecutive entries of B; an entry is settled in this step when its time
// is at most the tile's last time (or the tile ends A), and then
//   pos = a0 + #{tile entries < t},  c = P_{r-1}[pos]
// and P_r over the settled entries is a block scan with a carry across steps.
// Settled entries are a prefix of B's tile.  If all are settled the next step
// starts A at the last one's position; otherwise the tile is used up and A
// restarts past it, first jumping by a 128-way probe of A to within one tile
// of the first unsettled time.  Each step settles B's tile or moves A by a
// full tile, so a level reads A, B and P_{r-1} once, in coalesced tiles.
constexpr int kWBlock = 128;
constexpr int kWWaves = kWBlock / kWave;
constexpr int kWPer = 4;
constexpr int kWTile = kWBlock * kWPer;  // entries of B per step, of A per tile
constexpr int kDefaultWideBlocks = 4096;
constexpr int kMaxWideBlocks = 4096;

// Seven wavefronts per SIMD (72 VGPRs): measured 7% faster than the
// compiler's unbounded 105 VGPRs (4 per SIMD) on the batched workload.
__global__ __launch_bounds__(kWBlock, 7) void k_listcount_wide(SampleArgs A, uint64_t* pscratch) {
  __shared__ int64_t sA[kWTile];
  __shared__ uint64_t sP[kWTile + 1];
  __shared__ uint64_t s_wsum[kWWaves];
  __shared__ uint64_t s_wlo[kWWaves], s_whi[kWWaves];
  __shared__ uint32_t s_wset[kWWaves];
  __shared__ uint32_t s_lo[kMaxLists], s_len[kMaxLists];
  __shared__ uint32_t s_item, s_last_pos;
  __shared__ int64_t s_key0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t* Pbuf[2] = {pscratch + (uint64_t)blockIdx.x * 2 * (kWideCap + 1),
                       pscratch + ((uint64_t)blockIdx.x * 2 + 1) * (kWideCap + 1)};
  // Blocks past the item count leave at once (uniformly): the others keep
  // claiming until the counter passes the count, so every item is taken,
  // and an empty pass costs no contended claims.
  const uint32_t n_items = *A.wide_count;
  if (blockIdx.x >= n_items) return;
  sums_clear<1>(A);
  if (tid == 0) s_item = atomicAdd(A.wide_next, 1u);
  __syncthreads();
  uint32_t it = uni(s_item);
  while (it < n_items) {
    const uint32_t code = A.wide_code[it];
    uint32_t li;
    int j, d;
    decode(code, &li, &j, &d);
    const int l = A.plan.n_lists[j];
    if (tid < l) {
      const uint64_t wi = win_index(A, d, A.plan.list_pair[j][tid], li);
      s_lo[tid] = A.win_lo[wi];
      s_len[tid] = A.win_len[wi];
    }
    __syncthreads();
    uint32_t maxlen = 0;
    for (int r = 0; r < l; ++r) maxlen = s_len[r] > maxlen ? s_len[r] : maxlen;
    maxlen = uni(maxlen);
    U128 total{0, 0};
    bool sat = false;  // a level total reached 2^64
    if (maxlen <= (uint32_t)kWideCap) {
      // As in the one-wavefront pass: while T_r <= |L_r| T_{r-1} stays below
      // 2^64 the running carry is the exact level total (no 128-bit sums),
      // and below 2^32 the level's prefix sums are stored as 32-bit words.
      uint64_t t_prev = uni(s_len[0]);
      bool prev32 = false;
      for (int r = 1; r < l; ++r) {
        const uint32_t loA = uni(s_lo[r - 1]), nA = uni(s_len[r - 1]);
        const uint32_t loB = uni(s_lo[r]), nB = uni(s_len[r]);
        const uint64_t* Pprev = Pbuf[(r - 1) & 1];
        uint64_t* Pcur = Pbuf[r & 1];
        const uint32_t* Pprev32 = reinterpret_cast<const uint32_t*>(Pprev);
        uint32_t* Pcur32 = reinterpret_cast<uint32_t*>(Pcur);
        const bool keep = r + 1 < l;  // P_r is read by the next level
        uint64_t bound;
        const bool exact64 = !sat && !__builtin_mul_overflow((uint64_t)nB, t_prev, &bound);
        const bool cur32 = exact64 && bound < (1ull << 32);
        if (keep && tid == 0) {
          if (cur32)
            Pcur32[0] = 0u;
          else
            Pcur[0] = 0;
        }
        total = U128{0, 0};
        uint64_t carry = 0;
        uint32_t a0 = 0, b0 = 0;
        while (b0 < nB) {
          const uint32_t na = nA - a0 < (uint32_t)kWTile ? nA - a0 : (uint32_t)kWTile;
          const uint32_t nb = nB - b0 < (uint32_t)kWTile ? nB - b0 : (uint32_t)kWTile;
          for (uint32_t i = tid; i < na; i += kWBlock) sA[i] = A.pair_t[loA + a0 + i];
          for (uint32_t i = tid; i <= na; i += kWBlock)
            sP[i] = (r == 1) ? (uint64_t)(a0 + i)
                             : (prev32 ? (uint64_t)Pprev32[a0 + i] : Pprev[a0 + i]);
          int64_t key[kWPer];
#pragma unroll
          for (int e = 0; e < kWPer; ++e) {
            const uint32_t bi = (uint32_t)(tid * kWPer + e);
            key[e] = bi < nb ? A.pair_t[loB + b0 + bi] : INT64_MAX;
          }
          __syncthreads();
          const bool a_ends = a0 + na == nA;
          const int64_t a_last = na ? sA[na - 1] : INT64_MIN;
          uint64_t c[kWPer];
          uint32_t pl[kWPer];
          uint32_t nset = 0;
#pragma unroll
          for (int e = 0; e < kWPer; ++e) {
            const uint32_t bi = (uint32_t)(tid * kWPer + e);
            const bool set = bi < nb && (a_ends || key[e] <= a_last);
            pl[e] = set ? lower_bound<int64_t>(sA, 0u, na, key[e]) : 0u;
            c[e] = set ? sP[pl[e]] : 0ull;
            nset += set ? 1u : 0u;
          }
          // inclusive prefix of this thread's four counts, then across the block
          uint64_t run[kWPer];
#pragma unroll
          for (int e = 0; e < kWPer; ++e) run[e] = (e ? run[e - 1] : 0ull) + c[e];
          const uint64_t incl = scan_dpp(run[kWPer - 1]);
          if (!exact64) {
            U128 tsum{0, 0};
#pragma unroll
            for (int e = 0; e < kWPer; ++e) tsum = add128(tsum, U128{c[e], 0});
            // tsum.hi <= 3 (four values below 2^64 each)
            U128 wsum = wave_sum128_dpp(tsum.lo);
            wsum.hi += lane_u32(scan_dpp((uint32_t)tsum.hi), kWave - 1);
            if (lane == kWave - 1) {
              s_wlo[wave] = wsum.lo;
              s_whi[wave] = wsum.hi;
            }
          }
          const uint32_t wset = lane_u32(scan_dpp(nset), kWave - 1);
          if (lane == kWave - 1) {
            s_wsum[wave] = incl;
            s_wset[wave] = wset;
          }
          __syncthreads();
          uint64_t before = carry + incl - run[kWPer - 1];
          uint32_t nr = 0;
#pragma unroll
          for (int w = 0; w < kWWaves; ++w) {
            if (w < wave) before += s_wsum[w];
            nr += s_wset[w];
          }
          nr = uni(nr);
          if (keep) {
#pragma unroll
            for (int e = 0; e < kWPer; ++e) {
              const uint32_t bi = (uint32_t)(tid * kWPer + e);
              if (bi < nr) {
                if (cur32)
                  Pcur32[b0 + bi + 1] = (uint32_t)(before + run[e]);
                else
                  Pcur[b0 + bi + 1] = before + run[e];
              }
            }
          }
          if (!exact64) {
            U128 step{0, 0};
#pragma unroll
            for (int w = 0; w < kWWaves; ++w) step = add128(step, U128{s_wlo[w], s_whi[w]});
            total = add128(total, U128{uni64(step.lo), uni64(step.hi)});
          }
          uint64_t blk = 0;
#pragma unroll
          for (int w = 0; w < kWWaves; ++w) blk += s_wsum[w];
          carry += uni64(blk);
          // the next step's start in A
          if (nr == nb) {
#pragma unroll
            for (int e = 0; e < kWPer; ++e)
              if ((uint32_t)(tid * kWPer + e) == nb - 1) s_last_pos = pl[e];
          } else {
#pragma unroll
            for (int e = 0; e < kWPer; ++e)
              if ((uint32_t)(tid * kWPer + e) == nr) s_key0 = key[e];
          }
          __syncthreads();
          b0 += nr;
          if (nr == nb) {
            a0 += uni(s_last_pos);
          } else {
            a0 += na;
            const uint32_t rem = nA - a0;
            if (rem > (uint32_t)kWTile) {
              const int64_t key0 = uni64s(s_key0);
              const uint32_t stride = (rem + kWBlock - 1) / kWBlock;
              const uint64_t q = (uint64_t)a0 + (uint64_t)(tid + 1) * stride - 1;
              const bool below = q < nA && A.pair_t[loA + q] < key0;
              const uint32_t nb_below = (uint32_t)__syncthreads_count(below);
              a0 += uni(nb_below) * stride;
            }
          }
          __syncthreads();  // the tiles are rewritten by the next step
        }
        if (exact64) {
          t_prev = carry;
        } else {
          if (uni64(total.hi) != 0) sat = true;  // the 128-bit pass takes the item
          t_prev = total.hi ? ~0ull : total.lo;
        }
        prev32 = cur32;
        __threadfence_block();
        __syncthreads();  // P_r complete before the next level reads it
      }
      total = U128{t_prev, 0};
    }
    if (tid == 0) {
      if (maxlen > (uint32_t)kWideCap)
        A.big_code[atomicAdd(A.big_count, 1u)] = code;
      else if (sat)
        A.w128_code[atomicAdd(A.w128_count, 1u)] = code;
      else
        item_done(A, d, j, li, total.lo);
      s_item = atomicAdd(A.wide_next, 1u);
    }
    __syncthreads();
    it = uni(s_item);
  }
  __syncthreads();
  sums_flush<1>(A);
}

// One item's count X (128 bits) into a block slot.  The per-sample output X
// saturates at 2^64 - 1; cnt takes the exact value.  An importance-sampling
// term floor(X 2^64 / h) needs X < 2^64: beyond, the motif's overflow bit is
// set, as it is for a count of 2^128 or more (`ovf`).  Several threads may
// add to one slot (LDS atomics).
__device__ void item_done128(const SampleArgs& A, int d, int j, uint32_t li, U128 X, bool ovf,
                             BlockSums* slot) {
  const DeltaArgs& D = A.D[d];
  const uint64_t X64 = X.hi ? ~0ull : X.lo;  // saturated
  if (D.is && X.hi) ovf = true;
  if (ovf) flag_status(A, d, TC_F_OVERFLOW | TC_F_MOTIF(j));
  if (D.X) D.X[(uint64_t)j * A.k + A.c0 + li] = X64;
  const uint32_t hp = D.is ? A.samp_h[(uint64_t)d * A.chunk + li] : 1u;
  const U128 c = D.is ? contribution(X64, true, hp) : X;
  const bool nz = (X.lo | X.hi) != 0;
  atomicAdd((unsigned long long*)&slot->hits, nz ? 1ull : 0ull);
  if (nz) atomicMax((unsigned long long*)&slot->xmax, (unsigned long long)X64);
  if (D.m2 && nz) {
    const double v = __ddiv_rn(u128_to_double(X.lo, X.hi), (double)hp);
    atomicAdd(&slot->m2, __dmul_rn(v, v));
  }
  const uint64_t old = atomicAdd((unsigned long long*)&slot->lo, (unsigned long long)c.lo);
  const uint64_t add_hi = c.hi + ((old + c.lo < old) ? 1ull : 0ull);
  if (add_hi < c.hi) atomicOr(&slot->ovf, 1u);
  if (add_hi) {
    const uint64_t old_hi = atomicAdd((unsigned long long*)&slot->hi, (unsigned long long)add_hi);
    if (old_hi + add_hi < old_hi) atomicOr(&slot->ovf, 1u);
  }
}

// Items whose count reached 2^64 in a faster pass, lists up to kWideCap
// entries: the merge of k_listcount_wide in 128-bit arithmetic.  Each level
// merges L_{r-1} and L_r in tiles; P_{r-1} and P_r are 128-bit prefix sums
// (lo and hi words interleaved), and the block scan of the settled counts
// runs over 128-bit values with a carry across steps.  Any sum that passes
// 2^128 is reported as an overflow.  A block uses the prefix scratch of two
// merged-pass blocks, so the pass needs no workspace of its own.
__global__ __launch_bounds__(kWBlock) void k_listcount_w128(SampleArgs A, uint64_t* pscratch) {
  __shared__ int64_t sA[kWTile];
  __shared__ uint64_t sPlo[kWTile + 1], sPhi[kWTile + 1];
  __shared__ uint64_t s_wlo[kWWaves], s_whi[kWWaves];
  __shared__ uint32_t s_wset[kWWaves];
  __shared__ uint32_t s_lo[kMaxLists], s_len[kMaxLists];
  __shared__ uint32_t s_item, s_last_pos;
  __shared__ int64_t s_key0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t* Pbuf[2] = {pscratch + (uint64_t)blockIdx.x * 4 * (kWideCap + 1),
                       pscratch + ((uint64_t)blockIdx.x * 4 + 2) * (kWideCap + 1)};
  const uint32_t n_items = *A.w128_count;
  if (blockIdx.x >= n_items) return;  // uniform: the others claim every item
  sums_clear<1>(A);
  if (tid == 0) s_item = atomicAdd(A.w128_next, 1u);
  __syncthreads();
  uint32_t it = uni(s_item);
  while (it < n_items) {
    const uint32_t code = A.w128_code[it];
    uint32_t li;
    int j, d;
    decode(code, &li, &j, &d);
    const int l = A.plan.n_lists[j];
    if (tid < l) {
      const uint64_t wi = win_index(A, d, A.plan.list_pair[j][tid], li);
      s_lo[tid] = A.win_lo[wi];
      s_len[tid] = A.win_len[wi];
    }
    __syncthreads();
    uint32_t maxlen = 0;
    for (int r = 0; r < l; ++r) maxlen = s_len[r] > maxlen ? s_len[r] : maxlen;
    maxlen = uni(maxlen);
    bool ovf = false;
    U128 total{uni(s_len[0]), 0};
    if (maxlen <= (uint32_t)kWideCap) {
      for (int r = 1; r < l; ++r) {
        const uint32_t loA = uni(s_lo[r - 1]), nA = uni(s_len[r - 1]);
        const uint32_t loB = uni(s_lo[r]), nB = uni(s_len[r]);
        const uint64_t* Pprev = Pbuf[(r - 1) & 1];
        uint64_t* Pcur = Pbuf[r & 1];
        const bool keep = r + 1 < l;  // P_r is read by the next level
        if (keep && tid == 0) {
          Pcur[0] = 0;
          Pcur[1] = 0;
        }
        U128 carry{0, 0};
        uint32_t a0 = 0, b0 = 0;
        while (b0 < nB) {
          const uint32_t na = nA - a0 < (uint32_t)kWTile ? nA - a0 : (uint32_t)kWTile;
          const uint32_t nb = nB - b0 < (uint32_t)kWTile ? nB - b0 : (uint32_t)kWTile;
          for (uint32_t i = tid; i < na; i += kWBlock) sA[i] = A.pair_t[loA + a0 + i];
          for (uint32_t i = tid; i <= na; i += kWBlock) {
            if (r == 1) {
              sPlo[i] = (uint64_t)(a0 + i);
              sPhi[i] = 0;
            } else {
              sPlo[i] = Pprev[2 * (uint64_t)(a0 + i)];
              sPhi[i] = Pprev[2 * (uint64_t)(a0 + i) + 1];
            }
          }
          int64_t key[kWPer];
#pragma unroll
          for (int e = 0; e < kWPer; ++e) {
            const uint32_t bi = (uint32_t)(tid * kWPer + e);
            key[e] = bi < nb ? A.pair_t[loB + b0 + bi] : INT64_MAX;
          }
          __syncthreads();
          const bool a_ends = a0 + na == nA;
          const int64_t a_last = na ? sA[na - 1] : INT64_MIN;
          U128 c[kWPer];
          uint32_t pl[kWPer];
          uint32_t nset = 0;
#pragma unroll
          for (int e = 0; e < kWPer; ++e) {
            const uint32_t bi = (uint32_t)(tid * kWPer + e);
            const bool set = bi < nb && (a_ends || key[e] <= a_last);
            pl[e] = set ? lower_bound<int64_t>(sA, 0u, na, key[e]) : 0u;
            c[e] = set ? U128{sPlo[pl[e]], sPhi[pl[e]]} : U128{0, 0};
            nset += set ? 1u : 0u;
          }
          // inclusive prefix of this thread's counts, then across the wavefront
          U128 run[kWPer];
#pragma unroll
          for (int e = 0; e < kWPer; ++e) run[e] = e ? add128c(run[e - 1], c[e], &ovf) : c[0];
          const U128 mine = run[kWPer - 1];
          U128 inc = mine;
#pragma unroll
          for (int off = 1; off < kWave; off <<= 1) {
            const U128 o{__shfl_up(inc.lo, off, kWave), __shfl_up(inc.hi, off, kWave)};
            if (lane >= off) inc = add128c(inc, o, &ovf);
          }
          const uint32_t wset = lane_u32(scan_dpp(nset), kWave - 1);
          if (lane == kWave - 1) {
            s_wlo[wave] = inc.lo;
            s_whi[wave] = inc.hi;
            s_wset[wave] = wset;
          }
          __syncthreads();
          // this thread's exclusive prefix: the carry, the wavefronts before,
          // then the lanes before inside its wavefront
          U128 before = carry;
          uint32_t nr = 0;
          U128 blk{0, 0};
#pragma unroll
          for (int w = 0; w < kWWaves; ++w) {
            const U128 ws{s_wlo[w], s_whi[w]};
            if (w < wave) before = add128c(before, ws, &ovf);
            blk = add128c(blk, ws, &ovf);
            nr += s_wset[w];
          }
          nr = uni(nr);
          before = add128(before, U128{inc.lo - mine.lo,
                                       inc.hi - mine.hi - (inc.lo < mine.lo ? 1ull : 0ull)});
          if (keep) {
#pragma unroll
            for (int e = 0; e < kWPer; ++e) {
              const uint32_t bi = (uint32_t)(tid * kWPer + e);
              if (bi < nr) {
                const U128 v = add128(before, run[e]);
                Pcur[2 * (uint64_t)(b0 + bi + 1)] = v.lo;
                Pcur[2 * (uint64_t)(b0 + bi + 1) + 1] = v.hi;
              }
            }
          }
          carry = add128c(carry, U128{uni64(blk.lo), uni64(blk.hi)}, &ovf);
          // the next step's start in A (as in k_listcount_wide)
          if (nr == nb) {
#pragma unroll
            for (int e = 0; e < kWPer; ++e)
              if ((uint32_t)(tid * kWPer + e) == nb - 1) s_last_pos = pl[e];
          } else {
#pragma unroll
            for (int e = 0; e < kWPer; ++e)
              if ((uint32_t)(tid * kWPer + e) == nr) s_key0 = key[e];
          }
          __syncthreads();
          b0 += nr;
          if (nr == nb) {
            a0 += uni(s_last_pos);
          } else {
            a0 += na;
            const uint32_t rem = nA - a0;
            if (rem > (uint32_t)kWTile) {
              const int64_t key0 = uni64s(s_key0);
              const uint32_t stride = (rem + kWBlock - 1) / kWBlock;
              const uint64_t q = (uint64_t)a0 + (uint64_t)(tid + 1) * stride - 1;
              const bool below = q < nA && A.pair_t[loA + q] < key0;
              const uint32_t nb_below = (uint32_t)__syncthreads_count(below);
              a0 += uni(nb_below) * stride;
            }
          }
          __syncthreads();  // the tiles are rewritten by the next step
        }
        total = U128{uni64(carry.lo), uni64(carry.hi)};
        __threadfence_block();
        __syncthreads();  // P_r complete before the next level reads it
      }
    }
    const bool any_ovf = __syncthreads_or(ovf) != 0;
    if (tid == 0) {
      if (maxlen > (uint32_t)kWideCap)
        A.big_code[atomicAdd(A.big_count, 1u)] = code;
      else
        item_done128(A, d, j, li, total, any_ovf, sums_slot(A, 0, d, j));
      s_item = atomicAdd(A.w128_next, 1u);
    }
    __syncthreads();
    it = uni(s_item);
  }
  __syncthreads();
  sums_flush<1>(A);
}

// Items with a list longer than kWideCap: one thread per item, a merged time
// sweep in 128-bit counts.
__global__ __launch_bounds__(kSBlock) void k_listcount_big(SampleArgs A) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const uint32_t n_items = *A.big_count;
  if ((uint64_t)blockIdx.x * kSBlock >= n_items) return;  // uniform: no item for this block
  sums_clear<kSWaves>(A);
  __syncthreads();
  for (uint32_t it = blockIdx.x * kSBlock + tid; it < n_items; it += gridDim.x * kSBlock) {
    uint32_t li;
    int j, d;
    decode(A.big_code[it], &li, &j, &d);
    const int l = A.plan.n_lists[j];
    uint32_t ptr[kMaxLists], end[kMaxLists];
#pragma unroll
    for (int r = 0; r < kMaxLists; ++r) {
      ptr[r] = 0;
      end[r] = 0;
      if (r < l) {
        const uint64_t wi = win_index(A, d, A.plan.list_pair[j][r], li);
        ptr[r] = A.win_lo[wi];
        end[r] = ptr[r] + A.win_len[wi];
      }
    }
    bool ovf = false;
    const U128 X = sweep128<kMaxLists>(A.pair_t, ptr, end, l, &ovf);
    item_done128(A, d, j, li, X, ovf, sums_slot(A, wave, d, j));
  }
  __syncthreads();
  sums_flush<kSWaves>(A);
}

__global__ void k_zero_result(SampleArgs A) {
  const int nm = A.plan.n_motifs;
  for (int i = threadIdx.x; i < kSpread * A.nd * nm; i += blockDim.x)
    A.spread[i] = SpreadSums{0, 0, 0, 0, 0.0};
  for (int i = threadIdx.x; i < A.nd * nm; i += blockDim.x) {
    const int d = i / nm, j = i - d * nm;
    A.D[d].cnt[2 * j] = 0;
    A.D[d].cnt[2 * j + 1] = 0;
    A.D[d].hits[j] = 0;
    if (A.D[d].m2) A.D[d].m2[j] = 0.0;
    if (A.D[d].xmax) A.D[d].xmax[j] = 0;
  }
  if ((int)threadIdx.x < A.nd) *A.D[threadIdx.x].status = 0;
}

// estimate output pointers of the deltas, passed by value
struct EstPtrs {
  double* p[kMaxDeltas];
};

__global__ void k_store_ptrs(EstPtrs ep, double** dst) {
  if (threadIdx.x < kMaxDeltas) dst[threadIdx.x] = ep.p[threadIdx.x];
}

__global__ void k_zero_counters(uint32_t* p) {
  // item_count, (spare), wide_count, wide_next, big_count, mid_count,
  // w128_count, w128_next
  if (threadIdx.x < 8) p[threadIdx.x] = 0;
}

// C_hat = (cnt / k) * W, each integer rounded to nearest-even binary64; with
// a proposal, C_hat = ((cnt * 2^-64) / k) * Q
// One wavefront per (delta, motif): lane s holds copy s of the totals, and
// fixed-order wavefront sums give cnt (128-bit, with overflow), hits and m2.
__global__ __launch_bounds__(1024) void k_finalize(SampleArgs A, double* const* est) {
  const int nm = A.plan.n_motifs;
  const int lane = threadIdx.x & 63, wave = (int)uni(threadIdx.x >> 6);
  static_assert(kSpread == kWave, "one lane per copy of the totals");
  for (int i = wave; i < A.nd * nm; i += (int)(blockDim.x >> 6)) {  // uniform per wavefront
    const int d = i / nm, j = i - d * nm;
    const SpreadSums v = *spread_slot(A, lane, d, j);
    bool ovf = false;
    const U128 c128 = wave_sum128c(U128{v.lo, v.hi}, &ovf);
    ovf = __ballot(ovf) != 0;  // a carry seen on any lane's path
    uint64_t h = v.hits, xm = v.xmax;
    double sq = v.m2;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      h += __shfl_xor(h, off, kWave);
      sq += __shfl_xor(sq, off, kWave);
      const uint64_t o = __shfl_xor(xm, off, kWave);
      xm = o > xm ? o : xm;
    }
    if (lane == 0) {
      A.D[d].cnt[2 * j] = c128.lo;
      A.D[d].cnt[2 * j + 1] = c128.hi;
      A.D[d].hits[j] = h;
      if (A.D[d].m2) A.D[d].m2[j] = sq;
      if (A.D[d].xmax) A.D[d].xmax[j] = xm;
      if (ovf) atomicOr(A.D[d].status, TC_F_OVERFLOW | TC_F_MOTIF(j));
      const uint64_t W = A.D[d].S[A.m];
      double c = u128_to_double(c128.lo, c128.hi);
      if (A.D[d].is) c = ldexp(c, -64);
      // exhaustive mode: the count itself
      est[d][j] = A.exhaustive ? c
                               : ((W == 0) ? 0.0 : __dmul_rn(__ddiv_rn(c, (double)A.k), (double)W));
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < A.nd && *A.D[threadIdx.x].wstatus)
    atomicOr(A.D[threadIdx.x].status, *A.D[threadIdx.x].wstatus);
}

// ------------------------------------------------------------ workspace ----
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SampleTuning default_tuning() {
  SampleTuning t;
  t.chunk_log2 = kLiBits;
  t.path_blocks = 0;
  t.reg_waves = 40960;
  t.fast_waves = 8192;
  t.wide_blocks = kDefaultWideBlocks;
  t.reg_list_cap = 256;
  t.lds_list_cap = kKeyCap;
  return t;
}

static uint64_t chunk_for(uint64_t k, int nd, const SampleTuning& t) {
  const int lg = t.chunk_log2 < 10 ? 10 : (t.chunk_log2 > kLiBits ? kLiBits : t.chunk_log2);
  uint64_t c = (1ull << lg) / (uint64_t)nd;  // all deltas of a chunk within 2^kLiBits samples
  if (c > k) c = k;
  return c < 1 ? 1 : c;
}

static int fast_waves_for(const SampleTuning& t) {
  return t.fast_waves < 64 ? 64 : (t.fast_waves > kMaxFastWaves ? kMaxFastWaves : t.fast_waves);
}

static int wide_blocks_for(const SampleTuning& t) {
  return t.wide_blocks < 16 ? 16
                            : (t.wide_blocks > kMaxWideBlocks ? kMaxWideBlocks : t.wide_blocks);
}

struct SampleLayout {
  size_t win_lo, win_len, code, mid, wide, big, w128, counters, fast_p, wide_p, est_ptrs, samp_h,
      spread, total;
  uint64_t chunk, cap;
  int fast_waves, wide_blocks;
};

static SampleLayout sample_layout(uint64_t k, int nd, int32_t n_motifs, const SampleTuning& t) {
  SampleLayout L;
  L.chunk = chunk_for(k, nd, t);
  L.cap = L.chunk * (uint64_t)nd * (uint64_t)n_motifs;
  L.fast_waves = fast_waves_for(t);
  L.wide_blocks = wide_blocks_for(t);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  L.win_lo = take((size_t)nd * kMaxPairs * L.chunk * 4);
  L.win_len = take((size_t)nd * kMaxPairs * L.chunk * 4);
  L.code = take(L.cap * 4);
  L.mid = take(L.cap * 4);
  L.wide = take(L.cap * 4);
  L.big = take(L.cap * 4);
  L.w128 = take(L.cap * 4);
  L.counters = take(32);
  L.fast_p = take((size_t)L.fast_waves * 2 * (kKeyCap + 1) * 8);
  L.wide_p = take((size_t)L.wide_blocks * 2 * (kWideCap + 1) * 8);
  L.est_ptrs = take(kMaxDeltas * sizeof(double*));
  L.samp_h = take((size_t)nd * L.chunk * 4);
  L.spread = take((size_t)kSpread * nd * n_motifs * sizeof(SpreadSums));
  L.total = o;
  return L;
}

size_t sample_workspace_bytes(uint64_t k, int nd, int32_t n_motifs, const SampleTuning* t) {
  SampleTuning tt = t ? *t : default_tuning();
  if (!t) {  // room for any tuning
    tt.chunk_log2 = kLiBits;
    tt.fast_waves = kMaxFastWaves;
    tt.wide_blocks = kMaxWideBlocks;
  }
  return sample_layout(k, nd, n_motifs, tt).total;
}

tc_status sample_batch(const tc_graph* g, const tc_weights* const* w, int nd,
                       const MotifPlan& plan, uint64_t k, uint64_t seed, uint32_t stream_id,
                       uint64_t i0, tc_result* const* out, const SampleTuning& tune, void* ws,
                       size_t ws_bytes, hipStream_t st, bool exhaustive) {
  if (nd < 1 || nd > kMaxDeltas) return TC_E_ARG;
  const SampleLayout L = sample_layout(k, nd, plan.n_motifs, tune);
  if (!ws || ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  SampleArgs A;
  A.out_rec = (const uint4*)g->out_rec;
  A.in_rec = (const uint4*)g->in_rec;
  A.out_eid = g->out_eid;
  A.pair_t = g->pair_t;
  A.pair_hash = (const PairSlot*)g->pair_hash;
  A.pair_hash_log2 = g->pair_hash_log2;
  A.pair_skip = g->pair_skip;
  A.m = g->m;
  {
    const STree T = stree_layout(g->m);
    A.tree_levels = T.levels;
    for (int L2 = 0; L2 < kMaxTreeLevels; ++L2) A.tree_off[L2] = L2 <= T.levels ? T.offset[L2] : 0;
    // the lowest level whose tail of the tree still fits the LDS cache
    A.tree_cache_lo = T.levels + 1;  // none
    A.tree_cache_base = T.total_words;
    A.tree_cache_words = 0;
    for (int L2 = T.levels; L2 >= 1; --L2) {
      if (T.total_words - T.offset[L2] > (size_t)kTreeCache) break;
      A.tree_cache_lo = L2;
      A.tree_cache_base = T.offset[L2];
      A.tree_cache_words = (uint32_t)(T.total_words - T.offset[L2]);
    }
  }
  A.nd = nd;
  double* est_host[kMaxDeltas] = {};
  for (int d = 0; d < kMaxDeltas; ++d) {
    DeltaArgs& D = A.D[d];
    D = DeltaArgs{};
    if (d >= nd) continue;
    if (w[d]->m != g->m) return TC_E_ARG;
    D.prec = (const uint4*)w[d]->prec;
    D.S = w[d]->S;
    D.tree = (const uint64_t*)w[d]->scratch;
    D.wstatus = w[d]->status;
    D.delta = w[d]->delta;
    D.cnt = out[d]->cnt;
    D.hits = out[d]->hits;
    D.status = out[d]->status;
    D.e1 = out[d]->e1;
    D.e2 = out[d]->e2;
    D.e3 = out[d]->e3;
    D.X = out[d]->X;
    D.h = w[d]->h;
    // window factors only for a side that has an edge
    D.ps1 = w[d]->cls.mode1 != TC_SIDE_NONE ? w[d]->ps1 : nullptr;
    D.ps3 = w[d]->cls.mode3 != TC_SIDE_NONE ? w[d]->ps3 : nullptr;
    D.is = (D.h || D.ps1 || D.ps3) ? 1 : 0;
    D.P = out[d]->P;
    D.m2 = out[d]->m2;
    D.xmax = out[d]->xmax;
    est_host[d] = out[d]->estimate;
  }
  A.k = k;
  A.seed = seed;
  A.i0 = i0;
  A.stream_id = stream_id;
  A.exhaustive = exhaustive ? 1 : 0;
  A.chunk = (uint32_t)L.chunk;
  A.win_lo = (uint32_t*)(base + L.win_lo);
  A.win_len = (uint32_t*)(base + L.win_len);
  A.item_code = (uint32_t*)(base + L.code);
  A.mid_code = (uint32_t*)(base + L.mid);
  A.wide_code = (uint32_t*)(base + L.wide);
  A.big_code = (uint32_t*)(base + L.big);
  A.item_count = (uint32_t*)(base + L.counters);
  A.wide_count = A.item_count + 2;
  A.wide_next = A.item_count + 3;
  A.big_count = A.item_count + 4;
  A.mid_count = A.item_count + 5;
  A.w128_code = (uint32_t*)(base + L.w128);
  A.w128_count = A.item_count + 6;
  A.w128_next = A.item_count + 7;
  A.fast_p = (uint64_t*)(base + L.fast_p);
  A.samp_h = (uint32_t*)(base + L.samp_h);
  A.wide_p = (uint64_t*)(base + L.wide_p);
  A.spread = (SpreadSums*)(base + L.spread);
  A.plan = plan;
  A.lds_cap = (uint32_t)(tune.lds_list_cap < kWave ? kWave
                         : (tune.lds_list_cap > kKeyCap ? kKeyCap : tune.lds_list_cap));
  // the estimate pointers go to the device through a small kernel argument
  // copy, so the call stays capturable (no host-to-device memcpy)
  EstPtrs ep;
  for (int d = 0; d < kMaxDeltas; ++d) ep.p[d] = est_host[d];
  double** est_dev = (double**)(base + L.est_ptrs);
  hipLaunchKernelGGL(k_store_ptrs, dim3(1), dim3(kMaxDeltas), 0, st, ep, est_dev);
  hipLaunchKernelGGL(k_zero_result, dim3(1), dim3(1024), 0, st, A);
  const int nm = plan.n_motifs;
  const unsigned reg_waves = (unsigned)(tune.reg_waves < 64 ? 64 : tune.reg_waves);
  for (uint64_t c0 = 0; c0 < k; c0 += L.chunk) {
    A.c0 = c0;
    A.clen = (uint32_t)((k - c0) < L.chunk ? (k - c0) : L.chunk);
    A.tiles_per_delta = (A.clen + kSBlock - 1) / kSBlock;
    const uint32_t units = A.tiles_per_delta * (uint32_t)nd;
    const unsigned pblocks =
        (unsigned)((tune.path_blocks > 0 && (uint32_t)tune.path_blocks < units) ? tune.path_blocks
                                                                                : units);
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, A.item_count);
    {
      TimedLaunch tl("k_paths", st);
      // the compile-time form needs the class <-,+,<,>>, anchor edges in path
      // order and every list after the last anchor edge (anchor ranks 0, 1, 2)
      bool general = exhaustive || !same_class(plan.cls, kSpineClass) || plan.n_anchor != 3 ||
                     plan.order[0] != 0 || plan.order[1] != 1 || plan.order[2] != 2;
      for (int q = 0; q < plan.n_pairs; ++q) general = general || plan.pair_seg[q] != 2;
      hipLaunchKernelGGL(general ? k_paths<true> : k_paths<false>, dim3(pblocks), dim3(kSBlock),
                         sums_bytes(kSWaves, nd, nm) + tree_cache_at(plan.n_gates) +
                             (size_t)kTreeCache * 8,
                         st, A);
    }
    if (plan.max_lists >= 2) {
      {
        TimedLaunch tl("k_listcount_reg", st);
        // lists of up to 128 entries (two chunks per lane, fewer registers)
        // or up to 256 (four)
        if (tune.reg_list_cap <= 2 * kWave)
          hipLaunchKernelGGL(k_listcount_reg<2>, dim3(reg_waves), dim3(kWave),
                             sums_bytes(1, nd, nm), st, A);
        else
          hipLaunchKernelGGL(k_listcount_reg<4>, dim3(reg_waves), dim3(kWave),
                             sums_bytes(1, nd, nm), st, A);
      }
      {
        TimedLaunch tl("k_listcount_lds", st);
        if (A.lds_cap <= 512)
          hipLaunchKernelGGL(k_listcount_lds<512>, dim3((unsigned)L.fast_waves), dim3(kWave),
                             sums_bytes(1, nd, nm), st, A, A.fast_p);
        else
          hipLaunchKernelGGL(k_listcount_lds<kKeyCap>, dim3((unsigned)L.fast_waves), dim3(kWave),
                             sums_bytes(1, nd, nm), st, A, A.fast_p);
      }
      {
        TimedLaunch tl("k_listcount_wide", st);
        hipLaunchKernelGGL(k_listcount_wide, dim3((unsigned)L.wide_blocks), dim3(kWBlock),
                           sums_bytes(1, nd, nm), st, A, A.wide_p);
      }
      {
        // two merged-pass blocks' prefix scratch per block (wide_blocks is
        // at least 16)
        TimedLaunch tl("k_listcount_w128", st);
        hipLaunchKernelGGL(k_listcount_w128, dim3((unsigned)(L.wide_blocks / 2)), dim3(kWBlock),
                           sums_bytes(1, nd, nm), st, A, A.wide_p);
      }
      {
        TimedLaunch tl("k_listcount_big", st);
        // one thread per item: enough blocks for every CU (blocks with no
        // item leave at once)
        hipLaunchKernelGGL(k_listcount_big, dim3(1024), dim3(kSBlock), sums_bytes(kSWaves, nd, nm),
                           st, A);
      }
    }
  }
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, A, (double* const*)est_dev);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
