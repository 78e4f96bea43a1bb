// Preprocess(delta): per-edge window degrees and the exact integer CDF of the
// path weights (Algorithm Preprocess with Claim "count":
// w_e = d^-_u[t - delta, t] * d^+_v[t, t + delta], and for the other anchor
// classes d^{alpha_1}_u * d^{alpha_3}_v over the class's intervals, a side
// without an edge counting 1).  Described below for the class <-,+,<,>>.
//
// The window bounds are ranks of sorted query sequences in sorted adjacency
// arrays on the composite key (vertex, time): the out-CSR order p is sorted
// by (u, t), so lo_in[p] = #{in-CSR entries < (u, t - delta)} and
// lo_in[p] + a[p] = #{in-CSR entries <= (u, t)}; the in-CSR order q is sorted
// by (v, t), so v's out-window bounds are ranks of (v, t) and (v, t + delta)
// in the out-CSR.  Each rank sequence is one merge-path pass:
//   k_mp_split4   splits the merged sequence (queries + data) into tiles of
//                 kMPTile entries by a binary search on each tile diagonal,
//   k_mp_rank     stages the tile's data keys in LDS and ranks each of the
//                 tile's queries there,
// so every array is read once, coalesced.  Then:
//   k_combine     per p: v's window (the last rank pass stored it by edge id),
//                 writes lo_out, b and the 128-bit sum of a*b per 2048-edge
//                 tile.
//   k_scan_tiles  one block scans the tile sums in 128-bit arithmetic, so
//                 W >= 2^64 is detected exactly, and writes S[m] = W.
//   k_scan_apply  per tile: w = a*b, block-wide exclusive scan, plus the
//                 tile offset -> S[p].
#include <hip/hip_runtime.h>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kWBlock = 512;
constexpr int kWItems = 4;
constexpr int kWTile = kWBlock * kWItems;  // 2048 edges per tile

// ---- merge-path sorted search on (vertex, time) keys -------------------------
constexpr int kMPTile = 2048;   // merged entries (queries + data) per block
constexpr int kMPBlock = 512;

struct KeyCols {
  const int32_t* v;  // vertex column
  const int64_t* t;  // time column
  int64_t shift;     // added to every time of this side
};

// data entry (dv, dt) is ranked before query (qv, qt)
template <bool UPPER>
__device__ __forceinline__ bool before(int32_t dv, int64_t dt, int32_t qv, int64_t qt) {
  return dv < qv || (dv == qv && (UPPER ? dt <= qt : dt < qt));
}

// split[b] = number of queries among the first min(b * kMPTile, nq + nd)
// entries of the merge (a query is taken first unless a data entry is ranked
// before it), by a bisection on the diagonal.
// The four splits of the weights (two per window side) in one launch:
// blockIdx.y picks the job.  Each diagonal's search is a short serial chain,
// so one job alone leaves the GPU mostly idle.
struct SplitJob {
  KeyCols Q, D;
  uint32_t* split;
  int32_t upper;
};
struct SplitJobs {
  SplitJob j[4];
};

__global__ __launch_bounds__(256) void k_mp_split4(SplitJobs J, int64_t nq, int64_t nd,
                                                   int64_t nsplit) {
  const SplitJob& S = J.j[blockIdx.y];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nsplit) return;
  const int64_t d = b * kMPTile < nq + nd ? b * kMPTile : nq + nd;
  int64_t lo = d - nd > 0 ? d - nd : 0;
  int64_t hi = d < nq ? d : nq;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int64_t j = d - mid - 1;
    const bool bef = S.upper ? before<true>(S.D.v[j], S.D.t[j] + S.D.shift, S.Q.v[mid],
                                            S.Q.t[mid] + S.Q.shift)
                             : before<false>(S.D.v[j], S.D.t[j] + S.D.shift, S.Q.v[mid],
                                             S.Q.t[mid] + S.Q.shift);
    if (!bef)
      lo = mid + 1;
    else
      hi = mid;
  }
  S.split[b] = (uint32_t)lo;
}

// rank of every query of the tile: out[i] = rank, or with `sub`
// pair_out[i] = {sub[i], rank - sub[i]} (a window's start and length),
// stored at pair_out[eid[i]] when `eid` is given
template <bool UPPER>
__global__ __launch_bounds__(kMPBlock) void k_mp_rank(KeyCols Q, int64_t nq, KeyCols D, int64_t nd,
                                                      const uint32_t* __restrict__ split,
                                                      const uint32_t* __restrict__ sub,
                                                      uint32_t* __restrict__ out,
                                                      uint2* __restrict__ pair_out,
                                                      const int32_t* __restrict__ eid,
                                                      const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;  // a rejected graph: its arrays are not sorted
  __shared__ int32_t s_v[kMPTile];
  __shared__ int64_t s_t[kMPTile];
  const int64_t b = blockIdx.x;
  const int64_t d0 = b * kMPTile;
  const int64_t d1 = d0 + kMPTile < nq + nd ? d0 + kMPTile : nq + nd;
  const int64_t q0 = split[b], q1 = split[b + 1];
  const int64_t i0 = d0 - q0, i1 = d1 - q1;
  const int nd_t = (int)(i1 - i0);
  for (int k = threadIdx.x; k < nd_t; k += kMPBlock) {
    s_v[k] = D.v[i0 + k];
    s_t[k] = D.t[i0 + k] + D.shift;
  }
  __syncthreads();
  for (int64_t i = q0 + threadIdx.x; i < q1; i += kMPBlock) {
    const int32_t qv = Q.v[i];
    const int64_t qt = Q.t[i] + Q.shift;
    int lo = 0, n = nd_t;
    while (n > 0) {
      const int half = n >> 1;
      const int mid = lo + half;
      const bool go = before<UPPER>(s_v[mid], s_t[mid], qv, qt);
      lo = go ? mid + 1 : lo;
      n = go ? n - half - 1 : half;
    }
    const uint32_t rank = (uint32_t)(i0 + lo);
    if (pair_out) {
      const uint32_t s0 = sub[i];
      pair_out[eid ? eid[i] : i] = make_uint2(s0, rank - s0);
    } else {
      out[i] = sub ? rank - sub[i] : rank;
    }
  }
}

// per p: side 3's window (the last rank pass stored it by edge id), the path
// record, and the tile sums of a * b.  An absent side has the window {0, 1}
// (one position, no edge); side 1's is then written here too.
__global__ __launch_bounds__(kWBlock) void k_combine(const int32_t* __restrict__ out_eid,
                                                     const uint2* __restrict__ win_e,
                                                     uint32_t* __restrict__ lo_in,
                                                     uint32_t* __restrict__ a,
                                                     const int32_t* __restrict__ out_src,
                                                     const int32_t* __restrict__ out_dst,
                                                     const int64_t* __restrict__ out_t, int64_t m,
                                                     uint32_t* __restrict__ lo_out,
                                                     uint32_t* __restrict__ b_out,
                                                     uint4* __restrict__ prec,
                                                     uint64_t* __restrict__ tile_sums,
                                                     const uint32_t* __restrict__ gstatus,
                                                     int side1, int side3) {
  if (*gstatus) return;  // a rejected graph: its edge ids are not a permutation
  __shared__ U128 s_w[kWBlock / kWave];
  const int64_t start = (int64_t)blockIdx.x * kWTile;
  U128 acc{0, 0};
#pragma unroll 4
  for (int r = 0; r < kWItems; ++r) {
    const int64_t p = start + (int64_t)r * kWBlock + threadIdx.x;
    if (p < m) {
      const uint2 wq = side3 ? win_e[out_eid[p]] : make_uint2(0u, 1u);
      uint32_t l1 = 0, ap = 1;
      if (side1) {
        l1 = lo_in[p];
        ap = a[p];
      } else {
        lo_in[p] = 0;
        a[p] = 1;
      }
      const uint32_t bb = wq.y;
      lo_out[p] = wq.x;
      b_out[p] = bb;
      const int64_t t = out_t[p];
      prec[2 * p] = make_uint4(l1, ap, wq.x, bb);
      prec[2 * p + 1] =
          make_uint4((uint32_t)out_src[p], (uint32_t)out_dst[p], (uint32_t)t, (uint32_t)(t >> 32));
      acc = add128(acc, U128{(uint64_t)ap * (uint64_t)bb, 0});
    }
  }
  acc = wave_sum128(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    U128 t{0, 0};
    for (int w = 0; w < kWBlock / kWave; ++w) t = add128(t, s_w[w]);
    tile_sums[2 * blockIdx.x] = t.lo;
    tile_sums[2 * blockIdx.x + 1] = t.hi;
  }
}

// One block of 1024 threads: exclusive scan of the 128-bit tile sums; the
// offsets are stored modulo 2^64 (only meaningful when W < 2^64).
// A non-zero `upstream` word (the graph's build status, or the status of the
// weights a proposal is built on) makes the total 0 and is passed on.
__global__ __launch_bounds__(1024) void k_scan_tiles(const uint64_t* __restrict__ tile_sums,
                                                     int64_t ntiles, uint64_t* __restrict__ tile_off,
                                                     uint64_t* __restrict__ S, int64_t m,
                                                     uint32_t* __restrict__ status,
                                                     const uint32_t* __restrict__ upstream) {
  if (*upstream) {
    for (int64_t i = threadIdx.x; i < ntiles; i += 1024) tile_off[i] = 0;
    if (threadIdx.x == 0) {
      S[m] = 0;
      *status = *upstream & (TC_F_RANGE | TC_F_OVERFLOW);
    }
    return;
  }
  // Thread t owns the consecutive tiles [t c, (t + 1) c): it sums them with
  // independent loads, one block scan orders the thread sums, and it writes
  // its tiles' offsets from its exclusive prefix.
  __shared__ U128 s_w[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c = (ntiles + 1023) / 1024;
  const int64_t b0 = (int64_t)threadIdx.x * c;
  const int64_t b1 = b0 + c < ntiles ? b0 + c : ntiles;
  U128 v{0, 0};
#pragma unroll 8
  for (int64_t i = b0; i < b1; ++i) v = add128(v, U128{tile_sums[2 * i], tile_sums[2 * i + 1]});
  U128 inc = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    U128 o{__shfl_up(inc.lo, off, kWave), __shfl_up(inc.hi, off, kWave)};
    if (lane >= off) inc = add128(inc, o);
  }
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  U128 run{0, 0};
  for (int w = 0; w < wave; ++w) run = add128(run, s_w[w]);
  // exclusive prefix of this thread = waves before + inc - v
  run = add128(run, U128{inc.lo - v.lo, inc.hi - v.hi - (inc.lo < v.lo ? 1ull : 0ull)});
#pragma unroll 8
  for (int64_t i = b0; i < b1; ++i) {
    tile_off[i] = run.lo;  // modulo 2^64 (only used when W < 2^64)
    run = add128(run, U128{tile_sums[2 * i], tile_sums[2 * i + 1]});
  }
  if (threadIdx.x == 1023) {  // its run ends at the total
    U128 W{0, 0};
    for (int w = 0; w < 16; ++w) W = add128(W, s_w[w]);
    S[m] = W.lo;
    *status = (W.hi != 0) ? TC_F_OVERFLOW : 0u;
  }
}

// 128-bit tile sums of q = a * b * h (the proposal weights)
__global__ __launch_bounds__(kWBlock) void k_qtile_sums(const uint32_t* __restrict__ a,
                                                      const uint32_t* __restrict__ b,
                                                      const uint32_t* __restrict__ h, int64_t m,
                                                      uint64_t* __restrict__ tile_sums) {
  __shared__ U128 s_w[kWBlock / kWave];
  const int64_t start = (int64_t)blockIdx.x * kWTile;
  U128 acc{0, 0};
#pragma unroll 4
  for (int r = 0; r < kWItems; ++r) {
    const int64_t p = start + (int64_t)r * kWBlock + threadIdx.x;
    if (p < m) {
      const uint64_t w = (uint64_t)a[p] * (uint64_t)b[p];
      acc = add128(acc, U128{w * h[p], __umul64hi(w, (uint64_t)h[p])});
    }
  }
  acc = wave_sum128(acc);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    U128 t{0, 0};
    for (int w = 0; w < kWBlock / kWave; ++w) t = add128(t, s_w[w]);
    tile_sums[2 * blockIdx.x] = t.lo;
    tile_sums[2 * blockIdx.x + 1] = t.hi;
  }
}

// per tile: w = a * b (times h for the proposal), block-wide exclusive scan,
// plus the tile offset -> S[p]
template <bool H>
__global__ __launch_bounds__(kWBlock) void k_scan_apply(const uint32_t* __restrict__ a,
                                                      const uint32_t* __restrict__ b,
                                                      const uint32_t* __restrict__ h, int64_t m,
                                                      const uint64_t* __restrict__ tile_off,
                                                      uint64_t* __restrict__ S) {
  __shared__ uint64_t s_w[kWBlock / kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * kWTile + (int64_t)threadIdx.x * kWItems;
  uint64_t w[kWItems];
  uint64_t s = 0;
  if (p0 + kWItems <= m) {
    // kWItems consecutive words per array, as kWItems / 4 aligned 16-byte
    // loads (p0 is a multiple of kWItems): nothing past p0 + kWItems is read
    static_assert(kWItems % 4 == 0, "16-byte loads of whole items");
    uint32_t av[kWItems], bv[kWItems], hv[kWItems];
#pragma unroll
    for (int q = 0; q < kWItems / 4; ++q) {
      const uint4 aa = reinterpret_cast<const uint4*>(a + p0)[q];
      const uint4 bb = reinterpret_cast<const uint4*>(b + p0)[q];
      av[4 * q] = aa.x, av[4 * q + 1] = aa.y, av[4 * q + 2] = aa.z, av[4 * q + 3] = aa.w;
      bv[4 * q] = bb.x, bv[4 * q + 1] = bb.y, bv[4 * q + 2] = bb.z, bv[4 * q + 3] = bb.w;
      if (H) {
        const uint4 hh = reinterpret_cast<const uint4*>(h + p0)[q];
        hv[4 * q] = hh.x, hv[4 * q + 1] = hh.y, hv[4 * q + 2] = hh.z, hv[4 * q + 3] = hh.w;
      }
    }
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
      w[j] = (uint64_t)av[j] * (uint64_t)bv[j] * (H ? (uint64_t)hv[j] : 1ull);
      s += w[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
      const int64_t p = p0 + j;
      w[j] = (p < m) ? (uint64_t)a[p] * (uint64_t)b[p] * (H ? (uint64_t)h[p] : 1ull) : 0ull;
      s += w[j];
    }
  }
  const uint64_t inc = wave_inclusive_scan(s);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t run = tile_off[blockIdx.x] + inc - s;
  for (int q = 0; q < wave; ++q) run += s_w[q];
  if (p0 + kWItems <= m) {
    uint64_t out[kWItems];
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
      out[j] = run;
      run += w[j];
    }
    ulonglong2* S2 = reinterpret_cast<ulonglong2*>(S + p0);
#pragma unroll
    for (int j = 0; j < kWItems / 2; ++j) S2[j] = make_ulonglong2(out[2 * j], out[2 * j + 1]);
  } else {
#pragma unroll
    for (int j = 0; j < kWItems; ++j) {
      const int64_t p = p0 + j;
      if (p < m) S[p] = run;
      run += w[j];
    }
  }
}

// ---- 16-ary search tree over S ----------------------------------------------
// Level 0 is S itself, padded with all-ones words to a multiple of 16
// entries; level L holds S[16^L * i] (padded likewise) and the last level has
// at most 16 entries.  upper_bound(S, r) - 1 is then found by reading one
// 128-byte node per level: at each level the node is the last entry <= r of
// the level above, and counting its entries <= r gives the next index.
// All levels of the search tree over S in one launch (level L holds
// S[16^L i], or ~0 past m), plus S's padding to a multiple of 16: thread e
// below `words` writes tree word e, the next `pad` threads the padding.
struct TreeShape {
  int32_t levels;
  uint64_t offset[kMaxTreeLevels + 1];  // word offset of level L (1-based), then the total
};

__global__ __launch_bounds__(256) void k_tree(uint64_t* __restrict__ S, int64_t m,
                                              uint64_t* __restrict__ tree, TreeShape T,
                                              int64_t pad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t words = (int64_t)T.offset[T.levels + 1];
  if (e < words) {
    int L = 1;
    while (L < T.levels && (uint64_t)e >= T.offset[L + 1]) ++L;
    const uint64_t at = ((uint64_t)e - T.offset[L]) << (4 * L);
    tree[e] = (at <= (uint64_t)m) ? S[at] : ~0ull;
  } else if (e < words + pad) {
    S[m + 1 + (e - words)] = ~0ull;
  }
}

STree stree_layout(int64_t m) {
  STree T;
  T.levels = 0;
  int64_t n = m + 1;
  T.count[0] = ((n + 15) / 16) * 16;
  T.offset[0] = 0;  // level 0 lives in S
  size_t off = 0;
  while (n > 16) {
    n = (n + 15) / 16;
    ++T.levels;
    T.count[T.levels] = ((n + 15) / 16) * 16;
    T.offset[T.levels] = off;
    off += (size_t)T.count[T.levels];
  }
  T.total_words = off;
  return T;
}

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// search tree over w->S (padding first, then each level)
static void build_tree(tc_weights* w, hipStream_t st) {
  const int64_t m = w->m;
  const STree T = stree_layout(m);
  const int64_t pad = T.count[0] - (m + 1);
  TreeShape sh{};
  sh.levels = T.levels;
  for (int L = 1; L <= T.levels; ++L) sh.offset[L] = T.offset[L];
  sh.offset[T.levels + 1] = T.total_words;
  const int64_t n = (int64_t)T.total_words + pad;
  if (n > 0)
    hipLaunchKernelGGL(k_tree, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w->S, m,
                       (uint64_t*)w->scratch, sh, pad);
}

struct WeightsLayout {
  size_t lo_in, a, lo_out, b, S, status, tile_sums, tile_off, tree, lo_out_q, win_e, split, prec,
      total;
};

static WeightsLayout weights_layout(int64_t m) {
  WeightsLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  const size_t M = (size_t)m;
  const size_t ntiles = (size_t)((m + kWTile - 1) / kWTile);
  L.lo_in = take(M * 4);
  L.a = take(M * 4);
  L.lo_out = take(M * 4);
  L.b = take(M * 4);
  const STree T = stree_layout(m);
  L.S = take((size_t)T.count[0] * 8);
  L.tree = take(T.total_words * 8);
  L.status = take(4);
  L.tile_sums = take(ntiles * 16);
  L.tile_off = take(ntiles * 8);
  L.lo_out_q = take(M * 4);
  L.win_e = take(M * 8);
  L.split = take((size_t)4 * ((2 * M + kMPTile - 1) / kMPTile + 2) * 4);  // four jobs
  L.prec = take(M * 32);
  L.total = o;
  return L;
}

size_t weights_workspace_bytes(int64_t m) { return weights_layout(m).total; }

tc_status path_weights(const tc_graph* g, int64_t delta, const tc_class& cls, void* ws,
                       size_t ws_bytes, hipStream_t st, tc_weights* w) {
  const int64_t m = g->m;
  WeightsLayout L = weights_layout(m);
  if (ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  w->delta = delta;
  w->m = m;
  w->cls = cls;
  w->lo_in = (uint32_t*)(base + L.lo_in);
  w->a = (uint32_t*)(base + L.a);
  w->lo_out = (uint32_t*)(base + L.lo_out);
  w->b = (uint32_t*)(base + L.b);
  w->S = (uint64_t*)(base + L.S);
  w->status = (uint32_t*)(base + L.status);
  w->scratch = base + L.tree;  // search tree over S
  w->h = nullptr;
  w->prec = base + L.prec;
  uint64_t* tile_sums = (uint64_t*)(base + L.tile_sums);
  uint64_t* tile_off = (uint64_t*)(base + L.tile_off);
  const int64_t ntiles = (m + kWTile - 1) / kWTile;
  uint32_t* lo_out_q = (uint32_t*)(base + L.lo_out_q);
  uint2* win_e = (uint2*)(base + L.win_e);
  uint32_t* split = (uint32_t*)(base + L.split);
  const uint32_t* gst = (const uint32_t*)g->status;
  if (m > 0) {
    TimedLaunch tl("k_windows", st);
    const int64_t nsplit = (2 * m + kMPTile - 1) / kMPTile + 1;
    const unsigned sb = (unsigned)((nsplit + 255) / 256);
    const unsigned rb = (unsigned)(nsplit - 1);
    // (vertex, time) keys: the out-CSR sorted by (source, time), the in-CSR
    // by (destination, time)
    const KeyCols outk{g->out_src, g->out_t, 0};
    const KeyCols ink{g->in_dst, g->in_t, 0};
    const bool s1 = cls.mode1 != TC_SIDE_NONE, s3 = cls.mode3 != TC_SIDE_NONE;
    // Side 1: for every scan position p (out-CSR order, queries (u, t)) the
    // window of u's in- or out-edges; side 3: for every in-CSR position q
    // (queries (v, t): each edge seen from its destination) the window of
    // v's in- or out-edges.  A window [from, to] is the rank of (w, from)
    // counted with "<" and of (w, to) counted with "<=".
    auto shifted = [&](const KeyCols& q, int64_t sh) { return KeyCols{q.v, q.t, sh}; };
    const int64_t lo1 = cls.after1 ? 0 : -delta, hi1 = cls.after1 ? delta : 0;
    const int64_t lo3 = cls.after3 ? 0 : -delta, hi3 = cls.after3 ? delta : 0;
    const KeyCols d1 = cls.mode1 == TC_SIDE_IN ? ink : outk;
    const KeyCols d3 = cls.mode3 == TC_SIDE_IN ? ink : outk;
    uint32_t* sp[4];
    for (int c = 0; c < 4; ++c) sp[c] = split + (size_t)c * (size_t)(nsplit + 1);
    SplitJobs J{};
    int nj = 0;
    if (s1) {
      J.j[nj++] = SplitJob{shifted(outk, lo1), d1, sp[0], 0};
      J.j[nj++] = SplitJob{shifted(outk, hi1), d1, sp[1], 1};
    }
    if (s3) {
      J.j[nj++] = SplitJob{shifted(ink, lo3), d3, sp[2], 0};
      J.j[nj++] = SplitJob{shifted(ink, hi3), d3, sp[3], 1};
    }
    hipLaunchKernelGGL(k_mp_split4, dim3(sb, nj), dim3(256), 0, st, J, m, m, nsplit);
    if (s1) {
      hipLaunchKernelGGL(k_mp_rank<false>, dim3(rb), dim3(kMPBlock), 0, st, shifted(outk, lo1), m,
                         d1, m, (const uint32_t*)sp[0], (const uint32_t*)nullptr, w->lo_in,
                         (uint2*)nullptr, (const int32_t*)nullptr, gst);
      hipLaunchKernelGGL(k_mp_rank<true>, dim3(rb), dim3(kMPBlock), 0, st, shifted(outk, hi1), m,
                         d1, m, (const uint32_t*)sp[1], (const uint32_t*)w->lo_in, w->a,
                         (uint2*)nullptr, (const int32_t*)nullptr, gst);
    }
    if (s3) {
      hipLaunchKernelGGL(k_mp_rank<false>, dim3(rb), dim3(kMPBlock), 0, st, shifted(ink, lo3), m,
                         d3, m, (const uint32_t*)sp[2], (const uint32_t*)nullptr, lo_out_q,
                         (uint2*)nullptr, (const int32_t*)nullptr, gst);
      hipLaunchKernelGGL(k_mp_rank<true>, dim3(rb), dim3(kMPBlock), 0, st, shifted(ink, hi3), m,
                         d3, m, (const uint32_t*)sp[3], (const uint32_t*)lo_out_q,
                         (uint32_t*)nullptr, win_e, (const int32_t*)g->in_eid, gst);
    }
    hipLaunchKernelGGL(k_combine, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const int32_t*)g->out_eid, (const uint2*)win_e, w->lo_in, w->a,
                       (const int32_t*)g->out_src, (const int32_t*)g->out_dst,
                       (const int64_t*)g->out_t, m, w->lo_out, w->b, (uint4*)w->prec, tile_sums,
                       gst, s1 ? 1 : 0, s3 ? 1 : 0);
  }
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, (const uint64_t*)tile_sums, ntiles,
                     tile_off, w->S, m, w->status, gst);
  if (ntiles > 0) {
    TimedLaunch tl("k_scan_apply", st);
    hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint32_t*)w->a, (const uint32_t*)w->b, (const uint32_t*)nullptr, m,
                       (const uint64_t*)tile_off, w->S);
  }
  build_tree(w, st);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

// Proposal weights: windows borrowed from w, S = scan of a * b * h.
struct ProposalLayout {
  size_t S, tree, status, tile_sums, tile_off, total;
};

static ProposalLayout proposal_layout(int64_t m) {
  ProposalLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  const size_t ntiles = (size_t)((m + kWTile - 1) / kWTile);
  const STree T = stree_layout(m);
  L.S = take((size_t)T.count[0] * 8);
  L.tree = take(T.total_words * 8);
  L.status = take(4);
  L.tile_sums = take(ntiles * 16);
  L.tile_off = take(ntiles * 8);
  L.total = o;
  return L;
}

size_t proposal_workspace_bytes(int64_t m) { return proposal_layout(m).total; }

tc_status proposal_weights(const tc_weights* w, const uint32_t* h, void* ws, size_t ws_bytes,
                           hipStream_t st, tc_weights* wq) {
  const int64_t m = w->m;
  const ProposalLayout L = proposal_layout(m);
  if (ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  *wq = *w;
  wq->S = (uint64_t*)(base + L.S);
  wq->scratch = base + L.tree;
  wq->status = (uint32_t*)(base + L.status);
  wq->h = h;
  uint64_t* tile_sums = (uint64_t*)(base + L.tile_sums);
  uint64_t* tile_off = (uint64_t*)(base + L.tile_off);
  const int64_t ntiles = (m + kWTile - 1) / kWTile;
  if (ntiles > 0)
    hipLaunchKernelGGL(k_qtile_sums, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint32_t*)w->a, (const uint32_t*)w->b, h, m, tile_sums);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, (const uint64_t*)tile_sums, ntiles,
                     tile_off, wq->S, m, wq->status, (const uint32_t*)w->status);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint32_t*)w->a, (const uint32_t*)w->b, h, m,
                       (const uint64_t*)tile_off, wq->S);
  build_tree(wq, st);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
