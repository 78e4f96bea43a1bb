// Preprocess(delta): per-edge window degrees and the exact integer CDF of the
// path weights (Algorithm Preprocess with Claim "count":
// w_e = d^-_u[t - delta, t] * d^+_v[t, t + delta], and for the other anchor
// classes d^{alpha_1}_u * d^{alpha_3}_v over the class's intervals, a side
// without an edge counting 1), for one or several deltas of one class.
//
// The window bounds are ranks of sorted query sequences in sorted adjacency
// arrays on the composite key (vertex, time).  For the class <-,+,<,>>: the
// out-CSR order p is sorted by (u, t), so lo_in[p] = #{in-CSR entries <
// (u, t - delta)} and lo_in[p] + a[p] = #{in-CSR entries <= (u, t)}; the
// in-CSR order q is sorted by (v, t), so v's out-window bounds are ranks of
// (v, t) and (v, t + delta) in the out-CSR.  One bound of each side is the
// rank of the centre time itself and does not depend on delta.  Each side
// is one merge-path pass over its queries and data:
//   k_mp_split    splits the merged sequence (queries + data) into tiles of
//                 kMPTile entries by a binary search on each tile diagonal
//                 (both sides in one launch),
//   k_mp_rank     stages the tile's data keys in LDS, ranks each of the
//                 tile's queries there (the delta-free bound), and gallops
//                 from that bound to every delta's bound,
// so every array is read once per call, coalesced.  Side 3 comes out in
// in-CSR order: its pass writes one record per edge id holding the
// delta-free bound and every delta's rank, so a single scatter and a single
// gather carry all deltas to out-CSR order.  Then:
//   k_combine     per p: each delta's side-3 window from the record, the
//                 path records and the 128-bit tile sums of a*b per 2048-edge
//                 tile, for every delta.
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
// The splits of both sides' passes in one launch: blockIdx.y picks the job.  Two launches: every
// kSplitStride-th diagonal (and the last) bisects the whole range; the
// others bisect only between the splits of their two coarse neighbours (the
// split grows with the diagonal), a window of at most kSplitStride tiles
// whose probes stay in L2, where a full bisection reads a fresh line per
// probe.
constexpr int kMaxJobs = 2;
constexpr int64_t kSplitStride = 32;
struct SplitJob {
  KeyCols Q, D;
  uint32_t* split;
  int32_t upper;
};
struct SplitJobs {
  SplitJob j[kMaxJobs];
};

__device__ __forceinline__ uint32_t split_search(const SplitJob& S, int64_t d, int64_t lo,
                                                 int64_t hi) {
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
  return (uint32_t)lo;
}

// coarse: thread c takes diagonal index c * kSplitStride (or the last one)
__global__ __launch_bounds__(256) void k_mp_split_coarse(SplitJobs J, int64_t nq, int64_t nd,
                                                         int64_t nsplit) {
  const SplitJob& S = J.j[blockIdx.y];
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ncoarse = (nsplit - 1 + kSplitStride - 1) / kSplitStride + 1;
  if (c >= ncoarse) return;
  const int64_t b = c * kSplitStride < nsplit - 1 ? c * kSplitStride : nsplit - 1;
  const int64_t d = b * kMPTile < nq + nd ? b * kMPTile : nq + nd;
  const int64_t lo = d - nd > 0 ? d - nd : 0;
  const int64_t hi = d < nq ? d : nq;
  S.split[b] = split_search(S, d, lo, hi);
}

// fine: every other diagonal, inside its coarse neighbours' splits
__global__ __launch_bounds__(256) void k_mp_split(SplitJobs J, int64_t nq, int64_t nd,
                                                  int64_t nsplit) {
  const SplitJob& S = J.j[blockIdx.y];
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nsplit - 1 || b % kSplitStride == 0) return;
  const int64_t d = b * kMPTile < nq + nd ? b * kMPTile : nq + nd;
  const int64_t bl = b - b % kSplitStride;
  const int64_t br = bl + kSplitStride < nsplit - 1 ? bl + kSplitStride : nsplit - 1;
  int64_t lo = d - nd > 0 ? d - nd : 0;
  int64_t hi = d < nq ? d : nq;
  const int64_t sl = S.split[bl], sr = S.split[br];
  lo = sl > lo ? sl : lo;
  hi = sr < hi ? sr : hi;
  S.split[b] = split_search(S, d, lo, hi);
}

// One rank pass per side.  Query i's rank in the data with the centre time
// itself is the delta-free bound F; each delta's bound R is found from F by
// galloping over the data (probe F -/+ 1, 2, 4, ... until the probe crosses
// the delta's key, then bisect the last gap), reading the tile's LDS copy
// where the probe lies inside the tile and the data columns elsewhere.  A
// window before the centre time (BEFORE) has R = #{data < (w, t - delta)} <=
// F; one after it has R = #{data <= (w, t + delta)} >= F.  F counts the
// entries up to the centre time: "<=" for a closed window before it, "<" for
// one after it, and the reverse for a window open at the centre time (FU:
// F counts "<=").  Either way every entry from F on is not before a
// backward delta key and every entry below F is before a forward one, which
// the gallops need.  The pass stores:
//   RO_SIDE1  side 1's windows, for every delta: lo = F, len = R - F after
//             the centre time, lo = R, len = F - R before it;
//   RO_REC    side 3's record of query i's edge, at rec[eid[i] * stride]:
//             F, then every delta's R in delta order, then zeros.
// The inputs of a thread's queries are loaded before any of its stores, so
// no load waits behind a store it might alias.
enum { RO_SIDE1 = 1, RO_REC = 2 };
constexpr int kMaxRecWords = 12;
constexpr int kRankPer = kMPTile / kMPBlock;  // queries per thread at most
struct RankMode {
  int nd, chain;            // chain: deltas ascending, each gallop starts at the last bound
  int64_t dmax;             // the largest delta
  int64_t dsh[kMaxDeltas];  // +delta (window after the centre time) or -delta
  uint32_t* lo[kMaxDeltas];
  uint32_t* len[kMaxDeltas];
};

// record words per edge: the delta-free bound and one rank per delta,
// rounded up to 8 or a multiple of 16 bytes
__host__ __device__ constexpr int rec_stride(int nd) {
  const int w = 1 + nd;
  return w <= 2 ? 2 : ((w + 3) / 4) * 4;
}

// Data entries [lo, hi) are in LDS, entry j at index j - base.
struct TileKeys {
  const int32_t* s_v;
  const int64_t* s_t;
  int64_t base, lo, hi;
  KeyCols D;
  __device__ __forceinline__ void get(int64_t j, int32_t* v, int64_t* t) const {
    if (j >= lo && j < hi) {
      *v = s_v[j - base];
      *t = s_t[j - base];
    } else {
      *v = D.v[j];
      *t = D.t[j] + D.shift;
    }
  }
};

// Gallop from a bound F to the rank of (qv, qt): backwards with "<" when
// UPPER (every entry from F on is not before the key: F is the delta-free
// bound or a smaller delta's rank), forwards with "<=" otherwise (every
// entry below F is before it).  At most 2 log2(nd) + 2 probes.
template <bool UPPER>
__device__ __forceinline__ int64_t gallop(const TileKeys& K, int64_t nd, int64_t F, int32_t qv,
                                          int64_t qt) {
  int64_t lo, hi;  // entries <= lo are before the key, entries >= hi are not
  int32_t v;
  int64_t t;
  if (UPPER) {
    hi = F;
    lo = -1;
    for (int64_t step = 1;; step <<= 1) {
      const int64_t j = hi - step;
      if (j < 0) break;
      K.get(j, &v, &t);
      if (before<false>(v, t, qv, qt)) {
        lo = j;
        break;
      }
      hi = j;
    }
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      K.get(mid, &v, &t);
      if (before<false>(v, t, qv, qt))
        lo = mid;
      else
        hi = mid;
    }
  } else {
    lo = F - 1;
    hi = nd;
    for (int64_t step = 1;; step <<= 1) {
      const int64_t j = lo + step;
      if (j >= nd) break;
      K.get(j, &v, &t);
      if (!before<true>(v, t, qv, qt)) {
        hi = j;
        break;
      }
      lo = j;
    }
    while (hi - lo > 1) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      K.get(mid, &v, &t);
      if (before<true>(v, t, qv, qt))
        lo = mid;
      else
        hi = mid;
    }
  }
  return hi;
}

// The rank pass of one side (a compile-time mode and, for the record, delta
// count: the record's unrolled state would otherwise cost the side-1 pass
// registers and resident blocks)
// The first entry in (lo, hi] that is not before (qv, qt) (counted with
// "<=" when UQ), given that entry lo is before it (or lo = -1) and entry hi
// is not (or hi = nd): galloping inwards from both ends, then bisecting, so
// the cost follows the distance of the answer from the nearer end.
template <bool UQ>
__device__ __forceinline__ int64_t bracket(const TileKeys& K, int64_t lo, int64_t hi, int32_t qv,
                                           int64_t qt) {
  int32_t v;
  int64_t t;
  for (int64_t s = 1; hi - lo > 2 * s; s <<= 1) {
    const int64_t a = lo + s, b = hi - s;
    K.get(a, &v, &t);
    const bool pa = before<UQ>(v, t, qv, qt);
    K.get(b, &v, &t);
    const bool pb = before<UQ>(v, t, qv, qt);
    if (!pa) {
      hi = a;
      break;
    }
    if (pb) {
      lo = b;
      break;
    }
    lo = a;
    hi = b;
  }
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    K.get(mid, &v, &t);
    if (before<UQ>(v, t, qv, qt))
      lo = mid;
    else
      hi = mid;
  }
  return hi;
}

// Entries staged beside the tile for the delta windows that leave it: on
// the side the windows extend to (before the tile for windows before the
// centre time, after it otherwise), up to kExt entries, when the widest
// window of the tile's first (or last) query reaches past the tile.
constexpr int kExt = 1024;

template <bool BEFORE, bool FU, int MODE, int ND = 0>
__global__ __launch_bounds__(kMPBlock) void k_mp_rank(KeyCols Q, int64_t nq, KeyCols D, int64_t nd,
                                                      const uint32_t* __restrict__ split,
                                                      RankMode M, uint32_t* __restrict__ rec,
                                                      const int32_t* __restrict__ eid,
                                                      const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;  // a rejected graph: its arrays are not sorted
  __shared__ int32_t s_v[kMPTile + kExt];
  __shared__ int64_t s_t[kMPTile + kExt];
  __shared__ int s_ext;
  const int64_t b = blockIdx.x;
  const int64_t d0 = b * kMPTile;
  const int64_t d1 = d0 + kMPTile < nq + nd ? d0 + kMPTile : nq + nd;
  const int64_t q0 = split[b], q1 = split[b + 1];
  const int64_t i0 = d0 - q0, i1 = d1 - q1;
  const int nd_t = (int)(i1 - i0);
  // LDS index k holds data entry base + k; the tile starts at toff
  const int toff = BEFORE ? kExt : 0;
  const int64_t base = i0 - toff;
  for (int k = threadIdx.x; k < nd_t; k += kMPBlock) {
    s_v[toff + k] = D.v[i0 + k];
    s_t[toff + k] = D.t[i0 + k] + D.shift;
  }
  if (threadIdx.x == 0) {
    // does the widest window of the outermost query leave the tile?
    bool need = false;
    if (q0 < q1) {
      const int64_t qi = BEFORE ? q0 : q1 - 1;
      const int32_t v = Q.v[qi];
      const int64_t t = Q.t[qi] + Q.shift + (BEFORE ? -M.dmax : M.dmax);
      if (BEFORE && i0 > 0)
        need = !before<false>(D.v[i0 - 1], D.t[i0 - 1] + D.shift, v, t);
      else if (!BEFORE && i1 < nd)
        need = before<true>(D.v[i1], D.t[i1] + D.shift, v, t);
    }
    const int64_t room = BEFORE ? i0 : nd - i1;
    s_ext = need ? (int)(room < kExt ? room : kExt) : 0;
  }
  // this thread's queries: `per` consecutive ones (at most kRankPer),
  // loaded before any store
  const int per = (int)((q1 - q0 + kMPBlock - 1) / kMPBlock);
  const int64_t qb = q0 + (int64_t)threadIdx.x * per;
  const int mine = (int)(q1 - qb < 0 ? 0 : (q1 - qb < per ? q1 - qb : per));
  int32_t qv[kRankPer];
  int64_t qt[kRankPer], e[kRankPer];
#pragma unroll
  for (int r = 0; r < kRankPer; ++r) {
    const bool ok = r < mine;
    qv[r] = ok ? Q.v[qb + r] : 0;
    qt[r] = ok ? Q.t[qb + r] + Q.shift : 0;
    e[r] = MODE == RO_REC && ok ? eid[qb + r] : 0;
  }
  __syncthreads();
  const int ext = s_ext;
  if (ext > 0) {
    const int64_t x0 = BEFORE ? i0 - ext : i1;
    const int k0 = (int)(x0 - base);
    for (int k = threadIdx.x; k < ext; k += kMPBlock) {
      s_v[k0 + k] = D.v[x0 + k];
      s_t[k0 + k] = D.t[x0 + k] + D.shift;
    }
    __syncthreads();
  }
  if (mine == 0) return;
  const TileKeys K{s_v, s_t, base, BEFORE ? i0 - ext : i0, BEFORE ? i1 : i1 + ext, D};
  const int32_t* tv = s_v + toff;
  const int64_t* tt = s_t + toff;
  // delta-free bounds: a bisection of the tile for the first query, then
  // galloping on from the previous query's bound (the queries are sorted)
  int64_t F[kRankPer];
#pragma unroll
  for (int r = 0; r < kRankPer; ++r) {
    if (r >= mine) break;
    int lo, hi;
    if (r == 0) {
      lo = -1;
      hi = nd_t;
    } else {
      lo = (int)(F[r - 1] - i0) - 1;
      hi = nd_t;
      for (int s = 1;; s <<= 1) {
        const int j = lo + s;
        if (j >= nd_t) break;
        if (!before<FU>(tv[j], tt[j], qv[r], qt[r])) {
          hi = j;
          break;
        }
        lo = j;
      }
    }
    while (hi - lo > 1) {
      const int mid = lo + ((hi - lo) >> 1);
      if (before<FU>(tv[mid], tt[mid], qv[r], qt[r]))
        lo = mid;
      else
        hi = mid;
    }
    F[r] = i0 + hi;
  }
  // Each delta's bound: the thread's first query gallops from its
  // delta-free bound (or from the previous delta's bound when the deltas
  // ascend); every later query is bracketed by the previous query's bound
  // for the same delta (its keys are not larger) and, before the centre
  // time, by its own delta-free bound.
  if (MODE == RO_SIDE1) {
    int64_t from0 = F[0];
    for (int k = 0; k < M.nd; ++k) {
      const int64_t dk = M.dsh[k];
      int64_t prev = 0;
#pragma unroll
      for (int r = 0; r < kRankPer; ++r) {
        if (r >= mine) break;
        int64_t R;
        if (r == 0) {
          R = gallop<BEFORE>(K, nd, M.chain ? from0 : F[0], qv[0], qt[0] + dk);
          from0 = R;
        } else if (BEFORE) {
          R = bracket<false>(K, prev - 1, F[r], qv[r], qt[r] + dk);
        } else {
          R = gallop<false>(K, nd, F[r] > prev ? F[r] : prev, qv[r], qt[r] + dk);
        }
        prev = R;
        M.lo[k][qb + r] = (uint32_t)(BEFORE ? R : F[r]);
        M.len[k][qb + r] = (uint32_t)(BEFORE ? F[r] - R : R - F[r]);
      }
    }
  } else {
    constexpr int kStride = rec_stride(ND);
    int64_t prevR[ND > 0 ? ND : 1];
#pragma unroll
    for (int r = 0; r < kRankPer; ++r) {
      if (r >= mine) break;
      uint32_t w[kMaxRecWords];
#pragma unroll
      for (int j = 0; j < kMaxRecWords; ++j) w[j] = 0;
      w[0] = (uint32_t)F[r];
#pragma unroll
      for (int k = 0; k < ND; ++k) {
        const int64_t key = qt[r] + M.dsh[k];
        int64_t R;
        if (r == 0)
          R = gallop<BEFORE>(K, nd, M.chain && k > 0 ? prevR[k > 0 ? k - 1 : 0] : F[0], qv[0],
                            key);
        else if (BEFORE)
          R = bracket<false>(K, prevR[k] - 1, F[r], qv[r], key);
        else
          R = gallop<false>(K, nd, F[r] > prevR[k] ? F[r] : prevR[k], qv[r], key);
        prevR[k] = R;
        w[1 + k] = (uint32_t)R;
      }
      if (kStride == 2) {
        reinterpret_cast<uint2*>(rec)[e[r]] = make_uint2(w[0], w[1]);
      } else {
        uint4* r4 = reinterpret_cast<uint4*>(rec) + e[r] * (kStride / 4);
#pragma unroll
        for (int q = 0; q < kStride / 4; ++q)
          r4[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
      }
    }
  }
}

// the record pass for nd deltas (1..8)
template <bool BEFORE, bool FU>
static decltype(&k_mp_rank<BEFORE, FU, RO_REC, 1>) rec_kernel(int nd) {
  switch (nd) {
    case 1: return k_mp_rank<BEFORE, FU, RO_REC, 1>;
    case 2: return k_mp_rank<BEFORE, FU, RO_REC, 2>;
    case 3: return k_mp_rank<BEFORE, FU, RO_REC, 3>;
    case 4: return k_mp_rank<BEFORE, FU, RO_REC, 4>;
    case 5: return k_mp_rank<BEFORE, FU, RO_REC, 5>;
    case 6: return k_mp_rank<BEFORE, FU, RO_REC, 6>;
    case 7: return k_mp_rank<BEFORE, FU, RO_REC, 7>;
    default: return k_mp_rank<BEFORE, FU, RO_REC, 8>;
  }
}

// Per p, for every delta of the call: side 3's window from the record of
// p's edge, the path record, and the tile sums of a * b.  An absent side has
// the window {0, 1} (one position, no edge); side 1's is then written here.
struct CombineOut {
  int nd, side1, side3, after3, stride;
  uint32_t* lo_in[kMaxDeltas];
  uint32_t* a[kMaxDeltas];
  uint32_t* lo_out[kMaxDeltas];
  uint32_t* b[kMaxDeltas];
  uint4* prec[kMaxDeltas];
  uint64_t* tile_sums[kMaxDeltas];
};

__global__ __launch_bounds__(kWBlock) void k_combine(const int32_t* __restrict__ out_eid,
                                                     const uint32_t* __restrict__ rec,
                                                     const int32_t* __restrict__ out_src,
                                                     const int32_t* __restrict__ out_dst,
                                                     const int64_t* __restrict__ out_t, int64_t m,
                                                     CombineOut C,
                                                     const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;  // a rejected graph: its edge ids are not a permutation
  __shared__ U128 s_w[kMaxDeltas][kWBlock / kWave];
  const int64_t start = (int64_t)blockIdx.x * kWTile;
  U128 acc[kMaxDeltas];
#pragma unroll
  for (int i = 0; i < kMaxDeltas; ++i) acc[i] = U128{0, 0};
  for (int r = 0; r < kWItems; ++r) {
    const int64_t p = start + (int64_t)r * kWBlock + threadIdx.x;
    if (p < m) {
      uint32_t w[kMaxRecWords];
#pragma unroll
      for (int j = 0; j < kMaxRecWords; ++j) w[j] = 0;
      if (C.side3) {
        const int64_t e = out_eid[p];
        if (C.stride == 2) {
          const uint2 v = reinterpret_cast<const uint2*>(rec)[e];
          w[0] = v.x;
          w[1] = v.y;
        } else {
          const uint4* r4 = reinterpret_cast<const uint4*>(rec) + e * (C.stride / 4);
#pragma unroll
          for (int q = 0; q < kMaxRecWords / 4; ++q)
            if (q < C.stride / 4) {
              const uint4 v = r4[q];
              w[4 * q] = v.x, w[4 * q + 1] = v.y, w[4 * q + 2] = v.z, w[4 * q + 3] = v.w;
            }
        }
      }
      const int64_t t = out_t[p];
      const uint4 edge =
          make_uint4((uint32_t)out_src[p], (uint32_t)out_dst[p], (uint32_t)t, (uint32_t)(t >> 32));
#pragma unroll
      for (int i = 0; i < kMaxDeltas; ++i) {
        if (i < C.nd) {
          uint32_t l3 = 0, b3 = 1;
          if (C.side3) {
            const uint32_t f = w[0], rk = w[1 + i];
            l3 = C.after3 ? f : rk;
            b3 = C.after3 ? rk - f : f - rk;
          }
          uint32_t l1 = 0, a1 = 1;
          if (C.side1) {
            l1 = C.lo_in[i][p];
            a1 = C.a[i][p];
          } else {
            C.lo_in[i][p] = 0;
            C.a[i][p] = 1;
          }
          C.lo_out[i][p] = l3;
          C.b[i][p] = b3;
          C.prec[i][2 * p] = make_uint4(l1, a1, l3, b3);
          C.prec[i][2 * p + 1] = edge;
          acc[i] = add128(acc[i], U128{(uint64_t)a1 * (uint64_t)b3, 0});
        }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kMaxDeltas; ++i) {
    if (i < C.nd) {
      const U128 s = wave_sum128(acc[i]);
      if (lane == 0) s_w[i][wave] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < C.nd) {
    const int i = threadIdx.x;
    U128 t{0, 0};
    for (int q = 0; q < kWBlock / kWave; ++q) t = add128(t, s_w[i][q]);
    uint64_t* ts = nullptr;
#pragma unroll
    for (int j = 0; j < kMaxDeltas; ++j)
      if (j == i) ts = C.tile_sums[j];
    ts[2 * blockIdx.x] = t.lo;
    ts[2 * blockIdx.x + 1] = t.hi;
  }
}

// The 16-ary search tree over S (level L holds S[16^L i], ~0 past m; S
// itself padded with ~0 to a multiple of 16 words) is written by the scan
// kernels as S is formed: the apply pass stores S[p] into every level whose
// stride divides p < m, and the tile scan, which forms S[m], stores the
// entries at and past m and the padding.  Reading every 16th word of S back
// would fetch all of its lines.
struct TreeOut {
  uint64_t* tree;  // null: no tree
  int32_t levels;
  int64_t count0;                       // S padded to this many words
  uint64_t offset[kMaxTreeLevels + 1];  // word offset of level L (1-based), then the total
};

__device__ __forceinline__ void tree_put(const TreeOut& T, int64_t p, uint64_t s) {
  for (int L = 1; L <= T.levels; ++L) {
    if (p & (((int64_t)1 << (4 * L)) - 1)) break;
    T.tree[T.offset[L] + (uint64_t)(p >> (4 * L))] = s;
  }
}

// one thread: the padding of S and every level's entries at and past m
__device__ void tree_tail(const TreeOut& T, uint64_t* S, int64_t m, uint64_t W) {
  for (int64_t e = m + 1; e < T.count0; ++e) S[e] = ~0ull;
  for (int L = 1; L <= T.levels; ++L) {
    const int sh = 4 * L;
    const int64_t first = (m + ((int64_t)1 << sh) - 1) >> sh;  // first i with 16^L i >= m
    const int64_t cnt = (int64_t)(T.offset[L + 1] - T.offset[L]);
    for (int64_t i = first; i < cnt; ++i)
      T.tree[T.offset[L] + (uint64_t)i] = ((i << sh) == m) ? W : ~0ull;
  }
}

// One block of 1024 threads: exclusive scan of the 128-bit tile sums; the
// offsets are stored modulo 2^64 (only meaningful when W < 2^64).
// A non-zero `upstream` word (the graph's build status, or the status of the
// weights a proposal is built on) makes the total 0 and is passed on.
__device__ __forceinline__ void scan_tiles(const uint64_t* __restrict__ tile_sums,
                                           int64_t ntiles, uint64_t* __restrict__ tile_off,
                                           uint64_t* __restrict__ S, int64_t m,
                                           uint32_t* __restrict__ status,
                                           const uint32_t* __restrict__ upstream,
                                           const TreeOut& T) {
  if (*upstream) {
    for (int64_t i = threadIdx.x; i < ntiles; i += 1024) tile_off[i] = 0;
    if (threadIdx.x == 0) {
      S[m] = 0;
      *status = *upstream & (TC_F_RANGE | TC_F_OVERFLOW);
      if (T.tree) tree_tail(T, S, m, 0);
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
    if (T.tree) tree_tail(T, S, m, W.lo);
  }
}

__global__ __launch_bounds__(1024) void k_scan_tiles(const uint64_t* __restrict__ tile_sums,
                                                     int64_t ntiles, uint64_t* __restrict__ tile_off,
                                                     uint64_t* __restrict__ S, int64_t m,
                                                     uint32_t* __restrict__ status,
                                                     const uint32_t* __restrict__ upstream,
                                                     TreeOut T) {
  scan_tiles(tile_sums, ntiles, tile_off, S, m, status, upstream, T);
}

// the tile scans of every weights set of a call, one block each
struct ScanSets {
  const uint64_t* tile_sums[kMaxDeltas];
  uint64_t* tile_off[kMaxDeltas];
  uint64_t* S[kMaxDeltas];
  uint32_t* status[kMaxDeltas];
  TreeOut T[kMaxDeltas];
};
__global__ __launch_bounds__(1024) void k_scan_tiles_sets(ScanSets J, int64_t ntiles, int64_t m,
                                                          const uint32_t* __restrict__ upstream) {
  const int i = blockIdx.x;
  scan_tiles(J.tile_sums[i], ntiles, J.tile_off[i], J.S[i], m, J.status[i], upstream, J.T[i]);
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
                                                      uint64_t* __restrict__ S, TreeOut T) {
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
    // p0 is a multiple of kWItems: only it can be a multiple of 16
    if (T.tree && (p0 & 15) == 0) tree_put(T, p0, out[0]);
  } else {
    if (T.tree && p0 < m && (p0 & 15) == 0) tree_put(T, p0, run);
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

// where the scan kernels write the search tree over w->S
static TreeOut tree_out(const tc_weights* w) {
  const STree T = stree_layout(w->m);
  TreeOut o{};
  o.tree = (uint64_t*)w->scratch;
  o.levels = T.levels;
  o.count0 = T.count[0];
  for (int L = 1; L <= T.levels; ++L) o.offset[L] = T.offset[L];
  o.offset[T.levels + 1] = T.total_words;
  return o;
}

// The arrays one weights set owns (they stay valid as long as the workspace).
struct WeightsLayout {
  size_t lo_in, a, lo_out, b, S, tree, status, tile_sums, tile_off, prec, total;
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
  L.prec = take(M * 32);
  L.total = o;
  return L;
}

// A call over nd deltas: nd weights sets, then the scratch of the call (the
// side-3 records by edge id and the merge splits of both sides).
struct BatchLayout {
  size_t own, rec, split, total;
  int64_t nsplit;
};

static BatchLayout batch_layout(int64_t m, int nd) {
  BatchLayout L;
  L.own = weights_layout(m).total;
  L.nsplit = (2 * m + kMPTile - 1) / kMPTile + 1;
  L.rec = L.own * (size_t)nd;
  const size_t rec_bytes = align256((size_t)m * (size_t)rec_stride(nd) * 4 + 1);
  L.split = L.rec + rec_bytes;
  L.total = L.split + align256((size_t)kMaxJobs * (size_t)(L.nsplit + 1) * 4);
  return L;
}

size_t weights_workspace_bytes(int64_t m) { return batch_layout(m, 1).total; }
size_t weights_batch_workspace_bytes(int64_t m, int nd) { return batch_layout(m, nd).total; }

tc_status path_weights_batch(const tc_graph* g, const int64_t* deltas, int nd,
                             const tc_class& cls, void* ws, size_t ws_bytes, hipStream_t st,
                             tc_weights* w) {
  const int64_t m = g->m;
  if (nd < 1 || nd > kMaxDeltas) return TC_E_ARG;
  const BatchLayout B = batch_layout(m, nd);
  if (ws_bytes < B.total) return TC_E_WORKSPACE;
  const WeightsLayout L = weights_layout(m);
  const int64_t ntiles = (m + kWTile - 1) / kWTile;
  uint64_t* tile_sums[kMaxDeltas];
  uint64_t* tile_off[kMaxDeltas];
  for (int i = 0; i < nd; ++i) {
    char* base = (char*)ws + (size_t)i * B.own;
    tc_weights* W = &w[i];
    W->delta = deltas[i];
    W->m = m;
    W->cls = cls;
    W->lo_in = (uint32_t*)(base + L.lo_in);
    W->a = (uint32_t*)(base + L.a);
    W->lo_out = (uint32_t*)(base + L.lo_out);
    W->b = (uint32_t*)(base + L.b);
    W->S = (uint64_t*)(base + L.S);
    W->status = (uint32_t*)(base + L.status);
    W->scratch = base + L.tree;  // search tree over S
    W->h = nullptr;
    W->ps1 = W->ps3 = nullptr;
    W->prec = base + L.prec;
    tile_sums[i] = (uint64_t*)(base + L.tile_sums);
    tile_off[i] = (uint64_t*)(base + L.tile_off);
  }
  uint32_t* rec = (uint32_t*)((char*)ws + B.rec);
  uint32_t* split = (uint32_t*)((char*)ws + B.split);
  const uint32_t* gst = (const uint32_t*)g->status;
  if (m > 0) {
    TimedLaunch tl("k_windows", st);
    const int64_t nsplit = B.nsplit;
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
    // counted with "<" and of (w, to) counted with "<=".  The bound at the
    // centre time is delta-free: "<=" for a window before t, "<" for one
    // after it; each delta's bound is (w, t - delta) with "<" or
    // (w, t + delta) with "<=".
    const KeyCols d1 = cls.mode1 == TC_SIDE_IN ? ink : outk;
    const KeyCols d3 = cls.mode3 == TC_SIDE_IN ? ink : outk;
    SplitJobs J{};
    int nj = 0;
    auto job = [&](const KeyCols& q, const KeyCols& d, bool upper) {
      J.j[nj] = SplitJob{q, d, split + (size_t)nj * (size_t)(nsplit + 1), upper ? 1 : 0};
      return nj++;
    };
    int j1f = -1, j3f = -1;
    auto dshift = [&](int after, int64_t d) { return after ? d : -d; };
    // per side: the window's direction (bit 0 of `after`) and whether it is
    // open at the centre time (bit 1), which decide how F counts ties
    const bool before1 = (cls.after1 & 1) == 0, before3 = (cls.after3 & 1) == 0;
    const bool fu1 = before1 != ((cls.after1 & 2) != 0);
    const bool fu3 = before3 != ((cls.after3 & 2) != 0);
    if (s1) j1f = job(outk, d1, fu1);
    if (s3) j3f = job(ink, d3, fu3);
    if (nj > 0) {
      const int64_t ncoarse = (nsplit - 1 + kSplitStride - 1) / kSplitStride + 1;
      hipLaunchKernelGGL(k_mp_split_coarse, dim3((unsigned)((ncoarse + 255) / 256), nj), dim3(256),
                         0, st, J, m, m, nsplit);
      hipLaunchKernelGGL(k_mp_split, dim3(sb, nj), dim3(256), 0, st, J, m, m, nsplit);
    }
    auto rank_mode = [&]() {
      RankMode M{};
      M.nd = nd;
      M.chain = 1;
      M.dmax = deltas[0];
      for (int i = 1; i < nd; ++i) {
        if (deltas[i] < deltas[i - 1]) M.chain = 0;
        M.dmax = deltas[i] > M.dmax ? deltas[i] : M.dmax;
      }
      return M;
    };
    if (s1) {
      // side 1 in scan order: every delta's window straight into its set
      const SplitJob& S = J.j[j1f];
      RankMode M = rank_mode();
      for (int i = 0; i < nd; ++i) {
        M.dsh[i] = dshift(!before1, deltas[i]);
        M.lo[i] = w[i].lo_in;
        M.len[i] = w[i].a;
      }
      const auto kern = before1 ? (fu1 ? k_mp_rank<true, true, RO_SIDE1>
                                       : k_mp_rank<true, false, RO_SIDE1>)
                                : (fu1 ? k_mp_rank<false, true, RO_SIDE1>
                                       : k_mp_rank<false, false, RO_SIDE1>);
      hipLaunchKernelGGL(kern, dim3(rb), dim3(kMPBlock), 0, st, S.Q, m, S.D, m,
                         (const uint32_t*)S.split, M, (uint32_t*)nullptr, (const int32_t*)nullptr,
                         gst);
    }
    if (s3) {
      // side 3 in in-CSR order: one record per edge id
      const SplitJob& S = J.j[j3f];
      RankMode M = rank_mode();
      for (int i = 0; i < nd; ++i) M.dsh[i] = dshift(!before3, deltas[i]);
      const auto kern = before3 ? (fu3 ? rec_kernel<true, true>(nd) : rec_kernel<true, false>(nd))
                                : (fu3 ? rec_kernel<false, true>(nd)
                                       : rec_kernel<false, false>(nd));
      hipLaunchKernelGGL(kern, dim3(rb), dim3(kMPBlock), 0, st, S.Q, m, S.D, m,
                         (const uint32_t*)S.split, M, rec, (const int32_t*)g->in_eid, gst);
    }
    CombineOut C{};
    C.nd = nd;
    C.side1 = s1 ? 1 : 0;
    C.side3 = s3 ? 1 : 0;
    C.after3 = before3 ? 0 : 1;
    C.stride = rec_stride(nd);
    for (int i = 0; i < nd; ++i) {
      C.lo_in[i] = w[i].lo_in;
      C.a[i] = w[i].a;
      C.lo_out[i] = w[i].lo_out;
      C.b[i] = w[i].b;
      C.prec[i] = (uint4*)w[i].prec;
      C.tile_sums[i] = tile_sums[i];
    }
    hipLaunchKernelGGL(k_combine, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const int32_t*)g->out_eid, (const uint32_t*)rec,
                       (const int32_t*)g->out_src, (const int32_t*)g->out_dst,
                       (const int64_t*)g->out_t, m, C, gst);
  }
  ScanSets J{};
  for (int i = 0; i < nd; ++i) {
    J.tile_sums[i] = tile_sums[i];
    J.tile_off[i] = tile_off[i];
    J.S[i] = w[i].S;
    J.status[i] = w[i].status;
    J.T[i] = tree_out(&w[i]);
  }
  hipLaunchKernelGGL(k_scan_tiles_sets, dim3((unsigned)nd), dim3(1024), 0, st, J, ntiles, m, gst);
  for (int i = 0; i < nd; ++i) {
    const TreeOut& T = J.T[i];
    if (ntiles > 0) {
      TimedLaunch tl("k_scan_apply", st);
      hipLaunchKernelGGL(k_scan_apply<false>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                         (const uint32_t*)w[i].a, (const uint32_t*)w[i].b,
                         (const uint32_t*)nullptr, m, (const uint64_t*)tile_off[i], w[i].S, T);
    }
  }
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

tc_status path_weights(const tc_graph* g, int64_t delta, const tc_class& cls, void* ws,
                       size_t ws_bytes, hipStream_t st, tc_weights* w) {
  return path_weights_batch(g, &delta, 1, cls, ws, ws_bytes, st, w);
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
  const TreeOut T = tree_out(wq);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, (const uint64_t*)tile_sums, ntiles,
                     tile_off, wq->S, m, wq->status, (const uint32_t*)w->status, T);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_scan_apply<true>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint32_t*)w->a, (const uint32_t*)w->b, h, m,
                       (const uint64_t*)tile_off, wq->S, T);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}


// ---- window proposal (not part of the paper) ---------------------------------
// Per-entry factors g(deg) of the far endpoint of every in-CSR entry (an
// edge x -> u: x) and out-CSR entry (v -> y: y), deg the total degree:
// g(d) = min(cap, F_q(1 + d)) with F_0 = 1, F_1 = r4, F_2 = r2, F_3 = r2 r4,
// F_4 = r2^2, r2 = floor(sqrt(1 + d)), r4 = floor(sqrt(r2)) -- integer
// square roots, so the factors are exact and reproducible.
__device__ __forceinline__ uint64_t isqrt_u64(uint64_t v) {
  uint64_t r = (uint64_t)sqrt((double)v);
  while (r > 0 && r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

__device__ __forceinline__ uint32_t degree_factor(uint64_t d, int quarter, uint32_t cap) {
  const uint64_t r2 = isqrt_u64(1 + d), r4 = isqrt_u64(r2);
  const uint64_t f = quarter == 0 ? 1 : quarter == 1 ? r4 : quarter == 2 ? r2
                   : quarter == 3 ? r2 * r4 : r2 * r2;
  return (uint32_t)(f < cap ? f : cap);
}

__global__ __launch_bounds__(256) void k_window_factors(const int32_t* __restrict__ in_src,
                                                        const int32_t* __restrict__ out_dst,
                                                        const uint32_t* __restrict__ in_off,
                                                        const uint32_t* __restrict__ out_off,
                                                        int64_t m, int quarter, uint32_t cap,
                                                        uint32_t* __restrict__ f_in,
                                                        uint32_t* __restrict__ f_out,
                                                        const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;  // a rejected graph: its ids are not valid
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  auto deg = [&](int32_t v) -> uint64_t {
    return (uint64_t)(out_off[v + 1] - out_off[v]) + (uint64_t)(in_off[v + 1] - in_off[v]);
  };
  f_in[i] = degree_factor(deg(in_src[i]), quarter, cap);
  f_out[i] = degree_factor(deg(out_dst[i]), quarter, cap);
}

// 128-bit tile sums of a u32 array (tiles of kWTile entries)
__global__ __launch_bounds__(kWBlock) void k_u32_tile_sums(const uint32_t* __restrict__ v,
                                                         int64_t m,
                                                         uint64_t* __restrict__ tile_sums) {
  __shared__ uint64_t s_w[kWBlock / kWave];
  const int64_t start = (int64_t)blockIdx.x * kWTile;
  uint64_t acc = 0;
#pragma unroll
  for (int r = 0; r < kWItems; ++r) {
    const int64_t p = start + (int64_t)r * kWBlock + threadIdx.x;
    if (p < m) acc += v[p];
  }
  acc = wave_inclusive_scan(acc);
  if ((threadIdx.x & 63) == 63) s_w[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kWBlock / kWave; ++w) t += s_w[w];
    tile_sums[2 * blockIdx.x] = t;
    tile_sums[2 * blockIdx.x + 1] = 0;
  }
}

// exclusive prefix sums of u64 (or u32 widened) values per tile plus the
// tile offset; `out` has m + 1 words (the last is written by k_scan_tiles)
template <typename T>
__global__ __launch_bounds__(kWBlock) void k_prefix_apply(const T* __restrict__ v, int64_t m,
                                                        const uint64_t* __restrict__ tile_off,
                                                        uint64_t* __restrict__ out, TreeOut tr) {
  __shared__ uint64_t s_w[kWBlock / kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * kWTile + (int64_t)threadIdx.x * kWItems;
  uint64_t x[kWItems];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kWItems; ++j) {
    x[j] = p0 + j < m ? (uint64_t)v[p0 + j] : 0ull;
    s += x[j];
  }
  const uint64_t inc = wave_inclusive_scan(s);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t run = tile_off[blockIdx.x] + inc - s;
  for (int q = 0; q < wave; ++q) run += s_w[q];
  if (tr.tree && p0 < m && (p0 & 15) == 0) tree_put(tr, p0, run);
#pragma unroll
  for (int j = 0; j < kWItems; ++j) {
    if (p0 + j < m) out[p0 + j] = run;
    run += x[j];
  }
}

// the flag word starts as the weights' status (a rejected graph or an
// overflowed weight set passes on)
__global__ void k_copy_word(const uint32_t* __restrict__ from, uint32_t* __restrict__ to) {
  if (threadIdx.x == 0) *to = *from;
}

// q_p = h_p * G1_p * G3_p per scan position (G a side's factor sum over its
// window, the window size without factors, 1 for an absent side), stored in
// q and summed per tile in 128 bits.  A window sum of 2^32 or more, or a
// q_p of 2^64 or more, sets TC_F_OVERFLOW in *flag.
__global__ __launch_bounds__(kWBlock) void k_qwin_tiles(
    const uint32_t* __restrict__ lo1, const uint32_t* __restrict__ a,
    const uint32_t* __restrict__ lo3, const uint32_t* __restrict__ b,
    const uint32_t* __restrict__ h, const uint64_t* __restrict__ ps1,
    const uint64_t* __restrict__ ps3, int mode1, int mode3, int64_t m,
    uint64_t* __restrict__ q, uint64_t* __restrict__ tile_sums, uint32_t* __restrict__ flag,
    const uint32_t* __restrict__ gstatus) {
  // a rejected graph: its windows are undefined (the flag, set from the
  // weights' status, already makes Q = 0)
  if (*gstatus) return;
  __shared__ U128 s_w[kWBlock / kWave];
  const int64_t start = (int64_t)blockIdx.x * kWTile;
  U128 acc{0, 0};
  bool bad = false;
#pragma unroll
  for (int r = 0; r < kWItems; ++r) {
    const int64_t p = start + (int64_t)r * kWBlock + threadIdx.x;
    if (p < m) {
      uint64_t G1 = 1, G3 = 1;
      if (mode1 != TC_SIDE_NONE) G1 = ps1 ? ps1[lo1[p] + a[p]] - ps1[lo1[p]] : a[p];
      if (mode3 != TC_SIDE_NONE) G3 = ps3 ? ps3[lo3[p] + b[p]] - ps3[lo3[p]] : b[p];
      if (G1 > 0xFFFFFFFFull || G3 > 0xFFFFFFFFull) {
        bad = true;
        G1 = G1 > 0xFFFFFFFFull ? 0xFFFFFFFFull : G1;
        G3 = G3 > 0xFFFFFFFFull ? 0xFFFFFFFFull : G3;
      }
      const uint64_t g13 = G1 * G3;  // below 2^64
      const uint64_t hp = h ? (uint64_t)h[p] : 1ull;
      const U128 qq{g13 * hp, __umul64hi(g13, hp)};
      if (qq.hi) bad = true;
      q[p] = qq.lo;
      acc = add128(acc, qq);
    }
  }
  if (bad) atomicOr(flag, TC_F_OVERFLOW);
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

struct WindowLayout {
  size_t S, tree, status, flag, fstatus, tile_sums, tile_off, q, ps_in, ps_out, total;
};

static WindowLayout window_layout(int64_t m) {
  WindowLayout L;
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
  L.flag = take(4);
  L.fstatus = take(4);
  L.tile_sums = take(ntiles * 16);
  L.tile_off = take(ntiles * 8);
  L.q = take((size_t)m * 8);
  L.ps_in = take(((size_t)m + 1) * 8);
  L.ps_out = take(((size_t)m + 1) * 8);
  L.total = o;
  return L;
}

size_t window_proposal_workspace_bytes(int64_t m) { return window_layout(m).total; }

tc_status window_factors(const tc_graph* g, int quarter, uint32_t cap, uint32_t* f_in,
                         uint32_t* f_out, hipStream_t st) {
  const int64_t m = g->m;
  if (m > 0)
    hipLaunchKernelGGL(k_window_factors, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       (const int32_t*)g->in_src, (const int32_t*)g->out_dst,
                       (const uint32_t*)g->in_off, (const uint32_t*)g->out_off, m, quarter, cap,
                       f_in, f_out, (const uint32_t*)g->status);
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

tc_status proposal_window(const tc_graph* g, const tc_weights* w, const uint32_t* h,
                          const uint32_t* f_in, const uint32_t* f_out, void* ws, size_t ws_bytes,
                          hipStream_t st, tc_weights* wq) {
  const int64_t m = w->m;
  const WindowLayout L = window_layout(m);
  if (ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  *wq = *w;
  wq->S = (uint64_t*)(base + L.S);
  wq->scratch = base + L.tree;
  wq->status = (uint32_t*)(base + L.status);
  wq->h = h;
  uint32_t* flag = (uint32_t*)(base + L.flag);
  uint32_t* fstatus = (uint32_t*)(base + L.fstatus);
  uint64_t* tile_sums = (uint64_t*)(base + L.tile_sums);
  uint64_t* tile_off = (uint64_t*)(base + L.tile_off);
  uint64_t* q = (uint64_t*)(base + L.q);
  uint64_t* ps_in = f_in ? (uint64_t*)(base + L.ps_in) : nullptr;
  uint64_t* ps_out = f_out ? (uint64_t*)(base + L.ps_out) : nullptr;
  const int64_t ntiles = (m + kWTile - 1) / kWTile;
  const uint32_t* gst = (const uint32_t*)g->status;
  // prefix sums of the factors (m + 1 words each; the total lands in [m])
  auto prefix = [&](const uint32_t* f, uint64_t* ps) {
    if (ntiles > 0)
      hipLaunchKernelGGL(k_u32_tile_sums, dim3((unsigned)ntiles), dim3(kWBlock), 0, st, f, m,
                         tile_sums);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, (const uint64_t*)tile_sums,
                       ntiles, tile_off, ps, m, fstatus, gst, TreeOut{});
    if (ntiles > 0)
      hipLaunchKernelGGL(k_prefix_apply<uint32_t>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                         f, m, (const uint64_t*)tile_off, ps, TreeOut{});
  };
  if (ps_in) prefix(f_in, ps_in);
  if (ps_out) prefix(f_out, ps_out);
  auto side_ps = [&](int mode) -> const uint64_t* {
    return mode == TC_SIDE_IN ? ps_in : (mode == TC_SIDE_OUT ? ps_out : nullptr);
  };
  wq->ps1 = side_ps(w->cls.mode1);
  wq->ps3 = side_ps(w->cls.mode3);
  hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(64), 0, st, (const uint32_t*)w->status, flag);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_qwin_tiles, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint32_t*)w->lo_in, (const uint32_t*)w->a,
                       (const uint32_t*)w->lo_out, (const uint32_t*)w->b, h, wq->ps1, wq->ps3,
                       (int)w->cls.mode1, (int)w->cls.mode3, m, q, tile_sums, flag, gst);
  // a set flag (window sums or q_p out of range, or the weights' own status)
  // makes Q = 0 and is reported in wq->status
  const TreeOut T = tree_out(wq);
  hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, (const uint64_t*)tile_sums, ntiles,
                     tile_off, wq->S, m, wq->status, (const uint32_t*)flag, T);
  if (ntiles > 0)
    hipLaunchKernelGGL(k_prefix_apply<uint64_t>, dim3((unsigned)ntiles), dim3(kWBlock), 0, st,
                       (const uint64_t*)q, m, (const uint64_t*)tile_off, wq->S, T);
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
