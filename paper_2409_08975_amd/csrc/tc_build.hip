// Temporal adjacency build: validation, stable LSD radix sorts and CSR
// offsets.  The canonical orders are (t, eid) -> (src, t, eid) for the
// out-lists, (dst, t, eid) for the in-lists and (src, dst, t, eid) for the
// per-pair lists; each later sort is a stable sort of the previous order, so
// timestamp ties keep increasing edge id (section III-A assumes time-sorted
// per-vertex lists; the tie order is this library's convention).
//
// Radix sort design (gfx950, wave64): 8-bit digits, tiles of 4096 keys per
// 256-thread block.  A pass is (1) per-tile digit histograms written
// tile-major (each tile's 256 counts are one contiguous kilobyte), (2) a
// column scan of that [tiles][256] matrix that turns every count into the
// tile's global offset for its digit, (3) a
// scatter that ranks keys stably inside the tile with wavefront ballots
// (8 ballots give the lanes sharing a digit), stages the tile in LDS in
// digit order and writes each digit run to its global slot with coalesced
// stores.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kSortBlock = 256;
constexpr uint32_t kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2
constexpr int kSortItems = 16;
constexpr int kRecItems = 6;  // record-carrying sorts: 1536-entry tiles (LDS holds 16 B/entry)
constexpr int kRecTile = kSortBlock * kRecItems;
constexpr int kColChunk = 32;  // tiles per chunk of the histogram column scan

static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------ validation ---
__global__ void k_init_build(uint32_t* status, uint64_t* tminmax) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *status = 0;
    tminmax[0] = ~0ull;  // min of order-preserving keys
    tminmax[1] = 0ull;   // max
  }
}

// t is mapped to an order-preserving unsigned key (flip the sign bit)
__global__ __launch_bounds__(256) void k_validate(const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst,
                                                  const int64_t* __restrict__ t, int64_t m,
                                                  int32_t n, uint32_t* status, uint64_t* tminmax) {
  const int64_t lim = (int64_t)1 << 62;
  uint64_t mn = ~0ull, mx = 0;
  uint32_t bad = 0;
  auto check = [&](int32_t s, int32_t d, int64_t tt) {
    if (s < 0 || s >= n || d < 0 || d >= n || tt >= lim || tt <= -lim) bad = 1;
    const uint64_t key = (uint64_t)tt ^ (1ull << 63);
    mn = key < mn ? key : mn;
    mx = key > mx ? key : mx;
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // four edges per step, their loads issued together (all in bounds)
  for (; i + 3 * stride < m; i += 4 * stride) {
    int32_t sv[4], dv[4];
    int64_t tv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sv[u] = src[i + u * stride];
      dv[u] = dst[i + u * stride];
      tv[u] = t[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) check(sv[u], dv[u], tv[u]);
  }
  for (; i < m; i += stride) check(src[i], dst[i], t[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint64_t a = __shfl_xor(mn, off, kWave);
    uint64_t b = __shfl_xor(mx, off, kWave);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
    bad |= __shfl_xor(bad, off, kWave);
  }
  // one pair of atomics per block (not per wavefront): they all hit two words
  __shared__ uint64_t s_mn[4], s_mx[4];
  __shared__ uint32_t s_bad[4];
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_mn[wave] = mn;
    s_mx[wave] = mx;
    s_bad[wave] = bad;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      mn = s_mn[w] < mn ? s_mn[w] : mn;
      mx = s_mx[w] > mx ? s_mx[w] : mx;
      bad |= s_bad[w];
    }
    atomicMin((unsigned long long*)&tminmax[0], (unsigned long long)mn);
    atomicMax((unsigned long long*)&tminmax[1], (unsigned long long)mx);
    if (bad) atomicOr(status, TC_F_RANGE);
  }
}

// ----------------------------------------------------------- key making ----
template <typename K>
__global__ __launch_bounds__(256) void k_time_keys(const int64_t* __restrict__ t, int64_t m,
                                                   int64_t tmin, K* __restrict__ keys,
                                                   int32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    keys[i] = (K)(uint64_t)(t[i] - tmin);
    vals[i] = (int32_t)i;
  }
}

// keys[i] = vert[order[i]], vals[i] = order[i]
__global__ __launch_bounds__(256) void k_vertex_keys(const int32_t* __restrict__ vert,
                                                     const int32_t* __restrict__ order, int64_t m,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    int32_t e = order[i];
    keys[i] = (uint32_t)vert[e];
    vals[i] = e;
  }
}

// ----------------------------------------------------------- radix pass ----
// `dev_m` (optional) holds the element count on the device; m is then the
// capacity the grid was sized for.  A sort moves either (key, value) pairs
// from two arrays, or (V = NoVal) whole 16-byte records whose first word is
// the key.
struct NoVal {};
__device__ __forceinline__ uint32_t sort_key(uint32_t k) { return k; }
__device__ __forceinline__ uint64_t sort_key(uint64_t k) { return k; }
__device__ __forceinline__ uint32_t sort_key(const uint4& r) { return r.x; }

// Re-keying of a 16-byte edge record between the sorts of the build:
//   RX_NONE  identity
//   RX_OUT   (t, eid, src, dst) -> (src, eid, dst, t)   out-CSR input
//   RX_IN    (t, eid, src, dst) -> (dst, eid, src, t)   in-CSR input
//   RX_PAIR  (dst, eid, src, t) -> (src, eid, dst, t)   pair-index input
enum { RX_NONE = 0, RX_OUT = 1, RX_IN = 2, RX_PAIR = 3 };
__device__ __forceinline__ uint4 rec_xform(const uint4& r, int xf) {
  if (xf == RX_OUT) return make_uint4(r.z, r.y, r.w, r.x);
  if (xf == RX_IN) return make_uint4(r.w, r.y, r.z, r.x);
  if (xf == RX_PAIR) return make_uint4(r.z, r.y, r.x, r.w);
  return r;
}

// The input edge columns, read directly by the first pass of the time sort
// (which builds each record (t - t_min, eid, src, dst) as it loads it);
// t == nullptr for every other pass.
struct EdgeCols {
  const int32_t* src;
  const int32_t* dst;
  const int64_t* t;
  int64_t tmin;
};

// the re-keying of a sort with no pass (a key of zero bits), in place:
// every element is read and written by the same thread
__global__ __launch_bounds__(256) void k_rec_xform(uint4* __restrict__ a, int64_t m,
                                                   int xf1, uint4* __restrict__ out2, int xf2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const uint4 r = a[i];
    a[i] = rec_xform(r, xf1);
    if (out2) out2[i] = rec_xform(r, xf2);
  }
}


template <typename K, int ITEMS>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const K* __restrict__ keys, int64_t m,
                                                           int shift, uint32_t mask,
                                                           uint32_t* __restrict__ hist,
                                                           const uint32_t* __restrict__ dev_m,
                                                           EdgeCols ec) {
  __shared__ uint32_t s_h[256];
  if (dev_m) m = (int64_t)*dev_m < m ? (int64_t)*dev_m : m;
  s_h[threadIdx.x] = 0;
  __syncthreads();
  int64_t start = (int64_t)blockIdx.x * (kSortBlock * ITEMS);
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    int64_t i = start + (int64_t)r * kSortBlock + threadIdx.x;
    if (i < m) {
      const uint64_t key = ec.t ? (uint64_t)(ec.t[i] - ec.tmin) : (uint64_t)sort_key(keys[i]);
      atomicAdd(&s_h[(uint32_t)(key >> shift) & mask], 1u);
    }
  }
  __syncthreads();
  hist[(int64_t)blockIdx.x * 256 + threadIdx.x] = s_h[threadIdx.x];
}

// Column scan of the tile-major histogram: hist[t][d] becomes the position
// of tile t's first key of digit d in the pass output, i.e. the keys of all
// smaller digits plus the keys of digit d in tiles before t.  Three kernels:
// per-chunk column sums, an exclusive scan of each digit's chunk sums (which
// also leaves the digit totals in row `nchunks`), and an in-place walk of
// every chunk that adds the digit base.  Every access reads or writes whole
// 1 KB rows except the per-digit chunk scan, which touches nchunks*256 words.
__global__ __launch_bounds__(256) void k_col_sum(const uint32_t* __restrict__ hist,
                                                 int64_t ntiles, uint32_t* __restrict__ csum) {
  const int64_t t0 = (int64_t)blockIdx.x * kColChunk;
  const int d = threadIdx.x;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kColChunk; ++j) {
    // clamped index: every load is issued unconditionally
    const int64_t t = t0 + j < ntiles ? t0 + j : ntiles - 1;
    const uint32_t v = hist[t * 256 + d];
    s += (t0 + j < ntiles) ? v : 0u;
  }
  csum[(int64_t)blockIdx.x * 256 + d] = s;
}

// one block per digit (blockIdx.x), chunks spread over the block's threads
__global__ __launch_bounds__(256) void k_col_scan(uint32_t* __restrict__ csum, int64_t nchunks) {
  __shared__ uint32_t s_w[256 / kWave];
  const int d = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nchunks; base += 256) {
    const int64_t c = base + threadIdx.x;
    const uint32_t v = c < nchunks ? csum[c * 256 + d] : 0u;
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
      off += w < wave ? s_w[w] : 0u;
      tot += s_w[w];
    }
    if (c < nchunks) csum[c * 256 + d] = carry + off + inc - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) csum[nchunks * 256 + d] = carry;
}

// one block per chunk; thread d walks the chunk's tiles for digit d
__global__ __launch_bounds__(256) void k_col_apply(uint32_t* __restrict__ hist, int64_t ntiles,
                                                   const uint32_t* __restrict__ csum,
                                                   int64_t nchunks) {
  __shared__ uint32_t s_w[256 / kWave];
  const int d = threadIdx.x, lane = d & 63, wave = d >> 6;
  // digit base: exclusive scan of the digit totals over d
  const uint32_t tot = csum[nchunks * 256 + d];
  const uint32_t inc = wave_inclusive_scan(tot);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint32_t run = inc - tot;
  for (int w = 0; w < wave; ++w) run += s_w[w];
  run += csum[(int64_t)blockIdx.x * 256 + d];
  const int64_t t0 = (int64_t)blockIdx.x * kColChunk;
  uint32_t v[kColChunk];
#pragma unroll
  for (int j = 0; j < kColChunk; ++j) {
    const int64_t t = t0 + j < ntiles ? t0 + j : ntiles - 1;
    v[j] = hist[t * 256 + d];
  }
#pragma unroll
  for (int j = 0; j < kColChunk; ++j) {
    if (t0 + j < ntiles) hist[(t0 + j) * 256 + d] = run;
    run += v[j];
  }
}

size_t col_scan_scratch_elems(int64_t ntiles) {
  return (size_t)256 * ((ntiles + kColChunk - 1) / kColChunk + 1);
}

void col_scan(uint32_t* hist, int64_t ntiles, uint32_t* csum, hipStream_t st) {
  const int64_t nchunks = (ntiles + kColChunk - 1) / kColChunk;
  hipLaunchKernelGGL(k_col_sum, dim3((unsigned)nchunks), dim3(256), 0, st,
                     (const uint32_t*)hist, ntiles, csum);
  hipLaunchKernelGGL(k_col_scan, dim3(256), dim3(256), 0, st, csum, nchunks);
  hipLaunchKernelGGL(k_col_apply, dim3((unsigned)nchunks), dim3(256), 0, st, hist, ntiles,
                     (const uint32_t*)csum, nchunks);
}

template <typename K, typename V, int ITEMS>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const K* __restrict__ kin,
                                                              const V* __restrict__ vin,
                                                              K* __restrict__ kout,
                                                              V* __restrict__ vout, int64_t m,
                                                              int shift, int dbits,
                                                              const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ dev_m,
                                                              int xf1, K* __restrict__ kout2,
                                                              int xf2, EdgeCols ec) {
  // Each wavefront owns a contiguous quarter of the tile and ranks its keys
  // in order with ballots (no block barrier inside); one block-wide pass then
  // offsets every wavefront's digit counts by those of the wavefronts before
  // it, which keeps the pass stable.
  constexpr int kTile = kSortBlock * ITEMS;
  constexpr int kWaves = kSortBlock / kWave;
  constexpr int kSub = kWave * ITEMS;  // entries per wavefront
  constexpr bool kHasVal = !std::is_same<V, NoVal>::value;
  const uint32_t mask = (1u << dbits) - 1u;
  // XCD-aware tile order.  Workgroups are dealt to the XCDs round robin
  // (block b to XCD b mod 8), and each XCD has its own L2.  Neighbouring
  // tiles write neighbouring pieces of every digit run, so each XCD takes a
  // contiguous range of tiles: partial cache lines then meet in one L2
  // instead of being written back piecewise from several.
  const uint32_t nb = gridDim.x, xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds;
  const uint32_t q = nb / kXcds, rem = nb % kXcds;
  const uint32_t tile = xcd * q + (xcd < rem ? xcd : rem) + slot;
  if (dev_m) m = (int64_t)*dev_m < m ? (int64_t)*dev_m : m;
  if ((int64_t)tile * kTile >= m) return;
  __shared__ uint32_t s_base[256];
  __shared__ uint32_t s_excl[256];
  __shared__ uint32_t s_wcnt[kWaves][256];  // per-wavefront running digit counts
  __shared__ uint32_t s_wsum[kWaves];
  __shared__ K s_key[kTile];
  __shared__ V s_val[kHasVal ? kTile : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t start = (int64_t)tile * kTile;
  const int len = (int)((m - start) < kTile ? (m - start) : kTile);
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  s_base[tid] = hist[(int64_t)tile * 256 + tid];
#pragma unroll
  for (int w = 0; w < kWaves; ++w) s_wcnt[w][tid] = 0;
  __syncthreads();

  K key[ITEMS];
  V val[ITEMS];
  uint32_t rank[ITEMS];  // rank among the wavefront's keys of the same digit
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int idx = wave * kSub + r * kWave + lane;
    const bool valid = idx < len;
    if constexpr (std::is_same<K, uint4>::value) {
      if (ec.t) {  // uniform: the first pass of the time sort builds the records
        const int64_t g = start + idx;
        key[r] = valid ? make_uint4((uint32_t)(ec.t[g] - ec.tmin), (uint32_t)g,
                                    (uint32_t)ec.src[g], (uint32_t)ec.dst[g])
                       : K{};
      } else {
        key[r] = valid ? kin[start + idx] : K{};
      }
    } else {
      key[r] = valid ? kin[start + idx] : K{};
    }
    if constexpr (kHasVal) {
      if (valid) val[r] = vin[start + idx];
    }
    const uint32_t d = (uint32_t)(sort_key(key[r]) >> shift) & mask;
    uint64_t vb = __ballot(valid);
    uint64_t peers = valid ? vb : ~vb;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b >= dbits) break;  // uniform: the digit has dbits bits
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
    // read the running count before the leader of each digit group adds to it
    const uint32_t run = valid ? s_wcnt[wave][d] : 0u;
    rank[r] = run + below;
    __builtin_amdgcn_wave_barrier();
    if (valid && below == 0) s_wcnt[wave][d] = run + (uint32_t)__popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // thread tid owns digit tid: offsets of each wavefront's run of that digit
  {
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
      const uint32_t c = s_wcnt[w][tid];
      s_wcnt[w][tid] = tot;  // exclusive prefix over wavefronts
      tot += c;
    }
    const uint32_t inc = wave_inclusive_scan(tot);
    if (lane == 63) s_wsum[wave] = inc;
    __syncthreads();
    uint32_t off = inc - tot;
    for (int w = 0; w < wave; ++w) off += s_wsum[w];
    s_excl[tid] = off;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; ++r) {
    const int idx = wave * kSub + r * kWave + lane;
    if (idx < len) {
      const uint32_t d = (uint32_t)(sort_key(key[r]) >> shift) & mask;
      const uint32_t pos = s_excl[d] + s_wcnt[wave][d] + rank[r];
      s_key[pos] = key[r];
      if constexpr (kHasVal) s_val[pos] = val[r];
    }
  }
  __syncthreads();
  for (int i = tid; i < len; i += kSortBlock) {
    const K k = s_key[i];
    const uint32_t d = (uint32_t)(sort_key(k) >> shift) & mask;
    const int64_t gpos = (int64_t)s_base[d] + (i - (int64_t)s_excl[d]);
    if constexpr (std::is_same<K, uint4>::value) {
      // records: the last pass of a sort can re-key them for the next sort
      kout[gpos] = rec_xform(k, xf1);
      if (kout2) kout2[gpos] = rec_xform(k, xf2);
    } else {
      kout[gpos] = k;
    }
    if constexpr (kHasVal) vout[gpos] = s_val[i];
  }
}

// Sort (keys, vals) of length m by the low `bits` bits of the key, stably.
// Ping-pongs between (k0, v0) and (k1, v1); returns 0 if the result is in
// buffer 0, 1 if in buffer 1.
// returns -1 if the scan scratch is too small (nothing enqueued then)
// Records (K = uint4) leave the sort re-keyed by xf1, and if `extra` is given
// a second copy re-keyed by xf2 goes there.
template <typename K, typename V = int32_t, int ITEMS = kSortItems>
int radix_sort(K* k0, V* v0, K* k1, V* v1, int64_t m, int bits, uint32_t* hist,
               uint32_t* part, size_t part_elems, hipStream_t st,
               const uint32_t* dev_m = nullptr, int xf1 = RX_NONE, K* extra = nullptr,
               int xf2 = RX_NONE, const EdgeCols* first = nullptr) {
  if (m <= 0) return 0;
  constexpr int kTile = kSortBlock * ITEMS;
  const int64_t ntiles = (m + kTile - 1) / kTile;
  if (part_elems < col_scan_scratch_elems(ntiles)) return -1;
  int cur = 0;
  // ceil(bits / 8) passes with digit widths as equal as possible (narrow
  // ones first): fewer distinct digits per tile means longer runs in the
  // scatter's output, and fewer partly written cache lines
  const int npass = (bits + 7) / 8;
  if constexpr (std::is_same<K, uint4>::value) {
    if (npass == 0 && (xf1 != RX_NONE || extra))
      hipLaunchKernelGGL(k_rec_xform, dim3(blocks_for(m, 256)), dim3(256), 0, st, k0, m, xf1,
                         extra, xf2);
  }
  for (int p = 0, shift = 0; p < npass; ++p) {
    const bool last = p + 1 == npass;
    const int dbits = (bits - shift) / (npass - p);
    const uint32_t mask = (1u << dbits) - 1u;
    K* ki = cur ? k1 : k0;
    V* vi = cur ? v1 : v0;
    K* ko = cur ? k0 : k1;
    V* vo = cur ? v0 : v1;
    // with `first`, pass 0 reads the edge columns instead of k0 (K = uint4)
    const EdgeCols ec = (p == 0 && first) ? *first : EdgeCols{nullptr, nullptr, nullptr, 0};
    hipLaunchKernelGGL((k_radix_hist<K, ITEMS>), dim3((unsigned)ntiles), dim3(kSortBlock), 0, st,
                       (const K*)ki, m, shift, mask, hist, dev_m, ec);
    col_scan(hist, ntiles, part, st);
    {
      TimedLaunch tl("k_radix_scatter", st);
      hipLaunchKernelGGL((k_radix_scatter<K, V, ITEMS>), dim3((unsigned)ntiles), dim3(kSortBlock),
                         0, st, (const K*)ki, (const V*)vi, ko, vo, m, shift, dbits,
                         (const uint32_t*)hist, dev_m, last ? xf1 : (int)RX_NONE,
                         last ? extra : (K*)nullptr, last ? xf2 : (int)RX_NONE, ec);
    }
    cur ^= 1;
    shift += dbits;
  }
  return cur;
}

// -------------------------------------------------------- columns/offsets ---
// Gather the columns of one order.  key_col receives the sort key (the
// vertex), the optional other columns come from the input arrays.
__global__ __launch_bounds__(256) void k_gather_order(
    const uint32_t* __restrict__ skeys, const int32_t* __restrict__ order, int64_t m,
    const int32_t* __restrict__ other_v, const int64_t* __restrict__ t,
    int32_t* __restrict__ key_col, int32_t* __restrict__ other_col, int64_t* __restrict__ t_col,
    int32_t* __restrict__ eid_col, uint4* __restrict__ rec) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    int32_t e = order[i];
    if (key_col) key_col[i] = (int32_t)skeys[i];
    const int32_t o = other_v[e];
    const int64_t te = t[e];
    if (other_col) other_col[i] = o;
    t_col[i] = te;
    eid_col[i] = e;
    if (rec) rec[i] = make_uint4((uint32_t)o, (uint32_t)e, (uint32_t)te, (uint32_t)(te >> 32));
  }
}

// off[v] = first position whose sorted key is >= v, for v in [0, n]
__global__ __launch_bounds__(256) void k_offsets(const uint32_t* __restrict__ skeys, int64_t m,
                                                 int32_t n, uint32_t* __restrict__ off) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  int64_t prev = (i == 0) ? -1 : (int64_t)skeys[i - 1];
  int64_t cur = (i == m) ? (int64_t)n : (int64_t)skeys[i];
  for (int64_t v = prev + 1; v <= cur; ++v) off[v] = (uint32_t)i;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ a, int64_t n,
                                                  uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

// ----------------------------------------------------- pair-run hash table ---
// Every maximal run of equal (src, dst) in the pair index is one entry of an
// open-addressing table (linear probing, Fibonacci hashing of the 64-bit key
// src << 32 | dst).  A slot is 16 bytes {key, run start, run end}, so a hit
// costs one 16-byte load.  The capacity is a power of two above 1.25 m, so
// the load factor stays below 0.8 and a probe always reaches an empty slot.
__global__ __launch_bounds__(256) void k_hash_clear(PairSlot* __restrict__ tab, int64_t cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cap) {
    tab[i].key = kPairEmpty;
    tab[i].start = 0;
    tab[i].end = 0;
  }
}

// One thread per pair-index position.  The thread at the first position of
// a (src, dst) run finds where the run ends -- galloping over the sorted
// keys, then bisecting the last gap, so a run of length L costs O(log L)
// probes and most runs (a single edge) one -- and inserts {key, start, end}.
__global__ __launch_bounds__(256) void k_hash_insert(const uint32_t* __restrict__ psrc,
                                                     const int32_t* __restrict__ pdst, int64_t m,
                                                     PairSlot* __restrict__ tab, int log2cap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  auto key_at = [&](int64_t j) { return pair_key(psrc[j], (uint32_t)pdst[j]); };
  const uint64_t key = key_at(i);
  if (i > 0 && key_at(i - 1) == key) return;
  int64_t lo = i, hi, step = 1;  // key_at(lo) == key
  for (;;) {
    hi = lo + step;
    if (hi >= m || key_at(hi) != key) break;
    lo = hi;
    step <<= 1;
  }
  if (hi > m) hi = m;  // hi == m, or key_at(hi) != key
  while (hi - lo > 1) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (key_at(mid) == key)
      lo = mid;
    else
      hi = mid;
  }
  const uint64_t mask = (1ull << log2cap) - 1;
  uint64_t h = pair_hash(key, log2cap);
  for (uint64_t probe = 0; probe <= mask; ++probe) {
    const unsigned long long prev =
        atomicCAS((unsigned long long*)&tab[h].key, (unsigned long long)kPairEmpty,
                  (unsigned long long)key);
    if (prev == kPairEmpty) {
      tab[h].start = (uint32_t)i;
      tab[h].end = (uint32_t)hi;
      return;
    }
    h = (h + 1) & mask;
  }
}

// Sampled levels of the pair times: level k holds pair_t[16^k i].
__global__ __launch_bounds__(256) void k_pair_skip(const int64_t* __restrict__ pair_t, int64_t n1,
                                                   int64_t n2, int64_t n3,
                                                   int64_t* __restrict__ skip) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n1)
    skip[i] = pair_t[i << 4];
  else if (i < n1 + n2)
    skip[i] = pair_t[(i - n1) << 8];
  else if (i < n1 + n2 + n3)
    skip[i] = pair_t[(i - n1 - n2) << 12];
}

int pair_hash_log2(int64_t m) {
  int lg = 4;
  while (((int64_t)1 << lg) < m + m / 4 + 1) ++lg;
  return lg;
}

// ---------------------------------------------- sorts carrying their payload ---
// When the time range fits 32 bits every sort moves its whole record, one
// 16-byte word per edge: key (u32) + payload {eid, other vertex, t - t_min},
// so each column of the three orders comes out of the last pass in order,
// with no random gathers, and each digit run of a pass is one contiguous
// stretch of records.
__global__ __launch_bounds__(256) void k_rec_init(const int32_t* __restrict__ src,
                                                  const int32_t* __restrict__ dst,
                                                  const int64_t* __restrict__ t, int64_t m,
                                                  int64_t tmin, uint4* __restrict__ rec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m)
    rec[i] = make_uint4((uint32_t)(t[i] - tmin), (uint32_t)i, (uint32_t)src[i], (uint32_t)dst[i]);
}

// sorted (key, eid, other, t - t_min) -> columns of one order
// With `off` (n + 1 entries), also the CSR offsets of the sorted keys:
// off[v] = first position whose key is >= v, written by the thread of the
// position where the key passes v (grid of m + 1 threads).  With `skip`
// (the pair index), also the sampled levels skip_k[i] = t[16^k i], k = 1..3,
// from the times this pass writes anyway.
__global__ __launch_bounds__(256) void k_emit(const uint4* __restrict__ in, int64_t m,
                                              int64_t tmin, int32_t* __restrict__ key_col,
                                              int32_t* __restrict__ other_col,
                                              int64_t* __restrict__ t_col,
                                              int32_t* __restrict__ eid_col,
                                              uint4* __restrict__ rec, int32_t n,
                                              uint32_t* __restrict__ off,
                                              int64_t* __restrict__ skip) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const uint4 r = in[i];
    key_col[i] = (int32_t)r.x;
    const int64_t te = tmin + (int64_t)r.w;
    other_col[i] = (int32_t)r.z;
    t_col[i] = te;
    eid_col[i] = (int32_t)r.y;
    if (rec) rec[i] = make_uint4(r.z, r.y, (uint32_t)te, (uint32_t)(te >> 32));
    if (skip && (i & 15) == 0) {
      const int64_t n1 = skip_level_len(m, 1), n2 = skip_level_len(m, 2);
      skip[i >> 4] = te;
      if ((i & 255) == 0) skip[n1 + (i >> 8)] = te;
      if ((i & 4095) == 0) skip[n1 + n2 + (i >> 12)] = te;
    }
  }
  if (off && i <= m) {
    const int64_t prev = (i == 0) ? -1 : (int64_t)in[i - 1].x;
    const int64_t cur = (i == m) ? (int64_t)n : (int64_t)in[i].x;
    for (int64_t v = prev + 1; v <= cur; ++v) off[v] = (uint32_t)i;
  }
}

// --------------------------------------------------------------- layout ----
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct GraphLayout {
  size_t out_off, in_off, out_src, out_dst, out_eid, out_t, in_src, in_eid, in_dst, in_t,
      pair_dst, out_rec, in_rec,
      pair_eid, pair_t, pair_hash, pair_skip, status, tminmax, keys0, keys1, vals0, vals1, hist, part,
      part_elems, rr[4], total;
};

static GraphLayout graph_layout(int32_t n, int64_t m) {
  GraphLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes ? bytes : 1);
    return at;
  };
  const size_t M = (size_t)m;
  // histograms sized for the smaller (1536-entry) tiles of the record sorts
  const int64_t ntiles = (m + kRecTile - 1) / kRecTile;
  L.out_off = take(((size_t)n + 1) * 4);
  L.in_off = take(((size_t)n + 1) * 4);
  L.out_src = take(M * 4);
  L.out_dst = take(M * 4);
  L.out_eid = take(M * 4);
  L.out_t = take(M * 8);
  L.in_src = take(M * 4);
  L.in_eid = take(M * 4);
  L.in_dst = take(M * 4);
  L.in_t = take(M * 8);
  L.pair_dst = take(M * 4);
  L.pair_eid = take(M * 4);
  L.pair_t = take(M * 8);
  L.out_rec = take(M * 16);
  L.in_rec = take(M * 16);
  L.pair_hash = take(sizeof(PairSlot) << pair_hash_log2(m));
  L.pair_skip =
      take((size_t)(skip_level_len(m, 1) + skip_level_len(m, 2) + skip_level_len(m, 3)) * 8);
  // the status word and, 16 bytes on, the time min/max keys: one 32-byte
  // read-back after the validation
  L.status = take(32);
  L.tminmax = L.status + 16;
  // sort scratch: four 16-byte-record buffers for the record-carrying
  // sorts (two per concurrent branch), aliased by the
  // 64-bit-key buffers of the wide-time path (the two paths never run in the
  // same build)
  const size_t region = o;
  for (int b = 0; b < 4; ++b) L.rr[b] = take((M + 1) * 16);
  const size_t rec_end = o;
  o = region;
  L.keys0 = take((M + 1) * 8);
  L.keys1 = take((M + 1) * 8);
  L.vals0 = take((M + 1) * 4);
  L.vals1 = take((M + 1) * 4);
  if (o < rec_end) o = rec_end;
  L.hist = take((size_t)256 * ntiles * 4);
  // scan scratch of the histogram column scan
  L.part_elems = col_scan_scratch_elems(ntiles);
  L.part = take(L.part_elems * 4);
  L.total = o;
  return L;
}

// Second stream of a device for the build's independent branch, created once
// (default priority); the mutex also keeps two builds from interleaving their
// use of it and of its events.
struct SideStream {
  std::mutex mu;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, out_done = nullptr;
  bool ok = false, tried = false;
};
static SideStream g_side[64];

static SideStream* side_stream() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  SideStream* S = &g_side[dev];
  return S;
}

// with S->mu held
static bool side_ready(SideStream* S) {
  if (!S->tried) {
    S->tried = true;
    S->ok = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&S->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&S->out_done, hipEventDisableTiming) == hipSuccess;
  }
  return S->ok;
}

size_t graph_workspace_bytes(int32_t n, int64_t m) { return graph_layout(n, m).total; }

static int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }


// The pair-run table and the sampled pair times, from the pair index's
// sorted src keys.
static void clear_pair_hash(const tc_graph* g, hipStream_t st) {
  const int64_t cap = (int64_t)1 << g->pair_hash_log2;
  hipLaunchKernelGGL(k_hash_clear, dim3(blocks_for(cap, 256)), dim3(256), 0, st,
                     (PairSlot*)g->pair_hash, cap);
}

static void build_pair_hash(const uint32_t* psrc, const tc_graph* g, int64_t m, PairSlot* tab,
                            hipStream_t st, bool with_skip) {
  if (with_skip) {
    const int64_t n1 = skip_level_len(m, 1), n2 = skip_level_len(m, 2), n3 = skip_level_len(m, 3);
    hipLaunchKernelGGL(k_pair_skip, dim3(blocks_for(n1 + n2 + n3, 256)), dim3(256), 0, st,
                       (const int64_t*)g->pair_t, n1, n2, n3, g->pair_skip);
  }
  hipLaunchKernelGGL(k_hash_insert, dim3(blocks_for(m, 256)), dim3(256), 0, st, psrc,
                     (const int32_t*)g->pair_dst, m, tab, g->pair_hash_log2);
}

tc_status build_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      const int64_t* t, void* ws, size_t ws_bytes, hipStream_t st, tc_graph* g) {
  GraphLayout L = graph_layout(n, m);
  if (ws_bytes < L.total) return TC_E_WORKSPACE;
  char* base = (char*)ws;
  g->n = n;
  g->m = m;
  g->out_off = (uint32_t*)(base + L.out_off);
  g->in_off = (uint32_t*)(base + L.in_off);
  g->out_src = (int32_t*)(base + L.out_src);
  g->out_dst = (int32_t*)(base + L.out_dst);
  g->out_eid = (int32_t*)(base + L.out_eid);
  g->out_t = (int64_t*)(base + L.out_t);
  g->in_src = (int32_t*)(base + L.in_src);
  g->in_eid = (int32_t*)(base + L.in_eid);
  g->in_dst = (int32_t*)(base + L.in_dst);
  g->in_t = (int64_t*)(base + L.in_t);
  g->pair_dst = (int32_t*)(base + L.pair_dst);
  g->pair_eid = (int32_t*)(base + L.pair_eid);
  g->pair_t = (int64_t*)(base + L.pair_t);
  g->status = (uint32_t*)(base + L.status);
  g->pair_hash = (void*)(base + L.pair_hash);
  g->pair_hash_log2 = pair_hash_log2(m);
  g->pair_skip = (int64_t*)(base + L.pair_skip);
  g->out_rec = (void*)(base + L.out_rec);
  g->in_rec = (void*)(base + L.in_rec);
  uint64_t* tminmax = (uint64_t*)(base + L.tminmax);
  void* keys0 = base + L.keys0;
  void* keys1 = base + L.keys1;
  int32_t* vals0 = (int32_t*)(base + L.vals0);
  int32_t* vals1 = (int32_t*)(base + L.vals1);
  uint32_t* hist = (uint32_t*)(base + L.hist);
  uint32_t* part = (uint32_t*)(base + L.part);
  const size_t pe = L.part_elems;

  hipLaunchKernelGGL(k_init_build, dim3(1), dim3(64), 0, st, g->status, tminmax);
  if (m > 0) {
    unsigned vb = blocks_for(m, 256);
    if (vb > 1024) vb = 1024;
    hipLaunchKernelGGL(k_validate, dim3(vb), dim3(256), 0, st, src, dst, t, m, n, g->status,
                       tminmax);
  }
  // read back into pinned memory (one per host thread, kept for the
  // process): a pageable copy is staged, and its latency sits between the
  // validation and the first sort
  static thread_local uint64_t* pinned = nullptr;
  if (!pinned && hipHostMalloc((void**)&pinned, 32, hipHostMallocDefault) != hipSuccess)
    pinned = nullptr;
  uint64_t local[4] = {0, 0, 0, 0};
  uint64_t* rb = pinned ? pinned : local;
  if (hipMemcpyAsync(rb, g->status, 32, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return TC_E_HIP;
  if ((uint32_t)rb[0] != 0) return TC_E_RANGE;
  const int64_t tmin = m > 0 ? (int64_t)(rb[2] ^ (1ull << 63)) : 0;
  const int64_t tmax = m > 0 ? (int64_t)(rb[3] ^ (1ull << 63)) : 0;
  g->t_min = tmin;
  g->t_max = tmax;
  const unsigned eb = blocks_for(m > 0 ? m : 1, 256);

  const int tbits = bitlen((uint64_t)(tmax - tmin));
  const int vbits = bitlen((uint64_t)(n - 1));
  PairSlot* tab = (PairSlot*)g->pair_hash;
  if (m == 0) {
    clear_pair_hash(g, st);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->out_off, (int64_t)n + 1, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->in_off, (int64_t)n + 1, 0u);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    return TC_OK;
  }
  if (tbits <= 32) {
    // record-carrying sorts.  This stream sorts by time, then the in-CSR,
    // the pair index and the out-CSR (bandwidth bound).  A second stream
    // clears the run table during the sorts and builds it (random atomics,
    // latency bound) beside the out-CSR sort.  Four record buffers: the time
    // sort ping-pongs in 0 and 1, the in-CSR sort in 2 and the free one of
    // those, the pair sort in 3 and the one the in-CSR sort left free, and
    // the out-CSR sort in A (the time sort's result) and the in-CSR result.
    uint4* rr[4];
    for (int b = 0; b < 4; ++b) rr[b] = (uint4*)(base + L.rr[b]);
    auto sort_rec = [&](int from, int tmp, int bits, uint32_t* h, uint32_t* pt, hipStream_t s,
                        int xf1 = RX_NONE, int extra = -1, int xf2 = RX_NONE,
                        const EdgeCols* first = nullptr) -> int {
      const int w = radix_sort<uint4, NoVal, kRecItems>(
          rr[from], (NoVal*)nullptr, rr[tmp], (NoVal*)nullptr, m, bits, h, pt, pe, s, nullptr,
          xf1, extra < 0 ? (uint4*)nullptr : rr[extra], xf2, first);
      return w < 0 ? -1 : (w ? tmp : from);
    };
    SideStream* S = side_stream();
    std::unique_lock<std::mutex> lock;
    if (S) lock = std::unique_lock<std::mutex>(S->mu);
    const bool two = S && side_ready(S);
    hipStream_t s2 = two ? S->s : st;
    // time order.  Its first pass reads the edge columns and builds the
    // records as it loads them (with no pass, k_rec_init builds them); its
    // last pass leaves them re-keyed as the input of the out-CSR sort
    // (buffer A, the sort's own) and of the in-CSR sort (B)
    const EdgeCols ec{src, dst, t, tmin};
    if (tbits == 0)
      hipLaunchKernelGGL(k_rec_init, dim3(eb), dim3(256), 0, st, src, dst, t, m, tmin, rr[0]);
    const int A = sort_rec(0, 1, tbits, hist, part, st, RX_OUT, 2, RX_IN, tbits ? &ec : nullptr);
    if (A < 0) return TC_E_WORKSPACE;
    // the second stream clears the run table meanwhile (ordered after the
    // caller's earlier work on this stream)
    if (two) {
      if (hipEventRecord(S->fork, st) != hipSuccess ||
          hipStreamWaitEvent(s2, S->fork, 0) != hipSuccess)
        return TC_E_HIP;
    }
    clear_pair_hash(g, s2);
    const int B = 2, F = 1 - A;
    // in-CSR: stable by dst; a second copy of the result, re-keyed, is the
    // pair index input (buffer 3)
    const int I = sort_rec(B, F, vbits, hist, part, st, RX_NONE, 3, RX_PAIR);
    if (I < 0) return TC_E_WORKSPACE;
    const int Ifree = (I == B) ? F : B;
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st,
                       (const uint4*)rr[I], m, tmin, g->in_dst, g->in_src, g->in_t, g->in_eid,
                       (uint4*)g->in_rec, n, g->in_off, (int64_t*)nullptr);
    // pair index: the in-order (dst, t, eid) stably by src
    const int Pr = sort_rec(3, Ifree, vbits, hist, part, st);
    if (Pr < 0) return TC_E_WORKSPACE;
    const int Pfree = (Pr == 3) ? Ifree : 3;
    // the pair sort's spare buffer holds the pair sources
    uint32_t* psrc = (uint32_t*)rr[Pfree];
    hipLaunchKernelGGL(k_emit, dim3(eb), dim3(256), 0, st, (const uint4*)rr[Pr], m, tmin,
                       (int32_t*)psrc, g->pair_dst, g->pair_t, g->pair_eid, (uint4*)nullptr, n,
                       (uint32_t*)nullptr, g->pair_skip);
    if (two) {
      if (hipEventRecord(S->fork, st) != hipSuccess ||
          hipStreamWaitEvent(s2, S->fork, 0) != hipSuccess)
        return TC_E_HIP;
    }
    // second stream: the run table, after its clear (the pair emit wrote
    // the sampled levels)
    build_pair_hash(psrc, g, m, tab, s2, false);
    if (two && hipEventRecord(S->out_done, s2) != hipSuccess) return TC_E_HIP;
    // this stream, meanwhile: out-CSR (stable by src), with the in-CSR
    // records' buffer (emitted before the fork) as its spare
    const int R = sort_rec(A, I, vbits, hist, part, st);
    if (R < 0) return TC_E_WORKSPACE;
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st,
                       (const uint4*)rr[R], m, tmin, g->out_src, g->out_dst, g->out_t,
                       g->out_eid, (uint4*)g->out_rec, n, g->out_off, (int64_t*)nullptr);
    if (two && hipStreamWaitEvent(st, S->out_done, 0) != hipSuccess) return TC_E_HIP;
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    return TC_OK;
  }
  // wide time range: 64-bit time keys, columns gathered after each sort
  clear_pair_hash(g, st);
  // 1. time order: stable by t (initial order = eid)
  int32_t* torder;
  if (m > 0) {
    int where;
    if (tbits <= 32) {
      hipLaunchKernelGGL((k_time_keys<uint32_t>), dim3(eb), dim3(256), 0, st, t, m, tmin,
                         (uint32_t*)keys0, vals0);
      where = radix_sort<uint32_t>((uint32_t*)keys0, vals0, (uint32_t*)keys1, vals1, m, tbits,
                                   hist, part, pe, st);
    } else {
      hipLaunchKernelGGL((k_time_keys<uint64_t>), dim3(eb), dim3(256), 0, st, t, m, tmin,
                         (uint64_t*)keys0, vals0);
      where = radix_sort<uint64_t>((uint64_t*)keys0, vals0, (uint64_t*)keys1, vals1, m, tbits,
                                   hist, part, pe, st);
    }
    if (where < 0) return TC_E_WORKSPACE;
    torder = where ? vals1 : vals0;
  } else {
    torder = vals0;
  }
  // the time order is kept in the eid column of the pair index until the
  // pair sort needs it (pair_eid is rewritten at the end)
  int32_t* torder_keep = g->pair_eid;
  if (m > 0 &&
      hipMemcpyAsync(torder_keep, torder, (size_t)m * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return TC_E_HIP;
  uint32_t* k0 = (uint32_t*)keys0;
  uint32_t* k1 = (uint32_t*)keys1;
  // 2. out-CSR: stable by src
  if (m > 0) {
    hipLaunchKernelGGL(k_vertex_keys, dim3(eb), dim3(256), 0, st, src, torder_keep, m, k0, vals0);
    int w = radix_sort<uint32_t>(k0, vals0, k1, vals1, m, vbits, hist, part, pe, st);
    if (w < 0) return TC_E_WORKSPACE;
    uint32_t* sk = w ? k1 : k0;
    int32_t* sv = w ? vals1 : vals0;
    hipLaunchKernelGGL(k_gather_order, dim3(eb), dim3(256), 0, st, (const uint32_t*)sk,
                       (const int32_t*)sv, m, dst, t, g->out_src, g->out_dst, g->out_t,
                       g->out_eid, (uint4*)g->out_rec);
    hipLaunchKernelGGL(k_offsets, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st,
                       (const uint32_t*)sk, m, n, g->out_off);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->out_off, (int64_t)n + 1, 0u);
  }
  // 3. in-CSR: stable by dst
  if (m > 0) {
    hipLaunchKernelGGL(k_vertex_keys, dim3(eb), dim3(256), 0, st, dst, torder_keep, m, k0, vals0);
    int w = radix_sort<uint32_t>(k0, vals0, k1, vals1, m, vbits, hist, part, pe, st);
    if (w < 0) return TC_E_WORKSPACE;
    uint32_t* sk = w ? k1 : k0;
    int32_t* sv = w ? vals1 : vals0;
    hipLaunchKernelGGL(k_gather_order, dim3(eb), dim3(256), 0, st, (const uint32_t*)sk,
                       (const int32_t*)sv, m, src, t, g->in_dst, g->in_src, g->in_t,
                       g->in_eid, (uint4*)g->in_rec);
    hipLaunchKernelGGL(k_offsets, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st,
                       (const uint32_t*)sk, m, n, g->in_off);
  } else {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->in_off, (int64_t)n + 1, 0u);
  }
  // 4. pair index: the in-order (dst, t, eid) stably sorted by src
  if (m > 0) {
    hipLaunchKernelGGL(k_vertex_keys, dim3(eb), dim3(256), 0, st, src, g->in_eid, m, k0, vals0);
    int w = radix_sort<uint32_t>(k0, vals0, k1, vals1, m, vbits, hist, part, pe, st);
    if (w < 0) return TC_E_WORKSPACE;
    uint32_t* sk = w ? k1 : k0;
    int32_t* sv = w ? vals1 : vals0;
    hipLaunchKernelGGL(k_gather_order, dim3(eb), dim3(256), 0, st, (const uint32_t*)sk,
                       (const int32_t*)sv, m, dst, t, (int32_t*)nullptr, g->pair_dst, g->pair_t,
                       g->pair_eid, (uint4*)nullptr);
    // 5. pair-run hash table (the sorted src keys are still in sk)
    build_pair_hash(sk, g, m, tab, st, true);
  }
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
