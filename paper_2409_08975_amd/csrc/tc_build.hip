// Temporal adjacency build: validation, stable LSD radix sorts and CSR
// offsets.  The canonical orders are (t, eid) -> (src, t, eid) for the
// out-lists, (dst, t, eid) for the in-lists and (src, dst, t, eid) for the
// per-pair lists; each later sort is a stable sort of the previous order, so
// timestamp ties keep increasing edge id (section III-A assumes time-sorted
// per-vertex lists; the tie order is this library's convention).
//
// Radix sort design (gfx950, wave64): every sort moves 16-byte edge
// records, tiles of 1536 records per 256-thread block; the last pass of a
// vertex sort writes the graph's columns instead of records.  A pass is (1)
// per-tile digit histograms written tile-major (each tile's 256 or 512
// counts are one contiguous row), (2) a column scan of that [tiles][bins]
// matrix that turns every count into the tile's global offset for its digit,
// (3) a scatter that ranks keys stably inside the tile with wavefront
// ballots (one ballot per digit bit gives the lanes sharing a digit), stages
// the tile in LDS in digit order and writes each digit run to its global
// slot with coalesced stores.
//
// The whole build is one stream-ordered launch sequence: it allocates
// nothing, never waits on the device, and can be captured in a HIP graph.
// The validation result and the time range stay on the device; the time
// sort's passes read their plan from there (see BuildPlan).
#include <hip/hip_runtime.h>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

constexpr int kSortBlock = 256;
constexpr uint32_t kXcds = 8;  // accelerator complex dies of an MI355X, each with its own L2
constexpr int kRecItems = 6;  // record-carrying sorts: 1536-entry tiles (LDS holds 16 B/entry)
constexpr int kRecTile = kSortBlock * kRecItems;
constexpr int kColChunk = 32;  // tiles per chunk of the histogram column scan
constexpr int kMaxBins = 512;  // digits of at most 9 bits

static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------ validation ---
__global__ void k_init_build(uint32_t* status, uint64_t* tminmax) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    *status = 0;
    tminmax[0] = ~0ull;  // min of order-preserving keys
    tminmax[1] = 0ull;   // max
  }
}

// The validation, which also counts the low byte of every time per sort tile
// (tile-major rows of 256, as the radix histograms): the first pass of the
// time sort takes its digit counts from these rows once t_min is known
// (k_fold_hist), so it needs no histogram read of its own.  Each block walks
// tiles blockIdx.x, blockIdx.x + gridDim.x, ...
// t is mapped to an order-preserving unsigned key (flip the sign bit)
__global__ __launch_bounds__(kSortBlock) void k_validate(const int32_t* __restrict__ src,
                                                         const int32_t* __restrict__ dst,
                                                         const int64_t* __restrict__ t, int64_t m,
                                                         int32_t n, uint32_t* status,
                                                         uint64_t* tminmax,
                                                         uint32_t* __restrict__ hist) {
  const int64_t lim = (int64_t)1 << 62;
  uint64_t mn = ~0ull, mx = 0;
  uint32_t bad = 0;
  auto check = [&](int32_t s, int32_t d, int64_t tt) {
    if (s < 0 || s >= n || d < 0 || d >= n || tt >= lim || tt <= -lim) bad = 1;
    const uint64_t key = (uint64_t)tt ^ (1ull << 63);
    mn = key < mn ? key : mn;
    mx = key > mx ? key : mx;
  };
  __shared__ uint32_t s_h[256];
  const int64_t ntiles = (m + kRecTile - 1) / kRecTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t start = tile * kRecTile;
    int32_t sv[kRecItems], dv[kRecItems];
    int64_t tv[kRecItems];
#pragma unroll
    for (int r = 0; r < kRecItems; ++r) {  // the tile's loads issued together
      const int64_t i = start + (int64_t)r * kSortBlock + threadIdx.x;
      const bool in = i < m;
      sv[r] = in ? src[i] : 0;
      dv[r] = in ? dst[i] : 0;
      tv[r] = in ? t[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < kRecItems; ++r) {
      if (start + (int64_t)r * kSortBlock + threadIdx.x < m) {
        check(sv[r], dv[r], tv[r]);
        atomicAdd(&s_h[(uint32_t)(uint64_t)tv[r] & 255u], 1u);
      }
    }
    __syncthreads();
    hist[tile * 256 + threadIdx.x] = s_h[threadIdx.x];
    __syncthreads();  // the next tile clears s_h
  }
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

// ------------------------------------------------------------ sort plan ---
// Every sort of the build moves whole 16-byte edge records.  The time sort
// sorts the records by t - t_min, which needs up to 63 bits: up to four
// passes over the low 32 bits, then (only when the range is wider than 32
// bits) up to four over the high 32 bits.  How many of those eight launched
// passes do work, their digit widths and their ping-pong buffers are decided
// on the device from the validated time range (k_plan), so the host
// enqueues the same launches whatever the data and never waits for the
// device: the build is one stream-ordered sequence that a HIP graph can
// capture.  A pass with no work leaves at once.
constexpr int kTimePasses = 8;  // launched passes of the time sort (4 low + 4 high)

struct BuildPlan {
  int64_t tmin, tmax;  // time range (0, 0 for an empty or rejected input)
  uint32_t bad;        // the validation set TC_F_RANGE: nothing after it runs
  int32_t wide;        // the range needs more than 32 bits (high-word passes)
  int32_t npass;       // passes of the time sort that do work
  int32_t active[kTimePasses], order[kTimePasses], shift[kTimePasses], dbits[kTimePasses];
};

__device__ __forceinline__ int bitlen_dev(uint64_t x) { return x ? 64 - __clzll(x) : 0; }

// ceil(bits / 8) passes with digit widths as equal as possible (narrow ones
// first): fewer distinct digits per tile means longer runs in the scatter's
// output, and fewer partly written cache lines
__host__ __device__ inline void digit_plan(int bits, int npass, int i, int* shift, int* dbits) {
  int sh = 0;
  for (int q = 0; q < i; ++q) sh += (bits - sh) / (npass - q);
  *shift = sh;
  *dbits = (bits - sh) / (npass - i);
}

__global__ void k_plan(const uint32_t* __restrict__ status, const uint64_t* __restrict__ tminmax,
                       int64_t m, BuildPlan* __restrict__ P) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  BuildPlan B;
  B.bad = *status != 0 ? 1u : 0u;
  B.tmin = B.tmax = 0;
  B.wide = 0;
  B.npass = 0;
  for (int p = 0; p < kTimePasses; ++p) B.active[p] = B.order[p] = B.shift[p] = B.dbits[p] = 0;
  if (!B.bad && m > 0) {
    B.tmin = (int64_t)(tminmax[0] ^ (1ull << 63));
    B.tmax = (int64_t)(tminmax[1] ^ (1ull << 63));
    const int tbits = bitlen_dev((uint64_t)(B.tmax - B.tmin));
    const int lo = tbits < 32 ? tbits : 32, hi = tbits - lo;
    const int nlo = (lo + 7) / 8, nhi = (hi + 7) / 8;
    for (int i = 0; i < nlo; ++i) {
      B.active[i] = 1;
      B.order[i] = i;
      digit_plan(lo, nlo, i, &B.shift[i], &B.dbits[i]);
    }
    for (int i = 0; i < nhi; ++i) {
      B.active[4 + i] = 1;
      B.order[4 + i] = nlo + i;
      digit_plan(hi, nhi, i, &B.shift[4 + i], &B.dbits[4 + i]);
    }
    B.npass = nlo + nhi;
    B.wide = hi > 0 ? 1 : 0;
  }
  *P = B;
}

// The digit counts of the time sort's first pass from the validation's
// low-byte counts: its digit is the low w <= 8 bits of t - t_min (shift 0),
// so digit d counts the bytes b with (b - t_min) mod 2^w = d.  In place, one
// tile row at a time.
__global__ __launch_bounds__(256) void k_fold_hist(uint32_t* __restrict__ hist, int64_t ntiles,
                                                   const BuildPlan* __restrict__ plan) {
  if (plan->bad || !plan->active[0]) return;
  __shared__ uint32_t s_r[256];
  const uint32_t W = 1u << plan->dbits[0], tm = (uint32_t)(uint64_t)plan->tmin;
  const uint32_t d = threadIdx.x;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    s_r[d] = hist[tile * 256 + d];
    __syncthreads();
    uint32_t v = 0;
    if (d < W)
      for (uint32_t b = (d + tm) & (W - 1); b < 256; b += W) v += s_r[b];
    hist[tile * 256 + d] = v;
    __syncthreads();  // the next row overwrites s_r
  }
}

// ------------------------------------------------------------ radix pass ---
// Re-keying of a 16-byte edge record between the sorts of the build:
//   RX_NONE  identity
//   RX_OUT   (t, eid, src, dst) -> (src, eid, dst, t)   out-CSR input
//   RX_PAIR  (a, eid, b, t) -> (b, eid, a, t): the in-CSR input from the
//            out-CSR one as it is loaded, and the pair-index input from the
//            in-CSR order
enum { RX_NONE = 0, RX_OUT = 1, RX_PAIR = 3 };
__device__ __forceinline__ uint4 rec_xform(const uint4& r, int xf) {
  if (xf == RX_OUT) return make_uint4(r.z, r.y, r.w, r.x);
  if (xf == RX_PAIR) return make_uint4(r.z, r.y, r.x, r.w);
  return r;
}

// The input edge columns (read by the first pass of the time sort, which
// builds each record (t - t_min, eid, src, dst) as it loads it, and by the
// first high-word pass, which re-keys each record with the high word of
// t[eid] - t_min).
struct EdgeCols {
  const int32_t* src;
  const int32_t* dst;
  const int64_t* t;
};

// Where a pass reads its records from.
enum { SRC_BUF = 0, SRC_COLS = 1, SRC_HIGH = 2, SRC_INCOLS = 3 };

// The in-list columns as the pair sort's input: the 16-byte in-CSR records
// {src, eid, t} and the key column dst give the record (src, eid, dst,
// t - t_min) in in-CSR order, so no re-keyed copy of the in-CSR order is
// written for it.
struct InCols {
  const uint4* rec;
  const int32_t* key;
  const BuildPlan* plan;  // t_min
};

// The graph columns that the last pass of a vertex sort writes in place of
// its sorted records: for output position i with record (key, eid, other,
// t - t_min), key[i], other[i], t[i], eid[i], optionally the 16-byte record
// {other, eid, t} and, every 16th position, the sampled time levels.
struct EmitCols {
  const BuildPlan* plan;  // time base, the wide-range flag and the validation
  const int64_t* t_in;    // input times, read by edge id for wide ranges
  int32_t* key;
  int32_t* other;
  int64_t* t;
  int32_t* eid;
  uint4* rec;      // or null
  int64_t* skip;   // or null
};

// One launched radix pass.  With `plan` null the host planned it (the vertex
// sorts: bit counts follow from n); otherwise it is pass `pass` of the time
// sort and everything below `plan` is resolved on the device.
struct RecPass {
  const BuildPlan* plan;
  int pass;
  const uint4* in;  // host-planned input
  uint4* out;       // host-planned output
  uint4* buf[2];    // time sort: the ping-pong buffers (the sort ends in buf[0])
  int shift, dbits;
  int xfin;         // re-keying of the input as it is loaded (host-planned passes)
  int xf1;          // re-keying of the output (last pass of a sort)
  uint4* out2;      // second, re-keyed copy (last pass), or null
  int xf2;
  EdgeCols ec;
  EmitCols E;       // k_radix_scatter<..., true>: the columns out of the last pass
  InCols ic;        // host-planned input from the in-list columns (ic.rec non-null)
};

struct PassCfg {
  bool active;
  int shift, dbits, src, xfin, xf1, xf2;
  int64_t tmin;
  const uint4* in;
  uint4* out;
  uint4* out2;
  InCols ic;
};

__device__ __forceinline__ PassCfg resolve(const RecPass& R) {
  PassCfg c;
  c.tmin = 0;
  if (!R.plan) {
    c.active = true;
    c.shift = R.shift;
    c.dbits = R.dbits;
    c.src = R.ic.rec ? SRC_INCOLS : SRC_BUF;
    c.ic = R.ic;
    if (R.ic.rec) c.tmin = R.ic.plan->tmin;
    c.xfin = R.xfin;
    c.in = R.in;
    c.out = R.out;
    c.xf1 = R.xf1;
    c.out2 = R.out2;
    c.xf2 = R.xf2;
    return c;
  }
  const BuildPlan& P = *R.plan;
  const int p = R.pass;
  c.xfin = RX_NONE;
  c.ic = InCols{nullptr, nullptr, nullptr};
  c.active = P.active[p] != 0 && P.bad == 0;
  c.shift = P.shift[p];
  c.dbits = P.dbits[p];
  c.tmin = P.tmin;
  // active pass i of n writes buf[(n - 1 - i) & 1], so the last one writes
  // buf[0]; pass 0 reads the edge columns, the others the previous output
  const int i = P.order[p], n = P.npass;
  c.out = R.buf[(n - 1 - i) & 1];
  c.in = R.buf[(n - i) & 1];
  c.src = i == 0 ? SRC_COLS : (p == 4 ? SRC_HIGH : SRC_BUF);
  const bool last = i == n - 1;
  c.xf1 = last ? R.xf1 : RX_NONE;
  c.out2 = last ? R.out2 : nullptr;
  c.xf2 = last ? R.xf2 : RX_NONE;
  return c;
}

__device__ __forceinline__ uint4 load_rec(const PassCfg& c, const EdgeCols& ec, int64_t g) {
  if (c.src == SRC_COLS)
    return make_uint4((uint32_t)(uint64_t)(ec.t[g] - c.tmin), (uint32_t)g, (uint32_t)ec.src[g],
                      (uint32_t)ec.dst[g]);
  if (c.src == SRC_INCOLS) {
    const uint4 q = c.ic.rec[g];
    const int64_t te = (int64_t)(((uint64_t)q.w << 32) | q.z);
    return make_uint4(q.x, q.y, (uint32_t)c.ic.key[g], (uint32_t)(uint64_t)(te - c.tmin));
  }
  uint4 r = c.in[g];
  if (c.src == SRC_HIGH) r.x = (uint32_t)((uint64_t)(ec.t[r.y] - c.tmin) >> 32);
  return rec_xform(r, c.xfin);
}

// With no active time pass (every time equal): the records built from the
// edge columns, re-keyed like the last pass of the time sort would leave them.
__global__ __launch_bounds__(256) void k_rec_init(EdgeCols ec, int64_t m,
                                                  const BuildPlan* __restrict__ plan,
                                                  uint4* __restrict__ out, int xf1,
                                                  uint4* __restrict__ out2, int xf2) {
  if (plan->npass != 0 || plan->bad) return;
  // grid-stride: the launch is small, since it is idle for all but inputs
  // whose times are all equal
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint4 r = make_uint4((uint32_t)(uint64_t)(ec.t[i] - plan->tmin), (uint32_t)i,
                               (uint32_t)ec.src[i], (uint32_t)ec.dst[i]);
    out[i] = rec_xform(r, xf1);
    if (out2) out2[i] = rec_xform(r, xf2);
  }
}

// the re-keying of a vertex sort with no pass (n = 1): a[i] from in[i]
// (in == a allowed: every element is read and written by the same thread)
__global__ __launch_bounds__(256) void k_rec_xform(const uint4* in, int xfin, uint4* a, int64_t m,
                                                   int xf1, uint4* __restrict__ out2, int xf2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const uint4 r = rec_xform(in[i], xfin);
    a[i] = rec_xform(r, xf1);
    if (out2) out2[i] = rec_xform(r, xf2);
  }
}

template <int ITEMS, int BINS>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(RecPass R, int64_t m,
                                                           uint32_t* __restrict__ hist) {
  constexpr int kDig = BINS / kSortBlock;  // digits per thread
  __shared__ uint32_t s_h[BINS];
  const PassCfg c = resolve(R);
  if (!c.active) return;
  const uint32_t mask = (1u << c.dbits) - 1u;
  // one tile per block, or several when the grid is smaller than the tile
  // count (the passes that are usually idle)
  const int64_t ntiles = (m + kSortBlock * ITEMS - 1) / (kSortBlock * ITEMS);
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
#pragma unroll
    for (int q = 0; q < kDig; ++q) s_h[q * kSortBlock + threadIdx.x] = 0;
    __syncthreads();
    const int64_t start = tile * (kSortBlock * ITEMS);
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      int64_t i = start + (int64_t)r * kSortBlock + threadIdx.x;
      if (i < m) {
        const uint32_t key = c.src == SRC_COLS ? (uint32_t)(uint64_t)(R.ec.t[i] - c.tmin)
                                               : load_rec(c, R.ec, i).x;
        atomicAdd(&s_h[(key >> c.shift) & mask], 1u);
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kDig; ++q)
      hist[tile * BINS + q * kSortBlock + threadIdx.x] = s_h[q * kSortBlock + threadIdx.x];
    __syncthreads();  // the next tile clears s_h
  }
}

// Column scan of the tile-major histogram: hist[t][d] becomes the position
// of tile t's first key of digit d in the pass output, i.e. the keys of all
// smaller digits plus the keys of digit d in tiles before t.  Three kernels:
// per-chunk column sums, an exclusive scan of each digit's chunk sums (which
// also leaves the digit totals in row `nchunks`), and an in-place walk of
// every chunk that adds the digit base.  Every access reads or writes whole
// rows (BINS words) except the per-digit chunk scan, which touches
// nchunks*BINS words.  `gate` (time sort passes) skips a pass the plan
// leaves idle.
struct PassGate {
  const BuildPlan* plan;
  int pass;
};
__device__ __forceinline__ bool idle(const PassGate& G) {
  return G.plan && (G.plan->bad || !G.plan->active[G.pass]);
}

template <int BINS>
__global__ __launch_bounds__(256) void k_col_sum(const uint32_t* __restrict__ hist,
                                                 int64_t ntiles, uint32_t* __restrict__ csum,
                                                 PassGate gate) {
  if (idle(gate)) return;
  const int64_t t0 = (int64_t)blockIdx.x * kColChunk;
#pragma unroll
  for (int q = 0; q < BINS / 256; ++q) {
    const int d = q * 256 + threadIdx.x;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      // clamped index: every load is issued unconditionally
      const int64_t t = t0 + j < ntiles ? t0 + j : ntiles - 1;
      const uint32_t v = hist[t * BINS + d];
      s += (t0 + j < ntiles) ? v : 0u;
    }
    csum[(int64_t)blockIdx.x * BINS + d] = s;
  }
}

// one block per digit (blockIdx.x), chunks spread over the block's threads
template <int BINS>
__global__ __launch_bounds__(256) void k_col_scan(uint32_t* __restrict__ csum, int64_t nchunks,
                                                  PassGate gate) {
  if (idle(gate)) return;
  __shared__ uint32_t s_w[256 / kWave];
  const int d = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nchunks; base += 256) {
    const int64_t c = base + threadIdx.x;
    const uint32_t v = c < nchunks ? csum[c * BINS + d] : 0u;
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
      off += w < wave ? s_w[w] : 0u;
      tot += s_w[w];
    }
    if (c < nchunks) csum[c * BINS + d] = carry + off + inc - v;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) csum[nchunks * BINS + d] = carry;
}

// one block per chunk; thread tid walks the chunk's tiles for digits
// tid, tid + 256, ...
template <int BINS>
__global__ __launch_bounds__(256) void k_col_apply(uint32_t* __restrict__ hist, int64_t ntiles,
                                                   const uint32_t* __restrict__ csum,
                                                   int64_t nchunks, PassGate gate) {
  if (idle(gate)) return;
  constexpr int kDig = BINS / 256;
  __shared__ uint32_t s_w[kDig][256 / kWave];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t t0 = (int64_t)blockIdx.x * kColChunk;
  uint32_t carry = 0;  // totals of the digits below this group of 256
#pragma unroll
  for (int q = 0; q < kDig; ++q) {
    const int d = q * 256 + tid;
    // digit base: exclusive scan of the digit totals over d
    const uint32_t tot = csum[nchunks * BINS + d];
    const uint32_t inc = wave_inclusive_scan(tot);
    if (lane == 63) s_w[q][wave] = inc;
    __syncthreads();
    uint32_t run = carry + inc - tot, group = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) {
      run += w < wave ? s_w[q][w] : 0u;
      group += s_w[q][w];
    }
    carry += group;
    run += csum[(int64_t)blockIdx.x * BINS + d];
    uint32_t v[kColChunk];
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      const int64_t t = t0 + j < ntiles ? t0 + j : ntiles - 1;
      v[j] = hist[t * BINS + d];
    }
#pragma unroll
    for (int j = 0; j < kColChunk; ++j) {
      if (t0 + j < ntiles) hist[(t0 + j) * BINS + d] = run;
      run += v[j];
    }
  }
}

size_t col_scan_scratch_elems(int64_t ntiles, int bins) {
  return (size_t)bins * ((ntiles + kColChunk - 1) / kColChunk + 1);
}

template <int BINS>
void col_scan(uint32_t* hist, int64_t ntiles, uint32_t* csum, PassGate gate, hipStream_t st) {
  const int64_t nchunks = (ntiles + kColChunk - 1) / kColChunk;
  hipLaunchKernelGGL(k_col_sum<BINS>, dim3((unsigned)nchunks), dim3(256), 0, st,
                     (const uint32_t*)hist, ntiles, csum, gate);
  hipLaunchKernelGGL(k_col_scan<BINS>, dim3(BINS), dim3(256), 0, st, csum, nchunks, gate);
  hipLaunchKernelGGL(k_col_apply<BINS>, dim3((unsigned)nchunks), dim3(256), 0, st, hist, ntiles,
                     (const uint32_t*)csum, nchunks, gate);
}

// the columns of one sorted record at output position i (see EmitCols)
__device__ __forceinline__ void emit_cols(const EmitCols& E, int64_t m, int64_t i,
                                          const uint4& r) {
  const BuildPlan& P = *E.plan;
  const int64_t te = P.wide ? E.t_in[r.y] : P.tmin + (int64_t)r.w;
  E.key[i] = (int32_t)r.x;
  E.other[i] = (int32_t)r.z;
  E.t[i] = te;
  E.eid[i] = (int32_t)r.y;
  if (E.rec) E.rec[i] = make_uint4(r.z, r.y, (uint32_t)te, (uint32_t)(te >> 32));
  if (E.skip && (i & 15) == 0) {
    const int64_t n1 = skip_level_len(m, 1), n2 = skip_level_len(m, 2);
    E.skip[i >> 4] = te;
    if ((i & 255) == 0) E.skip[n1 + (i >> 8)] = te;
    if ((i & 4095) == 0) E.skip[n1 + n2 + (i >> 12)] = te;
  }
}

template <int ITEMS, int BINS, bool EMIT = false, bool LOOP = false>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(RecPass R, int64_t m,
                                                              const uint32_t* __restrict__ hist) {
  // Each wavefront owns a contiguous quarter of the tile and ranks its keys
  // in order with ballots (no block barrier inside); one block-wide pass then
  // offsets every wavefront's digit counts by those of the wavefronts before
  // it, which keeps the pass stable.
  static_assert(BINS == 256 || BINS == 512, "8- or 9-bit digits");
  constexpr int kTile = kSortBlock * ITEMS;
  constexpr int kWaves = kSortBlock / kWave;
  constexpr int kSub = kWave * ITEMS;  // entries per wavefront
  constexpr int kDig = BINS / kSortBlock;
  constexpr int kBits = BINS == 512 ? 9 : 8;
  static_assert(2 * kTile < 65536, "16-bit tile positions");
  const PassCfg c = resolve(R);
  if (!c.active) return;
  const int shift = c.shift, dbits = c.dbits;
  const uint32_t mask = (1u << dbits) - 1u;
  // s_base[d]: global position of digit d's run minus its start in the tile
  // s_pos[w][d]: wavefront w's running count of digit d, then the position
  //              in the tile of w's first key of digit d (16 bits suffice)
  __shared__ uint32_t s_base[BINS];
  __shared__ uint16_t s_pos[kWaves][BINS];
  __shared__ uint32_t s_wsum[kDig][kWaves];
  __shared__ uint4 s_key[kTile];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // One tile per block (the grid is the tile count), or with LOOP several
  // when the grid is smaller (a multiple of 8 blocks then, for the passes
  // that are usually idle).  XCD-aware tile order: workgroups are dealt to the XCDs round
  // robin (block b to XCD b mod 8), and each XCD has its own L2.
  // Neighbouring tiles write neighbouring pieces of every digit run, so each
  // XCD takes a contiguous range of tiles: partial cache lines then meet in
  // one L2 instead of being written back piecewise from several.
  const uint32_t nb = LOOP ? (uint32_t)((m + kTile - 1) / kTile) : gridDim.x;
  for (uint32_t vt = blockIdx.x; vt < nb; vt += gridDim.x) {
    const uint32_t xcd = vt % kXcds, slot = vt / kXcds;
    const uint32_t q = nb / kXcds, rem = nb % kXcds;
    const uint32_t tile = xcd * q + (xcd < rem ? xcd : rem) + slot;
    const int64_t start = (int64_t)tile * kTile;
    const int len = (int)((m - start) < kTile ? (m - start) : kTile);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

    uint32_t gbase[kDig];  // loaded now, used after the ranking
#pragma unroll
    for (int j = 0; j < kDig; ++j) gbase[j] = hist[(int64_t)tile * BINS + j * kSortBlock + tid];
#pragma unroll
    for (int w = 0; w < kWaves; ++w)
#pragma unroll
      for (int j = 0; j < kDig; ++j) s_pos[w][j * kSortBlock + tid] = 0;
    __syncthreads();

    uint4 key[ITEMS];
    uint32_t rank[ITEMS];  // rank among the wavefront's keys of the same digit
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int idx = wave * kSub + r * kWave + lane;
      const bool valid = idx < len;
      key[r] = valid ? load_rec(c, R.ec, start + idx) : uint4{};
      const uint32_t d = (key[r].x >> shift) & mask;
      uint64_t vb = __ballot(valid);
      uint64_t peers = valid ? vb : ~vb;
#pragma unroll
      for (int b = 0; b < kBits; ++b) {
        if (b < dbits) {  // uniform: the digit has dbits bits
          const bool bit = (d >> b) & 1u;
          const uint64_t bb = __ballot(bit);
          peers &= bit ? bb : ~bb;
        }
      }
      const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
      // read the running count before the leader of each digit group adds to it
      const uint32_t run = valid ? (uint32_t)s_pos[wave][d] : 0u;
      rank[r] = run + below;
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0) s_pos[wave][d] = (uint16_t)(run + (uint32_t)__popcll(peers));
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // thread tid owns digits tid, tid + 256, ...: the tile-local start of each
    // wavefront's run of that digit, digits in increasing order
    {
      uint32_t carry = 0;  // keys of the digit groups below
#pragma unroll
      for (int j = 0; j < kDig; ++j) {
        const int d = j * kSortBlock + tid;
        uint32_t cw[kWaves], tot = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          cw[w] = s_pos[w][d];
          tot += cw[w];
        }
        const uint32_t inc = wave_inclusive_scan(tot);
        if (lane == 63) s_wsum[j][wave] = inc;
        __syncthreads();
        uint32_t off = carry + inc - tot, group = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          off += w < wave ? s_wsum[j][w] : 0u;
          group += s_wsum[j][w];
        }
        carry += group;
        s_base[d] = gbase[j] - off;  // modulo 2^32; the sum below is exact
        uint32_t p = off;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          s_pos[w][d] = (uint16_t)p;
          p += cw[w];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
      const int idx = wave * kSub + r * kWave + lane;
      if (idx < len) {
        const uint32_t d = (key[r].x >> shift) & mask;
        s_key[(uint32_t)s_pos[wave][d] + rank[r]] = key[r];
      }
    }
    __syncthreads();
    const bool cols = EMIT && R.E.plan->bad == 0;
    for (int i = tid; i < len; i += kSortBlock) {
      const uint4 k = s_key[i];
      const uint32_t d = (k.x >> shift) & mask;
      const int64_t gpos = (int64_t)(s_base[d] + (uint32_t)i);
      // the last pass of a sort can re-key the records for the next sort, or
      // write the graph's columns instead of the records
      if (EMIT) {
        if (cols) emit_cols(R.E, m, gpos, k);
      } else {
        c.out[gpos] = rec_xform(k, c.xf1);
      }
      if (c.out2) c.out2[gpos] = rec_xform(k, c.xf2);
    }
    if (!LOOP) break;
    __syncthreads();  // the next tile reuses the LDS
  }
}

// One host-planned pass with BINS-entry digit histograms.
template <int ITEMS, int BINS>
void radix_pass(const RecPass& R, bool emit, int64_t m, int64_t ntiles, uint32_t* hist,
                uint32_t* part, hipStream_t st) {
  hipLaunchKernelGGL((k_radix_hist<ITEMS, BINS>), dim3((unsigned)ntiles), dim3(kSortBlock), 0,
                     st, R, m, hist);
  col_scan<BINS>(hist, ntiles, part, PassGate{nullptr, 0}, st);
  TimedLaunch tl("k_radix_scatter", st);
  if (emit)
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, BINS, true>), dim3((unsigned)ntiles),
                       dim3(kSortBlock), 0, st, R, m, (const uint32_t*)hist);
  else
    hipLaunchKernelGGL((k_radix_scatter<ITEMS, BINS>), dim3((unsigned)ntiles), dim3(kSortBlock),
                       0, st, R, m, (const uint32_t*)hist);
}

// Host-planned stable sort of m records by the low `bits` bits of their
// first word (a vertex id), ping-ponging between k0 and k1; returns 0 if the
// result is in k0, 1 if in k1, -1 if the scan scratch is too small (nothing
// enqueued then).  The result is re-keyed by xf1, and if `extra` is given a
// second copy re-keyed by xf2 goes there.  With `emit` the last pass writes
// the columns *emit instead of the sorted records (returns 2 then; with no
// pass at all the caller emits from k0).  With `in0` the first pass reads
// the records from there, re-keyed by xf_in as it loads them, and in0 is
// left as it was; with `ic` it reads them from the in-list columns (the
// caller passes ic only when the sort has a pass).  Digits are at most 8 bits wide,
// or at most 9 where that saves a pass (9, 17-18 and 25-27 bits: a 26-bit
// vertex id takes 8 + 9 + 9 instead of 6 + 6 + 7 + 7); a 9-bit pass moves
// twice the histogram rows, a few percent of the records' bytes.
template <int ITEMS>
int radix_sort(uint4* k0, uint4* k1, int64_t m, int bits, uint32_t* hist, uint32_t* part,
               size_t part_elems, hipStream_t st, int xf1 = RX_NONE, uint4* extra = nullptr,
               int xf2 = RX_NONE, const EmitCols* emit = nullptr, const uint4* in0 = nullptr,
               int xf_in = RX_NONE, const InCols* ic = nullptr) {
  if (m <= 0) return 0;
  constexpr int kTile = kSortBlock * ITEMS;
  const int64_t ntiles = (m + kTile - 1) / kTile;
  const int n8 = (bits + 7) / 8, n9 = (bits + 8) / 9;
  const bool nine = n9 < n8;
  const int npass = nine ? n9 : n8;
  if (part_elems < col_scan_scratch_elems(ntiles, nine ? 512 : 256)) return -1;
  int cur = 0;
  if (npass == 0 && (xf1 != RX_NONE || extra || in0))
    hipLaunchKernelGGL(k_rec_xform, dim3(blocks_for(m, 256)), dim3(256), 0, st,
                       in0 ? in0 : (const uint4*)k0, in0 ? xf_in : (int)RX_NONE, k0, m, xf1,
                       extra, xf2);
  int shift = 0;
  for (int p = 0; p < npass; ++p) {
    const bool last = p + 1 == npass;
    RecPass R{};
    R.plan = nullptr;
    R.in = p == 0 && in0 ? in0 : (cur ? k1 : k0);
    R.xfin = p == 0 && in0 ? xf_in : (int)RX_NONE;
    if (p == 0 && ic) R.ic = *ic;
    R.out = cur ? k0 : k1;
    // with 9-bit digits the narrow one goes last: the last pass writes the
    // longest runs, and an 8-bit pass takes 256-entry rows
    int sh, db;
    digit_plan(bits, npass, nine ? npass - 1 - p : p, &sh, &db);
    R.shift = shift;
    R.dbits = db;
    shift += db;
    R.xf1 = last ? xf1 : (int)RX_NONE;
    R.out2 = last ? extra : nullptr;
    R.xf2 = last ? xf2 : (int)RX_NONE;
    const bool em = last && emit;
    if (em) R.E = *emit;
    if (db > 8)
      radix_pass<ITEMS, 512>(R, em, m, ntiles, hist, part, st);
    else
      radix_pass<ITEMS, 256>(R, em, m, ntiles, hist, part, st);
    cur ^= 1;
  }
  return npass > 0 && emit ? 2 : cur;
}

// The time sort: kTimePasses launched passes planned on the device (see
// BuildPlan).  It reads the edge columns and leaves the time-ordered records
// re-keyed by xf1 in buf[0] and, if out2 is given, by xf2 in out2.  Its
// first pass takes its digit counts from the validation (k_fold_hist).
template <int ITEMS>
bool time_sort(const BuildPlan* plan, const EdgeCols& ec, uint4* b0, uint4* b1, int64_t m,
               uint32_t* hist, uint32_t* part, size_t part_elems, hipStream_t st, int xf1,
               uint4* out2, int xf2) {
  constexpr int kTile = kSortBlock * ITEMS;
  const int64_t ntiles = (m + kTile - 1) / kTile;
  if (part_elems < col_scan_scratch_elems(ntiles, 256)) return false;
  hipLaunchKernelGGL(k_rec_init, dim3(blocks_for(m, 256) < 2048 ? blocks_for(m, 256) : 2048),
                     dim3(256), 0, st, ec, m, plan, b0,
                     xf1, out2, xf2);
  for (int p = 0; p < kTimePasses; ++p) {
    RecPass R{};
    R.plan = plan;
    R.pass = p;
    R.buf[0] = b0;
    R.buf[1] = b1;
    R.xf1 = xf1;
    R.out2 = out2;
    R.xf2 = xf2;
    R.ec = ec;
    // the high-word passes work only for time ranges wider than 32 bits:
    // their launches take up to eight tiles per block, so that idle ones
    // cost a few microseconds
    const int64_t hb = ((ntiles + 63) / 64) * 8;
    const unsigned grid = (unsigned)(p >= 4 && hb < ntiles ? hb : ntiles);
    // pass 0 takes its counts from the validation's (k_fold_hist)
    if (p == 0)
      hipLaunchKernelGGL(k_fold_hist, dim3((unsigned)(ntiles < 2048 ? ntiles : 2048)), dim3(256),
                         0, st, hist, ntiles, plan);
    else
      hipLaunchKernelGGL((k_radix_hist<ITEMS, 256>), dim3(grid), dim3(kSortBlock), 0, st, R, m,
                         hist);
    col_scan<256>(hist, ntiles, part, PassGate{plan, p}, st);
    if (p >= 4)
      hipLaunchKernelGGL((k_radix_scatter<ITEMS, 256, false, true>), dim3(grid), dim3(kSortBlock),
                         0, st, R, m, (const uint32_t*)hist);
    else
      hipLaunchKernelGGL((k_radix_scatter<ITEMS, 256>), dim3(grid), dim3(kSortBlock), 0, st, R,
                         m, (const uint32_t*)hist);
  }
  return true;
}

// -------------------------------------------------------- columns/offsets ---
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
// probes and most runs (a single edge) one -- and inserts {key, start, end}:
// a compare-and-swap claims the slot's key, one 8-byte store fills the run.
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
      *reinterpret_cast<uint2*>(&tab[h].start) = make_uint2((uint32_t)i, (uint32_t)hi);
      return;
    }
    h = (h + 1) & mask;
  }
}

int pair_hash_log2(int64_t m) {
  int lg = 4;
  while (((int64_t)1 << lg) < m + m / 4 + 1) ++lg;
  return lg;
}

// sorted records (key, eid, other, t - t_min) -> columns of one order, for a
// graph of a single vertex (its vertex sorts have no pass whose last one
// would write the columns).  The time is t_min + the record's time word, or,
// when the range is wider than 32 bits, read back from the input by edge id.
// With `off` (n + 1 entries), also the CSR offsets of the sorted keys:
// off[v] = first position whose key is >= v, written by the thread of the
// position where the key passes v (grid of m + 1 threads).  With `skip`
// (the pair index), also the sampled levels skip_k[i] = t[16^k i], k = 1..3,
// from the times this pass writes anyway.  A rejected input (bad vertex id or
// time) writes nothing.
__global__ __launch_bounds__(256) void k_emit(const uint4* __restrict__ in, int64_t m,
                                              const BuildPlan* __restrict__ plan,
                                              const int64_t* __restrict__ t_in,
                                              int32_t* __restrict__ key_col,
                                              int32_t* __restrict__ other_col,
                                              int64_t* __restrict__ t_col,
                                              int32_t* __restrict__ eid_col,
                                              uint4* __restrict__ rec, int32_t n,
                                              uint32_t* __restrict__ off,
                                              int64_t* __restrict__ skip) {
  if (plan->bad) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    const uint4 r = in[i];
    key_col[i] = (int32_t)r.x;
    const int64_t te = plan->wide ? t_in[r.y] : plan->tmin + (int64_t)r.w;
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

// CSR offsets from a sorted key column: off[v] = first position whose key is
// at least v, for v in [0, n].  Each thread takes kOffItems consecutive
// positions (two 16-byte loads where the column allows), so the launch has
// an eighth of the blocks a thread per position would need.
constexpr int kOffItems = 8;
__global__ __launch_bounds__(256) void k_offsets(const int32_t* __restrict__ key, int64_t m,
                                                 const BuildPlan* __restrict__ plan, int32_t n,
                                                 uint32_t* __restrict__ off) {
  if (plan->bad) return;
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kOffItems;
  if (i0 > m) return;
  int32_t k[kOffItems];
  if (i0 + kOffItems <= m && ((uintptr_t)key & 15) == 0) {
    const int4 a = *(const int4*)(key + i0), b = *(const int4*)(key + i0 + 4);
    k[0] = a.x, k[1] = a.y, k[2] = a.z, k[3] = a.w, k[4] = b.x, k[5] = b.y, k[6] = b.z,
    k[7] = b.w;
  } else {
#pragma unroll
    for (int j = 0; j < kOffItems; ++j) k[j] = i0 + j < m ? key[i0 + j] : n;
  }
  int64_t prev = i0 == 0 ? -1 : (int64_t)key[i0 - 1];
#pragma unroll
  for (int j = 0; j < kOffItems; ++j) {
    const int64_t i = i0 + j;
    if (i <= m) {
      const int64_t cur = i == m ? (int64_t)n : (int64_t)k[j];
      for (int64_t v = prev + 1; v <= cur; ++v) off[v] = (uint32_t)i;
      prev = cur;
    }
  }
}

// the validation word and the time range of the plan, for tc_graph
__global__ void k_trange(const BuildPlan* __restrict__ plan, int64_t* __restrict__ tr) {
  if (threadIdx.x == 0) {
    tr[0] = plan->tmin;
    tr[1] = plan->tmax;
  }
}

// --------------------------------------------------------------- layout ----
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct GraphLayout {
  size_t out_off, in_off, out_src, out_dst, out_eid, out_t, in_src, in_eid, in_dst, in_t,
      pair_dst, out_rec, in_rec, pair_eid, pair_t, pair_hash, pair_skip, status, tminmax, trange,
      plan, hist, part, part_elems, rr[4], total;
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
  L.status = take(16);
  L.tminmax = take(16);
  L.trange = take(16);
  L.plan = take(sizeof(BuildPlan));
  // sort scratch: four 16-byte-record buffers
  for (int b = 0; b < 4; ++b) L.rr[b] = take((M + 1) * 16);
  L.hist = take((size_t)kMaxBins * ntiles * 4);
  // scan scratch of the histogram column scan
  L.part_elems = col_scan_scratch_elems(ntiles, kMaxBins);
  L.part = take(L.part_elems * 4);
  L.total = o;
  return L;
}

size_t graph_workspace_bytes(int32_t n, int64_t m) { return graph_layout(n, m).total; }

static int bitlen(uint64_t x) { return x ? 64 - __builtin_clzll(x) : 0; }

// The pair-run table from the pair index's sorted src keys.
static void clear_pair_hash(const tc_graph* g, hipStream_t st) {
  const int64_t cap = (int64_t)1 << g->pair_hash_log2;
  hipLaunchKernelGGL(k_hash_clear, dim3(blocks_for(cap, 256)), dim3(256), 0, st,
                     (PairSlot*)g->pair_hash, cap);
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
  g->t_range = (int64_t*)(base + L.trange);
  g->pair_hash = (void*)(base + L.pair_hash);
  g->pair_hash_log2 = pair_hash_log2(m);
  g->pair_skip = (int64_t*)(base + L.pair_skip);
  g->out_rec = (void*)(base + L.out_rec);
  g->in_rec = (void*)(base + L.in_rec);
  uint64_t* tminmax = (uint64_t*)(base + L.tminmax);
  BuildPlan* plan = (BuildPlan*)(base + L.plan);
  uint32_t* hist = (uint32_t*)(base + L.hist);
  uint32_t* part = (uint32_t*)(base + L.part);
  const size_t pe = L.part_elems;

  // validation and the sort plan, on the device
  hipLaunchKernelGGL(k_init_build, dim3(1), dim3(64), 0, st, g->status, tminmax);
  if (m > 0) {
    const int64_t ntiles = (m + kRecTile - 1) / kRecTile;
    hipLaunchKernelGGL(k_validate, dim3((unsigned)(ntiles < 1024 ? ntiles : 1024)),
                       dim3(kSortBlock), 0, st, src, dst, t, m, n, g->status, tminmax, hist);
  }
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, st, (const uint32_t*)g->status,
                     (const uint64_t*)tminmax, m, plan);
  hipLaunchKernelGGL(k_trange, dim3(1), dim3(64), 0, st, (const BuildPlan*)plan, g->t_range);
  clear_pair_hash(g, st);
  if (m == 0) {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->out_off, (int64_t)n + 1, 0u);
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for((int64_t)n + 1, 256)), dim3(256), 0, st,
                       g->in_off, (int64_t)n + 1, 0u);
    if (hipGetLastError() != hipSuccess) return TC_E_HIP;
    return TC_OK;
  }
  const int vbits = bitlen((uint64_t)(n - 1));
  const unsigned eb = blocks_for(m, 256);
  uint4* rr[4];
  for (int b = 0; b < 4; ++b) rr[b] = (uint4*)(base + L.rr[b]);
  // 1. time order, ending in rr[0] re-keyed as the out-CSR input
  const EdgeCols ec{src, dst, t};
  if (!time_sort<kRecItems>(plan, ec, rr[0], rr[1], m, hist, part, pe, st, RX_OUT, nullptr,
                            RX_NONE))
    return TC_E_WORKSPACE;
  // A vertex sort of rr[from] (spare rr[tmp]) whose last pass writes the
  // columns E; with no pass (n = 1) the records are emitted from rr[from].
  // With `in0` >= 0 the sort reads rr[in0] (re-keyed by xf_in) and leaves it
  // as it was, ping-ponging between rr[from] and rr[tmp]; with `ic` its first
  // pass reads the in-list columns instead of rr[from].
  auto sort_emit = [&](int from, int tmp, const EmitCols& E, uint32_t* off, int extra = -1,
                       int xf2 = RX_NONE, int in0 = -1, int xf_in = RX_NONE,
                       const InCols* ic = nullptr) -> bool {
    const int w = radix_sort<kRecItems>(rr[from], rr[tmp], m, vbits, hist, part, pe, st,
                                        RX_NONE, extra < 0 ? (uint4*)nullptr : rr[extra], xf2,
                                        &E, in0 < 0 ? (const uint4*)nullptr : rr[in0], xf_in,
                                        ic);
    if (w < 0) return false;
    if (w != 2)
      hipLaunchKernelGGL(k_emit, dim3(blocks_for(m + 1, 256)), dim3(256), 0, st,
                         (const uint4*)rr[w ? tmp : from], m, (const BuildPlan*)plan, t, E.key,
                         E.other, E.t, E.eid, E.rec, n, off, E.skip);
    else if (off)
      hipLaunchKernelGGL(k_offsets, dim3(blocks_for((m + kOffItems) / kOffItems, 256)),
                         dim3(256), 0, st, (const int32_t*)E.key, m, (const BuildPlan*)plan, n,
                         off);
    return true;
  };
  // 2. in-CSR: the time order read from rr[0] with src and dst swapped
  //    ((src, eid, dst, t) -> (dst, eid, src, t)), stable by dst, written as
  //    the in-list columns.  With a single vertex (no pass) a copy of the
  //    records re-keyed for the pair index goes to rr[3] instead.
  const bool one = vbits == 0;
  if (!sort_emit(2, 1,
                 EmitCols{plan, t, g->in_dst, g->in_src, g->in_t, g->in_eid, (uint4*)g->in_rec,
                          nullptr},
                 g->in_off, one ? 3 : -1, RX_PAIR, 0, RX_PAIR))
    return TC_E_WORKSPACE;
  // 3. pair index: the in-order (dst, t, eid), read from the in-list
  //    columns, stably by src; the pair sources go to the free buffer rr[2]
  int32_t* psrc = (int32_t*)rr[2];
  const InCols ic{(const uint4*)g->in_rec, g->in_dst, plan};
  if (!sort_emit(3, 1,
                 EmitCols{plan, t, psrc, g->pair_dst, g->pair_t, g->pair_eid, nullptr,
                          g->pair_skip},
                 nullptr, -1, RX_NONE, -1, RX_NONE, one ? nullptr : &ic))
    return TC_E_WORKSPACE;
  // 4. the run table (its clear was enqueued first)
  hipLaunchKernelGGL(k_hash_insert, dim3(eb), dim3(256), 0, st, (const uint32_t*)psrc,
                     (const int32_t*)g->pair_dst, m, (PairSlot*)g->pair_hash, g->pair_hash_log2);
  // 5. out-CSR: stable by src, from the time order in rr[0]
  if (!sort_emit(0, 1,
                 EmitCols{plan, t, g->out_src, g->out_dst, g->out_t, g->out_eid,
                          (uint4*)g->out_rec, nullptr},
                 g->out_off))
    return TC_E_WORKSPACE;
  if (hipGetLastError() != hipSuccess) return TC_E_HIP;
  return TC_OK;
}

}  // namespace tc
