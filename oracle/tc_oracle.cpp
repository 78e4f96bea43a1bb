// CPU oracle for temporal 3-path sampling (TEACUPS, Pan et al., ICDM 2024).
//
// TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
// reference that the GPU library is checked against.  Only the tests, the
// smoke check and the CPU-baseline leg of the benchmark may load it; the
// product path never calls it.  It shares no code with the HIP library.
//
// What it computes, step by step in the paper's order:
//   * time-sorted in/out adjacency and per-pair lists (section III-A: edges
//     sorted by time, per-vertex in/out lists sorted by time; section III-B:
//     the lists L_{u,v}),
//   * Preprocess: per-edge window degrees by binary search and
//     w_e = d^-_u[t-delta, t] * d^+_v[t, t+delta] (Claim "count",
//     Algorithm Preprocess), or for another anchor class (section III) the
//     product of its two sides' degrees over their intervals, a side with no
//     edge (a wedge) counting 1; their running total as an exact integer CDF,
//   * Sample: pick e with probability w_e / W by searching the CDF, then a
//     uniform edge inside each side's window (Algorithm Sample),
//   * CheckMotif + ListCount (Algorithms CheckMotif and ListCount),
//   * Estimate: C_hat = (cnt / k) * W (Algorithm Estimate),
//   * a definition-level backtracking count of M-matches (Definition of an
//     M-match, section I-A) and an exhaustive sum of CheckMotif over every
//     delta-centred 3-path (proof of Claim "est": sum_P C_P = C).
//
// Readings where the paper is silent or inconsistent (all listed in the
// design notes):
//   * windows are closed, [t-delta, t] and [t, t+delta], as in Claim "count"
//     and its proof; the match itself needs strict t1 < t2 < t3 (the order
//     condition of a match is an "iff", so ties are not matches); CheckMotif
//     therefore also rejects non-increasing times,
//   * equal timestamps inside a list are ordered by edge id (input index),
//   * the sampling distribution p_e = w_e / W is realised exactly as an
//     integer CDF S with a uniform integer r in [0, W),
//   * ListCount counts strictly increasing chains (ties are not matches) and
//     walks each pair of neighbouring lists with one forward pointer, which
//     is what its linear-time claim needs,
//   * the anchor of a motif holds its earliest edge (Algorithm Estimate):
//     a 3-path over four distinct vertices, or for three vertices a wedge
//     whose centre is the earliest edge; ties between candidates go to the
//     lexicographically smallest sorted ranks, then the smallest centre
//     rank, then the smallest rank of the edge at u,
//   * a non-anchor edge of rank r is looked for after the anchor time ranked
//     just below r and before the one ranked just above it, or up to the
//     first anchor time + delta (CheckMotif's list bounds), so for the
//     spine motifs every list is the pair's times in (t3, t1 + delta],
//   * exhaustive mode visits CDF rank r as the anchor p = UB(S, r) - 1 with
//     j1 = (r - S[p]) div b[p] and j3 = (r - S[p]) mod b[p].
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
// random numbers: as easy as 1, 2, 3", SC 2011) with counter
// (i mod 2^32, i div 2^32, attempt, stream) and key (seed mod 2^32,
// seed div 2^32).  Attempt n of sample i yields words x0..x3: x0|x1<<32 is
// the 64-bit draw for r, x2 for j1 and x3 for j3.  Each variable takes the
// first attempt whose word passes Lemire's rejection test ("Fast random
// integer generation in an interval", ACM TOMACS 2019), which makes every
// value exactly uniform.
#include <algorithm>
#include <parallel/algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>
#include <omp.h>

typedef unsigned __int128 u128;

namespace {

const uint64_t kU64Max = ~0ull;
const int64_t kTLimit = (int64_t)1 << 62;
const int kMaxAttempts = 1024;

enum { OR_OK = 0, OR_RANGE = 1, OR_OVERFLOW = 2, OR_RNG = 4, OR_ARG = 8 };

// An anchor class (section III: the 16 classes <alpha_1, alpha_3, beta_1,
// beta_3> of delta-centred 3-paths, and the wedges of the 3-vertex case):
// for the side at the centre edge's source u (side 1, edge e1) and the side
// at its destination v (side 3, edge e3), whether the side has an edge, whether
// that edge is an in-edge (-) or an out-edge (+) of u (resp. v), and whether
// it comes before the centre edge (window [t - delta, t]) or after it
// ([t, t + delta]).  Stored as 4 bytes {mode1, after1, mode3, after3}; bit 1
// of an `after` byte (2) opens the window at the centre time: [t - delta, t)
// or (t, t + delta].  A match's times increase strictly, so the open windows
// still hold every match's anchor (a variant of the closed windows of Claim
// "count", with a smaller W).
enum { SIDE_NONE = 0, SIDE_IN = 1, SIDE_OUT = 2 };
struct Class {
  int mode[2];   // side 1, side 3
  int after[2];
  int open[2];   // the window excludes the centre time
};
const Class kSpineClass = {{SIDE_IN, SIDE_OUT}, {0, 1}, {0, 0}};

bool parse_class(const uint8_t* c, Class* K) {
  if (!c) { *K = kSpineClass; return true; }
  for (int s = 0; s < 2; ++s) {
    K->mode[s] = c[2 * s];
    const int a = c[2 * s + 1];
    K->after[s] = a & 1;
    K->open[s] = (a >> 1) & 1;
    if (K->mode[s] > SIDE_OUT || a > 3) return false;
  }
  return K->mode[0] != SIDE_NONE || K->mode[1] != SIDE_NONE;
}

bool same_class(const Class& a, const Class& b) {
  for (int s = 0; s < 2; ++s) {
    if (a.mode[s] != b.mode[s]) return false;
    if (a.mode[s] != SIDE_NONE && a.after[s] != b.after[s]) return false;
  }
  return true;
}

// A motif with its anchor (Algorithm Estimate: an anchor path that holds
// the motif edge of time rank 0).  Edge i of the motif has rank i.
struct Motif {
  int nv, ne;
  int src[16], dst[16];
  Class cls;
  int aedge[3];   // motif edge of e1 (side 1), e2 (centre), e3 (side 3); -1 = no edge
  int na;         // anchor edges: 3 (a path) or 2 (a wedge)
  int order[3];   // anchor edges by increasing rank, as 0 = e1, 1 = e2, 2 = e3
  int slot[16];   // motif vertex -> position in phi = (x, u, v, y)
  int nl;         // non-anchor edges, in rank order
  int lslot_a[16], lslot_b[16], lseg[16];  // their pairs and segments
};

// The anchor of M (the choice the library makes too):
//  4 vertices: every (e1, e2, e3) of distinct motif edges that is a path
//    x - u - v - y over four distinct vertices, centre e2 = (u -> v) as
//    directed in the motif, holding rank 0; the one whose sorted ranks are
//    lexicographically smallest, then the smallest centre rank, then the
//    smallest e1 rank.
//  3 vertices: every (centre, side edge) pair of distinct motif edges over
//    three distinct vertices holding rank 0, the side edge meeting the
//    centre in one vertex; smallest sorted ranks, then smallest centre rank.
// Returns false when there is none (e.g. a 3-star).
bool compile_anchor(Motif* M) {
  const int ne = M->ne;
  int best[3] = {-1, -1, -1};
  long best_key = -1;
  auto touches = [&](int e, int a) { return M->src[e] == a || M->dst[e] == a; };
  auto other = [&](int e, int a) { return M->src[e] == a ? M->dst[e] : M->src[e]; };
  if (M->nv == 4) {
    for (int c = 0; c < ne; ++c) {
      const int U = M->src[c], V = M->dst[c];
      for (int e1 = 0; e1 < ne; ++e1) {
        if (e1 == c || !touches(e1, U) || touches(e1, V)) continue;
        const int X = other(e1, U);
        for (int e3 = 0; e3 < ne; ++e3) {
          if (e3 == c || e3 == e1 || !touches(e3, V) || touches(e3, U)) continue;
          const int Y = other(e3, V);
          if (Y == X) continue;
          if (c != 0 && e1 != 0 && e3 != 0) continue;
          int r[3] = {e1, c, e3};
          std::sort(r, r + 3);
          const long key = (((((long)r[0] * 16 + r[1]) * 16 + r[2]) * 16 + c) * 16 + e1);
          if (best_key < 0 || key < best_key) {
            best_key = key;
            best[0] = e1; best[1] = c; best[2] = e3;
          }
        }
      }
    }
  } else if (M->nv == 3) {
    for (int c = 0; c < ne; ++c) {
      const int U = M->src[c], V = M->dst[c];
      for (int e = 0; e < ne; ++e) {
        if (e == c || touches(e, U) == touches(e, V)) continue;  // meets exactly one end
        if (c != 0 && e != 0) continue;
        const int lo = std::min(c, e), hi = std::max(c, e);
        const long key = ((long)lo * 16 + hi) * 16 + c;
        if (best_key < 0 || key < best_key) {
          best_key = key;
          best[1] = c;
          best[0] = touches(e, U) ? e : -1;
          best[2] = touches(e, U) ? -1 : e;
        }
      }
    }
  }
  if (best_key < 0) return false;
  for (int i = 0; i < 3; ++i) M->aedge[i] = best[i];
  const int c = best[1], U = M->src[c], V = M->dst[c];
  for (int i = 0; i < 16; ++i) M->slot[i] = -1;
  M->slot[U] = 1;
  M->slot[V] = 2;
  M->na = 1;
  for (int s = 0; s < 2; ++s) {
    const int e = best[2 * s];
    const int at = s == 0 ? U : V;
    if (e < 0) {
      M->cls.mode[s] = SIDE_NONE;
      M->cls.after[s] = 0;
      continue;
    }
    ++M->na;
    M->cls.mode[s] = (M->dst[e] == at) ? SIDE_IN : SIDE_OUT;
    M->cls.after[s] = e > c ? 1 : 0;
    M->slot[other(e, at)] = s == 0 ? 0 : 3;
  }
  for (int v = 0; v < M->nv; ++v)
    if (M->slot[v] < 0) return false;  // a vertex the anchor does not reach
  // anchor edges by rank
  int k = 0;
  for (int r = 0; r < ne; ++r)
    for (int i = 0; i < 3; ++i)
      if (best[i] == r) M->order[k++] = i;
  // the other edges: lists, each bounded by the anchor edges around it
  M->nl = 0;
  for (int r = 0; r < ne; ++r) {
    if (r == best[0] || r == best[1] || r == best[2]) continue;
    int below = 0;
    for (int i = 0; i < 3; ++i)
      if (best[i] >= 0 && best[i] < r) ++below;
    M->lslot_a[M->nl] = M->slot[M->src[r]];
    M->lslot_b[M->nl] = M->slot[M->dst[r]];
    M->lseg[M->nl] = below - 1;
    ++M->nl;
  }
  return true;
}

bool parse_motif(const uint8_t* d, Motif* M) {
  M->nv = d[0];
  M->ne = d[1];
  if (M->nv < 3 || M->nv > 4 || M->ne < 2 || M->ne > 16) return false;
  for (int i = 0; i < M->ne; ++i) {
    M->src[i] = d[2 + i];
    M->dst[i] = d[18 + i];
    if (M->src[i] >= M->nv || M->dst[i] >= M->nv || M->src[i] == M->dst[i]) return false;
  }
  return compile_anchor(M);
}

struct Graph {
  int32_t n;
  int64_t m;
  std::vector<int32_t> src, dst;
  std::vector<int64_t> t;
  // canonical orders (vectors of edge ids)
  std::vector<int32_t> out_ord, in_ord, pair_ord;
  std::vector<uint32_t> out_off, in_off;  // [n+1]
  // gathered per-order columns
  std::vector<int64_t> out_t, in_t, pair_t;
  std::vector<int32_t> out_dst, in_src, pair_dst;
};

// ---- Philox4x32-10 (SC'11 definition) --------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void draw_block(uint64_t seed, uint32_t stream, uint64_t i, uint32_t attempt, uint32_t x[4]) {
  uint32_t ctr[4] = {(uint32_t)i, (uint32_t)(i >> 32), attempt, stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  philox4x32_10(ctr, key, x);
}

// Lemire: the draw x maps to floor(x * s / 2^b); it is rejected when the low
// b bits of x * s fall below (2^b - s) mod s, which leaves exactly
// floor(2^b / s) accepted draws per output value.
bool lemire64(uint64_t x, uint64_t s, uint64_t* out) {
  u128 p = (u128)x * s;
  uint64_t lo = (uint64_t)p;
  uint64_t thresh = (uint64_t)((((u128)1 << 64) - s) % s);
  if (lo < thresh) return false;
  *out = (uint64_t)(p >> 64);
  return true;
}

bool lemire32(uint32_t x, uint32_t s, uint32_t* out) {
  uint64_t p = (uint64_t)x * s;
  uint32_t lo = (uint32_t)p;
  uint32_t thresh = (uint32_t)((((uint64_t)1 << 32) - s) % s);
  if (lo < thresh) return false;
  *out = (uint32_t)(p >> 32);
  return true;
}

// ---- adjacency build --------------------------------------------------------
// Stable sort of edge ids; with several threads libstdc++'s parallel stable
// sort (a multiway merge sort), whose result is the same unique stable order.
template <typename Less>
void stable_sort_ids(std::vector<int32_t>& v, Less less, int nthreads) {
  if (nthreads > 1 && v.size() > 100000) {
    omp_set_num_threads(nthreads);
    __gnu_parallel::stable_sort(v.begin(), v.end(), less);
  } else {
    std::stable_sort(v.begin(), v.end(), less);
  }
}

int build(Graph& G, int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
          const int64_t* t, int nthreads) {
  G.n = n;
  G.m = m;
  for (int64_t e = 0; e < m; ++e) {
    if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n) return OR_RANGE;
    if (t[e] >= kTLimit || t[e] <= -kTLimit) return OR_RANGE;  // |t| < 2^62
  }
  G.src.assign(src, src + m);
  G.dst.assign(dst, dst + m);
  G.t.assign(t, t + m);
  std::vector<int32_t> ids(m);
  std::iota(ids.begin(), ids.end(), 0);
  // out lists: by (src, t, eid)
  G.out_ord = ids;
  stable_sort_ids(G.out_ord, [&](int32_t a, int32_t b) {
    if (G.src[a] != G.src[b]) return G.src[a] < G.src[b];
    return G.t[a] < G.t[b];
  }, nthreads);
  // in lists: by (dst, t, eid)
  G.in_ord = ids;
  stable_sort_ids(G.in_ord, [&](int32_t a, int32_t b) {
    if (G.dst[a] != G.dst[b]) return G.dst[a] < G.dst[b];
    return G.t[a] < G.t[b];
  }, nthreads);
  // pair lists L_{u,v}: by (src, dst, t, eid)
  G.pair_ord = ids;
  stable_sort_ids(G.pair_ord, [&](int32_t a, int32_t b) {
    if (G.src[a] != G.src[b]) return G.src[a] < G.src[b];
    if (G.dst[a] != G.dst[b]) return G.dst[a] < G.dst[b];
    return G.t[a] < G.t[b];
  }, nthreads);
  G.out_off.assign(n + 1, 0);
  G.in_off.assign(n + 1, 0);
  for (int64_t e = 0; e < m; ++e) {
    G.out_off[src[e] + 1]++;
    G.in_off[dst[e] + 1]++;
  }
  for (int32_t v = 0; v < n; ++v) {
    G.out_off[v + 1] += G.out_off[v];
    G.in_off[v + 1] += G.in_off[v];
  }
  G.out_t.resize(m); G.in_t.resize(m); G.pair_t.resize(m);
  G.out_dst.resize(m); G.in_src.resize(m); G.pair_dst.resize(m);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t p = 0; p < m; ++p) {
    G.out_t[p] = G.t[G.out_ord[p]];
    G.out_dst[p] = G.dst[G.out_ord[p]];
    G.in_t[p] = G.t[G.in_ord[p]];
    G.in_src[p] = G.src[G.in_ord[p]];
    G.pair_t[p] = G.t[G.pair_ord[p]];
    G.pair_dst[p] = G.dst[G.pair_ord[p]];
  }
  return OR_OK;
}

// Edges (a -> b) with time in the half-open interval (lo_t, hi_t]: returns
// [first, last) positions in the pair order.
void pair_window(const Graph& G, int32_t a, int32_t b, int64_t lo_t, int64_t hi_t,
                 int64_t* first, int64_t* last) {
  auto beg = G.pair_dst.begin() + G.out_off[a];
  auto end = G.pair_dst.begin() + G.out_off[a + 1];
  auto run = std::equal_range(beg, end, b);
  int64_t r0 = run.first - G.pair_dst.begin();
  int64_t r1 = run.second - G.pair_dst.begin();
  auto tb = G.pair_t.begin();
  *first = std::upper_bound(tb + r0, tb + r1, lo_t) - tb;
  *last = std::upper_bound(tb + r0, tb + r1, hi_t) - tb;
  if (*last < *first) *last = *first;
}

// ListCount: number of chains l_1 < l_2 < ... < l_l with l_r drawn from the
// sorted list L_r.  cnt_1 is all ones; cnt_r[i] sums cnt_{r-1}[j] over the
// entries of L_{r-1} strictly before L_r[i], found with one pointer that only
// moves forward.  Counts are kept in 128 bits; returns false only if a
// level's total reaches 2^128.
bool add_u128(u128* acc, u128 v) {
  const u128 r = *acc + v;
  const bool ok = r >= *acc;
  *acc = r;
  return ok;
}

bool list_count(const std::vector<std::vector<int64_t>>& L, u128* X) {
  size_t l = L.size();
  if (l == 0) { *X = 1; return true; }
  std::vector<u128> prev(L[0].size(), 1), cur;
  bool ok = true;
  for (size_t r = 1; r < l; ++r) {
    cur.assign(L[r].size(), 0);
    size_t j = 0;
    u128 run = 0;
    for (size_t i = 0; i < L[r].size(); ++i) {
      while (j < L[r - 1].size() && L[r - 1][j] < L[r][i]) {
        ok = add_u128(&run, prev[j]) && ok;
        ++j;
      }
      cur[i] = run;
    }
    u128 total = 0;
    for (u128 c : cur) ok = add_u128(&total, c) && ok;
    prev.swap(cur);
  }
  u128 s = 0;
  for (u128 c : prev) ok = add_u128(&s, c) && ok;
  *X = s;
  return ok;
}

// A per-sample count as one 64-bit word: saturated at 2^64 - 1.
uint64_t sat64(u128 x) { return (x >> 64) ? kU64Max : (uint64_t)x; }

// The edge of an anchor side at the centre edge's endpoint `at` (u for
// side 1, v for side 3): position `pos` of the in-CSR or the out-CSR.
int32_t side_edge(const Graph& G, int mode, int64_t pos) {
  return mode == SIDE_IN ? G.in_ord[pos] : G.out_ord[pos];
}

// CheckMotif (Algorithm CheckMotif, generalised to the anchor classes) for
// the anchor (e1, e2, e3) given by edge ids (-1 for an absent side): the
// number of M-matches in which these edges are the images of the motif's
// anchor edges.  phi = (x, u, v, y) with e2 = (u -> v); x is e1's other end
// at u, y is e3's other end at v.  The anchor must span distinct vertices,
// its times must strictly increase in rank order and lie within delta of
// the first; each other motif edge of rank r is then looked for among the
// edges of its pair with time after the anchor edge ranked just below r and
// before the one ranked just above it (or at most the first time + delta),
// and ListCount counts the strictly increasing chains through those lists.
int check_motif(const Graph& G, const Motif& M, int64_t delta, int32_t e1, int32_t e2,
                int32_t e3, u128* X) {
  *X = 0;
  const int32_t u = G.src[e2], v = G.dst[e2];
  int32_t phi[4] = {-1, u, v, -1};
  const int32_t ae[3] = {e1, e2, e3};
  for (int s = 0; s < 2; ++s) {
    const int32_t e = ae[2 * s];
    const int mode = M.cls.mode[s];
    if ((mode == SIDE_NONE) != (e < 0)) return OR_ARG;
    if (mode == SIDE_NONE) continue;
    const int32_t at = s == 0 ? u : v;
    if (mode == SIDE_IN && G.dst[e] != at) return OR_ARG;
    if (mode == SIDE_OUT && G.src[e] != at) return OR_ARG;
    phi[s == 0 ? 0 : 3] = mode == SIDE_IN ? G.src[e] : G.dst[e];
  }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (phi[i] >= 0 && phi[i] == phi[j]) return OR_OK;
  int64_t T[3];
  for (int k = 0; k < M.na; ++k) T[k] = G.t[ae[M.order[k]]];
  for (int k = 1; k < M.na; ++k)
    if (!(T[k - 1] < T[k])) return OR_OK;
  if (T[M.na - 1] - T[0] > delta) return OR_OK;
  std::vector<std::vector<int64_t>> L;
  for (int i = 0; i < M.nl; ++i) {
    const int sg = M.lseg[i];
    const int64_t lo = T[sg];
    const int64_t hi = sg + 1 < M.na ? T[sg + 1] - 1 : T[0] + delta;
    int64_t f, l;
    pair_window(G, phi[M.lslot_a[i]], phi[M.lslot_b[i]], lo, hi, &f, &l);
    L.emplace_back(G.pair_t.begin() + f, G.pair_t.begin() + l);
  }
  if (!list_count(L, X)) return OR_OVERFLOW;
  return OR_OK;
}

// Preprocess for an anchor class: per scan position p (out-CSR order, centre
// edge (u, v, t)) the window of each side -- the in- or out-edges of u
// (side 1) resp. v (side 3) with time in [t - delta, t] or [t, t + delta],
// closed -- as its first position in the in- or out-CSR and its size; an
// absent side counts 1.  w_p = a_p * b_p (Claim "count" and the remark after
// it: d^{alpha_1}_u times d^{alpha_3}_v over the class's intervals), S its
// exact running total.
int window_weights(const Graph& G, int64_t delta, const Class& K, uint32_t* lo1, uint32_t* a,
                   uint32_t* lo3, uint32_t* b, uint64_t* S, int nthreads) {
  int64_t m = G.m;
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t p = 0; p < m; ++p) {
    int32_t e = G.out_ord[p];
    const int32_t ends[2] = {G.src[e], G.dst[e]};
    int64_t t = G.t[e];
    uint32_t lo[2], cnt[2];
    for (int s = 0; s < 2; ++s) {
      if (K.mode[s] == SIDE_NONE) {
        lo[s] = 0;
        cnt[s] = 1;
        continue;
      }
      const int32_t w = ends[s];
      const std::vector<int64_t>& tt = K.mode[s] == SIDE_IN ? G.in_t : G.out_t;
      const std::vector<uint32_t>& off = K.mode[s] == SIDE_IN ? G.in_off : G.out_off;
      const int64_t from = K.after[s] ? t : t - delta;
      const int64_t to = K.after[s] ? t + delta : t;
      auto beg = tt.begin() + off[w], end = tt.begin() + off[w + 1];
      // an open window leaves out the times equal to the centre time
      const bool open_from = K.open[s] && K.after[s], open_to = K.open[s] && !K.after[s];
      const int64_t i0 = (open_from ? std::upper_bound(beg, end, from)
                                    : std::lower_bound(beg, end, from)) - tt.begin();
      const int64_t i1 = (open_to ? std::lower_bound(beg, end, to)
                                  : std::upper_bound(beg, end, to)) - tt.begin();
      lo[s] = (uint32_t)i0;
      cnt[s] = (uint32_t)(i1 - i0);
    }
    lo1[p] = lo[0];
    a[p] = cnt[0];
    lo3[p] = lo[1];
    b[p] = cnt[1];
  }
  u128 run = 0;
  int st = OR_OK;
  for (int64_t p = 0; p < m; ++p) {
    S[p] = (uint64_t)run;
    run += (u128)((uint64_t)a[p] * (uint64_t)b[p]);
  }
  if (run > kU64Max) st = OR_OVERFLOW;
  S[m] = (uint64_t)run;
  return st;
}

// The motifs of one call share the anchor's class, its number of edges and
// their rank order (so one sampled anchor serves every motif).
int parse_motifs(const uint8_t* motifs, int n, const Class& K, std::vector<Motif>* Ms) {
  Ms->resize(n);
  for (int j = 0; j < n; ++j) {
    if (!parse_motif(motifs + 34 * j, &(*Ms)[j])) return OR_ARG;
    const Motif& A = (*Ms)[0];
    const Motif& B = (*Ms)[j];
    if (!same_class(B.cls, K) || B.na != A.na) return OR_ARG;
    for (int k = 0; k < B.na; ++k)
      if (B.order[k] != A.order[k]) return OR_ARG;
  }
  return OR_OK;
}

double u128_over_k_times_w(u128 cnt, uint64_t k, uint64_t W) {
  return ((double)cnt / (double)k) * (double)W;
}

}  // namespace

extern "C" {

void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

int or_lemire64(uint64_t x, uint64_t s, uint64_t* out) { return lemire64(x, s, out) ? 1 : 0; }
int or_lemire32(uint32_t x, uint32_t s, uint32_t* out) { return lemire32(x, s, out) ? 1 : 0; }

void* or_graph_new(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                   const int64_t* t, int* status, int nthreads) {
  Graph* G = new Graph();
  *status = build(*G, n, m, src, dst, t, nthreads < 1 ? 1 : nthreads);
  if (*status != OR_OK) {
    delete G;
    return nullptr;
  }
  return G;
}

void or_graph_free(void* h) { delete (Graph*)h; }

void or_graph_orders(void* h, int32_t* out_ord, int32_t* in_ord, int32_t* pair_ord,
                     uint32_t* out_off, uint32_t* in_off) {
  Graph& G = *(Graph*)h;
  std::copy(G.out_ord.begin(), G.out_ord.end(), out_ord);
  std::copy(G.in_ord.begin(), G.in_ord.end(), in_ord);
  std::copy(G.pair_ord.begin(), G.pair_ord.end(), pair_ord);
  std::copy(G.out_off.begin(), G.out_off.end(), out_off);
  std::copy(G.in_off.begin(), G.in_off.end(), in_off);
}

int or_weights(void* h, int64_t delta, uint32_t* lo_in, uint32_t* a, uint32_t* lo_out,
               uint32_t* b, uint64_t* S, int nthreads) {
  if (delta < 0 || delta > kTLimit) return OR_ARG;
  return window_weights(*(Graph*)h, delta, kSpineClass, lo_in, a, lo_out, b, S, nthreads);
}

// Preprocess for the class given by 4 bytes {mode1, after1, mode3, after3}.
int or_weights_class(void* h, int64_t delta, const uint8_t* cls, uint32_t* lo1, uint32_t* a,
                     uint32_t* lo3, uint32_t* b, uint64_t* S, int nthreads) {
  Class K;
  if (delta < 0 || delta > kTLimit || !parse_class(cls, &K)) return OR_ARG;
  return window_weights(*(Graph*)h, delta, K, lo1, a, lo3, b, S, nthreads);
}

// The class of a motif's anchor (4 bytes), its number of anchor edges and
// their rank order; OR_ARG when the motif has no anchor.
int or_anchor(const uint8_t* motif, uint8_t* cls, int32_t* na, int32_t* order, int32_t* aedge) {
  Motif M;
  if (!parse_motif(motif, &M)) return OR_ARG;
  for (int s = 0; s < 2; ++s) {
    cls[2 * s] = (uint8_t)M.cls.mode[s];
    cls[2 * s + 1] = (uint8_t)M.cls.after[s];
  }
  *na = M.na;
  for (int k = 0; k < 3; ++k) {
    order[k] = k < M.na ? M.order[k] : -1;
    aedge[k] = M.aedge[k];
  }
  return OR_OK;
}

// One anchor given by edge ids (-1 for an absent side) -> CheckMotif count.
int or_check_motif(void* h, const uint8_t* motif, int64_t delta, int32_t e1, int32_t e2,
                   int32_t e3, uint64_t* X) {
  Motif M;
  if (!parse_motif(motif, &M)) return OR_ARG;
  u128 c = 0;
  const int st = check_motif(*(Graph*)h, M, delta, e1, e2, e3, &c);
  *X = sat64(c);
  return st;
}

// Estimate(M, k) for a batch of motifs that share the anchor (class `cls`,
// null = the <-,+,<,>> class): samples i0 .. i0+k-1 of (seed, stream).
// Optional per-sample outputs (null = off): e1/e2/e3 edge ids [k] (-1 for an
// absent side), X motif-major [n_motifs * k], P the scan position of the
// centre edge [k].  cnt holds (lo, hi) per motif; xmax (null = off) the
// largest X.
//
// With a proposal h (null = plain sampler), S must be the scan of
// q_p = w_p * h_p and Q = S[m]: the centre edge is drawn with probability
// q_p / Q, so a path P centred at p has probability h_p / Q and the
// unbiased per-sample value is Y = X * Q / h_p.  cnt then accumulates
// floor(X * 2^64 / h_p) in 128 bits and est = (cnt * 2^-64 / k) * Q.
// m2 (null = off) receives sum over samples of (X / h_p)^2 in binary64.
//
// With window factors (ps1 / ps3: prefix sums of per-entry factors over the
// CSR that side 1 / side 3 draws from, null = none; not part of the paper),
// S must be the scan of q_p = h_p * G1_p * G3_p, G the sum of the factors
// over the side's window, and each side's edge is the window entry j drawn
// with probability g_j / G (a uniform integer u in [0, G), then the entry
// whose prefix interval holds u).  A path then has probability
// h_p g1 g3 / Q and cnt accumulates floor(X * 2^64 / (h_p g1 g3)); the
// product must stay below 2^32 (else OR_OVERFLOW).
int or_sample_win(void* hg, int64_t delta, const uint8_t* cls, const uint32_t* lo1,
                  const uint32_t* a, const uint32_t* lo3, const uint32_t* b, const uint64_t* S,
                  const uint32_t* hq, const uint64_t* ps1, const uint64_t* ps3,
                  const uint8_t* motifs, int n_motifs, uint64_t k,
                  uint64_t seed, uint32_t stream, uint64_t i0, int32_t* e1o, int32_t* e2o,
                  int32_t* e3o, uint64_t* Xo, uint32_t* Po, uint64_t* cnt, uint64_t* hits,
                  double* est, double* m2o, uint64_t* xmax, int nthreads) {
  Graph& G = *(Graph*)hg;
  Class K;
  if (n_motifs < 1 || n_motifs > 16 || k < 1 || !parse_class(cls, &K)) return OR_ARG;
  std::vector<Motif> Ms;
  if (parse_motifs(motifs, n_motifs, K, &Ms) != OR_OK) return OR_ARG;
  const uint64_t W = S[G.m];  // W, or Q with a proposal
  if (K.mode[0] == SIDE_NONE) ps1 = nullptr;
  if (K.mode[1] == SIDE_NONE) ps3 = nullptr;
  const bool is_ = hq || ps1 || ps3;  // importance sampling
  std::vector<u128> c(n_motifs, 0);
  std::vector<uint64_t> hh(n_motifs, 0), mx(n_motifs, 0);
  std::vector<double> mm(n_motifs, 0.0);
  int status = OR_OK;
  if (W == 0) {
    for (uint64_t i = 0; i < k; ++i) {
      if (e1o) { e1o[i] = -1; e2o[i] = -1; e3o[i] = -1; }
      if (Po) Po[i] = 0xFFFFFFFFu;
      if (Xo) for (int j = 0; j < n_motifs; ++j) Xo[j * k + i] = 0;
    }
  } else {
    std::vector<std::vector<u128>> pc(nthreads, std::vector<u128>(n_motifs, 0));
    std::vector<std::vector<uint64_t>> ph(nthreads, std::vector<uint64_t>(n_motifs, 0));
    std::vector<std::vector<uint64_t>> px(nthreads, std::vector<uint64_t>(n_motifs, 0));
    std::vector<std::vector<double>> pm(nthreads, std::vector<double>(n_motifs, 0.0));
    std::vector<int> pst(nthreads, OR_OK);
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t ii = 0; ii < (int64_t)k; ++ii) {
      int tid = omp_get_thread_num();
      uint64_t i = i0 + (uint64_t)ii;
      uint32_t x[4];
      // r uniform in [0, W)
      uint64_t r = 0;
      bool ok = false;
      for (uint32_t n = 0; n < (uint32_t)kMaxAttempts && !ok; ++n) {
        draw_block(seed, stream, i, n, x);
        ok = lemire64((uint64_t)x[0] | ((uint64_t)x[1] << 32), W, &r);
      }
      if (!ok) { pst[tid] |= OR_RNG; continue; }
      // pick e with probability w_e / W (or q_e / Q): S[p] <= r < S[p+1]
      int64_t p = std::upper_bound(S, S + G.m + 1, r) - S - 1;
      // then an edge in each side's window (an absent side has one
      // position and takes no edge): uniform, or by the window factors
      auto pick = [&](const uint64_t* ps, uint32_t lo, uint32_t len, int word, uint32_t* j,
                      uint64_t* gj) -> bool {
        uint64_t span = len;
        if (ps) {
          span = ps[lo + len] - ps[lo];
          if (span > 0xFFFFFFFFull) {
            pst[tid] |= OR_OVERFLOW;
            span = 0xFFFFFFFFull;
          }
        }
        uint32_t u = 0;
        bool got = false;
        for (uint32_t n = 0; n < (uint32_t)kMaxAttempts && !got; ++n) {
          draw_block(seed, stream, i, n, x);
          got = lemire32(x[word], (uint32_t)span, &u);
        }
        if (!got) return false;
        *j = u;
        *gj = 1;
        if (ps) {
          // the entry whose prefix interval [ps[lo+j] - ps[lo], ps[lo+j+1] - ps[lo]) holds u
          *j = (uint32_t)(std::upper_bound(ps + lo, ps + lo + len + 1, ps[lo] + u) - (ps + lo) -
                          1);
          *gj = ps[lo + *j + 1] - ps[lo + *j];
        }
        return true;
      };
      uint32_t j1 = 0, j3 = 0;
      uint64_t g1 = 1, g3 = 1;
      if (!pick(K.mode[0] == SIDE_NONE ? nullptr : ps1, lo1[p], a[p], 2, &j1, &g1)) {
        pst[tid] |= OR_RNG;
        continue;
      }
      if (!pick(K.mode[1] == SIDE_NONE ? nullptr : ps3, lo3[p], b[p], 3, &j3, &g3)) {
        pst[tid] |= OR_RNG;
        continue;
      }
      int32_t e2 = G.out_ord[p];
      int32_t e1 = K.mode[0] == SIDE_NONE ? -1 : side_edge(G, K.mode[0], lo1[p] + j1);
      int32_t e3 = K.mode[1] == SIDE_NONE ? -1 : side_edge(G, K.mode[1], lo3[p] + j3);
      if (e1o) { e1o[ii] = e1; e2o[ii] = e2; e3o[ii] = e3; }
      if (Po) Po[ii] = (uint32_t)p;
      // the path's proposal factor h_p g1 g3 (below 2^32)
      u128 hpw = (u128)(hq ? hq[p] : 1u) * g1 * g3;
      if (hpw > 0xFFFFFFFFull) {
        pst[tid] |= OR_OVERFLOW;
        hpw = 0xFFFFFFFFull;
      }
      const uint32_t hp = (uint32_t)hpw;
      for (int j = 0; j < n_motifs; ++j) {
        u128 X = 0;
        int st = check_motif(G, Ms[j], delta, e1, e2, e3, &X);
        // an importance-sampling term floor(X 2^64 / h) needs X < 2^64
        if (is_ && (X >> 64)) st |= OR_OVERFLOW;
        // an overflow also names its motif (bit 8 + j)
        pst[tid] |= st | ((st & OR_OVERFLOW) ? (1 << (8 + j)) : 0);
        if (Xo) Xo[(uint64_t)j * k + ii] = sat64(X);
        u128 add = is_ ? ((X << 64) / hp) : X;
        if (!add_u128(&pc[tid][j], add)) pst[tid] |= OR_OVERFLOW | (1 << (8 + j));
        ph[tid][j] += X > 0;
        px[tid][j] = std::max(px[tid][j], sat64(X));
        const double v = (double)X / (double)hp;
        pm[tid][j] += v * v;
      }
    }
    for (int tid = 0; tid < nthreads; ++tid) {
      status |= pst[tid];
      for (int j = 0; j < n_motifs; ++j) {
        if (!add_u128(&c[j], pc[tid][j])) status |= OR_OVERFLOW | (1 << (8 + j));
        hh[j] += ph[tid][j];
        mm[j] += pm[tid][j];
        mx[j] = std::max(mx[j], px[tid][j]);
      }
    }
  }
  for (int j = 0; j < n_motifs; ++j) {
    cnt[2 * j] = (uint64_t)c[j];
    cnt[2 * j + 1] = (uint64_t)(c[j] >> 64);
    hits[j] = hh[j];
    if (W == 0) {
      est[j] = 0.0;
    } else if (is_) {
      const double cd = std::ldexp((double)c[j], -64);
      est[j] = (cd / (double)k) * (double)W;
    } else {
      est[j] = u128_over_k_times_w(c[j], k, W);
    }
    if (m2o) m2o[j] = mm[j];
    if (xmax) xmax[j] = mx[j];
  }
  return status;
}

int or_sample_cls(void* hg, int64_t delta, const uint8_t* cls, const uint32_t* lo1,
                  const uint32_t* a, const uint32_t* lo3, const uint32_t* b, const uint64_t* S,
                  const uint32_t* hq, const uint8_t* motifs, int n_motifs, uint64_t k,
                  uint64_t seed, uint32_t stream, uint64_t i0, int32_t* e1o, int32_t* e2o,
                  int32_t* e3o, uint64_t* Xo, uint32_t* Po, uint64_t* cnt, uint64_t* hits,
                  double* est, double* m2o, uint64_t* xmax, int nthreads) {
  return or_sample_win(hg, delta, cls, lo1, a, lo3, b, S, hq, nullptr, nullptr, motifs, n_motifs,
                       k, seed, stream, i0, e1o, e2o, e3o, Xo, Po, cnt, hits, est, m2o, xmax,
                       nthreads);
}

int or_sample_ex(void* hg, int64_t delta, const uint32_t* lo_in, const uint32_t* a,
                 const uint32_t* lo_out, const uint32_t* b, const uint64_t* S,
                 const uint32_t* hq, const uint8_t* motifs, int n_motifs, uint64_t k,
                 uint64_t seed, uint32_t stream, uint64_t i0, int32_t* e1o, int32_t* e2o,
                 int32_t* e3o, uint64_t* Xo, uint32_t* Po, uint64_t* cnt, uint64_t* hits,
                 double* est, double* m2o, int nthreads) {
  return or_sample_cls(hg, delta, nullptr, lo_in, a, lo_out, b, S, hq, motifs, n_motifs, k, seed,
                       stream, i0, e1o, e2o, e3o, Xo, Po, cnt, hits, est, m2o, nullptr, nthreads);
}

int or_sample(void* h, int64_t delta, const uint32_t* lo_in, const uint32_t* a,
              const uint32_t* lo_out, const uint32_t* b, const uint64_t* S,
              const uint8_t* motifs, int n_motifs, uint64_t k, uint64_t seed, uint32_t stream,
              uint64_t i0, int32_t* e1o, int32_t* e2o, int32_t* e3o, uint64_t* Xo,
              uint64_t* cnt, uint64_t* hits, double* est, int nthreads) {
  return or_sample_ex(h, delta, lo_in, a, lo_out, b, S, nullptr, motifs, n_motifs, k, seed,
                      stream, i0, e1o, e2o, e3o, Xo, nullptr, cnt, hits, est, nullptr, nthreads);
}

// Exhaustive mode: the anchors of ranks r0 .. r0 + count - 1 (clipped to W)
// in the order of the integer CDF -- rank r is centre p with
// S[p] <= r < S[p+1] and j = r - S[p] = j1 * b_p + j3 -- each run through
// CheckMotif for every motif.  Over all W ranks cnt is the exact count C
// (proof of Claim "est": every match has exactly one anchor), hits the
// anchors with a match, m2 the sum of X^2 (binary64) and xmax the largest X:
// the B statistics (number of matches sharing an anchor) over anchors with
// a match are cnt / hits, sqrt(m2 / hits - (cnt / hits)^2) and xmax.
// Per-rank outputs as in or_sample_cls (index r - r0); est = cnt in binary64.
int or_enumerate(void* hg, int64_t delta, const uint8_t* cls, const uint32_t* lo1,
                 const uint32_t* a, const uint32_t* lo3, const uint32_t* b, const uint64_t* S,
                 const uint8_t* motifs, int n_motifs, uint64_t r0, uint64_t count, int32_t* e1o,
                 int32_t* e2o, int32_t* e3o, uint64_t* Xo, uint64_t* cnt, uint64_t* hits,
                 double* est, double* m2o, uint64_t* xmax, int nthreads) {
  Graph& G = *(Graph*)hg;
  Class K;
  if (n_motifs < 1 || n_motifs > 16 || !parse_class(cls, &K)) return OR_ARG;
  std::vector<Motif> Ms;
  if (parse_motifs(motifs, n_motifs, K, &Ms) != OR_OK) return OR_ARG;
  const uint64_t W = S[G.m];
  std::vector<std::vector<u128>> pc(nthreads, std::vector<u128>(n_motifs, 0));
  std::vector<std::vector<uint64_t>> ph(nthreads, std::vector<uint64_t>(n_motifs, 0));
  std::vector<std::vector<uint64_t>> px(nthreads, std::vector<uint64_t>(n_motifs, 0));
  std::vector<std::vector<double>> pm(nthreads, std::vector<double>(n_motifs, 0.0));
  std::vector<int> pst(nthreads, OR_OK);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 256)
  for (int64_t ii = 0; ii < (int64_t)count; ++ii) {
    int tid = omp_get_thread_num();
    const uint64_t r = r0 + (uint64_t)ii;
    if (r >= W || r < r0) {
      if (e1o) { e1o[ii] = -1; e2o[ii] = -1; e3o[ii] = -1; }
      if (Xo) for (int j = 0; j < n_motifs; ++j) Xo[(uint64_t)j * count + ii] = 0;
      continue;
    }
    const int64_t p = std::upper_bound(S, S + G.m + 1, r) - S - 1;
    const uint64_t jj = r - S[p];
    const uint32_t j1 = (uint32_t)(jj / b[p]), j3 = (uint32_t)(jj % b[p]);
    int32_t e2 = G.out_ord[p];
    int32_t e1 = K.mode[0] == SIDE_NONE ? -1 : side_edge(G, K.mode[0], lo1[p] + j1);
    int32_t e3 = K.mode[1] == SIDE_NONE ? -1 : side_edge(G, K.mode[1], lo3[p] + j3);
    if (e1o) { e1o[ii] = e1; e2o[ii] = e2; e3o[ii] = e3; }
    for (int j = 0; j < n_motifs; ++j) {
      u128 X = 0;
      int st = check_motif(G, Ms[j], delta, e1, e2, e3, &X);
      if (!add_u128(&pc[tid][j], X)) st |= OR_OVERFLOW;
      pst[tid] |= st | ((st & OR_OVERFLOW) ? (1 << (8 + j)) : 0);
      if (Xo) Xo[(uint64_t)j * count + ii] = sat64(X);
      ph[tid][j] += X > 0;
      px[tid][j] = std::max(px[tid][j], sat64(X));
      pm[tid][j] += (double)X * (double)X;
    }
  }
  int status = OR_OK;
  for (int j = 0; j < n_motifs; ++j) {
    u128 c = 0;
    uint64_t h = 0, mx = 0;
    double mm = 0.0;
    for (int tid = 0; tid < nthreads; ++tid) {
      if (!add_u128(&c, pc[tid][j])) status |= OR_OVERFLOW | (1 << (8 + j));
      h += ph[tid][j];
      mm += pm[tid][j];
      mx = std::max(mx, px[tid][j]);
    }
    cnt[2 * j] = (uint64_t)c;
    cnt[2 * j + 1] = (uint64_t)(c >> 64);
    hits[j] = h;
    est[j] = (double)c;
    if (m2o) m2o[j] = mm;
    if (xmax) xmax[j] = mx;
  }
  for (int tid = 0; tid < nthreads; ++tid) status |= pst[tid];
  return status;
}

// Scan of the proposal weights q_p = a_p * b_p * h_p (exact, 128-bit
// running total): Q[p] = sum_{p' < p} q_p', Q[m] = Q.  Overflow if Q >= 2^64.
int or_proposal_scan(void* hg, const uint32_t* a, const uint32_t* b, const uint32_t* hq,
                     uint64_t* Q) {
  Graph& G = *(Graph*)hg;
  u128 run = 0;
  int st = OR_OK;
  for (int64_t p = 0; p < G.m; ++p) {
    Q[p] = (uint64_t)run;
    run += (u128)((uint64_t)a[p] * (uint64_t)b[p]) * hq[p];
    if (run > kU64Max) st = OR_OVERFLOW;
  }
  Q[G.m] = (uint64_t)run;
  return st;
}

// Window factors (not part of the paper): every in-CSR entry (an edge
// x -> u) gets g(deg x) and every out-CSR entry (an edge v -> y) g(deg y),
// deg the total degree (in + out) of the far endpoint, with
//   g(d) = min(cap, F_q(1 + d)),  F_0 = 1, F_1 = r4, F_2 = r2, F_3 = r2 r4,
//   F_4 = r2^2, where r2 = isqrt(1 + d) and r4 = isqrt(r2)
// (integer square roots, so about (1 + d)^(q / 4)).
static uint64_t isqrt64(uint64_t v) {
  uint64_t r = (uint64_t)std::sqrt((double)v);
  while (r > 0 && r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

static uint32_t degree_factor(uint64_t d, int quarter, uint32_t cap) {
  const uint64_t r2 = isqrt64(1 + d), r4 = isqrt64(r2);
  const uint64_t f = quarter == 0 ? 1 : quarter == 1 ? r4 : quarter == 2 ? r2
                   : quarter == 3 ? r2 * r4 : r2 * r2;
  return (uint32_t)std::min<uint64_t>(f, cap);
}

int or_window_factors(void* hg, int quarter, uint32_t cap, uint32_t* f_in, uint32_t* f_out) {
  Graph& G = *(Graph*)hg;
  if (quarter < 0 || quarter > 4 || cap < 1 || cap > 65535) return OR_ARG;
  auto deg = [&](int32_t v) -> uint64_t {
    return (uint64_t)(G.out_off[v + 1] - G.out_off[v]) + (uint64_t)(G.in_off[v + 1] - G.in_off[v]);
  };
  for (int64_t i = 0; i < G.m; ++i) {
    f_in[i] = degree_factor(deg(G.src[G.in_ord[i]]), quarter, cap);
    f_out[i] = degree_factor(deg(G.dst[G.out_ord[i]]), quarter, cap);
  }
  return OR_OK;
}

// Scan of the window proposal q_p = h_p * G1_p * G3_p (h null = 1): G of a
// side is the sum of the factors of its CSR (f_in for an in-edge side,
// f_out for an out-edge side; a null array counts 1 per entry) over the
// side's window, 1 for an absent side.  ps_in / ps_out (m + 1 words each)
// receive the prefix sums of f_in / f_out when given.  OR_OVERFLOW if a
// window sum reaches 2^32 or Q reaches 2^64.
int or_proposal_window(void* hg, const uint8_t* cls, const uint32_t* lo1, const uint32_t* a,
                       const uint32_t* lo3, const uint32_t* b, const uint32_t* hq,
                       const uint32_t* f_in, const uint32_t* f_out, uint64_t* ps_in,
                       uint64_t* ps_out, uint64_t* Q) {
  Graph& G = *(Graph*)hg;
  Class K;
  if (!parse_class(cls, &K)) return OR_ARG;
  if (f_in) {
    uint64_t s = 0;
    for (int64_t i = 0; i < G.m; ++i) { ps_in[i] = s; s += f_in[i]; }
    ps_in[G.m] = s;
  }
  if (f_out) {
    uint64_t s = 0;
    for (int64_t i = 0; i < G.m; ++i) { ps_out[i] = s; s += f_out[i]; }
    ps_out[G.m] = s;
  }
  int st = OR_OK;
  auto side_sum = [&](int mode, uint32_t lo, uint32_t len) -> u128 {
    if (mode == SIDE_NONE) return 1;
    const uint64_t* ps = mode == SIDE_IN ? (f_in ? ps_in : nullptr) : (f_out ? ps_out : nullptr);
    const uint64_t g = ps ? ps[lo + len] - ps[lo] : len;
    if (g > 0xFFFFFFFFull) st = OR_OVERFLOW;
    return g;
  };
  u128 run = 0;
  for (int64_t p = 0; p < G.m; ++p) {
    Q[p] = (uint64_t)run;
    const u128 q = (u128)(hq ? hq[p] : 1u) * side_sum(K.mode[0], lo1[p], a[p]) *
                   side_sum(K.mode[1], lo3[p], b[p]);
    run += q;
    if (run > kU64Max) st = OR_OVERFLOW;
  }
  Q[G.m] = (uint64_t)run;
  return st;
}

// Per-edge features of the learned proposal, in binary64, for every scan
// position p (centre edge e = (u, v, t)):
//   0 ln(1 + a)     in-window size of u in [t - delta, t]
//   1 ln(1 + b)     out-window size of v in [t, t + delta]
//   2 ln(1 + a b)   the path weight w_e
//   3 (t - t_first) / delta, t_first the earliest time in u's in-window
//   4 (t_last - t) / delta, t_last the latest time in v's out-window
//   5 ln(1 + #edges u -> v with time in [t - delta, t + delta])
//   6 ln(1 + #edges v -> u with time in [t - delta, t + delta])
//   7 ln(1 + M_in * M_out) / 2, with M_in the mean over u's in-window
//     edges (x -> u) of min(indeg(x), 65535)^2 and M_out the mean over v's
//     out-window edges (v -> y) of min(outdeg(y), 65535)^2 (0 if a window
//     is empty): how heavy the closing pairs y -> x of the paths through
//     the edge can be
// Features 3 and 4 are 0 when their window is empty or delta = 0.
void or_features(void* hg, int64_t delta, const uint32_t* lo_in, const uint32_t* a,
                 const uint32_t* lo_out, const uint32_t* b, double* F, int nthreads) {
  Graph& G = *(Graph*)hg;
  auto pair_count = [&](int32_t x, int32_t y, int64_t lo_t, int64_t hi_t) -> int64_t {
    auto beg = G.pair_dst.begin() + G.out_off[x];
    auto end = G.pair_dst.begin() + G.out_off[x + 1];
    auto run = std::equal_range(beg, end, y);
    auto tb = G.pair_t.begin();
    auto r0 = tb + (run.first - G.pair_dst.begin());
    auto r1 = tb + (run.second - G.pair_dst.begin());
    return std::upper_bound(r0, r1, hi_t) - std::lower_bound(r0, r1, lo_t);
  };
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t p = 0; p < G.m; ++p) {
    const int32_t e = G.out_ord[p];
    const int32_t u = G.src[e], v = G.dst[e];
    const int64_t t = G.t[e];
    double* f = F + 8 * p;
    f[0] = std::log1p((double)a[p]);
    f[1] = std::log1p((double)b[p]);
    f[2] = std::log1p((double)a[p] * (double)b[p]);
    f[3] = (a[p] > 0 && delta > 0) ? (double)(t - G.in_t[lo_in[p]]) / (double)delta : 0.0;
    f[4] = (b[p] > 0 && delta > 0)
               ? (double)(G.out_t[lo_out[p] + b[p] - 1] - t) / (double)delta
               : 0.0;
    f[5] = std::log1p((double)pair_count(u, v, t - delta, t + delta));
    f[6] = std::log1p((double)pair_count(v, u, t - delta, t + delta));
    auto cap2 = [](uint64_t d) -> uint64_t {
      const uint64_t c = d < 65535u ? d : 65535u;
      return c * c;
    };
    uint64_t s_in = 0, s_out = 0;
    for (uint32_t j = 0; j < a[p]; ++j) {
      const int32_t x = G.in_src[lo_in[p] + j];
      s_in += cap2(G.in_off[x + 1] - G.in_off[x]);
    }
    for (uint32_t j = 0; j < b[p]; ++j) {
      const int32_t y = G.out_dst[lo_out[p] + j];
      s_out += cap2(G.out_off[y + 1] - G.out_off[y]);
    }
    const double m_in = a[p] ? (double)s_in / (double)a[p] : 0.0;
    const double m_out = b[p] ? (double)s_out / (double)b[p] : 0.0;
    f[7] = 0.5 * std::log1p(m_in * m_out);
  }
}

// Sum of CheckMotif over every delta-centred <-,+,<,>> path (all W of them):
// by the proof of Claim "est" this equals the number of M-matches.  Also
// returns sum X^2 and the number of paths with X > 0.
int or_exhaustive(void* h, const uint8_t* motif, int64_t delta, const uint8_t* cls,
                  const uint32_t* lo1, const uint32_t* a, const uint32_t* lo3, const uint32_t* b,
                  uint64_t* sum_x, uint64_t* sum_x2, uint64_t* nonzero, int nthreads) {
  Graph& G = *(Graph*)h;
  Motif M;
  Class K;
  if (!parse_motif(motif, &M) || !parse_class(cls, &K) || !same_class(M.cls, K)) return OR_ARG;
  std::vector<u128> s1(nthreads, 0), s2(nthreads, 0);
  std::vector<uint64_t> nz(nthreads, 0);
  std::vector<int> pst(nthreads, OR_OK);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
  for (int64_t p = 0; p < G.m; ++p) {
    int tid = omp_get_thread_num();
    for (uint32_t j1 = 0; j1 < a[p]; ++j1)
      for (uint32_t j3 = 0; j3 < b[p]; ++j3) {
        u128 X = 0;
        const int32_t e1 = K.mode[0] == SIDE_NONE ? -1 : side_edge(G, K.mode[0], lo1[p] + j1);
        const int32_t e3 = K.mode[1] == SIDE_NONE ? -1 : side_edge(G, K.mode[1], lo3[p] + j3);
        pst[tid] |= check_motif(G, M, delta, e1, G.out_ord[p], e3, &X);
        if (!add_u128(&s1[tid], X) || (X >> 64) || !add_u128(&s2[tid], X * X))
          pst[tid] |= OR_OVERFLOW;
        nz[tid] += X > 0;
      }
  }
  u128 t1 = 0, t2 = 0;
  uint64_t tn = 0;
  int st = OR_OK;
  for (int i = 0; i < nthreads; ++i) { t1 += s1[i]; t2 += s2[i]; tn += nz[i]; st |= pst[i]; }
  sum_x[0] = (uint64_t)t1; sum_x[1] = (uint64_t)(t1 >> 64);
  sum_x2[0] = (uint64_t)t2; sum_x2[1] = (uint64_t)(t2 >> 64);
  *nonzero = tn;
  return st;
}

// Definition-level count of M-matches (section I-A): every assignment of
// distinct G-edges to the motif edges, in pi order with strictly increasing
// times, all within delta of the first, whose endpoints define a 1-1 map
// from V(H) into V(G).  Backtracking in pi order; candidates for rank r are
// read from the adjacency lists of already mapped endpoints.
namespace {
struct Brute {
  const Graph& G;
  const Motif& M;
  int64_t delta;
  int32_t phi[16];
  u128 count = 0;
  Brute(const Graph& g, const Motif& m, int64_t d) : G(g), M(m), delta(d) {
    for (int i = 0; i < 16; ++i) phi[i] = -1;
  }
  bool used(int32_t v) const {
    for (int i = 0; i < M.nv; ++i)
      if (phi[i] == v) return true;
    return false;
  }
  void extend(int r, int64_t t_first, int64_t t_prev) {
    if (r == M.ne) { count += 1; return; }
    int ha = M.src[r], hb = M.dst[r];
    int32_t ga = phi[ha], gb = phi[hb];
    int64_t hi = t_first + delta;
    if (ga >= 0 && gb >= 0) {
      int64_t f, l;
      pair_window(G, ga, gb, t_prev, hi, &f, &l);
      for (int64_t q = f; q < l; ++q) extend(r + 1, t_first, G.pair_t[q]);
    } else if (ga >= 0) {
      auto ob = G.out_t.begin();
      int64_t f = std::upper_bound(ob + G.out_off[ga], ob + G.out_off[ga + 1], t_prev) - ob;
      int64_t l = std::upper_bound(ob + G.out_off[ga], ob + G.out_off[ga + 1], hi) - ob;
      for (int64_t q = f; q < l; ++q) {
        int32_t w = G.out_dst[q];
        if (used(w)) continue;
        phi[hb] = w;
        extend(r + 1, t_first, G.out_t[q]);
        phi[hb] = -1;
      }
    } else if (gb >= 0) {
      auto ib = G.in_t.begin();
      int64_t f = std::upper_bound(ib + G.in_off[gb], ib + G.in_off[gb + 1], t_prev) - ib;
      int64_t l = std::upper_bound(ib + G.in_off[gb], ib + G.in_off[gb + 1], hi) - ib;
      for (int64_t q = f; q < l; ++q) {
        int32_t w = G.in_src[q];
        if (used(w)) continue;
        phi[ha] = w;
        extend(r + 1, t_first, G.in_t[q]);
        phi[ha] = -1;
      }
    } else {
      // only possible for a motif whose prefix is disconnected; scan all edges
      for (int64_t e = 0; e < G.m; ++e) {
        if (!(G.t[e] > t_prev && G.t[e] <= hi)) continue;
        int32_t s = G.src[e], d = G.dst[e];
        if (s == d || used(s) || used(d)) continue;
        phi[ha] = s; phi[hb] = d;
        extend(r + 1, t_first, G.t[e]);
        phi[ha] = -1; phi[hb] = -1;
      }
    }
  }
};
}  // namespace

int or_brute_count(void* h, const uint8_t* motif_bytes, int64_t delta, uint64_t* C,
                   int nthreads) {
  Graph& G = *(Graph*)h;
  Motif M;
  M.nv = motif_bytes[0];
  M.ne = motif_bytes[1];
  if (M.nv < 2 || M.nv > 16 || M.ne < 1 || M.ne > 16) return OR_ARG;
  for (int i = 0; i < M.ne; ++i) {
    M.src[i] = motif_bytes[2 + i];
    M.dst[i] = motif_bytes[18 + i];
  }
  std::vector<u128> part(nthreads, 0);
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 16)
  for (int64_t e = 0; e < G.m; ++e) {
    int32_t s = G.src[e], d = G.dst[e];
    if (s == d) continue;
    Brute bt(G, M, delta);
    bt.phi[M.src[0]] = s;
    bt.phi[M.dst[0]] = d;
    bt.extend(1, G.t[e], G.t[e]);
    part[omp_get_thread_num()] += bt.count;
  }
  u128 tot = 0;
  for (auto v : part) tot += v;
  C[0] = (uint64_t)tot;
  C[1] = (uint64_t)(tot >> 64);
  return OR_OK;
}

// ListCount on caller-provided sorted lists (for pinning against product
// enumeration): lists concatenated in `vals`, list r spans [off[r], off[r+1]);
// X receives the 128-bit count as (low, high) words.
int or_list_count(const int64_t* vals, const int64_t* off, int l, uint64_t* X) {
  std::vector<std::vector<int64_t>> L(l);
  for (int r = 0; r < l; ++r) L[r].assign(vals + off[r], vals + off[r + 1]);
  u128 c;
  const bool ok = list_count(L, &c);
  X[0] = (uint64_t)c;
  X[1] = (uint64_t)(c >> 64);
  return ok ? OR_OK : OR_OVERFLOW;
}

int or_max_threads(void) { return omp_get_max_threads(); }

// Window lengths of the lists of one delta-centred path (e1, e2, e3 by edge
// id) for one motif, in rank order; returns the number of lists, or -1 if
// the path fails CheckMotif's vertex and time tests.  Test diagnostics.
int or_list_lengths(void* h, const uint8_t* motif, int64_t delta, int32_t e1, int32_t e2,
                    int32_t e3, int64_t* lens) {
  Graph& G = *(Graph*)h;
  Motif M;
  if (!parse_motif(motif, &M)) return -2;
  const int32_t u = G.src[e2], v = G.dst[e2];
  int32_t phi[4] = {-1, u, v, -1};
  const int32_t ae[3] = {e1, e2, e3};
  for (int s = 0; s < 2; ++s) {
    const int32_t e = ae[2 * s];
    if ((M.cls.mode[s] == SIDE_NONE) != (e < 0)) return -2;
    if (e >= 0) phi[s == 0 ? 0 : 3] = M.cls.mode[s] == SIDE_IN ? G.src[e] : G.dst[e];
  }
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (phi[i] >= 0 && phi[i] == phi[j]) return -1;
  int64_t T[3];
  for (int k = 0; k < M.na; ++k) T[k] = G.t[ae[M.order[k]]];
  for (int k = 1; k < M.na; ++k)
    if (!(T[k - 1] < T[k])) return -1;
  if (T[M.na - 1] - T[0] > delta) return -1;
  for (int i = 0; i < M.nl; ++i) {
    const int sg = M.lseg[i];
    const int64_t hi = sg + 1 < M.na ? T[sg + 1] - 1 : T[0] + delta;
    int64_t f, l;
    pair_window(G, phi[M.lslot_a[i]], phi[M.lslot_b[i]], T[sg], hi, &f, &l);
    lens[i] = l - f;
  }
  return M.nl;
}

}  // extern "C"
