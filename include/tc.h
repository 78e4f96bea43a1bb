/* tc.h -- C ABI of the MI355X temporal 3-path sampling library (libtc.so).
 *
 * The library estimates the number of matches of a 3- or 4-vertex temporal
 * motif M = (H, pi, delta) in a directed temporal multigraph G by sampling
 * delta-centred 3-paths of the motif's anchor class, or wedges for 3-vertex
 * motifs (Pan, Bhalerao, Seshadhri, Talati, "Accurate and Fast Estimation
 * of Temporal Motifs using Path Sampling", ICDM 2024), and counts them
 * exactly by visiting every anchor (tc_exhaustive_count).  Problem
 * statement: section I-A (temporal multigraph, edges (u, v, t) with integer
 * t, parallel edges allowed; Definitions of a temporal motif and of an
 * M-match).  The three calls below are the three
 * phases of Algorithm Estimate: the time-sorted adjacency it assumes,
 * Preprocess (per-edge weights and their total W), and the loop of Sample +
 * CheckMotif that ends in C_hat = (cnt / k) * W.
 *
 * Conventions shared by every entry point:
 *   - Pointers marked (device) are HIP device pointers owned by the caller;
 *     (host) pointers are read during the call only.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Every call is stream-ordered and returns as soon as its kernels are
 *     enqueued (tc_autotune alone waits, for its timings).
 *   - The library allocates no device memory and creates no streams.  The
 *     caller provides workspaces of at
 *     least the size reported by the *_workspace_bytes queries, 256-byte
 *     aligned (as hipMalloc and torch allocations are: the 64-bit atomics
 *     and 16-byte records inside them need it); a null or misaligned
 *     workspace gives TC_E_ARG, a short one TC_E_WORKSPACE.  tc_graph and
 *     tc_weights then hold pointers into those workspaces (borrowed: keep the
 *     workspace alive while the struct is used).  There is no free call.
 *   - Host-checkable argument errors are returned synchronously and nothing
 *     is enqueued.  Data-dependent errors are recorded as bits of a device
 *     status word (TC_F_*); results guarded by a non-zero status word are
 *     undefined.  No C++ exception crosses this boundary.
 *   - Results are a pure function of the inputs (graph bytes, delta, motifs,
 *     k, seed, stream_id, i0), independent of launch configuration.
 *   - Calls on distinct workspaces/results may run concurrently.
 */
#ifndef TC_H_
#define TC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TC_OK = 0,
  TC_E_ARG = -1,          /* null pointer, bad size, bad delta or k            */
  TC_E_RANGE = -2,        /* reserved for host-side reporting of TC_F_RANGE     */
  TC_E_OVERFLOW = -3,     /* reserved for host-side reporting of TC_F_OVERFLOW  */
  TC_E_UNSUPPORTED = -4,  /* motif without an anchor path or wedge              */
  TC_E_WORKSPACE = -5,    /* workspace smaller than the query reported          */
  TC_E_HIP = -6           /* a HIP runtime call failed                          */
} tc_status;

/* Bits of a device status word. */
#define TC_F_RANGE 1u     /* bad vertex id or timestamp                              */
#define TC_F_OVERFLOW 2u  /* W >= 2^64; a count cnt >= 2^128; or, with a proposal
                             weight set, a per-sample X >= 2^64                     */
#define TC_F_RNG 4u       /* 1024 consecutive rejections in the range reduction       */
/* With TC_F_OVERFLOW from the sampler, bit 8 + j names each motif j whose
 * count overflowed; the counts of the other motifs of the call stay exact.
 * Per-sample counts X are exact up to 2^128 (ListCount in 128 bits where a
 * level's total reaches 2^64). */
#define TC_F_MOTIF(j) (1u << (8 + (j)))

/* A temporal motif: H's edges listed in pi order (edge i has time rank i),
 * vertices 0..nv-1 (nv = 3 or 4), 2 <= ne <= 16, no self-loops.  Its anchor S
 * (section III-B; Algorithm Estimate chooses an anchor holding the earliest
 * edge) is found by the library:
 *   nv = 4: a temporal 3-path x - u - v - y over four distinct vertices, its
 *     centre edge u -> v, holding rank 0: among all, the one with the
 *     lexicographically smallest sorted ranks, then the smallest centre
 *     rank, then the smallest rank of the edge at u;
 *   nv = 3: a wedge, centre edge u -> v plus one edge meeting u or v and
 *     reaching the third vertex, holding rank 0: smallest sorted ranks, then
 *     the smallest centre rank (so the centre is the earliest edge, the
 *     "base" edge of the wedge).
 * A motif with no such anchor (a 3-star, fewer than 3 vertices) gives
 * TC_E_UNSUPPORTED.  The anchor's class (tc_class) says which weights it is
 * sampled from; every other motif edge of rank r is looked for between the
 * anchor edges ranked just below and just above r (or up to the first
 * anchor time + delta), which is how CheckMotif bounds its lists. */
typedef struct {
  uint8_t nv, ne;
  uint8_t src[16], dst[16];
} tc_motif;

/* Anchor class (section III: the classes <alpha_1, alpha_3, beta_1, beta_3>
 * of delta-centred 3-paths, and the wedges of the 3-vertex case).  For the
 * side at the centre edge's source u (side 1) and at its destination v
 * (side 3): mode TC_SIDE_NONE (no edge: a wedge), TC_SIDE_IN (an in-edge,
 * alpha = -) or TC_SIDE_OUT (an out-edge, alpha = +); after = 0 for an edge
 * before the centre (window [t - delta, t], beta = <), 1 for one after it
 * ([t, t + delta], beta = >).  At least one side has an edge.  The class
 * <-,+,<,>> of the paper's presentation is {IN, 0, OUT, 1}.
 * TC_WINDOW_OPEN added to an `after` value opens that side's window at the
 * centre time: [t - delta, t) or (t, t + delta].  A match's times increase
 * strictly, so every match's anchor still lies in the open windows and the
 * estimate stays unbiased, with a weight total W no larger than the closed
 * windows' (a variant of Claim "count"; not in the paper).  Motif anchors
 * (tc_motif_anchor) report closed windows; a weights set of either kind
 * serves the motifs of its class. */
#define TC_SIDE_NONE 0
#define TC_SIDE_IN 1
#define TC_SIDE_OUT 2
#define TC_WINDOW_OPEN 2
typedef struct {
  uint8_t mode1, after1, mode3, after3;
} tc_class;

/* The anchor of a motif: its class, the number of anchor edges (3 for a
 * path, 2 for a wedge) and, in order[0..n_anchor-1], the anchor edges by
 * increasing rank (0 = the edge at u, 1 = the centre, 2 = the edge at v).
 * Errors: TC_E_ARG (null), TC_E_UNSUPPORTED (no anchor). */
tc_status tc_motif_anchor(const tc_motif *motif, tc_class *cls, int32_t *n_anchor,
                          int32_t *order);

/* Time-sorted temporal adjacency (section III-A assumes per-vertex in- and
 * out-lists sorted by time; section III-B uses the per-pair lists L_{u,v}).
 * Filled by tc_build_graph; all arrays (device) live in the graph workspace.
 *   out-CSR : edges sorted by (src, t, eid); out_off[v]..out_off[v+1]-1 are
 *             v's out-edges.  Position p in this order is the "scan order"
 *             used by the weights and the sampler.
 *   in-CSR  : edges sorted by (dst, t, eid); in_off as above.
 *   pair    : edges sorted by (src, dst, t, eid); shares out_off; each run
 *             of equal (src, dst) is also reachable through pair_hash.
 * eid is the edge's index in the input arrays; it breaks timestamp ties. */
typedef struct tc_graph {
  int32_t n;
  int64_t m;
  int64_t *t_range;                   /* [2] (device): t_min, t_max of the input
                                         (0, 0 when m = 0 or the input is rejected) */
  uint32_t *out_off;                  /* [n+1] */
  int32_t *out_src, *out_dst, *out_eid;
  int64_t *out_t;                     /* [m] each */
  uint32_t *in_off;                   /* [n+1] */
  int32_t *in_src, *in_eid, *in_dst;
  int64_t *in_t;                      /* [m] each */
  int32_t *pair_dst, *pair_eid;
  int64_t *pair_t;                    /* [m] each */
  uint32_t *status;                   /* device status word of the build       */
  void *pair_hash;                    /* run table of the pair index: 2^pair_hash_log2
                                         16-byte slots {u64 src<<32|dst, u32 start,
                                         u32 end}, open addressing, linear probing,
                                         empty key = all ones                     */
  int32_t pair_hash_log2;
  void *out_rec, *in_rec;             /* [m] 16-byte records of the two CSRs, one
                                         cache-line access per sampled end edge:
                                         {i32 other end (dst resp. src), i32 eid,
                                         i64 t}                                  */
  int64_t *pair_skip;                 /* sampled pair times for searches inside a
                                         run: level k = 1, 2, 3 holds
                                         pair_t[16^k i] for i < ceil(m / 16^k),
                                         the levels stored one after another     */
} tc_graph;

/* Per-edge window metadata and the exact integer CDF of the path weights,
 * all indexed by scan position p (out-CSR order), centre edge (u, v, t):
 *   lo_in[p], a[p]: side 1's window -- u's in-edges (in-CSR positions) or
 *              out-edges (out-CSR positions) with time in [t - delta, t] or
 *              [t, t + delta] as the class says: its first position and its
 *              size (d^{alpha_1}_u over the interval); 0 and 1 when side 1
 *              has no edge.  For the class {IN, 0, OUT, 1}: d^-_u[t - delta, t]
 *   lo_out[p], b[p]: side 3's window at v likewise (d^+_v[t, t + delta])
 *   S[p] = sum_{q < p} a[q] * b[q]  (exclusive scan), S[m] = W_delta.
 * Claim "count" and the remark after it give w_e = a * b; Algorithm
 * Preprocess computes it with four binary searches per edge.  Windows are
 * closed on both ends. */
typedef struct tc_weights {
  int64_t delta;
  int64_t m;
  uint32_t *lo_in, *a, *lo_out, *b;   /* [m] each (device) */
  uint64_t *S;                        /* [m+1] (device; followed by all-ones padding
                                         to a multiple of 16 words) */
  uint32_t *status;                   /* device word: TC_F_OVERFLOW if W >= 2^64 */
  void *scratch;                      /* 16-ary search tree over S (internal) */
  const uint32_t *h;                  /* NULL for the weights of the method; for a
                                         proposal weight set (tc_proposal_weights)
                                         the integer factor h[p] >= 1 per edge, and
                                         S is then the scan of q = a * b * h      */
  void *prec;                         /* [m] 32-byte path records {u32 lo_in, a,
                                         lo_out, b; i32 u, v; i64 t} of the scan
                                         positions (what the sampler needs of the
                                         centre edge, in one access)              */
  tc_class cls;                       /* anchor class of the windows           */
  const uint64_t *ps1, *ps3;          /* NULL, or for a window proposal set
                                         (tc_proposal_window) the prefix sums of
                                         the entry factors over the CSR that side 1
                                         resp. side 3 draws from ([m+1]); S is then
                                         the scan of q = h * G1 * G3              */
} tc_weights;

/* Outputs of tc_sample_estimate, all (device), caller-allocated.
 *   cnt[2j], cnt[2j+1] : low and high 64 bits of cnt_j = sum_i X_ij
 *   hits[j]            : number of samples with X_ij > 0
 *   estimate[j]        : C_hat_j = (cnt_j / k) * W in IEEE binary64, each
 *                        integer converted with round-to-nearest-even
 *   status             : TC_F_* bits (OR of the weights' status and the
 *                        sampler's own)
 *   e1, e2, e3         : optional [k] edge ids of the sampled path (NULL=off)
 *   X                  : optional [n_motifs * k], motif-major, saturated at
 *                        2^64 - 1 (cnt has the exact sum) (NULL = off)
 *   P                  : optional [k] scan position of the centre edge
 *                        (all ones when W = 0; NULL = off)
 *   m2                 : optional [n_motifs] sum over samples of
 *                        (X_ij / h_p)^2 in binary64 (h = 1 for the method's
 *                        weights), for variance estimates; its summation
 *                        order is not fixed (NULL = off)
 *   xmax               : optional [n_motifs] largest X_ij (NULL = off)
 * With a proposal weight set (w->h != NULL) the estimator is importance
 * sampling: a path centred at p has probability h[p] / Q, Q = S[m], and
 * contributes Y = X * Q / h[p].  cnt_j then holds the exact 128-bit sum of
 * floor(X_ij * 2^64 / h_p) and estimate[j] = ((cnt_j * 2^-64) / k) * Q.
 * cnt, hits, estimate, m2 and status are overwritten (not accumulated). */
typedef struct tc_result {
  uint64_t *cnt;
  uint64_t *hits;
  double *estimate;
  uint32_t *status;
  int32_t *e1, *e2, *e3;
  uint64_t *X;
  uint32_t *P;
  double *m2;
  uint64_t *xmax;
} tc_result;

/* Launch-shape choices of the sampler.  They change speed only, never a
 * result (every output is a pure function of the inputs).
 *   chunk_log2  log2 of the samples processed per chunk over all deltas
 *               (10..25; the queue and window scratch scale with it)
 *   path_blocks persistent blocks of the path kernel (0 = one per tile)
 *   reg_waves   wavefronts of the register ListCount pass
 *   fast_waves  wavefronts of the LDS-key ListCount pass (64..8192)
 *   wide_blocks 128-thread blocks of the merged ListCount pass for lists
 *               over lds_list_cap entries (16..4096; 1 MiB of workspace each)
 *   reg_list_cap  longest list the register ListCount pass takes: 128 or
 *               256 entries (two or four 64-entry chunks per lane); items
 *               with a longer list go to the LDS-key pass
 *   lds_list_cap  longest list the one-wavefront LDS-key pass takes
 *               (256..1024); items with a longer list go to the merged
 *               pass, where 128 lanes work on one item instead of 64 */
typedef struct {
  int32_t chunk_log2;
  int32_t path_blocks;
  int32_t reg_waves;
  int32_t fast_waves;
  int32_t wide_blocks;
  int32_t reg_list_cap;
  int32_t lds_list_cap;
} tc_tuning;

/* Library version string (host, static storage). */
const char *tc_version(void);

/* Workspace size in bytes for tc_build_graph with n vertices and m edges.
 * Errors: TC_E_ARG if bytes is NULL, n < 1, m < 0 or m >= 2^31. */
tc_status tc_graph_workspace_bytes(int32_t n, int64_t m, size_t *bytes);

/* Build the temporal adjacency of the multigraph given by src, dst, t
 * (device, [m] each, eid = index).  Requires 0 <= src, dst < n and
 * |t| < 2^62.  Enqueue only: the validation, the stable radix sorts (the
 * number of time-sort passes that do work is decided on the device from the
 * time range), the offsets and the pair-run table, all on `stream`, with no
 * host synchronisation and no allocation, so the call can be captured in a
 * HIP graph.  On TC_OK, *g describes the graph and its arrays are ready in
 * stream order.  A bad vertex id or time sets TC_F_RANGE in the device word
 * *g->status and leaves the arrays undefined; tc_path_weights on such a
 * graph reports TC_F_RANGE in its own status word with W = 0, and the
 * sampler then draws nothing.  The input arrays must stay alive until the
 * enqueued work has run.
 * Errors: TC_E_ARG (null pointers, n < 1, m < 0, m >= 2^31),
 * TC_E_WORKSPACE, TC_E_HIP. */
tc_status tc_build_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         const int64_t *t, void *ws, size_t ws_bytes, void *stream,
                         tc_graph *g);

/* Workspace size in bytes for tc_path_weights on a graph with m edges. */
tc_status tc_weights_workspace_bytes(int64_t m, size_t *bytes);

/* Preprocess(delta): window metadata and S for every edge (Algorithm
 * Preprocess with Claim "count") for the class {IN, 0, OUT, 1}.
 * 0 <= delta <= 2^62.  Enqueue only; W stays on the device as S[m];
 * TC_F_OVERFLOW is set in *w->status when the exact total reaches 2^64.
 * Errors: TC_E_ARG, TC_E_WORKSPACE, TC_E_HIP. */
tc_status tc_path_weights(const tc_graph *g, int64_t delta, void *ws, size_t ws_bytes,
                          void *stream, tc_weights *w);

/* Preprocess(delta) for any anchor class (section III; the weight of a
 * class is the product of its two sides' temporal degrees over the class's
 * intervals, the remark after Claim "count").  The same workspace size as
 * tc_path_weights.  Errors: as tc_path_weights, TC_E_ARG for a bad class. */
tc_status tc_path_weights_class(const tc_graph *g, int64_t delta, const tc_class *cls, void *ws,
                                size_t ws_bytes, void *stream, tc_weights *w);

/* Workspace size in bytes for tc_path_weights_batch with n_deltas deltas
 * (1..8) on a graph with m edges.  Errors: TC_E_ARG. */
tc_status tc_weights_batch_workspace_bytes(int64_t m, int32_t n_deltas, size_t *bytes);

/* Preprocess for n_deltas deltas (host array, 1..8, each 0..2^62) of one
 * anchor class (cls NULL: {IN, 0, OUT, 1}) in one launch sequence.  w (host
 * array of n_deltas) receives the weights of deltas[i] in w[i], equal word
 * for word to what tc_path_weights_class gives for that delta; all of them
 * live in ws, which must outlive their use.  Each side's window bound at the
 * centre time does not depend on delta and is ranked once; the side-3
 * windows of all deltas reach the out-CSR order in one scatter and one
 * gather.  Enqueue only.  Errors: TC_E_ARG, TC_E_WORKSPACE, TC_E_HIP. */
tc_status tc_path_weights_batch(const tc_graph *g, const int64_t *deltas, int32_t n_deltas,
                                const tc_class *cls, void *ws, size_t ws_bytes, void *stream,
                                tc_weights *w);

/* Workspace size in bytes for tc_sample_estimate with k samples and n_motifs
 * motifs (per-sample pair windows and the closure work queue of one chunk of
 * at most 2^25 samples).  Errors: TC_E_ARG (null, k < 1, n_motifs not in
 * 1..16). */
tc_status tc_sample_workspace_bytes(uint64_t k, int32_t n_motifs, size_t *bytes);

/* Estimate(M, k) for n_motifs motifs (host array, 1..16) whose anchors have
 * w's class, the same number of edges and the same rank order of those
 * edges (TC_E_ARG otherwise): samples i0 .. i0+k-1 (k >= 1) of the
 * counter-based stream
 * (seed, stream_id).  For each sample i (Algorithm Sample, then CheckMotif):
 *   Philox4x32-10 (Salmon et al., SC 2011) with counter
 *   (i mod 2^32, i div 2^32, attempt, stream_id) and key
 *   (seed mod 2^32, seed div 2^32) gives words x0..x3 per attempt;
 *   r = floor((x0 + 2^32 x1) * W / 2^64), j1 = floor(x2 * a_p / 2^32),
 *   j3 = floor(x3 * b_p / 2^32), each taken from the first attempt that
 *   passes Lemire's rejection test (exactly uniform);
 *   p is the edge with S[p] <= r < S[p+1]; e2 = out-CSR[p] = (u, v, t2),
 *   e1 = position lo_in[p] + j1 of the in- or out-CSR (side 1's mode),
 *   e3 = position lo_out[p] + j3 likewise (an absent side: no edge, -1);
 *   x is e1's other end, y is e3's other end, phi = (x, u, v, y);
 *   X = 0 unless the anchor's vertices are distinct, its times strictly
 *   increase in rank order and its last time is at most its first + delta;
 *   otherwise X = the number of strictly increasing chains, in rank order,
 *   of times of the motif's other edges, edge r taking the times of the pair
 *   (phi(src_r), phi(dst_r)) after the anchor time ranked just below r and
 *   before the one ranked just above it, or up to the first anchor time +
 *   delta (ListCount).  For the spine motifs (ranks 0, 1, 2 = 0->1->2->3)
 *   every list is the pair's times in (t3, t1 + delta].
 * W == 0 gives cnt = hits = 0, estimate 0, e* = -1, X = 0.
 * ws (device) is scratch of at least tc_sample_workspace_bytes(k, n_motifs)
 * bytes, reused across the call's chunks; calls that share it must be
 * stream-ordered.  Errors: TC_E_ARG, TC_E_UNSUPPORTED (motif shape),
 * TC_E_WORKSPACE, TC_E_HIP. */
tc_status tc_sample_estimate(const tc_graph *g, const tc_weights *w, const tc_motif *motifs,
                             int32_t n_motifs, uint64_t k, uint64_t seed, uint32_t stream_id,
                             uint64_t i0, void *ws, size_t ws_bytes, tc_result *out,
                             void *stream);

/* Exhaustive mode (the identity in the proof of Claim "est": every match has
 * exactly one anchor, so the sum of CheckMotif over all W anchors is the
 * count C): the anchors of ranks r0 .. r0 + count - 1 of the integer CDF,
 * rank r being the centre p with S[p] <= r < S[p+1] and the window picks
 * j1 = (r - S[p]) div b[p], j3 = (r - S[p]) mod b[p]; ranks at or past W
 * contribute nothing.  Outputs as tc_sample_estimate, sample index r - r0
 * (no random numbers are drawn): cnt = sum of X (exactly C when the ranks
 * cover 0 .. W-1), hits = anchors with a match, m2 = sum of X^2, xmax = the
 * largest X -- with hits, the statistics of B, the number of matches
 * sharing one anchor (B_avg = cnt / hits, B_std from m2, B_max = xmax);
 * estimate = cnt in binary64.  ws as for tc_sample_estimate with k = count.
 * Errors: as tc_sample_estimate (count >= 1). */
tc_status tc_exhaustive_count(const tc_graph *g, const tc_weights *w, const tc_motif *motifs,
                              int32_t n_motifs, uint64_t r0, uint64_t count, void *ws,
                              size_t ws_bytes, tc_result *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * tc_sample_estimate with the same arguments and results, but no workspace
 * argument.  Its scratch is a library-owned static device array of 80 MiB,
 * one per GPU, held until the process ends; the call allocates nothing and
 * clears what must start at zero.  Calls that overlap on one GPU (several
 * streams or threads at once) share that array and race: order them.
 * It runs in chunks of 2^16 samples; a call whose scratch would exceed the
 * array returns TC_E_WORKSPACE (no valid call does: any k, 1..16 motifs).
 * Errors: as tc_sample_estimate. */
tc_status tc_sample_estimate_noalloc(const tc_graph *g, const tc_weights *w,
                                     const tc_motif *motifs, int32_t n_motifs, uint64_t k,
                                     uint64_t seed, uint32_t stream_id, uint64_t i0,
                                     tc_result *out, void *stream);

/* Batched Estimate: n_deltas (1..8) weight sets of the same graph (one per
 * delta, from tc_path_weights, tc_path_weights_class or tc_path_weights_batch)
 * and n_motifs motifs sharing the anchor, in one
 * launch sequence: the path kernel is persistent over (delta, sample tile)
 * work and every ListCount pass serves all deltas.  Sample i of every delta
 * uses the counter of sample i of a single tc_sample_estimate call with the
 * same (seed, stream_id), so out[d] equals that call's result bit for bit.
 * out is a host array of n_deltas tc_result pointers; tuning may be NULL
 * (defaults).  Enqueue only, no host synchronisation, no allocation, no
 * memset: the sequence can be captured into a HIP graph and replayed.
 * Errors: as tc_sample_estimate. */
tc_status tc_batch_workspace_bytes(uint64_t k, int32_t n_deltas, int32_t n_motifs, size_t *bytes);
tc_status tc_batch_estimate(const tc_graph *g, const tc_weights *const *w, int32_t n_deltas,
                            const tc_motif *motifs, int32_t n_motifs, uint64_t k, uint64_t seed,
                            uint32_t stream_id, uint64_t i0, const tc_tuning *tuning, void *ws,
                            size_t ws_bytes, tc_result *const *out, void *stream);

/* Autotuner: times tc_batch_estimate with k_probe samples for candidate
 * tunings (coordinate descent over chunk_log2, path_blocks, reg_waves,
 * fast_waves, wide_blocks, reg_list_cap, lds_list_cap) with HIP events on
 * `stream`, and returns the fastest in *best
 * and its time in *best_ms.  Synchronises the stream; `out` receives the
 * probe results.  ws must hold tc_batch_workspace_bytes(k_probe, ...). */
tc_status tc_autotune(const tc_graph *g, const tc_weights *const *w, int32_t n_deltas,
                      const tc_motif *motifs, int32_t n_motifs, uint64_t k_probe, uint64_t seed,
                      void *ws, size_t ws_bytes, tc_result *const *out, void *stream,
                      tc_tuning *best, double *best_ms);

/* ---- Learned importance proposal (not part of the paper) -----------------
 * The sampler draws the centre edge with probability proportional to
 * q_p = w_p * h_p instead of w_p and corrects each sample by Q / h_p, which
 * keeps the estimate unbiased for any integers h_p >= 1 (see tc_result).
 * h comes from a small network g(f_p) over per-edge window features:
 * h = eps + (1 - eps) g, quantised to integers.  The network is
 * 8 -> 64 -> 64 -> 1 (ReLU, ReLU, sigmoid), TC_MLP_PARAMS float32
 * parameters in the order W1 [64][8] (row = unit), b1 [64], W2 [64][64],
 * b2 [64], w3 [64], b3; the kernels use bfloat16 copies of the weight
 * matrices, features and hidden activations with float32 accumulation. */
#define TC_MLP_PARAMS 4801

/* Features of every scan position p (centre edge (u, v, t)) into feat
 * (device, [m][8] bfloat16 bit patterns, 16 bytes per edge, 16-byte aligned):
 *   0 ln(1+a)  1 ln(1+b)  2 ln(1+a b)  3 (t - earliest time of u's in-window)/delta
 *   4 (latest time of v's out-window - t)/delta  5 ln(1 + #u->v edges with time
 *   in [t-delta, t+delta])  6 the same for v->u  7 ln(1 + M_in M_out) / 2 with
 *   M_in the mean of min(indeg(x), 65535)^2 over u's in-window edges x -> u and
 *   M_out the mean of min(outdeg(y), 65535)^2 over v's out-window edges v -> y
 *   (0 for an empty window); 3 and 4 are 0 for an empty window or delta = 0.
 * ws holds tc_features_workspace_bytes(m) bytes of scratch (prefix sums).
 * Errors: TC_E_ARG for null pointers or a weight set of another graph,
 * TC_E_WORKSPACE. */
tc_status tc_features_workspace_bytes(int64_t m, size_t *bytes);
tc_status tc_edge_features(const tc_graph *g, const tc_weights *w, uint16_t *feat, void *ws,
                           size_t ws_bytes, void *stream);

/* g[i] = network output for feature row i, i < n (device arrays). */
tc_status tc_mlp_forward(const float *params, const uint16_t *feat, int64_t n, float *g,
                         void *stream);

/* Workspace of tc_mlp_grad for n rows and of tc_mlp_train for one batch. */
tc_status tc_mlp_workspace_bytes(int64_t n, size_t *bytes);

/* Mean binary cross-entropy (*loss, device float) and its gradient
 * (grad, device [TC_MLP_PARAMS]) over n labels: label i uses feature row
 * rows[i] of the n_feat rows of feat (rows may be NULL: row i, then
 * n <= n_feat) and the closure outcome X[i] (X device [n], e.g. per-sample
 * counts and centre positions of the method's sampler): y_i = [X[i] > 0]
 * when label_cap = 0, else the soft label min(1, X[i] / label_cap) in
 * float32.  Labels whose row is >= n_feat are ignored (they add nothing;
 * the mean still divides by n).  Deterministic for a given n.
 * Errors: TC_E_ARG (null pointers, n < 1 or n >= 2^31, label_cap < 0),
 * TC_E_WORKSPACE. */
tc_status tc_mlp_grad(const float *params, const uint16_t *feat, int64_t n_feat,
                      const uint32_t *rows, const uint64_t *X, int64_t n, float label_cap,
                      float *grad, float *loss, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for the
 * 1-based step) on params with moments opt[0..P) and opt[P..2P) (device,
 * P = TC_MLP_PARAMS; start from zeros). */
tc_status tc_mlp_adam(float *params, float *opt, const float *grad, int64_t step, float lr,
                      void *stream);

/* Minibatch training: `epochs` passes over the n labels in a Philox-drawn
 * order per epoch (seed), batches of `batch` labels, one gradient and one
 * Adam step per batch (steps numbered from step0 + 1).  loss_per_epoch
 * (device [epochs], may be NULL) receives each epoch's mean loss.
 * Enqueue only.  Errors as tc_mlp_grad; batch in [32, 2^20]. */
tc_status tc_mlp_train(float *params, float *opt, const uint16_t *feat, int64_t n_feat,
                       const uint32_t *rows, const uint64_t *X, int64_t n, float label_cap,
                       int32_t batch, int32_t epochs, float lr, uint64_t seed, int64_t step0,
                       float *loss_per_epoch, void *ws, size_t ws_bytes, void *stream);

/* h[p] = max(1, floor((eps + (1 - eps) x[p]) * 2^s + 1/2)) with
 * s = clamp(63 - bitlen(W), 1, 16), W = w->S[m], and x = g clamped to
 * [0, 1] (NaN read as 0), every operation in float32.  With g_max non-NULL
 * (a device float the call overwrites) the scores are first normalised:
 * *g_max = max_p x[p] and x[p] is replaced by x[p] / *g_max when that is
 * positive, so the factors span [eps, 1] whatever the label base rate.
 * Then W * 2^s < 2^63 when W < 2^62, so the proposal total cannot
 * overflow.  eps in (0, 1]. */
tc_status tc_quantize_proposal(const tc_weights *w, const float *g, float eps, float *g_max,
                               uint32_t *h, void *stream);

/* Proposal weight set wq from w and h (device [m], h[p] >= 1): the same
 * window arrays (borrowed from w), S = exclusive scan of q = a * b * h with
 * Q = S[m] (128-bit exact; TC_F_OVERFLOW in *wq->status if Q >= 2^64), its
 * search tree, and wq->h = h.  Pass wq to tc_sample_estimate or
 * tc_batch_estimate for the importance-sampling estimate. */
tc_status tc_proposal_workspace_bytes(int64_t m, size_t *bytes);
tc_status tc_proposal_weights(const tc_graph *g, const tc_weights *w, const uint32_t *h,
                              void *ws, size_t ws_bytes, tc_weights *wq, void *stream);

/* ---- Window proposal (not part of the paper) ------------------------------
 * Importance sampling over the side edges as well as the centre edge: every
 * entry of the in-CSR and of the out-CSR carries an integer factor
 * f >= 1, a side's window has the factor sum G (1 for an absent side), the
 * centre edge p is drawn with probability q_p / Q, q_p = h_p * G1_p * G3_p
 * (h NULL = 1), and each side's edge is the window entry j drawn with
 * probability f_j / G: a uniform integer u < G (Lemire's test on the same
 * Philox word as the uniform pick), then the entry whose prefix interval
 * holds u.  A path has probability h_p f1 f3 / Q and contributes
 * X * Q / (h_p f1 f3); cnt holds the exact 128-bit sum of
 * floor(X 2^64 / (h_p f1 f3)) and estimate = ((cnt 2^-64) / k) * Q, as for
 * tc_proposal_weights.  The product h_p f1 f3 must stay below 2^32, each G
 * below 2^32 and Q below 2^64 (TC_F_OVERFLOW otherwise: the set's status
 * with Q = 0, or the sampler's).  With all factors 1 the draws equal those of
 * the method (or of the centre proposal h) position for position.
 *
 * tc_window_factors fills f_in[i] (in-CSR position i, an edge x -> u) and
 * f_out[o] (out-CSR position o, an edge v -> y) with min(cap, F(1 + d)) of
 * the far endpoint's total degree d (in + out): F = 1, r4, r2, r2 r4 or r2^2
 * for quarter = 0..4, with r2 = floor(sqrt(1 + d)), r4 = floor(sqrt(r2)),
 * about (1 + d)^(quarter/4).  cap in 1..65535.
 * tc_proposal_window builds the set wq from w (the method's weights: no h,
 * no factors): the window arrays are borrowed from w, S, its tree, the
 * prefix sums and the status live in ws.  f_in / f_out may be NULL (factor
 * 1 for that CSR).  Errors: TC_E_ARG, TC_E_WORKSPACE, TC_E_HIP. */
tc_status tc_window_factors(const tc_graph *g, int32_t quarter, uint32_t cap, uint32_t *f_in,
                            uint32_t *f_out, void *stream);
tc_status tc_proposal_window_workspace_bytes(int64_t m, size_t *bytes);
tc_status tc_proposal_window(const tc_graph *g, const tc_weights *w, const uint32_t *h,
                             const uint32_t *f_in, const uint32_t *f_out, void *ws,
                             size_t ws_bytes, tc_weights *wq, void *stream);

/* Profiling aid (not part of the method).  After tc_timing_enable(1) the
 * library records a pair of HIP events on the launch stream around each
 * launch of its main kernels ("k_windows", "k_scan_apply", "k_paths",
 * "k_listcount_reg", "k_radix_scatter").  tc_timing_read waits for the
 * recorded events of one kernel and returns the summed elapsed milliseconds
 * and the number of launches; tc_timing_reset drops all records.  Events are
 * created only while timing is enabled.  Errors: TC_E_ARG, TC_E_HIP. */
tc_status tc_timing_enable(int32_t on);
tc_status tc_timing_reset(void);
tc_status tc_timing_read(const char *kernel, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* TC_H_ */
