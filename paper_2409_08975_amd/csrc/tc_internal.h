// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tc.h"

namespace tc {

size_t graph_workspace_bytes(int32_t n, int64_t m);
tc_status build_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                      const int64_t* t, void* ws, size_t ws_bytes, hipStream_t st, tc_graph* g);

// Shape of the 16-ary search tree over S (level 0 = S padded to 16n words;
// levels 1..levels live in tc_weights.scratch at offset[L] words).
constexpr int kMaxTreeLevels = 16;
struct STree {
  int levels;
  int64_t count[kMaxTreeLevels];
  size_t offset[kMaxTreeLevels];
  size_t total_words;
};
STree stree_layout(int64_t m);

// Several deltas share one weights or sampling launch sequence.
constexpr int kMaxDeltas = 8;

size_t weights_workspace_bytes(int64_t m);
tc_status path_weights(const tc_graph* g, int64_t delta, const tc_class& cls, void* ws,
                       size_t ws_bytes, hipStream_t st, tc_weights* w);
// nd (1..kMaxDeltas) deltas of one class in one launch sequence; w[i] is
// what path_weights gives for deltas[i]
size_t weights_batch_workspace_bytes(int64_t m, int nd);
tc_status path_weights_batch(const tc_graph* g, const int64_t* deltas, int nd,
                             const tc_class& cls, void* ws, size_t ws_bytes, hipStream_t st,
                             tc_weights* w);

// Compiled form of a batch of motifs that share the anchor's class, its
// number of edges and their rank order.  phi = (x, u, v, y) are the vertex
// slots 0..3 (u -> v the centre edge, x the other end of the side-1 edge, y
// of the side-3 edge).  Every non-anchor motif edge becomes a list over a
// window key: a pair of slots and a segment s, the times after the anchor
// edge of rank position s and before the next one (or up to the first
// anchor time + delta).  The distinct window keys of the batch are searched
// once per sample (at most 16).
constexpr int kMaxMotifs = 16;
constexpr int kMaxLists = 13;
constexpr int kMaxPairs = 16;
// A motif's first list gates it: when that window is empty its count is 0
// and its other lists are never needed.  The gate keys are therefore
// searched for every accepted path, the others only for live motifs.
struct MotifPlan {
  int32_t n_motifs;
  int32_t n_pairs;
  int32_t max_lists;
  tc_class cls;                                 // the anchor class of every motif
  int32_t n_anchor;                             // 3 (path) or 2 (wedge)
  int32_t order[3];                             // anchor edges by rank: 0 = e1, 1 = centre, 2 = e3
  uint8_t pair_a[kMaxPairs], pair_b[kMaxPairs];  // vertex slots of each window key
  uint8_t pair_seg[kMaxPairs];                  // its segment
  int32_t n_lists[kMaxMotifs];
  uint8_t list_pair[kMaxMotifs][kMaxLists];     // window key of each list
  int32_t n_gates;
  uint8_t gate_pair[kMaxPairs];                 // distinct first-list keys
  uint8_t gate_index[kMaxPairs];                // key -> its gate index, or 0xFF
  uint16_t rest_mask[kMaxMotifs];               // other keys of each motif (not gates)
};

// The anchor of one motif (the rule stated in tc.h).
struct MotifAnchor {
  tc_class cls;
  int32_t n_anchor;
  int32_t order[3];
  int32_t aedge[3];  // motif edge of e1, centre, e3 (-1 = none)
  int32_t slot[16];  // motif vertex -> slot of phi
};
bool motif_anchor(const tc_motif& M, MotifAnchor* A);
bool same_class(const tc_class& a, const tc_class& b);
extern const tc_class kSpineClass;

tc_status compile_motifs(const tc_motif* motifs, int32_t n_motifs, MotifPlan* plan);

// Several deltas share one sampling launch sequence.
typedef tc_tuning SampleTuning;
SampleTuning default_tuning();
// Workspace of sample_batch; with t == NULL, room for any tuning.
size_t sample_workspace_bytes(uint64_t k, int nd, int32_t n_motifs, const SampleTuning* t);
// With `exhaustive` the samples are the anchors of CDF ranks i0 .. i0 + k - 1
// (no random numbers) and the estimate is the count itself.
tc_status sample_batch(const tc_graph* g, const tc_weights* const* w, int nd,
                       const MotifPlan& plan, uint64_t k, uint64_t seed, uint32_t stream_id,
                       uint64_t i0, tc_result* const* out, const SampleTuning& tune, void* ws,
                       size_t ws_bytes, hipStream_t st, bool exhaustive = false);

// Proposal weights (scan of a * b * h) and the learned proposal.
size_t proposal_workspace_bytes(int64_t m);
tc_status proposal_weights(const tc_weights* w, const uint32_t* h, void* ws, size_t ws_bytes,
                           hipStream_t st, tc_weights* wq);
// Window proposal (per-entry factors over the CSRs, q = h G1 G3).
tc_status window_factors(const tc_graph* g, int quarter, uint32_t cap, uint32_t* f_in,
                         uint32_t* f_out, hipStream_t st);
size_t window_proposal_workspace_bytes(int64_t m);
tc_status proposal_window(const tc_graph* g, const tc_weights* w, const uint32_t* h,
                          const uint32_t* f_in, const uint32_t* f_out, void* ws, size_t ws_bytes,
                          hipStream_t st, tc_weights* wq);
size_t features_workspace_bytes(int64_t m);
tc_status edge_features(const tc_graph* g, const tc_weights* w, uint16_t* feat, void* ws,
                        size_t ws_bytes, hipStream_t st);
tc_status mlp_forward(const float* params, const uint16_t* feat, int64_t n, float* g,
                      hipStream_t st);
size_t mlp_workspace_bytes(int64_t batch);
tc_status mlp_grad(const float* params, const uint16_t* feat, int64_t n_feat,
                   const uint32_t* rows, const uint64_t* X, int64_t n, float label_cap,
                   float* grad, float* loss, void* ws, size_t ws_bytes, hipStream_t st);
tc_status mlp_adam(float* params, float* opt, const float* grad, int64_t step, float lr,
                   hipStream_t st);
tc_status mlp_train(float* params, float* opt, const uint16_t* feat, int64_t n_feat,
                    const uint32_t* rows, const uint64_t* X, int64_t n, float label_cap,
                    int32_t batch, int32_t epochs, float lr,
                    uint64_t seed, int64_t step0, float* loss_per_epoch, void* ws,
                    size_t ws_bytes, hipStream_t st);
tc_status quantize_proposal(const tc_weights* w, const float* g, float eps, float* gmax,
                            uint32_t* hq, hipStream_t st);

// RAII timing of one launch site (active only after tc_timing_enable(1))
class TimedLaunch {
 public:
  TimedLaunch(const char* name, hipStream_t st);
  ~TimedLaunch();

 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace tc
