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

size_t weights_workspace_bytes(int64_t m);
tc_status path_weights(const tc_graph* g, int64_t delta, void* ws, size_t ws_bytes,
                       hipStream_t st, tc_weights* w);

// Compiled form of a batch of motifs that share the anchor 0->1->2->3:
// for motif j, ranks 3..ne-1 become lists over vertex slots of
// phi = (x, u, v, y).
constexpr int kMaxMotifs = 16;
constexpr int kMaxLists = 13;
struct MotifPlan {
  int32_t n_motifs;
  int32_t n_lists[kMaxMotifs];
  uint8_t a_slot[kMaxMotifs][kMaxLists];
  uint8_t b_slot[kMaxMotifs][kMaxLists];
};

tc_status compile_motifs(const tc_motif* motifs, int32_t n_motifs, MotifPlan* plan);

tc_status sample_estimate(const tc_graph* g, const tc_weights* w, const MotifPlan& plan,
                          uint64_t k, uint64_t seed, uint32_t stream_id, uint64_t i0,
                          tc_result* out, hipStream_t st);

}  // namespace tc
