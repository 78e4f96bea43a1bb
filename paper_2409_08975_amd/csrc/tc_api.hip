// extern "C" entry points declared in include/tc.h: argument checks, motif
// compilation and dispatch to the kernels of the other translation units.
#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {

tc_status compile_motifs(const tc_motif* motifs, int32_t n_motifs, MotifPlan* plan) {
  if (!motifs || n_motifs < 1 || n_motifs > kMaxMotifs) return TC_E_ARG;
  *plan = MotifPlan{};
  plan->n_motifs = n_motifs;
  for (int j = 0; j < n_motifs; ++j) {
    const tc_motif& M = motifs[j];
    if (M.nv != 4 || M.ne < 3 || M.ne > 16) return TC_E_UNSUPPORTED;
    for (int e = 0; e < M.ne; ++e)
      if (M.src[e] >= 4 || M.dst[e] >= 4 || M.src[e] == M.dst[e]) return TC_E_UNSUPPORTED;
    // anchor: ranks 0, 1, 2 form the directed 3-path 0 -> 1 -> 2 -> 3
    if (!(M.src[0] == 0 && M.dst[0] == 1 && M.src[1] == 1 && M.dst[1] == 2 && M.src[2] == 2 &&
          M.dst[2] == 3))
      return TC_E_UNSUPPORTED;
    // phi maps motif vertex 0..3 to (x, u, v, y), which are slots 0..3; each
    // later edge is a list over the pair (phi(src), phi(dst))
    plan->n_lists[j] = M.ne - 3;
    if (plan->n_lists[j] > plan->max_lists) plan->max_lists = plan->n_lists[j];
    for (int e = 3; e < M.ne; ++e) {
      int q = 0;
      while (q < plan->n_pairs &&
             !(plan->pair_a[q] == M.src[e] && plan->pair_b[q] == M.dst[e]))
        ++q;
      if (q == plan->n_pairs) {
        plan->pair_a[q] = M.src[e];
        plan->pair_b[q] = M.dst[e];
        plan->n_pairs++;
      }
      plan->list_pair[j][e - 3] = (uint8_t)q;
    }
  }
  return TC_OK;
}

}  // namespace tc

extern "C" {

const char* tc_version(void) { return "tc 0.1 gfx950"; }

tc_status tc_graph_workspace_bytes(int32_t n, int64_t m, size_t* bytes) {
  if (!bytes || n < 1 || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  *bytes = tc::graph_workspace_bytes(n, m);
  return TC_OK;
}

tc_status tc_build_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const int64_t* t, void* ws, size_t ws_bytes, void* stream, tc_graph* g) {
  if (!g || !ws || n < 1 || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  if (m > 0 && (!src || !dst || !t)) return TC_E_ARG;
  return tc::build_graph(n, m, src, dst, t, ws, ws_bytes, (hipStream_t)stream, g);
}

tc_status tc_weights_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  *bytes = tc::weights_workspace_bytes(m);
  return TC_OK;
}

tc_status tc_path_weights(const tc_graph* g, int64_t delta, void* ws, size_t ws_bytes,
                          void* stream, tc_weights* w) {
  if (!g || !w || !ws) return TC_E_ARG;
  if (delta < 0 || delta > ((int64_t)1 << 62)) return TC_E_ARG;
  return tc::path_weights(g, delta, ws, ws_bytes, (hipStream_t)stream, w);
}

tc_status tc_sample_workspace_bytes(uint64_t k, int32_t n_motifs, size_t* bytes) {
  if (!bytes || k < 1 || n_motifs < 1 || n_motifs > tc::kMaxMotifs) return TC_E_ARG;
  *bytes = tc::sample_workspace_bytes(k, n_motifs);
  return TC_OK;
}

tc_status tc_sample_estimate(const tc_graph* g, const tc_weights* w, const tc_motif* motifs,
                             int32_t n_motifs, uint64_t k, uint64_t seed, uint32_t stream_id,
                             uint64_t i0, void* ws, size_t ws_bytes, tc_result* out,
                             void* stream) {
  if (!g || !w || !out || !out->cnt || !out->hits || !out->estimate || !out->status) return TC_E_ARG;
  if (k < 1 || w->m != g->m) return TC_E_ARG;
  if ((out->e1 || out->e2 || out->e3) && !(out->e1 && out->e2 && out->e3)) return TC_E_ARG;
  tc::MotifPlan plan;
  tc_status s = tc::compile_motifs(motifs, n_motifs, &plan);
  if (s != TC_OK) return s;
  if (!ws) return TC_E_ARG;
  return tc::sample_estimate(g, w, plan, k, seed, stream_id, i0, out, ws, ws_bytes,
                             (hipStream_t)stream);
}

}  // extern "C"
