// Drives the library's host-side code (argument checks, workspace queries,
// the motif compiler) through the C ABI with random and invalid arguments,
// for a build whose host code carries AddressSanitizer and
// UndefinedBehaviorSanitizer.  Every call here returns before any GPU work.
#include <cstdint>
#include <cstdio>

#include "../../include/tc.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next() {
  rng_state ^= rng_state << 13;
  rng_state ^= rng_state >> 7;
  rng_state ^= rng_state << 17;
  return rng_state;
}

int main() {
  int bad = 0;
  size_t bytes = 0;
  if (tc_graph_workspace_bytes(1000, 20000, &bytes) != TC_OK || bytes == 0) ++bad;
  if (tc_graph_workspace_bytes(0, 10, &bytes) != TC_E_ARG) ++bad;
  if (tc_weights_workspace_bytes(-1, &bytes) != TC_E_ARG) ++bad;
  if (tc_sample_workspace_bytes(0, 1, &bytes) != TC_E_ARG) ++bad;
  if (tc_batch_workspace_bytes(10, 9, 1, &bytes) != TC_E_ARG) ++bad;
  int anchored = 0;
  for (int i = 0; i < 20000; ++i) {
    tc_motif M{};
    M.nv = (uint8_t)(2 + next() % 4);   // 2..5: some unsupported
    M.ne = (uint8_t)(next() % 18);      // 0..17: some out of range
    for (int e = 0; e < 16; ++e) {
      M.src[e] = (uint8_t)(next() % 6);
      M.dst[e] = (uint8_t)(next() % 6);
    }
    tc_class c;
    int32_t na, order[3];
    const tc_status s = tc_motif_anchor(&M, &c, &na, order);
    if (s == TC_OK) {
      ++anchored;
      if (na < 2 || na > 3) ++bad;
    } else if (s != TC_E_UNSUPPORTED) {
      ++bad;
    }
  }
  // host-checkable errors: nothing is enqueued
  tc_graph g{};
  tc_weights w{};
  g.m = w.m = 10;
  tc_result r{};
  tc_motif M{};
  M.nv = 4;
  M.ne = 4;
  const uint8_t s4[4] = {0, 1, 2, 3}, d4[4] = {1, 2, 3, 0};
  for (int e = 0; e < 4; ++e) { M.src[e] = s4[e]; M.dst[e] = d4[e]; }
  if (tc_build_graph(0, 1, nullptr, nullptr, nullptr, nullptr, 0, nullptr, &g) != TC_E_ARG) ++bad;
  if (tc_path_weights(&g, -1, (void*)1, 0, nullptr, &w) != TC_E_ARG) ++bad;
  if (tc_sample_estimate(&g, &w, &M, 1, 10, 1, 0, 0, (void*)256, 1, &r, nullptr) != TC_E_ARG) ++bad;
  if (tc_exhaustive_count(&g, &w, &M, 1, 0, 0, (void*)256, 1, &r, nullptr) != TC_E_ARG) ++bad;
  tc_class cz{0, 0, 0, 0};
  if (tc_path_weights_class(&g, 5, &cz, (void*)1, 0, nullptr, &w) != TC_E_ARG) ++bad;
  // batched Preprocess: sizes and host errors
  size_t b1 = 0, b2 = 0;
  if (tc_weights_batch_workspace_bytes(1000, 1, &b1) != TC_OK) ++bad;
  if (tc_weights_batch_workspace_bytes(1000, 2, &b2) != TC_OK || b2 <= b1) ++bad;
  if (tc_weights_batch_workspace_bytes(1000, 9, &b2) != TC_E_ARG) ++bad;
  tc_weights wb[8];
  const int64_t ds[3] = {5, -1, 7};
  if (tc_path_weights_batch(&g, ds, 3, nullptr, (void*)256, (size_t)1 << 40, nullptr, wb) !=
      TC_E_ARG)
    ++bad;
  if (tc_path_weights_batch(&g, ds, 1, &cz, (void*)256, (size_t)1 << 40, nullptr, wb) != TC_E_ARG)
    ++bad;
  if (tc_path_weights_batch(&g, ds, 1, nullptr, (void*)256, 16, nullptr, wb) != TC_E_WORKSPACE)
    ++bad;
  std::printf("abi driver: %d anchored random motifs, %d failures\n", anchored, bad);
  return bad == 0 && anchored > 0 ? 0 : 1;
}
