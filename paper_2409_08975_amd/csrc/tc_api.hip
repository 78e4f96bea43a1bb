// extern "C" entry points declared in include/tc.h: argument checks, motif
// compilation and dispatch to the kernels of the other translation units.
#include <hip/hip_runtime.h>

#include "tc_internal.h"

namespace tc {

const tc_class kSpineClass = {TC_SIDE_IN, 0, TC_SIDE_OUT, 1};

bool same_class(const tc_class& a, const tc_class& b) {
  if (a.mode1 != b.mode1 || a.mode3 != b.mode3) return false;
  // the window's direction only: a window open at the centre time serves
  // the same anchors
  if (a.mode1 != TC_SIDE_NONE && (a.after1 & 1) != (b.after1 & 1)) return false;
  if (a.mode3 != TC_SIDE_NONE && (a.after3 & 1) != (b.after3 & 1)) return false;
  return true;
}

// The anchor rule of tc.h: candidates hold rank 0 (edge index 0); the best
// has the smallest sorted ranks, then the smallest centre rank, then (paths)
// the smallest rank of the edge at u.
bool motif_anchor(const tc_motif& M, MotifAnchor* A) {
  const int ne = M.ne;
  auto meets = [&](int e, int vtx) { return M.src[e] == vtx || M.dst[e] == vtx; };
  auto far_end = [&](int e, int vtx) { return M.src[e] == vtx ? (int)M.dst[e] : (int)M.src[e]; };
  uint32_t best = 0xFFFFFFFFu;
  int e1b = -1, cb = -1, e3b = -1;
  for (int c = 0; c < ne; ++c) {
    const int U = M.src[c], V = M.dst[c];
    if (M.nv == 4) {
      for (int e1 = 0; e1 < ne; ++e1) {
        if (e1 == c || !meets(e1, U) || meets(e1, V)) continue;
        for (int e3 = 0; e3 < ne; ++e3) {
          if (e3 == c || e3 == e1 || !meets(e3, V) || meets(e3, U)) continue;
          if (far_end(e3, V) == far_end(e1, U)) continue;
          if (c != 0 && e1 != 0 && e3 != 0) continue;
          int r0 = e1, r1 = c, r2 = e3, tmp;
          if (r0 > r1) { tmp = r0; r0 = r1; r1 = tmp; }
          if (r1 > r2) { tmp = r1; r1 = r2; r2 = tmp; }
          if (r0 > r1) { tmp = r0; r0 = r1; r1 = tmp; }
          const uint32_t key = ((((uint32_t)r0 * 16 + r1) * 16 + r2) * 16 + c) * 16 + e1;
          if (key < best) { best = key; e1b = e1; cb = c; e3b = e3; }
        }
      }
    } else if (M.nv == 3) {
      for (int e = 0; e < ne; ++e) {
        if (e == c || meets(e, U) == meets(e, V)) continue;
        if (c != 0 && e != 0) continue;
        const uint32_t lo = c < e ? c : e, hi = c < e ? e : c;
        const uint32_t key = (lo * 16 + hi) * 16 + c;
        if (key < best) {
          best = key;
          cb = c;
          e1b = meets(e, U) ? e : -1;
          e3b = meets(e, U) ? -1 : e;
        }
      }
    }
  }
  if (cb < 0) return false;
  const int U = M.src[cb], V = M.dst[cb];
  for (int i = 0; i < 16; ++i) A->slot[i] = -1;
  A->slot[U] = 1;
  A->slot[V] = 2;
  A->aedge[0] = e1b;
  A->aedge[1] = cb;
  A->aedge[2] = e3b;
  A->n_anchor = 1;
  A->cls = tc_class{TC_SIDE_NONE, 0, TC_SIDE_NONE, 0};
  if (e1b >= 0) {
    ++A->n_anchor;
    A->cls.mode1 = M.dst[e1b] == U ? TC_SIDE_IN : TC_SIDE_OUT;
    A->cls.after1 = e1b > cb ? 1 : 0;
    A->slot[far_end(e1b, U)] = 0;
  }
  if (e3b >= 0) {
    ++A->n_anchor;
    A->cls.mode3 = M.dst[e3b] == V ? TC_SIDE_IN : TC_SIDE_OUT;
    A->cls.after3 = e3b > cb ? 1 : 0;
    A->slot[far_end(e3b, V)] = 3;
  }
  for (int vtx = 0; vtx < M.nv; ++vtx)
    if (A->slot[vtx] < 0) return false;
  int k = 0;
  for (int r = 0; r < ne; ++r)
    for (int i = 0; i < 3; ++i)
      if (A->aedge[i] == r) A->order[k++] = i;
  for (; k < 3; ++k) A->order[k] = -1;
  return true;
}

tc_status compile_motifs(const tc_motif* motifs, int32_t n_motifs, MotifPlan* plan) {
  if (!motifs || n_motifs < 1 || n_motifs > kMaxMotifs) return TC_E_ARG;
  *plan = MotifPlan{};
  plan->n_motifs = n_motifs;
  for (int j = 0; j < n_motifs; ++j) {
    const tc_motif& M = motifs[j];
    if (M.nv < 3 || M.nv > 4 || M.ne < 2 || M.ne > 16) return TC_E_UNSUPPORTED;
    for (int e = 0; e < M.ne; ++e)
      if (M.src[e] >= M.nv || M.dst[e] >= M.nv || M.src[e] == M.dst[e]) return TC_E_UNSUPPORTED;
    MotifAnchor A;
    if (!motif_anchor(M, &A)) return TC_E_UNSUPPORTED;
    // every motif of one call samples the same anchors
    if (j == 0) {
      plan->cls = A.cls;
      plan->n_anchor = A.n_anchor;
      for (int i = 0; i < 3; ++i) plan->order[i] = A.order[i];
    } else {
      if (!same_class(A.cls, plan->cls) || A.n_anchor != plan->n_anchor) return TC_E_ARG;
      for (int i = 0; i < A.n_anchor; ++i)
        if (A.order[i] != plan->order[i]) return TC_E_ARG;
    }
    // each later edge is a list over a window key (slot pair, segment)
    int nl = 0;
    for (int r = 0; r < M.ne; ++r) {
      if (r == A.aedge[0] || r == A.aedge[1] || r == A.aedge[2]) continue;
      int below = 0;
      for (int i = 0; i < 3; ++i)
        if (A.aedge[i] >= 0 && A.aedge[i] < r) ++below;
      const uint8_t sa = (uint8_t)A.slot[M.src[r]], sb = (uint8_t)A.slot[M.dst[r]];
      const uint8_t seg = (uint8_t)(below - 1);
      int q = 0;
      while (q < plan->n_pairs &&
             !(plan->pair_a[q] == sa && plan->pair_b[q] == sb && plan->pair_seg[q] == seg))
        ++q;
      if (q == plan->n_pairs) {
        if (plan->n_pairs == kMaxPairs) return TC_E_UNSUPPORTED;
        plan->pair_a[q] = sa;
        plan->pair_b[q] = sb;
        plan->pair_seg[q] = seg;
        plan->n_pairs++;
      }
      plan->list_pair[j][nl++] = (uint8_t)q;
    }
    plan->n_lists[j] = nl;
    if (nl > plan->max_lists) plan->max_lists = nl;
  }
  uint32_t gate_mask = 0;
  for (int j = 0; j < n_motifs; ++j)
    if (plan->n_lists[j] >= 1) gate_mask |= 1u << plan->list_pair[j][0];
  for (int q = 0; q < kMaxPairs; ++q) plan->gate_index[q] = 0xFF;
  for (int q = 0; q < plan->n_pairs; ++q)
    if (gate_mask & (1u << q)) {
      plan->gate_index[q] = (uint8_t)plan->n_gates;
      plan->gate_pair[plan->n_gates++] = (uint8_t)q;
    }
  for (int j = 0; j < n_motifs; ++j) {
    uint32_t mk = 0;
    for (int r = 1; r < plan->n_lists[j]; ++r) mk |= 1u << plan->list_pair[j][r];
    plan->rest_mask[j] = (uint16_t)(mk & ~gate_mask);
  }
  return TC_OK;
}

}  // namespace tc

extern "C" {

const char* tc_version(void) { return "tc 0.2 gfx950"; }

// a workspace: present and 256-byte aligned (the 64-bit atomics and 16-byte
// records inside it are laid out at 256-byte offsets from its start)
static bool ws_ok(const void* ws) { return ws && ((uintptr_t)ws & 255u) == 0; }

tc_status tc_graph_workspace_bytes(int32_t n, int64_t m, size_t* bytes) {
  if (!bytes || n < 1 || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  *bytes = tc::graph_workspace_bytes(n, m);
  return TC_OK;
}

tc_status tc_build_graph(int32_t n, int64_t m, const int32_t* src, const int32_t* dst,
                         const int64_t* t, void* ws, size_t ws_bytes, void* stream, tc_graph* g) {
  if (!g || !ws_ok(ws) || n < 1 || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  if (m > 0 && (!src || !dst || !t)) return TC_E_ARG;
  return tc::build_graph(n, m, src, dst, t, ws, ws_bytes, (hipStream_t)stream, g);
}

static bool class_ok(const tc_class* cls) {
  return cls->mode1 <= TC_SIDE_OUT && cls->mode3 <= TC_SIDE_OUT && cls->after1 <= 3 &&
         cls->after3 <= 3 && !(cls->mode1 == TC_SIDE_NONE && cls->mode3 == TC_SIDE_NONE);
}

tc_status tc_weights_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  *bytes = tc::weights_workspace_bytes(m);
  return TC_OK;
}

tc_status tc_path_weights(const tc_graph* g, int64_t delta, void* ws, size_t ws_bytes,
                          void* stream, tc_weights* w) {
  if (!g || !w || !ws_ok(ws)) return TC_E_ARG;
  if (delta < 0 || delta > ((int64_t)1 << 62)) return TC_E_ARG;
  return tc::path_weights(g, delta, tc::kSpineClass, ws, ws_bytes, (hipStream_t)stream, w);
}

tc_status tc_path_weights_class(const tc_graph* g, int64_t delta, const tc_class* cls, void* ws,
                                size_t ws_bytes, void* stream, tc_weights* w) {
  if (!g || !w || !ws_ok(ws) || !cls) return TC_E_ARG;
  if (delta < 0 || delta > ((int64_t)1 << 62)) return TC_E_ARG;
  if (!class_ok(cls)) return TC_E_ARG;
  return tc::path_weights(g, delta, *cls, ws, ws_bytes, (hipStream_t)stream, w);
}

tc_status tc_weights_batch_workspace_bytes(int64_t m, int32_t n_deltas, size_t* bytes) {
  if (!bytes || m < 0 || m >= ((int64_t)1 << 31) || n_deltas < 1 || n_deltas > tc::kMaxDeltas)
    return TC_E_ARG;
  *bytes = tc::weights_batch_workspace_bytes(m, n_deltas);
  return TC_OK;
}

tc_status tc_path_weights_batch(const tc_graph* g, const int64_t* deltas, int32_t n_deltas,
                                const tc_class* cls, void* ws, size_t ws_bytes, void* stream,
                                tc_weights* w) {
  if (!g || !deltas || !w || !ws_ok(ws)) return TC_E_ARG;
  if (n_deltas < 1 || n_deltas > tc::kMaxDeltas) return TC_E_ARG;
  for (int i = 0; i < n_deltas; ++i)
    if (deltas[i] < 0 || deltas[i] > ((int64_t)1 << 62)) return TC_E_ARG;
  if (cls && !class_ok(cls)) return TC_E_ARG;
  return tc::path_weights_batch(g, deltas, n_deltas, cls ? *cls : tc::kSpineClass, ws, ws_bytes,
                                (hipStream_t)stream, w);
}

tc_status tc_motif_anchor(const tc_motif* motif, tc_class* cls, int32_t* n_anchor,
                          int32_t* order) {
  if (!motif || !cls || !n_anchor || !order) return TC_E_ARG;
  const tc_motif& M = *motif;
  if (M.nv < 3 || M.nv > 4 || M.ne < 2 || M.ne > 16) return TC_E_UNSUPPORTED;
  for (int e = 0; e < M.ne; ++e)
    if (M.src[e] >= M.nv || M.dst[e] >= M.nv || M.src[e] == M.dst[e]) return TC_E_UNSUPPORTED;
  tc::MotifAnchor A;
  if (!tc::motif_anchor(M, &A)) return TC_E_UNSUPPORTED;
  *cls = A.cls;
  *n_anchor = A.n_anchor;
  for (int i = 0; i < 3; ++i) order[i] = A.order[i];
  return TC_OK;
}

tc_status tc_sample_workspace_bytes(uint64_t k, int32_t n_motifs, size_t* bytes) {
  if (!bytes || k < 1 || n_motifs < 1 || n_motifs > tc::kMaxMotifs) return TC_E_ARG;
  *bytes = tc::sample_workspace_bytes(k, 1, n_motifs, nullptr);
  return TC_OK;
}

tc_status tc_batch_workspace_bytes(uint64_t k, int32_t n_deltas, int32_t n_motifs, size_t* bytes) {
  if (!bytes || k < 1 || n_motifs < 1 || n_motifs > tc::kMaxMotifs || n_deltas < 1 ||
      n_deltas > tc::kMaxDeltas)
    return TC_E_ARG;
  *bytes = tc::sample_workspace_bytes(k, n_deltas, n_motifs, nullptr);
  return TC_OK;
}

static tc_status check_result(const tc_result* out) {
  if (!out || !out->cnt || !out->hits || !out->estimate || !out->status) return TC_E_ARG;
  if ((out->e1 || out->e2 || out->e3) && !(out->e1 && out->e2 && out->e3)) return TC_E_ARG;
  return TC_OK;
}

tc_status tc_batch_estimate(const tc_graph* g, const tc_weights* const* w, int32_t n_deltas,
                            const tc_motif* motifs, int32_t n_motifs, uint64_t k, uint64_t seed,
                            uint32_t stream_id, uint64_t i0, const tc_tuning* tuning, void* ws,
                            size_t ws_bytes, tc_result* const* out, void* stream) {
  if (!g || !w || !out || k < 1 || n_deltas < 1 || n_deltas > tc::kMaxDeltas) return TC_E_ARG;
  for (int d = 0; d < n_deltas; ++d) {
    if (!w[d] || w[d]->m != g->m) return TC_E_ARG;
    if (check_result(out[d]) != TC_OK) return TC_E_ARG;
  }
  tc::MotifPlan plan;
  tc_status s = tc::compile_motifs(motifs, n_motifs, &plan);
  if (s != TC_OK) return s;
  for (int d = 0; d < n_deltas; ++d)
    if (!tc::same_class(plan.cls, w[d]->cls)) return TC_E_ARG;
  if (!ws_ok(ws)) return TC_E_ARG;
  const tc::SampleTuning t = tuning ? *tuning : tc::default_tuning();
  return tc::sample_batch(g, w, n_deltas, plan, k, seed, stream_id, i0, out, t, ws, ws_bytes,
                          (hipStream_t)stream);
}

tc_status tc_sample_estimate(const tc_graph* g, const tc_weights* w, const tc_motif* motifs,
                             int32_t n_motifs, uint64_t k, uint64_t seed, uint32_t stream_id,
                             uint64_t i0, void* ws, size_t ws_bytes, tc_result* out,
                             void* stream) {
  if (!g || !w || check_result(out) != TC_OK) return TC_E_ARG;
  if (k < 1 || w->m != g->m) return TC_E_ARG;
  tc::MotifPlan plan;
  tc_status s = tc::compile_motifs(motifs, n_motifs, &plan);
  if (s != TC_OK) return s;
  if (!tc::same_class(plan.cls, w->cls)) return TC_E_ARG;
  if (!ws_ok(ws)) return TC_E_ARG;
  const tc_weights* wl[1] = {w};
  tc_result* ol[1] = {out};
  return tc::sample_batch(g, wl, 1, plan, k, seed, stream_id, i0, ol, tc::default_tuning(), ws,
                          ws_bytes, (hipStream_t)stream);
}

tc_status tc_exhaustive_count(const tc_graph* g, const tc_weights* w, const tc_motif* motifs,
                              int32_t n_motifs, uint64_t r0, uint64_t count, void* ws,
                              size_t ws_bytes, tc_result* out, void* stream) {
  if (!g || !w || check_result(out) != TC_OK) return TC_E_ARG;
  if (count < 1 || w->m != g->m || w->h || w->ps1 || w->ps3) return TC_E_ARG;
  tc::MotifPlan plan;
  tc_status s = tc::compile_motifs(motifs, n_motifs, &plan);
  if (s != TC_OK) return s;
  if (!tc::same_class(plan.cls, w->cls)) return TC_E_ARG;
  if (!ws_ok(ws)) return TC_E_ARG;
  const tc_weights* wl[1] = {w};
  tc_result* ol[1] = {out};
  return tc::sample_batch(g, wl, 1, plan, count, 0, 0, r0, ol, tc::default_tuning(), ws, ws_bytes,
                          (hipStream_t)stream, true);
}

tc_status tc_autotune(const tc_graph* g, const tc_weights* const* w, int32_t n_deltas,
                      const tc_motif* motifs, int32_t n_motifs, uint64_t k_probe, uint64_t seed,
                      void* ws, size_t ws_bytes, tc_result* const* out, void* stream,
                      tc_tuning* best, double* best_ms) {
  if (!best || !best_ms) return TC_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TC_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return TC_E_HIP;
  }
  auto run = [&](const tc_tuning& t, double* ms) -> tc_status {
    tc_status s = tc_batch_estimate(g, w, n_deltas, motifs, n_motifs, k_probe, seed, 0, 0, &t,
                                    ws, ws_bytes, out, stream);
    if (s != TC_OK) return s;  // warm
    if (hipEventRecord(e0, st) != hipSuccess) return TC_E_HIP;
    s = tc_batch_estimate(g, w, n_deltas, motifs, n_motifs, k_probe, seed, 0, 0, &t, ws,
                          ws_bytes, out, stream);
    if (s != TC_OK) return s;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
      return TC_E_HIP;
    float f = 0.f;
    if (hipEventElapsedTime(&f, e0, e1) != hipSuccess) return TC_E_HIP;
    *ms = f;
    return TC_OK;
  };
  tc_tuning cur = tc::default_tuning();
  double cur_ms = 0;
  tc_status s = run(cur, &cur_ms);
  // candidate values per knob (a knob with fewer repeats its last one)
  const int32_t cand[7][3] = {
      {23, 24, 25},         // chunk_log2
      {0, 1024, 4096},      // path_blocks
      {20480, 40960, 81920}, // reg_waves
      {2560, 5120, 8192},   // fast_waves
      {1024, 2048, 4096},   // wide_blocks
      {128, 256, 256},      // reg_list_cap: lanes hold 2 or 4 list entries
      {256, 512, 1024},     // lds_list_cap: 64 lanes per item up to it, 256 above
  };
  for (int dim = 0; dim < 7 && s == TC_OK; ++dim) {
    for (int c = 0; c < 3 && s == TC_OK; ++c) {
      if (c > 0 && cand[dim][c] == cand[dim][c - 1]) continue;
      tc_tuning t = cur;
      if (dim == 0) t.chunk_log2 = cand[dim][c];
      if (dim == 1) t.path_blocks = cand[dim][c];
      if (dim == 2) t.reg_waves = cand[dim][c];
      if (dim == 3) t.fast_waves = cand[dim][c];
      if (dim == 4) t.wide_blocks = cand[dim][c];
      if (dim == 5) t.reg_list_cap = cand[dim][c];
      if (dim == 6) t.lds_list_cap = cand[dim][c];
      double ms = 0;
      s = run(t, &ms);
      if (s == TC_OK && ms < cur_ms) {
        cur = t;
        cur_ms = ms;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != TC_OK) return s;
  *best = cur;
  *best_ms = cur_ms;
  return TC_OK;
}

static bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }
static const int64_t kMaxLabels = (int64_t)1 << 31;

tc_status tc_features_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0) return TC_E_ARG;
  *bytes = tc::features_workspace_bytes(m);
  return TC_OK;
}

tc_status tc_edge_features(const tc_graph* g, const tc_weights* w, uint16_t* feat, void* ws,
                           size_t ws_bytes, void* stream) {
  if (!g || !w || !feat || !ws_ok(ws) || w->m != g->m || !aligned16(feat)) return TC_E_ARG;
  if (!tc::same_class(w->cls, tc::kSpineClass)) return TC_E_UNSUPPORTED;
  return tc::edge_features(g, w, feat, ws, ws_bytes, (hipStream_t)stream);
}

tc_status tc_mlp_forward(const float* params, const uint16_t* feat, int64_t n, float* g,
                         void* stream) {
  if (!params || n < 0 || (n > 0 && (!feat || !g || !aligned16(feat)))) return TC_E_ARG;
  return tc::mlp_forward(params, feat, n, g, (hipStream_t)stream);
}

tc_status tc_mlp_workspace_bytes(int64_t n, size_t* bytes) {
  if (!bytes || n < 1 || n >= kMaxLabels) return TC_E_ARG;
  *bytes = tc::mlp_workspace_bytes(n);
  return TC_OK;
}

tc_status tc_mlp_grad(const float* params, const uint16_t* feat, int64_t n_feat,
                      const uint32_t* rows, const uint64_t* X, int64_t n, float label_cap,
                      float* grad, float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !feat || !X || !grad || !loss || !ws_ok(ws) || n < 1 || n >= kMaxLabels ||
      n_feat < 1 || (!rows && n > n_feat) || !aligned16(feat) || !(label_cap >= 0.0f))
    return TC_E_ARG;
  return tc::mlp_grad(params, feat, n_feat, rows, X, n, label_cap, grad, loss, ws, ws_bytes,
                      (hipStream_t)stream);
}

tc_status tc_mlp_adam(float* params, float* opt, const float* grad, int64_t step, float lr,
                      void* stream) {
  if (!params || !opt || !grad || step < 1) return TC_E_ARG;
  return tc::mlp_adam(params, opt, grad, step, lr, (hipStream_t)stream);
}

tc_status tc_mlp_train(float* params, float* opt, const uint16_t* feat, int64_t n_feat,
                       const uint32_t* rows, const uint64_t* X, int64_t n, float label_cap,
                       int32_t batch, int32_t epochs, float lr, uint64_t seed, int64_t step0,
                       float* loss_per_epoch, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !opt || !feat || !X || !ws_ok(ws) || n < 1 || n >= kMaxLabels || n_feat < 1 ||
      (!rows && n > n_feat) || batch < 32 || batch > (1 << 20) || epochs < 1 || step0 < 0 ||
      !aligned16(feat) || !(label_cap >= 0.0f))
    return TC_E_ARG;
  return tc::mlp_train(params, opt, feat, n_feat, rows, X, n, label_cap, batch, epochs, lr,
                       seed, step0, loss_per_epoch, ws, ws_bytes, (hipStream_t)stream);
}

tc_status tc_quantize_proposal(const tc_weights* w, const float* g, float eps, float* g_max,
                               uint32_t* h, void* stream) {
  if (!w || !g || !h || !(eps > 0.0f && eps <= 1.0f)) return TC_E_ARG;
  return tc::quantize_proposal(w, g, eps, g_max, h, (hipStream_t)stream);
}

tc_status tc_proposal_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0) return TC_E_ARG;
  *bytes = tc::proposal_workspace_bytes(m);
  return TC_OK;
}

tc_status tc_proposal_weights(const tc_graph* g, const tc_weights* w, const uint32_t* h,
                              void* ws, size_t ws_bytes, tc_weights* wq, void* stream) {
  if (!g || !w || !h || !ws_ok(ws) || !wq || w->m != g->m || w->h || w->ps1 || w->ps3 ||
      !aligned16(h))
    return TC_E_ARG;
  return tc::proposal_weights(w, h, ws, ws_bytes, (hipStream_t)stream, wq);
}

tc_status tc_window_factors(const tc_graph* g, int32_t quarter, uint32_t cap, uint32_t* f_in,
                            uint32_t* f_out, void* stream) {
  if (!g || !f_in || !f_out || quarter < 0 || quarter > 4 || cap < 1 || cap > 65535)
    return TC_E_ARG;
  return tc::window_factors(g, quarter, cap, f_in, f_out, (hipStream_t)stream);
}

tc_status tc_proposal_window_workspace_bytes(int64_t m, size_t* bytes) {
  if (!bytes || m < 0 || m >= ((int64_t)1 << 31)) return TC_E_ARG;
  *bytes = tc::window_proposal_workspace_bytes(m);
  return TC_OK;
}

tc_status tc_proposal_window(const tc_graph* g, const tc_weights* w, const uint32_t* h,
                             const uint32_t* f_in, const uint32_t* f_out, void* ws,
                             size_t ws_bytes, tc_weights* wq, void* stream) {
  if (!g || !w || !ws_ok(ws) || !wq || w->m != g->m || w->h || w->ps1 || w->ps3) return TC_E_ARG;
  return tc::proposal_window(g, w, h, f_in, f_out, ws, ws_bytes, (hipStream_t)stream, wq);
}

}  // extern "C"
