// tc_sample_estimate without a caller workspace: the sampler's scratch
// (per-sample pair windows, ListCount queues, prefix-sum scratch, per-block
// totals) lives in one file-scope device array per GPU, so the call itself
// allocates nothing.  For callers that cannot allocate device memory.
#include <hip/hip_runtime.h>

#include <mutex>

#include "tc_internal.h"

namespace tc {

// 80 MiB: the scratch of a one-delta call with 16 motifs in chunks of 2^16
// samples (pair windows 6 MiB, item queues 16 MiB, the LDS-key pass's prefix
// scratch for 1,024 wavefronts 16 MiB, the merged pass's for 32 blocks
// 32 MiB) fits with room to spare.  Each GPU the library runs on holds its
// own copy until the process ends.
constexpr size_t kNoAllocScratchBytes = (size_t)80 << 20;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

// Launch shape of the no-allocation call: chunks of 2^16 samples per delta
// and narrower ListCount passes, so that the scratch above is enough for
// any k and up to 16 motifs.  Results never depend on the launch shape.
static SampleTuning noalloc_tuning() {
  SampleTuning t = default_tuning();
  t.chunk_log2 = 16;
  t.fast_waves = 1024;
  t.wide_blocks = 32;
  return t;
}

// Device address of `scratch` on each device, looked up once per device
// with that device current (the array's name is only a host-side stand-in).
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

static tc_status scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return TC_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TC_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TC_OK;
}

}  // namespace tc

extern "C" tc_status tc_sample_estimate_noalloc(const tc_graph* g, const tc_weights* w,
                                                const tc_motif* motifs, int32_t n_motifs,
                                                uint64_t k, uint64_t seed, uint32_t stream_id,
                                                uint64_t i0, tc_result* out, void* stream) {
  if (!g || !w || !out || !out->cnt || !out->hits || !out->estimate || !out->status)
    return TC_E_ARG;
  if ((out->e1 || out->e2 || out->e3) && !(out->e1 && out->e2 && out->e3)) return TC_E_ARG;
  if (k < 1 || w->m != g->m) return TC_E_ARG;
  tc::MotifPlan plan;
  const tc_status s = tc::compile_motifs(motifs, n_motifs, &plan);
  if (s != TC_OK) return s;
  if (!tc::same_class(plan.cls, w->cls)) return TC_E_ARG;
  const tc::SampleTuning tune = tc::noalloc_tuning();
  if (tc::sample_workspace_bytes(k, 1, n_motifs, &tune) > tc::kNoAllocScratchBytes)
    return TC_E_WORKSPACE;
  void* ws = nullptr;
  const tc_status a = tc::scratch_address(&ws);
  if (a != TC_OK) return a;
  const tc_weights* wl[1] = {w};
  tc_result* ol[1] = {out};
  return tc::sample_batch(g, wl, 1, plan, k, seed, stream_id, i0, ol, tune, ws,
                          tc::kNoAllocScratchBytes, (hipStream_t)stream);
}
