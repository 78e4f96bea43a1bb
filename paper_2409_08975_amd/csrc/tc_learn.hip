// Learned importance proposal (an extension: the paper samples the centre
// edge with probability w_e / W; here with q_e / Q, q_e = w_e * h_e, and
// corrects each sample by Q / h_e, which keeps the estimate unbiased for any
// h >= 1).
//
//   k_features     per scan position p, eight window features of the centre
//                  edge (sizes of its in- and out-windows and of the path
//                  weight, the spans of the two windows relative to delta,
//                  the multi-edge counts of (u, v) and (v, u) around t, and
//                  the mean squared degree of the windows' far endpoints from
//                  prefix sums, k_deg2_*), stored as bfloat16.
//   k_mlp_forward  g = sigmoid(w3 . relu(W2 relu(W1 f + b1) + b2) + b3) for
//                  32 edges per wavefront: both hidden layers on MFMA
//                  (bfloat16 operands, float32 accumulation).  The
//                  accumulator layout of one layer is fed to the next as its
//                  B operand without a trip through LDS: within one MFMA the
//                  order of the contraction index is free, so the weights are
//                  loaded in the order in which each lane holds the
//                  activations.
//   k_mlp_grad     mean binary cross-entropy against y = [X > 0] (or the
//                  soft label min(1, X / cap)) and its
//                  gradient, per block (fixed row-to-block assignment):
//                  the same forward, dH1 = W2^T dZ2 on MFMA from registers,
//                  and the weight gradients dW2 = dZ2 H1^T and
//                  [dW1 | db1] = dZ1 [F | 1]^T on MFMA after an LDS
//                  transpose that puts edges on the contraction index.
//   k_mlp_reduce   sums the block partials in block order (deterministic),
//                  then either stores the gradient or takes an Adam step.
//   k_quantize     h_int = max(1, floor((eps + (1 - eps) g) 2^s + 1/2)),
//                  s = clamp(63 - bitlen(W), 1, 16), in float32 with no
//                  contraction, so the integer decision is reproducible;
//                  optionally g is first divided by its maximum over the
//                  edges (k_score_max), so that the scores span [0, 1].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "tc_device.h"
#include "tc_internal.h"

namespace tc {

// parameter vector: W1 [64][8], b1 [64], W2 [64][64], b2 [64], w3 [64], b3
constexpr int kIn = 8, kHid = 64;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kNParams = kOffB3 + 1;  // 4801
static_assert(kNParams == TC_MLP_PARAMS, "parameter count");

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// bfloat16 bits of a float, round to nearest even (NaN stays NaN)
// bfloat16 rounded to nearest even (the conversion instruction; single
// precision denormals are kept, so it agrees with the rounding rule on every
// value but NaN), NaN made quiet keeping its top bits; a select, not a
// branch, so a wavefront never splits here
__device__ __forceinline__ uint16_t bf16_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  const uint16_t rne = __builtin_bit_cast(uint16_t, (__bf16)f);
  return (u & 0x7FFFFFFFu) > 0x7F800000u ? (uint16_t)((u >> 16) | 0x40u) : rne;
}
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// two values that cannot be NaN (outputs of a ReLU), rounded to nearest even
// in one instruction: a in the low half, b in the high half
__device__ __forceinline__ uint32_t bf16x2_bits(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}
__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bf16_round(float f) { return bf16_val(bf16_bits(f)); }

// Row (within a 32-row block) of accumulator register v of a lane in half h
// (h = lane / 32) for the 32x32 MFMA output layout; the column is lane % 32.
__device__ __forceinline__ int drow(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

// Row of the input held at position s (0..7) of K-chunk kc = 2 * rb + c by a
// lane in half h, when a layer's output block rb feeds the next layer.
__device__ __forceinline__ int krow(int kc, int s, int h) {
  return 32 * (kc >> 1) + drow(8 * (kc & 1) + s, h);
}

__device__ __forceinline__ bf16x8 pack8(const uint16_t (&e)[8]) {
  s16x8 v;
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = (short)e[s];
  return __builtin_bit_cast(bf16x8, v);
}

// ---------------------------------------------------------------- features --
// Squared (capped) degree of the far endpoint of each adjacency entry: the
// source of an in-CSR entry (its in-degree) or the target of an out-CSR
// entry (its out-degree).  Capping at 2^16 - 1 keeps a window's sum below
// 2^63, so window sums taken from wrapping 64-bit prefix sums are exact.
struct Deg2 {
  const int32_t* end;   // in_src or out_dst
  const uint32_t* off;  // in_off or out_off
  __device__ __forceinline__ uint64_t operator()(int64_t i) const {
    const int32_t x = end[i];
    uint64_t d = (uint64_t)(off[x + 1] - off[x]);
    d = d < 65535u ? d : 65535u;
    return d * d;
  }
};

constexpr int kPBlock = 256, kPItems = 8, kPTile = kPBlock * kPItems;

// per tile: wrapping sum of the values
// Kernels that gather through the graph's vertex ids leave a rejected graph
// (non-zero build status) alone.
__global__ __launch_bounds__(kPBlock) void k_deg2_tiles(Deg2 f, int64_t m,
                                                       uint64_t* __restrict__ tile_sums,
                                                       const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;
  __shared__ uint64_t s_w[kPBlock / kWave];
  uint64_t s = 0;
  const int64_t p0 = (int64_t)blockIdx.x * kPTile + (int64_t)threadIdx.x * kPItems;
#pragma unroll
  for (int j = 0; j < kPItems; ++j)
    if (p0 + j < m) s += f(p0 + j);
  s = wave_sum64(s);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kPBlock / kWave; ++w) t += s_w[w];
    tile_sums[blockIdx.x] = t;
  }
}

// one block: exclusive wrapping scan of the tile sums (in place)
__global__ __launch_bounds__(1024) void k_deg2_scan_tiles(uint64_t* __restrict__ tile_sums,
                                                          int64_t ntiles) {
  __shared__ uint64_t s_w[16];
  __shared__ uint64_t s_carry;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < ntiles; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const uint64_t v = i < ntiles ? tile_sums[i] : 0;
    const uint64_t inc = wave_inclusive_scan(v);
    if (lane == 63) s_w[wave] = inc;
    __syncthreads();
    uint64_t pre = s_carry;
    for (int w = 0; w < wave; ++w) pre += s_w[w];
    if (i < ntiles) tile_sums[i] = pre + inc - v;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = pre + inc;
    __syncthreads();
  }
}

// per tile: exclusive prefix sums ps[i] (wrapping), ps[m] = total
__global__ __launch_bounds__(kPBlock) void k_deg2_apply(Deg2 f, int64_t m,
                                                       const uint64_t* __restrict__ tile_off,
                                                       uint64_t* __restrict__ ps,
                                                       const uint32_t* __restrict__ gstatus) {
  if (*gstatus) return;
  __shared__ uint64_t s_w[kPBlock / kWave];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t p0 = (int64_t)blockIdx.x * kPTile + (int64_t)threadIdx.x * kPItems;
  uint64_t v[kPItems];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kPItems; ++j) {
    v[j] = p0 + j < m ? f(p0 + j) : 0;
    s += v[j];
  }
  const uint64_t inc = wave_inclusive_scan(s);
  if (lane == 63) s_w[wave] = inc;
  __syncthreads();
  uint64_t run = tile_off[blockIdx.x] + inc - s;
  for (int q = 0; q < wave; ++q) run += s_w[q];
#pragma unroll
  for (int j = 0; j < kPItems; ++j) {
    if (p0 + j <= m) ps[p0 + j] = run;  // p0 + j == m stores the total
    run += v[j];
  }
}

__global__ __launch_bounds__(256) void k_features(
    const int32_t* __restrict__ out_src, const int32_t* __restrict__ out_dst,
    const int64_t* __restrict__ out_t, const int64_t* __restrict__ in_t,
    const int64_t* __restrict__ pair_t, const PairSlot* __restrict__ pair_hash,
    int32_t pair_hash_log2, const uint32_t* __restrict__ lo_in, const uint32_t* __restrict__ a,
    const uint32_t* __restrict__ lo_out, const uint32_t* __restrict__ b,
    const uint64_t* __restrict__ ps_in, const uint64_t* __restrict__ ps_out, int64_t delta,
    int64_t m, uint4* __restrict__ feat, const uint32_t* __restrict__ gstatus) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m || *gstatus) return;
  const int32_t u = out_src[p], v = out_dst[p];
  const int64_t t = out_t[p];
  const uint32_t ap = a[p], bp = b[p];
  float f[8];
  f[0] = log1pf((float)ap);
  f[1] = log1pf((float)bp);
  f[2] = log1pf((float)((uint64_t)ap * (uint64_t)bp));
  f[3] = (ap > 0 && delta > 0) ? (float)(t - in_t[lo_in[p]]) / (float)delta : 0.0f;
  f[4] = (bp > 0 && delta > 0) ? (float)(out_t[lo_out[p] + bp - 1] - t) / (float)delta : 0.0f;
  uint32_t r0, r1;
  pair_run(pair_hash, pair_hash_log2, u, v, &r0, &r1);
  f[5] = log1pf((float)(upper_bound<int64_t>(pair_t, r0, r1, t + delta) -
                        lower_bound<int64_t>(pair_t, r0, r1, t - delta)));
  pair_run(pair_hash, pair_hash_log2, v, u, &r0, &r1);
  f[6] = log1pf((float)(upper_bound<int64_t>(pair_t, r0, r1, t + delta) -
                        lower_bound<int64_t>(pair_t, r0, r1, t - delta)));
  // mean squared degree of the window ends (exact wrapping window sums)
  const uint32_t li = lo_in[p], lo = lo_out[p];
  const double m_in = ap ? (double)(ps_in[li + ap] - ps_in[li]) / (double)ap : 0.0;
  const double m_out = bp ? (double)(ps_out[lo + bp] - ps_out[lo]) / (double)bp : 0.0;
  f[7] = (float)(0.5 * log1p(m_in * m_out));
  uint32_t w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    w[i] = (uint32_t)bf16_bits(f[2 * i]) | ((uint32_t)bf16_bits(f[2 * i + 1]) << 16);
  feat[p] = make_uint4(w[0], w[1], w[2], w[3]);
}

// ------------------------------------------------------------ MLP pieces --
// Per-lane operand registers of the two MFMA layers.
struct MlpOps {
  s16x4 w1[2];      // layer 1, output block rb: W1[32 rb + i][4 h + s]
  bf16x8 w2[2][4];  // layer 2, output block ob, K-chunk kc: W2[32 ob + i][krow(kc, s, h)]
};

__device__ void load_ops(const float* __restrict__ P, int lane, MlpOps* o) {
  const int i = lane & 31, h = lane >> 5;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    s16x4 v;
#pragma unroll
    for (int s = 0; s < 4; ++s) v[s] = (short)bf16_bits(P[kOffW1 + (32 * rb + i) * kIn + 4 * h + s]);
    o->w1[rb] = v;
  }
#pragma unroll
  for (int ob = 0; ob < 2; ++ob)
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      uint16_t e[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) e[s] = bf16_bits(P[kOffW2 + (32 * ob + i) * kHid + krow(kc, s, h)]);
      o->w2[ob][kc] = pack8(e);
    }
}

// small vectors in LDS: b1, b2 (float32), w3 (bfloat16-rounded), b3
struct MlpVecs {
  float b1[kHid], b2[kHid], w3[kHid], b3;
};

__device__ void load_vecs(const float* __restrict__ P, MlpVecs* s) {
  for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
    s->b1[i] = P[kOffB1 + i];
    s->b2[i] = P[kOffB2 + i];
    s->w3[i] = bf16_round(P[kOffW3 + i]);
  }
  if (threadIdx.x == 0) s->b3 = P[kOffB3];
}

struct Fwd {
  f32x16 z1[2], z2[2];
  bf16x8 h1[4];  // layer-2 B operand chunks (relu(z1) in bfloat16)
  float z3;
};

// forward of 32 edges; fb = features 4h..4h+3 of edge lane % 32; z (zero)
// offsets every read of the small vectors
__device__ __forceinline__ void mlp_fwd(const MlpOps& o, const MlpVecs& sv, s16x4 fb, int h,
                                        Fwd* r, int z = 0) {
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    f32x16 c;
#pragma unroll
    for (int v = 0; v < 16; ++v) c[v] = sv.b1[32 * rb + drow(v, h) + z];
    r->z1[rb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(o.w1[rb], fb, c, 0, 0, 0);
  }
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const f32x16& z = r->z1[kc >> 1];
    const int s0 = 8 * (kc & 1);
    uint4 q;
    q.x = bf16x2_bits(fmaxf(z[s0], 0.0f), fmaxf(z[s0 + 1], 0.0f));
    q.y = bf16x2_bits(fmaxf(z[s0 + 2], 0.0f), fmaxf(z[s0 + 3], 0.0f));
    q.z = bf16x2_bits(fmaxf(z[s0 + 4], 0.0f), fmaxf(z[s0 + 5], 0.0f));
    q.w = bf16x2_bits(fmaxf(z[s0 + 6], 0.0f), fmaxf(z[s0 + 7], 0.0f));
    r->h1[kc] = __builtin_bit_cast(bf16x8, q);
  }
  float part = 0.0f;
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    f32x16 c;
#pragma unroll
    for (int v = 0; v < 16; ++v) c[v] = sv.b2[32 * ob + drow(v, h) + z];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc)
      c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.w2[ob][kc], r->h1[kc], c, 0, 0, 0);
    r->z2[ob] = c;
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
      const uint32_t pr = bf16x2_bits(fmaxf(c[v], 0.0f), fmaxf(c[v + 1], 0.0f));
      part += sv.w3[32 * ob + drow(v, h) + z] * __uint_as_float(pr << 16);
      part += sv.w3[32 * ob + drow(v + 1, h) + z] * __uint_as_float(pr & 0xFFFF0000u);
    }
  }
  part += __shfl_xor(part, 32, kWave);
  r->z3 = part + sv.b3;
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float softplusf(float x) {
  return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

__device__ __forceinline__ s16x4 load_feat4(const uint16_t* __restrict__ feat, int64_t row, int h) {
  const uint2 q = *reinterpret_cast<const uint2*>(feat + row * kIn + 4 * h);
  s16x4 v;
  v[0] = (short)(q.x & 0xFFFF);
  v[1] = (short)(q.x >> 16);
  v[2] = (short)(q.y & 0xFFFF);
  v[3] = (short)(q.y >> 16);
  return v;
}

// g for n rows of features (inference)
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ P,
                                                     const uint16_t* __restrict__ feat, int64_t n,
                                                     float* __restrict__ g) {
  __shared__ MlpVecs sv;
  load_vecs(P, &sv);
  MlpOps o;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  load_ops(P, lane, &o);
  __syncthreads();
  const int64_t tiles = (n + 31) / 32;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x / kWave);
  // one tile of 32 rows per wavefront at a time; the wavefront index is
  // uniform across its lanes, so the tile loop branches as a whole
  const int64_t wave_id = (int64_t)blockIdx.x * (blockDim.x / kWave) + uni(threadIdx.x >> 6);
  for (int64_t tile = wave_id; tile < tiles; tile += wstride) {
    const int64_t row = tile * 32 + (lane & 31);
    const s16x4 fb = row < n ? load_feat4(feat, row, h) : s16x4{0, 0, 0, 0};
    // The small vectors are read from LDS in every tile: an offset the
    // compiler cannot see to be zero keeps it from holding all 96 per-lane
    // values in registers, which would leave room for two wavefronts per SIMD.
    int z;
    asm volatile("v_mov_b32 %0, 0" : "=v"(z));
    Fwd r;
    mlp_fwd(o, sv, fb, h, &r, z);
    if (h == 0 && row < n) g[row] = sigmoidf(r.z3);
  }
}

// ------------------------------------------------------------ gradients ----
constexpr int kGradBlock = 256;
constexpr int kGradWaves = kGradBlock / kWave;
constexpr int kTS = 40;  // LDS row stride (bfloat16 entries) of a 64 x 32 tile

struct GradLds {
  MlpVecs sv;
  uint16_t w2b[kHid * kHid];  // W2 in bfloat16, row-major
  alignas(16) uint16_t dz2[kGradWaves][kHid * kTS];
  alignas(16) uint16_t h1[kGradWaves][kHid * kTS];
  alignas(16) uint16_t dz1[kGradWaves][kHid * kTS];
  alignas(16) uint16_t f[kGradWaves][32 * 8];
  float red[kGradWaves][kNParams + 1];
};

// Label row of item i of the current batch: index = (mul * (start + i) + add)
// mod n of the label arrays (a bijection of [0, n) when gcd(mul, n) = 1).
struct BatchMap {
  uint64_t mul, add, n, start;
  uint32_t count;
  uint64_t n_feat;  // feature rows; labels whose row is outside are ignored
  float label_cap;  // 0: y = [X > 0]; else y = min(1, X / label_cap)
};

// mul < n and start + i < n with n < 2^31, so the product fits 64 bits
__device__ __forceinline__ uint64_t batch_index(const BatchMap& bm, uint64_t i) {
  return (bm.mul * (bm.start + i) + bm.add) % bm.n;
}

// Partial loss and gradient of one block over its tiles of the batch; the
// tile-to-block assignment depends only on the launch shape.
__global__ __launch_bounds__(kGradBlock) void k_mlp_grad(const float* __restrict__ P,
                                                         const uint16_t* __restrict__ feat,
                                                         const uint32_t* __restrict__ rows,
                                                         const uint64_t* __restrict__ X,
                                                         BatchMap bm,
                                                         float* __restrict__ partial) {
  extern __shared__ char s_raw[];
  GradLds& L = *reinterpret_cast<GradLds*>(s_raw);
  load_vecs(P, &L.sv);
  const int lane = threadIdx.x & 63, h = lane >> 5, i = lane & 31, wave = threadIdx.x >> 6;
  MlpOps o;
  load_ops(P, lane, &o);
  for (int j = threadIdx.x; j < kHid * kHid; j += blockDim.x) L.w2b[j] = bf16_bits(P[kOffW2 + j]);
  __syncthreads();
  const float inv_n = 1.0f / (float)bm.count;
  f32x16 gW2[2][2], gW1[2];
#pragma unroll
  for (int a2 = 0; a2 < 2; ++a2) {
    gW1[a2] = f32x16{};
#pragma unroll
    for (int b2 = 0; b2 < 2; ++b2) gW2[a2][b2] = f32x16{};
  }
  float gb3 = 0.0f, loss = 0.0f;
  // this wave's partial gradient; w3 and b2 are accumulated here tile by tile
  float* red = L.red[wave];
  for (int j = lane; j <= kNParams; j += kWave) red[j] = 0.0f;
  uint16_t* tdz2 = L.dz2[wave];
  uint16_t* th1 = L.h1[wave];
  uint16_t* tdz1 = L.dz1[wave];
  uint16_t* tf = L.f[wave];
  const uint32_t tiles = (bm.count + 31) / 32;
  // uniform trip count over the block so the barriers below are uniform
  const uint32_t per_round = gridDim.x * kGradWaves;
  for (uint32_t base = blockIdx.x * kGradWaves; base < tiles; base += per_round) {
    const uint32_t tile = base + wave;
    const uint32_t item = tile * 32 + i;
    const bool in_batch = tile < tiles && item < bm.count;
    int64_t row = 0;
    float y = 0.0f;
    bool valid = in_batch;
    if (in_batch) {
      const uint64_t idx = batch_index(bm, item);
      row = rows ? (int64_t)rows[idx] : (int64_t)idx;
      const uint64_t xv = X[idx];
      y = bm.label_cap > 0.0f ? fminf(1.0f, __fdiv_rn((float)xv, bm.label_cap))
                              : (xv != 0 ? 1.0f : 0.0f);
      valid = (uint64_t)row < bm.n_feat;
    }
    const s16x4 fb = valid ? load_feat4(feat, row, h) : s16x4{0, 0, 0, 0};
    Fwd r;
    mlp_fwd(o, L.sv, fb, h, &r);
    const float gz = sigmoidf(r.z3);
    const float dz3 = valid ? (gz - y) * inv_n : 0.0f;
    if (h == 0 && valid) {
      loss += y * softplusf(-r.z3) + (1.0f - y) * softplusf(r.z3);
      gb3 += dz3;
    }
    // layer 3 and dZ2 (registers, rows drow(v, h) of block ob, edge i); the
    // w3 and b2 gradients are summed over the tile's 32 edges right away
    uint16_t dz2b[2][16];
#pragma unroll
    for (int ob = 0; ob < 2; ++ob)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rr = 32 * ob + drow(v, h);
        const float z2 = r.z2[ob][v];
        float s3 = dz3 * bf16_round(fmaxf(z2, 0.0f));
        const float d = z2 > 0.0f ? L.sv.w3[rr] * dz3 : 0.0f;
        float s2 = d;
        dz2b[ob][v] = bf16_bits(d);
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
          s3 += __shfl_xor(s3, off, kWave);
          s2 += __shfl_xor(s2, off, kWave);
        }
        if (i == 0) {
          red[kOffW3 + rr] += s3;
          red[kOffB2 + rr] += s2;
        }
      }
    // dH1 = W2^T dZ2, then dZ1 = dH1 * [z1 > 0]
    bf16x8 dzc[4];
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      uint16_t e[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) e[s] = dz2b[kc >> 1][8 * (kc & 1) + s];
      dzc[kc] = pack8(e);
    }
    // stage dZ2, H1, dZ1 and F with edges along rows for the weight gradients
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      f32x16 c = f32x16{};
#pragma unroll
      for (int kc = 0; kc < 4; ++kc) {
        // A operand of dH1 = W2^T dZ2: W2[krow(kc, s, h)][32 kb + i]
        uint16_t e[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) e[s] = L.w2b[krow(kc, s, h) * kHid + 32 * kb + i];
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pack8(e), dzc[kc], c, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int rr = 32 * kb + drow(v, h);
        const float z1 = r.z1[kb][v];
        tdz1[rr * kTS + i] = bf16_bits(z1 > 0.0f ? c[v] : 0.0f);
        th1[rr * kTS + i] = bf16_bits(fmaxf(z1, 0.0f));
        tdz2[rr * kTS + i] = dz2b[kb][v];
      }
    }
    {
      const uint2 q = {(uint32_t)(uint16_t)fb[0] | ((uint32_t)(uint16_t)fb[1] << 16),
                       (uint32_t)(uint16_t)fb[2] | ((uint32_t)(uint16_t)fb[3] << 16)};
      *reinterpret_cast<uint2*>(tf + i * 8 + 4 * h) = q;
    }
    __syncthreads();
    // dW2[32 ob + .][32 kb + .] += dZ2 H1^T and [dW1 | db1] += dZ1 [F | 1]^T,
    // contracting over the 32 edges (two K-chunks of 16)
#pragma unroll
    for (int e2 = 0; e2 < 2; ++e2) {
      const int col = 16 * e2 + 8 * h;
      bf16x8 Ad[2], Bh[2];
#pragma unroll
      for (int x2 = 0; x2 < 2; ++x2) {
        Ad[x2] = *reinterpret_cast<const bf16x8*>(tdz2 + (32 * x2 + i) * kTS + col);
        Bh[x2] = *reinterpret_cast<const bf16x8*>(th1 + (32 * x2 + i) * kTS + col);
      }
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
          gW2[ob][kb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ad[ob], Bh[kb], gW2[ob][kb], 0, 0, 0);
      // B of [F | 1]^T: column i < 8 is feature i of the edges, column 8 is 1
      uint16_t e[8];
#pragma unroll
      for (int s = 0; s < 8; ++s)
        e[s] = i < 8 ? tf[(col + s) * 8 + i] : (i == 8 ? (uint16_t)0x3F80u : (uint16_t)0);
      const bf16x8 Bf = pack8(e);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const bf16x8 A1 = *reinterpret_cast<const bf16x8*>(tdz1 + (32 * rb + i) * kTS + col);
        gW1[rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A1, Bf, gW1[rb], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // per-wave partials into LDS, then the block sum in wave order
#pragma unroll
  for (int ob = 0; ob < 2; ++ob)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rr = 32 * ob + drow(v, h);
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) red[kOffW2 + rr * kHid + 32 * kb + i] = gW2[ob][kb][v];
      if (i < 8) red[kOffW1 + rr * kIn + i] = gW1[ob][v];
      if (i == 8) red[kOffB1 + rr] = gW1[ob][v];
    }
  {
    float s3 = gb3, sl = loss;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      s3 += __shfl_xor(s3, off, kWave);
      sl += __shfl_xor(sl, off, kWave);
    }
    if (lane == 0) {
      red[kOffB3] = s3;
      red[kNParams] = sl;
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j <= kNParams; j += blockDim.x) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < kGradWaves; ++w) s += L.red[w][j];
    partial[(size_t)blockIdx.x * (kNParams + 1) + j] = s;
  }
}

size_t mlp_grad_lds_bytes() { return sizeof(GradLds); }

// Sum of the block partials in block order.  mode 0: grad[j] and *loss;
// mode 1: one Adam step on params with moments opt[0..n), opt[n..2n).
struct AdamArgs {
  float lr, beta1, beta2, eps;
  float omb1, omb2;  // 1 - beta, formed in binary64 and rounded once
  float bc1, bc2;    // 1 - beta^step
};

__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int nblocks,
                                                    int mode, float* __restrict__ grad,
                                                    float* __restrict__ loss, float loss_scale,
                                                    float* __restrict__ params,
                                                    float* __restrict__ opt, AdamArgs ad) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > kNParams || (j == kNParams && !loss)) return;
  float s = 0.0f;
  for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * (kNParams + 1) + j];
  if (j == kNParams) {
    // loss: sum over rows / batch size, scaled (e.g. 1 / batches per epoch)
    *loss += s * loss_scale;
    return;
  }
  if (mode == 0) {
    grad[j] = s;
    return;
  }
  float* m1 = opt;
  float* m2 = opt + kNParams;
  const float mj = ad.beta1 * m1[j] + ad.omb1 * s;
  const float vj = ad.beta2 * m2[j] + ad.omb2 * (s * s);
  m1[j] = mj;
  m2[j] = vj;
  const float mh = mj / ad.bc1, vh = vj / ad.bc2;
  params[j] -= ad.lr * mh / (sqrtf(vh) + ad.eps);
}

__global__ void k_zero_f32(float* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// ----------------------------------------------------------- quantisation --
// g clamped to [0, 1] (NaN read as 0)
__device__ __forceinline__ float clamp_score(float x) {
  if (!(x >= 0.0f)) x = 0.0f;
  return x > 1.0f ? 1.0f : x;
}

// max of the clamped scores (non-negative floats order like their bit patterns)
__global__ __launch_bounds__(256) void k_score_max(const float* __restrict__ g, int64_t m,
                                                   uint32_t* __restrict__ gmax_bits) {
  __shared__ uint32_t s_max;
  if (threadIdx.x == 0) s_max = 0u;
  __syncthreads();
  uint32_t b = 0u;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t v = __float_as_uint(clamp_score(g[p]));
    b = v > b ? v : b;
  }
  atomicMax(&s_max, b);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(gmax_bits, s_max);
}

__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

__global__ __launch_bounds__(256) void k_quantize(const float* __restrict__ g, int64_t m,
                                                  float eps, const uint64_t* __restrict__ S,
                                                  const float* __restrict__ gmax,
                                                  uint32_t* __restrict__ hq) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m) return;
  const uint64_t W = S[m];
  const int bitlen = W ? 64 - __clzll((long long)W) : 0;
  int s = 63 - bitlen;
  s = s < 1 ? 1 : (s > 16 ? 16 : s);
  float x = clamp_score(g[p]);
  if (gmax) {
    const float gm = *gmax;
    if (gm > 0.0f) x = __fdiv_rn(x, gm);
  }
  const float one_m = __fsub_rn(1.0f, eps);
  const float hv = __fadd_rn(eps, __fmul_rn(one_m, x));
  const float hs = __fmul_rn(hv, (float)(1u << s));
  const float r = floorf(__fadd_rn(hs, 0.5f));
  const uint32_t v = (uint32_t)r;
  hq[p] = v < 1u ? 1u : v;
}

// ------------------------------------------------------------- host side --
static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t features_workspace_bytes(int64_t m) {
  const size_t ntiles = (size_t)((m + 1 + kPTile - 1) / kPTile);
  return 2 * align256((size_t)(m + 1) * 8) + align256(ntiles * 8);
}

tc_status edge_features(const tc_graph* g, const tc_weights* w, uint16_t* feat, void* ws,
                        size_t ws_bytes, hipStream_t st) {
  const int64_t m = g->m;
  if (ws_bytes < features_workspace_bytes(m)) return TC_E_WORKSPACE;
  if (m == 0) return TC_OK;
  char* base = (char*)ws;
  uint64_t* ps_in = (uint64_t*)base;
  uint64_t* ps_out = (uint64_t*)(base + align256((size_t)(m + 1) * 8));
  uint64_t* tiles = (uint64_t*)(base + 2 * align256((size_t)(m + 1) * 8));
  // tiles cover indices 0..m so that the last one also stores ps[m]
  const int64_t ntiles = (m + 1 + kPTile - 1) / kPTile;
  const Deg2 fin{(const int32_t*)g->in_src, (const uint32_t*)g->in_off};
  const Deg2 fout{(const int32_t*)g->out_dst, (const uint32_t*)g->out_off};
  for (int side = 0; side < 2; ++side) {
    const Deg2 f = side == 0 ? fin : fout;
    uint64_t* ps = side == 0 ? ps_in : ps_out;
    hipLaunchKernelGGL(k_deg2_tiles, dim3((unsigned)ntiles), dim3(kPBlock), 0, st, f, m, tiles,
                       (const uint32_t*)g->status);
    hipLaunchKernelGGL(k_deg2_scan_tiles, dim3(1), dim3(1024), 0, st, tiles, ntiles);
    hipLaunchKernelGGL(k_deg2_apply, dim3((unsigned)ntiles), dim3(kPBlock), 0, st, f, m,
                       (const uint64_t*)tiles, ps, (const uint32_t*)g->status);
  }
  {
    TimedLaunch tl("k_features", st);
    hipLaunchKernelGGL(k_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st,
                       (const int32_t*)g->out_src, (const int32_t*)g->out_dst,
                       (const int64_t*)g->out_t, (const int64_t*)g->in_t,
                       (const int64_t*)g->pair_t, (const PairSlot*)g->pair_hash,
                       g->pair_hash_log2, w->lo_in, w->a, w->lo_out, w->b,
                       (const uint64_t*)ps_in, (const uint64_t*)ps_out, w->delta, m,
                       (uint4*)feat, (const uint32_t*)g->status);
  }
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

tc_status mlp_forward(const float* params, const uint16_t* feat, int64_t n, float* g,
                      hipStream_t st) {
  if (n > 0) {
    const int64_t tiles = (n + 31) / 32;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    TimedLaunch tl("k_mlp_forward", st);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, st, params, feat, n, g);
  }
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

int mlp_grad_blocks(int64_t count) {
  const int64_t tiles = (count + 31) / 32;
  int64_t b = (tiles + kGradWaves - 1) / kGradWaves;
  if (b > 512) b = 512;
  return b < 1 ? 1 : (int)b;
}

size_t mlp_workspace_bytes(int64_t batch) {
  return (size_t)mlp_grad_blocks(batch) * (kNParams + 1) * sizeof(float);
}

static tc_status launch_grad(const float* params, const uint16_t* feat, const uint32_t* rows,
                             const uint64_t* X, const BatchMap& bm, float* partial,
                             hipStream_t st) {
  const int nb = mlp_grad_blocks(bm.count);
  if (hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sizeof(GradLds)) != hipSuccess)
    return TC_E_HIP;
  TimedLaunch tl("k_mlp_grad", st);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)nb), dim3(kGradBlock), sizeof(GradLds), st,
                     params, feat, rows, X, bm, partial);
  return TC_OK;
}

tc_status mlp_grad(const float* params, const uint16_t* feat, int64_t n_feat, const uint32_t* rows,
                   const uint64_t* X, int64_t n, float label_cap, float* grad, float* loss,
                   void* ws, size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < mlp_workspace_bytes(n)) return TC_E_WORKSPACE;
  const BatchMap bm{1, 0, (uint64_t)n, 0, (uint32_t)n, (uint64_t)n_feat, label_cap};
  float* partial = (float*)ws;
  tc_status s = launch_grad(params, feat, rows, X, bm, partial, st);
  if (s != TC_OK) return s;
  hipLaunchKernelGGL(k_zero_f32, dim3(1), dim3(64), 0, st, loss, 1);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParams + 256) / 256), dim3(256), 0, st,
                     (const float*)partial, mlp_grad_blocks(n), 0, grad, loss, 1.0f / (float)n,
                     (float*)nullptr, (float*)nullptr, AdamArgs{});
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

static AdamArgs adam_args(int64_t step, float lr) {
  AdamArgs a;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.omb1 = (float)(1.0 - 0.9);
  a.omb2 = (float)(1.0 - 0.999);
  a.bc1 = (float)(1.0 - std::pow(0.9, (double)step));
  a.bc2 = (float)(1.0 - std::pow(0.999, (double)step));
  return a;
}

tc_status mlp_adam(float* params, float* opt, const float* grad, int64_t step, float lr,
                   hipStream_t st) {
  // the gradient is one "partial" of one block
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParams + 256) / 256), dim3(256), 0, st, grad, 1, 1,
                     (float*)nullptr, (float*)nullptr, 0.0f, params, opt, adam_args(step, lr));
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

static uint64_t gcd64(uint64_t a, uint64_t b) {
  while (b) {
    const uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

tc_status mlp_train(float* params, float* opt, const uint16_t* feat, int64_t n_feat,
                    const uint32_t* rows, const uint64_t* X, int64_t n, float label_cap,
                    int32_t batch, int32_t epochs, float lr,
                    uint64_t seed, int64_t step0, float* loss_per_epoch, void* ws,
                    size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < mlp_workspace_bytes(batch)) return TC_E_WORKSPACE;
  float* partial = (float*)ws;
  const int64_t nbatches = (n + batch - 1) / batch;
  if (loss_per_epoch)
    hipLaunchKernelGGL(k_zero_f32, dim3((epochs + 63) / 64), dim3(64), 0, st, loss_per_epoch,
                       epochs);
  int64_t step = step0;
  for (int32_t e = 0; e < epochs; ++e) {
    // a per-epoch bijection i -> (mul * i + add) mod n drawn from Philox
    const Words4 r = philox_block(seed, 0x4D4C5000u, (uint64_t)e, 0);
    uint64_t mul = n > 1 ? 1 + ((((uint64_t)r.x1 << 32) | r.x0) % (uint64_t)(n - 1)) : 1;
    while (gcd64(mul, (uint64_t)n) != 1) mul = mul + 1 < (uint64_t)n ? mul + 1 : 1;
    const uint64_t add = (((uint64_t)r.x3 << 32) | r.x2) % (uint64_t)n;
    for (int64_t bi = 0; bi < nbatches; ++bi) {
      const uint64_t start = (uint64_t)bi * (uint64_t)batch;
      const uint32_t count = (uint32_t)std::min<int64_t>(batch, n - (int64_t)start);
      const BatchMap bm{mul, add, (uint64_t)n, start, count, (uint64_t)n_feat, label_cap};
      tc_status s = launch_grad(params, feat, rows, X, bm, partial, st);
      if (s != TC_OK) return s;
      ++step;
      hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParams + 256) / 256), dim3(256), 0, st,
                         (const float*)partial, mlp_grad_blocks(count), 1, (float*)nullptr,
                         loss_per_epoch ? loss_per_epoch + e : (float*)nullptr,
                         1.0f / ((float)count * (float)nbatches), params, opt,
                         adam_args(step, lr));
    }
  }
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

tc_status quantize_proposal(const tc_weights* w, const float* g, float eps, float* gmax,
                            uint32_t* hq, hipStream_t st) {
  const int64_t m = w->m;
  if (gmax) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, (uint32_t*)gmax);
    if (m > 0) {
      int64_t blocks = (m + 255) / 256;
      if (blocks > 2048) blocks = 2048;
      hipLaunchKernelGGL(k_score_max, dim3((unsigned)blocks), dim3(256), 0, st, g, m,
                         (uint32_t*)gmax);
    }
  }
  if (m > 0)
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, g, m, eps,
                       (const uint64_t*)w->S, (const float*)gmax, hq);
  return hipGetLastError() == hipSuccess ? TC_OK : TC_E_HIP;
}

}  // namespace tc
