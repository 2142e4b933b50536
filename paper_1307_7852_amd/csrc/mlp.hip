// Learned partitioner: a two-layer network z = W2 relu(W1 (s x) + b1) + b2
// (d -> 256 -> 16) whose embedding replaces the raw points when the T
// divisions choose their split directions.  Training pairs are edges of a
// k-NN graph the method produced (positives) and uniform random pairs
// (negatives); the loss is the contrastive form of Hadsell, Chopra and
// LeCun (CVPR 2006), the optimiser Adam with bias correction (Kingma and
// Ba, ICLR 2015).  Master weights are FP32; the matrix products run on MFMA
// in BF16 with FP32 accumulation (or in FP32 for gradient checks).
//
// Every product is written as 32x32 output tiles built from 16-wide K
// slices.  A lane holds 8 values of a slice: lane half h the K indices
// 8h .. 8h+7 of its row (A operand) or column (B operand).  The BF16 form
// issues one v_mfma_f32_32x32x16_bf16 per slice; the FP32 form issues eight
// v_mfma_f32_32x32x2_f32, the e-th pairing index e of both halves.  Output
// element (i, j) sits in lane 32*((i/4)%2) + j, register 4*(i/8) + i%4.
#include "knng_dev.h"

#include <algorithm>

namespace knng {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int MH = KNNG_MLP_HIDDEN;
constexpr int ME = KNNG_MLP_EMB;
constexpr int WG = 256;   // four waves, 32 rows each

template <bool BF16>
__device__ __forceinline__ void mma16(f32x16& acc, const float (&a)[8], const float (&b)[8]) {
  if constexpr (BF16) {
    bf16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = (__bf16)a[e];
      bv[e] = (__bf16)b[e];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[e], b[e], acc, 0, 0, 0);
  }
}

// Row index (within a 32x32 tile) of output register r in lane half h.
__device__ __forceinline__ int tile_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ void load8(float (&v)[8], const float* p, bool ok) {
  if (ok) {
    float4 x = *(const float4*)p, y = *(const float4*)(p + 4);
    v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = 0.f;
  }
}

// ---------------------------------------------------------------- forward
// One wave per 32 rows.  Layer 1 is computed transposed (hidden units as
// tile rows, data rows as tile columns) so that each lane ends up with 16
// hidden values of its own data row; those feed layer 2 directly as the B
// operand, with the K order of layer 2 permuted to match (a permutation of
// the contraction index leaves the sum unchanged).
template <bool BF16, bool TRAIN, int NS>
__global__ __launch_bounds__(WG) void k_mlp_fwd(MlpArgs a) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, c32 = lane & 31;
  const int64_t base = ((int64_t)blockIdx.x * (WG / 64) + w) * 32;
  if (base >= a.R) return;   // whole wave idle; no barriers in this kernel
  const int d = a.d;
  const int64_t row = base + c32;
  const bool ok = row < a.R;
  const int64_t src = ok ? (a.rows ? (int64_t)a.rows[row] : row) : 0;
  const float* x = a.X + src * d;
  const float* W1 = a.params;
  const float* b1 = W1 + (size_t)MH * d;
  const float* W2 = b1 + MH;
  const float* b2 = W2 + (size_t)ME * MH;
  // x fragments (B operand of layer 1): slice s holds features 16s + 8h + e
  float xf[NS][8];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const int f = 16 * s + 8 * h;
    load8(xf[s], x + f, ok && f < d);
#pragma unroll
    for (int e = 0; e < 8; ++e) xf[s][e] *= a.scale;
  }
  f32x16 zacc = {0};
#pragma unroll 1
  for (int t = 0; t < MH / 32; ++t) {
    f32x16 acc = {0};
    const float* w1row = W1 + (size_t)(t * 32 + c32) * d;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      float wf[8];
      const int f = 16 * s + 8 * h;
      load8(wf, w1row + f, f < d);
      mma16<BF16>(acc, wf, xf[s]);
    }
    // acc[r]: hidden unit t*32 + tile_row(r, h) of data row `row`
    float hv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) hv[r] = fmaxf(acc[r] + b1[t * 32 + tile_row(r, h)], 0.f);
    if (TRAIN && ok) {
      float* hs = a.Hs + row * MH + t * 32;
#pragma unroll
      for (int g = 0; g < 4; ++g)
        *(float4*)(hs + 8 * g + 4 * h) = make_float4(hv[4 * g], hv[4 * g + 1], hv[4 * g + 2], hv[4 * g + 3]);
    }
    // layer 2, two K slices of 16 hidden units: slice q, element e of lane
    // half h is hidden unit t*32 + 16q + 8(e/4) + 4h + e%4 (= register 8q + e)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      float bf[8], af[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        bf[e] = hv[8 * q + e];
        const int hid = t * 32 + 16 * q + 8 * (e >> 2) + 4 * h + (e & 3);
        af[e] = c32 < ME ? W2[(size_t)c32 * MH + hid] : 0.f;
      }
      mma16<BF16>(zacc, af, bf);
    }
  }
  // zacc[r]: embedding unit tile_row(r, h) (< 16 for r < 8) of data row `row`
  if (ok) {
    float* z = a.Z + row * ME;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int e0 = 8 * g + 4 * h;
      *(float4*)(z + e0) = make_float4(zacc[4 * g] + b2[e0], zacc[4 * g + 1] + b2[e0 + 1], zacc[4 * g + 2] + b2[e0 + 2],
                                       zacc[4 * g + 3] + b2[e0 + 3]);
    }
  }
}

// Inference in BF16 (the embedding pass of a learned build): the same
// products as k_mlp_fwd<true, false, NS>, with the network's weights rounded
// to bfloat16 once per workgroup into LDS (rows padded by 8 halves) instead
// of being re-read from global memory by every wave.  Workgroups stride over
// tiles of 128 data rows.  Rounding a weight before or inside the MFMA's
// operand conversion gives the same bfloat16, so the result is bit for bit
// that of k_mlp_fwd.
template <int NS>
__global__ __launch_bounds__(WG) void k_mlp_embed(MlpArgs a, int64_t n_tiles) {
  constexpr int DP = NS * 16 + 8;
  __shared__ __bf16 w1s[MH * DP];
  __shared__ __bf16 w2s[ME * (MH + 8)];
  __shared__ float b1s[MH], b2s[ME];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, c32 = lane & 31;
  const int d = a.d;
  const float* W1 = a.params;
  const float* b1 = W1 + (size_t)MH * d;
  const float* W2 = b1 + MH;
  const float* b2 = W2 + (size_t)ME * MH;
  for (int e = threadIdx.x; e < MH * NS * 16; e += WG) {
    const int r = e / (NS * 16), c = e % (NS * 16);
    w1s[r * DP + c] = (__bf16)(c < d ? W1[(size_t)r * d + c] : 0.f);
  }
  for (int e = threadIdx.x; e < ME * MH; e += WG) w2s[(e / MH) * (MH + 8) + e % MH] = (__bf16)W2[e];
  for (int e = threadIdx.x; e < MH; e += WG) b1s[e] = b1[e];
  if (threadIdx.x < ME) b2s[threadIdx.x] = b2[threadIdx.x];
  __syncthreads();
  for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
    const int64_t row = tile * 128 + w * 32 + c32;
    const bool ok = row < a.R;
    const float* x = a.X + (ok ? row : 0) * d;
    bf16x8 xb[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) {
      float xf[8];
      const int f = 16 * s2 + 8 * h;
      load8(xf, x + f, ok && f < d);
#pragma unroll
      for (int e = 0; e < 8; ++e) xb[s2][e] = (__bf16)(xf[e] * a.scale);
    }
    f32x16 zacc = {0};
#pragma unroll 1
    for (int t = 0; t < MH / 32; ++t) {
      f32x16 acc = {0};
      const __bf16* w1row = w1s + (t * 32 + c32) * DP;
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) {
        const bf16x8 wb = *(const bf16x8*)(w1row + 16 * s2 + 8 * h);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wb, xb[s2], acc, 0, 0, 0);
      }
      float hv[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) hv[r] = fmaxf(acc[r] + b1s[t * 32 + tile_row(r, h)], 0.f);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        bf16x8 av, bv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          bv[e] = (__bf16)hv[8 * q + e];
          const int hid = t * 32 + 16 * q + 8 * (e >> 2) + 4 * h + (e & 3);
          av[e] = c32 < ME ? w2s[c32 * (MH + 8) + hid] : (__bf16)0.f;
        }
        zacc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, zacc, 0, 0, 0);
      }
    }
    if (ok) {
      float* z = a.Z + row * ME;
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        const int e0 = 8 * g + 4 * h;
        *(float4*)(z + e0) = make_float4(zacc[4 * g] + b2s[e0], zacc[4 * g + 1] + b2s[e0 + 1],
                                         zacc[4 * g + 2] + b2s[e0 + 2], zacc[4 * g + 3] + b2s[e0 + 3]);
      }
    }
  }
}

// ---------------------------------------------------------------- loss
// One thread per pair; pair p owns batch rows 2p and 2p+1.  Positives add
// |z_a - z_b|^2 / P, negatives lam * max(0, c - |z_a - z_b|^2) / N.
__global__ __launch_bounds__(256) void k_mlp_loss(MlpArgs a) {
  __shared__ float red[256];
  const int p = blockIdx.x * 256 + threadIdx.x;
  const int np = a.n_pos + a.n_neg;
  float term = 0.f;
  if (p < np) {
    const float* za = a.Z + (int64_t)(2 * p) * ME;
    const float* zb = za + ME;
    float dv[ME], l = 0.f;
#pragma unroll
    for (int e = 0; e < ME; ++e) {
      dv[e] = za[e] - zb[e];
      l = __builtin_fmaf(dv[e], dv[e], l);
    }
    float g;
    if (p < a.n_pos) {
      term = l / (float)a.n_pos;
      g = 2.0f / (float)a.n_pos;
    } else {
      const float hinge = a.margin - l;
      term = hinge > 0.f ? a.lam * hinge / (float)a.n_neg : 0.f;
      g = hinge > 0.f ? -2.0f * a.lam / (float)a.n_neg : 0.f;
    }
    float* ga = a.dZ + (int64_t)(2 * p) * ME;
#pragma unroll
    for (int e = 0; e < ME; ++e) {
      ga[e] = g * dv[e];
      ga[ME + e] = -g * dv[e];
    }
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.loss_part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------- backward
// dA1 = (dZ W2) * [h > 0]; one wave per 32 rows, tiles of 32 hidden units.
template <bool BF16>
__global__ __launch_bounds__(WG) void k_mlp_bwd_h(MlpArgs a) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, h = lane >> 5, c32 = lane & 31;
  const int64_t base = ((int64_t)blockIdx.x * (WG / 64) + w) * 32;
  if (base >= a.R) return;
  const int d = a.d;
  const float* W2 = a.params + (size_t)MH * d + MH;
  // A operand: dZ rows (data rows as tile rows), K = the 16 embedding units
  float af[8];
  load8(af, a.dZ + (base + c32) * ME + 8 * h, base + c32 < a.R);
#pragma unroll 1
  for (int t = 0; t < MH / 32; ++t) {
    float bf[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) bf[e] = W2[(size_t)(8 * h + e) * MH + t * 32 + c32];
    f32x16 acc = {0};
    mma16<BF16>(acc, af, bf);
    // acc[r]: data row base + tile_row(r, h), hidden unit t*32 + c32
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t ri = base + tile_row(r, h);
      if (ri < a.R) {
        const int64_t o = ri * MH + t * 32 + c32;
        a.dA[o] = a.Hs[o] > 0.f ? acc[r] : 0.f;
      }
    }
  }
}

// Weight gradients of one chunk of rows, written to that chunk's partial
// block (same layout as the parameters); chunks are summed in a fixed order
// afterwards, so the gradients do not depend on scheduling.
//   dW1 = dA1^T (s X),  db1 = sum dA1,  dW2 = dZ^T H,  db2 = sum dZ.
// Rows pass through LDS 16 at a time.  Each wave owns at most TPW dW1 tiles
// (hidden tile x feature tile) per sweep over the rows, and 2 dW2 tiles.
constexpr int TPW = 4;

template <bool BF16>
__global__ __launch_bounds__(WG) void k_mlp_wgrad(MlpArgs a) {
  extern __shared__ __align__(16) float sm[];
  const int d = a.d;
  const int DP = d + 4;                        // padded feature stride
  float* xs = sm;                              // [16][DP]
  float* dAs = xs + 16 * DP;                   // [16][MH + 4]
  float* hs = dAs + 16 * (MH + 4);             // [16][MH + 4]
  float* dzs = hs + 16 * (MH + 4);             // [16][ME]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, c32 = lane & 31;
  const int64_t r0 = (int64_t)blockIdx.x * a.chunk_rows;
  const int64_t r1 = r0 + a.chunk_rows < a.R ? r0 + a.chunk_rows : a.R;
  float* part = a.part + (size_t)blockIdx.x * a.n_params;
  const int ftiles = (d + 31) / 32;
  const int n1 = (MH / 32) * ftiles;           // dW1 tiles
  const int sweeps = (n1 + 4 * TPW - 1) / (4 * TPW);
  float db1 = 0.f, db2 = 0.f;                  // thread tid < MH: db1[tid]; tid < ME: db2[tid]
  for (int sw = 0; sw < sweeps; ++sw) {
    f32x16 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = (f32x16){0};
    f32x16 acc2[2] = {(f32x16){0}, (f32x16){0}};
    for (int64_t rb = r0; rb < r1; rb += 16) {
      __syncthreads();
      // stage 16 rows: scaled x, dA1, h, dZ (rows past r1 are zero)
      for (int i = tid; i < 16 * d; i += WG) {
        const int rr = i / d, f = i % d;
        const int64_t ri = rb + rr;
        xs[rr * DP + f] = ri < r1 ? a.X[(int64_t)a.rows[ri] * d + f] * a.scale : 0.f;
      }
      for (int i = tid; i < 16 * MH; i += WG) {
        const int rr = i / MH, c = i % MH;
        const int64_t ri = rb + rr;
        dAs[rr * (MH + 4) + c] = ri < r1 ? a.dA[ri * MH + c] : 0.f;
        hs[rr * (MH + 4) + c] = ri < r1 ? a.Hs[ri * MH + c] : 0.f;
      }
      for (int i = tid; i < 16 * ME; i += WG) {
        const int64_t ri = rb + i / ME;
        dzs[i] = ri < r1 ? a.dZ[ri * ME + i % ME] : 0.f;
      }
      __syncthreads();
      if (sw == 0) {
        if (tid < MH)
          for (int rr = 0; rr < 16; ++rr) db1 += dAs[rr * (MH + 4) + tid];
        if (tid < ME)
          for (int rr = 0; rr < 16; ++rr) db2 += dzs[rr * ME + tid];
      }
      // dW1 tiles of this sweep owned by wave w: indices sw*4*TPW + w*TPW + i
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int ti = sw * 4 * TPW + w * TPW + i;
        if (ti < n1) {   // uniform per wave
          const int ht = ti / ftiles, ft = ti % ftiles;
          float af[8], bf[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            af[e] = dAs[(8 * h + e) * (MH + 4) + ht * 32 + c32];
            const int f = ft * 32 + c32;
            bf[e] = f < d ? xs[(8 * h + e) * DP + f] : 0.f;
          }
          mma16<BF16>(acc[i], af, bf);
        }
      }
      if (sw == 0) {
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const int ht = w * 2 + i;   // 8 hidden tiles over 4 waves
          float af[8], bf[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            af[e] = c32 < ME ? dzs[(8 * h + e) * ME + c32] : 0.f;
            bf[e] = hs[(8 * h + e) * (MH + 4) + ht * 32 + c32];
          }
          mma16<BF16>(acc2[i], af, bf);
        }
      }
    }
    // write this sweep's dW1 tiles: element (hidden ht*32 + tile_row, feature ft*32 + c32)
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int ti = sw * 4 * TPW + w * TPW + i;
      if (ti < n1) {
        const int ht = ti / ftiles, ft = ti % ftiles;
        const int f = ft * 32 + c32;
        if (f < d) {
#pragma unroll
          for (int r = 0; r < 16; ++r) part[(size_t)(ht * 32 + tile_row(r, h)) * d + f] = acc[i][r];
        }
      }
    }
    if (sw == 0) {
      float* pW2 = part + (size_t)MH * d + MH;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ht = w * 2 + i;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int e = tile_row(r, h);
          if (e < ME) pW2[(size_t)e * MH + ht * 32 + c32] = acc2[i][r];
        }
      }
    }
  }
  if (tid < MH) part[(size_t)MH * d + tid] = db1;
  if (tid < ME) part[(size_t)MH * d + MH + (size_t)ME * MH + tid] = db2;
}

// grads[i] = sum over chunks c (in order) of part[c][i]; loss likewise.
__global__ __launch_bounds__(256) void k_mlp_reduce(MlpArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < a.n_params) {
    float s = 0.f;
    for (int c = 0; c < a.n_chunks; ++c) s += a.part[(size_t)c * a.n_params + i];
    a.grads[i] = s;
  }
  if (i == 0 && a.loss) {
    float l = 0.f;
    for (int b = 0; b < a.n_loss_parts; ++b) l += a.loss_part[b];
    *a.loss = l;
  }
}

// Adam with bias correction; bc1 = 1 - beta1^t and bc2 = 1 - beta2^t come
// from the host.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ params, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                  float b1, float b2, float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  params[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// Initial weights: W1 ~ U(-lim1, lim1), W2 ~ U(-lim2, lim2) from 24-bit
// uniforms of the counter generator; biases zero.
__global__ __launch_bounds__(256) void k_mlp_init(float* __restrict__ params, int d, uint64_t seed, float lim1,
                                                  float lim2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n1 = (int64_t)MH * d, nb1 = n1 + MH, n2 = nb1 + (int64_t)ME * MH, np = n2 + ME;
  if (i >= np) return;
  float val = 0.f;
  if (i < n1 || (i >= nb1 && i < n2)) {
    const uint64_t r = rand64(seed, TAG_MLP_INIT, 0, (uint32_t)i, 0);
    const float u = (float)(uint32_t)(r >> 40) * 0x1p-24f;
    val = (2.0f * u - 1.0f) * (i < n1 ? lim1 : lim2);
  }
  params[i] = val;
}

// Training pairs for step `step`: positives (i, ids[i][j]) for uniform i, j
// (a padded slot pairs i with itself, which adds nothing to the loss),
// negatives (a, b) uniform.  Integers in [0, n) come from the high half of
// a 64-bit product, which needs n < 2^32.
__global__ __launch_bounds__(256) void k_mlp_sample(const uint32_t* __restrict__ ids, int64_t n, int k, uint64_t seed,
                                                    uint32_t step, int n_pos, int n_neg, uint32_t* __restrict__ rows) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n_pos + n_neg) return;
  const bool pos = p < n_pos;
  const uint64_t r = rand64(seed, pos ? TAG_MLP_POS : TAG_MLP_NEG, step & 0xFFF, (uint32_t)p, step >> 12);
  const uint32_t i = (uint32_t)(((r >> 32) * (uint64_t)n) >> 32);
  uint32_t j;
  if (pos) {
    const uint32_t s = (uint32_t)(((r & 0xFFFFFFFFull) * (uint64_t)k) >> 32);
    j = ids[(int64_t)i * k + s];
    if (j == KNNG_NONE) j = i;
  } else {
    j = (uint32_t)(((r & 0xFFFFFFFFull) * (uint64_t)n) >> 32);
  }
  rows[2 * p] = i;
  rows[2 * p + 1] = j;
}

// Fraction of pairs whose endpoints share a leaf: leaf labels per point,
// then a count.
__global__ __launch_bounds__(256) void k_leaf_labels(const uint32_t* __restrict__ perm, const int64_t* __restrict__ leaf_off,
                                                     int64_t n_leaves, uint32_t* __restrict__ label) {
  const int64_t L = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (L >= n_leaves) return;
  for (int64_t j = leaf_off[L] + (threadIdx.x & 63); j < leaf_off[L + 1]; j += 64) label[perm[j]] = (uint32_t)L;
}

__global__ __launch_bounds__(256) void k_pair_same(const uint32_t* __restrict__ label, const uint32_t* __restrict__ pairs,
                                                   int64_t np, unsigned long long* __restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool same = p < np && label[pairs[2 * p]] == label[pairs[2 * p + 1]];
  const uint64_t b = __ballot(same);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(count, (unsigned long long)__popcll(b));
}

template <bool BF16, bool TRAIN>
hipError_t launch_fwd_t(const MlpArgs& a, hipStream_t s) {
  const unsigned grid = (unsigned)((a.R + (WG / 64) * 32 - 1) / ((WG / 64) * 32));
  if (grid == 0) return hipSuccess;
  const int ns = (a.d + 15) / 16;
  if (ns <= 2) hipLaunchKernelGGL((k_mlp_fwd<BF16, TRAIN, 2>), dim3(grid), dim3(WG), 0, s, a);
  else if (ns <= 4) hipLaunchKernelGGL((k_mlp_fwd<BF16, TRAIN, 4>), dim3(grid), dim3(WG), 0, s, a);
  else if (ns <= 8) hipLaunchKernelGGL((k_mlp_fwd<BF16, TRAIN, 8>), dim3(grid), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL((k_mlp_fwd<BF16, TRAIN, 16>), dim3(grid), dim3(WG), 0, s, a);
  return hipGetLastError();
}

}  // namespace

size_t mlp_wgrad_lds(int d) { return (size_t)(16 * (d + 4) + 2 * 16 * (MH + 4) + 16 * ME) * 4; }

hipError_t launch_mlp_forward(const MlpArgs& a, bool train, hipStream_t s) {
  if (a.bf16 && !train && !a.rows && a.d <= 128 && a.d % 16 == 0) {   // inference over the rows of X
    const int64_t n_tiles = (a.R + 127) / 128;
    if (n_tiles == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<int64_t>(n_tiles, (int64_t)cu_count() * 2);
    const int ns = a.d / 16;
    if (ns <= 2) hipLaunchKernelGGL(k_mlp_embed<2>, dim3(grid), dim3(WG), 0, s, a, n_tiles);
    else if (ns <= 4) hipLaunchKernelGGL(k_mlp_embed<4>, dim3(grid), dim3(WG), 0, s, a, n_tiles);
    else hipLaunchKernelGGL(k_mlp_embed<8>, dim3(grid), dim3(WG), 0, s, a, n_tiles);
    return hipGetLastError();
  }
  if (a.bf16) return train ? launch_fwd_t<true, true>(a, s) : launch_fwd_t<true, false>(a, s);
  return train ? launch_fwd_t<false, true>(a, s) : launch_fwd_t<false, false>(a, s);
}

// Loss, dZ, dA1, chunk partials, reduction into a.grads (and *a.loss).
hipError_t launch_mlp_backward(const MlpArgs& a, hipStream_t s) {
  const int np = a.n_pos + a.n_neg;
  hipLaunchKernelGGL(k_mlp_loss, dim3((np + 255) / 256), dim3(256), 0, s, a);
  const unsigned gr = (unsigned)((a.R + (WG / 64) * 32 - 1) / ((WG / 64) * 32));
  if (a.bf16) hipLaunchKernelGGL(k_mlp_bwd_h<true>, dim3(gr), dim3(WG), 0, s, a);
  else hipLaunchKernelGGL(k_mlp_bwd_h<false>, dim3(gr), dim3(WG), 0, s, a);
  const size_t lds = mlp_wgrad_lds(a.d);
  if (a.bf16) hipLaunchKernelGGL(k_mlp_wgrad<true>, dim3(a.n_chunks), dim3(WG), lds, s, a);
  else hipLaunchKernelGGL(k_mlp_wgrad<false>, dim3(a.n_chunks), dim3(WG), lds, s, a);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((a.n_params + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                           float eps, float bc1, float bc2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, params, g, m, v, n, lr, b1, b2,
                     eps, bc1, bc2);
  return hipGetLastError();
}

hipError_t launch_mlp_init(float* params, int d, uint64_t seed, float lim1, float lim2, hipStream_t s) {
  const int64_t np = (int64_t)MH * d + MH + (int64_t)ME * MH + ME;
  hipLaunchKernelGGL(k_mlp_init, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, params, d, seed, lim1, lim2);
  return hipGetLastError();
}

hipError_t launch_mlp_sample(const uint32_t* ids, int64_t n, int k, uint64_t seed, uint32_t step, int n_pos, int n_neg,
                             uint32_t* rows, hipStream_t s) {
  const int np = n_pos + n_neg;
  hipLaunchKernelGGL(k_mlp_sample, dim3((np + 255) / 256), dim3(256), 0, s, ids, n, k, seed, step, n_pos, n_neg, rows);
  return hipGetLastError();
}

hipError_t launch_coleaf(const uint32_t* perm, const int64_t* leaf_off, int64_t n_leaves, uint32_t* label,
                         const uint32_t* pairs, int64_t np, unsigned long long* count, hipStream_t s) {
  hipError_t e = launch_fill_u32((uint32_t*)count, 0u, 2, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_leaf_labels, dim3((unsigned)((n_leaves + 3) / 4)), dim3(256), 0, s, perm, leaf_off, n_leaves,
                     label);
  if (np > 0) hipLaunchKernelGGL(k_pair_same, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, label, pairs, np, count);
  return hipGetLastError();
}

}  // namespace knng
