// Device helpers shared by the gfx950 kernels (wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "knng_internal.h"

namespace knng {

constexpr int WAVE = 64;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Float with the total order used for split keys: -0 ranks as +0, then the
// IEEE order maps monotonically onto unsigned integers.
__device__ __forceinline__ uint32_t ordered_key(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) == 0) u = 0;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// (distance, id) packed so that unsigned order is (distance, id) order for
// distance >= 0; the empty entry (KNNG_NONE, +inf) packs to all ones.
__device__ __forceinline__ uint64_t pack_did(float d, uint32_t id) {
  return id == KNNG_NONE ? ~0ull : (((uint64_t)__float_as_uint(d)) << 32) | id;
}
__device__ __forceinline__ float key_dist(uint64_t k) {
  return k == ~0ull ? __int_as_float(0x7F800000) : __uint_as_float((uint32_t)(k >> 32));
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return k == ~0ull ? KNNG_NONE : (uint32_t)k; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = __shfl_xor((unsigned)(v & 0xFFFFFFFFu), m);
  uint32_t hi = __shfl_xor((unsigned)(v >> 32), m);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((unsigned)(v & 0xFFFFFFFFu), src);
  uint32_t hi = __shfl((unsigned)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int delta) {
  uint32_t lo = __shfl_up((unsigned)(v & 0xFFFFFFFFu), delta);
  uint32_t hi = __shfl_up((unsigned)(v >> 32), delta);
  return ((uint64_t)hi << 32) | lo;
}

// Element e-1 of a wave-distributed array (element e = r*64 + lane); `none`
// before the first element.  All lanes must call it.
template <int R>
__device__ __forceinline__ uint64_t prev_elem(const uint64_t (&v)[R], int r, int lane, uint64_t none) {
  uint64_t up = shfl_up_u64(v[r], 1);
  uint64_t last = r > 0 ? shfl_u64(v[r > 0 ? r - 1 : 0], 63) : none;
  return lane == 0 ? last : up;
}
template <int R>
__device__ __forceinline__ uint32_t prev_elem(const uint32_t (&v)[R], int r, int lane, uint32_t none) {
  uint32_t up = __shfl_up(v[r], 1);
  uint32_t last = r > 0 ? (uint32_t)__shfl(v[r > 0 ? r - 1 : 0], 63) : none;
  return lane == 0 ? last : up;
}

// Canonical squared distance between two rows of d floats (d % 4 == 0),
// computed by one group of 16 lanes: lane g of the group owns the float4
// chunks g, g+16, g+32, ...; each of its four components accumulates
// fma(diff, diff, acc) in increasing chunk order; the lane sums
// (a0 + a1) + (a2 + a3); the group then adds across lanes with an xor
// butterfly (8, 4, 2, 1).  Every lane of the group returns the same value,
// and dist2(x, y) == dist2(y, x) bit for bit.  All 16 lanes must take part.
__device__ __forceinline__ float dist2_g16(const float* __restrict__ x, const float* __restrict__ y, int d, int g) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  const float4* xv = (const float4*)x;
  const float4* yv = (const float4*)y;
  int nc = d >> 2;
  for (int c = g; c < nc; c += 16) {
    float4 u = xv[c], w = yv[c];
    float e0 = u.x - w.x, e1 = u.y - w.y, e2 = u.z - w.z, e3 = u.w - w.w;
    a0 = __builtin_fmaf(e0, e0, a0);
    a1 = __builtin_fmaf(e1, e1, a1);
    a2 = __builtin_fmaf(e2, e2, a2);
    a3 = __builtin_fmaf(e3, e3, a3);
  }
  float s = (a0 + a1) + (a2 + a3);
  s += __shfl_xor(s, 8, 16);
  s += __shfl_xor(s, 4, 16);
  s += __shfl_xor(s, 2, 16);
  s += __shfl_xor(s, 1, 16);
  return s;
}

// Same as dist2_g16 with the first row already held by the lane as its
// float4 chunks (xr[i] = chunk g + 16 i).
template <int NCH>
__device__ __forceinline__ float dist2_g16_reg(const float4 (&xr)[NCH], const float* __restrict__ y, int d, int g) {
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  const float4* yv = (const float4*)y;
  int nc = d >> 2;
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    int c = g + 16 * i;
    if (c < nc) {
      float4 u = xr[i], w = yv[c];
      float e0 = u.x - w.x, e1 = u.y - w.y, e2 = u.z - w.z, e3 = u.w - w.w;
      a0 = __builtin_fmaf(e0, e0, a0);
      a1 = __builtin_fmaf(e1, e1, a1);
      a2 = __builtin_fmaf(e2, e2, a2);
      a3 = __builtin_fmaf(e3, e3, a3);
    }
  }
  float s = (a0 + a1) + (a2 + a3);
  s += __shfl_xor(s, 8, 16);
  s += __shfl_xor(s, 4, 16);
  s += __shfl_xor(s, 2, 16);
  s += __shfl_xor(s, 1, 16);
  return s;
}

// dist2_g16_reg for four rows at once (the same arithmetic for each pair);
// the four rows' loads are in flight together.
template <int NCH>
__device__ __forceinline__ void dist2_g16_reg4(const float4 (&xr)[NCH], const float* const (&y)[4], int d, int g,
                                               float (&out)[4]) {
  float a[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0.f;
  const int nc = d >> 2;
#pragma unroll
  for (int i = 0; i < NCH; ++i) {
    const int c = g + 16 * i;
    if (c < nc) {
      float4 w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = ((const float4*)y[u])[c];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 x = xr[i];
        float e0 = x.x - w[u].x, e1 = x.y - w[u].y, e2 = x.z - w[u].z, e3 = x.w - w[u].w;
        a[u][0] = __builtin_fmaf(e0, e0, a[u][0]);
        a[u][1] = __builtin_fmaf(e1, e1, a[u][1]);
        a[u][2] = __builtin_fmaf(e2, e2, a[u][2]);
        a[u][3] = __builtin_fmaf(e3, e3, a[u][3]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    float s = (a[u][0] + a[u][1]) + (a[u][2] + a[u][3]);
    s += __shfl_xor(s, 8, 16);
    s += __shfl_xor(s, 4, 16);
    s += __shfl_xor(s, 2, 16);
    s += __shfl_xor(s, 1, 16);
    out[u] = s;
  }
}

// Bitonic sort across the wave of R registers per lane: element e = r*64+lane.
// Sorts blocks of SEG consecutive elements ascending (SEG = 64*R sorts all).
template <int R, int SEG, typename K>
__device__ __forceinline__ void wave_bitonic(K (&v)[R], int lane) {
#pragma unroll
  for (int size = 2; size <= SEG; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride / 64;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if ((r & rs) == 0) {
            int e = r * 64 + lane;
            bool asc = (size == SEG) ? true : ((e & size) == 0);
            K a = v[r], b = v[r + rs];
            bool sw = asc ? (a > b) : (a < b);
            v[r] = sw ? b : a;
            v[r + rs] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int e = r * 64 + lane;
          K o;
          if constexpr (sizeof(K) == 8) o = shfl_xor_u64(v[r], stride);
          else o = __shfl_xor(v[r], stride);
          bool asc = (size == SEG) ? true : ((e & size) == 0);
          bool lower = (lane & stride) == 0;
          // lower element keeps the min when ascending
          bool take_min = (lower == asc);
          v[r] = take_min ? (o < v[r] ? o : v[r]) : (o > v[r] ? o : v[r]);
        }
      }
    }
  }
}

// Exclusive prefix count of `flag` over the wave (in lane order) and total.
__device__ __forceinline__ int wave_prefix_count(bool flag, int lane, int* total) {
  uint64_t b = __ballot(flag);
  *total = __popcll(b);
  uint64_t below = lane == 0 ? 0ull : (b & ((~0ull) >> (64 - lane)));
  return __popcll(below);
}

}  // namespace knng
