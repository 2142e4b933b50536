// Rows scaled to unit length for the cosine distance (Definition 1 names it
// beside the Euclidean distance): the squared Euclidean distance of two unit
// rows is 2 (1 - cos theta), which ranks like the cosine distance, so the
// whole method runs unchanged on the scaled rows.
//
// The arithmetic is fixed so that any implementation can reproduce it bit
// for bit: the squared norm is summed over the features left to right in
// float32, each product and each sum rounded on its own (no fused
// multiply-add), then the square root and every quotient are correctly
// rounded.  A zero row stays zero.
#include "knng_dev.h"

namespace knng {

namespace {

constexpr int NR_ROWS = 64;   // rows per workgroup
constexpr int NR_COLS = 64;   // features staged per step

// 256 threads, 64 rows: a 64 x 64 tile of X is staged through LDS with
// coalesced loads; thread r < 64 then walks its row's 64 values in feature
// order.  The quotients are written with coalesced stores.
__global__ __launch_bounds__(256) void k_normalize(const float* __restrict__ X, int64_t n, int d,
                                                   float* __restrict__ Xn) {
#pragma clang fp contract(off)
  __shared__ float tile[NR_ROWS][NR_COLS + 1];
  __shared__ float nrm[NR_ROWS];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * NR_ROWS;
  float acc = 0.f;
  for (int c0 = 0; c0 < d; c0 += NR_COLS) {
    for (int e = tid; e < NR_ROWS * NR_COLS; e += 256) {
      const int r = e / NR_COLS, c = e % NR_COLS;
      const int64_t row = r0 + r;
      tile[r][c] = (row < n && c0 + c < d) ? X[row * d + c0 + c] : 0.f;
    }
    __syncthreads();
    if (tid < NR_ROWS) {
      const int cn = d - c0 < NR_COLS ? d - c0 : NR_COLS;
      for (int c = 0; c < cn; ++c) {
        const float x = tile[tid][c];
        const float sq = x * x;
        acc = acc + sq;
      }
    }
    __syncthreads();
  }
  if (tid < NR_ROWS) nrm[tid] = __builtin_sqrtf(acc);   // correctly rounded (no fast-math flags)
  __syncthreads();
  for (int e = tid; e < NR_ROWS * d; e += 256) {
    const int r = e / d, c = e % d;
    const int64_t row = r0 + r;
    if (row < n) {
      const float q = nrm[r];
      const float x = X[row * d + c];
      Xn[row * d + c] = q > 0.f ? x / q : 0.f;   // correctly rounded quotient
    }
  }
}

}  // namespace

hipError_t launch_normalize(const float* X, int64_t n, int d, float* Xn, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((n + NR_ROWS - 1) / NR_ROWS);
  hipLaunchKernelGGL(k_normalize, dim3(blocks), dim3(256), 0, s, X, n, d, Xn);
  return hipGetLastError();
}

}  // namespace knng
