// One level of a random division (Section 3.1; appendix median bipartition;
// Section 3.4 principal direction): project every point of every internal
// node, select each node's split key by a 3-pass radix select over the
// ordered key bits, and stable-partition the node's segment of the
// permutation.  A node's segment is always sorted by point id (children keep
// their parent's order and the root is 0..n-1), so the (key, id) order of
// the split is "key, then position in the segment".
#include "knng_dev.h"

#include <algorithm>

namespace knng {

namespace {

constexpr int DIV_THREADS = 256;
constexpr int HB[3] = {(int)HIST_B0, (int)HIST_B1, (int)HIST_B2};
__constant__ int c_hist_base[3] = {0, (int)HIST_B0, (int)(HIST_B0 + HIST_B1)};

// --------------------------------------------------------------- block scans
__device__ __forceinline__ int block_excl_scan(int v, int* sh, int* total) {
  // 256 threads = 4 waves
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int s = sh[i];
    base += (i < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// After histogram pass q of a level: each segment's key prefix after q + 1
// passes and the rank of the left child's last key inside that prefix, from
// the previous pass's (prefix, rank) and one scan of pass q's histogram.  One
// workgroup per segment, once per pass; the pass kernels of every chunk of
// the segment then read two words instead of walking the histograms.
__global__ __launch_bounds__(DIV_THREADS) void k_resolve_step(DivideLevelArgs a, int q) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  __shared__ int sh[16];
  const uint32_t sl = blockIdx.x;
  uint32_t* g = a.hist + (size_t)sl * HIST_TOTAL;
  uint32_t pre = 0, r = a.segs[sl].left;
  if (q > 0) {
    pre = g[HIST_PR + 2 * (q - 1)];
    r = g[HIST_PR + 2 * (q - 1) + 1];
  }
  const uint32_t* h = g + c_hist_base[q];
  const int per = HB[q] / DIV_THREADS;   // 8 or 4 bins per thread
  const int b0 = threadIdx.x * per;
  int mysum = 0;
  for (int i = 0; i < per; ++i) mysum += (int)h[b0 + i];
  int tot;
  const int before = block_excl_scan(mysum, sh, &tot);
  if ((uint32_t)before <= r && r < (uint32_t)(before + mysum)) {   // exactly one thread
    uint32_t c = before;
    for (int i = 0; i < per; ++i) {
      const uint32_t hv = h[b0 + i];
      if (r < c + hv) {
        const int bits = (q == 2) ? 10 : 11;
        g[HIST_PR + 2 * q] = (pre << bits) | (uint32_t)(b0 + i);
        g[HIST_PR + 2 * q + 1] = r - c;
        break;
      }
      c += hv;
    }
  }
}

// --------------------------------------------------------------- direction
__device__ void load_direction(const DivideLevelArgs& a, const SegDesc& sd, float* dir, bool first_item) {
  for (int j = threadIdx.x; j < a.d; j += DIV_THREADS) {
    float v;
    if (a.dirs) v = a.dirs[(size_t)sd.dir_index * a.d + j];
    else if (a.pca_iters > 0) v = a.pca_dirs[(size_t)sd.dir_index * a.d + j];
    else v = rp_entry(a.seed, sd.t, sd.v, (uint32_t)j);
    dir[j] = v;
    if (a.dirs_out && first_item) a.dirs_out[(size_t)sd.dir_index * a.d + j] = v;
  }
  __syncthreads();
}

// key = a . x in float32, left to right, every product and sum rounded.
__device__ __forceinline__ float dot_seq(const float* __restrict__ x, const float* __restrict__ a, int d) {
#pragma clang fp contract(off)
  float acc = 0.f;
  const float4* xv = (const float4*)x;
  const int c4 = d >> 2;
  int c = 0;
  // eight float4 (a 128-byte line of the row) in flight per step; the
  // products and sums still run left to right
  for (; c + 8 <= c4; c += 8) {
    float4 u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = xv[c + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float* ak = a + 4 * (c + k);
      float p0 = u[k].x * ak[0];
      acc = acc + p0;
      float p1 = u[k].y * ak[1];
      acc = acc + p1;
      float p2 = u[k].z * ak[2];
      acc = acc + p2;
      float p3 = u[k].w * ak[3];
      acc = acc + p3;
    }
  }
  if (c < c4) {   // the last 1..7 float4, all loads in flight together
    const int r = c4 - c;
    float4 u[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) u[k] = k < r ? xv[c + k] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k < r) {
        const float* ak = a + 4 * (c + k);
        float p0 = u[k].x * ak[0];
        acc = acc + p0;
        float p1 = u[k].y * ak[1];
        acc = acc + p1;
        float p2 = u[k].z * ak[2];
        acc = acc + p2;
        float p3 = u[k].w * ak[3];
        acc = acc + p3;
      }
    }
  }
  return acc;
}

// Four bytes of the one-byte copy of X as the float4 of X they hold.
__device__ __forceinline__ float4 bytes4(uint32_t b) {
  return make_float4((float)(b & 0xFFu), (float)((b >> 8) & 0xFFu), (float)((b >> 16) & 0xFFu), (float)(b >> 24));
}

// dot_seq on a row of the one-byte copy: the same values in the same order,
// so the same result.  A 128-value block (eight 16-byte loads, the whole row
// at d = 128) is in flight at once, a quarter of the float row's bytes.
__device__ __forceinline__ float dot_seq_u8(const uint8_t* __restrict__ x, const float* __restrict__ a, int d) {
#pragma clang fp contract(off)
  float acc = 0.f;
  const int c4 = d >> 2;
  int c = 0;
  auto quad = [&](uint32_t wb, int cc) {
    const float4 u = bytes4(wb);
    const float* ak = a + 4 * cc;
    float p0 = u.x * ak[0];
    acc = acc + p0;
    float p1 = u.y * ak[1];
    acc = acc + p1;
    float p2 = u.z * ak[2];
    acc = acc + p2;
    float p3 = u.w * ak[3];
    acc = acc + p3;
  };
  if ((d & 15) == 0) {
    const uint4* xv = (const uint4*)x;
    for (; c + 32 <= c4; c += 32) {
      uint4 w[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = xv[c / 4 + k];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        quad(w[k].x, c + 4 * k);
        quad(w[k].y, c + 4 * k + 1);
        quad(w[k].z, c + 4 * k + 2);
        quad(w[k].w, c + 4 * k + 3);
      }
    }
  }
  const uint32_t* xw = (const uint32_t*)x;
  for (; c + 8 <= c4; c += 8) {
    uint32_t w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = xw[c + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) quad(w[k], c + k);
  }
  for (; c < c4; ++c) quad(xw[c], c);
  return acc;
}

// --------------------------------------------------------------- kernels
__global__ __launch_bounds__(DIV_THREADS) void k_proj_hist0(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  extern __shared__ float dir[];
  __shared__ uint32_t lh[HIST_B0];
  const ItemDesc it = a.items[blockIdx.x];
  const SegDesc sd = a.segs[it.seg];
  const bool hist = a.small == 0u;   // uniform: small segments are selected in LDS instead
  if (hist)
    for (int b = threadIdx.x; b < (int)HIST_B0; b += DIV_THREADS) lh[b] = 0;
  load_direction(a, sd, dir, it.start == sd.off);
  const size_t base = (size_t)it.slot * (size_t)a.n;
  const bool u8 = a.X8 && (*a.flags & EXACT_U8) != 0u;   // uniform
  for (uint32_t i = threadIdx.x; i < it.len; i += DIV_THREADS) {
    size_t pos = base + it.start + i;
    uint32_t row = a.perm_in[pos];
    float key = u8 ? dot_seq_u8(a.X8 + (size_t)row * a.d, dir, a.d) : dot_seq(a.X + (size_t)row * a.d, dir, a.d);
    uint32_t uk = ordered_key(key);
    a.ukeys[pos] = uk;
    if (hist) atomicAdd(&lh[uk >> 21], 1u);
  }
  if (!hist) return;
  __syncthreads();
  uint32_t* gh = a.hist + (size_t)it.seg * HIST_TOTAL;
  for (int b = threadIdx.x; b < (int)HIST_B0; b += DIV_THREADS)
    if (lh[b]) atomicAdd(&gh[b], lh[b]);
}

__global__ __launch_bounds__(DIV_THREADS) void k_hist_pass(DivideLevelArgs a, int pass) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  __shared__ uint32_t lh[HIST_B1];
  const ItemDesc it = a.items[blockIdx.x];
  const uint32_t prefix = a.hist[(size_t)it.seg * HIST_TOTAL + HIST_PR + 2 * (pass - 1)];   // from k_resolve_step
  int nb = HB[pass];
  for (int b = threadIdx.x; b < nb; b += DIV_THREADS) lh[b] = 0;
  __syncthreads();
  int shift_pre = pass == 1 ? 21 : 10;
  const uint32_t* uks = a.ukeys + (size_t)it.slot * (size_t)a.n + it.start;
  for (uint32_t i = threadIdx.x; i < it.len; i += DIV_THREADS) {
    uint32_t uk = uks[i];
    if ((uk >> shift_pre) == prefix) {
      uint32_t dg = pass == 1 ? ((uk >> 10) & 0x7FF) : (uk & 0x3FF);
      atomicAdd(&lh[dg], 1u);
    }
  }
  __syncthreads();
  uint32_t* gh = a.hist + (size_t)it.seg * HIST_TOTAL + c_hist_base[pass];
  for (int b = threadIdx.x; b < nb; b += DIV_THREADS)
    if (lh[b]) atomicAdd(&gh[b], lh[b]);
}

// A level whose segments all hold at most DIV_SMALL points: one workgroup
// per segment loads the segment's keys into LDS, finds the key of rank
// `left` by four 8-bit radix passes over LDS histograms, and writes the
// stable partition (keys below it, then the first `need` keys equal to it,
// left; the rest right, each side in position order) -- the same pivot,
// count and order as the histogram passes and chunked scatter of larger
// segments.  The segment's first item does the work; copy items copy.
__global__ __launch_bounds__(DIV_THREADS) void k_small_partition(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  __shared__ uint32_t keys[DIV_SMALL];
  __shared__ uint32_t hb[256];
  __shared__ uint32_t pick[2];
  __shared__ int sh[16];
  const ItemDesc it = a.items[blockIdx.x];
  const size_t base = (size_t)it.slot * (size_t)a.n;
  const uint32_t* pin = a.perm_in + base;
  uint32_t* pout = a.perm_out + base;
  if (it.seg == 0xFFFFFFFFu) {   // positions outside this level's internal nodes
    for (uint32_t i = threadIdx.x; i < it.len; i += DIV_THREADS) pout[it.start + i] = pin[it.start + i];
    return;
  }
  const SegDesc sd = a.segs[it.seg];
  if (it.start != sd.off) return;   // uniform: not the segment's first item
  const uint32_t m = sd.m;
  for (uint32_t i = threadIdx.x; i < m; i += DIV_THREADS) keys[i] = a.ukeys[base + sd.off + i];
  uint32_t prefix = 0, r = sd.left;   // rank of the pivot among the segment's keys
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hb[threadIdx.x] = 0;   // 256 threads, 256 bins
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < m; i += DIV_THREADS) {
      const uint32_t uk = keys[i];
      if (pass == 0 || (uk >> (shift + 8)) == prefix) atomicAdd(&hb[(uk >> shift) & 255u], 1u);
    }
    __syncthreads();
    const int c = (int)hb[threadIdx.x];
    int tot;
    const int before = block_excl_scan(c, sh, &tot);
    if ((uint32_t)before <= r && r < (uint32_t)(before + c)) {   // exactly one thread
      pick[0] = threadIdx.x;
      pick[1] = (uint32_t)before;
    }
    __syncthreads();
    prefix = (prefix << 8) | pick[0];
    r -= pick[1];
    __syncthreads();   // pick and hb are rewritten by the next pass
  }
  const uint32_t pivot = prefix, need = r;   // need: keys equal to the pivot that go left
  int less_before = 0, eq_before = 0;
  for (uint32_t t0 = 0; t0 < m; t0 += DIV_THREADS) {
    const uint32_t i = t0 + threadIdx.x;
    const bool valid = i < m;
    const uint32_t uk = valid ? keys[i] : 0xFFFFFFFFu;
    const int isl = valid && uk < pivot, ise = valid && uk == pivot;
    int tl, te;
    const int rl = block_excl_scan(isl, sh, &tl);
    const int re = block_excl_scan(ise, sh, &te);
    if (valid) {
      const uint32_t nless = (uint32_t)(less_before + rl), neq = (uint32_t)(eq_before + re);
      uint32_t dest;
      if (isl) dest = sd.off + nless + (neq < need ? neq : need);
      else if (ise && neq < need) dest = sd.off + nless + neq;
      else dest = sd.off + sd.left + (i - nless - (neq < need ? neq : need));
      pout[dest] = pin[sd.off + i];
    }
    less_before += tl;
    eq_before += te;
  }
}

__global__ __launch_bounds__(DIV_THREADS) void k_part_count(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  __shared__ int sh[16];
  const ItemDesc it = a.items[blockIdx.x];
  const uint32_t pivot = a.hist[(size_t)it.seg * HIST_TOTAL + HIST_PR + 4];   // the left child's last key
  int nl = 0, ne = 0;
  const uint32_t* uks = a.ukeys + (size_t)it.slot * (size_t)a.n + it.start;
  for (uint32_t i = threadIdx.x; i < it.len; i += DIV_THREADS) {
    uint32_t uk = uks[i];
    nl += uk < pivot;
    ne += uk == pivot;
  }
  int tl, te;
  block_excl_scan(nl, sh, &tl);
  block_excl_scan(ne, sh, &te);
  if (threadIdx.x == 0) {
    a.chunk_cnt[2 * blockIdx.x] = (uint32_t)tl;
    a.chunk_cnt[2 * blockIdx.x + 1] = (uint32_t)te;
  }
}

__global__ __launch_bounds__(DIV_THREADS) void k_part_scatter(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  __shared__ int sh[16];
  const ItemDesc it = a.items[blockIdx.x];
  const size_t base = (size_t)it.slot * (size_t)a.n;
  const uint32_t* pin = a.perm_in + base;
  uint32_t* pout = a.perm_out + base;
  if (it.seg == 0xFFFFFFFFu) {   // positions outside this level's internal nodes
    for (uint32_t i = threadIdx.x; i < it.len; i += DIV_THREADS) pout[it.start + i] = pin[it.start + i];
    return;
  }
  const SegDesc sd = a.segs[it.seg];
  const uint32_t pivot = a.hist[(size_t)it.seg * HIST_TOTAL + HIST_PR + 4];   // from k_resolve_step
  const uint32_t need = a.hist[(size_t)it.seg * HIST_TOTAL + HIST_PR + 5];
  // counts of the segment's earlier chunks
  int pl = 0, pe = 0;
  for (uint32_t c = sd.first_item + threadIdx.x; c < blockIdx.x; c += DIV_THREADS) {
    pl += (int)a.chunk_cnt[2 * c];
    pe += (int)a.chunk_cnt[2 * c + 1];
  }
  int less_before, eq_before;
  block_excl_scan(pl, sh, &less_before);
  block_excl_scan(pe, sh, &eq_before);
  uint32_t base_idx = it.start - sd.off;
  for (uint32_t t0 = 0; t0 < it.len; t0 += DIV_THREADS) {
    uint32_t i = t0 + threadIdx.x;
    bool valid = i < it.len;
    uint32_t uk = valid ? a.ukeys[base + it.start + i] : 0xFFFFFFFFu;
    int isl = valid && uk < pivot, ise = valid && uk == pivot;
    int tl, te;
    int rl = block_excl_scan(isl, sh, &tl);
    int re = block_excl_scan(ise, sh, &te);
    if (valid) {
      uint32_t nless = (uint32_t)(less_before + rl);   // less-than elements before this one
      uint32_t neq = (uint32_t)(eq_before + re);        // equal elements before this one
      uint32_t idx = base_idx + i;
      uint32_t dest;
      if (isl) {
        dest = sd.off + nless + (neq < need ? neq : need);
      } else if (ise && neq < need) {
        dest = sd.off + nless + neq;
      } else {
        uint32_t lbefore = nless + (neq < need ? neq : need);
        dest = sd.off + sd.left + (idx - lbefore);
      }
      pout[dest] = pin[it.start + i];
    }
    less_before += tl;
    eq_before += te;
  }
}

// Principal direction of one node's sample by FP32 power iteration (Section
// 3.4 takes the principal direction of points sampled from the subset), with
// the whole sample in LDS (d <= PCA_LDS_DMAX).  t = Y v: a thread per sample
// row, float4 over the columns.  w = Y^T t: a thread per (column quad, slab
// of rows); slab partials are added in a fixed order (four chains).  The
// mean is formed the same way.  The sample, start vector, iteration count
// and sign rule are those of k_pca_dirs.
// U8 = false: the sample is stored as floats, rows padded to d + 4 floats
// (float4 reads of one column by consecutive rows fall in different banks),
// and centred in place.  U8 = true (every value of X an integer in 0..255):
// the rows are kept as bytes, padded to d + 4 bytes, and centred as they are
// read; (float)byte - mean is the value the float form stores, so the
// direction is the same bit for bit, and the quarter-size stage lets four
// nodes share a CU.  Both forms are launched; each returns at once unless the
// data check chose it.  Workgroups stride over the level's segments.
constexpr int PCA_LDS_DMAX = 136;   // 256 (d + 4) + 2d + 256 + 1024 floats fit 150 KB

template <bool U8>
__global__ __launch_bounds__(DIV_THREADS) void k_pca_lds(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  const bool u8 = a.X8 && (*a.flags & EXACT_U8) != 0u;   // uniform
  if (u8 != U8) return;
  extern __shared__ float smem[];
  const int d = a.d;
  const int ld = d + 4;                        // row stride: floats (U8: bytes)
  const int cw = d >> 2;                       // column quads
  const int G = DIV_THREADS / cw;              // row slabs
  float* Y = smem;                             // 256 x ld floats
  uint8_t* Yb = reinterpret_cast<uint8_t*>(smem);   // 256 x ld bytes
  float* v = U8 ? smem + 64 * ld : Y + 256 * ld;    // d
  float* mu = v + d;                           // d
  float* tt = mu + d;                          // 256
  float4* part = (float4*)(tt + 256);          // G x cw
  // the sample's row ids share the partials' room: read only while staging,
  // before the first partial is written (each segment starts after a barrier)
  uint32_t* rows = reinterpret_cast<uint32_t*>(part);
  __shared__ float red[DIV_THREADS / 64];
  __shared__ float red2[DIV_THREADS / 64];
  __shared__ int redi[DIV_THREADS / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int q = tid % cw, g = tid / cw;
  for (uint32_t seg = blockIdx.x; seg < a.n_segs; seg += gridDim.x) {
  const SegDesc sd = a.segs[seg];
  const uint32_t m = sd.m;
  const uint32_t s = m < 256 ? m : 256;
  uint32_t wd = m / s;
  if (wd < 1) wd = 1;
  if (tid < (int)s) {
    uint32_t pos = (uint32_t)(((uint64_t)tid * m) / s) + (uint32_t)(rand64(a.seed, TAG_SAMPLE, sd.t, sd.v, tid) % wd);
    rows[tid] = a.perm_in[(size_t)sd.slot * (size_t)a.n + sd.off + pos];
  }
  for (int j = tid; j < d; j += DIV_THREADS) v[j] = rp_entry(a.seed, sd.t, sd.v, (uint32_t)j);
  __syncthreads();
  // raw sample -> LDS, 8 loads in flight per thread
  {
    const int tot = (int)s * cw;
    for (int e0 = tid; e0 < tot; e0 += DIV_THREADS * 8) {
      if constexpr (U8) {
        uint32_t wb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int e = e0 + u * DIV_THREADS;
          wb[u] = e < tot ? ((const uint32_t*)(a.X8 + (size_t)rows[e / cw] * d))[e % cw] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int e = e0 + u * DIV_THREADS;
          if (e < tot) *(uint32_t*)(Yb + (e / cw) * ld + 4 * (e % cw)) = wb[u];
        }
      } else {
        float4 buf[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int e = e0 + u * DIV_THREADS;
          buf[u] = e < tot ? ((const float4*)(a.X + (size_t)rows[e / cw] * d))[e % cw] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          int e = e0 + u * DIV_THREADS;
          if (e < tot) *(float4*)(Y + (e / cw) * ld + 4 * (e % cw)) = buf[u];
        }
      }
    }
  }
  __syncthreads();
  bool centred = false;
  // column quad qq of sample row i, centred once the mean is known
  auto yq = [&](uint32_t i, int qq) -> float4 {
    if constexpr (U8) {
      const uint32_t b = *(const uint32_t*)(Yb + i * ld + 4 * qq);
      float4 y = make_float4((float)(b & 0xFFu), (float)((b >> 8) & 0xFFu), (float)((b >> 16) & 0xFFu), (float)(b >> 24));
      if (centred) {
        const float4 m4 = *(const float4*)(mu + 4 * qq);
        y.x -= m4.x; y.y -= m4.y; y.z -= m4.z; y.w -= m4.w;
      }
      return y;
    } else {
      return *(const float4*)(Y + i * ld + 4 * qq);
    }
  };
  const uint32_t rps = (s + G - 1) / G;        // rows per slab
  // column sums over a slab of rows, weighted by wt[i] (or 1), into part[g][q]
  auto slab_sums = [&](const float* wt) {
    if (g < G) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      const uint32_t i0 = g * rps, i1 = min(s, i0 + rps);
#pragma unroll 8
      for (uint32_t i = i0; i < i1; ++i) {
        const float4 y = yq(i, q);
        const float c = wt ? wt[i] : 1.f;
        acc.x = __builtin_fmaf(y.x, c, acc.x);
        acc.y = __builtin_fmaf(y.y, c, acc.y);
        acc.z = __builtin_fmaf(y.z, c, acc.z);
        acc.w = __builtin_fmaf(y.w, c, acc.w);
      }
      part[g * cw + q] = acc;
    }
    __syncthreads();
  };
  // slab partials of column quad qq summed in four interleaved chains (slab
  // g into chain g mod 4), then (c0 + c1) + (c2 + c3): a fixed order whose
  // dependent chain is a quarter as long (G reaches 64 at d = 16)
  auto col_total = [&](int qq) -> float4 {
    float4 c[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    auto add = [](float4& r, const float4 p4) { r.x += p4.x; r.y += p4.y; r.z += p4.z; r.w += p4.w; };
    int gg = 0;
    for (; gg + 4 <= G; gg += 4) {
#pragma unroll
      for (int j = 0; j < 4; ++j) add(c[j], part[(gg + j) * cw + qq]);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j)
      if (gg + j < G) add(c[j], part[(gg + j) * cw + qq]);
    add(c[0], c[1]);
    add(c[2], c[3]);
    add(c[0], c[2]);
    return c[0];
  };

  // mean and centring
  slab_sums(nullptr);
  if (tid < cw) {
    const float4 t4 = col_total(tid);
    const float is = 1.0f / (float)s;
    mu[4 * tid + 0] = t4.x * is;
    mu[4 * tid + 1] = t4.y * is;
    mu[4 * tid + 2] = t4.z * is;
    mu[4 * tid + 3] = t4.w * is;
  }
  __syncthreads();
  if constexpr (!U8) {
    for (int e = tid; e < (int)s * cw; e += DIV_THREADS) {
      float4* yr = (float4*)(Y + (e / cw) * ld + 4 * (e % cw));
      const float4 m4 = *(const float4*)(mu + 4 * (e % cw));
      float4 y = *yr;
      y.x -= m4.x; y.y -= m4.y; y.z -= m4.z; y.w -= m4.w;
      *yr = y;
    }
  }
  // The float stage is centred in place; the byte stage stays raw and is
  // centred algebraically: (y_i - mu).v = y_i.v - mu.v, so t = Y v costs a
  // conversion and an FMA per byte plus one scalar per row, and w = Y^T t
  // needs no centring at all because a centred sample's t sums to zero
  // (sum_i (y_i - mu) = 0 for the sample mean mu).
  centred = !U8;
  auto block_sum2 = [&](float& x, float& y) {
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_xor(x, o);
      y += __shfl_xor(y, o);
    }
    if (lane == 0) {
      red[wv] = x;
      red2[wv] = y;
    }
    __syncthreads();
    x = 0.f;
    y = 0.f;
    for (int i = 0; i < DIV_THREADS / 64; ++i) {
      x += red[i];
      y += red2[i];
    }
    __syncthreads();
  };
  // normalise the start vector (and, for bytes, mu.v of the unit vector)
  float nn = 0.f, mv = 0.f;
  for (int j = tid; j < d; j += DIV_THREADS) {
    nn += v[j] * v[j];
    if constexpr (U8) mv = __builtin_fmaf(mu[j], v[j], mv);
  }
  block_sum2(nn, mv);
  float cmv;   // mu . v of the current unit v (bytes only)
  {
    const float inv = nn > 0.f ? 1.0f / sqrtf(nn) : 0.f;
    for (int j = tid; j < d; j += DIV_THREADS) v[j] *= inv;
    cmv = mv * inv;
  }
  __syncthreads();
  for (int itr = 0; itr < a.pca_iters; ++itr) {
    if (tid < (int)s) {   // t = Y v
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 8
      for (int c = 0; c < cw; ++c) {
        const float4 y = yq(tid, c);
        const float4 vv = *(const float4*)(v + 4 * c);
        acc.x = __builtin_fmaf(y.x, vv.x, acc.x);
        acc.y = __builtin_fmaf(y.y, vv.y, acc.y);
        acc.z = __builtin_fmaf(y.z, vv.z, acc.z);
        acc.w = __builtin_fmaf(y.w, vv.w, acc.w);
      }
      const float dot = (acc.x + acc.y) + (acc.z + acc.w);
      tt[tid] = U8 ? dot - cmv : dot;
    }
    __syncthreads();
    slab_sums(tt);   // w = Y^T t, by slabs
    float sq = 0.f, mw = 0.f;
    float4 w4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < cw) {
      w4 = col_total(tid);
      sq = w4.x * w4.x + w4.y * w4.y + w4.z * w4.z + w4.w * w4.w;
      if constexpr (U8) {
        const float4 m4 = *(const float4*)(mu + 4 * tid);
        mw = m4.x * w4.x + m4.y * w4.y + m4.z * w4.z + m4.w * w4.w;
      }
    }
    block_sum2(sq, mw);
    if (sq > 0.f) {
      const float iv = 1.0f / sqrtf(sq);
      if (tid < cw) *(float4*)(v + 4 * tid) = make_float4(w4.x * iv, w4.y * iv, w4.z * iv, w4.w * iv);
      cmv = mw * iv;
    }
    __syncthreads();
  }
  // sign: the largest-magnitude entry positive, lowest index on ties
  float best = -1.f;
  int bj = 0x7FFFFFFF;
  for (int j = tid; j < d; j += DIV_THREADS) {
    float av = fabsf(v[j]);
    if (av > best) { best = av; bj = j; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    float ob = __shfl_xor(best, o);
    int oj = __shfl_xor(bj, o);
    if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
  }
  if (lane == 0) { red[wv] = best; redi[wv] = bj; }
  __syncthreads();
  best = red[0]; bj = redi[0];
  for (int i = 1; i < DIV_THREADS / 64; ++i)
    if (red[i] > best || (red[i] == best && redi[i] < bj)) { best = red[i]; bj = redi[i]; }
  const float sg = v[bj] < 0.f ? -1.f : 1.f;
  for (int j = tid; j < d; j += DIV_THREADS) a.pca_dirs[(size_t)sd.dir_index * d + j] = sg * v[j];
  __syncthreads();   // the next segment overwrites the stage, v and red
  }
}

// Principal direction for d <= 16 (the learned division's embedding): one
// wave per node, no workgroup barriers.  The sample (the positions, start
// vector, iteration count and sign rule of k_pca_lds) sits in registers,
// four rows per lane; butterfly sums give every lane the sample mean and the
// centred sample's d x d scatter matrix Y^T Y, which goes through LDS so
// that lane j keeps its row j; each power iteration v <- Y^T Y v / |Y^T Y v|
// is then one row product per lane and a gather of the d results.
constexpr int PCA_COV_DMAX = 16;

__global__ __launch_bounds__(DIV_THREADS) void k_pca_cov(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  constexpr int D = PCA_COV_DMAX;
  __shared__ float cov_s[DIV_THREADS / 64][D * D];
  const int d = a.d;
  const int lane = threadIdx.x & 63;
  const int wpb = DIV_THREADS / 64;
  const int64_t nw = (int64_t)gridDim.x * wpb;
  auto wsum = [](float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
  };
  for (int64_t seg = (int64_t)blockIdx.x * wpb + (threadIdx.x >> 6); seg < a.n_segs; seg += nw) {
    const SegDesc sd = a.segs[seg];
    const uint32_t m = sd.m;
    const uint32_t s = m < 256 ? m : 256;
    uint32_t wd = m / s;
    if (wd < 1) wd = 1;
    float y[4][D];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const uint32_t i = (uint32_t)lane + 64u * r;
      const bool in = i < s;
      uint32_t row = 0;
      if (in) {
        const uint32_t pos = (uint32_t)(((uint64_t)i * m) / s) + (uint32_t)(rand64(a.seed, TAG_SAMPLE, sd.t, sd.v, i) % wd);
        row = a.perm_in[(size_t)sd.slot * (size_t)a.n + sd.off + pos];
      }
      const float* xr = a.X + (size_t)row * d;
#pragma unroll
      for (int j4 = 0; j4 < D / 4; ++j4) {
        const float4 v4 = (in && 4 * j4 < d) ? ((const float4*)xr)[j4] : make_float4(0.f, 0.f, 0.f, 0.f);
        y[r][4 * j4] = v4.x;
        y[r][4 * j4 + 1] = v4.y;
        y[r][4 * j4 + 2] = v4.z;
        y[r][4 * j4 + 3] = v4.w;
      }
    }
    const float is = 1.0f / (float)s;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const float mu = wsum((y[0][j] + y[1][j]) + (y[2][j] + y[3][j])) * is;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if ((uint32_t)lane + 64u * r < s) y[r][j] -= mu;   // rows past the sample stay zero
    }
    // scatter matrix into LDS (both halves), then lane j keeps row j of it
    float* Cs = cov_s[threadIdx.x >> 6];
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
      for (int l = j; l < D; ++l) {
        float c = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) c = __builtin_fmaf(y[r][j], y[r][l], c);
        c = wsum(c);
        if (lane == 0) {
          Cs[j * D + l] = c;
          Cs[l * D + j] = c;
        }
      }
    wave_sync();
    float crow[D];
#pragma unroll
    for (int l = 0; l < D; ++l) crow[l] = Cs[(lane & (D - 1)) * D + l];
    wave_sync();   // the next node overwrites Cs
    float v[D];
    float nn = 0.f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      v[j] = j < d ? rp_entry(a.seed, sd.t, sd.v, (uint32_t)j) : 0.f;
      nn = __builtin_fmaf(v[j], v[j], nn);
    }
    const float inv0 = nn > 0.f ? 1.0f / sqrtf(nn) : 0.f;
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] *= inv0;
    for (int itr = 0; itr < a.pca_iters; ++itr) {
      // lane j forms (Y^T Y v)_j; every lane then gathers all of them
      float acc = 0.f;
#pragma unroll
      for (int l = 0; l < D; ++l) acc = __builtin_fmaf(crow[l], v[l], acc);
      float w[D];
      float sq = 0.f;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        w[j] = __shfl(acc, j);
        sq = __builtin_fmaf(w[j], w[j], sq);
      }
      if (sq > 0.f) {
        const float iv = 1.0f / sqrtf(sq);
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = w[j] * iv;
      }
    }
    // sign: the largest-magnitude entry positive, lowest index on ties
    float best = -1.f, sg = 1.f;
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < d && fabsf(v[j]) > best) {
        best = fabsf(v[j]);
        sg = v[j] < 0.f ? -1.f : 1.f;
      }
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (lane == j && j < d) a.pca_dirs[(size_t)sd.dir_index * d + j] = sg * v[j];
  }
}

// Principal direction for d > PCA_LDS_DMAX: the centred sample is read from
// global memory (L2) in every iteration; same sample, start, iterations and
// sign rule as k_pca_lds.
__global__ __launch_bounds__(DIV_THREADS) void k_pca_dirs(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  extern __shared__ float smem[];
  const int d = a.d;
  float* mu = smem;               // d
  float* v = mu + d;              // d
  float* tt = v + d;              // 256
  __shared__ uint32_t rows[256];
  __shared__ float red[DIV_THREADS / 64];
  __shared__ int redi[DIV_THREADS / 64];
  const SegDesc sd = a.segs[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t m = sd.m;
  uint32_t s = m < 256 ? m : 256;
  uint32_t wd = m / s;
  if (wd < 1) wd = 1;
  if (threadIdx.x < s) {
    uint32_t pos = (uint32_t)(((uint64_t)threadIdx.x * m) / s) +
                   (uint32_t)(rand64(a.seed, TAG_SAMPLE, sd.t, sd.v, threadIdx.x) % wd);
    rows[threadIdx.x] = a.perm_in[(size_t)sd.slot * (size_t)a.n + sd.off + pos];
  }
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) v[j] = rp_entry(a.seed, sd.t, sd.v, (uint32_t)j);
  __syncthreads();
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) {
    float acc = 0.f;
    for (uint32_t i = 0; i < s; ++i) acc += a.X[(size_t)rows[i] * d + j];
    mu[j] = acc / (float)s;
  }
  __syncthreads();
  auto yval = [&](uint32_t i, int j) -> float { return a.X[(size_t)rows[i] * d + j] - mu[j]; };
  auto block_sum = [&](float x) -> float {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    if (lane == 0) red[wv] = x;
    __syncthreads();
    float r = 0.f;
    for (int i = 0; i < DIV_THREADS / 64; ++i) r += red[i];
    __syncthreads();
    return r;
  };
  // normalise the start vector
  float nn = 0.f;
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) nn += v[j] * v[j];
  nn = block_sum(nn);
  float inv = nn > 0.f ? 1.0f / sqrtf(nn) : 0.f;
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) v[j] *= inv;
  __syncthreads();
  for (int itr = 0; itr < a.pca_iters; ++itr) {
    if (threadIdx.x < s) {
      float acc0 = 0.f, acc1 = 0.f;
      int j = 0;
      for (; j + 1 < d; j += 2) {
        acc0 = __builtin_fmaf(yval(threadIdx.x, j), v[j], acc0);
        acc1 = __builtin_fmaf(yval(threadIdx.x, j + 1), v[j + 1], acc1);
      }
      for (; j < d; ++j) acc0 = __builtin_fmaf(yval(threadIdx.x, j), v[j], acc0);
      tt[threadIdx.x] = acc0 + acc1;
    }
    __syncthreads();
    float sq = 0.f;
    float wj[(4096 + DIV_THREADS - 1) / DIV_THREADS];
    int nj = 0;
    for (int j = threadIdx.x; j < d; j += DIV_THREADS, ++nj) {
      float acc0 = 0.f, acc1 = 0.f;
      uint32_t i = 0;
      for (; i + 1 < s; i += 2) {
        acc0 = __builtin_fmaf(yval(i, j), tt[i], acc0);
        acc1 = __builtin_fmaf(yval(i + 1, j), tt[i + 1], acc1);
      }
      for (; i < s; ++i) acc0 = __builtin_fmaf(yval(i, j), tt[i], acc0);
      wj[nj] = acc0 + acc1;
      sq += wj[nj] * wj[nj];
    }
    sq = block_sum(sq);
    if (sq > 0.f) {
      float iv = 1.0f / sqrtf(sq);
      nj = 0;
      for (int j = threadIdx.x; j < d; j += DIV_THREADS, ++nj) v[j] = wj[nj] * iv;
    }
    __syncthreads();
  }
  // sign: the largest-magnitude entry positive, lowest index on ties
  float best = -1.f;
  int bj = 0x7FFFFFFF;
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) {
    float av = fabsf(v[j]);
    if (av > best) { best = av; bj = j; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    float ob = __shfl_xor(best, o);
    int oj = __shfl_xor(bj, o);
    if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
  }
  if (lane == 0) { red[wv] = best; redi[wv] = bj; }
  __syncthreads();
  best = red[0]; bj = redi[0];
  for (int i = 1; i < DIV_THREADS / 64; ++i)
    if (red[i] > best || (red[i] == best && redi[i] < bj)) { best = red[i]; bj = redi[i]; }
  float sg = v[bj] < 0.f ? -1.f : 1.f;
  for (int j = threadIdx.x; j < d; j += DIV_THREADS) a.pca_dirs[(size_t)sd.dir_index * d + j] = sg * v[j];
}

// Principal direction for PCA_LDS_DMAX < d <= PCA_ROWS_DMAX, one pass over
// the sample per iteration: w = Y^T (Y v) is the sum over sample rows of
// (y_i - mu) t_i with t_i = (y_i - mu) . v, so a wave that holds a whole
// row (lane l: float4 chunks l, l + 64, ... of it; NC4 of them) forms t_i by
// a wave sum and adds the row times t_i into its own partial of w in
// registers.  Waves take rows w, w + 4, ...; their partials are added in
// wave order.  Every wave keeps the whole of v and mu, so only the partials
// of w and the mean cross waves (through LDS).  Same sample, start vector,
// iteration count and sign rule as k_pca_lds; the sums run in another
// order.  The sample is read once per iteration (coalesced rows, four in
// flight per wave) instead of twice.
constexpr int PCA_ROWS_DMAX = 1024;

__device__ __forceinline__ float wave_sum_f(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  return x;   // the same value in every lane (each step adds a pair in both orders)
}

template <int NC4>
__global__ __launch_bounds__(DIV_THREADS) void k_pca_rows(DivideLevelArgs a) {
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  constexpr int NW = DIV_THREADS / 64;
  constexpr int RU = 4;            // rows in flight per wave
  __shared__ uint32_t rows[256];
  __shared__ float4 part[NW][64 * NC4];
  const SegDesc sd = a.segs[blockIdx.x];
  const int d = a.d, c4 = d >> 2;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint32_t m = sd.m;
  const uint32_t s = m < 256 ? m : 256;
  uint32_t wd = m / s;
  if (wd < 1) wd = 1;
  if (threadIdx.x < s) {
    uint32_t pos = (uint32_t)(((uint64_t)threadIdx.x * m) / s) +
                   (uint32_t)(rand64(a.seed, TAG_SAMPLE, sd.t, sd.v, threadIdx.x) % wd);
    rows[threadIdx.x] = a.perm_in[(size_t)sd.slot * (size_t)a.n + sd.off + pos];
  }
  bool ok[NC4];
  float4 v[NC4];
#pragma unroll
  for (int c = 0; c < NC4; ++c) {
    const int q = lane + 64 * c;   // this lane's float4 chunk c: columns 4q .. 4q + 3
    ok[c] = q < c4;
    v[c] = ok[c] ? make_float4(rp_entry(a.seed, sd.t, sd.v, 4 * q), rp_entry(a.seed, sd.t, sd.v, 4 * q + 1),
                               rp_entry(a.seed, sd.t, sd.v, 4 * q + 2), rp_entry(a.seed, sd.t, sd.v, 4 * q + 3))
                 : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  // the rows of this wave, RU at a time; rows past the sample load row 0
  // and are not used
  auto load_rows = [&](uint32_t i0, float4 (&y)[RU][NC4]) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const uint32_t i = i0 + (uint32_t)(NW * u);
      const float4* yr = reinterpret_cast<const float4*>(a.X + (size_t)rows[i < s ? i : 0] * d);
#pragma unroll
      for (int c = 0; c < NC4; ++c) y[u][c] = ok[c] ? yr[lane + 64 * c] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto add4 = [](float4& r, const float4 x) { r.x += x.x; r.y += x.y; r.z += x.z; r.w += x.w; };
  // partials of the waves added in wave order into every wave's registers
  auto gather = [&](float4 (&acc)[NC4], float4 (&out)[NC4]) {
#pragma unroll
    for (int c = 0; c < NC4; ++c) part[wv][lane + 64 * c] = acc[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC4; ++c) {
      float4 r = part[0][lane + 64 * c];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) add4(r, part[w2][lane + 64 * c]);
      out[c] = r;
    }
    __syncthreads();   // part is written again by the next gather
  };
  // mean
  float4 mu[NC4];
  {
    float4 acc[NC4];
#pragma unroll
    for (int c = 0; c < NC4; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t i0 = wv; i0 < s; i0 += NW * RU) {
      float4 y[RU][NC4];
      load_rows(i0, y);
#pragma unroll
      for (int u = 0; u < RU; ++u)
        if (i0 + (uint32_t)(NW * u) < s) {
#pragma unroll
          for (int c = 0; c < NC4; ++c) add4(acc[c], y[u][c]);
        }
    }
    gather(acc, mu);
    const float fs = (float)s;
#pragma unroll
    for (int c = 0; c < NC4; ++c) mu[c] = make_float4(mu[c].x / fs, mu[c].y / fs, mu[c].z / fs, mu[c].w / fs);
  }
  auto dot4 = [](const float4 x, const float4 y, float acc) {
    acc = __builtin_fmaf(x.x, y.x, acc);
    acc = __builtin_fmaf(x.y, y.y, acc);
    acc = __builtin_fmaf(x.z, y.z, acc);
    return __builtin_fmaf(x.w, y.w, acc);
  };
  // normalise the start vector (every wave holds all of it)
  {
    float nn = 0.f;
#pragma unroll
    for (int c = 0; c < NC4; ++c) nn = dot4(v[c], v[c], nn);
    nn = wave_sum_f(nn);
    const float inv = nn > 0.f ? 1.0f / sqrtf(nn) : 0.f;
#pragma unroll
    for (int c = 0; c < NC4; ++c) v[c] = make_float4(v[c].x * inv, v[c].y * inv, v[c].z * inv, v[c].w * inv);
  }
  for (int itr = 0; itr < a.pca_iters; ++itr) {
    float4 acc[NC4];
#pragma unroll
    for (int c = 0; c < NC4; ++c) acc[c] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (uint32_t i0 = wv; i0 < s; i0 += NW * RU) {
      float4 y[RU][NC4];
      load_rows(i0, y);
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (i0 + (uint32_t)(NW * u) >= s) break;   // uniform
        float t = 0.f;
#pragma unroll
        for (int c = 0; c < NC4; ++c) {
          float4& yc = y[u][c];
          yc.x -= mu[c].x; yc.y -= mu[c].y; yc.z -= mu[c].z; yc.w -= mu[c].w;   // padded chunks stay 0
          t = dot4(yc, v[c], t);
        }
        t = wave_sum_f(t);
#pragma unroll
        for (int c = 0; c < NC4; ++c) {
          acc[c].x = __builtin_fmaf(y[u][c].x, t, acc[c].x);
          acc[c].y = __builtin_fmaf(y[u][c].y, t, acc[c].y);
          acc[c].z = __builtin_fmaf(y[u][c].z, t, acc[c].z);
          acc[c].w = __builtin_fmaf(y[u][c].w, t, acc[c].w);
        }
      }
    }
    float4 w4[NC4];
    gather(acc, w4);
    float sq = 0.f;
#pragma unroll
    for (int c = 0; c < NC4; ++c) sq = dot4(w4[c], w4[c], sq);
    sq = wave_sum_f(sq);
    if (sq > 0.f) {
      const float iv = 1.0f / sqrtf(sq);
#pragma unroll
      for (int c = 0; c < NC4; ++c) v[c] = make_float4(w4[c].x * iv, w4[c].y * iv, w4[c].z * iv, w4[c].w * iv);
    }
  }
  // sign: the largest-magnitude entry positive, lowest index on ties (every
  // wave holds v; wave 0 decides and writes)
  if (wv != 0) return;
  float best = -1.f;
  int bj = 0x7FFFFFFF;
  float bv = 0.f;
#pragma unroll
  for (int c = 0; c < NC4; ++c) {
    const int j0 = 4 * (lane + 64 * c);
    const float e[4] = {v[c].x, v[c].y, v[c].z, v[c].w};
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (ok[c] && fabsf(e[u]) > best) { best = fabsf(e[u]); bj = j0 + u; bv = e[u]; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const float ob = __shfl_xor(best, o);
    const int oj = __shfl_xor(bj, o);
    const float ov = __shfl_xor(bv, o);
    if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; bv = ov; }
  }
  const float sg = bv < 0.f ? -1.f : 1.f;
  float4* out = reinterpret_cast<float4*>(a.pca_dirs + (size_t)sd.dir_index * d);
#pragma unroll
  for (int c = 0; c < NC4; ++c)
    if (ok[c]) out[lane + 64 * c] = make_float4(sg * v[c].x, sg * v[c].y, sg * v[c].z, sg * v[c].w);
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = value;
}

// slots consecutive copies of 0..n-1
__global__ void k_iota(uint32_t* p, uint32_t n, uint32_t slots) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t tot = (size_t)n * slots;
  for (; i < tot; i += stride) p[i] = (uint32_t)(i % n);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, p, value, count);
  return hipGetLastError();
}

hipError_t launch_iota(uint32_t* p, uint32_t n, uint32_t slots, hipStream_t s) {
  size_t blocks = ((size_t)n * slots + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_iota, dim3((unsigned)blocks), dim3(256), 0, s, p, n, slots);
  return hipGetLastError();
}

hipError_t launch_divide_level(const DivideLevelArgs& a, hipStream_t s) {
  hipError_t e;
  if (!a.small && (e = launch_fill_u32(a.hist, 0u, (size_t)a.n_segs * HIST_TOTAL, s)) != hipSuccess) return e;
  if (a.pca_iters > 0 && !a.dirs) {
    size_t base = (size_t)(2 * a.d + 256) * sizeof(float);
    if (a.d <= PCA_COV_DMAX) {
      const unsigned blocks = (unsigned)std::min<size_t>((a.n_segs + 3) / 4, (size_t)cu_count() * 8);
      hipLaunchKernelGGL(k_pca_cov, dim3(blocks), dim3(DIV_THREADS), 0, s, a);
    } else if (a.d <= PCA_LDS_DMAX) {
      const int cw = a.d / 4, G = DIV_THREADS / cw;
      const size_t tail = (2 * (size_t)a.d + 256 + (size_t)G * cw * 4) * sizeof(float);
      const size_t shm = (size_t)256 * (a.d + 4) * sizeof(float) + tail;
      const size_t shm8 = (size_t)256 * (a.d + 4) + tail;   // 256 (d + 4) is a multiple of 16
      static bool attr = false;
      if (!attr) {
        e = hipFuncSetAttribute((const void*)k_pca_lds<false>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e != hipSuccess) return e;
        attr = true;
      }
      // as many workgroups as the CUs' LDS holds at once (160 KB each, with
      // the kernel's 48 static bytes), at most eight per CU; they stride
      // over the segments
      const unsigned cus = (unsigned)cu_count();
      auto grid = [&](size_t bytes) {
        const size_t per_cu = std::max<size_t>(1, std::min<size_t>(8, (160 * 1024) / (bytes + 48)));
        return dim3((unsigned)std::min<size_t>(a.n_segs, per_cu * cus));
      };
      hipLaunchKernelGGL(k_pca_lds<false>, grid(shm), dim3(DIV_THREADS), shm, s, a);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (a.X8) hipLaunchKernelGGL(k_pca_lds<true>, grid(shm8), dim3(DIV_THREADS), shm8, s, a);
    } else if (a.d <= PCA_ROWS_DMAX) {
      const int nc4 = (a.d / 4 + 63) / 64;
      if (nc4 == 1) hipLaunchKernelGGL(k_pca_rows<1>, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a);
      else if (nc4 == 2) hipLaunchKernelGGL(k_pca_rows<2>, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a);
      else if (nc4 == 3) hipLaunchKernelGGL(k_pca_rows<3>, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a);
      else hipLaunchKernelGGL(k_pca_rows<4>, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a);
    } else {
      hipLaunchKernelGGL(k_pca_dirs, dim3(a.n_segs), dim3(DIV_THREADS), base, s, a);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_proj_hist0, dim3(a.n_split), dim3(DIV_THREADS), (size_t)a.d * sizeof(float), s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.small) {
    hipLaunchKernelGGL(k_small_partition, dim3(a.n_items), dim3(DIV_THREADS), 0, s, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_resolve_step, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a, 0);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hist_pass, dim3(a.n_split), dim3(DIV_THREADS), 0, s, a, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_resolve_step, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a, 1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_hist_pass, dim3(a.n_split), dim3(DIV_THREADS), 0, s, a, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_resolve_step, dim3(a.n_segs), dim3(DIV_THREADS), 0, s, a, 2);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_count, dim3(a.n_split), dim3(DIV_THREADS), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_scatter, dim3(a.n_items), dim3(DIV_THREADS), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
