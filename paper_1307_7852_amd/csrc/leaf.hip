// Exact k-NN inside every leaf subset (Section 3.1's brute-force subgraph).
//
// One workgroup per leaf: 8 waves by default (4 for k + rerank_m > 32);
// the wave count and the K-chunk width are tunable per shape.  The leaf's
// members stream through LDS in tiles of 32 candidates x KC features
// (double-buffered, staged once for all waves; rows padded so operand reads
// are bank-conflict free).  Each wave owns 32 queries whose fragments sit in
// registers as the B operand, the tile supplies the A operand:
//   G[c][q] = x_c . x_q   (v_mfma_f32_32x32x2_f32, or v_mfma_f32_32x32x16_bf16
//                          on leaf-centred BF16 data)
// so every lane holds 16 candidates of one query per tile.  Each becomes a
// 32-bit key: the approximate squared distance |x_q|^2 + |x_c|^2 - 2 G as a
// float with its 11 low mantissa bits replaced by the candidate's position
// in the leaf.  Nonnegative normal floats order like their bit patterns, so
// keeping a sorted top-KP list per lane costs one v_med3_f32 per list entry
// and candidate.  The two lanes that share a query (each saw half of the
// candidates) merge their lists; the KP survivors are re-scored with the
// canonical FP32 distance, sorted by (distance, id) and the first k written.
// A row whose k-th exact distance is not safely below every rejected
// candidate's lower bound (from the truncated key and the Gram's error bound)
// is redone exactly by k_leaf_exact.
//
// Member norms, the leaf's exactness flag (all-integer data with small norms
// makes the FP32 Gram exact) and the largest norm come from the per-point
// norms the data check wrote (k_exact_check: one pass over X per launch or
// build); only a centred BF16 leaf forms its norms while its first pass
// stages the tiles.  On integer data the keys carry the exact distance and
// need no re-rank (see make_ikey).
#include "knng_dev.h"

#include <algorithm>
#include <type_traits>

namespace knng {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int QPW = 32;            // queries per wave
constexpr int TILE = 32;           // candidates per tile
constexpr int TILE_BUFS = 4;       // tile buffers in LDS: staged two steps ahead, a barrier every second step
static_assert((TILE_BUFS & (TILE_BUFS - 1)) == 0, "buffer rotation is a mask");
constexpr int MU_MAX = 2048;       // BF16 path: d <= 2048
constexpr uint32_t POS_MASK = 0x7FFu;          // position bits of a key (leaf <= 2048)
constexpr uint32_t KEY_NONE = 0x7F7FFFFFu;     // FLT_MAX: above every key
constexpr uint32_t KEY_VALID = 0x7F000000u;    // keys at or above this are padding
constexpr float PAD_NORM = 3e38f;              // norm given to padding rows (keys land above KEY_VALID)
constexpr float KEY_FLOOR = 0x1p-100f;         // keeps every key a normal float

template <int KP, int W>
struct Cfg {
  static constexpr int WAVES = W;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int QPB = QPW * WAVES;   // queries per pass
  static constexpr int LS = KP + 1;         // list stride per query in LDS
};

// Integer data (every value integral, every norm <= 2^22; for the BF16 Gram
// also |x| <= 256) makes |x_q|^2 + |x_c|^2 - 2G an exact integer D.  Then
// the key carries D itself: (min(D, KEY_DSAT) << 11) | position, still a
// nonnegative float bit pattern below the NaN range (denormals included;
// the kernels keep them).  A list of such keys is ordered exactly by
// (distance, position) = (distance, id), so it needs no re-rank; a row whose
// k-th key is saturated goes to the exact kernel.
constexpr uint32_t KEY_DSAT = 1044478u;   // (KEY_DSAT << 11) | 2047 < KEY_NONE

__device__ __forceinline__ float make_ikey(float dv, uint32_t pos) {
  const uint32_t D = (uint32_t)fminf(fmaxf(dv, 0.f), (float)KEY_DSAT);   // dv is an exact integer
  return __uint_as_float((D << 11) | pos);
}

__device__ __forceinline__ float make_key(float dv, uint32_t pos) {
  float v = fmaxf(dv, KEY_FLOOR);
  return __uint_as_float((__float_as_uint(v) & ~POS_MASK) | pos);
}
__device__ __forceinline__ float key_value(uint32_t key) { return __uint_as_float(key & ~POS_MASK); }

// Inserts x into the ascending list L (the largest entry falls off).
template <int KP>
__device__ __forceinline__ void list_insert(float (&L)[KP], float x) {
#pragma unroll
  for (int j = KP - 1; j > 0; --j) L[j] = __builtin_amdgcn_fmed3f(L[j - 1], x, L[j]);
  L[0] = fminf(L[0], x);
}

// The same on the first KI entries only (the rest keep what they hold):
// enough wherever only the KI smallest keys are ever read.
template <int KI, int KP>
__device__ __forceinline__ void list_insert_head(float (&L)[KP], float x) {
  static_assert(KI <= KP, "head longer than the list");
#pragma unroll
  for (int j = KI - 1; j > 0; --j) L[j] = __builtin_amdgcn_fmed3f(L[j - 1], x, L[j]);
  // keys are nonnegative floats, ordered as their bit patterns: an integer
  // minimum needs no canonicalising of x
  L[0] = __uint_as_float(min(__float_as_uint(L[0]), __float_as_uint(x)));
}

// Eight canonical distances: two query rows, four candidates each (dist2_g16's arithmetic per pair).
__device__ __forceinline__ void dist2_g16_x8(const float* __restrict__ xa, const float* const (&ya)[4],
                                             const float* __restrict__ xb, const float* const (&yb)[4], int d, int g,
                                             float (&oa)[4], float (&ob)[4]) {
  float a[8][4];
#pragma unroll
  for (int u = 0; u < 8; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0.f;
  const int nc = d >> 2;
  for (int c = g; c < nc; c += 16) {
    float4 xva = ((const float4*)xa)[c], xvb = ((const float4*)xb)[c];
    float4 w[8];
#pragma unroll
    for (int u = 0; u < 4; ++u) { w[u] = ((const float4*)ya[u])[c]; w[4 + u] = ((const float4*)yb[u])[c]; }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float4 xv = u < 4 ? xva : xvb;
      float e0 = xv.x - w[u].x, e1 = xv.y - w[u].y, e2 = xv.z - w[u].z, e3 = xv.w - w[u].w;
      a[u][0] = __builtin_fmaf(e0, e0, a[u][0]);
      a[u][1] = __builtin_fmaf(e1, e1, a[u][1]);
      a[u][2] = __builtin_fmaf(e2, e2, a[u][2]);
      a[u][3] = __builtin_fmaf(e3, e3, a[u][3]);
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    float s = (a[u][0] + a[u][1]) + (a[u][2] + a[u][3]);
    s += __shfl_xor(s, 8, 16);
    s += __shfl_xor(s, 4, 16);
    s += __shfl_xor(s, 2, 16);
    s += __shfl_xor(s, 1, 16);
    if (u < 4) oa[u] = s; else ob[u - 4] = s;
  }
}

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
// Two floats rounded to BF16 (to nearest even) in one 32-bit word, a low.
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const f32x2 f = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2));
}

// Tile element types: FP32 rows padded by 4 floats, BF16 rows by 8 halves;
// either way consecutive rows start 16 bytes apart modulo the bank width.
template <int KC, bool BF16>
struct TileT {
  static constexpr int STRIDE = BF16 ? (KC + 8) : (KC + 4);   // elements per row
  using E = typename std::conditional<BF16, __bf16, float>::type;
  E v[TILE * STRIDE];
};

template <int KC, int KP, bool BF16, int W>
struct LeafShared {
  using C = Cfg<KP, W>;
  uint32_t ids[KNNG_MAX_LEAF];
  float nrm[KNNG_MAX_LEAF];                 // member norms (centred BF16: of the rounded centred rows)
  TileT<KC, BF16> tile[TILE_BUFS];
  float mu[BF16 ? MU_MAX : 1];
  uint32_t max_n;                           // largest member norm (float bits)
  int flag;                                 // every value integral and every norm <= 2^22 (BF16: |value| <= 256)
  float qn[C::WAVES][QPW];                  // query norms, as used in the keys
  uint32_t lst[C::WAVES][QPW * C::LS];      // merged top-KP keys per query
  float dst[C::WAVES][QPW * C::LS];         // their canonical distances
};

// Query fragments in registers: lane (h, q) owns features [h*HALF, h*HALF+HALF)
// of each KC-wide chunk; MFMA step s uses feature h*HALF + s (FP32) or
// h*HALF + 8 s .. +7 (BF16).  Tiles use the same mapping for the candidates,
// so the contraction covers every feature exactly once.
template <int KC, bool BF16>
struct QFrag {
  static constexpr int HALF = KC / 2;
  static constexpr int N4 = HALF / 4;
  static constexpr int N8 = HALF / 8;
  float4 f[BF16 ? 1 : N4];
  bf16x8 b[BF16 ? N8 : 1];
  __device__ __forceinline__ void load(const float* __restrict__ row, int kc, int d, int h, const float* mu, bool ok) {
    if constexpr (!BF16) {
#pragma unroll
      for (int i = 0; i < N4; ++i) {
        int c = kc + h * HALF + 4 * i;
        f[i] = (ok && c < d) ? *(const float4*)(row + c) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    } else {
      // two 16-byte loads per 8 features (d is a multiple of 4, rows and c
      // are 16-byte aligned), centred with the leaf mean and rounded
#pragma unroll
      for (int i = 0; i < N8; ++i) {
        const int c = kc + h * HALF + 8 * i;
        const bool ok0 = ok && c < d, ok1 = ok && c + 4 < d;
        const float4 v0 = ok0 ? *(const float4*)(row + c) : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 v1 = ok1 ? *(const float4*)(row + c + 4) : make_float4(0.f, 0.f, 0.f, 0.f);
        b[i][0] = (__bf16)(ok0 ? v0.x - mu[c] : 0.f);
        b[i][1] = (__bf16)(ok0 ? v0.y - mu[c + 1] : 0.f);
        b[i][2] = (__bf16)(ok0 ? v0.z - mu[c + 2] : 0.f);
        b[i][3] = (__bf16)(ok0 ? v0.w - mu[c + 3] : 0.f);
        b[i][4] = (__bf16)(ok1 ? v1.x - mu[c + 4] : 0.f);
        b[i][5] = (__bf16)(ok1 ? v1.y - mu[c + 5] : 0.f);
        b[i][6] = (__bf16)(ok1 ? v1.z - mu[c + 6] : 0.f);
        b[i][7] = (__bf16)(ok1 ? v1.w - mu[c + 7] : 0.f);
      }
    }
  }
};

// Clears bit EXACT_FP32 of *flags if some value of X is not an integer or
// some row norm exceeds 2^22, EXACT_BF16 also if some |value| > 256, and
// EXACT_U8 if some value is not one of 0, 1, ..., 255 (-0 counts as 0: a
// zero's sign never changes a sum that starts from +0, so the byte copy's +0
// gives the same projections).  Writes every row's
// squared norm to pnorm, with the sign bit set when the row holds a
// non-integer.  16 lanes per row.
__global__ __launch_bounds__(256) void k_exact_check(const float* __restrict__ X, int64_t n, int d,
                                                     unsigned int* __restrict__ flags, float* __restrict__ pnorm) {
  const int64_t row = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 4;
  const int gl = threadIdx.x & 15;
  bool integral = true, small = true, byte = true;
  float nrm = 0.f;
  if (row < n) {
    const float4* xr = (const float4*)(X + row * d);
    for (int c = gl; c < (d >> 2); c += 16) {
      const float4 v = xr[c];
      integral = integral && v.x == rintf(v.x) && v.y == rintf(v.y) && v.z == rintf(v.z) && v.w == rintf(v.w);
      small = small && fabsf(v.x) <= 256.f && fabsf(v.y) <= 256.f && fabsf(v.z) <= 256.f && fabsf(v.w) <= 256.f;
      byte = byte && v.x >= 0.f && v.y >= 0.f && v.z >= 0.f && v.w >= 0.f && v.x <= 255.f && v.y <= 255.f &&
             v.z <= 255.f && v.w <= 255.f;
      nrm = __builtin_fmaf(v.x, v.x, __builtin_fmaf(v.y, v.y, __builtin_fmaf(v.z, v.z, __builtin_fmaf(v.w, v.w, nrm))));
    }
  }
  nrm += __shfl_xor(nrm, 8, 16);
  nrm += __shfl_xor(nrm, 4, 16);
  nrm += __shfl_xor(nrm, 2, 16);
  nrm += __shfl_xor(nrm, 1, 16);
  // the row is integral when all 16 lanes of its group found only integers
  const unsigned long long nonint = __ballot(!integral);
  const bool row_int = ((nonint >> (threadIdx.x & 48)) & 0xFFFFull) == 0ull;
  if (row < n && gl == 0) pnorm[row] = row_int ? nrm : -nrm;
  const bool ok32 = integral && !(nrm > 4194304.0f);
  const bool bad32 = __any(!ok32), bad16 = __any(!(ok32 && small)), bad8 = __any(!(integral && byte));
  const unsigned int clear = (bad32 ? EXACT_FP32 : 0u) | (bad16 ? EXACT_BF16 : 0u) | (bad8 ? EXACT_U8 : 0u);
  // a wave writes only bits that are still set, so the atomics stay few
  if ((threadIdx.x & 63) == 0 && clear != 0u && (__atomic_load_n(flags, __ATOMIC_RELAXED) & clear) != 0u)
    atomicAnd(flags, ~clear);
}

// One leaf: members perm[off .. off+m), rows written to ids/dist (already
// offset to the leaf's division).  `key` names the leaf in the fallback list.
template <int KC, int KP, bool BF16, int W, int KT, bool PAIR>
__device__ __forceinline__ void leaf_body(const LeafArgs& a, LeafShared<KC, KP, BF16, W>& S, const uint32_t* __restrict__ perm,
                                          uint32_t* __restrict__ ids_out, float* __restrict__ dist_out, int64_t off,
                                          int m, uint32_t key) {
  using C = Cfg<KP, W>;
  using Tile = TileT<KC, BF16>;
  constexpr int LS = C::LS;
  const int tid = threadIdx.x, lane = tid & 63, h = lane >> 5, r32 = lane & 31;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave index, uniform (a scalar)
  const int d = a.d, k = a.k;
  const uint32_t L = key;
  if (m <= 0) return;
  if (m > KNNG_MAX_LEAF) {   // every row goes to the exact kernel
    for (int i = tid; i < m; i += C::THREADS) {
      unsigned long long slot = atomicAdd(&a.diag->fallback_count, 1ull);
      atomicAdd(&a.diag->leaf_fallback, 1ull);
      if (slot < a.fallback_cap) {   // capacity: every point of every division once
        a.fallback[2 * slot] = L;
        a.fallback[2 * slot + 1] = (uint32_t)i;
      }
    }
    return;
  }
  for (int i = tid; i < m; i += C::THREADS) S.ids[i] = perm[off + i];
  if (tid == 0) {
    S.flag = 1;
    S.max_n = 0u;
  }
  // exact integer keys when the whole data set allows them (uniform)
  const bool ikey = (__builtin_amdgcn_readfirstlane(a.diag->exact_flags) & (BF16 ? EXACT_BF16 : EXACT_FP32)) != 0u;   // uniform
  __syncthreads();
  // ---- BF16: leaf mean, coalesced (threads over features x row groups).
  // A leaf whose values are all integers of magnitude <= 256 is BF16-exact
  // as it stands: then it is not centred (centring would make it inexact),
  // and with norms <= 2^22 its BF16 Gram with FP32 accumulation is exact.
  if (BF16 && ikey) {   // exact as it stands: no centring
    for (int j = tid; j < d; j += C::THREADS) S.mu[BF16 ? j : 0] = 0.f;
    __syncthreads();
  } else if constexpr (BF16) {
    float* part = reinterpret_cast<float*>(&S.tile[0]);   // >= THREADS floats, free until staging
    const int dd = d < C::THREADS ? d : C::THREADS;
    const int G = C::THREADS / dd;
    for (int jb = 0; jb < d; jb += dd) {
      const int jl = tid % dd, g = tid / dd, j = jb + jl;
      float acc = 0.f;
      bool ex = true;
      if (g < G && j < d)
        for (int i = g; i < m; i += G) {
          const float v = a.X[(size_t)S.ids[i] * d + j];
          acc += v;
          ex = ex && v == rintf(v) && fabsf(v) <= 256.f;
        }
      if (!ex) S.flag = 0;
      if (g < G) part[g * dd + jl] = acc;
      __syncthreads();
      if (tid < dd && jb + tid < d) {
        float s = 0.f;
        for (int gg = 0; gg < G; ++gg) s += part[gg * dd + tid];
        S.mu[jb + tid] = s / (float)m;
      }
      __syncthreads();
    }
    if (S.flag) {   // uniform: every thread reads the flag after the last barrier
      for (int j = tid; j < d; j += C::THREADS) S.mu[j] = 0.f;
      __syncthreads();
    }
  }
  // Member norms of uncentred rows come from the per-point norms (sign bit:
  // the row holds a non-integer); padding rows up to the tile boundary get
  // PAD_NORM.  Centred BF16 rows get theirs while the first pass stages them.
  const bool pre_norms = !BF16 || ikey;   // uniform
  if (pre_norms) {
    const int mt = (m + TILE - 1) / TILE * TILE;
    float mx = 0.f;
    bool bad = false;
    for (int i = tid; i < mt; i += C::THREADS) {
      float v = PAD_NORM;
      if (i < m) {
        const float pn = a.pnorm[S.ids[i]];
        v = fabsf(pn);
        bad = bad || (__float_as_uint(pn) >> 31) != 0u || v > 4194304.0f;   // 2^22: partial Gram sums stay exact
        mx = fmaxf(mx, v);
      }
      S.nrm[i] = v;
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    if (__any(bad) && lane == 0) S.flag = 0;
    if (lane == 0) atomicMax(&S.max_n, __float_as_uint(mx));
    __syncthreads();
  }
  const float eps_c = 2.0f * (float)(d + 4) * 5.9604645e-8f;   // 2 (d+4) 2^-24
  const float INF = __int_as_float(0x7F800000);

  constexpr int HALF = KC / 2;
  constexpr int F4_PER_ROW = KC / 4;
  constexpr int TILE_F4 = TILE * F4_PER_ROW;
  constexpr int STAGE_F4 = (TILE_F4 + C::THREADS - 1) / C::THREADS;   // float4 per thread per tile chunk
  const int nchunk = (d + KC - 1) / KC;
  const int ntile = (m + TILE - 1) / TILE;
  const int nsteps = ntile * nchunk;
  // st / nchunk as a multiply-high by M = ceil(2^32 / nchunk): exact for
  // st < 2^32 / nchunk, far above any step count here
  const uint32_t nch_m = nchunk == 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)nchunk - 1u) / (uint64_t)nchunk);
  auto step_tile = [&](int st) -> int { return nchunk == 1 ? st : (int)__umulhi((uint32_t)st, nch_m); };
  // PAIR (rows of several chunks): tiles go in pairs, chunk by chunk --
  // (tile 2p, chunk c), (tile 2p + 1, chunk c), (2p, c + 1), ... -- so one
  // load of a wave's query fragment of chunk c serves both tiles, while the
  // pair's other partial Gram waits in a second accumulator; an odd last
  // tile goes alone.  Each tile still takes its chunks in increasing order.
  const bool pair = PAIR && nchunk > 1;                      // uniform
  const int full = pair ? (ntile >> 1) * 2 * nchunk : 0;     // steps of whole pairs
  auto step_tc = [&](int st, int& tile, int& kci) {
    if (!pair) {
      tile = step_tile(st);
      kci = st - tile * nchunk;
    } else if (st < full) {
      const int pr = st / (2 * nchunk), r = st - pr * 2 * nchunk;
      tile = 2 * pr + (r & 1);
      kci = r >> 1;
    } else {
      tile = ntile - 1;
      kci = st - full;
    }
  };

  // Integer keys straight from the Gram (integer data, exact in the Gram's
  // input type, one chunk, leaves of at most 512; in BF16 such leaves are
  // not centred): with the query scaled by -2 and the accumulator
  // starting at 2^23 + |x_c|^2 + M (M: the leaf's largest member norm), the
  // Gram ends at 2^23 + D', where D' = D - |x_q|^2 + M is an integer in
  // [0, 4M] that ranks the lane's candidates as D does.  Every partial sum
  // is an integer in (2^22, 2^24), so all of it is exact, and the float's
  // bits are 0x4B000000 + D'.  With 4M below FK_DSAT, D' shifted above a
  // 9-bit position stays below KEY_NONE and the exponent shifts out, so one
  // funnel shift of (bits, position << 23) by 23 forms the key.  The true
  // distance D' + |x_q|^2 - M is restored for the k written entries.
  constexpr uint32_t FK_BITS = 9u;
  constexpr uint32_t FK_DSAT = (KEY_NONE >> FK_BITS) - 1u;   // (FK_DSAT << 9) | 511 < KEY_NONE
  bool fastkey = false;
  {
    const float mxn = __uint_as_float(S.max_n);
    fastkey = ikey && nchunk == 1 && m <= (1 << FK_BITS) && 4.0f * mxn < (float)FK_DSAT;   // uniform
    if (fastkey) {
      const float off = mxn + 8388608.0f;
      for (int i = tid; i < m; i += C::THREADS) S.nrm[i] += off;   // padding rows keep PAD_NORM
      __syncthreads();
    }
  }

  // global -> registers for step st (tile st / nchunk, chunk st % nchunk).
  // Every thread issues all STAGE_F4 loads unconditionally, so the number of
  // loads in flight is fixed and the Gram's MFMAs need not wait for this
  // prefetch: rows past the leaf repeat its last member (the padding norm
  // keeps them out of every list); columns past d read column 0 and are
  // zeroed when the values are stored (a select there, after the load, not
  // around it), which a d that is a multiple of KC never needs.
  const bool dfull = d % KC == 0 && TILE_F4 % C::THREADS == 0;   // uniform
  auto stage_load = [&](int st, float4 (&rg)[STAGE_F4]) {
    int t, kci;
    step_tc(st, t, kci);
    const int c0 = t * TILE, kc = kci * KC;
#pragma unroll
    for (int u = 0; u < STAGE_F4; ++u) {
      int e = tid + u * C::THREADS;
      int row = e / F4_PER_ROW, col = (e % F4_PER_ROW) * 4;
      int cp = c0 + row;
      const bool colok = e < TILE_F4 && kc + col < d;
      const int cpc = cp < m ? cp : m - 1;
      // element offset id * d + column as one 32 x 32 + 64-bit multiply-add
      const uint64_t eo = (uint64_t)S.ids[cpc] * (uint32_t)d + (uint32_t)(colok ? kc + col : 0);
      const float4 v = *(const float4*)(a.X + eo);
      rg[u] = v;
    }
  };
  // registers -> LDS; on the first pass of a centred BF16 leaf also the
  // member norms (rows of a tile are held by F4_PER_ROW consecutive lanes,
  // reduced by shuffles)
  auto stage_store = [&](int st, int buf, const float4 (&rg)[STAGE_F4], bool norms) {
    int t, kci;
    step_tc(st, t, kci);
    const int c0 = t * TILE, kc = kci * KC;
#pragma unroll
    for (int u = 0; u < STAGE_F4; ++u) {
      int e = tid + u * C::THREADS;
      int row = e / F4_PER_ROW, col = (e % F4_PER_ROW) * 4;
      float4 v = rg[u];
      if (!dfull && !(e < TILE_F4 && kc + col < d)) v = make_float4(0.f, 0.f, 0.f, 0.f);   // padded features
      float sq;
      if constexpr (!BF16) {
        if (e < TILE_F4) *(float4*)&S.tile[buf].v[row * Tile::STRIDE + col] = v;
        sq = __builtin_fmaf(v.x, v.x, __builtin_fmaf(v.y, v.y, __builtin_fmaf(v.z, v.z, v.w * v.w)));
      } else if (ikey) {
        // integers of magnitude <= 256, not centred: exact in BF16, and the
        // load already zeroed the features past d (no norms are formed here)
        if (e < TILE_F4) *(uint2*)&S.tile[buf].v[row * Tile::STRIDE + col] = make_uint2(pack_bf16(v.x, v.y), pack_bf16(v.z, v.w));
        sq = 0.f;
      } else {
        const bool in = e < TILE_F4 && kc + col < d;   // padded features stay exactly zero
        const float4 m4 = make_float4(S.mu[kc + col], S.mu[kc + col + 1], S.mu[kc + col + 2], S.mu[kc + col + 3]);
        // the four halves in one 8-byte store; the norm is of the rounded values
        const uint32_t lo = in ? pack_bf16(v.x - m4.x, v.y - m4.y) : 0u;
        const uint32_t hi = in ? pack_bf16(v.z - m4.z, v.w - m4.w) : 0u;
        if (e < TILE_F4) *(uint2*)&S.tile[buf].v[row * Tile::STRIDE + col] = make_uint2(lo, hi);
        const float t0 = __uint_as_float(lo << 16), t1 = __uint_as_float(lo & 0xFFFF0000u);
        const float t2 = __uint_as_float(hi << 16), t3 = __uint_as_float(hi & 0xFFFF0000u);
        sq = __builtin_fmaf(t0, t0, __builtin_fmaf(t1, t1, __builtin_fmaf(t2, t2, t3 * t3)));
      }
      if (norms) {   // uniform
#pragma unroll
        for (int o = F4_PER_ROW / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, F4_PER_ROW);
        if (e < TILE_F4 && (e % F4_PER_ROW) == 0) {
          int cp = c0 + row;
          float tot = (cp < m) ? ((kci == 0) ? sq : S.nrm[cp] + sq) : PAD_NORM;
          S.nrm[cp] = tot;
          if (kci == nchunk - 1 && cp < m) {
            atomicMax(&S.max_n, __float_as_uint(tot));
            if (tot > 4194304.0f) S.flag = 0;   // 2^22: partial Gram sums stay exact
          }
        }
      }
    }
  };

  // Tiles are staged two steps ahead into four LDS buffers with a barrier
  // after every second step, so the waves of a SIMD may drift apart by a
  // step (one's key insertion overlapping the other's MFMAs).  A store at
  // step s goes to the buffer read at s + 2 (last read at s - 2), and the
  // barrier between them orders both.  A pass followed by another over the
  // same leaf stages that pass's first two tiles in its last two steps;
  // bufbase keeps the buffer rotation running across passes.
  // BF16 steps are short (one BF16 MFMA does the work of eight FP32 ones),
  // so there a tile's global loads are issued one step earlier still: the
  // loads of step st feed the store of step st + 1, carried in `pend`.
  constexpr bool DEEP = BF16 && KP <= 16;   // (with longer lists the registers run out)
  float4 pend[STAGE_F4];
  int bufbase = 0;
  bool staged = false;
  for (int qb = 0; qb < m; qb += C::QPB) {
    const bool first = qb == 0;
    const bool follow = qb + C::QPB < m;      // another pass comes after this one
    const int qbase = qb + w * QPW;
    const bool wave_on = qbase < m;           // uniform per wave
    const int qpos = qbase + r32;             // this lane's query
    const bool qok = qpos < m;
    const float* qrow = a.X + (size_t)S.ids[qok ? qpos : 0] * d;
    QFrag<KC, BF16> qf;
    // query norm over the lane's half of every chunk, then across the pair
    float nq = 0.f;
    if (wave_on) {
      if (nchunk == 1) {
        qf.load(qrow, 0, d, h, S.mu, qok);
        if constexpr (!BF16) {
#pragma unroll
          for (int i = 0; i < QFrag<KC, BF16>::N4; ++i) {
            nq = __builtin_fmaf(qf.f[i].x, qf.f[i].x, nq);
            nq = __builtin_fmaf(qf.f[i].y, qf.f[i].y, nq);
            nq = __builtin_fmaf(qf.f[i].z, qf.f[i].z, nq);
            nq = __builtin_fmaf(qf.f[i].w, qf.f[i].w, nq);
          }
        } else {
#pragma unroll
          for (int i = 0; i < QFrag<KC, BF16>::N8; ++i)
#pragma unroll
            for (int e = 0; e < 8; ++e) nq = __builtin_fmaf((float)qf.b[i][e], (float)qf.b[i][e], nq);
        }
      } else {
        for (int kc = 0; kc < d; kc += KC) {
#pragma unroll 4
          for (int c = kc + h * HALF; c < kc + h * HALF + HALF; c += 4) {
            float4 v = (qok && c < d) ? *(const float4*)(qrow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
            if (BF16 && qok && c < d) {
              v.x = bf16_round(v.x - S.mu[c]);
              v.y = bf16_round(v.y - S.mu[c + 1]);
              v.z = bf16_round(v.z - S.mu[c + 2]);
              v.w = bf16_round(v.w - S.mu[c + 3]);
            }
            nq = __builtin_fmaf(v.x, v.x, nq);
            nq = __builtin_fmaf(v.y, v.y, nq);
            nq = __builtin_fmaf(v.z, v.z, nq);
            nq = __builtin_fmaf(v.w, v.w, nq);
          }
        }
      }
      nq += __shfl_xor(nq, 32);
      if (h == 0) S.qn[w][r32] = nq;
      if (fastkey) {   // scaling by -2 is exact in either type
        if constexpr (!BF16) {
#pragma unroll
          for (int i = 0; i < QFrag<KC, BF16>::N4; ++i) {
            qf.f[i].x *= -2.0f;
            qf.f[i].y *= -2.0f;
            qf.f[i].z *= -2.0f;
            qf.f[i].w *= -2.0f;
          }
        } else {
#pragma unroll
          for (int i = 0; i < QFrag<KC, BF16>::N8; ++i)
#pragma unroll
            for (int e = 0; e < 8; ++e) qf.b[i][e] = (__bf16)(-2.0f * (float)qf.b[i][e]);
        }
      }
    }
    float Lk[KP];
#pragma unroll
    for (int j = 0; j < KP; ++j) Lk[j] = __uint_as_float(KEY_NONE);
    f32x16 acc0 = {0};
    f32x16 acc_o = {0};   // PAIR: the other tile's partial Gram
    if (!staged) {
      for (int s0 = 0; s0 < 2 && s0 < nsteps; ++s0) {
        float4 rg[STAGE_F4];
        stage_load(s0, rg);
        stage_store(s0, (s0 + bufbase) & (TILE_BUFS - 1), rg, first && !pre_norms);
      }
      if constexpr (DEEP) stage_load(2 < nsteps ? 2 : 0, pend);   // the tile step 0 stores
    }
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
      const int buf = (st + bufbase) & (TILE_BUFS - 1);
      int tl, kci;
      step_tc(st, tl, kci);
      const int c0 = tl * TILE;
      // the query chunk is loaded before the next tile's prefetch so that the
      // MFMAs wait only for the older loads and the prefetch stays in flight
      // (in a pair, by its first tile only)
      if (wave_on && nchunk > 1 && !(pair && st < full && (st & 1))) qf.load(qrow, kci * KC, d, h, S.mu, qok);
      float4 rg[STAGE_F4];
      // step st stages step st + 2 of this pass, or of the next pass over
      // the leaf, or else re-stages its own tile into a buffer nobody reads
      // again, so every step issues the same loads
      const int ahead = st + 2;
      const bool more = ahead < nsteps;
      const bool carry = !more && follow && nsteps >= 2;   // the next pass's step ahead - nsteps
      const int nxt = more ? ahead : carry ? ahead - nsteps : st;
      if constexpr (DEEP) {
        // this step loads the tile the next step stores (step st + 3, in
        // this pass or the next) and stores the one loaded by the last step
        const int ahead3 = st + 3;
        const int nxt3 = ahead3 < nsteps ? ahead3 : (follow && nsteps >= 4) ? ahead3 - nsteps : st;
        stage_load(nxt3, rg);
      } else {
        stage_load(nxt, rg);
      }
      if (wave_on) {
        if constexpr (!BF16) {
          // one accumulation chain (back-to-back dependent MFMAs of one shape
          // need no wait); a chunk that starts a tile starts from the zero
          // constant, so the accumulator needs no clearing
          const float4* trow = reinterpret_cast<const float4*>(&S.tile[buf].v[r32 * Tile::STRIDE + h * HALF]);
          // the tile's next 16 bytes are read while the current ones feed MFMAs
          auto chain = [&](int i0) __attribute__((always_inline)) {
            float4 nx = trow[i0];
#pragma unroll
            for (int i = 0; i < HALF / 4; ++i) {
              if (i < i0) continue;
              const float4 cv = nx;
              if (i + 1 < HALF / 4) nx = trow[i + 1];
              acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.x, qf.f[i].x, acc0, 0, 0, 0);
              acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.y, qf.f[i].y, acc0, 0, 0, 0);
              acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.z, qf.f[i].z, acc0, 0, 0, 0);
              acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.w, qf.f[i].w, acc0, 0, 0, 0);
            }
          };
          if (fastkey) {
            // register r: candidate c0 + 8(r/4) + 4h + r%4, as the keys read it
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const float4 n = *reinterpret_cast<const float4*>(&S.nrm[c0 + 8 * g + 4 * h]);
              acc0[4 * g] = n.x;
              acc0[4 * g + 1] = n.y;
              acc0[4 * g + 2] = n.z;
              acc0[4 * g + 3] = n.w;
            }
            chain(0);
          } else if (kci == 0) {
            const float4 cv = trow[0];
            const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.x, qf.f[0].x, zero, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.y, qf.f[0].y, acc0, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.z, qf.f[0].z, acc0, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(cv.w, qf.f[0].w, acc0, 0, 0, 0);
            chain(1);
          } else {
            chain(0);
          }
        } else {
          const bf16x8* trow = reinterpret_cast<const bf16x8*>(&S.tile[buf].v[r32 * Tile::STRIDE + h * HALF]);
          if (fastkey) {   // one chain from the norms, as in the FP32 form
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const float4 n = *reinterpret_cast<const float4*>(&S.nrm[c0 + 8 * g + 4 * h]);
              acc0[4 * g] = n.x;
              acc0[4 * g + 1] = n.y;
              acc0[4 * g + 2] = n.z;
              acc0[4 * g + 3] = n.w;
            }
#pragma unroll
            for (int i = 0; i < HALF / 8; ++i) acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[i], qf.b[i], acc0, 0, 0, 0);
          } else {
            // two interleaved chains, the second one local to the step and
            // added in at its end (a chain carried across steps would be
            // carried, and copied, through the fast form's steps as well);
            // a tile's first chunk starts both from the zero constant
            const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            f32x16 acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[1], qf.b[1], zero, 0, 0, 0);
            if (kci == 0) acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[0], qf.b[0], zero, 0, 0, 0);
            else acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[0], qf.b[0], acc0, 0, 0, 0);
#pragma unroll
            for (int i = 2; i < HALF / 8; ++i) {
              if (i % 2 == 0) acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[i], qf.b[i], acc0, 0, 0, 0);
              else acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(trow[i], qf.b[i], acc1, 0, 0, 0);
            }
            acc0 += acc1;
          }
        }
        if (kci == nchunk - 1) {
          // register r holds candidate c0 + 8(r/4) + 4h + r%4 against this lane's query
          float4 n4[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) n4[g] = *reinterpret_cast<const float4*>(&S.nrm[c0 + 8 * g + 4 * h]);
          const uint32_t pbase = (uint32_t)(c0 + 4 * h);
          const bool diag = (c0 == qbase);   // uniform: the tile holding the wave's own queries
          const bool ragged = c0 + TILE > m;  // uniform: the last tile has padding rows
          // The tile's 16 keys per lane, then the masks (uniform branch: only
          // the tile holding the wave's own queries, or padding rows when the
          // keys are integers), then one insertion for all key forms.
          // EXACT: integer keys; FAST: keys from the Gram's bits, their
          // position without the lane half 4h (bit 2, set before the halves
          // merge); KI: list entries kept (integer keys need only the k
          // smallest: KP/2, 5KP/8, 3KP/4 or KP, the first that holds k)
          float x[16];
          auto make_keys = [&](auto exact_tag, auto fast_tag) {
            constexpr bool EXACT = decltype(exact_tag)::value;
            constexpr bool FAST = decltype(fast_tag)::value;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              const int cl = 8 * (r >> 2) + (r & 3);
              if constexpr (FAST) {
                // (bits << 9) | position; padding rows are masked below
                x[r] = __uint_as_float(__builtin_amdgcn_alignbit(__float_as_uint(acc0[r]), (uint32_t)(c0 + cl) << 23, 23u));
              } else {
                const float nc = (r & 3) == 0 ? n4[r >> 2].x : (r & 3) == 1 ? n4[r >> 2].y : (r & 3) == 2 ? n4[r >> 2].z : n4[r >> 2].w;
                const float dv = __builtin_fmaf(-2.0f, acc0[r], nq + nc);
                x[r] = EXACT ? make_ikey(dv, pbase + (uint32_t)cl) : make_key(dv, pbase + (uint32_t)cl);
              }
            }
            if (diag || (EXACT && ragged)) {
#pragma unroll
              for (int r = 0; r < 16; ++r) {
                const int cl = 8 * (r >> 2) + (r & 3);
                if (diag && (cl + 4 * h == r32)) x[r] = __uint_as_float(KEY_NONE);
                if (EXACT && ragged && (int)pbase + cl >= m) x[r] = __uint_as_float(KEY_NONE);
              }
            }
          };
          auto insert = [&](auto len_tag) {
            constexpr int KI = decltype(len_tag)::value;
#pragma unroll
            for (int r = 0; r < 16; ++r) list_insert_head<KI>(Lk, x[r]);
          };
          using T_ = std::true_type;
          using F_ = std::false_type;
          if (fastkey) make_keys(T_{}, T_{});
          else if (ikey) make_keys(T_{}, F_{});
          else make_keys(F_{}, F_{});
          if constexpr (KT > 0) {   // the tier fixed by the instance (KT >= k)
            if (ikey) insert(std::integral_constant<int, KT>{});
            else insert(std::integral_constant<int, KP>{});   // float keys keep the whole list
          } else {
            const int kt = ikey ? k : KP;
            if (kt <= KP / 2) insert(std::integral_constant<int, KP / 2>{});
            else if (kt <= KP / 2 + KP / 8) insert(std::integral_constant<int, KP / 2 + KP / 8>{});
            else if (kt <= KP - KP / 4) insert(std::integral_constant<int, KP - KP / 4>{});
            else insert(std::integral_constant<int, KP>{});
          }
        }
        if constexpr (PAIR) {
          if (pair && st < full) {   // uniform: hand over to the pair's other tile
            const f32x16 tmp = acc0;
            acc0 = acc_o;
            acc_o = tmp;
          }
        }
      }
      if constexpr (DEEP) {
        stage_store(nxt, (ahead + bufbase) & (TILE_BUFS - 1), pend, first && more && !pre_norms);
#pragma unroll
        for (int u = 0; u < STAGE_F4; ++u) pend[u] = rg[u];
      } else {
        stage_store(nxt, (ahead + bufbase) & (TILE_BUFS - 1), rg, first && more && !pre_norms);
      }
      if ((st & 1) || st + 1 == nsteps) __syncthreads();
    }
    staged = follow && nsteps >= 2;
    bufbase = (nsteps + bufbase) & (TILE_BUFS - 1);   // the buffer of the next pass's step 0
    if (!wave_on) continue;                   // no barrier below this point
    // ---- merge the two half-lists of each query: the KP smallest of both
    {
      if (fastkey && h) {   // the lane half's position bit (KEY_NONE has it set already)
#pragma unroll
        for (int j = 0; j < KP; ++j) Lk[j] = __uint_as_float(__float_as_uint(Lk[j]) | 4u);
      }
      float P[KP];
#pragma unroll
      for (int j = 0; j < KP; ++j) P[j] = __shfl_xor(Lk[j], 32);
#pragma unroll
      for (int j = 0; j < KP; ++j) Lk[j] = fminf(Lk[j], P[KP - 1 - j]);
#pragma unroll
      for (int s = KP / 2; s > 0; s >>= 1) {
#pragma unroll
        for (int j = 0; j < KP; ++j) {
          if ((j & s) == 0) {
            float lo = fminf(Lk[j], Lk[j + s]), hi = fmaxf(Lk[j], Lk[j + s]);
            Lk[j] = lo;
            Lk[j + s] = hi;
          }
        }
      }
      if (ikey) {
        // exact keys: the merged list is the answer in (distance, id) order;
        // the two lanes of a query write alternate slots
        if (qok) {
          const uint32_t qid = S.ids[qpos];
          // a saturated entry among the written ones (the list is ascending,
          // so the last valid one is the largest) carries neither its true
          // distance nor its (distance, id) order: the row is redone exactly.
          // Rows of leaves with at most k members have padding at slot k - 1,
          // so the check covers every written slot, not only the k-th.
          bool sat = false;
          // fast keys: D' in the bits above pbits, D = D' + |x_q|^2 - M (exact)
          const uint32_t psh = fastkey ? FK_BITS : 11u;
          const uint32_t pmask = (1u << psh) - 1u;
          const uint32_t dsat = fastkey ? FK_DSAT : KEY_DSAT;
          const float dshift = fastkey ? nq - __uint_as_float(S.max_n) : 0.f;
#pragma unroll
          for (int j = 0; j < KP; ++j) {
            const uint32_t kk = __float_as_uint(Lk[j]);
            const bool none = kk == KEY_NONE;
            if (j < k) sat = sat || (!none && (kk >> psh) >= dsat);
            if (j < k && (j & 1) == h) {
              ids_out[(size_t)qid * a.list_row + j] = none ? KNNG_NONE : S.ids[kk & pmask];
              dist_out[(size_t)qid * a.list_row + j] = none ? INF : (float)(kk >> psh) + dshift;
            }
          }
          if (sat && h == 0) {
            unsigned long long sl = atomicAdd(&a.diag->fallback_count, 1ull);
            atomicAdd(&a.diag->leaf_fallback, 1ull);
            if (sl < a.fallback_cap) {
              a.fallback[2 * sl] = L;
              a.fallback[2 * sl + 1] = (uint32_t)qpos;
            }
          }
        }
        continue;
      }
      if (h == 0) {
#pragma unroll
        for (int j = 0; j < KP; ++j) S.lst[w][r32 * LS + j] = __float_as_uint(Lk[j]);
      }
    }
    wave_sync();
    // ---- exact re-rank: groups of 16 lanes, eight pairs (two list blocks) in flight at a time
    {
      const int g = lane >> 4, gl = lane & 15;
      for (int blk2 = 0; blk2 < QPW * KP; blk2 += 32) {
        const float* xq[2];
        const float* xc[2][4];
        bool ok[2][4];
        int ee[2][4], qjv[2];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int blk = blk2 + 16 * b;
          const int qj = blk / KP;
          qjv[b] = qj;
          const int qp = qbase + qj;
          xq[b] = a.X + (size_t)S.ids[qp < m ? qp : 0] * d;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            ee[b][u] = (blk % KP) + g + 4 * u;
            uint32_t kk = S.lst[w][qj * LS + ee[b][u]];
            ok[b][u] = kk < KEY_VALID && qp < m;
            int cp = ok[b][u] ? (int)(kk & POS_MASK) : 0;
            xc[b][u] = a.X + (size_t)S.ids[cp] * d;
          }
        }
        float dd[2][4];
        dist2_g16_x8(xq[0], xc[0], xq[1], xc[1], d, gl, dd[0], dd[1]);
        if (gl == 0) {
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int u = 0; u < 4; ++u) S.dst[w][qjv[b] * LS + ee[b][u]] = ok[b][u] ? dd[b][u] : INF;
        }
      }
    }
    wave_sync();
    // ---- sort each query's KP (distance, id) keys; blocks of KP over the wave
    constexpr int R = (QPW * KP) / 64;
    uint64_t kv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int e = r * 64 + lane;
      int qj = e / KP, slot = e % KP;
      uint32_t kk = S.lst[w][qj * LS + slot];
      kv[r] = kk < KEY_VALID ? pack_did(S.dst[w][qj * LS + slot], S.ids[kk & POS_MASK]) : ~0ull;
    }
    wave_bitonic<R, KP, uint64_t>(kv, lane);
    const float max_n = __uint_as_float(S.max_n);
    const bool exact_gram = S.flag;
    // write rows, check the certificate on slot k-1
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int e = r * 64 + lane;
      int qj = e / KP, slot = e % KP;
      int qp = qbase + qj;
      if (qp < m && slot < k) {
        uint32_t qid = S.ids[qp];
        ids_out[(size_t)qid * a.list_row + slot] = key_id(kv[r]);
        dist_out[(size_t)qid * a.list_row + slot] = key_dist(kv[r]);
        if (slot == k - 1) {
          // every candidate outside the list has a key at least the KP-th's
          uint32_t kl = S.lst[w][qj * LS + KP - 1];
          bool cert = true;
          if (kl < KEY_VALID) {
            float vlast = key_value(kl) - 2.0f * KEY_FLOOR;
            float nq = S.qn[w][qj];
            float lb;
            if (exact_gram) {
              lb = vlast;
            } else if (BF16) {
              float e32 = eps_c * (nq + max_n);
              // rounding each centred row to BF16 moves it by at most 2^-8 of its norm
              float delta = (0.00390625f + 1.2e-7f) * 1.0025f * (sqrtf(nq) + sqrtf(max_n)) * 1.001f;
              float rt = sqrtf(fmaxf(vlast - e32, 0.f)) - delta;
              lb = rt > 0.f ? rt * rt * 0.9999f : 0.f;
            } else {
              lb = vlast - eps_c * (nq + max_n);
            }
            float dk = key_dist(kv[r]);
            cert = lb > dk * (1.0f + 2e-6f);
          }
          if (!cert) {
            unsigned long long sl = atomicAdd(&a.diag->fallback_count, 1ull);
            atomicAdd(&a.diag->leaf_fallback, 1ull);
            if (sl < a.fallback_cap) {
              a.fallback[2 * sl] = L;
              a.fallback[2 * sl + 1] = (uint32_t)qp;
            }
          }
        }
      }
    }
    wave_sync();
  }
}

// Single-division mode: one workgroup per leaf.  Batched mode: a persistent
// grid; each workgroup takes the next leaf from the work list (largest
// first) until the list is exhausted, so every workgroup reaches the exit.
template <int KC, int KP, bool BF16, int W, int KT, bool PAIR>
__global__ __launch_bounds__((Cfg<KP, W>::THREADS)) void k_leaf(LeafArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using Sh = LeafShared<KC, KP, BF16, W>;
  Sh& S = *reinterpret_cast<Sh*>(smem_raw);
  __shared__ uint32_t next;
  if (a.skip && *a.skip) return;   // uniform: a later division of a stopped build
  // the index of the following work item is taken when a leaf starts, so
  // the atomic's round trip overlaps the leaf's own loads
  if (a.work && threadIdx.x == 0) next = atomicAdd(a.counter, 1u);
  uint32_t following = 0;
  unsigned long long rows = 0;   // members of this workgroup's leaves, added to the diagnostics once
  // single-division mode runs one pass of the loop for leaf blockIdx.x
  for (uint32_t pass = 0;; ++pass) {
    uint32_t idx;
    if (a.work) {
      __syncthreads();
      idx = __builtin_amdgcn_readfirstlane(next);   // every thread read the same value: a scalar
      __syncthreads();
      if (idx >= a.n_work) break;
      if (threadIdx.x == 0) following = atomicAdd(a.counter, 1u);
    } else {
      if (pass > 0) break;
      idx = blockIdx.x;
    }
    const uint32_t* perm = a.perm;
    uint32_t* ids_out = a.ids;
    float* dist_out = a.dist;
    int64_t off;
    int m;
    if (a.work) {
      const LeafWork wk = a.work[idx];
      perm += (size_t)wk.slot * a.n;
      ids_out += (size_t)wk.slot * a.list_slot;
      dist_out += (size_t)wk.slot * a.list_slot;
      off = (int64_t)wk.off;
      m = (int)wk.m;
    } else {
      off = a.leaf_off[idx];
      m = (int)(a.leaf_off[idx + 1] - off);
    }
    leaf_body<KC, KP, BF16, W, KT, PAIR>(a, S, perm, ids_out, dist_out, off, m, idx);
    if (m > 0) rows += (unsigned long long)m;
    if (a.work && threadIdx.x == 0) next = following;
    __syncthreads();
  }
  if (threadIdx.x == 0 && rows) atomicAdd(&a.diag->leaf_rows, rows);
}

// Exact row: distances from one member to every other member of its leaf,
// streamed in chunks of 2048 through an LDS bitonic sort; keeps the first k
// by (distance, id).
__global__ __launch_bounds__(256) void k_leaf_exact(LeafArgs a) {
  __shared__ uint64_t keys[2048 + 64];
  __shared__ uint64_t best[64];
  if (a.skip && *a.skip) return;   // uniform
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  unsigned long long cnt = a.diag->fallback_count;
  if (cnt > a.fallback_cap) cnt = a.fallback_cap;
  for (unsigned long long it = blockIdx.x; it < cnt; it += gridDim.x) {
    const uint32_t L = a.fallback[2 * it], qp = a.fallback[2 * it + 1];
    int64_t off, m;
    const uint32_t* perm = a.perm;
    uint32_t* ids_out = a.ids;
    float* dist_out = a.dist;
    if (a.work) {
      const LeafWork wk = a.work[L];
      off = (int64_t)wk.off;
      m = wk.m;
      perm += (size_t)wk.slot * a.n;
      ids_out += (size_t)wk.slot * a.list_slot;
      dist_out += (size_t)wk.slot * a.list_slot;
    } else {
      off = a.leaf_off[L];
      m = a.leaf_off[L + 1] - off;
    }
    const uint32_t qid = perm[off + qp];
    const float* xq = a.X + (size_t)qid * a.d;
    if (tid < 64) best[tid] = ~0ull;
    __syncthreads();
    for (int64_t c0 = 0; c0 < m; c0 += 2048) {
      // 16 groups of 16 lanes score candidates c0 + gid, c0 + gid + 16, ...
      const int gid = tid >> 4, gl = tid & 15;
      for (int j = gid; j < 2048; j += 16) {
        int64_t cp = c0 + j;
        uint64_t key = ~0ull;
        if (cp < m) {   // uniform across the 16-lane group
          uint32_t cid = perm[off + cp];
          float dd = dist2_g16(xq, a.X + (size_t)cid * a.d, a.d, gl);
          if (cp != (int64_t)qp) key = pack_did(dd, cid);
        }
        if (gl == 0) keys[j] = key;
      }
      if (tid < 64) keys[2048 + tid] = best[tid];
      __syncthreads();
      // bitonic sort of 2048 keys (the 64 kept ones ride along below)
      for (int size = 2; size <= 2048; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          for (int e = tid; e < 2048; e += 256) {
            int p = e ^ stride;
            if (p > e) {
              bool asc = (e & size) == 0;
              uint64_t x = keys[e], y = keys[p];
              if (asc ? (x > y) : (x < y)) { keys[e] = y; keys[p] = x; }
            }
          }
          __syncthreads();
        }
      }
      // merge the sorted chunk's first k with the kept list (wave 0)
      if (wv == 0) {
        uint64_t x = lane < a.k ? keys[lane] : ~0ull;
        uint64_t y = lane < a.k ? keys[2048 + lane] : ~0ull;
        // 128-element sort of the two lists in registers, keep first k
        uint64_t v[2] = {x, y};
        wave_bitonic<2, 128, uint64_t>(v, lane);
        if (lane < 64) best[lane] = lane < a.k ? v[0] : ~0ull;
      }
      __syncthreads();
    }
    if (tid < a.k) {
      ids_out[(size_t)qid * a.list_row + tid] = key_id(best[tid]);
      dist_out[(size_t)qid * a.list_row + tid] = key_dist(best[tid]);
    }
    __syncthreads();
  }
}

template <int KC, int KP, bool BF16, int W, int KT, bool PAIR = false>
hipError_t launch_leaf_t(const LeafArgs& a, hipStream_t s) {
  using Sh = LeafShared<KC, KP, BF16, W>;
  if constexpr (sizeof(Sh) + 64 > 160 * 1024) {
    return hipErrorInvalidConfiguration;   // this tile shape does not fit a CU's LDS
  } else {
    size_t shm = sizeof(Sh);
    auto kern = k_leaf<KC, KP, BF16, W, KT, PAIR>;
    constexpr int THREADS = Cfg<KP, W>::THREADS;
    static int per_cu = 0;
    if (per_cu == 0) {
      hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
      int occ = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, THREADS, shm);
      per_cu = (e == hipSuccess && occ > 0) ? occ : 1;
    }
    if (a.prepare_only) return hipSuccess;
    if (a.work) {
      hipError_t e = launch_fill_u32(a.counter, 0u, 1, s);
      if (e != hipSuccess) return e;
      unsigned grid = (unsigned)std::min<uint64_t>(a.n_work, (uint64_t)a.grid * per_cu);
      if (grid == 0) return hipSuccess;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(THREADS), shm, s, a);
    } else {
      hipLaunchKernelGGL(kern, dim3((unsigned)a.n_leaves), dim3(THREADS), shm, s, a);
    }
    return hipGetLastError();
  }
}

template <int KC, int KP, bool BF16>
hipError_t launch_leaf_w(const LeafArgs& a, hipStream_t s) {
  const int w = a.waves ? a.waves : (KP <= 32 ? 8 : 4);
  if (w == 8) {
    // rows of more than one chunk: tiles in pairs (one query fragment load
    // serves two tiles)
    if (a.d > KC) return launch_leaf_t<KC, KP, BF16, 8, 0, true>(a, s);
    // the common shape (d in (64, 128], k + rerank_m <= 16, 8 waves) has an
    // instance per list-length tier, so its steps hold one insertion
    if constexpr (KC == 128 && KP == 16) {
      if (a.k <= KP / 2) return launch_leaf_t<KC, KP, BF16, 8, KP / 2>(a, s);
      if (a.k <= KP / 2 + KP / 8) return launch_leaf_t<KC, KP, BF16, 8, KP / 2 + KP / 8>(a, s);
      if (a.k <= KP - KP / 4) return launch_leaf_t<KC, KP, BF16, 8, KP - KP / 4>(a, s);
      return launch_leaf_t<KC, KP, BF16, 8, KP>(a, s);
    } else {
      return launch_leaf_t<KC, KP, BF16, 8, 0>(a, s);
    }
  }
  if (w == 4) return launch_leaf_t<KC, KP, BF16, 4, 0>(a, s);
  return hipErrorInvalidValue;
}

template <int KC, bool BF16>
hipError_t launch_leaf_kp(const LeafArgs& a, hipStream_t s) {
  if (a.kp <= 16) return launch_leaf_w<KC, 16, BF16>(a, s);
  if (a.kp <= 32) return launch_leaf_w<KC, 32, BF16>(a, s);
  return launch_leaf_w<KC, 64, BF16>(a, s);
}

template <bool BF16>
hipError_t launch_leaf_kc(const LeafArgs& a, hipStream_t s) {
  const int kc = a.kc ? a.kc : (a.d <= 32 ? 32 : a.d <= 64 ? 64 : 128);
  if (kc == 32) return launch_leaf_kp<32, BF16>(a, s);
  if (kc == 64) return launch_leaf_kp<64, BF16>(a, s);
  if (kc == 128) return launch_leaf_kp<128, BF16>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace

// X as bytes (each value clamped to [0, 255]): sixteen values per thread,
// four 16-byte loads and one 16-byte store; the last thread of a ragged end
// goes four values at a time.
__global__ __launch_bounds__(256) void k_byte_copy(const float* __restrict__ X, int64_t count, uint8_t* __restrict__ x8) {
  const int64_t e0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 16;
  if (e0 >= count) return;
  auto pack = [](float4 v) -> uint32_t {
    const uint32_t b0 = (uint32_t)fminf(fmaxf(v.x, 0.f), 255.f), b1 = (uint32_t)fminf(fmaxf(v.y, 0.f), 255.f);
    const uint32_t b2 = (uint32_t)fminf(fmaxf(v.z, 0.f), 255.f), b3 = (uint32_t)fminf(fmaxf(v.w, 0.f), 255.f);
    return b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
  };
  const float4* xv = (const float4*)(X + e0);
  if (e0 + 16 <= count) {
    const float4 v0 = xv[0], v1 = xv[1], v2 = xv[2], v3 = xv[3];
    *(uint4*)(x8 + e0) = make_uint4(pack(v0), pack(v1), pack(v2), pack(v3));
  } else {
    for (int64_t e = e0; e < count; e += 4) *(uint32_t*)(x8 + e) = pack(*(const float4*)(X + e));
  }
}

hipError_t launch_data_check(const float* X, int64_t n, int d, uint32_t* flags, float* pnorm, uint8_t* x8,
                             hipStream_t s) {
  hipError_t e = launch_fill_u32(flags, EXACT_FP32 | EXACT_BF16 | EXACT_U8, 1, s);
  if (e != hipSuccess || n <= 0) return e;
  hipLaunchKernelGGL(k_exact_check, dim3((unsigned)((n * 16 + 255) / 256)), dim3(256), 0, s, X, n, d, flags, pnorm);
  if ((e = hipGetLastError()) != hipSuccess || !x8) return e;
  const int64_t count = n * (int64_t)d;
  hipLaunchKernelGGL(k_byte_copy, dim3((unsigned)((count / 16 + 256) / 256)), dim3(256), 0, s, X, count, x8);
  return hipGetLastError();
}

hipError_t launch_leaf(const LeafArgs& a, hipStream_t s) {
  hipError_t e;
  if (a.prepare_only) return a.precision == KNNG_BF16 ? launch_leaf_kc<true>(a, s) : launch_leaf_kc<false>(a, s);
  if ((e = launch_fill_u32((uint32_t*)&a.diag->fallback_count, 0u, 2, s)) != hipSuccess) return e;
  if (!a.data_checked && (e = launch_data_check(a.X, a.n, a.d, &a.diag->exact_flags, a.pnorm, nullptr, s)) != hipSuccess)
    return e;
  e = a.precision == KNNG_BF16 ? launch_leaf_kc<true>(a, s) : launch_leaf_kc<false>(a, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_leaf_exact, dim3(1024), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
