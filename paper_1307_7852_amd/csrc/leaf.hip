// Exact k-NN inside every leaf subset (Section 3.1's brute-force subgraph).
//
// One workgroup (4 waves) per leaf.  The leaf's members stream through LDS in
// tiles of 32 candidates x KC features (double-buffered, staged once for all
// four waves, rows padded so the MFMA operand reads are bank-conflict free).
// Each wave owns 32 queries (fragments in registers) and computes
//   G[c][q] = x_c . x_q         (v_mfma_f32_32x32x2_f32, or the BF16 form
//                                v_mfma_f32_32x32x16_bf16 on leaf-centred data)
//   s[c][q] = |x_c|^2 - 2 G     (the query's own norm is constant per row)
// A lane holds one query and 16 of every tile's 32 candidates; it keeps its
// best KP candidates in a sorted register list fed through a small LDS
// queue, so lanes with nothing to insert do not stall the others.  The two
// lanes sharing a query exchange thresholds after every tile and merge their
// lists in registers at the end.  The KP survivors are re-scored with the
// canonical FP32 distance, sorted by (distance, id), and the first k written.
// A row whose k-th exact distance is not safely below every rejected
// candidate's lower bound (from the Gram's error bound) is redone exactly by
// k_leaf_exact.
#include "knng_dev.h"

#include <algorithm>
#include <type_traits>

namespace knng {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int LEAF_THREADS = 256;
constexpr int QPW = 32;            // queries per wave
constexpr int QPB = 128;           // queries per block pass
constexpr int TILE = 32;           // candidates per tile
constexpr int QUEUE = 8;           // per-lane queue slots (half a tile's share)
constexpr int MU_MAX = 2048;       // BF16 path: d <= 2048

template <int KP>
__device__ __forceinline__ void list_insert(float (&v)[KP], int (&p)[KP], float x, int px) {
#pragma unroll
  for (int s = KP - 1; s > 0; --s) {
    bool sh = x < v[s - 1];
    bool tk = x < v[s];
    float nv = sh ? v[s - 1] : x;
    int np = sh ? p[s - 1] : px;
    v[s] = tk ? nv : v[s];
    p[s] = tk ? np : p[s];
  }
  bool t0 = x < v[0];
  v[0] = t0 ? x : v[0];
  p[0] = t0 ? px : p[0];
}

// (value, position) order with the empty entry (-1 as unsigned) last.
__device__ __forceinline__ bool vp_less(float va, int pa, float vb, int pb) {
  return va < vb || (va == vb && (unsigned)pa < (unsigned)pb);
}

// Lanes l and l^32 hold sorted lists of the same query; both end with the
// first KP of the union, sorted (a bitonic merge: the element-wise minimum of
// one list and the other reversed holds the KP smallest, then half-cleaners).
template <int KP>
__device__ __forceinline__ void pair_merge(float (&v)[KP], int (&p)[KP]) {
  float ov[KP];
  int op[KP];
#pragma unroll
  for (int s = 0; s < KP; ++s) {
    ov[s] = __shfl_xor(v[s], 32);
    op[s] = __shfl_xor(p[s], 32);
  }
#pragma unroll
  for (int s = 0; s < KP; ++s) {
    float bv = ov[KP - 1 - s];
    int bp = op[KP - 1 - s];
    bool tb = vp_less(bv, bp, v[s], p[s]);
    v[s] = tb ? bv : v[s];
    p[s] = tb ? bp : p[s];
  }
#pragma unroll
  for (int stride = KP / 2; stride > 0; stride >>= 1) {
#pragma unroll
    for (int s = 0; s < KP; ++s) {
      if ((s & stride) == 0) {
        bool sw = vp_less(v[s + stride], p[s + stride], v[s], p[s]);
        float tv = v[s];
        int tp = p[s];
        v[s] = sw ? v[s + stride] : v[s];
        p[s] = sw ? p[s + stride] : p[s];
        v[s + stride] = sw ? tv : v[s + stride];
        p[s + stride] = sw ? tp : p[s + stride];
      }
    }
  }
}

// Four canonical distances from one row to four rows (identical arithmetic
// to dist2_g16 for each pair; the loads of all five rows are in flight together).
__device__ __forceinline__ void dist2_g16_x4(const float* __restrict__ x, const float* const (&y)[4], int d, int g,
                                             float (&out)[4]) {
  float a[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u) a[u][0] = a[u][1] = a[u][2] = a[u][3] = 0.f;
  const int nc = d >> 2;
  for (int c = g; c < nc; c += 16) {
    float4 xv = ((const float4*)x)[c];
    float4 w[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = ((const float4*)y[u])[c];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float e0 = xv.x - w[u].x, e1 = xv.y - w[u].y, e2 = xv.z - w[u].z, e3 = xv.w - w[u].w;
      a[u][0] = __builtin_fmaf(e0, e0, a[u][0]);
      a[u][1] = __builtin_fmaf(e1, e1, a[u][1]);
      a[u][2] = __builtin_fmaf(e2, e2, a[u][2]);
      a[u][3] = __builtin_fmaf(e3, e3, a[u][3]);
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

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// Tile element types: FP32 rows padded by 4 floats, BF16 rows by 8 halves;
// either way consecutive rows start 16 bytes apart modulo the bank width.
template <int KC, bool BF16>
struct TileT {
  static constexpr int STRIDE = BF16 ? (KC + 8) : (KC + 4);   // elements per row
  using E = typename std::conditional<BF16, __bf16, float>::type;
  E v[TILE * STRIDE];
};

template <int KC, int KP, bool BF16>
struct LeafShared {
  uint32_t ids[KNNG_MAX_LEAF];
  float nrm[KNNG_MAX_LEAF];
  TileT<KC, BF16> tile[2];
  float mu[BF16 ? MU_MAX : 1];
  float red[8];
  int flag;
  // per wave: the tile loop's queues (64 x QUEUE float2), then the re-rank
  // buffers (positions, approximate values, exact distances: 3 x QPW x KP)
  alignas(16) unsigned char scratch[4][(64 * QUEUE * 8 > 12 * QPW * KP) ? 64 * QUEUE * 8 : 12 * QPW * KP];
};

// Query fragments in registers: lane (h, r) owns features [h*HALF, h*HALF+HALF)
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
#pragma unroll
      for (int i = 0; i < N8; ++i) {
        int c = kc + h * HALF + 8 * i;
#pragma unroll
        for (int e = 0; e < 8; ++e) b[i][e] = (__bf16)((ok && c + e < d) ? row[c + e] - mu[c + e] : 0.f);
      }
    }
  }
};

// One leaf: members perm[off .. off+m), rows written to ids/dist (already
// offset to the leaf's division).  `key` names the leaf in the fallback list.
template <int KC, int KP, bool BF16>
__device__ __forceinline__ void leaf_body(const LeafArgs& a, LeafShared<KC, KP, BF16>& S, const uint32_t* __restrict__ perm,
                          uint32_t* __restrict__ ids_out, float* __restrict__ dist_out, int64_t off, int m, uint32_t key) {
  using Tile = TileT<KC, BF16>;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, h = lane >> 5, r32 = lane & 31;
  const int d = a.d, k = a.k;
  const uint32_t L = key;
  if (m <= 0) return;
  if (tid == 0) atomicAdd(&a.diag->leaf_rows, (unsigned long long)m);
  if (m > KNNG_MAX_LEAF) {   // every row goes to the exact kernel
    for (int i = tid; i < m; i += LEAF_THREADS) {
      unsigned long long slot = atomicAdd(&a.diag->fallback_count, 1ull);
      atomicAdd(&a.diag->leaf_fallback, 1ull);
      if (slot < a.fallback_cap) {   // capacity: every point of every division once
        a.fallback[2 * slot] = L;
        a.fallback[2 * slot + 1] = (uint32_t)i;
      }
    }
    return;
  }
  for (int i = tid; i < m; i += LEAF_THREADS) S.ids[i] = perm[off + i];
  if (tid == 0) S.flag = 1;
  __syncthreads();
  // ---- prologue: leaf mean (BF16), member norms, exactness flag, norm bounds
  if constexpr (BF16) {
    for (int j = tid; j < d; j += LEAF_THREADS) {
      float acc = 0.f;
      for (int i = 0; i < m; ++i) acc += a.X[(size_t)S.ids[i] * d + j];
      S.mu[j] = acc / (float)m;
    }
    __syncthreads();
  }
  float my_max_n = 0.f, my_max_c = 0.f;
  int all_int = 1;
  for (int i = w; i < m; i += 4) {            // a wave per member row, lanes over features
    const float* x = a.X + (size_t)S.ids[i] * d;
    float nacc = 0.f, cacc = 0.f;
    for (int j = lane; j < d; j += 64) {
      float v = x[j];
      if (BF16) {
        float c = v - S.mu[j];
        float t = bf16_round(c);
        nacc = __builtin_fmaf(t, t, nacc);
        cacc = __builtin_fmaf(c, c, cacc);
      } else {
        nacc = __builtin_fmaf(v, v, nacc);
        all_int &= (v == rintf(v));
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      nacc += __shfl_xor(nacc, o);
      cacc += __shfl_xor(cacc, o);
    }
    if (!BF16) all_int &= (nacc <= 4194304.0f);   // 2^22: every Gram partial sum exact
    if (lane == 0) S.nrm[i] = nacc;
    my_max_n = fmaxf(my_max_n, nacc);
    my_max_c = fmaxf(my_max_c, cacc);
  }
  if (lane == 0) { S.red[w] = my_max_n; S.red[4 + w] = my_max_c; }
  if (!all_int) S.flag = 0;
  __syncthreads();
  const float max_n = fmaxf(fmaxf(S.red[0], S.red[1]), fmaxf(S.red[2], S.red[3]));
  const float max_c = sqrtf(fmaxf(fmaxf(S.red[4], S.red[5]), fmaxf(S.red[6], S.red[7])));
  const bool exact_gram = !BF16 && S.flag;
  const float eps_c = 2.0f * (float)(d + 4) * 5.9604645e-8f;   // 2 (d+4) 2^-24

  unsigned char* scr = S.scratch[w];
  float2* myq = reinterpret_cast<float2*>(scr) + lane * QUEUE;
  constexpr int HALF = KC / 2;
  constexpr int F4_PER_ROW = KC / 4;
  constexpr int STAGE_F4 = TILE * F4_PER_ROW / LEAF_THREADS;   // float4 per thread per tile chunk
  static_assert(STAGE_F4 >= 1, "tile too small for the block");
  const int nchunk = (d + KC - 1) / KC;
  const int ntile = (m + TILE - 1) / TILE;
  const int nsteps = ntile * nchunk;

  // global -> registers for step st (tile st / nchunk, chunk st % nchunk)
  auto stage_load = [&](int st, float4 (&rg)[STAGE_F4]) {
    int c0 = (st / nchunk) * TILE, kc = (st % nchunk) * KC;
#pragma unroll
    for (int u = 0; u < STAGE_F4; ++u) {
      int e = tid + u * LEAF_THREADS;
      int row = e / F4_PER_ROW, col = (e % F4_PER_ROW) * 4;
      int cp = c0 + row;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (cp < m && kc + col < d) v = *(const float4*)(a.X + (size_t)S.ids[cp] * d + kc + col);
      rg[u] = v;
    }
  };
  auto stage_store = [&](int st, int buf, const float4 (&rg)[STAGE_F4]) {
    int kc = (st % nchunk) * KC;
#pragma unroll
    for (int u = 0; u < STAGE_F4; ++u) {
      int e = tid + u * LEAF_THREADS;
      int row = e / F4_PER_ROW, col = (e % F4_PER_ROW) * 4;
      if constexpr (!BF16) {
        *(float4*)&S.tile[buf].v[row * Tile::STRIDE + col] = rg[u];
      } else {
        float4 v = rg[u];
        bool in = kc + col < d;   // padded features stay exactly zero
        __bf16* dst = &S.tile[buf].v[row * Tile::STRIDE + col];
        dst[0] = (__bf16)(in ? v.x - S.mu[kc + col] : 0.f);
        dst[1] = (__bf16)(in ? v.y - S.mu[kc + col + 1] : 0.f);
        dst[2] = (__bf16)(in ? v.z - S.mu[kc + col + 2] : 0.f);
        dst[3] = (__bf16)(in ? v.w - S.mu[kc + col + 3] : 0.f);
      }
    }
  };

  for (int qb = 0; qb < m; qb += QPB) {
    const int qbase = qb + w * QPW;
    const bool wave_on = qbase < m;           // uniform per wave
    const int qpos = qbase + r32;
    const bool qok = qpos < m;
    const float* qrow = a.X + (size_t)S.ids[qok ? qpos : 0] * d;
    QFrag<KC, BF16> qf;
    if (nchunk == 1 && wave_on) qf.load(qrow, 0, d, h, S.mu, qok);
    float lv[KP];
    int lp[KP];
#pragma unroll
    for (int s = 0; s < KP; ++s) { lv[s] = __int_as_float(0x7F800000); lp[s] = -1; }
    float thr_pair = __int_as_float(0x7F800000);
    f32x16 acc0 = {0}, acc1 = {0};
    {
      float4 rg[STAGE_F4];
      stage_load(0, rg);
      stage_store(0, 0, rg);
    }
    __syncthreads();
    for (int st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      const int c0 = (st / nchunk) * TILE, kci = st % nchunk;
      float4 rg[STAGE_F4];
      const bool more = st + 1 < nsteps;
      if (more) stage_load(st + 1, rg);
      if (wave_on) {
        if (nchunk > 1) qf.load(qrow, kci * KC, d, h, S.mu, qok);
        if (kci == 0) {
#pragma unroll
          for (int r = 0; r < 16; ++r) { acc0[r] = 0.f; acc1[r] = 0.f; }
        }
        if constexpr (!BF16) {
          const float4* trow = reinterpret_cast<const float4*>(&S.tile[buf].v[r32 * Tile::STRIDE + h * HALF]);
#pragma unroll
          for (int i = 0; i < HALF / 4; ++i) {
            float4 av = trow[i];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.x, qf.f[i].x, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.y, qf.f[i].y, acc1, 0, 0, 0);
            acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.z, qf.f[i].z, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(av.w, qf.f[i].w, acc1, 0, 0, 0);
          }
        } else {
          const bf16x8* trow = reinterpret_cast<const bf16x8*>(&S.tile[buf].v[r32 * Tile::STRIDE + h * HALF]);
#pragma unroll
          for (int i = 0; i < HALF / 8; ++i) {
            bf16x8 av = trow[i];
            if (i % 2 == 0) acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, qf.b[i], acc0, 0, 0, 0);
            else acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, qf.b[i], acc1, 0, 0, 0);
          }
        }
        if (kci == nchunk - 1) {
          // filter this tile into the lane's queue, half a tile at a time
#pragma unroll
          for (int half = 0; half < 2; ++half) {
            int cnt = 0;
#pragma unroll
            for (int rr = 0; rr < 8; ++rr) {
              const int r = half * 8 + rr;
              int ci = 8 * (r >> 2) + 4 * h + (r & 3);
              int cp = c0 + ci;
              float g = acc0[r] + acc1[r];
              float sv = (cp < m ? S.nrm[cp] : 0.f) - 2.0f * g;
              bool ok = qok && cp < m && cp != qpos && (sv < lv[KP - 1]) && (sv <= thr_pair);
              if (ok) myq[cnt] = make_float2(sv, __int_as_float(cp));
              cnt += ok ? 1 : 0;
            }
            for (int q = 0; __any(q < cnt); ++q) {
              if (q < cnt) {
                float2 e = myq[q];
                if (e.x < lv[KP - 1]) list_insert<KP>(lv, lp, e.x, __float_as_int(e.y));
              }
            }
          }
          thr_pair = __shfl_xor(lv[KP - 1], 32);
        }
      }
      if (more) stage_store(st + 1, buf ^ 1, rg);
      __syncthreads();
    }
    if (!wave_on) continue;                   // no barrier below this point
    // ---- merge the two half-lists of each query (both lanes end with it)
    pair_merge<KP>(lv, lp);
    int* pb = reinterpret_cast<int*>(scr);                       // [QPW][KP] candidate positions
    float* vbuf = reinterpret_cast<float*>(scr) + QPW * KP;      // [QPW][KP] approximate values
    float* dex = reinterpret_cast<float*>(scr) + 2 * QPW * KP;   // [QPW][KP] exact distances
    wave_sync();
    if (h == 0) {
#pragma unroll
      for (int s2 = 0; s2 < KP; ++s2) { pb[r32 * KP + s2] = lp[s2]; vbuf[r32 * KP + s2] = lv[s2]; }
    }
    wave_sync();
    // ---- exact re-rank: groups of 16 lanes, four pairs of one query at a time
    {
      const int g = lane >> 4, gl = lane & 15;
      for (int blk = 0; blk < QPW * KP; blk += 16) {
        const int qj = blk / KP;
        const int qp = qbase + qj;
        const float* xq = a.X + (size_t)S.ids[qp < m ? qp : 0] * d;
        const float* xc[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int cp = pb[blk + g + 4 * u];
          ok[u] = cp >= 0 && qp < m;
          xc[u] = a.X + (size_t)S.ids[ok[u] ? cp : 0] * d;
        }
        float dd[4];
        dist2_g16_x4(xq, xc, d, gl, dd);
        if (gl == 0) {
#pragma unroll
          for (int u = 0; u < 4; ++u) dex[blk + g + 4 * u] = ok[u] ? dd[u] : __int_as_float(0x7F800000);
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
      int cp = pb[e];
      kv[r] = cp >= 0 ? pack_did(dex[e], S.ids[cp]) : ~0ull;
    }
    wave_bitonic<R, KP, uint64_t>(kv, lane);
    // write rows, check the certificate on slot k-1
#pragma unroll
    for (int r = 0; r < R; ++r) {
      int e = r * 64 + lane;
      int qj = e / KP, slot = e % KP;
      int qp = qbase + qj;
      if (qp < m && slot < k) {
        uint32_t qid = S.ids[qp];
        ids_out[(size_t)qid * k + slot] = key_id(kv[r]);
        dist_out[(size_t)qid * k + slot] = key_dist(kv[r]);
        if (slot == k - 1) {
          // worst rejected candidate: the KP-th approximate value, if the list was full
          float vlast = vbuf[qj * KP + KP - 1];
          bool full = pb[qj * KP + KP - 1] >= 0;
          bool cert = true;
          if (full && !exact_gram) {
            float nq = S.nrm[qp];
            float dt = nq + vlast;                         // approximate distance of the boundary
            float e32 = eps_c * (nq + max_n);
            float lb;
            if (BF16) {
              float xq = 0.f;
              const float* xr = a.X + (size_t)qid * d;
              for (int j = 0; j < d; ++j) { float c = xr[j] - S.mu[j]; xq = __builtin_fmaf(c, c, xq); }
              float delta = (0.00390625f + 1.2e-7f) * (sqrtf(xq) + max_c) * 1.001f;
              float rt = sqrtf(fmaxf(dt - e32, 0.f)) - delta;
              lb = rt > 0.f ? rt * rt * 0.9999f : 0.f;
            } else {
              lb = dt - e32;
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
template <int KC, int KP, bool BF16>
__global__ __launch_bounds__(LEAF_THREADS, 2) void k_leaf(LeafArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  using Sh = LeafShared<KC, KP, BF16>;
  Sh& S = *reinterpret_cast<Sh*>(smem_raw);
  __shared__ uint32_t next;
  // single-division mode runs one pass of the loop for leaf blockIdx.x
  for (uint32_t pass = 0;; ++pass) {
    uint32_t idx;
    if (a.work) {
      if (threadIdx.x == 0) next = atomicAdd(a.counter, 1u);
      __syncthreads();
      idx = next;
      __syncthreads();
      if (idx >= a.n_work) break;
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
      ids_out += (size_t)wk.slot * a.n * a.k;
      dist_out += (size_t)wk.slot * a.n * a.k;
      off = (int64_t)wk.off;
      m = (int)wk.m;
    } else {
      off = a.leaf_off[idx];
      m = (int)(a.leaf_off[idx + 1] - off);
    }
    leaf_body<KC, KP, BF16>(a, S, perm, ids_out, dist_out, off, m, idx);
    __syncthreads();
  }
}

// Exact row: distances from one member to every other member of its leaf,
// streamed in chunks of 2048 through an LDS bitonic sort; keeps the first k
// by (distance, id).
__global__ __launch_bounds__(256) void k_leaf_exact(LeafArgs a) {
  __shared__ uint64_t keys[2048 + 64];
  __shared__ uint64_t best[64];
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
      ids_out += (size_t)wk.slot * a.n * a.k;
      dist_out += (size_t)wk.slot * a.n * a.k;
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
      ids_out[(size_t)qid * a.k + tid] = key_id(best[tid]);
      dist_out[(size_t)qid * a.k + tid] = key_dist(best[tid]);
    }
    __syncthreads();
  }
}

template <int KC, int KP, bool BF16>
hipError_t launch_leaf_t(const LeafArgs& a, hipStream_t s) {
  size_t shm = sizeof(LeafShared<KC, KP, BF16>);
  auto kern = k_leaf<KC, KP, BF16>;
  static int per_cu = 0;
  if (per_cu == 0) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    int occ = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)kern, LEAF_THREADS, shm);
    per_cu = (e == hipSuccess && occ > 0) ? occ : 1;
  }
  if (a.work) {
    hipError_t e = launch_fill_u32(a.counter, 0u, 1, s);
    if (e != hipSuccess) return e;
    unsigned grid = (unsigned)std::min<uint64_t>(a.n_work, (uint64_t)a.grid * per_cu);
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(LEAF_THREADS), shm, s, a);
  } else {
    hipLaunchKernelGGL(kern, dim3((unsigned)a.n_leaves), dim3(LEAF_THREADS), shm, s, a);
  }
  return hipGetLastError();
}

template <int KC, bool BF16>
hipError_t launch_leaf_kp(const LeafArgs& a, hipStream_t s) {
  if (a.kp <= 16) return launch_leaf_t<KC, 16, BF16>(a, s);
  if (a.kp <= 32) return launch_leaf_t<KC, 32, BF16>(a, s);
  return launch_leaf_t<KC, 64, BF16>(a, s);
}

}  // namespace

hipError_t launch_leaf(const LeafArgs& a, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32((uint32_t*)&a.diag->fallback_count, 0u, 2, s)) != hipSuccess) return e;
  if (a.precision == KNNG_BF16) {
    if (a.d <= 32) e = launch_leaf_kp<32, true>(a, s);
    else if (a.d <= 64) e = launch_leaf_kp<64, true>(a, s);
    else e = launch_leaf_kp<128, true>(a, s);
  } else {
    if (a.d <= 32) e = launch_leaf_kp<32, false>(a, s);
    else if (a.d <= 64) e = launch_leaf_kp<64, false>(a, s);
    else e = launch_leaf_kp<128, false>(a, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_leaf_exact, dim3(1024), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
