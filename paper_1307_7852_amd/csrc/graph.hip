// Combination of base graphs (Section 3.1) and neighbourhood propagation
// rounds (Section 3.2, first-order form of Theorem 1, with the pairwise
// updating of Section 3.4).  All kernels work one wave per point and keep
// candidate sets in registers, sorted with wave-wide bitonic networks; they
// are bound by the gathers of neighbour lists and candidate rows.
#include "knng_dev.h"

#include <algorithm>

namespace knng {

namespace {

// ---------------------------------------------------------------- merge
// Row p: the union of n_lists lists of k (distance, id) entries, duplicates
// dropped, first k by (distance, id).  The same pair always carries the same
// FP32 distance (one canonical distance routine), so duplicates sort next to
// each other.
template <int R>
__global__ __launch_bounds__(256) void k_merge(int64_t n, int k, int n_lists, const uint32_t* __restrict__ ids_in,
                                                const float* __restrict__ dist_in, uint32_t* __restrict__ ids_out,
                                                float* __restrict__ dist_out, int64_t ls, int64_t rs,
                                                const uint32_t* __restrict__ n_used) {
  __shared__ uint64_t sk[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 4 + w;
  if (p >= n) return;
  if (n_used) n_lists = min(n_lists, (int)*n_used);   // lists of divisions that ran
  const int tot = n_lists * k;
  uint64_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int e = r * 64 + lane;
    uint64_t key = ~0ull;
    if (e < tot) {
      int li = e / k, j = e % k;
      size_t idx = (size_t)li * ls + (size_t)p * rs + j;
      key = pack_did(dist_in[idx], ids_in[idx]);
    }
    v[r] = key;
  }
  if constexpr (R > 1) {
    // The first list's largest key bounds the union's k-th: only keys below
    // it (besides that list) can enter.  When those fit one register beside
    // the first list (the usual case), one 64-wide sort replaces the wider one.
    uint64_t mx = lane < k ? v[0] : 0ull;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t lo = __shfl_xor((uint32_t)mx, o), hi = __shfl_xor((uint32_t)(mx >> 32), o);
      const uint64_t x = ((uint64_t)hi << 32) | lo;
      mx = x > mx ? x : mx;
    }
    int S = 0;
    sk[w][lane] = ~0ull;
    wave_sync();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = r * 64 + lane;
      const bool in = e >= k && v[r] < mx;
      int cnt;
      const int slot = k + S + wave_prefix_count(in, lane, &cnt);
      if (in && slot < 64) sk[w][slot] = v[r];
      S += cnt;
    }
    wave_sync();
    if (k + S <= 64) {   // uniform
      uint64_t u[1];
      u[0] = lane < k ? v[0] : sk[w][lane];
      wave_bitonic<1, 64, uint64_t>(u, lane);
      const uint64_t pv = prev_elem<1>(u, 0, lane, ~0ull);
      const bool uniq = u[0] != ~0ull && key_id(pv) != key_id(u[0]);
      int cnt;
      const int slot = wave_prefix_count(uniq, lane, &cnt);
      if (uniq && slot < k) {
        ids_out[(size_t)p * k + slot] = key_id(u[0]);
        dist_out[(size_t)p * k + slot] = key_dist(u[0]);
      }
      for (int s2 = cnt + lane; s2 < k; s2 += 64) {
        ids_out[(size_t)p * k + s2] = KNNG_NONE;
        dist_out[(size_t)p * k + s2] = __int_as_float(0x7F800000);
      }
      return;
    }
  }
  wave_bitonic<R, 64 * R, uint64_t>(v, lane);
  int base = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    uint64_t pv = prev_elem<R>(v, r, lane, ~0ull);
    bool uniq = v[r] != ~0ull && key_id(pv) != key_id(v[r]);
    int cnt;
    int slot = base + wave_prefix_count(uniq, lane, &cnt);
    if (uniq && slot < k) {
      ids_out[(size_t)p * k + slot] = key_id(v[r]);
      dist_out[(size_t)p * k + slot] = key_dist(v[r]);
    }
    base += cnt;
  }
  // pad
  for (int s = base + lane; s < k; s += 64) {
    ids_out[(size_t)p * k + s] = KNNG_NONE;
    dist_out[(size_t)p * k + s] = __int_as_float(0x7F800000);
  }
}

// Thread-per-point merge for the configured list lengths (k = 10, 20): the
// thread keeps p's k best keys sorted in registers, starting from its first
// list (sorted and duplicate-free), and walks every other list in order
// until an entry no longer beats its current k-th (the rest of that list
// cannot either).  An entry equal to a kept key is the same (distance, id)
// pair found by another division and is skipped.  The first PF entries of
// up to G lists are loaded together (8-byte pieces: k is even), so a thread
// waits for memory once per group instead of once per entry; the rest of a
// list is read only when its PF-th entry still entered.
template <int K>
__global__ __launch_bounds__(256) void k_merge_pt(int64_t n, int n_lists, const uint32_t* __restrict__ ids_in,
                                                  const float* __restrict__ dist_in, uint32_t* __restrict__ ids_out,
                                                  float* __restrict__ dist_out, int64_t ls, int64_t rs,
                                                  const uint32_t* __restrict__ n_used) {
  static_assert(K % 2 == 0, "pairs of entries are loaded together");
  constexpr int PF = 4, G = 8;
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  if (n_used) n_lists = min(n_lists, (int)*n_used);
  const uint32_t* ib = ids_in + (size_t)p * rs;
  const float* db = dist_in + (size_t)p * rs;
  uint64_t L[K];
  {
    uint2 iv[K / 2];
    float2 dv[K / 2];
#pragma unroll
    for (int j = 0; j < K / 2; ++j) {
      iv[j] = ((const uint2*)ib)[j];
      dv[j] = ((const float2*)db)[j];
    }
#pragma unroll
    for (int j = 0; j < K / 2; ++j) {
      L[2 * j] = pack_did(dv[j].x, iv[j].x);
      L[2 * j + 1] = pack_did(dv[j].y, iv[j].y);
    }
  }
  auto insert = [&](uint64_t x) -> bool {   // false: x cannot enter (nor can anything after it)
    if (x >= L[K - 1]) return false;
    bool dup = false;
#pragma unroll
    for (int i = 0; i < K; ++i) dup = dup || x == L[i];
    if (!dup) {
#pragma unroll
      for (int i = K - 1; i > 0; --i) L[i] = x < L[i - 1] ? L[i - 1] : (x < L[i] ? x : L[i]);
      L[0] = x < L[0] ? x : L[0];
    }
    return true;
  };
  for (int t0 = 1; t0 < n_lists; t0 += G) {
    uint2 iv[G][PF / 2];
    float2 dv[G][PF / 2];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int t = t0 + g < n_lists ? t0 + g : 0;   // past the last list: re-read list 0 (ignored)
#pragma unroll
      for (int j = 0; j < PF / 2; ++j) {
        iv[g][j] = ((const uint2*)(ib + (size_t)t * ls))[j];
        dv[g][j] = ((const float2*)(db + (size_t)t * ls))[j];
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (t0 + g >= n_lists) break;
      bool more = true;
#pragma unroll
      for (int j = 0; j < PF / 2 && more; ++j) {
        more = insert(pack_did(dv[g][j].x, iv[g][j].x));
        if (more) more = insert(pack_did(dv[g][j].y, iv[g][j].y));
      }
      if (more) {   // the list's first PF entries all entered: read on
        const uint32_t* it = ib + (size_t)(t0 + g) * ls;
        const float* dt = db + (size_t)(t0 + g) * ls;
        for (int j = PF; j < K; ++j)
          if (!insert(pack_did(dt[j], it[j]))) break;
      }
    }
  }
  uint32_t* io = ids_out + (size_t)p * K;
  float* dout = dist_out + (size_t)p * K;
#pragma unroll
  for (int j = 0; j < K / 2; ++j) {
    ((uint2*)io)[j] = make_uint2(key_id(L[2 * j]), key_id(L[2 * j + 1]));
    ((float2*)dout)[j] = make_float2(key_dist(L[2 * j]), key_dist(L[2 * j + 1]));
  }
}

// ---------------------------------------------------------------- propagation, forward part
// Blocks are dealt to the 8 XCDs round-robin; remapping block b to a
// contiguous range per XCD keeps the points one XCD works on (and so the
// candidate rows its L2 holds) neighbours in the visiting order.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
  uint32_t q = nb / 8, r = nb % 8, x = b % 8, j = b / 8;
  return x * q + (x < r ? x : r) + j;
}

// Wave per point p:
//   1. C_p = ids of N(q) for q in N(p), duplicates, p and N(p) dropped (LDS hash);
//   2. score every candidate with the canonical distance (16 lanes each);
//   3. first k by (distance, id) of N(p) and C_p -> forward list;
//   4. pairwise: propose p to every scored o when (D, p) beats o's frozen
//      k-th entry (anything else could never enter o's list).
template <int R1, int R2, int NCH>
__global__ __launch_bounds__(256) void k_prop_forward(PropArgs a) {
  __shared__ uint32_t cand_s[4][64 * R1];
  __shared__ float cd_s[4][64 * R1];
  __shared__ __align__(16) uint32_t htab[4][128 * R1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t vis = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * 4 + w;
  if (vis >= a.n) return;
  const int64_t p = a.order ? (int64_t)a.order[vis] : vis;   // points in spatial order
  const int k = a.k, d = a.d;
  uint32_t nb = lane < k ? a.ids_in[(size_t)p * k + lane] : KNNG_NONE;
  float nbd = lane < k ? a.dist_in[(size_t)p * k + lane] : __int_as_float(0x7F800000);
  // 1. C_p: the ids of N(q) for q in N(p), deduplicated through a per-wave
  //    open-addressing table in LDS that first receives p and N(p), so those
  //    are dropped too.  The candidates come out in table-race order; every
  //    later step depends only on the set (keys are (distance, id)).
  constexpr int TBL = 128 * R1;   // >= 2 (k^2) > k^2 + k + 1 entries
  constexpr int LOG2_TBL = 7 + (R1 >= 2) + (R1 >= 4) + (R1 >= 8) + (R1 >= 16);
  static_assert((1 << LOG2_TBL) == TBL, "table size");
  uint32_t* ht = htab[w];
  for (int i = lane; i < TBL; i += 64) ht[i] = KNNG_NONE;
  wave_sync();
  auto insert = [&](uint32_t id) -> bool {   // true: id was not in the table yet
    uint32_t h = (id * 0x9E3779B1u) >> (32 - LOG2_TBL);
    for (;;) {   // ends: the table always has empty slots
      const uint32_t old = atomicCAS(&ht[h], KNNG_NONE, id);
      if (old == KNNG_NONE) return true;
      if (old == id) return false;
      h = (h + 1) & (TBL - 1);
    }
  };
  if (lane < k && nb != KNNG_NONE) insert(nb);
  if (lane == 63) insert((uint32_t)p);
  wave_sync();
  int U = 0;
#pragma unroll
  for (int r = 0; r < R1; ++r) {
    const int e = r * 64 + lane;
    uint32_t o = KNNG_NONE;
    const int qi = e / k;
    const uint32_t q = __shfl(nb, qi < 64 ? qi : 0);
    if (e < k * k && q != KNNG_NONE) o = a.ids_in[(size_t)q * k + (e % k)];
    const bool u = o != KNNG_NONE && insert(o);
    int cnt;
    const int slot = U + wave_prefix_count(u, lane, &cnt);
    if (u) cand_s[w][slot] = o;
    U += cnt;
  }
  wave_sync();
  // 2. score: lane group g takes candidates g, g+4, ...; p's row in registers
  //    (NCH float4 chunks per lane; NCH == 0 reads it from memory each time)
  const int g = lane >> 4, gl = lane & 15;
  const float* xp = a.X + (size_t)p * d;
  // Byte rows (every value of X an integer in 0..255, d <= 256 and a
  // multiple of 8): the squared distance is an integer below 2^24, formed in
  // integers as |x|^2 + |y|^2 - 2 x.y with four-byte dot products, so it is
  // exactly dist2_g16's value.  A lane holds 8 consecutive bytes of p (block
  // gl, and gl + 16 when d > 128) and reads one 8-byte piece of each
  // candidate row: eight rows per lane group are in flight.
  // NB 8-value blocks per lane: one up to d = 128 (NCH <= 2), two up to 256
  constexpr int NB = NCH >= 3 ? 2 : 1;
  const bool u8 = NCH >= 1 && NCH <= 4 && a.X8 && (a.diag->exact_flags & EXACT_U8) != 0u && (d & 7) == 0 &&
                  d <= 128 * NB;   // uniform
  if (u8) {
    constexpr int R8 = 8;
    const int nb = d >> 3;
    uint2 xw[NB];
    uint32_t x2[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int blk = gl + 16 * b;
      xw[b] = blk < nb ? *(const uint2*)(a.X8 + (size_t)p * d + 8 * blk) : make_uint2(0u, 0u);
      x2[b] = __builtin_amdgcn_udot4(xw[b].x, xw[b].x, __builtin_amdgcn_udot4(xw[b].y, xw[b].y, 0u, false), false);
    }
    for (int base = 0; base < U; base += 4 * R8) {
      // every lane loads (lanes past the row read block 0 and drop the sum
      // afterwards), so no branch sits between the loads and their use
      uint2 wr[R8][NB];
#pragma unroll
      for (int j = 0; j < R8; ++j) {
        const int ci = base + g + 4 * j;
        const uint32_t o = ci < U ? cand_s[w][ci] : (uint32_t)p;
        const uint8_t* yr = a.X8 + (size_t)o * d;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int blk = gl + 16 * b;
          wr[j][b] = *(const uint2*)(yr + 8 * (blk < nb ? blk : 0));
        }
      }
#pragma unroll
      for (int j = 0; j < R8; ++j) {
        uint32_t acc = 0u;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const uint2 y = wr[j][b];
          const uint32_t yy = __builtin_amdgcn_udot4(y.x, y.x, __builtin_amdgcn_udot4(y.y, y.y, 0u, false), false);
          const uint32_t xy = __builtin_amdgcn_udot4(xw[b].x, y.x, __builtin_amdgcn_udot4(xw[b].y, y.y, 0u, false), false);
          // the block's sum of (x - y)^2: nonnegative, so the unsigned
          // arithmetic wraps back to it
          const uint32_t part = x2[b] + yy - 2u * xy;
          acc += gl + 16 * b < nb ? part : 0u;
        }
        acc += __shfl_xor(acc, 8, 16);
        acc += __shfl_xor(acc, 4, 16);
        acc += __shfl_xor(acc, 2, 16);
        acc += __shfl_xor(acc, 1, 16);
        const int ci = base + g + 4 * j;
        if (gl == 0 && ci < U) cd_s[w][ci] = (float)acc;
      }
    }
  } else if constexpr (NCH > 0) {
    float4 xr[NCH];
#pragma unroll
    for (int i = 0; i < NCH; ++i) {
      int cc = gl + 16 * i;
      xr[i] = (cc < (d >> 2)) ? ((const float4*)xp)[cc] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // four candidates per lane group in flight: base + g + 4j
    for (int base = 0; base < U; base += 16) {
      const float* yr[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int ci = base + g + 4 * j;
        const uint32_t o = ci < U ? cand_s[w][ci] : (uint32_t)p;
        yr[j] = a.X + (size_t)o * d;
      }
      float dd[4];
      dist2_g16_reg4<NCH>(xr, yr, d, gl, dd);
      if (gl == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (base + g + 4 * j < U) cd_s[w][base + g + 4 * j] = dd[j];
      }
    }
  } else {
    for (int base = 0; base < U; base += 4) {
      int ci = base + g;
      uint32_t o = ci < U ? cand_s[w][ci] : (uint32_t)p;
      float dd = dist2_g16(xp, a.X + (size_t)o * d, d, gl);
      if (gl == 0 && ci < U) cd_s[w][ci] = dd;
    }
  }
  wave_sync();
  if (lane == 0) atomicAdd(&a.diag->prop_candidates[blockIdx.x & (DIAG_SLOTS - 1)], (unsigned long long)U);
  // 3. first k of N(p) and C_p.  N(p) is sorted and C_p holds none of its
  //    ids, so only the candidates keyed below N(p)'s k-th can enter (W of
  //    them, few once the graph is good): none leaves N(p) as it is; up to
  //    8 are inserted one by one; up to 64 - k are sorted with N(p) in one
  //    register; more, and all k + U keys are sorted.
  const uint64_t nbkey = lane < k ? pack_did(nbd, nb) : ~0ull;
  const uint64_t kth_p = shfl_u64(nbkey, k - 1);
  uint64_t* wkeys = reinterpret_cast<uint64_t*>(htab[w]);   // the table's room: free after step 1
  int W = 0;
  for (int base = 0; base < U; base += 64) {
    const int ci = base + lane;
    const uint64_t key = ci < U ? pack_did(cd_s[w][ci], cand_s[w][ci]) : ~0ull;
    const bool win = key < kth_p;
    int cnt;
    const int slot = W + wave_prefix_count(win, lane, &cnt);
    if (win && slot < 64 - k) wkeys[slot] = key;
    W += cnt;
  }
  uint64_t v[R2];
  if (k + W <= 64) {
    wave_sync();
    if (W <= 8) {
      v[0] = nbkey;
      for (int i = 0; i < W; ++i) {   // the largest entry falls off
        const uint64_t x = wkeys[i];
        const uint64_t prev = shfl_up_u64(v[0], 1);
        if (x < v[0]) v[0] = (lane == 0 || x > prev) ? x : prev;
      }
    } else {
      uint64_t v1[1] = {lane < k ? nbkey : lane < k + W ? wkeys[lane - k] : ~0ull};
      wave_bitonic<1, 64, uint64_t>(v1, lane);
      v[0] = v1[0];
    }
  } else {
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      int e = r * 64 + lane;
      uint64_t key = ~0ull;
      if (e < k) key = nbkey;                       // e == lane here
      else if (e - k < U) key = pack_did(cd_s[w][e - k], cand_s[w][e - k]);
      v[r] = key;
    }
    wave_bitonic<R2, 64 * R2, uint64_t>(v, lane);
  }
  uint32_t* oi = a.pairwise ? a.fwd_ids : a.ids_out;
  float* od = a.pairwise ? a.fwd_dist : a.dist_out;
  if (lane < k) {
    oi[(size_t)p * k + lane] = key_id(v[0]);
    od[(size_t)p * k + lane] = key_dist(v[0]);
  }
  if (!a.pairwise) return;
  // 4. reverse proposals into p's own slots
  uint32_t* slots = a.prop_buf + (size_t)p * a.slot_cap * 2;
  int np = 0;
  for (int base = 0; base < U; base += 64) {
    int ci = base + lane;
    bool ok = false;
    uint32_t o = 0;
    float dd = 0.f;
    if (ci < U) {
      o = cand_s[w][ci];
      dd = cd_s[w][ci];
      ok = pack_did(dd, (uint32_t)p) < a.kth[o];
    }
    int tot;
    int pre = np + wave_prefix_count(ok, lane, &tot);
    if (ok) {
      slots[2 * pre] = o;
      slots[2 * pre + 1] = __float_as_uint(dd);
      atomicAdd(&a.cnt[o], 1u);
    }
    np += tot;
  }
  if (lane == 0) {
    a.prop_n[p] = (uint32_t)np;
    atomicAdd(&a.diag->prop_proposals[blockIdx.x & (DIAG_SLOTS - 1)], (unsigned long long)np);
  }
}

// Every point's frozen k-th key, packed: the proposal test reads this
// dense n x 8-byte array instead of two scattered words of the lists.
__global__ __launch_bounds__(256) void k_prop_kth(PropArgs a) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= a.n) return;
  const size_t e = (size_t)p * a.k + a.k - 1;
  a.kth[p] = pack_did(a.dist_in[e], a.ids_in[e]);
}

// ---------------------------------------------------------------- scan (exclusive, n+1 entries)
__global__ __launch_bounds__(1024) void k_scan_blocks(const uint32_t* in, uint32_t* out, uint32_t* bsum, int64_t cnt) {
  __shared__ uint32_t ws[16];
  int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  uint32_t v = i < cnt ? in[i] : 0u;
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t x = v;
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) ws[w] = x;
  __syncthreads();
  uint32_t base = 0;
  for (int j = 0; j < w; ++j) base += ws[j];
  if (i < cnt) out[i] = base + x - v;
  if (threadIdx.x == 1023) bsum[blockIdx.x] = base + x;
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t* bsum, int nb) {
  // single block: exclusive scan of nb block sums in place (nb <= 1024 * 16)
  __shared__ uint32_t part[1024];
  int per = (nb + 1023) / 1024;
  int b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += bsum[b0 + i];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    uint32_t y = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - s;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      uint32_t t = bsum[b0 + i];
      bsum[b0 + i] = run;
      run += t;
    }
}

__global__ void k_scan_add(uint32_t* out, const uint32_t* bsum, int64_t cnt) {
  int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  if (i < cnt) out[i] += bsum[blockIdx.x];
}

// Proposals into per-destination buckets; leaves cnt[] at zero again.
__global__ __launch_bounds__(256) void k_prop_scatter(PropArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= a.n) return;
  const uint32_t np = a.prop_n[p];
  const uint32_t* slots = a.prop_buf + (size_t)p * a.slot_cap * 2;
  for (uint32_t j = lane; j < np; j += 64) {
    uint32_t dst = slots[2 * j];
    uint32_t pos = a.offs[dst] + atomicSub(&a.cnt[dst], 1u) - 1u;
    a.bucket[2 * pos] = (uint32_t)p;
    a.bucket[2 * pos + 1] = slots[2 * j + 1];
  }
}

// Row p: first k by (distance, id) of its forward list and its bucket.
template <int R>
__global__ __launch_bounds__(256) void k_prop_final(PropArgs a) {
  __shared__ uint64_t kept[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * 4 + w;
  if (p >= a.n) return;
  const int k = a.k;
  const uint32_t b0 = a.offs[p], b1 = a.offs[p + 1];
  if (b0 == b1) {   // no proposals for p: its forward list is final
    if (lane < k) {
      a.ids_out[(size_t)p * k + lane] = a.fwd_ids[(size_t)p * k + lane];
      a.dist_out[(size_t)p * k + lane] = a.fwd_dist[(size_t)p * k + lane];
    }
    return;
  }
  uint64_t keep = lane < k ? pack_did(a.fwd_dist[(size_t)p * k + lane], a.fwd_ids[(size_t)p * k + lane]) : ~0ull;
  // Only proposals below the forward list's k-th key can enter.  When those
  // fit one register beside the list (the usual case), one 64-wide sort
  // gives the answer.
  if (b1 - b0 <= 64) {   // uniform
    const uint32_t klo = __shfl((uint32_t)keep, k - 1), khi = __shfl((uint32_t)(keep >> 32), k - 1);
    const uint64_t kth = ((uint64_t)khi << 32) | klo;
    const uint32_t j = b0 + (uint32_t)lane;
    const uint64_t key = j < b1 ? pack_did(__uint_as_float(a.bucket[2 * j + 1]), a.bucket[2 * j]) : ~0ull;
    const bool in = key < kth;
    int S;
    const int slot = k + wave_prefix_count(in, lane, &S);
    if (k + S <= 64) {   // uniform
      kept[w][lane] = ~0ull;
      wave_sync();
      if (in) kept[w][slot] = key;
      wave_sync();
      uint64_t v[1];
      v[0] = lane < k ? keep : kept[w][lane];
      wave_bitonic<1, 64, uint64_t>(v, lane);
      const uint64_t pv = prev_elem<1>(v, 0, lane, ~0ull);
      const bool uniq = v[0] != ~0ull && key_id(pv) != key_id(v[0]);
      int cnt;
      const int out = wave_prefix_count(uniq, lane, &cnt);
      wave_sync();
      kept[w][lane] = ~0ull;
      wave_sync();
      if (uniq && out < k) kept[w][out] = v[0];
      wave_sync();
      if (lane < k) {
        const uint64_t r = kept[w][lane];
        a.ids_out[(size_t)p * k + lane] = key_id(r);
        a.dist_out[(size_t)p * k + lane] = key_dist(r);
      }
      return;
    }
  }
  const uint32_t chunk = 64 * (R - 1);   // register 0 carries the kept list
  uint32_t pos = b0;
  do {
    uint64_t v[R];
    v[0] = keep;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      uint32_t j = pos + (uint32_t)((r - 1) * 64 + lane);
      v[r] = j < b1 ? pack_did(__uint_as_float(a.bucket[2 * j + 1]), a.bucket[2 * j]) : ~0ull;
    }
    pos += chunk;
    wave_bitonic<R, 64 * R, uint64_t>(v, lane);
    // drop adjacent duplicates (same id carries the same distance) and keep the first k
    kept[w][lane] = ~0ull;
    wave_sync();
    int base = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint64_t pv = prev_elem<R>(v, r, lane, ~0ull);
      bool uniq = v[r] != ~0ull && key_id(pv) != key_id(v[r]);
      int cnt;
      int slot = base + wave_prefix_count(uniq, lane, &cnt);
      if (uniq && slot < k) kept[w][slot] = v[r];
      base += cnt;
    }
    wave_sync();
    keep = kept[w][lane];
    wave_sync();
  } while (pos < b1);
  if (lane < k) {
    a.ids_out[(size_t)p * k + lane] = key_id(keep);
    a.dist_out[(size_t)p * k + lane] = key_dist(keep);
  }
}

// ---------------------------------------------------------------- propagation, queue form
// One wave per point p with a queue of (distance to p, id) keys and an
// open-addressing table of the ids seen so far (p, N(p) and every evaluated
// point), both in LDS.  Best-first pass (Section 3.2): the queue starts with
// N(p); the smallest unpopped key is popped (a popped key keeps its slot with
// bit 63 set) and its neighbours not seen yet are evaluated in list order
// and queued, until visit_max points have been evaluated or nothing is left
// to pop.  FIRST: the first-order round of Theorem 1 for k > 31 (only the
// entries of N(p) are popped and nothing limits the evaluations: the
// candidates are N(N(p)) minus p and N(p), as in k_prop_forward).  Then p
// keeps the first k by (distance, id) of N(p) and the evaluated points, and
// with pairwise updating proposes itself to every evaluated point whose
// frozen k-th entry it beats.
template <int NCH, bool FIRST>
__global__ __launch_bounds__(256) void k_prop_queue(PropArgs a, int qcap, int log2_tbl, int wave_bytes) {
  extern __shared__ __align__(16) unsigned char qsm[];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wpb = blockDim.x >> 6;
  const int64_t vis = (int64_t)xcd_contiguous(blockIdx.x, gridDim.x) * wpb + w;
  if (vis >= a.n) return;   // whole waves; no workgroup barrier below
  uint64_t* Q = (uint64_t*)(qsm + (size_t)w * wave_bytes);
  uint32_t* ht = (uint32_t*)(Q + qcap);
  const int tbl = 1 << log2_tbl;
  const int64_t p = a.order ? (int64_t)a.order[vis] : vis;
  const int k = a.k, d = a.d;
  constexpr uint64_t POPPED = 1ull << 63;
  for (int i = lane; i < tbl; i += 64) ht[i] = KNNG_NONE;
  wave_sync();
  auto slot0 = [&](uint32_t id) { return (id * 0x9E3779B1u) >> (32 - log2_tbl); };
  auto seen = [&](uint32_t id) -> bool {   // ends: the table always has empty slots
    for (uint32_t h = slot0(id);; h = (h + 1) & (tbl - 1)) {
      const uint32_t x = ht[h];
      if (x == id) return true;
      if (x == KNNG_NONE) return false;
    }
  };
  auto insert = [&](uint32_t id) {
    for (uint32_t h = slot0(id);; h = (h + 1) & (tbl - 1)) {
      const uint32_t old = atomicCAS(&ht[h], KNNG_NONE, id);
      if (old == KNNG_NONE || old == id) return;
    }
  };
  const uint32_t nb = lane < k ? a.ids_in[(size_t)p * k + lane] : KNNG_NONE;
  const float nbd = lane < k ? a.dist_in[(size_t)p * k + lane] : __int_as_float(0x7F800000);
  const bool valid = nb != KNNG_NONE;
  if (valid) insert(nb);
  wave_sync();
  if (lane == 0) insert((uint32_t)p);
  int nvalid;
  const int vslot = wave_prefix_count(valid, lane, &nvalid);
  if (valid) Q[vslot] = pack_did(nbd, nb);
  wave_sync();

  // p's row for the scoring: byte rows (see k_prop_forward) or float4 chunks
  const int g = lane >> 4, gl = lane & 15;
  constexpr int NB = NCH >= 3 ? 2 : 1;
  const bool u8 = NCH >= 1 && NCH <= 4 && a.X8 && (a.diag->exact_flags & EXACT_U8) != 0u && (d & 7) == 0 &&
                  d <= 128 * NB;   // uniform
  const int nblk = d >> 3;
  uint2 xw[NB];
  uint32_t x2[NB];
  float4 xr[NCH > 0 ? NCH : 1];
  if (u8) {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int blk = gl + 16 * b;
      xw[b] = blk < nblk ? *(const uint2*)(a.X8 + (size_t)p * d + 8 * blk) : make_uint2(0u, 0u);
      x2[b] = __builtin_amdgcn_udot4(xw[b].x, xw[b].x, __builtin_amdgcn_udot4(xw[b].y, xw[b].y, 0u, false), false);
    }
  } else if constexpr (NCH > 0) {
#pragma unroll
    for (int i = 0; i < NCH; ++i) {
      const int cc = gl + 16 * i;
      xr[i] = (cc < (d >> 2)) ? ((const float4*)(a.X + (size_t)p * d))[cc] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  // scores the cnt candidates whose ids sit in Q[b0 .. b0 + cnt) and stores
  // their (distance, id) keys there
  auto score = [&](int b0, int cnt) {
    if (u8) {
      constexpr int R8 = 8;
      for (int base = 0; base < cnt; base += 4 * R8) {
        uint2 wr[R8][NB];
#pragma unroll
        for (int j = 0; j < R8; ++j) {
          const int ci = base + g + 4 * j;
          const uint32_t o = ci < cnt ? (uint32_t)Q[b0 + ci] : (uint32_t)p;
          const uint8_t* yr = a.X8 + (size_t)o * d;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const int blk = gl + 16 * b;
            wr[j][b] = *(const uint2*)(yr + 8 * (blk < nblk ? blk : 0));
          }
        }
#pragma unroll
        for (int j = 0; j < R8; ++j) {
          uint32_t acc = 0u;   // |x|^2 + |y|^2 - 2 x.y per block, as in k_prop_forward
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const uint2 y = wr[j][b];
            const uint32_t yy = __builtin_amdgcn_udot4(y.x, y.x, __builtin_amdgcn_udot4(y.y, y.y, 0u, false), false);
            const uint32_t xy = __builtin_amdgcn_udot4(xw[b].x, y.x, __builtin_amdgcn_udot4(xw[b].y, y.y, 0u, false), false);
            const uint32_t part = x2[b] + yy - 2u * xy;
            acc += gl + 16 * b < nblk ? part : 0u;
          }
          acc += __shfl_xor(acc, 8, 16);
          acc += __shfl_xor(acc, 4, 16);
          acc += __shfl_xor(acc, 2, 16);
          acc += __shfl_xor(acc, 1, 16);
          const int ci = base + g + 4 * j;
          if (gl == 0 && ci < cnt) Q[b0 + ci] = pack_did((float)acc, (uint32_t)Q[b0 + ci]);
        }
      }
    } else if constexpr (NCH > 0) {
      for (int base = 0; base < cnt; base += 16) {
        const float* yr[4];
        uint32_t oid[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int ci = base + g + 4 * j;
          oid[j] = ci < cnt ? (uint32_t)Q[b0 + ci] : (uint32_t)p;
          yr[j] = a.X + (size_t)oid[j] * d;
        }
        float dd[4];
        dist2_g16_reg4<NCH>(xr, yr, d, gl, dd);
        if (gl == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (base + g + 4 * j < cnt) Q[b0 + base + g + 4 * j] = pack_did(dd[j], oid[j]);
        }
      }
    } else {
      const float* xp = a.X + (size_t)p * d;
      for (int base = 0; base < cnt; base += 4) {
        const int ci = base + g;
        const uint32_t o = ci < cnt ? (uint32_t)Q[b0 + ci] : (uint32_t)p;
        const float dd = dist2_g16(xp, a.X + (size_t)o * d, d, gl);
        if (gl == 0 && ci < cnt) Q[b0 + ci] = pack_did(dd, o);
      }
    }
    wave_sync();
  };

  int qlen = nvalid;
  int budget = FIRST ? k * k : a.visit_max;
  while (budget > 0) {
    const int lim = FIRST ? nvalid : qlen;   // FIRST pops only the entries of N(p)
    uint64_t mn = ~0ull;
    for (int i = lane; i < lim; i += 64) {
      const uint64_t x = Q[i];
      mn = x < mn ? x : mn;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint64_t y = shfl_xor_u64(mn, o);
      mn = y < mn ? y : mn;
    }
    if (mn & POPPED) break;   // uniform: every key popped (or none queued)
    for (int i = lane; i < lim; i += 64)
      if (Q[i] == mn) Q[i] = mn | POPPED;   // keys are unique: one owner
    const uint32_t q = key_id(mn);
    const uint32_t o = lane < k ? a.ids_in[(size_t)q * k + lane] : KNNG_NONE;
    const bool fresh = o != KNNG_NONE && !seen(o);
    int cnt;
    const int rank = wave_prefix_count(fresh, lane, &cnt);
    const int ntake = cnt < budget ? cnt : budget;
    wave_sync();
    if (fresh && rank < budget) {   // the first `budget` new ones in q's list order
      insert(o);
      Q[qlen + rank] = (uint64_t)o;
    }
    wave_sync();
    score(qlen, ntake);
    qlen += ntake;
    budget -= ntake;
  }
  const int V = qlen - nvalid;
  if (lane == 0) atomicAdd(&a.diag->prop_candidates[blockIdx.x & (DIAG_SLOTS - 1)], (unsigned long long)V);
  // p keeps the first k of N(p) and the evaluated points; only keys below the
  // current k-th can enter
  uint64_t keep = lane < k ? pack_did(nbd, nb) : ~0ull;
  uint64_t kth = shfl_u64(keep, k - 1);
  for (int base = nvalid; base < qlen; base += 64) {
    const int i = base + lane;
    const uint64_t x = i < qlen ? (Q[i] & ~POPPED) : ~0ull;
    const bool in = x < kth;
    if (!__any(in)) continue;   // uniform
    uint64_t v[2] = {keep, in ? x : ~0ull};
    wave_bitonic<2, 128, uint64_t>(v, lane);
    keep = lane < k ? v[0] : ~0ull;
    kth = shfl_u64(keep, k - 1);
  }
  uint32_t* oi = a.pairwise ? a.fwd_ids : a.ids_out;
  float* od = a.pairwise ? a.fwd_dist : a.dist_out;
  if (lane < k) {
    oi[(size_t)p * k + lane] = key_id(keep);
    od[(size_t)p * k + lane] = key_dist(keep);
  }
  if (!a.pairwise) return;
  uint32_t* slots = a.prop_buf + (size_t)p * a.slot_cap * 2;
  int np = 0;
  for (int base = nvalid; base < qlen; base += 64) {
    const int i = base + lane;
    bool ok = false;
    uint32_t o = 0;
    float dd = 0.f;
    if (i < qlen) {
      const uint64_t x = Q[i] & ~POPPED;
      o = key_id(x);
      dd = key_dist(x);
      ok = pack_did(dd, (uint32_t)p) < a.kth[o];
    }
    int tot;
    const int pre = np + wave_prefix_count(ok, lane, &tot);
    if (ok) {
      slots[2 * pre] = o;
      slots[2 * pre + 1] = __float_as_uint(dd);
      atomicAdd(&a.cnt[o], 1u);
    }
    np += tot;
  }
  if (lane == 0) {
    a.prop_n[p] = (uint32_t)np;
    atomicAdd(&a.diag->prop_proposals[blockIdx.x & (DIAG_SLOTS - 1)], (unsigned long long)np);
  }
}

// ---------------------------------------------------------------- effective rate
// Thread per point: the ids of p's list m that none of its lists 0..m-1
// holds, summed over the workgroup and added to diag->rate_new[m].
template <int KM>
__global__ __launch_bounds__(256) void k_rate_count(int64_t n, int k, int m, const uint32_t* __restrict__ lists,
                                                    int64_t ls, int64_t rs, DiagDev* diag) {
  __shared__ unsigned long long part[4];
  if (diag->stop) return;   // uniform: the rule has already fired
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  unsigned long long nw = 0;
  if (p < n) {
    uint32_t cur[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) cur[j] = j < k ? lists[(size_t)m * ls + (size_t)p * rs + j] : KNNG_NONE;
    uint64_t found = 0;
    for (int t = 0; t < m; ++t)
      for (int jj = 0; jj < k; ++jj) {
        const uint32_t x = lists[(size_t)t * ls + (size_t)p * rs + jj];
        if (x == KNNG_NONE) continue;
#pragma unroll
        for (int j = 0; j < KM; ++j)
          if (cur[j] == x) found |= 1ull << j;
      }
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (cur[j] != KNNG_NONE && !((found >> j) & 1ull)) ++nw;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nw += shfl_xor_u64(nw, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = nw;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long s = part[0] + part[1] + part[2] + part[3];
    if (s) atomicAdd(&diag->rate_new[m], s);
  }
}

// r_m = new_m / total_m with total_m = total_{m-1} + new_m; the divisions
// stop once 1000 new_m < rate_permille total_m (integer arithmetic).
__global__ void k_rate_decide(DiagDev* diag, int m, int rate_permille) {
  if (threadIdx.x != 0 || diag->stop) return;
  const unsigned long long nw = diag->rate_new[m];
  const unsigned long long tot = (m > 0 ? diag->rate_total[m - 1] : 0ull) + nw;
  diag->rate_total[m] = tot;
  diag->div_used = (unsigned)(m + 1);
  if (1000ull * nw < (unsigned long long)rate_permille * tot) diag->stop = 1u;
}

template <int NCH, bool FIRST>
hipError_t launch_queue_n(const PropArgs& a, hipStream_t s) {
  const int budget0 = FIRST ? a.k * a.k : a.visit_max;
  const int qcap = a.k + budget0;
  const int ent = a.k + 1 + budget0;
  int log2_tbl = 6;
  while ((1 << log2_tbl) < ent + ent / 2) ++log2_tbl;
  const int wave_bytes = (qcap * 8 + (4 << log2_tbl) + 15) & ~15;
  const int wpb = std::max(1, std::min(4, (160 * 1024) / wave_bytes));
  const size_t shm = (size_t)wpb * wave_bytes;
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  auto kern = k_prop_queue<NCH, FIRST>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const unsigned blocks = (unsigned)((a.n + wpb - 1) / wpb);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * wpb), shm, s, a, qcap, log2_tbl, wave_bytes);
  return hipGetLastError();
}

template <bool FIRST>
hipError_t launch_queue(const PropArgs& a, hipStream_t s) {
  const int nc = a.d / 4;
  if (nc <= 16) return launch_queue_n<1, FIRST>(a, s);
  if (nc <= 32) return launch_queue_n<2, FIRST>(a, s);
  if (nc <= 64) return launch_queue_n<4, FIRST>(a, s);
  if (nc <= 128) return launch_queue_n<8, FIRST>(a, s);
  if (nc <= 256) return launch_queue_n<16, FIRST>(a, s);
  return launch_queue_n<0, FIRST>(a, s);
}

template <int R>
hipError_t launch_merge_r(int64_t n, int k, int n_lists, const uint32_t* ids_in, const float* dist_in,
                          uint32_t* ids_out, float* dist_out, hipStream_t s, int64_t ls, int64_t rs,
                          const uint32_t* n_used) {
  unsigned blocks = (unsigned)((n + 3) / 4);
  hipLaunchKernelGGL(k_merge<R>, dim3(blocks), dim3(256), 0, s, n, k, n_lists, ids_in, dist_in, ids_out, dist_out, ls,
                     rs, n_used);
  return hipGetLastError();
}

template <int R1, int R2, int NCH>
hipError_t launch_fwd(const PropArgs& a, hipStream_t s) {
  unsigned blocks = (unsigned)((a.n + 3) / 4);
  hipLaunchKernelGGL((k_prop_forward<R1, R2, NCH>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int R1, int R2>
hipError_t launch_fwd_d(const PropArgs& a, hipStream_t s) {
  int nc = a.d / 4;   // float4 chunks; lane owns ceil(nc/16)
  if (nc <= 16) return launch_fwd<R1, R2, 1>(a, s);
  if (nc <= 32) return launch_fwd<R1, R2, 2>(a, s);
  if (nc <= 64) return launch_fwd<R1, R2, 4>(a, s);
  if (nc <= 128) return launch_fwd<R1, R2, 8>(a, s);
  if (nc <= 256) return launch_fwd<R1, R2, 16>(a, s);
  return launch_fwd<R1, R2, 0>(a, s);
}

}  // namespace

hipError_t launch_merge(int64_t n, int k, int n_lists, const uint32_t* ids_in, const float* dist_in,
                        uint32_t* ids_out, float* dist_out, hipStream_t s, int64_t ls, int64_t rs,
                        const uint32_t* n_used) {
  const bool al8 = (((uintptr_t)ids_in | (uintptr_t)dist_in | (uintptr_t)ids_out | (uintptr_t)dist_out) & 7) == 0;
  if ((k == 10 || k == 20) && al8) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    if (k == 10)
      hipLaunchKernelGGL(k_merge_pt<10>, dim3(blocks), dim3(256), 0, s, n, n_lists, ids_in, dist_in, ids_out, dist_out,
                         ls, rs, n_used);
    else
      hipLaunchKernelGGL(k_merge_pt<20>, dim3(blocks), dim3(256), 0, s, n, n_lists, ids_in, dist_in, ids_out, dist_out,
                         ls, rs, n_used);
    return hipGetLastError();
  }
  int tot = n_lists * k;
  if (tot <= 64) return launch_merge_r<1>(n, k, n_lists, ids_in, dist_in, ids_out, dist_out, s, ls, rs, n_used);
  if (tot <= 128) return launch_merge_r<2>(n, k, n_lists, ids_in, dist_in, ids_out, dist_out, s, ls, rs, n_used);
  if (tot <= 256) return launch_merge_r<4>(n, k, n_lists, ids_in, dist_in, ids_out, dist_out, s, ls, rs, n_used);
  if (tot <= 512) return launch_merge_r<8>(n, k, n_lists, ids_in, dist_in, ids_out, dist_out, s, ls, rs, n_used);
  if (tot <= 1024) return launch_merge_r<16>(n, k, n_lists, ids_in, dist_in, ids_out, dist_out, s, ls, rs, n_used);
  return hipErrorInvalidValue;
}

hipError_t launch_effective_rate(int64_t n, int k, int m, const uint32_t* lists_ids, int64_t ls, int64_t rs,
                                 int rate_permille, DiagDev* diag, hipStream_t s) {
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (k <= 16) hipLaunchKernelGGL(k_rate_count<16>, dim3(blocks), dim3(256), 0, s, n, k, m, lists_ids, ls, rs, diag);
  else if (k <= 32) hipLaunchKernelGGL(k_rate_count<32>, dim3(blocks), dim3(256), 0, s, n, k, m, lists_ids, ls, rs, diag);
  else hipLaunchKernelGGL(k_rate_count<64>, dim3(blocks), dim3(256), 0, s, n, k, m, lists_ids, ls, rs, diag);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rate_decide, dim3(1), dim3(64), 0, s, diag, m, rate_permille);
  return hipGetLastError();
}

hipError_t launch_propagate_round(const PropArgs& a, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32((uint32_t*)a.diag->prop_candidates, 0u, 4 * DIAG_SLOTS, s)) != hipSuccess) return e;
  if (a.pairwise) {
    if ((e = launch_fill_u32(a.cnt, 0u, (size_t)a.n + 1, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_prop_kth, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // R1 registers hold the k^2 gathered ids, R2 the k + k^2 keys of the
  // final selection: the smallest power-of-two widths that fit
  int kk = a.k * a.k, kt = a.k * a.k + a.k;
  if (a.visit_max > 0) e = launch_queue<false>(a, s);
  else if (kt > 1024) e = launch_queue<true>(a, s);
  else if (kk <= 64 && kt <= 128) e = launch_fwd_d<1, 2>(a, s);
  else if (kk <= 128 && kt <= 128) e = launch_fwd_d<2, 2>(a, s);
  else if (kk <= 128 && kt <= 256) e = launch_fwd_d<2, 4>(a, s);
  else if (kk <= 256 && kt <= 256) e = launch_fwd_d<4, 4>(a, s);
  else if (kk <= 256 && kt <= 512) e = launch_fwd_d<4, 8>(a, s);
  else if (kk <= 512 && kt <= 512) e = launch_fwd_d<8, 8>(a, s);
  else if (kk <= 512 && kt <= 1024) e = launch_fwd_d<8, 16>(a, s);
  else if (kk <= 1024 && kt <= 1024) e = launch_fwd_d<16, 16>(a, s);
  else return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  if (!a.pairwise) return hipSuccess;
  int64_t cnt = a.n + 1;
  unsigned nb = (unsigned)((cnt + 1023) / 1024);
  hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(1024), 0, s, a.cnt, a.offs, a.block_sums, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, a.block_sums, (int)nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(1024), 0, s, a.offs, a.block_sums, cnt);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  unsigned blocks = (unsigned)((a.n + 3) / 4);
  hipLaunchKernelGGL(k_prop_scatter, dim3(blocks), dim3(256), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_prop_final<2>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace knng
