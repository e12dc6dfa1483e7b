// Dense contractions of the path on the matrix cores (MFMA):
//   * query preparation: Pq = P q for a batch (Supplementary G computes Pq
//     once per query) plus, with pivots, the scores |x|^2 - 2 q.x that pick
//     each query's start point;
//   * the node table P c of every node;
//   * brute-force kNN (the recall ground truth of Section 1, and the graph
//     build's self-join): candidate scores in split bf16 precision, then an
//     exact float32 re-rank.
// All are C[i][j] = sum_k A[i][k] B[j][k] with A, B row-major and k
// contiguous.  One 256-thread block computes a 64 x 64 tile; each wave owns
// a 32 x 32 quarter as 2 x 2 blocks of 16 x 16 MFMA tiles (fp32
// v_mfma_f32_16x16x4f32 for Pq and P c; the pivot scores and the kNN
// candidate scores use the bf16 instructions described with them).  K
// advances in slabs of 32 staged through LDS.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 32, LDT = BK + 1;

// Stage A rows [r0, r0+64) and B rows [c0, c0+64), k in [k0, k0+32), into
// LDS (zero outside the matrices).
__device__ __forceinline__ void stage(const float* __restrict__ A, int64_t rows,
                                      const float* __restrict__ B, int64_t cols, int K,
                                      int64_t r0, int64_t c0, int k0, float* As, float* Bs) {
  const int t = threadIdx.x;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = (t >> 3) + 32 * h;
    const int kc = (t & 7) * 4;
    float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
    const int kk = k0 + kc;
    if (kk < K) {
      if (r0 + row < rows) va = *reinterpret_cast<const float4*>(A + (r0 + row) * (int64_t)K + kk);
      if (c0 + row < cols) vb = *reinterpret_cast<const float4*>(B + (c0 + row) * (int64_t)K + kk);
    }
    float* a = As + row * LDT + kc;
    float* b = Bs + row * LDT + kc;
    a[0] = va.x; a[1] = va.y; a[2] = va.z; a[3] = va.w;
    b[0] = vb.x; b[1] = vb.y; b[2] = vb.z; b[3] = vb.w;
  }
}

// acc[bi][bj] covers rows wr + 16 bi + 4 (l/16) + v, cols wc + 16 bj + l%16
__device__ __forceinline__ void tile_mma(const float* __restrict__ A, int64_t rows,
                                         const float* __restrict__ B, int64_t cols, int K,
                                         int64_t r0, int64_t c0, float* As, float* Bs,
                                         f4v acc[2][2]) {
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    stage(A, rows, B, cols, K, r0, c0, k0, As, Bs);
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int kk = ks + (l >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[(wr + 16 * i + (l & 15)) * LDT + kk];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[(wc + 16 * j + (l & 15)) * LDT + kk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
}

__global__ void __launch_bounds__(256) k_gemm_store(const float* A, int64_t rows, const float* B,
                                                    int64_t cols, int K, float* C, int64_t ldc) {
  __shared__ float As[BM * LDT], Bs[BN * LDT];
  const int64_t r0 = (int64_t)blockIdx.y * BM, c0 = (int64_t)blockIdx.x * BN;
  f4v acc[2][2];
  tile_mma(A, rows, B, cols, K, r0, c0, As, Bs, acc);
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + wr + 16 * i + 4 * (l >> 4) + v;
        const int64_t col = c0 + wc + 16 * j + (l & 15);
        if (row < rows && col < cols) C[row * ldc + col] = acc[i][j][v];
      }
}

// Pq = P q for a batch: B's first rpad rows are P (zero rows past r).
__global__ void __launch_bounds__(256) k_qprep(const float* Q, int64_t nq, const float* B, int cols,
                                               int K, int rpad, float* Pq) {
  __shared__ float As[BM * LDT], Bs[BN * LDT];
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const int64_t c0 = (int64_t)blockIdx.x * BN;
  f4v acc[2][2];
  tile_mma(Q, nq, B, cols, K, r0, c0, As, Bs, acc);
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = r0 + wr + 16 * i + 4 * (l >> 4) + v;
        const int64_t col = c0 + wc + 16 * j + (l & 15);
        if (col < rpad && row < nq) Pq[row * rpad + col] = acc[i][j][v];
      }
}

// Pq for long vectors: a workgroup owns 16 queries (many more workgroups
// than 64-row tiles give, so the latency of each K slab overlaps across
// them) and walks the columns in groups of 64, wave w taking columns
// 16 w .. 16 w + 15 of a group.  The next slab's global loads are in flight
// while the current one is multiplied (LDS double buffer).  The MFMA steps
// and their operands are those of k_qprep, so Pq is the same bits.
constexpr int kQpRows = 16;

__global__ void __launch_bounds__(256) k_qprep_rows(const float* __restrict__ Q, int64_t nq,
                                                    const float* __restrict__ B, int cols, int K,
                                                    int rpad, float* __restrict__ Pq) {
  __shared__ float As[2][kQpRows * LDT], Bs[2][BN * LDT];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int64_t r0 = (int64_t)blockIdx.x * kQpRows;
  const int srow = t >> 3, kc = (t & 7) * 4;  // staging: row t / 8 (and + 32), 4 elements
  for (int c0 = 0; c0 < rpad; c0 += BN) {
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb0 = ra, rb1 = ra;
    auto load = [&](int k0) {
      const int kk = k0 + kc;
      ra = make_float4(0.f, 0.f, 0.f, 0.f);
      rb0 = ra;
      rb1 = ra;
      if (kk < K) {
        if (srow < kQpRows && r0 + srow < nq) ra = *reinterpret_cast<const float4*>(Q + (r0 + srow) * (int64_t)K + kk);
        if (c0 + srow < cols) rb0 = *reinterpret_cast<const float4*>(B + (int64_t)(c0 + srow) * K + kk);
        if (c0 + srow + 32 < cols) rb1 = *reinterpret_cast<const float4*>(B + (int64_t)(c0 + srow + 32) * K + kk);
      }
    };
    f4v acc = f4v{0.f, 0.f, 0.f, 0.f};
    load(0);
    int buf = 0;
    for (int k0 = 0; k0 < K; k0 += BK, buf ^= 1) {
      if (srow < kQpRows) {
        float* a = &As[buf][srow * LDT + kc];
        a[0] = ra.x; a[1] = ra.y; a[2] = ra.z; a[3] = ra.w;
      }
      float* b0 = &Bs[buf][srow * LDT + kc];
      b0[0] = rb0.x; b0[1] = rb0.y; b0[2] = rb0.z; b0[3] = rb0.w;
      float* b1 = &Bs[buf][(srow + 32) * LDT + kc];
      b1[0] = rb1.x; b1[1] = rb1.y; b1[2] = rb1.z; b1[3] = rb1.w;
      __syncthreads();
      if (k0 + BK < K) load(k0 + BK);
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        const int kk = ks + (l >> 4);
        const float a = As[buf][(l & 15) * LDT + kk];
        const float b = Bs[buf][(16 * w + (l & 15)) * LDT + kk];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + 4 * (l >> 4) + v;
      const int col = c0 + 16 * w + (l & 15);
      if (col < rpad && row < nq) Pq[row * rpad + col] = acc[v];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- pivots
// Entry choice by the nearest pivot, in two stages.
//
// Stage 1 (k_pivot_scores) ranks pivots by s = |p|^2 - 2 q.p on the bf16
// matrix cores (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+8)
// and B[8(l/16)..+8)[l%16]; D[4(l/16)+v][l%16]).  Pivot rows were rounded to
// bf16 once when the tables were built; query rows are rounded on load
// (both exact for integers up to 256); products accumulate in float32.  One
// wave owns 16 queries and one of kPivSplit pivot ranges, walks that range in
// 16-pivot tiles, and keeps in every lane the lowest (score, pivot) of the
// columns that land on it (no cross-lane work in the loop); at the end each
// query row keeps the best kPivKeep of its 16 stripe minima, so a query has
// kPivCand = kPivSplit kPivKeep candidates.  Many short ranges give enough
// waves to hide the latency of the pivot tiles, which come from L2.
//
// Stage 2 (k_qfinish, one wave per query) sorts the candidates by score and
// re-ranks the best kPivRerank by exact float32 direct differences; the
// nearest (ties to the smaller pivot index) becomes the entry.
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
constexpr int kPivSplit = 16;                    // pivot ranges per 16-query tile
constexpr int kPivKeep = 4;                      // candidates kept per query and range
constexpr int kPivCand = kPivKeep * kPivSplit;   // candidates per query (= 64, one per lane)
constexpr int kPivRerank = 16;            // candidates re-ranked exactly
constexpr int kPivKs = 8;                 // 32-wide k-steps of a query held in registers
constexpr int kPivGroup = 4;              // pivot tiles sharing one chunk of query fragments
constexpr int kPivTiles = 2;              // 16-row query tiles per wave
constexpr int kPivRows = 16 * kPivTiles;  // queries per wave

static_assert(kPivCand == 64, "k_qfinish sorts one candidate per lane");

// ascending sort of one key per lane within each aligned group of 16 lanes
__device__ __forceinline__ uint64_t sort16(uint64_t v) {
  const int g = lane_id() & 15;
#pragma unroll
  for (int k = 2; k <= 16; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const uint64_t o = shfl_xor_u64(v, j);
      const bool take_min = ((g & j) == 0) == ((g & k) == 0 || k == 16);
      v = take_min ? (v < o ? v : o) : (v < o ? o : v);
    }
  }
  return v;
}

__device__ __forceinline__ b8v load_query_frag(const float* __restrict__ Q, int64_t nq, int m,
                                              int64_t row, int k) {
  float v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = 0.f;
  if (row < nq) {
    const float* src = Q + row * (int64_t)m;
    if (k < m) {
      const float4 x = *reinterpret_cast<const float4*>(src + k);
      v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    if (k + 4 < m) {
      const float4 x = *reinterpret_cast<const float4*>(src + k + 4);
      v[4] = x.x; v[5] = x.y; v[6] = x.z; v[7] = x.w;
    }
  }
  b8v r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (__bf16)v[e];
  return r;
}

// Per-lane running minima of four score rows: the lowest score and its
// pivot.  Columns reach a lane in increasing order, so a strict comparison
// keeps the smaller pivot of equal scores, which is the order of the
// (score, pivot) keys built at the end (-0 and +0 compare equal, as their
// keys do).
struct PivBest {
  float s[4];
  int c[4];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      s[v] = __int_as_float(0x7f800000);
      c[v] = -1;
    }
  }
  // one 16x16 score tile (pn = |p|^2 of this lane's column, loaded with the tile)
  __device__ __forceinline__ void fold(const f4v& acc, int col, int npiv, float pn) {
    if (col >= npiv) return;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float sc = pn - 2.f * acc[v];
      if (sc < s[v] || c[v] < 0) {
        s[v] = sc;
        c[v] = col;
      }
    }
  }
  __device__ __forceinline__ uint64_t key(int v) const {
    return c[v] < 0 ? ~0ull : (((uint64_t)order_bits(s[v]) << 32) | (uint32_t)c[v]);
  }
};

// grid: ceil(nq / kPivRows) * kPivSplit waves, 4 per block; PB [npad][kpad] bf16
// and pnorm [npad], npad = kPivSplit * range with range a multiple of 32,
// rows >= npiv zero; cand [nq][kPivCand].
// KS: 32-wide k-steps (kpad = 32 KS) when the query fits in registers
// (KS <= kPivKs); KS = 0 is the general path that streams the query in
// chunks of kPivKs steps.  The pivot tile of the next iteration is loaded
// while the current one is multiplied (two register sets).
template <int KS>
__global__ void __launch_bounds__(256) k_pivot_scores(const float* __restrict__ Q, int64_t nq, int m,
                                                      const __bf16* __restrict__ PB,
                                                      const float* __restrict__ pnorm, int npiv,
                                                      int kpad, int range,
                                                      uint64_t* __restrict__ cand) {
  // one wave: kPivRows queries (kPivTiles 16-row MFMA tiles share every pivot
  // tile it loads) x one pivot range
  constexpr int NT = kPivTiles;
  const int64_t wid = (int64_t)blockIdx.x * 4 + uniform_i(threadIdx.x / 64);
  const int64_t q0 = (wid / kPivSplit) * kPivRows;
  const int split = (int)(wid % kPivSplit);
  if (q0 >= nq) return;  // whole waves only
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = 8 * (l >> 4);
  const int c_beg = split * range;
  PivBest best[NT];
#pragma unroll
  for (int u = 0; u < NT; ++u) best[u].init();
  if constexpr (KS > 0) {
    b8v a[NT][KS];
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int i = 0; i < KS; ++i) a[u][i] = load_query_frag(Q, nq, m, q0 + 16 * u + lr, 32 * i + lk);
    // range is a multiple of 32 and PB / pnorm hold every padded row, so the
    // loop loads unconditionally: bx (tile t) is multiplied while by (tile
    // t + 16) is in flight and the other way round, and the wait counts stay
    // exact (no loads under branches)
    const __bf16* base = PB + (int64_t)(c_beg + lr) * kpad + lk;
    const float* pbase = pnorm + c_beg + lr;
    b8v bx[KS], by[KS];
#pragma unroll
    for (int i = 0; i < KS; ++i) bx[i] = *reinterpret_cast<const b8v*>(base + 32 * i);
    float px = pbase[0], py;
    for (int t = 0; t < range; t += 32) {
#pragma unroll
      for (int i = 0; i < KS; ++i)
        by[i] = *reinterpret_cast<const b8v*>(base + (int64_t)(t + 16) * kpad + 32 * i);
      py = pbase[t + 16];
      f4v c[NT];
#pragma unroll
      for (int u = 0; u < NT; ++u) c[u] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < KS; ++i)
#pragma unroll
        for (int u = 0; u < NT; ++u) c[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], bx[i], c[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < NT; ++u) best[u].fold(c[u], c_beg + t + lr, npiv, px);
      // next tile pair (the last iteration reloads its own first tile, unused)
      const int tn = t + 32 < range ? t + 32 : t;
#pragma unroll
      for (int i = 0; i < KS; ++i)
        bx[i] = *reinterpret_cast<const b8v*>(base + (int64_t)tn * kpad + 32 * i);
      px = pbase[tn];
#pragma unroll
      for (int u = 0; u < NT; ++u) c[u] = f4v{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int i = 0; i < KS; ++i)
#pragma unroll
        for (int u = 0; u < NT; ++u) c[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], by[i], c[u], 0, 0, 0);
#pragma unroll
      for (int u = 0; u < NT; ++u) best[u].fold(c[u], c_beg + t + 16 + lr, npiv, py);
    }
  } else {
    // long vectors: the k dimension is walked in chunks of kPivKs steps whose
    // query fragments stay in registers across a group of kPivGroup pivot
    // tiles, so each fragment is loaded and rounded once per group instead
    // of once per tile; every tile still accumulates its k-steps in
    // ascending order
    constexpr int TG = kPivGroup;
    const int ksteps = kpad / 32;
    const int ntile = range / 16;
    for (int t0 = 0; t0 < ntile; t0 += TG) {
      f4v c[TG][NT];
#pragma unroll
      for (int g = 0; g < TG; ++g)
#pragma unroll
        for (int u = 0; u < NT; ++u) c[g][u] = f4v{0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < ksteps; k0 += kPivKs) {
        b8v a[NT][kPivKs];
#pragma unroll
        for (int i = 0; i < kPivKs; ++i)
#pragma unroll
          for (int u = 0; u < NT; ++u)
            if (k0 + i < ksteps) a[u][i] = load_query_frag(Q, nq, m, q0 + 16 * u + lr, 32 * (k0 + i) + lk);
#pragma unroll
        for (int g = 0; g < TG; ++g) {
          if (t0 + g >= ntile) break;
          const __bf16* brow = PB + (int64_t)(c_beg + 16 * (t0 + g) + lr) * kpad + lk;
#pragma unroll
          for (int i = 0; i < kPivKs; ++i) {
            if (k0 + i >= ksteps) break;
            const b8v b = *reinterpret_cast<const b8v*>(brow + 32 * (k0 + i));
#pragma unroll
            for (int u = 0; u < NT; ++u)
              c[g][u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u][i], b, c[g][u], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int g = 0; g < TG; ++g) {
        if (t0 + g >= ntile) break;
        const int col = c_beg + 16 * (t0 + g) + lr;
        const float pn = pnorm[col];
#pragma unroll
        for (int u = 0; u < NT; ++u) best[u].fold(c[g][u], col, npiv, pn);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NT; ++u) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // row 4(l/16)+v of tile u: its 16 stripe minima, ascending
      const uint64_t srt = sort16(best[u].key(v));
      const int64_t row = q0 + 16 * u + 4 * (l >> 4) + v;
      if (lr < kPivKeep && row < nq) cand[row * kPivCand + split * kPivKeep + lr] = srt;
    }
  }
}

// The same scores and candidates for long vectors (the query does not fit in
// registers), for a workgroup of four waves that owns 64 queries and one
// pivot range, walked in passes of 256 pivots (wave w takes pivots 64 w ..
// 64 w + 63 of a pass).  Per 32-wide k-step the workgroup stages the 64
// query rows once through LDS (rounded to bf16 on the way), and each wave
// reads its own pivot fragments straight from memory (the waves' pivots are
// disjoint); both are loaded one step ahead, so the next step's loads are in
// flight during the current step's 16 MFMAs per wave.  The tiles accumulate
// their k-steps in ascending order with the same operands as
// k_pivot_scores, so scores, stripe minima and candidates are the same
// bits.  At the end the four waves' stripe minima (stripe = pivot column
// mod 16 within the range) are combined through LDS.
constexpr int kPlQ = 64;     // queries per workgroup
constexpr int kPlP = 256;    // pivots per pass
constexpr int kPlRow = 40;   // LDS row pitch of the query slab in bf16 elements (32 + 8)

__global__ void __launch_bounds__(256) k_pivot_scores_lds(const float* __restrict__ Q, int64_t nq, int m,
                                                          const __bf16* __restrict__ PB,
                                                          const float* __restrict__ pnorm, int npiv,
                                                          int kpad, int range,
                                                          uint64_t* __restrict__ cand) {
  // query slabs (2 x 64 x 40 bf16) during the k loop, then the stripe
  // minima (64 rows x 4 waves x 16 stripes)
  __shared__ __align__(16) uint64_t lds_raw[kPlQ * 4 * 16];
  __bf16* sA = reinterpret_cast<__bf16*>(lds_raw);
  static_assert(2 * kPlQ * kPlRow * 2 <= kPlQ * 4 * 16 * 8, "slabs fit the stripe area");
  const int tid = threadIdx.x;
  const int w = uniform_i(tid >> 6), l = tid & 63, lr = l & 15, lk = 8 * (l >> 4);
  const int64_t q0 = (int64_t)blockIdx.x * kPlQ;
  const int split = blockIdx.y;
  const int c_beg = split * range;
  const int ksteps = kpad / 32;
  // staging role: query row tid / 4, elements 8 (tid % 4) .. +8 of the k-step
  const int arow = tid >> 2, acol = 8 * (tid & 3);
  const int64_t aq = q0 + arow;
  const float* asrc = Q + (aq < nq ? aq : 0) * (int64_t)m;
  PivBest best[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) best[i].init();
  const b8v zero8 = b8v{(__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f,
                        (__bf16)0.f, (__bf16)0.f};
  for (int pass = 0; pass < range; pass += kPlP) {
    // this lane's pivot row of each of the wave's four tiles
    const __bf16* brow[4];
    bool bok[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int rel = pass + 64 * w + 16 * j + lr;
      bok[j] = rel < range;
      brow[j] = PB + (int64_t)(c_beg + (bok[j] ? rel : 0)) * kpad + lk;
    }
    float4 ra0, ra1;
    b8v bcur[4], bnxt[4];
    auto load_a = [&](int ks) {
      const int k = 32 * ks + acol;
      ra0 = make_float4(0.f, 0.f, 0.f, 0.f);
      ra1 = ra0;
      if (aq < nq) {
        if (k < m) ra0 = *reinterpret_cast<const float4*>(asrc + k);
        if (k + 4 < m) ra1 = *reinterpret_cast<const float4*>(asrc + k + 4);
      }
    };
    auto load_b = [&](int ks, b8v* dst) {
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[j] = bok[j] ? *reinterpret_cast<const b8v*>(brow[j] + 32 * ks) : zero8;
    };
    f4v acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
    load_a(0);
    load_b(0, bcur);
    for (int ks = 0; ks < ksteps; ++ks) {
      __bf16* slab = sA + (ks & 1) * (kPlQ * kPlRow);
      {
        b8v av;
        av[0] = (__bf16)ra0.x; av[1] = (__bf16)ra0.y; av[2] = (__bf16)ra0.z; av[3] = (__bf16)ra0.w;
        av[4] = (__bf16)ra1.x; av[5] = (__bf16)ra1.y; av[6] = (__bf16)ra1.z; av[7] = (__bf16)ra1.w;
        *reinterpret_cast<b8v*>(slab + arow * kPlRow + acol) = av;
      }
      __syncthreads();
      if (ks + 1 < ksteps) {
        load_a(ks + 1);
        load_b(ks + 1, bnxt);
      }
      b8v a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = *reinterpret_cast<const b8v*>(slab + (16 * i + lr) * kPlRow + lk);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bcur[j], acc[i][j], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) bcur[j] = bnxt[j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (bok[j]) {
        const int col = c_beg + pass + 64 * w + 16 * j + lr;
        const float pn = pnorm[col];
#pragma unroll
        for (int i = 0; i < 4; ++i) best[i].fold(acc[i][j], col, npiv, pn);
      }
    }
    __syncthreads();  // the next pass restages the slabs
  }
  // stripe minima of the four waves: S[row][wave][stripe]
  uint64_t* S = lds_raw;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) S[((16 * i + 4 * (l >> 4) + v) * 4 + w) * 16 + lr] = best[i].key(v);
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int row = 16 * w + 4 * it + (l >> 4);
    uint64_t mn = S[(row * 4) * 16 + lr];
#pragma unroll
    for (int ww = 1; ww < 4; ++ww) {
      const uint64_t o = S[(row * 4 + ww) * 16 + lr];
      mn = o < mn ? o : mn;
    }
    const uint64_t srt = sort16(mn);
    if (lr < kPivKeep && q0 + row < nq) cand[(q0 + row) * kPivCand + split * kPivKeep + lr] = srt;
  }
}

// Per query (one wave): |q|^2, then (with candidates) the exact re-rank.
// PF: float32 pivot rows [npiv][m].
__global__ void k_qfinish(const float* __restrict__ Q, int64_t nq, int m,
                          const float* __restrict__ PF, const int32_t* __restrict__ piv_ids,
                          int npiv, const uint64_t* __restrict__ cand, float* __restrict__ qq,
                          int32_t* __restrict__ entries, int ip) {
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + uniform_i(threadIdx.x / 64);
  if (q >= nq) return;
  const int l = threadIdx.x & 63;
  const float* qv = Q + q * m;
  float acc = 0.f;
  for (int j = l; j < m; j += 64) acc += qv[j] * qv[j];
  acc = wave_sum(acc);
  if (l == 0) qq[q] = acc;
  if (cand == nullptr || entries == nullptr) return;
  const uint64_t key = bitonic_sort<64>(cand[q * kPivCand + l]);
  // four lanes per candidate; candidate ci is the ci-th lowest score
  const int ci = l >> 2, part = l & 3;
  const uint64_t ck = shfl_u64(key, ci);
  const int col = (int)(uint32_t)ck;
  const bool valid = ck != ~0ull && col >= 0 && col < npiv;
  float d = 0.f;
  if (valid) {
    const float4* p4 = reinterpret_cast<const float4*>(PF + (int64_t)col * m);
    const float4* q4 = reinterpret_cast<const float4*>(qv);
    if (ip) {
      for (int j = part; j < m / 4; j += 4) {
        const float4 x = q4[j], y = p4[j];
        d -= x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
      }
    } else {
      for (int j = part; j < m / 4; j += 4) {
        const float4 x = q4[j], y = p4[j];
        const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
        d += dx * dx + dy * dy + dz * dz + dw * dw;
      }
    }
  }
  d += shfl_xor_f(d, 1);
  d += shfl_xor_f(d, 2);
  uint64_t mine = (valid && ci < kPivRerank) ? make_key(d, col) : ~0ull;
#pragma unroll
  for (int o = 4; o < 64; o <<= 1) {
    const uint64_t other = shfl_xor_u64(mine, o);
    mine = other < mine ? other : mine;
  }
  if (l == 0) entries[q] = piv_ids[mine == ~0ull ? 0 : key_id(mine)];
}

__global__ void k_pack_bf16_rows(const float* __restrict__ src, int rows, int m, int rows_pad,
                                 int kpad, __bf16* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows_pad * kpad) return;
  const int row = (int)(i / kpad), k = (int)(i % kpad);
  dst[i] = (__bf16)((row < rows && k < m) ? src[(int64_t)row * m + k] : 0.f);
}

}  // namespace

hipError_t launch_gemm_nt(const float* A, int64_t rows, const float* B, int64_t cols, int K,
                          float* C, int64_t ldc, hipStream_t s) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((unsigned)((cols + BN - 1) / BN), (unsigned)((rows + BM - 1) / BM));
  hipLaunchKernelGGL(k_gemm_store, grid, dim3(256), 0, s, A, rows, B, cols, K, C, ldc);
  return hipGetLastError();
}

size_t query_prep_scratch_bytes(const Tables& t, int64_t nq) {
  return t.npiv > 0 ? (size_t)nq * kPivCand * sizeof(uint64_t) : 0;
}

int pivot_pad_rows(int npiv) { return (npiv + 32 * kPivSplit - 1) / (32 * kPivSplit) * (32 * kPivSplit); }
int pivot_kpad(int m) { return (m + 31) / 32 * 32; }

hipError_t launch_pack_pivots(const float* src, int npiv, int m, __bf16* dst, hipStream_t s) {
  const int rows_pad = pivot_pad_rows(npiv), kpad = pivot_kpad(m);
  const int64_t total = (int64_t)rows_pad * kpad;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack_bf16_rows, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src,
                     npiv, m, rows_pad, kpad, dst);
  return hipGetLastError();
}

hipError_t launch_query_prep(const Tables& t, const float* Q, int64_t nq, float* qq, float* Pq,
                             int32_t* entries, void* scratch, hipStream_t s, bool need_pq) {
  if (nq == 0) return hipSuccess;
  const int rpad = rpad_of(t.r);
  const int rcols = (rpad + BN - 1) / BN * BN;  // P block padded to whole tiles
  const bool piv = t.npiv > 0 && entries != nullptr;
  uint64_t* cand = piv ? reinterpret_cast<uint64_t*>(scratch) : nullptr;
  if (t.r > 0 && need_pq) {
    // Pq = P q in float32 MFMA (the estimate needs full precision)
    if (t.m > 128) {
      hipLaunchKernelGGL(k_qprep_rows, dim3((unsigned)((nq + kQpRows - 1) / kQpRows)), dim3(256), 0, s, Q,
                         nq, t.qprep_B, rcols, t.m, rpad, Pq);
    } else {
      dim3 grid((unsigned)(rcols / BN), (unsigned)((nq + BM - 1) / BM));
      hipLaunchKernelGGL(k_qprep, grid, dim3(256), 0, s, Q, nq, t.qprep_B, rcols, t.m, rpad, Pq);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (piv) {
    const int64_t waves = (nq + kPivRows - 1) / kPivRows * kPivSplit;
    const int range = pivot_pad_rows(t.npiv) / kPivSplit;
    const int kpad = pivot_kpad(t.m);
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    const float* pn = t.piv_norm;
    if (kpad > 128) {
      // long vectors: operands staged through LDS (same candidates)
      const dim3 g2((unsigned)((nq + kPlQ - 1) / kPlQ), (unsigned)kPivSplit);
      hipLaunchKernelGGL(k_pivot_scores_lds, g2, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad,
                         range, cand);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    } else switch (kpad / 32) {
      case 1: hipLaunchKernelGGL(k_pivot_scores<1>, grid, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad, range, cand); break;
      case 2: hipLaunchKernelGGL(k_pivot_scores<2>, grid, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad, range, cand); break;
      case 3: hipLaunchKernelGGL(k_pivot_scores<3>, grid, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad, range, cand); break;
      case 4: hipLaunchKernelGGL(k_pivot_scores<4>, grid, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad, range, cand); break;
      default: hipLaunchKernelGGL(k_pivot_scores<0>, grid, block, 0, s, Q, nq, t.m, t.piv_b16, pn, t.npiv, kpad, range, cand); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int wpb = 4;
  hipLaunchKernelGGL(k_qfinish, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb), 0, s, Q,
                     nq, t.m, t.qprep_B + (int64_t)rcols * t.m, t.piv_ids, t.npiv, cand, qq,
                     piv ? entries : nullptr, t.metric == FINGER_IP ? 1 : 0);
  return hipGetLastError();
}

// ------------------------------------------------------------ exact kNN

namespace {

// candidates kept beyond k for the exact re-rank: a true neighbour is lost
// only if 16 others sit within the split-precision score error (about 1e-5
// relative) of it; integer data up to 256 scores exactly
constexpr int kKnnSlack = 16;

// Candidate scores for the kNN on the bf16 matrix cores, in split precision:
// each float x is staged as hi = bf16(x) and lo = bf16(x - hi), and
// A.B ~ hi.hi' + hi.lo' + lo.hi' (the dropped lo.lo' term is below 2^-16 of
// |x||y|), accumulated in float32 by v_mfma_f32_16x16x32_bf16.  The scores
// only choose the k + kKnnSlack candidates that k_knn_final re-ranks by exact
// float32 differences.  LDS: hi/lo tiles of A and B, 64 rows x 32 k, rows
// padded to 40 elements (80 bytes) so a lane's 16-byte fragment read stays
// aligned.
typedef __bf16 b4v __attribute__((ext_vector_type(4)));
constexpr int kX3Row = 40;
constexpr int kX3Tile = BM * kX3Row;                      // elements per hi or lo tile
constexpr int kX3Bytes = 4 * kX3Tile * 2;                 // Ahi, Alo, Bhi, Blo
static_assert(kX3Bytes >= BM * 65 * 4, "the score tile reuses the staging area");

__device__ __forceinline__ void stage_x3(const float* __restrict__ A, int64_t rows,
                                         const float* __restrict__ B, int64_t cols, int K,
                                         int64_t r0, int64_t c0, int k0, __bf16* S) {
  const int t = threadIdx.x;
  __bf16* Ahi = S;
  __bf16* Alo = S + kX3Tile;
  __bf16* Bhi = S + 2 * kX3Tile;
  __bf16* Blo = S + 3 * kX3Tile;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int row = (t >> 3) + 32 * h;
    const int kc = (t & 7) * 4;
    float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
    const int kk = k0 + kc;
    if (kk < K) {
      if (r0 + row < rows) va = *reinterpret_cast<const float4*>(A + (r0 + row) * (int64_t)K + kk);
      if (c0 + row < cols) vb = *reinterpret_cast<const float4*>(B + (c0 + row) * (int64_t)K + kk);
    }
    const float xa[4] = {va.x, va.y, va.z, va.w};
    const float xb[4] = {vb.x, vb.y, vb.z, vb.w};
    b4v ha, la, hb, lb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      ha[e] = (__bf16)xa[e];
      la[e] = (__bf16)(xa[e] - (float)ha[e]);
      hb[e] = (__bf16)xb[e];
      lb[e] = (__bf16)(xb[e] - (float)hb[e]);
    }
    // four elements = one 8-byte LDS write per tile (row * 80 + kc * 2 is
    // 8-byte aligned)
    *reinterpret_cast<b4v*>(Ahi + row * kX3Row + kc) = ha;
    *reinterpret_cast<b4v*>(Alo + row * kX3Row + kc) = la;
    *reinterpret_cast<b4v*>(Bhi + row * kX3Row + kc) = hb;
    *reinterpret_cast<b4v*>(Blo + row * kX3Row + kc) = lb;
  }
}

// acc[bi][bj] covers rows wr + 16 bi + 4 (l/16) + v, cols wc + 16 bj + l%16
// (the same layout as tile_mma)
__device__ __forceinline__ void tile_mma_x3(const float* __restrict__ A, int64_t rows,
                                            const float* __restrict__ B, int64_t cols, int K,
                                            int64_t r0, int64_t c0, __bf16* S, f4v acc[2][2]) {
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  const int fo = (l & 15) * kX3Row + 8 * (l >> 4);   // this lane's fragment in a 16-row block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    stage_x3(A, rows, B, cols, K, r0, c0, k0, S);
    __syncthreads();
    b8v ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      ah[i] = *reinterpret_cast<const b8v*>(S + (wr + 16 * i) * kX3Row + fo);
      al[i] = *reinterpret_cast<const b8v*>(S + kX3Tile + (wr + 16 * i) * kX3Row + fo);
      bh[i] = *reinterpret_cast<const b8v*>(S + 2 * kX3Tile + (wc + 16 * i) * kX3Row + fo);
      bl[i] = *reinterpret_cast<const b8v*>(S + 3 * kX3Tile + (wc + 16 * i) * kX3Row + fo);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
      }
  }
}

// Each block: 64 queries x a contiguous range of data columns.  The running
// best KK (approximate d2, id) per query live in LDS as sorted lists.  The
// tile loop waits on LDS and on the global loads of the next tile, so
// occupancy pays: registers are capped so that four waves share a SIMD (the
// LDS lists admit four blocks per CU in any case).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_knn_tiles(const float* Q, int64_t nq, const float* X, int64_t n, int K, const float* qn,
            const float* xn, int KK, int64_t chunk, uint64_t* out, int nchunks, int ip) {
  extern __shared__ __align__(16) char smem[];
  __bf16* S = reinterpret_cast<__bf16*>(smem);
  uint64_t* lists = reinterpret_cast<uint64_t*>(smem + kX3Bytes);
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const int64_t cbeg = (int64_t)blockIdx.x * chunk;
  const int64_t cend = min(n, cbeg + chunk);
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  for (int i = threadIdx.x; i < BM * KK; i += blockDim.x) lists[i] = ~0ull;
  int* cnts = reinterpret_cast<int*>(lists + BM * KK);        // fill of each row's list
  uint64_t* nk = reinterpret_cast<uint64_t*>(cnts + BM) + w * 64; // this wave's sorted new keys
  for (int i = threadIdx.x; i < BM; i += blockDim.x) cnts[i] = 0;
  for (int64_t c0 = cbeg; c0 < cend; c0 += BN) {
    f4v acc[2][2];
    tile_mma_x3(Q, nq, X, cend, K, r0, c0, S, acc);
    __syncthreads();
    float* Ct = reinterpret_cast<float*>(smem);  // 64 x 65 tile of approximate d2
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = wr + 16 * i + 4 * (l >> 4) + v;
          const int cl = wc + 16 * j + (l & 15);
          const int64_t row = r0 + rr, col = c0 + cl;
          float d = __int_as_float(0x7f800000);
          if (row < nq && col < cend)
            d = ip ? -acc[i][j][v] : fmaxf(qn[row] + xn[col] - 2.f * acc[i][j][v], 0.f);
          Ct[rr * 65 + cl] = d;
        }
    __syncthreads();
    // this wave's 16 rows: read every row's score and current worst key
    // first, so the LDS reads are in flight together (most rows admit
    // nothing once their lists are full)
    float dr[BM / 4];
    uint64_t wr_[BM / 4];
#pragma unroll
    for (int s4 = 0; s4 < BM / 4; ++s4) {
      const int rr = w + 4 * s4;
      dr[s4] = Ct[rr * 65 + l];
      const int cnt = cnts[rr];
      wr_[s4] = cnt < KK ? ~0ull : lists[rr * KK + KK - 1];
    }
#pragma unroll 1
    for (int s4 = 0; s4 < BM / 4; ++s4) {
      const int rr = w + 4 * s4;
      uint64_t* L = lists + rr * KK;
      const float d = dr[s4];
      const uint64_t key = (d < __int_as_float(0x7f800000)) ? make_key(d, (int)(c0 + l)) : ~0ull;
      const bool in = key < wr_[s4];
      const uint64_t bm = ballot(in);
      const int na = popc64(bm);
      if (na == 0) continue;
      const int cnt = cnts[rr];
      const uint64_t v = bitonic_sort<64>(in ? key : ~0ull);
      nk[l] = v;
      wave_lds_sync();
      // existing entries move right by the number of new keys below them
      uint64_t mine[3];
      int pos[3];
      int nm = 0;
      for (int i = l; i < cnt; i += 64) {
        const uint64_t kk = L[i];
        int lo = 0, hi = na;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (nk[mid] < kk) lo = mid + 1; else hi = mid;
        }
        mine[nm] = kk;
        pos[nm] = i + lo;
        ++nm;
      }
      int pv = KK;
      if (l < na) {
        int lo = 0, hi = cnt;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (L[mid] < v) lo = mid + 1; else hi = mid;
        }
        pv = l + lo;
      }
      wave_lds_sync();
      for (int t = 0; t < nm; ++t)
        if (pos[t] < KK) L[pos[t]] = mine[t];
      if (l < na && pv < KK) L[pv] = v;
      if (l == 0) cnts[rr] = min(cnt + na, KK);
      wave_lds_sync();
    }
  }
  __syncthreads();
  for (int s = 0; s < 16; ++s) {
    const int rr = w + 4 * s;
    const int64_t row = r0 + rr;
    if (row >= nq) continue;
    for (int i = l; i < KK; i += 64)
      out[(row * nchunks + blockIdx.x) * KK + i] = lists[rr * KK + i];
  }
}

// Per query (one wave): gather the chunk lists, keep the KK best keys,
// re-rank them by direct float32 differences and emit the best k by (d2, id).
__global__ void k_knn_final(const float* Q, int64_t nq, const float* X, int m, int k, int KK,
                            int nchunks, const uint64_t* cand, int32_t* ids, float* dist, int ip) {
  extern __shared__ __align__(16) char smem[];
  const int wib = threadIdx.x / 64, l = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + wib;
  const int total = nchunks * KK;
  uint64_t* buf = reinterpret_cast<uint64_t*>(smem) + (int64_t)wib * (total + 2 * KK);
  uint64_t* sel = buf + total;
  if (q >= nq) return;
  const uint64_t* c = cand + q * total;
  // threshold: the smallest per-chunk KK-th key bounds the global KK-th
  uint64_t th = ~0ull;
  for (int ch = 0; ch < nchunks; ++ch) {
    const uint64_t v = c[ch * KK + KK - 1];
    th = v < th ? v : th;
  }
  int nsel = 0;
  for (int b0 = 0; b0 < total; b0 += 64) {
    const int i = b0 + l;
    const uint64_t v = i < total ? c[i] : ~0ull;
    const bool in = v != ~0ull && v <= th;
    const uint64_t bm = ballot(in);
    if (in) buf[nsel + mask_rank(bm)] = v;
    nsel += popc64(bm);
  }
  wave_lds_sync();
  // rank-select the KK smallest of buf[0..nsel)
  const int keep = min(KK, nsel);
  for (int i = l; i < nsel; i += 64) {
    const uint64_t v = buf[i];
    int rk = 0;
    for (int t = 0; t < nsel; ++t) rk += buf[t] < v ? 1 : 0;
    if (rk < keep) sel[rk] = v;
  }
  wave_lds_sync();
  // exact re-rank
  const float* qv = Q + q * m;
  uint64_t* ex = sel + KK;
  for (int t = 0; t < keep; ++t) {
    const int id = key_id(sel[t]);
    const float* xv = X + (int64_t)id * m;
    float d = 0.f;
    if (ip)
      for (int j = l; j < m; j += 64) d -= qv[j] * xv[j];
    else
      for (int j = l; j < m; j += 64) { float u = qv[j] - xv[j]; d += u * u; }
    d = wave_sum(d);
    if (l == 0) ex[t] = make_key(d, id);
  }
  wave_lds_sync();
  for (int i = l; i < keep; i += 64) {
    const uint64_t v = ex[i];
    int rk = 0;
    for (int t = 0; t < keep; ++t) rk += ex[t] < v ? 1 : 0;
    if (rk < k) {
      ids[q * k + rk] = key_id(v);
      dist[q * k + rk] = key_d2(v);
    }
  }
  for (int i = keep + l; i < k; i += 64) {
    ids[q * k + i] = -1;
    dist[q * k + i] = __int_as_float(0x7f800000);
  }
}

int knn_chunks(int64_t n, int64_t nq) {
  const int64_t qtiles = (nq + BM - 1) / BM;
  int64_t want = (2048 + qtiles - 1) / qtiles;  // aim for >= 2048 blocks
  int64_t maxc = (n + BN - 1) / BN;
  int64_t c = want < 1 ? 1 : want;
  if (c > maxc) c = maxc;
  if (c > 16) c = 16;
  return (int)c;
}

}  // namespace

size_t exact_knn_ws_bytes(int64_t n, int m, int64_t nq, int k) {
  const int KK = k + kKnnSlack;
  const int nch = knn_chunks(n, nq);
  size_t b = 0;
  b += ((size_t)n * 4 + 255) / 256 * 256;             // data norms
  b += ((size_t)nq * 4 + 255) / 256 * 256;            // query norms
  b += ((size_t)nq * nch * KK * 8 + 255) / 256 * 256; // candidates
  (void)m;
  return b;
}

hipError_t launch_exact_knn(const float* data, int64_t n, int m, const float* Q, int64_t nq,
                            int k, int metric, int32_t* ids, float* dist, void* ws,
                            hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const int KK = k + kKnnSlack;
  const int nch = knn_chunks(n, nq);
  char* p = static_cast<char*>(ws);
  float* xn = reinterpret_cast<float*>(p);
  p += ((size_t)n * 4 + 255) / 256 * 256;
  float* qn = reinterpret_cast<float*>(p);
  p += ((size_t)nq * 4 + 255) / 256 * 256;
  uint64_t* cand = reinterpret_cast<uint64_t*>(p);
  hipError_t e = launch_row_norms(data, n, m, xn, s);
  if (e != hipSuccess) return e;
  e = launch_row_norms(Q, nq, m, qn, s);
  if (e != hipSuccess) return e;
  const int64_t ntile = (n + BN - 1) / BN;
  const int64_t chunk = (ntile + nch - 1) / nch * BN;
  const int lds = kX3Bytes + BM * KK * 8 + BM * 4 + 4 * 64 * 8;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_knn_tiles),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)nch, (unsigned)((nq + BM - 1) / BM));
  hipLaunchKernelGGL(k_knn_tiles, grid, dim3(256), lds, s, Q, nq, data, n, m, qn, xn, KK, chunk,
                     cand, nch, metric == FINGER_IP ? 1 : 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int wpb = 2;
  const int flds = wpb * (nch * KK + 2 * KK) * 8;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_knn_final),
                          hipFuncAttributeMaxDynamicSharedMemorySize, flds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_final, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb), flds, s,
                     Q, nq, data, m, k, KK, nch, cand, ids, dist, metric == FINGER_IP ? 1 : 0);
  return hipGetLastError();
}

}  // namespace finger
