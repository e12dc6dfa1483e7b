// Dense contractions of the path on the fp32 matrix cores (MFMA):
//   * query preparation: Pq = P q for a batch (Supplementary G computes Pq
//     once per query) plus, with pivots, the scores |x|^2 - 2 q.x that pick
//     each query's start point;
//   * the node table P c of every node;
//   * brute-force kNN (the recall ground truth of Section 1).
// All are C[i][j] = sum_k A[i][k] B[j][k] with A, B row-major and k
// contiguous.  One 256-thread block computes a 64 x 64 tile; each wave owns
// a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f32_16x16x4f32.  K advances
// in slabs of 32 staged through LDS.
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

// Query prep: columns [0, rpad) of B are P (zero rows past r), columns
// [rpad, rpad + npiv) are pivot vectors.  Stores Pq and, per 64-column tile,
// the two best pivot scores |x|^2 - 2 q.x of each query.
__global__ void __launch_bounds__(256) k_qprep(const float* Q, int64_t nq, const float* B,
                                               const float* Bnorm, int cols, int K, int rpad,
                                               int pcols, int pend, float* Pq, float2* best,
                                               int ntiles) {
  __shared__ float As[BM * LDT], Bs[BN * LDT];
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const int64_t c0 = (int64_t)blockIdx.x * BN;
  f4v acc[2][2];
  tile_mma(Q, nq, B, cols, K, r0, c0, As, Bs, acc);
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  __syncthreads();
  // scores to LDS (reuse As as a 64 x 65 tile)
  float* Ct = As;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = wr + 16 * i + 4 * (l >> 4) + v;
        const int cl = wc + 16 * j + (l & 15);
        const int64_t row = r0 + rr, col = c0 + cl;
        const float c = acc[i][j][v];
        if (col < rpad) {
          if (row < nq) Pq[row * rpad + col] = c;
        }
        Ct[rr * 65 + cl] = (col >= pcols && col < pend) ? Bnorm[col] - 2.f * c
                                                         : __int_as_float(0x7f800000);
      }
  __syncthreads();
  if (c0 + BN <= pcols || ntiles == 0) return;
  // per query row: the best two (score, column) of this tile
  const int tile = (int)(blockIdx.x) - pcols / BN;
  for (int rr = w; rr < BM; rr += 4) {
    const int64_t row = r0 + rr;
    float s = Ct[rr * 65 + l];
    int col = (int)c0 + l;
    // min over the wave, ties to the smaller column
    float s1 = s;
    int c1 = col;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      float so = __shfl_xor(s1, o, 64);
      int co = __shfl_xor(c1, o, 64);
      if (so < s1 || (so == s1 && co < c1)) { s1 = so; c1 = co; }
    }
    float s2 = (col == c1) ? __int_as_float(0x7f800000) : s;
    int c2 = col;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      float so = __shfl_xor(s2, o, 64);
      int co = __shfl_xor(c2, o, 64);
      if (so < s2 || (so == s2 && co < c2)) { s2 = so; c2 = co; }
    }
    if (l == 0 && row < nq && tile >= 0) {
      best[(row * ntiles + tile) * 2] = make_float2(s1, __int_as_float(c1));
      best[(row * ntiles + tile) * 2 + 1] = make_float2(s2, __int_as_float(c2));
    }
  }
}

// Pivot scores |x|^2 - 2 q.x on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+8) and
// B[8(l/16)..+8)[l%16]; D[4(l/16)+v][l%16]).  Queries and pivots are rounded
// to bf16 (exact for integers up to 256), products accumulate in float32.
// The scores only rank candidates: the final choice is re-ranked with exact
// float32 distances in k_qfinish.  Per 64-column tile, each query keeps its
// two best (score, column).
typedef __bf16 b8v __attribute__((ext_vector_type(8)));
constexpr int PK = 32, PLD = 40;  // K slab and padded LDS row (bf16 elements)

__global__ void __launch_bounds__(256) k_pivot_scores(const float* Q, int64_t nq, const float* B,
                                                      const float* Bnorm, int pcols, int pend,
                                                      int K, float2* best, int ntiles) {
  __shared__ __align__(16) __bf16 As[BM * PLD], Bs[BN * PLD];
  __shared__ float Ct[BM * 65];
  const int64_t r0 = (int64_t)blockIdx.y * BM;
  const int tile = blockIdx.x;
  const int64_t c0 = pcols + (int64_t)tile * BN;
  const int w = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += PK) {
    __syncthreads();
    // stage: 64 rows x 32 k of each operand, 8 elements per thread
    {
      const int row = threadIdx.x >> 2, kc = (threadIdx.x & 3) * 8;
      float va[8], vb[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) { va[e] = 0.f; vb[e] = 0.f; }
      if (k0 + kc < K) {  // K % 4 == 0 and slabs of 8 never straddle K when K % 8 == 0
        const int64_t qa = r0 + row, cb = c0 + row;
#pragma unroll
        for (int e = 0; e < 8; e += 4) {
          if (k0 + kc + e < K) {
            if (qa < nq) {
              const float4 v = *reinterpret_cast<const float4*>(Q + qa * K + k0 + kc + e);
              va[e] = v.x; va[e + 1] = v.y; va[e + 2] = v.z; va[e + 3] = v.w;
            }
            if (cb < pend) {
              const float4 v = *reinterpret_cast<const float4*>(B + cb * K + k0 + kc + e);
              vb[e] = v.x; vb[e + 1] = v.y; vb[e + 2] = v.z; vb[e + 3] = v.w;
            }
          }
        }
      }
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        As[row * PLD + kc + e] = (__bf16)va[e];
        Bs[row * PLD + kc + e] = (__bf16)vb[e];
      }
    }
    __syncthreads();
    b8v a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      a[i] = *reinterpret_cast<const b8v*>(&As[(wr + 16 * i + (l & 15)) * PLD + 8 * (l >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j)
      b[j] = *reinterpret_cast<const b8v*>(&Bs[(wc + 16 * j + (l & 15)) * PLD + 8 * (l >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = wr + 16 * i + 4 * (l >> 4) + v;
        const int cl = wc + 16 * j + (l & 15);
        const int64_t col = c0 + cl;
        Ct[rr * 65 + cl] = col < pend ? Bnorm[col] - 2.f * acc[i][j][v] : __int_as_float(0x7f800000);
      }
  __syncthreads();
  for (int rr = w; rr < BM; rr += 4) {
    const int64_t row = r0 + rr;
    const float s = Ct[rr * 65 + l];
    const int col = (int)c0 + l;
    float s1 = s;
    int c1 = col;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float so = __shfl_xor(s1, o, 64);
      const int co = __shfl_xor(c1, o, 64);
      if (so < s1 || (so == s1 && co < c1)) { s1 = so; c1 = co; }
    }
    float s2 = (col == c1) ? __int_as_float(0x7f800000) : s;
    int c2 = col;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const float so = __shfl_xor(s2, o, 64);
      const int co = __shfl_xor(c2, o, 64);
      if (so < s2 || (so == s2 && co < c2)) { s2 = so; c2 = co; }
    }
    if (l == 0 && row < nq) {
      best[(row * ntiles + tile) * 2] = make_float2(s1, __int_as_float(c1));
      best[(row * ntiles + tile) * 2 + 1] = make_float2(s2, __int_as_float(c2));
    }
  }
}

// Per query (one wave): norms, then among the per-tile best pivot scores
// the 8 lowest are re-ranked by exact direct differences; the nearest
// pivot (ties to the smaller pivot index) becomes the entry.
__global__ void k_qfinish(const float* Q, int64_t nq, int m, const float* B, int pcols,
                          const int32_t* piv_ids, int npiv, const float2* best, int ntiles,
                          float* qq, int32_t* entries) {
  const int64_t q = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (q >= nq) return;
  const int l = threadIdx.x & 63;
  const float* qv = Q + q * m;
  float acc = 0.f;
  for (int j = l; j < m; j += 64) acc += qv[j] * qv[j];
  acc = wave_sum(acc);
  if (l == 0) qq[q] = acc;
  if (ntiles == 0 || entries == nullptr) return;
  // 4 best candidates by score (each lane scans a strided subset)
  float cs[4];
  int cc[4];
  for (int i = 0; i < 4; ++i) { cs[i] = __int_as_float(0x7f800000); cc[i] = 0x7fffffff; }
  for (int i = l; i < 2 * ntiles; i += 64) {
    float2 b = best[q * 2 * ntiles + i];
    float s = b.x;
    int c = __float_as_int(b.y);
    if (!(s < __int_as_float(0x7f800000))) continue;
    // insert into the lane's sorted 4-list
    for (int t = 0; t < 4; ++t) {
      if (s < cs[t] || (s == cs[t] && c < cc[t])) {
        float ts = cs[t]; int tc = cc[t];
        cs[t] = s; cc[t] = c; s = ts; c = tc;
      }
    }
  }
  float bestd = __int_as_float(0x7f800000);
  int bestc = 0x7fffffff;
  for (int round = 0; round < 8; ++round) {
    // wave-wide minimum of the lanes' heads
    float s1 = cs[0];
    int c1 = cc[0];
    for (int o = 32; o >= 1; o >>= 1) {
      float so = __shfl_xor(s1, o, 64);
      int co = __shfl_xor(c1, o, 64);
      if (so < s1 || (so == s1 && co < c1)) { s1 = so; c1 = co; }
    }
    if (!(s1 < __int_as_float(0x7f800000))) break;
    if (cc[0] == c1) {  // pop the head
      for (int t = 0; t < 3; ++t) { cs[t] = cs[t + 1]; cc[t] = cc[t + 1]; }
      cs[3] = __int_as_float(0x7f800000); cc[3] = 0x7fffffff;
    }
    // exact distance to pivot column c1
    const float* pv = B + (int64_t)c1 * m;
    float d = 0.f;
    for (int j = l; j < m; j += 64) { float t = qv[j] - pv[j]; d += t * t; }
    d = wave_sum(d);
    const int pidx = c1 - pcols;
    if (d < bestd || (d == bestd && pidx < bestc)) { bestd = d; bestc = pidx; }
  }
  if (bestc < 0 || bestc >= npiv) bestc = 0;  // only for non-finite scores
  if (l == 0) entries[q] = piv_ids[bestc];
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
  const int ntiles = t.npiv > 0 ? (t.npiv + BN - 1) / BN : 0;
  return (size_t)nq * ntiles * 2 * sizeof(float2);
}

hipError_t launch_query_prep(const Tables& t, const float* Q, int64_t nq, float* qq, float* Pq,
                             int32_t* entries, float* scratch, hipStream_t s, bool need_pq) {
  if (nq == 0) return hipSuccess;
  const int rpad = rpad_of(t.r);
  const int rcols = (rpad + BN - 1) / BN * BN;  // P block padded to whole tiles
  const int ntiles = t.npiv > 0 ? (t.npiv + BN - 1) / BN : 0;
  float2* best = reinterpret_cast<float2*>(scratch);
  if (t.r > 0 && need_pq) {
    // Pq = P q in float32 MFMA (the estimate needs full precision)
    dim3 grid((unsigned)(rcols / BN), (unsigned)((nq + BM - 1) / BM));
    hipLaunchKernelGGL(k_qprep, grid, dim3(256), 0, s, Q, nq, t.qprep_B, t.qprep_Bnorm, rcols, t.m,
                       rpad, rcols, rcols, Pq, best, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (ntiles > 0) {
    dim3 grid((unsigned)ntiles, (unsigned)((nq + BM - 1) / BM));
    hipLaunchKernelGGL(k_pivot_scores, grid, dim3(256), 0, s, Q, nq, t.qprep_B, t.qprep_Bnorm,
                       rcols, rcols + t.npiv, t.m, best, ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int wpb = 4;
  hipLaunchKernelGGL(k_qfinish, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb), 0, s, Q,
                     nq, t.m, t.qprep_B, rcols, t.piv_ids, t.npiv, best, ntiles, qq,
                     ntiles > 0 ? entries : nullptr);
  return hipGetLastError();
}

// ------------------------------------------------------------ exact kNN

namespace {

constexpr int kKnnSlack = 32;

// Each block: 64 queries x a contiguous range of data columns.  The running
// best KK (approximate d2, id) per query live in LDS as sorted lists.
__global__ void __launch_bounds__(256) k_knn_tiles(const float* Q, int64_t nq, const float* X,
                                                   int64_t n, int K, const float* qn,
                                                   const float* xn, int KK, int64_t chunk,
                                                   uint64_t* out, int nchunks) {
  extern __shared__ __align__(16) char smem[];
  float* As = reinterpret_cast<float*>(smem);
  float* Bs = As + BM * LDT;
  uint64_t* lists = reinterpret_cast<uint64_t*>(smem + 2 * BM * LDT * sizeof(float));
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
    tile_mma(Q, nq, X, cend, K, r0, c0, As, Bs, acc);
    __syncthreads();
    float* Ct = As;  // 64 x 65 tile of approximate d2
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
          if (row < nq && col < cend) d = fmaxf(qn[row] + xn[col] - 2.f * acc[i][j][v], 0.f);
          Ct[rr * 65 + cl] = d;
        }
    __syncthreads();
    for (int rr = w; rr < BM; rr += 4) {
      uint64_t* L = lists + rr * KK;
      const int cnt = cnts[rr];
      const uint64_t worst = cnt < KK ? ~0ull : L[KK - 1];
      const float d = Ct[rr * 65 + l];
      const uint64_t key = (d < __int_as_float(0x7f800000)) ? make_key(d, (int)(c0 + l)) : ~0ull;
      const bool in = key < worst;
      const uint64_t bm = ballot(in);
      const int na = popc64(bm);
      if (na == 0) continue;
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
                            int nchunks, const uint64_t* cand, int32_t* ids, float* dist) {
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
  (void)metric;
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
  const int lds = 2 * BM * LDT * (int)sizeof(float) + BM * KK * 8 + BM * 4 + 4 * 64 * 8;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_knn_tiles),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)nch, (unsigned)((nq + BM - 1) / BM));
  hipLaunchKernelGGL(k_knn_tiles, grid, dim3(256), lds, s, Q, nq, data, n, m, qn, xn, KK, chunk,
                     cand, nch);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int wpb = 2;
  const int flds = wpb * (nch * KK + 2 * KK) * 8;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_knn_final),
                          hipFuncAttributeMaxDynamicSharedMemorySize, flds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_knn_final, dim3((unsigned)((nq + wpb - 1) / wpb)), dim3(64 * wpb), flds, s,
                     Q, nq, data, m, k, KK, nch, cand, ids, dist);
  return hipGetLastError();
}

}  // namespace finger
