// Flat proximity graph on the GPU: the k nearest other points of every
// point (the exact kNN kernels with k + 1 and the point itself dropped),
// symmetrization by two stable radix sorts of the 2nk directed edges (by
// target, then by (source, distance)), HNSW's neighbour-selection heuristic
// for rows longer than the degree cap (one wavefront per row), and the
// pieces of the reachability repair (BFS levels and the nearest reached node
// with a free slot).  The repair's outer loop runs on the host (api.hip):
// each step depends on the previous one.
//
// Edge e of the 2nk directed edges: e < nk is the kNN edge (e / k -> ids[e])
// and e >= nk the reverse of kNN edge e - nk.  Both carry the kNN list's
// distance, a float32 sum of squared differences whose value does not depend
// on the direction, so a pair listed from both ends sorts into adjacent
// equal entries and the duplicate is dropped.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace finger {
namespace {

struct Edge {
  uint32_t src, dst;
  float d;
};

__device__ __forceinline__ Edge edge_of(uint32_t e, int64_t nk, int k, const int32_t* ids,
                                        const float* dk) {
  Edge r;
  if ((int64_t)e < nk) {
    r.src = e / (uint32_t)k;
    r.dst = (uint32_t)ids[e];
    r.d = dk[e];
  } else {
    const uint32_t f = e - (uint32_t)nk;
    r.src = (uint32_t)ids[f];
    r.dst = f / (uint32_t)k;
    r.d = dk[f];
  }
  return r;
}

// row i of a query batch starting at point `first`
__global__ void k_drop_self(const int32_t* ids1, const float* d1, int64_t n, int k1, int k,
                            int32_t* ids, float* dk, int64_t first, int64_t id_offset) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = 0;
  for (int t = 0; t < k1 && o < k; ++t) {
    const int32_t v = ids1[i * k1 + t];
    if (v == (int32_t)(first + i)) continue;
    ids[i * k + o] = (int32_t)(v + id_offset);
    dk[i * k + o] = d1[i * k1 + t];
    ++o;
  }
}

__global__ void k_keys_dst(int64_t ne, int64_t nk, int k, const int32_t* ids, const float* dk,
                           uint32_t* keys, uint32_t* vals) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  keys[e] = edge_of((uint32_t)e, nk, k, ids, dk).dst;
  vals[e] = (uint32_t)e;
}

__global__ void k_keys_src_d(int64_t ne, int64_t nk, int k, const int32_t* ids, const float* dk,
                             const uint32_t* perm, uint64_t* keys) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ne) return;
  const Edge g = edge_of(perm[x], nk, k, ids, dk);
  keys[x] = ((uint64_t)g.src << 32) | order_bits(g.d);
}

// flag[x] = 1 unless sorted edge x repeats the (source, target) of x - 1;
// cnt[source] counts the kept edges of each row
__global__ void k_dedupe(int64_t ne, int64_t nk, int k, const int32_t* ids, const float* dk,
                         const uint32_t* perm, uint32_t* flag, uint32_t* cnt) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ne) return;
  const Edge g = edge_of(perm[x], nk, k, ids, dk);
  uint32_t f = 1;
  if (x > 0) {
    const Edge p = edge_of(perm[x - 1], nk, k, ids, dk);
    f = (p.src != g.src || p.dst != g.dst) ? 1u : 0u;
  }
  flag[x] = f;
  if (f) atomicAdd(&cnt[g.src], 1u);
}

__global__ void k_fill_rows(int64_t ne, int64_t nk, int k, const int32_t* ids, const float* dk,
                            const uint32_t* perm, const uint32_t* flag, const uint32_t* pos,
                            int32_t* nbr, float* nd) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= ne || flag[x] == 0) return;
  const Edge g = edge_of(perm[x], nk, k, ids, dk);
  nbr[pos[x]] = (int32_t)g.dst;
  nd[pos[x]] = g.d;
}

template <int G, int T4>
__device__ __forceinline__ void load_vec(const float4* data, int m4, int id, int lg, bool valid,
                                         float4 (&v)[T4]) {
  const float4* row = data + (int64_t)(valid ? id : 0) * m4;
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const int j = lg + G * t;
    v[t] = (valid && j < m4) ? row[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <int G, int T4>
__device__ __forceinline__ float sq_dist(const float4 (&a)[T4], const float4 (&b)[T4]) {
  float acc = 0.f;
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const float dx = a[t].x - b[t].x, dy = a[t].y - b[t].y;
    const float dz = a[t].z - b[t].z, dw = a[t].w - b[t].w;
    acc += dx * dx + dy * dy + dz * dz + dw * dw;
  }
  return group_sum<G>(acc);
}

// One wavefront per row.  Short rows are copied; a long row is scanned in
// (distance, id) order and a candidate kept iff fewer than W are kept and it
// is strictly closer to the base than to every kept neighbour.  Lane t holds
// the t-th kept id.
template <int G, int T4>
__global__ __launch_bounds__(256) void k_prune(const float4* data, int64_t n, int m4,
                                               const uint32_t* indptr, const int32_t* nbr,
                                               const float* nd, int W, int32_t* out) {
  constexpr int NPAR = 64 / G;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (i >= n) return;
  const int lg = lane % G, grp = lane / G;
  const uint32_t off = indptr[i];
  const int deg = (int)(indptr[i + 1] - off);
  int32_t* row = out + i * W;
  if (deg <= W) {
    for (int t = lane; t < W; t += 64) row[t] = t < deg ? nbr[off + t] : -1;
    return;
  }
  int kept = -1;
  int kc = 0;
  for (int c = 0; c < deg && kc < W; ++c) {
    const int id = uniform_i(nbr[off + c]);
    const float dc = uniform_f(nd[off + c]);
    float4 xc[T4];
    load_vec<G, T4>(data, m4, id, lg, true, xc);
    bool reject = false;
    for (int p0 = 0; p0 < kc && !reject; p0 += NPAR) {
      const int t = p0 + grp;
      const bool valid = t < kc;
      const int kid = shfl_i(kept, valid ? t : 0);
      float4 xt[T4];
      load_vec<G, T4>(data, m4, kid, lg, valid, xt);
      const float dd = sq_dist<G, T4>(xc, xt);
      reject = ballot(valid && !(dc < dd)) != 0;
    }
    if (!reject) {
      if (lane == kc) kept = id;
      ++kc;
    }
  }
  for (int t = lane; t < W; t += 64) row[t] = t < kc ? kept : -1;
}

__global__ void k_degrees(const int32_t* G, int64_t n, int W, int32_t* deg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = 0;
  for (int t = 0; t < W; ++t) d += G[i * W + t] >= 0 ? 1 : 0;
  deg[i] = d;
}

__global__ void k_bfs_level(const int32_t* G, int W, const int32_t* frontier, int64_t fsize,
                            uint32_t* reached, int32_t* next, uint32_t* next_count) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= fsize * W) return;
  const int64_t f = frontier[idx / W];
  const int32_t v = G[f * W + idx % W];
  if (v >= 0 && atomicExch(&reached[v], 1u) == 0u) next[atomicAdd(next_count, 1u)] = v;
}

// smallest (squared distance to u, id) over reached nodes with a free slot
template <int G, int T4>
__global__ __launch_bounds__(256) void k_nearest_free(const float4* data, int64_t n, int m4, int u,
                                                      const uint32_t* reached, const int32_t* deg,
                                                      int W, unsigned long long* best) {
  constexpr int NPAR = 64 / G;
  __shared__ uint64_t red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lg = lane % G, grp = lane / G;
  float4 xu[T4];
  load_vec<G, T4>(data, m4, u, lg, true, xu);
  uint64_t mine = ~0ull;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t b = ((int64_t)blockIdx.x * (blockDim.x / 64) + w) * NPAR; b < n; b += waves * NPAR) {
    const int64_t v = b + grp;
    const bool ok = v < n && reached[v] != 0u && deg[v] < W;
    float4 xv[T4];
    load_vec<G, T4>(data, m4, (int)v, lg, ok, xv);
    const float d = sq_dist<G, T4>(xu, xv);
    if (ok) {
      const uint64_t key = make_key(d, (int)v);
      mine = key < mine ? key : mine;
    }
  }
  if constexpr (G < 64) { const uint64_t o = shfl_xor_u64(mine, G); mine = o < mine ? o : mine; }
  if constexpr (G < 32) { const uint64_t o = shfl_xor_u64(mine, 2 * G); mine = o < mine ? o : mine; }
  if (lane == 0) red[w] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t b = red[0];
    for (int t = 1; t < (int)(blockDim.x / 64); ++t) b = red[t] < b ? red[t] : b;
    if (b != ~0ull) atomicMin(best, (unsigned long long)b);
  }
}

inline unsigned blocks_for(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_drop_self(const int32_t* ids1, const float* d1, int64_t n, int k1, int k,
                            int32_t* ids, float* dk, int64_t first, int64_t id_offset, hipStream_t s) {
  hipLaunchKernelGGL(k_drop_self, dim3(blocks_for(n)), dim3(256), 0, s, ids1, d1, n, k1, k, ids, dk,
                     first, id_offset);
  return hipGetLastError();
}

hipError_t launch_sym_keys_dst(int64_t n, int k, const int32_t* ids, const float* dk, uint32_t* keys,
                               uint32_t* vals, hipStream_t s) {
  const int64_t nk = n * k, ne = 2 * nk;
  hipLaunchKernelGGL(k_keys_dst, dim3(blocks_for(ne)), dim3(256), 0, s, ne, nk, k, ids, dk, keys, vals);
  return hipGetLastError();
}

hipError_t launch_sym_keys_src_d(int64_t n, int k, const int32_t* ids, const float* dk,
                                 const uint32_t* perm, uint64_t* keys, hipStream_t s) {
  const int64_t nk = n * k, ne = 2 * nk;
  hipLaunchKernelGGL(k_keys_src_d, dim3(blocks_for(ne)), dim3(256), 0, s, ne, nk, k, ids, dk, perm, keys);
  return hipGetLastError();
}

hipError_t launch_sym_dedupe(int64_t n, int k, const int32_t* ids, const float* dk,
                             const uint32_t* perm, uint32_t* flag, uint32_t* cnt, hipStream_t s) {
  const int64_t nk = n * k, ne = 2 * nk;
  hipLaunchKernelGGL(k_dedupe, dim3(blocks_for(ne)), dim3(256), 0, s, ne, nk, k, ids, dk, perm, flag, cnt);
  return hipGetLastError();
}

hipError_t launch_sym_fill(int64_t n, int k, const int32_t* ids, const float* dk, const uint32_t* perm,
                           const uint32_t* flag, const uint32_t* pos, int32_t* nbr, float* nd,
                           hipStream_t s) {
  const int64_t nk = n * k, ne = 2 * nk;
  hipLaunchKernelGGL(k_fill_rows, dim3(blocks_for(ne)), dim3(256), 0, s, ne, nk, k, ids, dk, perm,
                     flag, pos, nbr, nd);
  return hipGetLastError();
}

hipError_t radix_sort_u32(void* tmp, size_t& tmp_bytes, const uint32_t* kin, uint32_t* kout,
                          const uint32_t* vin, uint32_t* vout, int64_t count, int end_bit, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, (int)count, 0,
                                            end_bit, s);
}

hipError_t radix_sort_u64(void* tmp, size_t& tmp_bytes, const uint64_t* kin, uint64_t* kout,
                          const uint32_t* vin, uint32_t* vout, int64_t count, int end_bit, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, kin, kout, vin, vout, (int)count, 0,
                                            end_bit, s);
}

hipError_t exclusive_sum_u32(void* tmp, size_t& tmp_bytes, const uint32_t* in, uint32_t* out,
                             int64_t count, hipStream_t s) {
  return hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, in, out, (int)count, s);
}

hipError_t launch_prune(const float* data, int64_t n, int m, const uint32_t* indptr,
                        const int32_t* nbr, const float* nd, int W, int32_t* out, hipStream_t s) {
  const float4* d4 = reinterpret_cast<const float4*>(data);
  const int m4 = m / 4;
  const dim3 grid(blocks_for(n, 4)), block(256);
#define FINGER_PRUNE(G_, T_) hipLaunchKernelGGL((k_prune<G_, T_>), grid, block, 0, s, d4, n, m4, indptr, nbr, nd, W, out)
  if (m4 <= 16) FINGER_PRUNE(16, 1);
  else if (m4 <= 32) FINGER_PRUNE(16, 2);
  else if (m4 <= 64) FINGER_PRUNE(16, 4);
  else if (m4 <= 128) FINGER_PRUNE(16, 8);
  else if (m4 <= 256) FINGER_PRUNE(64, 4);
  else FINGER_PRUNE(64, 8);
#undef FINGER_PRUNE
  return hipGetLastError();
}

hipError_t launch_degrees(const int32_t* G, int64_t n, int W, int32_t* deg, hipStream_t s) {
  hipLaunchKernelGGL(k_degrees, dim3(blocks_for(n)), dim3(256), 0, s, G, n, W, deg);
  return hipGetLastError();
}

hipError_t launch_bfs_level(const int32_t* G, int W, const int32_t* frontier, int64_t fsize,
                            uint32_t* reached, int32_t* next, uint32_t* next_count, hipStream_t s) {
  if (fsize == 0) return hipSuccess;
  hipLaunchKernelGGL(k_bfs_level, dim3(blocks_for(fsize * W)), dim3(256), 0, s, G, W, frontier, fsize,
                     reached, next, next_count);
  return hipGetLastError();
}

hipError_t launch_nearest_free(const float* data, int64_t n, int m, int u, const uint32_t* reached,
                               const int32_t* deg, int W, unsigned long long* best, hipStream_t s) {
  const float4* d4 = reinterpret_cast<const float4*>(data);
  const int m4 = m / 4;
  const dim3 grid((unsigned)std::min<int64_t>(4096, (n + 15) / 16)), block(256);
#define FINGER_NEAR(G_, T_) hipLaunchKernelGGL((k_nearest_free<G_, T_>), grid, block, 0, s, d4, n, m4, u, reached, deg, W, best)
  if (m4 <= 16) FINGER_NEAR(16, 1);
  else if (m4 <= 32) FINGER_NEAR(16, 2);
  else if (m4 <= 64) FINGER_NEAR(16, 4);
  else if (m4 <= 128) FINGER_NEAR(16, 8);
  else if (m4 <= 256) FINGER_NEAR(64, 4);
  else FINGER_NEAR(64, 8);
#undef FINGER_NEAR
  return hipGetLastError();
}

}  // namespace finger
