// Start points from the upper layers of an HNSW-style hierarchy: the greedy
// descent HNSW runs above layer 0 (its layer search with a result list of
// one), for a batch of queries, one wavefront per query.
//
// Per hop the wave reads the current node's row in the current layer (one
// coalesced load of up to 64 ids), evaluates every listed neighbour exactly
// (G lanes per neighbour, float4 loads of the point, DPP group sums), and
// moves to the neighbour of smallest (d, id) key if that key is below the
// current node's; otherwise it drops one layer and keeps the node.  Keys
// strictly decrease, so every layer ends after at most as many hops as it has
// nodes; the hop cap (n per layer) only bounds the loop for the compiler.
// Neighbours seen at an earlier hop are evaluated again (no visited set):
// their keys are above the current node's, so only the evaluation count
// differs from a search that remembers them.
#include <algorithm>

#include "device_common.h"
#include "internal.h"

namespace finger {
namespace {

struct DescendArgs {
  const float4* data;
  const float4* q;
  int64_t nq;
  int m4;
  const int32_t* row0;   // [n] first upper row of each node
  const int32_t* upper;  // [rows][width]
  int width;
  int top_level;
  int top;
  int64_t max_hops;
  int ip;
  int32_t* out;
  int32_t* calls;
};

// distance of this lane group's node (id < 0: none), summed over the group
template <int G, int T4>
__device__ __forceinline__ float group_dist(const DescendArgs& a, const float4 (&qv)[T4],
                                            const float4 (&xv)[T4]) {
  float acc = 0.f;
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    if (a.ip) {
      acc -= qv[t].x * xv[t].x + qv[t].y * xv[t].y + qv[t].z * xv[t].z + qv[t].w * xv[t].w;
    } else {
      const float dx = qv[t].x - xv[t].x, dy = qv[t].y - xv[t].y;
      const float dz = qv[t].z - xv[t].z, dw = qv[t].w - xv[t].w;
      acc += dx * dx + dy * dy + dz * dz + dw * dw;
    }
  }
  return group_sum<G>(acc);
}

template <int G, int T4>
__device__ __forceinline__ void load_point(const DescendArgs& a, int id, int lg, float4 (&xv)[T4]) {
  const float4* row = a.data + (int64_t)(id < 0 ? 0 : id) * a.m4;
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const int j = lg + G * t;
    xv[t] = (id >= 0 && j < a.m4) ? row[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

__device__ __forceinline__ uint64_t min_u64(uint64_t x, uint64_t y) { return x < y ? x : y; }

template <int G, int T4>
__global__ __launch_bounds__(256) void k_descend(DescendArgs a) {
  constexpr int NPAR = 64 / G;   // neighbours per pass
  constexpr int U = 4;           // passes with loads in flight together
  constexpr int CHUNK = NPAR * U;
  const int lane = threadIdx.x & 63;
  const int64_t qi = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (qi >= a.nq) return;  // uniform per wave
  const int lg = lane % G, grp = lane / G;

  float4 qv[T4];
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const int j = lg + G * t;
    qv[t] = j < a.m4 ? a.q[qi * a.m4 + j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }

  int cur = a.top;
  uint64_t ck;
  {
    float4 xv[T4];
    load_point<G, T4>(a, cur, lg, xv);
    ck = make_key(group_dist<G, T4>(a, qv, xv), cur);
    ck = readlane_u64(ck, 0);
  }
  int calls = 1;

  for (int layer = a.top_level; layer >= 1; --layer) {
    for (int64_t hop = 0; hop < a.max_hops; ++hop) {
      const int row = uniform_i(a.row0[cur]) + layer - 1;
      const int32_t* rp = a.upper + (int64_t)row * a.width;
      const int nb = lane < a.width ? rp[lane] : -1;
      calls += popc64(ballot(nb >= 0));
      uint64_t best = ~0ull;
      for (int p0 = 0; p0 < a.width; p0 += CHUNK) {
        int id[U];
        float4 xv[U][T4];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int s = p0 + u * NPAR + grp;
          id[u] = shfl_i(nb, s < 64 ? s : 0);
          if (s >= a.width) id[u] = -1;
          load_point<G, T4>(a, id[u], lg, xv[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const float d = group_dist<G, T4>(a, qv, xv[u]);
          if (id[u] >= 0) best = min_u64(best, make_key(d, id[u]));
        }
      }
      if constexpr (G < 64) best = min_u64(best, shfl_xor_u64(best, G));
      if constexpr (G < 32) best = min_u64(best, shfl_xor_u64(best, 2 * G));
      best = readlane_u64(best, 0);
      if (!(best < ck)) break;
      ck = best;
      cur = key_id(best);
    }
  }
  if (lane == 0) {
    a.out[qi] = cur;
    if (a.calls != nullptr) a.calls[qi] = calls;
  }
}

template <int G, int T4>
hipError_t launch(const DescendArgs& a, hipStream_t s) {
  const int wpb = 4;
  const int64_t blocks = (a.nq + wpb - 1) / wpb;
  hipLaunchKernelGGL((k_descend<G, T4>), dim3((unsigned)blocks), dim3(64 * wpb), 0, s, a);
  return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* p, uint32_t value, size_t count) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = value;
}

}  // namespace

hipError_t launch_fill_u32(void* p, uint32_t value, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const size_t blocks = std::min<size_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s,
                     static_cast<uint32_t*>(p), value, count);
  return hipGetLastError();
}

hipError_t launch_descend(const Tables& t, const float* Q, int64_t nq, int32_t* out, int32_t* calls,
                          hipStream_t s) {
  if (nq == 0) return hipSuccess;
  DescendArgs a;
  a.data = reinterpret_cast<const float4*>(t.data);
  a.q = reinterpret_cast<const float4*>(Q);
  a.nq = nq;
  a.m4 = t.m / 4;
  a.row0 = t.h_row0;
  a.upper = t.h_upper;
  a.width = t.h_width;
  a.top_level = t.h_top_level;
  a.top = t.h_top;
  a.max_hops = t.n;
  a.ip = t.metric == FINGER_IP ? 1 : 0;
  a.out = out;
  a.calls = calls;
  const int m4 = a.m4;
  if (m4 <= 16) return launch<16, 1>(a, s);
  if (m4 <= 32) return launch<16, 2>(a, s);
  if (m4 <= 64) return launch<16, 4>(a, s);
  if (m4 <= 128) return launch<16, 8>(a, s);
  if (m4 <= 256) return launch<64, 4>(a, s);
  return launch<64, 8>(a, s);
}

}  // namespace finger
