// Batched greedy graph search (Algorithm 1) and FINGER's approximate greedy
// search (Algorithm 4 with the estimate of Algorithm 3 in the factorized
// form of Supplementary G), one wavefront per query.
//
// Per-wave state:
//   T      the best ef_eff keys (d2, id) found so far, sorted; bit 31 of an
//          id marks "expanded".  The unexpanded entries of T play the role
//          of the candidate queue C.  Up to ef_max = 64, T sits in registers
//          (lane i holds entry i); longer lists sit in LDS, where every entry
//          below a running index (hint) is expanded, so the search for the
//          next centre starts there.
// and in LDS:
//   V      the visited set: open addressing with linear probing over
//          buckets of four slots; a probe run longer than vis_probe slots
//          continues in a per-wave table in the workspace; when both are
//          full the query reports an overflow.
//   w      P q_res for the current centre (screening only).
//   scratch compacted neighbour ids / flags, the query and P q.
//
// One expansion:
//   1. pick the best unexpanded entry c of T;
//   2. one round trip brings c's adjacency row (one id per lane), and when
//      screening: c.c, P c, alpha_d and rho_d of every slot, and (prefetch
//      variant) every slot's edge code;
//   3. test-and-set V for the neighbours;
//   4. screening: w = Pq - alpha_q P c, then per new slot
//      t_hat = w.u_d / |w|, the distribution-matching map and Eq. 2; a slot
//      is skipped iff its estimate exceeds ub = worst d2 of T at the start of
//      the expansion (the non-prefetch variants load codes of new slots
//      only, after step 3).  The coalesced layout reads 1 KB of the centre's
//      code block per load instruction; the per-lane layout gives each lane
//      32 consecutive elements of one slot's code;
//   5. gather the survivors' vectors (G lanes per vector, float4 loads) and
//      reduce (q - x)^2 across the group;
//   6. merge admitted keys into T by rank (ballots over T, broadcast reads
//      of the few new keys), no sort.
// Loads whose lanes are conditional are raw buffer loads with the masked
// lanes sent past the end of the buffer, not loads inside branches: the
// compiler merges the wait counts of the paths around a branched load,
// which made later work wait for loads it does not use.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

constexpr uint32_t kExpanded = 0x80000000u;
// FINGER search that also writes the gate-training log (internal mode)
constexpr int kModeLog = 3;

// code elements one lane holds: 32 (128 bytes of fp32, 64 of bf16, 32 of
// fp8), so a rank-64 code is two lanes and a screen of 32 slots one pass
template <int CODE>
constexpr int chunk_elems() { return 32; }
__host__ __device__ inline int chunk_elems_rt(int) { return 32; }

struct KArgs {
  const float* data;
  const int32_t* graph;
  int64_t n;
  int m, m4, deg;
  const float* queries;
  int64_t nq;
  // FINGER tables
  int r, rpad;
  int cpr;    // lanes (code chunks) per code row = rpad / chunk_elems
  int spp;    // slots per screening pass = 64 / cpr
  const float* cc;
  const float* pc;
  const float* alpha;
  const float* rho;
  const void* codes;
  const float* scale;
  float mu, dm_scale, mu_hat, eps;
  // per-query inputs
  const float* qq;
  const float* pq;
  const int32_t* entries;
  int entry;
  const int32_t* kq;
  const int32_t* efq;
  int k_all, ef_all, k_max, ef_max, warmup;
  // outputs
  int32_t* out_ids;
  float* out_dist;
  int32_t* counters;
  // scheduling / scratch
  int32_t* queue;
  int persistent;
  // one ef class of a partitioned launch: the queries are qlist[0..*qcount);
  // with nclass > 0 instead one launch over all classes, qlist holding class
  // c's queries at qlist + c list_stride and qcount[c] of them, served from
  // the last (largest) class down
  const int32_t* qlist;
  const int32_t* qcount;
  int nclass;
  int64_t list_stride;
  int ip;     // inner-product metric: distance -q.x
  int32_t* spill;
  int spill_slots;
  int vis_cap;
  int vis_buckets;  // LDS buckets of four slots a visited test examines
  int waves_per_block;
  int coalesced;  // FINGER mode: use the coalesced screen where it applies
  int lds_wave_bytes;
  int lds_shared_bytes;
  // gate (weights transposed: W1T [in][H], W2T [H][H], W3 [H]; biases float)
  const uint16_t* gate_w;
  const float* gate_b;
  int gate_in, gate_h;
  float eps_gate;
  float gate_band;  // > 0: the gate decides only edges within gate_band ub^2 of the bound
  // gate-training log
  float* log_x;
  float* log_y;
  int64_t log_cap;
  int64_t* log_count;
};

// Raw buffer resources (stride 0): the fourth descriptor word for gfx9-family
// parts, and a byte offset past any block the kernels describe (such a load
// returns zeros without touching memory).
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufPastEnd = 0x40000000;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, kBufWord3);
}
// 4-byte element i of a buffer, or zero when !valid (no memory access)
__device__ __forceinline__ uint32_t buf_u32(__amdgpu_buffer_rsrc_t r, int i, bool valid) {
  return __builtin_amdgcn_raw_buffer_load_b32(r, valid ? 4 * i : kBufPastEnd, 0, 0);
}

__device__ __forceinline__ uint32_t hash_id(int id) { return (uint32_t)id * 2654435761u; }

// Exact membership test-and-insert.  visit_lds returns 1 if id was new, 0
// if already visited, -1 if its probe run in LDS is full (visit_spill then
// continues it in the workspace table: it sets spilled, and overflow when
// that table is exhausted too, the id then treated as visited).
// The LDS table is probed linearly in buckets of four slots: one 16-byte
// read examines a bucket; an id present there is visited; otherwise the id
// goes into the bucket's first empty slot, and only a full bucket moves the
// probe on.  All lanes claim their slots in the same compare-and-swap (one
// LDS round trip for the wave, whichever slot each lane needs); lanes of one
// bucket saw the same slots empty, so a lane that lost its slot to another
// lane tries the next one.  Slots only ever fill, so an id is always in the
// first empty slot of its probe sequence or before it; lanes with the same
// id see the same bucket and race for the same slot, so an id is inserted
// once.
__device__ __forceinline__ int visit_lds(int id, int* __restrict__ tab, uint32_t cap_mask, int buckets) {
  uint32_t h = (hash_id(id) >> 7) & cap_mask & ~3u;
#pragma unroll 1
  for (int p = 0; p < buckets; ++p) {
    const int4 b = *reinterpret_cast<const int4*>(tab + h);
    if ((b.x == id) | (b.y == id) | (b.z == id) | (b.w == id)) return 0;
#pragma unroll 1
    for (int e = b.x == -1 ? 0 : (b.y == -1 ? 1 : (b.z == -1 ? 2 : (b.w == -1 ? 3 : 4))); e < 4; ++e) {
      const int old = atomicCAS(&tab[h + e], -1, id);
      if (old == -1) return 1;
      if (old == id) return 0;
    }
    h = (h + 4) & cap_mask;
  }
  return -1;
}

// Empty a wave's workspace table (slots: a power of two >= 64, the table
// 16-byte aligned), visible to the wave's later atomics.
__device__ __forceinline__ void clear_spill(int* spill, int slots) {
  int4* t4 = reinterpret_cast<int4*>(spill);
  for (int i = lane_id(); i < slots / 4; i += 64) t4[i] = make_int4(-1, -1, -1, -1);
  __threadfence_block();
}

// The rest of the probe, in the wave's table in the workspace.
__device__ __forceinline__ int visit_spill(int id, int* __restrict__ spill, uint32_t spill_mask, bool& spilled,
                                           bool& overflow) {
  spilled = true;
  uint32_t g = (hash_id(id ^ 0x5bd1e995) >> 5) & spill_mask;
#pragma unroll 1
  for (uint32_t p = 0; p <= spill_mask; ++p) {
    const int old = atomicCAS(&spill[g], -1, id);
    if (old == -1) return 1;
    if (old == id) return 0;
    g = (g + 1) & spill_mask;
  }
  overflow = true;
  return 0;
}

// One lane's 32-element chunk of an edge code, kept in its stored form.
template <int CODE>
struct Chunk;

template <>
struct Chunk<FINGER_CODE_F32> {
  float4 v[8];
  __device__ __forceinline__ void load(const void* base, int64_t elem) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + elem);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = p[i];
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __device__ __forceinline__ float at(int e) const {
    const float4 q = v[e >> 2];
    const int k = e & 3;
    return k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
  }
  __device__ __forceinline__ float dot(const float* __restrict__ w) const {
    const float4* w4 = reinterpret_cast<const float4*>(w);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float4 a = w4[i];
      s += a.x * v[i].x + a.y * v[i].y + a.z * v[i].z + a.w * v[i].w;
    }
    return s;
  }
};

template <>
struct Chunk<FINGER_CODE_BF16> {
  uint4 v[4];
  __device__ __forceinline__ void load(const void* base, int64_t elem) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint16_t*>(base) + elem);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = p[i];
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  __device__ __forceinline__ static float lo(uint32_t x) { return __uint_as_float(x << 16); }
  __device__ __forceinline__ static float hi(uint32_t x) { return __uint_as_float(x & 0xffff0000u); }
  __device__ __forceinline__ float at(int e) const {
    const uint4 q = v[e >> 3];
    const int k = (e & 7) >> 1;
    const uint32_t x = k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
    return (e & 1) ? hi(x) : lo(x);
  }
  __device__ __forceinline__ float dot(const float* __restrict__ w) const {
    const float4* w4 = reinterpret_cast<const float4*>(w);
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 a = w4[2 * i], b = w4[2 * i + 1];
      s += a.x * lo(v[i].x) + a.y * hi(v[i].x) + a.z * lo(v[i].y) + a.w * hi(v[i].y);
      s += b.x * lo(v[i].z) + b.y * hi(v[i].z) + b.z * lo(v[i].w) + b.w * hi(v[i].w);
    }
    return s;
  }
};

template <>
struct Chunk<FINGER_CODE_FP8E4M3> {
  uint4 v[2];
  __device__ __forceinline__ void load(const void* base, int64_t elem) {
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(base) + elem);
    v[0] = p[0];
    v[1] = p[1];
  }
  __device__ __forceinline__ void zero() { v[0] = v[1] = make_uint4(0u, 0u, 0u, 0u); }
  // gfx950's packed conversion decodes OCP E4M3 (two bytes per half word)
  typedef float f2v __attribute__((ext_vector_type(2)));
  __device__ __forceinline__ float at(int e) const {
    const uint4 q = v[e >> 4];
    const int k = (e & 15) >> 2;
    const uint32_t x = k == 0 ? q.x : (k == 1 ? q.y : (k == 2 ? q.z : q.w));
    return e4m3_to_f((uint8_t)(x >> (8 * (e & 3))));
  }
  __device__ __forceinline__ float dot(const float* __restrict__ w) const {
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint32_t x[4] = {v[i].x, v[i].y, v[i].z, v[i].w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 a = reinterpret_cast<const float4*>(w)[4 * i + j];
        const f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[j], false);
        const f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[j], true);
        s += a.x * lo.x + a.y * lo.y + a.z * hi.x + a.w * hi.y;
      }
    }
    return s;
  }
};

// sum over aligned groups of g lanes, g a runtime power of two <= 64
__device__ __forceinline__ float group_sum_rt(float v, int g) {
  if (g >= 2) v += dpp_f<kDppXor1>(v);
  if (g >= 4) v += dpp_f<kDppXor2>(v);
  if (g >= 8) v += dpp_f<kDppHalfMirror>(v);
  if (g >= 16) v += dpp_f<kDppMirror>(v);
  if (g >= 32) v += shfl_xor_f(v, 16);
  if (g >= 64) v += shfl_xor_f(v, 32);
  return v;
}

// ------------------------------------------------ coalesced screening
// FINGER mode with code rows of at most 256 bytes and at most 32 slots per
// node: a node's codes are one contiguous block of deg x CB bytes, and load
// instruction i of a screen covers its bytes [1024 i, 1024 i + 1024): lane
// l holds the 16 bytes at 1024 i + 16 l, i.e. piece p = l % LC of slot
// i SPI + l / LC (LC = CB / 16 lanes per code, SPI = 64 / LC codes per
// instruction).  Every lane multiplies its pieces with the same FE-element
// fragment of w (held in registers) and the LC / 2 partial dot products of
// a group of LC lanes are summed by a transposed butterfly of DPP moves
// inside the group, after which lane p of the group holds the full dot
// product of instruction p / 2, i.e. of slot (p / 2) SPI + l / LC.
template <int CODE>
constexpr int code_esz() { return CODE == FINGER_CODE_F32 ? 4 : (CODE == FINGER_CODE_BF16 ? 2 : 1); }

// partial dot product of one 16-byte piece with the lane's w fragment
template <int CODE>
__device__ __forceinline__ float piece_dot(const uint4& v, const float* __restrict__ w);
template <>
__device__ __forceinline__ float piece_dot<FINGER_CODE_F32>(const uint4& v, const float* __restrict__ w) {
  return w[0] * __uint_as_float(v.x) + w[1] * __uint_as_float(v.y) + w[2] * __uint_as_float(v.z) +
         w[3] * __uint_as_float(v.w);
}
template <>
__device__ __forceinline__ float piece_dot<FINGER_CODE_BF16>(const uint4& v, const float* __restrict__ w) {
  const uint32_t x[4] = {v.x, v.y, v.z, v.w};
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    s += w[2 * j] * __uint_as_float(x[j] << 16) + w[2 * j + 1] * __uint_as_float(x[j] & 0xffff0000u);
  return s;
}
template <>
__device__ __forceinline__ float piece_dot<FINGER_CODE_FP8E4M3>(const uint4& v, const float* __restrict__ w) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const uint32_t x[4] = {v.x, v.y, v.z, v.w};
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const f2v lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[j], false);
    const f2v hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[j], true);
    s += w[4 * j] * lo.x + w[4 * j + 1] * lo.y + w[4 * j + 2] * hi.x + w[4 * j + 3] * hi.y;
  }
  return s;
}

// one butterfly step: K values -> K / 2; the lane whose partner (under the
// DPP pairing CTRL) sits below it keeps the upper half
template <int K, int CTRL>
__device__ __forceinline__ void bfly_split(float* v, bool upper) {
#pragma unroll
  for (int j = 0; j < K / 2; ++j) {
    const float keep = upper ? v[j + K / 2] : v[j];
    const float send = upper ? v[j] : v[j + K / 2];
    v[j] = keep + dpp_f<CTRL>(send);
  }
}

// v[0..LC/2): this lane's partials of instructions 0..LC/2-1; returns the
// group's sum for instruction p / 2 (p = lane within the group).  Pairings:
// row_mirror (i <-> 15 - i) splits on bit 3, row_half_mirror (i <-> 7 - i)
// on bit 2, quad swaps on bits 1 and 0.
template <int LC>
__device__ __forceinline__ float bfly_reduce(float* v, int p) {
  if constexpr (LC >= 16) bfly_split<8, kDppMirror>(v, (p & 8) != 0);
  if constexpr (LC >= 8) bfly_split<4, kDppHalfMirror>(v, (p & 4) != 0);
  if constexpr (LC >= 4) bfly_split<2, kDppXor2>(v, (p & 2) != 0);
  return v[0] + dpp_f<kDppXor1>(v[0]);
}

template <int G, int T4>
__device__ __forceinline__ void load_query(const KArgs& a, int64_t qi, float4* qv) {
  const int lg = lane_id() & (G - 1);
  const float4* q4 = reinterpret_cast<const float4*>(a.queries + qi * a.m);
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    const int j = lg + G * t;
    qv[t] = j < a.m4 ? q4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// exact squared distances of the `cnt` ids in ids_lds[0..cnt) to the query;
// lane l (l < cnt) receives the distance of ids_lds[l].  G lanes share one
// vector; NP groups of 64/G vectors are in flight together; each group sum
// is handed to its lane by a cross-lane read (no LDS round trip).
// qv: the query chunks this lane needs, either in registers or (qlds) read
// from the wave's LDS copy of the query when needed
template <int G, int T4, int NP>
__device__ __forceinline__ float exact_dists(const KArgs& a, const float4* qv, const float4* qlds,
                                             const int* __restrict__ ids_lds, int cnt) {
  constexpr int NPP = 64 / G;
  const int l = lane_id();
  const int lg = l & (G - 1);
  const int slot = l / G;
  float mine = 0.f;
  if (a.m4 == G * T4 && !a.ip) {
    // the lanes' pieces cover the vector exactly (m = 512 G T4 / 128): no
    // range tests.  Slots past cnt load the first id's vector again (lines
    // the same instruction already requests) instead of branching; their
    // sums are never handed out.
    for (int p0 = 0; p0 < cnt; p0 += NP * NPP) {
      float4 xv[NP][T4];
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        const int ph = p0 + h * NPP + slot;
        const int id = ids_lds[ph < cnt ? ph : 0];
        const float4* x4 = reinterpret_cast<const float4*>(a.data + (int64_t)id * a.m) + lg;
#pragma unroll
        for (int t = 0; t < T4; ++t) xv[h][t] = x4[G * t];
      }
#pragma unroll
      for (int h = 0; h < NP; ++h) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < T4; ++t) {
          const float4 q = qlds != nullptr ? qlds[lg + G * t] : qv[t];
          const float dx = q.x - xv[h][t].x, dy = q.y - xv[h][t].y;
          const float dz = q.z - xv[h][t].z, dw = q.w - xv[h][t].w;
          acc += dx * dx + dy * dy + dz * dz + dw * dw;
        }
        acc = group_sum<G>(acc);
        const int want = l - p0 - h * NPP;
        const float got = __shfl(acc, (want >= 0 && want < NPP ? want : 0) * G, 64);
        if (want >= 0 && want < NPP) mine = got;
      }
    }
    return mine;
  }
  // Other shapes: every lane loads, with no branch (so that the waits count
  // exactly and one pass's sums overlap the next pass's loads): slots past
  // cnt load the first id's vector again, pieces past m reload the last
  // piece of the vector and are zeroed after the load.
  for (int p0 = 0; p0 < cnt; p0 += NP * NPP) {
    float4 xv[NP][T4];
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      const int ph = p0 + h * NPP + slot;
      const float4* x4 = reinterpret_cast<const float4*>(a.data + (int64_t)ids_lds[ph < cnt ? ph : 0] * a.m);
#pragma unroll
      for (int t = 0; t < T4; ++t) {
        const int j = lg + G * t;
        const float4 v = x4[j < a.m4 ? j : a.m4 - 1];
        xv[h][t] = j < a.m4 ? v : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      float acc = 0.f;
      if (a.ip) {
        // inner-product metric: the distance is -q.x
#pragma unroll
        for (int t = 0; t < T4; ++t) {
          const int j = lg + G * t;
          const float4 q = qlds != nullptr ? (j < a.m4 ? qlds[j] : make_float4(0.f, 0.f, 0.f, 0.f)) : qv[t];
          acc -= q.x * xv[h][t].x + q.y * xv[h][t].y + q.z * xv[h][t].z + q.w * xv[h][t].w;
        }
      } else {
#pragma unroll
        for (int t = 0; t < T4; ++t) {
          const int j = lg + G * t;
          const float4 q = qlds != nullptr ? (j < a.m4 ? qlds[j] : make_float4(0.f, 0.f, 0.f, 0.f)) : qv[t];
          const float dx = q.x - xv[h][t].x, dy = q.y - xv[h][t].y;
          const float dz = q.z - xv[h][t].z, dw = q.w - xv[h][t].w;
          acc += dx * dx + dy * dy + dz * dz + dw * dw;
        }
      }
      acc = group_sum<G>(acc);
      // vector p0 + h NPP + s sits in lanes [s G, s G + G); lane p0 + h NPP + s takes it
      const int want = l - p0 - h * NPP;
      const float got = __shfl(acc, (want >= 0 && want < NPP ? want : 0) * G, 64);
      if (want >= 0 && want < NPP) mine = got;
    }
  }
  return mine;
}

typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  return (uint16_t)(__float_as_uint(round_bf16(f)) >> 16);
}
__device__ __forceinline__ b8v ld_b8(const uint16_t* p) { return *reinterpret_cast<const b8v*>(p); }

// The gate network on E <= 32 edges whose features (bf16, zero padded to
// k1 columns) are rows of featb: 16-row tiles through the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+8) and
// B[8(l/16)..+8)[l%16]; D[4(l/16)+v][l%16]), float32 accumulation, hidden
// activations rounded to bf16 after the ReLU (the training kernels' rule).
// b1v[nt] is b1 + W1[:, 0:r] w/|w| for hidden unit 16 nt + l%16 (shared by
// the expansion's edges).  Writes yv[0..E).
__device__ __forceinline__ void gate_tiles(const GateLayout& GL, const uint16_t* __restrict__ W,
                                           const float* __restrict__ B, const float b1v[4],
                                           const uint16_t* __restrict__ featb,
                                           uint16_t* __restrict__ h1b, float* __restrict__ yv,
                                           int E) {
  const int l = lane_id();
  const int lr = l & 15, lk = 8 * (l >> 4), g = l >> 4;
  const int NT = GL.hp / 16;
  const uint16_t* W1e = W + GL.w1e;
  const uint16_t* W2 = W + GL.w2;
  const uint16_t* W3 = W + GL.w3;
  for (int mt = 0; 16 * mt < E; ++mt) {
    f4v acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < GL.k1 / 32; ++ks) {
      const b8v A = ld_b8(featb + (16 * mt + lr) * GL.k1 + 32 * ks + lk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        if (nt < NT)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              A, ld_b8(W1e + (16 * nt + lr) * GL.k1 + 32 * ks + lk), acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
      if (nt < NT)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          h1b[(16 * mt + 4 * g + v) * GL.k2 + 16 * nt + lr] = bf16_bits(fmaxf(acc[nt][v] + b1v[nt], 0.f));
    wave_lds_sync();
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < GL.k2 / 32; ++ks) {
      const b8v A = ld_b8(h1b + (16 * mt + lr) * GL.k2 + 32 * ks + lk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        if (nt < NT)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              A, ld_b8(W2 + (16 * nt + lr) * GL.k2 + 32 * ks + lk), acc[nt], 0, 0, 0);
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      if (nt < NT) {
        const float w3 = bf16_to_f(W3[16 * nt + lr]);
        const float b2 = B[GL.hp + 16 * nt + lr];
#pragma unroll
        for (int v = 0; v < 4; ++v) part[v] += w3 * round_bf16(fmaxf(acc[nt][v] + b2, 0.f));
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) part[v] += shfl_xor_f(part[v], o);
    if (lr == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * mt + 4 * g + v;
        if (row < E) yv[row] = part[v] + B[2 * GL.hp];
      }
    }
    wave_lds_sync();
  }
}

template <int MODE, int CODE, int G, int T4, bool PREFETCH, int LC>
__device__ __forceinline__ void search_body(const KArgs& a) {
  // LC > 0: the coalesced screen (FINGER mode only); the query then stays in
  // registers when a lane needs at most four float4 of it and holds at most
  // four code pieces
  static_assert(LC == 0 || MODE == FINGER_MODE_FINGER, "coalesced screen is for FINGER mode");
  constexpr bool kCoal = LC > 0;
  constexpr bool kQReg = MODE == FINGER_MODE_PLAIN || (kCoal && T4 <= 4 && LC <= 8);
  constexpr int kFE = 16 / code_esz<CODE>();          // code elements per 16-byte piece
  constexpr int kSPI = kCoal ? 64 / LC : 1;           // slots per load instruction
  constexpr int kNI = kCoal ? LC / 2 : 1;             // load instructions for 32 slots
  extern __shared__ __align__(16) char smem[];
  const int l = lane_id();
  // wave-uniform values are kept in scalar registers (readfirstlane), so the
  // address arithmetic that depends only on them runs on the scalar unit
  const int wib = uniform_i(threadIdx.x / 64);
  char* base = smem + a.lds_shared_bytes + wib * a.lds_wave_bytes;
  // T: [ef_max] distances, then [ef_max] ids with the expanded bit (merged
  // in place).  Pointers are formed from the LDS base so that the compiler
  // keeps them in the LDS address space (ds_read/ds_write, not flat)
  float* TD = reinterpret_cast<float*>(base);
  int* TI = reinterpret_cast<int*>(base + 4 * a.ef_max);
  // V starts 16-byte aligned (its buckets are read 16 bytes at a time)
  const int t_bytes = (8 * a.ef_max + 15) & ~15;
  int* vis = reinterpret_cast<int*>(base + t_bytes);
  int* cid = reinterpret_cast<int*>(base + t_bytes + 4 * a.vis_cap);
  int* cflag = reinterpret_cast<int*>(cid + 64);
  float* wv = reinterpret_cast<float*>(cflag + 64);  // [rpad] (screening)
  float* pqv = wv + a.rpad;                          // [rpad] this query's Pq
  float4* qsh = reinterpret_cast<float4*>(pqv + a.rpad);  // [m] the query (screening modes)
  float* feat = reinterpret_cast<float*>(qsh) + (MODE != FINGER_MODE_PLAIN ? a.m : 0);
  // gated: feat = [spp][r + 4], then [64] hidden
  // the other screening modes keep the query in LDS (registers go to the screen)
  const float4* qlds = kQReg ? nullptr : qsh;

  const uint16_t* gw = nullptr;
  const float* gb = nullptr;
  GateLayout GL{};
  uint16_t* featb = nullptr;  // gated: per-wave edge features [32][k1] bf16
  uint16_t* h1b = nullptr;    // gated: hidden activations [32][k2] bf16
  float* yv = nullptr;        // gated: outputs [32]
  if constexpr (MODE == FINGER_MODE_GATED) {
    // the packed weights (about 29 KB at r = 64, 64 hidden units) are read
    // through the caches: every wave of the CU reads the same lines, and
    // LDS stays with the per-query state (more resident waves)
    GL = gate_layout(a.r, a.gate_h);
    gw = a.gate_w;
    gb = a.gate_b;
    featb = reinterpret_cast<uint16_t*>(feat);
    h1b = featb + 32 * GL.k1;
    yv = reinterpret_cast<float*>(h1b + 32 * GL.k2);
    // the padding columns must read as zero (they meet zero weights)
    for (int i = l; i < 32 * (GL.k1 + GL.k2); i += 64) featb[i] = 0;
    wave_lds_sync();
  }

  const int wave_global = blockIdx.x * a.waves_per_block + wib;
  const int total_waves = gridDim.x * a.waves_per_block;
  int* spill = a.spill + (int64_t)wave_global * a.spill_slots;
  const uint32_t cap_mask = (uint32_t)a.vis_cap - 1u;
  const uint32_t spill_mask = (uint32_t)a.spill_slots - 1u;
  bool spill_ready = false;  // this wave's workspace table has been emptied
  // screening lane roles: code lanes hold chunk ch of slot (p0 + l / cpr)
  constexpr int kChunk = chunk_elems<CODE>();
  const int cpr = a.cpr;
  const int csub = l / cpr;
  const int ch = l - csub * cpr;

  // edge-code chunk, zeroed once so that lanes whose slot is not loaded hold
  // defined values; their dot products are masked out
  Chunk<CODE> code;
  code.zero();
  // coalesced screen: piece lp of the codes of slots i kSPI + lg, and the
  // slot whose decision this lane computes
  const int lp = kCoal ? l % (kCoal ? LC : 1) : 0;
  const int lg = kCoal ? l / (kCoal ? LC : 1) : 0;
  const int myslot = (lp >> 1) * kSPI + lg;

  int64_t nq_here = a.nq;
  if (a.nclass > 0) {
    nq_here = 0;
    for (int c = 0; c < a.nclass; ++c) nq_here += uniform_i(a.qcount[c]);
  } else if (a.qcount != nullptr) {
    nq_here = uniform_i(*a.qcount);
  }
  for (int64_t it = 0;; ++it) {
    int64_t qi;
    if (a.persistent) {
      int got = 0;
      if (l == 0) got = atomicAdd(a.queue, 1);
      qi = uniform_i(__shfl(got, 0, 64));
    } else {
      qi = (int64_t)wave_global + it * total_waves;
    }
    if (qi >= nq_here) break;
    if (a.nclass > 0) {
      // queue position -> query, the largest ef class first
      int64_t r = qi;
      for (int c = a.nclass - 1; c >= 0; --c) {
        const int64_t cn = uniform_i(a.qcount[c]);
        if (r < cn) {
          qi = uniform_i(a.qlist[c * a.list_stride + r]);
          break;
        }
        r -= cn;
      }
    } else if (a.qlist != nullptr) {
      qi = uniform_i(a.qlist[qi]);
    }

    const int k = a.kq ? a.kq[qi] : a.k_all;
    const int ef = a.efq ? a.efq[qi] : a.ef_all;
    int status = 0;
    int ef_eff = max(ef, k);
    if (ef_eff > a.ef_max) {
      ef_eff = a.ef_max;
      status |= 2;
    }

    float4 qv[kQReg ? T4 : 1];
    if constexpr (kQReg) {
      load_query<G, T4>(a, qi, qv);
    } else {
      const float4* q4 = reinterpret_cast<const float4*>(a.queries + qi * a.m);
      for (int j = l; j < a.m4; j += 64) qsh[j] = q4[j];
    }
    float qq = 0.f;
    if constexpr (MODE != FINGER_MODE_PLAIN) {
      qq = a.qq[qi];
      for (int i = l; i < a.rpad; i += 64) pqv[i] = a.pq[qi * a.rpad + i];
    }

    for (int i = l; i < a.vis_cap; i += 64) vis[i] = -1;
    wave_lds_sync();
    bool spilled = false, overflow = false;

    const int entry = a.entries ? a.entries[qi] : a.entry;
    if (l == 0) {
      // (the table was just emptied: the entry lands in its first bucket)
      visit_lds(entry, vis, cap_mask, a.vis_buckets);
      cid[0] = entry;
    }
    wave_lds_sync();
    const float d_entry = exact_dists<G, T4, 1>(a, qv, qlds, cid, 1);
    // T lives in registers when it fits one entry per lane (ef_max <= 64):
    // lane i holds entry i as td (distance) and ti (id with the expanded
    // bit); selection and merge then read no memory.  Larger lists live in
    // LDS (TD, TI) and are scanned and merged in blocks of 64.
    const bool treg = a.ef_max <= 64;
    float td = d_entry;
    int ti = entry;
    if (!treg && l == 0) {
      TD[0] = d_entry;
      TI[0] = entry;
    }
    wave_lds_sync();
    int tn = 1;
    int n_exp = 0, n_exact = 1, n_scr = 0, n_skip = 0, n_vis = 1, n_prep = 0;
    int hint = 0;  // LDS list: every entry of T below this index is expanded

    while (true) {
      // 1. the best unexpanded entry of T (in LDS: scanning from the block
      // that holds index hint)
      int j = -1, cur = -1;
      float dcur, ub2;
      if (treg) {
        const uint64_t bm = ballot(l < tn && ((uint32_t)ti & kExpanded) == 0u);
        if (bm == 0ull) break;
        j = __ffsll((unsigned long long)bm) - 1;
        cur = __builtin_amdgcn_readlane(ti, j);
        dcur = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(td), j));
        ub2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(td), tn - 1));
        if (l == j) ti = (int)((uint32_t)ti | kExpanded);
      } else {
        for (int b0 = hint & ~63; b0 < tn; b0 += 64) {
          const int i = b0 + l;
          const int raw = i < tn ? TI[i] : (int)kExpanded;
          const uint64_t bm = ballot(((uint32_t)raw & kExpanded) == 0u);
          if (bm) {
            const int s0 = __ffsll((unsigned long long)bm) - 1;
            j = b0 + s0;
            cur = __builtin_amdgcn_readlane(raw, s0);
            break;
          }
        }
        if (j < 0) break;
        hint = j + 1;
        dcur = uniform_f(TD[j]);
        ub2 = uniform_f(TD[tn - 1]);
        wave_lds_sync();
        if (l == 0) TI[j] = (int)((uint32_t)cur | kExpanded);
      }
      ++n_exp;

      const bool screening = (MODE != FINGER_MODE_PLAIN) && n_exp > a.warmup && tn == ef_eff;
      // 2. one round trip: adjacency (+ screening inputs)
      // (buffer loads answer lanes past the degree with zeros and no access;
      // with no branch around them the waits below count exactly which
      // loads they need)
      int nb = (int)buf_u32(buf_rsrc(a.graph + (int64_t)cur * a.deg, 4 * a.deg), l, l < a.deg);
      if (l >= a.deg) nb = -1;
      float al = 0.f, rh = 0.f, ccv = 0.f;
      // P c of the centre, element l + 64 t in pcv[t] (rpad <= 256), read in
      // this round trip so that forming w below waits on no memory access
      // (a wait there would also drain the code loads issued before it)
      float pcv[4] = {0.f, 0.f, 0.f, 0.f};
      // coalesced screen: this lane's piece of P c, the fp8 scale, and the
      // code pieces (zero where not loaded, so that nothing carries over
      // from one expansion to the next)
      float pcf[kCoal ? kFE : 1];
      float sclv = 1.f;
      uint4 craw[kNI];
#pragma unroll
      for (int i = 0; i < kNI; ++i) craw[i] = make_uint4(0u, 0u, 0u, 0u);
      if constexpr (kCoal) {
        // requested on every expansion, with every lane masked off when this
        // one does not screen: no branch, so the wait for the row below
        // leaves these in flight through the visited test
        al = __uint_as_float(buf_u32(buf_rsrc(a.alpha + (int64_t)cur * a.deg, 4 * a.deg), myslot,
                                     screening && myslot < a.deg));
        rh = __uint_as_float(buf_u32(buf_rsrc(a.rho + (int64_t)cur * a.deg, 4 * a.deg), myslot,
                                     screening && myslot < a.deg));
        ccv = __uint_as_float(buf_u32(buf_rsrc(a.cc + cur, 4), 0, screening));
        const __amdgpu_buffer_rsrc_t pcr = buf_rsrc(a.pc + (int64_t)cur * a.rpad, 4 * a.rpad);
#pragma unroll
        for (int t = 0; t < kFE / 4; ++t) {
          const float4 v = __builtin_bit_cast(
              float4, __builtin_amdgcn_raw_buffer_load_b128(pcr, screening ? 4 * (lp * kFE + 4 * t) : kBufPastEnd,
                                                            0, 0));
          pcf[4 * t] = v.x;
          pcf[4 * t + 1] = v.y;
          pcf[4 * t + 2] = v.z;
          pcf[4 * t + 3] = v.w;
        }
        if constexpr (CODE == FINGER_CODE_FP8E4M3)
          sclv = __uint_as_float(buf_u32(buf_rsrc(a.scale + cur, 4), 0, screening));
        if constexpr (PREFETCH) {
          const __amdgpu_buffer_rsrc_t cbr = buf_rsrc(
              static_cast<const char*>(a.codes) + (int64_t)cur * a.deg * (LC * 16), a.deg * (LC * 16));
#pragma unroll
          for (int i = 0; i < kNI; ++i)
            craw[i] = __builtin_bit_cast(
                uint4, __builtin_amdgcn_raw_buffer_load_b128(
                           cbr, screening && i * kSPI + lg < a.deg ? (64 * i + l) * 16 : kBufPastEnd, 0, 0));
        }
      } else if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) {
          if (csub < a.deg) {
            al = a.alpha[(int64_t)cur * a.deg + csub];
            rh = a.rho[(int64_t)cur * a.deg + csub];
            if constexpr (PREFETCH)
              code.load(a.codes, ((int64_t)cur * a.deg + csub) * a.rpad + ch * kChunk);
          }
          ccv = a.cc[cur];
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (l + 64 * t < a.rpad) pcv[t] = a.pc[(int64_t)cur * a.rpad + l + 64 * t];
        }
      }
      // 3. visited test-and-set
      int isnew = 0;
      if (nb >= 0) isnew = visit_lds(nb, vis, cap_mask, a.vis_buckets);
      if (ballot(isnew < 0) != 0ull) {
        // the wave's workspace table holds whatever the caller's memory held
        // until the wave first needs it; it is emptied then, and every query
        // that used it empties it again at its end
        if (!spill_ready) {
          clear_spill(spill, a.spill_slots);
          spill_ready = true;
        }
        if (isnew < 0) isnew = visit_spill(nb, spill, spill_mask, spilled, overflow);
      }
      const uint64_t newm = ballot(isnew != 0);
      const int S = popc64(newm);
      n_vis += S;
      if (S == 0) continue;

      uint64_t survm = newm;
      bool logging = false;
      int64_t log_base = 0;
      if constexpr (kCoal) {
        if (screening) {
          // 4. screening, coalesced: codes of the new slots (unless requested
          // with the adjacency row), one 1 KB span of the block per instruction
          n_scr += S;
          ++n_prep;
          if constexpr (!PREFETCH) {
            // buffer loads over this node's code block: a lane whose slot is
            // not new reads past the block's end, which the hardware answers
            // with zeros and no memory access.  No branch surrounds the loads,
            // so forming w below waits only for the row's screening inputs
            // while the codes are in flight.
            const __amdgpu_buffer_rsrc_t cbr = buf_rsrc(
                static_cast<const char*>(a.codes) + (int64_t)cur * a.deg * (LC * 16), a.deg * (LC * 16));
            // (newm has no bit at or past the row's degree: those lanes hold no id)
#pragma unroll
            for (int i = 0; i < kNI; ++i) {
              const bool ld = (newm >> (i * kSPI + lg)) & 1ull;
              craw[i] = __builtin_bit_cast(
                  uint4, __builtin_amdgcn_raw_buffer_load_b128(cbr, ld ? (64 * i + l) * 16 : kBufPastEnd, 0, 0));
            }
          }
          // query side (Section 3.2 and Supplementary G), as below; w is
          // formed piecewise: this lane's kFE elements of Pq - alpha_q P c
          const float qc = a.ip ? -dcur : 0.5f * (qq + ccv - dcur);
          const float aq = ccv > 0.f ? qc / ccv : 0.f;
          const float rq2 = fmaxf(qq - aq * qc, 0.f);
          const float rq = sqrtf(rq2);
          float wf[kFE];
          float w2 = 0.f;
          const float4* pq4 = reinterpret_cast<const float4*>(pqv + lp * kFE);
#pragma unroll
          for (int t = 0; t < kFE / 4; ++t) {
            const float4 q = pq4[t];
            wf[4 * t] = q.x - aq * pcf[4 * t];
            wf[4 * t + 1] = q.y - aq * pcf[4 * t + 1];
            wf[4 * t + 2] = q.z - aq * pcf[4 * t + 2];
            wf[4 * t + 3] = q.w - aq * pcf[4 * t + 3];
          }
#pragma unroll
          for (int e = 0; e < kFE; ++e) w2 += wf[e] * wf[e];
          w2 = group_sum<LC>(w2);
          const float inv_w = w2 > 0.f ? 1.0f / sqrtf(w2) : 0.f;
          float part[kNI];
#pragma unroll
          for (int i = 0; i < kNI; ++i) part[i] = piece_dot<CODE>(craw[i], wf);
          const float dot = bfly_reduce<LC>(part, lp);
          // Algorithm 3 and Eq. 2 for slot myslot (lanes with even lp decide)
          const bool slot_new = myslot < a.deg && ((newm >> myslot) & 1ull);
          const float t_hat = dot * sclv * inv_w;
          const float t = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
          const float da = aq - al;
          const float est = a.ip ? -(aq * al * ccv + rq * rh * t) : da * da * ccv + rq2 + rh * rh - 2.f * rq * rh * t;
          const int skip_here = (slot_new && est > ub2) ? 1 : 0;
          // adjacency lane s takes the decision of lane (s % kSPI) LC + 2 (s / kSPI)
          const int src = l < a.deg ? (l % kSPI) * LC + 2 * (l / kSPI) : 0;
          const bool skip_l = __shfl(skip_here, src, 64) != 0;
          const bool keep = isnew && !skip_l;
          survm = ballot(keep);
          n_skip += S - popc64(survm);
        }
      } else if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) {
          // 4. screening
          n_scr += S;
          ++n_prep;
          // codes of the new slots of the first pass (slot csub), unless
          // requested with the adjacency row; chunks of visited or padding
          // slots keep stale values, their dot products are masked out
          if constexpr (!PREFETCH) {
            if (csub < a.deg && ((newm >> csub) & 1ull))
              code.load(a.codes, ((int64_t)cur * a.deg + csub) * a.rpad + ch * kChunk);
          }
          // query side (Section 3.2 and Supplementary G): q.c from the exact
          // d2 of the centre, alpha_q, |q_res|^2, w = Pq - alpha_q P c
          // (inner-product metric: T holds -q.c itself)
          const float qc = a.ip ? -dcur : 0.5f * (qq + ccv - dcur);
          const float aq = ccv > 0.f ? qc / ccv : 0.f;
          const float rq2 = fmaxf(qq - aq * qc, 0.f);
          const float rq = sqrtf(rq2);
          float w2 = 0.f;
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int i = l + 64 * t;
            if (i < a.rpad) {
              const float w = pqv[i] - aq * pcv[t];
              wv[i] = w;
              w2 += w * w;
            }
          }
          w2 = wave_sum(w2);
          const float inv_w = w2 > 0.f ? 1.0f / sqrtf(w2) : 0.f;
          const float scl = (CODE == FINGER_CODE_FP8E4M3) ? a.scale[cur] : 1.f;
          const float ub = sqrtf(ub2);
          const float inv_ub = ub > 0.f ? 1.f / ub : 0.f;
          logging = (MODE == kModeLog);
          if (logging) {
            unsigned long long got = 0;
            if (l == 0) got = atomicAdd((unsigned long long*)a.log_count, (unsigned long long)S);
            log_base = (int64_t)shfl_u64((uint64_t)got, 0);
          }
          wave_lds_sync();
          float b1v[4] = {0.f, 0.f, 0.f, 0.f};
          if constexpr (MODE == FINGER_MODE_GATED) {
            // shared part of the gate's first layer, b1 + W1[:, 0:r] w/|w|,
            // one lane per hidden unit, then spread to the MFMA column layout
            float base1 = 0.f;
            if (l < GL.hp) {
              base1 = gb[l];
              for (int i = 0; i < a.r; ++i) base1 += bf16_to_f(gw[i * GL.hp + l]) * round_bf16(wv[i] * inv_w);
            }
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) b1v[nt] = __shfl(base1, 16 * nt + (l & 15), 64);
          }
          bool skip_l = false;  // the decision for this lane's adjacency slot
          // one screening pass over slots [p0, p0 + spp): this lane holds
          // chunk ch of slot p0 + csub in cd, with that slot's alpha and rho
          auto screen_pass = [&](int p0, const Chunk<CODE>& cd, float al, float rh) {
            const int slot = p0 + csub;
            const bool slot_new = slot < a.deg && ((newm >> slot) & 1ull);
            const Chunk<CODE>& code = cd;
            const float dot = group_sum_rt(slot_new ? code.dot(wv + ch * kChunk) : 0.f, cpr);
            const float t_hat = dot * scl * inv_w;
            const float da = aq - al;
            const float proj = da * da * ccv;
            float t;
            if (MODE == kModeLog && slot_new) {
              const int64_t row = log_base + popc64(newm & ((1ull << slot) - 1ull));
              if (row < a.log_cap) {
                // features in the layout finger_gate_attach documents
                float* x = a.log_x + row * (int64_t)(2 * a.r + 4);
                for (int e = 0; e < kChunk; ++e) {
                  const int idx = ch * kChunk + e;
                  if (idx < a.r) {
                    x[idx] = wv[idx] * inv_w;
                    x[a.r + idx] = code.at(e) * scl;
                  }
                }
                if (ch == 0) {
                  x[2 * a.r] = t_hat;
                  x[2 * a.r + 1] = rq * inv_ub;
                  x[2 * a.r + 2] = rh * inv_ub;
                  x[2 * a.r + 3] = proj * inv_ub * inv_ub;
                }
              }
            }
            if constexpr (MODE == FINGER_MODE_GATED) {
              // Algorithm 3's matched cosine first; with a band, the gate
              // decides only the edges whose matched estimate lies within
              // gate_band ub^2 of the bound (the others keep Algorithm 3's
              // decision), without a band every new edge.  The gated edges
              // of this pass become the rows of a feature tile (compacted in
              // slot order) evaluated on the matrix cores; a pass without
              // one skips the network.
              const float t_dm = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
              const float est_dm = proj + rq2 + rh * rh - 2.f * rq * rh * t_dm;
              const bool gated_edge = slot_new && (a.gate_band <= 0.f || fabsf(est_dm - ub2) <= a.gate_band * ub2);
              // one bit per gated slot, at the slot's first lane
              const uint64_t gm = ballot(gated_edge && ch == 0);
              const int E = popc64(gm);
              const int row = gated_edge ? popc64(gm & ((1ull << (csub * cpr)) - 1ull)) : 0;
              if (E > 0) {
                if (gated_edge) {
                  uint16_t* fr = featb + row * GL.k1;
                  for (int e = 0; e < kChunk; ++e) {
                    const int idx = ch * kChunk + e;
                    if (idx < a.r) fr[idx] = bf16_bits(code.at(e) * scl);
                  }
                  if (ch == 0) {
                    fr[a.r] = bf16_bits(t_hat);
                    fr[a.r + 1] = bf16_bits(rq * inv_ub);
                    fr[a.r + 2] = bf16_bits(rh * inv_ub);
                    fr[a.r + 3] = bf16_bits(proj * inv_ub * inv_ub);
                  }
                }
                wave_lds_sync();
                gate_tiles(GL, gw, gb, b1v, featb, h1b, yv, E);
                t = gated_edge ? yv[row] + a.eps_gate : t_dm;
                wave_lds_sync();
              } else {
                t = t_dm;
              }
            } else {
              t = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
            }
            // Eq. 2 (L2), or -(q_proj.d_proj + |q_res| |d_res| t) (inner product)
            const float est = a.ip ? -(aq * al * ccv + rq * rh * t)
                                   : proj + rq2 + rh * rh - 2.f * rq * rh * t;
            // skip iff the estimate exceeds ub (both squared); slot s of this
            // pass is decided in lane (s - p0) cpr and handed to lane s
            const int rel = l - p0;
            const bool in_pass = rel >= 0 && rel < a.spp;
            const int sk = __shfl(est > ub2 ? 1 : 0, (in_pass ? rel : 0) * cpr, 64);
            if (in_pass) skip_l = sk != 0;
          };
          screen_pass(0, code, al, rh);
          if (a.spp < a.deg) {
            // further passes (r > 64: more slots than one pass holds) load as they go
            for (int p0 = a.spp; p0 < a.deg; p0 += a.spp) {
              const int slot = p0 + csub;
              float alx = 0.f, rhx = 0.f;
              if (slot < a.deg) {
                alx = a.alpha[(int64_t)cur * a.deg + slot];
                rhx = a.rho[(int64_t)cur * a.deg + slot];
              }
              if (slot < a.deg && ((newm >> slot) & 1ull))
                code.load(a.codes, ((int64_t)cur * a.deg + slot) * a.rpad + ch * kChunk);
              screen_pass(p0, code, alx, rhx);
            }
          }
          // back in adjacency lanes
          const bool keep = isnew && !skip_l;
          survm = ballot(keep);
          n_skip += S - popc64(survm);
          if (logging) {
            // every screened edge gets its exact distance for the log; the
            // skip decision is kept per compacted position for admission
            const int rk = mask_rank(newm);
            wave_lds_sync();
            if (isnew) {
              cid[rk] = nb;
              cflag[rk] = keep ? 0 : 1;
            }
            survm = newm;
            wave_lds_sync();
          }
        }
      }
      // compact the survivors into cid (logging did it already)
      if (!logging) {
        wave_lds_sync();
        if ((survm >> l) & 1ull) cid[mask_rank(survm)] = nb;
        wave_lds_sync();
      }
      const int S2 = popc64(survm);
      if (S2 == 0) continue;
      // 5. exact distances of the survivors
      // plain search keeps two passes of vectors in flight; after screening
      // few neighbours survive and one pass is enough
      const float dmine = exact_dists<G, T4, MODE == FINGER_MODE_PLAIN ? 2 : 1>(a, qv, qlds, cid, S2);

      // 6. admission: lanes 0..S2-1 hold (dmine, cid)
      uint64_t key = ~0ull;
      bool adm = false;
      bool was_skipped = false;
      const uint64_t worst_key =
          treg ? make_key(__int_as_float(__builtin_amdgcn_readlane(__float_as_int(td), tn - 1)),
                          (int)((uint32_t)__builtin_amdgcn_readlane(ti, tn - 1) & ~kExpanded))
               : make_key(uniform_f(TD[tn - 1]), uniform_i((int)((uint32_t)TI[tn - 1] & ~kExpanded)));
      if (l < S2) {
        if (logging) {
          was_skipped = cflag[l] != 0;
          const int64_t row = log_base + l;
          if (row < a.log_cap) {
            a.log_y[2 * row] = dmine;
            a.log_y[2 * row + 1] = ub2;
          }
        }
        key = make_key(dmine, cid[l]);
        adm = !was_skipped && (tn < ef_eff || key < worst_key);
      }
      n_exact += S2 - popc64(ballot(was_skipped));
      const uint64_t am = ballot(adm);
      const int NA = popc64(am);
      if (NA == 0) continue;
      // merge in place, by ranks, with the new keys read across lanes: T
      // entry i moves right by the number of new keys below it; a new key
      // lands at (new keys below it) + (T keys below it).  Blocks of 64
      // entries go from the last one down, so that every entry is read
      // before anything lands on it (entries only move right); the blocks
      // wholly below the smallest new key keep their places untouched.
      int my_pos = 0;
      if (treg) {
        // T in registers: a new key's place is (new keys below it) + (T keys
        // below it); lane p then takes the new key placed at p, or else T
        // entry p - (new keys placed below p), read across lanes
        const uint64_t tk = l < tn ? make_key(td, (int)((uint32_t)ti & ~kExpanded)) : ~0ull;
        for (uint64_t mm = am; mm; mm &= mm - 1ull) {
          const int src = __ffsll((unsigned long long)mm) - 1;
          const uint64_t kj = readlane_u64(key, src);
          my_pos += kj < key ? 1 : 0;
          const int below = popc64(ballot(tk < kj));
          if (l == src) my_pos += below;
        }
        uint64_t placed = 0ull, nk = 0ull;
        for (uint64_t mm = am; mm; mm &= mm - 1ull) {
          const int src = __ffsll((unsigned long long)mm) - 1;
          const int pos = __builtin_amdgcn_readlane(my_pos, src);
          if (pos < ef_eff) {
            placed |= 1ull << pos;
            const uint64_t kj = readlane_u64(key, src);
            if (l == pos) nk = kj;
          }
        }
        const int from = l - popc64(placed & ((1ull << l) - 1ull));
        const float od = __shfl(td, from, 64);
        const int oi = __shfl(ti, from, 64);
        const bool mine_new = ((placed >> l) & 1ull) != 0ull;
        td = mine_new ? key_d2(nk) : od;
        ti = mine_new ? key_id(nk) : oi;
        tn = min(tn + NA, ef_eff);
        continue;
      }
      uint64_t kmin = ~0ull;
      int kmin_src = 0;
      for (uint64_t mm = am; mm; mm &= mm - 1ull) {
        const int src = __ffsll((unsigned long long)mm) - 1;
        const uint64_t kj = readlane_u64(key, src);
        my_pos += kj < key ? 1 : 0;
        if (kj < kmin) {
          kmin = kj;
          kmin_src = src;
        }
      }
      for (int b0 = (tn - 1) & ~63; b0 >= 0; b0 -= 64) {
        const int i = b0 + l;
        const bool valid = i < tn;
        const int raw = valid ? TI[i] : 0;
        const float d = valid ? TD[i] : 0.f;
        const uint64_t tk = valid ? make_key(d, (int)((uint32_t)raw & ~kExpanded)) : ~0ull;
        const int last = min(tn - b0, 64) - 1;
        if (readlane_u64(tk, last) < kmin) {
          // this block and those before it lie below every new key
          my_pos += b0 + last + 1;
          break;
        }
        int shift = 0;
        for (uint64_t mm = am; mm; mm &= mm - 1ull) {
          const int src = __ffsll((unsigned long long)mm) - 1;
          const uint64_t kj = readlane_u64(key, src);
          shift += kj < tk ? 1 : 0;
          const int below = popc64(ballot(tk < kj));
          if (l == src) my_pos += below;
        }
        if (valid && shift > 0 && i + shift < ef_eff) {
          TD[i + shift] = d;
          TI[i + shift] = raw;
        }
      }
      if (adm && my_pos < ef_eff) {
        TD[my_pos] = key_d2(key);
        TI[my_pos] = key_id(key);
      }
      // entries below the smallest new key's place did not move
      hint = min(hint, __builtin_amdgcn_readlane(my_pos, kmin_src));
      tn = min(tn + NA, ef_eff);
      wave_lds_sync();
    }

    // output: the first k keys of T
    {
      for (int jx = l; jx < a.k_max; jx += 64) {
        int id = -1;
        float d = __int_as_float(0x7f800000);
        if (jx < k && jx < tn) {
          // (T in registers: tn <= 64, so jx is this lane's entry)
          id = (int)((uint32_t)(treg ? ti : TI[jx]) & ~kExpanded);
          d = treg ? td : TD[jx];
        }
        a.out_ids[qi * a.k_max + jx] = id;
        a.out_dist[qi * a.k_max + jx] = d;
      }
    }
    const bool any_over = ballot(overflow) != 0ull;
    const bool any_spill = ballot(spilled) != 0ull;
    if (a.counters != nullptr && l == 0) {
      int32_t* c = a.counters + qi * FINGER_NCOUNTERS;
      c[0] = n_exp;
      c[1] = n_exact;
      c[2] = n_scr;
      c[3] = n_skip;
      c[4] = n_vis;
      c[5] = n_prep;
      c[6] = status | (any_over ? 1 : 0);
    }
    if (any_spill) {
      // leave the spill table empty for the next query on this wave slot
      clear_spill(spill, a.spill_slots);
    }
    wave_lds_sync();
  }
}

template <int MODE, int CODE, int G, int T4, bool PF, int LC>
__global__ void __launch_bounds__(256) k_search(KArgs a) {
  search_body<MODE, CODE, G, T4, PF, LC>(a);
}

// FINGER screening: hold the register budget of four waves per SIMD (the
// search is latency bound, so resident waves matter more than a few spills)
template <int MODE, int CODE, int G, int T4, bool PF, int LC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_search_w4(KArgs a) {
  search_body<MODE, CODE, G, T4, PF, LC>(a);
}

template <typename F>
hipError_t launch_fn(F fn, const KArgs& a, int blocks, int lds, hipStream_t s) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * a.waves_per_block), lds, s, a);
  return hipGetLastError();
}

template <int MODE, int CODE, int G, int T4, bool PF, int LC>
hipError_t launch_k(const KArgs& a, int blocks, int lds, hipStream_t s) {
  // the register cap applies up to m = 512; beyond, a vector needs 8 float4
  // per lane and the capped build spills heavily (there it also returned
  // run-to-run differing results with BF16 codes requested ahead, so the
  // uncapped build is used)
  if constexpr (MODE == FINGER_MODE_FINGER && G < 64)
    return launch_fn(k_search_w4<MODE, CODE, G, T4, PF, LC>, a, blocks, lds, s);
  else
    return launch_fn(k_search<MODE, CODE, G, T4, PF, LC>, a, blocks, lds, s);
}

template <int MODE, int CODE, bool PF, int LC>
hipError_t launch_dims_lc(const KArgs& a, int blocks, int lds, hipStream_t s) {
  if (a.m4 <= 32) return launch_k<MODE, CODE, 8, 4, PF, LC>(a, blocks, lds, s);
  if (a.m4 <= 128) return launch_k<MODE, CODE, 32, 4, PF, LC>(a, blocks, lds, s);
  return launch_k<MODE, CODE, 64, 8, PF, LC>(a, blocks, lds, s);
}

template <int MODE, int CODE, bool PF>
hipError_t launch_dims(const KArgs& a, int blocks, int lds, hipStream_t s) {
  if constexpr (MODE == FINGER_MODE_FINGER) {
    // the coalesced screen where a code row is 32..256 bytes and a node has
    // at most 32 slots
    const int cb = a.rpad * code_esz<CODE>();
    if (a.coalesced && a.deg <= 32) {
      if (cb == 256) return launch_dims_lc<MODE, CODE, PF, 16>(a, blocks, lds, s);
      if (cb == 128) return launch_dims_lc<MODE, CODE, PF, 8>(a, blocks, lds, s);
      if constexpr (CODE != FINGER_CODE_F32) {
        if (cb == 64) return launch_dims_lc<MODE, CODE, PF, 4>(a, blocks, lds, s);
      }
      if constexpr (CODE == FINGER_CODE_FP8E4M3) {
        if (cb == 32) return launch_dims_lc<MODE, CODE, PF, 2>(a, blocks, lds, s);
      }
    }
  }
  return launch_dims_lc<MODE, CODE, PF, 0>(a, blocks, lds, s);
}

template <int MODE, bool PF>
hipError_t launch_codes_pf(const KArgs& a, int code, int blocks, int lds, hipStream_t s) {
  if (code == FINGER_CODE_BF16) return launch_dims<MODE, FINGER_CODE_BF16, PF>(a, blocks, lds, s);
  if (code == FINGER_CODE_FP8E4M3) return launch_dims<MODE, FINGER_CODE_FP8E4M3, PF>(a, blocks, lds, s);
  return launch_dims<MODE, FINGER_CODE_F32, PF>(a, blocks, lds, s);
}

// PF_ALLOWED false: the mode always loads codes after the visited test
template <int MODE, bool PF_ALLOWED = true>
hipError_t launch_codes(const KArgs& a, int code, bool pf, int blocks, int lds, hipStream_t s) {
  if constexpr (PF_ALLOWED)
    if (pf) return launch_codes_pf<MODE, true>(a, code, blocks, lds, s);
  return launch_codes_pf<MODE, false>(a, code, blocks, lds, s);
}

int wave_bytes(int ef_max, int vis_cap, int r, int m, int gate_in) {
  const int rpad = rpad_of(r);
  int b = ((8 * ef_max + 15) & ~15) + 4 * vis_cap + 64 * 4 * 2 + 8 * rpad + (r > 0 ? 4 * m : 0);
  if (gate_in > 0) {
    // edge features [32][k1] and hidden activations [32][k2] in bf16, outputs [32]
    const GateLayout GL = gate_layout(r, 64);
    b += 2 * 32 * (GL.k1 + GL.k2) + 4 * 32;
  }
  return (b + 15) & ~15;
}

void fill_common(KArgs& a, const Tables& t) {
  a.ip = t.metric == FINGER_IP ? 1 : 0;
  a.data = t.data;
  a.graph = t.graph;
  a.n = t.n;
  a.m = t.m;
  a.m4 = t.m / 4;
  a.deg = t.deg;
  a.r = t.r;
  a.rpad = rpad_of(t.r);
  a.cpr = a.rpad > 0 ? a.rpad / chunk_elems_rt(t.code_type) : 1;
  a.spp = 64 / a.cpr;
  a.cc = t.cc;
  a.pc = t.pc;
  a.alpha = t.alpha;
  a.rho = t.rho;
  a.codes = t.codes;
  a.scale = t.scale;
  a.mu = (float)t.mu;
  a.dm_scale = (float)(t.sigma_hat > 0 ? t.sigma / t.sigma_hat : 1.0);
  a.mu_hat = (float)t.mu_hat;
  a.eps = (float)t.eps;
}

}  // namespace

int search_lds_bytes(int ef_max, int vis_cap, int r, int m, int gate_in) {
  return wave_bytes(ef_max, vis_cap, r, m, gate_in);
}

bool search_prefetch_supported(const Tables& t) {
  // the first screening pass covers every slot, so all codes can be issued
  // with the adjacency row
  return t.r > 0 && t.deg <= 64 / (rpad_of(t.r) / chunk_elems_rt(t.code_type));
}

hipError_t launch_search(const Tables& t, const SearchLaunch& L, hipStream_t s) {
  KArgs a{};
  fill_common(a, t);
  a.queries = L.queries;
  a.nq = L.nq;
  a.qq = L.qq;
  a.pq = L.pq;
  a.entries = L.entries;
  a.entry = L.entry;
  a.kq = L.kq;
  a.efq = L.efq;
  a.k_all = L.k_all;
  a.ef_all = L.ef_all;
  a.k_max = L.k_max;
  a.ef_max = L.ef_max;
  a.warmup = L.warmup;
  a.out_ids = L.out_ids;
  a.out_dist = L.out_dist;
  a.counters = L.counters;
  a.queue = L.queue;
  a.persistent = L.persistent;
  a.qlist = L.qlist;
  a.qcount = L.qcount;
  a.nclass = L.nclass;
  a.list_stride = L.list_stride;
  a.spill = L.spill;
  a.spill_slots = L.spill_slots_per_wave;
  a.vis_cap = L.vis_cap;
  a.vis_buckets = L.vis_probe / 4;
  a.log_x = L.log_x;
  a.log_y = L.log_y;
  a.log_cap = L.log_cap;
  a.log_count = L.log_count;
  const bool gated = L.mode == FINGER_MODE_GATED;
  a.gate_w = gated ? t.gate_w : nullptr;
  a.gate_b = gated ? t.gate_b : nullptr;
  a.gate_in = gated ? t.gate_in : 0;
  a.gate_h = gated ? t.gate_h : 0;
  a.eps_gate = (float)t.eps_gate;
  a.gate_band = L.gate_band;
  // one query wave per workgroup keeps LDS allocation fine grained
  a.waves_per_block = 1;
  a.coalesced = L.coalesced;
  a.lds_shared_bytes = 0;
  a.lds_wave_bytes = wave_bytes(L.ef_max, L.vis_cap, L.mode == FINGER_MODE_PLAIN ? 0 : t.r, t.m,
                                gated ? a.gate_in : 0);
  const int lds = a.lds_shared_bytes + a.waves_per_block * a.lds_wave_bytes;
  const int blocks = (L.waves + a.waves_per_block - 1) / a.waves_per_block;
  const bool pf = L.prefetch && search_prefetch_supported(t);
  if (L.mode == FINGER_MODE_PLAIN)
    return launch_dims<FINGER_MODE_PLAIN, FINGER_CODE_F32, false>(a, blocks, lds, s);
  if (L.mode == FINGER_MODE_FINGER && L.log_x != nullptr)
    return launch_codes<kModeLog>(a, t.code_type, pf, blocks, lds, s);
  if (L.mode == FINGER_MODE_FINGER) return launch_codes<FINGER_MODE_FINGER>(a, t.code_type, pf, blocks, lds, s);
  return launch_codes<FINGER_MODE_GATED, false>(a, t.code_type, false, blocks, lds, s);
}

// ------------------------------------------------------ ef classes

namespace {

// One block: every query's class (the first bound >= its ef_eff = max(ef,
// K), the last class for anything above), appended to that class's list
// lists[c nq ..] (order inside a class is not fixed: a query's search does
// not depend on the others); counts[c] and the lists drive the per-class
// launches.
__global__ void __launch_bounds__(1024) k_ef_classes(const int32_t* __restrict__ kq,
                                                     const int32_t* __restrict__ efq, int64_t nq,
                                                     int k_all, int ef_all, ClassBounds cb,
                                                     int32_t* __restrict__ counts,
                                                     int32_t* __restrict__ lists) {
  __shared__ int cnt[kMaxEfClasses];
  const int t = threadIdx.x;
  if (t < kMaxEfClasses) cnt[t] = 0;
  __syncthreads();
  for (int64_t i = t; i < nq; i += blockDim.x) {
    const int k = kq ? kq[i] : k_all;
    const int ef = efq ? efq[i] : ef_all;
    const int e = ef > k ? ef : k;
    int c = 0;
    while (c + 1 < cb.n && e > cb.bound[c]) ++c;
    lists[(int64_t)c * nq + atomicAdd(&cnt[c], 1)] = (int32_t)i;
  }
  __syncthreads();
  if (t < cb.n) counts[t] = cnt[t];
}

}  // namespace

hipError_t launch_ef_classes(const int32_t* kq, const int32_t* efq, int64_t nq, int k_all, int ef_all,
                             const ClassBounds& cb, int32_t* counts, int32_t* lists, hipStream_t s) {
  hipLaunchKernelGGL(k_ef_classes, dim3(1), dim3(1024), 0, s, kq, efq, nq, k_all, ef_all, cb, counts, lists);
  return hipGetLastError();
}

// ------------------------------------------------- estimate test kernel

namespace {
// One wave per (query, centre, slot) item, computing exactly what the
// search's screening step computes for that edge.
template <int CODE>
__global__ void k_estimate_edges(KArgs a, const int32_t* qi, const int32_t* ci,
                                 const int32_t* si, int64_t items, float* est, float* that) {
  extern __shared__ __align__(16) float wsm[];
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  float* wv = wsm + (threadIdx.x / 64) * a.rpad;
  if (item >= items) return;
  const int l = lane_id();
  const int q = qi[item], c = ci[item], slot = si[item];
  // the exact d2(q, c) the search has in T
  const float4* q4 = reinterpret_cast<const float4*>(a.queries + (int64_t)q * a.m);
  const float4* c4 = reinterpret_cast<const float4*>(a.data + (int64_t)c * a.m);
  float acc = 0.f;
  for (int j = l; j < a.m4; j += 64) {
    const float4 x = q4[j], y = c4[j];
    if (a.ip) {
      acc -= x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
    } else {
      const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
      acc += dx * dx + dy * dy + dz * dz + dw * dw;
    }
  }
  const float dcur = wave_sum(acc);
  const float qq = a.qq[q];
  const float ccv = a.cc[c];
  const float qc = a.ip ? -dcur : 0.5f * (qq + ccv - dcur);
  const float aq = ccv > 0.f ? qc / ccv : 0.f;
  const float rq2 = fmaxf(qq - aq * qc, 0.f);
  const float rq = sqrtf(rq2);
  float w2 = 0.f;
  for (int e = l; e < a.rpad; e += 64) {
    const float w = a.pq[(int64_t)q * a.rpad + e] - aq * a.pc[(int64_t)c * a.rpad + e];
    wv[e] = w;
    w2 += w * w;
  }
  w2 = wave_sum(w2);
  wave_lds_sync();
  const float inv_w = w2 > 0.f ? 1.0f / sqrtf(w2) : 0.f;
  float dot = 0.f;
  constexpr int kChunk = chunk_elems<CODE>();
  if (l < a.cpr) {
    Chunk<CODE> code;
    code.load(a.codes, ((int64_t)c * a.deg + slot) * a.rpad + l * kChunk);
    dot = code.dot(wv + l * kChunk);
  }
  dot = wave_sum(dot);
  const float scl = (CODE == FINGER_CODE_FP8E4M3) ? a.scale[c] : 1.f;
  const float t_hat = dot * scl * inv_w;
  const float ad = a.alpha[(int64_t)c * a.deg + slot];
  const float rd = a.rho[(int64_t)c * a.deg + slot];
  const float t = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
  const float da = aq - ad;
  if (l == 0) {
    est[item] = a.ip ? -(aq * ad * ccv + rq * rd * t) : da * da * ccv + rq2 + rd * rd - 2.f * rq * rd * t;
    that[item] = t_hat;
  }
}
}  // namespace

hipError_t launch_estimate_edges(const Tables& t, const float* Q, const float* qq,
                                 const float* Pq, const int32_t* qi, const int32_t* ci,
                                 const int32_t* si, int64_t items, float* est, float* that,
                                 hipStream_t s) {
  if (items == 0) return hipSuccess;
  KArgs a{};
  fill_common(a, t);
  a.queries = Q;
  a.qq = qq;
  a.pq = Pq;
  const int wpb = 4;
  const int blocks = (int)((items + wpb - 1) / wpb);
  const int lds = wpb * a.rpad * 4;
  if (t.code_type == FINGER_CODE_BF16)
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_BF16>, dim3(blocks), dim3(64 * wpb), lds, s, a,
                       qi, ci, si, items, est, that);
  else if (t.code_type == FINGER_CODE_FP8E4M3)
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_FP8E4M3>, dim3(blocks), dim3(64 * wpb), lds, s,
                       a, qi, ci, si, items, est, that);
  else
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_F32>, dim3(blocks), dim3(64 * wpb), lds, s, a,
                       qi, ci, si, items, est, that);
  return hipGetLastError();
}

}  // namespace finger
