// Batched greedy graph search (Algorithm 1) and FINGER's approximate greedy
// search (Algorithm 4 with the estimate of Algorithm 3 in the factorized
// form of Supplementary G), one wavefront per query.
//
// Per-wave state lives in LDS:
//   T      the best ef_eff keys (d2, id) found so far, sorted, double
//          buffered; bit 31 of an id marks "expanded".  The unexpanded
//          entries of T play the role of the candidate queue C.
//   V      the visited set: open addressing with linear probing; a probe
//          run longer than kLdsProbes continues in a per-wave table in the
//          workspace, so the set stays exact.
//   w      P q_res for the current centre (screening only).
//   scratch compacted neighbour ids / distances / admitted keys / flags.
//
// One expansion:
//   1. pick the best unexpanded entry c of T;
//   2. one round trip brings c's adjacency row (one id per lane), and when
//      screening: c.c, P c, alpha_d and rho_d of every slot, and (prefetch
//      variant) every slot's edge code;
//   3. test-and-set V for the neighbours;
//   4. screening: w = Pq - alpha_q P c, then per new slot
//      t_hat = w.u_d / |w| (code chunks of 32 elements, one per lane, w
//      read from LDS), the distribution-matching map and Eq. 2; a slot is
//      skipped iff its estimate exceeds ub = worst d2 of T at the start of
//      the expansion (the non-prefetch variant loads codes of new slots only,
//      after step 3);
//   5. gather the survivors' vectors (G lanes per vector, float4 loads) and
//      reduce (q - x)^2 across the group;
//   6. merge admitted keys into T by rank (ballots over T, broadcast reads of
//      the few new keys), no sort.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

constexpr uint32_t kExpanded = 0x80000000u;
// FINGER search that also writes the gate-training log (internal mode)
constexpr int kModeLog = 3;
constexpr int kLdsProbes = 24;
// code elements one lane holds: 64 bytes of fp32 or bf16, 32 bytes of fp8
template <int CODE>
constexpr int chunk_elems() { return CODE == FINGER_CODE_F32 ? 16 : 32; }
__host__ __device__ inline int chunk_elems_rt(int code) { return code == FINGER_CODE_F32 ? 16 : 32; }

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
  int32_t* spill;
  int spill_slots;
  int vis_cap;
  int waves_per_block;
  int lds_wave_bytes;
  int lds_shared_bytes;
  // gate (weights transposed: W1T [in][H], W2T [H][H], W3 [H]; biases float)
  const uint16_t* gate_w;
  const float* gate_b;
  int gate_in, gate_h;
  float eps_gate;
  // gate-training log
  float* log_x;
  float* log_y;
  int64_t log_cap;
  int64_t* log_count;
};

__device__ __forceinline__ uint32_t hash_id(int id) { return (uint32_t)id * 2654435761u; }

// Exact membership test-and-insert.  Returns 1 if id was new, 0 if already
// visited; sets spilled when the global table was touched, overflow when
// both tables were exhausted (the id is then treated as visited).
__device__ __forceinline__ int visit(int id, int* __restrict__ tab, uint32_t cap_mask,
                                     int* __restrict__ spill, uint32_t spill_mask,
                                     bool& spilled, bool& overflow) {
  uint32_t h = (hash_id(id) >> 7) & cap_mask;
#pragma unroll 1
  for (int p = 0; p < kLdsProbes; ++p) {
    const int old = atomicCAS(&tab[h], -1, id);
    if (old == -1) return 1;
    if (old == id) return 0;
    h = (h + 1) & cap_mask;
  }
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
  float4 v[4];
  __device__ __forceinline__ void load(const void* base, int64_t elem) {
    const float4* p = reinterpret_cast<const float4*>(static_cast<const float*>(base) + elem);
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = p[i];
  }
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
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
    for (int i = 0; i < 4; ++i) {
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
  for (int s = g >> 1; s >= 1; s >>= 1) v += shfl_xor_f(v, s);
  return v;
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
// results go to d_lds[0..cnt).  G lanes share one vector; NP passes of
// 64/G vectors are in flight together.
// qv: the query chunks this lane needs, either in registers or (qlds) read
// from the wave's LDS copy of the query when needed
template <int G, int T4, int NP>
__device__ __forceinline__ void exact_dists(const KArgs& a, const float4* qv, const float4* qlds,
                                            const int* __restrict__ ids_lds, int cnt,
                                            float* __restrict__ d_lds) {
  constexpr int NPP = 64 / G;
  const int l = lane_id();
  const int lg = l & (G - 1);
  const int slot = l / G;
  for (int p0 = 0; p0 < cnt; p0 += NP * NPP) {
    float4 xv[NP][T4];
    int p[NP];
#pragma unroll
    for (int h = 0; h < NP; ++h) p[h] = p0 + h * NPP + slot;
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      if (p[h] < cnt) {
        const float4* x4 = reinterpret_cast<const float4*>(a.data + (int64_t)ids_lds[p[h]] * a.m);
#pragma unroll
        for (int t = 0; t < T4; ++t) {
          const int j = lg + G * t;
          xv[h][t] = j < a.m4 ? x4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int t = 0; t < T4; ++t) xv[h][t] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int h = 0; h < NP; ++h) {
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < T4; ++t) {
        const int j = lg + G * t;
        const float4 q = qlds != nullptr ? (j < a.m4 ? qlds[j] : make_float4(0.f, 0.f, 0.f, 0.f)) : qv[t];
        const float dx = q.x - xv[h][t].x, dy = q.y - xv[h][t].y;
        const float dz = q.z - xv[h][t].z, dw = q.w - xv[h][t].w;
        acc += dx * dx + dy * dy + dz * dz + dw * dw;
      }
      acc = group_sum<G>(acc);
      if (lg == 0 && p[h] < cnt) d_lds[p[h]] = acc;
    }
  }
  wave_lds_sync();
}

// Gate network on one edge: every lane owns one hidden unit (lanes >= H
// idle).  base1 = b1 + W1[:, 0:r] (w/|w|) is shared by the expansion's
// edges; u (r floats) and the 4 scalars s are this edge's features in LDS.
__device__ __forceinline__ float gate_edge(const KArgs& a, const uint16_t* __restrict__ W,
                                           const float* __restrict__ B, float base1,
                                           const float* __restrict__ u, const float* s,
                                           float* __restrict__ hbuf) {
  const int l = lane_id();
  const int H = a.gate_h, r = a.r;
  const uint16_t* W1T = W;                           // [in][H]
  const uint16_t* W2T = W + (int64_t)a.gate_in * H;  // [H][H]
  const uint16_t* W3 = W2T + H * H;                  // [H]
  float z = base1;
  if (l < H) {
    for (int i = 0; i < r; ++i) z += bf16_to_f(W1T[(r + i) * H + l]) * u[i];
#pragma unroll
    for (int c = 0; c < 4; ++c) z += bf16_to_f(W1T[(2 * r + c) * H + l]) * s[c];
  }
  const float h1 = l < H ? round_bf16(fmaxf(z, 0.f)) : 0.f;
  hbuf[l] = h1;
  wave_lds_sync();
  float z2 = l < H ? B[H + l] : 0.f;
  if (l < H)
    for (int i = 0; i < H; ++i) z2 += bf16_to_f(W2T[i * H + l]) * hbuf[i];
  const float h2 = l < H ? round_bf16(fmaxf(z2, 0.f)) : 0.f;
  const float y = wave_sum(l < H ? bf16_to_f(W3[l]) * h2 : 0.f) + B[2 * H];
  wave_lds_sync();
  return y;
}

template <int MODE, int CODE, int G, int T4, bool PREFETCH>
__device__ __forceinline__ void search_body(const KArgs& a) {
  extern __shared__ __align__(16) char smem[];
  const int l = lane_id();
  const int wib = threadIdx.x / 64;
  char* base = smem + a.lds_shared_bytes + wib * a.lds_wave_bytes;
  float* tD[2];
  int* tI[2];
  tD[0] = reinterpret_cast<float*>(base);
  tI[0] = reinterpret_cast<int*>(base + 4 * a.ef_max);
  tD[1] = reinterpret_cast<float*>(base + 8 * a.ef_max);
  tI[1] = reinterpret_cast<int*>(base + 12 * a.ef_max);
  int* vis = reinterpret_cast<int*>(base + 16 * a.ef_max);
  uint64_t* ck = reinterpret_cast<uint64_t*>(base + 16 * a.ef_max + 4 * a.vis_cap);
  int* cid = reinterpret_cast<int*>(ck + 64);
  float* cd = reinterpret_cast<float*>(cid + 64);
  int* cflag = reinterpret_cast<int*>(cd + 64);
  float* wv = reinterpret_cast<float*>(cflag + 64);  // [rpad] (screening)
  float* pqv = wv + a.rpad;                          // [rpad] this query's Pq
  float4* qsh = reinterpret_cast<float4*>(pqv + a.rpad);  // [m] the query (screening modes)
  float* feat = reinterpret_cast<float*>(qsh) + (MODE != FINGER_MODE_PLAIN ? a.m : 0);
  // gated: feat = [spp][r + 4], then [64] hidden
  // screening modes keep the query in LDS (registers go to the screen)
  const float4* qlds = (MODE != FINGER_MODE_PLAIN) ? qsh : nullptr;

  const uint16_t* gw = nullptr;
  const float* gb = nullptr;
  if constexpr (MODE == FINGER_MODE_GATED) {
    uint16_t* sw = reinterpret_cast<uint16_t*>(smem);
    const int nw = a.gate_h * a.gate_in + a.gate_h * a.gate_h + a.gate_h;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) sw[i] = a.gate_w[i];
    float* sb = reinterpret_cast<float*>(smem + ((2 * nw + 15) & ~15));
    for (int i = threadIdx.x; i < 2 * a.gate_h + 1; i += blockDim.x) sb[i] = a.gate_b[i];
    __syncthreads();
    gw = sw;
    gb = sb;
  }

  const int wave_global = blockIdx.x * a.waves_per_block + wib;
  const int total_waves = gridDim.x * a.waves_per_block;
  int* spill = a.spill + (int64_t)wave_global * a.spill_slots;
  const uint32_t cap_mask = (uint32_t)a.vis_cap - 1u;
  const uint32_t spill_mask = (uint32_t)a.spill_slots - 1u;
  // screening lane roles: code lanes hold chunk ch of slot (p0 + l / cpr)
  constexpr int kChunk = chunk_elems<CODE>();
  const int cpr = a.cpr;
  const int csub = l / cpr;
  const int ch = l - csub * cpr;

  for (int64_t it = 0;; ++it) {
    int64_t qi;
    if (a.persistent) {
      int got = 0;
      if (l == 0) got = atomicAdd(a.queue, 1);
      qi = uniform_i(__shfl(got, 0, 64));
    } else {
      qi = (int64_t)wave_global + it * total_waves;
    }
    if (qi >= a.nq) break;

    const int k = a.kq ? a.kq[qi] : a.k_all;
    const int ef = a.efq ? a.efq[qi] : a.ef_all;
    int status = 0;
    int ef_eff = max(ef, k);
    if (ef_eff > a.ef_max) {
      ef_eff = a.ef_max;
      status |= 2;
    }

    float4 qv[MODE == FINGER_MODE_PLAIN ? T4 : 1];
    if constexpr (MODE == FINGER_MODE_PLAIN) {
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
      visit(entry, vis, cap_mask, spill, spill_mask, spilled, overflow);
      cid[0] = entry;
    }
    wave_lds_sync();
    exact_dists<G, T4, 1>(a, qv, qlds, cid, 1, cd);
    int cur_buf = 0;
    if (l == 0) {
      tD[0][0] = cd[0];
      tI[0][0] = entry;
    }
    wave_lds_sync();
    int tn = 1;
    int n_exp = 0, n_exact = 1, n_scr = 0, n_skip = 0, n_vis = 1, n_prep = 0;

    while (true) {
      float* TD = tD[cur_buf];
      int* TI = tI[cur_buf];
      // 1. the best unexpanded entry of T
      int j = -1;
      for (int b0 = 0; b0 < tn; b0 += 64) {
        const int i = b0 + l;
        const bool un = i < tn && ((uint32_t)TI[i] & kExpanded) == 0u;
        const uint64_t bm = ballot(un);
        if (bm) {
          j = b0 + __ffsll((unsigned long long)bm) - 1;
          break;
        }
      }
      if (j < 0) break;
      const int cur = TI[j];
      const float dcur = TD[j];
      const float ub2 = TD[tn - 1];
      wave_lds_sync();
      if (l == 0) TI[j] = (int)((uint32_t)cur | kExpanded);
      ++n_exp;

      const bool screening = (MODE != FINGER_MODE_PLAIN) && n_exp > a.warmup && tn == ef_eff;
      // 2. one round trip: adjacency (+ screening inputs)
      int nb = -1;
      if (l < a.deg) nb = a.graph[(int64_t)cur * a.deg + l];
      float al = 0.f, rh = 0.f, ccv = 0.f, pc0 = 0.f;
      Chunk<CODE> code;
      if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) {
          if (csub < a.deg) {
            al = a.alpha[(int64_t)cur * a.deg + csub];
            rh = a.rho[(int64_t)cur * a.deg + csub];
            if constexpr (PREFETCH)
              code.load(a.codes, ((int64_t)cur * a.deg + csub) * a.rpad + ch * kChunk);
          }
          ccv = a.cc[cur];
          if (l < a.rpad) pc0 = a.pc[(int64_t)cur * a.rpad + l];
        }
      }
      // 3. visited test-and-set
      int isnew = 0;
      if (nb >= 0) isnew = visit(nb, vis, cap_mask, spill, spill_mask, spilled, overflow);
      const uint64_t newm = ballot(isnew != 0);
      const int S = popc64(newm);
      n_vis += S;
      if (S == 0) continue;

      uint64_t survm = newm;
      bool logging = false;
      int64_t log_base = 0;
      if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) {
          // 4. screening
          n_scr += S;
          ++n_prep;
          // query side (Section 3.2 and Supplementary G): q.c from the exact
          // d2 of the centre, alpha_q, |q_res|^2, w = Pq - alpha_q P c
          const float qc = 0.5f * (qq + ccv - dcur);
          const float aq = ccv > 0.f ? qc / ccv : 0.f;
          const float rq2 = fmaxf(qq - aq * qc, 0.f);
          const float rq = sqrtf(rq2);
          float w2 = 0.f;
          for (int i = l; i < a.rpad; i += 64) {
            const float pc = i < 64 ? pc0 : a.pc[(int64_t)cur * a.rpad + i];
            const float w = pqv[i] - aq * pc;
            wv[i] = w;
            w2 += w * w;
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
          float base1 = 0.f;
          if constexpr (MODE == FINGER_MODE_GATED) {
            // shared part of the gate's first layer: b1 + W1[:, 0:r] w/|w|
            if (l < a.gate_h) {
              base1 = gb[l];
              for (int i = 0; i < a.r; ++i) base1 += bf16_to_f(gw[i * a.gate_h + l]) * round_bf16(wv[i] * inv_w);
            }
          }
          for (int p0 = 0; p0 < a.deg; p0 += a.spp) {
            const int slot = p0 + csub;
            const bool slot_new = slot < a.deg && ((newm >> slot) & 1ull);
            if (p0 > 0 && slot < a.deg) {
              al = a.alpha[(int64_t)cur * a.deg + slot];
              rh = a.rho[(int64_t)cur * a.deg + slot];
            }
            if (!PREFETCH || p0 > 0) {
              if (slot_new) code.load(a.codes, ((int64_t)cur * a.deg + slot) * a.rpad + ch * kChunk);
              else code.zero();
            }
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
              // stage this pass's edge features, then run the gate edge by edge
              float* fu = feat + (int64_t)csub * (a.r + 4);
              if (slot_new) {
                for (int e = 0; e < kChunk; ++e) {
                  const int idx = ch * kChunk + e;
                  if (idx < a.r) fu[idx] = round_bf16(code.at(e) * scl);
                }
                if (ch == 0) {
                  fu[a.r] = round_bf16(t_hat);
                  fu[a.r + 1] = round_bf16(rq * inv_ub);
                  fu[a.r + 2] = round_bf16(rh * inv_ub);
                  fu[a.r + 3] = round_bf16(proj * inv_ub * inv_ub);
                }
              }
              wave_lds_sync();
              float* hbuf = feat + (int64_t)a.spp * (a.r + 4);
              const uint64_t pm = ballot(slot_new && ch == 0);
              float mine = 0.f;
              for (uint64_t mm = pm; mm; mm &= mm - 1ull) {
                const int src = __ffsll((unsigned long long)mm) - 1;
                const float* f = feat + (int64_t)(src / cpr) * (a.r + 4);
                const float y = gate_edge(a, gw, gb, base1, f, f + a.r, hbuf);
                if (l == src) mine = y;
              }
              t = mine + a.eps_gate;
            } else {
              t = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
            }
            const float est = proj + rq2 + rh * rh - 2.f * rq * rh * t;
            // skip iff the estimate exceeds ub (both squared)
            if (slot_new && ch == 0) cflag[slot] = est > ub2 ? 1 : 0;
          }
          wave_lds_sync();
          // back in adjacency lanes
          const bool keep = isnew && cflag[l] == 0;
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
      exact_dists<G, T4, MODE == FINGER_MODE_PLAIN ? 2 : 1>(a, qv, qlds, cid, S2, cd);

      // 6. admission: lanes 0..S2-1 hold (cd, cid)
      uint64_t key = ~0ull;
      bool adm = false;
      bool was_skipped = false;
      const uint64_t worst_key = make_key(TD[tn - 1], (int)((uint32_t)TI[tn - 1] & ~kExpanded));
      if (l < S2) {
        const float d = cd[l];
        if (logging) {
          was_skipped = cflag[l] != 0;
          const int64_t row = log_base + l;
          if (row < a.log_cap) {
            a.log_y[2 * row] = d;
            a.log_y[2 * row + 1] = ub2;
          }
        }
        key = make_key(d, cid[l]);
        adm = !was_skipped && (tn < ef_eff || key < worst_key);
      }
      n_exact += S2 - popc64(ballot(was_skipped));
      const uint64_t am = ballot(adm);
      const int NA = popc64(am);
      if (NA == 0) continue;
      wave_lds_sync();
      if (adm) ck[mask_rank(am)] = key;
      wave_lds_sync();
      // ranks: new key jn lands at (#new keys below it) + (#T keys below
      // it); T entry i moves right by the number of new keys below it
      float* ND = tD[cur_buf ^ 1];
      int* NI = tI[cur_buf ^ 1];
      for (int i = l; i < tn; i += 64) {
        const int raw = TI[i];
        const float d = TD[i];
        const uint64_t tk = make_key(d, (int)((uint32_t)raw & ~kExpanded));
        int shift = 0;
        for (int jn = 0; jn < NA; ++jn) shift += ck[jn] < tk ? 1 : 0;  // broadcast reads
        if (i + shift < ef_eff) {
          ND[i + shift] = d;
          NI[i + shift] = raw;
        }
      }
      const uint64_t mykey = l < NA ? ck[l] : ~0ull;
      int my_pos = 0;
      for (int jn = 0; jn < NA; ++jn) {
        const uint64_t kj = ck[jn];
        my_pos += (kj < mykey) ? 1 : 0;
        int below = 0;
        for (int b0 = 0; b0 < tn; b0 += 64) {
          const int i = b0 + l;
          const bool lt = i < tn && make_key(TD[i], (int)((uint32_t)TI[i] & ~kExpanded)) < kj;
          below += popc64(ballot(lt));
        }
        if (l == jn) my_pos += below;
      }
      if (l < NA && my_pos < ef_eff) {
        ND[my_pos] = key_d2(mykey);
        NI[my_pos] = key_id(mykey);
      }
      tn = min(tn + NA, ef_eff);
      cur_buf ^= 1;
      wave_lds_sync();
    }

    // output: the first k keys of T
    {
      const float* TD = tD[cur_buf];
      const int* TI = tI[cur_buf];
      for (int jx = l; jx < a.k_max; jx += 64) {
        int id = -1;
        float d = __int_as_float(0x7f800000);
        if (jx < k && jx < tn) {
          id = (int)((uint32_t)TI[jx] & ~kExpanded);
          d = TD[jx];
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
      for (int i = l; i < a.spill_slots; i += 64) spill[i] = -1;
      __threadfence_block();
    }
    wave_lds_sync();
  }
}

template <int MODE, int CODE, int G, int T4, bool PF>
__global__ void __launch_bounds__(256) k_search(KArgs a) {
  search_body<MODE, CODE, G, T4, PF>(a);
}

// FINGER screening: hold the register budget of four waves per SIMD (the
// search is latency bound, so resident waves matter more than a few spills)
template <int MODE, int CODE, int G, int T4, bool PF>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_search_w4(KArgs a) {
  search_body<MODE, CODE, G, T4, PF>(a);
}

template <int MODE, int CODE, int G, int T4, bool PF>
hipError_t launch_k(const KArgs& a, int blocks, int lds, hipStream_t s) {
  auto fn = MODE == FINGER_MODE_FINGER ? k_search_w4<MODE, CODE, G, T4, PF>
                                       : k_search<MODE, CODE, G, T4, PF>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * a.waves_per_block), lds, s, a);
  return hipGetLastError();
}

template <int MODE, int CODE, bool PF>
hipError_t launch_dims(const KArgs& a, int blocks, int lds, hipStream_t s) {
  if (a.m4 <= 32) return launch_k<MODE, CODE, 8, 4, PF>(a, blocks, lds, s);
  if (a.m4 <= 128) return launch_k<MODE, CODE, 32, 4, PF>(a, blocks, lds, s);
  return launch_k<MODE, CODE, 64, 8, PF>(a, blocks, lds, s);
}

template <int MODE>
hipError_t launch_codes(const KArgs& a, int code, bool pf, int blocks, int lds, hipStream_t s) {
  if (code == FINGER_CODE_BF16)
    return pf ? launch_dims<MODE, FINGER_CODE_BF16, true>(a, blocks, lds, s)
              : launch_dims<MODE, FINGER_CODE_BF16, false>(a, blocks, lds, s);
  if (code == FINGER_CODE_FP8E4M3)
    return pf ? launch_dims<MODE, FINGER_CODE_FP8E4M3, true>(a, blocks, lds, s)
              : launch_dims<MODE, FINGER_CODE_FP8E4M3, false>(a, blocks, lds, s);
  return pf ? launch_dims<MODE, FINGER_CODE_F32, true>(a, blocks, lds, s)
            : launch_dims<MODE, FINGER_CODE_F32, false>(a, blocks, lds, s);
}

int gate_shared_bytes(int gate_h, int gate_in) {
  if (gate_h <= 0) return 0;
  const int nw = gate_h * gate_in + gate_h * gate_h + gate_h;
  return ((2 * nw + 15) & ~15) + ((4 * (2 * gate_h + 1) + 15) & ~15);
}

int wave_bytes(int ef_max, int vis_cap, int r, int m, int gate_in) {
  const int rpad = rpad_of(r);
  int b = 16 * ef_max + 4 * vis_cap + 64 * 8 + 64 * 4 * 3 + 8 * rpad + (r > 0 ? 4 * m : 0);
  if (gate_in > 0) {
    const int spp = 64 / (rpad / 16);  // at most this many slots per pass
    b += 4 * (spp * (r + 4) + 64);
  }
  return (b + 15) & ~15;
}

void fill_common(KArgs& a, const Tables& t) {
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

int search_lds_bytes(int ef_max, int vis_cap, int r, int m, int gate_h, int gate_in) {
  return gate_shared_bytes(gate_h, gate_in) + wave_bytes(ef_max, vis_cap, r, m, gate_in);
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
  a.spill = L.spill;
  a.spill_slots = L.spill_slots_per_wave;
  a.vis_cap = L.vis_cap;
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
  // plain and FINGER: one query wave per workgroup keeps LDS allocation fine
  // grained; the gated mode shares its weights among 4 waves
  a.waves_per_block = gated ? 4 : 1;
  a.lds_shared_bytes = gated ? gate_shared_bytes(a.gate_h, a.gate_in) : 0;
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
  return launch_codes<FINGER_MODE_GATED>(a, t.code_type, false, blocks, lds, s);
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
    const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
    acc += dx * dx + dy * dy + dz * dz + dw * dw;
  }
  const float dcur = wave_sum(acc);
  const float qq = a.qq[q];
  const float ccv = a.cc[c];
  const float qc = 0.5f * (qq + ccv - dcur);
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
    est[item] = da * da * ccv + rq2 + rd * rd - 2.f * rq * rd * t;
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
