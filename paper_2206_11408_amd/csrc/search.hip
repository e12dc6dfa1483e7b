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
//   scratch compacted neighbour ids / distances / sorted new keys.
// One expansion: pick the best unexpanded entry of T; read its adjacency
// row (one 4-byte id per lane, coalesced); test-and-set V; in FINGER mode
// screen the new neighbours with the estimate against ub = worst d2 of T at
// the start of the expansion; gather the survivors' vectors (G lanes per
// vector, float4 loads) and reduce (q - x)^2 across the group; merge the
// admitted keys into T (bitonic sort of at most 64 keys + rank-based merge).
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

constexpr uint32_t kExpanded = 0x80000000u;
constexpr int kLdsProbes = 24;

struct KArgs {
  const float* data;
  const int32_t* graph;
  int64_t n;
  int m, m4, deg;
  const float* queries;
  int64_t nq;
  // FINGER tables
  int r, rpad, rg;  // rg = lanes per code row (rpad / 16)
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
  // gate
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
// visited; sets *spilled when the global table was touched, *overflow when
// both tables were exhausted (the id is then treated as visited).
__device__ __forceinline__ int visit(int id, int* __restrict__ tab, uint32_t cap_mask,
                                     int* __restrict__ spill, uint32_t spill_mask,
                                     bool& spilled, bool& overflow) {
  uint32_t h = (hash_id(id) >> 7) & cap_mask;
#pragma unroll 1
  for (int p = 0; p < kLdsProbes; ++p) {
    int old = atomicCAS(&tab[h], -1, id);
    if (old == -1) return 1;
    if (old == id) return 0;
    h = (h + 1) & cap_mask;
  }
  spilled = true;
  uint32_t g = (hash_id(id ^ 0x5bd1e995) >> 5) & spill_mask;
#pragma unroll 1
  for (uint32_t p = 0; p <= spill_mask; ++p) {
    int old = atomicCAS(&spill[g], -1, id);
    if (old == -1) return 1;
    if (old == id) return 0;
    g = (g + 1) & spill_mask;
  }
  overflow = true;
  return 0;
}

// number of keys among the sorted LDS keys (d[i], id[i] & ~flag), i < cnt,
// that are below x; cnt <= 2^steps
__device__ __forceinline__ int rank_in_T(const float* __restrict__ d, const int* __restrict__ id,
                                         int cnt, uint64_t x, int top) {
  int pos = 0;
#pragma unroll 1
  for (int step = top; step > 0; step >>= 1) {
    int probe = pos + step;
    if (probe <= cnt) {
      uint64_t kk = make_key(d[probe - 1], (int)((uint32_t)id[probe - 1] & ~kExpanded));
      if (kk < x) pos = probe;
    }
  }
  return pos;
}

__device__ __forceinline__ int rank_in_keys(const uint64_t* __restrict__ k, int cnt, uint64_t x) {
  int pos = 0;
#pragma unroll
  for (int step = 64; step > 0; step >>= 1) {
    int probe = pos + step;
    if (probe <= cnt && k[probe - 1] < x) pos = probe;
  }
  return pos;
}

template <int CODE>
__device__ __forceinline__ void load_code16(const void* codes, int64_t row, int rpad, int chunk,
                                            float* u) {
  if constexpr (CODE == FINGER_CODE_F32) {
    const float4* p = reinterpret_cast<const float4*>(
        static_cast<const float*>(codes) + row * rpad + chunk * 16);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float4 v = p[i];
      u[4 * i] = v.x; u[4 * i + 1] = v.y; u[4 * i + 2] = v.z; u[4 * i + 3] = v.w;
    }
  } else if constexpr (CODE == FINGER_CODE_BF16) {
    const uint4* p = reinterpret_cast<const uint4*>(
        static_cast<const uint16_t*>(codes) + row * rpad + chunk * 16);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      uint4 v = p[i];
      uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        u[8 * i + 2 * j] = __uint_as_float(w[j] << 16);
        u[8 * i + 2 * j + 1] = __uint_as_float(w[j] & 0xffff0000u);
      }
    }
  } else {
    const uint4* p = reinterpret_cast<const uint4*>(
        static_cast<const uint8_t*>(codes) + row * rpad + chunk * 16);
    uint4 v = p[0];
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
      for (int b = 0; b < 4; ++b) u[4 * j + b] = e4m3_to_f((uint8_t)(w[j] >> (8 * b)));
    }
  }
}

// sum over aligned groups of g lanes, g a runtime power of two <= 16
__device__ __forceinline__ float group_sum_rt(float v, int g) {
  for (int s = g >> 1; s >= 1; s >>= 1) v += shfl_xor_f(v, s);
  return v;
}

// Per-expansion screening prep (the query side of Supplementary G): from
// the exact d2 of the centre, q.c by the law of cosines (Section 3.2),
// alpha_q = q.c / c.c, ||q_res||^2 = ||q||^2 - alpha_q q.c and the chunk of
// w = P q_res = Pq - alpha_q P c this lane holds.
struct Prep {
  float alpha_q, rq2, rq, cc, inv_w;
  float w[16];
};

__device__ __forceinline__ void screen_prep(const KArgs& a, int cur, float dcur, float qq,
                                            const float* pqv, int chunk, Prep& s) {
  const float cc = a.cc[cur];
  const float qc = 0.5f * (qq + cc - dcur);
  const float aq = cc > 0.f ? qc / cc : 0.f;
  s.cc = cc;
  s.alpha_q = aq;
  s.rq2 = fmaxf(qq - aq * qc, 0.f);
  s.rq = sqrtf(s.rq2);
  const float4* pcp = reinterpret_cast<const float4*>(a.pc + (int64_t)cur * a.rpad + chunk * 16);
  float part = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float4 v = pcp[i];
    s.w[4 * i] = pqv[4 * i] - aq * v.x;
    s.w[4 * i + 1] = pqv[4 * i + 1] - aq * v.y;
    s.w[4 * i + 2] = pqv[4 * i + 2] - aq * v.z;
    s.w[4 * i + 3] = pqv[4 * i + 3] - aq * v.w;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) part += s.w[i] * s.w[i];
  const float w2 = group_sum_rt(part, a.rg);
  s.inv_w = w2 > 0.f ? 1.0f / sqrtf(w2) : 0.f;
}

// Algorithm 3 + Eq. 2 for one edge given its t_hat
__device__ __forceinline__ float finger_est(const KArgs& a, const Prep& s, float t_hat,
                                            float alpha_d, float rho_d) {
  const float t = (t_hat - a.mu_hat) * a.dm_scale + a.mu + a.eps;
  const float da = s.alpha_q - alpha_d;
  return da * da * s.cc + s.rq2 + rho_d * rho_d - 2.f * s.rq * rho_d * t;
}

// Gated estimate: the network replaces the distribution-matching map.
// Every lane of the group evaluates the same small MLP on its edge features
// held in LDS; weights are bf16 in LDS, accumulation in float.
__device__ float gate_eval(const KArgs& a, const uint16_t* __restrict__ w,
                           const float* __restrict__ b, const float* __restrict__ x) {
  const int in = a.gate_in, H = a.gate_h;
  float h1[64];
  for (int j = 0; j < H; ++j) {
    float acc = b[j];
    const uint16_t* wr = w + (int64_t)j * in;
    for (int i = 0; i < in; ++i) acc += bf16_to_f(wr[i]) * x[i];
    h1[j] = fmaxf(acc, 0.f);
  }
  const uint16_t* W2 = w + (int64_t)H * in;
  const uint16_t* W3 = W2 + H * H;
  float out = b[2 * H];
  for (int j = 0; j < H; ++j) {
    float acc = b[H + j];
    const uint16_t* wr = W2 + j * H;
    for (int i = 0; i < H; ++i) acc += bf16_to_f(wr[i]) * h1[i];
    out += bf16_to_f(W3[j]) * fmaxf(acc, 0.f);
  }
  return out;
}

template <int G, int T4>
__device__ __forceinline__ void load_query(const KArgs& a, int64_t qi, float4* qv) {
  const int lg = lane_id() & (G - 1);
  const float4* q4 = reinterpret_cast<const float4*>(a.queries + qi * a.m);
#pragma unroll
  for (int t = 0; t < T4; ++t) {
    int j = lg + G * t;
    qv[t] = j < a.m4 ? q4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// exact squared distances of `cnt` ids listed in ids_lds[0..cnt) to the
// query; results go to d_lds[0..cnt)
template <int G, int T4>
__device__ __forceinline__ void exact_dists(const KArgs& a, const float4* qv,
                                            const int* __restrict__ ids_lds, int cnt,
                                            float* __restrict__ d_lds) {
  constexpr int NPP = 64 / G;
  const int l = lane_id();
  const int lg = l & (G - 1);
  const int slot = l / G;
  for (int p0 = 0; p0 < cnt; p0 += 2 * NPP) {
    float4 xv[2][T4];
    int p[2] = {p0 + slot, p0 + NPP + slot};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (p[h] < cnt) {
        const int id = ids_lds[p[h]];
        const float4* x4 = reinterpret_cast<const float4*>(a.data + (int64_t)id * a.m);
#pragma unroll
        for (int t = 0; t < T4; ++t) {
          int j = lg + G * t;
          xv[h][t] = j < a.m4 ? x4[j] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int t = 0; t < T4; ++t) xv[h][t] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      float acc = 0.f;
#pragma unroll
      for (int t = 0; t < T4; ++t) {
        if (lg + G * t < a.m4) {
          float dx = qv[t].x - xv[h][t].x, dy = qv[t].y - xv[h][t].y;
          float dz = qv[t].z - xv[h][t].z, dw = qv[t].w - xv[h][t].w;
          acc += dx * dx + dy * dy + dz * dz + dw * dw;
        }
      }
      acc = group_sum<G>(acc);
      if (lg == 0 && p[h] < cnt) d_lds[p[h]] = acc;
    }
  }
  wave_lds_sync();
}

template <int MODE, int CODE, int G, int T4>
__global__ void __launch_bounds__(256) k_search(KArgs a) {
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
  float* feat = reinterpret_cast<float*>(cflag + 64);  // gated: 64/rg rows of gate_in floats

  // gate weights staged once per block
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
  int top = 1;
  while (top * 2 <= a.ef_max) top *= 2;

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
    int ef = a.efq ? a.efq[qi] : a.ef_all;
    int status = 0;
    int ef_eff = max(ef, k);
    if (ef_eff > a.ef_max) { ef_eff = a.ef_max; status |= 2; }

    float4 qv[T4];
    load_query<G, T4>(a, qi, qv);
    const float qq = (MODE != FINGER_MODE_PLAIN) ? a.qq[qi] : 0.f;
    float pqv[16];
    const int chunk = (MODE != FINGER_MODE_PLAIN) ? (l % a.rg) : 0;
    if constexpr (MODE != FINGER_MODE_PLAIN) {
      const float4* pq4 = reinterpret_cast<const float4*>(a.pq + qi * a.rpad + chunk * 16);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float4 v = pq4[i];
        pqv[4 * i] = v.x; pqv[4 * i + 1] = v.y; pqv[4 * i + 2] = v.z; pqv[4 * i + 3] = v.w;
      }
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
    exact_dists<G, T4>(a, qv, cid, 1, cd);
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
      // select the best unexpanded entry of T
      int j = -1;
      for (int b0 = 0; b0 < tn; b0 += 64) {
        int i = b0 + l;
        bool un = i < tn && ((uint32_t)TI[i] & kExpanded) == 0u;
        uint64_t bm = ballot(un);
        if (bm) { j = b0 + __ffsll((unsigned long long)bm) - 1; break; }
      }
      if (j < 0) break;
      const int cur = TI[j];
      const float dcur = TD[j];
      wave_lds_sync();
      if (l == 0) TI[j] = (int)((uint32_t)cur | kExpanded);
      ++n_exp;

      const bool screening = (MODE != FINGER_MODE_PLAIN) && n_exp > a.warmup && tn == ef_eff;
      const float ub2 = TD[tn - 1];
      int nb = -1;
      float al = 0.f, rh = 0.f;
      if (l < a.deg) {
        nb = a.graph[(int64_t)cur * a.deg + l];
        if (screening) {
          al = a.alpha[(int64_t)cur * a.deg + l];
          rh = a.rho[(int64_t)cur * a.deg + l];
        }
      }
      Prep sp;
      if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) screen_prep(a, cur, dcur, qq, pqv, chunk, sp);
      }
      int isnew = 0;
      if (nb >= 0) isnew = visit(nb, vis, cap_mask, spill, spill_mask, spilled, overflow);
      const uint64_t newm = ballot(isnew != 0);
      const int S = popc64(newm);
      n_vis += S;
      if (S == 0) continue;
      // compact the new neighbours: cid[p] = id, cflag[p] = slot
      const int rk = mask_rank(newm);
      if (isnew) {
        cid[rk] = nb;
        cflag[rk] = l;
      }
      wave_lds_sync();

      uint64_t survm = newm;
      bool logging = false;
      int64_t log_base = 0;
      if constexpr (MODE != FINGER_MODE_PLAIN) {
        if (screening) {
          n_scr += S;
          ++n_prep;
          logging = (MODE == FINGER_MODE_FINGER) && a.log_x != nullptr;
          if (logging) {
            unsigned long long got = 0;
            if (l == 0) got = atomicAdd((unsigned long long*)a.log_count, (unsigned long long)S);
            log_base = (int64_t)shfl_u64((uint64_t)got, 0);
          }
          const int cpp = 64 / a.rg;
          const int sub = l / a.rg;
          const float scl = (CODE == FINGER_CODE_FP8E4M3) ? a.scale[cur] : 1.f;
          const float ub = sqrtf(ub2);
          const float inv_ub = ub > 0.f ? 1.f / ub : 0.f;
          for (int p0 = 0; p0 < S; p0 += cpp) {
            const int p = p0 + sub;
            float dot = 0.f;
            float u[16];
            int slot = 0;
            if (p < S) {
              slot = cflag[p];
              load_code16<CODE>(a.codes, (int64_t)cur * a.deg + slot, a.rpad, chunk, u);
#pragma unroll
              for (int i = 0; i < 16; ++i) dot += sp.w[i] * u[i];
            } else {
#pragma unroll
              for (int i = 0; i < 16; ++i) u[i] = 0.f;
            }
            dot = group_sum_rt(dot, a.rg);
            const float t_hat = dot * scl * sp.inv_w;
            // alpha_d and rho_d were read by adjacency lane `slot`
            const float ad = __shfl(al, slot, 64);
            const float rd = __shfl(rh, slot, 64);
            const float da = sp.alpha_q - ad;
            float* x = nullptr;
            if constexpr (MODE == FINGER_MODE_GATED) {
              x = feat + (int64_t)sub * a.gate_in;
            } else {
              if (logging && p < S && log_base + p < a.log_cap)
                x = a.log_x + (log_base + p) * (int64_t)(2 * a.r + 4);
            }
            if (x != nullptr && p < S) {
              // features of this edge, in the layout finger_gate_attach documents
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                const int e = chunk * 16 + i;
                if (e < a.r) {
                  x[e] = sp.w[i] * sp.inv_w;
                  x[a.r + e] = u[i] * scl;
                }
              }
              if (chunk == 0) {
                x[2 * a.r] = t_hat;
                x[2 * a.r + 1] = sp.rq * inv_ub;
                x[2 * a.r + 2] = rd * inv_ub;
                x[2 * a.r + 3] = da * da * sp.cc * inv_ub * inv_ub;
              }
            }
            float est;
            if constexpr (MODE == FINGER_MODE_GATED) {
              wave_lds_sync();
              float t = 0.f;
              if (p < S && chunk == 0) t = gate_eval(a, gw, gb, x) + a.eps_gate;
              est = da * da * sp.cc + sp.rq2 + rd * rd - 2.f * sp.rq * rd * t;
              wave_lds_sync();
            } else {
              est = finger_est(a, sp, t_hat, ad, rd);
            }
            // skip iff the estimate exceeds ub (both squared)
            if (p < S && chunk == 0) cd[p] = (est > ub2) ? 1.f : 0.f;
          }
          wave_lds_sync();
          // back in adjacency lanes: this lane's neighbour sits at position rk
          const bool keep = isnew && cd[rk] == 0.f;
          survm = ballot(keep);
          n_skip += S - popc64(survm);
          wave_lds_sync();
          if (logging) {
            // every screened edge gets its exact distance for the log; the
            // skip decision is kept per position for the admission step
            if (isnew) cflag[rk] = keep ? 0 : 1;
            survm = newm;
          } else {
            const int r2 = mask_rank(survm);
            if (keep) cid[r2] = nb;
          }
          wave_lds_sync();
        }
      }
      const int S2 = popc64(survm);
      if (S2 == 0) continue;
      exact_dists<G, T4>(a, qv, cid, S2, cd);

      // admission candidates: lanes 0..S2-1 hold (cd, cid)
      uint64_t key = ~0ull;
      bool adm = false;
      bool was_skipped = false;
      if (l < S2) {
        const float d = cd[l];
        const int id = cid[l];
        if (logging) {
          was_skipped = cflag[l] != 0;
          const int64_t row = log_base + l;
          if (row < a.log_cap) {
            a.log_y[2 * row] = d;
            a.log_y[2 * row + 1] = ub2;
          }
        }
        key = make_key(d, id);
        adm = !was_skipped &&
              (tn < ef_eff ||
               key < make_key(TD[tn - 1], (int)((uint32_t)TI[tn - 1] & ~kExpanded)));
      }
      n_exact += S2 - popc64(ballot(was_skipped));
      const uint64_t am = ballot(adm);
      const int NA = popc64(am);
      if (NA == 0) continue;
      // compact admitted keys to lanes 0..NA-1 via LDS, then sort
      wave_lds_sync();
      if (adm) ck[mask_rank(am)] = key;
      wave_lds_sync();
      uint64_t v = l < NA ? ck[l] : ~0ull;
      v = bitonic_sort<64>(v);
      wave_lds_sync();
      if (l < NA) ck[l] = v;
      wave_lds_sync();
      // merge T (sorted) with the NA sorted keys into the other buffer
      float* ND = tD[cur_buf ^ 1];
      int* NI = tI[cur_buf ^ 1];
      for (int i = l; i < tn; i += 64) {
        const int idf = TI[i];
        const uint64_t kk = make_key(TD[i], (int)((uint32_t)idf & ~kExpanded));
        const int pos = i + rank_in_keys(ck, NA, kk);
        if (pos < ef_eff) {
          ND[pos] = TD[i];
          NI[pos] = idf;
        }
      }
      if (l < NA) {
        const int pos = l + rank_in_T(TD, TI, tn, v, top);
        if (pos < ef_eff) {
          ND[pos] = key_d2(v);
          NI[pos] = key_id(v);
        }
      }
      tn = min(tn + NA, ef_eff);
      cur_buf ^= 1;
      wave_lds_sync();
    }

    // output: the first k keys of T
    {
      float* TD = tD[cur_buf];
      int* TI = tI[cur_buf];
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
      for (int i = l; i < a.spill_slots; i += 64) spill[i] = -1;
      __threadfence_block();
    }
    wave_lds_sync();
  }
}

template <int MODE, int CODE, int G, int T4>
hipError_t launch_k(const KArgs& a, int blocks, int lds, hipStream_t s) {
  auto fn = k_search<MODE, CODE, G, T4>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * a.waves_per_block), lds, s, a);
  return hipGetLastError();
}

template <int MODE, int CODE>
hipError_t launch_dims(const KArgs& a, int blocks, int lds, hipStream_t s) {
  if (a.m4 <= 32) return launch_k<MODE, CODE, 8, 4>(a, blocks, lds, s);
  if (a.m4 <= 128) return launch_k<MODE, CODE, 32, 4>(a, blocks, lds, s);
  return launch_k<MODE, CODE, 64, 8>(a, blocks, lds, s);
}

template <int MODE>
hipError_t launch_codes(const KArgs& a, int code, int blocks, int lds, hipStream_t s) {
  if (code == FINGER_CODE_BF16) return launch_dims<MODE, FINGER_CODE_BF16>(a, blocks, lds, s);
  if (code == FINGER_CODE_FP8E4M3) return launch_dims<MODE, FINGER_CODE_FP8E4M3>(a, blocks, lds, s);
  return launch_dims<MODE, FINGER_CODE_F32>(a, blocks, lds, s);
}

int gate_shared_bytes(int gate_h, int gate_in) {
  if (gate_h <= 0) return 0;
  const int nw = gate_h * gate_in + gate_h * gate_h + gate_h;
  return ((2 * nw + 15) & ~15) + ((4 * (2 * gate_h + 1) + 15) & ~15);
}

int wave_bytes(int ef_max, int vis_cap, int r, int gate_in) {
  (void)r;
  int b = 16 * ef_max + 4 * vis_cap + 64 * 8 + 64 * 4 * 3;
  if (gate_in > 0) b += 64 * gate_in * 4;
  return (b + 15) & ~15;
}

}  // namespace

int search_lds_bytes(int ef_max, int vis_cap, int r, int gate_h, int gate_in) {
  return gate_shared_bytes(gate_h, gate_in) + wave_bytes(ef_max, vis_cap, r, gate_in);
}

hipError_t launch_search(const Tables& t, const SearchLaunch& L, hipStream_t s) {
  KArgs a{};
  a.data = t.data;
  a.graph = t.graph;
  a.n = t.n;
  a.m = t.m;
  a.m4 = t.m / 4;
  a.deg = t.deg;
  a.queries = L.queries;
  a.nq = L.nq;
  a.r = t.r;
  a.rpad = (t.r + 15) / 16 * 16;
  a.rg = a.rpad > 0 ? a.rpad / 16 : 1;
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
  // one query wave per workgroup keeps LDS allocation fine grained; the
  // gated mode shares its weights among 4 waves
  a.waves_per_block = gated ? 4 : 1;
  a.lds_shared_bytes = gated ? gate_shared_bytes(a.gate_h, a.gate_in) : 0;
  a.lds_wave_bytes = wave_bytes(L.ef_max, L.vis_cap, t.r, gated ? a.gate_in : 0);
  const int lds = a.lds_shared_bytes + a.waves_per_block * a.lds_wave_bytes;
  const int blocks = (L.waves + a.waves_per_block - 1) / a.waves_per_block;
  if (L.mode == FINGER_MODE_PLAIN) return launch_dims<FINGER_MODE_PLAIN, FINGER_CODE_F32>(a, blocks, lds, s);
  if (L.mode == FINGER_MODE_FINGER) return launch_codes<FINGER_MODE_FINGER>(a, t.code_type, blocks, lds, s);
  return launch_codes<FINGER_MODE_GATED>(a, t.code_type, blocks, lds, s);
}

// ------------------------------------------------- estimate test kernel

namespace {
template <int CODE>
__global__ void k_estimate_edges(KArgs a, const int32_t* qi, const int32_t* ci,
                                 const int32_t* si, int64_t items, float* est, float* that) {
  const int64_t item = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (item >= items) return;
  const int l = lane_id();
  const int q = qi[item], c = ci[item], slot = si[item];
  // exact d2(q, c) as the search has it from T
  const float4* q4 = reinterpret_cast<const float4*>(a.queries + (int64_t)q * a.m);
  const float4* c4 = reinterpret_cast<const float4*>(a.data + (int64_t)c * a.m);
  float acc = 0.f;
  for (int j = l; j < a.m4; j += 64) {
    float4 x = q4[j], y = c4[j];
    float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z, dw = x.w - y.w;
    acc += dx * dx + dy * dy + dz * dz + dw * dw;
  }
  const float dcur = wave_sum(acc);
  const int chunk = l % a.rg;
  float pqv[16];
  const float4* pq4 = reinterpret_cast<const float4*>(a.pq + (int64_t)q * a.rpad + chunk * 16);
  for (int i = 0; i < 4; ++i) {
    float4 v = pq4[i];
    pqv[4 * i] = v.x; pqv[4 * i + 1] = v.y; pqv[4 * i + 2] = v.z; pqv[4 * i + 3] = v.w;
  }
  Prep sp;
  screen_prep(a, c, dcur, a.qq[q], pqv, chunk, sp);
  float u[16];
  load_code16<CODE>(a.codes, (int64_t)c * a.deg + slot, a.rpad, chunk, u);
  float dot = 0.f;
  for (int i = 0; i < 16; ++i) dot += sp.w[i] * u[i];
  dot = group_sum_rt(dot, a.rg);
  const float scl = (CODE == FINGER_CODE_FP8E4M3) ? a.scale[c] : 1.f;
  const float t_hat = dot * scl * sp.inv_w;
  const float ad = a.alpha[(int64_t)c * a.deg + slot];
  const float rd = a.rho[(int64_t)c * a.deg + slot];
  if (l == 0) {
    est[item] = finger_est(a, sp, t_hat, ad, rd);
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
  a.data = t.data;
  a.m = t.m;
  a.m4 = t.m / 4;
  a.deg = t.deg;
  a.queries = Q;
  a.r = t.r;
  a.rpad = (t.r + 15) / 16 * 16;
  a.rg = a.rpad / 16;
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
  a.qq = qq;
  a.pq = Pq;
  const int wpb = 4;
  const int blocks = (int)((items + wpb - 1) / wpb);
  if (t.code_type == FINGER_CODE_BF16)
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_BF16>, dim3(blocks), dim3(64 * wpb), 0, s, a,
                       qi, ci, si, items, est, that);
  else if (t.code_type == FINGER_CODE_FP8E4M3)
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_FP8E4M3>, dim3(blocks), dim3(64 * wpb), 0, s,
                       a, qi, ci, si, items, est, that);
  else
    hipLaunchKernelGGL(k_estimate_edges<FINGER_CODE_F32>, dim3(blocks), dim3(64 * wpb), 0, s, a,
                       qi, ci, si, items, est, that);
  return hipGetLastError();
}

}  // namespace finger
