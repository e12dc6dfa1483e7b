// FINGER construction kernels (Algorithm 2) and the precomputed tables of
// Supplementary G.  Statistics that set the basis and the distribution
// matching constants are accumulated in float64 with fixed-order
// reductions, so a build is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

// SplitMix64 (Steele, Lea, Flood 2014): the j-th output of the stream
// seeded with `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t j) {
  uint64_t z = seed + (j + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// one thread per row: ids in [0, n), no self loop, valid prefix then -1,
// no repeats.  bad[0] counts offending rows.
__global__ void k_validate_graph(const int32_t* g, int64_t n, int deg, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t* row = g + i * deg;
  bool ok = true, ended = false;
  for (int j = 0; j < deg; ++j) {
    const int32_t v = row[j];
    if (v < 0) {
      if (v != -1) ok = false;
      ended = true;
      continue;
    }
    if (ended || v >= n || v == i) ok = false;
    for (int t = 0; t < j; ++t)
      if (row[t] == v) ok = false;
  }
  if (!ok) atomicAdd(bad, 1);
}

__global__ void k_check_ids(const int32_t* ids, int64_t cnt, int64_t n, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt && (ids[i] < 0 || ids[i] >= n)) atomicAdd(bad, 1);
}

// sample i -> (c, d, d') or (-1, -1, -1) when c has fewer than two neighbours
__global__ void k_sample_pairs(const int32_t* g, int64_t n, int deg, int64_t ns, uint64_t seed,
                               int32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ns) return;
  const int64_t c = (ns == n) ? i : (int64_t)(splitmix64(seed, 3ull * (uint64_t)i) % (uint64_t)n);
  const int32_t* row = g + c * deg;
  int d = 0;
  while (d < deg && row[d] >= 0) ++d;
  if (d < 2) {
    out[3 * i] = -1;
    out[3 * i + 1] = -1;
    out[3 * i + 2] = -1;
    return;
  }
  const uint64_t a = splitmix64(seed, 3ull * (uint64_t)i + 1ull) % (uint64_t)d;
  const uint64_t b = (a + 1ull + splitmix64(seed, 3ull * (uint64_t)i + 2ull) % (uint64_t)(d - 1)) %
                     (uint64_t)d;
  out[3 * i] = (int32_t)c;
  out[3 * i + 1] = row[a];
  out[3 * i + 2] = row[b];
}

// Eq. 1 in float64: d_res = d - (c.d / c.c) c for both neighbours of each
// kept sample (one wave per sample)
__global__ void k_residuals(const float* X, int m, const int32_t* smp, int64_t ns, double* r1,
                            double* r2) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= ns) return;
  const int l = threadIdx.x & 63;
  const float* c = X + (int64_t)smp[3 * i] * m;
  const float* d = X + (int64_t)smp[3 * i + 1] * m;
  const float* e = X + (int64_t)smp[3 * i + 2] * m;
  double cc = 0, cd = 0, ce = 0;
  for (int j = l; j < m; j += 64) {
    const double cj = c[j];
    cc += cj * cj;
    cd += cj * (double)d[j];
    ce += cj * (double)e[j];
  }
  for (int o = 32; o >= 1; o >>= 1) {
    cc += __shfl_xor(cc, o, 64);
    cd += __shfl_xor(cd, o, 64);
    ce += __shfl_xor(ce, o, 64);
  }
  const double ad = cc > 0 ? cd / cc : 0.0, ae = cc > 0 ? ce / cc : 0.0;
  for (int j = l; j < m; j += 64) {
    r1[i * m + j] = (double)d[j] - ad * (double)c[j];
    r2[i * m + j] = (double)e[j] - ae * (double)c[j];
  }
}

// partial Gram matrices: block (ti, tj, part) sums rows of its part into a
// 32 x 32 tile of R^T R
__global__ void __launch_bounds__(256) k_gram_part(const double* R, int64_t ns, int m, int parts,
                                                   double* partial) {
  __shared__ double Ai[32][33], Aj[32][33];
  const int ti = blockIdx.x, tj = blockIdx.y, part = blockIdx.z;
  const int64_t per = (ns + parts - 1) / parts;
  const int64_t b0 = part * per, b1 = min(ns, b0 + per);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // ty 0..7
  double acc[4] = {0, 0, 0, 0};
  for (int64_t s0 = b0; s0 < b1; s0 += 32) {
    __syncthreads();
    for (int rr = ty; rr < 32; rr += 8) {
      const int64_t srow = s0 + rr;
      const int ci = ti * 32 + tx, cj = tj * 32 + tx;
      Ai[rr][tx] = (srow < b1 && ci < m) ? R[srow * m + ci] : 0.0;
      Aj[rr][tx] = (srow < b1 && cj < m) ? R[srow * m + cj] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < 32; ++rr) {
      const double bj = Aj[rr][tx];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += Ai[rr][ty + 8 * q] * bj;
    }
  }
  for (int q = 0; q < 4; ++q) {
    const int i = ti * 32 + ty + 8 * q, j = tj * 32 + tx;
    if (i < m && j < m) partial[((int64_t)part * m + i) * m + j] = acc[q];
  }
}

__global__ void k_gram_reduce(const double* partial, int parts, int64_t mm, double* M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mm) return;
  double s = 0;
  for (int p = 0; p < parts; ++p) s += partial[p * mm + i];
  M[i] = s;
}

// X_i = cos(d_res, d'_res), Y_i = cos(P d_res, P d'_res) in float64 (one
// wave per sample; a zero vector has cosine 0)
__global__ void k_pair_cos(const double* r1, const double* r2, int64_t ns, int m,
                           const double* P, int r, double* xy) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= ns) return;
  const int l = threadIdx.x & 63;
  const double* a = r1 + i * m;
  const double* b = r2 + i * m;
  double ab = 0, aa = 0, bb = 0;
  for (int j = l; j < m; j += 64) {
    ab += a[j] * b[j];
    aa += a[j] * a[j];
    bb += b[j] * b[j];
  }
  double pab = 0, paa = 0, pbb = 0;
  for (int k = l; k < r; k += 64) {
    const double* p = P + (int64_t)k * m;
    double pa = 0, pb = 0;
    for (int j = 0; j < m; ++j) {
      pa += p[j] * a[j];
      pb += p[j] * b[j];
    }
    pab += pa * pb;
    paa += pa * pa;
    pbb += pb * pb;
  }
  for (int o = 32; o >= 1; o >>= 1) {
    ab += __shfl_xor(ab, o, 64);
    aa += __shfl_xor(aa, o, 64);
    bb += __shfl_xor(bb, o, 64);
    pab += __shfl_xor(pab, o, 64);
    paa += __shfl_xor(paa, o, 64);
    pbb += __shfl_xor(pbb, o, 64);
  }
  if (l == 0) {
    const double den = sqrt(aa * bb), pden = sqrt(paa * pbb);
    xy[2 * i] = den > 0 ? ab / den : 0.0;
    xy[2 * i + 1] = pden > 0 ? pab / pden : 0.0;
  }
}

// fixed-order float64 sums over the samples (one block of 1024 threads)
//   stage 0: sum X, sum Y
//   stage 1: sum (X - mu)^2, sum (Y - mu_hat)^2
//   stage 2: sum |(Y - mu_hat) scale + mu - X|
__global__ void __launch_bounds__(1024) k_dm_sums(const double* xy, int64_t ns, double mu,
                                                  double mu_hat, double scale, int stage,
                                                  double* out) {
  __shared__ double s0[1024], s1[1024];
  double a = 0, b = 0;
  for (int64_t i = threadIdx.x; i < ns; i += blockDim.x) {
    const double x = xy[2 * i], y = xy[2 * i + 1];
    if (stage == 0) { a += x; b += y; }
    else if (stage == 1) { a += (x - mu) * (x - mu); b += (y - mu_hat) * (y - mu_hat); }
    else if (stage == 2) { a += fabs((y - mu_hat) * scale + mu - x); }
    else { a += (x - mu) * (y - mu_hat); }
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s0[threadIdx.x] += s0[threadIdx.x + w];
      s1[threadIdx.x] += s1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = s0[0]; out[1] = s1[0]; }
}

__global__ void k_row_norms(const float* X, int64_t n, int m, float* out) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= n) return;
  const int l = threadIdx.x & 63;
  const float* x = X + i * m;
  float a = 0.f;
  for (int j = l; j < m; j += 64) a += x[j] * x[j];
  a = wave_sum(a);
  if (l == 0) out[i] = a;
}

__global__ void k_normalize_rows(const float* X, int64_t n, int m, float* Y) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= n) return;
  const int l = threadIdx.x & 63;
  const float* x = X + i * m;
  double a = 0;
  for (int j = l; j < m; j += 64) a += (double)x[j] * x[j];
  for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o, 64);
  const double inv = a > 0 ? 1.0 / sqrt(a) : 0.0;
  for (int j = l; j < m; j += 64) Y[i * m + j] = (float)(x[j] * inv);
}

__global__ void k_gather_rows(const float* X, int m, const int32_t* ids, int64_t cnt, float* Y) {
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
  if (i >= cnt) return;
  const int l = threadIdx.x & 63;
  const float* x = X + (int64_t)ids[i] * m;
  for (int j = l; j < m; j += 64) Y[i * m + j] = x[j];
}

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// float -> OCP FP8 E4M3, round to nearest even, saturating at +-448.
// Written from the format: 1 sign bit, 4 exponent bits (bias 7), 3 mantissa
// bits; normals 2^(e-7) (1 + m/8) for e = 1..15 (e = 15, m = 7 is NaN, so
// the largest finite value is 448); subnormals 2^-6 m/8.
__device__ __forceinline__ uint8_t f_to_e4m3(float f) {
  const uint32_t sign = (__float_as_uint(f) >> 24) & 0x80u;
  float a = fabsf(f);
  if (!(a < 464.f)) return (uint8_t)(sign | 0x7Eu);  // >= 464 rounds past 448: saturate
  if (a >= 448.f) return (uint8_t)(sign | 0x7Eu);
  // quantum of the binade holding a: 2^(E-3) for normals, 2^-9 below 2^-6
  int E;
  frexpf(a, &E);  // a = f * 2^E, f in [0.5, 1) -> binade exponent E - 1
  int e = E - 1;
  if (e < -6) e = -6;
  const float q = ldexpf(1.0f, e - 3);
  const float k = rintf(a / q);  // round half to even on the quantum grid
  const float v = k * q;         // exactly representable
  if (v == 0.f) return (uint8_t)sign;
  int E2;
  frexpf(v, &E2);
  int ev = E2 - 1;  // v may have moved up one binade
  uint32_t code;
  if (ev < -6) {
    code = (uint32_t)(v / ldexpf(1.0f, -9));  // subnormal: m = v / 2^-9
  } else {
    const float mant = v / ldexpf(1.0f, ev) - 1.0f;  // in [0, 1)
    code = ((uint32_t)(ev + 7) << 3) | (uint32_t)rintf(mant * 8.0f);
  }
  if (code > 0x7Eu) code = 0x7Eu;
  return (uint8_t)(sign | code);
}

// Per node c (one wave): alpha_d, rho_d and u_d for every slot (Supplementary
// G), then the stored code.  LDS: c [m], Pc [rpad], u rows [deg][rpad].
__global__ void k_edge_codes(const float* X, int m, const int32_t* g, int64_t n, int deg,
                             const float* cc, const float* pc, int r, int rpad, int code_type,
                             float* alpha, float* rho, void* codes, float* scale) {
  extern __shared__ __align__(16) float sm[];
  const int wib = threadIdx.x / 64, l = threadIdx.x & 63;
  const int wpb = blockDim.x / 64;
  float* cv = sm + (int64_t)wib * (m + rpad + deg * rpad);
  float* pcc = cv + m;
  float* U = pcc + rpad;
  const int64_t c = (int64_t)blockIdx.x * wpb + wib;
  if (c >= n) return;
  const float* xc = X + c * m;
  for (int j = l; j < m; j += 64) cv[j] = xc[j];
  for (int j = l; j < rpad; j += 64) pcc[j] = pc[c * rpad + j];
  wave_lds_sync();
  const float ccv = cc[c];
  float amax = 0.f;
  for (int s = 0; s < deg; ++s) {
    const int d = g[c * deg + s];
    float a = 0.f, rr = 0.f;
    if (d >= 0) {
      const float* xd = X + (int64_t)d * m;
      float dot = 0.f;
      for (int j = l; j < m; j += 64) dot += cv[j] * xd[j];
      dot = wave_sum(dot);
      a = ccv > 0.f ? dot / ccv : 0.f;
      float r2 = 0.f;
      for (int j = l; j < m; j += 64) {
        const float t = xd[j] - a * cv[j];
        r2 += t * t;
      }
      rr = sqrtf(wave_sum(r2));
      float nu = 0.f;
      for (int j = l; j < rpad; j += 64) {
        const float v = (j < r) ? pc[(int64_t)d * rpad + j] - a * pcc[j] : 0.f;
        U[s * rpad + j] = v;
        nu += v * v;
      }
      nu = wave_sum(nu);
      const float inv = nu > 0.f ? 1.0f / sqrtf(nu) : 0.f;
      for (int j = l; j < rpad; j += 64) {
        const float v = U[s * rpad + j] * inv;
        U[s * rpad + j] = v;
        amax = fmaxf(amax, fabsf(v));
      }
    } else {
      for (int j = l; j < rpad; j += 64) U[s * rpad + j] = 0.f;
    }
    if (l == 0) {
      alpha[c * deg + s] = a;
      rho[c * deg + s] = rr;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  wave_lds_sync();
  const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
  if (code_type == FINGER_CODE_FP8E4M3 && l == 0) scale[c] = sc;
  if (code_type != FINGER_CODE_FP8E4M3 && l == 0 && scale != nullptr) scale[c] = 1.0f;
  const int64_t base = c * deg * (int64_t)rpad;
  for (int i = l; i < deg * rpad; i += 64) {
    const float v = U[i];
    if (code_type == FINGER_CODE_F32) static_cast<float*>(codes)[base + i] = v;
    else if (code_type == FINGER_CODE_BF16) static_cast<uint16_t*>(codes)[base + i] = f_to_bf16(v);
    else static_cast<uint8_t*>(codes)[base + i] = f_to_e4m3(v / sc);
  }
}

}  // namespace

hipError_t launch_validate_graph(const int32_t* graph, int64_t n, int deg, int32_t* bad,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_validate_graph, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, graph,
                     n, deg, bad);
  return hipGetLastError();
}

hipError_t launch_check_ids(const int32_t* ids, int64_t cnt, int64_t n, int32_t* bad,
                            hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_ids, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, ids, cnt,
                     n, bad);
  return hipGetLastError();
}

hipError_t launch_sample_pairs(const int32_t* graph, int64_t n, int deg, int64_t ns,
                               uint64_t seed, int32_t* samples, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_pairs, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, s, graph,
                     n, deg, ns, seed, samples);
  return hipGetLastError();
}

hipError_t launch_residuals_f64(const float* data, int m, const int32_t* samples, int64_t ns,
                                double* res1, double* res2, hipStream_t s) {
  hipLaunchKernelGGL(k_residuals, dim3((unsigned)((ns + 3) / 4)), dim3(256), 0, s, data, m,
                     samples, ns, res1, res2);
  return hipGetLastError();
}

int gram_parts(int64_t ns, int m) {
  const int tiles = (m + 31) / 32;
  int parts = (int)((1024 + tiles * tiles - 1) / (tiles * tiles));
  if (parts > 64) parts = 64;
  if (parts < 1) parts = 1;
  if (parts > ns) parts = (int)(ns > 0 ? ns : 1);
  return parts;
}

hipError_t launch_gram_f64(const double* R, int64_t ns, int m, double* M, hipStream_t s) {
  // M has room for gram_parts(ns, m) partial m x m blocks after the result
  const int tiles = (m + 31) / 32;
  const int parts = gram_parts(ns, m);
  double* partial = M + (int64_t)m * m;
  hipLaunchKernelGGL(k_gram_part, dim3(tiles, tiles, parts), dim3(256), 0, s, R, ns, m, parts,
                     partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, partial,
                     parts, mm, M);
  return hipGetLastError();
}

hipError_t launch_pair_cosines(const double* res1, const double* res2, int64_t ns, int m,
                               const double* P64, int r, double* xy, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_cos, dim3((unsigned)((ns + 3) / 4)), dim3(256), 0, s, res1, res2, ns,
                     m, P64, r, xy);
  return hipGetLastError();
}

hipError_t launch_dm_sums(const double* xy, int64_t ns, double mu, double mu_hat, double scale,
                          int stage, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dm_sums, dim3(1), dim3(1024), 0, s, xy, ns, mu, mu_hat, scale, stage, out);
  return hipGetLastError();
}

hipError_t launch_row_norms(const float* X, int64_t n, int m, float* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_norms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, m, out);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(const float* X, int64_t n, int m, float* Y, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_normalize_rows, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, X, n, m, Y);
  return hipGetLastError();
}

hipError_t launch_gather_rows(const float* X, int m, const int32_t* ids, int64_t cnt, float* Y,
                              hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((cnt + 3) / 4)), dim3(256), 0, s, X, m, ids,
                     cnt, Y);
  return hipGetLastError();
}

hipError_t launch_edge_codes(const Tables& t, hipStream_t s) {
  const int rpad = rpad_of(t.r);
  const int per = t.m + rpad + t.deg * rpad;
  int wpb = (int)(160 * 1024 / (per * (int)sizeof(float)));
  if (wpb > 4) wpb = 4;
  if (wpb < 1) return hipErrorInvalidValue;
  const int lds = wpb * per * (int)sizeof(float);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_edge_codes),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_edge_codes, dim3((unsigned)((t.n + wpb - 1) / wpb)), dim3(64 * wpb), lds,
                     s, t.data, t.m, t.graph, t.n, t.deg, t.cc, t.pc, t.r, rpad, t.code_type,
                     t.alpha, t.rho, t.codes, t.scale);
  return hipGetLastError();
}

}  // namespace finger
