// Learned skip gate (an extension beyond the paper): a perceptron
// in -> H -> H -> 1 with ReLU, trained to predict cos(q_res, d_res) from the
// screening features the search logs.  Training runs on the bf16 matrix
// cores: operands are rounded to bfloat16, products accumulate in float32.
// Weight layout (float):
//   W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1].
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

constexpr int kTS = 32;  // samples per training tile (one MFMA k step)

__device__ __forceinline__ float rbf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}
__device__ __forceinline__ uint16_t bfbits(float f) { return (uint16_t)(__float_as_uint(rbf(f)) >> 16); }

struct Off {
  int64_t w1, b1, w2, b2, w3, b3, total;
};

__host__ __device__ inline Off offsets(int in, int H) {
  Off o;
  o.w1 = 0;
  o.b1 = (int64_t)H * in;
  o.w2 = o.b1 + H;
  o.b2 = o.w2 + (int64_t)H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + H;
  o.total = o.b3 + 1;
  return o;
}

typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint16_t u8v __attribute__((ext_vector_type(8)));

__device__ __forceinline__ b8v as_b8(u8v v) { return __builtin_bit_cast(b8v, v); }
__device__ __forceinline__ b8v lds_b8(const uint16_t* p) {
  return as_b8(*reinterpret_cast<const u8v*>(p));
}
// 8 consecutive float weights w[0..8) (those at or past `valid` read as 0)
// rounded to bf16: one MFMA operand fragment
__device__ __forceinline__ b8v glb_b8(const float* __restrict__ w, int valid) {
  u8v r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = e < valid ? bfbits(w[e]) : (uint16_t)0;
  return as_b8(r);
}

// Tile shapes: inp = in rounded up to 32, hp = H rounded up to 16 (NT tiles
// of 16 hidden units), kh = hp rounded up to 32 (the k extent of layer 2).
struct Dims {
  int in, H, inp, hp, kh, NT;
};
__host__ __device__ inline Dims dims_of(int in, int H) {
  Dims d;
  d.in = in;
  d.H = H;
  d.inp = (in + 31) / 32 * 32;
  d.hp = (H + 15) / 16 * 16;
  d.kh = (d.hp + 31) / 32 * 32;
  d.NT = d.hp / 16;
  return d;
}

// LDS of one training wave (bf16 bits): xs [32][inp], xT [inp][32],
// h1s [32][kh], h1T [hp][32], d2s [32][kh], d2T [hp][32], d1T [hp][32],
// w2T [hp][kh] (W2 transposed)
__host__ __device__ inline int train_lds_elems(const Dims& d) {
  return 2 * kTS * d.inp + 2 * kTS * d.kh + 3 * d.hp * kTS + d.hp * d.kh;
}

// The forward pass of one tile of 32 samples on the bf16 matrix cores
// (v_mfma_f32_16x16x32_bf16; lane l holds A[l%16][8(l/16)..+8), B[8(l/16)..
// +8)[l%16], and D[4(l/16)+v][l%16]).  Operands are bf16, products
// accumulate in float32, biases are added in float32, hidden activations
// are rounded to bf16 after the ReLU.  Leaves z1/z2 (pre-activations, D
// layout: [mt][nt][v] for sample 16 mt + 4(l/16) + v, unit 16 nt + l%16) in
// registers, h1 in LDS, and returns y of samples 16 mt + 4 (l/16) + v in
// yv[mt][v] (every lane of the 16-lane group).
__device__ __forceinline__ void tile_forward(const float* __restrict__ w, const Dims& D, const Off& o,
                                             const uint16_t* __restrict__ xs, uint16_t* __restrict__ h1s,
                                             uint16_t* __restrict__ h1T, float z1[2][4][4],
                                             float z2[2][4][4], float yv[2][4]) {
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = 8 * (l >> 4), g = l >> 4;
  // layer 1: Z1 = X W1^T + b1
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f4v acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < D.inp / 32; ++ks) {
      const b8v A = lds_b8(xs + (16 * mt + lr) * D.inp + 32 * ks + lk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        if (nt < D.NT) {
          const int j = 16 * nt + lr, k0 = 32 * ks + lk;
          const b8v B = j < D.H ? glb_b8(w + o.w1 + (int64_t)j * D.in + k0, D.in - k0) : as_b8(u8v{0, 0, 0, 0, 0, 0, 0, 0});
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[nt], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      const float b1 = (nt < D.NT && j < D.H) ? w[o.b1 + j] : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float z = acc[nt][v] + b1;
        z1[mt][nt][v] = z;
        if (nt < D.NT) {
          const uint16_t hb = bfbits(fmaxf(z, 0.f));
          const int sidx = 16 * mt + 4 * g + v;
          h1s[sidx * D.kh + j] = hb;
          h1T[j * kTS + sidx] = hb;
        }
      }
    }
  }
  // padding columns of h1s (kh > hp) read as zero
  for (int i = l; i < kTS * (D.kh - D.hp); i += 64) {
    const int sidx = i / (D.kh - D.hp), c = D.hp + i % (D.kh - D.hp);
    h1s[sidx * D.kh + c] = 0;
  }
  __syncthreads();
  // layer 2: Z2 = H1 W2^T + b2, then y = W3 . relu(Z2) + b3
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f4v acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < D.kh / 32; ++ks) {
      const b8v A = lds_b8(h1s + (16 * mt + lr) * D.kh + 32 * ks + lk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        if (nt < D.NT) {
          const int j = 16 * nt + lr, k0 = 32 * ks + lk;
          const b8v B = j < D.H ? glb_b8(w + o.w2 + (int64_t)j * D.H + k0, D.H - k0) : as_b8(u8v{0, 0, 0, 0, 0, 0, 0, 0});
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[nt], 0, 0, 0);
        }
      }
    }
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      const bool live = nt < D.NT && j < D.H;
      const float b2 = live ? w[o.b2 + j] : 0.f;
      const float w3 = live ? rbf(w[o.w3 + j]) : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float z = acc[nt][v] + b2;
        z2[mt][nt][v] = z;
        part[v] += w3 * rbf(fmaxf(z, 0.f));
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) part[v] += __shfl_xor(part[v], off, 64);
      yv[mt][v] = part[v] + w[o.b3];
    }
  }
}

// stage a tile of 32 samples (rows past B are zero) as bf16: xs and xT
__device__ __forceinline__ void stage_x(const float* __restrict__ x, int64_t B, int64_t s0, const Dims& D,
                                        uint16_t* __restrict__ xs, uint16_t* __restrict__ xT) {
  const int l = threadIdx.x & 63;
  for (int i = l; i < kTS * D.inp; i += 64) {
    const int sidx = i / D.inp, k = i % D.inp;
    const int64_t s = s0 + sidx;
    const uint16_t v = (s < B && k < D.in) ? bfbits(x[s * D.in + k]) : (uint16_t)0;
    xs[sidx * D.inp + k] = v;
    xT[k * kTS + sidx] = v;
  }
}

// y = f(x) for every sample, one tile of 32 per wave
__global__ void __launch_bounds__(64) k_mlp_fwd(const float* w, int in, int H, const float* x, int64_t B,
                                                float* y) {
  extern __shared__ __align__(16) uint16_t lds[];
  const Dims D = dims_of(in, H);
  const Off o = offsets(in, H);
  uint16_t* xs = lds;
  uint16_t* xT = xs + kTS * D.inp;
  uint16_t* h1s = xT + kTS * D.inp;
  uint16_t* h1T = h1s + kTS * D.kh;
  const int64_t s0 = (int64_t)blockIdx.x * kTS;
  stage_x(x, B, s0, D, xs, xT);
  __syncthreads();
  float z1[2][4][4], z2[2][4][4], yv[2][4];
  tile_forward(w, D, o, xs, h1s, h1T, z1, z2, yv);
  const int l = threadIdx.x & 63;
  if ((l & 15) == 0) {
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t s = s0 + 16 * mt + 4 * (l >> 4) + v;
        if (s < B) y[s] = yv[mt][v];
      }
  }
}

// Backward of the mean squared error over the batch, one tile of 32
// samples per wave, on the matrix cores: dL/dy = 2 (y - t) / B,
// dz2 = dL/dy W3 [z2 > 0], dz1 = (dz2 W2) [z1 > 0], and the weight
// gradients dz2^T h1, dz1^T x and dL/dy^T h2 as products over the tile's
// samples (bf16 operands: x, h1, h2, dz1, dz2 and the weights; float32
// accumulation); bias gradients are float32 sums of the float32 dz.  Each
// wave writes its partial gradient (layout of the weights) and its sum of
// squared errors; k_reduce_parts adds the partials in wave order.
__global__ void __launch_bounds__(64) k_mlp_bwd(const float* w, int in, int H, const float* x,
                                                const float* tgt, int64_t B, float* partial,
                                                float* loss_part) {
  extern __shared__ __align__(16) uint16_t lds[];
  const Dims D = dims_of(in, H);
  const Off o = offsets(in, H);
  uint16_t* xs = lds;
  uint16_t* xT = xs + kTS * D.inp;
  uint16_t* h1s = xT + kTS * D.inp;
  uint16_t* d2s = h1s + kTS * D.kh;
  uint16_t* h1T = d2s + kTS * D.kh;
  uint16_t* d2T = h1T + D.hp * kTS;
  uint16_t* d1T = d2T + D.hp * kTS;
  uint16_t* w2T = d1T + D.hp * kTS;
  const int l = threadIdx.x & 63;
  const int lr = l & 15, lk = 8 * (l >> 4), g = l >> 4;
  const int64_t s0 = (int64_t)blockIdx.x * kTS;
  stage_x(x, B, s0, D, xs, xT);
  // W2 transposed (w2T[i][j] = W2[j][i]), zero padded, for dz2 W2
  for (int i = l; i < D.hp * D.kh; i += 64) {
    const int ii = i / D.kh, jj = i % D.kh;
    w2T[i] = (ii < D.H && jj < D.H) ? bfbits(w[o.w2 + (int64_t)jj * D.H + ii]) : (uint16_t)0;
  }
  __syncthreads();
  float z1[2][4][4], z2[2][4][4], yv[2][4];
  tile_forward(w, D, o, xs, h1s, h1T, z1, z2, yv);
  float* out = partial + (int64_t)blockIdx.x * o.total;
  // output error of samples 16 mt + 4 g + v
  float dy[2][4];
  float se = 0.f, sdy = 0.f;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t s = s0 + 16 * mt + 4 * g + v;
      const float e = s < B ? yv[mt][v] - tgt[s] : 0.f;
      dy[mt][v] = 2.f * e / (float)B;
      se += e * e;
      sdy += dy[mt][v];
    }
  // dz2, and the layer-3 and layer-2 bias gradients
  float gw3[4] = {0.f, 0.f, 0.f, 0.f}, gb2[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    const int j = 16 * nt + lr;
    const bool live = nt < D.NT && j < D.H;
    const float w3 = live ? rbf(w[o.w3 + j]) : 0.f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float z = z2[mt][nt][v];
        const float d = z > 0.f ? dy[mt][v] * w3 : 0.f;
        gw3[nt] += dy[mt][v] * rbf(fmaxf(z, 0.f));
        gb2[nt] += d;
        if (nt < D.NT) {
          const int sidx = 16 * mt + 4 * g + v;
          const uint16_t db = bfbits(d);
          d2s[sidx * D.kh + j] = db;
          d2T[j * kTS + sidx] = db;
        }
      }
  }
  for (int i = l; i < kTS * (D.kh - D.hp); i += 64) {
    const int sidx = i / (D.kh - D.hp), c = D.hp + i % (D.kh - D.hp);
    d2s[sidx * D.kh + c] = 0;
  }
  // sums over the 4 row groups (lanes l, l^16, l^32, l^48 hold one unit)
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    gw3[nt] += __shfl_xor(gw3[nt], 16, 64);
    gw3[nt] += __shfl_xor(gw3[nt], 32, 64);
    gb2[nt] += __shfl_xor(gb2[nt], 16, 64);
    gb2[nt] += __shfl_xor(gb2[nt], 32, 64);
  }
  if (g == 0) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      if (nt < D.NT && j < D.H) {
        out[o.w3 + j] = gw3[nt];
        out[o.b2 + j] = gb2[nt];
      }
    }
  }
  // sum over the tile: every lane's terms, then across lanes in a fixed order
#pragma unroll
  for (int off = 16; off < 64; off <<= 1) {
    se += __shfl_xor(se, off, 64);
    sdy += __shfl_xor(sdy, off, 64);
  }
  if (l == 0) {
    out[o.b3] = sdy;
    loss_part[blockIdx.x] = se;
  }
  __syncthreads();
  // dz1 = (dz2 W2) [z1 > 0]
  float gb1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    f4v acc[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) acc[nt] = f4v{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < D.kh / 32; ++ks) {
      const b8v A = lds_b8(d2s + (16 * mt + lr) * D.kh + 32 * ks + lk);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt)
        if (nt < D.NT)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              A, lds_b8(w2T + (16 * nt + lr) * D.kh + 32 * ks + lk), acc[nt], 0, 0, 0);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      if (nt < D.NT) {
        const int j = 16 * nt + lr;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float d = z1[mt][nt][v] > 0.f ? acc[nt][v] : 0.f;
          gb1[nt] += d;
          d1T[j * kTS + 16 * mt + 4 * g + v] = bfbits(d);
        }
      }
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    gb1[nt] += __shfl_xor(gb1[nt], 16, 64);
    gb1[nt] += __shfl_xor(gb1[nt], 32, 64);
  }
  if (g == 0) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int j = 16 * nt + lr;
      if (nt < D.NT && j < D.H) out[o.b1 + j] = gb1[nt];
    }
  }
  __syncthreads();
  // dW2 = dz2^T h1 (one MFMA per 16 x 16 tile: k = the tile's 32 samples)
  for (int jt = 0; jt < D.NT; ++jt) {
    const b8v A = lds_b8(d2T + (16 * jt + lr) * kTS + lk);
    for (int it = 0; it < D.NT; ++it) {
      f4v acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, lds_b8(h1T + (16 * it + lr) * kTS + lk),
                                                        f4v{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const int i = 16 * it + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * jt + 4 * g + v;
        if (j < D.H && i < D.H) out[o.w2 + (int64_t)j * D.H + i] = acc[v];
      }
    }
  }
  // dW1 = dz1^T x
  for (int jt = 0; jt < D.NT; ++jt) {
    const b8v A = lds_b8(d1T + (16 * jt + lr) * kTS + lk);
    for (int kt = 0; kt < D.inp / 16; ++kt) {
      f4v acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, lds_b8(xT + (16 * kt + lr) * kTS + lk),
                                                        f4v{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      const int k = 16 * kt + lr;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * jt + 4 * g + v;
        if (j < D.H && k < D.in) out[o.w1 + (int64_t)j * D.in + k] = acc[v];
      }
    }
  }
}

// grad[i] = sum over waves of partial[w][i], in wave order (deterministic)
__global__ void k_reduce_parts(const float* partial, int parts, int64_t P, float* grad,
                               const float* loss_part, float* loss, int64_t B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) {
    float s = 0.f;
    for (int p = 0; p < parts; ++p) s += partial[(int64_t)p * P + i];
    grad[i] = s;
  }
  if (i == 0 && loss != nullptr) {
    float s = 0.f;
    for (int p = 0; p < parts; ++p) s += loss_part[p];
    *loss = s / (float)B;
  }
}

// per-block sums of |t - y| in float64, each block over a contiguous range
// in index order and then a fixed tree (deterministic for a given grid)
__global__ void __launch_bounds__(256) k_abs_err_parts(const float* y, const float* t, int64_t rows,
                                                       int64_t per_block, double* parts) {
  __shared__ double red[256];
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = b0 + per_block < rows ? b0 + per_block : rows;
  double s = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += 256) s += fabs((double)t[i] - (double)y[i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) parts[blockIdx.x] = red[0];
}

__global__ void k_adam(float* w, const float* g, float* m1, float* m2, int64_t cnt, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// bf16 weights for the search kernel (layout GateLayout, hidden units
// padded to Hp with zero weights and biases):
//   W1s [r][Hp]   first-layer columns of the shared query features w/|w|,
//                 transposed so that one lane per hidden unit reads in order
//   W1e [Hp][K1]  first-layer columns of the per-edge features, row-major
//                 and zero padded to K1 = 32 ceil((r + 4) / 32) (MFMA B tiles)
//   W2  [Hp][K2]  second layer, zero padded to K2 = 32 ceil(Hp / 32)
//   W3  [Hp]
// biases (float): b1 [Hp], b2 [Hp], b3
__global__ void k_pack_gate(const float* w, int in, int H, uint16_t* wbf, float* b) {
  const Off o = offsets(in, H);
  const GateLayout L = gate_layout((in - 4) / 2, H);
  const int r = L.r;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < L.total;
       i += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    if (i < L.w1e) {
      const int inp = (int)(i / L.hp), hid = (int)(i % L.hp);  // W1s[inp][hid] = W1[hid][inp]
      if (hid < H) v = w[o.w1 + (int64_t)hid * in + inp];
    } else if (i < L.w2) {
      const int64_t k = i - L.w1e;
      const int hid = (int)(k / L.k1), c = (int)(k % L.k1);
      if (hid < H && c < r + 4) v = w[o.w1 + (int64_t)hid * in + r + c];
    } else if (i < L.w3) {
      const int64_t k = i - L.w2;
      const int hid = (int)(k / L.k2), c = (int)(k % L.k2);
      if (hid < H && c < H) v = w[o.w2 + (int64_t)hid * H + c];
    } else {
      const int hid = (int)(i - L.w3);
      if (hid < H) v = w[o.w3 + hid];
    }
    wbf[i] = (uint16_t)(__float_as_uint(rbf(v)) >> 16);
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L.hp) {
    b[i] = i < H ? w[o.b1 + i] : 0.f;
    b[L.hp + i] = i < H ? w[o.b2 + i] : 0.f;
  }
  if (i == 0) b[2 * L.hp] = w[o.b3];
}

// cos(q_res, d_res) from a logged row through Eq. 2
__global__ void k_gate_targets(const float* x, const float* y, int64_t rows, int r, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const float* f = x + i * (int64_t)(2 * r + 4);
  const float d2 = y[2 * i], ub2 = y[2 * i + 1];
  const float ub = sqrtf(ub2);
  const float rq = f[2 * r + 1] * ub, rd = f[2 * r + 2] * ub, proj = f[2 * r + 3] * ub2;
  const float den = 2.f * rq * rd;
  out[i] = den > 0.f ? (proj + rq * rq + rd * rd - d2) / den : 0.f;
}

}  // namespace

hipError_t launch_gate_targets(const float* x, const float* y, int64_t rows, int r, float* out,
                               hipStream_t s) {
  if (rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gate_targets, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, x, y,
                     rows, r, out);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* w, int in, int H, const float* x, int64_t B, float* y,
                              hipStream_t s) {
  if (B == 0) return hipSuccess;
  const Dims D = dims_of(in, H);
  const int lds = (2 * kTS * D.inp + 2 * kTS * D.kh) * 2;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_fwd),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((B + kTS - 1) / kTS)), dim3(64), lds, s, w, in, H, x,
                     B, y);
  return hipGetLastError();
}

size_t mlp_backward_scratch_bytes(int in, int H, int64_t B) {
  const int64_t parts = (B + kTS - 1) / kTS;
  return (size_t)(parts * offsets(in, H).total + parts) * sizeof(float);
}

hipError_t launch_mlp_backward(const float* w, int in, int H, const float* x, const float* tgt,
                               int64_t B, float* grad, float* loss, void* scratch_v, hipStream_t s) {
  const Off o = offsets(in, H);
  const Dims D = dims_of(in, H);
  const int64_t parts = (B + kTS - 1) / kTS;
  float* scratch = static_cast<float*>(scratch_v);
  const int lds = train_lds_elems(D) * 2;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_bwd),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)parts), dim3(64), lds, s, w, in, H, x, tgt, B, scratch,
                     scratch + parts * o.total);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((o.total + 255) / 256)), dim3(256), 0, s,
                     scratch, (int)parts, o.total, grad, scratch + parts * o.total, loss, B);
  return hipGetLastError();
}

int abs_err_blocks(int64_t rows) {
  const int64_t per = 65536;
  return (int)((rows + per - 1) / per);
}

hipError_t launch_abs_err_parts(const float* y, const float* t, int64_t rows, double* parts,
                                hipStream_t s) {
  const int64_t per = 65536;
  hipLaunchKernelGGL(k_abs_err_parts, dim3((unsigned)abs_err_blocks(rows)), dim3(256), 0, s, y, t, rows,
                     per, parts);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m1, float* m2, int64_t cnt, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, w, g, m1, m2,
                     cnt, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack_gate(const float* w_dev, int in, int H, uint16_t* wbf, float* b,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_pack_gate, dim3(64), dim3(256), 0, s, w_dev, in, H, wbf, b);
  return hipGetLastError();
}

}  // namespace finger
