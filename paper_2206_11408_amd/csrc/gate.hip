// Learned skip gate (an extension beyond the paper): a perceptron
// in -> H -> H -> 1 with ReLU, trained to predict cos(q_res, d_res) from the
// screening features the search logs.  Operands are rounded to bfloat16,
// products accumulate in float32.  Weight layout (float):
//   W1 [H][in], b1 [H], W2 [H][H], b2 [H], W3 [H], b3 [1].
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "internal.h"

namespace finger {

namespace {

constexpr int kHMax = 64;
constexpr int kBwdRows = 64;  // samples per backward block

__device__ __forceinline__ float rbf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

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

// forward of one sample, keeping pre-activations for the backward pass
__device__ __forceinline__ float fwd_one(const float* __restrict__ w, int in, int H,
                                         const float* __restrict__ x, float* z1, float* h1,
                                         float* z2, float* h2) {
  const Off o = offsets(in, H);
#pragma unroll
  for (int j = 0; j < kHMax; ++j) z1[j] = j < H ? w[o.b1 + j] : 0.f;
  for (int i = 0; i < in; ++i) {
    const float xi = rbf(x[i]);
#pragma unroll
    for (int j = 0; j < kHMax; ++j)
      if (j < H) z1[j] += rbf(w[o.w1 + (int64_t)j * in + i]) * xi;
  }
#pragma unroll
  for (int j = 0; j < kHMax; ++j) h1[j] = rbf(fmaxf(z1[j], 0.f));
#pragma unroll
  for (int j = 0; j < kHMax; ++j) {
    float acc = j < H ? w[o.b2 + j] : 0.f;
    if (j < H)
      for (int i = 0; i < H; ++i) acc += rbf(w[o.w2 + (int64_t)j * H + i]) * h1[i];
    z2[j] = acc;
    h2[j] = rbf(fmaxf(acc, 0.f));
  }
  float y = w[o.b3];
#pragma unroll
  for (int j = 0; j < kHMax; ++j)
    if (j < H) y += rbf(w[o.w3 + j]) * h2[j];
  return y;
}

__global__ void k_mlp_fwd(const float* w, int in, int H, const float* x, int64_t B, float* y) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  float z1[kHMax], h1[kHMax], z2[kHMax], h2[kHMax];
  y[b] = fwd_one(w, in, H, x + b * in, z1, h1, z2, h2);
}

// Backward of the mean squared error over the batch.  Block p handles
// samples [p*64, p*64+64): each thread first runs one sample forward and
// backward to its pre-activation gradients (kept in LDS), then the block
// forms its partial parameter gradients (sums over its samples in a fixed
// order) and writes them to partial[p].
__global__ void __launch_bounds__(kBwdRows) k_mlp_bwd(const float* w, int in, int H,
                                                      const float* x, const float* tgt, int64_t B,
                                                      float* partial, float* loss_part) {
  extern __shared__ __align__(16) float sm[];
  float* sx = sm;                           // [64][in] bf16-rounded inputs
  float* sh1 = sx + kBwdRows * in;          // [64][H]
  float* sd1 = sh1 + kBwdRows * H;          // [64][H]  dL/dz1
  float* sh2 = sd1 + kBwdRows * H;          // [64][H]
  float* sd2 = sh2 + kBwdRows * H;          // [64][H]  dL/dz2
  float* sdy = sd2 + kBwdRows * H;          // [64]
  const Off o = offsets(in, H);
  const int t = threadIdx.x;
  const int64_t b = (int64_t)blockIdx.x * kBwdRows + t;
  float z1[kHMax], h1[kHMax], z2[kHMax], h2[kHMax];
  float dy = 0.f, se = 0.f;
  if (b < B) {
    const float* xb = x + b * in;
    const float y = fwd_one(w, in, H, xb, z1, h1, z2, h2);
    const float e = y - tgt[b];
    se = e * e;
    dy = 2.f * e / (float)B;
    for (int i = 0; i < in; ++i) sx[t * in + i] = rbf(xb[i]);
  } else {
    for (int i = 0; i < in; ++i) sx[t * in + i] = 0.f;
#pragma unroll
    for (int j = 0; j < kHMax; ++j) { z1[j] = 0.f; h1[j] = 0.f; z2[j] = 0.f; h2[j] = 0.f; }
  }
  float d2[kHMax];
#pragma unroll
  for (int j = 0; j < kHMax; ++j) d2[j] = (j < H && z2[j] > 0.f) ? dy * rbf(w[o.w3 + j]) : 0.f;
#pragma unroll
  for (int j = 0; j < kHMax; ++j) {
    if (j < H) {
      float acc = 0.f;
      for (int k = 0; k < H; ++k) acc += rbf(w[o.w2 + (int64_t)k * H + j]) * d2[k];
      sd1[t * H + j] = z1[j] > 0.f ? acc : 0.f;
      sh1[t * H + j] = h1[j];
      sh2[t * H + j] = h2[j];
      sd2[t * H + j] = d2[j];
    }
  }
  sdy[t] = dy;
  // loss partial (fixed-order tree over the block)
  __shared__ float red[kBwdRows];
  red[t] = se;
  __syncthreads();
  for (int s = kBwdRows / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) loss_part[blockIdx.x] = red[0];
  float* out = partial + (int64_t)blockIdx.x * o.total;
  // parameter gradients, each a sum over the block's samples in order
  for (int64_t pidx = t; pidx < o.total; pidx += kBwdRows) {
    float g = 0.f;
    if (pidx < o.b1) {
      const int j = (int)(pidx / in), i = (int)(pidx % in);
      for (int s = 0; s < kBwdRows; ++s) g += sd1[s * H + j] * sx[s * in + i];
    } else if (pidx < o.w2) {
      const int j = (int)(pidx - o.b1);
      for (int s = 0; s < kBwdRows; ++s) g += sd1[s * H + j];
    } else if (pidx < o.b2) {
      const int j = (int)((pidx - o.w2) / H), i = (int)((pidx - o.w2) % H);
      for (int s = 0; s < kBwdRows; ++s) g += sd2[s * H + j] * sh1[s * H + i];
    } else if (pidx < o.w3) {
      const int j = (int)(pidx - o.b2);
      for (int s = 0; s < kBwdRows; ++s) g += sd2[s * H + j];
    } else if (pidx < o.b3) {
      const int j = (int)(pidx - o.w3);
      for (int s = 0; s < kBwdRows; ++s) g += sdy[s] * sh2[s * H + j];
    } else {
      for (int s = 0; s < kBwdRows; ++s) g += sdy[s];
    }
    out[pidx] = g;
  }
}

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
  hipLaunchKernelGGL(k_mlp_fwd, dim3((unsigned)((B + 127) / 128)), dim3(128), 0, s, w, in, H, x,
                     B, y);
  return hipGetLastError();
}

size_t mlp_backward_scratch_floats(int in, int H, int64_t B) {
  const int64_t parts = (B + kBwdRows - 1) / kBwdRows;
  return (size_t)(parts * offsets(in, H).total + parts);
}

hipError_t launch_mlp_backward(const float* w, int in, int H, const float* x, const float* tgt,
                               int64_t B, float* grad, float* loss, hipStream_t s) {
  const Off o = offsets(in, H);
  const int64_t parts = (B + kBwdRows - 1) / kBwdRows;
  float* scratch = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&scratch),
                                (size_t)(parts * o.total + parts) * sizeof(float), s);
  if (e != hipSuccess) return e;
  const int lds = (kBwdRows * in + 4 * kBwdRows * H + kBwdRows) * (int)sizeof(float);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_bwd),
                          hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_mlp_bwd, dim3((unsigned)parts), dim3(kBwdRows), lds, s, w, in, H, x, tgt,
                       B, scratch, scratch + parts * o.total);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((o.total + 255) / 256)), dim3(256), 0, s,
                       scratch, (int)parts, o.total, grad, scratch + parts * o.total, loss, B);
    e = hipGetLastError();
  }
  hipError_t e2 = hipFreeAsync(scratch, s);
  return e != hipSuccess ? e : e2;
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
