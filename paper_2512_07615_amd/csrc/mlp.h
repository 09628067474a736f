// Rank-predictor network: a multilayer perceptron 33 -> 128 -> 128 -> 128
// -> 1 (ReLU on the hidden layers, linear output), FP32, with hand-written
// forward, backward (mean squared error) and Adam kernels.
//
// Input of one sample: the spectrum of a truncation around its cut -- the
// 32 singular values sigma_{r-16} .. sigma_{r+15} of the previous step (r the
// rank it kept), as log10(sigma / sigma_1) / 8, absent values as -2 -- and
// the step index / 1000.  Output: the change of the rank at the next step,
// divided by 16.
//
// Parameters live in one FP32 array: W1 (33 x 128, row-major: input row,
// output column), b1, W2 (128 x 128), b2, W3, b3, W4 (128 x 1), b4.
#pragma once
#include "common.h"

namespace mpslbm {

constexpr int MLP_IN = 33;
constexpr int MLP_H = 128;
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_IN * MLP_H;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_H * MLP_H;
constexpr int MLP_W4 = MLP_B3 + MLP_H;
constexpr int MLP_B4 = MLP_W4 + MLP_H;
constexpr int MLP_NPARAM = MLP_B4 + 1;

__global__ void k_fill_f32(float* p, float v, long cnt) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < cnt;
       e += (long)gridDim.x * blockDim.x)
    p[e] = v;
}

// Z = X W + b (B x O), A = relu(Z) or Z; one thread per output element
__global__ void k_dense_fwd(const float* X, int I, const float* W, const float* b, int O,
                            float* Z, float* A, int B, int relu) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)B * O) return;
  const int s = (int)(e / O), o = (int)(e % O);
  float z = b[o];
  const float* x = X + (long)s * I;
  for (int i = 0; i < I; ++i) z += x[i] * W[(long)i * O + o];
  Z[e] = z;
  A[e] = relu ? fmaxf(z, 0.0f) : z;
}

// dY = 2 (Y - T) / B (Y, T: B x 1) and the loss mean (Y - T)^2, one block
__global__ void k_mse_grad(const float* Y, const float* T, int B, float* dY, float* loss) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int s = threadIdx.x; s < B; s += blockDim.x) {
    const float d = Y[s] - T[s];
    dY[s] = 2.0f * d / (float)B;
    acc += (double)d * d;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0 && loss) *loss = (float)(acc / B);
}

// dX = dZ W^T (B x I), times relu'(Zprev) when the layer below has a ReLU
__global__ void k_dense_bwd_x(const float* dZ, int O, const float* W, int I, const float* Zprev,
                              float* dX, int B) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)B * I) return;
  const int s = (int)(e / I), i = (int)(e % I);
  const float* dz = dZ + (long)s * O;
  const float* w = W + (long)i * O;
  float g = 0.0f;
  for (int o = 0; o < O; ++o) g += dz[o] * w[o];
  if (Zprev && !(Zprev[e] > 0.0f)) g = 0.0f;
  dX[e] = g;
}

// dW = X^T dZ (I x O) and db = column sums of dZ; one thread per (i, o),
// threads with i == I produce db
__global__ void k_dense_bwd_w(const float* X, int I, const float* dZ, int O, int B, float* dW,
                              float* db) {
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)(I + 1) * O) return;
  const int i = (int)(e / O), o = (int)(e % O);
  float g = 0.0f;
  if (i < I) {
    for (int s = 0; s < B; ++s) g += X[(long)s * I + i] * dZ[(long)s * O + o];
    dW[(long)i * O + o] = g;
  } else {
    for (int s = 0; s < B; ++s) g += dZ[(long)s * O + o];
    db[o] = g;
  }
}

// Adam (Kingma and Ba, 2015) with bias correction factors c1 = 1 - beta1^t,
// c2 = 1 - beta2^t
__global__ void k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float c1,
                       float c2) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[e] + (1.0f - b1) * g[e];
  const float vv = b2 * v[e] + (1.0f - b2) * g[e] * g[e];
  m[e] = mm;
  v[e] = vv;
  p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// He-uniform weights (bound sqrt(6 / fan_in)) from a counter-based
// generator (the SplitMix64 finaliser of Steele, Lea and Flood, 2014, applied
// to seed + golden-ratio increment times the element index), zero biases
__global__ void k_mlp_init(float* p, uint64_t seed) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= MLP_NPARAM) return;
  int fan = 0;
  if (e < MLP_B1) fan = MLP_IN;
  else if (e >= MLP_W2 && e < MLP_B2) fan = MLP_H;
  else if (e >= MLP_W3 && e < MLP_B3) fan = MLP_H;
  else if (e >= MLP_W4 && e < MLP_B4) fan = MLP_H;
  if (fan == 0) {
    p[e] = 0.0f;
    return;
  }
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(e + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);  // [0, 1)
  p[e] = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan));
}

// Activations and gradients of one batch; device buffers sized for bmax.
struct Mlp {
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  float *z1, *a1, *z2, *a2, *z3, *a3, *y, *dy, *d3, *d2, *d1, *loss;
  int bmax = 0;
  long t = 0;  // Adam steps taken

  template <typename Alloc>
  void setup(int bmax_, Alloc alloc, uint64_t seed, hipStream_t st) {
    bmax = bmax_;
    p = (float*)alloc(4L * MLP_NPARAM);
    g = (float*)alloc(4L * MLP_NPARAM);
    m = (float*)alloc(4L * MLP_NPARAM);
    v = (float*)alloc(4L * MLP_NPARAM);
    float** acts[] = {&z1, &a1, &z2, &a2, &z3, &a3, &d3, &d2, &d1};
    for (float** a : acts) *a = (float*)alloc(4L * bmax * MLP_H);
    y = (float*)alloc(4L * bmax);
    dy = (float*)alloc(4L * bmax);
    loss = (float*)alloc(64);
    hipLaunchKernelGGL(k_mlp_init, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, p, seed);
    hipLaunchKernelGGL(k_fill_f32, dim3(64), dim3(256), 0, st, m, 0.0f, (long)MLP_NPARAM);
    hipLaunchKernelGGL(k_fill_f32, dim3(64), dim3(256), 0, st, v, 0.0f, (long)MLP_NPARAM);
  }
  static unsigned blocks(long n) { return (unsigned)((n + 255) / 256); }
  // y (B) = f(X), X: B x 33 on the device, B <= bmax
  void forward(const float* X, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st, X, MLP_IN,
                       (const float*)(p + MLP_W1), (const float*)(p + MLP_B1), MLP_H, z1, a1, B, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st,
                       (const float*)a1, MLP_H, (const float*)(p + MLP_W2),
                       (const float*)(p + MLP_B2), MLP_H, z2, a2, B, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st,
                       (const float*)a2, MLP_H, (const float*)(p + MLP_W3),
                       (const float*)(p + MLP_B3), MLP_H, z3, a3, B, 1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(blocks(B)), dim3(256), 0, st, (const float*)a3, MLP_H,
                       (const float*)(p + MLP_W4), (const float*)(p + MLP_B4), 1, y, y, B, 0);
  }
  // loss and gradient g of the mean squared error against T (B) after forward
  void backward(const float* X, const float* T, int B, hipStream_t st) {
    hipLaunchKernelGGL(k_mse_grad, dim3(1), dim3(256), 0, st, (const float*)y, T, B, dy, loss);
    // layer 4: dW4, db4; d3 = dy W4^T relu'(z3)
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((MLP_H + 1) * 1L)), dim3(256), 0, st,
                       (const float*)a3, MLP_H, (const float*)dy, 1, B, g + MLP_W4, g + MLP_B4);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st,
                       (const float*)dy, 1, (const float*)(p + MLP_W4), MLP_H, (const float*)z3,
                       d3, B);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((MLP_H + 1L) * MLP_H)), dim3(256), 0, st,
                       (const float*)a2, MLP_H, (const float*)d3, MLP_H, B, g + MLP_W3,
                       g + MLP_B3);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st,
                       (const float*)d3, MLP_H, (const float*)(p + MLP_W3), MLP_H,
                       (const float*)z2, d2, B);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((MLP_H + 1L) * MLP_H)), dim3(256), 0, st,
                       (const float*)a1, MLP_H, (const float*)d2, MLP_H, B, g + MLP_W2,
                       g + MLP_B2);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(blocks((long)B * MLP_H)), dim3(256), 0, st,
                       (const float*)d2, MLP_H, (const float*)(p + MLP_W2), MLP_H,
                       (const float*)z1, d1, B);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(blocks((MLP_IN + 1L) * MLP_H)), dim3(256), 0, st, X,
                       MLP_IN, (const float*)d1, MLP_H, B, g + MLP_W1, g + MLP_B1);
  }
  void adam(float lr, hipStream_t st) {
    ++t;
    const float c1 = 1.0f - powf(0.9f, (float)t), c2 = 1.0f - powf(0.999f, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(MLP_NPARAM)), dim3(256), 0, st, p, (const float*)g, m,
                       v, MLP_NPARAM, lr, c1, c2);
  }
};

}  // namespace mpslbm
