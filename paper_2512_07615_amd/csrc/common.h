// Shared device/host definitions of the MPS-LBM library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <stdexcept>
#include <string>

namespace mpslbm {

constexpr int MAXN = 10;     // maximum number of sites (N <= 1024)
constexpr int PHYS = 8;      // physical dimension of a site (x, y, z bits)
constexpr int WG = 256;      // threads per workgroup for the batched kernels
constexpr int MAXB = 64;     // maximum batch of a single launch

// Device memory source of a handle: the caller's callbacks (for example a
// framework's caching allocator), each called with the handle's stream, or
// hipMalloc / hipFree when none are registered.
struct Allocator {
  void* (*alloc)(size_t bytes, void* stream, void* ctx) = nullptr;
  void (*free_)(void* ptr, void* stream, void* ctx) = nullptr;
  void* ctx = nullptr;
};

// Error carried through the host code as an exception (never crosses the ABI).
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIP_OK(expr)                                                              \
  do {                                                                            \
    hipError_t _e = (expr);                                                       \
    if (_e != hipSuccess)                                                         \
      throw ::mpslbm::Error(-3, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Device-resident descriptor of one MPS.  Core k (0-based) is stored packed,
// row-major with shape (r[k], 8, r[k+1]) at data + off[k]; the space reserved
// for it is cap[k] * 8 * cap[k+1] elements.  Ranks are updated on the device
// by the truncation kernels, so the host never needs to read them in a step.
template <typename T>
struct MpsDev {
  T* data;
  long off[MAXN];
  int cap[MAXN + 1];
  int r[MAXN + 1];
  int n;
  int pad;
};

template <typename T>
struct MpsList {
  MpsDev<T>* p[MAXB];
};

// Coefficient a * rho_0^p of a term (p in {1, 0, -1, -2}); d selects the
// domain whose rho_0 applies when several domains are advanced together.
// The scalars live in one device array (rho_0 of the domains first); s > 0
// multiplies the coefficient by entry s of that array as well (a factor the
// device updates every step, such as a time-dependent face velocity).
struct Coef {
  double a;
  int p : 4;
  int d : 12;
  int s : 16;
};

__host__ __device__ inline double coef_value(Coef c, const double* rho0) {
  double v = c.a;
  if (c.p != 0) {
    const double r = rho0[c.d];
    switch (c.p) {
      case 1: v *= r; break;
      case -1: v /= r; break;
      case -2: v /= r * r; break;
      default: break;
    }
  }
  if (c.s > 0) v *= rho0[c.s];
  return v;
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum for a 256-thread workgroup; `red` has >= 4 entries.
// Block-wide copy of cnt doubles.  Each thread issues eight loads before
// its stores, so that the latencies of global loads overlap instead of
// adding up one iteration at a time.
__device__ __forceinline__ void block_copy(double* dst, const double* src, long cnt) {
  constexpr int U = 8;
  const long st = blockDim.x;
  for (long e0 = threadIdx.x; e0 < cnt; e0 += U * st) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = e0 + u * st;
      v[u] = e < cnt ? src[e] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = e0 + u * st;
      if (e < cnt) dst[e] = v[u];
    }
  }
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  int nw = (blockDim.x + 63) >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  __syncthreads();
  return s;
}

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace mpslbm
