// Bandwidth-bound MPS kernels (gfx950): block-diagonal addition, the
// shift-MPO application as a pure gather, rank-1 plane masks, copies and
// small reductions.  Every kernel reads the bond dimensions from the device
// descriptors, so launches are sized by capacity and need no host sync.
#pragma once
#include "common.h"

namespace mpslbm {

template <typename T>
__device__ inline T* core_ptr(MpsDev<T>* m, int k) { return m->data + m->off[k]; }

// ---------------------------------------------------------------------------
// dst = ca * A + cb * B: block-diagonal cores, bonds add (add equation of
// the paper).  The coefficients scale the first core of each block.
// grid: (chunks, n, count); n >= 2.
struct CoefArr {
  Coef c[MAXB];
};

template <typename T>
__global__ void k_add(MpsList<T> dst, MpsList<T> A, MpsList<T> B, CoefArr coefs,
                      const double* rho0) {
  int pr = blockIdx.z, k = blockIdx.y;
  MpsDev<T>* d = dst.p[pr];
  MpsDev<T>* a = A.p[pr];
  MpsDev<T>* b = B.p[pr];
  const int n = a->n;
  if (k >= n) return;
  const int al = a->r[k], ar = a->r[k + 1], bl = b->r[k], br = b->r[k + 1];
  const int dl = (k == 0) ? 1 : al + bl;
  const int dr = (k == n - 1) ? 1 : ar + br;
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    d->r[0] = 1;
    d->r[n] = 1;
    for (int j = 1; j < n; ++j) d->r[j] = a->r[j] + b->r[j];
  }
  double ca = 1.0, cb = 1.0;
  if (k == 0) {
    ca = coef_value(coefs.c[2 * pr], rho0);
    cb = coef_value(coefs.c[2 * pr + 1], rho0);
  }
  const T* pa = core_ptr(a, k);
  const T* pb = core_ptr(b, k);
  T* pd = core_ptr(d, k);
  const long tot = (long)dl * PHYS * dr;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const int l = (int)(e / (PHYS * dr));
    const int rem = (int)(e % (PHYS * dr));
    const int s = rem / dr, r = rem % dr;
    double v = 0.0;
    if (k == 0) {
      v = (r < ar) ? ca * (double)pa[(long)s * ar + r] : cb * (double)pb[(long)s * br + (r - ar)];
    } else if (k == n - 1) {
      v = (l < al) ? (double)pa[(long)l * PHYS + s] : (double)pb[(long)(l - al) * PHYS + s];
    } else if (l < al && r < ar) {
      v = (double)pa[((long)l * PHYS + s) * ar + r];
    } else if (l >= al && r >= ar) {
      v = (double)pb[((long)(l - al) * PHYS + s) * br + (r - ar)];
    }
    pd[e] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// Streaming shift along one axis: out(x) = in(x - c), c = +-1, written as
// the MPO of a binary incrementer/decrementer acting on one bit of each
// site (Section 2.5: the shift MPO has bond dimension 2; here its entries
// are generated from the carry rule instead of being stored).  With
// d = -c, in(x) is read at x + d.  At site k (k = 0 most significant) the
// output bit y and the carry coming from the less significant sites give
// the input bit y ^ carry and the carry passed on:
//   d = +1 (increment): carry_out = y & carry_in
//   d = -1 (decrement): carry_out = !y & carry_in
// The least significant site receives carry_in = 1.  At the most
// significant site a carry_out of 1 means the source lies outside the
// domain: cyclic shifts keep it (wrap-around), non-cyclic ones drop it.
// Result core k: [(cout, a), s_out, (cin, a')] with bonds 2 r.
// grid: (chunks, n, count)
struct IntArr {
  int v[MAXB];
};

struct RankArr {
  int r[MAXN + 1];
};

template <typename T>
__global__ void k_shift(MpsList<T> dst, MpsList<T> src, IntArr axis_arr, IntArr dir_arr,
                        IntArr cyc_arr) {
  int pr = blockIdx.z, k = blockIdx.y;
  MpsDev<T>* d = dst.p[pr];
  MpsDev<T>* a = src.p[pr];
  const int n = a->n;
  if (k >= n) return;
  const int axis = axis_arr.v[pr], dd = -dir_arr.v[pr], cyclic = cyc_arr.v[pr];
  const int bit = 2 - axis;  // sigma = 4 x + 2 y + z
  int al = a->r[k], ar = a->r[k + 1];
  int gl = (k == 0) ? 1 : 2;          // left MPO bond (cout) extent
  int gr = (k == n - 1) ? 1 : 2;      // right MPO bond (cin) extent
  int dl = gl * al, dr = gr * ar;
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    d->r[0] = 1;
    d->r[n] = 1;
    for (int j = 1; j < n; ++j) d->r[j] = 2 * a->r[j];
  }
  const T* pa = core_ptr(a, k);
  T* pd = core_ptr(d, k);
  long tot = (long)dl * PHYS * dr;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    int L = (int)(e / (PHYS * dr));
    int rem = (int)(e % (PHYS * dr));
    int so = rem / dr, R = rem % dr;
    int cout_idx = (k == 0) ? -1 : L / al;
    int aa = (k == 0) ? L : L % al;
    int cin = (k == n - 1) ? 1 : R / ar;
    int ap = (k == n - 1) ? R : R % ar;
    int y = (so >> bit) & 1;
    int xin = y ^ cin;
    int cout = (dd > 0) ? (y & cin) : ((y ^ 1) & cin);
    bool ok;
    if (k == 0) ok = cyclic ? true : (cout == 0);
    else ok = (cout == cout_idx);
    T v = (T)0;
    if (ok) {
      int si = (so & ~(1 << bit)) | (xin << bit);
      v = pa[((long)aa * PHYS + si) * ar + ap];
    }
    pd[e] = v;
  }
}

// ---------------------------------------------------------------------------
// dst = m_B (.) src for the plane x_axis = index (rank-1 mask): exact
// slicing of the physical index, ranks unchanged.  grid: (chunks, n, count)
template <typename T>
__global__ void k_slice(MpsList<T> dst, MpsList<T> src, IntArr axis_arr, IntArr idx_arr) {
  int pr = blockIdx.z, k = blockIdx.y;
  MpsDev<T>* d = dst.p[pr];
  MpsDev<T>* a = src.p[pr];
  const int n = a->n;
  if (k >= n) return;
  int axis = axis_arr.v[pr], index = idx_arr.v[pr];
  int want = (index >> (n - 1 - k)) & 1;
  int bit = 2 - axis;
  int al = a->r[k], ar = a->r[k + 1];
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0)
    for (int j = 0; j <= n; ++j) d->r[j] = a->r[j];
  const T* pa = core_ptr(a, k);
  T* pd = core_ptr(d, k);
  long tot = (long)al * PHYS * ar;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    int s = (int)((e / ar) % PHYS);
    pd[e] = (((s >> bit) & 1) == want) ? pa[e] : (T)0;
  }
}

// dst = coef * src (copy of ranks and cores; the coefficient scales core 0).
template <typename T>
__global__ void k_copy_scaled(MpsList<T> dst, MpsList<T> src, CoefArr coefs,
                              const double* rho0) {
  int pr = blockIdx.z, k = blockIdx.y;
  MpsDev<T>* d = dst.p[pr];
  MpsDev<T>* a = src.p[pr];
  const int n = a->n;
  if (k >= n) return;
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0)
    for (int j = 0; j <= n; ++j) d->r[j] = a->r[j];
  double c = (k == 0) ? coef_value(coefs.c[pr], rho0) : 1.0;
  const T* pa = core_ptr(a, k);
  T* pd = core_ptr(d, k);
  long tot = (long)a->r[k] * PHYS * a->r[k + 1];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    pd[e] = (T)(c * (double)pa[e]);
}

// Rank-1 MPS with every core = 1 (the unit MPS) or a plane-restricted one.
template <typename T>
__global__ void k_set_ones(MpsList<T> dst, int count) {
  int pr = blockIdx.x;
  if (pr >= count) return;
  MpsDev<T>* d = dst.p[pr];
  const int n = d->n;
  if (threadIdx.x == 0)
    for (int j = 0; j <= n; ++j) d->r[j] = 1;
  for (int e = threadIdx.x; e < n * PHYS; e += blockDim.x) {
    int k = e / PHYS, s = e % PHYS;
    core_ptr(d, k)[s] = (T)1;
  }
}

// <1, X> for each MPS: chain of vector-matrix products, FP64 accumulation.
// One workgroup per MPS; out[pr] = result.  Optionally out2 = out * scale2.
template <typename T>
__global__ __launch_bounds__(256) void k_inner_ones(MpsList<T> src, double* out, int count) {
  __shared__ double v[1024];
  __shared__ double vn[1024];
  int pr = blockIdx.x;
  if (pr >= count) return;
  MpsDev<T>* a = src.p[pr];
  const int n = a->n;
  if (threadIdx.x == 0) v[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    int rl = a->r[k], rr = a->r[k + 1];
    const T* c = core_ptr(a, k);
    for (int j = threadIdx.x; j < rr; j += blockDim.x) {
      double acc = 0.0;
      for (int l = 0; l < rl; ++l) {
        double sl = 0.0;
        const T* row = c + (long)l * PHYS * rr + j;
        for (int s = 0; s < PHYS; ++s) sl += (double)row[s * rr];
        acc += v[l] * sl;
      }
      vn[j] = acc;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < rr; j += blockDim.x) v[j] = vn[j];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[pr] = v[0];
}

// delta2[pr] = tol^2 * ||core_{n-1}||^2 / (n-1) (centre at the last site
// after left orthogonalisation); norm2 kept for the discarded-weight ratio.
// Inner product <A, B> = sum over all indices of A B, by the left
// environment E_k = sum_s A_k[s]^T E_{k-1} B_k[s] (E_0 = 1), two launches a
// site.  First half: T[a][s][b'] = sum_b E[a][b] B_k[b][s][b'].
template <typename T>
__global__ __launch_bounds__(256) void k_ip_half(const MpsDev<T>* A, const MpsDev<T>* B, int k,
                                                 const double* E, double* Tm) {
  const int ra = A->r[k], rb = B->r[k], rb1 = B->r[k + 1];
  const long row = (long)PHYS * rb1;
  const long tot = (long)ra * row;
  const T* Bk = B->data + B->off[k];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const long a = e / row, sb = e % row;
    double acc = 0.0;
    for (int b = 0; b < rb; ++b) acc += E[a * rb + b] * (double)Bk[b * row + sb];
    Tm[e] = acc;
  }
}

// Second half: E_k[a'][b'] = sum_{a, s} A_k[a][s][a'] T[a][s][b'].
template <typename T>
__global__ __launch_bounds__(256) void k_ip_env(const MpsDev<T>* A, const MpsDev<T>* B, int k,
                                                const double* Tm, double* E) {
  const int ra = A->r[k], ra1 = A->r[k + 1], rb1 = B->r[k + 1];
  const long tot = (long)ra1 * rb1;
  const T* Ak = A->data + A->off[k];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    const long a1 = e / rb1, b1 = e % rb1;
    double acc = 0.0;
    for (long as = 0; as < (long)ra * PHYS; ++as)
      acc += (double)Ak[as * ra1 + a1] * Tm[as * rb1 + b1];
    E[e] = acc;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_round_threshold(MpsList<T> src, double tol,
                                                         double* delta2, double* norm2,
                                                         int count) {
  __shared__ double red[8];
  int pr = blockIdx.x;
  if (pr >= count) return;
  MpsDev<T>* a = src.p[pr];
  const int n = a->n;
  const T* c = core_ptr(a, n - 1);
  long tot = (long)a->r[n - 1] * PHYS * a->r[n];
  double acc = 0.0;
  for (long e = threadIdx.x; e < tot; e += blockDim.x) acc += (double)c[e] * (double)c[e];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) {
    norm2[pr] = acc;
    delta2[pr] = (n > 1) ? tol * tol * acc / (double)(n - 1) : 0.0;
  }
}

// Copy a packed matrix (rows x cols at ld cols) from a workspace into core k
// of each MPS (the shape is taken from the MPS ranks after the update).
// Two such copies in one launch (blockIdx.z picks the pair member); the
// cores have fixed slots, so the two never overlap.
template <typename T>
__global__ void k_store_core2(MpsList<T> dst, const T* tmp0, long slot0, int k0, const T* tmp1,
                              long slot1, int k1) {
  const int pr = blockIdx.y, k = blockIdx.z ? k1 : k0;
  MpsDev<T>* d = dst.p[pr];
  const long tot = (long)d->r[k] * PHYS * d->r[k + 1];
  const T* s = (blockIdx.z ? tmp1 + pr * slot1 : tmp0 + pr * slot0);
  T* o = core_ptr(d, k);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    o[e] = s[e];
}

template <typename T>
__global__ void k_store_core(MpsList<T> dst, const T* tmp, long slot, int k) {
  int pr = blockIdx.y;
  MpsDev<T>* d = dst.p[pr];
  long tot = (long)d->r[k] * PHYS * d->r[k + 1];
  const T* s = tmp + pr * slot;
  T* o = core_ptr(d, k);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    o[e] = s[e];
}

// ---------------------------------------------------------------------------
// Dense helpers (initialisation and read-back).
// scale order: linear index of sigma_1..sigma_n (sigma_1 most significant)
// from (x, y, z): bit k of each coordinate goes to site k.
__device__ inline long scale_index(int x, int y, int z, int n) {
  long idx = 0;
  for (int k = 0; k < n; ++k) {
    int sh = n - 1 - k;
    int s = (((x >> sh) & 1) << 2) | (((y >> sh) & 1) << 1) | ((z >> sh) & 1);
    idx = idx * PHYS + s;
  }
  return idx;
}

// out[q][scale(x,y,z)] = in[q][x][y][z] (to_scale = 1) or the inverse.
template <typename TI, typename TO>
__global__ void k_scale_permute(const TI* in, TO* out, int n, int nfields, int to_scale) {
  long N = 1L << n, N3 = N * N * N;
  long tot = N3 * nfields;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    long q = e / N3, r = e % N3;
    int x = (int)(r / (N * N)), y = (int)((r / N) % N), z = (int)(r % N);
    long si = scale_index(x, y, z, n);
    if (to_scale) out[q * N3 + si] = (TO)in[e];
    else out[e] = (TO)in[q * N3 + si];
  }
}

// Initial equilibrium populations f_i = (1 - m) w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)
__global__ void k_feq_dense(const double* rho, const double* u, const uint8_t* solid,
                            double* f, long N3, const int* cvec, const double* w, int q) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    double r = rho[e], ux = u[e], uy = u[N3 + e], uz = u[2 * N3 + e];
    double fl = solid ? (solid[e] ? 0.0 : 1.0) : 1.0;
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < q; ++i) {
      double cu = cvec[3 * i] * ux + cvec[3 * i + 1] * uy + cvec[3 * i + 2] * uz;
      f[i * N3 + e] = fl * w[i] * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
    }
  }
}

// Counter-based standard normals (splitmix64 hash + Box-Muller) for the
// randomized range finder of the initial decomposition.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
template <typename T>
__global__ void k_gauss(T* out, long count, uint64_t seed) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    uint64_t h1 = splitmix64(seed ^ (2 * (uint64_t)e));
    uint64_t h2 = splitmix64(seed ^ (2 * (uint64_t)e + 1));
    double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740993.0);
    double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
    out[e] = (T)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
}

// Non-finite scan of every core of a list (sets *flag = 1).
template <typename T>
__global__ void k_nonfinite(MpsList<T> src, int* flag) {
  int pr = blockIdx.z, k = blockIdx.y;
  MpsDev<T>* a = src.p[pr];
  if (k >= a->n) return;
  long tot = (long)a->r[k] * PHYS * a->r[k + 1];
  const T* c = core_ptr(a, k);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    double v = (double)c[e];
    if (!(v == v) || v - v != 0.0) *flag = 1;
  }
}

}  // namespace mpslbm

namespace mpslbm {
// per-block sums over entries of (a - b)^2 (out[block]) and b^2
// (out[gridDim.x + block]), FP64, for the mask decomposition error
template <typename T>
__global__ __launch_bounds__(256) void k_diff_norm(const T* a, const T* b, long count,
                                                   double* out) {
  __shared__ double red[8];
  double d = 0.0, q = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x) {
    double x = (double)a[e], y = (double)b[e];
    d += (x - y) * (x - y);
    q += y * y;
  }
  d = block_sum(d, red);
  q = block_sum(q, red);
  if (threadIdx.x == 0) {
    out[blockIdx.x] = d;
    out[gridDim.x + blockIdx.x] = q;
  }
}
}  // namespace mpslbm
