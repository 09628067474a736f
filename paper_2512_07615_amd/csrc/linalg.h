// Small dense linear algebra for MPS rounding and centre shifts (gfx950):
//  * QR of tall-skinny problems by Householder reflections in FP64 (one
//    workgroup per matrix), robust to rank deficiency; a Cholesky-QR
//    pipeline (Gram products on MFMA) is kept for full-rank fast paths;
//  * one-sided (Hestenes) Jacobi SVD in FP64, one workgroup per matrix,
//    cyclic round-robin pairing, followed by sorting, the truncation-rank
//    rule and packing of the kept singular vectors.
#pragma once
#include "gemm.h"

namespace mpslbm {

// One QR problem: A (m x s) read through strides; Q (m x p) written packed
// row-major (ld = p), R (p x s) FP64 packed row-major, p = min(m, s).
template <typename T>
struct QrProb {
  const T* A;
  long sAm, sAk;
  int m, s, p;
  int valid;
  T* Q;
  double* R;
};

// Per-problem FP64 workspace of the QR pipeline (capacity-sized slots).
struct QrWork {
  double* G;     // s x s
  double* R1;    // s x s   (R of pass 1, 2, 3 overwrite in turn)
  double* Racc;  // s x s   accumulated R
  double* Rt;    // s x s   temporary product
  double* Rinv;  // s x s
  double* Q1;    // m x s
  double* Q2;    // m x s
  long sq;       // slot stride of the s x s buffers
  long mq;       // slot stride of the m x s buffers
};

template <typename T, typename F>
__global__ void k_qr_prep(F f, QrProb<T>* qp, int nprob) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nprob) return;
  QrProb<T> q = f.get(i);
  if (q.valid) q.p = q.m < q.s ? q.m : q.s;
  qp[i] = q;
}

// ---- GEMM functors over materialised QR problems -------------------------
// Gram: G = X^T X, X = A (pass 1, T) or Q1/Q2 (FP64).
template <typename T>
struct GramA {
  const QrProb<T>* qp; QrWork w;
  __device__ GemmDesc<T, T, double> get(int i) const {
    GemmDesc<T, T, double> d = gemm_empty<T, T, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    d.A = q.A; d.B = q.A; d.C = w.G + i * w.sq;
    d.M = q.s; d.N = q.s; d.K = q.m;
    d.sAm = q.sAk; d.sAk = q.sAm; d.sBk = q.sAm; d.sBn = q.sAk;
    d.sCm = q.s; d.sCn = 1; d.valid = 1;
    return d;
  }
};
template <typename T>
struct GramQ {
  const QrProb<T>* qp; QrWork w; int which;  // 1: Q1, 2: Q2
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    const double* X = (which == 1 ? w.Q1 : w.Q2) + i * w.mq;
    d.A = X; d.B = X; d.C = w.G + i * w.sq;
    d.M = q.s; d.N = q.s; d.K = q.m;
    d.sAm = 1; d.sAk = q.s; d.sBk = q.s; d.sBn = 1;
    d.sCm = q.s; d.sCn = 1; d.valid = 1;
    return d;
  }
};
// Q_next = X * Rinv ; pass 1 reads A (T), later passes FP64 workspaces.
template <typename T>
struct ApplyRinvA {
  const QrProb<T>* qp; QrWork w;
  __device__ GemmDesc<T, double, double> get(int i) const {
    GemmDesc<T, double, double> d = gemm_empty<T, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    d.A = q.A; d.B = w.Rinv + i * w.sq; d.C = w.Q1 + i * w.mq;
    d.M = q.m; d.N = q.s; d.K = q.s;
    d.sAm = q.sAm; d.sAk = q.sAk; d.sBk = q.s; d.sBn = 1; d.sCm = q.s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct ApplyRinvQ {
  const QrProb<T>* qp; QrWork w; int from;  // 1: Q1 -> Q2
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    d.A = w.Q1 + i * w.mq; d.B = w.Rinv + i * w.sq; d.C = w.Q2 + i * w.mq;
    d.M = q.m; d.N = q.s; d.K = q.s;
    d.sAm = q.s; d.sAk = 1; d.sBk = q.s; d.sBn = 1; d.sCm = q.s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct ApplyRinvFinal {  // Q = Q2 * Rinv -> output (type T, ld = p = s)
  const QrProb<T>* qp; QrWork w;
  __device__ GemmDesc<double, double, T> get(int i) const {
    GemmDesc<double, double, T> d = gemm_empty<double, double, T>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    d.A = w.Q2 + i * w.mq; d.B = w.Rinv + i * w.sq; d.C = q.Q;
    d.M = q.m; d.N = q.s; d.K = q.s;
    d.sAm = q.s; d.sAk = 1; d.sBk = q.s; d.sBn = 1; d.sCm = q.s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
// Racc <- R1 * Racc (upper triangular products), into Rt then swapped by caller.
template <typename T>
struct RMul {
  const QrProb<T>* qp; const double* L; long sL; const double* Rr; long sR; double* out;
  long sO;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    d.A = L + i * sL; d.B = Rr + i * sR; d.C = out + i * sO;
    d.M = q.s; d.N = q.s; d.K = q.s;
    d.sAm = q.s; d.sAk = 1; d.sBk = q.s; d.sBn = 1; d.sCm = q.s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// Cholesky G (+ shift) = R^T R (R upper) and R^{-1}; one workgroup per
// problem.  `shift_factor` > 0 adds shift_factor * trace(G) to the diagonal
// (shifted Cholesky-QR); non-positive pivots are clamped to a tiny value so
// that rank-deficient inputs still produce an orthonormal Q.
template <typename T>
__global__ __launch_bounds__(256) void k_chol_inv(const QrProb<T>* qp, QrWork w, int pass,
                                                  int lds_elems) {
  extern __shared__ double sh[];
  __shared__ double red[8];
  __shared__ double piv;
  QrProb<T> q = qp[blockIdx.x];
  if (!q.valid || q.m <= q.s) return;
  const int s = q.s, tid = threadIdx.x;
  double* Gg = w.G + blockIdx.x * w.sq;
  double* R = w.R1 + blockIdx.x * w.sq;
  double* Ri = w.Rinv + blockIdx.x * w.sq;
  double* G = (s * s <= lds_elems) ? sh : Gg;
  if (G != Gg)
    for (int e = tid; e < s * s; e += blockDim.x) G[e] = Gg[e];
  __syncthreads();
  double tr = 0.0;
  for (int e = tid; e < s; e += blockDim.x) tr += G[e * s + e];
  tr = block_sum(tr, red);
  double shift = 0.0;
  if (pass == 1) {
    const double u = 1.1102230246251565e-16;
    shift = 11.0 * ((double)q.m * s + (double)s * (s + 1)) * u * tr;
  }
  const double floor_piv = (tr > 0.0 ? tr : 1.0) * 1e-300 + 1e-300;
  if (shift > 0.0)
    for (int e = tid; e < s; e += blockDim.x) G[e * s + e] += shift;
  __syncthreads();
  // right-looking Cholesky on the upper triangle: R[j][c] for c >= j
  for (int j = 0; j < s; ++j) {
    if (tid == 0) {
      double dj = G[j * s + j];
      if (!(dj > floor_piv)) dj = floor_piv;
      piv = sqrt(dj);
    }
    __syncthreads();
    double rjj = piv;
    for (int c = j + tid; c < s; c += blockDim.x) {
      double v = (c == j) ? rjj : G[j * s + c] / rjj;
      G[j * s + c] = v;
    }
    __syncthreads();
    int rem = s - j - 1;
    long tot = (long)rem * rem;
    for (long e = tid; e < tot; e += blockDim.x) {
      int a = j + 1 + (int)(e / rem), b = j + 1 + (int)(e % rem);
      if (b >= a) G[a * s + b] -= G[j * s + a] * G[j * s + b];
    }
    __syncthreads();
  }
  // export R (zero below the diagonal)
  for (int e = tid; e < s * s; e += blockDim.x) {
    int a = e / s, b = e % s;
    R[e] = (b >= a) ? G[e] : 0.0;
  }
  __syncthreads();
  // R^{-1}: column c solves R x = e_c by back substitution (one thread per column)
  for (int c = tid; c < s; c += blockDim.x) {
    for (int i = 0; i < s; ++i) Ri[i * s + c] = 0.0;
    Ri[c * s + c] = 1.0 / G[c * s + c];
    for (int i = c - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i + 1; k <= c; ++k) acc += G[i * s + k] * Ri[k * s + c];
      Ri[i * s + c] = -acc / G[i * s + i];
    }
  }
}

// m <= s: Q = I_m, R = A (copied to FP64).
template <typename T>
__global__ void k_qr_identity(const QrProb<T>* qp) {
  QrProb<T> q = qp[blockIdx.y];
  if (!q.valid || q.m > q.s) return;
  long tot = (long)q.m * q.m + (long)q.m * q.s;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    if (e < (long)q.m * q.m) {
      int a = (int)(e / q.m), b = (int)(e % q.m);
      q.Q[e] = (T)(a == b ? 1.0 : 0.0);
    } else {
      long f = e - (long)q.m * q.m;
      int a = (int)(f / q.s), b = (int)(f % q.s);
      q.R[f] = (double)q.A[a * q.sAm + b * q.sAk];
    }
  }
}

// Copy accumulated R into the problem's output (p = s case).
template <typename T>
__global__ void k_qr_export_r(const QrProb<T>* qp, const double* Racc, long sq) {
  QrProb<T> q = qp[blockIdx.y];
  if (!q.valid || q.m <= q.s) return;
  const double* src = Racc + blockIdx.y * sq;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q.s * q.s;
       e += gridDim.x * blockDim.x)
    q.R[e] = src[e];
}

// ---------------------------------------------------------------------------
// Householder QR (FP64), one workgroup per problem, for m > s.  Reflectors
// follow the usual convention H = I - tau v v^T, v_0 = 1,
// beta = -sign(alpha) ||x||; a column that is already zero below the
// diagonal gets tau = 0.  Q = H_0 ... H_{p-1} [I; 0] is formed explicitly,
// so it is orthonormal for every input, rank-deficient ones included.
// Working copies live in LDS when they fit, else in the FP64 workspaces.
template <typename T>
__global__ __launch_bounds__(256) void k_householder(const QrProb<T>* qp, QrWork w,
                                                     int lds_elems, double* flops) {
  extern __shared__ double sh[];
  __shared__ double tau_s[1024];
  __shared__ double red[8];
  __shared__ double bcast[2];
  QrProb<T> q = qp[blockIdx.x];
  if (!q.valid || q.m <= q.s) return;
  const int m = q.m, s = q.s, p = q.p, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nw = blockDim.x >> 6;
  const bool in_lds = (long)m * s + (long)m * p <= lds_elems;
  double* Wk = in_lds ? sh : w.Q1 + blockIdx.x * w.mq;
  double* Qw = in_lds ? sh + (long)m * s : w.Q2 + blockIdx.x * w.mq;
  for (long e = tid; e < (long)m * s; e += blockDim.x) {
    int i = (int)(e % m), c = (int)(e / m);
    Wk[e] = (double)q.A[(long)i * q.sAm + (long)c * q.sAk];
  }
  __syncthreads();
  for (int j = 0; j < p; ++j) {
    double* col = Wk + (long)j * m;
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += blockDim.x) part += col[i] * col[i];
    part = block_sum(part, red);
    if (tid == 0) {
      double alpha = col[j];
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (part > 0.0) {
        double nrm = sqrt(alpha * alpha + part);
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      tau_s[j] = tau;
      bcast[0] = scale;
      bcast[1] = beta;
    }
    __syncthreads();
    const double scale = bcast[0], beta = bcast[1], tau = tau_s[j];
    if (tau != 0.0)
      for (int i = j + 1 + tid; i < m; i += blockDim.x) col[i] *= scale;
    __syncthreads();
    if (tid == 0) col[j] = beta;
    if (tau != 0.0) {
      for (int c = j + 1 + wv; c < s; c += nw) {
        double* cc = Wk + (long)c * m;
        const double cj = cc[j];  // read by every lane before lane 0 updates it
        double acc = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) acc += col[i] * cc[i];
        acc = wave_sum(acc) + cj;
        acc *= tau;
        for (int i = j + 1 + lane; i < m; i += 64) cc[i] -= acc * col[i];
        if (lane == 0) cc[j] -= acc;
      }
    }
    __syncthreads();
  }
  // R (p x s), zero below the diagonal
  for (long e = tid; e < (long)p * s; e += blockDim.x) {
    int i = (int)(e / s), c = (int)(e % s);
    q.R[e] = (c >= i) ? Wk[(long)c * m + i] : 0.0;
  }
  // Q = H_0 ... H_{p-1} [I; 0]
  for (long e = tid; e < (long)m * p; e += blockDim.x) {
    int i = (int)(e % m), c = (int)(e / m);
    Qw[e] = (i == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int j = p - 1; j >= 0; --j) {
    const double tau = tau_s[j];
    if (tau != 0.0) {
      const double* v = Wk + (long)j * m;
      for (int c = j + wv; c < p; c += nw) {
        double* cc = Qw + (long)c * m;
        const double cj = cc[j];  // read by every lane before lane 0 updates it
        double acc = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) acc += v[i] * cc[i];
        acc = wave_sum(acc) + cj;
        acc *= tau;
        for (int i = j + 1 + lane; i < m; i += 64) cc[i] -= acc * v[i];
        if (lane == 0) cc[j] -= acc;
      }
    }
    __syncthreads();
  }
  for (long e = tid; e < (long)m * p; e += blockDim.x) {
    int i = (int)(e / p), c = (int)(e % p);
    q.Q[e] = (T)Qw[(long)c * m + i];
  }
  if (flops && tid == 0) {
    // reflector generation 2(m-j), trailing update 4(m-j)(s-j-1), Q formation 4(m-j)(p-j)
    double f = 0.0;
    for (int j = 0; j < p; ++j)
      f += 2.0 * (m - j) + 4.0 * (m - j) * (s - j - 1) + 4.0 * (m - j) * (p - j);
    atomicAdd(flops, f);
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi SVD (FP64) with truncation.
// L (rows x cols, column-major, ld = rows) and W (cols x cols, column-major)
// are rotated in place: L W = U S.  Afterwards singular values are sorted,
// the rank is chosen by the tail rule (smallest r >= 1 with
// sum_{j >= r} s_j^2 <= delta2, capped at chi) and the kept columns are
// packed: US (rows x r, row-major, ld r) and Wk (cols x r, row-major, ld r).
struct SvdProb {
  double* L;
  double* W;
  int rows, cols;
  int valid;
  double delta2;   // per-bond threshold
  int chi;
  int* rank_out;   // where the chosen rank is stored (an MPS bond)
  double* US;      // rows x r
  double* Wk;      // cols x r
  double* sv;      // singular values (sorted) out, length cols (may be null)
  double* disc;    // discarded weight out (may be null)
  int* fail;       // incremented when the sweep limit is hit (may be null)
};

template <typename F>
__global__ void k_svd_prep(F f, SvdProb* sp, int nprob) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nprob) sp[i] = f.get(i);
}

__global__ __launch_bounds__(256) void k_jacobi_svd(const SvdProb* sp, int lds_elems,
                                                    int max_sweeps, double* flops) {
  extern __shared__ double sh[];
  __shared__ int rotated;
  __shared__ int perm[1024];
  __shared__ double red[8];
  SvdProb p = sp[blockIdx.x];
  if (!p.valid) return;
  const int m = p.rows, n = p.cols, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nwaves = blockDim.x >> 6;
  bool in_lds = (long)m * n + (long)n * n <= lds_elems;
  double* L = in_lds ? sh : p.L;
  double* W = in_lds ? sh + (long)m * n : p.W;
  if (in_lds)
    for (long e = tid; e < (long)m * n; e += blockDim.x) L[e] = p.L[e];
  for (long e = tid; e < (long)n * n; e += blockDim.x) W[e] = ((e / n) == (e % n)) ? 1.0 : 0.0;
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double tol = eps * sqrt((double)(m > 1 ? m : 1));
  const int P = (n % 2) ? n + 1 : n;  // players (one dummy if odd)
  double work = 0.0;  // algorithmic flops of this wave (pairs tested, rotations applied)
  int sweep = 0;
  for (; sweep < max_sweeps && n > 1; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int t = 0; t < P - 1; ++t) {
      for (int k = wv; k < P / 2; k += nwaves) {
        int i1, i2;
        if (k == 0) { i1 = t; i2 = P - 1; }
        else { i1 = (t + k) % (P - 1); i2 = (t - k + (P - 1)) % (P - 1); }
        if (i1 >= n || i2 >= n) continue;
        int a = i1 < i2 ? i1 : i2, b = i1 < i2 ? i2 : i1;
        double* ca = L + (long)a * m;
        double* cb = L + (long)b * m;
        double al = 0, be = 0, ga = 0;
        for (int r = lane; r < m; r += 64) {
          double x = ca[r], y = cb[r];
          al += x * x; be += y * y; ga += x * y;
        }
        al = wave_sum(al); be = wave_sum(be); ga = wave_sum(ga);
        work += 6.0 * m;
        // relative orthogonality test; sqrt(al) sqrt(be) avoids underflow of al * be
        if (ga == 0.0 || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        double zeta = (be - al) / (2.0 * ga);
        double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double cs = 1.0 / sqrt(1.0 + tt * tt), sn = cs * tt;
        for (int r = lane; r < m; r += 64) {
          double x = ca[r], y = cb[r];
          ca[r] = cs * x - sn * y;
          cb[r] = sn * x + cs * y;
        }
        double* wa = W + (long)a * n;
        double* wb = W + (long)b * n;
        for (int r = lane; r < n; r += 64) {
          double x = wa[r], y = wb[r];
          wa[r] = cs * x - sn * y;
          wb[r] = sn * x + cs * y;
        }
        if (lane == 0) rotated = 1;
        work += 6.0 * m + 6.0 * n;
      }
      __syncthreads();
    }
    int any = rotated;
    __syncthreads();
    if (!any) break;
  }
  if (sweep >= max_sweeps && tid == 0 && p.fail) atomicAdd(p.fail, 1);
  if (flops && lane == 0) atomicAdd(flops, work);
  // singular values = column norms (stored temporarily in W's spare? use global sv)
  double* sv = p.sv;
  // column norms into a scratch region: reuse perm-sorted pass with LDS array
  __shared__ double nrm[1024];
  __shared__ int nonfin;
  if (tid == 0) nonfin = 0;
  __syncthreads();
  for (int c = wv; c < n; c += nwaves) {
    double acc = 0.0;
    for (int r = lane; r < m; r += 64) acc += L[(long)c * m + r] * L[(long)c * m + r];
    acc = wave_sum(acc);
    if (lane == 0) {
      double v = sqrt(acc);
      // a non-finite norm is ranked last and reported; the sort below must
      // stay a permutation whatever the values
      if (!(v <= 1.7976931348623157e308)) {
        nonfin = 1;
        v = -1.0;
      }
      nrm[c] = v;
    }
  }
  __syncthreads();
  if (tid == 0 && nonfin && p.fail) atomicAdd(p.fail + 1, 1);
  // sort descending (rank by counting; ties by index)
  for (int c = tid; c < n; c += blockDim.x) {
    int pos = 0;
    double v = nrm[c];
    for (int o = 0; o < n; ++o) {
      double u = nrm[o];
      if (u > v || (u == v && o < c)) ++pos;
    }
    perm[pos] = c;
  }
  __syncthreads();
  __shared__ int rsel;
  __shared__ double dsel;
  if (tid == 0) {
    // tail[r] = sum_{j >= r} s_j^2 ; choose smallest r >= 1 with tail <= delta2
    double tail = 0.0;
    int r = n;
    double tail_at_r = 0.0;
    // walk from the end accumulating
    double acc = 0.0;
    int best = n;
    for (int j = n - 1; j >= 1; --j) {
      acc += nrm[perm[j]] * nrm[perm[j]];
      if (acc <= p.delta2) { best = j; tail_at_r = acc; } else break;
    }
    r = best;
    if (r > p.chi) {
      r = p.chi;
      tail = 0.0;
      for (int j = r; j < n; ++j) tail += nrm[perm[j]] * nrm[perm[j]];
      tail_at_r = tail;
    }
    if (r < 1) r = 1;
    rsel = r;
    dsel = tail_at_r;
    if (p.rank_out) *p.rank_out = r;
    if (p.disc) *p.disc = tail_at_r;
  }
  __syncthreads();
  const int r = rsel;
  if (sv)
    for (int j = tid; j < n; j += blockDim.x) sv[j] = nrm[perm[j]];
  // pack kept columns: US[row][j] = L[perm[j]][row]; Wk[row][j] = W[perm[j]][row]
  for (long e = tid; e < (long)m * r; e += blockDim.x) {
    int row = (int)(e / r), j = (int)(e % r);
    p.US[e] = L[(long)perm[j] * m + row];
  }
  for (long e = tid; e < (long)n * r; e += blockDim.x) {
    int row = (int)(e / r), j = (int)(e % r);
    p.Wk[e] = W[(long)perm[j] * n + row];
  }
  (void)red;
  (void)dsel;
}

}  // namespace mpslbm
