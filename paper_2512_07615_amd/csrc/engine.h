// Host orchestration of the MPS-LBM operations on one GPU.
//
// Every operation is a short sequence of batched kernel launches on the
// engine's stream.  Bond dimensions live in device memory (MpsDev::r), so
// launches are sized by the host-known capacities and an operation never
// waits for the device.  MPS objects come from a pool of capacity-sized
// buffers and are referred to by pool index on the host.
#pragma once
#include <type_traits>
#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <cstring>
#include <string>
#include <vector>

#include "linalg.h"
#include "mpsops.h"
#include "rsvd.h"

namespace mpslbm {

// Velocity sets, opposite velocities stored as neighbours (opp(i) = i +- 1).
// D3Q19: rest (1/3), 6 axis (1/18), 12 edge velocities (1/36).  D3Q15, the
// set of the paper's 3D runs (Section 4.1): rest (2/9), 6 axis (1/9), 8
// corner velocities (1/72).  Both have c_s^2 = 1/3 and the same
// second-order equilibrium.
constexpr int QMAX = 19;
struct LatticeTab {
  int q;
  int c[QMAX][3];
  int opp[QMAX];
  double w[QMAX];
};
static const LatticeTab kD3Q19 = {
    19,
    {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
     {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1}, {-1, 0, -1}, {1, 0, -1},
     {-1, 0, 1}, {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}},
    {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17},
    {1.0 / 3.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0}};
static const LatticeTab kD3Q15 = {
    15,
    {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
     {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1},
     {-1, 1, 1}, {1, -1, -1}},
    {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13},
    {2.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
     1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0, 1.0 / 72.0,
     1.0 / 72.0}};

template <typename T>
struct Mps {
  MpsDev<T>* dev = nullptr;
  T* data = nullptr;
  int n = 0;
  int cap[MAXN + 1];
  long off[MAXN];
  long total = 0;
};

template <typename T>
__device__ inline int max_bond(const MpsDev<T>* m) {
  int b = 1;
  for (int k = 1; k < m->n; ++k) b = m->r[k] > b ? m->r[k] : b;
  return b;
}

// Product factor order: the factor with the larger maximum bond is the
// candidate (the "first factor" of the variational product); ties keep the
// written order.
template <typename T>
__device__ inline void prod_order(MpsDev<T>* x, MpsDev<T>* y, MpsDev<T>** B, MpsDev<T>** C) {
  if (max_bond(y) > max_bond(x)) {
    *B = y;
    *C = x;
  } else {
    *B = x;
    *C = y;
  }
}

// ============================================================================
// QR problem functors
// left unfolding of core k: m = 8 r_k, s = r_{k+1}
template <typename T>
struct FnQrLeft {
  MpsList<T> L; int k; T* qout; long qslot; double* rout; long rslot;
  __device__ QrProb<T> get(int i) const {
    MpsDev<T>* m = L.p[i];
    QrProb<T> q;
    q.A = core_ptr(m, k);
    q.m = PHYS * m->r[k];
    q.s = m->r[k + 1];
    q.sAm = q.s; q.sAk = 1;
    q.p = 0; q.valid = 1;
    q.Q = qout + i * qslot;
    q.R = rout + i * rslot;
    return q;
  }
};
// transpose of the right unfolding of core k: m = 8 r_{k+1}, s = r_k
template <typename T>
struct FnQrRightT {
  MpsList<T> L; int k; T* qout; long qslot; double* rout; long rslot;
  __device__ QrProb<T> get(int i) const {
    MpsDev<T>* m = L.p[i];
    QrProb<T> q;
    q.A = core_ptr(m, k);
    q.m = PHYS * m->r[k + 1];
    q.s = m->r[k];
    q.sAm = 1; q.sAk = q.m;
    q.p = 0; q.valid = 1;
    q.Q = qout + i * qslot;
    q.R = rout + i * rslot;
    return q;
  }
};
// dense matrix problems (initial decomposition): A_i = base + i*stride, m x s row-major
template <typename T>
struct FnQrDense {
  const T* A; long astride; int m, s; T* qout; long qslot; double* rout; long rslot;
  __device__ QrProb<T> get(int i) const {
    QrProb<T> q;
    q.A = A + i * astride;
    q.m = m; q.s = s; q.sAm = s; q.sAk = 1;
    q.p = 0; q.valid = 1;
    q.Q = qout + i * qslot;
    q.R = rout + i * rslot;
    return q;
  }
};

template <typename T>
__global__ void k_qr_copy_sq(const QrProb<T>* qp, const double* src, double* dst, long sq) {
  QrProb<T> q = qp[blockIdx.y];
  if (!q.valid || q.m <= q.s) return;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < q.s * q.s; e += gridDim.x * blockDim.x)
    dst[blockIdx.y * sq + e] = src[blockIdx.y * sq + e];
}

// rank updates after a QR of a core: left form r_{k+1} = p, right form r_k = p
template <typename T>
__global__ void k_set_rank_from_qr(MpsList<T> L, const QrProb<T>* qp, int bond, int cnt) {
  int i = threadIdx.x;
  if (i < cnt) L.p[i]->r[bond] = qp[i].p;
}

// ============================================================================
// GEMM functors of the rounding sweep
// tmp = R (p x s) * core_{k+1} (s x 8 r_{k+2})
template <typename T>
struct FnRTimesCore {
  MpsList<T> L; const QrProb<T>* qp; T* tmp; long slot; int k;
  __device__ GemmDesc<double, T, T> get(int i) const {
    GemmDesc<double, T, T> d = gemm_empty<double, T, T>();
    MpsDev<T>* m = L.p[i];
    QrProb<T> q = qp[i];
    int s = q.s, p = q.p, rr = m->r[k + 2];
    d.A = q.R; d.B = core_ptr(m, k + 1); d.C = tmp + i * slot;
    d.M = p; d.N = PHYS * rr; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = PHYS * rr; d.sBn = 1; d.sCm = PHYS * rr; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
// tmp = core_{k-1} ((r_{k-1} 8) x s) * X (s x r), X = US (rounding) or R'^T (canonicalisation)
template <typename T>
struct FnCoreTimesUS {
  MpsList<T> L; const QrProb<T>* qp; const double* US; long sus; T* tmp; long slot; int k;
  __device__ GemmDesc<T, double, T> get(int i) const {
    GemmDesc<T, double, T> d = gemm_empty<T, double, T>();
    MpsDev<T>* m = L.p[i];
    QrProb<T> q = qp[i];
    int s = q.s, r = m->r[k], rl = m->r[k - 1];
    d.A = core_ptr(m, k - 1); d.B = US + i * sus; d.C = tmp + i * slot;
    d.M = rl * PHYS; d.N = r; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct FnCoreTimesRt {
  MpsList<T> L; const QrProb<T>* qp; T* tmp; long slot; int k;
  __device__ GemmDesc<T, double, T> get(int i) const {
    GemmDesc<T, double, T> d = gemm_empty<T, double, T>();
    MpsDev<T>* m = L.p[i];
    QrProb<T> q = qp[i];
    int s = q.s, p = q.p, rl = m->r[k - 1];
    d.A = core_ptr(m, k - 1); d.B = q.R; d.C = tmp + i * slot;
    d.M = rl * PHYS; d.N = p; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = 1; d.sBn = s; d.sCm = p; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
// core_k = Wk^T (r x p) * Q'^T (p x 8 r_{k+1})
template <typename T>
struct FnWtQt {
  MpsList<T> L; const QrProb<T>* qp; const double* Wk; long swk; int k;
  __device__ GemmDesc<double, T, T> get(int i) const {
    GemmDesc<double, T, T> d = gemm_empty<double, T, T>();
    MpsDev<T>* m = L.p[i];
    QrProb<T> q = qp[i];
    int r = m->r[k], p = q.p, mm = q.m;
    d.A = Wk + i * swk; d.B = q.Q; d.C = core_ptr(m, k);
    d.M = r; d.N = mm; d.K = p;
    d.sAm = 1; d.sAk = r; d.sBk = 1; d.sBn = p; d.sCm = mm; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// SVD problem of the truncation step: L = R'^T (rows s, cols p) is R' read
// column-major; delta2 and the rank slot come from the MPS of entry i.
template <typename T>
struct FnSvdTrunc {
  MpsList<T> L; const QrProb<T>* qp; int k; double* W; long sw; double* US; double* Wk;
  long sus; const double* delta2; double* disc; int chi; int* fail; double* spectra;
  long sstride;
  __device__ SvdProb get(int i) const {
    QrProb<T> q = qp[i];
    SvdProb p;
    p.L = q.R; p.W = W + i * sw; p.Lw = q.R;  // rotated in place when not in LDS
    p.rows = q.s; p.cols = q.p; p.valid = 1;
    p.delta2 = delta2[i]; p.chi = chi;
    p.rank_out = &L.p[i]->r[k];
    p.US = US + i * sus; p.Wk = Wk + i * sus;
    p.sv = spectra ? spectra + i * sstride : nullptr;
    p.disc = disc + i * (MAXN + 1) + k;
    p.fail = fail;
    return p;
  }
};

__global__ void k_round_finish(const double* disc, const double* norm2, double* stats, int cnt) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < cnt; ++i) {
    double s = 0.0;
    for (int k = 0; k <= MAXN; ++k) s += disc[i * (MAXN + 1) + k];
    double ratio = norm2[i] > 0.0 ? s / norm2[i] : 0.0;
    if (ratio > stats[0]) stats[0] = ratio;
  }
}

// store the transposed Q' (m x p) as core k (p x m)
template <typename T>
__global__ void k_store_core_T(MpsList<T> L, const QrProb<T>* qp, int k) {
  int i = blockIdx.y;
  QrProb<T> q = qp[i];
  T* o = core_ptr(L.p[i], k);
  long tot = (long)q.m * q.p;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x) {
    int j = (int)(e / q.m), r = (int)(e % q.m);
    o[e] = q.Q[(long)r * q.p + j];
  }
}

// ============================================================================
// Variational product functors (Section 2.3).  Environments:
//  Lenv[k] (rD_k, rB_k, rC_k): sites 0..k-1 contracted;  Renv[k]: sites k..n-1.
// Local optimum at site p:  A_p = sum L[a,b,c] B[b,s,b'] C[c,s,c'] R[a',b',c']
//  G1: T1[a][c][s][b'] = sum_b L[a][b][c] B[b][s][b']       (batched over a)
//  G2: T2[a][s][b'][c'] = sum_c T1[a][c][s][b'] C[c][s][c']  (batched over a, s)
//  G3: A[a][s][a'] = sum_{b'c'} T2[a][s][b'c'] R[a'][b'c']
// Left environment after the centre moves right (reuses T2 of site p):
//  G3L: Lenv[p+1][a'][b'c'] = sum_{a s} A[a][s][a'] T2[a][s][b'c']
// Right environment after the centre moves left:
//  H1: U1[a'][c'][s][b] = sum_{b'} R[a'][b'][c'] B[b][s][b']  (batched over a', s)
//  H2: U2[s][a'][b][c] = sum_{c'} U1[a'][c'][s][b] C[c][s][c'] (batched over s, a')
//  (s before b in U1, so that the operand of H2 at fixed s is read in
//  contiguous rows)
//  H3: Renv[p][a][b c] = sum_{s a'} A[a][s][a'] U2[s][a'][b c]
// Environments of problem i at bond k start at env + i * estride + eoff[k]
// (each bond sized by its capacities r_A r_B r_C).  With `fixed` set, X is
// the candidate (the obstacle products, whose result keeps the population's
// bonds); otherwise the factor with the larger maximal bond is.
template <typename T>
struct ProdCtx {
  MpsList<T> D, X, Y;
  T* envL; T* envR; long estride;
  T* T1; T* T2; long tcap;
  long eoff[MAXN + 2];
  int fixed;
  __device__ void get(int i, MpsDev<T>** d, MpsDev<T>** b, MpsDev<T>** c) const {
    *d = D.p[i];
    if (fixed) {
      *b = X.p[i];
      *c = Y.p[i];
    } else {
      prod_order(X.p[i], Y.p[i], b, c);
    }
  }
  __device__ T* L(int i, int k) const { return envL + i * estride + eoff[k]; }
  __device__ T* R(int i, int k) const { return envR + i * estride + eoff[k]; }
};

template <typename T, typename Tacc>
struct FnG1 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a = D->r[p], b = B->r[p], cc = C->r[p], b2 = B->r[p + 1];
    g.A = c.L(i, p); g.B = core_ptr(B, p); g.C = c.T1 + i * c.tcap;
    g.M = cc; g.N = PHYS * b2; g.K = b; g.nb1 = a; g.nb2 = 1;
    g.sAm = 1; g.sAk = cc; g.bA1 = (long)b * cc;
    g.sBk = PHYS * b2; g.sBn = 1;
    g.sCm = PHYS * b2; g.sCn = 1; g.bC1 = (long)cc * PHYS * b2;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnG2 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a = D->r[p], cc = C->r[p], b2 = B->r[p + 1], c2 = C->r[p + 1];
    g.A = c.T1 + i * c.tcap; g.B = core_ptr(C, p); g.C = c.T2 + i * c.tcap;
    g.M = b2; g.N = c2; g.K = cc; g.nb1 = PHYS; g.nb2 = a;
    g.sAm = 1; g.sAk = PHYS * b2; g.bA1 = b2; g.bA2 = (long)cc * PHYS * b2;
    g.sBk = PHYS * c2; g.sBn = 1; g.bB1 = c2; g.bB2 = 0;
    g.sCm = c2; g.sCn = 1; g.bC1 = (long)b2 * c2; g.bC2 = (long)PHYS * b2 * c2;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnG3 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a = D->r[p], a2 = D->r[p + 1], b2 = B->r[p + 1], c2 = C->r[p + 1];
    g.A = c.T2 + i * c.tcap; g.B = c.R(i, p + 1); g.C = core_ptr(D, p);
    g.M = PHYS * a; g.N = a2; g.K = b2 * c2;
    g.sAm = (long)b2 * c2; g.sAk = 1; g.sBk = 1; g.sBn = (long)b2 * c2;
    g.sCm = a2; g.sCn = 1;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnG3L {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a = D->r[p], a2 = D->r[p + 1], b2 = B->r[p + 1], c2 = C->r[p + 1];
    g.A = core_ptr(D, p); g.B = c.T2 + i * c.tcap; g.C = c.L(i, p + 1);
    g.M = a2; g.N = b2 * c2; g.K = PHYS * a;
    g.sAm = 1; g.sAk = a2; g.sBk = (long)b2 * c2; g.sBn = 1;
    g.sCm = (long)b2 * c2; g.sCn = 1;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnH1 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a2 = D->r[p + 1], b = B->r[p], b2 = B->r[p + 1], c2 = C->r[p + 1];
    g.A = c.R(i, p + 1); g.B = core_ptr(B, p); g.C = c.T1 + i * c.tcap;
    g.M = c2; g.N = b; g.K = b2; g.nb1 = a2; g.nb2 = PHYS;
    g.sAm = 1; g.sAk = c2; g.bA1 = (long)b2 * c2;
    g.sBk = 1; g.sBn = PHYS * b2; g.bB2 = b2;
    g.sCm = PHYS * b; g.sCn = 1; g.bC1 = (long)c2 * PHYS * b; g.bC2 = b;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnH2 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a2 = D->r[p + 1], b = B->r[p], cc = C->r[p], c2 = C->r[p + 1];
    g.A = c.T1 + i * c.tcap; g.B = core_ptr(C, p); g.C = c.T2 + i * c.tcap;
    g.M = b; g.N = cc; g.K = c2; g.nb1 = PHYS; g.nb2 = a2;
    g.sAm = 1; g.sAk = PHYS * b; g.bA1 = b; g.bA2 = (long)c2 * PHYS * b;
    g.sBk = 1; g.sBn = PHYS * c2; g.bB1 = c2; g.bB2 = 0;
    g.sCm = cc; g.sCn = 1; g.bC1 = (long)a2 * b * cc; g.bC2 = (long)b * cc;
    g.valid = 1;
    return g;
  }
};
template <typename T, typename Tacc>
struct FnH3 {
  ProdCtx<T> c; int p;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>*D, *B, *C;
    c.get(i, &D, &B, &C);
    int a = D->r[p], a2 = D->r[p + 1], b = B->r[p], cc = C->r[p];
    g.A = core_ptr(D, p); g.B = c.T2 + i * c.tcap; g.C = c.R(i, p);
    g.M = a; g.N = b * cc; g.K = PHYS * a2;
    g.sAm = PHYS * a2; g.sAk = 1; g.sBk = (long)b * cc; g.sBn = 1;
    g.sCm = (long)b * cc; g.sCn = 1;
    g.valid = 1;
    return g;
  }
};

// D <- copy of the candidate factor; environment boundaries = 1
template <typename T>
__global__ void k_prod_init(ProdCtx<T> c, int n) {
  int i = blockIdx.y, k = blockIdx.x;
  MpsDev<T>*D, *B, *C;
  c.get(i, &D, &B, &C);
  if (k == 0 && threadIdx.x == 0) {
    for (int j = 0; j <= n; ++j) D->r[j] = B->r[j];
    c.L(i, 0)[0] = (T)1;
    c.R(i, n)[0] = (T)1;
  }
  if (k >= n) return;
  long tot = (long)B->r[k] * PHYS * B->r[k + 1];
  const T* s = core_ptr(B, k);
  T* o = core_ptr(D, k);
  for (long e = threadIdx.x; e < tot; e += blockDim.x) o[e] = s[e];
}

// ============================================================================
// dense-contraction functor: T_{k+1} (rows x 8 r_{k+1}) = T_k (rows x r_k) * core_k
template <typename T>
struct FnContract {
  MpsList<T> L; const T* in; T* out; long slot; long rows; int k;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    MpsDev<T>* m = L.p[i];
    int rl = m->r[k], rr = m->r[k + 1];
    g.A = in + i * slot; g.B = core_ptr(m, k); g.C = out + i * slot;
    g.M = (int)rows; g.N = PHYS * rr; g.K = rl;
    g.sAm = rl; g.sAk = 1; g.sBk = PHYS * rr; g.sBn = 1; g.sCm = PHYS * rr; g.sCn = 1;
    g.valid = 1;
    return g;
  }
};

// initial decomposition functors (shapes host-known)
template <typename T>
struct FnDense {
  const T* A; long sa; const T* B; long sb; T* C; long sc;
  int M, N, K; long sAm, sAk, sBk, sBn;
  __device__ GemmDesc<T, T, T> get(int i) const {
    GemmDesc<T, T, T> g = gemm_empty<T, T, T>();
    g.A = A + i * sa; g.B = B + i * sb; g.C = C + i * sc;
    g.M = M; g.N = N; g.K = K;
    g.sAm = sAm; g.sAk = sAk; g.sBk = sBk; g.sBn = sBn; g.sCm = N; g.sCn = 1;
    g.valid = 1;
    return g;
  }
};

template <typename T>
__global__ void k_set_identity_core(MpsList<T> L, int k, int m) {
  int i = blockIdx.y;
  T* o = core_ptr(L.p[i], k);
  long tot = (long)m * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    o[e] = (e / m == e % m) ? (T)1 : (T)0;
}

template <typename T>
__global__ void k_set_ranks(MpsList<T> L, RankArr r, int cnt) {
  int i = threadIdx.x;
  if (i >= cnt) return;
  for (int k = 0; k <= L.p[i]->n; ++k) L.p[i]->r[k] = r.r[k];
}

template <typename T>
__global__ void k_copy_plain(const T* src, T* dst, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

template <typename T>
__global__ void k_moments_dense(const T* f, double* out, long N3, int what, const int* cvec,
                                int q) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    double rho = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < q; ++i) {
      double v = (double)f[i * N3 + e];
      rho += v;
      jx += cvec[3 * i] * v;
      jy += cvec[3 * i + 1] * v;
      jz += cvec[3 * i + 2] * v;
    }
    if (what == 1) {
      out[e] = rho;
    } else {
      double s = 1.0;
      if (what == 3) s = (rho != 0.0) ? 1.0 / rho : 0.0;
      out[e] = jx * s;
      out[N3 + e] = jy * s;
      out[2 * N3 + e] = jz * s;
    }
  }
}

// sum over cells of |j / rho|^2 (0 where rho = 0) of the dense
// populations, added into *out
template <typename T>
__global__ __launch_bounds__(256) void k_u2_sum(const T* f, long N3, const int* cvec, int q,
                                                double* out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    double rho = 0, jx = 0, jy = 0, jz = 0;
    for (int i = 0; i < q; ++i) {
      const double v = (double)f[i * N3 + e];
      rho += v;
      jx += cvec[3 * i] * v;
      jy += cvec[3 * i + 1] * v;
      jz += cvec[3 * i + 2] * v;
    }
    if (rho != 0.0) acc += (jx * jx + jy * jy + jz * jz) / (rho * rho);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// out[0] = sum of the n partial sums in index order (one thread: the same
// order, hence the same bits, on every call)
__global__ void k_sum_in_order(const double* part, int n, double* out) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += part[i];
  out[0] = s;
}

// fill kernel (used instead of memset nodes in code that may be captured)
__global__ void k_fill_f64(double* p, double v, long cnt) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < cnt; e += (long)gridDim.x * blockDim.x)
    p[e] = v;
}

template <typename T>
__global__ void k_copy_ranks(MpsDev<T>* dst, const MpsDev<T>* src) {
  const int k = threadIdx.x;
  if (k <= src->n) dst->r[k] = src->r[k];
}

__global__ void k_div_scalar(const double* a, double b, double* out) {
  if (threadIdx.x == 0) out[0] = a[0] / b;
}

// ============================================================================
// FP32 policy: rank-revealing Cholesky-QR2 and Gram-eigen truncation.
template <typename T>
struct FCqGram1 {  // G = A^T A
  const QrProb<T>* qp; CholWork w;
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
struct FCqQ1 {  // Q1 = A B1 (m x rho1)
  const QrProb<T>* qp; CholWork w;
  __device__ GemmDesc<T, double, double> get(int i) const {
    GemmDesc<T, double, double> d = gemm_empty<T, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    int r1 = w.rank[2 * i];
    d.A = q.A; d.B = w.B1 + i * w.sq; d.C = w.Q1 + i * w.mq;
    d.M = q.m; d.N = r1; d.K = q.s;
    d.sAm = q.sAm; d.sAk = q.sAk; d.sBk = r1; d.sBn = 1; d.sCm = r1; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct FCqGram2 {  // G = Q1^T Q1 (rho1 x rho1)
  const QrProb<T>* qp; CholWork w;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    int r1 = w.rank[2 * i];
    const double* X = w.Q1 + i * w.mq;
    d.A = X; d.B = X; d.C = w.G + i * w.sq;
    d.M = r1; d.N = r1; d.K = q.m;
    d.sAm = 1; d.sAk = r1; d.sBk = r1; d.sBn = 1; d.sCm = r1; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct FCqQ {  // Q = Q1 B2 (m x rho2) -> output
  const QrProb<T>* qp; CholWork w;
  __device__ GemmDesc<double, double, T> get(int i) const {
    GemmDesc<double, double, T> d = gemm_empty<double, double, T>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    int r1 = w.rank[2 * i], r2 = w.rank[2 * i + 1];
    d.A = w.Q1 + i * w.mq; d.B = w.B2 + i * w.sq; d.C = q.Q;
    d.M = q.m; d.N = r2; d.K = r1;
    d.sAm = r1; d.sAk = 1; d.sBk = r2; d.sBn = 1; d.sCm = r2; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct FCqR {  // R = R2 R1 (rho2 x s) -> output
  const QrProb<T>* qp; CholWork w;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    QrProb<T> q = qp[i];
    if (!q.valid || q.m <= q.s) return d;
    int r1 = w.rank[2 * i], r2 = w.rank[2 * i + 1];
    d.A = w.R2 + i * w.sq; d.B = w.R1 + i * w.sq; d.C = q.R;
    d.M = r2; d.N = q.s; d.K = r1;
    d.sAm = r1; d.sAk = 1; d.sBk = q.s; d.sBn = 1; d.sCm = q.s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
// pass-2 rank into p; an all-zero Q (A = 0) becomes e_0 so Q stays orthonormal.
// Problems with m <= s, which the Cholesky passes skip, get Q = I_m and R = A
// (in FP64) here.  With set_rank, the final p of problem i also becomes rank
// `bond` of the i-th MPS of L (every problem, as after any QR of a core).
template <typename T>
__global__ void k_cq_finish(QrProb<T>* qp, const int* rank, int nprob, MpsList<T> L, int bond,
                            int set_rank) {
  int i = blockIdx.x;
  if (i >= nprob) return;
  QrProb<T> q = qp[i];
  int pfin = q.p;
  if (q.valid && q.m > q.s) {
    __shared__ double red[8];
    int r2 = rank[2 * i + 1];
    double acc = 0.0;
    for (int e = threadIdx.x; e < q.m; e += blockDim.x) acc += fabs((double)q.Q[(long)e * r2]);
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) {
      qp[i].p = r2;
      if (acc == 0.0) q.Q[0] = (T)1;
    }
    pfin = r2;
  } else if (q.valid) {
    const long tot = (long)q.m * q.m + (long)q.m * q.s;
    for (long e = threadIdx.x; e < tot; e += blockDim.x) {
      if (e < (long)q.m * q.m) {
        const int a = (int)(e / q.m), b = (int)(e % q.m);
        q.Q[e] = (T)(a == b ? 1.0 : 0.0);
      } else {
        const long f = e - (long)q.m * q.m;
        const int a = (int)(f / q.s), b = (int)(f % q.s);
        q.R[f] = (double)q.A[a * q.sAm + b * q.sAk];
      }
    }
  }
  if (set_rank && threadIdx.x == 0) L.p[i]->r[bond] = pfin;
}

// Widen a rank-deficient Q (m x p, ld p) to m x s (ld s) with zero columns,
// R to s rows with zero rows, so that a caller with host-fixed bond sizes sees
// the Householder layout (Q^T Q is then a projector, Q Q^T A = A still holds).
// One workgroup per problem; tmp holds m*s elements per problem.
template <typename T>
__global__ void k_qr_widen(QrProb<T>* qp, T* tmp, long tslot, int nprob) {
  int i = blockIdx.x;
  if (i >= nprob) return;
  QrProb<T> q = qp[i];
  if (!q.valid || q.m <= q.s || q.p >= q.s) return;
  T* t = tmp + i * tslot;
  long mp = (long)q.m * q.p;
  for (long e = threadIdx.x; e < mp; e += blockDim.x) t[e] = q.Q[e];
  __syncthreads();
  for (long e = threadIdx.x; e < (long)q.m * q.s; e += blockDim.x) {
    long row = e / q.s;
    int col = (int)(e % q.s);
    q.Q[e] = col < q.p ? t[row * q.p + col] : (T)0;
  }
  // R is p x s (ld s): rows p..s-1 become zero
  for (long e = (long)q.p * q.s + threadIdx.x; e < (long)q.s * q.s; e += blockDim.x) q.R[e] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) qp[i].p = q.s;
}

template <typename T>
__global__ void k_rank_dims(MpsList<T> L, int k, int* out, int cnt) {
  int i = threadIdx.x;
  if (i < cnt) out[i] = L.p[i]->r[k];
}

// Gram of the right unfolding M (r_k x 8 r_{k+1}) of core k: G = M M^T (FP64)
template <typename T>
struct FGramM {
  MpsList<T> L; int k; double* G; long sq;
  __device__ GemmDesc<T, T, double> get(int i) const {
    GemmDesc<T, T, double> d = gemm_empty<T, T, double>();
    MpsDev<T>* m = L.p[i];
    int s = m->r[k], c = PHYS * m->r[k + 1];
    d.A = core_ptr(m, k); d.B = core_ptr(m, k); d.C = G + i * sq;
    d.M = s; d.N = s; d.K = c;
    d.sAm = c; d.sAk = 1; d.sBk = 1; d.sBn = c; d.sCm = s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
template <typename T>
struct FnEigTrunc {
  MpsList<T> L; int k; double* Rp; long sq; const int* crank; double* US; double* Ut; long sus;
  const double* delta2; double* disc; int chi; int* fail;
  const int* s0 = nullptr;    // bond sizes before truncation (randomized path on)
  const int* skip = nullptr;  // problems already truncated by the randomized path
  float* feat = nullptr;      // rank-predictor features of this bond (MLP_IN per problem)
  float stepf = 0.0f;
  __device__ EigProb get(int i) const {
    EigProb p;
    p.feat = feat ? feat + i * MLP_IN : nullptr;
    p.stepf = stepf;
    p.A = Rp + i * sq;  // R P^T (c x s, row-major) read as its transpose
    p.s = s0 ? s0[i] : L.p[i]->r[k];
    p.c = crank[i];
    p.valid = (skip && skip[i]) ? 0 : 1;
    p.delta2 = delta2[i];
    p.chi = chi;
    p.rank_out = &L.p[i]->r[k];
    p.US = US + i * sus;
    p.Ut = Ut + i * sus;
    p.disc = disc + i * (MAXN + 1) + k;
    p.fail = fail;
    return p;
  }
};
// core_k <- Ut (r x s) M (s x 8 r_{k+1}) into tmp
template <typename T>
struct FUtM {
  MpsList<T> L; const EigProb* ep; T* tmp; long slot; int k;
  __device__ GemmDesc<double, T, T> get(int i) const {
    GemmDesc<double, T, T> d = gemm_empty<double, T, T>();
    MpsDev<T>* m = L.p[i];
    int s = ep[i].s, r = m->r[k], c = PHYS * m->r[k + 1];
    d.A = ep[i].Ut; d.B = core_ptr(m, k); d.C = tmp + i * slot;
    d.M = r; d.N = c; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = c; d.sBn = 1; d.sCm = c; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
// core_{k-1} <- core_{k-1} ((8 r_{k-1}) x s) US (s x r) into tmp
template <typename T>
struct FCoreUS2 {
  MpsList<T> L; const EigProb* ep; T* tmp; long slot; int k;
  __device__ GemmDesc<T, double, T> get(int i) const {
    GemmDesc<T, double, T> d = gemm_empty<T, double, T>();
    MpsDev<T>* m = L.p[i];
    int s = ep[i].s, r = m->r[k], rl = m->r[k - 1];
    d.A = core_ptr(m, k - 1); d.B = ep[i].US; d.C = tmp + i * slot;
    d.M = rl * PHYS; d.N = r; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// ============================================================================
// TT-SVD of dense fields (Section 2.1, svd-comp equation).  At site k the
// remainder M (8 r_k x rest, row-major, rest = 8^(n-1-k)) is factored as
// M^T = Q R (Householder; Q = I when rest <= 8 r_k) and R^T = U S W^T (Jacobi
// SVD with the rank rule), so that M = U S (Q W)^T: the kept columns of U are
// core k and S W^T Q^T is the next remainder.
template <typename T>
struct FnTtQr {
  MpsList<T> L; const T* cur; long slot; int k; long rest; T* qout; double* rout; long rslot;
  __device__ QrProb<T> get(int i) const {
    QrProb<T> q;
    q.A = cur + i * slot;
    q.m = (int)rest;
    q.s = PHYS * L.p[i]->r[k];
    q.sAm = 1; q.sAk = rest;
    q.p = 0; q.valid = 1;
    q.Q = qout + i * slot;
    q.R = rout + i * rslot;
    return q;
  }
};

template <typename T>
struct FnTtSvd {
  MpsList<T> L; const QrProb<T>* qp; int k; double* W; long wslot; double* US; double* Wk;
  long uslot; long wkslot; double* sv; long svslot; const double* delta2; double* disc; int chi;
  int* fail;
  __device__ SvdProb get(int i) const {
    QrProb<T> q = qp[i];
    SvdProb p;
    p.L = q.R; p.Lw = q.R; p.W = W + i * wslot;
    p.rows = q.s; p.cols = q.p; p.valid = 1;
    p.delta2 = delta2[i]; p.chi = chi;
    p.rank_out = &L.p[i]->r[k + 1];
    p.US = US + i * uslot; p.Wk = Wk + i * wkslot;
    p.sv = sv + i * svslot;
    p.disc = disc + i;
    p.fail = fail;
    return p;
  }
};

// core k = U_r (U S with column j divided by s_j); Wk column j scaled by s_j
template <typename T>
__global__ void k_tt_core(MpsList<T> L, int k, const QrProb<T>* qp, const double* US, double* Wk,
                          long uslot, long wkslot, const double* sv, long svslot) {
  const int i = blockIdx.y;
  MpsDev<T>* d = L.p[i];
  const int m = PHYS * d->r[k], r = d->r[k + 1], p = qp[i].p;
  const double* us = US + i * uslot;
  double* wk = Wk + i * wkslot;
  const double* s = sv + i * svslot;
  T* core = core_ptr(d, k);
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)m * r;
       e += (long)gridDim.x * blockDim.x) {
    double sg = s[e % r];
    core[e] = (T)(sg > 0.0 ? us[e] / sg : 0.0);
  }
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)p * r;
       e += (long)gridDim.x * blockDim.x)
    wk[e] *= s[e % r];
}

// next remainder (r x rest) = (Wk S)^T (r x p) * Q^T (p x rest)
template <typename T>
struct FnTtNext {
  MpsList<T> L; const QrProb<T>* qp; const double* Wk; long uslot; T* nxt; long slot; int k;
  long rest;
  __device__ GemmDesc<double, T, T> get(int i) const {
    GemmDesc<double, T, T> d = gemm_empty<double, T, T>();
    QrProb<T> q = qp[i];
    const int r = L.p[i]->r[k + 1];
    d.A = Wk + i * uslot; d.B = q.Q; d.C = nxt + i * slot;
    d.M = r; d.N = (int)rest; d.K = q.p;
    d.sAm = 1; d.sAk = r;
    d.sBk = 1; d.sBn = q.p;
    d.sCm = rest; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

template <typename T>
__global__ void k_dense_delta2(const T* W, long N3, int cnt, double f, double* out) {
  __shared__ double red[8];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (long e = threadIdx.x; e < N3; e += blockDim.x) {
    double v = (double)W[i * N3 + e];
    acc += v * v;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[i] = f * acc;
}

// ============================================================================
template <typename T>
class Engine {
 public:
  typedef T Tacc;
  int n = 0, chi = 1;
  double tol = 0.0;
  hipStream_t st = nullptr;
  int capb[MAXN + 1];  // capacity bond of pooled MPS: 2 min(chi, full-rank bound)
  int cpb[MAXN + 1];   // bond bound of rounded MPS: min(chi, full-rank bound)
  int maxbond = 1;
  long maxcore = 0;
  long estride = 0, tcap = 0;  // product workspaces per problem (largest profile)
  long ws_env = 0, ws_t = 0;     // elements allocated for envL/envR and T1/T2
  int lds_elems = 8000;
  int js_elems = 8000;  // dynamic LDS (doubles) of k_jacobi_eig_split
  std::vector<Mps<T>> pool;
  std::vector<int> freelist;
  std::vector<void*> allocs;
  QrProb<T>* qp = nullptr;
  QrWork qw;
  T* qtmp = nullptr;
  double* rbuf = nullptr;
  long qslot = 0, rslot = 0;
  T* ctmp = nullptr;
  SvdProb* sp = nullptr;
  double* svdW = nullptr;
  double* svdUS = nullptr;
  double* svdWk = nullptr;
  long sw = 0, sus = 0;
  double* rdelta = nullptr;
  double* rnorm = nullptr;
  double* rdisc = nullptr;
  double* stats = nullptr;  // [0] max discarded ratio of the current step
  int* istats = nullptr;    // [0] SVD sweep-limit hits, [1] non-finite flag,
                            // [2] Jacobi sweeps, [3] Jacobi problems (totals)
  T* envL = nullptr;
  T* envR = nullptr;
  T* T1 = nullptr;
  T* T2 = nullptr;
  // FP32 policy: rank-revealing Cholesky-QR2 and Gram-eigen truncation
  bool fast = false;
  CholWork cw;
  int* cq_n = nullptr;  // [2 * MAXB] dims of the two Cholesky passes
  EigProb* ep = nullptr;
  double eps_rank = 1e-14;
  // second Cholesky-QR pass skipped when the first already left the Gram
  // within this distance of the identity (far below FP32 resolution)
  double cq_skip = 1e-9;
  int pbatch = 1;
  int sweeps = 2;
  long roundings = 0, products = 0;
  // rank-predicted randomized truncation (FP32/BF16): predictions are the
  // ranks chosen in the previous step by the same rounding call, problem
  // slot and bond (the step's schedule is fixed)
  static constexpr int RS_CALLS = 1024;
  bool rsvd = false;
  int rs_over = 16;
  // Jacobi of the FP32 truncation: column pairs count as orthogonal at a
  // relative 1e-9, which leaves the eigenvectors orthonormal to 1e-9: the
  // level at which the FP32 Cholesky-QR already accepts a Q, and far below
  // the rounding of the FP32 cores they become (about 1e-7)
  double eig_orth_tol = 1e-9;
  int rs_call = 0;
  int* rs_pred = nullptr;   // [RS_CALLS][MAXN + 1][MAXB]
  int* rs_dims = nullptr;
  EigProb* rs_ep = nullptr;
  RsWork rw;
  void enable_rsvd(int oversample, unsigned long long seed) {
    if (rs_pred) return;
    rsvd = true;
    rs_over = oversample > 0 ? oversample : 16;
    const long sq = cw.sq;
    rw.sq = sq;
    double** mats[] = {&rw.Y, &rw.T, &rw.B, &rw.R, &rw.B2, &rw.R2,
                       &rw.Q, &rw.Q2, &rw.W, &rw.USt, &rw.Utt};
    for (double** m : mats) *m = (double*)dalloc(8 * sq * MAXB);
    // one Gaussian test matrix, drawn once from the seed and shared by all
    // problems and calls: read as c x l with leading dimension l, any
    // prefix of it is an i.i.d. Gaussian matrix of that shape
    rw.som = (long)PHYS * sq;
    rw.Om = (double*)dalloc(8 * rw.som);
    hipLaunchKernelGGL(k_gauss<double>, dim3((unsigned)std::min<long>(1024, (rw.som + 255) / 256)),
                       dim3(256), 0, st, rw.Om, rw.som,
                       (uint64_t)(0x9E3779B97F4A7C15ull ^ (uint64_t)seed));
    int** ints[] = {&rw.s0, &rw.ell, &rw.rank1, &rw.rank2, &rw.rankT, &rw.rsel, &rw.acc};
    for (int** v : ints) *v = (int*)dalloc(4 * MAXB);
    rw.tries = (int*)dalloc(4 * 4);
    rw.budget = (double*)dalloc(8 * MAXB);
    rw.disc = (double*)dalloc(8 * MAXB);
    rw.trG = (double*)dalloc(8 * MAXB);
    rs_dims = (int*)dalloc(4 * MAXB);
    rs_ep = (EigProb*)dalloc(sizeof(EigProb) * MAXB);
    rs_pred = (int*)dalloc(4L * RS_CALLS * (MAXN + 1) * MAXB);
    HIP_OK(hipMemset(rs_pred, 0xFF, 4L * RS_CALLS * (MAXN + 1) * MAXB));  // -1: no prediction
    HIP_OK(hipMemset(rw.tries, 0, 16));
  }

  // Threads of the truncation's Jacobi at bond k: the columns it rotates
  // number at most the rank of the unfolding, which the full bound of the
  // bond caps below the storage capacity (twice the bond for sums); 16 lanes
  // per pair (every row of a column up to 128 in registers) for up to 8, 32,
  // 64 or 128 columns take one, four, eight or sixteen waves.
  int eig_threads(int scap, int k) const {
    const int c = std::min(scap, full_bound(n, k));
    return c <= 8 ? 64 : c <= 32 ? 256 : c <= 64 ? 512 : 1024;
  }

  // learned rank predictor: features of the last step per (call, bond,
  // problem), a ring of training samples (features of step t, rank change
  // from t to t + 1, divided by 16) and the network
  static constexpr int SMP_CAP = 1 << 16;
  bool mlp_on = false, mlp_trained = false;
  Mlp mlp;
  float* rs_feat = nullptr;  // [RS_CALLS][MAXN + 1][MAXB][MLP_IN]
  float* smp_x = nullptr;    // [SMP_CAP][MLP_IN]
  float* smp_t = nullptr;    // [SMP_CAP]
  int* smp_n = nullptr;      // samples written (total)
  int* smp_slot = nullptr;   // [MAXB] pending sample of each problem of a bond, -1: none
  float* mlp_x = nullptr;    // [MAXB][MLP_IN] inputs of one bond
  int* rs_pred2 = nullptr;   // [MAXB] ranks used to size the sketches of one bond
  double* mlp_err = nullptr; // [3]: sum |rhat - r|, sum |r_prev - r|, count
  long long step_count = 0;
  float first_loss = -1.0f, last_loss = -1.0f;
  void enable_mlp(unsigned long long seed) {
    if (mlp_on) return;
    mlp_on = true;
    rs_feat = (float*)dalloc(4L * RS_CALLS * (MAXN + 1) * MAXB * MLP_IN);
    smp_x = (float*)dalloc(4L * SMP_CAP * MLP_IN);
    smp_t = (float*)dalloc(4L * SMP_CAP);
    smp_n = (int*)dalloc(64);
    smp_slot = (int*)dalloc(4L * MAXB);
    mlp_x = (float*)dalloc(4L * MAXB * MLP_IN);
    rs_pred2 = (int*)dalloc(4L * MAXB);
    mlp_err = (double*)dalloc(64);
    HIP_OK(hipMemset(smp_n, 0, 64));
    HIP_OK(hipMemset(mlp_err, 0, 64));
    mlp.setup(1024, [this](size_t b) { return dalloc(b); }, seed ^ 0x5EEDull, st);
  }
  // Adam epochs over the collected samples in batches of up to 1024;
  // returns the mean squared error of the last epoch
  float train_mlp(int epochs, float lr) {
    int n = 0;
    HIP_OK(hipMemcpyAsync(&n, smp_n, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    n = std::min(n, SMP_CAP);
    if (n < 16) throw Error(-1, "fewer than 16 predictor samples collected");
    float loss_sum = 0.0f;
    for (int ep = 0; ep < epochs; ++ep) {
      loss_sum = 0.0f;
      int nb = 0;
      for (int off = 0; off < n; off += mlp.bmax) {
        const int B = std::min(mlp.bmax, n - off);
        mlp.forward(smp_x + (long)off * MLP_IN, B, st);
        mlp.backward(smp_x + (long)off * MLP_IN, smp_t + off, B, st);
        mlp.adam(lr, st);
        float l = 0.0f;
        HIP_OK(hipMemcpyAsync(&l, mlp.loss, 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        loss_sum += l;
        ++nb;
      }
      loss_sum /= nb;
      if (first_loss < 0.0f) first_loss = loss_sum;
    }
    last_loss = loss_sum;
    mlp_trained = true;
    HIP_OK(hipMemset(mlp_err, 0, 64));
    return loss_sum;
  }

  // randomized attempt at bond k of one rounding call (see rsvd.h)
  void rs_attempt(MpsList<T> L, int k, int cnt, int* predk, int scap, int chi_cap,
                  float* featk) {
    const long sq = rw.sq;
    const int lds = lds_elems * 8;
    const int* plan = predk;
    if (mlp_on) {
      // inputs of this bond (last step's spectra), pending samples, and the
      // network's ranks once it is trained
      hipLaunchKernelGGL(k_mlp_gather, dim3(1), dim3(64), 0, st, (const float*)featk,
                         (const int*)predk, mlp_x, smp_x, smp_t, smp_n, smp_slot, SMP_CAP, cnt);
      if (mlp_trained) {
        mlp.forward(mlp_x, cnt, st);
        hipLaunchKernelGGL(k_mlp_rank<T>, dim3(1), dim3(64), 0, st, L, k, (const int*)predk,
                           (const float*)mlp.y, rs_pred2, cnt);
        plan = rs_pred2;
      }
    }
    hipLaunchKernelGGL(k_rs_plan<T>, dim3(cnt), dim3(256), 0, st, L, k, plan, rs_over,
                       (const double*)cw.G, rw, cnt);
    typedef double D;
    launch_gemm<T, D, D, D>(FRsMOm<T>{L, k, rw}, cnt, scap, scap, 1, st);
    launch_gemm<D, D, D, D>(FRsGram<T>{L, k, rw.Y, rw.T, rw.ell, sq}, cnt, scap, scap, 1, st);
    launch_chol(scap, cnt, (const int*)rw.ell, 1, rw.T, sq, rw.B, rw.R, rw.rank1, eps_rank,
                lds_elems, cnt, 1, (double*)nullptr, 0.0);
    launch_gemm<D, D, D, D>(FRsXB<T>{L, k, rw.Y, rw.B, rw.Q, rw.ell, rw.rank1, sq}, cnt, scap,
                            scap, 1, st);
    launch_gemm<D, D, D, D>(FRsGram<T>{L, k, rw.Q, rw.T, rw.rank1, sq}, cnt, scap, scap, 1, st);
    launch_chol(scap, cnt, (const int*)rw.rank1, 1, rw.T, sq, rw.B2, rw.R2, rw.rank2, 1e-28,
                lds_elems, cnt, 1, (double*)nullptr, cq_skip);
    launch_gemm<D, D, D, D>(FRsXB<T>{L, k, rw.Q, rw.B2, rw.Q2, rw.rank1, rw.rank2, sq}, cnt, scap,
                            scap, 1, st);
    launch_gemm<D, D, D, D>(FRsGQ<T>{L, k, cw.G, rw}, cnt, scap, scap, 1, st);
    launch_gemm<D, D, D, D>(FRsQtW<T>{L, k, rw}, cnt, scap, scap, 1, st);
    hipLaunchKernelGGL(k_rs_budget, dim3(cnt), dim3(256), 0, st, (const double*)rdelta, rw, cnt);
    hipLaunchKernelGGL(k_rs_dims_T, dim3(1), dim3(64), 0, st, rw, rs_dims, cnt);
    launch_chol(scap, cnt, (const int*)rs_dims, 1, rw.T, sq, rw.B, rw.R, rw.rankT, eps_rank,
                lds_elems, cnt, 0, (double*)nullptr, 0.0);
    hipLaunchKernelGGL(k_eig_prep<FnRsEig>, dim3(1), dim3(64), 0, st,
                       FnRsEig{rw, chi_cap, istats, featk, 0.001f * (float)step_count}, rs_ep,
                       cnt);
    hipLaunchKernelGGL(k_jacobi_eig, dim3(cnt), dim3(eig_threads(scap, k)), lds, st,
                       (const EigProb*)rs_ep, lds_elems, 40, (double*)nullptr, eig_orth_tol);
    hipLaunchKernelGGL(k_rs_accept<T>, dim3(1), dim3(64), 0, st, L, k, (const double*)rdelta,
                       chi_cap, rw, rdisc, cnt);
    launch_gemm<D, D, D, D>(FRsUS{rw, svdUS, sus}, cnt, scap, scap, 1, st);
    launch_gemm<D, D, D, D>(FRsUt{rw, svdWk, sus}, cnt, scap, scap, 1, st);
    hipLaunchKernelGGL(k_rs_dims_full<T>, dim3(1), dim3(64), 0, st, L, k, rw, cq_n, cnt);
    HIP_OK(hipGetLastError());
  }
  // Truncation eigendecompositions of the cnt problems in ep whose factors
  // may have 129-256 rows: column blocks spread over JS_PARTS workgroups per
  // problem (k_jacobi_eig_split), at most JS_LAUNCH problems per launch so
  // that the workgroups of a launch fit the GPU together.
  static constexpr int JS_LAUNCH = 32;
  JsSync js{};
  void eig_split(int cnt) {
    if (!js.nrm) {
      js.nrm = (double*)dalloc(8 * JS_NRM_SLOT * JS_LAUNCH);
      js.count = (unsigned*)dalloc(4 * JS_LAUNCH);
    }
    for (int off = 0; off < cnt; off += JS_LAUNCH) {
      const int c = std::min(JS_LAUNCH, cnt - off);
      hipLaunchKernelGGL(k_js_reset, dim3(1), dim3(64), 0, st, js.count, c);
      const int blocks = ((c + 7) / 8) * 8 * JS_PARTS;
      hipLaunchKernelGGL(k_jacobi_eig_split, dim3(blocks), dim3(JS_THREADS), (size_t)js_elems * 8,
                         st, (const EigProb*)(ep + off), c, js, js_elems, 40, kf(1), eig_orth_tol);
    }
    HIP_OK(hipGetLastError());
  }

  // Pivoted Cholesky of nprob Grams of order at most ncap: the 1024-thread
  // kernel up to CPB_MAXN, the 512-thread one (blocked with the Gram in
  // global memory up to CHOL_WIDE_MAXN) above.
  template <typename... A>
  void launch_chol(int ncap, int nprob, A... args) {
    if (ncap > CPB_MAXN)
      hipLaunchKernelGGL(k_chol_piv_wide, dim3(nprob), dim3(CHOL_WIDE_THREADS),
                         (size_t)lds_elems * 8, st, args...);
    else
      hipLaunchKernelGGL(k_chol_piv, dim3(nprob), dim3(CHOL_THREADS), (size_t)lds_elems * 8, st,
                         args...);
  }

  // timing of one kernel class: HIP events around each of its launches
  int tkind = 0;
  std::vector<hipEvent_t> evs;
  size_t ev_next = 0;
  long long tlaunches = 0;
  double tms = 0.0;
  double* kflops = nullptr;  // device counter of the class's algorithmic flops

  void timing(int kind) {
    flush_events();
    tkind = kind;
    tlaunches = 0;
    tms = 0.0;
    if (!kflops) kflops = (double*)dalloc(64);
    HIP_OK(hipMemsetAsync(kflops, 0, 8, st));
    if (kind && evs.empty()) {
      evs.resize(8192);
      for (auto& e : evs) HIP_OK(hipEventCreate(&e));
    }
  }
  void tbegin(int kind) {
    if (tkind != kind) return;
    if (ev_next + 2 > evs.size()) flush_events();
    HIP_OK(hipEventRecord(evs[ev_next], st));
  }
  void tend(int kind) {
    if (tkind != kind) return;
    HIP_OK(hipEventRecord(evs[ev_next + 1], st));
    ev_next += 2;
    ++tlaunches;
  }
  double* kf(int kind) const { return tkind == kind ? kflops : nullptr; }
  void flush_events() {
    if (ev_next == 0) return;
    HIP_OK(hipStreamSynchronize(st));
    for (size_t i = 0; i + 1 < ev_next; i += 2) {
      float ms = 0.f;
      HIP_OK(hipEventElapsedTime(&ms, evs[i], evs[i + 1]));
      tms += ms;
    }
    ev_next = 0;
  }

  // every device buffer of the engine comes from here (and goes back
  // through dfree), through the handle's allocator on the engine's stream
  Allocator al;
  void* dalloc(size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (al.alloc) {
      p = al.alloc(bytes, (void*)st, al.ctx);
      if (!p) throw Error(-2, "device allocation of " + std::to_string(bytes) + " bytes failed");
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw Error(-2, "device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    try {
      allocs.push_back(p);
    } catch (...) {
      dfree(p);
      throw;
    }
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    if (al.free_)
      al.free_(p, (void*)st, al.ctx);
    else
      (void)hipFree(p);
  }
  ~Engine() {
    (void)hipStreamSynchronize(st);
    for (void* p : allocs) dfree(p);
    for (auto& e : evs) (void)hipEventDestroy(e);
  }

  static int full_bound(int n, int k) {
    long a = 1, b = 1;
    for (int j = 0; j < k && a < (1 << 20); ++j) a *= 8;
    for (int j = 0; j < n - k && b < (1 << 20); ++j) b *= 8;
    long m = a < b ? a : b;
    return (int)(m > (1 << 20) ? (1 << 20) : m);
  }

  void setup(int n_, int chi_, double tol_, hipStream_t s, int npool, int pbatch_) {
    n = n_; chi = chi_; tol = tol_; st = s; pbatch = pbatch_;
    capb[0] = capb[n] = 1;
    cpb[0] = cpb[n] = 1;
    maxbond = 1;
    for (int k = 1; k < n; ++k) {
      int fb = full_bound(n, k);
      cpb[k] = std::min(chi, fb);
      capb[k] = 2 * cpb[k];
      maxbond = std::max(maxbond, capb[k]);
    }
    maxcore = 0;
    for (int k = 0; k < n; ++k) maxcore = std::max(maxcore, (long)capb[k] * PHYS * capb[k + 1]);
    int dev = 0, lds = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    long want = std::min<long>(lds, 147456) - 16384;
    lds_elems = (int)std::max<long>(want / 8, 1024);
    if (hipFuncSetAttribute((const void*)k_jacobi_svd, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_householder<T>,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_chol_piv, hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_chol_piv_wide,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_jacobi_eig,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_jacobi_eig_split,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            lds_elems * 8) != hipSuccess) {
      (void)hipGetLastError();
      lds_elems = (65536 - 16384) / 8;
    }
    // the split eigendecomposition holds two padded column blocks; below
    // that it runs the single-workgroup body on its first part
    js_elems = lds_elems;
    const long js_need = 2L * JS_BS * JS_LD;
    if (js_need > lds_elems && js_need * 8 + 16384 <= lds &&
        hipFuncSetAttribute((const void*)k_jacobi_eig_split,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(js_need * 8)) == hipSuccess)
      js_elems = (int)js_need;
    (void)hipGetLastError();
    for (int i = 0; i < npool; ++i) pool.push_back(make_mps(capb));
    freelist.clear();
    for (int i = npool - 1; i >= 0; --i) freelist.push_back(i);
    int scap = maxbond, mcap = PHYS * maxbond;
    qp = (QrProb<T>*)dalloc(sizeof(QrProb<T>) * MAXB);
    long sq = (long)scap * scap, mq = (long)mcap * scap;
    qw.sq = sq; qw.mq = mq;
    qw.G = (double*)dalloc(8 * sq * MAXB);
    qw.R1 = (double*)dalloc(8 * sq * MAXB);
    qw.Racc = (double*)dalloc(8 * sq * MAXB);
    qw.Rt = (double*)dalloc(8 * sq * MAXB);
    qw.Rinv = (double*)dalloc(8 * sq * MAXB);
    qw.Q1 = (double*)dalloc(8 * mq * MAXB);
    qw.Q2 = (double*)dalloc(8 * mq * MAXB);
    qslot = mq;  // Q is m x p with p <= s
    rslot = sq;  // R is p x s; in the m <= s case it is m x s with m <= s
    qtmp = (T*)dalloc(sizeof(T) * qslot * MAXB);
    rbuf = (double*)dalloc(8 * rslot * MAXB);
    ctmp = (T*)dalloc(sizeof(T) * maxcore * MAXB);
    sp = (SvdProb*)dalloc(sizeof(SvdProb) * MAXB);
    sw = sq;   // W is p x p
    sus = sq;  // US is s x r, Wk is p x r
    svdW = (double*)dalloc(8 * sw * MAXB);
    svdUS = (double*)dalloc(8 * sus * MAXB);
    svdWk = (double*)dalloc(8 * sus * MAXB);
    rdelta = (double*)dalloc(8 * MAXB);
    rnorm = (double*)dalloc(8 * MAXB);
    rdisc = (double*)dalloc(8 * MAXB * (MAXN + 1));
    stats = (double*)dalloc(8 * 16);
    istats = (int*)dalloc(4 * 16);
    HIP_OK(hipMemsetAsync(stats, 0, 8 * 16, st));
    HIP_OK(hipMemsetAsync(istats, 0, 4 * 16, st));
    fast = (sizeof(T) == 4);
    cw.sq = sq; cw.mq = mq;
    cw.G = (double*)dalloc(8 * sq * MAXB);
    cw.B1 = (double*)dalloc(8 * sq * MAXB);
    cw.R1 = (double*)dalloc(8 * sq * MAXB);
    cw.B2 = (double*)dalloc(8 * sq * MAXB);
    cw.R2 = (double*)dalloc(8 * sq * MAXB);
    cw.Q1 = (double*)dalloc(8 * mq * MAXB);
    cw.rank = (int*)dalloc(4 * 4 * MAXB);  // [0, 2 MAXB): per-problem pairs (pass 1, pass 2)
    cq_n = (int*)dalloc(4 * 2 * MAXB);
    ep = (EigProb*)dalloc(sizeof(EigProb) * MAXB);
    reserve_products(cpb);
  }

  // Product workspaces for a second factor of capacity profile ccp (the
  // candidate and the result are at most cpb): environment of bond k holds
  // cpb[k]^2 ccp[k] elements; the intermediates of a site update hold the
  // largest of T1 (a c 8 b'), T2 (a 8 b' c'), U1 (a' c' 8 b), U2 (8 a' b c).
  // Grows the buffers when a profile needs more (at initialisation only).
  void prod_sizes(const int* ccp, long* eoff, long* stride, long* tsz) const {
    long off = 0;
    for (int k = 0; k <= n; ++k) {
      eoff[k] = off;
      off += (long)cpb[k] * cpb[k] * ccp[k];
    }
    eoff[n + 1] = off;
    *stride = off;
    long tc = 1;
    for (int k = 0; k < n; ++k) {
      const long a = cpb[k], a2 = cpb[k + 1], c = ccp[k], c2 = ccp[k + 1];
      tc = std::max({tc, a * c * PHYS * a2, a * PHYS * a2 * c2, a2 * c2 * PHYS * a,
                     PHYS * a2 * a * c});
    }
    *tsz = tc;
  }
  void free_alloc(void* p) {
    if (!p) return;
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        dfree(p);
        allocs.erase(allocs.begin() + i);
        return;
      }
  }
  void reserve_products(const int* ccp) {
    long eoff[MAXN + 2], stride = 0, tsz = 0;
    prod_sizes(ccp, eoff, &stride, &tsz);
    estride = std::max(estride, stride);
    tcap = std::max(tcap, tsz);
    if (estride * pbatch > ws_env) {
      HIP_OK(hipStreamSynchronize(st));
      free_alloc(envL);
      free_alloc(envR);
      envL = (T*)dalloc(sizeof(T) * estride * pbatch);
      envR = (T*)dalloc(sizeof(T) * estride * pbatch);
      ws_env = estride * pbatch;
    }
    if (tcap * pbatch > ws_t) {
      HIP_OK(hipStreamSynchronize(st));
      free_alloc(T1);
      free_alloc(T2);
      T1 = (T*)dalloc(sizeof(T) * tcap * pbatch);
      T2 = (T*)dalloc(sizeof(T) * tcap * pbatch);
      ws_t = tcap * pbatch;
    }
  }

  Mps<T> make_mps(const int* cap) {
    Mps<T> m;
    m.n = n;
    long off = 0;
    for (int k = 0; k <= n; ++k) m.cap[k] = cap[k];
    for (int k = 0; k < n; ++k) {
      m.off[k] = off;
      off += (long)cap[k] * PHYS * cap[k + 1];
    }
    m.total = off;
    m.data = (T*)dalloc(sizeof(T) * off);
    m.dev = (MpsDev<T>*)dalloc(sizeof(MpsDev<T>));
    MpsDev<T> h;
    memset(&h, 0, sizeof(h));
    h.data = m.data;
    h.n = n;
    for (int k = 0; k < n; ++k) h.off[k] = m.off[k];
    for (int k = 0; k <= n; ++k) {
      h.cap[k] = cap[k];
      h.r[k] = 1;
    }
    HIP_OK(hipMemcpy(m.dev, &h, sizeof(h), hipMemcpyHostToDevice));
    HIP_OK(hipMemset(m.data, 0, sizeof(T) * off));
    return m;
  }

  // An MPS of its own capacity profile outside the recycled pool (geometry
  // masks, decomposed once and only read afterwards); never released.
  int add_fixed(const int* cap) {
    pool.push_back(make_mps(cap));
    return (int)pool.size() - 1;
  }

  // frees the storage of an add_fixed object (its index is not reused)
  void drop_fixed(int i) {
    free_alloc(pool[i].data);
    free_alloc(pool[i].dev);
    pool[i].data = nullptr;
    pool[i].dev = nullptr;
  }

  int acquire() {
    if (freelist.empty()) {
      // grow the pool (memory stays bounded by the peak number of live MPS)
      pool.push_back(make_mps(capb));
      return (int)pool.size() - 1;
    }
    int i = freelist.back();
    freelist.pop_back();
    return i;
  }
  // slots that release() must not recycle (the populations a captured step
  // reads stay untouched until the step has finished with them)
  std::vector<char> pinned;
  void release(int i) {
    if (i < 0) return;
    if (i < (int)pinned.size() && pinned[i]) return;
    freelist.push_back(i);
  }
  MpsDev<T>* D(int i) const { return pool[i].dev; }
  // grid-stride chunks for kernels walking one core of capacity size
  int chunks() const { return (int)std::max<long>(1, std::min<long>(64, (maxcore + 255) / 256)); }
  int chunks_q() const {
    long e = (long)PHYS * maxbond * maxbond;
    return (int)std::max<long>(1, std::min<long>(64, (e + 255) / 256));
  }

  MpsList<T> list_idx(const std::vector<int>& v, size_t off, int cnt) const {
    MpsList<T> l;
    memset(&l, 0, sizeof(l));
    for (int i = 0; i < cnt; ++i) l.p[i] = D(v[off + i]);
    return l;
  }

  // Product contractions: in the working type, or (BF16 policy, FP32
  // storage) with operands rounded to BF16 on a BF16 MFMA, FP32 accumulate.
  // product contractions: 0 in the storage type, 1 on BF16 MFMA (operands
  // rounded), 2 on BF16 MFMA with three-term operand splitting
  int bf16_products = 0;
  template <typename F>
  void pgemm(const F& f, int nprob, int mcap, int ncap, int bcap, hipStream_t s,
             double* flops = nullptr, int kcap = 0) {
    const int acc = bf16_products == 2 ? 3 : bf16_products == 1 ? 2 : sizeof(Tacc) == 8 ? 0 : 1;
    int ts = GT;
    const KSplit ks = ksplit(nprob, mcap, ncap, bcap, kcap, acc, &ts);
    if constexpr (std::is_same<T, float>::value) {
      if (bf16_products == 1) {
        if (ts == 2 * GT)
          launch_gemm<T, T, T, float, F, 1, 2 * GT>(f, nprob, mcap, ncap, bcap, s, flops, ks);
        else
          launch_gemm<T, T, T, float, F, 1>(f, nprob, mcap, ncap, bcap, s, flops, ks);
        return;
      }
      if (bf16_products == 2) {
        if (ts == 2 * GT)
          launch_gemm<T, T, T, float, F, 2, 2 * GT>(f, nprob, mcap, ncap, bcap, s, flops, ks);
        else
          launch_gemm<T, T, T, float, F, 2>(f, nprob, mcap, ncap, bcap, s, flops, ks);
        return;
      }
    }
    launch_gemm<T, T, T, Tacc>(f, nprob, mcap, ncap, bcap, s, flops, ks);
  }

  // Split of K for contractions whose K capacity exceeds 512: the share
  // count comes from the autotuner's table for the contraction's class
  // (arithmetic, capacities, problem and batch counts) once it has been
  // tuned, else one share per 256 columns of K, at most 8.  The partial
  // tiles go to a workspace that grows on demand (the first, eager step
  // reaches its peak before any capture).  The BF16 product contractions
  // also take their tile edge from the table (64, or 128 where it was
  // faster; *ts), whatever their K.  A table entry holds the share count
  // plus TILE128 for the larger tile.
  double* kws = nullptr;
  size_t kws_bytes = 0;
  typedef std::tuple<int, int, int, int, int, int> KClass;  // acc, m, n, k, nprob, batch
  std::map<KClass, int> ktab;  // tuned share counts (+ TILE128)
  std::set<KClass> kseen;      // classes met and not tuned yet
  static constexpr int TILE128 = 16;
  KSplit ksplit(int nprob, int mcap, int ncap, int bcap, int kcap, int acc = 0,
                int* ts = nullptr) {
    if (ts) *ts = GT;
    const bool bf16 = ts && acc >= 2;  // a product contraction on BF16 MFMA
    if ((kcap < 512 && !bf16) || nprob <= 0 || mcap <= 0 || ncap <= 0 || bcap <= 0)
      return KSplit{nullptr, 1};
    const KClass key(acc, mcap, ncap, kcap, nprob, bcap);
    int sp;
    auto it = ktab.find(key);
    if (it != ktab.end()) {
      sp = it->second;
      if (sp & TILE128) {
        if (ts) *ts = 2 * GT;
        sp &= ~TILE128;
      }
    } else {
      kseen.insert(key);
      sp = kcap < 512 ? 1 : std::min(8, kcap / 256);
    }
    if (sp < 2) return KSplit{nullptr, 1};
    return KSplit{kworkspace(nprob, mcap, ncap, bcap, sp, ts ? *ts : GT), sp};
  }
  double* kworkspace(int nprob, int mcap, int ncap, int bcap, int sp, int tsz = GT) {
    const size_t need = (size_t)nprob * bcap * ceil_div(mcap, tsz) * ceil_div(ncap, tsz) * sp *
                        tsz * tsz * sizeof(double);
    if (need > kws_bytes) {
      kws = (double*)dalloc(need);
      kws_bytes = need;
    }
    return kws;
  }

  // ---- split-K and tile autotuner -------------------------------------------
  // Every class met since the last tuning is timed at its capacity shape on
  // scratch operands (one shared A and B, a C per problem and batch entry)
  // for 1, 2, 4 and 8 shares of K (each share at least one slice of GK),
  // and for the BF16 modes with tiles of 64 and of 128: one warm-up launch
  // and three timed ones with HIP events per candidate; the fastest is kept.
  // Returns the number of classes tuned.
  template <typename TA, int MODE>
  struct FTune {
    const TA* A; const TA* B; void* C; int M, N, K, nb;
    __device__ GemmDesc<TA, TA, TA> get(int i) const {
      GemmDesc<TA, TA, TA> d = gemm_empty<TA, TA, TA>();
      d.A = A; d.B = B; d.C = (TA*)C + (long)i * nb * M * N;
      d.M = M; d.N = N; d.K = K; d.nb1 = nb;
      d.sAm = K; d.sAk = 1; d.sBk = N; d.sBn = 1; d.sCm = N; d.sCn = 1;
      d.bC1 = (long)M * N;
      d.valid = 1;
      return d;
    }
  };
  template <typename TA, typename Tacc, int MODE, int TS>
  void time_class(const KClass& c, void* A, void* B, void* C, hipEvent_t e0, hipEvent_t e1,
                  int code, int& best, float& tbest) {
    int acc, m, nn, kk, np, nb;
    std::tie(acc, m, nn, kk, np, nb) = c;
    const FTune<TA, MODE> f{(const TA*)A, (const TA*)B, C, m, nn, kk, nb};
    for (int sp = 1; sp <= 8; sp *= 2) {
      if (sp > 1 && ((long)sp * GK > kk || kk < 512)) break;
      const KSplit ks =
          sp > 1 ? KSplit{kworkspace(np, m, nn, nb, sp, TS), sp} : KSplit{nullptr, 1};
      launch_gemm<TA, TA, TA, Tacc, FTune<TA, MODE>, MODE, TS>(f, np, m, nn, nb, st, nullptr, ks);
      HIP_OK(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r)
        launch_gemm<TA, TA, TA, Tacc, FTune<TA, MODE>, MODE, TS>(f, np, m, nn, nb, st, nullptr,
                                                                 ks);
      HIP_OK(hipEventRecord(e1, st));
      HIP_OK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIP_OK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < tbest) {
        tbest = ms;
        best = sp | code;
      }
    }
  }
  template <typename TA, typename Tacc, int MODE>
  int tune_class(const KClass& c, void* A, void* B, void* C) {
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int best = 1;
    float tbest = 1e30f;
    time_class<TA, Tacc, MODE, GT>(c, A, B, C, e0, e1, 0, best, tbest);
    if constexpr (MODE != 0)
      time_class<TA, Tacc, MODE, 2 * GT>(c, A, B, C, e0, e1, TILE128, best, tbest);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
  }
  int autotune() {
    int tuned = 0;
    for (const KClass& c : kseen) {
      if (ktab.count(c)) continue;
      int acc, m, nn, kk, np, nb;
      std::tie(acc, m, nn, kk, np, nb) = c;
      const size_t ea = (size_t)m * kk, eb = (size_t)kk * nn, ec = (size_t)np * nb * m * nn;
      const size_t w = acc == 0 ? 8 : 4;
      // scratch operands, freed one by one afterwards: the split-K
      // workspace may grow while a class is timed and must stay
      void* A = dalloc(w * ea);
      void* B = dalloc(w * eb);
      void* C = dalloc(w * ec);
      HIP_OK(hipMemsetAsync(A, 0, w * ea, st));
      HIP_OK(hipMemsetAsync(B, 0, w * eb, st));
      int sp = 1;
      if (acc == 0) sp = tune_class<double, double, 0>(c, A, B, C);
      else if (acc == 1) sp = tune_class<float, float, 0>(c, A, B, C);
      else if (acc == 2) sp = tune_class<float, float, 1>(c, A, B, C);
      else sp = tune_class<float, float, 2>(c, A, B, C);
      HIP_OK(hipStreamSynchronize(st));
      free_alloc(C);
      free_alloc(B);
      free_alloc(A);
      ktab[c] = sp;
      ++tuned;
    }
    kseen.clear();
    return tuned;
  }

  // ------------------------------------------------------------ QR op
  template <typename F>
  // With rank_list, the Cholesky path also stores each problem's final rank
  // as rank `bond` of the MPS of *rank_list (the Householder path leaves that
  // to the caller).
  void qr(const F& f, int nprob, int mcap, int scap, const MpsList<T>* rank_list = nullptr,
          int bond = 0) {
    if (nprob <= 0) return;
    hipLaunchKernelGGL((k_qr_prep<T, F>), dim3(1), dim3(64), 0, st, f, qp, nprob,
                       fast ? cq_n : (int*)nullptr);
    if (fast) {
      qr_cholesky(nprob, mcap, scap, rank_list, bond);
      return;
    }
    hipLaunchKernelGGL(k_qr_identity<T>, dim3(chunks_q(), nprob), dim3(256), 0, st,
                       (const QrProb<T>*)qp);
    tbegin(2);
    hipLaunchKernelGGL(k_householder<T>, dim3(nprob), dim3(256), (size_t)lds_elems * 8, st,
                       (const QrProb<T>*)qp, qw, lds_elems, kf(2));
    tend(2);
    HIP_OK(hipGetLastError());
  }

  // rank-revealing Cholesky-QR2 of the materialised problems (m > s)
  void qr_cholesky(int nprob, int mcap, int scap, const MpsList<T>* rank_list, int bond) {
    size_t lds = (size_t)lds_elems * 8;
    CholWork w = cw;
    launch_gemm<T, T, double, double>(FCqGram1<T>{qp, w}, nprob, scap, scap, 1, st, nullptr,
                                      ksplit(nprob, scap, scap, 1, mcap));
    tbegin(4);
    // ranks land interleaved: pass 1 in rank[2 i], pass 2 in rank[2 i + 1]
    launch_chol(scap, nprob, (const int*)cq_n, 1, w.G, w.sq, w.B1, w.R1, w.rank, eps_rank,
                lds_elems, nprob, 1, kf(4), 0.0, 2, cq_n + MAXB);
    tend(4);
    launch_gemm<T, double, double, double>(FCqQ1<T>{qp, w}, nprob, mcap, scap, 1, st);
    launch_gemm<double, double, double, double>(FCqGram2<T>{qp, w}, nprob, scap, scap, 1, st,
                                                nullptr, ksplit(nprob, scap, scap, 1, mcap));
    tbegin(4);
    launch_chol(scap, nprob, (const int*)(cq_n + MAXB), 1, w.G, w.sq, w.B2, w.R2, w.rank + 1,
                1e-28, lds_elems, nprob, 1, kf(4), cq_skip, 2);
    tend(4);
    launch_gemm<double, double, T, double>(FCqQ<T>{qp, w}, nprob, mcap, scap, 1, st);
    launch_gemm<double, double, double, double>(FCqR<T>{qp, w}, nprob, scap, scap, 1, st);
    hipLaunchKernelGGL(k_cq_finish<T>, dim3(nprob), dim3(256), 0, st, qp, (const int*)w.rank,
                       nprob, rank_list ? *rank_list : MpsList<T>{}, bond, rank_list ? 1 : 0);
    HIP_OK(hipGetLastError());
  }

  // ------------------------------------------------------------ rounding
  // Rounding (TT-rounding as a centre sweep): QR orthogonalisation from the
  // left moves the centre to the last site; truncated SVDs then shift it
  // back to the first site (svd-move equation), truncating only at the
  // centre with per-bond threshold tol^2 ||X||^2 / (n - 1) and rank cap chi.
  void round(const std::vector<int>& X, int chi_cap = -1, double tol_r = -1.0) {
    if (chi_cap < 0) chi_cap = chi;
    if (tol_r < 0) tol_r = tol;
    for (size_t off = 0; off < X.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, X.size() - off);
      round_list(list_idx(X, off, cnt), cnt, chi_cap, tol_r);
    }
  }

  void round_list(MpsList<T> L, int cnt, int chi_cap, double tol_r) {
    roundings += cnt;
    dim3 blk(256);
    for (int k = 0; k < n - 1; ++k) {
      int mcap = capb[k] * PHYS, scap = capb[k + 1];
      // the rank update r_{k+1} = p reads nothing that the product R core
      // needs (it takes p and s from the QR problem)
      qr(FnQrLeft<T>{L, k, qtmp, qslot, rbuf, rslot}, cnt, mcap, scap, &L, k + 1);
      launch_gemm<double, T, T, double>(FnRTimesCore<T>{L, qp, ctmp, maxcore, k}, cnt, scap,
                                        PHYS * capb[k + 2], 1, st);
      if (!fast)
        hipLaunchKernelGGL(k_set_rank_from_qr<T>, dim3(1), dim3(64), 0, st, L,
                           (const QrProb<T>*)qp, k + 1, cnt);
      hipLaunchKernelGGL(k_store_core2<T>, dim3(chunks(), cnt, 2), blk, 0, st, L, (const T*)qtmp,
                         qslot, k, (const T*)ctmp, maxcore, k + 1);
    }
    hipLaunchKernelGGL(k_round_threshold<T>, dim3(cnt), blk, 0, st, L, tol_r, rdelta, rnorm, cnt);
    hipLaunchKernelGGL(k_fill_f64, dim3(3), dim3(256), 0, st, rdisc, 0.0, (long)MAXB * (MAXN + 1));
    const int call = rs_call++;
    const bool rs_now = fast && rsvd && call < RS_CALLS;
    for (int k = n - 1; k >= 1 && fast; --k) {
      int scap = capb[k], ccap = PHYS * capb[k + 1];
      int* predk = rs_now ? rs_pred + ((long)call * (MAXN + 1) + k) * MAXB : nullptr;
      float* featk =
          (rs_now && mlp_on) ? rs_feat + (((long)call * (MAXN + 1) + k) * MAXB) * MLP_IN : nullptr;
      launch_gemm<T, T, double, double>(FGramM<T>{L, k, cw.G, cw.sq}, cnt, scap, scap, 1, st,
                                        nullptr, ksplit(cnt, scap, scap, 1, ccap));
      if (rs_now)
        rs_attempt(L, k, cnt, predk, scap, chi_cap, featk);
      else
        hipLaunchKernelGGL(k_rank_dims<T>, dim3(1), dim3(64), 0, st, L, k, cq_n, cnt);
      tbegin(4);
      launch_chol(scap, cnt, (const int*)cq_n, 1, cw.G, cw.sq, cw.B1, cw.R1, cw.rank, eps_rank,
                  lds_elems, cnt, 0, kf(4));
      tend(4);
      hipLaunchKernelGGL(k_eig_prep<FnEigTrunc<T>>, dim3(1), dim3(64), 0, st,
                         FnEigTrunc<T>{L, k, cw.R1, cw.sq, (const int*)cw.rank, svdUS, svdWk,
                                       sus, rdelta, rdisc, chi_cap, istats,
                                       rs_now ? (const int*)rw.s0 : nullptr,
                                       rs_now ? (const int*)rw.acc : nullptr, featk,
                                       0.001f * (float)step_count},
                         ep, cnt);
      tbegin(1);
      if (scap > 128 && std::min(scap, full_bound(n, k)) > 128)
        eig_split(cnt);
      else
        hipLaunchKernelGGL(k_jacobi_eig, dim3(cnt), dim3(eig_threads(scap, k)),
                           (size_t)lds_elems * 8, st, (const EigProb*)ep, lds_elems, 40, kf(1),
                           eig_orth_tol);
      tend(1);
      launch_gemm<double, T, T, double>(FUtM<T>{L, ep, qtmp, qslot, k}, cnt, scap, ccap, 1, st);
      launch_gemm<T, double, T, double>(FCoreUS2<T>{L, ep, ctmp, maxcore, k}, cnt,
                                        PHYS * capb[k - 1], scap, 1, st);
      hipLaunchKernelGGL(k_store_core2<T>, dim3(chunks(), cnt, 2), blk, 0, st, L, (const T*)qtmp,
                         qslot, k, (const T*)ctmp, maxcore, k - 1);
      if (rs_now && mlp_on)
        hipLaunchKernelGGL(k_mlp_target<T>, dim3(1), dim3(64), 0, st, L, k, (const int*)predk,
                           (const int*)rs_pred2, mlp_trained ? 1 : 0, smp_t, smp_slot, mlp_err,
                           cnt);
      if (rs_now) hipLaunchKernelGGL(k_rs_store<T>, dim3(1), dim3(64), 0, st, L, k, predk, cnt);
    }
    for (int k = n - 1; k >= 1 && !fast; --k) {
      int mcap = PHYS * capb[k + 1], scap = capb[k];
      qr(FnQrRightT<T>{L, k, qtmp, qslot, rbuf, rslot}, cnt, mcap, scap);
      hipLaunchKernelGGL(k_svd_prep<FnSvdTrunc<T>>, dim3(1), dim3(64), 0, st,
                         FnSvdTrunc<T>{L, (const QrProb<T>*)qp, k, svdW, sw, svdUS, svdWk, sus,
                                       rdelta, rdisc, chi_cap, istats, nullptr, 0},
                         sp, cnt);
      tbegin(1);
      hipLaunchKernelGGL(k_jacobi_svd, dim3(cnt), dim3(scap <= 64 ? 512 : 1024),
                         (size_t)lds_elems * 8, st, (const SvdProb*)sp, lds_elems, 40, kf(1));
      tend(1);
      launch_gemm<T, double, T, double>(FnCoreTimesUS<T>{L, qp, svdUS, sus, ctmp, maxcore, k},
                                        cnt, capb[k - 1] * PHYS, scap, 1, st);
      launch_gemm<double, T, T, double>(FnWtQt<T>{L, qp, svdWk, sus, k}, cnt, scap, mcap, 1, st);
      hipLaunchKernelGGL(k_store_core<T>, dim3(chunks(), cnt), blk, 0, st, L, (const T*)ctmp, maxcore,
                         k - 1);
    }
    hipLaunchKernelGGL(k_round_finish, dim3(1), dim3(64), 0, st, (const double*)rdisc,
                       (const double*)rnorm, stats, cnt);
    HIP_OK(hipGetLastError());
  }

  // ------------------------------------------------------------ additions
  // dst_i = c2i * a_i + c2i+1 * b_i (block-diagonal cores)
  void add(const std::vector<int>& dst, const std::vector<int>& a, const std::vector<int>& b,
           const std::vector<Coef>& coefs, const double* rho0) {
    const int per = MAXB / 2;
    for (size_t off = 0; off < dst.size(); off += per) {
      int cnt = (int)std::min<size_t>(per, dst.size() - off);
      CoefArr ca;
      memset(&ca, 0, sizeof(ca));
      for (int i = 0; i < cnt; ++i) {
        ca.c[2 * i] = coefs[2 * (off + i)];
        ca.c[2 * i + 1] = coefs[2 * (off + i) + 1];
      }
      hipLaunchKernelGGL(k_add<T>, dim3(chunks(), n, cnt), dim3(256), 0, st, list_idx(dst, off, cnt),
                         list_idx(a, off, cnt), list_idx(b, off, cnt), ca, rho0);
    }
    HIP_OK(hipGetLastError());
  }

  void copy_scaled(const std::vector<int>& dst, const std::vector<int>& src,
                   const std::vector<Coef>& coefs, const double* rho0) {
    for (size_t off = 0; off < dst.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, dst.size() - off);
      CoefArr ca;
      memset(&ca, 0, sizeof(ca));
      for (int i = 0; i < cnt; ++i) ca.c[i] = coefs[off + i];
      hipLaunchKernelGGL(k_copy_scaled<T>, dim3(chunks(), n, cnt), dim3(256), 0, st,
                         list_idx(dst, off, cnt), list_idx(src, off, cnt), ca, rho0);
    }
    HIP_OK(hipGetLastError());
  }

  struct Term {
    Coef c;
    int obj;
  };

  // Batched sums, each a pairwise tree: adjacent items are added and
  // rounded level by level, an odd last item is carried up.  Terms with a
  // zero constant coefficient are dropped.  Returns a fresh object per sum.
  std::vector<int> sums(const std::vector<std::vector<Term>>& S, const double* rho0) {
    struct Item {
      Coef c;
      int obj;
      bool owned;
    };
    std::vector<std::vector<Item>> items(S.size());
    for (size_t s = 0; s < S.size(); ++s)
      for (const Term& t : S[s])
        if (!(t.c.p == 0 && t.c.a == 0.0)) items[s].push_back({t.c, t.obj, false});
    for (;;) {
      std::vector<int> dst, a, b;
      std::vector<Coef> co;
      std::vector<std::pair<size_t, size_t>> where;
      for (size_t s = 0; s < items.size(); ++s) {
        auto& it = items[s];
        for (size_t j = 0; j + 1 < it.size(); j += 2) {
          dst.push_back(acquire());
          a.push_back(it[j].obj);
          b.push_back(it[j + 1].obj);
          co.push_back(it[j].c);
          co.push_back(it[j + 1].c);
          where.push_back({s, j});
        }
      }
      if (dst.empty()) break;
      add(dst, a, b, co, rho0);
      round(dst);
      // rebuild item lists
      size_t q = 0;
      for (size_t s = 0; s < items.size(); ++s) {
        auto& it = items[s];
        if (it.size() < 2) continue;
        std::vector<Item> nx;
        for (size_t j = 0; j + 1 < it.size(); j += 2) {
          if (it[j].owned) release(it[j].obj);
          if (it[j + 1].owned) release(it[j + 1].obj);
          nx.push_back({Coef{1.0, 0}, dst[q++], true});
        }
        if (it.size() % 2) nx.push_back(it.back());
        it = nx;
      }
    }
    std::vector<int> out(S.size(), -1);
    std::vector<int> cd, cs;
    std::vector<Coef> cc;
    for (size_t s = 0; s < items.size(); ++s) {
      auto& it = items[s];
      if (it.empty()) {
        int o = acquire();
        set_zero(o);
        out[s] = o;
      } else if (it[0].owned && it[0].c.p == 0 && it[0].c.a == 1.0) {
        out[s] = it[0].obj;
      } else {
        int o = acquire();
        cd.push_back(o);
        cs.push_back(it[0].obj);
        cc.push_back(it[0].c);
        out[s] = o;
        if (it[0].owned) release_later_.push_back(it[0].obj);
      }
    }
    if (!cd.empty()) copy_scaled(cd, cs, cc, rho0);
    for (int o : release_later_) release(o);
    release_later_.clear();
    return out;
  }
  std::vector<int> release_later_;

  void set_zero(int o) {
    std::vector<int> v{o};
    MpsList<T> l = list_idx(v, 0, 1);
    hipLaunchKernelGGL(k_set_ones<T>, dim3(1), dim3(64), 0, st, l, 1);
    std::vector<Coef> c{Coef{0.0, 0}};
    copy_scaled(v, v, c, nullptr);
  }

  void set_ones(int o) {
    std::vector<int> v{o};
    hipLaunchKernelGGL(k_set_ones<T>, dim3(1), dim3(64), 0, st, list_idx(v, 0, 1), 1);
    HIP_OK(hipGetLastError());
  }

  // ------------------------------------------------------------ products
  // Variational compressed Hadamard products (Section 2.3): candidate = the
  // higher-rank factor, right-canonicalised by QR; environments; sweeps
  // 1 -> n -> 1 (twice by default) with a QR centre shift after every
  // local update.
  // With ccp given, the second factor of every pair has that capacity
  // profile and the first factor is the candidate (obstacle products);
  // otherwise both factors are rounded pool MPS and the candidate is the
  // one with the larger maximal bond.
  std::vector<int> prods(const std::vector<std::pair<int, int>>& P, const int* ccp = nullptr) {
    std::vector<int> out(P.size());
    for (size_t i = 0; i < P.size(); ++i) out[i] = acquire();
    for (size_t off = 0; off < P.size(); off += pbatch) {
      int cnt = (int)std::min<size_t>(pbatch, P.size() - off);
      std::vector<int> d(cnt), x(cnt), y(cnt);
      for (int i = 0; i < cnt; ++i) {
        d[i] = out[off + i];
        x[i] = P[off + i].first;
        y[i] = P[off + i].second;
      }
      prod_list(list_idx(d, 0, cnt), list_idx(x, 0, cnt), list_idx(y, 0, cnt), cnt,
                ccp ? ccp : cpb, ccp ? 1 : 0);
    }
    return out;
  }

  void prod_list(MpsList<T> Dl, MpsList<T> Xl, MpsList<T> Yl, int cnt, const int* ccp,
                 int fixed) {
    products += cnt;
    ProdCtx<T> c;
    c.D = Dl; c.X = Xl; c.Y = Yl;
    c.envL = envL; c.envR = envR; c.T1 = T1; c.T2 = T2;
    long stride = 0, tsz = 0;
    prod_sizes(ccp, c.eoff, &stride, &tsz);
    if (stride > estride || tsz > tcap) throw Error(-1, "product workspaces not reserved");
    c.estride = estride;
    c.tcap = tcap;
    c.fixed = fixed;
    dim3 blk(256);
    hipLaunchKernelGGL(k_prod_init<T>, dim3(n + 1, cnt), blk, 0, st, c, n);
    // right-canonicalise the candidate
    for (int k = n - 1; k >= 1; --k) {
      qr(FnQrRightT<T>{Dl, k, qtmp, qslot, rbuf, rslot}, cnt, PHYS * cpb[k + 1], cpb[k]);
      launch_gemm<T, double, T, double>(FnCoreTimesRt<T>{Dl, qp, ctmp, maxcore, k}, cnt,
                                        PHYS * cpb[k - 1], cpb[k], 1, st);
      hipLaunchKernelGGL(k_set_rank_from_qr<T>, dim3(1), dim3(64), 0, st, Dl,
                         (const QrProb<T>*)qp, k, cnt);
      hipLaunchKernelGGL(k_store_core_T<T>, dim3(chunks(), cnt), blk, 0, st, Dl, (const QrProb<T>*)qp,
                         k);
      hipLaunchKernelGGL(k_store_core<T>, dim3(chunks(), cnt), blk, 0, st, Dl, (const T*)ctmp, maxcore,
                         k - 1);
    }
    for (int k = n - 1; k >= 1; --k) right_env(c, k, cnt, ccp);
    std::vector<int> pos;
    for (int k = 0; k < n; ++k) pos.push_back(k);
    for (int k = n - 2; k >= 0; --k) pos.push_back(k);
    std::vector<int> one = pos;
    for (int s = 1; s < sweeps; ++s) pos.insert(pos.end(), one.begin() + 1, one.end());
    for (size_t idx = 0; idx < pos.size(); ++idx) {
      int p = pos[idx];
      local_update(c, p, cnt, ccp);
      if (idx + 1 == pos.size()) break;
      int nxt = pos[idx + 1];
      if (nxt > p) {
        qr(FnQrLeft<T>{Dl, p, qtmp, qslot, rbuf, rslot}, cnt, PHYS * cpb[p], cpb[p + 1]);
        hipLaunchKernelGGL(k_set_rank_from_qr<T>, dim3(1), dim3(64), 0, st, Dl,
                           (const QrProb<T>*)qp, p + 1, cnt);
        hipLaunchKernelGGL(k_store_core<T>, dim3(chunks(), cnt), blk, 0, st, Dl, (const T*)qtmp, qslot,
                           p);
        tbegin(3);
        pgemm(FnG3L<T, Tacc>{c, p}, cnt, cpb[p + 1], cpb[p + 1] * ccp[p + 1], 1, st, kf(3),
              PHYS * cpb[p]);
        tend(3);
      } else {
        qr(FnQrRightT<T>{Dl, p, qtmp, qslot, rbuf, rslot}, cnt, PHYS * cpb[p + 1], cpb[p]);
        hipLaunchKernelGGL(k_set_rank_from_qr<T>, dim3(1), dim3(64), 0, st, Dl,
                           (const QrProb<T>*)qp, p, cnt);
        hipLaunchKernelGGL(k_store_core_T<T>, dim3(chunks(), cnt), blk, 0, st, Dl,
                           (const QrProb<T>*)qp, p);
        right_env(c, p, cnt, ccp);
      }
    }
    HIP_OK(hipGetLastError());
  }

  // Launch capacities: bonds of the result and the candidate are at most
  // cpb, those of the second factor at most ccp.
  void local_update(const ProdCtx<T>& c, int p, int cnt, const int* ccp) {
    tbegin(3);
    pgemm(FnG1<T, Tacc>{c, p}, cnt, ccp[p], PHYS * cpb[p + 1], cpb[p], st, kf(3));
    tend(3);
    tbegin(3);
    pgemm(FnG2<T, Tacc>{c, p}, cnt, cpb[p + 1], ccp[p + 1], PHYS * cpb[p], st, kf(3));
    tend(3);
    tbegin(3);
    pgemm(FnG3<T, Tacc>{c, p}, cnt, PHYS * cpb[p], cpb[p + 1], 1, st, kf(3),
          cpb[p + 1] * ccp[p + 1]);
    tend(3);
  }

  void right_env(const ProdCtx<T>& c, int p, int cnt, const int* ccp) {
    tbegin(3);
    pgemm(FnH1<T, Tacc>{c, p}, cnt, ccp[p + 1], cpb[p], PHYS * cpb[p + 1], st, kf(3));
    tend(3);
    tbegin(3);
    pgemm(FnH2<T, Tacc>{c, p}, cnt, cpb[p], ccp[p], PHYS * cpb[p + 1], st, kf(3));
    tend(3);
    tbegin(3);
    pgemm(FnH3<T, Tacc>{c, p}, cnt, cpb[p], cpb[p] * ccp[p], 1, st, kf(3), PHYS * cpb[p + 1]);
    tend(3);
  }

  // ------------------------------------------------------------ shifts, slices
  void shift(const std::vector<int>& dst, const std::vector<int>& src, const std::vector<int>& ax,
             const std::vector<int>& dir, const std::vector<int>& cyc) {
    for (size_t off = 0; off < dst.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, dst.size() - off);
      IntArr a, d, c;
      for (int i = 0; i < cnt; ++i) {
        a.v[i] = ax[off + i];
        d.v[i] = dir[off + i];
        c.v[i] = cyc[off + i];
      }
      hipLaunchKernelGGL(k_shift<T>, dim3(chunks(), n, cnt), dim3(256), 0, st, list_idx(dst, off, cnt),
                         list_idx(src, off, cnt), a, d, c);
    }
    HIP_OK(hipGetLastError());
  }

  // A two-term sum ca a + cb b, rounded.
  struct PairSum {
    Coef ca;
    int a;
    Coef cb;
    int b;
  };

  // Streaming f_new(x) = f(x - c): every item is shifted along its nonzero
  // axes in x, y, z order, each shift followed by rounding.  Level L of the
  // batch holds the L-th shift of every item, so each item sees the same
  // sequence of operations as in an axis-by-axis schedule, in as many levels
  // as an item has nonzero components (two for D3Q19, three for D3Q15).  The pair sums, if
  // any, are assembled and rounded together with the first level; their
  // results go to *pair_out.  Returns fresh objects.
  std::vector<int> stream(const std::vector<int>& src, const std::vector<const int*>& cvec,
                          const std::vector<const int*>& axis_open, const double* rho0 = nullptr,
                          const std::vector<PairSum>& pairs = {},
                          std::vector<int>* pair_out = nullptr) {
    std::vector<int> cur = src;
    std::vector<bool> owned(src.size(), false);
    std::vector<int> next_ax(src.size(), 0);
    for (int level = 0; level < 3; ++level) {
      std::vector<int> dst, s, a, d, cy, who;
      for (size_t i = 0; i < src.size(); ++i) {
        int ax = next_ax[i];
        while (ax < 3 && cvec[i][ax] == 0) ++ax;
        next_ax[i] = ax < 3 ? ax + 1 : 3;
        if (ax == 3) continue;
        dst.push_back(acquire());
        s.push_back(cur[i]);
        a.push_back(ax);
        d.push_back(cvec[i][ax]);
        cy.push_back(axis_open[i][ax] ? 0 : 1);
        who.push_back((int)i);
      }
      std::vector<int> pd;
      if (level == 0 && !pairs.empty()) {
        std::vector<int> pa, pb;
        std::vector<Coef> pc;
        for (const PairSum& q : pairs) {
          pd.push_back(acquire());
          pa.push_back(q.a);
          pb.push_back(q.b);
          pc.push_back(q.ca);
          pc.push_back(q.cb);
        }
        add(pd, pa, pb, pc, rho0);
        if (pair_out) *pair_out = pd;
      }
      if (dst.empty() && pd.empty()) break;
      if (!dst.empty()) shift(dst, s, a, d, cy);
      std::vector<int> all = dst;
      all.insert(all.end(), pd.begin(), pd.end());
      round(all);
      for (size_t j = 0; j < who.size(); ++j) {
        int i = who[j];
        if (owned[i]) release(cur[i]);
        cur[i] = dst[j];
        owned[i] = true;
      }
    }
    // items with c = 0 get a copy so that every result is a fresh object
    std::vector<int> cd, cs;
    std::vector<Coef> cc;
    for (size_t i = 0; i < src.size(); ++i)
      if (!owned[i]) {
        int o = acquire();
        cd.push_back(o);
        cs.push_back(cur[i]);
        cc.push_back(Coef{1.0, 0});
        cur[i] = o;
      }
    if (!cd.empty()) copy_scaled(cd, cs, cc, nullptr);
    return cur;
  }

  std::vector<int> slice(const std::vector<int>& src, const std::vector<int>& ax,
                         const std::vector<int>& idx) {
    std::vector<int> dst(src.size());
    for (size_t i = 0; i < src.size(); ++i) dst[i] = acquire();
    for (size_t off = 0; off < dst.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, dst.size() - off);
      IntArr a, d;
      for (int i = 0; i < cnt; ++i) {
        a.v[i] = ax[off + i];
        d.v[i] = idx[off + i];
      }
      hipLaunchKernelGGL(k_slice<T>, dim3(chunks(), n, cnt), dim3(256), 0, st, list_idx(dst, off, cnt),
                         list_idx(src, off, cnt), a, d);
    }
    HIP_OK(hipGetLastError());
    return dst;
  }

  // <1, X> into out[i] (device doubles)
  void inner_ones(const std::vector<int>& src, double* out) {
    for (size_t off = 0; off < src.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, src.size() - off);
      hipLaunchKernelGGL(k_inner_ones<T>, dim3(cnt), dim3(256), 0, st, list_idx(src, off, cnt),
                         out + off, cnt);
    }
    HIP_OK(hipGetLastError());
  }

  // ------------------------------------------------------------ dense I/O
  // Contract objects to dense scale-ordered arrays: out[i * N^3 + ...]
  // <a, b> of two objects into out[0] (device, FP64), by the left
  // environment (k_ip_half / k_ip_env); workspaces from the allocator.
  void inner_pair(int a, int b, double* out) {
    long ecap = 1, tcap = 1;
    for (int k = 0; k < n; ++k) {
      ecap = std::max(ecap, (long)pool[a].cap[k + 1] * pool[b].cap[k + 1]);
      tcap = std::max(tcap, (long)pool[a].cap[k] * PHYS * pool[b].cap[k + 1]);
    }
    double* Ev = (double*)dalloc(8 * ecap);
    double* Tm = (double*)dalloc(8 * tcap);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, Ev, 1.0, 1L);
    for (int k = 0; k < n; ++k) {
      const long th = (long)pool[a].cap[k] * PHYS * pool[b].cap[k + 1];
      const long te = (long)pool[a].cap[k + 1] * pool[b].cap[k + 1];
      hipLaunchKernelGGL(k_ip_half<T>, dim3(ceil_div(std::min(th, 2048L * 256), 256)), dim3(256),
                         0, st, (const MpsDev<T>*)D(a), (const MpsDev<T>*)D(b), k,
                         (const double*)Ev, Tm);
      hipLaunchKernelGGL(k_ip_env<T>, dim3(ceil_div(std::min(te, 2048L * 256), 256)), dim3(256),
                         0, st, (const MpsDev<T>*)D(a), (const MpsDev<T>*)D(b), k,
                         (const double*)Tm, Ev);
    }
    hipLaunchKernelGGL(k_copy_plain<double>, dim3(1), dim3(64), 0, st, (const double*)Ev, out, 1L);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    free_alloc(Tm);
    free_alloc(Ev);
  }

  void to_dense(const std::vector<int>& src, T* out, T* work) {
    long N3 = 1L << (3 * n);
    for (size_t off = 0; off < src.size(); off += MAXB) {
      int cnt = (int)std::min<size_t>(MAXB, src.size() - off);
      MpsList<T> L = list_idx(src, off, cnt);
      T* a = work;
      T* b = out + off * N3;
      // T_0 = 1 (rows = 1, r_0 = 1)
      std::vector<T> ones(cnt, (T)1);
      for (int i = 0; i < cnt; ++i)
        HIP_OK(hipMemcpyAsync(a + i * N3, &ones[i], sizeof(T), hipMemcpyHostToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
      long rows = 1;
      for (int k = 0; k < n; ++k) {
        T* dst = (k % 2 == 0) ? b : a;
        T* srcb = (k % 2 == 0) ? a : b;
        // launch capacity: the largest storage bound of the objects
        int ncap = 1;
        for (int i = 0; i < cnt; ++i) ncap = std::max(ncap, pool[src[off + i]].cap[k + 1]);
        // ensure the final result lands in `b`: n steps alternate a->b->a...
        launch_gemm<T, T, T, Tacc>(FnContract<T>{L, srcb, dst, N3, rows, k}, cnt, (int)rows,
                                   PHYS * ncap, 1, st);
        rows *= PHYS;
      }
      if (n % 2 == 0) {
        // last write went to `a`
        int ch = (int)std::max<long>(1, std::min<long>(2048, (N3 * cnt + 255) / 256));
        hipLaunchKernelGGL(k_copy_plain<T>, dim3(ch), dim3(256), 0, st, (const T*)a, b, N3 * cnt);
      }
    }
    HIP_OK(hipGetLastError());
  }

  // TT-SVD of cnt dense scale-ordered fields W (slot N^3 each; overwritten)
  // into the MPS objs, truncating each bond by the rank rule at tol_r
  // (threshold tol_r^2 ||W||^2 / (n - 1)) and rank cap chi_r.  Every SVD is
  // the FP64 Householder + Jacobi pair, whatever the precision policy.
  void tt_svd(T* W, int cnt, const std::vector<int>& objs, int chi_r, double tol_r) {
    const long N3 = 1L << (3 * n);
    MpsList<T> L = list_idx(objs, 0, cnt);
    RankArr ones;
    for (int k = 0; k <= MAXN; ++k) ones.r[k] = 1;
    hipLaunchKernelGGL(k_set_ranks<T>, dim3(1), dim3(64), 0, st, L, ones, cnt);
    // at site k the remainder has 8 r_k <= 8 min(chi_r, 8^k) rows and
    // rest = 8^(n-1-k) columns; its QR has p = min(rows, rest) and the SVD
    // acts on p columns, at most 1024 in one workgroup.  Slots hold the
    // largest p x rows (R, U S) and p x p (W, W_k) of all sites.
    long slot = 1, pmax = 1;
    {
      long rest = N3;
      for (int k = 0; k < n - 1; ++k) {
        rest /= PHYS;
        const long rows = (long)PHYS * std::min<long>(chi_r, full_bound(n, k));
        const long p = std::min(rest, rows);
        if (p > 1024)
          throw Error(-5, "initial decomposition needs an SVD wider than 1024 columns "
                          "(reduce chi_max or chi_mask_max)");
        slot = std::max(slot, p * rows);
        pmax = std::max(pmax, p);
      }
    }
    for (int o : objs)
      for (int k = 1; k < n; ++k)
        if (pool[o].cap[k] < std::min(chi_r, full_bound(n, k)))
          throw Error(-1, "decomposition target smaller than its rank bound");
    std::vector<void*> tmp;
    auto tdalloc = [&](size_t b) {
      void* q = dalloc(b);
      tmp.push_back(q);
      return q;
    };
    T* nxt = (T*)tdalloc(sizeof(T) * N3 * cnt);
    T* Qb = (T*)tdalloc(sizeof(T) * N3 * cnt);
    double* Rb = (double*)tdalloc(8 * slot * cnt);
    double* Wb = (double*)tdalloc(8 * pmax * pmax * cnt);
    double* USb = (double*)tdalloc(8 * slot * cnt);
    double* Wkb = (double*)tdalloc(8 * pmax * pmax * cnt);
    double* svb = (double*)tdalloc(8 * pmax * cnt);
    double* d2 = (double*)tdalloc(8 * cnt);
    double* disc = (double*)tdalloc(8 * cnt);
    QrWork tw = qw;
    tw.Q1 = (double*)tdalloc(8 * N3 * cnt);
    tw.Q2 = (double*)tdalloc(8 * N3 * cnt);
    tw.mq = N3;
    hipLaunchKernelGGL(k_dense_delta2<T>, dim3(cnt), dim3(256), 0, st, (const T*)W, N3, cnt,
                       tol_r * tol_r / (double)(n > 1 ? n - 1 : 1), d2);
    T* cur = W;
    long rest = N3;
    for (int k = 0; k < n - 1; ++k) {
      rest /= PHYS;
      const long rows = (long)PHYS * std::min<long>(chi_r, full_bound(n, k));
      hipLaunchKernelGGL((k_qr_prep<T, FnTtQr<T>>), dim3(1), dim3(64), 0, st,
                         FnTtQr<T>{L, cur, N3, k, rest, Qb, Rb, slot}, qp, cnt);
      int ch = (int)std::max<long>(1, std::min<long>(2048, (rest * rows + 255) / 256));
      hipLaunchKernelGGL(k_qr_identity<T>, dim3(ch, cnt), dim3(256), 0, st, (const QrProb<T>*)qp);
      hipLaunchKernelGGL(k_householder<T>, dim3(cnt), dim3(256), (size_t)lds_elems * 8, st,
                         (const QrProb<T>*)qp, tw, lds_elems, (double*)nullptr);
      hipLaunchKernelGGL(k_svd_prep<FnTtSvd<T>>, dim3(1), dim3(64), 0, st,
                         FnTtSvd<T>{L, (const QrProb<T>*)qp, k, Wb, pmax * pmax, USb, Wkb,
                                    slot, pmax * pmax, svb, pmax, d2, disc, chi_r, istats},
                         sp, cnt);
      hipLaunchKernelGGL(k_jacobi_svd, dim3(cnt), dim3(1024), (size_t)lds_elems * 8, st,
                         (const SvdProb*)sp, lds_elems, 60, (double*)nullptr);
      hipLaunchKernelGGL(k_tt_core<T>, dim3(64, cnt), dim3(256), 0, st, L, k, (const QrProb<T>*)qp,
                         (const double*)USb, Wkb, slot, pmax * pmax, (const double*)svb, pmax);
      launch_gemm<double, T, T, double>(
          FnTtNext<T>{L, (const QrProb<T>*)qp, Wkb, pmax * pmax, nxt, N3, k, rest}, cnt,
          (int)std::min<long>(chi_r, full_bound(n, k + 1)), (int)rest, 1, st);
      std::swap(cur, nxt);
    }
    hipLaunchKernelGGL(k_store_core<T>, dim3(chunks(), cnt), dim3(256), 0, st, L, (const T*)cur, N3,
                       n - 1);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    for (void* q : tmp) free_alloc(q);
  }
};

}  // namespace mpslbm
