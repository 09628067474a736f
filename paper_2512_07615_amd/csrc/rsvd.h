// Rank-predicted randomized truncation (FP32 and BF16 policies).
//
// At a bond whose rank in the previous step, r_hat, is known, the
// truncation of the core unfolding M (s x c, FP64 Gram G = M M^T) is first
// tried on a sketch of width l = r_hat + p < s instead of the full s x s
// problem: a randomized range finder (Halko, Martinsson and Tropp, SIAM
// Review 53 (2011), algorithm 4.1) followed by a Rayleigh-Ritz step on the
// Gram (their algorithm 5.3 in Gram form):
//   Y = M Omega, Omega Gaussian (c x l);  Q = orth(Y) (Cholesky-QR2);
//   T = Q^T G Q;  T = V diag(lambda) V^T;  U = Q V.
// The sketch is taken from M itself, not from a power of G: the FP64 Gram of
// Y then resolves singular values of M down to 1e-7 of the largest, as the
// full path does.
// Projecting M onto span(U_r) discards exactly trace(G) - sum_{j<=r}
// lambda_j, so the rank rule is applied with the exact discarded weight:
// the eigen step of T receives the allowance delta^2 - (trace G - trace T).
// The sketch is accepted when the rule is met at some r strictly inside it
// (r < rank of Q, r <= chi), or, at bonds held at chi, when its discarded
// weight is provably within 5% of the optimal rank-chi truncation's (see
// k_rs_accept); every other problem falls back to the full
// eigendecomposition of G.  Accepted and fallback problems write the same
// outputs (US = U_r Sigma_r, Ut = Sigma_r^{-1} U_r^T, bond rank, discarded
// weight), so the rest of the rounding is unchanged.
#pragma once
#include "linalg.h"
#include "mlp.h"

namespace mpslbm {

// Work arrays of the randomized path; matrices use slots of sq doubles.
struct RsWork {
  double* Om;     // c x l Gaussian test matrix, shared (som doubles)
  double* Y;      // s x l: M Omega
  double* T;      // Grams of the orthonormalisation, then Q^T G Q
  double* B;      // P R11^{-1} of the pivoted Cholesky passes
  double* R;      // R P^T of the pivoted Cholesky passes
  double* B2;
  double* R2;
  double* Q;      // s x rank1
  double* Q2;     // s x rank2 (orthonormal basis of the sketch)
  double* W;      // s x rank2: G Q2
  double* USt;    // rank2 x r
  double* Utt;    // r x rank2
  int* s0;        // bond dimension before the truncation
  int* ell;       // sketch width, 0 = not attempted
  int* rank1;     // rank of the first Cholesky-QR pass
  int* rank2;     // rank of the second pass (columns of Q2)
  int* rankT;     // numerical rank of T
  int* rsel;      // rank chosen on the sketch
  int* acc;       // 1 = sketch accepted
  int* tries;     // [0] problems attempted, [1] accepted (totals)
  double* budget; // delta^2 - (trace G - trace T)
  double* disc;   // tail of the spectrum of T beyond rsel
  double* trG;    // trace of G
  long sq;
  long som;       // slot of Om (8 sq: c <= 8 s_cap)
};

// Sketch width from the prediction (pred[i] < 1: none) and clearing of the
// per-problem state; the trace of G on the way.
template <typename T>
__global__ void k_rs_plan(MpsList<T> L, int k, const int* pred, int over, const double* G,
                          RsWork w, int cnt) {
  const int i = blockIdx.x;
  if (i >= cnt) return;
  __shared__ double red[8];
  const int s = L.p[i]->r[k];
  double a = 0.0;
  for (int j = threadIdx.x; j < s; j += blockDim.x) a += G[i * w.sq + (long)j * s + j];
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    const int pr = pred ? pred[i] : -1;
    const int l = (pr > 0 && pr + over < s) ? pr + over : 0;
    w.ell[i] = l;
    w.s0[i] = s;
    w.rank1[i] = 0;
    w.rank2[i] = 0;
    w.rankT[i] = 0;
    w.acc[i] = 0;
    w.trG[i] = a;
    w.budget[i] = -1.0;
    if (l > 0) atomicAdd(w.tries, 1);
  }
}

// Y (s x l) = M Omega, M the right unfolding of core k (s x c, row-major)
template <typename T>
struct FRsMOm {
  MpsList<T> L; int k; RsWork w;
  __device__ GemmDesc<T, double, double> get(int i) const {
    GemmDesc<T, double, double> d = gemm_empty<T, double, double>();
    const int l = w.ell[i];
    if (l <= 0) return d;
    MpsDev<T>* m = L.p[i];
    const int s = m->r[k], c = PHYS * m->r[k + 1];
    d.A = core_ptr(m, k); d.B = w.Om; d.C = w.Y + i * w.sq;
    d.M = s; d.N = l; d.K = c;
    d.sAm = c; d.sAk = 1; d.sBk = l; d.sBn = 1; d.sCm = l; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// out (n x n) = X^T X for X (s x n, ld n); n = dims[i] (0: skipped)
template <typename T>
struct FRsGram {
  MpsList<T> L; int k; const double* X; double* out; const int* dims; long sq;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    const int nn = dims[i];
    if (nn <= 0) return d;
    const int s = L.p[i]->r[k];
    d.A = X + i * sq; d.B = X + i * sq; d.C = out + i * sq;
    d.M = nn; d.N = nn; d.K = s;
    d.sAm = 1; d.sAk = nn; d.sBk = nn; d.sBn = 1; d.sCm = nn; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// C (s x r) = X (s x n, ld n) Bm (n x r, ld r); n = dn[i], r = dr[i]
template <typename T>
struct FRsXB {
  MpsList<T> L; int k; const double* X; const double* Bm; double* C; const int* dn;
  const int* dr; long sq;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    const int nn = dn[i], r = dr[i];
    if (nn <= 0 || r <= 0) return d;
    const int s = L.p[i]->r[k];
    d.A = X + i * sq; d.B = Bm + i * sq; d.C = C + i * sq;
    d.M = s; d.N = r; d.K = nn;
    d.sAm = nn; d.sAk = 1; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// W (s x rho) = G Q2, rho = rank2
template <typename T>
struct FRsGQ {
  MpsList<T> L; int k; const double* G; RsWork w;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    const int r = w.rank2[i];
    if (w.ell[i] <= 0 || r <= 0) return d;
    const int s = L.p[i]->r[k];
    d.A = G + i * w.sq; d.B = w.Q2 + i * w.sq; d.C = w.W + i * w.sq;
    d.M = s; d.N = r; d.K = s;
    d.sAm = s; d.sAk = 1; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// T (rho x rho) = Q2^T W
template <typename T>
struct FRsQtW {
  MpsList<T> L; int k; RsWork w;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    const int r = w.rank2[i];
    if (w.ell[i] <= 0 || r <= 0) return d;
    const int s = L.p[i]->r[k];
    d.A = w.Q2 + i * w.sq; d.B = w.W + i * w.sq; d.C = w.T + i * w.sq;
    d.M = r; d.N = r; d.K = s;
    d.sAm = 1; d.sAk = r; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// allowance left for the tail of T: delta^2 - (trace G - trace T)
__global__ void k_rs_budget(const double* delta2, RsWork w, int cnt) {
  const int i = blockIdx.x;
  if (i >= cnt) return;
  __shared__ double red[8];
  const int r = w.rank2[i];
  if (w.ell[i] <= 0 || r <= 0) return;
  double a = 0.0;
  for (int j = threadIdx.x; j < r; j += blockDim.x) a += w.T[i * w.sq + (long)j * r + j];
  a = block_sum(a, red);
  if (threadIdx.x == 0) w.budget[i] = delta2[i] - fmax(w.trG[i] - a, 0.0);
}

// dims of the eigen problem of T
__global__ void k_rs_dims_T(RsWork w, int* out, int cnt) {
  const int i = threadIdx.x;
  if (i < cnt) out[i] = w.ell[i] > 0 ? w.rank2[i] : 0;
}

// eigen problem of T; rank and tail go to the sketch's own arrays
struct FnRsEig {
  RsWork w; int chi; int* fail;
  float* feat = nullptr;  // rank-predictor features (Ritz values of the sketch)
  float stepf = 0.0f;
  __device__ EigProb get(int i) const {
    EigProb p;
    p.feat = feat ? feat + i * MLP_IN : nullptr;
    p.stepf = stepf;
    p.A = w.R + i * w.sq;  // R P^T of the Cholesky of T, read as its transpose
    p.s = w.rank2[i];
    p.c = w.rankT[i];
    p.valid = (w.ell[i] > 0 && w.rank2[i] > 0) ? 1 : 0;
    p.delta2 = w.budget[i];  // negative: the rule keeps min(rank, chi)
    p.chi = chi;
    p.rank_out = w.rsel + i;
    p.US = w.USt + i * w.sq;
    p.Ut = w.Utt + i * w.sq;
    p.disc = w.disc + i;
    p.fail = fail;
    return p;
  }
};

// Acceptance; the bond rank and the discarded weight of accepted problems.
// With ex = trace G - trace T (the weight outside the sketch) and tail the
// Ritz values of T beyond the chosen rank r < rank of Q:
//  * tolerance-bound: ex + tail <= delta^2, the rule of the full path holds
//    with the exact discarded weight;
//  * cap-bound (r = chi): the Ritz values beyond chi alone exceed delta^2;
//    as the j-th Ritz value never exceeds the j-th eigenvalue of G (Cauchy
//    interlacing), the optimal rank-chi discarded weight d* is at least
//    tail, so the full path also keeps chi, and the sketch discards
//    ex + tail <= (1 + RS_CAP_SLACK) d* when ex <= RS_CAP_SLACK * tail.
constexpr double RS_CAP_SLACK = 0.05;
template <typename T>
__global__ void k_rs_accept(MpsList<T> L, int k, const double* delta2, int chi, RsWork w,
                            double* disc_out, int cnt) {
  const int i = threadIdx.x;
  if (i >= cnt) return;
  int a = 0;
  const double ex = delta2[i] - w.budget[i];
  if (w.ell[i] > 0 && w.rank2[i] > 0) {
    const int r = w.rsel[i];
    const double tail = w.disc[i];
    if (r >= 1 && r < w.rank2[i]) {
      if (w.budget[i] >= 0.0 && tail <= w.budget[i]) a = 1;
      else if (r == chi && tail > delta2[i] && ex <= RS_CAP_SLACK * tail) a = 1;
    }
  }
  w.acc[i] = a;
  if (a) {
    L.p[i]->r[k] = w.rsel[i];
    // trace G - sum of the kept Ritz values
    disc_out[i * (MAXN + 1) + k] = ex + w.disc[i];
    atomicAdd(w.tries + 1, 1);
  }
}

// dims of the full path: accepted problems are switched off
template <typename T>
__global__ void k_rs_dims_full(MpsList<T> L, int k, const RsWork w, int* out, int cnt) {
  const int i = threadIdx.x;
  if (i < cnt) out[i] = w.acc[i] ? 0 : L.p[i]->r[k];
}

// accepted outputs: US (s x r, ld r) = Q2 USt;  Ut (r x s, ld s) = Utt Q2^T
struct FRsUS {
  RsWork w; double* US; long sus;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    if (!w.acc[i]) return d;
    const int s = w.s0[i], r = w.rsel[i], rho = w.rank2[i];
    d.A = w.Q2 + i * w.sq; d.B = w.USt + i * w.sq; d.C = US + i * sus;
    d.M = s; d.N = r; d.K = rho;
    d.sAm = rho; d.sAk = 1; d.sBk = r; d.sBn = 1; d.sCm = r; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};
struct FRsUt {
  RsWork w; double* Ut; long sus;
  __device__ GemmDesc<double, double, double> get(int i) const {
    GemmDesc<double, double, double> d = gemm_empty<double, double, double>();
    if (!w.acc[i]) return d;
    const int s = w.s0[i], r = w.rsel[i], rho = w.rank2[i];
    d.A = w.Utt + i * w.sq; d.B = w.Q2 + i * w.sq; d.C = Ut + i * sus;
    d.M = r; d.N = s; d.K = rho;
    d.sAm = rho; d.sAk = 1; d.sBk = 1; d.sBn = rho; d.sCm = s; d.sCn = 1;
    d.valid = 1;
    return d;
  }
};

// ---- learned rank predictor (see mlp.h) ------------------------------------
// Inputs of one bond from the previous step's features, and a pending
// training sample for every problem that has them (predk[i] > 0).
__global__ void k_mlp_gather(const float* featk, const int* predk, float* x, float* smp_x,
                             float* smp_t, int* smp_n, int* smp_slot, int cap, int cnt) {
  const int i = threadIdx.x;
  if (i >= cnt) return;
  if (predk[i] <= 0) {
    smp_slot[i] = -1;
    for (int q = 0; q < MLP_IN; ++q) x[i * MLP_IN + q] = 0.0f;
    return;
  }
  const int slot = atomicAdd(smp_n, 1) % cap;
  for (int q = 0; q < MLP_IN; ++q) {
    const float f = featk[i * MLP_IN + q];
    x[i * MLP_IN + q] = f;
    smp_x[(long)slot * MLP_IN + q] = f;
  }
  smp_t[slot] = 0.0f;
  smp_slot[i] = slot;
}

// predicted rank: the previous rank plus 16 times the network's output,
// within [1, current bond]; -1 where there is no previous rank
template <typename T>
__global__ void k_mlp_rank(MpsList<T> L, int k, const int* predk, const float* y, int* out,
                           int cnt) {
  const int i = threadIdx.x;
  if (i >= cnt) return;
  const int rp = predk[i];
  if (rp <= 0) {
    out[i] = -1;
    return;
  }
  const int s = L.p[i]->r[k];
  int r = rp + (int)lrintf(16.0f * y[i]);
  out[i] = r < 1 ? 1 : (r > s ? s : r);
}

// after the truncation: targets of the pending samples (rank change / 16)
// and, once trained, the absolute rank errors of the network and of the
// previous-rank predictor
template <typename T>
__global__ void k_mlp_target(MpsList<T> L, int k, const int* predk, const int* pred2,
                             int trained, float* smp_t, const int* smp_slot, double* err,
                             int cnt) {
  const int i = threadIdx.x;
  if (i >= cnt) return;
  const int slot = smp_slot[i];
  if (slot < 0) return;
  const int r = L.p[i]->r[k], rp = predk[i];
  smp_t[slot] = (float)(r - rp) / 16.0f;
  if (trained) {
    atomicAdd(err, (double)abs(pred2[i] - r));
    atomicAdd(err + 1, (double)abs(rp - r));
    atomicAdd(err + 2, 1.0);
  }
}

// the chosen ranks become the next step's predictions
template <typename T>
__global__ void k_rs_store(MpsList<T> L, int k, int* pred, int cnt) {
  const int i = threadIdx.x;
  if (i < cnt) pred[i] = L.p[i]->r[k];
}

}  // namespace mpslbm
