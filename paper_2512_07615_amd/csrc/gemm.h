// Grouped, strided, batched GEMM on MFMA (gfx950).
//
// C = alpha * A * B + beta * C for many small problems in one launch.  A
// problem is produced on the device by a functor (so shapes may depend on
// bond dimensions that live in device memory); the launch grid covers the
// host-known capacity and workgroups whose tile or batch entry is outside
// the actual problem exit at once.
//
// Tiles are 64x64 per 256-thread workgroup (four waves, 32x32 each = 2x2
// MFMA 16x16 blocks), K staged through LDS 64 at a time, the next slice
// loaded into registers while the current one is multiplied.  Operands are read
// through arbitrary element strides and converted to the accumulation type
// Tacc on the way into LDS; Tacc = double uses v_mfma_f64_16x16x4f64,
// Tacc = float uses v_mfma_f32_16x16x4f32.
#pragma once
#include "common.h"

namespace mpslbm {

template <typename TA, typename TB, typename TC>
struct GemmDesc {
  const TA* A;
  const TB* B;
  TC* C;
  int M, N, K;
  int nb1, nb2;  // batch entry b = b1 + nb1 * b2
  long sAm, sAk, sBk, sBn, sCm, sCn;
  long bA1, bB1, bC1, bA2, bB2, bC2;
  double alpha, beta;
  int valid;
};

template <typename TA, typename TB, typename TC>
__host__ __device__ inline GemmDesc<TA, TB, TC> gemm_empty() {
  GemmDesc<TA, TB, TC> d;
  d.A = nullptr; d.B = nullptr; d.C = nullptr;
  d.M = d.N = d.K = 0; d.nb1 = d.nb2 = 1;
  d.sAm = d.sAk = d.sBk = d.sBn = d.sCm = d.sCn = 0;
  d.bA1 = d.bB1 = d.bC1 = d.bA2 = d.bB2 = d.bC2 = 0;
  d.alpha = 1.0; d.beta = 0.0; d.valid = 0;
  return d;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Operand layouts of the 16x16x4 MFMAs: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16]; the four accumulator registers of lane l hold
// column l % 16 and, per register v, row 4 (l / 16) + v for FP32 but row
// l / 16 + 4 v for FP64 (checked on gfx950 with a one-wave probe).
template <typename Tacc> struct MfmaT;
template <> struct MfmaT<double> {
  typedef d4 V;
  __device__ static V op(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <> struct MfmaT<float> {
  typedef f4 V;
  __device__ static V op(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static int row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

constexpr int GT = 64;   // tile edge
constexpr int GK = 64;   // K slice staged through LDS per step

// Round to nearest even BF16 (bit pattern: gfx950's v_cvt_pk_bf16_f32)
// and back.
__device__ inline short bf16_bits(float f) { return __builtin_bit_cast(short, (__bf16)f); }
__device__ inline float bf16_value(short b) {
  return __uint_as_float(((unsigned)(unsigned short)b) << 16);
}
// x = h + m + l with h, m, l BF16: each term the nearest BF16 to what the
// earlier terms leave; the remainders are exact in FP32, and the three
// terms hold 24 significant bits, so the split is exact for normal x
// whose remainders stay normal
__device__ inline void bf16_split3(float x, short& h, short& m, short& l) {
  h = bf16_bits(x);
  const float r1 = x - bf16_value(h);
  m = bf16_bits(r1);
  const float r2 = r1 - bf16_value(m);
  l = bf16_bits(r2);
}

// MODE 0: MFMA in the accumulation type; MODE 1 (Tacc = float): operands
// rounded to BF16, BF16 MFMA with FP32 accumulation; MODE 2 (Tacc = float):
// each FP32 operand split exactly into three BF16 terms x = h + m + l (each
// the BF16 rounding of what the previous ones leave), and the six products
// of combined order up to l (hh, hm, mh, hl, mm, lh) accumulated on BF16
// MFMA in FP32, which carries the product to about FP32 accuracy.
// Split K: with split > 1 each of `split` workgroups of a tile multiplies
// one contiguous share of K (a multiple of GK) and stores its partial tile
// in ws; k_gemm_reduce then sums the shares in a fixed order.
struct KSplit {
  double* ws;
  int split;
};

// BF16 modes on gfx950's v_mfma_f32_16x16x32_bf16: lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16], j = 0..7 (one K
// tile of 32 per instruction), with the accumulator layout of the 16x16x4
// FP32 MFMA (checked with a one-wave probe of exact integer products).  The
// operands are converted once, when a K slice is staged: rounded (MODE 1)
// or split into three BF16 terms (MODE 2), stored K-contiguous per row of A
// and per column of B (row stride BKP) so that a lane's eight K values are
// one 16-byte LDS read.  These modes stage K slices of GKB = 32 (the three
// BF16 terms of a 64 x 64 x 32 slice take 30 KB of LDS), so that four
// workgroups share a CU and hide each other's staging and LDS latency.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
constexpr int GKB = 32;
constexpr int BKP = GKB + 8;  // 80-byte rows: an odd number of 16-byte units

// TS: tile edge, 64 or (BF16 modes) 128; each of the four waves computes
// one (TS/2) x (TS/2) quarter of the tile.
template <typename TA, typename TB, typename TC, typename Tacc, typename F, int MODE = 0,
          int TS = GT>
__global__ __launch_bounds__(256) void k_gemm(F f, int tiles_cap, int batch_cap, double* flops,
                                              KSplit ks) {
  static_assert(TS == GT || (MODE != 0 && TS == 2 * GT), "tile edge");
  typedef typename MfmaT<Tacc>::V V;
  // K slice staged through LDS: 64 for FP32, 32 for FP64 (34 KB of LDS, so
  // that four workgroups share a CU) and the BF16 modes
  constexpr int GKM = (MODE == 0 && sizeof(Tacc) == 4) ? GK : GKB;
  constexpr int WT = TS / 2, NBW = WT / 16;  // a wave's quarter, in 16 x 16 blocks
  constexpr size_t SM0 = 2 * sizeof(Tacc) * GKM * (GT + 1);
  constexpr size_t SMB = (MODE == 2 ? 6 : 2) * sizeof(short) * TS * BKP;
  __shared__ __attribute__((aligned(16))) char smem[MODE == 0 ? SM0 : SMB];
  Tacc (*As)[GT + 1] = reinterpret_cast<Tacc (*)[GT + 1]>(smem);
  Tacc (*Bs)[GT + 1] = reinterpret_cast<Tacc (*)[GT + 1]>(smem + sizeof(Tacc) * GKM * (GT + 1));
  // BF16 tiles: A terms [TS rows][BKP], then B terms [TS columns][BKP]
  short* const Ab = reinterpret_cast<short*>(smem);
  constexpr int NT = MODE == 2 ? 3 : 1;
  short* const Bb = Ab + NT * TS * BKP;
  long wg = blockIdx.x;
  const int kseg = (int)(wg % ks.split);
  wg /= ks.split;
  int tile = (int)(wg % tiles_cap);
  long rest = wg / tiles_cap;
  int b = (int)(rest % batch_cap);
  int prob = (int)(rest / batch_cap);
  GemmDesc<TA, TB, TC> d = f.get(prob);
  if (!d.valid) return;
  if (b >= d.nb1 * d.nb2) return;
  int tn = (d.N + TS - 1) / TS;
  int tm = (d.M + TS - 1) / TS;
  if (tile >= tm * tn || d.M <= 0 || d.N <= 0) return;
  if (flops && tile == 0 && kseg == 0 && threadIdx.x == 0) atomicAdd(flops, 2.0 * d.M * d.N * d.K);
  // share of K: [kb, ke)
  const int kc = ((d.K + ks.split - 1) / ks.split + GK - 1) / GK * GK;
  const int kb = kseg * kc, ke = d.K < kb + kc ? d.K : kb + kc;
  int ti = tile / tn, tj = tile % tn;
  int b1 = b % d.nb1, b2 = b / d.nb1;
  const TA* A = d.A + b1 * d.bA1 + b2 * d.bA2;
  const TB* B = d.B + b1 * d.bB1 + b2 * d.bB2;
  TC* C = d.C + b1 * d.bC1 + b2 * d.bC2;
  int m0 = ti * TS, n0 = tj * TS;
  int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int wm = w >> 1, wn = w & 1;
  V acc[NBW][NBW];
  for (int i = 0; i < NBW; ++i)
    for (int j = 0; j < NBW; ++j)
      for (int v = 0; v < 4; ++v) acc[i][j][v] = 0;
  const bool a_k_contig = (d.sAk == 1);
  const bool b_n_contig = (d.sBn == 1);
  // Software pipeline: the operands of the next K slice are loaded into
  // registers while the MFMAs work on the slice in LDS, so global latency
  // is paid once per K slice rather than per instruction.
  constexpr int LQ = TS * GKM / 256;  // elements of each operand per thread
  Tacc ra[LQ], rb[LQ];
  // Element q of this thread's share of a slice.  FP32/FP64 (MODE 0): one
  // element per 256 threads, the contiguous index fastest.  BF16 modes:
  // four runs of four consecutive K values of one row of A or column of B
  // (q = 4 i + j), so that the converted terms go to LDS as 8-byte writes;
  // lanes still walk the contiguous index of the operand.
  constexpr int TPR = GKM / 4;  // threads per row (column) of a K-contiguous operand
  auto a_pos = [&](int q, int& mm, int& kk) {
    if constexpr (MODE == 0) {
      const int e = tid + 256 * q;
      if (a_k_contig) { mm = e / GKM; kk = e % GKM; } else { mm = e % GT; kk = e / GT; }
    } else {
      const int i = q >> 2, j = q & 3;
      if (a_k_contig) { mm = tid / TPR + (256 / TPR) * i; kk = 4 * (tid % TPR) + j; }
      else { mm = tid % TS; kk = 4 * (tid / TS) + 4 * (256 / TS) * i + j; }
    }
  };
  auto b_pos = [&](int q, int& nn, int& kb) {
    if constexpr (MODE == 0) {
      const int e = tid + 256 * q;
      if (b_n_contig) { kb = e / GT; nn = e % GT; } else { nn = e / GKM; kb = e % GKM; }
    } else {
      const int i = q >> 2, j = q & 3;
      if (b_n_contig) { nn = tid % TS; kb = 4 * (tid / TS) + 4 * (256 / TS) * i + j; }
      else { nn = tid / TPR + (256 / TPR) * i; kb = 4 * (tid % TPR) + j; }
    }
  };
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < LQ; ++q) {
      int mm, kk;
      a_pos(q, mm, kk);
      const int gm = m0 + mm, gk = k0 + kk;
      ra[q] = (gm < d.M && gk < ke) ? (Tacc)A[gm * d.sAm + gk * d.sAk] : (Tacc)0;
      int nn, kb;
      b_pos(q, nn, kb);
      const int gn = n0 + nn, gk2 = k0 + kb;
      rb[q] = (gn < d.N && gk2 < ke) ? (Tacc)B[gk2 * d.sBk + gn * d.sBn] : (Tacc)0;
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += GKM) {
    if constexpr (MODE == 0) {
#pragma unroll
      for (int q = 0; q < LQ; ++q) {
        int mm, kk, nn, kb;
        a_pos(q, mm, kk);
        b_pos(q, nn, kb);
        As[kk][mm] = ra[q];
        Bs[kb][nn] = rb[q];
      }
    } else {
      // a run of four K values -> NT terms of four BF16 each, 8-byte writes
      typedef short s4 __attribute__((ext_vector_type(4)));
#pragma unroll
      for (int i = 0; i < LQ / 4; ++i) {
        int mm, kk, nn, kb;
        a_pos(4 * i, mm, kk);
        b_pos(4 * i, nn, kb);
        s4 ta[NT], tb[NT];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if constexpr (MODE == 1) {
            ta[0][j] = bf16_bits((float)ra[4 * i + j]);
            tb[0][j] = bf16_bits((float)rb[4 * i + j]);
          } else {
            short x0, x1, x2;
            bf16_split3((float)ra[4 * i + j], x0, x1, x2);
            ta[0][j] = x0; ta[1][j] = x1; ta[2][j] = x2;
            bf16_split3((float)rb[4 * i + j], x0, x1, x2);
            tb[0][j] = x0; tb[1][j] = x1; tb[2][j] = x2;
          }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          *reinterpret_cast<s4*>(Ab + t * TS * BKP + mm * BKP + kk) = ta[t];
          *reinterpret_cast<s4*>(Bb + t * TS * BKP + nn * BKP + kb) = tb[t];
        }
      }
    }
    __syncthreads();
    if (k0 + GKM < ke) fetch(k0 + GKM);
    const int kvalid = ke - k0;  // K columns of this slice that are not padding
    if constexpr (MODE == 2) {
#pragma unroll
      for (int ks = 0; ks < GKM / 32; ++ks) {
        if (ks * 32 < kvalid) {
          const int kof = ks * 32 + 8 * (lane >> 4);
          bf8 ah[NBW], am[NBW], al[NBW], bh[NBW], bm[NBW], bl[NBW];
#pragma unroll
          for (int h = 0; h < NBW; ++h) {
            const int ra_ = (wm * WT + 16 * h + (lane & 15)) * BKP + kof;
            const int cb_ = (wn * WT + 16 * h + (lane & 15)) * BKP + kof;
            ah[h] = *reinterpret_cast<const bf8*>(Ab + ra_);
            am[h] = *reinterpret_cast<const bf8*>(Ab + TS * BKP + ra_);
            al[h] = *reinterpret_cast<const bf8*>(Ab + 2 * TS * BKP + ra_);
            bh[h] = *reinterpret_cast<const bf8*>(Bb + cb_);
            bm[h] = *reinterpret_cast<const bf8*>(Bb + TS * BKP + cb_);
            bl[h] = *reinterpret_cast<const bf8*>(Bb + 2 * TS * BKP + cb_);
          }
#pragma unroll
          for (int i = 0; i < NBW; ++i)
#pragma unroll
            for (int jj = 0; jj < NBW; ++jj) {
              // smallest terms first
              V c = acc[i][jj];
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[jj], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bm[jj], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[jj], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[i], bh[jj], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bm[jj], c, 0, 0, 0);
              c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[jj], c, 0, 0, 0);
              acc[i][jj] = c;
            }
        }
      }
    } else if constexpr (MODE == 1) {
#pragma unroll
      for (int ks = 0; ks < GKM / 32; ++ks) {
        if (ks * 32 < kvalid) {
          const int kof = ks * 32 + 8 * (lane >> 4);
          bf8 av[NBW], bv[NBW];
#pragma unroll
          for (int h = 0; h < NBW; ++h) {
            av[h] = *reinterpret_cast<const bf8*>(Ab + (wm * WT + 16 * h + (lane & 15)) * BKP + kof);
            bv[h] = *reinterpret_cast<const bf8*>(Bb + (wn * WT + 16 * h + (lane & 15)) * BKP + kof);
          }
#pragma unroll
          for (int i = 0; i < NBW; ++i)
#pragma unroll
            for (int jj = 0; jj < NBW; ++jj)
              acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[jj], acc[i][jj], 0, 0, 0);
        }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < GKM / 4; ++ks) {
        if (ks * 4 < kvalid) {
          int kr = ks * 4 + (lane >> 4);
          Tacc a0 = As[kr][wm * 32 + (lane & 15)];
          Tacc a1 = As[kr][wm * 32 + 16 + (lane & 15)];
          Tacc bb0 = Bs[kr][wn * 32 + (lane & 15)];
          Tacc bb1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
          acc[0][0] = MfmaT<Tacc>::op(a0, bb0, acc[0][0]);
          acc[0][1] = MfmaT<Tacc>::op(a0, bb1, acc[0][1]);
          acc[1][0] = MfmaT<Tacc>::op(a1, bb0, acc[1][0]);
          acc[1][1] = MfmaT<Tacc>::op(a1, bb1, acc[1][1]);
        }
      }
    }
    __syncthreads();
  }
  if (ks.split > 1) {
    double* W = ks.ws + ((((long)prob * batch_cap + b) * tiles_cap + tile) * ks.split + kseg) *
                            (TS * TS);
#pragma unroll
    for (int i = 0; i < NBW; ++i)
#pragma unroll
      for (int j = 0; j < NBW; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * WT + i * 16 + MfmaT<Tacc>::row(lane, v);
          const int col = wn * WT + j * 16 + (lane & 15);
          W[row * TS + col] = (double)acc[i][j][v];
        }
    return;
  }
  const double alpha = d.alpha, beta = d.beta;
#pragma unroll
  for (int i = 0; i < NBW; ++i)
#pragma unroll
    for (int j = 0; j < NBW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = m0 + wm * WT + i * 16 + MfmaT<Tacc>::row(lane, v);
        int col = n0 + wn * WT + j * 16 + (lane & 15);
        if (row < d.M && col < d.N) {
          TC* p = C + row * d.sCm + col * d.sCn;
          double val = alpha * (double)acc[i][j][v];
          if (beta != 0.0) val += beta * (double)(*p);
          *p = (TC)val;
        }
      }
}

// Sum of the split-K partial tiles in share order, then C = alpha sum + beta C.
// Each output tile is shared by RQ workgroups (an eighth of its entries
// each), so that one pass of loads covers a workgroup's part and the launch
// spreads over RQ times as many CUs.
constexpr int RQ = 8;
template <typename TA, typename TB, typename TC, typename F, int TS = GT>
__global__ __launch_bounds__(256) void k_gemm_reduce(F f, int tiles_cap, int batch_cap, KSplit ks) {
  long wg = blockIdx.x;
  const int part = (int)(wg % RQ);
  wg /= RQ;
  int tile = (int)(wg % tiles_cap);
  long rest = wg / tiles_cap;
  int b = (int)(rest % batch_cap);
  int prob = (int)(rest / batch_cap);
  GemmDesc<TA, TB, TC> d = f.get(prob);
  if (!d.valid) return;
  if (b >= d.nb1 * d.nb2) return;
  int tn = (d.N + TS - 1) / TS;
  int tm = (d.M + TS - 1) / TS;
  if (tile >= tm * tn || d.M <= 0 || d.N <= 0) return;
  int ti = tile / tn, tj = tile % tn;
  int b1 = b % d.nb1, b2 = b / d.nb1;
  TC* C = d.C + b1 * d.bC1 + b2 * d.bC2;
  const double* W = ks.ws + (((long)prob * batch_cap + b) * tiles_cap + tile) * ks.split * (TS * TS);
  // two outputs per thread, the loads of all their shares issued together,
  // then each output summed in share order
  constexpr int OUT = 2, PART = TS * TS / RQ;
  const int e_end = (part + 1) * PART;
  for (int e0 = part * PART + threadIdx.x; e0 < e_end; e0 += OUT * blockDim.x) {
    double v[OUT][8];
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
      const int e = e0 + o * blockDim.x;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[o][q] = (e < e_end && q < ks.split) ? W[(long)q * (TS * TS) + e] : 0.0;
    }
#pragma unroll
    for (int o = 0; o < OUT; ++o) {
      const int e = e0 + o * blockDim.x;
      const int row = ti * TS + e / TS, col = tj * TS + e % TS;
      if (e >= e_end || row >= d.M || col >= d.N) continue;
      double sum = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < ks.split) sum += v[o][q];
      TC* p = C + row * d.sCm + col * d.sCn;
      double val = d.alpha * sum;
      if (d.beta != 0.0) val += d.beta * (double)(*p);
      *p = (TC)val;
    }
  }
}

// Launch helper: grid = nprob * batch_cap * tiles_cap (each host-known caps),
// times ks.split when K is split (ks.ws then holds
// nprob * batch_cap * tiles_cap * split tiles of TS x TS doubles).
template <typename TA, typename TB, typename TC, typename Tacc, typename F, int MODE = 0,
          int TS = GT>
inline void launch_gemm(const F& f, int nprob, int mcap, int ncap, int batch_cap,
                        hipStream_t s, double* flops = nullptr, KSplit ks = KSplit{nullptr, 1}) {
  if (nprob <= 0 || mcap <= 0 || ncap <= 0 || batch_cap <= 0) return;
  if (ks.split < 1 || !ks.ws) ks.split = 1;
  int tiles = ceil_div(mcap, TS) * ceil_div(ncap, TS);
  long grid = (long)nprob * batch_cap * tiles;
  if (grid <= 0) return;
  hipLaunchKernelGGL((k_gemm<TA, TB, TC, Tacc, F, MODE, TS>), dim3((unsigned)(grid * ks.split)),
                     dim3(256), 0, s, f, tiles, batch_cap, flops, ks);
  if (ks.split > 1)
    hipLaunchKernelGGL((k_gemm_reduce<TA, TB, TC, F, TS>), dim3((unsigned)(grid * RQ)), dim3(256),
                       0, s, f, tiles, batch_cap, ks);
  HIP_OK(hipGetLastError());
}

}  // namespace mpslbm
