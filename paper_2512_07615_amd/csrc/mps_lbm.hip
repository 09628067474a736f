// C ABI and step schedule of the MI355X MPS lattice Boltzmann library.
//
// One BGK step on the MPS populations of a D3Q19 or D3Q15 velocity set
// (Section 3.2 of the paper), in this order:
//  1. rho = sum_i f_i and j_a = sum_i c_ia f_i (sums, rounded pairwise);
//  2. rho_0 = <1, rho> / N_fluid;
//  3. r ~ 1/rho: Taylor-2 about rho_0, r = (1/rho_0)(1 - e + e (.) e) with
//     e = rho/rho_0 - 1, or Newton-Schulz y <- y (.) (2 - rho (.) y);
//  4. j_eq = j + tau g rho, u_a = j_eq,a (.) r, Pi_ab = j_eq,a (.) u_b;
//  5. BGK: f_i <- (1 - w) f_i + w w_i [S0 + 3 c_i.j_eq + 4.5 c_i c_i : Pi],
//     S0 = rho - 1.5 tr Pi, w = 1/tau;
//  6. streaming by shift MPOs, one axis at a time, rounded after each;
//  7. open faces: f_i += m_B (.) b(f_ihat post-collision, rho_b, u_b);
//  8. obstacles: f_i <- f_i - m_O (.) f_i + S(c_i)(m_O (.) f_ihat).
// Every sum is a pairwise tree (adjacent pairs, odd last term carried up)
// rounded after each addition; the CPU oracle follows the same schedule.
// Roundings that do not depend on each other share one batch: the j_eq sums
// run with the first sums of step 3, each population's streaming shifts are
// batched by their order (two levels for D3Q19 edges, three for D3Q15
// corners), and the first pair of the
// obstacle sum runs with the first shift level of the reflected part.  This
// changes which launch carries an operation, never the operations applied to
// one MPS or their order.
#include "../../include/mps_lbm.h"

#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "engine.h"

using namespace mpslbm;

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

namespace {

struct Sim {
  virtual ~Sim() {}
  virtual int domains() const = 0;
  virtual void step(int nsteps) = 0;
  virtual void to_dense(int d, int what, double* out) = 0;
  virtual void observables(int d, mps_lbm_obs* o) = 0;
  virtual void set_timing(int kind) = 0;
  virtual void kstats(mps_lbm_kstats* o) = 0;
  virtual int get_mps(int d, int which, double* out, size_t out_len, int* bonds) = 0;
  virtual long cells(int d) const = 0;
  virtual int velocities(int d) const = 0;
  virtual double kinetic_energy(int d) = 0;
  virtual void capture() = 0;
  virtual float train_predictor(int epochs, float lr) = 0;
  virtual int autotune() = 0;
  virtual void predictor_info(mps_lbm_predictor_info* o) = 0;
  virtual int numeric_status() = 0;
  virtual bool fatal_seen() const = 0;
  virtual void raise_flags(int nonfinite, int sweep_limit) = 0;
  virtual void rank_model(float* w, int load) = 0;
  virtual void set_face_profile(int d, int face, const double* coef, double dt) = 0;
  virtual void set_region(int d, const int* lo, const int* hi, double rho_ref) = 0;
  // pieces of capture() for a handle whose domains form several groups
  virtual void capture_prepare() {}
  virtual void capture_record() {}
  virtual void capture_finish() {}
  virtual void count_step() {}
};

// Copy MPS i of S into MPS i of D (same capacity profile), converting the
// element type: ranks and the cores in use.
template <typename Ts, typename Td>
__global__ void k_convert_mps(MpsList<Ts> S, MpsList<Td> Dl, int n) {
  const int i = blockIdx.z, k = blockIdx.y;
  const MpsDev<Ts>* a = S.p[i];
  MpsDev<Td>* b = Dl.p[i];
  if (blockIdx.x == 0 && k == 0 && (int)threadIdx.x <= n) b->r[threadIdx.x] = a->r[threadIdx.x];
  if (k >= n) return;
  const long tot = (long)a->r[k] * PHYS * a->r[k + 1];
  const Ts* x = a->data + a->off[k];
  Td* y = b->data + b->off[k];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    y[e] = (Td)x[e];
}

// Chain of two MPS (Appendix D): the la cores of a (coarse grid) followed by
// the lb cores of b (fine grid) form the MPS of their tensor product; the
// bond between them is 1.  Grid (chunks, la + lb).
template <typename Ts, typename Td>
__global__ void k_chain_mps(const MpsDev<Ts>* a, int la, const MpsDev<Ts>* b, int lb,
                            MpsDev<Td>* d) {
  const int k = blockIdx.y;
  if (blockIdx.x == 0 && k == 0) {
    const int j = threadIdx.x;
    if (j <= la) d->r[j] = a->r[j];
    if (j >= 1 && j <= lb) d->r[la + j] = b->r[j];
  }
  const MpsDev<Ts>* src = k < la ? a : b;
  const int ks = k < la ? k : k - la;
  const long tot = (long)src->r[ks] * PHYS * src->r[ks + 1];
  const Ts* x = src->data + src->off[ks];
  Td* y = d->data + d->off[k];
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < tot;
       e += (long)gridDim.x * blockDim.x)
    y[e] = (Td)x[e];
}

// Dense solid of a coarse layout (side 2^(n-k)) with the fine unit geometry
// (side 2^k) in each of its solid cells (Appendix D composition).
__global__ void k_compose_solid(const uint8_t* outer, const uint8_t* inner, uint8_t* out, int n,
                                int k) {
  const long N3 = 1L << (3 * n);
  const int N = 1 << n, L = 1 << (n - k), K = 1 << k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    const int x = (int)(e >> (2 * n)), y = (int)((e >> n) & (N - 1)), z = (int)(e & (N - 1));
    const long eo = ((long)(x >> k) * L + (y >> k)) * L + (z >> k);
    const long ei = ((long)(x & (K - 1)) * K + (y & (K - 1))) * K + (z & (K - 1));
    out[e] = (outer[eo] != 0 && inner[ei] != 0) ? 1 : 0;
  }
}

__global__ void k_u8_to_f64(const uint8_t* in, double* out, long count) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < count;
       e += (long)gridDim.x * blockDim.x)
    out[e] = in[e] ? 1.0 : 0.0;
}

__global__ void k_add_flags(int* istats, int sweep_limit, int nonfinite) {
  if (threadIdx.x == 0) {
    istats[0] += sweep_limit;
    istats[1] += nonfinite;
  }
}

__global__ void k_div_vec(const double* num, const double* den, double* out, int cnt) {
  int i = threadIdx.x;
  if (i < cnt) out[i] = num[i] / den[i];
}

// State of one domain: its configuration and the pool indices of its MPS.
struct Domain {
  mps_lbm_config cfg;
  int f[19];
  int mask = -1;
  int fplane[6];
  double n_fluid = 0.0;
  double mask_err = 0.0;
  double face_err = 0.0;
  // region of interest of the pressure metric (Section 4.2)
  int region = -1;
  double region_cells = 0.0;
  double region_rho = 1.0;
  double region_err = 0.0;
};

// Time profile of a velocity face: the face velocity is scaled by
// phi(t) = c0 + c1 (1 - e^(-c2 t)) + c3 t^c4 e^(-c5 t), t = steps taken x dt
// (Section 4.1 inflows: a ramp and a pulse).
struct FaceProf {
  double c[6];
  double dt;
  int on;
  int pad;
};

// Per-step face scales: entry fs + j (j = 6 d + face) of the scalar array
// becomes phi(t) for a profiled face and 1 otherwise; entry cnt counts the
// steps taken, read before it is advanced.  One workgroup.
__global__ void k_face_time(const FaceProf* prof, double* sc, int fs, int cnt, int nf) {
  const int j = threadIdx.x;
  const double steps = sc[cnt];
  if (j < nf) {
    const FaceProf p = prof[j];
    double v = 1.0;
    if (p.on) {
      const double t = steps * p.dt;
      v = p.c[0] + p.c[1] * (1.0 - exp(-p.c[2] * t));
      if (p.c[3] != 0.0) v += p.c[3] * pow(t, p.c[4]) * exp(-p.c[5] * t);
    }
    sc[fs + j] = v;
  }
  __syncthreads();
  if (j == 0) sc[cnt] = steps + 1.0;
}

// Dense [x][y][z] indicator of the fluid cells of the box lo <= x < hi
// (solid read from the scale-ordered mask field, > 1/2 = solid; NULL = no
// solid), and its cell count added to *count.
template <typename T>
__global__ __launch_bounds__(256) void k_box_fluid(const T* mask_s, double* out, int n, int x0,
                                                   int y0, int z0, int x1, int y1, int z1,
                                                   double* count) {
  __shared__ double red[4];
  const long N3 = 1L << (3 * n);
  const int N = 1 << n;
  double c = 0.0;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    const int x = (int)(e >> (2 * n)), y = (int)((e >> n) & (N - 1)), z = (int)(e & (N - 1));
    const bool in = x >= x0 && x < x1 && y >= y0 && y < y1 && z >= z0 && z < z1;
    const bool solid = mask_s && (double)mask_s[scale_index(x, y, z, n)] > 0.5;
    const double v = (in && !solid) ? 1.0 : 0.0;
    out[e] = v;
    c += v;
  }
  c = block_sum(c, red);
  if (threadIdx.x == 0) atomicAdd(count, c);
}

// Obstacle geometry given as a coarse layout outer [L][L][L] (L = 2^l) and
// the fine unit geometry inner [K][K][K] (K = 2^(n-l)) repeated in each of
// its solid cells (Appendix D); host arrays, 1 = solid.
struct MaskParts {
  const uint8_t* outer;
  int l;
  const uint8_t* inner;
};

// dense [x][y][z] field: 1 on the fluid cells of the plane x_ax = idx
__global__ void k_face_plane(const uint8_t* solid, double* out, int n, int ax, int idx) {
  const long N3 = 1L << (3 * n);
  const int N = 1 << n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < N3;
       e += (long)gridDim.x * blockDim.x) {
    const int c[3] = {(int)(e >> (2 * n)), (int)((e >> n) & (N - 1)), (int)(e & (N - 1))};
    out[e] = (c[ax] == idx && !(solid && solid[e])) ? 1.0 : 0.0;
  }
}

// One engine advancing D domains of equal n, chi and precision together:
// every operation of the step is issued once for the MPS of all domains, so
// launches carry D times as many problems (Sections 3.2 and 2).
template <typename T>
struct SimT : Sim {
  typedef typename Engine<T>::Term Term;
  typedef typename Engine<T>::PairSum PairSum;
  Engine<T> E;
  std::unique_ptr<Engine<double>> X;  // FP64 island (reduced-precision policies)
  int one64 = -1;
  hipStream_t st;
  int n, N, D;
  const LatticeTab* lat = &kD3Q19;  // velocity set of every domain
  int Q = 19;
  long N3;
  std::vector<Domain> dom;
  int one = -1;
  double* rho0 = nullptr;   // device [D]
  double* nfl = nullptr;    // device [D]: fluid cell counts
  double* sbuf = nullptr;   // device sums of a step (rho_0 numerators, norms)
  FaceProf* fprof = nullptr;     // device [6 D] velocity-face time profiles
  std::vector<FaceProf> hprof;   // host copy
  int fs_off() const { return D + 8; }
  int cnt_off() const { return D + 8 + 6 * D; }
  int* cvec_dev = nullptr;
  double* w_dev = nullptr;
  long long steps = 0;
  long long last_roundings = 0, last_products = 0;

  SimT(const mps_lbm_config* cfgs, int count, hipStream_t s, const Allocator& al) : st(s) {
    const mps_lbm_config& c = cfgs[0];
    E.al = al;
    E.st = s;
    D = count;
    n = c.n;
    N = 1 << n;
    N3 = 1L << (3 * n);
    lat = c.lattice == MPS_LBM_D3Q15 ? &kD3Q15 : &kD3Q19;
    Q = lat->q;
    dom.resize(D);
    for (int d = 0; d < D; ++d) {
      dom[d].cfg = cfgs[d];
      for (int i = 0; i < 6; ++i) dom[d].fplane[i] = -1;
    }
    E.sweeps = c.sweeps;
    E.bf16_products = c.precision == MPS_LBM_BF16 ? 1 : c.precision == MPS_LBM_BF16X3 ? 2 : 0;
    E.setup(n, c.chi_max, c.tol, s, 96 + 160 * D, std::min(MAXB, Q * D));
    if (sizeof(T) == 4) {
      // FP64 island of the reduced-precision policies: the inverse density
      // (its sums and products) runs in an FP64 engine on the same stream
      X.reset(new Engine<double>());
      X->al = al;
      X->sweeps = c.sweeps;
      X->setup(n, c.chi_max, c.tol, s, 8 + 8 * D, std::min(MAXB, D));
      // its truncations use the factorisations of the reduced-precision
      // policies (rank-revealing Cholesky-QR2 and Gram eigendecomposition,
      // all in FP64) on FP64 data: directions below about 3e-8 of the
      // largest singular value count as zero (FP64 Gram resolution) and the
      // eigenvectors are orthonormal to 1e-12
      X->fast = true;
      X->eps_rank = 1e-15;
      X->eig_orth_tol = 1e-12;
      one64 = X->acquire();
      X->set_ones(one64);
    }
    if (c.rank_predictor) E.enable_rsvd(c.rank_oversample, c.seed);
    if (c.rank_predictor == 2) E.enable_mlp(c.seed);
    // scalars of the step: rho_0 per domain, then the per-step face scales
    // (6 per domain, Coef::s) and the count of steps taken
    rho0 = (double*)E.dalloc(8 * (cnt_off() + 1));
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(256), 0, st, rho0 + fs_off(), 1.0, 6L * D);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, rho0 + cnt_off(), 0.0, 1L);
    hprof.assign(6 * D, FaceProf{});
    fprof = (FaceProf*)E.dalloc(sizeof(FaceProf) * 6 * D);
    HIP_OK(hipMemcpy(fprof, hprof.data(), sizeof(FaceProf) * 6 * D, hipMemcpyHostToDevice));
    nfl = (double*)E.dalloc(8 * (D + 8));
    sbuf = (double*)E.dalloc(8 * (19 * D + 64));
    int cvec[3 * QMAX];
    double w[QMAX];
    for (int i = 0; i < Q; ++i) {
      for (int a = 0; a < 3; ++a) cvec[3 * i + a] = lat->c[i][a];
      w[i] = lat->w[i];
    }
    cvec_dev = (int*)E.dalloc(sizeof(cvec));
    w_dev = (double*)E.dalloc(sizeof(w));
    HIP_OK(hipMemcpy(cvec_dev, cvec, sizeof(cvec), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(w_dev, w, sizeof(w), hipMemcpyHostToDevice));
    one = E.acquire();
    E.set_ones(one);
  }

  int domains() const override { return D; }
  int velocities(int) const override { return Q; }
  long cells(int) const override { return N3; }

  int dense_chunks(long count) const {
    return (int)std::max<long>(1, std::min<long>(2048, (count + 255) / 256));
  }

  // dense -> MPS: TT-SVD (Section 2.1, svd-comp equation) of cnt
  // scale-ordered fields W, truncated at (chi_r, tol_r).  W is overwritten.
  // W holds the same fields scale-ordered in the working type.  Under the
  // reduced-precision policies the decomposition runs in the FP64 engine on
  // the FP64 fields (so that ranks are decided as in FP64 arithmetic) and the
  // cores are then converted; objects of the recycled pool go through pool
  // objects of the FP64 engine, others (the obstacle masks, capacity cap)
  // through a fixed FP64 object of that profile.
  void dense_to_mps(const double* dense, T* W, int cnt, const std::vector<int>& objs, int chi_r,
                    double tol_r, const int* cap = nullptr) {
    if (!X) {
      E.tt_svd(W, cnt, objs, chi_r, tol_r);
      return;
    }
    double* W64 = (double*)X->dalloc(8 * N3 * cnt);
    hipLaunchKernelGGL((k_scale_permute<double, double>), dim3(dense_chunks(cnt * N3)), dim3(256),
                       0, st, dense, W64, n, cnt, 1);
    std::vector<int> xo(cnt);
    for (int i = 0; i < cnt; ++i) xo[i] = cap ? X->add_fixed(cap) : X->acquire();
    X->tt_svd(W64, cnt, xo, chi_r, tol_r);
    for (size_t off = 0; off < xo.size(); off += MAXB) {
      const int c = (int)std::min<size_t>(MAXB, xo.size() - off);
      hipLaunchKernelGGL((k_convert_mps<double, T>), dim3(E.chunks(), n, c), dim3(256), 0, st,
                         X->list_idx(xo, off, c), E.list_idx(objs, off, c), n);
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    X->free_alloc(W64);
    for (int o : xo) {
      if (cap)
        X->drop_fixed(o);
      else
        X->release(o);
    }
  }

  // Decomposition error ||m - m~|| / ||m|| of MPS obj against the dense
  // scale-ordered field Wref (synchronises).
  double decomposition_error(int obj, const T* Wref) {
    T* back = (T*)E.dalloc(sizeof(T) * N3);
    T* work = (T*)E.dalloc(sizeof(T) * N3);
    E.to_dense({obj}, back, work);
    // per-block partial sums, then their sums in a fixed order
    const int nb = std::min(256, dense_chunks(N3));
    double* part = (double*)E.dalloc(8 * 2 * nb);
    hipLaunchKernelGGL(k_diff_norm<T>, dim3(nb), dim3(256), 0, st, (const T*)back, Wref, N3,
                       part);
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, st, (const double*)part, nb, sbuf);
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, st, (const double*)(part + nb), nb,
                       sbuf + 1);
    double hnorm[2];
    HIP_OK(hipMemcpyAsync(hnorm, sbuf, 16, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    E.free_alloc(part);
    E.free_alloc(work);
    E.free_alloc(back);
    return hnorm[1] > 0 ? std::sqrt(hnorm[0] / hnorm[1]) : 0.0;
  }

  // capacity profile of the obstacle masks: min(chi_mask_max, 8^k, 8^(n-k)),
  // no cap when chi_mask_max <= 0 (the mask at machine precision)
  int mask_cap(int k) const {
    const int c = dom[0].cfg.chi_mask_max > 0 ? dom[0].cfg.chi_mask_max : (1 << 30);
    return (k == 0 || k == n) ? 1 : std::min(c, Engine<T>::full_bound(n, k));
  }
  int mcp[MAXN + 1];    // product launch capacities of the masks' bonds
  bool any_mask = false;

  // Obstacle mask of domain d as the tensor product of a coarse layout
  // (l sites) and a fine unit geometry (n - l sites), Appendix D: each part
  // is decomposed by TT-SVD at tol_mask (rank cap chi_mask_max, if any) on
  // its own grid in FP64, and the two MPS are chained into one mask object
  // whose capacities are exactly the resulting bonds.
  void tensor_mask(Domain& dm, const MaskParts& mp, std::vector<void*>& staged) {
    const mps_lbm_config& cfg = dm.cfg;
    const int chi_mask = cfg.chi_mask_max > 0 ? cfg.chi_mask_max : (1 << 30);
    const int len[2] = {mp.l, n - mp.l};
    const uint8_t* part[2] = {mp.outer, mp.inner};
    Engine<double> sub[2];
    int obj[2];
    MpsDev<double> hd[2];
    for (int p = 0; p < 2; ++p) {
      const int m = len[p];
      const long M3 = 1L << (3 * m);
      sub[p].al = E.al;
      sub[p].setup(m, std::min(cfg.chi_max, 16), cfg.tol_mask, st, 0, 1);
      uint8_t* du8 = (uint8_t*)E.dalloc(M3);
      staged.push_back(du8);
      HIP_OK(hipMemcpyAsync(du8, part[p], M3, hipMemcpyHostToDevice, st));
      double* dv = (double*)sub[p].dalloc(8 * M3);
      double* Wv = (double*)sub[p].dalloc(8 * M3);
      hipLaunchKernelGGL(k_u8_to_f64, dim3(dense_chunks(M3)), dim3(256), 0, st,
                         (const uint8_t*)du8, dv, M3);
      hipLaunchKernelGGL((k_scale_permute<double, double>), dim3(dense_chunks(M3)), dim3(256), 0,
                         st, (const double*)dv, Wv, m, 1, 1);
      int cap[MAXN + 1];
      for (int k = 0; k <= m; ++k)
        cap[k] = (k == 0 || k == m) ? 1 : std::min(chi_mask, Engine<double>::full_bound(m, k));
      obj[p] = sub[p].add_fixed(cap);
      sub[p].tt_svd(Wv, 1, {obj[p]}, chi_mask, cfg.tol_mask);
      HIP_OK(hipMemcpyAsync(&hd[p], sub[p].D(obj[p]), sizeof(MpsDev<double>),
                            hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      sub[p].free_alloc(Wv);
      sub[p].free_alloc(dv);
    }
    int cap[MAXN + 1];
    for (int k = 0; k <= mp.l; ++k) cap[k] = hd[0].r[k];
    for (int k = 0; k <= n - mp.l; ++k) cap[mp.l + k] = hd[1].r[k];
    if (cap[mp.l] != 1) throw Error(-3, "tensor-product mask: parts are not closed MPS");
    dm.mask = E.add_fixed(cap);
    hipLaunchKernelGGL((k_chain_mps<double, T>), dim3(E.chunks(), n), dim3(256), 0, st,
                       (const MpsDev<double>*)sub[0].D(obj[0]), mp.l,
                       (const MpsDev<double>*)sub[1].D(obj[1]), n - mp.l, E.D(dm.mask));
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    for (int p = 0; p < 2; ++p) sub[p].drop_fixed(obj[p]);
  }

  // Initial state of domain d from dense fields (all synchronous).  The
  // obstacle geometry is the dense solid field, or, when mp is given, the
  // composition of its two parts.
  void init_domain(int d, const double* rho, const double* u, const double* fin,
                   const uint8_t* solid, const MaskParts* mp = nullptr) {
    Domain& dm = dom[d];
    const mps_lbm_config& cfg = dm.cfg;
    // dense staging, released at the end (the masks allocated on the way
    // stay)
    std::vector<void*> staged;
    auto stage = [&](size_t bytes) {
      void* p = E.dalloc(bytes);
      staged.push_back(p);
      return p;
    };
    double* dd = (double*)stage(8 * N3 * Q);
    T* W = (T*)stage(sizeof(T) * N3 * Q);
    uint8_t* dsolid = nullptr;
    if (solid) {
      dsolid = (uint8_t*)stage(N3);
      HIP_OK(hipMemcpy(dsolid, solid, N3, hipMemcpyHostToDevice));
    } else if (mp) {
      const long L3 = 1L << (3 * mp->l), K3 = 1L << (3 * (n - mp->l));
      uint8_t* o = (uint8_t*)stage(L3);
      uint8_t* i = (uint8_t*)stage(K3);
      HIP_OK(hipMemcpy(o, mp->outer, L3, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(i, mp->inner, K3, hipMemcpyHostToDevice));
      dsolid = (uint8_t*)stage(N3);
      hipLaunchKernelGGL(k_compose_solid, dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const uint8_t*)o, (const uint8_t*)i, dsolid, n, n - mp->l);
    }
    if (dsolid) {
      hipLaunchKernelGGL(k_u8_to_f64, dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const uint8_t*)dsolid, dd, N3);
      hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const double*)dd, W, n, 1, 1);
      T* Wkeep = (T*)stage(sizeof(T) * N3);
      hipLaunchKernelGGL(k_copy_plain<T>, dim3(dense_chunks(N3)), dim3(256), 0, st, (const T*)W,
                         Wkeep, N3);
      if (mp) {
        tensor_mask(dm, *mp, staged);
      } else {
        // obstacle mask (objects equation): TT-SVD of the solid field at
        // tol_mask in an MPS of its own capacity, by default uncapped, i.e.
        // at machine precision (the mask bond dimension of Section 5.2)
        int cap[MAXN + 1];
        for (int k = 0; k <= n; ++k) cap[k] = mask_cap(k);
        dm.mask = E.add_fixed(cap);
        const int chi_mask = cfg.chi_mask_max > 0 ? cfg.chi_mask_max : (1 << 30);
        dense_to_mps(dd, W, 1, {dm.mask}, chi_mask, cfg.tol_mask, cap);
      }
      dm.mask_err = decomposition_error(dm.mask, Wkeep);
      E.inner_ones({dm.mask}, sbuf + 2);
      double ones_m = 0.0;
      MpsDev<T> md;
      HIP_OK(hipMemcpyAsync(&ones_m, sbuf + 2, 8, hipMemcpyDeviceToHost, st));
      HIP_OK(hipMemcpyAsync(&md, E.D(dm.mask), sizeof(md), hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      dm.n_fluid = (double)N3 - ones_m;
      if (!any_mask)
        for (int k = 0; k <= n; ++k) mcp[k] = 1;
      any_mask = true;
      for (int k = 0; k <= n; ++k) mcp[k] = std::max(mcp[k], md.r[k]);
    } else {
      dm.n_fluid = (double)N3;
    }
    HIP_OK(hipMemcpyAsync(nfl + d, &dm.n_fluid, 8, hipMemcpyHostToDevice, st));
    // face masks m_B (boundaries equations): the fluid cells of each open
    // face plane, decomposed from that dense field at tol_mask; they enter
    // population sums, so their rank is capped at chi_max
    for (int ax = 0; ax < 3; ++ax) {
      if (!cfg.axis_open[ax]) continue;
      for (int side = 0; side < 2; ++side) {
        int face = 2 * ax + side;
        if (cfg.face_bc[face] == MPS_LBM_BC_NONE) continue;
        hipLaunchKernelGGL(k_face_plane, dim3(dense_chunks(N3)), dim3(256), 0, st,
                           (const uint8_t*)dsolid, dd, n, ax, side == 0 ? 0 : N - 1);
        hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(N3)), dim3(256), 0,
                           st, (const double*)dd, W, n, 1, 1);
        T* Wkeep = (T*)stage(sizeof(T) * N3);
        hipLaunchKernelGGL(k_copy_plain<T>, dim3(dense_chunks(N3)), dim3(256), 0, st,
                           (const T*)W, Wkeep, N3);
        dm.fplane[face] = E.acquire();
        dense_to_mps(dd, W, 1, {dm.fplane[face]}, cfg.chi_max, cfg.tol_mask);
        dm.face_err = std::max(dm.face_err, decomposition_error(dm.fplane[face], Wkeep));
      }
    }
    // initial populations
    if (fin) {
      HIP_OK(hipMemcpy(dd, fin, 8 * N3 * Q, hipMemcpyHostToDevice));
    } else {
      double* drho = (double*)stage(8 * N3);
      double* du = (double*)stage(8 * N3 * 3);
      HIP_OK(hipMemcpy(drho, rho, 8 * N3, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(du, u, 8 * N3 * 3, hipMemcpyHostToDevice));
      hipLaunchKernelGGL(k_feq_dense, dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const double*)drho, (const double*)du, (const uint8_t*)dsolid, dd, N3,
                         (const int*)cvec_dev, (const double*)w_dev, Q);
    }
    hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(Q * N3)), dim3(256), 0,
                       st, (const double*)dd, W, n, Q, 1);
    std::vector<int> objs(Q);
    for (int i = 0; i < Q; ++i) objs[i] = dm.f[i] = E.acquire();
    dense_to_mps(dd, W, Q, objs, cfg.chi_max, cfg.tol);
    HIP_OK(hipStreamSynchronize(st));
    for (void* p : staged) E.free_alloc(p);
  }

  // After every domain is initialised: product workspaces for the masks'
  // bond profile (the obstacle products' second factor).
  void finish_init() {
    if (any_mask) E.reserve_products(mcp);
  }

  // Objects of E copied into fresh objects of X (to FP64) and back.
  std::vector<int> to_island(const std::vector<int>& src) {
    std::vector<int> dst(src.size());
    for (size_t i = 0; i < src.size(); ++i) dst[i] = X->acquire();
    for (size_t off = 0; off < src.size(); off += MAXB) {
      const int cnt = (int)std::min<size_t>(MAXB, src.size() - off);
      hipLaunchKernelGGL((k_convert_mps<T, double>), dim3(E.chunks(), n, cnt), dim3(256), 0, st,
                         E.list_idx(src, off, cnt), X->list_idx(dst, off, cnt), n);
    }
    HIP_OK(hipGetLastError());
    return dst;
  }
  std::vector<int> from_island(const std::vector<int>& src) {
    std::vector<int> dst(src.size());
    for (size_t i = 0; i < src.size(); ++i) dst[i] = E.acquire();
    for (size_t off = 0; off < src.size(); off += MAXB) {
      const int cnt = (int)std::min<size_t>(MAXB, src.size() - off);
      hipLaunchKernelGGL((k_convert_mps<double, T>), dim3(E.chunks(), n, cnt), dim3(256), 0, st,
                         X->list_idx(src, off, cnt), E.list_idx(dst, off, cnt), n);
    }
    HIP_OK(hipGetLastError());
    return dst;
  }

  // Inverse density of every domain (Section 3.2; Appendix B) on engine Q
  // with its unit MPS one_q: Taylor-2 about rho_0, r = (1/rho_0)(1 - e +
  // e (.) e) with e = rho/rho_0 - 1, or Newton-Schulz from 1/rho_0.  The
  // first sums of the chosen form are rounded together with the sums
  // `extra` (appended; their results are returned in *extra_out).
  template <typename U>
  std::vector<int> inverse_density(Engine<U>& Q, int one_q, const std::vector<int>& rho,
                                   const std::vector<std::vector<typename Engine<U>::Term>>& extra,
                                   std::vector<int>* extra_out) {
    typedef typename Engine<U>::Term TermU;
    const mps_lbm_config& c0 = dom[0].cfg;
    auto first = [&](std::vector<std::vector<TermU>> SF) {
      SF.insert(SF.end(), extra.begin(), extra.end());
      std::vector<int> o = Q.sums(SF, rho0);
      if (extra_out) extra_out->assign(o.begin() + D, o.end());
      o.resize(D);
      return o;
    };
    std::vector<int> r(D);
    if (c0.inv_rho_mode == MPS_LBM_INV_TAYLOR2) {
      std::vector<std::vector<TermU>> SE(D);
      for (int d = 0; d < D; ++d) SE[d] = {{Coef{1.0, -1, d}, rho[d]}, {Coef{-1.0, 0, d}, one_q}};
      std::vector<int> e = first(SE);
      std::vector<std::pair<int, int>> pe;
      for (int d = 0; d < D; ++d) pe.push_back({e[d], e[d]});
      std::vector<int> ee = Q.prods(pe);
      std::vector<std::vector<TermU>> SR(D);
      for (int d = 0; d < D; ++d)
        SR[d] = {{Coef{1.0, -1, d}, one_q}, {Coef{-1.0, -1, d}, e[d]}, {Coef{1.0, -1, d}, ee[d]}};
      r = Q.sums(SR, rho0);
      for (int d = 0; d < D; ++d) {
        Q.release(e[d]);
        Q.release(ee[d]);
      }
    } else {
      std::vector<std::vector<TermU>> SY(D);
      for (int d = 0; d < D; ++d)
        SY[d] = {{Coef{2.0, -1, d}, one_q}, {Coef{-1.0, -2, d}, rho[d]}};
      std::vector<int> y = first(SY);
      for (int it = 1; it < c0.inv_rho_iters; ++it) {
        std::vector<std::pair<int, int>> p1;
        for (int d = 0; d < D; ++d) p1.push_back({rho[d], y[d]});
        std::vector<int> ry = Q.prods(p1);
        std::vector<std::vector<TermU>> ST(D);
        for (int d = 0; d < D; ++d) ST[d] = {{Coef{2.0, 0, d}, one_q}, {Coef{-1.0, 0, d}, ry[d]}};
        std::vector<int> t = Q.sums(ST, rho0);
        std::vector<std::pair<int, int>> p2;
        for (int d = 0; d < D; ++d) p2.push_back({y[d], t[d]});
        std::vector<int> y2 = Q.prods(p2);
        for (int d = 0; d < D; ++d) {
          Q.release(ry[d]);
          Q.release(t[d]);
          Q.release(y[d]);
        }
        y = y2;
      }
      r = y;
    }
    return r;
  }

  // ---------------------------------------------------------------- step
  void step_once() {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, E.stats, 0.0, 1L);
    hipLaunchKernelGGL(k_face_time, dim3(1), dim3(((6 * D + 63) / 64) * 64), 0, st,
                       (const FaceProf*)fprof, rho0, fs_off(), cnt_off(), 6 * D);
    E.rs_call = 0;
    E.roundings = 0;
    E.products = 0;
    static const int PI[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    // 1. moments rho, j_a (4 sums per domain)
    std::vector<std::vector<Term>> S(4 * D);
    for (int d = 0; d < D; ++d) {
      for (int i = 0; i < Q; ++i) S[4 * d].push_back({Coef{1.0, 0, d}, dom[d].f[i]});
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < Q; ++i)
          if (lat->c[i][a]) S[4 * d + 1 + a].push_back({Coef{(double)lat->c[i][a], 0, d}, dom[d].f[i]});
    }
    std::vector<int> mom = E.sums(S, rho0);
    std::vector<int> rho(D), j(3 * D);
    std::vector<int> rl(D);
    for (int d = 0; d < D; ++d) {
      rho[d] = mom[4 * d];
      for (int a = 0; a < 3; ++a) j[3 * d + a] = mom[4 * d + 1 + a];
    }
    // 2. rho_0 = <1, rho> / N_fluid
    E.inner_ones(rho, sbuf);
    hipLaunchKernelGGL(k_div_vec, dim3(1), dim3(std::max(64, ((D + 63) / 64) * 64)), 0, st,
                       (const double*)sbuf, (const double*)nfl, rho0, D);
    // 4a. j_eq = j + tau g rho on the forced axes; these sums need only the
    // moments, so they are rounded together with the first sums of step 3
    std::vector<int> jeq(3 * D);
    std::vector<std::vector<Term>> SJ;
    std::vector<int> which;
    for (int d = 0; d < D; ++d)
      for (int a = 0; a < 3; ++a) {
        const double ga = dom[d].cfg.g[a];
        if (ga != 0.0) {
          SJ.push_back({{Coef{1.0, 0, d}, j[3 * d + a]}, {Coef{dom[d].cfg.tau * ga, 0, d}, rho[d]}});
          which.push_back(3 * d + a);
        } else {
          jeq[3 * d + a] = j[3 * d + a];
        }
      }
    // 3. inverse density (every domain of a handle uses the same mode); the
    // j_eq sums need only the moments and are rounded with its first sums,
    // or, with the FP64 island, on their own
    std::vector<int> r(D), jq;
    if (X) {
      X->roundings = 0;
      X->products = 0;
      std::vector<int> rho64 = to_island(rho);
      std::vector<int> r64 = inverse_density(*X, one64, rho64, {}, nullptr);
      r = from_island(r64);
      for (int d = 0; d < D; ++d) {
        X->release(rho64[d]);
        X->release(r64[d]);
      }
      if (!SJ.empty()) jq = E.sums(SJ, rho0);
    } else {
      r = inverse_density(E, one, rho, SJ, &jq);
    }
    for (size_t q = 0; q < which.size(); ++q) {
      E.release(j[which[q]]);
      jeq[which[q]] = jq[q];
    }
    // 4b. u = j_eq (.) r, Pi_ab = j_eq,a (.) u_b
    std::vector<std::pair<int, int>> pu;
    for (int d = 0; d < D; ++d)
      for (int a = 0; a < 3; ++a) pu.push_back({jeq[3 * d + a], r[d]});
    std::vector<int> u = E.prods(pu);  // u[3 d + a]
    std::vector<std::pair<int, int>> pp;
    for (int d = 0; d < D; ++d)
      for (int q = 0; q < 6; ++q) pp.push_back({jeq[3 * d + PI[q][0]], u[3 * d + PI[q][1]]});
    std::vector<int> Pi = E.prods(pp);  // Pi[6 d + q]
    std::vector<std::vector<Term>> SS(D);
    for (int d = 0; d < D; ++d)
      SS[d] = {{Coef{1.0, 0, d}, rho[d]}, {Coef{-1.5, 0, d}, Pi[6 * d]},
               {Coef{-1.5, 0, d}, Pi[6 * d + 1]}, {Coef{-1.5, 0, d}, Pi[6 * d + 2]}};
    std::vector<int> S0 = E.sums(SS, rho0);
    // 5. BGK relaxation
    std::vector<std::vector<Term>> SB(Q * D);
    for (int d = 0; d < D; ++d) {
      const double om = 1.0 / dom[d].cfg.tau;
      for (int i = 0; i < Q; ++i) {
        const double wi = lat->w[i];
        std::vector<Term>& t = SB[Q * d + i];
        t.push_back({Coef{1.0 - om, 0, d}, dom[d].f[i]});
        t.push_back({Coef{om * wi, 0, d}, S0[d]});
        for (int a = 0; a < 3; ++a)
          if (lat->c[i][a]) t.push_back({Coef{3.0 * om * wi * lat->c[i][a], 0, d}, jeq[3 * d + a]});
        for (int q = 0; q < 6; ++q) {
          const int a = PI[q][0], b = PI[q][1];
          const int coef = lat->c[i][a] * lat->c[i][b] * (a == b ? 1 : 2);
          if (coef) t.push_back({Coef{4.5 * om * wi * coef, 0, d}, Pi[6 * d + q]});
        }
      }
    }
    std::vector<int> fpost = E.sums(SB, rho0);  // fpost[Q d + i]
    for (int d = 0; d < D; ++d) {
      for (int i = 0; i < Q; ++i) E.release(dom[d].f[i]);
      E.release(rho[d]);
      E.release(r[d]);
      E.release(S0[d]);
      for (int q = 0; q < 6; ++q) E.release(Pi[6 * d + q]);
      for (int a = 0; a < 3; ++a) E.release(jeq[3 * d + a]);
    }
    // 7a. open-face boundary terms (post-collision f_ihat and u)
    std::vector<std::vector<Term>> bterms(Q * D);
    std::vector<int> btemp;
    {
      struct Face { int d, ax, side, typ, idx; };
      std::vector<Face> faces;
      for (int d = 0; d < D; ++d)
        for (int ax = 0; ax < 3; ++ax) {
          if (!dom[d].cfg.axis_open[ax]) continue;
          for (int side = 0; side < 2; ++side) {
            const int typ = dom[d].cfg.face_bc[2 * ax + side];
            if (typ != MPS_LBM_BC_NONE) faces.push_back({d, ax, side, typ, side == 0 ? 0 : N - 1});
          }
        }
      // u restricted to the pressure faces, rounded; then the uu products
      std::vector<int> us, uax, uid;
      for (const Face& F : faces)
        if (F.typ == MPS_LBM_BC_PRESSURE)
          for (int a = 0; a < 3; ++a) {
            us.push_back(u[3 * F.d + a]);
            uax.push_back(F.ax);
            uid.push_back(F.idx);
          }
      std::vector<int> uB;
      if (!us.empty()) {
        uB = E.slice(us, uax, uid);
        E.round(uB);
      }
      std::vector<std::pair<int, int>> pq;
      for (size_t fp = 0; fp * 3 < uB.size(); ++fp)
        for (int q = 0; q < 6; ++q) pq.push_back({uB[3 * fp + PI[q][0]], uB[3 * fp + PI[q][1]]});
      std::vector<int> uu = pq.empty() ? std::vector<int>() : E.prods(pq);
      for (int o : uB) E.release(o);
      for (int o : uu) btemp.push_back(o);
      // plane slices of the incoming populations
      std::vector<int> src, axs, ids, fent;
      for (size_t q = 0; q < faces.size(); ++q) {
        const Face& F = faces[q];
        const int entering = F.side == 0 ? 1 : -1;
        for (int i = 0; i < Q; ++i)
          if (lat->c[i][F.ax] == entering) {
            src.push_back(fpost[Q * F.d + lat->opp[i]]);
            axs.push_back(F.ax);
            ids.push_back(F.idx);
            fent.push_back((int)q * Q + i);
          }
      }
      std::vector<int> fo = src.empty() ? std::vector<int>() : E.slice(src, axs, ids);
      for (int o : fo) btemp.push_back(o);
      int pface = 0;  // running index of pressure faces (order of uB / uu)
      std::vector<int> pidx(faces.size(), -1);
      for (size_t q = 0; q < faces.size(); ++q)
        if (faces[q].typ == MPS_LBM_BC_PRESSURE) pidx[q] = pface++;
      for (size_t t = 0; t < fent.size(); ++t) {
        const int q = fent[t] / Q, i = fent[t] % Q;
        const Face& F = faces[q];
        const Domain& dm = dom[F.d];
        const int face = 2 * F.ax + F.side;
        const int fp = dm.fplane[face];
        const double c[3] = {(double)lat->c[i][0], (double)lat->c[i][1], (double)lat->c[i][2]};
        std::vector<Term>& bt = bterms[Q * F.d + i];
        if (F.typ == MPS_LBM_BC_VELOCITY) {
          const double* ub = dm.cfg.face_val[face];
          const double cu = c[0] * ub[0] + c[1] * ub[1] + c[2] * ub[2];
          bt.push_back({Coef{1.0, 0, F.d}, fo[t]});
          // u_b(t) = u_b phi(t): phi is the face's per-step scale
          bt.push_back({Coef{6.0 * lat->w[i] * cu, cu == 0.0 ? 0 : 1, F.d, fs_off() + 6 * F.d + face},
                        fp});
        } else {
          const double rb = dm.cfg.face_val[face][0];
          const double kk = 2.0 * lat->w[i] * rb;
          bt.push_back({Coef{-1.0, 0, F.d}, fo[t]});
          bt.push_back({Coef{kk, 0, F.d}, fp});
          for (int p = 0; p < 6; ++p) {
            const int a = PI[p][0], b = PI[p][1];
            const double coef = (a == b) ? kk * (4.5 * c[a] * c[a] - 1.5) : kk * 9.0 * c[a] * c[b];
            if (coef != 0.0) bt.push_back({Coef{coef, 0, F.d}, uu[6 * pidx[q] + p]});
          }
        }
      }
    }
    // 6. streaming (f_0 does not move)
    std::vector<int> src;
    std::vector<const int*> cv, ao;
    for (int d = 0; d < D; ++d)
      for (int i = 1; i < Q; ++i) {
        src.push_back(fpost[Q * d + i]);
        cv.push_back(lat->c[i]);
        ao.push_back(dom[d].cfg.axis_open);
      }
    std::vector<int> fs1 = E.stream(src, cv, ao);
    std::vector<int> fs(Q * D);
    for (int d = 0; d < D; ++d) {
      fs[Q * d] = fpost[Q * d];
      for (int i = 1; i < Q; ++i) fs[Q * d + i] = fs1[(Q - 1) * d + i - 1];
    }
    // 7b. add the boundary terms
    {
      std::vector<std::vector<Term>> SBC;
      std::vector<int> which;
      for (int q = 0; q < Q * D; ++q) {
        if (bterms[q].empty()) continue;
        std::vector<Term> t{{Coef{1.0, 0, q / Q}, fs[q]}};
        t.insert(t.end(), bterms[q].begin(), bterms[q].end());
        SBC.push_back(t);
        which.push_back(q);
      }
      if (!SBC.empty()) {
        std::vector<int> o = E.sums(SBC, rho0);
        for (size_t q = 0; q < which.size(); ++q) {
          E.release(fs[which[q]]);
          fs[which[q]] = o[q];
        }
      }
    }
    for (int o : btemp) E.release(o);
    for (int d = 0; d < D; ++d) {
      for (int i = 1; i < Q; ++i) E.release(fpost[Q * d + i]);
      for (int a = 0; a < 3; ++a) E.release(u[3 * d + a]);
    }
    // 8. obstacle bounce-back
    {
      std::vector<int> dd;
      for (int d = 0; d < D; ++d)
        if (dom[d].mask >= 0) dd.push_back(d);
      if (!dd.empty()) {
        std::vector<std::pair<int, int>> pm;
        for (int d : dd)
          for (int i = 1; i < Q; ++i) pm.push_back({fs[Q * d + i], dom[d].mask});
        // candidate = the population (its bonds are those the result keeps)
        std::vector<int> g1 = E.prods(pm, mcp);  // g1[18 k + i - 1]
        std::vector<int> hs;
        std::vector<const int*> hc, ha;
        for (size_t k = 0; k < dd.size(); ++k)
          for (int i = 1; i < Q; ++i) {
            hs.push_back(g1[(Q - 1) * k + lat->opp[i] - 1]);
            hc.push_back(lat->c[i]);
            ha.push_back(dom[dd[k]].cfg.axis_open);
          }
        // the sum f_i - g1_i + h_i is a pairwise tree: its first pair
        // (f_i - g1_i) is rounded together with the first shift level of h
        std::vector<PairSum> pre;
        for (size_t k = 0; k < dd.size(); ++k) {
          const int d = dd[k];
          for (int i = 1; i < Q; ++i)
            pre.push_back({Coef{1.0, 0, d}, fs[Q * d + i], Coef{-1.0, 0, d}, g1[(Q - 1) * k + i - 1]});
        }
        std::vector<int> fg;
        std::vector<int> h = E.stream(hs, hc, ha, rho0, pre, &fg);
        std::vector<std::vector<Term>> SO;
        for (size_t k = 0; k < dd.size(); ++k) {
          const int d = dd[k];
          for (int i = 1; i < Q; ++i)
            SO.push_back({{Coef{1.0, 0, d}, fg[(Q - 1) * k + i - 1]},
                          {Coef{1.0, 0, d}, h[(Q - 1) * k + i - 1]}});
        }
        std::vector<int> o = E.sums(SO, rho0);
        for (size_t k = 0; k < dd.size(); ++k) {
          const int d = dd[k];
          for (int i = 1; i < Q; ++i) {
            E.release(fs[Q * d + i]);
            E.release(g1[(Q - 1) * k + i - 1]);
            E.release(h[(Q - 1) * k + i - 1]);
            E.release(fg[(Q - 1) * k + i - 1]);
            fs[Q * d + i] = o[(Q - 1) * k + i - 1];
          }
        }
      }
    }
    for (int d = 0; d < D; ++d)
      for (int i = 0; i < Q; ++i) dom[d].f[i] = fs[Q * d + i];
    last_roundings = E.roundings + (X ? X->roundings : 0);
    last_products = E.products + (X ? X->products : 0);
  }

  void step(int nsteps) override {
    for (int s = 0; s < nsteps; ++s) {
      if (gexec) {
        HIP_OK(hipGraphLaunch(gexec, st));
      } else {
        step_once();
      }
      ++steps;
      E.step_count = steps;
    }
    HIP_OK(hipGetLastError());
  }

  // Graph mode: one eager step brings the MPS pool to its peak size, then
  // the next step is recorded into a HIP graph followed by copies that move
  // the new populations back into the slots the step read from, so that the
  // recorded launches (fixed pointers) are valid for every later step.
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  // capture in three pieces, so that a handle of several groups can record
  // all of them into one graph: prepare (one eager step, pin the slots the
  // populations live in), record (inside an open capture: the step and the
  // copies back into those slots), finish (unpin)
  std::vector<std::array<int, 19>> home;
  int saved_tkind = 0;
  void capture_prepare() override {
    step(1);
    HIP_OK(hipStreamSynchronize(st));
    home.assign(D, std::array<int, 19>{});
    for (int d = 0; d < D; ++d)
      for (int i = 0; i < Q; ++i) home[d][i] = dom[d].f[i];
    // the step releases its input populations half-way; during recording
    // their slots are pinned so that no result or temporary lands in them
    // and the final copies cannot overwrite a source still to be copied
    E.pinned.assign(E.pool.size(), 0);
    for (int d = 0; d < D; ++d)
      for (int i = 0; i < Q; ++i) E.pinned[home[d][i]] = 1;
    saved_tkind = E.tkind;
    E.tkind = 0;
  }
  void capture_record() override {
    step_once();
    for (int d = 0; d < D; ++d)
      for (int i = 0; i < Q; ++i) {
        const int now = dom[d].f[i], h = home[d][i];
        const long tot = E.pool[now].total;
        hipLaunchKernelGGL(k_copy_plain<T>, dim3(dense_chunks(tot)), dim3(256), 0, st,
                           (const T*)E.pool[now].data, E.pool[h].data, tot);
        hipLaunchKernelGGL(k_copy_ranks<T>, dim3(1), dim3(64), 0, st, E.D(h),
                           (const MpsDev<T>*)E.D(now));
        E.release(now);
        dom[d].f[i] = h;
      }
  }
  void capture_finish() override {
    E.tkind = saved_tkind;
    E.pinned.clear();
  }
  void count_step() override {
    ++steps;
    E.step_count = steps;
  }

  void capture() override {
    if (gexec) return;
    if (!st) throw Error(-1, "graph capture needs a non-default stream");
    capture_prepare();
    HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      capture_record();
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(st, &g);
      if (g) (void)hipGraphDestroy(g);
      capture_finish();
      throw;
    }
    HIP_OK(hipStreamEndCapture(st, &graph));
    capture_finish();
    HIP_OK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }

  ~SimT() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
  }

  void to_dense(int d, int what, double* out) override {
    std::vector<void*> tmp;
    auto tdalloc = [&](size_t b) {
      void* q = E.dalloc(b);
      tmp.push_back(q);
      return q;
    };
    size_t bytes = sizeof(T) * N3 * Q;
    T* buf = (T*)tdalloc(bytes);
    T* work = (T*)tdalloc(bytes);
    std::vector<int> objs(dom[d].f, dom[d].f + Q);
    E.to_dense(objs, buf, work);
    long nout = (what == MPS_LBM_POPS) ? Q * N3 : (what == MPS_LBM_RHO ? N3 : 3 * N3);
    double* res = (double*)tdalloc(8 * nout);
    if (what == MPS_LBM_POPS) {
      hipLaunchKernelGGL((k_scale_permute<T, double>), dim3(dense_chunks(Q * N3)), dim3(256), 0,
                         st, (const T*)buf, res, n, Q, 0);
    } else {
      double* mom = (double*)tdalloc(8 * nout);
      hipLaunchKernelGGL(k_moments_dense<T>, dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const T*)buf, mom, N3, what, (const int*)cvec_dev, Q);
      hipLaunchKernelGGL((k_scale_permute<double, double>), dim3(dense_chunks(nout)), dim3(256), 0,
                         st, (const double*)mom, res, n, (int)(nout / N3), 0);
    }
    HIP_OK(hipMemcpyAsync(out, res, 8 * nout, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (void* q : tmp) E.free_alloc(q);
  }

  // Kinetic energy (Section 4.2): (1 / (2 N^3)) sum_x |u_x|^2 with
  // u = j / rho of the dense contraction of the state (0 where rho = 0).
  double kinetic_energy(int d) override {
    std::vector<void*> tmp;
    auto tdalloc = [&](size_t b) {
      void* q = E.dalloc(b);
      tmp.push_back(q);
      return q;
    };
    T* buf = (T*)tdalloc(sizeof(T) * N3 * Q);
    T* work = (T*)tdalloc(sizeof(T) * N3 * Q);
    const int nb = std::min(1024, dense_chunks(N3));
    double* acc = (double*)tdalloc(8 * (nb + 1));
    std::vector<int> objs(dom[d].f, dom[d].f + Q);
    E.to_dense(objs, buf, work);
    // per-block partial sums, then their sum in a fixed order
    hipLaunchKernelGGL(k_u2_sum<T>, dim3(nb), dim3(256), 0, st, (const T*)buf, N3,
                       (const int*)cvec_dev, Q, acc + 1);
    hipLaunchKernelGGL(k_sum_in_order, dim3(1), dim3(64), 0, st, (const double*)(acc + 1), nb, acc);
    double s = 0.0;
    HIP_OK(hipMemcpyAsync(&s, acc, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (void* q : tmp) E.free_alloc(q);
    return 0.5 * s / (double)N3;
  }

  // Numerical health after a synchronisation: a non-finite value seen in
  // the state is sticky (every later data read and step reports it); new
  // Jacobi sweep-limit hits are reported once.
  int seen_fail = 0;
  bool nonfinite_seen = false;
  int numeric_status() override {
    int ist[2] = {0, 0}, isx[2] = {0, 0};
    HIP_OK(hipMemcpyAsync(ist, E.istats, 8, hipMemcpyDeviceToHost, st));
    if (X) HIP_OK(hipMemcpyAsync(isx, X->istats, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    ist[0] += isx[0];
    ist[1] += isx[1];
    if (ist[1] > 0) nonfinite_seen = true;
    if (nonfinite_seen) return fail(MPS_LBM_ENUMERIC, "a non-finite value appeared in the state");
    if (ist[0] > seen_fail) {
      const int k = ist[0] - seen_fail;
      seen_fail = ist[0];
      return fail(MPS_LBM_ENUMERIC, std::to_string(k) +
                                        " singular value decompositions hit the sweep limit");
    }
    return MPS_LBM_OK;
  }
  bool fatal_seen() const override { return nonfinite_seen; }
  void raise_flags(int nonfinite, int sweep_limit) override {
    hipLaunchKernelGGL(k_add_flags, dim3(1), dim3(64), 0, st, E.istats, sweep_limit, nonfinite);
    HIP_OK(hipGetLastError());
  }

  void rank_model(float* w, int load) override {
    if (!E.mlp_on) throw Error(MPS_LBM_EUNSUPPORTED, "the learned rank predictor is off");
    const size_t b = sizeof(float) * MLP_NPARAM;
    if (load) {
      if (gexec) throw Error(MPS_LBM_EUNSUPPORTED, "loading weights after graph capture");
      HIP_OK(hipMemcpyAsync(E.mlp.p, w, b, hipMemcpyHostToDevice, st));
      HIP_OK(hipStreamSynchronize(st));
      E.mlp_trained = true;
    } else {
      HIP_OK(hipMemcpyAsync(w, E.mlp.p, b, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
    }
  }

  int get_mps(int d, int which, double* out, size_t out_len, int* bonds) override {
    if (which >= Q && which != MPS_LBM_MPS_MASK)
      return fail(MPS_LBM_EINVAL, "population index beyond the lattice's velocities");
    int idx = which < Q ? dom[d].f[which] : dom[d].mask;
    if (idx < 0) return fail(MPS_LBM_EINVAL, "no obstacle mask in this simulation");
    MpsDev<T> md;
    HIP_OK(hipMemcpyAsync(&md, E.D(idx), sizeof(md), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    size_t need = 0;
    for (int k = 0; k <= n; ++k) bonds[k] = md.r[k];
    for (int k = 0; k < n; ++k) need += (size_t)md.r[k] * PHYS * md.r[k + 1];
    if (!out) return MPS_LBM_OK;
    if (out_len < need) return fail(MPS_LBM_EINVAL, "out_len too small");
    std::vector<T> tmp(need);
    size_t pos = 0;
    for (int k = 0; k < n; ++k) {
      size_t cnt = (size_t)md.r[k] * PHYS * md.r[k + 1];
      HIP_OK(hipMemcpyAsync(tmp.data() + pos, md.data + md.off[k], sizeof(T) * cnt,
                            hipMemcpyDeviceToHost, st));
      pos += cnt;
    }
    HIP_OK(hipStreamSynchronize(st));
    for (size_t e = 0; e < need; ++e) out[e] = (double)tmp[e];
    return MPS_LBM_OK;
  }

  void set_timing(int kind) override { E.timing(kind); }

  int autotune() override {
    if (gexec) throw Error(MPS_LBM_EUNSUPPORTED, "autotuning after graph capture");
    if (steps == 0) throw Error(MPS_LBM_EINVAL, "no step taken yet");
    return E.autotune();
  }

  float train_predictor(int epochs, float lr) override {
    if (!E.mlp_on) throw Error(MPS_LBM_EUNSUPPORTED, "the learned rank predictor is off");
    if (gexec) throw Error(MPS_LBM_EUNSUPPORTED, "training after graph capture");
    return E.train_mlp(epochs, lr);
  }

  void predictor_info(mps_lbm_predictor_info* o) override {
    memset(o, 0, sizeof(*o));
    if (!E.mlp_on) return;
    int nsmp = 0;
    double err[3] = {0, 0, 0};
    HIP_OK(hipMemcpyAsync(&nsmp, E.smp_n, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(err, E.mlp_err, 24, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    o->samples = nsmp;
    o->trained = E.mlp_trained ? 1 : 0;
    o->first_loss = E.first_loss;
    o->last_loss = E.last_loss;
    o->predictions = (long long)err[2];
    o->mlp_abs_err = err[2] > 0 ? err[0] / err[2] : 0.0;
    o->prev_abs_err = err[2] > 0 ? err[1] / err[2] : 0.0;
  }

  void kstats(mps_lbm_kstats* o) override {
    E.flush_events();
    double fl = 0.0;
    if (E.kflops) HIP_OK(hipMemcpy(&fl, E.kflops, 8, hipMemcpyDeviceToHost));
    o->launches = E.tlaunches;
    o->total_ms = E.tms;
    o->flops = fl;
  }

  void set_face_profile(int d, int face, const double* coef, double dt) override {
    const mps_lbm_config& cfg = dom[d].cfg;
    if (cfg.face_bc[face] != MPS_LBM_BC_VELOCITY)
      throw Error(-1, "a time profile applies to a velocity face");
    FaceProf p{};
    for (int c = 0; c < 6; ++c) p.c[c] = coef ? coef[c] : 0.0;
    p.dt = dt;
    p.on = coef ? 1 : 0;
    hprof[6 * d + face] = p;
    HIP_OK(hipMemcpyAsync(fprof + 6 * d + face, &hprof[6 * d + face], sizeof(FaceProf),
                          hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
  }

  // Region of interest of the pressure metric (Section 4.2): the fluid
  // cells of the box lo <= x < hi as an MPS, decomposed from that dense
  // indicator like the obstacle mask (tol_mask, no cap, FP64 ranks); the
  // solid cells are read back from the obstacle mask.
  void set_region(int d, const int* lo, const int* hi, double rho_ref) override {
    for (int a = 0; a < 3; ++a)
      if (lo[a] < 0 || hi[a] > N || lo[a] >= hi[a]) throw Error(-1, "region box outside the grid");
    Domain& dm = dom[d];
    const mps_lbm_config& cfg = dm.cfg;
    std::vector<void*> staged;
    auto stage = [&](size_t bytes) {
      void* p = E.dalloc(bytes);
      staged.push_back(p);
      return p;
    };
    try {
      T* ms = nullptr;
      if (dm.mask >= 0) {
        ms = (T*)stage(sizeof(T) * N3);
        T* work = (T*)stage(sizeof(T) * N3);
        E.to_dense({dm.mask}, ms, work);
      }
      double* dd = (double*)stage(8 * N3);
      T* W = (T*)stage(sizeof(T) * N3);
      T* Wkeep = (T*)stage(sizeof(T) * N3);
      double* cnt = (double*)stage(8);
      hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, cnt, 0.0, 1L);
      hipLaunchKernelGGL(k_box_fluid<T>, dim3(std::min(1024, dense_chunks(N3))), dim3(256), 0, st,
                         (const T*)ms, dd, n, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], cnt);
      double cells = 0.0;
      HIP_OK(hipMemcpyAsync(&cells, cnt, 8, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      if (!(cells > 0.0)) throw Error(-1, "the region holds no fluid cell");
      hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const double*)dd, W, n, 1, 1);
      hipLaunchKernelGGL(k_copy_plain<T>, dim3(dense_chunks(N3)), dim3(256), 0, st, (const T*)W,
                         Wkeep, N3);
      int cap[MAXN + 1];
      for (int k = 0; k <= n; ++k) cap[k] = mask_cap(k);
      const int obj = E.add_fixed(cap);
      try {
        const int chi_mask = cfg.chi_mask_max > 0 ? cfg.chi_mask_max : (1 << 30);
        dense_to_mps(dd, W, 1, {obj}, chi_mask, cfg.tol_mask, cap);
        dm.region_err = decomposition_error(obj, Wkeep);
      } catch (...) {
        E.drop_fixed(obj);
        throw;
      }
      if (dm.region >= 0) E.drop_fixed(dm.region);
      dm.region = obj;
      dm.region_cells = cells;
      dm.region_rho = rho_ref;
    } catch (...) {
      (void)hipStreamSynchronize(st);
      for (void* p : staged) E.free_alloc(p);
      throw;
    }
    HIP_OK(hipStreamSynchronize(st));
    for (void* p : staged) E.free_alloc(p);
  }

  void observables(int d, mps_lbm_obs* o) override {
    memset(o, 0, sizeof(*o));
    const Domain& dm = dom[d];
    std::vector<int> objs(dm.f, dm.f + Q);
    E.inner_ones(objs, sbuf);
    double s[19];
    double stat[2] = {0, 0};
    int ist[7] = {0, 0, 0, 0, 0, 0, 0};
    HIP_OK(hipMemcpyAsync(s, sbuf, 8 * Q, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(stat, E.stats, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ist, E.istats, 28, hipMemcpyDeviceToHost, st));
    double r0 = 0.0;
    HIP_OK(hipMemcpyAsync(&r0, rho0 + d, 8, hipMemcpyDeviceToHost, st));
    std::vector<MpsDev<T>> descs(Q);
    for (int i = 0; i < Q; ++i)
      HIP_OK(hipMemcpyAsync(&descs[i], E.D(dm.f[i]), sizeof(MpsDev<T>), hipMemcpyDeviceToHost, st));
    MpsDev<T> md;
    if (dm.mask >= 0) HIP_OK(hipMemcpyAsync(&md, E.D(dm.mask), sizeof(md), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    o->step = steps;
    for (int i = 0; i < Q; ++i) {
      o->mass += s[i];
      for (int a = 0; a < 3; ++a) o->momentum[a] += lat->c[i][a] * s[i];
    }
    o->rho0 = r0;
    o->n_fluid = dm.n_fluid;
    double nv = 0.0;
    int mb = 1;
    for (int i = 0; i < Q; ++i) {
      for (int k = 1; k < n; ++k) {
        o->bonds[i][k - 1] = descs[i].r[k];
        mb = std::max(mb, descs[i].r[k]);
      }
      for (int k = 0; k < n; ++k) nv += (double)descs[i].r[k] * PHYS * descs[i].r[k + 1];
    }
    o->max_bond = mb;
    o->nvps = nv;
    o->compression = nv > 0 ? (double)Q * (double)N3 / nv : 0.0;
    o->max_discarded = stat[0];
    int mk = 1;
    if (dm.mask >= 0)
      for (int k = 1; k < n; ++k) mk = std::max(mk, md.r[k]);
    o->mask_bond = dm.mask >= 0 ? mk : 0;
    o->mask_trunc_err = dm.mask_err;
    o->face_trunc_err = dm.face_err;
    o->roundings = last_roundings;
    o->products = last_products;
    o->svd_failures = ist[0];
    o->nonfinite = ist[1];
    o->jacobi_sweeps = ist[3] > 0 ? (double)ist[2] / ist[3] : 0.0;
    o->jacobi_sweeps_wide = ist[5] > 0 ? (double)ist[4] / ist[5] : 0.0;
    o->jacobi_cols_wide = ist[5] > 0 ? (double)ist[6] / ist[5] : 0.0;
    o->lds_bytes = E.lds_elems * 8;
    if (E.rs_pred) {
      int t[2] = {0, 0};
      HIP_OK(hipMemcpy(t, E.rw.tries, 8, hipMemcpyDeviceToHost));
      o->rs_attempted = t[0];
      o->rs_accepted = t[1];
    }
    if (dm.region >= 0) {
      // Delta p / p_0 = <m_D, rho> / (rho_ref |D|) - 1 with
      // <m_D, rho> = sum_i <m_D, f_i> (Section 4.2)
      double ip = 0.0;
      for (int i = 0; i < Q; ++i) {
        E.inner_pair(dm.f[i], dm.region, sbuf);
        double v = 0.0;
        HIP_OK(hipMemcpy(&v, sbuf, 8, hipMemcpyDeviceToHost));
        ip += v;
      }
      o->dp_p0 = ip / (dm.region_rho * dm.region_cells) - 1.0;
      o->region_cells = dm.region_cells;
      o->region_trunc_err = dm.region_err;
    }
  }
};

// Domains of different shapes or policies in one handle: each group of
// domains that share n, the velocity set, chi_max, chi_mask_max, precision,
// tol, sweeps, the inverse-density mode and the rank-predictor settings is
// one batched SimT with a stream of its own (default priority).  A step
// forks from the handle's stream to the group streams and joins back
// through events, so that the groups' launches (most of them latency-bound
// and far from filling the chip) overlap; the graph mode records the same
// fork and join, one graph with a branch per group.
struct MultiSim : Sim {
  std::vector<std::pair<int, int>> where;  // domain -> (group, index in it)
  hipStream_t st = nullptr;                // the handle's stream
  std::vector<hipStream_t> gs;             // one per group
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<std::unique_ptr<Sim>> g;

  void make_streams(int ngroups) {
    HIP_OK(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
    for (int i = 0; i < ngroups; ++i) {
      hipStream_t s = nullptr;
      HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      gs.push_back(s);
      hipEvent_t e = nullptr;
      HIP_OK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      join_ev.push_back(e);
    }
  }
  ~MultiSim() {
    (void)hipStreamSynchronize(st);
    for (hipStream_t s : gs) (void)hipStreamSynchronize(s);
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    g.clear();  // the groups free their memory on their streams
    for (hipEvent_t e : join_ev) (void)hipEventDestroy(e);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    for (hipStream_t s : gs) (void)hipStreamDestroy(s);
  }
  Sim& of(int d) const { return *g[where[d].first]; }
  int loc(int d) const { return where[d].second; }
  // work already on the handle's stream precedes a group call
  Sim& synced(int d) const {
    HIP_OK(hipStreamSynchronize(st));
    return of(d);
  }
  void fork() {
    HIP_OK(hipEventRecord(fork_ev, st));
    for (hipStream_t s : gs) HIP_OK(hipStreamWaitEvent(s, fork_ev, 0));
  }
  void join() {
    for (size_t i = 0; i < gs.size(); ++i) {
      HIP_OK(hipEventRecord(join_ev[i], gs[i]));
      HIP_OK(hipStreamWaitEvent(st, join_ev[i], 0));
    }
  }

  int domains() const override { return (int)where.size(); }
  void step(int nsteps) override {
    for (int s = 0; s < nsteps; ++s) {
      if (gexec) {
        HIP_OK(hipGraphLaunch(gexec, st));
        for (auto& x : g) x->count_step();
      } else {
        fork();
        for (auto& x : g) x->step(1);
        join();
      }
    }
    HIP_OK(hipGetLastError());
  }
  void to_dense(int d, int what, double* out) override {
    synced(d).to_dense(loc(d), what, out);
  }
  void observables(int d, mps_lbm_obs* o) override { synced(d).observables(loc(d), o); }
  void set_timing(int kind) override {
    for (auto& x : g) x->set_timing(kind);
  }
  void kstats(mps_lbm_kstats* o) override {
    mps_lbm_kstats sum{0, 0.0, 0.0};
    for (auto& x : g) {
      mps_lbm_kstats k{0, 0.0, 0.0};
      x->kstats(&k);
      sum.launches += k.launches;
      sum.total_ms += k.total_ms;
      sum.flops += k.flops;
    }
    *o = sum;
  }
  int get_mps(int d, int which, double* out, size_t out_len, int* bonds) override {
    return synced(d).get_mps(loc(d), which, out, out_len, bonds);
  }
  long cells(int d) const override { return of(d).cells(loc(d)); }
  int velocities(int d) const override { return of(d).velocities(loc(d)); }
  double kinetic_energy(int d) override { return synced(d).kinetic_energy(loc(d)); }
  void capture() override {
    if (gexec) return;
    if (!st) throw Error(-1, "graph capture needs a non-default stream");
    HIP_OK(hipStreamSynchronize(st));
    for (auto& x : g) x->capture_prepare();
    HIP_OK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    try {
      fork();
      for (auto& x : g) x->capture_record();
      join();
    } catch (...) {
      hipGraph_t gg = nullptr;
      (void)hipStreamEndCapture(st, &gg);
      if (gg) (void)hipGraphDestroy(gg);
      for (auto& x : g) x->capture_finish();
      throw;
    }
    HIP_OK(hipStreamEndCapture(st, &graph));
    for (auto& x : g) x->capture_finish();
    HIP_OK(hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0));
  }
  // the rank predictor and the numerical-failure hook address the first group
  float train_predictor(int epochs, float lr) override {
    HIP_OK(hipStreamSynchronize(st));
    return g[0]->train_predictor(epochs, lr);
  }
  int autotune() override {
    HIP_OK(hipStreamSynchronize(st));
    int n = 0;
    for (auto& x : g) n += x->autotune();
    return n;
  }
  void predictor_info(mps_lbm_predictor_info* o) override { synced(0).predictor_info(o); }
  int numeric_status() override {
    HIP_OK(hipStreamSynchronize(st));
    for (auto& x : g) {
      const int r = x->numeric_status();
      if (r) return r;
    }
    return MPS_LBM_OK;
  }
  bool fatal_seen() const override {
    for (auto& x : g)
      if (x->fatal_seen()) return true;
    return false;
  }
  void raise_flags(int nonfinite, int sweep_limit) override {
    synced(0).raise_flags(nonfinite, sweep_limit);
  }
  void rank_model(float* w, int load) override { synced(0).rank_model(w, load); }
  void set_face_profile(int d, int face, const double* coef, double dt) override {
    synced(d).set_face_profile(loc(d), face, coef, dt);
  }
  void set_region(int d, const int* lo, const int* hi, double rho_ref) override {
    synced(d).set_region(loc(d), lo, hi, rho_ref);
  }
};

// the fields that domains advanced by one batched engine must share
static bool same_group(const mps_lbm_config& a, const mps_lbm_config& b) {
  return a.n == b.n && a.lattice == b.lattice && a.chi_max == b.chi_max &&
         a.chi_mask_max == b.chi_mask_max && a.precision == b.precision && a.tol == b.tol &&
         a.sweeps == b.sweeps && a.inv_rho_mode == b.inv_rho_mode &&
         a.inv_rho_iters == b.inv_rho_iters && a.rank_predictor == b.rank_predictor &&
         a.rank_oversample == b.rank_oversample;
}

}  // namespace

struct mps_lbm {
  std::unique_ptr<Sim> sim;
};

// process-wide allocator, read when a handle is created
static Allocator g_alloc;

// Scratch of mps_lbm_mlp_gradient_device: the activations and deltas of the
// predictor network for one batch of at most MLP_SCRATCH_BATCH samples
// (nine B x 128 layers and two B-vectors, 4.7 MB).  Every GPU the library
// runs on holds its own copy until the process ends; its address on a
// device comes from hipGetSymbolAddress, once per device.
constexpr int MLP_SCRATCH_BATCH = 1024;
constexpr long MLP_SCRATCH_FLOATS = (9L * MLP_H + 2) * MLP_SCRATCH_BATCH;
static __device__ __align__(256) float scratch[MLP_SCRATCH_FLOATS];

constexpr int SCRATCH_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[SCRATCH_DEVICES];

// device address of `scratch` on the current device
static float* scratch_on_current_device() {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= SCRATCH_DEVICES)
    throw Error(MPS_LBM_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(MPS_LBM_EHIP, "no device address for the scratch array");
    g_scratch_ptr[dev] = (float*)p;
  }
  return g_scratch_ptr[dev];
}

// Runs an entry point body; no C++ exception leaves it.
template <typename F>
static int guarded(F&& body) {
  try {
    return body();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(MPS_LBM_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  } catch (...) {
    return fail(MPS_LBM_EHIP, "unknown exception");
  }
}

extern "C" {

void mps_lbm_default_config(mps_lbm_config* c) {
  if (!c) return;
  memset(c, 0, sizeof(*c));
  c->n = 4;
  c->lattice = MPS_LBM_D3Q19;
  c->chi_max = 16;
  c->chi_mask_max = 0;
  c->tol = 1e-10;
  c->tol_mask = 1e-12;
  c->tau = 0.8;
  c->inv_rho_mode = MPS_LBM_INV_TAYLOR2;
  c->inv_rho_iters = 2;
  c->precision = MPS_LBM_FP64;
  c->sweeps = 2;
  c->seed = 2512;
  c->rank_predictor = 0;
  c->rank_oversample = 16;
}

int mps_lbm_set_allocator(void* (*alloc)(size_t, void*, void*), void (*free_)(void*, void*, void*),
                          void* ctx) {
  if ((alloc == nullptr) != (free_ == nullptr))
    return fail(MPS_LBM_EINVAL, "alloc and free must both be given or both be NULL");
  g_alloc.alloc = alloc;
  g_alloc.free_ = free_;
  g_alloc.ctx = alloc ? ctx : nullptr;
  return MPS_LBM_OK;
}

static int validate(const mps_lbm_config* c) {
  if (!c) return fail(MPS_LBM_EINVAL, "config is NULL");
  if (c->n < 2 || c->n > MPS_LBM_MAX_SITES) return fail(MPS_LBM_EINVAL, "n out of range");
  if (c->lattice != MPS_LBM_D3Q19 && c->lattice != MPS_LBM_D3Q15)
    return fail(MPS_LBM_EINVAL, "unknown lattice");
  if (c->chi_max < 1) return fail(MPS_LBM_EINVAL, "chi_max < 1");
  if (c->chi_max > 512) return fail(MPS_LBM_EUNSUPPORTED, "chi_max > 512");
  if (!(c->tau > 0.5)) return fail(MPS_LBM_EINVAL, "tau must exceed 1/2");
  if (!(c->tol >= 0.0) || !(c->tol_mask >= 0.0)) return fail(MPS_LBM_EINVAL, "negative tol");
  if (c->inv_rho_mode != MPS_LBM_INV_TAYLOR2 && c->inv_rho_mode != MPS_LBM_INV_NEWTON)
    return fail(MPS_LBM_EINVAL, "unknown inverse-density mode");
  if (c->inv_rho_mode == MPS_LBM_INV_NEWTON && c->inv_rho_iters < 1)
    return fail(MPS_LBM_EINVAL, "inv_rho_iters < 1");
  if (c->precision != MPS_LBM_FP64 && c->precision != MPS_LBM_FP32 &&
      c->precision != MPS_LBM_BF16 && c->precision != MPS_LBM_BF16X3)
    return fail(MPS_LBM_EINVAL, "unknown precision");
  if (c->sweeps < 1) return fail(MPS_LBM_EINVAL, "sweeps < 1");
  if (c->rank_predictor < 0 || c->rank_predictor > 2)
    return fail(MPS_LBM_EINVAL, "rank_predictor must be 0, 1 or 2");
  if (c->rank_predictor && c->rank_oversample < 1)
    return fail(MPS_LBM_EINVAL, "rank_oversample < 1");
  if (c->rank_predictor && c->precision == MPS_LBM_FP64)
    return fail(MPS_LBM_EUNSUPPORTED, "the rank predictor runs with the FP32 and BF16 policies");
  for (int a = 0; a < 3; ++a) {
    if (c->axis_open[a] != 0 && c->axis_open[a] != 1) return fail(MPS_LBM_EINVAL, "axis_open");
    for (int s = 0; s < 2; ++s) {
      int t = c->face_bc[2 * a + s];
      if (t < 0 || t > 2) return fail(MPS_LBM_EINVAL, "unknown face bc");
      if (t != 0 && !c->axis_open[a]) return fail(MPS_LBM_EINVAL, "bc on a periodic axis");
      if (t == MPS_LBM_BC_PRESSURE && !(c->face_val[2 * a + s][0] > 0.0))
        return fail(MPS_LBM_EINVAL, "pressure face needs rho_b > 0");
    }
  }
  return MPS_LBM_OK;
}

// One batched engine for the domains idx of cfgs (equal group fields).
static std::unique_ptr<Sim> make_group(const mps_lbm_config* cfgs, const std::vector<int>& idx,
                                       const double* const* rho, const double* const* u,
                                       const double* const* f, const uint8_t* const* solid,
                                       hipStream_t st, const MaskParts* mp) {
  std::vector<mps_lbm_config> gc;
  for (int d : idx) gc.push_back(cfgs[d]);
  auto build = [&](auto* s) {
    std::unique_ptr<Sim> keep(s);
    for (size_t j = 0; j < idx.size(); ++j) {
      const int d = idx[j];
      s->init_domain((int)j, rho ? rho[d] : nullptr, u ? u[d] : nullptr, f ? f[d] : nullptr,
                     solid ? solid[d] : nullptr, mp);
    }
    s->finish_init();
    return keep;
  };
  if (gc[0].precision == MPS_LBM_FP64)
    return build(new SimT<double>(gc.data(), (int)gc.size(), st, g_alloc));
  return build(new SimT<float>(gc.data(), (int)gc.size(), st, g_alloc));
}

static int create(const mps_lbm_config* cfgs, int count, const double* const* rho,
                  const double* const* u, const double* const* f, const uint8_t* const* solid,
                  void* hip_stream, mps_lbm_t** out, const MaskParts* mp = nullptr) {
  return guarded([&]() -> int {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      return fail(MPS_LBM_EHIP, "no HIP device");
    }
    std::unique_ptr<mps_lbm> h(new mps_lbm());
    hipStream_t st = (hipStream_t)hip_stream;
    // group the domains by the fields a batched engine needs equal, in the
    // order of their first appearance
    std::vector<std::vector<int>> groups;
    std::vector<std::pair<int, int>> where(count);
    for (int d = 0; d < count; ++d) {
      size_t gi = 0;
      while (gi < groups.size() && !same_group(cfgs[groups[gi][0]], cfgs[d])) ++gi;
      if (gi == groups.size()) groups.emplace_back();
      where[d] = {(int)gi, (int)groups[gi].size()};
      groups[gi].push_back(d);
    }
    if (groups.size() == 1) {
      h->sim = make_group(cfgs, groups[0], rho, u, f, solid, st, mp);
    } else {
      std::unique_ptr<MultiSim> ms(new MultiSim());
      ms->st = st;
      ms->where = where;
      ms->make_streams((int)groups.size());
      for (size_t i = 0; i < groups.size(); ++i)
        ms->g.push_back(make_group(cfgs, groups[i], rho, u, f, solid, ms->gs[i], mp));
      h->sim = std::move(ms);
    }
    *out = h.release();
    g_last_error.clear();
    return MPS_LBM_OK;
  });
}

int mps_lbm_init_from_field(const mps_lbm_config* cfg, const double* rho, const double* u,
                            const double* f, const uint8_t* solid, void* hip_stream,
                            mps_lbm_t** out) {
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int v = validate(cfg);
  if (v) return v;
  if (!f && (!rho || !u)) return fail(MPS_LBM_EINVAL, "need f or both rho and u");
  return create(cfg, 1, &rho, &u, &f, &solid, hip_stream, out);
}

int mps_lbm_init_tensor_mask(const mps_lbm_config* cfg, const double* rho, const double* u,
                             const double* f, const uint8_t* solid_outer, int l,
                             const uint8_t* solid_inner, void* hip_stream, mps_lbm_t** out) {
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int v = validate(cfg);
  if (v) return v;
  if (!f && (!rho || !u)) return fail(MPS_LBM_EINVAL, "need f or both rho and u");
  if (!solid_outer || !solid_inner) return fail(MPS_LBM_EINVAL, "mask parts are NULL");
  if (l < 2 || cfg->n - l < 2)
    return fail(MPS_LBM_EINVAL, "each mask part needs at least 2 sites (2 <= l <= n - 2)");
  const MaskParts mp{solid_outer, l, solid_inner};
  const uint8_t* none = nullptr;
  return create(cfg, 1, &rho, &u, &f, &none, hip_stream, out, &mp);
}

int mps_lbm_init_batch(const mps_lbm_config* cfgs, int count, const double* const* rho,
                       const double* const* u, const uint8_t* const* solid, void* hip_stream,
                       mps_lbm_t** out) {
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || count < 1) return fail(MPS_LBM_EINVAL, "need count >= 1 configurations");
  if (!rho || !u) return fail(MPS_LBM_EINVAL, "rho and u are NULL");
  for (int d = 0; d < count; ++d) {
    int v = validate(cfgs + d);
    if (v) return v;
    if (!rho[d] || !u[d]) return fail(MPS_LBM_EINVAL, "rho[d] or u[d] is NULL");
  }
  return create(cfgs, count, rho, u, nullptr, solid, hip_stream, out);
}

int mps_lbm_capture_step(mps_lbm_t* h) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  return guarded([&]() -> int {
    h->sim->capture();
    return MPS_LBM_OK;
  });
}

int mps_lbm_domains(const mps_lbm_t* h) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  return h->sim->domains();
}

int mps_lbm_step(mps_lbm_t* h, int nsteps) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(MPS_LBM_EINVAL, "nsteps < 0");
  if (h->sim->fatal_seen())
    return fail(MPS_LBM_ENUMERIC, "the state holds non-finite values; no step taken");
  return guarded([&]() -> int {
    h->sim->step(nsteps);
    return MPS_LBM_OK;
  });
}

int mps_lbm_to_dense_domain(mps_lbm_t* h, int domain, int what, double* out, size_t out_len) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  if (what < MPS_LBM_POPS || what > MPS_LBM_VEL) return fail(MPS_LBM_EINVAL, "bad what");
  if (domain < 0 || domain >= h->sim->domains()) return fail(MPS_LBM_EINVAL, "bad domain");
  const long N3 = h->sim->cells(domain);
  const long Q = h->sim->velocities(domain);
  size_t need = (size_t)((what == MPS_LBM_POPS) ? Q * N3 : (what == MPS_LBM_RHO ? N3 : 3 * N3));
  if (out_len < need) return fail(MPS_LBM_EINVAL, "out_len too small");
  return guarded([&]() -> int {
    const int ns = h->sim->numeric_status();
    if (ns) return ns;
    h->sim->to_dense(domain, what, out);
    return MPS_LBM_OK;
  });
}

int mps_lbm_kinetic_energy(mps_lbm_t* h, int domain, double* e_kin) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!e_kin) return fail(MPS_LBM_EINVAL, "e_kin is NULL");
  if (domain < 0 || domain >= h->sim->domains()) return fail(MPS_LBM_EINVAL, "bad domain");
  return guarded([&]() -> int {
    const int ns = h->sim->numeric_status();
    if (ns) return ns;
    *e_kin = h->sim->kinetic_energy(domain);
    return MPS_LBM_OK;
  });
}

int mps_lbm_to_dense(mps_lbm_t* h, int what, double* out, size_t out_len) {
  return mps_lbm_to_dense_domain(h, 0, what, out, out_len);
}

int mps_lbm_get_mps(mps_lbm_t* h, int which, double* out, size_t out_len, int* bonds) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!bonds) return fail(MPS_LBM_EINVAL, "bonds is NULL");
  if (which < 0 || which > MPS_LBM_MPS_MASK) return fail(MPS_LBM_EINVAL, "bad which");
  return guarded([&]() -> int {
    const int ns = h->sim->numeric_status();
    if (ns) return ns;
    return h->sim->get_mps(0, which, out, out_len, bonds);
  });
}

int mps_lbm_observables_domain(mps_lbm_t* h, int domain, mps_lbm_obs* out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  if (domain < 0 || domain >= h->sim->domains()) return fail(MPS_LBM_EINVAL, "bad domain");
  return guarded([&]() -> int {
    h->sim->observables(domain, out);
    return MPS_LBM_OK;
  });
}

int mps_lbm_observables(mps_lbm_t* h, mps_lbm_obs* out) {
  return mps_lbm_observables_domain(h, 0, out);
}

int mps_lbm_kernel_timing(mps_lbm_t* h, int kind) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (kind < MPS_LBM_K_NONE || kind > MPS_LBM_K_CHOLESKY) return fail(MPS_LBM_EINVAL, "bad kind");
  return guarded([&]() -> int {
    h->sim->set_timing(kind);
    return MPS_LBM_OK;
  });
}

int mps_lbm_kernel_stats(mps_lbm_t* h, mps_lbm_kstats* out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  return guarded([&]() -> int {
    h->sim->kstats(out);
    return MPS_LBM_OK;
  });
}

int mps_lbm_train_rank_predictor(mps_lbm_t* h, int epochs, double lr, double* loss_out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (epochs < 1) return fail(MPS_LBM_EINVAL, "epochs < 1");
  if (!(lr > 0.0) || !(lr < 1.0)) return fail(MPS_LBM_EINVAL, "lr outside (0, 1)");
  return guarded([&]() -> int {
    const float l = h->sim->train_predictor(epochs, (float)lr);
    if (loss_out) *loss_out = l;
    return MPS_LBM_OK;
  });
}

int mps_lbm_load_rank_model(mps_lbm_t* h, const float* weights, size_t n) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!weights) return fail(MPS_LBM_EINVAL, "weights is NULL");
  if (n != (size_t)MLP_NPARAM) return fail(MPS_LBM_EINVAL, "weights must hold 37505 floats");
  return guarded([&]() -> int {
    h->sim->rank_model(const_cast<float*>(weights), 1);
    return MPS_LBM_OK;
  });
}

int mps_lbm_get_rank_model(mps_lbm_t* h, float* weights, size_t n) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!weights) return fail(MPS_LBM_EINVAL, "weights is NULL");
  if (n < (size_t)MLP_NPARAM) return fail(MPS_LBM_EINVAL, "n below 37505");
  return guarded([&]() -> int {
    h->sim->rank_model(weights, 0);
    return MPS_LBM_OK;
  });
}

int mps_lbm_autotune(mps_lbm_t* h, int* classes_tuned) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  return guarded([&]() -> int {
    const int n = h->sim->autotune();
    if (classes_tuned) *classes_tuned = n;
    return MPS_LBM_OK;
  });
}

int mps_lbm_rank_predictor_info(mps_lbm_t* h, mps_lbm_predictor_info* out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  return guarded([&]() -> int {
    h->sim->predictor_info(out);
    return MPS_LBM_OK;
  });
}

int mps_lbm_set_face_profile(mps_lbm_t* h, int domain, int face, const double* coef,
                             double dt) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (domain < 0 || domain >= h->sim->domains()) return fail(MPS_LBM_EINVAL, "no such domain");
  if (face < 0 || face > 5) return fail(MPS_LBM_EINVAL, "face outside [0, 5]");
  if (coef) {
    for (int c = 0; c < 6; ++c)
      if (!std::isfinite(coef[c])) return fail(MPS_LBM_EINVAL, "non-finite profile coefficient");
    if (coef[4] < 0.0) return fail(MPS_LBM_EINVAL, "profile exponent c4 < 0");
    if (!std::isfinite(dt) || dt < 0.0) return fail(MPS_LBM_EINVAL, "dt < 0");
  }
  return guarded([&]() -> int {
    h->sim->set_face_profile(domain, face, coef, dt);
    return MPS_LBM_OK;
  });
}

int mps_lbm_set_region(mps_lbm_t* h, int domain, const int* lo, const int* hi, double rho_ref) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (domain < 0 || domain >= h->sim->domains()) return fail(MPS_LBM_EINVAL, "no such domain");
  if (!lo || !hi) return fail(MPS_LBM_EINVAL, "lo or hi is NULL");
  if (!std::isfinite(rho_ref) || !(rho_ref > 0.0)) return fail(MPS_LBM_EINVAL, "rho_ref <= 0");
  return guarded([&]() -> int {
    h->sim->set_region(domain, lo, hi, rho_ref);
    return MPS_LBM_OK;
  });
}

int mps_lbm_debug_raise_flags(mps_lbm_t* h, int nonfinite, int sweep_limit) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (nonfinite < 0 || sweep_limit < 0) return fail(MPS_LBM_EINVAL, "negative count");
  return guarded([&]() -> int {
    h->sim->raise_flags(nonfinite, sweep_limit);
    return MPS_LBM_OK;
  });
}

int mps_lbm_mlp_gradient(const float* params, const float* x, const float* t, int batch,
                         float* loss, float* grad) {
  if (!params || !x || !t || !loss || !grad) return fail(MPS_LBM_EINVAL, "NULL argument");
  if (batch < 1 || batch > 1024) return fail(MPS_LBM_EINVAL, "batch outside [1, 1024]");
  std::vector<void*> mem;
  const Allocator al = g_alloc;
  auto release = [&]() {
    for (void* p : mem) {
      if (al.free_)
        al.free_(p, nullptr, al.ctx);
      else
        (void)hipFree(p);
    }
    mem.clear();
  };
  const int rc = guarded([&]() -> int {
    auto alloc = [&mem, &al](size_t b) -> void* {
      void* p = nullptr;
      if (al.alloc) {
        p = al.alloc(b, nullptr, al.ctx);
      } else if (hipMalloc(&p, b) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
      }
      if (!p) throw Error(MPS_LBM_ENOMEM, "device allocation failed");
      mem.push_back(p);
      return p;
    };
    Mlp m;
    m.setup(batch, alloc, 0, nullptr);
    float* dx = (float*)alloc(4L * batch * MLP_IN);
    float* dt = (float*)alloc(4L * batch);
    HIP_OK(hipMemcpy(m.p, params, 4L * MLP_NPARAM, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dx, x, 4L * batch * MLP_IN, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dt, t, 4L * batch, hipMemcpyHostToDevice));
    m.forward(dx, batch, nullptr);
    m.backward(dx, dt, batch, nullptr);
    HIP_OK(hipMemcpy(grad, m.g, 4L * MLP_NPARAM, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(loss, m.loss, 4, hipMemcpyDeviceToHost));
    return MPS_LBM_OK;
  });
  (void)hipDeviceSynchronize();
  release();
  return rc;
}

int mps_lbm_mlp_gradient_device(const float* params, const float* x, const float* t, int batch,
                                float* loss, float* grad, void* hip_stream) {
  if (!params || !x || !t || !loss || !grad) return fail(MPS_LBM_EINVAL, "NULL argument");
  if (batch < 1 || batch > MLP_SCRATCH_BATCH)
    return fail(MPS_LBM_EINVAL, "batch outside [1, 1024] (the scratch holds 1024 samples)");
  return guarded([&]() -> int {
    float* s = scratch_on_current_device();
    hipStream_t st = (hipStream_t)hip_stream;
    // the network's buffers: the caller's parameters, gradient and loss, the
    // activations and deltas packed into the scratch
    Mlp m;
    m.p = const_cast<float*>(params);
    m.g = grad;
    m.loss = loss;
    m.bmax = batch;
    float** acts[] = {&m.z1, &m.a1, &m.z2, &m.a2, &m.z3, &m.a3, &m.d3, &m.d2, &m.d1};
    long off = 0;
    for (float** a : acts) {
      *a = s + off;
      off += (long)batch * MLP_H;
    }
    m.y = s + off;
    off += batch;
    m.dy = s + off;
    m.forward(x, batch, st);
    m.backward(x, t, batch, st);
    HIP_OK(hipGetLastError());
    return MPS_LBM_OK;
  });
}

void mps_lbm_destroy(mps_lbm_t* h) {
  try {
    delete h;
  } catch (...) {
  }
}

const char* mps_lbm_last_error(void) { return g_last_error.c_str(); }

const char* mps_lbm_version(void) { return "mps-lbm-gfx950 0.2"; }

}  // extern "C"
