// C ABI and step schedule of the MI355X MPS lattice Boltzmann library.
//
// One D3Q19 BGK step on MPS populations (Section 3.2 of the paper), in this
// order:
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
#include "../../include/mps_lbm.h"

#include <cmath>
#include <cstring>
#include <memory>
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
  virtual void step(int nsteps) = 0;
  virtual void to_dense(int what, double* out) = 0;
  virtual void observables(mps_lbm_obs* o) = 0;
  virtual void set_timing(int kind) = 0;
  virtual void kstats(mps_lbm_kstats* o) = 0;
  virtual int get_mps(int which, double* out, size_t out_len, int* bonds) = 0;
};

template <typename T>
struct SimT : Sim {
  typedef typename Engine<T>::Term Term;
  mps_lbm_config cfg;
  Engine<T> E;
  hipStream_t st;
  int n, N;
  long N3;
  int f[19];
  int one = -1, mask = -1, fluid = -1;
  int fplane[6];
  double* rho0 = nullptr;   // device scalar
  double* scratch = nullptr;
  double n_fluid = 0.0;
  double mask_err = 0.0;
  long long steps = 0;
  int chi_mask = 1;

  SimT(const mps_lbm_config& c, hipStream_t s) : cfg(c), st(s) {
    n = c.n;
    N = 1 << n;
    N3 = 1L << (3 * n);
    for (int i = 0; i < 6; ++i) fplane[i] = -1;
    E.sweeps = c.sweeps;
    E.setup(n, c.chi_max, c.tol, s, 256, 19);
    rho0 = (double*)E.dalloc(8 * 64);
    scratch = (double*)E.dalloc(8 * 64);
    chi_mask = c.chi_mask_max > 0 ? std::min(c.chi_mask_max, c.chi_max) : c.chi_max;
  }

  // --- dense -> MPS: TT-SVD (Section 2.1, svd-comp equation) of cnt
  // scale-ordered fields W, truncated at (chi_r, tol_r).  W is overwritten.
  int dense_chunks(long count) const {
    return (int)std::max<long>(1, std::min<long>(2048, (count + 255) / 256));
  }

  void dense_to_mps(T* W, int cnt, const std::vector<int>& objs, int chi_r, double tol_r) {
    E.tt_svd(W, cnt, objs, chi_r, tol_r);
  }

  void free_last(int k) {
    for (int i = 0; i < k && !E.allocs.empty(); ++i) {
      (void)hipFree(E.allocs.back());
      E.allocs.pop_back();
    }
  }

  void init(const double* rho, const double* u, const double* fin, const uint8_t* solid) {
    int cvec[57];
    double w[19];
    for (int i = 0; i < 19; ++i) {
      for (int a = 0; a < 3; ++a) cvec[3 * i + a] = kC[i][a];
      w[i] = kW(i);
    }
    int* dc = (int*)E.dalloc(sizeof(cvec));
    double* dw = (double*)E.dalloc(sizeof(w));
    HIP_OK(hipMemcpy(dc, cvec, sizeof(cvec), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dw, w, sizeof(w), hipMemcpyHostToDevice));
    cvec_dev = dc;
    one = E.acquire();
    E.set_ones(one);
    // obstacle mask
    double* dd = (double*)E.dalloc(8 * N3 * 19);  // dense staging (FP64)
    T* W = (T*)E.dalloc(sizeof(T) * N3 * 19);
    uint8_t* dsolid = nullptr;
    if (solid) {
      dsolid = (uint8_t*)E.dalloc(N3);
      HIP_OK(hipMemcpy(dsolid, solid, N3, hipMemcpyHostToDevice));
      std::vector<double> hs(N3);
      for (long e = 0; e < N3; ++e) hs[e] = solid[e] ? 1.0 : 0.0;
      HIP_OK(hipMemcpy(dd, hs.data(), 8 * N3, hipMemcpyHostToDevice));
      hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(N3)), dim3(256), 0, st,
                         (const double*)dd, W, n, 1, 1);
      mask = E.acquire();
      T* Wkeep = (T*)E.dalloc(sizeof(T) * N3);
      hipLaunchKernelGGL(k_copy_plain<T>, dim3(dense_chunks(N3)), dim3(256), 0, st, (const T*)W, Wkeep,
                         N3);
      dense_to_mps(W, 1, {mask}, chi_mask, cfg.tol_mask);
      // decomposition error of the mask
      T* back = (T*)E.dalloc(sizeof(T) * N3);
      T* work = (T*)E.dalloc(sizeof(T) * N3);
      E.to_dense({mask}, back, work);
      HIP_OK(hipMemsetAsync(scratch, 0, 16, st));
      hipLaunchKernelGGL(k_diff_norm<T>, dim3(std::min(256, dense_chunks(N3))), dim3(256), 0, st, (const T*)back,
                         (const T*)Wkeep, N3, scratch);
      double hnorm[2];
      HIP_OK(hipMemcpyAsync(hnorm, scratch, 16, hipMemcpyDeviceToHost, st));
      E.inner_ones({mask}, scratch + 2);
      double ones_m = 0.0;
      HIP_OK(hipMemcpyAsync(&ones_m, scratch + 2, 8, hipMemcpyDeviceToHost, st));
      HIP_OK(hipStreamSynchronize(st));
      mask_err = hnorm[1] > 0 ? std::sqrt(hnorm[0] / hnorm[1]) : 0.0;
      n_fluid = (double)N3 - ones_m;
      free_last(3);
      // fluid = round(1 - m)
      fluid = E.acquire();
      E.add({fluid}, {one}, {mask}, {Coef{1.0, 0}, Coef{-1.0, 0}}, nullptr);
      E.round({fluid}, cfg.chi_max, cfg.tol_mask);
    } else {
      n_fluid = (double)N3;
      fluid = one;
    }
    // open-face planes of the fluid indicator
    for (int ax = 0; ax < 3; ++ax) {
      if (!cfg.axis_open[ax]) continue;
      for (int side = 0; side < 2; ++side) {
        int face = 2 * ax + side;
        if (cfg.face_bc[face] == MPS_LBM_BC_NONE) continue;
        std::vector<int> o = E.slice({fluid}, {ax}, {side == 0 ? 0 : N - 1});
        fplane[face] = o[0];
      }
    }
    // initial populations
    if (fin) {
      HIP_OK(hipMemcpy(dd, fin, 8 * N3 * 19, hipMemcpyHostToDevice));
    } else {
      double* drho = (double*)E.dalloc(8 * N3);
      double* du = (double*)E.dalloc(8 * N3 * 3);
      HIP_OK(hipMemcpy(drho, rho, 8 * N3, hipMemcpyHostToDevice));
      HIP_OK(hipMemcpy(du, u, 8 * N3 * 3, hipMemcpyHostToDevice));
      hipLaunchKernelGGL(k_feq_dense, dim3(dense_chunks(N3)), dim3(256), 0, st, (const double*)drho,
                         (const double*)du, (const uint8_t*)dsolid, dd, N3, (const int*)dc,
                         (const double*)dw);
      HIP_OK(hipStreamSynchronize(st));
      free_last(2);
    }
    hipLaunchKernelGGL((k_scale_permute<double, T>), dim3(dense_chunks(19 * N3)), dim3(256), 0,
                       st, (const double*)dd, W, n, 19, 1);
    std::vector<int> objs(19);
    for (int i = 0; i < 19; ++i) objs[i] = f[i] = E.acquire();
    dense_to_mps(W, 19, objs, cfg.chi_max, cfg.tol);
    HIP_OK(hipStreamSynchronize(st));
    // release the dense staging (W, dd, and the solid copy)
    (void)hipFree(W);
    (void)hipFree(dd);
    if (dsolid) (void)hipFree(dsolid);
    E.allocs.erase(std::remove_if(E.allocs.begin(), E.allocs.end(),
                                  [&](void* p) { return p == W || p == dd || p == dsolid; }),
                   E.allocs.end());
  }
  int* cvec_dev = nullptr;

  // ---------------------------------------------------------------- step
  void step_once() {
    HIP_OK(hipMemsetAsync(E.stats, 0, 8, st));
    E.roundings = 0;
    E.products = 0;
    const double tau = cfg.tau, om = 1.0 / tau;
    // 1. moments
    std::vector<std::vector<Term>> S(4);
    for (int i = 0; i < 19; ++i) S[0].push_back({Coef{1.0, 0}, f[i]});
    for (int a = 0; a < 3; ++a)
      for (int i = 0; i < 19; ++i)
        if (kC[i][a]) S[1 + a].push_back({Coef{(double)kC[i][a], 0}, f[i]});
    std::vector<int> mom = E.sums(S, rho0);
    int rho = mom[0];
    int j[3] = {mom[1], mom[2], mom[3]};
    // 2. rho_0
    E.inner_ones({rho}, scratch);
    hipLaunchKernelGGL(k_div_scalar, dim3(1), dim3(64), 0, st, (const double*)scratch, n_fluid,
                       rho0);
    // 3. inverse density
    int r = -1;
    if (cfg.inv_rho_mode == MPS_LBM_INV_TAYLOR2) {
      int e = E.sums({{{Coef{1.0, -1}, rho}, {Coef{-1.0, 0}, one}}}, rho0)[0];
      int ee = E.prods({{e, e}})[0];
      r = E.sums({{{Coef{1.0, -1}, one}, {Coef{-1.0, -1}, e}, {Coef{1.0, -1}, ee}}}, rho0)[0];
      E.release(e);
      E.release(ee);
    } else {
      int y = E.sums({{{Coef{2.0, -1}, one}, {Coef{-1.0, -2}, rho}}}, rho0)[0];
      for (int it = 1; it < cfg.inv_rho_iters; ++it) {
        int ry = E.prods({{rho, y}})[0];
        int t = E.sums({{{Coef{2.0, 0}, one}, {Coef{-1.0, 0}, ry}}}, rho0)[0];
        int y2 = E.prods({{y, t}})[0];
        E.release(ry);
        E.release(t);
        E.release(y);
        y = y2;
      }
      r = y;
    }
    // 4. j_eq, u, Pi
    int jeq[3];
    {
      std::vector<std::vector<Term>> SJ;
      std::vector<int> which;
      for (int a = 0; a < 3; ++a) {
        if (cfg.g[a] != 0.0) {
          SJ.push_back({{Coef{1.0, 0}, j[a]}, {Coef{tau * cfg.g[a], 0}, rho}});
          which.push_back(a);
        } else {
          jeq[a] = j[a];
        }
      }
      if (!SJ.empty()) {
        std::vector<int> o = E.sums(SJ, rho0);
        for (size_t q = 0; q < which.size(); ++q) {
          E.release(j[which[q]]);
          jeq[which[q]] = o[q];
        }
      }
    }
    std::vector<int> u = E.prods({{jeq[0], r}, {jeq[1], r}, {jeq[2], r}});
    static const int PI[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    std::vector<std::pair<int, int>> pp;
    for (int q = 0; q < 6; ++q) pp.push_back({jeq[PI[q][0]], u[PI[q][1]]});
    std::vector<int> Pi = E.prods(pp);
    int S0 = E.sums({{{Coef{1.0, 0}, rho}, {Coef{-1.5, 0}, Pi[0]}, {Coef{-1.5, 0}, Pi[1]},
                      {Coef{-1.5, 0}, Pi[2]}}},
                    rho0)[0];
    // 5. BGK
    std::vector<std::vector<Term>> SB(19);
    for (int i = 0; i < 19; ++i) {
      double wi = kW(i);
      SB[i].push_back({Coef{1.0 - om, 0}, f[i]});
      SB[i].push_back({Coef{om * wi, 0}, S0});
      for (int a = 0; a < 3; ++a)
        if (kC[i][a]) SB[i].push_back({Coef{3.0 * om * wi * kC[i][a], 0}, jeq[a]});
      for (int q = 0; q < 6; ++q) {
        int a = PI[q][0], b = PI[q][1];
        int coef = kC[i][a] * kC[i][b] * (a == b ? 1 : 2);
        if (coef) SB[i].push_back({Coef{4.5 * om * wi * coef, 0}, Pi[q]});
      }
    }
    std::vector<int> fpost = E.sums(SB, rho0);
    for (int i = 0; i < 19; ++i) E.release(f[i]);
    E.release(rho);
    E.release(r);
    E.release(S0);
    for (int q = 0; q < 6; ++q) E.release(Pi[q]);
    for (int a = 0; a < 3; ++a) E.release(jeq[a]);
    // 7a. open-face boundary terms (need post-collision f_ihat and u)
    std::vector<std::vector<Term>> bterms(19);
    std::vector<int> btemp;
    for (int ax = 0; ax < 3; ++ax) {
      if (!cfg.axis_open[ax]) continue;
      for (int side = 0; side < 2; ++side) {
        int face = 2 * ax + side;
        int typ = cfg.face_bc[face];
        if (typ == MPS_LBM_BC_NONE) continue;
        int idx = side == 0 ? 0 : N - 1;
        int entering = side == 0 ? 1 : -1;
        int fp = fplane[face];
        std::vector<int> uu;
        if (typ == MPS_LBM_BC_PRESSURE) {
          std::vector<int> uB = E.slice({u[0], u[1], u[2]}, {ax, ax, ax}, {idx, idx, idx});
          E.round(uB);
          std::vector<std::pair<int, int>> pq;
          for (int q = 0; q < 6; ++q) pq.push_back({uB[PI[q][0]], uB[PI[q][1]]});
          uu = E.prods(pq);
          for (int o : uB) E.release(o);
          for (int o : uu) btemp.push_back(o);
        }
        std::vector<int> ent;
        for (int i = 0; i < 19; ++i)
          if (kC[i][ax] == entering) ent.push_back(i);
        std::vector<int> src, axs, ids;
        for (int i : ent) {
          src.push_back(fpost[kOpp[i]]);
          axs.push_back(ax);
          ids.push_back(idx);
        }
        std::vector<int> fo = E.slice(src, axs, ids);
        for (int o : fo) btemp.push_back(o);
        for (size_t q = 0; q < ent.size(); ++q) {
          int i = ent[q];
          double c[3] = {(double)kC[i][0], (double)kC[i][1], (double)kC[i][2]};
          if (typ == MPS_LBM_BC_VELOCITY) {
            const double* ub = cfg.face_val[face];
            double cu = c[0] * ub[0] + c[1] * ub[1] + c[2] * ub[2];
            bterms[i].push_back({Coef{1.0, 0}, fo[q]});
            bterms[i].push_back({Coef{6.0 * kW(i) * cu, cu == 0.0 ? 0 : 1}, fp});
          } else {
            double rb = cfg.face_val[face][0];
            double kk = 2.0 * kW(i) * rb;
            bterms[i].push_back({Coef{-1.0, 0}, fo[q]});
            bterms[i].push_back({Coef{kk, 0}, fp});
            for (int p = 0; p < 6; ++p) {
              int a = PI[p][0], b = PI[p][1];
              double coef = (a == b) ? kk * (4.5 * c[a] * c[a] - 1.5) : kk * 9.0 * c[a] * c[b];
              if (coef != 0.0) bterms[i].push_back({Coef{coef, 0}, uu[p]});
            }
          }
        }
      }
    }
    // 6. streaming (f_0 does not move)
    std::vector<int> src;
    std::vector<const int*> cv;
    for (int i = 1; i < 19; ++i) {
      src.push_back(fpost[i]);
      cv.push_back(kC[i]);
    }
    std::vector<int> fs1 = E.stream(src, cv, cfg.axis_open);
    int fs[19];
    fs[0] = fpost[0];
    for (int i = 1; i < 19; ++i) fs[i] = fs1[i - 1];
    // 7b. add boundary terms
    {
      std::vector<std::vector<Term>> SBC;
      std::vector<int> which;
      for (int i = 0; i < 19; ++i) {
        if (bterms[i].empty()) continue;
        std::vector<Term> t{{Coef{1.0, 0}, fs[i]}};
        t.insert(t.end(), bterms[i].begin(), bterms[i].end());
        SBC.push_back(t);
        which.push_back(i);
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
    for (int i = 1; i < 19; ++i) E.release(fpost[i]);
    for (int a = 0; a < 3; ++a) E.release(u[a]);
    // 8. obstacle bounce-back
    if (mask >= 0) {
      std::vector<std::pair<int, int>> pm;
      for (int i = 1; i < 19; ++i) pm.push_back({fs[i], mask});
      std::vector<int> g1 = E.prods(pm);
      int g[19];
      g[0] = -1;
      for (int i = 1; i < 19; ++i) g[i] = g1[i - 1];
      std::vector<int> hs;
      std::vector<const int*> hc;
      for (int i = 1; i < 19; ++i) {
        hs.push_back(g[kOpp[i]]);
        hc.push_back(kC[i]);
      }
      std::vector<int> h = E.stream(hs, hc, cfg.axis_open);
      std::vector<std::vector<Term>> SO;
      for (int i = 1; i < 19; ++i)
        SO.push_back({{Coef{1.0, 0}, fs[i]}, {Coef{-1.0, 0}, g[i]}, {Coef{1.0, 0}, h[i - 1]}});
      std::vector<int> o = E.sums(SO, rho0);
      for (int i = 1; i < 19; ++i) {
        E.release(fs[i]);
        E.release(g[i]);
        E.release(h[i - 1]);
        fs[i] = o[i - 1];
      }
    }
    for (int i = 0; i < 19; ++i) f[i] = fs[i];
    last_roundings = E.roundings;
    last_products = E.products;
  }
  long long last_roundings = 0, last_products = 0;

  void step(int nsteps) override {
    for (int s = 0; s < nsteps; ++s) {
      step_once();
      ++steps;
    }
    HIP_OK(hipGetLastError());
  }

  void to_dense(int what, double* out) override {
    T* buf = nullptr;
    T* work = nullptr;
    double* mom = nullptr;
    double* res = nullptr;
    size_t bytes = sizeof(T) * N3 * 19;
    HIP_OK(hipMalloc(&buf, bytes));
    HIP_OK(hipMalloc(&work, bytes));
    std::vector<int> objs(f, f + 19);
    E.to_dense(objs, buf, work);
    long nout = (what == MPS_LBM_POPS) ? 19 * N3 : (what == MPS_LBM_RHO ? N3 : 3 * N3);
    HIP_OK(hipMalloc(&res, 8 * nout));
    if (what == MPS_LBM_POPS) {
      hipLaunchKernelGGL((k_scale_permute<T, double>), dim3(dense_chunks(19 * N3)), dim3(256), 0,
                         st, (const T*)buf, res, n, 19, 0);
    } else {
      HIP_OK(hipMalloc(&mom, 8 * nout));
      hipLaunchKernelGGL(k_moments_dense<T>, dim3(dense_chunks(N3)), dim3(256), 0, st, (const T*)buf, mom,
                         N3, what, (const int*)cvec_dev);
      hipLaunchKernelGGL((k_scale_permute<double, double>), dim3(dense_chunks(nout)), dim3(256), 0, st,
                         (const double*)mom, res, n, (int)(nout / N3), 0);
    }
    HIP_OK(hipMemcpyAsync(out, res, 8 * nout, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    (void)hipFree(buf);
    (void)hipFree(work);
    (void)hipFree(res);
    if (mom) (void)hipFree(mom);
  }

  int get_mps(int which, double* out, size_t out_len, int* bonds) override {
    int idx = which < 19 ? f[which] : mask;
    if (idx < 0) return fail(MPS_LBM_EINVAL, "no obstacle mask in this simulation");
    MpsDev<T> d;
    HIP_OK(hipMemcpyAsync(&d, E.D(idx), sizeof(d), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    size_t need = 0;
    for (int k = 0; k <= n; ++k) bonds[k] = d.r[k];
    for (int k = 0; k < n; ++k) need += (size_t)d.r[k] * PHYS * d.r[k + 1];
    if (!out) return MPS_LBM_OK;
    if (out_len < need) return fail(MPS_LBM_EINVAL, "out_len too small");
    std::vector<T> tmp(need);
    size_t pos = 0;
    for (int k = 0; k < n; ++k) {
      size_t cnt = (size_t)d.r[k] * PHYS * d.r[k + 1];
      HIP_OK(hipMemcpyAsync(tmp.data() + pos, d.data + d.off[k], sizeof(T) * cnt,
                            hipMemcpyDeviceToHost, st));
      pos += cnt;
    }
    HIP_OK(hipStreamSynchronize(st));
    for (size_t e = 0; e < need; ++e) out[e] = (double)tmp[e];
    return MPS_LBM_OK;
  }

  void set_timing(int kind) override { E.timing(kind); }

  void kstats(mps_lbm_kstats* o) override {
    E.flush_events();
    double fl = 0.0;
    if (E.kflops) HIP_OK(hipMemcpy(&fl, E.kflops, 8, hipMemcpyDeviceToHost));
    o->launches = E.tlaunches;
    o->total_ms = E.tms;
    o->flops = fl;
  }

  void observables(mps_lbm_obs* o) override {
    memset(o, 0, sizeof(*o));
    std::vector<int> objs(f, f + 19);
    E.inner_ones(objs, scratch);
    double s[19];
    double stat[2] = {0, 0};
    int ist[4] = {0, 0, 0, 0};
    HIP_OK(hipMemcpyAsync(s, scratch, 8 * 19, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(stat, E.stats, 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ist, E.istats, 16, hipMemcpyDeviceToHost, st));
    double r0 = 0.0;
    HIP_OK(hipMemcpyAsync(&r0, rho0, 8, hipMemcpyDeviceToHost, st));
    std::vector<MpsDev<T>> descs(19);
    for (int i = 0; i < 19; ++i)
      HIP_OK(hipMemcpyAsync(&descs[i], E.D(f[i]), sizeof(MpsDev<T>), hipMemcpyDeviceToHost, st));
    MpsDev<T> md;
    if (mask >= 0) HIP_OK(hipMemcpyAsync(&md, E.D(mask), sizeof(md), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    o->step = steps;
    for (int i = 0; i < 19; ++i) {
      o->mass += s[i];
      for (int a = 0; a < 3; ++a) o->momentum[a] += kC[i][a] * s[i];
    }
    o->rho0 = r0;
    o->n_fluid = n_fluid;
    double nv = 0.0;
    int mb = 1;
    for (int i = 0; i < 19; ++i) {
      for (int k = 1; k < n; ++k) {
        o->bonds[i][k - 1] = descs[i].r[k];
        mb = std::max(mb, descs[i].r[k]);
      }
      for (int k = 0; k < n; ++k) nv += (double)descs[i].r[k] * PHYS * descs[i].r[k + 1];
    }
    o->max_bond = mb;
    o->nvps = nv;
    o->compression = nv > 0 ? 19.0 * (double)N3 / nv : 0.0;
    o->max_discarded = stat[0];
    int mk = 1;
    if (mask >= 0)
      for (int k = 1; k < n; ++k) mk = std::max(mk, md.r[k]);
    o->mask_bond = mask >= 0 ? mk : 0;
    o->mask_trunc_err = mask_err;
    o->roundings = last_roundings;
    o->products = last_products;
    o->svd_failures = ist[0];
    o->nonfinite = ist[1];
    o->jacobi_sweeps = ist[3] > 0 ? (double)ist[2] / ist[3] : 0.0;
    o->lds_bytes = E.lds_elems * 8;
  }
};

}  // namespace

struct mps_lbm {
  std::unique_ptr<Sim> sim;
};

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
}

static int validate(const mps_lbm_config* c) {
  if (!c) return fail(MPS_LBM_EINVAL, "config is NULL");
  if (c->n < 2 || c->n > MPS_LBM_MAX_SITES) return fail(MPS_LBM_EINVAL, "n out of range");
  if (c->lattice != MPS_LBM_D3Q19) return fail(MPS_LBM_EINVAL, "unknown lattice");
  if (c->chi_max < 1) return fail(MPS_LBM_EINVAL, "chi_max < 1");
  if (c->chi_max > 512) return fail(MPS_LBM_EUNSUPPORTED, "chi_max > 512");
  if (!(c->tau > 0.5)) return fail(MPS_LBM_EINVAL, "tau must exceed 1/2");
  if (!(c->tol >= 0.0) || !(c->tol_mask >= 0.0)) return fail(MPS_LBM_EINVAL, "negative tol");
  if (c->inv_rho_mode != MPS_LBM_INV_TAYLOR2 && c->inv_rho_mode != MPS_LBM_INV_NEWTON)
    return fail(MPS_LBM_EINVAL, "unknown inverse-density mode");
  if (c->inv_rho_mode == MPS_LBM_INV_NEWTON && c->inv_rho_iters < 1)
    return fail(MPS_LBM_EINVAL, "inv_rho_iters < 1");
  if (c->precision != MPS_LBM_FP64 && c->precision != MPS_LBM_FP32)
    return fail(MPS_LBM_EINVAL, "unknown precision");
  if (c->sweeps < 1) return fail(MPS_LBM_EINVAL, "sweeps < 1");
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

int mps_lbm_init_from_field(const mps_lbm_config* cfg, const double* rho, const double* u,
                            const double* f, const uint8_t* solid, void* hip_stream,
                            mps_lbm_t** out) {
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  *out = nullptr;
  int v = validate(cfg);
  if (v) return v;
  if (!f && (!rho || !u)) return fail(MPS_LBM_EINVAL, "need f or both rho and u");
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      (void)hipGetLastError();
      return fail(MPS_LBM_EHIP, "no HIP device");
    }
    std::unique_ptr<mps_lbm> h(new mps_lbm());
    hipStream_t st = (hipStream_t)hip_stream;
    if (cfg->precision == MPS_LBM_FP64) {
      auto* s = new SimT<double>(*cfg, st);
      h->sim.reset(s);
      s->init(rho, u, f, solid);
    } else {
      auto* s = new SimT<float>(*cfg, st);
      h->sim.reset(s);
      s->init(rho, u, f, solid);
    }
    *out = h.release();
    g_last_error.clear();
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  }
}

int mps_lbm_step(mps_lbm_t* h, int nsteps) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(MPS_LBM_EINVAL, "nsteps < 0");
  try {
    h->sim->step(nsteps);
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  }
}

int mps_lbm_to_dense(mps_lbm_t* h, int what, double* out, size_t out_len) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  if (what < MPS_LBM_POPS || what > MPS_LBM_VEL) return fail(MPS_LBM_EINVAL, "bad what");
  SimT<double>* sd = dynamic_cast<SimT<double>*>(h->sim.get());
  SimT<float>* sf = dynamic_cast<SimT<float>*>(h->sim.get());
  long N3 = sd ? sd->N3 : sf->N3;
  size_t need = (size_t)((what == MPS_LBM_POPS) ? 19 * N3 : (what == MPS_LBM_RHO ? N3 : 3 * N3));
  if (out_len < need) return fail(MPS_LBM_EINVAL, "out_len too small");
  try {
    h->sim->to_dense(what, out);
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  }
}

int mps_lbm_get_mps(mps_lbm_t* h, int which, double* out, size_t out_len, int* bonds) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!bonds) return fail(MPS_LBM_EINVAL, "bonds is NULL");
  if (which < 0 || which > MPS_LBM_MPS_MASK) return fail(MPS_LBM_EINVAL, "bad which");
  try {
    return h->sim->get_mps(which, out, out_len, bonds);
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  }
}

int mps_lbm_observables(mps_lbm_t* h, mps_lbm_obs* out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  try {
    h->sim->observables(out);
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::exception& e) {
    return fail(MPS_LBM_EHIP, e.what());
  }
}

int mps_lbm_kernel_timing(mps_lbm_t* h, int kind) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (kind < MPS_LBM_K_NONE || kind > MPS_LBM_K_CHOLESKY) return fail(MPS_LBM_EINVAL, "bad kind");
  try {
    h->sim->set_timing(kind);
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

int mps_lbm_kernel_stats(mps_lbm_t* h, mps_lbm_kstats* out) {
  if (!h || !h->sim) return fail(MPS_LBM_EINVAL, "handle is NULL");
  if (!out) return fail(MPS_LBM_EINVAL, "out is NULL");
  try {
    h->sim->kstats(out);
    return MPS_LBM_OK;
  } catch (const Error& e) {
    return fail(e.code, e.what());
  }
}

void mps_lbm_destroy(mps_lbm_t* h) { delete h; }

const char* mps_lbm_last_error(void) { return g_last_error.c_str(); }

const char* mps_lbm_version(void) { return "mps-lbm-gfx950 0.1"; }

}  // extern "C"
