// Separable preconditioner for the TT solve.
//
// P = c0 a0 (x) m1 (x) m2 + c1 m0 (x) a1 (x) m2 + c2 m0 (x) m1 (x) a2 is the
// stiffness operator of the parametric cube with constant coefficients: a_d and
// m_d are the 1-D stiffness and mass matrices of the solution B-splines on the
// interior indices (the selector matrices d and m of Section 4.2.1 with a unit
// factor), and c_d is the mean of R_dd over the parametric domain.  With the
// generalised eigenbasis a_d V_d = m_d V_d diag(lambda_d), V_d^T m_d V_d = I,
// P^-1 = (V0 (x) V1 (x) V2) D^-1 (V0 (x) V1 (x) V2)^T, D = sum_d c_d lambda_d.
// D^-1 is not low-rank, so 1/s is replaced by an exponential sum
// sum_t w_t exp(-tau_t s) (trapezoidal rule for 1/s = int exp(t - s e^t) dt),
// which turns the diagonal scaling into a sum of rank-1 scalings of the TT
// cores; the result is re-compressed.  This is not part of the paper (which
// solves with AMEn); it only changes how fast the TT-CG iteration converges,
// not the solution it converges to.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <memory>
#include <vector>

#include "precond.hpp"
#include "problem.hpp"

namespace ttiga {

__global__ void k_band_to_dense(int n, int p, const double* __restrict__ M, double* __restrict__ D) {
  const long total = (long)n * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e / n, j = e % n;
    const int t = j - i + p;
    D[e] = (t >= 0 && t <= 2 * p) ? M[(long)i * (2 * p + 1) + t] : 0.0;
  }
}

// v[a][b] = sum_q w_q G[a][q][b]
__global__ void k_weighted_core_sum(int ra, int Q, int rb, const double* __restrict__ G,
                                    const double* __restrict__ w, double* __restrict__ v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ra * rb) return;
  const int a = e / rb, b = e % rb;
  double s = 0.0;
  for (int q = 0; q < Q; ++q) s += w[q] * G[((long)a * Q + q) * rb + b];
  v[e] = s;
}

// tab[t][i] = scale_t * exp(-tau_t * c * lam[i])
__global__ void k_exp_table(int R, int n, const double* __restrict__ tau, const double* __restrict__ scale,
                            double c, const double* __restrict__ lam, double* __restrict__ tab) {
  const long total = (long)R * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int t = e / n, i = e % n;
    tab[e] = scale[t] * exp(-tau[t] * c * lam[i]);
  }
}

// Core k of sum_t (diag(tab0_t) (x) diag(tab1_t) (x) diag(tab2_t)) x: block structure in t.
__global__ void k_exp_hadamard(int k, int R, int n, int ra, int rb, const double* __restrict__ X,
                               const double* __restrict__ tab, double* __restrict__ O) {
  const int oa = (k == 0) ? 1 : R * ra;
  const int ob = (k == 2) ? 1 : R * rb;
  const long total = (long)oa * n * ob;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int ib = e % ob;
    const int i = (e / ob) % n;
    const int ia = e / ((long)ob * n);
    double v = 0.0;
    if (k == 0) {
      const int t = ib / rb, b = ib % rb;
      v = tab[(long)t * n + i] * X[(long)i * rb + b];
    } else if (k == 2) {
      const int t = ia / ra, a = ia % ra;
      v = tab[(long)t * n + i] * X[(long)a * n + i];
    } else {
      const int t = ia / ra, a = ia % ra, t2 = ib / rb, b = ib % rb;
      if (t == t2) v = tab[(long)t * n + i] * X[((long)a * n + i) * rb + b];
    }
    O[e] = v;
  }
}

__global__ void k_square(double* __restrict__ x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= x[i];
}

static std::shared_ptr<EigenBasis> eigenbasis(Problem& P, int d) {
  Context& ctx = *P.ctx;
  const int p = P.p, band = 2 * p + 1;
  const int n = P.n[d], Q = P.Q[d], m = P.hi[d] - P.lo[d];
  const std::array<int, 5> key = {n, p, P.g, P.lo[d], P.hi[d]};
  PlanCache& pc = *ctx.plans;
  {
    std::unique_lock<std::mutex> lk(pc.mu);
    while (true) {
      auto it = pc.map.find(key);
      if (it != pc.map.end()) return std::static_pointer_cast<EigenBasis>(it->second);
      if (pc.busy.insert(key).second) break;  // this caller computes it
      pc.cv.wait(lk);
    }
  }
  // whatever happens below, the key leaves `busy` and waiters look again
  struct Done {
    PlanCache& pc;
    const std::array<int, 5>& key;
    ~Done() {
      {
        std::lock_guard<std::mutex> lk(pc.mu);
        pc.busy.erase(key);
      }
      pc.cv.notify_all();
    }
  } done{pc, key};
  auto e = std::make_shared<EigenBasis>();
  e->ni = m;
  DBuf ones(ctx.alloc, sizeof(double) * Q);
  fill(ctx, ones.d(), Q, 1.0);
  DBuf mb(ctx.alloc, sizeof(double) * n * band), ab(ctx.alloc, sizeof(double) * n * band);
  launch_assemble_band(ctx, n, p, P.g, 1, 1, ones.d(), P.tab_w[d].d(), P.tab_B[d].d(), P.tab_B[d].d(), mb.d());
  launch_assemble_band(ctx, n, p, P.g, 1, 1, ones.d(), P.tab_w[d].d(), P.tab_D[d].d(), P.tab_D[d].d(), ab.d());
  DBuf mi(ctx.alloc, sizeof(double) * m * band), ai(ctx.alloc, sizeof(double) * m * band);
  launch_slice_band(ctx, n, p, P.lo[d], m, 1, 1, mb.d(), mi.d());
  launch_slice_band(ctx, n, p, P.lo[d], m, 1, 1, ab.d(), ai.d());
  DBuf Md(ctx.alloc, sizeof(double) * m * m), Ad(ctx.alloc, sizeof(double) * m * m);
  hipLaunchKernelGGL(k_band_to_dense, dim3(grid_for((long)m * m)), dim3(256), 0, ctx.stream, m, p, mi.d(), Md.d());
  hipLaunchKernelGGL(k_band_to_dense, dim3(grid_for((long)m * m)), dim3(256), 0, ctx.stream, m, p, ai.d(), Ad.d());
  TTIGA_HIP(hipGetLastError());
  DBuf Rm(ctx.alloc, sizeof(double) * m * m), Rmi(ctx.alloc, sizeof(double) * m * m);
  TTIGA_CHECK(cholesky_inverse(ctx, Md.d(), m, Rm.d(), Rmi.d()), TTIGA_E_ARG,
              "1-D mass matrix is not positive definite");
  // S = Rmi^T A Rmi, symmetric positive semi-definite; its SVD is its eigendecomposition
  DBuf T1(ctx.alloc, sizeof(double) * m * m), S(ctx.alloc, sizeof(double) * m * m);
  gemm(ctx, false, false, m, m, m, 1.0, Ad.d(), m, 0, Rmi.d(), m, 0, 0.0, T1.d(), m, 0);
  gemm(ctx, true, false, m, m, m, 1.0, Rmi.d(), m, 0, T1.d(), m, 0, 0.0, S.d(), m, 0);
  DBuf U(ctx.alloc, sizeof(double) * m * m), W(ctx.alloc, sizeof(double) * m * m);
  // with the Dirichlet cut S is positive definite: S = L L^T (pivoted Cholesky, full rank)
  // and the left singular vectors of L are the eigenvectors of S, sigma^2 its eigenvalues
  // (Jacobi on L converges in about a third of the sweeps of Jacobi on S); a singular S
  // keeps the Jacobi SVD of S itself, whose null vectors the fast diagonalisation needs
  DBuf Lc(ctx.alloc, sizeof(double) * m * m);
  const int k = pivoted_cholesky(ctx, S.d(), m, Lc.d(), 2.220446049250313e-16);
  e->lam = DBuf(ctx.plan_alloc, sizeof(double) * m);
  e->V = DBuf(ctx.plan_alloc, sizeof(double) * m * m);
  if (ctx.plan_stream && ctx.plan_stream != ctx.stream) {
    // plan memory may have been released by work still queued on the plan allocator's
    // stream: this stream writes it only after that work
    hipEvent_t ev;
    TTIGA_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    TTIGA_HIP(hipEventRecord(ev, ctx.plan_stream));
    TTIGA_HIP(hipStreamWaitEvent(ctx.stream, ev, 0));
    TTIGA_HIP(hipEventDestroy(ev));
  }
  if (k == m) {
    svd_small(ctx, Lc.d(), false, m, m, m, U.d(), e->lam.d(), nullptr, "jacobi_eig");
    hipLaunchKernelGGL(k_square, dim3((m + 255) / 256), dim3(256), 0, ctx.stream, e->lam.d(), m);
    TTIGA_HIP(hipGetLastError());
    gemm(ctx, false, false, m, m, m, 1.0, Rmi.d(), m, 0, U.d(), m, 0, 0.0, e->V.d(), m, 0);
  } else {
    svd_small(ctx, S.d(), false, m, m, m, U.d(), e->lam.d(), W.d());
    gemm(ctx, false, false, m, m, m, 1.0, Rmi.d(), m, 0, W.d(), m, 0, 0.0, e->V.d(), m, 0);
  }
  double* h = ctx.host(2);
  TTIGA_HIP(hipMemcpyAsync(h, e->lam.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  TTIGA_HIP(hipMemcpyAsync(h + 1, e->lam.d() + (m - 1), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();  // the plan is complete before other streams can find it
  e->lam_max = h[0];
  e->lam_min = h[1];
  std::lock_guard<std::mutex> lk(pc.mu);
  auto ins = pc.map.emplace(key, e);
  return std::static_pointer_cast<EigenBasis>(ins.first->second);
}

void Precond::setup(Problem& P) {
  Context& ctx = *P.ctx;
  for (int d = 0; d < 3; ++d) {
    eb[d] = eigenbasis(P, d);
    ni[d] = eb[d]->ni;
    lam_min[d] = eb[d]->lam_min;
    lam_max[d] = eb[d]->lam_max;
  }
  // c_d = mean of R_dd over the parametric cube, from its TT cores
  for (int d = 0; d < 3; ++d) {
    const TT& Rt = P.R[d];
    c[d] = 1.0;
    if (Rt.zero()) continue;
    DBuf v[3];
    for (int k = 0; k < 3; ++k) {
      v[k] = DBuf(ctx.alloc, sizeof(double) * Rt.r[k] * Rt.r[k + 1]);
      hipLaunchKernelGGL(k_weighted_core_sum, dim3((Rt.r[k] * Rt.r[k + 1] + 255) / 256), dim3(256), 0, ctx.stream,
                         Rt.r[k], P.Q[k], Rt.r[k + 1], Rt.c[k].d(), P.tab_w[k].d(), v[k].d());
    }
    TTIGA_HIP(hipGetLastError());
    DBuf t01(ctx.alloc, sizeof(double) * Rt.r[2]), res(ctx.alloc, sizeof(double));
    gemm(ctx, false, false, 1, Rt.r[2], Rt.r[1], 1.0, v[0].d(), Rt.r[1], 0, v[1].d(), Rt.r[2], 0, 0.0, t01.d(), Rt.r[2], 0);
    gemm(ctx, false, false, 1, 1, Rt.r[2], 1.0, t01.d(), Rt.r[2], 0, v[2].d(), 1, 0, 0.0, res.d(), 1, 0);
    double* h = ctx.host(1);
    TTIGA_HIP(hipMemcpyAsync(h, res.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
    ctx.sync();
    if (h[0] > 0.0 && std::isfinite(h[0])) c[d] = h[0];
  }
  // exponential sum for 1/s on [s_min, s_max]: nodes t_k = t_lo + k h, tau = e^t, w = h e^t
  double smin = 0.0, smax = 0.0;
  for (int d = 0; d < 3; ++d) {
    smin += c[d] * std::max(lam_min[d], 0.0);
    smax += c[d] * lam_max[d];
  }
  if (!(smin > 0.0)) smin = 1e-12 * smax;
  s_min = smin;
  s_max = smax;
  const double lo_tail = 0.05, hi_tail = 3.0, target = 0.25;
  std::vector<double> tau, wt;
  for (double h : {4.0, 3.5, 3.0, 2.5, 2.0, 1.6, 1.3, 1.0, 0.8}) {
    tau.clear();
    wt.clear();
    const double t_lo = std::log(lo_tail / smax), t_hi = std::log(hi_tail / smin);
    for (double t = t_lo; t <= t_hi + h; t += h) {
      tau.push_back(std::exp(t));
      wt.push_back(h * std::exp(t));
    }
    double err = 0.0;
    for (int k = 0; k <= 400; ++k) {
      const double s = smin * std::pow(smax / smin, k / 400.0);
      double acc = 0.0;
      for (size_t j = 0; j < tau.size(); ++j) acc += wt[j] * std::exp(-tau[j] * s);
      err = std::max(err, std::fabs(s * acc - 1.0));
    }
    approx_err = err;
    if (err <= target) break;
  }
  R = (int)tau.size();
  std::vector<double> ones(R, 1.0);
  DBuf dtau(ctx.alloc, sizeof(double) * R), dw(ctx.alloc, sizeof(double) * R), d1(ctx.alloc, sizeof(double) * R);
  TTIGA_HIP(hipMemcpyAsync(dtau.d(), tau.data(), sizeof(double) * R, hipMemcpyHostToDevice, ctx.stream));
  TTIGA_HIP(hipMemcpyAsync(dw.d(), wt.data(), sizeof(double) * R, hipMemcpyHostToDevice, ctx.stream));
  TTIGA_HIP(hipMemcpyAsync(d1.d(), ones.data(), sizeof(double) * R, hipMemcpyHostToDevice, ctx.stream));
  for (int d = 0; d < 3; ++d) {
    etab[d] = DBuf(ctx.alloc, sizeof(double) * R * ni[d]);
    hipLaunchKernelGGL(k_exp_table, dim3(grid_for((long)R * ni[d])), dim3(256), 0, ctx.stream, R, ni[d],
                       dtau.d(), d == 0 ? dw.d() : d1.d(), c[d], eb[d]->lam.d(), etab[d].d());
  }
  TTIGA_HIP(hipGetLastError());
  ctx.sync();  // host vectors above go out of scope
  ready = true;
}

void Precond::apply(Context& ctx, const TT& r, TT& z, double eps, int max_rank, int& hint) {
  if (r.zero()) {
    z.set_zero(r.n);
    return;
  }
  TT w;
  tt_copy(ctx, r, w);
  for (int d = 0; d < 3; ++d) tt_mode_product(ctx, w, d, eb[d]->V.d(), true);
  int rr[4] = {1, R * w.r[1], R * w.r[2], 1};
  TT hz;
  hz.alloc(ctx, w.n, rr);
  for (int k = 0; k < 3; ++k) {
    const long total = (long)hz.core_elems(k);
    ProfScope prof(ctx, "precond_scaling", (double)total, 8.0 * (total + (double)w.core_elems(k)));
    hipLaunchKernelGGL(k_exp_hadamard, dim3(grid_for(total)), dim3(256), 0, ctx.stream, k, R, w.n[k],
                       w.r[k], w.r[k + 1], w.c[k].d(), etab[k].d(), hz.c[k].d());
  }
  TTIGA_HIP(hipGetLastError());
  tt_round_auto(ctx, hz, eps, max_rank, hint);
  for (int d = 0; d < 3; ++d) tt_mode_product(ctx, hz, d, eb[d]->V.d(), false);
  z = std::move(hz);
}

}  // namespace ttiga
