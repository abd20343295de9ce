// Accuracy and compression of a TT solution, evaluated in TT format (Section 5).
//
// The relative L2 error of eq. L2norm, with squares and a root (the printed formula has
// neither; its squared-and-rooted form is the relative L2 norm), is
//   ||u_h - u||^2 = sum_q w_q det J_q (u_h(xi_q) - u(x(xi_q)))^2
// over a tensor Gauss grid of p + extra points per knot span.  Everything is a TT on that
// grid: u_h's cores contracted with the B-spline values (exact, the ranks of the solution;
// the interior cores plus the Dirichlet data on the boundary coefficients),
// the exact solution sampled at the mapped points and the weights w0 w1 w2 det J, both
// compressed by TT-SVD at 1e-13.  The difference E = u_h - u is formed as a TT sum and
// rounded by Householder orthogonalisation (no cancellation between the two parts), and
// sum_q W_q E_q^2 is contracted core by core: with L[c][a][a'] the left interface,
//   X[(q d)][(a a')] = sum_c W[c][q][d] L[c][a][a'],
//   T_d[a][q][b'] = sum_a' X[(q d)][a][a'] E[a'][q][b']      (one product per q),
//   L'[d][b][b'] = sum_{a q} E[a][q][b] T_d[a][q][b'],
// all GEMMs of the library's one kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "problem.hpp"

namespace ttiga {

// Tolerance of the compressed exact solution and weights: far below any error worth measuring.
static constexpr double kErrorGridEps = 1e-13;

double tt_weighted_sqnorm(Context& ctx, const TT& E, const TT& W) {
  if (E.zero() || W.zero()) return 0.0;
  DBuf L(ctx.alloc, sizeof(double));
  fill(ctx, L.d(), 1, 1.0);
  for (int k = 0; k < 3; ++k) {
    const int re0 = E.r[k], re1 = E.r[k + 1], rw0 = W.r[k], rw1 = W.r[k + 1], Q = E.n[k];
    TTIGA_CHECK(W.n[k] == Q, TTIGA_E_ARG, "weighted norm: mode sizes differ");
    // X[(q d)][(a a')] = sum_c W[c][(q d)] L[c][(a a')]
    DBuf X(ctx.alloc, sizeof(double) * (size_t)Q * rw1 * re0 * re0);
    gemm(ctx, true, false, Q * rw1, re0 * re0, rw0, 1.0, W.c[k].d(), (long)Q * rw1, 0, L.d(), (long)re0 * re0, 0,
         0.0, X.d(), (long)re0 * re0, 0);
    DBuf Ln(ctx.alloc, sizeof(double) * (size_t)rw1 * re1 * re1);
    DBuf T(ctx.alloc, sizeof(double) * (size_t)re0 * Q * re1);
    for (int d = 0; d < rw1; ++d) {
      // per q: T[a][q][:] = X[(q d)] (re0 x re0) E[:, q, :] (re0 x re1)
      gemm(ctx, false, false, re0, re1, re0, 1.0, X.d() + (size_t)d * re0 * re0, re0, (long)rw1 * re0 * re0,
           E.c[k].d(), (long)Q * re1, re1, 0.0, T.d(), (long)Q * re1, re1, Q);
      // Ln[d] = E^T T over the merged (a q) index
      gemm(ctx, true, false, re1, re1, re0 * Q, 1.0, E.c[k].d(), re1, 0, T.d(), re1, 0, 0.0,
           Ln.d() + (size_t)d * re1 * re1, re1, 0);
    }
    L = std::move(Ln);
  }
  double* h = ctx.host(1);
  TTIGA_HIP(hipMemcpyAsync(h, L.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  return h[0];
}

void Problem::l2_error(int exact_kind, const double* prm, int extra, double out[3]) {
  TTIGA_CHECK(solved, TTIGA_E_STATE, "no solution yet");
  TTIGA_CHECK(exact_kind == TTIGA_EXACT_MANUFACTURED_ANNULUS || exact_kind == TTIGA_EXACT_RADIAL_LOG ||
                  exact_kind == TTIGA_EXACT_SINE_XY,
              TTIGA_E_ARG, "unknown exact solution");
  TTIGA_CHECK(extra >= 0 && p + extra <= 16, TTIGA_E_ARG, "error grid: p + extra must be at most 16");
  ExactDev ex{};
  ex.kind = exact_kind;
  if (exact_kind == TTIGA_EXACT_RADIAL_LOG) {
    TTIGA_CHECK(prm != nullptr, TTIGA_E_ARG, "radial log solution needs r_in, r_out, u_in, u_out");
    for (int i = 0; i < 4; ++i) ex.prm[i] = prm[i];
    TTIGA_CHECK(ex.prm[0] > 0.0 && ex.prm[1] > ex.prm[0], TTIGA_E_ARG, "radial log: need 0 < r_in < r_out");
  }
  Context& c = *ctx;
  const int ge = p + extra;
  int Qe[3];
  DBuf xi[3], w[3], B[3], D[3], span[3], GB[3], GD[3];
  for (int d = 0; d < 3; ++d) {
    Qe[d] = E[d] * ge;
    xi[d] = DBuf(c.alloc, sizeof(double) * Qe[d]);
    w[d] = DBuf(c.alloc, sizeof(double) * Qe[d]);
    B[d] = DBuf(c.alloc, sizeof(double) * Qe[d] * (p + 1));
    D[d] = DBuf(c.alloc, sizeof(double) * Qe[d] * (p + 1));
    launch_basis_tables(c, n[d], p, ge, sknots_d[d].d(), xi[d].d(), w[d].d(), B[d].d(), D[d].d());
    span[d] = DBuf(c.alloc, sizeof(int) * Qe[d]);
    GB[d] = DBuf(c.alloc, sizeof(double) * Qe[d] * (pg[d] + 1));
    GD[d] = DBuf(c.alloc, sizeof(double) * Qe[d] * (pg[d] + 1));
    launch_geo_tables(c, Qe[d], xi[d].d(), 1, m[d], pg[d], gknots_d[d].d(), span[d].as<int>(), GB[d].d(),
                      GD[d].d());
  }
  const GeoDev gd = geo_dev(span, GB, GD);
  const double* wp[3] = {w[0].d(), w[1].d(), w[2].d()};
  // the exact solution (t = 0) and the weights (t = 1) as TTs on the error grid
  TT fac[2];
  DBuf st8(c.alloc, sizeof(double) * 8);
  auto thresholds = [&](std::vector<double>& delta) {
    double* h = c.host(8);
    TTIGA_HIP(hipMemcpyAsync(h, st8.d(), 8 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    TTIGA_CHECK(h[7] > 0.0, TTIGA_E_DETJ, "min det J <= 0 on the error grid");
    delta.assign(2, 0.0);
    for (int t = 0; t < 2; ++t) delta[t] = h[t] == 0.0 ? -1.0 : kErrorGridEps * std::sqrt(h[t]) / std::sqrt(2.0);
  };
  const size_t total = (size_t)Qe[0] * Qe[1] * Qe[2];
  const size_t slab = sizeof(double) * 2 * (size_t)Qe[0] * Qe[2];
  const size_t whole_limit = size_t(2) << 30;
  if (slab * Qe[1] <= whole_limit || Qe[0] <= 64 || (size_t)Qe[1] * Qe[2] <= 64) {
    DBuf G(c.alloc, sizeof(double) * 2 * total);
    launch_exact_grid(c, gd, ex, wp, Qe, 0, Qe[1], G.d(), st8.d());
    std::vector<double> delta;
    thresholds(delta);
    for (int t = 0; t < 2; ++t) {
      if (delta[t] < 0.0) {
        fac[t].set_zero(Qe);
        continue;
      }
      tt_compress_dense(c, G.d() + t * total, Qe, delta[t], fac[t], 0);
    }
  } else {
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>(Qe[1], whole_limit / slab));
    auto produce = [&](int b, int cnt, double* buf) { launch_exact_grid(c, gd, ex, wp, Qe, b, cnt, buf, st8.d()); };
    tt_compress_streamed(c, 2, Qe, chunk, produce, thresholds, fac, 0);
  }
  // the solution on the error grid: its cores times the B-spline values
  TT U;
  if (!u.zero()) {
    U.alloc(c, Qe, u.r);
    for (int d = 0; d < 3; ++d)
      launch_eval_core(c, u.r[d], u.r[d + 1], Qe[d], ge, p, lo[d], hi[d] - lo[d], B[d].d(), u.c[d].d(), U.c[d].d());
  } else {
    U.set_zero(Qe);
  }
  // plus the Dirichlet data on the boundary coefficients (all n of them)
  if (!ug.zero()) {
    TT G, sum;
    G.alloc(c, Qe, ug.r);
    for (int d = 0; d < 3; ++d)
      launch_eval_core(c, ug.r[d], ug.r[d + 1], Qe[d], ge, p, 0, n[d], B[d].d(), ug.c[d].d(), G.c[d].d());
    tt_axpby(c, 1.0, U, 1.0, G, sum);
    U = std::move(sum);
  }
  TT Ediff;
  tt_axpby(c, 1.0, U, -1.0, fac[0], Ediff);
  tt_round(c, Ediff, kErrorGridEps, -1.0, 0);
  const double e2 = tt_weighted_sqnorm(c, Ediff, fac[1]);
  const double u2 = tt_weighted_sqnorm(c, fac[0], fac[1]);
  out[1] = std::sqrt(std::max(e2, 0.0));
  out[2] = std::sqrt(std::max(u2, 0.0));
  out[0] = out[2] > 0.0 ? out[1] / out[2] : 0.0;
}

// Compression ratios of the assembled operator and load vector and of the solution (full
// grid entries over TT entries): K against its sparse IGA matrix (the Kronecker pattern of
// 1-D bands, prod_d (n_d (2p+1) - p (p+1)) non-zeros) and against the dense N x N matrix;
// F against N values; u against the N_I interior values.
void Problem::compression_ratios(double out[4]) {
  TTIGA_CHECK(assembled, TTIGA_E_STATE, "problem not assembled");
  const int band = 2 * p + 1;
  double nnz = 1.0, N = 1.0, NI = 1.0, k_tt = 0.0, k_dense_tt = 0.0, f_tt = 0.0, u_tt = 0.0;
  for (int d = 0; d < 3; ++d) {
    nnz *= (double)n[d] * band - (double)p * (p + 1);
    N *= n[d];
    NI *= hi[d] - lo[d];
    k_tt += (double)K.r[d] * n[d] * band * K.r[d + 1];
    k_dense_tt += (double)K.r[d] * n[d] * n[d] * K.r[d + 1];
    f_tt += (double)F.r[d] * n[d] * F.r[d + 1];
    if (solved) u_tt += (double)u.r[d] * u.n[d] * u.r[d + 1];
  }
  out[0] = k_tt > 0.0 ? nnz / k_tt : 0.0;
  out[1] = k_dense_tt > 0.0 ? N * N / k_dense_tt : 0.0;
  out[2] = f_tt > 0.0 ? N / f_tt : 0.0;
  out[3] = u_tt > 0.0 ? NI / u_tt : 0.0;
}

}  // namespace ttiga
