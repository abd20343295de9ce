// Problem description, assembly driver and TT solve.
//
// Assembly (Sections 4.2-4.3):
//   1. per direction, Gauss nodes/weights on the solution spans and the solution
//      and geometry B-spline tables there;
//   2. the seven factor tensors R_00..R_12, f det J on the Gauss grid (eq. Rxi, ffinal);
//   3. TT-SVD of each factor: R components to a threshold relative to the largest
//      ||R_ij||_F (identically vanishing components become rank 0), f det J
//      relative to its own norm;
//   4. banded TT-matrix cores of the nine K_ij (selector a_ij^(d)), summed with
//      TT-rounding after each addition; TT cores of F;
//   5. Dirichlet indices cut from the cores; constant face data lifted into the
//      right-hand side F_I - (K u_g)_I.
// Solve: conjugate gradients on TT tensors with TT-rounding of every update
// (truncated TT-CG), true-residual replacement every 10 iterations and at the
// stopping test.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "iga.hpp"

#include "problem.hpp"

namespace ttiga {

static const int kTermOrder[9][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 0},
                                     {0, 2}, {2, 0}, {1, 2}, {2, 1}};

static int r_index(int i, int j) {
  const int a = std::min(i, j), b = std::max(i, j);
  static const int tab[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
  return tab[a][b];
}

static double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

static void check_knots(const double* k, int len, int p) {
  TTIGA_CHECK(k != nullptr, TTIGA_E_ARG, "null knot vector");
  for (int i = 0; i + 1 < len; ++i)
    TTIGA_CHECK(k[i] <= k[i + 1], TTIGA_E_KNOTS, "knot vector is not non-decreasing");
  for (int i = 0; i <= p; ++i) {
    TTIGA_CHECK(k[i] == k[0], TTIGA_E_KNOTS, "knot vector start multiplicity != p+1");
    TTIGA_CHECK(k[len - 1 - i] == k[len - 1], TTIGA_E_KNOTS, "knot vector end multiplicity != p+1");
  }
  TTIGA_CHECK(k[p + 1] > k[0] || len == 2 * (p + 1), TTIGA_E_KNOTS,
              "knot vector end multiplicity exceeds p+1");
  TTIGA_CHECK(k[len - p - 2] < k[len - 1] || len == 2 * (p + 1), TTIGA_E_KNOTS,
              "knot vector end multiplicity exceeds p+1");
  TTIGA_CHECK(k[0] == 0.0 && k[len - 1] == 1.0, TTIGA_E_KNOTS, "knot vectors must span [0, 1]");
}

Problem::Problem(Context* c, const ttiga_geometry* geo, const ttiga_discretization* disc,
                 const ttiga_source* src, const ttiga_dirichlet* bc, const ttiga_options* opt)
    : ctx(c) {
  TTIGA_CHECK(geo && disc && src && bc && opt, TTIGA_E_ARG, "null problem description");
  // geometry
  size_t nctrl = 1;
  for (int d = 0; d < 3; ++d) {
    pg[d] = geo->degree[d];
    m[d] = geo->n_ctrl[d];
    TTIGA_CHECK(pg[d] >= 1 && pg[d] <= 8, TTIGA_E_ARG, "geometry degree must be in [1, 8]");
    TTIGA_CHECK(m[d] >= pg[d] + 1, TTIGA_E_ARG, "geometry needs n_ctrl >= degree + 1");
    const int len = m[d] + pg[d] + 1;
    check_knots(geo->knots[d], len, pg[d]);
    gknots[d].assign(geo->knots[d], geo->knots[d] + len);
    nctrl *= (size_t)m[d];
  }
  TTIGA_CHECK(geo->ctrl_xyz != nullptr, TTIGA_E_ARG, "null control points");
  ctrl.assign(geo->ctrl_xyz, geo->ctrl_xyz + 3 * nctrl);
  weights.assign(nctrl, 1.0);
  if (geo->weights) {
    weights.assign(geo->weights, geo->weights + nctrl);
    for (double w : weights) TTIGA_CHECK(w > 0.0 && std::isfinite(w), TTIGA_E_GEOM, "weights must be positive");
  }
  for (double v : ctrl) TTIGA_CHECK(std::isfinite(v), TTIGA_E_GEOM, "non-finite control point");
  // discretisation
  p = disc->degree;
  TTIGA_CHECK(p >= 1 && p <= 8, TTIGA_E_ARG, "solution degree must be in [1, 8]");
  g = disc->n_gauss > 0 ? disc->n_gauss : p + 1;
  TTIGA_CHECK(g >= 1 && g <= 8, TTIGA_E_ARG, "n_gauss must be in [0, 8]");
  for (int d = 0; d < 3; ++d) {
    n[d] = disc->n_basis[d];
    TTIGA_CHECK(n[d] >= p + 1, TTIGA_E_ARG, "n_basis must be >= degree + 1");
    TTIGA_CHECK(n[d] <= (1 << 20), TTIGA_E_ARG, "n_basis too large");
    E[d] = n[d] - p;
    Q[d] = E[d] * g;
  }
  // source
  src_kind = src->kind;
  TTIGA_CHECK(src_kind == TTIGA_SOURCE_ZERO || src_kind == TTIGA_SOURCE_MANUFACTURED_ANNULUS ||
                  src_kind == TTIGA_SOURCE_FOURIER,
              TTIGA_E_ARG, "unknown source kind");
  if (src_kind == TTIGA_SOURCE_FOURIER) {
    TTIGA_CHECK(src->n_modes >= 0 && src->n_modes <= 4096, TTIGA_E_ARG, "bad n_modes");
    TTIGA_CHECK(src->n_modes == 0 || (src->a && src->k && src->phi), TTIGA_E_ARG, "null Fourier data");
    TTIGA_CHECK(src->scale > 0.0, TTIGA_E_ARG, "Fourier scale must be positive");
    src_a.assign(src->a, src->a + src->n_modes);
    src_k.assign(src->k, src->k + 3 * src->n_modes);
    src_phi.assign(src->phi, src->phi + src->n_modes);
  }
  for (int d = 0; d < 3; ++d) src_origin[d] = src->origin[d];
  src_scale = src->scale > 0.0 ? src->scale : 1.0;
  // boundary data
  for (int f = 0; f < 6; ++f) {
    bc_kind[f] = bc->kind[f];
    bc_value[f] = bc->value[f];
    TTIGA_CHECK(bc_kind[f] >= TTIGA_BC_NATURAL && bc_kind[f] <= TTIGA_BC_TRACTION, TTIGA_E_ARG,
                "unknown boundary kind");
  }
  // constant data on any faces: lifted by a TT of rank at most the number of such faces
  lift = false;
  for (int f = 0; f < 6; ++f) lift = lift || (bc_kind[f] == TTIGA_BC_CONSTANT && bc_value[f] != 0.0);
  for (int d = 0; d < 3; ++d) {
    lo[d] = is_dirichlet(bc_kind[2 * d]) ? 1 : 0;
    hi[d] = is_dirichlet(bc_kind[2 * d + 1]) ? n[d] - 1 : n[d];
    TTIGA_CHECK(hi[d] - lo[d] >= 1, TTIGA_E_ARG, "no interior unknowns");
  }
  // options
  opts = *opt;
  TTIGA_CHECK(opts.tt_eps > 0.0 && opts.tt_eps < 1.0, TTIGA_E_ARG, "tt_eps must be in (0, 1)");
  TTIGA_CHECK(opts.assembly_eps >= 0.0 && opts.assembly_eps < 1.0, TTIGA_E_ARG, "assembly_eps must be in [0, 1)");
  TTIGA_CHECK(opts.rel_res_tol > 0.0, TTIGA_E_ARG, "rel_res_tol must be positive");
  TTIGA_CHECK(opts.max_iter > 0, TTIGA_E_ARG, "max_iter must be positive");
  TTIGA_CHECK(opts.precision == TTIGA_FP64 || opts.precision == TTIGA_FP32 || opts.precision == TTIGA_BF16,
              TTIGA_E_ARG, "precision must be TTIGA_FP64, TTIGA_FP32 or TTIGA_BF16");
  TTIGA_CHECK(opts.precision == TTIGA_FP64 || opts.precond == 1, TTIGA_E_ARG,
              "mixed precision refines around the preconditioned solver (precond = 1)");
  if (opts.max_rank <= 0) opts.max_rank = 1 << 20;
}

void Problem::upload() {
  Context& c = *ctx;
  const size_t nctrl = (size_t)m[0] * m[1] * m[2];
  DBuf xyz(c.alloc, sizeof(double) * 3 * nctrl), w(c.alloc, sizeof(double) * nctrl);
  TTIGA_HIP(hipMemcpyAsync(xyz.d(), ctrl.data(), sizeof(double) * 3 * nctrl, hipMemcpyHostToDevice, c.stream));
  TTIGA_HIP(hipMemcpyAsync(w.d(), weights.data(), sizeof(double) * nctrl, hipMemcpyHostToDevice, c.stream));
  Pw = DBuf(c.alloc, sizeof(double) * 4 * nctrl);
  launch_homogeneous(c, (long)nctrl, xyz.d(), w.d(), Pw.d());
  // host sources of the asynchronous copies below: they must outlive the copies, so they live
  // until the stream has drained at the end of this function
  std::vector<double> knots_h[3], modes_h;
  for (int d = 0; d < 3; ++d) {
    gknots_d[d] = DBuf(c.alloc, sizeof(double) * gknots[d].size());
    TTIGA_HIP(hipMemcpyAsync(gknots_d[d].d(), gknots[d].data(), sizeof(double) * gknots[d].size(),
                             hipMemcpyHostToDevice, c.stream));
    // open uniform solution knots: p+1 zeros, e/E for e = 1..E-1, p+1 ones
    std::vector<double>& kn = knots_h[d];
    kn.resize(n[d] + p + 1);
    for (int i = 0; i < (int)kn.size(); ++i) {
      const int e = std::min(std::max(i - p, 0), E[d]);
      kn[i] = (e == E[d]) ? 1.0 : (double)e / E[d];
    }
    sknots_d[d] = DBuf(c.alloc, sizeof(double) * kn.size());
    TTIGA_HIP(hipMemcpyAsync(sknots_d[d].d(), kn.data(), sizeof(double) * kn.size(),
                             hipMemcpyHostToDevice, c.stream));
  }
  const int nm = (int)src_a.size();
  if (nm > 0) {
    modes_d = DBuf(c.alloc, sizeof(double) * 5 * nm);
    std::vector<double>& h = modes_h;
    h.resize(5 * nm);
    std::memcpy(h.data(), src_a.data(), sizeof(double) * nm);
    std::memcpy(h.data() + nm, src_k.data(), sizeof(double) * 3 * nm);
    std::memcpy(h.data() + 4 * nm, src_phi.data(), sizeof(double) * nm);
    TTIGA_HIP(hipMemcpyAsync(modes_d.d(), h.data(), sizeof(double) * 5 * nm, hipMemcpyHostToDevice, c.stream));
  }
  c.sync();  // the host vectors above go out of scope after this
}

SourceDev Problem::source_dev() const {
  SourceDev s{};
  s.kind = src_kind;
  s.n_modes = (int)src_a.size();
  if (s.n_modes > 0) {
    s.a = modes_d.d();
    s.k = modes_d.d() + s.n_modes;
    s.phi = modes_d.d() + 4 * s.n_modes;
  }
  for (int d = 0; d < 3; ++d) s.origin[d] = src_origin[d];
  s.scale = src_scale;
  s.int_kmax = -1;
  if (src_kind == TTIGA_SOURCE_FOURIER) {
    int km = 0;
    bool integral = true;
    for (double v : src_k) {
      if (!(std::fabs(v) <= kMaxIntWave) || v != std::floor(v)) integral = false;
      else km = std::max(km, (int)std::fabs(v));
    }
    if (integral) s.int_kmax = km;
  }
  return s;
}

void Problem::build_tables() {
  Context& c = *ctx;
  for (int d = 0; d < 3; ++d) {
    const int Qd = Q[d];
    tab_xi[d] = DBuf(c.alloc, sizeof(double) * Qd);
    tab_w[d] = DBuf(c.alloc, sizeof(double) * Qd);
    tab_B[d] = DBuf(c.alloc, sizeof(double) * Qd * (p + 1));
    tab_D[d] = DBuf(c.alloc, sizeof(double) * Qd * (p + 1));
    launch_basis_tables(c, n[d], p, g, sknots_d[d].d(), tab_xi[d].d(), tab_w[d].d(), tab_B[d].d(),
                        tab_D[d].d());
    gtab_span[d] = DBuf(c.alloc, sizeof(int) * Qd);
    gtab_B[d] = DBuf(c.alloc, sizeof(double) * Qd * (pg[d] + 1));
    gtab_D[d] = DBuf(c.alloc, sizeof(double) * Qd * (pg[d] + 1));
    launch_geo_tables(c, Qd, tab_xi[d].d(), 1, m[d], pg[d], gknots_d[d].d(), gtab_span[d].as<int>(),
                      gtab_B[d].d(), gtab_D[d].d());
  }
}

GeoDev Problem::geo_dev(const DBuf* span, const DBuf* B, const DBuf* D) const {
  GeoDev gd{};
  for (int d = 0; d < 3; ++d) {
    gd.pg[d] = pg[d];
    gd.m[d] = m[d];
    gd.span[d] = span[d].as<int>();
    gd.B[d] = B[d].d();
    gd.D[d] = D[d].d();
  }
  gd.Pw = Pw.d();
  return gd;
}

// Host-side index choices of the cross approximation (columns, extra rows, probe points)
// come from a SplitMix64 stream seeded from the context counter, which restarts at every
// assembly, so they do not depend on what ran before.
static uint64_t splitmix(uint64_t& state) {
  uint64_t z = (state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// idx0[e], idx1[e], idx2[e] for e = (x a1 + y) a2 + z: the grid points of the product of three
// index lists (a null list: 0 .. a-1)
__global__ void k_product_indices(int a0, int a1, int a2, const int* __restrict__ L0, const int* __restrict__ L1,
                                  const int* __restrict__ L2, int* __restrict__ i0, int* __restrict__ i1,
                                  int* __restrict__ i2) {
  const long total = (long)a0 * a1 * a2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int z = (int)(e % a2);
    const long t = e / a2;
    const int y = (int)(t % a1), x = (int)(t / a1);
    i0[e] = L0 ? L0[x] : x;
    i1[e] = L1 ? L1[y] : y;
    i2[e] = L2 ? L2[z] : z;
  }
}

// The seven factors at the product of three index lists (device lists, null: the whole range),
// into out[7][a0 a1 a2].
static void sample_product(Context& c, const GeoDev& gd, const SourceDev& sd, const int* L0, int a0, const int* L1,
                           int a1, const int* L2, int a2, double* out) {
  const long cnt = (long)a0 * a1 * a2;
  DBuf idx(c.alloc, sizeof(int) * 3 * cnt);
  int* di = idx.as<int>();
  hipLaunchKernelGGL(k_product_indices, dim3(grid_for(cnt)), dim3(256), 0, c.stream, a0, a1, a2, L0, L1, L2, di,
                     di + cnt, di + 2 * cnt);
  TTIGA_HIP(hipGetLastError());
  launch_factors_at(c, gd, sd, cnt, di, di + cnt, di + 2 * cnt, out, nullptr);
}

// Second level of the cross approximation: with the first-mode bases U_t (Q0 x k_t), the
// interpolation rows I and P_t^+ = U_t[I, :]^+, the coefficient tensor X_t = P_t^+ A_t[I, :, :]
// (k_t x Q1 x Q2) is approximated in the same way along its last mode instead of being formed:
//  a. L2 random third-direction indices j: the fibres X_t[:, :, j] from the samples A[I, :, j]
//     (|I| Q1 L2 points), their column basis V_t ((k_t Q1) x k2_t, truncated at 0.1 eps of the
//     largest metric sample scale), L2 doubling while a rank comes within 12 of it;
//  b. interpolation rows R_t of V_t (pivoted Gram-Schmidt on its rows, as for U_t); the rows
//     (a, i1) need the samples A[I, i1, :] for the distinct i1 of all R_t plus 8 random ones
//     (|I| |S| Q2 points), giving X_t[R_t, :];
//  c. X_t ~= V_t D_t with D_t the least-squares solution over all the sampled rows (a, i1),
//     i1 in S, of X_t (k_t |S| rows: the pivots and the rest of their slices, an oversampling
//     that keeps the interpolation well conditioned); the TT of the factor is (U_t, V_t as
//     k_t x Q1 x k2_t, D_t), rounded at eps of its scale like the TT-SVD path.
// Declines (the caller samples the whole slices) when a basis comes within 12 of its largest
// sample, when the sampled rows of V_t are ill-conditioned or when the grid is too small for it
// to pay; the caller also takes the slices when the result fails the probe check.
bool Problem::cross_second_level(const GeoDev& gd, const SourceDev& sd, TT* fac, ttiga_assembly_stats& s,
                                 const std::vector<DBuf>& U, const std::vector<int>& k, const std::vector<int>& I,
                                 const DBuf& Id, const std::vector<DBuf>& Pinv, double* scale, uint64_t& rs) {
  Context& c = *ctx;
  const int n1 = Q[1], n2 = Q[2];
  const int nI = (int)I.size();
  const double eps = assembly_eps();
  auto rnd = [&](int hi) { return (int)(splitmix(rs) % (uint64_t)hi); };
  const int cap = std::min(n2 / 2, 256);
  if (cap < 32 || n1 < 8) return false;
  int L2 = std::min(cap, 48);
  std::vector<DBuf> V(7);
  std::vector<int> k2(7, 0);
  while (true) {
    // a. the fibres A[i0, i1, j] for i0 in I, all i1, the L2 chosen j
    std::vector<int> J(L2);
    for (int q = 0; q < L2; ++q) J[q] = rnd(n2);
    const long cnt = (long)nI * n1 * L2;
    DBuf Jd(c.alloc, sizeof(int) * L2), Af(c.alloc, sizeof(double) * 7 * cnt);
    TTIGA_HIP(hipMemcpyAsync(Jd.d(), J.data(), sizeof(int) * L2, hipMemcpyHostToDevice, c.stream));
    sample_product(c, gd, sd, Id.as<int>(), nI, nullptr, n1, Jd.as<int>(), L2, Af.d());
    s.samples += cnt;
    // C_t = P_t^+ A_t[I, :, J]: (k_t) x (Q1 L2), read as (k_t Q1) x L2
    std::vector<DBuf> C(7);
    DBuf csq(c.alloc, sizeof(double) * 7);
    fill(c, csq.d(), 7, 0.0);
    for (int t = 0; t < 7; ++t) {
      if (!k[t]) continue;
      C[t] = DBuf(c.alloc, sizeof(double) * (size_t)k[t] * n1 * L2);
      gemm(c, false, false, k[t], n1 * L2, nI, 1.0, Pinv[t].d(), nI, 0, Af.d() + (size_t)t * cnt, (long)n1 * L2, 0,
           0.0, C[t].d(), (long)n1 * L2, 0);
      sumsq_reduce(c, C[t].d(), (size_t)k[t] * n1 * L2, csq.d() + t);
    }
    double* hc = c.host(7);
    TTIGA_HIP(hipMemcpyAsync(hc, csq.d(), 7 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();  // J goes out of scope
    double cmax = 0.0;
    for (int t = 0; t < 6; ++t) cmax = std::max(cmax, std::sqrt(std::max(hc[t], 0.0)));
    bool saturated = false;
    for (int t = 0; t < 7; ++t) {
      const double cs = t < 6 ? cmax : std::sqrt(std::max(hc[6], 0.0));
      k2[t] = (k[t] && cs > 0.0 && (long)k[t] * n1 >= L2) ? column_basis(c, C[t].d(), k[t] * n1, L2, 0.1 * eps * cs, V[t])
                                                         : 0;
      if (k[t] && (long)k[t] * n1 < L2) return false;
      if (k2[t] > L2 - 12) saturated = true;
    }
    if (!saturated) break;
    if (L2 == cap) return false;
    L2 = std::min(cap, 2 * L2);
  }
  // b. interpolation rows (a, i1) of each V_t; the distinct i1 of all of them plus 8 random
  std::vector<std::vector<int>> R(7);
  std::vector<char> pick(n1, 0);
  for (int t = 0; t < 7; ++t) {
    if (!k2[t]) continue;
    DBuf rows(c.alloc, sizeof(int) * k2[t]);
    pivot_rows(c, V[t].d(), k[t] * n1, k2[t], rows.as<int>());
    R[t].resize(k2[t]);
    TTIGA_HIP(hipMemcpyAsync(R[t].data(), rows.d(), sizeof(int) * k2[t], hipMemcpyDeviceToHost, c.stream));
    c.sync();
    for (int r : R[t]) pick[r % n1] = 1;
  }
  for (int e = 0; e < 8; ++e) pick[rnd(n1)] = 1;
  std::vector<int> S;
  for (int i1 = 0; i1 < n1; ++i1)
    if (pick[i1]) S.push_back(i1);
  const int nS = (int)S.size();
  if (2 * nS > n1) return false;
  // the samples A[i0, i1, :] for i0 in I, i1 in S; E_t = P_t^+ A_t[I, S, :] (k_t x |S| Q2)
  const long cnt = (long)nI * nS * n2;
  DBuf Sd(c.alloc, sizeof(int) * nS), As(c.alloc, sizeof(double) * 7 * cnt);
  TTIGA_HIP(hipMemcpyAsync(Sd.d(), S.data(), sizeof(int) * nS, hipMemcpyHostToDevice, c.stream));
  sample_product(c, gd, sd, Id.as<int>(), nI, Sd.as<int>(), nS, nullptr, n2, As.d());
  s.samples += cnt;
  c.sync();  // S may go out of scope
  // c. D_t = V_t[S_t, :]^+ X_t[S_t, :], least squares over every sampled row (a, i1 in S) of X_t
  // (k_t |S| rows, the pivots R_t among them), and the TT (U_t, V_t, D_t)
  double nrm[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int t = 0; t < 7; ++t) {
    if (!k2[t]) {
      fac[t].set_zero(Q);
      continue;
    }
    const int kt = k[t], k2t = k2[t], ms = kt * nS;
    if (ms < k2t) return false;
    // E = P_t^+ A_t[I, S, :]: k_t x |S| Q2, read as (k_t |S|) x Q2 with row a |S| + q
    DBuf E(c.alloc, sizeof(double) * (size_t)ms * n2);
    gemm(c, false, false, kt, nS * n2, nI, 1.0, Pinv[t].d(), nI, 0, As.d() + (size_t)t * cnt, (long)nS * n2, 0, 0.0,
         E.d(), (long)nS * n2, 0);
    // the same rows of V_t: row a Q1 + S[q]
    std::vector<int> vr(ms);
    for (int a = 0; a < kt; ++a)
      for (int q = 0; q < nS; ++q) vr[(size_t)a * nS + q] = a * n1 + S[q];
    DBuf vrd(c.alloc, sizeof(int) * ms), VS(c.alloc, sizeof(double) * (size_t)ms * k2t);
    TTIGA_HIP(hipMemcpyAsync(vrd.d(), vr.data(), sizeof(int) * ms, hipMemcpyHostToDevice, c.stream));
    gather_rows(c, V[t].d(), k2t, vrd.as<int>(), ms, VS.d());
    // V_S = Qv Rv, Rv = Ur diag(sv) Wr^T: D = Wr diag(1/sv) Ur^T Qv^T E
    DBuf Qv(c.alloc, sizeof(double) * (size_t)ms * k2t), Rv(c.alloc, sizeof(double) * k2t * k2t),
        Ur(c.alloc, sizeof(double) * k2t * k2t), Sv(c.alloc, sizeof(double) * k2t), Wr(c.alloc, sizeof(double) * k2t * k2t);
    qr_tall(c, VS.d(), false, ms, k2t, k2t, Qv.d(), Rv.d());
    svd_small(c, Rv.d(), false, k2t, k2t, k2t, Ur.d(), Sv.d(), Wr.d());
    double* h = c.host(2);
    TTIGA_HIP(hipMemcpyAsync(h, Sv.d(), sizeof(double), hipMemcpyDeviceToHost, c.stream));
    TTIGA_HIP(hipMemcpyAsync(h + 1, Sv.d() + (k2t - 1), sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();  // vr goes out of scope
    if (!(h[1] > 1e-8 * h[0])) return false;
    DBuf T1(c.alloc, sizeof(double) * (size_t)k2t * n2), T2(c.alloc, sizeof(double) * (size_t)k2t * n2),
        WS(c.alloc, sizeof(double) * k2t * k2t);
    gemm(c, true, false, k2t, n2, ms, 1.0, Qv.d(), k2t, 0, E.d(), n2, 0, 0.0, T1.d(), n2, 0);
    gemm(c, true, false, k2t, n2, k2t, 1.0, Ur.d(), k2t, 0, T1.d(), n2, 0, 0.0, T2.d(), n2, 0);
    scale_cols_inv(c, Wr.d(), k2t, k2t, Sv.d(), WS.d());
    TT tt;
    const int rr[4] = {1, kt, k2t, 1};
    tt.alloc(c, Q, rr);
    copy(c, tt.c[0].d(), U[t].d(), (size_t)Q[0] * kt);
    copy(c, tt.c[1].d(), V[t].d(), (size_t)kt * n1 * k2t);
    gemm(c, false, false, k2t, n2, k2t, 1.0, WS.d(), k2t, 0, T2.d(), n2, 0, 0.0, tt.c[2].d(), n2, 0);
    nrm[t] = std::sqrt(std::max(tt_dot_sync(c, tt, tt), 0.0));
    fac[t] = std::move(tt);
  }
  double rmax = 0.0;
  for (int t = 0; t < 6; ++t) rmax = std::max(rmax, nrm[t]);
  s.max_R_norm = rmax;
  for (int t = 0; t < 7; ++t) scale[t] = t < 6 ? rmax : nrm[6];
  for (int t = 0; t < 7; ++t) {
    if (fac[t].zero()) continue;
    if (scale[t] == 0.0) {
      fac[t].set_zero(Q);
      continue;
    }
    tt_round(c, fac[t], 0.0, eps * scale[t] / std::sqrt(2.0), opts.max_rank);
  }
  return true;
}

// Cross approximation of the first unfolding A_(0) (Q0 x Q1 Q2) of the seven factors, the
// sampled-entries alternative to full-grid TT-SVD (the role TT-cross plays in the paper):
//  1. L random columns (fibres along the first direction, shared by the factors); per
//     factor the orthonormal basis U of their span (truncated SVD at 1e-2 eps relative);
//     a basis within 8 of L means the columns may miss directions: L doubles;
//  2. interpolation rows: the pivoted rows of each U (column-pivoted QR of U^T), their
//     union I plus 8 random rows;
//  3. X = U[I, :]^+ A[I, :], so that A_(0) ~= U X (interpolation through the rows I): by a
//     second level of the same construction along the last mode (cross_second_level), or
//     from the slices A[I, :, :] only (|I| of Q0), streamed in second-direction chunks, when
//     the second level declines or its result fails the probe check of step 5;
//  4. ||A||_F ~= ||X||_F sets the thresholds; U, X continue as in TT-SVD (truncated SVD
//     of X, dense factorisation of the rest);
//  5. 2048 random grid points compare the TTs with directly sampled values: a factor
//     off by more than 10 eps (its threshold scale, RMS per point) rejects the result
//     and the caller falls back to TT-SVD.
bool Problem::compress_cross(const GeoDev& gd, const SourceDev& sd, TT* fac, ttiga_assembly_stats& s) {
  Context& c = *ctx;
  const int n0 = Q[0], n1 = Q[1], n2 = Q[2];
  const long M = (long)n1 * n2;
  const double eps = assembly_eps();
  uint64_t rs = c.rng_counter;
  auto rnd = [&](int hi) { return (int)(splitmix(rs) % (uint64_t)hi); };
  static const bool trace = [] {
    const char* e = std::getenv("TTIGA_TRACE_CROSS");
    return e && e[0] == '1';
  }();
  auto reject = [&](const char* why) {
    if (trace) std::fprintf(stderr, "[cross] rejected: %s\n", why);
    return false;
  };
  const int cap = std::min(n0 / 2, 256);
  int L = std::min(cap, 48);
  std::vector<DBuf> U(7);
  std::vector<int> k(7, 0);
  while (true) {
    // 1. column fibres
    std::vector<int> hi0((size_t)n0 * L), hi1((size_t)n0 * L), hi2((size_t)n0 * L);
    for (int j = 0; j < L; ++j) {
      const int a = rnd(n1), b = rnd(n2);
      for (int i = 0; i < n0; ++i) {
        hi0[(size_t)i * L + j] = i;
        hi1[(size_t)i * L + j] = a;
        hi2[(size_t)i * L + j] = b;
      }
    }
    const long cnt = (long)n0 * L;
    DBuf idx(c.alloc, sizeof(int) * 3 * cnt), Cf(c.alloc, sizeof(double) * 7 * cnt);
    int* di = idx.as<int>();
    TTIGA_HIP(hipMemcpyAsync(di, hi0.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, c.stream));
    TTIGA_HIP(hipMemcpyAsync(di + cnt, hi1.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, c.stream));
    TTIGA_HIP(hipMemcpyAsync(di + 2 * cnt, hi2.data(), sizeof(int) * cnt, hipMemcpyHostToDevice, c.stream));
    launch_factors_at(c, gd, sd, cnt, di, di + cnt, di + 2 * cnt, Cf.d(), nullptr);
    s.samples += cnt;
    c.sync();  // the host index arrays go out of scope
    // the metric entries share one scale (the largest of their samples), as in the TT-SVD
    // thresholds: an entry that vanishes analytically is sampled as roundoff and must
    // come out empty, not as a full-rank basis of noise
    DBuf csq(c.alloc, sizeof(double) * 7);
    fill(c, csq.d(), 7, 0.0);
    for (int t = 0; t < 7; ++t) sumsq_reduce(c, Cf.d() + (size_t)t * cnt, (size_t)cnt, csq.d() + t);
    double* hc = c.host(7);
    TTIGA_HIP(hipMemcpyAsync(hc, csq.d(), 7 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    double cmax = 0.0;
    for (int t = 0; t < 6; ++t) cmax = std::max(cmax, std::sqrt(std::max(hc[t], 0.0)));
    const double cscale[7] = {cmax, cmax, cmax, cmax, cmax, cmax, std::sqrt(std::max(hc[6], 0.0))};
    bool saturated = false;
    if (n0 > L) {
      // the seven bases in batched factorisations (the same bits as one at a time)
      double dl[7];
      for (int t = 0; t < 7; ++t) dl[t] = 0.1 * eps * cscale[t];
      int kb[7];
      DBuf Ub[7];
      column_basis_batched(c, 7, Cf.d(), cnt, n0, L, dl, kb, Ub);
      for (int t = 0; t < 7; ++t) {
        k[t] = cscale[t] > 0.0 ? kb[t] : 0;
        if (k[t] > 0) U[t] = std::move(Ub[t]);
      }
    } else {
      for (int t = 0; t < 7; ++t)
        k[t] = cscale[t] > 0.0 ? column_basis(c, Cf.d() + (size_t)t * cnt, n0, L, 0.1 * eps * cscale[t], U[t]) : 0;
    }
    for (int t = 0; t < 7; ++t)
      if (k[t] > L - 8) saturated = true;
    if (trace)
      std::fprintf(stderr, "[cross] L %d column ranks %d %d %d %d %d %d %d\n", L, k[0], k[1], k[2], k[3], k[4], k[5],
                   k[6]);
    if (!saturated) break;
    if (L == cap) return reject("column ranks saturate the largest sample");
    L = std::min(cap, 2 * L);
  }
  // 2. interpolation rows
  std::vector<char> pick(n0, 0);
  for (int t = 0; t < 7; ++t) {
    if (k[t] == 0) continue;
    DBuf rows(c.alloc, sizeof(int) * k[t]);
    pivot_rows(c, U[t].d(), n0, k[t], rows.as<int>());
    std::vector<int> hr(k[t]);
    TTIGA_HIP(hipMemcpyAsync(hr.data(), rows.d(), sizeof(int) * k[t], hipMemcpyDeviceToHost, c.stream));
    c.sync();
    for (int r : hr) pick[r] = 1;
  }
  for (int e = 0; e < 8; ++e) pick[rnd(n0)] = 1;
  std::vector<int> I;
  for (int i = 0; i < n0; ++i)
    if (pick[i]) I.push_back(i);
  const int nI = (int)I.size();
  if (trace) std::fprintf(stderr, "[cross] %d interpolation rows of %d\n", nI, n0);
  if (2 * nI > n0) return reject("interpolation rows cover half the grid");
  DBuf Id(c.alloc, sizeof(int) * nI);
  TTIGA_HIP(hipMemcpyAsync(Id.d(), I.data(), sizeof(int) * nI, hipMemcpyHostToDevice, c.stream));
  // interpolation operators X = P^+ A[I, :] with P = U[I, :] (|I| x k)
  std::vector<DBuf> Pinv(7), X(7);
  for (int t = 0; t < 7; ++t) {
    if (k[t] == 0) continue;
    const int kt = k[t];
    DBuf P(c.alloc, sizeof(double) * nI * kt), Up(c.alloc, sizeof(double) * nI * kt),
        Sp(c.alloc, sizeof(double) * kt), Vp(c.alloc, sizeof(double) * kt * kt);
    gather_rows(c, U[t].d(), kt, Id.as<int>(), nI, P.d());
    svd_small(c, P.d(), false, nI, kt, kt, Up.d(), Sp.d(), Vp.d());
    double* h = c.host(2);
    TTIGA_HIP(hipMemcpyAsync(h, Sp.d(), sizeof(double), hipMemcpyDeviceToHost, c.stream));
    TTIGA_HIP(hipMemcpyAsync(h + 1, Sp.d() + (kt - 1), sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    if (!(h[1] > 1e-8 * h[0])) return reject("interpolation rows do not determine the basis");
    // P^+ = V S^-1 U^T
    DBuf VS(c.alloc, sizeof(double) * kt * kt);
    scale_cols_inv(c, Vp.d(), kt, kt, Sp.d(), VS.d());
    Pinv[t] = DBuf(c.alloc, sizeof(double) * kt * nI);
    gemm(c, false, true, kt, nI, kt, 1.0, VS.d(), kt, 0, Up.d(), kt, 0, 0.0, Pinv[t].d(), nI, 0);
  }
  double scale[7];
  // the whole-slice path of step 3
  auto slices = [&]() {
    for (int t = 0; t < 7; ++t)
      if (k[t]) X[t] = DBuf(c.alloc, sizeof(double) * (size_t)k[t] * M);
    {
      const size_t slab = sizeof(double) * 7 * (size_t)nI * n2;
      const int chunk = (int)std::max<size_t>(1, std::min<size_t>(n1, (size_t(2) << 30) / slab));
      DBuf buf(c.alloc, slab * chunk), st(c.alloc, sizeof(double) * 8);
      for (int b = 0; b < n1; b += chunk) {
        const int cn = std::min(chunk, n1 - b);
        const long w = (long)cn * n2;
        launch_factors_grid(c, gd, sd, Q, b, cn, buf.d(), st.d(), false, Id.as<int>(), nI);
        for (int t = 0; t < 7; ++t)
          if (k[t])
            gemm(c, false, false, k[t], (int)w, nI, 1.0, Pinv[t].d(), nI, 0, buf.d() + (size_t)t * nI * w, w, 0,
                 0.0, X[t].d() + (size_t)b * n2, M, 0);
      }
      s.samples += (long long)nI * M;
    }
    // 4. thresholds from ||X|| and the TT-SVD tail
    DBuf ssq(c.alloc, sizeof(double) * 7);
    fill(c, ssq.d(), 7, 0.0);
    for (int t = 0; t < 7; ++t)
      if (k[t]) sumsq_reduce(c, X[t].d(), (size_t)k[t] * M, ssq.d() + t);
    double* h = c.host(7);
    TTIGA_HIP(hipMemcpyAsync(h, ssq.d(), 7 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    double nrm[7], rmax = 0.0;
    for (int t = 0; t < 7; ++t) nrm[t] = std::sqrt(std::max(h[t], 0.0));
    for (int t = 0; t < 6; ++t) rmax = std::max(rmax, nrm[t]);
    s.max_R_norm = rmax;
    for (int t = 0; t < 7; ++t) scale[t] = t < 6 ? rmax : nrm[6];
    for (int t = 0; t < 7; ++t) {
      if (k[t] == 0 || nrm[t] == 0.0) {
        fac[t].set_zero(Q);
        continue;
      }
      tt_from_first_unfolding(c, U[t].d(), k[t], X[t].d(), Q, eps * scale[t] / std::sqrt(2.0), 0, fac[t],
                              opts.max_rank);
    }
    for (int t = 0; t < 7; ++t) X[t].reset();
  };
  // 5. probe check on random grid points: every factor's RMS error per point within 10 eps of its
  // threshold scale spread over the grid
  auto probe = [&]() {
    const int P = 2048;
    std::vector<int> p0(P), p1(P), p2(P);
    for (int q = 0; q < P; ++q) {
      p0[q] = rnd(n0);
      p1[q] = rnd(n1);
      p2[q] = rnd(n2);
    }
    DBuf pid(c.alloc, sizeof(int) * 3 * P), ref(c.alloc, sizeof(double) * 7 * P), got(c.alloc, sizeof(double) * 7 * P);
    int* dp = pid.as<int>();
    TTIGA_HIP(hipMemcpyAsync(dp, p0.data(), sizeof(int) * P, hipMemcpyHostToDevice, c.stream));
    TTIGA_HIP(hipMemcpyAsync(dp + P, p1.data(), sizeof(int) * P, hipMemcpyHostToDevice, c.stream));
    TTIGA_HIP(hipMemcpyAsync(dp + 2 * P, p2.data(), sizeof(int) * P, hipMemcpyHostToDevice, c.stream));
    launch_factors_at(c, gd, sd, P, dp, dp + P, dp + 2 * P, ref.d(), nullptr);
    for (int t = 0; t < 7; ++t) tt_eval_points(c, fac[t], P, dp, dp + P, dp + 2 * P, got.d() + (size_t)t * P);
    std::vector<double> hr((size_t)7 * P), hg((size_t)7 * P);
    TTIGA_HIP(hipMemcpyAsync(hr.data(), ref.d(), sizeof(double) * 7 * P, hipMemcpyDeviceToHost, c.stream));
    TTIGA_HIP(hipMemcpyAsync(hg.data(), got.d(), sizeof(double) * 7 * P, hipMemcpyDeviceToHost, c.stream));
    c.sync();
    s.samples += P;
    const double npts = (double)n0 * M;
    bool ok = true;
    for (int t = 0; t < 7; ++t) {
      double e2 = 0.0;
      for (int q = 0; q < P; ++q) {
        const double d = hg[(size_t)t * P + q] - hr[(size_t)t * P + q];
        e2 += d * d;
      }
      const double rms = std::sqrt(e2 / P), allowed = 10.0 * eps * scale[t] / std::sqrt(npts);
      if (trace) std::fprintf(stderr, "[cross] factor %d probe rms %.3e allowed %.3e\n", t, rms, allowed);
      if (!(rms <= allowed) && !(scale[t] == 0.0 && e2 == 0.0)) ok = false;
    }
    return ok;
  };
  // 3. the coefficients X_t = P_t^+ A_t[I, :] (k_t x Q1 Q2): by a second cross approximation of X_t
  // viewed as (k_t Q1) x Q2 when it succeeds (samples of O(Q r^2)) and passes the probe check,
  // else from the whole slices A_t[I, :, :] (|I| Q1 Q2 samples)
  if (cross_second_level(gd, sd, fac, s, U, k, I, Id, Pinv, scale, rs)) {
    if (probe()) {
      if (trace) std::fprintf(stderr, "[cross] second level accepted\n");
      return true;
    }
    if (trace) std::fprintf(stderr, "[cross] second level failed its probe check: whole slices\n");
  }
  slices();
  if (!probe()) return reject("probe error above 10 eps");
  return true;
}

void Problem::assemble(ttiga_assembly_stats* st) {
  Context& c = *ctx;
  ttiga_assembly_stats s{};
  double t0 = now_ms();
  c.rng_counter = kAssembleSeed;
  build_tables();
  // 2. factor tensors on the Gauss grid, 3. TT compression
  const size_t total = (size_t)Q[0] * Q[1] * Q[2];
  const size_t slab_bytes = sizeof(double) * 7 * (size_t)Q[0] * Q[2];
  const size_t kWholeLimit = size_t(2) << 30;
  const bool streamed = (opts.sample_chunk_bytes > 0 || slab_bytes * Q[1] > kWholeLimit) &&
                        Q[0] > kExactSvdSize && (size_t)Q[1] * Q[2] > (size_t)kExactSvdSize;
  const GeoDev gd = geo_dev(gtab_span, gtab_B, gtab_D);
  const SourceDev sd = source_dev();
  DBuf st8(c.alloc, sizeof(double) * 8);
  const double eps = assembly_eps();
  double t1 = 0.0;
  // norms, det J check and the compression thresholds from the 8 gathered statistics
  auto thresholds = [&](std::vector<double>& delta) {
    double* h = c.host(8);
    TTIGA_HIP(hipMemcpyAsync(h, st8.d(), 8 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    double sumsq[7];
    for (int f = 0; f < 7; ++f) sumsq[f] = h[f];
    s.min_detJ = h[7];
    double rmax = 0.0;
    for (int f = 0; f < 6; ++f) rmax = std::max(rmax, std::sqrt(sumsq[f]));
    s.max_R_norm = rmax;
    min_detJ = s.min_detJ;
    if (!(s.min_detJ > 0.0))
      throw Error(TTIGA_E_DETJ, "min det J = " + std::to_string(s.min_detJ) + " <= 0 on the Gauss grid");
    const double dR = eps * rmax / std::sqrt(2.0);
    const double dF = eps * std::sqrt(sumsq[6]) / std::sqrt(2.0);
    delta.assign(7, 0.0);
    for (int f = 0; f < 7; ++f) delta[f] = (sumsq[f] == 0.0) ? -1.0 : (f < 6 ? dR : dF);
    t1 = now_ms();
    s.time_ms[0] = t1 - t0;
  };
  TT fac[7];
  const bool cross = opts.compression == TTIGA_COMPRESS_AUTO && Q[0] > 2 * kExactSvdSize &&
                     (size_t)Q[1] * Q[2] > (size_t)(2 * kExactSvdSize) && detj_rows_fit(gd);
  bool done = false;
  if (cross) {
    // det J on the whole grid (the E_DETJ guarantee), then the cross approximation
    GeoDev gdj = gd;
    gdj.xi2 = tab_xi[2].d();
    gdj.knots2 = gknots_d[2].d();
    launch_detj_min(c, gdj, Q, st8.d());
    double* h = c.host(1);
    TTIGA_HIP(hipMemcpyAsync(h, st8.d(), sizeof(double), hipMemcpyDeviceToHost, c.stream));
    c.sync();
    s.min_detJ = min_detJ = h[0];
    if (!(s.min_detJ > 0.0))
      throw Error(TTIGA_E_DETJ, "min det J = " + std::to_string(s.min_detJ) + " <= 0 on the Gauss grid");
    done = compress_cross(gd, sd, fac, s);
    s.compression_path = done ? 2 : 3;
    t1 = now_ms();
    s.time_ms[0] = t1 - t0;
  }
  if (done) {
  } else if (streamed || cross) {
    if (!cross) s.compression_path = 1;
    s.samples += 2 * (long long)total;
    const size_t budget = opts.sample_chunk_bytes > 0 ? opts.sample_chunk_bytes : kWholeLimit;
    const int chunk = (int)std::max<size_t>(1, std::min<size_t>(Q[1], budget / slab_bytes));
    auto produce = [&](int b, int cnt, double* buf) {
      launch_factors_grid(c, gd, sd, Q, b, cnt, buf, st8.d(), b > 0);
    };
    tt_compress_streamed(c, 7, Q, chunk, produce, thresholds, fac, opts.max_rank);
  } else {
    s.compression_path = 0;
    s.samples += (long long)total;
    DBuf Fac(c.alloc, sizeof(double) * 7 * total);
    launch_factors_grid(c, gd, sd, Q, 0, Q[1], Fac.d(), st8.d(), false);
    std::vector<double> delta;
    thresholds(delta);
    for (int f = 0; f < 7; ++f) {
      if (delta[f] < 0.0) { fac[f].set_zero(Q); continue; }
      tt_compress_dense(c, Fac.d() + f * total, Q, delta[f], fac[f], opts.max_rank);
    }
  }
  for (int f = 0; f < 6; ++f) R[f] = std::move(fac[f]);
  fJ = std::move(fac[6]);
  c.sync();
  double t2 = now_ms();
  s.time_ms[1] = t2 - t1;
  for (int f = 0; f < 6; ++f)
    for (int k = 0; k < 4; ++k) s.rank_R[f][k] = R[f].r[k];
  for (int k = 0; k < 4; ++k) s.rank_fJ[k] = fJ.r[k];
  // 4. K as the rounded sum of the nine components, F from f det J
  const int band = 2 * p + 1;
  int nb[3] = {n[0] * band, n[1] * band, n[2] * band};
  K.set_zero(nb);
  for (int tI = 0; tI < 9; ++tI) {
    const int i = kTermOrder[tI][0], j = kTermOrder[tI][1];
    const TT& Rt = R[r_index(i, j)];
    if (Rt.zero()) continue;
    TT term;
    term.alloc(c, nb, Rt.r);
    for (int d = 0; d < 3; ++d) {
      const double* row = (d == i) ? tab_D[d].d() : tab_B[d].d();
      const double* col = (d == j) ? tab_D[d].d() : tab_B[d].d();
      launch_assemble_band(c, n[d], p, g, Rt.r[d], Rt.r[d + 1], Rt.c[d].d(), tab_w[d].d(), row, col,
                           term.c[d].d());
    }
    if (K.zero()) {
      K = std::move(term);
    } else {
      TT sum;
      tt_axpby(c, 1.0, K, 1.0, term, sum);
      tt_round(c, sum, eps, -1.0, opts.max_rank);
      K = std::move(sum);
    }
  }
  if (!fJ.zero()) {
    F.alloc(c, n, fJ.r);
    for (int d = 0; d < 3; ++d)
      launch_assemble_vec(c, n[d], p, g, fJ.r[d], fJ.r[d + 1], fJ.c[d].d(), tab_w[d].d(), tab_B[d].d(),
                          F.c[d].d());
  } else {
    F.set_zero(n);
  }
  for (int f = 0; f < 6; ++f)
    if (bc_kind[f] == TTIGA_BC_TRACTION && bc_value[f] != 0.0) add_traction(f, eps);
  c.sync();
  double t3 = now_ms();
  s.time_ms[2] = t3 - t2;
  for (int k = 0; k < 4; ++k) {
    s.rank_K[k] = K.r[k];
    s.rank_F[k] = F.r[k];
  }
  // 5. boundary reduction
  reduce_boundary();
  c.sync();
  s.time_ms[3] = now_ms() - t3;
  assembled = true;
  solved = false;
  if (st) *st = s;
}

// The flux of a traction face f (Section 3.1: the boundary term of the weak form on a natural
// face with du/dn = g): F_a += g int_face N_a dS.  On the face xi_d = 0 (or 1) only the first
// (last) B-spline of direction d is non-zero, and equals 1; over the two tangential directions
// i < j the integral is the Gauss sum of w_i w_j J_s N_ai N_aj with the surface element
// J_s = |dx/dxi_i x dx/dxi_j|.  J_s on the tangential Gauss grid is compressed to a rank-r
// two-mode TT (TT-SVD at 1e-2 eps of its norm), each mode contracted against the B-splines
// like the cores of F, and the face vector g e_end placed in mode d: a TT of rank r added to F.
void Problem::add_traction(int f, double eps) {
  Context& c = *ctx;
  const int d = f / 2, side = f % 2;
  const int i = d == 0 ? 1 : 0, j = d == 2 ? 1 : 2;
  // geometry tables: the tangential directions at their Gauss points, direction d at xi_d = side
  DBuf xi1(c.alloc, sizeof(double)), span[3], GB[3], GD[3];
  const double xv = (double)side;
  TTIGA_HIP(hipMemcpyAsync(xi1.d(), &xv, sizeof(double), hipMemcpyHostToDevice, c.stream));
  for (int e = 0; e < 3; ++e) {
    const int cnt = e == d ? 1 : Q[e];
    span[e] = DBuf(c.alloc, sizeof(int) * cnt);
    GB[e] = DBuf(c.alloc, sizeof(double) * cnt * (pg[e] + 1));
    GD[e] = DBuf(c.alloc, sizeof(double) * cnt * (pg[e] + 1));
    launch_geo_tables(c, cnt, e == d ? xi1.d() : tab_xi[e].d(), 1, m[e], pg[e], gknots_d[e].d(), span[e].as<int>(),
                      GB[e].d(), GD[e].d());
  }
  c.sync();  // the host value xv is read by the copy above
  const GeoDev gd = geo_dev(span, GB, GD);
  const int Qi = Q[i], Qj = Q[j];
  DBuf Js(c.alloc, sizeof(double) * (size_t)Qi * Qj);
  launch_surface_jac(c, gd, d, Qi, Qj, Js.d());
  DBuf nrm(c.alloc, sizeof(double));
  fill(c, nrm.d(), 1, 0.0);
  sumsq_reduce(c, Js.d(), (size_t)Qi * Qj, nrm.d());
  double* h = c.host(1);
  TTIGA_HIP(hipMemcpyAsync(h, nrm.d(), sizeof(double), hipMemcpyDeviceToHost, c.stream));
  c.sync();
  TTIGA_CHECK(h[0] > 0.0, TTIGA_E_GEOM, "traction face has zero area");
  TT S;  // J_s as a TT over (Q_i, Q_j, 1)
  const int shape[3] = {Qi, Qj, 1};
  tt_compress_dense(c, Js.d(), shape, 1e-2 * eps * std::sqrt(h[0]), S, opts.max_rank);
  const int r = S.r[1];
  // cores of the face load: ranks (1, r, 1, 1) for d = 0 ... in the order of the directions
  int rr[4];
  if (d == 0) { rr[0] = 1; rr[1] = 1; rr[2] = r; rr[3] = 1; }
  else if (d == 1) { rr[0] = 1; rr[1] = r; rr[2] = r; rr[3] = 1; }
  else { rr[0] = 1; rr[1] = r; rr[2] = 1; rr[3] = 1; }
  TT Fs;
  Fs.alloc(c, n, rr);
  // mode i: the first core of S (1 x Q_i x r) against the B-splines; mode j: the second core
  // times the third (r x Q_j x 1) against the B-splines
  DBuf Sj(c.alloc, sizeof(double) * (size_t)r * Qj);
  gemm(c, false, false, r * Qj, 1, S.r[2], 1.0, S.c[1].d(), S.r[2], 0, S.c[2].d(), 1, 0, 0.0, Sj.d(), 1, 0);
  launch_assemble_vec(c, n[i], p, g, 1, r, S.c[0].d(), tab_w[i].d(), tab_B[i].d(), Fs.c[i].d());
  launch_assemble_vec(c, n[j], p, g, r, 1, Sj.d(), tab_w[j].d(), tab_B[j].d(), Fs.c[j].d());
  // mode d: g e_end, times the identity over the rank when d sits between i and j
  const int rd = d == 1 ? r : 1;
  std::vector<double> core((size_t)rd * n[d] * rd, 0.0);
  for (int a = 0; a < rd; ++a) core[((size_t)a * n[d] + (side ? n[d] - 1 : 0)) * rd + a] = bc_value[f];
  TTIGA_HIP(hipMemcpyAsync(Fs.c[d].d(), core.data(), sizeof(double) * core.size(), hipMemcpyHostToDevice,
                           c.stream));
  c.sync();
  if (F.zero()) {
    F = std::move(Fs);
  } else {
    TT sum;
    tt_axpby(c, 1.0, F, 1.0, Fs, sum);
    tt_round(c, sum, eps * 1e-2, -1.0, opts.max_rank);
    F = std::move(sum);
  }
}

void Problem::reduce_boundary() {
  Context& c = *ctx;
  const int band = 2 * p + 1;
  int ni[3];
  for (int d = 0; d < 3; ++d) ni[d] = hi[d] - lo[d];
  int nbi[3] = {ni[0] * band, ni[1] * band, ni[2] * band};
  if (K.zero()) throw Error(TTIGA_E_GEOM, "stiffness operator is zero");
  KII.alloc(c, nbi, K.r);
  for (int d = 0; d < 3; ++d)
    launch_slice_band(c, n[d], p, lo[d], ni[d], K.r[d], K.r[d + 1], K.c[d].d(), KII.c[d].d());
  TT FI;
  if (!F.zero()) {
    FI.alloc(c, ni, F.r);
    for (int d = 0; d < 3; ++d)
      launch_slice_vec(c, n[d], lo[d], ni[d], F.r[d], F.r[d + 1], F.c[d].d(), FI.c[d].d());
  } else {
    FI.set_zero(ni);
  }
  if (lift) {
    // u_g: the face constants on the Dirichlet faces, 0 inside, the later face in face order
    // winning where faces meet.  With m_f the indicator of face f (rank 1: the end vector of
    // its direction times ones), u_g = sum_f c_f m_f prod_{f' > f Dirichlet} (1 - m_f'), and
    // every term is rank 1: per direction the face's end vector (or ones) times, for each
    // later Dirichlet face of that direction, ones with that face's end zeroed.
    ug.set_zero(n);
    for (int f = 0; f < 6; ++f) {
      if (bc_kind[f] != TTIGA_BC_CONSTANT || bc_value[f] == 0.0) continue;
      TT term;
      int r1[4] = {1, 1, 1, 1};
      term.alloc(c, n, r1);
      for (int d = 0; d < 3; ++d) {
        std::vector<double> v(n[d], 1.0);
        if (d == f / 2) {
          std::fill(v.begin(), v.end(), 0.0);
          v[f % 2 == 0 ? 0 : n[d] - 1] = 1.0;
        }
        for (int g2 = f + 1; g2 < 6; ++g2)
          if (g2 / 2 == d && is_dirichlet(bc_kind[g2])) v[g2 % 2 == 0 ? 0 : n[d] - 1] = 0.0;
        if (d == 0)
          for (double& x : v) x *= bc_value[f];
        TTIGA_HIP(hipMemcpyAsync(term.c[d].d(), v.data(), sizeof(double) * n[d], hipMemcpyHostToDevice,
                                 c.stream));
        c.sync();
      }
      TT acc;
      tt_axpby(c, 1.0, ug, 1.0, term, acc);
      ug = std::move(acc);
    }
    TT Kug, KugI;
    tt_matvec_banded(c, K, p, ug, Kug);
    KugI.alloc(c, ni, Kug.r);
    for (int d = 0; d < 3; ++d)
      launch_slice_vec(c, n[d], lo[d], ni[d], Kug.r[d], Kug.r[d + 1], Kug.c[d].d(), KugI.c[d].d());
    TT sum;
    tt_axpby(c, 1.0, FI, -1.0, KugI, sum);
    tt_round(c, sum, assembly_eps() * 1e-2, -1.0, opts.max_rank);
    rhs = std::move(sum);
  } else {
    ug.set_zero(n);
    rhs = std::move(FI);
  }
}

// Upper estimate of the device memory one assembly + solve needs, for admission by an
// executor: the larger of the sampling/compression phase (whole-grid samples and one
// TT-SVD's temporaries, or one streamed chunk, the shared sketch matrix and the seven
// projections with their QR) and the solve phase (a few trains of rank 48 times the
// operator band, the product and preconditioner trains at the same rank), plus the
// resident tables.  Overruns are served from the executor's pool, so an estimate that is
// low costs admission accuracy, not correctness.
size_t Problem::footprint_estimate() const {
  const double Q0 = Q[0], Q1 = Q[1], Q2 = Q[2];
  const double pts = Q0 * Q1 * Q2, slab = 7.0 * Q0 * Q2 * 8.0;
  const double whole_limit = 2.0 * 1073741824.0;
  const bool streamed = (opts.sample_chunk_bytes > 0 || slab * Q1 > whole_limit) &&
                        Q[0] > kExactSvdSize && Q1 * Q2 > kExactSvdSize;
  double sampling;
  if (streamed) {
    const double budget = opts.sample_chunk_bytes > 0 ? (double)opts.sample_chunk_bytes : whole_limit;
    const double chunk = std::max(1.0, std::min(Q1, std::floor(budget / slab)));
    sampling = slab * chunk + Q1 * Q2 * 48.0 * 8.0 * (1.0 + 7.0 + 2.0) + 64.0 * Q0 * 48.0 * 8.0;
  } else {
    sampling = 7.0 * pts * 8.0 + 3.0 * pts * 8.0;
  }
  const double nmax = std::max(n[0], std::max(n[1], n[2]));
  const double rbar = std::min(48, opts.max_rank > 0 ? opts.max_rank : 48);
  const double solve = 40.0 * rbar * rbar * nmax * (2.0 * p + 1.0) * 8.0;
  const double tables = 8.0 * (Q0 + Q1 + Q2) * (4.0 * (p + 1) + 8.0) + 8.0 * 4.0 * m[0] * m[1] * m[2];
  return (size_t)(std::max(sampling, solve) + tables + (64u << 20));
}

void Problem::solve(ttiga_solve_stats* st) {
  TTIGA_CHECK(assembled, TTIGA_E_STATE, "solve before assemble");
  Context& c = *ctx;
  ttiga_solve_stats s{};
  const double t0 = now_ms();
  c.rng_counter = kSolveSeed;
  int ni[3];
  for (int d = 0; d < 3; ++d) ni[d] = hi[d] - lo[d];
  u.set_zero(ni);
  if (rhs.zero()) {
    s.iterations = 0;
    s.rel_res = 0.0;
    s.status = TTIGA_OK;
  } else if (opts.solver == TTIGA_SOLVER_AMEN) {
    TTIGA_CHECK(opts.precision == TTIGA_FP64, TTIGA_E_ARG, "the AMEn solve runs in FP64 only");
    const double ts = now_ms();
    if (!pc.ready) pc.setup(*this);
    s.precond_setup_ms = now_ms() - ts;
    solve_amen(s);
  } else if (opts.precond) {
    const double ts = now_ms();
    if (!pc.ready) pc.setup(*this);
    s.precond_setup_ms = now_ms() - ts;
    if (opts.precision == TTIGA_FP64)
      solve_pcg(s);
    else
      solve_mixed(s);
  } else {
    solve_cg(s);
  }
  for (int k = 0; k < 4; ++k) s.rank_u[k] = u.r[k];
  c.sync();
  s.time_ms = now_ms() - t0;
  solved = true;
  last_solve = s;
  if (st) *st = s;
  if (s.status != TTIGA_OK)
    throw Error(s.status, opts.solver == TTIGA_SOLVER_AMEN ? "AMEn did not reach rel_res_tol within its sweeps"
                                                           : "TT-CG did not reach rel_res_tol within max_iter");
}

// Products K x whose explicit cores (ranks rK rx) would exceed this many bytes are rounded
// as they are formed (tt_matvec_round) instead of being stored and rounded afterwards.
static constexpr size_t kFusedProductBytes = size_t(1) << 30;

// ||b - K x|| / ||b||, with the residual train b - K x rounded at eps_x (replaces r).
// exact_norm: the norm is that of the unrounded train: Householder orthogonalisation of the
// concatenated cores of [b, -K x] loses no digits to the cancellation, and the first SVD of
// the right-to-left sweep reads the norm before anything is truncated (a randomised sketch
// could only underestimate it); the plain CG stops on this norm, and the preconditioned
// solves report it at their end.  Otherwise (the residual replacements inside PCG, whose
// stopping test is the preconditioned estimate) a train of rank above 160 is rounded by the
// randomised sketch at loose tolerances, and the norm returned is that of the rounded train.  With Kf
// given and a product too large to store, the residual train is formed already rounded and
// the norm is that of the rounded train.
double true_residual(Context& c, const Matvec& mv, const TT& b, const TT& x, double nb, double eps_x, int max_rank,
                     TT& r, int& hint, const TT* Kf, int p, bool exact_norm) {
  if (Kf && matvec_product_bytes(*Kf, x) > kFusedProductBytes) {
    tt_matvec_round(c, *Kf, p, x, -1.0, &b, 1.0, eps_x, max_rank, hint, r);
    return std::sqrt(std::max(tt_dot_sync(c, r, r), 0.0)) / nb;
  }
  TT Kx, tr;
  mv(x, Kx);
  tt_axpby(c, 1.0, b, -1.0, Kx, tr);
  // trains of modest rank take the deterministic rounding anyway: it is the cheaper one there
  if (exact_norm || eps_x < 1e-9 || std::max(tr.r[1], tr.r[2]) <= 160) {
    double nrm = 0.0;
    tt_round(c, tr, eps_x, -1.0, max_rank, &nrm);
    r = std::move(tr);
    return nrm / nb;
  }
  tt_round_auto(c, tr, eps_x, max_rank, hint);
  r = std::move(tr);
  return std::sqrt(std::max(tt_dot_sync(c, r, r), 0.0)) / nb;
}

// Truncated TT-CG: conjugate gradients with TT-rounding of every update, the
// iterate kept at min(eps, tol/10) because truncating x moves the residual by up
// to kappa times the truncation; true residual every 10 iterations and at the test.
void Problem::solve_cg(ttiga_solve_stats& s) {
  Context& c = *ctx;
  const double tol = opts.rel_res_tol;
  const double eps = std::min(opts.tt_eps, 0.3 * tol);
  const double eps_x = std::min(opts.tt_eps, 0.1 * tol);
  const Matvec mv = [&](const TT& v, TT& out) { tt_matvec_banded(c, KII, p, v, out); };
  int max_seen = 0;
  auto seen = [&](const TT& t) {
    for (int k = 1; k < 3; ++k) max_seen = std::max(max_seen, t.r[k]);
  };
  const double nb = std::sqrt(std::max(tt_dot_sync(c, rhs, rhs), 0.0));
  TT r, pdir;
  tt_copy(c, rhs, r);
  tt_copy(c, rhs, pdir);
  double rho = tt_dot_sync(c, r, r);
  int it = 0, hq = 8, hx = 8, hr = 8, hp = 8;
  bool conv = false;
  double true_res = 1.0;
  while (it < opts.max_iter) {
    ++it;
    TT q;
    if (matvec_product_bytes(KII, pdir) > kFusedProductBytes) {
      tt_matvec_round(c, KII, p, pdir, 1.0, nullptr, 0.0, eps, opts.max_rank, hq, q);
      seen(q);
    } else {
      tt_matvec_banded(c, KII, p, pdir, q);
      seen(q);
      tt_round_auto(c, q, eps, opts.max_rank, hq);
    }
    const double alpha = rho / tt_dot_sync(c, pdir, q);
    TT xn, rn;
    tt_axpby(c, 1.0, u, alpha, pdir, xn);
    tt_round_auto(c, xn, eps_x, opts.max_rank, hx);
    u = std::move(xn);
    tt_axpby(c, 1.0, r, -alpha, q, rn);
    tt_round_auto(c, rn, eps, opts.max_rank, hr);
    r = std::move(rn);
    const double est = std::sqrt(std::max(tt_dot_sync(c, r, r), 0.0)) / nb;
    if (it % 10 == 0 || est <= tol) {
      true_res = true_residual(c, mv, rhs, u, nb, eps_x, opts.max_rank, r, hr, &KII, p);
      if (true_res <= tol) {
        conv = true;
        break;
      }
    }
    const double rho_new = tt_dot_sync(c, r, r);
    const double beta = rho_new / rho;
    rho = rho_new;
    TT pn;
    tt_axpby(c, 1.0, r, beta, pdir, pn);
    tt_round_auto(c, pn, eps, opts.max_rank, hp);
    pdir = std::move(pn);
    seen(u);
  }
  if (!conv) {
    TT tmp;
    true_res = true_residual(c, mv, rhs, u, nb, eps_x, 0, tmp, hr, &KII, p);
  }
  s.iterations = it;
  s.rel_res = true_res;
  s.max_rank_seen = max_seen;
  s.status = conv ? TTIGA_OK : TTIGA_E_NOTCONV;
}

// Flexible preconditioned truncated TT-CG (Polak-Ribiere beta, clipped at 0),
// preconditioner applied with a loose re-compression.  The directions, residuals and
// products shrink with the error, so they are truncated with a relaxed relative
// tolerance eps_k = 0.1 tol / est_k (est_k the current error estimate, capped at 1e-3):
// their absolute truncation error stays at the tol level, as in relaxed inexact
// Krylov methods, instead of resolving ever finer detail of ever smaller vectors
// (which makes their TT ranks grow every iteration).  With the preconditioner
// the stopping test is ||P^-1 r|| <= tol ||x||: since P^-1 K is close to the
// identity, P^-1 r estimates the error x - u itself, so the test bounds the
// relative 2-norm error of the iterate; the plain residual of a truncated iterate
// is amplified by kappa(K) and would stall near kappa * eps.  The test is
// confirmed on the true residual b - K x every 10 iterations and before stopping.
PcgRun Problem::pcg_run(const TT& b, TT& x, double tol, double eps_floor, int max_iter,
                        const LowpTT* Klp, int& max_seen, bool report_exact) {
  Context& c = *ctx;
  const Matvec mv = [&](const TT& v, TT& out) {
    if (Klp)
      tt_matvec_banded_lp(c, *Klp, p, v, out);
    else
      tt_matvec_banded(c, KII, p, v, out);
  };
  // every rounding inside the iteration injects a relative error into the residual
  // recursion, so it must sit below the error target; truncating the iterate by a
  // relative delta moves P^-1 r by about delta (P^-1 K is near the identity), so the
  // iterate takes the same tolerance; the preconditioner only needs two digits
  const double eps0 = eps_floor;
  const double eps_x = eps_floor;
  double eps = eps0;
  double best = 1.0;
  int best_it = 0;
  auto seen = [&](const TT& t) {
    for (int k = 1; k < 3; ++k) max_seen = std::max(max_seen, t.r[k]);
  };
  const double nb = std::sqrt(std::max(tt_dot_sync(c, b, b), 0.0));
  TT r, z, pdir;
  tt_copy(c, b, r);
  int hq = 8, hx = 8, hr = 8, hp = 8, hz = 8;
  auto eps_p = [&]() { return std::max(eps, 1e-2); };
  pc.apply(c, r, z, eps_p(), opts.max_rank, hz);
  tt_copy(c, z, pdir);
  double rho = tt_dot_sync(c, r, z);
  // a product too large to store is rounded as it is formed, with the FP64 operator (also
  // inside a mixed-precision refinement, whose low-precision product forms the cores)
  const TT* Kf = &KII;
  PcgRun o;
  while (o.it < max_iter) {
    ++o.it;
    TT q;
    if (Kf && matvec_product_bytes(*Kf, pdir) > kFusedProductBytes) {
      tt_matvec_round(c, *Kf, p, pdir, 1.0, nullptr, 0.0, eps, opts.max_rank, hq, q);
      seen(q);
    } else {
      mv(pdir, q);
      seen(q);
      tt_round_auto(c, q, eps, opts.max_rank, hq);
    }
    const double alpha = rho / tt_dot_sync(c, pdir, q);
    TT xn, rn;
    tt_axpby(c, 1.0, x, alpha, pdir, xn);
    tt_round_auto(c, xn, eps_x, opts.max_rank, hx);
    x = std::move(xn);
    seen(x);
    tt_axpby(c, 1.0, r, -alpha, q, rn);
    tt_round_auto(c, rn, eps, opts.max_rank, hr);
    TT r_old = std::move(r);
    r = std::move(rn);
    bool replaced = false;
    if (o.it % 10 == 0) {
      o.true_res = true_residual(c, mv, b, x, nb, eps_x, opts.max_rank, r, hr, Kf, p, false);
      replaced = true;
    }
    pc.apply(c, r, z, eps_p(), opts.max_rank, hz);
    seen(z);
    // r.z, z.z, x.x and r_old.z (the Polak-Ribiere term) with one synchronisation
    double dd[4];
    auto dots = [&]() {
      const TT* xs[4] = {&r, &z, &x, &r_old};
      const TT* ys[4] = {&z, &z, &x, &z};
      tt_dots_sync(c, xs, ys, 4, dd);
      o.pres = std::sqrt(std::max(dd[1], 0.0) / std::max(dd[2], 1e-300));
    };
    dots();
    if (o.pres <= tol && !replaced) {
      o.true_res = true_residual(c, mv, b, x, nb, eps_x, opts.max_rank, r, hr, Kf, p, false);
      pc.apply(c, r, z, eps_p(), opts.max_rank, hz);
      dots();
    }
    const double rho_new = dd[0];
    if (o.pres <= tol) {
      o.conv = true;
      break;
    }
    eps = std::min(1e-3, std::max(eps0, 0.1 * tol / std::max(o.pres, 1e-300)));
    // stagnation: no halving of the best preconditioned residual in 15 iterations
    if (o.pres < 0.5 * best) {
      best = o.pres;
      best_it = o.it;
    } else if (o.it - best_it >= 15) {
      break;
    }
    const double beta = std::max(0.0, (rho_new - dd[3]) / rho);
    rho = rho_new;
    TT pn;
    tt_axpby(c, 1.0, z, beta, pdir, pn);
    tt_round_auto(c, pn, eps, opts.max_rank, hp);
    pdir = std::move(pn);
  }
  // the reported true residual (exact norm of the unrounded b - K x when asked for)
  if (report_exact || !o.conv) {
    TT tmp;
    o.true_res = true_residual(c, mv, b, x, nb, eps_x, 0, tmp, hr, Kf, p, report_exact);
  }
  return o;
}

// Flexible preconditioned truncated TT-CG in FP64 on K_II u = rhs.
void Problem::solve_pcg(ttiga_solve_stats& s) {
  const double tol = opts.rel_res_tol;
  int max_seen = 0;
  const PcgRun o = pcg_run(rhs, u, tol, std::min(opts.tt_eps, 0.3 * tol), opts.max_iter, nullptr, max_seen, true);
  s.iterations = o.it;
  s.rel_res = o.true_res;
  s.rel_pres = o.pres;
  s.max_rank_seen = max_seen;
  s.precond_terms = pc.R;
  s.precond_err = pc.approx_err;
  s.status = o.conv ? TTIGA_OK : TTIGA_E_NOTCONV;
}

// Mixed precision by iterative refinement: the operator is stored in FP32 or BF16 (the
// cores of K_II rounded once), and each correction d solves K d = r with the same
// flexible PCG whose products K v take the low-precision cores with FP32 arithmetic,
// to a loose relative tolerance t; its dense contractions with the operator (the products
// rounded as they are formed) and the preconditioner's transforms run on the FP32 MFMA product
// (operator products in BF16 mode: BF16) with FP32 accumulation.  The roundings' sketches and
// Gram matrices stay FP64: the trains they round are differences such as b - K d whose parts
// are far larger than the result, so FP32 contractions of them lose the result's digits (the
// mixed C2 batch lost accuracy to 5e-5 and speed 7x when they ran in FP32).  The update u + d, the residual r = rhs - K u (FP64
// product), its rounding, the preconditioned error estimate and every QR/SVD stay in
// FP64.  A correction of relative accuracy t reduces the error by about
// max(t, kappa u_low); with FP32 (u = 6e-8) that is a few steps for any mesh here,
// with BF16 (u = 3.9e-3) only small meshes contract at all, so a step that does not
// halve the estimate ends the refinement (E_NOTCONV).  Since a correction is only
// needed to relative accuracy t, the residual it starts from and the trains inside its
// solve are truncated relative to their own norms at a fraction of t, not at the final
// tolerance: the residual of an accurate iterate is rough, and resolving it to 1e-8 of
// its norm would cost ranks in the hundreds for digits the correction cannot use.
void Problem::solve_mixed(ttiga_solve_stats& s) {
  Context& c = *ctx;
  if (Klp.r[1] == 0) tt_to_lowp(c, KII, opts.precision, Klp);
  const Matvec mv = [&](const TT& v, TT& out) { tt_matvec_banded(c, KII, p, v, out); };
  const double tol = opts.rel_res_tol;
  const double eps_x = std::min(opts.tt_eps, 0.3 * tol);
  const double floor_in = opts.precision == TTIGA_BF16 ? 3e-2 : 1e-3;
  const double eps_r = std::max(eps_x, floor_in);
  const double nb = std::sqrt(std::max(tt_dot_sync(c, rhs, rhs), 0.0));
  TT r;
  tt_copy(c, rhs, r);
  double est = 1.0, prev = 1e300, true_res = 1.0;
  int inner = 0, steps = 0, max_seen = 0, hx = 8, hr = 8, hz = 8;
  bool conv = false;
  while (steps < kMaxRefineSteps && inner < opts.max_iter) {
    ++steps;
    const double tol_in = std::max(floor_in, 0.3 * tol / est);
    TT d;
    d.set_zero(u.n);
    PcgRun o;
    {
      // the correction's operator products rounded as they are formed and its preconditioner
      // transforms on the low-precision MFMA product
      struct LowpScope {
        Context& c;
        LowpScope(Context& cc, int dt) : c(cc) { c.lowp = dt; }
        ~LowpScope() { c.lowp = 0; }
      } scope(c, opts.precision);
      o = pcg_run(r, d, tol_in, std::min(0.1, 0.3 * tol_in), opts.max_iter - inner, &Klp, max_seen, false);
    }
    inner += o.it;
    if (d.zero()) break;
    TT un;
    tt_axpby(c, 1.0, u, 1.0, d, un);
    tt_round_auto(c, un, eps_x, opts.max_rank, hx);
    u = std::move(un);
    true_res = true_residual(c, mv, rhs, u, nb, eps_r, opts.max_rank, r, hr, &KII, p, false);
    TT z;
    pc.apply(c, r, z, 1e-2, opts.max_rank, hz);
    double dd[2];
    const TT* xs[2] = {&z, &u};
    tt_dots_sync(c, xs, xs, 2, dd);
    est = std::sqrt(std::max(dd[0], 0.0) / std::max(dd[1], 1e-300));
    if (est <= tol) {
      conv = true;
      break;
    }
    if (est > 0.5 * prev) break;  // the low-precision corrections no longer contract
    prev = est;
  }
  {
    // the reported true residual: exact norm of the unrounded rhs - K u
    TT tmp;
    true_res = true_residual(c, mv, rhs, u, nb, eps_x, 0, tmp, hr, &KII, p, true);
  }
  s.iterations = inner;
  s.refine_steps = steps;
  s.rel_res = true_res;
  s.rel_pres = est;
  s.max_rank_seen = max_seen;
  s.precond_terms = pc.R;
  s.precond_err = pc.approx_err;
  s.status = conv ? TTIGA_OK : TTIGA_E_NOTCONV;
}

const TT* Problem::which(int w) const {
  if (w == TTIGA_WHICH_K) return &K;
  if (w == TTIGA_WHICH_F) return &F;
  if (w == TTIGA_WHICH_KII) return &KII;
  if (w == TTIGA_WHICH_RHS) return &rhs;
  if (w >= TTIGA_WHICH_FACTOR0 && w < TTIGA_WHICH_FACTOR0 + 6) return &R[w - TTIGA_WHICH_FACTOR0];
  if (w == TTIGA_WHICH_FACTOR0 + 6) return &fJ;
  return nullptr;
}

void Problem::sample_points(const double* pts, size_t count, double* out, double* det_out) {
  Context& c = *ctx;
  TTIGA_CHECK(pts && out && count > 0, TTIGA_E_ARG, "sample_factors: null or empty input");
  for (size_t q = 0; q < 3 * count; ++q)
    TTIGA_CHECK(pts[q] >= 0.0 && pts[q] <= 1.0, TTIGA_E_ARG, "sample point outside [0,1]^3");
  DBuf P(c.alloc, sizeof(double) * 3 * count);
  TTIGA_HIP(hipMemcpyAsync(P.d(), pts, sizeof(double) * 3 * count, hipMemcpyHostToDevice, c.stream));
  DBuf span[3], B[3], D[3];
  for (int d = 0; d < 3; ++d) {
    span[d] = DBuf(c.alloc, sizeof(int) * count);
    B[d] = DBuf(c.alloc, sizeof(double) * count * (pg[d] + 1));
    D[d] = DBuf(c.alloc, sizeof(double) * count * (pg[d] + 1));
    launch_geo_tables(c, (int)count, P.d() + d, 3, m[d], pg[d], gknots_d[d].d(), span[d].as<int>(),
                      B[d].d(), D[d].d());
  }
  DBuf O(c.alloc, sizeof(double) * 7 * count), Dt(c.alloc, sizeof(double) * count);
  launch_factors_points(c, geo_dev(span, B, D), source_dev(), (long)count, O.d(), Dt.d());
  TTIGA_HIP(hipMemcpyAsync(out, O.d(), sizeof(double) * 7 * count, hipMemcpyDeviceToHost, c.stream));
  if (det_out)
    TTIGA_HIP(hipMemcpyAsync(det_out, Dt.d(), sizeof(double) * count, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

}  // namespace ttiga
