// One TT-IGA problem: validated host copy of the description plus its device state.
#pragma once

#include <functional>
#include <vector>

#include "iga.hpp"
#include "precond.hpp"

namespace ttiga {

// sketch seeds of the assembly and of the solve (see Context::rng_counter)
constexpr uint64_t kAssembleSeed = 0xa55e3b1e00000000ull;
constexpr uint64_t kSolveSeed = 0x501fe00000000000ull;

// Outcome of one flexible PCG run.
struct PcgRun {
  int it = 0;
  double pres = 1.0, true_res = 1.0;
  bool conv = false;
};

constexpr int kMaxRefineSteps = 12;

using Matvec = std::function<void(const TT&, TT&)>;

// ||b - K x|| / ||b|| with the residual train b - K x rounded at eps_x into r (problem.hip)
double true_residual(Context& c, const Matvec& mv, const TT& b, const TT& x, double nb, double eps_x, int max_rank,
                     TT& r, int& hint, const TT* Kf = nullptr, int p = 0, bool exact_norm = true);

// faces with Dirichlet data (their end indices are cut from the cores)
inline bool is_dirichlet(int kind) { return kind == TTIGA_BC_ZERO || kind == TTIGA_BC_CONSTANT; }

struct Problem {
  Context* ctx;
  // description
  int pg[3], m[3];
  std::vector<double> gknots[3], ctrl, weights;
  int p, g, n[3], E[3], Q[3];
  int src_kind;
  std::vector<double> src_a, src_k, src_phi;
  double src_origin[3], src_scale;
  int bc_kind[6];
  double bc_value[6];
  bool lift = false;  // non-zero constant Dirichlet data on some face
  int lo[3], hi[3];  // interior index range per direction
  ttiga_options opts;
  // device inputs
  DBuf Pw, gknots_d[3], sknots_d[3], modes_d;
  // per-direction tables at the Gauss nodes
  DBuf tab_xi[3], tab_w[3], tab_B[3], tab_D[3];
  DBuf gtab_span[3], gtab_B[3], gtab_D[3];
  // TT state
  TT R[6], fJ, K, F, KII, rhs, u;
  TT ug;  // full-grid coefficients of the Dirichlet data (zero inside), when lift
  LowpTT Klp;  // K_II in FP32 or BF16 for the mixed-precision solve
  Precond pc;
  double min_detJ = 0.0;
  bool assembled = false, solved = false;
  ttiga_solve_stats last_solve{};

  Problem(Context* c, const ttiga_geometry* geo, const ttiga_discretization* disc,
          const ttiga_source* src, const ttiga_dirichlet* bc, const ttiga_options* opt);
  void assemble(ttiga_assembly_stats* st);
  void solve(ttiga_solve_stats* st);
  const TT* which(int w) const;
  void sample_points(const double* pts, size_t count, double* out, double* det_out);
  void upload();  // device copies of the small inputs
  // relative L2 error of the solution against an exact solution on a Gauss grid of p + extra
  // points per span, evaluated in TT format: out = {relative, ||u_h - u||, ||u||}
  void l2_error(int exact_kind, const double* prm, int extra, double out[3]);
  // {K vs sparse, K vs dense, F, u} compression ratios (entries of the full-grid object over TT entries)
  void compression_ratios(double out[4]);
  size_t footprint_estimate() const;

 private:
  // relative tolerance of the assembly (factor compression, rounded K and F)
  double assembly_eps() const { return opts.assembly_eps > 0.0 ? opts.assembly_eps : opts.tt_eps; }
  bool compress_cross(const GeoDev& gd, const SourceDev& sd, TT* fac, ttiga_assembly_stats& s);
  bool cross_second_level(const GeoDev& gd, const SourceDev& sd, TT* fac, ttiga_assembly_stats& s,
                          const std::vector<DBuf>& U, const std::vector<int>& k, const std::vector<int>& I,
                          const DBuf& Id, const std::vector<DBuf>& Pinv, double* scale, uint64_t& rs);
  void solve_cg(ttiga_solve_stats& s);
  void solve_pcg(ttiga_solve_stats& s);
  void solve_mixed(ttiga_solve_stats& s);
  void solve_amen(ttiga_solve_stats& s);
  PcgRun pcg_run(const TT& b, TT& x, double tol, double eps_floor, int max_iter, const LowpTT* Klp,
                 int& max_seen, bool report_exact);
  void build_tables();
  void add_traction(int face, double eps);
  void reduce_boundary();
  SourceDev source_dev() const;
  GeoDev geo_dev(const DBuf* span, const DBuf* B, const DBuf* D) const;
};

}  // namespace ttiga

struct ttiga_problem {
  ttiga::Problem* impl;
};
