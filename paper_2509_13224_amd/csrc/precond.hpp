// Separable (fast-diagonalisation) preconditioner in TT form; see precond.hip.
#pragma once

#include "runtime.hpp"

namespace ttiga {

struct Problem;

struct Precond {
  bool ready = false;
  int ni[3] = {0, 0, 0};
  DBuf V[3], lam[3], etab[3];
  double c[3] = {1, 1, 1};
  double lam_min[3] = {0, 0, 0}, lam_max[3] = {0, 0, 0};
  double s_min = 0, s_max = 0, approx_err = 0;
  int R = 0;
  void setup(Problem& P);
  // z ~= P^-1 r, re-compressed with relative tolerance eps
  void apply(Context& ctx, const TT& r, TT& z, double eps, int max_rank, int& hint);
};

}  // namespace ttiga
