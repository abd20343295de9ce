// Separable (fast-diagonalisation) preconditioner in TT form; see precond.hip.
#pragma once

#include "runtime.hpp"

namespace ttiga {

struct Problem;

// Generalised eigenbasis of the 1-D interior stiffness/mass pencil (a, m) of one
// direction: V^T m V = I, V^T a V = diag(lam), eigenvalues descending.  It depends
// only on the knot vector, degree, quadrature and the boundary cut, so it is
// computed once per discretisation and shared.
struct EigenBasis {
  int ni = 0;
  DBuf V, lam;
  double lam_min = 0.0, lam_max = 0.0;
};

struct Precond {
  bool ready = false;
  int ni[3] = {0, 0, 0};
  std::shared_ptr<EigenBasis> eb[3];
  DBuf etab[3];
  double c[3] = {1, 1, 1};
  double lam_min[3] = {0, 0, 0}, lam_max[3] = {0, 0, 0};
  double s_min = 0, s_max = 0, approx_err = 0;
  int R = 0;
  void setup(Problem& P);
  // z ~= P^-1 r, re-compressed with relative tolerance eps
  void apply(Context& ctx, const TT& r, TT& z, double eps, int max_rank, int& hint);
};

}  // namespace ttiga
