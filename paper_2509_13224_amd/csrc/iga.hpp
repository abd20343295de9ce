// Device-side descriptions of the geometry and source, and the IGA kernel launchers.
#pragma once

#include "runtime.hpp"

namespace ttiga {

// Geometry tables for one sampling: per direction the span index and the p_g+1
// non-zero geometry basis values / derivatives at each sample coordinate.
struct GeoDev {
  int pg[3];
  int m[3];            // control points per direction
  const double* Pw;    // [m0][m1][m2][4] homogeneous control net
  const int* span[3];  // per sample coordinate
  const double* B[3];
  const double* D[3];
  // for the det J pass over the Gauss grid: the third direction's sample coordinates and the
  // geometry's knot vector in that direction (null elsewhere)
  const double* xi2 = nullptr;
  const double* knots2 = nullptr;
};

struct SourceDev {
  int kind;
  int n_modes;
  const double* a;    // device
  const double* k;    // device, n_modes x 3
  const double* phi;  // device
  double origin[3];
  double scale;
  // largest |k| component when every wave vector is integral and at most kMaxIntWave
  // (the phases e^{i pi k.x} are then products of powers of three unit phasors), else -1
  int int_kmax;
};

// An exact solution u(x) of the problem, for measuring a solution's L2 error.
struct ExactDev {
  int kind;       // TTIGA_EXACT_*
  double prm[4];  // radial log: r_in, r_out, u_in, u_out
};

constexpr int kMaxIntWave = 8;
constexpr int kMaxRowModes = 64;  // Fourier modes whose phase shifts the row kernel caches

void launch_basis_tables(Context& ctx, int n, int p, int g, const double* knots, double* xi,
                         double* w, double* B, double* D);
void launch_geo_tables(Context& ctx, int count, const double* xi, int stride, int nb, int pg,
                       const double* knots, int* span, double* B, double* D);
// Samples the slabs b0 .. b0+c1-1 of the second direction into F[7][Q0][c1][Q2]; stats8
// receives (or, with accumulate, is merged with) the 7 sums of squares and min det J.
// rows0 (device, nrows0 entries) restricts the first direction to the listed indices
// (F[7][nrows0][c1][Q2]).
void launch_factors_grid(Context& ctx, const GeoDev& geo, const SourceDev& src, const int* Q,
                         int b0, int c1, double* F, double* stats8, bool accumulate = false,
                         const int* rows0 = nullptr, int nrows0 = 0);
// Minimum of det J over the whole Gauss grid into *min_out (device), nothing else; needs
// detj_rows_fit (the rows of a block in LDS: at most 170 control points in the third direction).
bool detj_rows_fit(const GeoDev& geo);
void launch_detj_min(Context& ctx, const GeoDev& geo, const int* Q, double* min_out);
// Grid points (i0[q], i1[q], i2[q]) (device index arrays): out[7][count], det (optional).
void launch_factors_at(Context& ctx, const GeoDev& geo, const SourceDev& src, long count, const int* i0,
                       const int* i1, const int* i2, double* out, double* det);
// Error grid: the exact solution and w0 w1 w2 det J of the slabs b0 .. b0+c1-1 of the second
// direction into F[2][Q0][c1][Q2]; stats8 gets their sums of squares (slots 0, 1) and min det J
// (slot 7).  w[d]: the quadrature weights per direction.
void launch_exact_grid(Context& ctx, const GeoDev& geo, const ExactDev& ex, const double* const* w, const int* Q,
                       int b0, int c1, double* F, double* stats8);
// |dx/dxi_i x dx/dxi_j| on the Qi x Qj tangential grid of a face xi_d = const (the geometry
// tables of direction d hold the face's single point)
void launch_surface_jac(Context& ctx, const GeoDev& geo, int d, int Qi, int Qj, double* out);
// out[a][q][b] = sum_j B[q][j] U[a][e_q + j - lo][b] (the solution core on a grid of g points per
// span; U has ni interior indices starting at global index lo)
void launch_eval_core(Context& ctx, int ra, int rb, int Q, int g, int p, int lo, int ni, const double* B,
                      const double* U, double* out);
void launch_factors_points(Context& ctx, const GeoDev& geo, const SourceDev& src, long count,
                           double* out, double* det);
void launch_assemble_band(Context& ctx, int n, int p, int g, int ra, int rb, const double* G,
                          const double* w, const double* Brow, const double* Bcol, double* M);
void launch_assemble_vec(Context& ctx, int n, int p, int g, int ra, int rb, const double* G,
                         const double* w, const double* B, double* V);
void launch_slice_band(Context& ctx, int n, int p, int lo, int n2, int ra, int rb, const double* M,
                       double* O);
void launch_slice_vec(Context& ctx, int n, int lo, int n2, int ra, int rb, const double* V, double* O);
void launch_homogeneous(Context& ctx, long count, const double* xyz, const double* wts, double* Pw);

}  // namespace ttiga
