/*
 * ttiga.h - C ABI of the TT-IGA library for MI355X (gfx950).
 *
 * The library assembles the isogeometric stiffness operator and load vector of
 * the 3-D Poisson problem in tensor-train (TT) form and solves the reduced
 * system in TT.  All arithmetic runs in HIP kernels on one GPU; the host code
 * behind this header only validates arguments, sizes buffers and sequences
 * kernel launches.
 *
 * Problem statement (Section 3.1): -Laplace u = f on the image of a NURBS
 * solid (Section 2.3), u = u_bar on Dirichlet faces, zero traction elsewhere.
 * Discretisation (Section 3.3): B-spline solution space of degree p with n
 * basis functions per parametric direction (open uniform knots, i.e. the
 * h-refined space), stiffness K and load F of eqs. Kfinal / ffinal.
 * TT assembly (Sections 4.2.1 and 4.2.2): metric factors R_ij and f det J are
 * sampled at Gauss points, compressed to TT with tolerance eps and contracted
 * against 1-D B-spline matrices; the nine K_ij are summed with TT-rounding
 * after each addition.  Boundary conditions (Section 4.3) reduce the system to
 * the interior unknowns.  The TT solve is the paper's AMEn (Section 4.1.2) or a
 * preconditioned truncated TT-CG (options.solver).
 *
 * Conventions
 *   - Flattened multi-index: (i0 * n1 + i1) * n2 + i2 (first direction slowest),
 *     the lexicographic order of Section 4.1.1.
 *   - TT cores are stored in the paper's order G_k[r_{k-1}][n_k][r_k], row-major,
 *     r_0 = r_3 = 1 (Section 4.1.1).
 *   - TT-matrix cores are stored banded: M_k[r_{k-1}][n_k][2p+1][r_k], entry
 *     (i, t) holds the 1-D column j = i + t - p; entries whose j falls outside
 *     [0, n_k) are zero.  Only |i - j| <= p can be non-zero because the 1-D
 *     factors are products of B-splines whose supports overlap only then.
 *   - Face order for boundary data: xi0=0, xi0=1, xi1=0, xi1=1, xi2=0, xi2=1.
 *   - Every call returns TTIGA_OK (0), TTIGA_PENDING (1) or a negative error.
 *     No C++ exception crosses this interface.  ttiga_last_error() returns
 *     the message of the last failing call on the calling thread.
 *   - All device work is enqueued on the stream bound to the context; calls
 *     that fill a stats struct or copy to host memory synchronise it.
 *   - A context is not thread-safe: one thread drives it at a time.
 */
#ifndef TTIGA_H
#define TTIGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TTIGA_VERSION_MAJOR 0
#define TTIGA_VERSION_MINOR 1

#define TTIGA_OK 0
#define TTIGA_PENDING 1
#define TTIGA_E_ARG (-1)       /* null pointer, bad size, unsupported option */
#define TTIGA_E_KNOTS (-2)     /* non-monotone knots, wrong length, end multiplicity != p+1 */
#define TTIGA_E_GEOM (-3)      /* non-positive weight */
#define TTIGA_E_DETJ (-4)      /* min det J <= 0 at some Gauss point (folded map) */
#define TTIGA_E_OOM (-5)       /* workspace exhausted */
#define TTIGA_E_ADMISSION (-6) /* server: request does not fit now */
#define TTIGA_E_NOTCONV (-7)   /* iteration limit reached; solution and stats still valid */
#define TTIGA_E_RANKCAP (-8)   /* a TT rank exceeded options.max_rank */
#define TTIGA_E_STATE (-9)     /* call out of order (e.g. solve before assemble) */
#define TTIGA_E_HIP (-10)      /* HIP runtime error; text in ttiga_last_error() */

#define TTIGA_SOURCE_ZERO 0
#define TTIGA_SOURCE_MANUFACTURED_ANNULUS 1 /* forcing of u = sin(pi r) sin(2 theta) sin(pi z) */
#define TTIGA_SOURCE_FOURIER 2              /* sum_m a_m sin(pi k_m.(x - origin)/scale + phi_m) */

/* Exact solutions for ttiga_l2_error (Section 5): the manufactured field of the quarter
 * annulus workload; the radial Laplace solution between coaxial cylinders of radii
 * r_in < r_out with u = u_in at r_in and u_out at r_out (the ring of Section 5.2),
 * params = {r_in, r_out, u_in, u_out}; the L-shape solution of Section 5.1 for
 * f = sin(pi x) sin(pi y). */
#define TTIGA_EXACT_MANUFACTURED_ANNULUS 1 /* u = sin(pi r) sin(2 theta) sin(pi z) */
#define TTIGA_EXACT_RADIAL_LOG 2           /* u = (u_in ln(r_out/r) + u_out ln(r/r_in)) / ln(r_out/r_in) */
#define TTIGA_EXACT_SINE_XY 3              /* u = sin(pi x) sin(pi y) / (2 pi^2) */

#define TTIGA_BC_NATURAL 0  /* zero traction: nothing to impose */
#define TTIGA_BC_ZERO 1     /* homogeneous Dirichlet */
#define TTIGA_BC_CONSTANT 2 /* u = value on the face */
#define TTIGA_BC_TRACTION 3 /* natural face with the flux du/dn = value (outward normal): adds
                               value * int_face N_a dS to F (Section 3.1) */

#define TTIGA_FP64 0
#define TTIGA_FP32 1
#define TTIGA_BF16 2

typedef struct ttiga_ctx ttiga_ctx;
typedef struct ttiga_problem ttiga_problem;
typedef struct ttiga_tt ttiga_tt; /* library-owned TT tensor (results of standalone ops) */

/* NURBS solid (Section 2.3): degree, open knot vectors (end multiplicity
 * degree+1, length n_ctrl+degree+1), control points [n0][n1][n2][3] C-order,
 * weights [n0][n1][n2] or NULL for a B-spline solid.  Host pointers. */
typedef struct {
  int degree[3];
  int n_ctrl[3];
  const double* knots[3];
  const double* ctrl_xyz;
  const double* weights;
} ttiga_geometry;

/* Solution space (Section 3.3): degree p, n basis per direction (n >= p+1),
 * n_gauss Gauss-Legendre points per knot span (0 means p+1, at most 8). */
typedef struct {
  int degree;
  int n_basis[3];
  int n_gauss;
} ttiga_discretization;

/* Source term f (Section 3.1).  For FOURIER: n_modes entries in a, phi and
 * n_modes x 3 in k (host pointers, C order). */
typedef struct {
  int kind;
  int n_modes;
  const double* a;
  const double* k;
  const double* phi;
  double origin[3];
  double scale;
} ttiga_source;

/* Boundary data per face (Section 3.1, u = u_bar on Gamma_D). */
typedef struct {
  int kind[6];
  double value[6];
} ttiga_dirichlet;

typedef struct {
  double tt_eps;      /* TT tolerance of compression and rounding */
  double rel_res_tol; /* plain TT-CG: stop when ||F_I - K_II u||_2 <= tol ||F_I||_2;
                         with precond: when ||P^-1 (F_I - K_II u)||_2 <= tol ||u||_2, an
                         estimate of the relative error of u (P^-1 K is near the identity) */
  int max_iter;
  int max_rank;       /* cap on every TT rank; exceeding it fails with E_RANKCAP */
  int precision;      /* TTIGA_FP64; or TTIGA_FP32 / TTIGA_BF16: K_II stored in that type and
                         its products with FP32 arithmetic inside the corrections of an
                         iterative refinement whose residual, updates and roundings are
                         FP64 (needs precond = 1) */
  int precond;        /* 1: separable Laplacian preconditioner, 0: plain TT-CG */
  size_t sample_chunk_bytes; /* 0: automatic (the Gauss-grid factor samples are held whole
                         up to 2 GiB, beyond that sampled and compressed in chunks of
                         second-direction slabs of at most 2 GiB); > 0: always stream in
                         chunks of at most this many bytes (at least one slab) when the
                         first direction has more than 64 Gauss points */
  int compression;    /* TTIGA_COMPRESS_AUTO (0): grids above 64 points per direction are
                         compressed by cross approximation of the first unfolding (sampled
                         column fibers, pivoted interpolation slices), verified on random
                         grid points, with TT-SVD as the fallback; TTIGA_COMPRESS_SVD (1):
                         TT-SVD of the whole (or streamed) Gauss-grid samples only */
  double assembly_eps; /* 0: tt_eps; > 0: relative tolerance of the assembly alone (factor
                         compression, the TT-rounded sums K and F, the lifted right-hand
                         side), independent of the solve's roundings.  The solution of a
                         non-separable geometry can move by far more than tt_eps when the
                         compressed operator drops a small singular value, so callers that
                         need the solution to about tt_eps set this well below it. */
  int solver;         /* TTIGA_SOLVER_CG (0): truncated TT-CG, preconditioned when precond = 1;
                         TTIGA_SOLVER_AMEN (1): the AMEn solve of Section 4.1.2 (alternating
                         local solves of one core, enrichment by the residual), FP64 only, with
                         local systems preconditioned by the projection of the separable
                         preconditioner whatever precond says; it stops on the same test as the
                         preconditioned TT-CG, ||P^-1 (F_I - K_II u)|| <= tol ||u|| */
} ttiga_options;

#define TTIGA_SOLVER_CG 0
#define TTIGA_SOLVER_AMEN 1

#define TTIGA_COMPRESS_AUTO 0
#define TTIGA_COMPRESS_SVD 1

typedef struct {
  int status;
  int rank_R[6][4];  /* TT ranks of R_00, R_11, R_22, R_01, R_02, R_12 (all 0: dropped) */
  int rank_fJ[4];    /* TT ranks of f det J */
  int rank_K[4];     /* TT ranks of the assembled K (before boundary reduction) */
  int rank_F[4];
  double min_detJ;
  double max_R_norm;  /* max_ij ||R_ij||_F over the Gauss grid */
  double time_ms[4];  /* basis+geometry, compression, core assembly+rounding, boundary */
  int compression_path; /* 0 TT-SVD of the whole grid, 1 streamed TT-SVD, 2 cross approximation,
                           3 cross rejected by its probe check, then streamed TT-SVD */
  long long samples;  /* factor sample points evaluated (det J-only points not counted) */
} ttiga_assembly_stats;

typedef struct {
  int status;
  int iterations;
  double rel_res;    /* true ||F_I - K_II u|| / ||F_I|| of the returned solution */
  double rel_pres;   /* ||P^-1 r|| / ||u||, the error estimate of the stopping test (precond only) */
  int rank_u[4];
  int max_rank_seen;
  int precond_terms; /* exponential-sum terms of the preconditioner (0: none) */
  double precond_err;/* max relative error of that sum on the spectrum interval */
  double precond_setup_ms; /* preconditioner set-up time within time_ms */
  double time_ms;
  int refine_steps;  /* mixed precision: FP64 refinement steps (iterations counts the inner ones) */
  int local_iterations; /* AMEn: CG iterations of all local solves (iterations counts half-sweeps) */
} ttiga_solve_stats;

/* Plain views of caller-owned device TT data (used by the standalone ops). */
typedef struct {
  int n[3];
  int r[4];
  const double* core[3]; /* device pointers, layout [r_k][n_k][r_{k+1}] */
} ttiga_tt_view;

typedef struct {
  int n[3];
  int p;                 /* half band width; 2p+1 band entries per row */
  int r[4];
  const double* core[3]; /* device pointers, layout [r_k][n_k][2p+1][r_{k+1}] */
} ttiga_ttm_view;

int ttiga_version(int* major, int* minor);

/* Context on HIP device `device`, enqueuing on `hip_stream` (a hipStream_t,
 * owned by the caller, NULL = the null stream). */
int ttiga_create(int device, void* hip_stream, ttiga_ctx** out);
int ttiga_destroy(ttiga_ctx* ctx);

/* Device memory for all library allocations: [dev_ptr, dev_ptr + bytes) is
 * sub-allocated by the library and must outlive the context and every
 * problem created on it.  Without a workspace the library allocates device
 * memory itself.  May be called once, before the first allocation. */
int ttiga_set_workspace(ttiga_ctx* ctx, void* dev_ptr, size_t bytes);

const char* ttiga_last_error(void);

/* Host-only check of a problem description (no device work): the status
 * ttiga_problem_create would return for it before touching the GPU. */
int ttiga_validate(const ttiga_geometry* geo, const ttiga_discretization* disc, const ttiga_source* src,
                   const ttiga_dirichlet* bc, const ttiga_options* opt);

/* Copy and validate one problem description.  The inputs may be freed on return. */
int ttiga_problem_create(ttiga_ctx* ctx, const ttiga_geometry* geo, const ttiga_discretization* disc,
                         const ttiga_source* src, const ttiga_dirichlet* bc, const ttiga_options* opt,
                         ttiga_problem** out);
int ttiga_problem_destroy(ttiga_problem* prob);

/* Assembly (Sections 4.2-4.3): basis tables, geometry factors at the Gauss
 * grid, TT compression, TT cores of the nine K_ij and of F, sum + rounding,
 * boundary reduction.  K and F stay on the device, owned by the problem. */
int ttiga_assemble(ttiga_problem* prob, ttiga_assembly_stats* stats);

/* TT solve of the reduced system K_II u_I = F_I - K_IB u_B (Section 4.3) with the
 * assembled TT operator and right-hand side.  options.solver = TTIGA_SOLVER_AMEN runs the
 * paper's solver (Section 4.1.2: AMEn, alternating local solves of one core with residual
 * enrichment; FP64); TTIGA_SOLVER_CG runs truncated TT-CG (precond = 0) or flexible
 * preconditioned TT-CG (precond = 1), optionally inside FP64 iterative refinement
 * (precision FP32/BF16).  The solution TT stays on the device, owned by the problem.
 * Errors: E_STATE before ttiga_assemble; E_ARG for AMEn with a precision other than FP64;
 * E_RANKCAP when a rounded TT needs more than max_rank; E_NOTCONV when the tolerance is
 * not met in max_iter iterations (AMEn: half-sweeps, at most 60) (the solution and stats
 * are still valid); E_HIP / E_OOM on device failures. */
int ttiga_solve(ttiga_problem* prob, ttiga_solve_stats* stats);

/* Ranks and mode sizes of the interior solution TT u_I (Section 4.1.1 format: ranks
 * r_0 = 1, r_1, r_2, r_3 = 1, modes n_d - (number of Dirichlet faces in direction d)),
 * so that a caller can size the buffer of ttiga_get_solution.  E_STATE before a solve. */
int ttiga_solution_ranks(const ttiga_problem* prob, int ranks[4], int n[3]);

/* The solution TT of Section 4.1.2 (the output of the solve): copies the interior
 * cores, concatenated in paper order [r0][n1][r1] | [r1][n2][r2] | [r2][n3][r3],
 * row-major FP64, into caller-owned host memory `dst` holding `count` doubles.
 * E_ARG if dst is null or count is below the total; E_STATE before a solve. */
int ttiga_get_solution(const ttiga_problem* prob, double* dst, size_t count);

/* Accuracy of the solution (Section 5, eq. L2norm read with squares and a root): the
 * relative L2 error ||u_h - u||_L2(Omega) / ||u||_L2(Omega) against an exact solution u
 * (TTIGA_EXACT_*; params as listed there, else NULL), by Gauss quadrature with
 * p + extra_gauss points per knot span on the exact geometry (dOmega = det J dxi), all of it
 * evaluated in TT format on the device: u_h on the grid from the solution cores, u and
 * w det J compressed by TT-SVD at 1e-13, their difference rounded by Householder sweeps and
 * its weighted square norm contracted core by core.  out = {relative error, ||u_h - u||,
 * ||u||} (host).  E_STATE before a solve; E_ARG on an unknown kind, bad parameters or
 * p + extra_gauss > 16; E_DETJ if det J <= 0 on the error grid. */
int ttiga_l2_error(ttiga_problem* prob, int exact_kind, const double* params, int extra_gauss, double out[3]);

/* Compression ratios (entries of the full-grid object over entries of its TT cores, the
 * figure the paper reports for its operators and vectors in Section 5): out[0] K^TT (banded
 * cores) against the sparse IGA stiffness matrix, whose non-zeros are
 * prod_d (n_d (2p+1) - p (p+1)); out[1] K^TT against the dense N x N matrix (dense TT-matrix
 * cores r n n r' counted); out[2] F^TT against N values; out[3] the solution TT against the
 * N_I interior values (0 before a solve).  E_STATE before ttiga_assemble. */
int ttiga_compression_ratios(ttiga_problem* prob, double out[4]);

/* Which TT of an assembled problem a query refers to. */
#define TTIGA_WHICH_K 0        /* full K, banded TT-matrix cores */
#define TTIGA_WHICH_F 1        /* full F */
#define TTIGA_WHICH_KII 2      /* interior K_II, banded */
#define TTIGA_WHICH_RHS 3      /* F_I - K_IB u_B */
#define TTIGA_WHICH_FACTOR0 10 /* +f, f = 0..6: TT of R_00, R_11, R_22, R_01, R_02, R_12, f det J */

/* Ranks and mode sizes of an assembled TT; for the banded matrices n is the
 * number of rows per direction and `band` is set to 2p+1 (1 for tensors).
 * Ranks are all zero for a factor that was truncated to the zero tensor. */
int ttiga_problem_tt_info(const ttiga_problem* prob, int which, int ranks[4], int n[3], int* band);

/* Copy the cores of an assembled TT to host memory (paper order, concatenated). */
int ttiga_problem_tt_copy(const ttiga_problem* prob, int which, double* dst, size_t count);

/* Geometry factors (eq. Rxi and the integrand of eq. ffinal) at `count`
 * parametric points pts[count][3] (host, each coordinate in [0,1]):
 * out[7][count] (host) = R_00, R_11, R_22, R_01, R_02, R_12, f det J,
 * det_out[count] (host, may be NULL).  Same kernel as the Gauss-grid sampling. */
int ttiga_sample_factors(ttiga_problem* prob, const double* pts, size_t count, double* out,
                         double* det_out);

/* Standalone banded TT-matvec y = K x on caller device data: y is written to a
 * library-owned TT (ranks r_K * r_x), returned in *out (free with ttiga_tt_free). */
int ttiga_tt_matvec(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, ttiga_tt** out);

/* Dense FP64 product C[b] = alpha op(A[b]) op(B[b]) + beta C[b] on the context stream:
 * the kernel behind the core contractions of this library (TT-matrix x TT-vector,
 * Section 4.1.1; the QR/SVD products of TT-rounding), exposed for parity tests and tile
 * tuning.  Row-major device operands: op(A) is M x K (A stored M x K with leading
 * dimension lda, or K x M when ta != 0), op(B) is K x N (B stored K x N with ldb, or
 * N x K when tb != 0), C is M x N with ldc; batch >= 1 products at element strides sA,
 * sB, sC.  plan: NULL for the library's own choice (its tuned table, else its shape
 * rule), else {bm, bn, kchunk} with (bm, bn) one of (64, 64), (128, 64), (64, 128), (64, 16),
 * (16, 64) and
 * kchunk 0 (the whole contraction in one pass) or a multiple of 32 (the contraction cut
 * into chunks of that length, partials summed in chunk order).  Synchronises the stream.
 * E_ARG on null pointers, M, N, K or batch < 1, a leading dimension shorter than a row, a
 * plan outside that set, or batch times chunks above 65535; the partial-tile workspace of
 * a split product comes from the context's allocator (E_OOM). */
int ttiga_gemm_f64(ttiga_ctx* ctx, int ta, int tb, int M, int N, int K, double alpha, const double* A,
                   long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
                   long sC, int batch, const int* plan);

/* The product of ttiga_gemm_f64 with both operands rounded to dtype (TTIGA_FP32, or
 * TTIGA_BF16 through FP32; round to nearest even) as they are staged, MFMA in that type with
 * FP32 accumulation, FP64 in and out: the contraction of the mixed-precision solves' inner
 * corrections (their Gram matrices, preconditioner transforms and rounded operator products).
 * Arguments as ttiga_gemm_f64 without a plan; E_ARG also for any other dtype. */
int ttiga_gemm_lowp(ttiga_ctx* ctx, int dtype, int ta, int tb, int M, int N, int K, double alpha, const double* A,
                    long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
                    long sC, int batch);

/* The same product with the operator cores rounded to dtype (TTIGA_FP32 or TTIGA_BF16,
 * round to nearest even; BF16 through FP32), the vector cores to FP32, FP32 products
 * and band sums, and the result cores in FP64: the contraction of the mixed-precision
 * solve, exposed for accuracy checks and timing. */
int ttiga_tt_matvec_lowp(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, int dtype,
                         ttiga_tt** out);

/* Rounded product y = round(alpha K x + beta z, eps) without forming the product cores
 * (the TT solve's residual and operator products when K x would be large, e.g. the
 * complex-geometry configuration): a randomised rounding whose Gaussian TT sketch, of
 * width sketch_rank + 10 widened by 12 while the rounded rank saturates it, is contracted
 * through the K and x cores one at a time, followed by the deterministic rounding
 * (Oseledets 2011) of the small sketched train at relative eps.  z may be NULL (then beta
 * is ignored); its mode sizes must equal x's.  The sketch is drawn from the context's
 * counter exactly as the rounding of an explicit train draws it.  Result in a library-owned
 * TT (*out, free with ttiga_tt_free); E_ARG on size mismatches. */
int ttiga_tt_matvec_round(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, double alpha,
                          const ttiga_tt_view* z, double beta, double eps, int sketch_rank, ttiga_tt** out);

/* Standalone TT-rounding (Oseledets 2011, used after each summation of
 * Section 4.2.1): y = round(x, eps) with per-unfolding threshold
 * eps * ||x||_F / sqrt(2). */
int ttiga_tt_round(ttiga_ctx* ctx, const ttiga_tt_view* x, double eps, ttiga_tt** out);

/* Standalone TT inner product <x, y> (left-to-right contraction), result to host. */
int ttiga_tt_dot(ttiga_ctx* ctx, const ttiga_tt_view* x, const ttiga_tt_view* y, double* out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): ttiga_tt_dot with its temporaries in a fixed 64 MiB
 * device array per GPU (held until the process ends) instead of the workspace, so the call
 * allocates nothing, does not synchronise, and writes <x, y> to the caller's device double
 * out_dev on the context stream (the same bits as ttiga_tt_dot).  Views as for ttiga_tt_dot
 * (caller-owned device cores).  E_ARG when the contraction needs more scratch than 64 MiB
 * (e.g. ranks above 128 at mode sizes of 256; the message gives the need), on null or
 * mismatched views; E_STATE while profiling (ttiga_profile) is on.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other threads)
 * race, so a caller serialises them. */
int ttiga_tt_dot_noalloc(ttiga_ctx* ctx, const ttiga_tt_view* x, const ttiga_tt_view* y, double* out_dev);

/* TT-SVD of a dense device tensor A[n0][n1][n2] with absolute per-unfolding
 * threshold delta (randomised range finder above 64 points per mode). */
int ttiga_tt_compress(ttiga_ctx* ctx, const double* A, const int n[3], double delta, ttiga_tt** out);

/* Per-kernel-class timing: HIP events recorded around each instrumented launch
 * on the context stream, plus the algorithmic flops and bytes of the launch
 * (operation counts of the method, not of any padding).  enable = 1 starts,
 * 0 stops, -1 clears the counters. */
typedef struct {
  char name[32];
  long launches;
  double total_ms;
  double flops;
  double bytes;
} ttiga_kernel_stat;

int ttiga_profile(ttiga_ctx* ctx, int enable);

/* Copies up to `capacity` entries; *count receives the number of kernel classes. */
int ttiga_profile_read(ttiga_ctx* ctx, ttiga_kernel_stat* out, int capacity, int* count);

int ttiga_tt_info(const ttiga_tt* t, int ranks[4], int n[3]);
int ttiga_tt_copy(const ttiga_tt* t, double* dst, size_t count); /* to host, paper order */
int ttiga_tt_free(ttiga_tt* t);
/* Device view of a library-owned TT (pointers valid until ttiga_tt_free). */
int ttiga_tt_view_of(const ttiga_tt* t, ttiga_tt_view* view);

/* ------------------------------------------------------------------------
 * Many independent problems at once.
 *
 * Each problem is the whole pipeline of Sections 4.2-4.3 followed by the TT
 * solve, as in ttiga_assemble + ttiga_solve.  An executor runs them on several
 * lanes: one host worker thread and one HIP stream each (default priority),
 * so the latency-bound steps of different problems (small QR/SVD sweeps,
 * host-side rank decisions) overlap on the device.  Device memory comes from a
 * pool carved out of the context's workspace; a problem starts only when its
 * footprint estimate fits what the running problems leave of the pool
 * (continuous batching: a problem is admitted as soon as a lane and the
 * memory free up), and every problem runs in an arena of that size (overruns
 * are served from the pool).  The sketch seeds are reset per problem and every
 * reduction has a fixed order, so a result does not depend on the other
 * problems in the mix or on the lane it ran on.
 * ------------------------------------------------------------------------ */
typedef struct {
  const ttiga_geometry* geo;
  const ttiga_discretization* disc;
  const ttiga_source* src;
  const ttiga_dirichlet* bc;
  const ttiga_options* opt;
} ttiga_request;

typedef struct {
  int status;               /* TTIGA_OK, TTIGA_E_NOTCONV (solution still valid) or the error */
  int lane;                 /* executor lane that ran it */
  int rank_u[4];            /* solution TT ranks (all 0 if there is no solution) */
  int n[3];                 /* interior sizes of the solution */
  ttiga_assembly_stats assembly;
  ttiga_solve_stats solve;
  double queue_ms;          /* submission -> start */
  double run_ms;            /* start -> solution resident */
  double latency_ms;        /* submission -> solution resident */
  size_t footprint_bytes;   /* admitted footprint estimate */
  size_t peak_bytes;        /* high-water mark of the problem's device memory */
  char error[128];          /* message of a failed problem */
} ttiga_result;

/* Host-only: footprint estimate (bytes) that admission uses for a request. */
int ttiga_footprint(const ttiga_request* req, size_t* bytes);

/* Batched mode: assemble and solve count problems on `lanes` lanes within
 * hbm_budget bytes of the context's workspace (0: the largest free block less
 * 1 GiB).  Problems start largest footprint first.  On return solutions[i] is
 * a library-owned TT on the context (free with ttiga_tt_free), or NULL when
 * problem i failed; results[i] holds its status and statistics.  The call
 * itself fails only on bad arguments or when the pool cannot be set up; a
 * problem that fails does not affect the others.  Each lane is a host thread
 * with its own HIP stream; lanes overlap on the device only when the HIP
 * runtime gives every active stream its own hardware queue
 * (GPU_MAX_HW_QUEUES >= lanes + the caller's streams, set before the runtime
 * starts).  Per-discretisation plans (the preconditioner's 1-D eigenbases)
 * are computed once per context, kept in its workspace, and shared by all
 * batches and servers built on it. */
int ttiga_solve_batch(ttiga_ctx* ctx, int count, const ttiga_request* reqs, int lanes,
                      size_t hbm_budget, ttiga_tt** solutions, ttiga_result* results);

/* Serving mode.  A server owns a pool of hbm_budget bytes of the context's
 * workspace and `lanes` lanes.  ttiga_server_submit copies and validates the
 * request and queues it (first come, first served; a later problem that fits
 * may start before an earlier one that does not, a bounded number of times);
 * it returns TTIGA_E_ADMISSION when the request's footprint exceeds the whole
 * pool or `max_queue` requests are already waiting.  ttiga_server_poll
 * returns TTIGA_PENDING while the request waits or runs (wait_ms > 0 blocks up
 * to that long, < 0 until it is done) and TTIGA_OK once `out` holds the
 * result.  Solutions stay resident in the pool until ttiga_server_release.
 * Submit, poll, solution access and release may be called from any thread. */
typedef struct ttiga_server ttiga_server;

int ttiga_server_create(ttiga_ctx* ctx, size_t hbm_budget, int lanes, int max_queue,
                        ttiga_server** out);
int ttiga_server_submit(ttiga_server* srv, const ttiga_request* req, unsigned long long* ticket);
int ttiga_server_poll(ttiga_server* srv, unsigned long long ticket, int wait_ms, ttiga_result* out);
/* Device view of a finished request's solution (valid until release). */
int ttiga_server_solution(ttiga_server* srv, unsigned long long ticket, ttiga_tt_view* view);
/* Host copy of a finished request's solution cores, paper order. */
int ttiga_server_copy_solution(ttiga_server* srv, unsigned long long ticket, double* dst, size_t count);
int ttiga_server_release(ttiga_server* srv, unsigned long long ticket);
/* Waits for running and queued requests, then frees the pool and the lanes. */
int ttiga_server_destroy(ttiga_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* TTIGA_H */
