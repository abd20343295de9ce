"""ctypes binding of libttiga.so (the C ABI in include/ttiga.h).

Argument marshalling only: every step of assembly and solve runs in the
library's HIP kernels.  PyTorch provides device memory (workspace and operand
buffers) and the stream; nothing here computes on the CPU.  Loading fails
loudly when the library has not been built.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libttiga.so")

TTIGA_OK = 0
TTIGA_PENDING = 1
TTIGA_E_ARG = -1
TTIGA_E_KNOTS = -2
TTIGA_E_GEOM = -3
TTIGA_E_DETJ = -4
TTIGA_E_OOM = -5
TTIGA_E_ADMISSION = -6
TTIGA_E_NOTCONV = -7
TTIGA_E_RANKCAP = -8
TTIGA_SOLVER_CG = 0
TTIGA_SOLVER_AMEN = 1
TTIGA_E_STATE = -9
TTIGA_E_HIP = -10

WHICH_K, WHICH_F, WHICH_KII, WHICH_RHS, WHICH_FACTOR0 = 0, 1, 2, 3, 10
TTIGA_EXACT_MANUFACTURED_ANNULUS, TTIGA_EXACT_RADIAL_LOG, TTIGA_EXACT_SINE_XY = 1, 2, 3

EXPORTED = (
    "ttiga_version", "ttiga_create", "ttiga_destroy", "ttiga_set_workspace", "ttiga_last_error",
    "ttiga_validate", "ttiga_problem_create", "ttiga_problem_destroy", "ttiga_assemble", "ttiga_solve",
    "ttiga_solution_ranks", "ttiga_get_solution", "ttiga_l2_error", "ttiga_compression_ratios",
    "ttiga_problem_tt_info", "ttiga_problem_tt_copy",
    "ttiga_sample_factors", "ttiga_gemm_f64", "ttiga_gemm_lowp", "ttiga_tt_matvec", "ttiga_tt_matvec_round", "ttiga_tt_round", "ttiga_tt_dot",
    "ttiga_tt_dot_noalloc",
    "ttiga_tt_compress", "ttiga_tt_matvec_lowp", "ttiga_tt_info", "ttiga_tt_copy", "ttiga_tt_free", "ttiga_profile",
    "ttiga_profile_read", "ttiga_tt_view_of", "ttiga_footprint", "ttiga_solve_batch",
    "ttiga_server_create", "ttiga_server_submit", "ttiga_server_poll", "ttiga_server_solution",
    "ttiga_server_copy_solution", "ttiga_server_release", "ttiga_server_destroy",
)

c_int_p = ctypes.POINTER(ctypes.c_int)
c_dbl_p = ctypes.POINTER(ctypes.c_double)


class Geometry(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int * 3), ("n_ctrl", ctypes.c_int * 3),
                ("knots", c_dbl_p * 3), ("ctrl_xyz", c_dbl_p), ("weights", c_dbl_p)]


class Discretization(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int), ("n_basis", ctypes.c_int * 3), ("n_gauss", ctypes.c_int)]


class Source(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n_modes", ctypes.c_int), ("a", c_dbl_p), ("k", c_dbl_p),
                ("phi", c_dbl_p), ("origin", ctypes.c_double * 3), ("scale", ctypes.c_double)]


class Dirichlet(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int * 6), ("value", ctypes.c_double * 6)]


class Options(ctypes.Structure):
    _fields_ = [("tt_eps", ctypes.c_double), ("rel_res_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("max_rank", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int),
                ("sample_chunk_bytes", ctypes.c_size_t), ("compression", ctypes.c_int),
                ("assembly_eps", ctypes.c_double), ("solver", ctypes.c_int)]


class AssemblyStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("rank_R", (ctypes.c_int * 4) * 6),
                ("rank_fJ", ctypes.c_int * 4), ("rank_K", ctypes.c_int * 4),
                ("rank_F", ctypes.c_int * 4), ("min_detJ", ctypes.c_double),
                ("max_R_norm", ctypes.c_double), ("time_ms", ctypes.c_double * 4),
                ("compression_path", ctypes.c_int), ("samples", ctypes.c_longlong)]


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("rel_res", ctypes.c_double),
                ("rel_pres", ctypes.c_double), ("rank_u", ctypes.c_int * 4), ("max_rank_seen", ctypes.c_int),
                ("precond_terms", ctypes.c_int), ("precond_err", ctypes.c_double),
                ("precond_setup_ms", ctypes.c_double), ("time_ms", ctypes.c_double),
                ("refine_steps", ctypes.c_int), ("local_iterations", ctypes.c_int)]


class TTView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("r", ctypes.c_int * 4), ("core", ctypes.c_void_p * 3)]


class TTMView(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("p", ctypes.c_int), ("r", ctypes.c_int * 4),
                ("core", ctypes.c_void_p * 3)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_long), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("geo", ctypes.POINTER(Geometry)), ("disc", ctypes.POINTER(Discretization)),
                ("src", ctypes.POINTER(Source)), ("bc", ctypes.POINTER(Dirichlet)),
                ("opt", ctypes.POINTER(Options))]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("lane", ctypes.c_int), ("rank_u", ctypes.c_int * 4),
                ("n", ctypes.c_int * 3), ("assembly", AssemblyStats), ("solve", SolveStats),
                ("queue_ms", ctypes.c_double), ("run_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("footprint_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("error", ctypes.c_char * 128)]


def _result_dict(r):
    return dict(status=r.status, lane=r.lane, rank_u=list(r.rank_u), n=list(r.n),
                iterations=r.solve.iterations, rel_res=r.solve.rel_res, rel_pres=r.solve.rel_pres,
                max_rank_seen=r.solve.max_rank_seen, rank_K=list(r.assembly.rank_K),
                refine_steps=r.solve.refine_steps, local_iterations=r.solve.local_iterations,
                assembly_ms=list(r.assembly.time_ms),
                compression_path=r.assembly.compression_path, solve_ms=r.solve.time_ms,
                precond_setup_ms=r.solve.precond_setup_ms, queue_ms=r.queue_ms, run_ms=r.run_ms, latency_ms=r.latency_ms,
                footprint_bytes=r.footprint_bytes, peak_bytes=r.peak_bytes, error=r.error.decode())


class TTIGAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ttiga error {code}: {msg}")
        self.code = code


_LIB = None


def load(path=LIB_PATH):
    """Load libttiga.so and declare its signatures; raises if it is missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with paper_2509_13224_amd/build.py")
    lib = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    sig = {
        "ttiga_version": (ctypes.c_int, [c_int_p, c_int_p]),
        "ttiga_create": (ctypes.c_int, [ctypes.c_int, vp, ctypes.POINTER(vp)]),
        "ttiga_destroy": (ctypes.c_int, [vp]),
        "ttiga_set_workspace": (ctypes.c_int, [vp, vp, ctypes.c_size_t]),
        "ttiga_last_error": (ctypes.c_char_p, []),
        "ttiga_problem_create": (ctypes.c_int, [vp, ctypes.POINTER(Geometry), ctypes.POINTER(Discretization),
                                                ctypes.POINTER(Source), ctypes.POINTER(Dirichlet),
                                                ctypes.POINTER(Options), ctypes.POINTER(vp)]),
        "ttiga_validate": (ctypes.c_int, [ctypes.POINTER(Geometry), ctypes.POINTER(Discretization),
                                          ctypes.POINTER(Source), ctypes.POINTER(Dirichlet),
                                          ctypes.POINTER(Options)]),
        "ttiga_problem_destroy": (ctypes.c_int, [vp]),
        "ttiga_assemble": (ctypes.c_int, [vp, ctypes.POINTER(AssemblyStats)]),
        "ttiga_solve": (ctypes.c_int, [vp, ctypes.POINTER(SolveStats)]),
        "ttiga_solution_ranks": (ctypes.c_int, [vp, c_int_p, c_int_p]),
        "ttiga_get_solution": (ctypes.c_int, [vp, c_dbl_p, ctypes.c_size_t]),
        "ttiga_l2_error": (ctypes.c_int, [vp, ctypes.c_int, c_dbl_p, ctypes.c_int, c_dbl_p]),
        "ttiga_compression_ratios": (ctypes.c_int, [vp, c_dbl_p]),
        "ttiga_problem_tt_info": (ctypes.c_int, [vp, ctypes.c_int, c_int_p, c_int_p, c_int_p]),
        "ttiga_problem_tt_copy": (ctypes.c_int, [vp, ctypes.c_int, c_dbl_p, ctypes.c_size_t]),
        "ttiga_sample_factors": (ctypes.c_int, [vp, c_dbl_p, ctypes.c_size_t, c_dbl_p, c_dbl_p]),
        "ttiga_gemm_f64": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, vp, ctypes.c_long, ctypes.c_long, vp, ctypes.c_long,
                                          ctypes.c_long, ctypes.c_double, vp, ctypes.c_long, ctypes.c_long,
                                          ctypes.c_int, c_int_p]),
        "ttiga_gemm_lowp": (ctypes.c_int, [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_double, vp, ctypes.c_long, ctypes.c_long, vp,
                                           ctypes.c_long, ctypes.c_long, ctypes.c_double, vp, ctypes.c_long,
                                           ctypes.c_long, ctypes.c_int]),
        "ttiga_tt_matvec": (ctypes.c_int, [vp, ctypes.POINTER(TTMView), ctypes.POINTER(TTView),
                                           ctypes.POINTER(vp)]),
        "ttiga_tt_matvec_lowp": (ctypes.c_int, [vp, ctypes.POINTER(TTMView), ctypes.POINTER(TTView), ctypes.c_int,
                                                ctypes.POINTER(vp)]),
        "ttiga_tt_round": (ctypes.c_int, [vp, ctypes.POINTER(TTView), ctypes.c_double, ctypes.POINTER(vp)]),
        "ttiga_tt_matvec_round": (ctypes.c_int, [vp, ctypes.POINTER(TTMView), ctypes.POINTER(TTView), ctypes.c_double,
                                                 ctypes.POINTER(TTView), ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                 ctypes.POINTER(vp)]),
        "ttiga_tt_dot": (ctypes.c_int, [vp, ctypes.POINTER(TTView), ctypes.POINTER(TTView), c_dbl_p]),
        "ttiga_tt_dot_noalloc": (ctypes.c_int, [vp, ctypes.POINTER(TTView), ctypes.POINTER(TTView), vp]),
        "ttiga_tt_compress": (ctypes.c_int, [vp, vp, c_int_p, ctypes.c_double, ctypes.POINTER(vp)]),
        "ttiga_tt_info": (ctypes.c_int, [vp, c_int_p, c_int_p]),
        "ttiga_tt_copy": (ctypes.c_int, [vp, c_dbl_p, ctypes.c_size_t]),
        "ttiga_tt_free": (ctypes.c_int, [vp]),
        "ttiga_profile": (ctypes.c_int, [vp, ctypes.c_int]),
        "ttiga_profile_read": (ctypes.c_int, [vp, ctypes.POINTER(KernelStat), ctypes.c_int, c_int_p]),
        "ttiga_tt_view_of": (ctypes.c_int, [vp, ctypes.POINTER(TTView)]),
        "ttiga_footprint": (ctypes.c_int, [ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_size_t)]),
        "ttiga_solve_batch": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(Request), ctypes.c_int,
                                             ctypes.c_size_t, ctypes.POINTER(vp), ctypes.POINTER(Result)]),
        "ttiga_server_create": (ctypes.c_int, [vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(vp)]),
        "ttiga_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request),
                                               ctypes.POINTER(ctypes.c_ulonglong)]),
        "ttiga_server_poll": (ctypes.c_int, [vp, ctypes.c_ulonglong, ctypes.c_int, ctypes.POINTER(Result)]),
        "ttiga_server_solution": (ctypes.c_int, [vp, ctypes.c_ulonglong, ctypes.POINTER(TTView)]),
        "ttiga_server_copy_solution": (ctypes.c_int, [vp, ctypes.c_ulonglong, c_dbl_p, ctypes.c_size_t]),
        "ttiga_server_release": (ctypes.c_int, [vp, ctypes.c_ulonglong]),
        "ttiga_server_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def _check(lib, code, ok=(TTIGA_OK,)):
    if code not in ok:
        raise TTIGAError(code, lib.ttiga_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(c_dbl_p)


def _ranks_of(cores):
    return [1, cores[0].shape[-1], cores[1].shape[-1], 1]


def split_cores(flat, n, r, band=1):
    """Concatenated paper-order cores -> list of arrays [r_k][n_k][(band)][r_{k+1}]."""
    out, off = [], 0
    for k in range(3):
        cnt = r[k] * n[k] * band * r[k + 1]
        shape = (r[k], n[k], band, r[k + 1]) if band > 1 else (r[k], n[k], r[k + 1])
        out.append(np.asarray(flat[off:off + cnt]).reshape(shape))
        off += cnt
    return out


class Context:
    """ttiga_create on a device and stream (default: torch's current stream on cuda:0).

    The library sub-allocates everything from one torch-owned device buffer of
    ``workspace_bytes`` (default 1 GiB); 0 lets the library allocate by itself.
    """

    def __init__(self, device=0, stream=None, workspace_bytes=1 << 30):
        import torch
        self.lib = load()
        self.torch = torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.device = device
        self._ws = None
        if workspace_bytes:
            self._ws = torch.empty(int(workspace_bytes), dtype=torch.uint8, device=f"cuda:{device}")
            _check(self.lib, self.lib.ttiga_set_workspace(self.h, ctypes.c_void_p(self._ws.data_ptr()),
                                                          ctypes.c_size_t(self._ws.numel())))

    def close(self):
        if self.h:
            self.lib.ttiga_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- profiling
    def profile(self, enable):
        _check(self.lib, self.lib.ttiga_profile(self.h, int(enable)))

    def profile_read(self):
        cnt = ctypes.c_int()
        _check(self.lib, self.lib.ttiga_profile_read(self.h, None, 0, ctypes.byref(cnt)))
        arr = (KernelStat * max(cnt.value, 1))()
        _check(self.lib, self.lib.ttiga_profile_read(self.h, arr, cnt.value, ctypes.byref(cnt)))
        return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                           flops=arr[i].flops, bytes=arr[i].bytes)
                for i in range(cnt.value)}

    # ---------------------------------------------------------------- problems
    def problem_create(self, pr, precond=0):
        return ProblemHandle(self, pr, precond)

    def solve_batch(self, problems, lanes=4, hbm_budget=0, precond=1):
        """ttiga_solve_batch over workloads.Problem descriptions.

        Returns a list of (result dict, solution cores on the host or None)."""
        count = len(problems)
        reqs, keep = make_requests(problems, precond)
        sols = (ctypes.c_void_p * max(count, 1))()
        res = (Result * max(count, 1))()
        _check(self.lib, self.lib.ttiga_solve_batch(self.h, count, reqs, int(lanes), ctypes.c_size_t(hbm_budget),
                                                    sols, res))
        out = []
        for i in range(count):
            cores = self._take(ctypes.c_void_p(sols[i])) if sols[i] else None
            out.append((_result_dict(res[i]), cores))
        return out

    def server(self, hbm_budget=0, lanes=4, max_queue=1024):
        return Server(self, hbm_budget, lanes, max_queue)

    # ---------------------------------------------------------------- standalone ops
    def _view(self, cores_dev):
        v = TTView()
        for k in range(3):
            v.n[k] = cores_dev[k].shape[1]
            v.core[k] = cores_dev[k].data_ptr()
        r = _ranks_of(cores_dev)
        for k in range(4):
            v.r[k] = r[k]
        return v

    def _take(self, handle):
        r = (ctypes.c_int * 4)()
        n = (ctypes.c_int * 3)()
        _check(self.lib, self.lib.ttiga_tt_info(handle, r, n))
        r, n = list(r), list(n)
        total = sum(r[k] * n[k] * r[k + 1] for k in range(3))
        flat = np.zeros(max(total, 1))
        _check(self.lib, self.lib.ttiga_tt_copy(handle, _dptr(flat), ctypes.c_size_t(flat.size)))
        self.lib.ttiga_tt_free(handle)
        if r[1] == 0:
            return None
        return split_cores(flat, n, r)

    def gemm_f64(self, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch=1, sA=0, sB=0, sC=0,
                 plan=None):
        """ttiga_gemm_f64 on device float64 tensors A, B, C (row-major, leading dimensions and
        batch strides in elements); plan = (bm, bn, kchunk) or None for the library's choice."""
        pl = (ctypes.c_int * 3)(*plan) if plan is not None else None
        _check(self.lib, self.lib.ttiga_gemm_f64(self.h, int(ta), int(tb), M, N, K, float(alpha), A.data_ptr(), lda,
                                                 sA, B.data_ptr(), ldb, sB, float(beta), C.data_ptr(), ldc, sC,
                                                 batch, pl))

    def gemm_lowp(self, dtype, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch=1, sA=0, sB=0, sC=0):
        """ttiga_gemm_lowp: the product with operands rounded to dtype (1 FP32, 2 BF16), MFMA in
        that type with FP32 accumulation; device float64 tensors in and out."""
        _check(self.lib, self.lib.ttiga_gemm_lowp(self.h, int(dtype), int(ta), int(tb), M, N, K, float(alpha),
                                                  A.data_ptr(), lda, sA, B.data_ptr(), ldb, sB, float(beta),
                                                  C.data_ptr(), ldc, sC, batch))

    def tt_matvec(self, K_cores_dev, p, x_cores_dev, dtype=None, copy=True):
        """y = K x; K banded cores [r][n][2p+1][r'] and x cores [r][n][r'] as device tensors.

        dtype TTIGA_FP32 / TTIGA_BF16 (1 / 2) selects the low-precision product.  copy=False
        frees the result on the device without copying it (timing runs) and returns None."""
        kv = TTMView()
        kv.p = p
        rK = [1, K_cores_dev[0].shape[-1], K_cores_dev[1].shape[-1], 1]
        for k in range(3):
            kv.n[k] = K_cores_dev[k].shape[1]
            kv.core[k] = K_cores_dev[k].data_ptr()
        for k in range(4):
            kv.r[k] = rK[k]
        xv = self._view(x_cores_dev)
        h = ctypes.c_void_p()
        if dtype:
            _check(self.lib, self.lib.ttiga_tt_matvec_lowp(self.h, ctypes.byref(kv), ctypes.byref(xv), int(dtype),
                                                           ctypes.byref(h)))
        else:
            _check(self.lib, self.lib.ttiga_tt_matvec(self.h, ctypes.byref(kv), ctypes.byref(xv), ctypes.byref(h)))
        if not copy:
            self.lib.ttiga_tt_free(h)
            return None
        return self._take(h)

    def tt_matvec_round(self, K_cores_dev, p, x_cores_dev, eps, alpha=1.0, z_cores_dev=None, beta=0.0,
                        sketch_rank=8):
        """round(alpha K x + beta z, eps) without forming K x (ttiga_tt_matvec_round)."""
        kv = TTMView()
        kv.p = p
        rK = [1, K_cores_dev[0].shape[-1], K_cores_dev[1].shape[-1], 1]
        for k in range(3):
            kv.n[k] = K_cores_dev[k].shape[1]
            kv.core[k] = K_cores_dev[k].data_ptr()
        for k in range(4):
            kv.r[k] = rK[k]
        xv = self._view(x_cores_dev)
        zp = ctypes.byref(self._view(z_cores_dev)) if z_cores_dev is not None else None
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_tt_matvec_round(self.h, ctypes.byref(kv), ctypes.byref(xv), ctypes.c_double(alpha),
                                                        zp, ctypes.c_double(beta), ctypes.c_double(eps),
                                                        ctypes.c_int(sketch_rank), ctypes.byref(h)))
        return self._take(h)

    def tt_round(self, cores_dev, eps):
        v = self._view(cores_dev)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_tt_round(self.h, ctypes.byref(v), ctypes.c_double(eps), ctypes.byref(h)))
        return self._take(h)

    def tt_dot(self, x_dev, y_dev):
        a, b = self._view(x_dev), self._view(y_dev)
        out = ctypes.c_double()
        _check(self.lib, self.lib.ttiga_tt_dot(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(out)))
        return out.value

    def tt_dot_noalloc(self, x_dev, y_dev, out_dev):
        """ttiga_tt_dot_noalloc: <x, y> written to the device float64 tensor out_dev (one
        element) on the context stream, without allocating; the caller synchronises."""
        a, b = self._view(x_dev), self._view(y_dev)
        _check(self.lib, self.lib.ttiga_tt_dot_noalloc(self.h, ctypes.byref(a), ctypes.byref(b),
                                                       ctypes.c_void_p(out_dev.data_ptr())))

    def tt_compress(self, A_dev, delta):
        n = (ctypes.c_int * 3)(*A_dev.shape)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_tt_compress(self.h, ctypes.c_void_p(A_dev.data_ptr()), n,
                                                    ctypes.c_double(delta), ctypes.byref(h)))
        return self._take(h)


def describe(pr, precond=0):
    """ctypes structs of a workloads.Problem; returns (structs tuple, keep-alive list)."""
    geo = pr.geometry
    keep = []

    def arr(x):
        a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
        keep.append(a)
        return a

    g = Geometry()
    for d in range(3):
        g.degree[d] = int(geo.degree[d])
        g.n_ctrl[d] = int(geo.ctrl.shape[d])
        g.knots[d] = _dptr(arr(geo.knots[d]))
    g.ctrl_xyz = _dptr(arr(geo.ctrl))
    g.weights = _dptr(arr(geo.weights)) if geo.weights is not None else None
    disc = Discretization()
    disc.degree = int(pr.disc.degree)
    for d in range(3):
        disc.n_basis[d] = int(pr.disc.n_basis[d])
    disc.n_gauss = int(pr.disc.n_gauss)
    src = Source()
    src.kind = int(pr.source.kind)
    src.n_modes = int(len(pr.source.a))
    src.a = _dptr(arr(pr.source.a))
    src.k = _dptr(arr(np.asarray(pr.source.k).reshape(-1, 3)))
    src.phi = _dptr(arr(pr.source.phi))
    for d in range(3):
        src.origin[d] = float(pr.source.origin[d])
    src.scale = float(pr.source.scale)
    bc = Dirichlet()
    for f in range(6):
        bc.kind[f] = int(pr.dirichlet.kind[f])
        bc.value[f] = float(pr.dirichlet.value[f])
    o = Options()
    o.tt_eps = pr.options.tt_eps
    o.rel_res_tol = pr.options.rel_res_tol
    o.max_iter = pr.options.max_iter
    o.max_rank = pr.options.max_rank
    o.precision = pr.options.precision
    o.precond = precond
    o.sample_chunk_bytes = int(getattr(pr.options, "sample_chunk_bytes", 0))
    o.compression = int(getattr(pr.options, "compression", 0))
    o.assembly_eps = float(getattr(pr.options, "assembly_eps", 0.0))
    o.solver = int(getattr(pr.options, "solver", TTIGA_SOLVER_CG))
    return (g, disc, src, bc, o), keep


def make_requests(problems, precond=1):
    """ctypes array of ttiga_request for a list of workloads.Problem (plus keep-alive list)."""
    keep = []
    reqs = (Request * max(len(problems), 1))()
    for i, pr in enumerate(problems):
        structs, k = describe(pr, precond)
        keep.append((structs, k))
        g, disc, src, bc, o = structs
        reqs[i].geo = ctypes.pointer(g)
        reqs[i].disc = ctypes.pointer(disc)
        reqs[i].src = ctypes.pointer(src)
        reqs[i].bc = ctypes.pointer(bc)
        reqs[i].opt = ctypes.pointer(o)
    return reqs, keep


def footprint(pr, precond=1):
    """ttiga_footprint: the admission estimate in bytes (host only)."""
    lib = load()
    reqs, keep = make_requests([pr], precond)
    out = ctypes.c_size_t()
    _check(lib, lib.ttiga_footprint(reqs, ctypes.byref(out)))
    return out.value


class Server:
    """ttiga_server_*: continuous batching of TT-IGA solves on one context."""

    def __init__(self, ctx, hbm_budget=0, lanes=4, max_queue=1024):
        self.ctx, self.lib = ctx, ctx.lib
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_server_create(ctx.h, ctypes.c_size_t(hbm_budget), int(lanes),
                                                      int(max_queue), ctypes.byref(h)))
        self.h = h

    def submit(self, pr, precond=1):
        """Returns a ticket; raises TTIGAError (code TTIGA_E_ADMISSION) when refused."""
        reqs, keep = make_requests([pr], precond)
        t = ctypes.c_ulonglong()
        _check(self.lib, self.lib.ttiga_server_submit(self.h, reqs, ctypes.byref(t)))
        return t.value

    def poll(self, ticket, wait_ms=0):
        """None while pending, else the result dict."""
        r = Result()
        code = _check(self.lib, self.lib.ttiga_server_poll(self.h, ticket, int(wait_ms), ctypes.byref(r)),
                      (TTIGA_OK, TTIGA_PENDING))
        return None if code == TTIGA_PENDING else _result_dict(r)

    def solution(self, ticket):
        """Host copy of the solution cores (paper order)."""
        v = TTView()
        _check(self.lib, self.lib.ttiga_server_solution(self.h, ticket, ctypes.byref(v)))
        r, n = list(v.r), list(v.n)
        total = sum(r[k] * n[k] * r[k + 1] for k in range(3))
        flat = np.zeros(max(total, 1))
        _check(self.lib, self.lib.ttiga_server_copy_solution(self.h, ticket, _dptr(flat), ctypes.c_size_t(flat.size)))
        if r[1] == 0:
            return None
        return split_cores(flat, n, r)

    def release(self, ticket):
        _check(self.lib, self.lib.ttiga_server_release(self.h, ticket))

    def close(self):
        if self.h:
            self.lib.ttiga_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def validate(pr, precond=0):
    """ttiga_validate: host-only status of a description (0 = acceptable)."""
    lib = load()
    (g, disc, src, bc, o), keep = describe(pr, precond)
    code = lib.ttiga_validate(ctypes.byref(g), ctypes.byref(disc), ctypes.byref(src), ctypes.byref(bc),
                              ctypes.byref(o))
    return code, lib.ttiga_last_error().decode()


class ProblemHandle:
    """ttiga_problem_create from a workloads.Problem description."""

    def __init__(self, ctx, pr, precond=0):
        self.ctx, self.lib = ctx, ctx.lib
        (g, disc, src, bc, o), keep = describe(pr, precond)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.ttiga_problem_create(ctx.h, ctypes.byref(g), ctypes.byref(disc), ctypes.byref(src),
                                                       ctypes.byref(bc), ctypes.byref(o), ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.ttiga_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def assemble(self):
        st = AssemblyStats()
        _check(self.lib, self.lib.ttiga_assemble(self.h, ctypes.byref(st)))
        return dict(rank_R=[list(r) for r in st.rank_R], rank_fJ=list(st.rank_fJ), rank_K=list(st.rank_K),
                    rank_F=list(st.rank_F), min_detJ=st.min_detJ, max_R_norm=st.max_R_norm,
                    time_ms=list(st.time_ms), compression_path=st.compression_path, samples=st.samples)

    def solve(self, allow_notconv=False):
        st = SolveStats()
        ok = (TTIGA_OK, TTIGA_E_NOTCONV) if allow_notconv else (TTIGA_OK,)
        code = _check(self.lib, self.lib.ttiga_solve(self.h, ctypes.byref(st)), ok)
        return dict(status=code, iterations=st.iterations, rel_res=st.rel_res, rel_pres=st.rel_pres,
                    rank_u=list(st.rank_u), max_rank_seen=st.max_rank_seen, precond_terms=st.precond_terms,
                    precond_err=st.precond_err, precond_setup_ms=st.precond_setup_ms, time_ms=st.time_ms,
                    refine_steps=st.refine_steps, local_iterations=st.local_iterations)

    def l2_error(self, exact_kind, params=None, extra_gauss=3):
        """ttiga_l2_error: relative L2 error of the solution against an exact solution, evaluated
        in TT format on the device (p + extra_gauss Gauss points per span)."""
        out = (ctypes.c_double * 3)()
        prm = (ctypes.c_double * 4)(*params) if params is not None else None
        _check(self.lib, self.lib.ttiga_l2_error(self.h, int(exact_kind), prm, int(extra_gauss), out))
        return dict(rel_l2=out[0], err_norm=out[1], exact_norm=out[2])

    def compression_ratios(self):
        """ttiga_compression_ratios: full-grid entries over TT entries for K (against the sparse
        and the dense matrix), F and the solution."""
        out = (ctypes.c_double * 4)()
        _check(self.lib, self.lib.ttiga_compression_ratios(self.h, out))
        return dict(K_sparse=out[0], K_dense=out[1], F=out[2], u=out[3])

    def solution(self):
        r = (ctypes.c_int * 4)()
        n = (ctypes.c_int * 3)()
        _check(self.lib, self.lib.ttiga_solution_ranks(self.h, r, n))
        r, n = list(r), list(n)
        total = sum(r[k] * n[k] * r[k + 1] for k in range(3))
        flat = np.zeros(max(total, 1))
        _check(self.lib, self.lib.ttiga_get_solution(self.h, _dptr(flat), ctypes.c_size_t(flat.size)))
        if r[1] == 0:
            return None
        return split_cores(flat, n, r)

    def tt(self, which):
        r = (ctypes.c_int * 4)()
        n = (ctypes.c_int * 3)()
        band = ctypes.c_int()
        _check(self.lib, self.lib.ttiga_problem_tt_info(self.h, which, r, n, ctypes.byref(band)))
        r, n, band = list(r), list(n), band.value
        total = sum(r[k] * n[k] * band * r[k + 1] for k in range(3))
        flat = np.zeros(max(total, 1))
        _check(self.lib, self.lib.ttiga_problem_tt_copy(self.h, which, _dptr(flat), ctypes.c_size_t(flat.size)))
        if r[1] == 0:
            return None
        return split_cores(flat, n, r, band)

    def sample_factors(self, pts):
        pts = np.ascontiguousarray(np.asarray(pts, dtype=np.float64))
        count = pts.shape[0]
        out = np.zeros((7, count))
        det = np.zeros(count)
        _check(self.lib, self.lib.ttiga_sample_factors(self.h, _dptr(pts), ctypes.c_size_t(count), _dptr(out), _dptr(det)))
        return out, det
