"""ctypes binding of libssmap (include/ssmap.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels. If the built
library is missing this module raises at load time; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SSMAP_LIB", os.path.join(HERE, "libssmap.so"))

SSMAP_OK = 0
SSMAP_EINVAL = -1
SSMAP_ENOMEM = -2
SSMAP_EDEVICE = -3
SSMAP_ENONFINITE = -4
SSMAP_ENODEV = -5
STATUS_NAMES = {0: "SSMAP_OK", -1: "SSMAP_EINVAL", -2: "SSMAP_ENOMEM", -3: "SSMAP_EDEVICE",
                -4: "SSMAP_ENONFINITE", -5: "SSMAP_ENODEV"}

PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
KERNELS = {"auto": 0, "unfused": 1, "fused": 2, "gemm": 3, "split": 4}
SSMAP_KEEP_AUX = 1
SSMAP_MONITOR_PRIMAL = 4
SSMAP_WARM_START = 8
MAX_HIST = 512

EXPORTS = ["ssmap_create", "ssmap_solve", "ssmap_solve_device", "ssmap_solve_device_noalloc",
           "ssmap_get_aux",
           "ssmap_get_stats", "ssmap_get_singular_values", "ssmap_last_error",
           "ssmap_destroy", "ssmap_version", "ssmap_set_mask", "ssmap_set_reference",
           "ssmap_set_initial", "ssmap_tune_beta",
           "ssmap_batch_create", "ssmap_batch_set_mask", "ssmap_batch_solve", "ssmap_batch_solve_device",
           "ssmap_batch_get_stats", "ssmap_batch_get_job_stats", "ssmap_batch_last_error",
           "ssmap_batch_destroy",
           "ssmap_server_create", "ssmap_server_add_dictionary", "ssmap_server_submit",
           "ssmap_server_submit_masked", "ssmap_server_pump", "ssmap_server_poll",
           "ssmap_server_get_job_stats", "ssmap_server_drain",
           "ssmap_server_get_stats", "ssmap_server_last_error", "ssmap_server_destroy"]
SSMAP_AUTOTUNE = 2
MAX_CLASSES = 16
NOALLOC_MAX_BYTES = 64 << 20     # SSMAP_NOALLOC_MAX_BYTES


class Steps(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("xi_p", ctypes.c_double), ("rank", ctypes.c_int),
                ("precision", ctypes.c_int), ("check_every", ctypes.c_int),
                ("flags", ctypes.c_int), ("kernel", ctypes.c_int), ("reserved", ctypes.c_int),
                ("stop_tol", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("rank", ctypes.c_int), ("rank_padded", ctypes.c_int), ("precision", ctypes.c_int),
                ("kernel", ctypes.c_int), ("iters", ctypes.c_int), ("n_hist", ctypes.c_int),
                ("xi_p", ctypes.c_double), ("tau", ctypes.c_double), ("dtd_norm", ctypes.c_double),
                ("sigma_max", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("project_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double),
                ("output_ms", ctypes.c_double), ("device_bytes", ctypes.c_double),
                ("gemm_ms", ctypes.c_double), ("gemm_flops", ctypes.c_double),
                ("hist_iter", ctypes.c_int * MAX_HIST),
                ("hist_objective", ctypes.c_double * MAX_HIST),
                ("hist_dual", ctypes.c_double * MAX_HIST),
                ("hist_znorm", ctypes.c_double * MAX_HIST),
                ("hist_primal", ctypes.c_double * MAX_HIST),
                ("hist_dfcs", ctypes.c_double * MAX_HIST),
                ("hist_dfcs_f", ctypes.c_double * MAX_HIST),
                ("gemm_library", ctypes.c_int)]


class BatchStats(ctypes.Structure):
    _fields_ = [("njobs", ctypes.c_int), ("nclasses", ctypes.c_int), ("solo_jobs", ctypes.c_int),
                ("iters", ctypes.c_int), ("voxels", ctypes.c_double),
                ("project_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double),
                ("output_ms", ctypes.c_double), ("autotune_ms", ctypes.c_double),
                ("class_precision", ctypes.c_int * MAX_CLASSES),
                ("class_rank_padded", ctypes.c_int * MAX_CLASSES),
                ("class_jobs", ctypes.c_int * MAX_CLASSES),
                ("class_bricks", ctypes.c_int * MAX_CLASSES),
                ("class_brick_y", ctypes.c_int * MAX_CLASSES),
                ("class_brick_z", ctypes.c_int * MAX_CLASSES)]


JOB_STATES = {0: "queued", 1: "running", 2: "done"}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_double), ("streams", ctypes.c_int),
                ("reserved", ctypes.c_int * 3)]


class JobInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("status", ctypes.c_int), ("rank", ctypes.c_int),
                ("rank_padded", ctypes.c_int), ("precision", ctypes.c_int), ("iters", ctypes.c_int),
                ("xi_p", ctypes.c_double), ("state_bytes", ctypes.c_double),
                ("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("classes", ctypes.c_int), ("streams", ctypes.c_int),
                ("budget_bytes", ctypes.c_double), ("in_use_bytes", ctypes.c_double),
                ("peak_bytes", ctypes.c_double), ("voxel_iterations", ctypes.c_double)]


class SsmapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str | None = None) -> ctypes.CDLL:
    """Load libssmap.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise OSError(f"libssmap.so not built at {p}; run __graft_entry__.build()")
    lib = ctypes.CDLL(p)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int
    lib.ssmap_create.argtypes = [dp, ip, ip, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(vp)]
    lib.ssmap_create.restype = ip
    lib.ssmap_solve.argtypes = [vp, dp, ctypes.c_double, ctypes.POINTER(Steps), ip, dp]
    lib.ssmap_solve.restype = ip
    lib.ssmap_solve_device.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(Steps), ip, vp, vp]
    lib.ssmap_solve_device.restype = ip
    lib.ssmap_solve_device_noalloc.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(Steps), ip,
                                               vp, vp]
    lib.ssmap_solve_device_noalloc.restype = ip
    lib.ssmap_get_aux.argtypes = [vp, dp, dp]
    lib.ssmap_get_aux.restype = ip
    lib.ssmap_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.ssmap_get_stats.restype = ip
    lib.ssmap_get_singular_values.argtypes = [vp, dp, ip, ctypes.POINTER(ctypes.c_int)]
    lib.ssmap_get_singular_values.restype = ip
    lib.ssmap_last_error.argtypes = [vp]
    lib.ssmap_last_error.restype = ctypes.c_char_p
    lib.ssmap_destroy.argtypes = [vp]
    lib.ssmap_destroy.restype = None
    lib.ssmap_set_mask.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
    lib.ssmap_set_mask.restype = ip
    lib.ssmap_set_reference.argtypes = [vp, dp]
    lib.ssmap_set_reference.restype = ip
    lib.ssmap_set_initial.argtypes = [vp, dp, dp]
    lib.ssmap_set_initial.restype = ip
    lib.ssmap_tune_beta.argtypes = [vp, dp, ctypes.c_double, ctypes.POINTER(Steps), ip, dp, ip,
                                    dp, dp]
    lib.ssmap_tune_beta.restype = ip
    lib.ssmap_version.argtypes = []
    lib.ssmap_version.restype = ctypes.c_char_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.ssmap_batch_create.argtypes = [ip, pp, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(vp)]
    lib.ssmap_batch_create.restype = ip
    lib.ssmap_batch_set_mask.argtypes = [vp, ip, ctypes.POINTER(ctypes.c_uint8)]
    lib.ssmap_batch_set_mask.restype = ip
    lib.ssmap_batch_solve.argtypes = [vp, pp, dp, ctypes.POINTER(Steps), ip, pp]
    lib.ssmap_batch_solve.restype = ip
    lib.ssmap_batch_solve_device.argtypes = [vp, pp, dp, ctypes.POINTER(Steps), ip, pp, vp]
    lib.ssmap_batch_solve_device.restype = ip
    lib.ssmap_batch_get_stats.argtypes = [vp, ctypes.POINTER(BatchStats)]
    lib.ssmap_batch_get_stats.restype = ip
    lib.ssmap_batch_get_job_stats.argtypes = [vp, ip, ctypes.POINTER(Stats)]
    lib.ssmap_batch_get_job_stats.restype = ip
    lib.ssmap_batch_last_error.argtypes = [vp]
    lib.ssmap_batch_last_error.restype = ctypes.c_char_p
    lib.ssmap_batch_destroy.argtypes = [vp]
    lib.ssmap_batch_destroy.restype = None
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.ssmap_server_create.argtypes = [ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.ssmap_server_create.restype = ip
    lib.ssmap_server_add_dictionary.argtypes = [vp, dp, ip, ip, ctypes.POINTER(ctypes.c_int)]
    lib.ssmap_server_add_dictionary.restype = ip
    lib.ssmap_server_submit.argtypes = [vp, ip, i64p, vp, ctypes.c_double, ctypes.POINTER(Steps),
                                        ip, vp, i64p]
    lib.ssmap_server_submit.restype = ip
    lib.ssmap_server_submit_masked.argtypes = [vp, ip, i64p, ctypes.POINTER(ctypes.c_uint8), vp,
                                               ctypes.c_double, ctypes.POINTER(Steps), ip, vp, i64p]
    lib.ssmap_server_submit_masked.restype = ip
    lib.ssmap_server_pump.argtypes = [vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    lib.ssmap_server_pump.restype = ip
    lib.ssmap_server_poll.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(JobInfo)]
    lib.ssmap_server_poll.restype = ip
    lib.ssmap_server_get_job_stats.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(Stats)]
    lib.ssmap_server_get_job_stats.restype = ip
    lib.ssmap_server_drain.argtypes = [vp]
    lib.ssmap_server_drain.restype = ip
    lib.ssmap_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ssmap_server_get_stats.restype = ip
    lib.ssmap_server_last_error.argtypes = [vp]
    lib.ssmap_server_last_error.restype = ctypes.c_char_p
    lib.ssmap_server_destroy.argtypes = [vp]
    lib.ssmap_server_destroy.restype = None
    if path is None:
        _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_steps(beta, xi_p=0.0, rank=0, precision="fp64", check_every=0, keep_aux=False,
               kernel="auto", autotune=False, stop_tol=0.0, primal=False, warm=False) -> Steps:
    flags = (SSMAP_KEEP_AUX if keep_aux else 0) | (SSMAP_AUTOTUNE if autotune else 0) | \
        (SSMAP_MONITOR_PRIMAL if primal else 0) | (SSMAP_WARM_START if warm else 0)
    return Steps(beta=float(beta), xi_p=float(xi_p), rank=int(rank),
                 precision=PRECISIONS[precision] if isinstance(precision, str) else int(precision),
                 check_every=int(check_every), flags=flags,
                 kernel=KERNELS[kernel] if isinstance(kernel, str) else int(kernel), reserved=0,
                 stop_tol=float(stop_tol))


# ------------------------------------------------------------------ C names
def ssmap_create(K: np.ndarray, grid) -> int:
    """Returns the context handle (int); raises SsmapError on failure."""
    lib = load()
    K = np.ascontiguousarray(K, dtype=np.float64)
    P, Q = K.shape
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    out = ctypes.c_void_p()
    st = lib.ssmap_create(_dptr(K), P, Q, g, ctypes.byref(out))
    if st != SSMAP_OK:
        raise SsmapError(st, lib.ssmap_last_error(None).decode())
    return out.value


def _check(ctx, st):
    if st != SSMAP_OK:
        raise SsmapError(st, load().ssmap_last_error(ctx).decode())


def ssmap_solve(ctx: int, M: np.ndarray, lam: float, steps: Steps, iters: int, N: int, Q: int):
    M = np.ascontiguousarray(M, dtype=np.float64)
    F = np.empty((N, Q), dtype=np.float64)
    _check(ctx, load().ssmap_solve(ctx, _dptr(M), float(lam), ctypes.byref(steps), int(iters),
                                   _dptr(F)))
    return F


def ssmap_solve_device(ctx: int, dM: int, lam: float, steps: Steps, iters: int, dF: int,
                       stream: int = 0):
    _check(ctx, load().ssmap_solve_device(ctx, ctypes.c_void_p(dM), float(lam),
                                          ctypes.byref(steps), int(iters), ctypes.c_void_p(dF),
                                          ctypes.c_void_p(stream)))


def ssmap_solve_device_noalloc(ctx: int, dM: int, lam: float, steps: Steps, iters: int, dF: int,
                               stream: int = 0):
    _check(ctx, load().ssmap_solve_device_noalloc(ctx, ctypes.c_void_p(dM), float(lam),
                                                  ctypes.byref(steps), int(iters),
                                                  ctypes.c_void_p(dF), ctypes.c_void_p(stream)))


def ssmap_get_aux(ctx: int, N: int, Q: int):
    f = np.empty((N, Q), dtype=np.float64)
    d = np.empty((N, Q), dtype=np.float64)
    _check(ctx, load().ssmap_get_aux(ctx, _dptr(f), _dptr(d)))
    return f, d


def ssmap_get_stats(ctx: int) -> dict:
    s = Stats()
    _check(ctx, load().ssmap_get_stats(ctx, ctypes.byref(s)))
    return _stats_dict(s)


def _stats_dict(s: "Stats") -> dict:
    n = s.n_hist
    return dict(rank=s.rank, rank_padded=s.rank_padded, precision=s.precision, kernel=s.kernel,
                iters=s.iters, xi_p=s.xi_p, tau=s.tau, dtd_norm=s.dtd_norm,
                sigma_max=s.sigma_max, setup_ms=s.setup_ms, project_ms=s.project_ms,
                iterate_ms=s.iterate_ms, output_ms=s.output_ms, device_bytes=s.device_bytes,
                gemm_ms=s.gemm_ms, gemm_flops=s.gemm_flops, hist_iter=list(s.hist_iter[:n]), hist_objective=list(s.hist_objective[:n]),
                hist_dual=list(s.hist_dual[:n]), hist_znorm=list(s.hist_znorm[:n]),
                hist_primal=list(s.hist_primal[:n]), hist_dfcs=list(s.hist_dfcs[:n]),
                hist_dfcs_f=list(s.hist_dfcs_f[:n]), gemm_library=s.gemm_library)


def ssmap_get_singular_values(ctx: int) -> np.ndarray:
    lib = load()
    n = ctypes.c_int()
    _check(ctx, lib.ssmap_get_singular_values(ctx, None, 0, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.float64)
    _check(ctx, lib.ssmap_get_singular_values(ctx, _dptr(out), n.value, ctypes.byref(n)))
    return out


def ssmap_last_error(ctx: int | None) -> str:
    return load().ssmap_last_error(ctx).decode()


def ssmap_destroy(ctx: int | None) -> None:
    load().ssmap_destroy(ctx)


def ssmap_set_mask(ctx: int, mask) -> None:
    """mask: N booleans (voxel order of M's rows), or None for the whole box."""
    if mask is None:
        _check(ctx, load().ssmap_set_mask(ctx, None))
        return
    mk = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
    _check(ctx, load().ssmap_set_mask(ctx, mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def ssmap_set_reference(ctx: int, f_star) -> None:
    """f_star: (N, Q) float64 reference map for DFCS, or None to remove it."""
    if f_star is None:
        _check(ctx, load().ssmap_set_reference(ctx, None))
        return
    f = np.ascontiguousarray(f_star, dtype=np.float64)
    _check(ctx, load().ssmap_set_reference(ctx, _dptr(f)))


def ssmap_set_initial(ctx: int, z0, d0) -> None:
    """z0, d0: (N, Q) float64 initial iterate for warm starts (None: zeros);
    both None removes it."""
    zs = None if z0 is None else np.ascontiguousarray(z0, dtype=np.float64)
    ds = None if d0 is None else np.ascontiguousarray(d0, dtype=np.float64)
    _check(ctx, load().ssmap_set_initial(ctx, None if zs is None else _dptr(zs),
                                         None if ds is None else _dptr(ds)))


def ssmap_tune_beta(ctx: int, M: np.ndarray, lam: float, steps: Steps, iters: int, betas):
    """Returns (best beta, objectives per candidate)."""
    M = np.ascontiguousarray(M, dtype=np.float64)
    b = np.ascontiguousarray(betas, dtype=np.float64)
    J = np.empty(b.size)
    best = ctypes.c_double()
    _check(ctx, load().ssmap_tune_beta(ctx, _dptr(M), float(lam), ctypes.byref(steps), int(iters),
                                       _dptr(b), int(b.size), _dptr(J), ctypes.byref(best)))
    return best.value, J


def ssmap_version() -> str:
    return load().ssmap_version().decode()


# ------------------------------------------------------------------ convenience
class Mapper:
    """One dictionary on one grid (owns an ssmap context)."""

    def __init__(self, K: np.ndarray, grid):
        self.K = np.ascontiguousarray(K, dtype=np.float64)
        self.P, self.Q = self.K.shape
        self.grid = tuple(int(v) for v in grid)
        self.N = self.grid[0] * self.grid[1] * self.grid[2]
        self.ctx = ssmap_create(self.K, self.grid)

    def solve(self, M, lam, beta, iters, **kw) -> np.ndarray:
        return ssmap_solve(self.ctx, M, lam, make_steps(beta, **kw), iters, self.N, self.Q)

    def solve_torch(self, M, lam, beta, iters, F=None, stream=None, noalloc=False, **kw):
        """Device solve on torch tensors (float64 for fp64, float32 otherwise);
        `noalloc` calls the allocation-free entry point."""
        import torch
        steps = make_steps(beta, **kw)
        dt = torch.float64 if steps.precision == 0 else torch.float32
        if M.dtype != dt or not M.is_cuda or not M.is_contiguous():
            raise ValueError(f"M must be a contiguous device tensor of {dt}")
        if M.shape != (self.N, self.P):
            raise ValueError("M must be (N, P)")
        if F is None:
            F = torch.empty((self.N, self.Q), dtype=dt, device=M.device)
        if F.dtype != dt or not F.is_contiguous() or F.shape != (self.N, self.Q):
            raise ValueError("F must be a contiguous (N, Q) tensor of the I/O type")
        s = stream if stream is not None else torch.cuda.current_stream(M.device)
        fn = ssmap_solve_device_noalloc if noalloc else ssmap_solve_device
        fn(self.ctx, M.data_ptr(), lam, steps, iters, F.data_ptr(), s.cuda_stream)
        return F

    def aux(self):
        return ssmap_get_aux(self.ctx, self.N, self.Q)

    def stats(self) -> dict:
        return ssmap_get_stats(self.ctx)

    def singular_values(self) -> np.ndarray:
        return ssmap_get_singular_values(self.ctx)

    def set_mask(self, mask) -> None:
        ssmap_set_mask(self.ctx, mask)

    def set_reference(self, f_star) -> None:
        if f_star is not None and np.shape(f_star) != (self.N, self.Q):
            raise ValueError("f_star must be (N, Q)")
        ssmap_set_reference(self.ctx, f_star)

    def set_initial(self, z0=None, d0=None) -> None:
        """Initial iterate (z^0, d^0) for solves with warm=True."""
        for x in (z0, d0):
            if x is not None and np.shape(x) != (self.N, self.Q):
                raise ValueError("z0 and d0 must be (N, Q)")
        ssmap_set_initial(self.ctx, z0, d0)

    def tune_beta(self, M, lam, iters, betas, **kw):
        """Patch heuristic for beta; returns (best beta, objectives)."""
        return ssmap_tune_beta(self.ctx, M, lam, make_steps(1.0, **kw), iters, betas)

    def close(self):
        if self.ctx:
            ssmap_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ batches
def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*ptrs)


def ssmap_batch_create(Ks, grids) -> int:
    lib = load()
    Ks = [np.ascontiguousarray(K, dtype=np.float64) for K in Ks]
    n = len(Ks)
    P = (ctypes.c_int * n)(*[K.shape[0] for K in Ks])
    Q = (ctypes.c_int * n)(*[K.shape[1] for K in Ks])
    g = (ctypes.c_int64 * (3 * n))(*[int(v) for gr in grids for v in gr])
    out = ctypes.c_void_p()
    st = lib.ssmap_batch_create(n, _ptr_array([K.ctypes.data for K in Ks]), P, Q, g,
                                ctypes.byref(out))
    if st != SSMAP_OK:
        raise SsmapError(st, lib.ssmap_batch_last_error(None).decode())
    return out.value


def _bcheck(b, st):
    if st != SSMAP_OK:
        raise SsmapError(st, load().ssmap_batch_last_error(b).decode())


def ssmap_batch_get_job_stats(b, job: int) -> dict:
    s = Stats()
    _bcheck(b, load().ssmap_batch_get_job_stats(b, int(job), ctypes.byref(s)))
    return _stats_dict(s)


def ssmap_batch_set_mask(b, job: int, mask) -> None:
    """mask: N_job booleans, or None for the whole box."""
    if mask is None:
        _bcheck(b, load().ssmap_batch_set_mask(b, int(job), None))
        return
    mk = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
    _bcheck(b, load().ssmap_batch_set_mask(b, int(job), mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))


def ssmap_batch_solve(b, Ms, lams, steps_list, iters, shapes):
    """Host solve; shapes[j] = (N_j, Q_j). Returns a list of (N_j, Q_j) maps."""
    Ms = [np.ascontiguousarray(M, dtype=np.float64) for M in Ms]
    Fs = [np.empty(sh, dtype=np.float64) for sh in shapes]
    n = len(Ms)
    steps = (Steps * n)(*steps_list)
    lam = (ctypes.c_double * n)(*[float(x) for x in lams])
    _bcheck(b, load().ssmap_batch_solve(b, _ptr_array([M.ctypes.data for M in Ms]), lam, steps,
                                        int(iters), _ptr_array([F.ctypes.data for F in Fs])))
    return Fs


def ssmap_batch_solve_device(b, dMs, lams, steps_list, iters, dFs, stream=0):
    n = len(dMs)
    steps = (Steps * n)(*steps_list)
    lam = (ctypes.c_double * n)(*[float(x) for x in lams])
    _bcheck(b, load().ssmap_batch_solve_device(b, _ptr_array(dMs), lam, steps, int(iters),
                                               _ptr_array(dFs), ctypes.c_void_p(stream)))


def ssmap_batch_get_stats(b) -> dict:
    s = BatchStats()
    _bcheck(b, load().ssmap_batch_get_stats(b, ctypes.byref(s)))
    c = s.nclasses
    return dict(njobs=s.njobs, nclasses=c, solo_jobs=s.solo_jobs, iters=s.iters, voxels=s.voxels,
                project_ms=s.project_ms, iterate_ms=s.iterate_ms, output_ms=s.output_ms,
                autotune_ms=s.autotune_ms,
                classes=[dict(precision=s.class_precision[i], rank_padded=s.class_rank_padded[i],
                              jobs=s.class_jobs[i], bricks=s.class_bricks[i],
                              brick=(16, s.class_brick_y[i], s.class_brick_z[i]))
                         for i in range(c)])


def ssmap_batch_last_error(b) -> str:
    return load().ssmap_batch_last_error(b).decode()


def ssmap_batch_destroy(b) -> None:
    load().ssmap_batch_destroy(b)


class BatchMapper:
    """Many problems solved together (owns an ssmap batch)."""

    def __init__(self, Ks, grids):
        self.Ks = [np.ascontiguousarray(K, dtype=np.float64) for K in Ks]
        self.grids = [tuple(int(v) for v in g) for g in grids]
        self.N = [g[0] * g[1] * g[2] for g in self.grids]
        self.b = ssmap_batch_create(self.Ks, self.grids)

    def job_stats(self, job) -> dict:
        return ssmap_batch_get_job_stats(self.b, job)

    def set_mask(self, job, mask) -> None:
        if mask is not None and np.size(mask) != self.N[job]:
            raise ValueError("mask must have N_job entries")
        ssmap_batch_set_mask(self.b, job, mask)

    def solve(self, Ms, lams, betas, iters, **kw):
        steps = [make_steps(bt, **kw) for bt in betas]
        return ssmap_batch_solve(self.b, Ms, lams, steps, iters,
                                 [(n, K.shape[1]) for n, K in zip(self.N, self.Ks)])

    def solve_torch(self, Ms, lams, betas, iters, Fs=None, stream=None, **kw):
        import torch
        steps = [make_steps(bt, **kw) for bt in betas]
        if Fs is None:
            Fs = [torch.empty((n, K.shape[1]), dtype=M.dtype, device=M.device)
                  for n, K, M in zip(self.N, self.Ks, Ms)]
        for M, F, n, K in zip(Ms, Fs, self.N, self.Ks):
            if not (M.is_cuda and M.is_contiguous() and M.shape == (n, K.shape[0])):
                raise ValueError("each M must be a contiguous (N, P) device tensor")
            if not (F.is_contiguous() and F.shape == (n, K.shape[1]) and F.dtype == M.dtype):
                raise ValueError("each F must be a contiguous (N, Q) tensor of M's type")
        s = stream if stream is not None else torch.cuda.current_stream(Ms[0].device)
        ssmap_batch_solve_device(self.b, [M.data_ptr() for M in Ms], lams, steps, iters,
                                 [F.data_ptr() for F in Fs], s.cuda_stream)
        return Fs

    def stats(self) -> dict:
        return ssmap_batch_get_stats(self.b)

    def close(self):
        if self.b:
            ssmap_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def _scheck(sv, st):
    if st != SSMAP_OK:
        raise SsmapError(st, load().ssmap_server_last_error(sv).decode())


def ssmap_server_create(hbm_budget: float, streams: int = 0) -> int:
    lib = load()
    opts = ServerOpts(float(hbm_budget), int(streams))
    out = ctypes.c_void_p()
    st = lib.ssmap_server_create(ctypes.byref(opts), ctypes.byref(out))
    if st != SSMAP_OK:
        raise SsmapError(st, lib.ssmap_server_last_error(None).decode())
    return out.value


def ssmap_server_add_dictionary(sv, K: np.ndarray) -> int:
    K = np.ascontiguousarray(K, dtype=np.float64)
    d = ctypes.c_int()
    _scheck(sv, load().ssmap_server_add_dictionary(sv, _dptr(K), K.shape[0], K.shape[1],
                                                    ctypes.byref(d)))
    return d.value


def ssmap_server_submit(sv, dict_id, grid, dM, lam, steps, iters, dF, mask=None) -> int:
    """Queue a job; `mask` (N values, nonzero = inside, copied) makes it a masked job."""
    g = (ctypes.c_int64 * 3)(*[int(v) for v in grid])
    jid = ctypes.c_int64()
    if mask is None:
        st = load().ssmap_server_submit(sv, int(dict_id), g, ctypes.c_void_p(dM), float(lam),
                                        ctypes.byref(steps), int(iters), ctypes.c_void_p(dF),
                                        ctypes.byref(jid))
    else:
        mk = np.ascontiguousarray(np.asarray(mask).reshape(-1) != 0, dtype=np.uint8)
        if mk.size != int(grid[0]) * int(grid[1]) * int(grid[2]):
            raise ValueError("mask must hold one value per voxel")
        st = load().ssmap_server_submit_masked(sv, int(dict_id), g,
                                               mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                               ctypes.c_void_p(dM), float(lam), ctypes.byref(steps),
                                               int(iters), ctypes.c_void_p(dF), ctypes.byref(jid))
    _scheck(sv, st)
    return jid.value


def ssmap_server_pump(sv, horizon_ms: float) -> int:
    n = ctypes.c_int()
    _scheck(sv, load().ssmap_server_pump(sv, float(horizon_ms), ctypes.byref(n)))
    return n.value


def ssmap_server_poll(sv, job_id) -> dict:
    i = JobInfo()
    _scheck(sv, load().ssmap_server_poll(sv, int(job_id), ctypes.byref(i)))
    return dict(state=JOB_STATES[i.state], status=i.status, rank=i.rank,
                rank_padded=i.rank_padded, precision=i.precision, iters=i.iters, xi_p=i.xi_p,
                state_bytes=i.state_bytes, submit_ms=i.submit_ms, admit_ms=i.admit_ms,
                done_ms=i.done_ms)


def ssmap_server_get_job_stats(sv, job_id) -> dict:
    """Monitoring record of a finished served job (history empty when unmonitored)."""
    s = Stats()
    _scheck(sv, load().ssmap_server_get_job_stats(sv, int(job_id), ctypes.byref(s)))
    return _stats_dict(s)


def ssmap_server_drain(sv) -> None:
    _scheck(sv, load().ssmap_server_drain(sv))


def ssmap_server_get_stats(sv) -> dict:
    s = ServerStats()
    _scheck(sv, load().ssmap_server_get_stats(sv, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def ssmap_server_last_error(sv) -> str:
    return load().ssmap_server_last_error(sv).decode()


def ssmap_server_destroy(sv) -> None:
    load().ssmap_server_destroy(sv)


class Server:
    """Served jobs on device tensors (owns an ssmap server). Keeps each job's
    M and F tensors alive until the job is done."""

    def __init__(self, hbm_budget: float, streams: int = 0):
        self.sv = ssmap_server_create(hbm_budget, streams)
        self.dicts = {}
        self.live = {}

    def add_dictionary(self, K: np.ndarray) -> int:
        d = ssmap_server_add_dictionary(self.sv, K)
        self.dicts[d] = np.asarray(K).shape
        return d

    def submit(self, dict_id, grid, M, lam, beta, iters, F=None, ready=False, mask=None, **kw) -> int:
        """Queue a job on device tensor M (N, P), float64 for fp64 and float32
        otherwise; returns its id. Unless `ready`, the current torch stream is
        synchronized first so that M is complete when the server reads it.
        `mask` (N values, nonzero = inside) makes it a masked job."""
        import torch
        P, Q = self.dicts[dict_id]
        N = int(grid[0]) * int(grid[1]) * int(grid[2])
        steps = make_steps(beta, **kw)
        dt = torch.float64 if steps.precision == 0 else torch.float32
        if not (M.is_cuda and M.is_contiguous() and M.dtype == dt and tuple(M.shape) == (N, P)):
            raise ValueError(f"M must be a contiguous (N, P) device tensor of {dt}")
        if F is None:
            F = torch.empty((N, Q), dtype=dt, device=M.device)
        if not (F.is_cuda and F.is_contiguous() and F.dtype == dt and tuple(F.shape) == (N, Q)):
            raise ValueError(f"F must be a contiguous (N, Q) device tensor of {dt}")
        if not ready:
            torch.cuda.current_stream(M.device).synchronize()
        jid = ssmap_server_submit(self.sv, dict_id, grid, M.data_ptr(), lam, steps, iters,
                                  F.data_ptr(), mask=mask)
        self.live[jid] = (M, F)
        return jid

    def pump(self, horizon_ms: float = 5.0) -> int:
        return ssmap_server_pump(self.sv, horizon_ms)

    def poll(self, job_id) -> dict:
        info = ssmap_server_poll(self.sv, job_id)
        return info

    def job_stats(self, job_id) -> dict:
        return ssmap_server_get_job_stats(self.sv, job_id)

    def result(self, job_id):
        """F of a finished job (None while it runs); releases the job's tensors."""
        info = ssmap_server_poll(self.sv, job_id)
        if info["state"] != "done":
            return None
        M, F = self.live.pop(job_id, (None, None))
        if info["status"] != SSMAP_OK:
            raise SsmapError(info["status"], f"job {job_id} failed")
        return F

    def drain(self) -> None:
        ssmap_server_drain(self.sv)

    def stats(self) -> dict:
        return ssmap_server_get_stats(self.sv)

    def close(self):
        if self.sv:
            ssmap_server_destroy(self.sv)
            self.sv = None
            self.live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
