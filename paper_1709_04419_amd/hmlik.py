"""Thin Python binding of libhmlik (include/hmlik.h) with the same names.

Argument marshalling only: every step of the likelihood evaluation runs in
the library's HIP kernels.  There is no CPU fallback: if the shared library
is missing or cannot be loaded, importing this module raises.

Arrays: coordinates are (n, 2) float64; Z is (n,) or (n, r) float64, either
a numpy array (host) or a torch CUDA tensor (device pointer, read on the
context's stream).
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmlik.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1709_04419_amd.build`")
# One HIP runtime per process: torch ships its own libamdhip64 (soname
# libamdhip64.so.7, loaded under the unversioned name).  Loading torch first
# makes the library bind to that same runtime, so that torch tensors and
# streams can be handed to it; loading the library first would give the
# process two runtimes, and torch would then find no GPU.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

(HM_OK, HM_ERR_ARG, HM_ERR_NOT_SPD, HM_ERR_OOM, HM_ERR_DEVICE, HM_ERR_INTERNAL, HM_ERR_CANCELLED,
 HM_ERR_BUSY) = range(8)
HM_FP64, HM_MIXED = 0, 1
HM_OP_L, HM_OP_LT, HM_OP_C, HM_OP_SOLVE, HM_OP_C_EXACT = range(5)


class hm_theta(C.Structure):
    _fields_ = [("sigma2", C.c_double), ("ell", C.c_double), ("nu", C.c_double),
                ("nugget", C.c_double)]


class hm_tree_opts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("eta", C.c_double)]


class hm_approx(C.Structure):
    _fields_ = [("fixed_rank", C.c_int32), ("eps", C.c_double), ("prec", C.c_int32),
                ("refine_max_iter", C.c_int32), ("refine_tol", C.c_double)]


class hm_result(C.Structure):
    _fields_ = [("loglik", C.c_double), ("logdet", C.c_double), ("quadform", C.c_double),
                ("n", C.c_int64), ("max_rank", C.c_int32), ("rank_capped", C.c_int32),
                ("bytes_C", C.c_int64), ("bytes_L", C.c_int64), ("status", C.c_int32),
                ("fail_pivot", C.c_int32), ("fail_block", C.c_int64), ("refine_quad", C.c_double),
                ("refine_resid", C.c_double), ("refine_iters", C.c_int32), ("reserved", C.c_int32),
                ("t_assemble", C.c_double), ("t_factor", C.c_double), ("t_solve", C.c_double)]


class hm_server_opts(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("hbm_budget", C.c_int64)]


class hm_request_stats(C.Structure):
    _fields_ = [("t_queue", C.c_double), ("t_latency", C.c_double), ("steps", C.c_int32),
                ("peak_batch", C.c_int32)]


_P = C.c_void_p
_sig = {
    "hm_ctx_create": (C.c_int, [C.c_int, _P, C.POINTER(_P)]),
    "hm_ctx_destroy": (None, [_P]),
    "hm_dataset_create": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.POINTER(hm_tree_opts), C.c_int32,
                                    C.POINTER(_P)]),
    "hm_dataset_destroy": (None, [_P]),
    "hm_dataset_set_z": (C.c_int, [_P, _P, C.c_int32, C.c_int32]),
    "hm_assemble": (C.c_int, [_P, C.POINTER(hm_theta), C.POINTER(hm_approx)]),
    "hm_factor": (C.c_int, [_P]),
    "hm_solve": (C.c_int, [_P, C.POINTER(hm_result)]),
    "hm_loglik": (C.c_int, [_P, C.POINTER(hm_theta), C.POINTER(hm_approx), C.POINTER(hm_result)]),
    "hm_tune_schedule": (C.c_int, [_P, C.POINTER(hm_theta), C.POINTER(hm_approx)]),
    "hm_loglik_batch": (C.c_int, [_P, C.c_int32, C.POINTER(_P), C.POINTER(hm_theta), C.POINTER(hm_approx),
                                  C.POINTER(hm_result)]),
    "hm_dataset_info": (C.c_int, [_P, _P, _P, _P, _P, _P]),
    "hm_dataset_export_tree": (C.c_int, [_P, _P, _P, _P]),
    "hm_dataset_export_blocks": (C.c_int, [_P, _P, _P]),
    "hm_get_block": (C.c_int, [_P, C.c_int64, _P, C.POINTER(C.c_int32)]),
    "hm_factor_flops": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "hm_get_term": (C.c_int, [_P, C.c_int64, _P, C.POINTER(C.c_int32), C.POINTER(C.c_int64),
                              C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "hm_test_truncate": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                                   _P, _P, C.POINTER(C.c_int32), _P]),
    "hm_truncate_noalloc": (C.c_int, [_P, _P, C.c_int64, _P, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                                      _P, _P, _P]),
    "hm_dataset_keep_matrix": (C.c_int, [_P, C.c_int32]),
    "hm_apply": (C.c_int, [_P, C.c_int32, _P, _P, C.c_int32, C.c_int32]),
    "hm_simulate": (C.c_int, [_P, C.POINTER(hm_theta), C.POINTER(hm_approx), _P, _P, C.c_int32, C.c_int32]),
    "hm_inverse_accuracy": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_double)]),
    "hm_exact_block": (C.c_int, [_P, C.c_int64, C.c_int64, C.c_int64, C.c_int64, _P, C.c_int64, C.c_int32]),
    "hm_dataset_footprint": (C.c_int, [_P, _P, _P, _P]),
    "hm_dataset_release": (C.c_int, [_P]),
    "hm_server_create": (C.c_int, [_P, C.POINTER(hm_server_opts), C.POINTER(_P)]),
    "hm_server_submit": (C.c_int, [_P, _P, C.POINTER(hm_theta), C.POINTER(hm_approx), C.POINTER(C.c_uint64)]),
    "hm_server_poll": (C.c_int, [_P, C.c_uint64, C.c_int32, C.POINTER(hm_result), C.POINTER(hm_request_stats),
                                 C.POINTER(C.c_int32)]),
    "hm_server_cancel": (C.c_int, [_P, C.c_uint64]),
    "hm_server_destroy": (None, [_P]),
    "hm_status_string": (C.c_char_p, [C.c_int]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class HMError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {hm_status_string(status)} (status {status})")
        self.status = status


def hm_status_string(s: int) -> str:
    return _lib.hm_status_string(int(s)).decode()


def _check(s, where):
    if s != HM_OK:
        raise HMError(s, where)


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if isinstance(a, np.ndarray) else C.c_void_p(int(a.data_ptr()))


def _device_f64(t, ctx, what):
    """A torch tensor handed to the library as a device pointer must be float64
    and live on the context's GPU (the library reads 8 bytes per entry there)."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a numpy array or a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{what}: torch tensor must be float64, got {t.dtype}")
    if not t.is_cuda or t.device.index != ctx.device:
        raise ValueError(f"{what}: torch tensor must be on cuda:{ctx.device}, got {t.device}")
    return t


class Context:
    """hm_ctx_create / hm_ctx_destroy.  stream: a torch.cuda.Stream, a raw
    hipStream_t as int, or None for the default stream."""

    def __init__(self, device: int = 0, stream=None):
        h = _P()
        raw = None
        if stream is not None:
            raw = getattr(stream, "cuda_stream", stream)
        _check(_lib.hm_ctx_create(int(device), C.c_void_p(raw) if raw else None, C.byref(h)),
               "hm_ctx_create")
        self._h = h
        self.device = int(device)
        self._datasets = weakref.WeakSet()
        self._servers = weakref.WeakSet()

    def close(self):
        """Destroys the context, closing its servers and then its datasets first
        (neither may outlive the context it was created in)."""
        if self._h:
            for sv in list(self._servers):
                sv.close()
            for ds in list(self._datasets):
                ds.close()
            _lib.hm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Dataset:
    """hm_dataset_*: trees, schedule and device storage for one set of locations."""

    def __init__(self, ctx: Context, coords, leaf_size: int = 64, eta: float = 2.0):
        """coords: (n, 2) float64, a numpy array or a torch CUDA tensor on the
        context's device."""
        if isinstance(coords, np.ndarray) or not hasattr(coords, "data_ptr"):
            P = np.ascontiguousarray(coords, dtype=np.float64)
            on_dev = 0
        else:
            P = _device_f64(coords, ctx, "coords").contiguous()
            on_dev = 1
        if P.ndim != 2 or P.shape[1] != 2:
            raise ValueError("coords must be (n, 2)")
        self.ctx = ctx
        self.n = int(P.shape[0])
        opts = hm_tree_opts(int(leaf_size), float(eta))
        h = _P()
        _check(_lib.hm_dataset_create(ctx._h, _ptr(P), C.c_int64(self.n), 2, C.byref(opts), on_dev, C.byref(h)),
               "hm_dataset_create")
        self._h = h
        self.r = 0
        ctx._datasets.add(self)

    def close(self):
        if getattr(self, "_h", None):
            _lib.hm_dataset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_z(self, Z):
        on_dev = not isinstance(Z, np.ndarray)
        if on_dev:
            Z = _device_f64(Z, self.ctx, "Z")
            if Z.dim() == 1:
                Z = Z[:, None]
            Zc = Z.t().contiguous()     # column-major (n, r) == row-major (r, n)
            r = Zc.shape[0]
            if Zc.shape[1] != self.n:
                raise ValueError("Z has the wrong length")
            _check(_lib.hm_dataset_set_z(self._h, C.c_void_p(int(Zc.data_ptr())), r, 1),
                   "hm_dataset_set_z")
        else:
            Z = np.asarray(Z, dtype=np.float64)
            if Z.ndim == 1:
                Z = Z[:, None]
            if Z.shape[0] != self.n:
                raise ValueError("Z has the wrong length")
            r = Z.shape[1]
            Zc = np.asfortranarray(Z)
            _check(_lib.hm_dataset_set_z(self._h, C.c_void_p(Zc.ctypes.data), r, 0), "hm_dataset_set_z")
        self.r = r

    @staticmethod
    def _args(theta, nugget, eps, rank, prec=HM_FP64, refine_max_iter=0, refine_tol=0.0):
        sigma2, ell, nu = theta
        return (hm_theta(sigma2, ell, nu, nugget),
                hm_approx(int(rank), float(eps), int(prec), int(refine_max_iter), float(refine_tol)))

    def assemble(self, theta, nugget, eps=0.0, rank=0, prec=HM_FP64, refine_max_iter=0, refine_tol=0.0):
        th, ap = self._args(theta, nugget, eps, rank, prec, refine_max_iter, refine_tol)
        _check(_lib.hm_assemble(self._h, C.byref(th), C.byref(ap)), "hm_assemble")

    def factor(self) -> int:
        s = _lib.hm_factor(self._h)
        if s not in (HM_OK, HM_ERR_NOT_SPD):
            raise HMError(s, "hm_factor")
        return s

    def solve(self):
        out = (hm_result * self.r)()
        s = _lib.hm_solve(self._h, out)
        if s not in (HM_OK, HM_ERR_NOT_SPD):
            raise HMError(s, "hm_solve")
        return _results(out)

    def loglik(self, theta, nugget, eps=0.0, rank=0, prec=HM_FP64, refine_max_iter=0, refine_tol=0.0):
        """Eq. (4) for every column of Z; returns a dict of arrays.  prec=HM_MIXED
        selects the mixed-precision form with iterative refinement of C~^{-1} Z
        (at most refine_max_iter corrections, stopping at relative residual
        refine_tol)."""
        th, ap = self._args(theta, nugget, eps, rank, prec, refine_max_iter, refine_tol)
        out = (hm_result * self.r)()
        s = _lib.hm_loglik(self._h, C.byref(th), C.byref(ap), out)
        if s not in (HM_OK, HM_ERR_NOT_SPD):
            raise HMError(s, "hm_loglik")
        return _results(out)

    def tune_schedule(self, theta, nugget, eps=0.0, rank=0, prec=HM_FP64) -> int:
        """hm_tune_schedule: one timed evaluation, then the level assignment of
        the factorisation's tasks is re-balanced (results unchanged)."""
        th, ap = self._args(theta, nugget, eps, rank, prec)
        s = _lib.hm_tune_schedule(self._h, C.byref(th), C.byref(ap))
        if s not in (HM_OK, HM_ERR_NOT_SPD):
            raise HMError(s, "hm_tune_schedule")
        return s

    def info(self):
        vals = [C.c_int64() for _ in range(5)]
        _check(_lib.hm_dataset_info(self._h, *[C.byref(v) for v in vals]), "hm_dataset_info")
        return dict(zip(("n", "nclusters", "nblocks", "ntasks", "nlevels"), (v.value for v in vals)))

    def footprint(self):
        """hm_dataset_footprint: dict(resident_bytes, factor_bytes, attached)."""
        res, fac, att = C.c_int64(), C.c_int64(), C.c_int32()
        _check(_lib.hm_dataset_footprint(self._h, C.byref(res), C.byref(fac), C.byref(att)),
               "hm_dataset_footprint")
        return dict(resident_bytes=res.value, factor_bytes=fac.value, attached=bool(att.value))

    def release(self):
        """hm_dataset_release: frees the factor storage until the next evaluation."""
        _check(_lib.hm_dataset_release(self._h), "hm_dataset_release")

    def keep_matrix(self, keep: bool = True):
        """hm_dataset_keep_matrix: later assemblies keep a copy of C~ (for HM_OP_C)."""
        _check(_lib.hm_dataset_keep_matrix(self._h, 1 if keep else 0), "hm_dataset_keep_matrix")

    def apply(self, op: int, W):
        """hm_apply: Y = op W (HM_OP_*) for W of shape (n,) or (n, r), numpy
        (host) or a float64 torch tensor on the context's GPU (device)."""
        on_dev = not isinstance(W, np.ndarray)
        if on_dev:
            W = _device_f64(W, self.ctx, "W")
            vec = W.dim() == 1
            Wc = (W[:, None] if vec else W).t().contiguous()
            r = Wc.shape[0]
            Yc = Wc.new_empty(Wc.shape)
            _check(_lib.hm_apply(self._h, int(op), _ptr(Wc), _ptr(Yc), r, 1), "hm_apply")
            Y = Yc.t()
            return Y[:, 0] if vec else Y
        W = np.asarray(W, dtype=np.float64)
        vec = W.ndim == 1
        Wf = np.asfortranarray(W[:, None] if vec else W)
        if Wf.shape[0] != self.n:
            raise ValueError("W has the wrong length")
        Y = np.empty_like(Wf, order="F")
        _check(_lib.hm_apply(self._h, int(op), _ptr(Wf), _ptr(Y), Wf.shape[1], 0), "hm_apply")
        return Y[:, 0] if vec else Y

    def simulate(self, theta, nugget, W, eps=0.0, rank=0):
        """hm_simulate: Z = L~(theta) W (host arrays, (n,) or (n, r))."""
        th, ap = self._args(theta, nugget, eps, rank)
        W = np.asarray(W, dtype=np.float64)
        vec = W.ndim == 1
        Wf = np.asfortranarray(W[:, None] if vec else W)
        Z = np.empty_like(Wf, order="F")
        _check(_lib.hm_simulate(self._h, C.byref(th), C.byref(ap), _ptr(Wf), _ptr(Z), Wf.shape[1], 0),
               "hm_simulate")
        return Z[:, 0] if vec else Z

    def inverse_accuracy(self, x0, iters: int = 10) -> float:
        """hm_inverse_accuracy: ||I - (L~ L~^T)^{-1} C||_2 by `iters` power steps from x0."""
        x = np.ascontiguousarray(x0, dtype=np.float64)
        out = C.c_double()
        _check(_lib.hm_inverse_accuracy(self._h, _ptr(x), int(iters), C.byref(out)), "hm_inverse_accuracy")
        return out.value

    def exact_block(self, i0: int, ni: int, j0: int, nj: int, device: bool = False):
        """hm_exact_block: C(i0:i0+ni, j0:j0+nj) of the exact covariance at the
        last assembled theta, input order; a numpy array, or with device=True a
        float64 torch tensor on the context's GPU (column-major storage)."""
        if device:
            import torch
            buf = torch.empty((nj, ni), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
            _check(_lib.hm_exact_block(self._h, i0, ni, j0, nj, _ptr(buf), max(ni, 1), 1), "hm_exact_block")
            return buf.t()
        out = np.empty((ni, nj), dtype=np.float64, order="F")
        _check(_lib.hm_exact_block(self._h, i0, ni, j0, nj, _ptr(out), max(ni, 1), 0), "hm_exact_block")
        return out

    def export_tree(self):
        inf = self.info()
        perm = np.empty(self.n, dtype=np.int64)
        ranges = np.empty((inf["nclusters"], 2), dtype=np.int64)
        boxes = np.empty((inf["nclusters"], 4), dtype=np.float64)
        _check(_lib.hm_dataset_export_tree(self._h, _ptr(perm), _ptr(ranges), _ptr(boxes)),
               "hm_dataset_export_tree")
        return perm, ranges, boxes

    def export_blocks(self):
        inf = self.info()
        rc = np.empty((inf["nblocks"], 4), dtype=np.int64)
        kind = np.empty(inf["nblocks"], dtype=np.int8)
        _check(_lib.hm_dataset_export_blocks(self._h, _ptr(rc), _ptr(kind)), "hm_dataset_export_blocks")
        return rc, kind

    def factor_flops(self) -> float:
        """hm_factor_flops: algorithmic flops of the last factorization."""
        f = C.c_double()
        _check(_lib.hm_factor_flops(self._h, C.byref(f)), "hm_factor_flops")
        return f.value

    def get_term(self, term: int):
        """Update term `term`: dict(kind, A, B, factor) (factor None for kind 2)."""
        kind, k = C.c_int32(), C.c_int32()
        A, B, rows = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.hm_get_term(self._h, C.c_int64(term), None, C.byref(kind), C.byref(A), C.byref(B),
                                C.byref(rows), C.byref(k)), "hm_get_term")
        fac = None
        if kind.value != 2:
            buf = np.empty(max(1, rows.value * 64), dtype=np.float64)
            _check(_lib.hm_get_term(self._h, C.c_int64(term), _ptr(buf), C.byref(kind), C.byref(A), C.byref(B),
                                    C.byref(rows), C.byref(k)), "hm_get_term")
            fac = buf[:rows.value * k.value].reshape(k.value, rows.value).T.copy()
        return dict(kind=kind.value, A=A.value, B=B.value, factor=fac)

    def get_block(self, block: int, rows: int, cols: int):
        """Dense leaf -> (rows, cols) array; low-rank leaf -> (U, V)."""
        buf = np.empty((rows + cols) * 64 if rows * cols < (rows + cols) * 64 else rows * cols,
                       dtype=np.float64)
        k = C.c_int32()
        _check(_lib.hm_get_block(self._h, C.c_int64(block), _ptr(buf), C.byref(k)), "hm_get_block")
        if k.value < 0:
            return buf[:rows * cols].reshape(cols, rows).T.copy()
        kk = k.value
        U = buf[:rows * kk].reshape(kk, rows).T.copy()
        V = buf[rows * kk:rows * kk + cols * kk].reshape(kk, cols).T.copy()
        return U, V


def test_truncate(ds: "Dataset", X, Y=None, eps=0.0, rank=0):
    """hm_test_truncate: device truncation of X Y^T, or of the explicit matrix X
    when Y is None; returns (U, V, [total, phase1, phase2, phase3] seconds)."""
    X = np.asfortranarray(X, dtype=np.float64)
    if Y is None:
        m, n = X.shape
        r = 0
        yp = None
    else:
        Y = np.asfortranarray(Y, dtype=np.float64)
        m, r = X.shape
        n = Y.shape[0]
        yp = _ptr(Y)
    U = np.zeros((m, 64), order="F")
    V = np.zeros((n, 64), order="F")
    k = C.c_int32()
    sec = (C.c_double * 4)()
    _check(_lib.hm_test_truncate(ds._h, _ptr(X), m, yp, n, r, float(eps), int(rank), _ptr(U), _ptr(V),
                                 C.byref(k), sec), "hm_test_truncate")
    kk = k.value
    Uo = np.asarray(U.reshape(-1, order="F")[:m * kk].reshape(kk, m).T)
    Vo = np.asarray(V.reshape(-1, order="F")[:n * kk].reshape(kk, n).T)
    return Uo, Vo, list(sec)


def loglik_batch(ctx: "Context", datasets, thetas, nuggets, eps=0.0, rank=0):
    """hm_loglik_batch: eq. (4) for several datasets in one call; dataset i at
    thetas[i] with nuggets[i] and accuracy eps[i] / rank[i] (eps and rank may
    also be single values).  Returns one result dict per dataset."""
    m = len(datasets)
    eps = list(eps) if np.ndim(eps) else [eps] * m
    rank = list(rank) if np.ndim(rank) else [rank] * m
    th = (hm_theta * m)()
    ap = (hm_approx * m)()
    hs = (_P * m)()
    for i, ds in enumerate(datasets):
        t, a = ds._args(thetas[i], nuggets[i], eps[i], rank[i])
        th[i] = t
        ap[i] = a
        hs[i] = ds._h.value
    total = sum(ds.r for ds in datasets)
    out = (hm_result * total)()
    s = _lib.hm_loglik_batch(ctx._h, m, hs, th, ap, out)
    if s not in (HM_OK, HM_ERR_NOT_SPD):
        raise HMError(s, "hm_loglik_batch")
    res, off = [], 0
    for ds in datasets:
        res.append(_results(out[off:off + ds.r]))
        off += ds.r
    return res


class Server:
    """hm_server_*: continuous-batching request server on a context's resident
    datasets.  While it is open, the context's direct evaluation calls raise
    HMError with status HM_ERR_BUSY."""

    def __init__(self, ctx: Context, max_active: int = 8, hbm_budget: int = 0):
        opts = hm_server_opts(int(max_active), int(hbm_budget))
        h = _P()
        _check(_lib.hm_server_create(ctx._h, C.byref(opts), C.byref(h)), "hm_server_create")
        self._h = h
        self.ctx = ctx
        self._r = {}
        ctx._servers.add(self)

    def submit(self, ds: Dataset, theta, nugget, eps=0.0, rank=0) -> int:
        th, ap = ds._args(theta, nugget, eps, rank)
        t = C.c_uint64()
        _check(_lib.hm_server_submit(self._h, ds._h, C.byref(th), C.byref(ap), C.byref(t)), "hm_server_submit")
        self._r[t.value] = ds.r
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """None while the request runs (wait=False); else the result dict of
        Dataset.loglik plus 'request_status', 't_queue', 't_latency', 'steps'
        and 'peak_batch'.  The ticket is retired once its result is returned."""
        r = self._r.get(ticket, 1)
        out = (hm_result * max(1, r))()
        st = hm_request_stats()
        done = C.c_int32()
        s = _lib.hm_server_poll(self._h, C.c_uint64(ticket), 1 if wait else 0, out, C.byref(st), C.byref(done))
        if s == HM_ERR_ARG and not done.value:
            raise HMError(s, "hm_server_poll")
        if not done.value:
            return None
        self._r.pop(ticket, None)
        res = _results(out[:r])
        res.update(request_status=s, t_queue=st.t_queue, t_latency=st.t_latency, steps=st.steps,
                   peak_batch=st.peak_batch)
        return res

    def cancel(self, ticket: int):
        _check(_lib.hm_server_cancel(self._h, C.c_uint64(ticket)), "hm_server_cancel")

    def close(self):
        if getattr(self, "_h", None):
            _lib.hm_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _results(out):
    keys = ("loglik", "logdet", "quadform", "n", "max_rank", "rank_capped", "bytes_C", "bytes_L", "status",
            "fail_pivot", "fail_block", "refine_quad", "refine_resid", "refine_iters", "t_assemble", "t_factor",
            "t_solve")
    return {k: np.array([getattr(o, k) for o in out]) for k in keys}
