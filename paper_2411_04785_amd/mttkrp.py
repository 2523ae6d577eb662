"""ctypes binding of libmttkrp (C ABI in include/mttkrp.h).

Argument marshalling only: every computation runs in the HIP library.  Torch
is used for device memory (``tensor.data_ptr()``) and streams
(``torch.cuda.current_stream().cuda_stream``).  The library is loaded on
first use; if ``libmttkrp.so`` has not been built the call raises -- there is
no fallback path.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MTK_LIBRARY") or os.path.join(_HERE, "libmttkrp.so")

MTK_OK, MTK_EINVAL, MTK_ENOMEM, MTK_EHIP, MTK_ENOTSPD, MTK_EUNSUPPORTED, MTK_EBUDGET, MTK_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7
FP32, BF16X3, FP8_E4M3, BF16X6 = 0, 1, 2, 3
PREC_NAMES = {"fp32": FP32, "bf16x3": BF16X3, "bf16x6": BF16X6, "fp8": FP8_E4M3, "fp8_e4m3": FP8_E4M3}
STATUS_NAMES = {0: "MTK_OK", -1: "MTK_EINVAL", -2: "MTK_ENOMEM", -3: "MTK_EHIP", -4: "MTK_ENOTSPD",
                -5: "MTK_EUNSUPPORTED", -6: "MTK_EBUDGET", -7: "MTK_EAGAIN"}

EXPORTED = ["mtk_create", "mtk_destroy", "mtk_last_error", "mtk_check", "mtk_reserve",
            "mtk_quantize_fp8", "mttkrp", "mttkrp_noalloc", "mttkrp_nway", "als_sweep_nway", "mtk_coo_create", "mtk_coo_destroy", "mtk_coo_nnz", "mttkrp_coo", "als_sweep_coo",
            "mttkrp_dimtree", "mtk_sweep_uses_dimtree", "gram_solve", "mtk_fit",
            "als_sweep", "als_run", "als_run_extrapolated", "mtk_graph_reset",
            "mtk_server_create", "mtk_server_submit", "mtk_server_poll", "mtk_server_stats",
            "mtk_server_request_bytes", "mtk_server_destroy"]


class MtkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NotSPDError(MtkError):
    pass


class Tensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("data_t", ctypes.c_void_p), ("dims", ctypes.c_int64 * 3),
                ("fmt", ctypes.c_int32), ("slice_exp", ctypes.c_void_p)]


class ServerStat(ctypes.Structure):
    _fields_ = [("resident", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("bytes_in_use", ctypes.c_uint64),
                ("peak_bytes_in_use", ctypes.c_uint64), ("device_bytes", ctypes.c_uint64),
                ("steps", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("R", ctypes.c_int32),
                ("dims", ctypes.c_int64 * 3), ("fit", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmttkrp.so (raises FileNotFoundError if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(f"{LIB_PATH} not built: run `python -m paper_2411_04785_amd.build`")
    # torch carries its own HIP runtime under the same soname as the system
    # one the library links against; whichever is loaded first serves the
    # process, and torch finds no device on the other.  Load torch's first.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, d = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    P3 = ctypes.c_void_p * 3
    sig = {
        "mtk_create": (i32, [ctypes.POINTER(vp), i32]),
        "mtk_destroy": (i32, [vp]),
        "mtk_last_error": (ctypes.c_char_p, [vp]),
        "mtk_check": (i32, [vp, vp]),
        "mtk_reserve": (i32, [vp, ctypes.POINTER(i64), i64, i32]),
        "mtk_quantize_fp8": (i32, [vp, vp, ctypes.POINTER(i64), vp, vp, vp, vp]),
        "mttkrp": (i32, [vp, ctypes.POINTER(Tensor), P3, i64, i32, i32, vp, vp]),
        "mttkrp_noalloc": (i32, [vp, ctypes.POINTER(Tensor), P3, i64, i32, i32, vp, vp]),
        "mttkrp_nway": (i32, [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(vp), i64, i32, i32, vp, vp]),
        "als_sweep_nway": (i32, [vp, vp, i32, ctypes.POINTER(i64), ctypes.POINTER(vp), vp, i64, i32, i32, vp]),
        "mtk_coo_create": (i32, [vp, ctypes.POINTER(i64), i64, P3, vp, vp, ctypes.POINTER(vp)]),
        "mtk_coo_destroy": (i32, [vp]),
        "mtk_coo_nnz": (i64, [vp]),
        "mttkrp_coo": (i32, [vp, vp, P3, i64, i32, vp, vp]),
        "als_sweep_coo": (i32, [vp, vp, P3, vp, i64, i32, vp]),
        "mttkrp_dimtree": (i32, [vp, ctypes.POINTER(Tensor), P3, i64, i32, i32, vp, vp]),
        "mtk_sweep_uses_dimtree": (i32, [ctypes.POINTER(i64), i64, i32]),
        "gram_solve": (i32, [vp, P3, ctypes.POINTER(i64), i64, i32, vp, vp, vp, vp]),
        "mtk_fit": (i32, [vp, ctypes.POINTER(Tensor), P3, vp, i64, ctypes.POINTER(d), vp]),
        "als_sweep": (i32, [vp, ctypes.POINTER(Tensor), P3, vp, i64, i32, i32, ctypes.POINTER(d), vp]),
        "als_run": (i32, [vp, ctypes.POINTER(Tensor), P3, vp, i64, i32, i32, d, ctypes.POINTER(d),
                          ctypes.POINTER(i32), ctypes.POINTER(d), vp]),
        "als_run_extrapolated": (i32, [vp, ctypes.POINTER(Tensor), P3, vp, i64, i32, i32, d, i32,
                                       ctypes.POINTER(d), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(d), vp]),
        "mtk_graph_reset": (i32, [vp]),
        "mtk_server_create": (i32, [ctypes.POINTER(vp), i32, ctypes.c_uint64, i32]),
        "mtk_server_submit": (i32, [vp, i64, vp, ctypes.POINTER(i64), i64, i32, i32, P3, P3, vp]),
        "mtk_server_poll": (i32, [vp, ctypes.POINTER(Result), i32, ctypes.POINTER(i32), d]),
        "mtk_server_stats": (i32, [vp, ctypes.POINTER(ServerStat)]),
        "mtk_server_request_bytes": (ctypes.c_uint64, [ctypes.POINTER(i64), i64, i32]),
        "mtk_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _dims(d: Sequence[int]):
    return (ctypes.c_int64 * 3)(*[int(x) for x in d])


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _prec(p) -> int:
    return PREC_NAMES[p] if isinstance(p, str) else int(p)


class CooTensor:
    """An mtk_coo: a sparse tensor held on the device in the library's form."""

    def __init__(self, L, h, dims, nnz):
        self._L, self.h, self.dims, self.nnz = L, h, tuple(dims), nnz

    def close(self):
        if getattr(self, "h", None):
            self._L.mtk_coo_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


class Context:
    """An mtk_ctx on one device."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.mtk_create(ctypes.byref(h), int(device))
        if st != MTK_OK:
            raise MtkError(st, f"mtk_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self._L.mtk_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st: int):
        if st == MTK_OK:
            return
        msg = self._L.mtk_last_error(self.h).decode()
        if st == MTK_ENOTSPD:
            raise NotSPDError(st, msg)
        raise MtkError(st, msg)

    # -- C ABI calls ---------------------------------------------------------
    def check(self, stream=None):
        self._chk(self._L.mtk_check(self.h, _stream(stream)))

    def reserve(self, dims, R, prec):
        self._chk(self._L.mtk_reserve(self.h, _dims(dims), int(R), _prec(prec)))

    def quantize_fp8(self, x, q_out=None, exp_out=None, transposed=False, stream=None):
        """x: CUDA float32 (I,J,K).  Returns (codes uint8, exponents int32), or
        (codes, exponents, slice-transposed codes) with ``transposed=True``."""
        import torch
        if q_out is None:
            q_out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
        if exp_out is None:
            exp_out = torch.empty(x.shape[0], dtype=torch.int32, device=x.device)
        qt = None
        if transposed:
            qt = torch.empty((x.shape[0], x.shape[2], x.shape[1]), dtype=torch.uint8, device=x.device)
        self._chk(self._L.mtk_quantize_fp8(self.h, _ptr(x), _dims(x.shape), _ptr(q_out), _ptr(qt), _ptr(exp_out),
                                           _stream(stream)))
        return (q_out, exp_out, qt) if transposed else (q_out, exp_out)

    @staticmethod
    def tensor_desc(X, slice_exp=None, dims=None, X_t=None) -> Tensor:
        import torch
        fmt = FP8_E4M3 if X.dtype == torch.uint8 else FP32
        d = dims if dims is not None else X.shape
        return Tensor(_ptr(X), _ptr(X_t), _dims(d), fmt, _ptr(slice_exp))

    def mttkrp(self, X, factors, mode: int, prec="fp32", out=None, slice_exp=None, R=None, stream=None,
               desc: Optional[Tensor] = None, X_t=None):
        import torch
        R = int(R if R is not None else next(f for f in factors if f is not None).shape[1])
        d = desc or self.tensor_desc(X, slice_exp, X_t=X_t)
        if out is None:
            rows = d.dims[mode] if 0 <= int(mode) < 3 else 1     # invalid modes are rejected by the library
            out = torch.empty((rows, R), dtype=torch.float32, device=X.device)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.mttkrp(self.h, ctypes.byref(d), fp, R, int(mode), _prec(prec), _ptr(out),
                                 _stream(stream)))
        return out

    def mttkrp_noalloc(self, X, factors, mode: int, out, prec="fp32", slice_exp=None, R=None, stream=None,
                       X_t=None):
        """mttkrp into a caller-provided ``out`` with no device allocation (the
        library's static scratch; calls on one device must not overlap)."""
        R = int(R if R is not None else next(f for f in factors if f is not None).shape[1])
        d = self.tensor_desc(X, slice_exp, X_t=X_t)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.mttkrp_noalloc(self.h, ctypes.byref(d), fp, R, int(mode), _prec(prec), _ptr(out),
                                         _stream(stream)))
        return out

    def mttkrp_nway(self, X, factors, mode: int, prec="fp32", out=None, R=None, stream=None):
        """Mode-n MTTKRP of an N-way FP32 tensor (3 <= N <= 8)."""
        import torch
        R = int(R if R is not None else next(f for f in factors if f is not None).shape[1])
        n = X.dim()
        if out is None:
            rows = X.shape[mode] if 0 <= int(mode) < n else 1
            out = torch.empty((rows, R), dtype=torch.float32, device=X.device)
        dims = (ctypes.c_int64 * n)(*[int(d) for d in X.shape])
        fp = (ctypes.c_void_p * n)(*[_ptr(f) for f in factors])
        self._chk(self._L.mttkrp_nway(self.h, _ptr(X), n, dims, fp, R, int(mode), _prec(prec), _ptr(out),
                                      _stream(stream)))
        return out

    def als_sweep_nway(self, X, factors, lam, nsweeps: int, prec="fp32", stream=None):
        """CP-ALS sweeps of an N-way FP32 tensor, factors (FP32) and lam (FP64)
        updated in place."""
        n = X.dim()
        dims = (ctypes.c_int64 * n)(*[int(d) for d in X.shape])
        fp = (ctypes.c_void_p * n)(*[_ptr(f) for f in factors])
        self._chk(self._L.als_sweep_nway(self.h, _ptr(X), n, dims, fp, _ptr(lam), int(factors[0].shape[1]),
                                         _prec(prec), int(nsweeps), _stream(stream)))

    def coo_create(self, dims, idx, vals, stream=None):
        """Sparse tensor from coordinates: idx = three device int32 tensors
        (nnz each), vals = device float32 (nnz); returns a CooTensor."""
        dims = [int(d) for d in dims]
        nnz = int(vals.numel())
        h = ctypes.c_void_p()
        ip = (ctypes.c_void_p * 3)(*[_ptr(i) for i in idx])
        self._chk(self._L.mtk_coo_create(self.h, _dims(dims), nnz, ip, _ptr(vals), _stream(stream), ctypes.byref(h)))
        return CooTensor(self._L, h, dims, nnz)

    def mttkrp_coo(self, t, factors, mode: int, out=None, R=None, stream=None):
        """Mode-n MTTKRP of a CooTensor (FP32)."""
        import torch
        R = int(R if R is not None else next(f for f in factors if f is not None).shape[1])
        if out is None:
            rows = t.dims[mode] if 0 <= int(mode) < 3 else 1
            dev = next(f for f in factors if f is not None).device
            out = torch.empty((rows, R), dtype=torch.float32, device=dev)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.mttkrp_coo(self.h, t.h, fp, R, int(mode), _ptr(out), _stream(stream)))
        return out

    def als_sweep_coo(self, t, factors, lam, nsweeps: int, stream=None):
        """CP-ALS sweeps on a CooTensor, factors (float32) and lam (float64)
        updated in place."""
        R = int(factors[0].shape[1])
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.als_sweep_coo(self.h, t.h, fp, _ptr(lam), R, int(nsweeps), _stream(stream)))

    def mttkrp_dimtree(self, X, factors, mode: int, prec="fp32", out=None, R=None, stream=None):
        """Mode-0 / mode-1 MTTKRP through Y = X x3 C (the sweep's dimension tree)."""
        import torch
        R = int(R if R is not None else next(f for f in factors if f is not None).shape[1])
        d = self.tensor_desc(X)
        if out is None:
            rows = d.dims[mode] if 0 <= int(mode) < 3 else 1     # invalid modes are rejected by the library
            out = torch.empty((rows, R), dtype=torch.float32, device=X.device)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.mttkrp_dimtree(self.h, ctypes.byref(d), fp, R, int(mode), _prec(prec), _ptr(out),
                                         _stream(stream)))
        return out

    @staticmethod
    def sweep_uses_dimtree(dims, R: int, prec="fp32") -> bool:
        return bool(lib().mtk_sweep_uses_dimtree(_dims(dims), int(R), _prec(prec)))

    def gram_solve(self, factors, dims, mode: int, M, factor_out=None, lambda_out=None, R=None, stream=None):
        import torch
        R = int(R if R is not None else M.shape[1])
        if factor_out is None:
            factor_out = torch.empty_like(M)
        if lambda_out is None:
            lambda_out = torch.empty(R, dtype=torch.float64, device=M.device)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        self._chk(self._L.gram_solve(self.h, fp, _dims(dims), R, int(mode), _ptr(M), _ptr(factor_out),
                                     _ptr(lambda_out), _stream(stream)))
        return factor_out, lambda_out

    def fit(self, X, factors, lam, slice_exp=None, stream=None, X_t=None) -> float:
        d = self.tensor_desc(X, slice_exp, X_t=X_t)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        out = ctypes.c_double()
        self._chk(self._L.mtk_fit(self.h, ctypes.byref(d), fp, _ptr(lam), int(factors[0].shape[1]),
                                  ctypes.byref(out), _stream(stream)))
        return out.value

    def als_sweep(self, X, factors, lam, nsweeps: int, prec="fp32", slice_exp=None, with_fit=False,
                  stream=None, X_t=None):
        """In-place CP-ALS sweeps on device factors (FP32) and lambda (FP64).
        Returns the per-sweep fits (numpy) if with_fit else None."""
        d = self.tensor_desc(X, slice_exp, X_t=X_t)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        fits = np.zeros(max(1, nsweeps)) if with_fit else None
        fptr = fits.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if with_fit else None
        self._chk(self._L.als_sweep(self.h, ctypes.byref(d), fp, _ptr(lam), int(factors[0].shape[1]),
                                    _prec(prec), int(nsweeps), fptr, _stream(stream)))
        return fits[:nsweeps] if with_fit else None

    def als_run(self, X, factors, lam, max_sweeps: int, prec="fp32", tol: float = 0.0, slice_exp=None,
                final_fit=True, stream=None, X_t=None):
        """CP-ALS until the per-sweep fit changes by less than tol (at most
        max_sweeps).  Returns (per-sweep fits, sweeps run, direct fit of the
        final model or None)."""
        d = self.tensor_desc(X, slice_exp, X_t=X_t)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        fits = np.zeros(max(1, max_sweeps))
        done = ctypes.c_int(0)
        ff = ctypes.c_double(float("nan"))
        self._chk(self._L.als_run(self.h, ctypes.byref(d), fp, _ptr(lam), int(factors[0].shape[1]), _prec(prec),
                                  int(max_sweeps), float(tol), fits.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  ctypes.byref(done), ctypes.byref(ff) if final_fit else None, _stream(stream)))
        return fits[:done.value], done.value, (ff.value if final_fit else None)

    def als_run_extrapolated(self, X, factors, lam, max_sweeps: int, ls_start: int = 2, prec="fp32",
                             tol: float = 0.0, slice_exp=None, final_fit=True, stream=None, X_t=None):
        """als_run with an extrapolation candidate after every sweep >=
        ls_start.  Returns (per-sweep kept fits, accepted flags, sweeps run,
        direct fit of the final model or None)."""
        d = self.tensor_desc(X, slice_exp, X_t=X_t)
        fp = (ctypes.c_void_p * 3)(*[_ptr(f) for f in factors])
        fits = np.zeros(max(1, max_sweeps))
        acc = np.zeros(max(1, max_sweeps), dtype=np.int32)
        done = ctypes.c_int(0)
        ff = ctypes.c_double(float("nan"))
        self._chk(self._L.als_run_extrapolated(
            self.h, ctypes.byref(d), fp, _ptr(lam), int(factors[0].shape[1]), _prec(prec), int(max_sweeps),
            float(tol), int(ls_start), fits.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            acc.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), ctypes.byref(done),
            ctypes.byref(ff) if final_fit else None, _stream(stream)))
        return fits[:done.value], acc[:done.value].astype(bool), done.value, (ff.value if final_fit else None)

    def graph_reset(self):
        self._chk(self._L.mtk_graph_reset(self.h))


class Server:
    """mtk_server: continuous batching of CP-ALS decompositions on one device
    (every resident request advances one mode update per scheduler step; a
    step is a captured graph of grouped launches over all of them).

    submit() copies the host inputs; results land in host arrays owned by
    this object until poll() returns them."""

    def __init__(self, device: int = 0, budget_bytes: int = 200 * 10**9, max_slots: int = 8):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.mtk_server_create(ctypes.byref(h), int(device), int(budget_bytes), int(max_slots))
        if st != MTK_OK:
            raise MtkError(st, "mtk_server_create failed")
        self.h = h
        self._live = {}

    @staticmethod
    def request_bytes(dims, R: int, prec="fp32") -> int:
        """Device bytes a request takes while resident (0 if invalid)."""
        return int(lib().mtk_server_request_bytes(_dims(dims), int(R), _prec(prec)))

    def submit(self, rid: int, X: np.ndarray, init: Sequence[np.ndarray], prec="fp32", sweeps: int = 10):
        X = np.ascontiguousarray(X, dtype=np.float32)
        init = [np.ascontiguousarray(f, dtype=np.float32) for f in init]
        R = init[0].shape[1]
        outs = [np.empty((d, R), np.float32) for d in X.shape]
        lam = np.empty(R, np.float64)
        ip = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in init])
        op = (ctypes.c_void_p * 3)(*[f.ctypes.data for f in outs])
        st = self._L.mtk_server_submit(self.h, int(rid), X.ctypes.data, _dims(X.shape), int(R), _prec(prec),
                                       int(sweeps), ip, op, lam.ctypes.data)
        if st != MTK_OK:
            raise MtkError(st, f"mtk_server_submit(id={rid}) failed")
        self._live[int(rid)] = (outs, lam)

    def poll(self, timeout_s: float = 0.0, cap: int = 64):
        """Finished requests as dicts (id, status, fit, factors, lambda, times)."""
        buf = (Result * cap)()
        n = ctypes.c_int(0)
        st = self._L.mtk_server_poll(self.h, buf, cap, ctypes.byref(n), float(timeout_s))
        if st not in (MTK_OK, MTK_EAGAIN):
            raise MtkError(st, "mtk_server_poll failed")
        res = []
        for k in range(n.value):
            r = buf[k]
            outs, lam = self._live.pop(int(r.id), (None, None))
            res.append({"id": int(r.id), "status": int(r.status), "R": int(r.R), "dims": tuple(r.dims),
                        "fit": float(r.fit), "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "factors": outs, "lambda": lam})
        return res

    def stats(self):
        st = ServerStat()
        self._L.mtk_server_stats(self.h, ctypes.byref(st))
        return {k: getattr(st, k) for k, _ in ServerStat._fields_}

    def close(self):
        if getattr(self, "h", None):
            self._L.mtk_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
