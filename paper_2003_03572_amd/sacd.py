"""Thin Python binding of libsacd (include/sacd.h).

Argument marshalling only: every step of SaCD runs in the HIP library.
PyTorch provides device memory (through the allocator callback) and the HIP
stream the library orders its work on.  The library must be built
(``python -m paper_2003_03572_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SACD_LIB") or os.path.join(_HERE, "lib", "libsacd.so")

PREC_FP32 = 0
PREC_MIXED_BF16 = 1
UPDATE_GS = 0
UPDATE_JACOBI = 1

KERNEL_MTTKRP = 0
KERNEL_UPDATE = 1
KERNEL_IMPORTANCE = 2

_STATUS = {0: "ok", -1: "invalid argument", -2: "index out of range", -3: "out of device memory",
           -4: "bad state", -5: "device error", -6: "non-finite or degenerate value"}


class SacdError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__(f"{what}: {_STATUS.get(status, status)} ({detail})")
        self.status = status


class _Stats(C.Structure):
    _fields_ = [("k", C.c_int64), ("lipschitz", C.c_double), ("ti", C.c_double),
                ("flip", C.c_int32), ("n_selected", C.c_int64), ("objective", C.c_double)]


class _ServerConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_slots", C.c_int32), ("max_iter", C.c_int32),
                ("tol", C.c_double), ("precision", C.c_int), ("use_graphs", C.c_int32)]


class _ServerStats(C.Structure):
    _fields_ = [("running", C.c_int32), ("queued", C.c_int32), ("bytes_in_use", C.c_int64),
                ("peak_bytes", C.c_int64), ("steps", C.c_int64), ("graph_builds", C.c_int64),
                ("graph_launches", C.c_int64), ("eager_launches", C.c_int64),
                ("sec_admit", C.c_double), ("sec_tables", C.c_double), ("sec_iterate", C.c_double),
                ("sec_retire", C.c_double)]


JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED, JOB_CANCELLED = 0, 1, 2, 3, 4

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class _Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("release", _RELEASE_FN), ("user", C.c_void_p)]


_lib = None


def lib():
    """Load libsacd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libsacd.so is not built ({LIB_PATH}); run "
                               "python -m paper_2003_03572_amd.build")
        L = C.CDLL(LIB_PATH)
        p, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "sacd_create_tensor": [p, i64, p, p, p, p, C.POINTER(p)],
            "sacd_tensor_info": [p, p, p, p, p],
            "sacd_tensor_mode_coo": [p, i32, p, p, p],
            "sacd_init_factors": [p, i32, C.c_uint64, C.c_int, C.c_int, C.POINTER(p)],
            "sacd_init_factors_columns": [p, i32, C.c_uint64, i32, C.POINTER(p)],
            "sacd_sweep": [p, i32],
            "sacd_iterate": [p, i32],
            "sacd_fit": [p, p, p],
            "sacd_run_until": [p, dbl, i32, p, p],
            "sacd_get_factor": [p, i32, p],
            "sacd_set_factor": [p, i32, p],
            "sacd_get_state": [p, i32, p, p, p],
            "sacd_set_state": [p, i32, p, dbl, i64],
            "sacd_get_stats": [p, i32, p],
            "sacd_get_column_counts": [p, i32, p],
            "sacd_get_diagnostics": [p, i32, p, p, p],
            "sacd_set_diagnostics": [p, i32],
            "sacd_time_kernel": [p, i32, i32, i32, p],
            "sacd_timing_prepare": [p, i32],
            "sacd_iterate_timed": [p, i32, p, p],
            "sacd_kernel_bytes": [p, i32, i32, p],
            "sacd_model_bytes": [p, p],
            "sacd_job_bytes": [p, i64, i32, C.c_int, p, p],
            "sacd_rmse": [p, i64, p, p, p],
            "sacd_rmse_static": [p, i64, p, p, p],
            "sacd_pd": [p, i32, p],
            "sacd_server_create": [p, p, p, C.POINTER(p)],
            "sacd_server_submit": [p, p, i64, p, p, i32, C.c_uint64, p],
            "sacd_server_step": [p, p, p],
            "sacd_server_finished": [p, p, i32, p],
            "sacd_server_poll": [p, i64, p, p, p, p],
            "sacd_server_result": [p, i64, i32, p],
            "sacd_server_release": [p, i64],
            "sacd_server_cancel": [p, i64],
            "sacd_server_set_budget": [p, i64],
            "sacd_server_stats": [p, p],
            "sacd_create_ntensor": [i32, p, i64, p, p, p, p, C.POINTER(p)],
            "sacd_ntensor_info": [p, p, p, p, p, p],
            "sacd_ntensor_mode_coo": [p, i32, p, p, p],
            "sacd_init_nfactors": [p, i32, C.c_uint64, C.POINTER(p)],
            "sacd_nsweep": [p, i32],
            "sacd_niterate": [p, i32],
            "sacd_niterate_timed": [p, i32, p, p],
            "sacd_nfit": [p, p, p],
            "sacd_nrun_until": [p, dbl, i32, p, p],
            "sacd_get_nfactor": [p, i32, p],
            "sacd_set_nfactor": [p, i32, p],
            "sacd_get_nstate": [p, i32, p, p, p],
            "sacd_set_nstate": [p, i32, p, dbl, i64],
            "sacd_get_nstats": [p, i32, p],
            "sacd_get_ncolumn_counts": [p, i32, p],
            "sacd_get_ndiagnostics": [p, i32, p, p, p],
            "sacd_set_ndiagnostics": [p, i32],
            "sacd_nmodel_bytes": [p, p],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.sacd_destroy_tensor.argtypes = [p]
        L.sacd_destroy_tensor.restype = None
        L.sacd_destroy_model.argtypes = [p]
        L.sacd_destroy_model.restype = None
        L.sacd_server_destroy.argtypes = [p]
        L.sacd_server_destroy.restype = None
        L.sacd_destroy_ntensor.argtypes = [p]
        L.sacd_destroy_ntensor.restype = None
        L.sacd_destroy_nmodel.argtypes = [p]
        L.sacd_destroy_nmodel.restype = None
        L.sacd_last_error.restype = C.c_char_p
        L.sacd_status_string.restype = C.c_char_p
        L.sacd_version.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SacdError(rc, what, lib().sacd_last_error().decode(errors="replace"))


def _dptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


class TorchAllocator:
    """Device allocator backed by torch's caching allocator."""

    def __init__(self, device: torch.device):
        self.device = device
        self.live = {}
        self._alloc = _ALLOC_FN(self._do_alloc)
        self._release = _RELEASE_FN(self._do_release)
        self.struct = _Allocator(self._alloc, self._release, None)

    def _do_alloc(self, nbytes, user):
        try:
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except Exception:  # out of memory: the library reports SACD_ERR_NO_MEMORY
            return None
        ptr = t.data_ptr()
        self.live[ptr] = t
        return ptr

    def _do_release(self, ptr, user):
        self.live.pop(ptr, None)


class Tensor:
    """A sparse 3-way tensor resident on the GPU (sacd_create_tensor)."""

    def __init__(self, dims: Sequence[int], idx: torch.Tensor, vals: torch.Tensor,
                 stream: Optional[torch.cuda.Stream] = None, torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the SaCD library runs on the GPU only")
        self.device = idx.device if idx.is_cuda else torch.device("cuda", torch.cuda.current_device())
        idx = idx.to(self.device, torch.int32).contiguous().view(-1, 3)
        vals = vals.to(self.device, torch.float32).contiguous().view(-1)
        if idx.shape[0] != vals.shape[0]:
            raise ValueError("idx and vals disagree on nnz")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.alloc = TorchAllocator(self.device) if torch_allocator else None
        d = (C.c_int64 * 3)(*[int(x) for x in dims])
        h = C.c_void_p()
        # the input must be complete before the library's stream reads it
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().sacd_create_tensor(d, idx.shape[0], _dptr(idx), _dptr(vals),
                                        C.byref(self.alloc.struct) if self.alloc else None,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "sacd_create_tensor")
        self._h = h
        self._models = 0

    @classmethod
    def from_numpy(cls, dims, idx: np.ndarray, vals: np.ndarray, **kw) -> "Tensor":
        dev = torch.device("cuda", torch.cuda.current_device())
        return cls(dims, torch.from_numpy(np.ascontiguousarray(idx, np.int32)).to(dev),
                   torch.from_numpy(np.ascontiguousarray(vals, np.float32)).to(dev), **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().sacd_destroy_tensor(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        d = (C.c_int64 * 3)()
        nnz, n2, by = C.c_int64(), C.c_double(), C.c_int64()
        _check(lib().sacd_tensor_info(self._h, d, C.byref(nnz), C.byref(n2), C.byref(by)),
               "sacd_tensor_info")
        return dict(dims=tuple(d), nnz=nnz.value, norm2=n2.value, device_bytes=by.value)

    @property
    def dims(self) -> Tuple[int, int, int]:
        return self.info()["dims"]

    @property
    def nnz(self) -> int:
        return self.info()["nnz"]

    @property
    def norm2(self) -> float:
        return self.info()["norm2"]

    def mode_coo(self, mode: int):
        info = self.info()
        nnz = info["nnz"]
        coords = torch.empty((max(nnz, 1), 3), dtype=torch.int32, device=self.device)
        vals = torch.empty(max(nnz, 1), dtype=torch.float32, device=self.device)
        ptr = torch.empty(info["dims"][mode] + 1, dtype=torch.int64, device=self.device)
        _check(lib().sacd_tensor_mode_coo(self._h, mode, _dptr(coords), _dptr(vals), _dptr(ptr)),
               "sacd_tensor_mode_coo")
        return coords[:nnz], vals[:nnz], ptr


class Model:
    """SaCD model of rank R over a Tensor (sacd_init_factors)."""

    def __init__(self, tensor: Tensor, rank: int, seed: int, precision: int = PREC_FP32,
                 update: int = UPDATE_GS, columns: int = 0):
        """columns > 0: the column-at-a-time form with blocks of that many
        columns (FP32, Gauss-Seidel; sacd_init_factors_columns)."""
        self.t = tensor
        self.R = int(rank)
        h = C.c_void_p()
        if columns:
            if precision != PREC_FP32 or update != UPDATE_GS:
                raise ValueError("the column-at-a-time form is FP32 Gauss-Seidel")
            _check(lib().sacd_init_factors_columns(tensor._h, self.R, C.c_uint64(seed), int(columns),
                                                   C.byref(h)), "sacd_init_factors_columns")
        else:
            _check(lib().sacd_init_factors(tensor._h, self.R, C.c_uint64(seed), precision, update,
                                           C.byref(h)), "sacd_init_factors")
        self._h = h
        self.dims = tensor.dims

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().sacd_destroy_model(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, mode: int):
        _check(lib().sacd_sweep(self._h, mode), "sacd_sweep")

    def iterate(self, n: int = 1):
        _check(lib().sacd_iterate(self._h, n), "sacd_iterate")

    def fit(self) -> Tuple[float, float]:
        fit, f = C.c_double(), C.c_double()
        _check(lib().sacd_fit(self._h, C.byref(fit), C.byref(f)), "sacd_fit")
        return fit.value, f.value

    def run_until(self, tol: float, max_iter: int, record=None) -> Tuple[int, float]:
        """Outer iterations until the relative fit change is below tol (from the
        second on) or max_iter (sacd_run_until).  With `record` (a path, or a
        text file open for writing) the same iterations run sweep by sweep and
        each sweep writes one JSON line: iteration, mode, the mode's sweep
        counter k, objective f (eq. 6), fit, total importance ti (eq. 25), the
        eq. 27 branch (flip), the number of selected elements |E| and L."""
        if record is None:
            it, fit = C.c_int32(), C.c_double()
            _check(lib().sacd_run_until(self._h, float(tol), int(max_iter), C.byref(it), C.byref(fit)),
                   "sacd_run_until")
            return it.value, fit.value
        if int(max_iter) < 1 or not float(tol) >= 0.0:
            raise ValueError("max_iter < 1 or tol < 0")
        nx = float(np.sqrt(self.t.norm2))
        if not nx > 0.0:
            raise ValueError("||X|| = 0: the fit is undefined")
        own = isinstance(record, (str, os.PathLike))
        fh = open(record, "w") if own else record
        try:
            prev = fit = 0.0
            it = 0
            for it in range(1, int(max_iter) + 1):
                for n in range(3):
                    self.sweep(n)
                    s = self.stats(n)
                    fit = 1.0 - float(np.sqrt(max(s["f"], 0.0))) / nx
                    fh.write(json.dumps(dict(iter=it, mode=n, k=s["k"], f=s["f"], fit=fit, ti=s["ti"],
                                             flip=s["flip"], nsel=s["nsel"], L=s["L"])) + "\n")
                if it >= 2 and abs(fit - prev) < float(tol) * abs(prev):
                    break
                prev = fit
            return it, fit
        finally:
            if own:
                fh.close()

    def factor(self, mode: int) -> torch.Tensor:
        out = torch.empty((self.dims[mode], self.R), dtype=torch.float32, device=self.t.device)
        _check(lib().sacd_get_factor(self._h, mode, _dptr(out)), "sacd_get_factor")
        return out

    def set_factor(self, mode: int, A: torch.Tensor):
        A = A.to(self.t.device, torch.float32).contiguous()
        if tuple(A.shape) != (self.dims[mode], self.R):
            raise ValueError("factor shape mismatch")
        torch.cuda.current_stream(self.t.device).synchronize()
        _check(lib().sacd_set_factor(self._h, mode, _dptr(A)), "sacd_set_factor")

    def state(self, mode: int):
        zp = torch.empty((self.dims[mode], self.R), dtype=torch.float32, device=self.t.device)
        ti, k = C.c_double(), C.c_int64()
        _check(lib().sacd_get_state(self._h, mode, _dptr(zp), C.byref(ti), C.byref(k)),
               "sacd_get_state")
        return zp, ti.value, k.value

    def set_state(self, mode: int, zprev: torch.Tensor, ti_prev: float, k: int):
        zp = zprev.to(self.t.device, torch.float32).contiguous()
        if tuple(zp.shape) != (self.dims[mode], self.R):
            raise ValueError("zprev shape mismatch")
        torch.cuda.current_stream(self.t.device).synchronize()
        _check(lib().sacd_set_state(self._h, mode, _dptr(zp), float(ti_prev), int(k)),
               "sacd_set_state")

    def stats(self, mode: int) -> dict:
        s = _Stats()
        _check(lib().sacd_get_stats(self._h, mode, C.byref(s)), "sacd_get_stats")
        return dict(k=s.k, L=s.lipschitz, ti=s.ti, flip=bool(s.flip), nsel=s.n_selected,
                    f=s.objective)

    def column_counts(self, mode: int) -> np.ndarray:
        """|e_r|: elements of each column selected in the last sweep of `mode`."""
        out = np.zeros(self.R, np.int64)
        _check(lib().sacd_get_column_counts(self._h, mode, out.ctypes.data_as(C.c_void_p)),
               "sacd_get_column_counts")
        return out

    def set_diagnostics(self, on: bool):
        _check(lib().sacd_set_diagnostics(self._h, int(bool(on))), "sacd_set_diagnostics")

    def diagnostics(self, mode: int):
        I = self.dims[mode]
        M = torch.empty((I, self.R), dtype=torch.float32, device=self.t.device)
        sel = torch.empty((I, self.R), dtype=torch.uint8, device=self.t.device)
        G = np.empty((self.R, self.R), np.float64)
        _check(lib().sacd_get_diagnostics(self._h, mode, _dptr(M), _dptr(sel),
                                          G.ctypes.data_as(C.c_void_p)), "sacd_get_diagnostics")
        return M, sel.bool(), G

    def rmse(self, idx, vals) -> float:
        """eq. 30 on the given (held-out) entries: idx (n, 3), vals (n,)."""
        idx = torch.as_tensor(np.ascontiguousarray(idx, np.int32) if isinstance(idx, np.ndarray) else idx)
        vals = torch.as_tensor(np.ascontiguousarray(vals, np.float32) if isinstance(vals, np.ndarray) else vals)
        idx = idx.to(self.t.device, torch.int32).contiguous().view(-1, 3)
        vals = vals.to(self.t.device, torch.float32).contiguous().view(-1)
        self.t.stream.wait_stream(torch.cuda.current_stream(self.t.device))
        out = C.c_double()
        _check(lib().sacd_rmse(self._h, idx.shape[0], _dptr(idx), _dptr(vals), C.byref(out)), "sacd_rmse")
        return out.value

    def rmse_static(self, idx: torch.Tensor, vals: torch.Tensor, out: torch.Tensor):
        """sacd_rmse_static: eq. 30 into out (device, 2 float64: RMSE, out-of-range
        flag) on the model's stream, with no allocation and no synchronisation.
        idx (n, 3) int32 and vals (n,) float32 are device tensors."""
        if idx.dtype != torch.int32 or vals.dtype != torch.float32 or out.dtype != torch.float64:
            raise TypeError("idx int32, vals float32, out float64")
        if not (idx.is_cuda and vals.is_cuda and out.is_cuda) or out.numel() < 2:
            raise ValueError("device tensors; out holds 2 values")
        if not (idx.is_contiguous() and vals.is_contiguous() and out.is_contiguous()):
            raise ValueError("contiguous tensors")
        n = vals.numel()
        if idx.numel() != 3 * n:
            raise ValueError("idx is not n x 3")
        dev = self.t.device
        self.t.stream.wait_stream(torch.cuda.current_stream(dev))  # inputs ready
        _check(lib().sacd_rmse_static(self._h, n, _dptr(idx), _dptr(vals), _dptr(out)), "sacd_rmse_static")
        torch.cuda.current_stream(dev).wait_stream(self.t.stream)  # out ready for later torch work

    def pd(self, mode: int = 2) -> float:
        """Pattern distinctiveness (eq. pd) of the columns of factor `mode`."""
        out = C.c_double()
        _check(lib().sacd_pd(self._h, mode, C.byref(out)), "sacd_pd")
        return out.value

    def time_kernel(self, which: int, mode: int, reps: int) -> float:
        ms = C.c_float()
        _check(lib().sacd_time_kernel(self._h, which, mode, reps, C.byref(ms)), "sacd_time_kernel")
        return ms.value

    def timing_prepare(self, n_iters: int):
        """Create the HIP events for n_iters timed iterations (see iterate_timed)."""
        _check(lib().sacd_timing_prepare(self._h, n_iters), "sacd_timing_prepare")

    def iterate_timed(self, n_iters: int, sweeps: bool = False):
        """n_iters outer iterations, the same work as iterate() but enqueued
        launch by launch with HIP events around the MTTKRP launches and at the
        end of every sweep.  Waits for them; returns the MTTKRP kernel
        milliseconds as a list of n_iters [mode 0, 1, 2], and with sweeps=True
        also the whole sweeps' milliseconds in the same form."""
        out = (C.c_float * (3 * n_iters))()
        sw = (C.c_float * (3 * n_iters))()
        _check(lib().sacd_iterate_timed(self._h, n_iters, out, sw), "sacd_iterate_timed")
        mt = [[out[3 * i + n] for n in range(3)] for i in range(n_iters)]
        if not sweeps:
            return mt
        return mt, [[sw[3 * i + n] for n in range(3)] for i in range(n_iters)]

    def kernel_bytes(self, which: int, mode: int) -> float:
        b = C.c_double()
        _check(lib().sacd_kernel_bytes(self._h, which, mode, C.byref(b)), "sacd_kernel_bytes")
        return b.value

    def device_bytes(self) -> int:
        b = C.c_int64()
        _check(lib().sacd_model_bytes(self._h, C.byref(b)), "sacd_model_bytes")
        return b.value

    def synchronize(self):
        self.t.stream.synchronize()



class NTensor:
    """A sparse N-way tensor resident on the GPU (sacd_create_ntensor)."""

    def __init__(self, dims: Sequence[int], idx: torch.Tensor, vals: torch.Tensor,
                 stream: Optional[torch.cuda.Stream] = None, torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the SaCD library runs on the GPU only")
        self.N = len(dims)
        self.device = idx.device if idx.is_cuda else torch.device("cuda", torch.cuda.current_device())
        idx = idx.to(self.device, torch.int32).contiguous().view(-1, self.N)
        vals = vals.to(self.device, torch.float32).contiguous().view(-1)
        if idx.shape[0] != vals.shape[0]:
            raise ValueError("idx and vals disagree on nnz")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.alloc = TorchAllocator(self.device) if torch_allocator else None
        d = (C.c_int64 * self.N)(*[int(x) for x in dims])
        h = C.c_void_p()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(lib().sacd_create_ntensor(self.N, d, idx.shape[0], _dptr(idx), _dptr(vals),
                                         C.byref(self.alloc.struct) if self.alloc else None,
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "sacd_create_ntensor")
        self._h = h

    @classmethod
    def from_numpy(cls, dims, idx: np.ndarray, vals: np.ndarray, **kw) -> "NTensor":
        dev = torch.device("cuda", torch.cuda.current_device())
        return cls(dims, torch.from_numpy(np.ascontiguousarray(idx, np.int32)).to(dev),
                   torch.from_numpy(np.ascontiguousarray(vals, np.float32)).to(dev), **kw)

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().sacd_destroy_ntensor(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        n = C.c_int32()
        d = (C.c_int64 * 8)()
        nnz, n2, by = C.c_int64(), C.c_double(), C.c_int64()
        _check(lib().sacd_ntensor_info(self._h, C.byref(n), d, C.byref(nnz), C.byref(n2), C.byref(by)),
               "sacd_ntensor_info")
        return dict(N=n.value, dims=tuple(d[:n.value]), nnz=nnz.value, norm2=n2.value, device_bytes=by.value)

    @property
    def dims(self) -> Tuple[int, ...]:
        return self.info()["dims"]

    @property
    def nnz(self) -> int:
        return self.info()["nnz"]

    @property
    def norm2(self) -> float:
        return self.info()["norm2"]

    def mode_coo(self, mode: int):
        info = self.info()
        nnz = info["nnz"]
        coords = torch.empty((max(nnz, 1), self.N), dtype=torch.int32, device=self.device)
        vals = torch.empty(max(nnz, 1), dtype=torch.float32, device=self.device)
        ptr = torch.empty(info["dims"][mode] + 1, dtype=torch.int64, device=self.device)
        _check(lib().sacd_ntensor_mode_coo(self._h, mode, _dptr(coords), _dptr(vals), _dptr(ptr)),
               "sacd_ntensor_mode_coo")
        return coords[:nnz], vals[:nnz], ptr


class NModel:
    """SaCD model of rank R over an NTensor (sacd_init_nfactors): FP32,
    Gauss-Seidel; an iteration sweeps modes 0, ..., N - 1."""

    def __init__(self, tensor: NTensor, rank: int, seed: int):
        self.t = tensor
        self.R = int(rank)
        self.N = tensor.N
        h = C.c_void_p()
        _check(lib().sacd_init_nfactors(tensor._h, self.R, C.c_uint64(seed), C.byref(h)), "sacd_init_nfactors")
        self._h = h
        self.dims = tensor.dims

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().sacd_destroy_nmodel(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, mode: int):
        _check(lib().sacd_nsweep(self._h, mode), "sacd_nsweep")

    def iterate(self, n: int = 1):
        _check(lib().sacd_niterate(self._h, n), "sacd_niterate")

    def iterate_timed(self, n_iters: int):
        """(MTTKRP ms, sweep ms), each an (n_iters, N) array."""
        mt = np.zeros(n_iters * self.N, np.float32)
        sw = np.zeros(n_iters * self.N, np.float32)
        _check(lib().sacd_niterate_timed(self._h, int(n_iters), mt.ctypes.data_as(C.c_void_p),
                                         sw.ctypes.data_as(C.c_void_p)), "sacd_niterate_timed")
        return mt.reshape(n_iters, self.N), sw.reshape(n_iters, self.N)

    def fit(self) -> Tuple[float, float]:
        fit, f = C.c_double(), C.c_double()
        _check(lib().sacd_nfit(self._h, C.byref(fit), C.byref(f)), "sacd_nfit")
        return fit.value, f.value

    def run_until(self, tol: float, max_iter: int) -> Tuple[int, float]:
        it, fit = C.c_int32(), C.c_double()
        _check(lib().sacd_nrun_until(self._h, float(tol), int(max_iter), C.byref(it), C.byref(fit)),
               "sacd_nrun_until")
        return it.value, fit.value

    def factor(self, mode: int) -> torch.Tensor:
        out = torch.empty((self.dims[mode], self.R), dtype=torch.float32, device=self.t.device)
        _check(lib().sacd_get_nfactor(self._h, mode, _dptr(out)), "sacd_get_nfactor")
        return out

    def set_factor(self, mode: int, A: torch.Tensor):
        A = A.to(self.t.device, torch.float32).contiguous()
        if tuple(A.shape) != (self.dims[mode], self.R):
            raise ValueError("factor shape mismatch")
        torch.cuda.current_stream(self.t.device).synchronize()
        _check(lib().sacd_set_nfactor(self._h, mode, _dptr(A)), "sacd_set_nfactor")

    def state(self, mode: int):
        zp = torch.empty((self.dims[mode], self.R), dtype=torch.float32, device=self.t.device)
        ti, k = C.c_double(), C.c_int64()
        _check(lib().sacd_get_nstate(self._h, mode, _dptr(zp), C.byref(ti), C.byref(k)), "sacd_get_nstate")
        return zp, ti.value, k.value

    def set_state(self, mode: int, zprev: torch.Tensor, ti_prev: float, k: int):
        zp = zprev.to(self.t.device, torch.float32).contiguous()
        if tuple(zp.shape) != (self.dims[mode], self.R):
            raise ValueError("zprev shape mismatch")
        torch.cuda.current_stream(self.t.device).synchronize()
        _check(lib().sacd_set_nstate(self._h, mode, _dptr(zp), float(ti_prev), int(k)), "sacd_set_nstate")

    def stats(self, mode: int) -> dict:
        s = _Stats()
        _check(lib().sacd_get_nstats(self._h, mode, C.byref(s)), "sacd_get_nstats")
        return dict(k=s.k, L=s.lipschitz, ti=s.ti, flip=bool(s.flip), nsel=s.n_selected, f=s.objective)

    def column_counts(self, mode: int) -> np.ndarray:
        out = np.zeros(self.R, np.int64)
        _check(lib().sacd_get_ncolumn_counts(self._h, mode, out.ctypes.data_as(C.c_void_p)),
               "sacd_get_ncolumn_counts")
        return out

    def set_diagnostics(self, on: bool):
        _check(lib().sacd_set_ndiagnostics(self._h, int(bool(on))), "sacd_set_ndiagnostics")

    def diagnostics(self, mode: int):
        I = self.dims[mode]
        M = torch.empty((I, self.R), dtype=torch.float32, device=self.t.device)
        sel = torch.empty((I, self.R), dtype=torch.uint8, device=self.t.device)
        G = np.empty((self.R, self.R), np.float64)
        _check(lib().sacd_get_ndiagnostics(self._h, mode, _dptr(M), _dptr(sel), G.ctypes.data_as(C.c_void_p)),
               "sacd_get_ndiagnostics")
        return M, sel.bool(), G

    def device_bytes(self) -> int:
        b = C.c_int64()
        _check(lib().sacd_nmodel_bytes(self._h, C.byref(b)), "sacd_nmodel_bytes")
        return b.value

    def synchronize(self):
        self.t.stream.synchronize()


def job_bytes(dims: Sequence[int], nnz: int, rank: int, precision: int = PREC_FP32) -> Tuple[int, int]:
    """Upper bounds (resident, transient) of the device bytes of a job."""
    d = (C.c_int64 * 3)(*[int(x) for x in dims])
    a, b = C.c_int64(), C.c_int64()
    _check(lib().sacd_job_bytes(d, int(nnz), int(rank), int(precision), C.byref(a), C.byref(b)),
           "sacd_job_bytes")
    return a.value, b.value


class Server:
    """Many factorization jobs resident on the GPU, iterated together
    (sacd_server_*)."""

    def __init__(self, budget_bytes: int, max_slots: int = 256, max_iter: int = 500,
                 tol: float = 1e-4, precision: int = PREC_FP32, use_graphs: bool = True,
                 stream: Optional[torch.cuda.Stream] = None, torch_allocator: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the SaCD library runs on the GPU only")
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.alloc = TorchAllocator(self.device) if torch_allocator else None
        cfg = _ServerConfig(int(budget_bytes), int(max_slots), int(max_iter), float(tol),
                            int(precision), int(bool(use_graphs)))
        h = C.c_void_p()
        _check(lib().sacd_server_create(C.byref(cfg), C.byref(self.alloc.struct) if self.alloc else None,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h)),
               "sacd_server_create")
        self._h = h

    def submit(self, dims, idx: np.ndarray, vals: np.ndarray, rank: int, seed: int) -> int:
        idx = np.ascontiguousarray(idx, np.int32).reshape(-1, 3)
        vals = np.ascontiguousarray(vals, np.float32).reshape(-1)
        d = (C.c_int64 * 3)(*[int(x) for x in dims])
        t = C.c_int64()
        _check(lib().sacd_server_submit(self._h, d, idx.shape[0], idx.ctypes.data_as(C.c_void_p),
                                        vals.ctypes.data_as(C.c_void_p), int(rank), C.c_uint64(seed),
                                        C.byref(t)), "sacd_server_submit")
        return t.value

    def step(self) -> Tuple[int, int]:
        r, q = C.c_int32(), C.c_int32()
        _check(lib().sacd_server_step(self._h, C.byref(r), C.byref(q)), "sacd_server_step")
        return r.value, q.value

    def finished(self):
        n = C.c_int32()
        _check(lib().sacd_server_finished(self._h, None, 0, C.byref(n)), "sacd_server_finished")
        buf = (C.c_int64 * max(n.value, 1))()
        _check(lib().sacd_server_finished(self._h, buf, n.value, C.byref(n)), "sacd_server_finished")
        return [buf[i] for i in range(n.value)]

    def poll(self, ticket: int) -> dict:
        st, it = C.c_int32(), C.c_int32()
        fit, f = C.c_double(), C.c_double()
        rc = lib().sacd_server_poll(self._h, int(ticket), C.byref(st), C.byref(it), C.byref(fit),
                                    C.byref(f))
        if rc != 0 and st.value != JOB_FAILED:
            _check(rc, "sacd_server_poll")
        return dict(state=st.value, iters=it.value, fit=fit.value, f=f.value, status=rc)

    def result(self, ticket: int, dims: Sequence[int], rank: int):
        out = []
        for n in range(3):
            A = np.empty((int(dims[n]), int(rank)), np.float32)
            _check(lib().sacd_server_result(self._h, int(ticket), n, A.ctypes.data_as(C.c_void_p)),
                   "sacd_server_result")
            out.append(A)
        return out

    def release(self, ticket: int):
        _check(lib().sacd_server_release(self._h, int(ticket)), "sacd_server_release")

    def cancel(self, ticket: int):
        _check(lib().sacd_server_cancel(self._h, int(ticket)), "sacd_server_cancel")

    def set_budget(self, budget_bytes: int):
        _check(lib().sacd_server_set_budget(self._h, int(budget_bytes)), "sacd_server_set_budget")

    def stats(self) -> dict:
        s = _ServerStats()
        _check(lib().sacd_server_stats(self._h, C.byref(s)), "sacd_server_stats")
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().sacd_server_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
