"""Python binding of the FP64 CPU oracle of SaCD (oracle/sacd_oracle.c).

TEST INFRASTRUCTURE ONLY.  The oracle checks the GPU library; only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.
It shares no code with the GPU library and never imports it.

Paper: Balasubramaniam, Nayak, Yuen, "Efficient Nonnegative Tensor
Factorization via Saturating Coordinate Descent" (arXiv 2003.03572).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle_sacd.so")
SRC_PATH = os.path.join(_HERE, "sacd_oracle.c")

UPDATE_GS = 0
UPDATE_JACOBI = 1


SRC_N_PATH = os.path.join(_HERE, "sacd_oracle_n.c")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math; OpenMP for the
    loops whose iterations are independent)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wextra", "-o", tmp, SRC_PATH, SRC_N_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        p = C.c_void_p
        i64, i32, dbl = C.c_int64, C.c_int, C.c_double
        L.ora_tensor_create.argtypes = [p, i64, p, p, C.POINTER(p)]
        L.ora_tensor_destroy.argtypes = [p]
        L.ora_tensor_destroy.restype = None
        L.ora_tensor_nnz.argtypes = [p]
        L.ora_tensor_nnz.restype = i64
        L.ora_tensor_norm2.argtypes = [p]
        L.ora_tensor_norm2.restype = dbl
        L.ora_tensor_mode_coo.argtypes = [p, i32, p, p, p]
        L.ora_mttkrp.argtypes = [p, i32, i32, p, p, p, p]
        L.ora_splitmix64.argtypes = [C.c_uint64, i64, p]
        L.ora_splitmix64.restype = None
        L.ora_cd_delta.argtypes = [dbl, dbl, dbl]
        L.ora_cd_delta.restype = dbl
        L.ora_importance.argtypes = [dbl, dbl, dbl]
        L.ora_importance.restype = dbl
        L.ora_select.argtypes = [i64, dbl, dbl, i32]
        L.ora_select.restype = i32
        L.ora_model_create.argtypes = [p, i32, C.c_uint64, i32, C.POINTER(p)]
        L.ora_model_destroy.argtypes = [p]
        L.ora_model_destroy.restype = None
        L.ora_model_get_factor.argtypes = [p, i32, p]
        L.ora_model_set_factor.argtypes = [p, i32, p]
        L.ora_model_get_state.argtypes = [p, i32, p, p, p]
        L.ora_model_set_state.argtypes = [p, i32, p, dbl, i64]
        L.ora_model_force_flip.argtypes = [p, i32]
        L.ora_model_force_flip.restype = None
        L.ora_model_set_tie_tol.argtypes = [p, dbl]
        L.ora_model_set_tie_tol.restype = None
        L.ora_sweep.argtypes = [p, i32]
        L.ora_sweep_info.argtypes = [p, i32, p, p, p, p, p, p]
        L.ora_sweep_band.argtypes = [p, i32, p, p, p]
        L.ora_sweep_undo.argtypes = [p, i32]
        L.ora_sttvp.argtypes = [p, i32, i32, i32, p, p, p, p]
        L.oran_tensor_create.argtypes = [i32, p, i64, p, p, C.POINTER(p)]
        L.oran_tensor_destroy.argtypes = [p]
        L.oran_tensor_destroy.restype = None
        L.oran_tensor_nnz.argtypes = [p]
        L.oran_tensor_nnz.restype = i64
        L.oran_tensor_norm2.argtypes = [p]
        L.oran_tensor_norm2.restype = dbl
        L.oran_tensor_mode_coo.argtypes = [p, i32, p, p, p]
        L.oran_mttkrp.argtypes = [p, i32, i32, p, p]
        L.oran_model_create.argtypes = [p, i32, C.c_uint64, C.POINTER(p)]
        L.oran_model_destroy.argtypes = [p]
        L.oran_model_destroy.restype = None
        L.oran_model_get_factor.argtypes = [p, i32, p]
        L.oran_model_set_factor.argtypes = [p, i32, p]
        L.oran_model_get_state.argtypes = [p, i32, p, p, p]
        L.oran_model_set_state.argtypes = [p, i32, p, dbl, i64]
        L.oran_sweep.argtypes = [p, i32]
        L.oran_sweep_info.argtypes = [p, i32, p, p, p, p, p]
        L.oran_sweep_band.argtypes = [p, i32, p, p, p]
        L.oran_row_outcome.argtypes = [p, i32, i64, p, p]
        L.oran_objective.argtypes = [p]
        L.oran_objective.restype = dbl
        L.ora_model_set_columns.argtypes = [p, i32]
        L.ora_set_threads.argtypes = [i32]
        L.ora_set_threads.restype = i32
        L.ora_row_outcome.argtypes = [p, i32, i64, p, p]
        L.ora_objective.argtypes = [p]
        L.ora_objective.restype = dbl
        L.ora_fit.argtypes = [p, p, p]
        L.ora_run_until.argtypes = [p, dbl, i32, p, p, p]
        L.ora_rmse.argtypes = [p, i64, p, p, p]
        L.ora_pd.argtypes = [p, i32, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


class Tensor:
    """Sparse 3-way tensor (observed set Omega, Sec. 3)."""

    def __init__(self, dims, idx: np.ndarray, vals: np.ndarray):
        self.dims = tuple(int(d) for d in dims)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
        vals = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1)
        if idx.shape[0] != vals.shape[0]:
            raise ValueError("idx and vals disagree on nnz")
        d = np.array(self.dims, dtype=np.int64)
        h = C.c_void_p()
        _check(lib().ora_tensor_create(_ptr(d), idx.shape[0], _ptr(idx), _ptr(vals),
                                       C.byref(h)), "ora_tensor_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.ora_tensor_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    @property
    def nnz(self) -> int:
        return int(lib().ora_tensor_nnz(self._h))

    @property
    def norm2(self) -> float:
        return float(lib().ora_tensor_norm2(self._h))

    def mode_coo(self, mode: int):
        """(coords (nnz x 3: i_n, i_a, i_b), vals, ptr) sorted for `mode`."""
        nnz = self.nnz
        coords = np.empty((nnz, 3), np.int32)
        vals = np.empty(nnz, np.float32)
        ptr = np.empty(self.dims[mode] + 1, np.int64)
        _check(lib().ora_tensor_mode_coo(self._h, mode, _ptr(coords), _ptr(vals), _ptr(ptr)),
               "ora_tensor_mode_coo")
        return coords, vals, ptr

    def sttvp(self, mode: int, r: int, factors) -> np.ndarray:
        """Column r of the MTTKRP of `mode` (Sec. 4.4 column form)."""
        R = factors[0].shape[1]
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
        m = np.empty(self.dims[mode], np.float64)
        _check(lib().ora_sttvp(self._h, mode, R, r, _ptr(fs[0]), _ptr(fs[1]), _ptr(fs[2]), _ptr(m)),
               "ora_sttvp")
        return m

    def mttkrp(self, mode: int, factors) -> np.ndarray:
        R = factors[0].shape[1]
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
        M = np.empty((self.dims[mode], R), np.float64)
        _check(lib().ora_mttkrp(self._h, mode, R, _ptr(fs[0]), _ptr(fs[1]), _ptr(fs[2]), _ptr(M)),
               "ora_mttkrp")
        return M


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, np.uint64)
    lib().ora_splitmix64(C.c_uint64(seed), count, _ptr(out))
    return out


def cd_delta(a: float, g: float, h: float) -> float:
    return float(lib().ora_cd_delta(a, g, h))


def importance(g: float, delta: float, L: float) -> float:
    return float(lib().ora_importance(g, delta, L))


def select(k: int, z: float, zprev: float, flip: bool) -> bool:
    return bool(lib().ora_select(k, z, zprev, int(flip)))


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's parallel loops (n < 1: unchanged); returns the
    count in use.  Results are bit-identical for any count."""
    return int(lib().ora_set_threads(int(n)))


class Model:
    """SaCD state for one tensor (Alg. 1): factors, Grams, Z^{k-1}, ti^{k-1}, k."""

    def __init__(self, tensor: Tensor, R: int, seed: int, update: int = UPDATE_GS):
        self.t = tensor
        self.R = int(R)
        h = C.c_void_p()
        _check(lib().ora_model_create(tensor._h, self.R, C.c_uint64(seed), update, C.byref(h)),
               "ora_model_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.ora_model_destroy(h)
            except Exception:  # interpreter shutdown
                pass
            self._h = None

    def factor(self, mode: int) -> np.ndarray:
        out = np.empty((self.t.dims[mode], self.R), np.float64)
        _check(lib().ora_model_get_factor(self._h, mode, _ptr(out)), "get_factor")
        return out

    def set_factor(self, mode: int, A: np.ndarray):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (self.t.dims[mode], self.R)
        _check(lib().ora_model_set_factor(self._h, mode, _ptr(A)), "set_factor")

    def state(self, mode: int):
        zp = np.empty((self.t.dims[mode], self.R), np.float64)
        ti = C.c_double()
        k = C.c_int64()
        _check(lib().ora_model_get_state(self._h, mode, _ptr(zp), C.byref(ti), C.byref(k)),
               "get_state")
        return zp, ti.value, k.value

    def set_state(self, mode: int, zprev: np.ndarray, ti_prev: float, k: int):
        zp = np.ascontiguousarray(zprev, dtype=np.float64)
        assert zp.shape == (self.t.dims[mode], self.R)
        _check(lib().ora_model_set_state(self._h, mode, _ptr(zp), float(ti_prev), int(k)),
               "set_state")

    def set_columns(self, cb: int):
        """Column-at-a-time form with blocks of cb columns (0: row form)."""
        _check(lib().ora_model_set_columns(self._h, int(cb)), "set_columns")

    def force_flip(self, v: int):
        lib().ora_model_force_flip(self._h, int(v))

    def set_tie_tol(self, tau: float):
        lib().ora_model_set_tie_tol(self._h, float(tau))

    def sweep(self, mode: int):
        _check(lib().ora_sweep(self._h, mode), "ora_sweep")

    def undo_sweep(self, mode: int):
        """Restore the state before the last sweep of `mode` (factor, Gram,
        Z^{k-1}, ti^{k-1}, k and the band of Z^{k-1})."""
        _check(lib().ora_sweep_undo(self._h, mode), "ora_sweep_undo")

    def info(self, mode: int) -> dict:
        """Record of the last sweep of `mode` with its tie band.  kind: 0
        decided, 1 exact zero (decided), 2 zero-gradient tie, 3 margin tie;
        tie = kind >= 2."""
        I, R = self.t.dims[mode], self.R
        M = np.empty((I, R), np.float64)
        G0 = np.empty((I, R), np.float64)
        z = np.empty((I, R), np.float64)
        sel = np.empty((I, R), np.uint8)
        H = np.empty((R, R), np.float64)
        sc = np.empty(8, np.float64)
        _check(lib().ora_sweep_info(self._h, mode, _ptr(M), _ptr(G0), _ptr(z), _ptr(sel),
                                    _ptr(H), _ptr(sc)), "sweep_info")
        band = np.empty((I, R), np.float64)
        kind = np.empty((I, R), np.uint8)
        bs = np.empty(5, np.float64)
        _check(lib().ora_sweep_band(self._h, mode, _ptr(band), _ptr(kind), _ptr(bs)), "sweep_band")
        return dict(M=M, G0=G0, z=z, sel=sel.astype(bool), H=H,
                    L=sc[0], ti=sc[1], flip=bool(sc[2]), ti_prev=sc[3], f=sc[4],
                    nsel=int(sc[5]), inner=sc[6], model=sc[7],
                    band=band, kind=kind, tie=kind >= 2, band_ti=bs[0], tie_global=bool(bs[1]),
                    n_exact_zero=int(bs[2]), n_zero_grad=int(bs[3]), n_margin=int(bs[4]))

    def row_outcome(self, mode: int, q: int, sel: np.ndarray) -> np.ndarray:
        """Row q of the last sweep of `mode` updated under decisions `sel`."""
        sel = np.ascontiguousarray(sel, np.uint8).reshape(-1)
        assert sel.shape[0] == self.R
        out = np.empty(self.R, np.float64)
        _check(lib().ora_row_outcome(self._h, mode, int(q), _ptr(sel), _ptr(out)), "row_outcome")
        return out

    def objective(self) -> float:
        return float(lib().ora_objective(self._h))

    def fit(self):
        fit = C.c_double()
        f = C.c_double()
        _check(lib().ora_fit(self._h, C.byref(fit), C.byref(f)), "ora_fit")
        return fit.value, f.value

    def rmse(self, idx: np.ndarray, vals: np.ndarray) -> float:
        """eq. 30 on the given (held-out) entries."""
        idx = np.ascontiguousarray(idx, np.int32).reshape(-1, 3)
        vals = np.ascontiguousarray(vals, np.float32).reshape(-1)
        out = C.c_double()
        _check(lib().ora_rmse(self._h, idx.shape[0], _ptr(idx), _ptr(vals), C.byref(out)), "ora_rmse")
        return out.value

    def pd(self, mode: int = 2) -> float:
        """Pattern distinctiveness (eq. pd) of the columns of factor `mode`."""
        out = C.c_double()
        _check(lib().ora_pd(self._h, mode, C.byref(out)), "ora_pd")
        return out.value

    def run_until(self, tol: float, max_iter: int):
        trace = np.zeros(max_iter, np.float64)
        it = C.c_int()
        fit = C.c_double()
        _check(lib().ora_run_until(self._h, float(tol), int(max_iter), C.byref(it), C.byref(fit),
                                   _ptr(trace)), "ora_run_until")
        return it.value, fit.value, trace[: it.value]


class NTensor:
    """Sparse N-way tensor (Sec. 3, N modes)."""

    def __init__(self, dims, idx: np.ndarray, vals: np.ndarray):
        self.dims = tuple(int(d) for d in dims)
        self.N = len(self.dims)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, self.N)
        vals = np.ascontiguousarray(vals, dtype=np.float32).reshape(-1)
        d = np.array(self.dims, dtype=np.int64)
        h = C.c_void_p()
        _check(lib().oran_tensor_create(self.N, _ptr(d), idx.shape[0], _ptr(idx), _ptr(vals), C.byref(h)),
               "oran_tensor_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.oran_tensor_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def nnz(self) -> int:
        return int(lib().oran_tensor_nnz(self._h))

    @property
    def norm2(self) -> float:
        return float(lib().oran_tensor_norm2(self._h))

    def mode_coo(self, mode: int):
        nnz = self.nnz
        coords = np.empty((nnz, self.N), np.int32)
        vals = np.empty(nnz, np.float32)
        ptr = np.empty(self.dims[mode] + 1, np.int64)
        _check(lib().oran_tensor_mode_coo(self._h, mode, _ptr(coords), _ptr(vals), _ptr(ptr)), "mode_coo")
        return coords, vals, ptr

    def mttkrp(self, mode: int, factors) -> np.ndarray:
        R = factors[0].shape[1]
        fs = [np.ascontiguousarray(f, dtype=np.float64) for f in factors]
        arr = (C.c_void_p * self.N)(*[f.ctypes.data for f in fs])
        M = np.empty((self.dims[mode], R), np.float64)
        _check(lib().oran_mttkrp(self._h, mode, R, arr, _ptr(M)), "oran_mttkrp")
        return M


class NModel:
    """SaCD state of an N-way tensor: factors, Grams, Z^{k-1}, ti^{k-1}, k."""

    def __init__(self, tensor: NTensor, R: int, seed: int):
        self.t = tensor
        self.R = int(R)
        h = C.c_void_p()
        _check(lib().oran_model_create(tensor._h, self.R, C.c_uint64(seed), C.byref(h)), "oran_model_create")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            try:
                _lib.oran_model_destroy(h)
            except Exception:
                pass
            self._h = None

    def factor(self, mode: int) -> np.ndarray:
        out = np.empty((self.t.dims[mode], self.R), np.float64)
        _check(lib().oran_model_get_factor(self._h, mode, _ptr(out)), "get_factor")
        return out

    def set_factor(self, mode: int, A: np.ndarray):
        A = np.ascontiguousarray(A, dtype=np.float64)
        assert A.shape == (self.t.dims[mode], self.R)
        _check(lib().oran_model_set_factor(self._h, mode, _ptr(A)), "set_factor")

    def state(self, mode: int):
        zp = np.empty((self.t.dims[mode], self.R), np.float64)
        ti, k = C.c_double(), C.c_int64()
        _check(lib().oran_model_get_state(self._h, mode, _ptr(zp), C.byref(ti), C.byref(k)), "get_state")
        return zp, ti.value, k.value

    def set_state(self, mode: int, zprev: np.ndarray, ti_prev: float, k: int):
        zp = np.ascontiguousarray(zprev, dtype=np.float64)
        _check(lib().oran_model_set_state(self._h, mode, _ptr(zp), float(ti_prev), int(k)), "set_state")

    def sweep(self, mode: int):
        _check(lib().oran_sweep(self._h, mode), "oran_sweep")

    def info(self, mode: int) -> dict:
        """Record of the last sweep of `mode` with its tie band (keys as the
        three-way Model.info, without G0)."""
        I, R = self.t.dims[mode], self.R
        M = np.empty((I, R), np.float64)
        z = np.empty((I, R), np.float64)
        sel = np.empty((I, R), np.uint8)
        H = np.empty((R, R), np.float64)
        sc = np.empty(8, np.float64)
        _check(lib().oran_sweep_info(self._h, mode, _ptr(M), _ptr(z), _ptr(sel), _ptr(H), _ptr(sc)), "info")
        band = np.empty((I, R), np.float64)
        kind = np.empty((I, R), np.uint8)
        bs = np.empty(5, np.float64)
        _check(lib().oran_sweep_band(self._h, mode, _ptr(band), _ptr(kind), _ptr(bs)), "sweep_band")
        return dict(M=M, z=z, sel=sel.astype(bool), H=H, L=sc[0], ti=sc[1], flip=bool(sc[2]), ti_prev=sc[3],
                    f=sc[4], nsel=int(sc[5]), inner=sc[6], model=sc[7],
                    band=band, kind=kind, tie=kind >= 2, band_ti=bs[0], tie_global=bool(bs[1]),
                    n_exact_zero=int(bs[2]), n_zero_grad=int(bs[3]), n_margin=int(bs[4]))

    def row_outcome(self, mode: int, q: int, sel: np.ndarray) -> np.ndarray:
        """Row q of the last sweep of `mode` updated under decisions `sel`."""
        sel = np.ascontiguousarray(sel, np.uint8).reshape(-1)
        assert sel.shape[0] == self.R
        out = np.empty(self.R, np.float64)
        _check(lib().oran_row_outcome(self._h, mode, int(q), _ptr(sel), _ptr(out)), "row_outcome")
        return out

    def objective(self) -> float:
        return float(lib().oran_objective(self._h))
