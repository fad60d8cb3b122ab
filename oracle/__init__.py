"""FP64 CPU oracle for Parallel SGLD matrix factorisation (arXiv:1506.01418).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package to check and time the GPU library.  The
product path never imports it, and it imports nothing from the product.

The arithmetic lives in ``psgld_oracle.c`` (plain C, double precision); this
module only compiles it with gcc, marshals numpy arrays through ctypes and
keeps the chain state between calls.  See the C file's header for what is
computed and which passage of the paper each step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "psgld_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAG_NOISE_OFF = 1
FLAG_FREEZE_W = 2
FLAG_FREEZE_H = 4
STREAM_W = 0
STREAM_H = 1
PRIOR_KINDS = {"exponential": 0, "gaussian": 1}


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction; OpenMP
    threads over the blocks of a part and the rows/columns of the sweep)."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


PART_ORDERS = {"cyclic": 0, "random": 1}


class _Cfg(C.Structure):
    _fields_ = [("I", C.c_int64), ("J", C.c_int64), ("K", C.c_int32), ("B", C.c_int32),
                ("beta", C.c_double), ("phi", C.c_double), ("mu_floor", C.c_double),
                ("prior_kind", C.c_int32), ("mirror", C.c_int32),
                ("lambda_w", C.c_double), ("lambda_h", C.c_double),
                ("eps_a", C.c_double), ("eps_t0", C.c_double), ("eps_gamma", C.c_double),
                ("seed", C.c_uint64), ("burn_in", C.c_int64), ("thin", C.c_int32),
                ("flags", C.c_uint32), ("part_order", C.c_int32)]


_P = C.c_void_p


class _State(C.Structure):
    _fields_ = [("nnz", C.c_int64), ("row", _P), ("col", _P), ("val", _P),
                ("nho", C.c_int64), ("hrow", _P), ("hcol", _P),
                ("row_piece", _P), ("col_piece", _P),
                ("W", _P), ("H", _P), ("t", C.c_int64),
                ("sumW", _P), ("sumW2", _P), ("sumH", _P), ("sumH2", _P),
                ("n_kept", C.c_int64), ("ho_sum", _P), ("ho_cnt", _P)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.oracle_philox4x32_10.argtypes = [_P, _P, _P]
        L.oracle_normals.argtypes = [C.c_uint64, C.c_int64, C.c_uint32, C.c_int64, C.c_int32, _P, _P]
        L.oracle_partition.argtypes = [C.c_int64, C.c_int32, _P]
        L.oracle_partition.restype = C.c_int
        L.oracle_dbeta.argtypes = [C.c_double, C.c_double, C.c_double]
        L.oracle_dbeta.restype = C.c_double
        L.oracle_eps.argtypes = [C.POINTER(_Cfg), C.c_int64]
        L.oracle_eps.restype = C.c_double
        L.oracle_part_sizes.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), _P]
        L.oracle_drift.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), C.c_int32, _P, _P]
        L.oracle_drift.restype = C.c_int
        L.oracle_loglik.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), _P]
        L.oracle_loglik.restype = C.c_int
        L.oracle_run.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), C.c_int64, _P, _P]
        L.oracle_run.restype = C.c_int
        L.oracle_prepare.argtypes = [C.POINTER(_Cfg), C.POINTER(_State)]
        L.oracle_prepare.restype = _P
        L.oracle_release.argtypes = [_P]
        L.oracle_release.restype = None
        L.oracle_run_prepared.argtypes = [C.POINTER(_Cfg), C.POINTER(_State), _P, C.c_int64, _P, _P]
        L.oracle_run_prepared.restype = C.c_int
        L.oracle_threads.argtypes = [C.c_int]
        L.oracle_threads.restype = C.c_int
        L.oracle_part_at.argtypes = [C.POINTER(_Cfg), C.c_int64, _P, C.c_int64]
        L.oracle_part_at.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> np.ndarray:
    """Raw Philox4x32-10 block for one 128-bit counter and 64-bit key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def normals(seed: int, t: int, stream: int, index: int, K: int):
    """The K standard normals (and Box-Muller radii) of one factor row/column."""
    z = np.zeros(K)
    r = np.zeros(K)
    lib().oracle_normals(seed, t, stream, index, K, _ptr(z), _ptr(r))
    return z, r


def partition(n: int, B: int) -> np.ndarray:
    """Piece index of every element of [n] under the contiguous B-partition."""
    out = np.zeros(n, dtype=np.int32)
    if lib().oracle_partition(n, B, _ptr(out)) != 0:
        raise ValueError("partition needs 1 <= B <= n")
    return out


def dbeta(v: float, mu: float, beta: float) -> float:
    return lib().oracle_dbeta(float(v), float(mu), float(beta))


def threads(n: int = 0) -> int:
    """Sets the oracle's thread count when n >= 1; returns the count in use.
    Results do not depend on it (bitwise)."""
    return int(lib().oracle_threads(int(n)))


# ---------------------------------------------------------------- the chain
@dataclass
class Config:
    I: int
    J: int
    K: int
    B: int
    beta: float = 2.0
    phi: float = 1.0
    prior: str = "gaussian"
    lambda_w: float = 1.0
    lambda_h: float = 1.0
    mirror: bool = False
    eps_a: float = 1e-3
    eps_t0: float = 1.0
    eps_gamma: float = 0.51
    seed: int = 0
    burn_in: int = 0
    thin: int = 1
    flags: int = 0
    mu_floor: float = 1e-6
    part_order: str = "cyclic"    # or "random": parts drawn with probability |part| / N

    def c(self) -> _Cfg:
        return _Cfg(self.I, self.J, self.K, self.B, self.beta, self.phi, self.mu_floor,
                    PRIOR_KINDS[self.prior], int(bool(self.mirror)), self.lambda_w, self.lambda_h,
                    self.eps_a, self.eps_t0, self.eps_gamma, self.seed, self.burn_in, self.thin,
                    self.flags, PART_ORDERS[self.part_order])

    def eps(self, t: int) -> float:
        return lib().oracle_eps(C.byref(self.c()), t)


class Chain:
    """One PSGLD chain in FP64.  W is I x K and H is K x J (the paper's
    orientation).  With mirroring on, the initial factors are mirrored on
    load so that the chain starts on the non-negative orthant."""

    def __init__(self, cfg: Config, row, col, val, W0, H0, hrow=None, hcol=None,
                 row_piece=None, col_piece=None):
        self.cfg = cfg
        self.row = np.ascontiguousarray(row, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.hrow = np.ascontiguousarray(hrow if hrow is not None else [], dtype=np.int32)
        self.hcol = np.ascontiguousarray(hcol if hcol is not None else [], dtype=np.int32)
        self.row_piece = np.ascontiguousarray(
            row_piece if row_piece is not None else partition(cfg.I, cfg.B), dtype=np.int32)
        self.col_piece = np.ascontiguousarray(
            col_piece if col_piece is not None else partition(cfg.J, cfg.B), dtype=np.int32)
        W = np.array(W0, dtype=np.float64).reshape(cfg.I, cfg.K)
        H = np.array(H0, dtype=np.float64).reshape(cfg.K, cfg.J)
        if cfg.mirror:
            W, H = np.abs(W), np.abs(H)
        self.W = np.ascontiguousarray(W)
        self.H = np.ascontiguousarray(H)
        self.t = 0
        self.sumW = np.zeros_like(self.W)
        self.sumW2 = np.zeros_like(self.W)
        self.sumH = np.zeros_like(self.H)
        self.sumH2 = np.zeros_like(self.H)
        self.n_kept = 0
        self.ho_sum = np.zeros(len(self.hrow))
        self.ho_cnt = np.zeros(len(self.hrow), dtype=np.int64)
        self._prep = None   # bucketing of the entries by (part, block), made on first run

    def __del__(self):
        if getattr(self, "_prep", None):
            lib().oracle_release(self._prep)
            self._prep = None

    def _prepared(self):
        if self._prep is None:
            self._prep = lib().oracle_prepare(C.byref(self.cfg.c()), C.byref(self._state()))
            if not self._prep:
                raise ValueError("oracle_prepare failed (invalid input or out of memory)")
        return self._prep

    def _state(self) -> _State:
        return _State(len(self.row), _ptr(self.row), _ptr(self.col), _ptr(self.val),
                      len(self.hrow), _ptr(self.hrow), _ptr(self.hcol),
                      _ptr(self.row_piece), _ptr(self.col_piece),
                      _ptr(self.W), _ptr(self.H), self.t,
                      _ptr(self.sumW), _ptr(self.sumW2), _ptr(self.sumH), _ptr(self.sumH2),
                      self.n_kept, _ptr(self.ho_sum), _ptr(self.ho_cnt))

    def set_state(self, W, H, t: int):
        self.W = np.ascontiguousarray(np.array(W, dtype=np.float64).reshape(self.cfg.I, self.cfg.K))
        self.H = np.ascontiguousarray(np.array(H, dtype=np.float64).reshape(self.cfg.K, self.cfg.J))
        self.t = int(t)

    def run(self, n_iter: int, bounds: bool = False):
        """Run n_iter iterations.  With bounds=True, return the per-parameter
        magnitude scales (c_W, c_H) of the last iteration."""
        st = self._state()
        bW = np.zeros_like(self.W) if bounds else None
        bH = np.zeros_like(self.H) if bounds else None
        rc = lib().oracle_run_prepared(C.byref(self.cfg.c()), C.byref(st), self._prepared(), n_iter,
                                       _ptr(bW), _ptr(bH))
        self.t = st.t
        self.n_kept = st.n_kept
        if rc != 0:
            raise FloatingPointError(f"oracle_run failed with status {rc} at t={self.t}")
        return (bW, bH) if bounds else None

    def drift(self, p: int):
        dW = np.zeros_like(self.W)
        dH = np.zeros_like(self.H)
        rc = lib().oracle_drift(C.byref(self.cfg.c()), C.byref(self._state()), p, _ptr(dW), _ptr(dH))
        if rc != 0:
            raise ValueError(f"oracle_drift status {rc}")
        return dW, dH

    def part_sizes(self) -> np.ndarray:
        out = np.zeros(self.cfg.B, dtype=np.int64)
        lib().oracle_part_sizes(C.byref(self.cfg.c()), C.byref(self._state()), _ptr(out))
        return out

    def part_at(self, t: int) -> int:
        """The part iteration t uses (cyclic, or drawn per Condition 2)."""
        n_p = self.part_sizes()
        return int(lib().oracle_part_at(C.byref(self.cfg.c()), t, _ptr(n_p), int(n_p.sum())))

    def loglik(self) -> float:
        out = np.zeros(1)
        if lib().oracle_loglik(C.byref(self.cfg.c()), C.byref(self._state()), _ptr(out)) != 0:
            raise ValueError("oracle_loglik failed")
        return float(out[0])

    def posterior_mean(self):
        n = max(self.n_kept, 1)
        return self.sumW / n, self.sumH / n

    def posterior_var(self):
        n = max(self.n_kept, 1)
        mW, mH = self.sumW / n, self.sumH / n
        return self.sumW2 / n - mW * mW, self.sumH2 / n - mH * mH

    def heldout_prediction(self) -> np.ndarray:
        return self.ho_sum / np.maximum(self.ho_cnt, 1)

    def heldout_rmse(self, hval) -> float:
        pred = self.heldout_prediction()
        return float(np.sqrt(np.mean((np.asarray(hval, dtype=np.float64) - pred) ** 2)))
