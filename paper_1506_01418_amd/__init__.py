"""Python binding of libpsgld, the MI355X (gfx950) Parallel SGLD library.

The functions here carry the names of the C ABI in ``include/psgld.h`` and
only marshal arguments: every step of the sampler runs in the HIP kernels of
``libpsgld.so``.  There is no CPU fallback: if the library has not been built
(``python -m paper_1506_01418_amd.build``) importing this package fails.

``PSGLD`` is a thin convenience wrapper around one context.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsgld.so")

PSGLD_OK = 0
PSGLD_E_ARG = -1
PSGLD_E_STATE = -2
PSGLD_E_NOMEM = -3
PSGLD_E_DEVICE = -4
PSGLD_E_NUMERIC = -5
PSGLD_E_UNSUPPORTED = -6
STATUS_NAMES = {0: "OK", -1: "E_ARG", -2: "E_STATE", -3: "E_NOMEM", -4: "E_DEVICE",
                -5: "E_NUMERIC", -6: "E_UNSUPPORTED"}

PSGLD_PRIOR_EXPONENTIAL = 0
PSGLD_PRIOR_GAUSSIAN = 1
PSGLD_FP32 = 0
PSGLD_BF16_DENSE = 1
PSGLD_BF16_DENSE_VALUES = 2
PSGLD_TEST_NOISE_OFF = 1
PSGLD_TEST_FREEZE_W = 2
PSGLD_TEST_FREEZE_H = 4


class PsgldError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class psgld_likelihood(C.Structure):
    _fields_ = [("beta", C.c_double), ("phi", C.c_double)]


class psgld_prior(C.Structure):
    _fields_ = [("kind", C.c_int32), ("lambda_w", C.c_double), ("lambda_h", C.c_double),
                ("mirror", C.c_int32)]


class psgld_eps_schedule(C.Structure):
    _fields_ = [("a", C.c_double), ("t0", C.c_double), ("gamma", C.c_double)]


# allocator hooks of psgld_options: void *dev_alloc(size_t, void *), void dev_free(void *, size_t, void *)
DEV_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
DEV_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class psgld_options(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("burn_in", C.c_int64), ("thin", C.c_int32),
                ("precision", C.c_int32), ("dense_threshold", C.c_double),
                ("mu_floor", C.c_double), ("row_piece", C.c_void_p), ("col_piece", C.c_void_p),
                ("stream", C.c_void_p), ("test_flags", C.c_uint32), ("device", C.c_int32),
                ("graph_iters", C.c_int32), ("persistent", C.c_int32), ("part_order", C.c_int32),
                ("dense_min_cols", C.c_int32), ("persistent_grid", C.c_int32),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN), ("alloc_user", C.c_void_p)]


class psgld_server_options(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_active", C.c_int32), ("iters_per_tick", C.c_int32),
                ("device", C.c_int32), ("persistent", C.c_int32),
                ("dev_alloc", DEV_ALLOC_FN), ("dev_free", DEV_FREE_FN), ("alloc_user", C.c_void_p)]


class TorchAllocator:
    """The allocator hooks of psgld_options backed by PyTorch's caching
    allocator on `device`, with blocks tied to `stream` (a hipStream_t handle,
    0 = the device's default stream).  Keep the object alive as long as any
    context created with its hooks.  Counts the bytes it holds."""

    def __init__(self, device=0, stream=0, fail_after=None):
        import torch
        self._torch = torch
        self.device = int(device)
        self.stream = int(stream or 0)
        self.held = {}              # ptr -> bytes
        self.calls = 0
        self.fail_after = fail_after   # test hook: return NULL from this call on
        self.alloc_fn = DEV_ALLOC_FN(self._alloc)
        self.free_fn = DEV_FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        self.calls += 1
        if self.fail_after is not None and self.calls > self.fail_after:
            return None
        try:
            p = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
        except Exception:
            return None
        self.held[p] = int(nbytes)
        return p

    def _free(self, ptr, nbytes, user):
        if ptr in self.held:
            del self.held[ptr]
            self._torch.cuda.caching_allocator_delete(ptr)

    @property
    def bytes(self):
        return sum(self.held.values())

    def install(self, opt):
        opt.dev_alloc = self.alloc_fn
        opt.dev_free = self.free_fn
        opt.alloc_user = None


class psgld_job(C.Structure):
    _fields_ = [("I", C.c_int64), ("J", C.c_int64), ("K", C.c_int32), ("B", C.c_int32),
                ("lik", psgld_likelihood), ("prior", psgld_prior), ("seed", C.c_uint64),
                ("burn_in", C.c_int64), ("thin", C.c_int32), ("precision", C.c_int32),
                ("dense_threshold", C.c_double), ("dense_min_cols", C.c_int32),
                ("sched", psgld_eps_schedule), ("n_iter", C.c_int64),
                ("nnz", C.c_int64), ("row", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("dense", C.c_void_p), ("mask", C.c_void_p), ("n_heldout", C.c_int64),
                ("hrow", C.c_void_p), ("hcol", C.c_void_p), ("hval", C.c_void_p),
                ("W0", C.c_void_p), ("H0", C.c_void_p)]


PSGLD_JOB_QUEUED, PSGLD_JOB_RUNNING, PSGLD_JOB_DONE, PSGLD_JOB_FAILED = 0, 1, 2, 3
PSGLD_PART_CYCLIC, PSGLD_PART_RANDOM = 0, 1


_P = C.c_void_p
_I64 = C.c_int64
_ST = C.c_int

# name -> (argtypes, restype); the exported symbols of include/psgld.h
SIGNATURES = {
    "psgld_default_options": ([C.POINTER(psgld_options)], None),
    "psgld_create": ([_I64, _I64, C.c_int32, C.c_int32, C.POINTER(psgld_likelihood),
                      C.POINTER(psgld_prior), C.POINTER(psgld_options), C.POINTER(_P)], _ST),
    "psgld_load_coo": ([_P, _I64, _P, _P, _P], _ST),
    "psgld_load_dense": ([_P, _P, _P], _ST),
    "psgld_load_heldout": ([_P, _I64, _P, _P, _P], _ST),
    "psgld_set_factors": ([_P, _P, _P], _ST),
    "psgld_step": ([_P, _I64, C.POINTER(psgld_eps_schedule)], _ST),
    "psgld_step_static": ([_P, _I64, C.POINTER(psgld_eps_schedule)], _ST),
    "psgld_step_batch": ([_P, C.c_int32, _P, _P], _ST),
    "psgld_sync": ([_P], _ST),
    "psgld_set_schedule": ([_P, C.c_int32, C.c_int32], _ST),
    "psgld_schedule_info": ([_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)], _ST),
    "psgld_tune": ([_P, _P, C.c_int32, C.c_int32, C.POINTER(psgld_eps_schedule), C.POINTER(C.c_int32)], _ST),
    "psgld_get_factors": ([_P, _P, _P], _ST),
    "psgld_posterior_mean": ([_P, _P, _P], _ST),
    "psgld_posterior_var": ([_P, _P, _P], _ST),
    "psgld_num_samples": ([_P, C.POINTER(_I64)], _ST),
    "psgld_heldout_predictions": ([_P, _P], _ST),
    "psgld_heldout_rmse": ([_P, C.POINTER(C.c_double)], _ST),
    "psgld_log_likelihood": ([_P, C.POINTER(C.c_double)], _ST),
    "psgld_iteration": ([_P, C.POINTER(_I64)], _ST),
    "psgld_part_sizes": ([_P, _P, C.POINTER(_I64)], _ST),
    "psgld_get_state": ([_P, _P, C.POINTER(C.c_size_t)], _ST),
    "psgld_set_state": ([_P, _P, C.c_size_t], _ST),
    "psgld_memory_bytes": ([_P, C.POINTER(_I64)], _ST),
    "psgld_get_stream": ([_P, C.POINTER(_P)], _ST),
    "psgld_last_error": ([_P], C.c_char_p),
    "psgld_balanced_pieces": ([_I64, _P, C.c_int32, _P], _ST),
    "psgld_part_at": ([_P, _I64, _P], _ST),
    "psgld_server_create": ([C.POINTER(psgld_server_options), _P], _ST),
    "psgld_server_estimate_bytes": ([C.POINTER(psgld_job), _P], _ST),
    "psgld_server_submit": ([_P, C.POINTER(psgld_job), _P], _ST),
    "psgld_server_tick": ([_P, _P, _P, _P], _ST),
    "psgld_server_job_info": ([_P, _I64, _P, _P, _P, _P], _ST),
    "psgld_server_job_result": ([_P, _I64, _P, _P, _P, _P, _P], _ST),
    "psgld_server_release": ([_P, _I64], _ST),
    "psgld_server_last_error": ([_P], C.c_char_p),
    "psgld_server_job_error": ([_P, _I64], C.c_char_p),
    "psgld_server_destroy": ([_P], None),
    "psgld_destroy": ([_P], None),
    "psgld_philox_blocks": ([_I64, _P, _P, _P, C.c_int32], _ST),
    "psgld_normals": ([_I64, C.c_uint64, _P, _P, _P, C.c_int32, _P, _P, C.c_int32], _ST),
}

_lib = None


def lib():
    """The loaded libpsgld.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1506_01418_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check(status, ctx=None):
    if status != PSGLD_OK:
        msg = lib().psgld_last_error(ctx)
        raise PsgldError(status, msg.decode() if msg else "")


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ------------------------------------------------------------ C-named wrappers
def psgld_default_options() -> psgld_options:
    o = psgld_options()
    lib().psgld_default_options(C.byref(o))
    return o


def psgld_create(I, J, K, B, lik: psgld_likelihood, prior: psgld_prior,
                 opt: Optional[psgld_options] = None):
    out = C.c_void_p()
    st = lib().psgld_create(I, J, K, B, C.byref(lik), C.byref(prior),
                            C.byref(opt) if opt is not None else None, C.byref(out))
    _check(st, None)
    return out


def psgld_load_coo(ctx, row, col, val):
    row, col, val = _arr(row, np.int32), _arr(col, np.int32), _arr(val, np.float32)
    _check(lib().psgld_load_coo(ctx, len(row), _ptr(row), _ptr(col), _ptr(val)), ctx)


def psgld_load_dense(ctx, V, train_mask=None):
    V = _arr(V, np.float32)
    m = None if train_mask is None else _arr(train_mask, np.uint8)
    _check(lib().psgld_load_dense(ctx, _ptr(V), _ptr(m)), ctx)


def psgld_load_heldout(ctx, row, col, val=None):
    row, col = _arr(row, np.int32), _arr(col, np.int32)
    v = None if val is None else _arr(val, np.float32)
    _check(lib().psgld_load_heldout(ctx, len(row), _ptr(row), _ptr(col), _ptr(v)), ctx)


def psgld_set_factors(ctx, W, H):
    W, H = _arr(W, np.float32), _arr(H, np.float32)
    _check(lib().psgld_set_factors(ctx, _ptr(W), _ptr(H)), ctx)


def psgld_step(ctx, n_iter, sched: psgld_eps_schedule):
    _check(lib().psgld_step(ctx, int(n_iter), C.byref(sched)), ctx)


def psgld_step_static(ctx, n_iter, sched: psgld_eps_schedule):
    _check(lib().psgld_step_static(ctx, int(n_iter), C.byref(sched)), ctx)


def psgld_step_batch(ctxs, n_iter, scheds):
    """n_iter[j] iterations of ctxs[j] with scheds[j] (psgld_eps_schedule)."""
    n = len(ctxs)
    arr = (C.c_void_p * max(n, 1))(*ctxs)
    its = _arr(n_iter, np.int64)
    sch = (psgld_eps_schedule * max(n, 1))(*scheds)
    st = lib().psgld_step_batch(arr, n, _ptr(its), C.cast(sch, C.c_void_p))
    if st != PSGLD_OK:
        bad = next((c for c in ctxs if lib().psgld_last_error(c)), ctxs[0] if ctxs else None)
        _check(st, bad)


def psgld_balanced_pieces(weight, B) -> np.ndarray:
    """Piece of every element, weights balanced over B pieces (host only)."""
    w = _arr(weight, np.int64)
    out = np.zeros(len(w), dtype=np.int32)
    st = lib().psgld_balanced_pieces(len(w), _ptr(w), int(B), _ptr(out))
    if st != PSGLD_OK:
        raise PsgldError(st, "psgld_balanced_pieces: need len(weight) >= B >= 1 and weights >= 0")
    return out


def balanced_pieces_for(row, col, I, J, B):
    """Row and column pieces balancing training entries (+1 per row or
    column for its own update) over the B pieces."""
    wr = np.bincount(np.asarray(row), minlength=I).astype(np.int64) + 1
    wc = np.bincount(np.asarray(col), minlength=J).astype(np.int64) + 1
    return psgld_balanced_pieces(wr, B), psgld_balanced_pieces(wc, B)


def psgld_tune(ctx, candidates, iters, sched: psgld_eps_schedule) -> int:
    cand = _arr(candidates, np.int32)
    out = C.c_int32()
    _check(lib().psgld_tune(ctx, _ptr(cand), len(cand), int(iters), C.byref(sched), C.byref(out)), ctx)
    return out.value


def psgld_schedule_info(ctx):
    """(entries per group, quads per lane, lanes per group) of the sparse schedule."""
    e, q, l_ = C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib().psgld_schedule_info(ctx, C.byref(e), C.byref(q), C.byref(l_)), ctx)
    return e.value, q.value, l_.value


def psgld_sync(ctx):
    _check(lib().psgld_sync(ctx), ctx)


def psgld_get_factors(ctx, I, J, K):
    W = np.zeros((I, K), np.float32)
    H = np.zeros((K, J), np.float32)
    _check(lib().psgld_get_factors(ctx, _ptr(W), _ptr(H)), ctx)
    return W, H


def psgld_posterior_mean(ctx, I, J, K):
    W = np.zeros((I, K))
    H = np.zeros((K, J))
    _check(lib().psgld_posterior_mean(ctx, _ptr(W), _ptr(H)), ctx)
    return W, H


def psgld_posterior_var(ctx, I, J, K):
    W = np.zeros((I, K))
    H = np.zeros((K, J))
    _check(lib().psgld_posterior_var(ctx, _ptr(W), _ptr(H)), ctx)
    return W, H


def psgld_num_samples(ctx) -> int:
    s = C.c_int64()
    _check(lib().psgld_num_samples(ctx, C.byref(s)), ctx)
    return s.value


def psgld_heldout_predictions(ctx, n):
    out = np.zeros(n)
    _check(lib().psgld_heldout_predictions(ctx, _ptr(out)), ctx)
    return out


def psgld_heldout_rmse(ctx) -> float:
    r = C.c_double()
    _check(lib().psgld_heldout_rmse(ctx, C.byref(r)), ctx)
    return r.value


def psgld_log_likelihood(ctx) -> float:
    r = C.c_double()
    _check(lib().psgld_log_likelihood(ctx, C.byref(r)), ctx)
    return r.value


def psgld_iteration(ctx) -> int:
    t = C.c_int64()
    _check(lib().psgld_iteration(ctx, C.byref(t)), ctx)
    return t.value


def psgld_part_sizes(ctx, B):
    n_p = np.zeros(B, np.int64)
    N = C.c_int64()
    _check(lib().psgld_part_sizes(ctx, _ptr(n_p), C.byref(N)), ctx)
    return n_p, N.value


def psgld_get_state(ctx) -> bytes:
    size = C.c_size_t(0)
    _check(lib().psgld_get_state(ctx, None, C.byref(size)), ctx)
    buf = C.create_string_buffer(size.value)
    _check(lib().psgld_get_state(ctx, buf, C.byref(size)), ctx)
    return buf.raw


def psgld_set_state(ctx, state: bytes):
    buf = C.create_string_buffer(state, len(state))
    _check(lib().psgld_set_state(ctx, buf, len(state)), ctx)


def psgld_memory_bytes(ctx) -> int:
    b = C.c_int64()
    _check(lib().psgld_memory_bytes(ctx, C.byref(b)), ctx)
    return b.value


def psgld_get_stream(ctx) -> int:
    s = C.c_void_p()
    _check(lib().psgld_get_stream(ctx, C.byref(s)), ctx)
    return s.value or 0


def psgld_last_error(ctx) -> str:
    m = lib().psgld_last_error(ctx)
    return m.decode() if m else ""


def psgld_destroy(ctx):
    lib().psgld_destroy(ctx)


def psgld_philox_blocks(ctr, key, device=0):
    ctr = _arr(ctr, np.uint32).reshape(-1, 4)
    key = _arr(key, np.uint32).reshape(-1, 2)
    out = np.zeros_like(ctr)
    _check(lib().psgld_philox_blocks(len(ctr), _ptr(ctr), _ptr(key), _ptr(out), device))
    return out


def psgld_normals(seed, t, stream, index, K, device=0):
    t, stream, index = _arr(t, np.int64), _arr(stream, np.uint32), _arr(index, np.int64)
    n = len(t)
    z = np.zeros((n, K), np.float32)
    r = np.zeros((n, K), np.float32)
    _check(lib().psgld_normals(n, seed, _ptr(t), _ptr(stream), _ptr(index), K, _ptr(z), _ptr(r),
                               device))
    return z, r


# ------------------------------------------------------------ convenience class
class PSGLD:
    """One sampler context.  Arguments mirror psgld_create and psgld_options."""

    def __init__(self, I, J, K, B, beta=2.0, phi=1.0, prior="gaussian", lambda_w=1.0,
                 lambda_h=1.0, mirror=False, seed=0, burn_in=0, thin=1, precision=PSGLD_FP32,
                 dense_threshold=0.3, mu_floor=1e-6, row_piece=None, col_piece=None,
                 stream: Optional[int] = None, test_flags=0, device=0, graph_iters=-1, persistent=0,
                 part_order="cyclic", dense_min_cols=256, persistent_grid=0, allocator=None):
        """allocator: None (the library's hipMalloc) or an object with an
        install(opt) method setting the hooks, e.g. TorchAllocator; the
        string "torch" makes a TorchAllocator on `device` tied to `stream`,
        or to PyTorch's current stream when no stream is given (then the
        context also runs on that stream, unless it is the default stream)."""
        self.I, self.J, self.K, self.B = int(I), int(J), int(K), int(B)
        lik = psgld_likelihood(beta, phi)
        pr = psgld_prior(PSGLD_PRIOR_EXPONENTIAL if prior == "exponential" else PSGLD_PRIOR_GAUSSIAN,
                         lambda_w, lambda_h, int(bool(mirror)))
        opt = psgld_default_options()
        opt.seed, opt.burn_in, opt.thin = seed, burn_in, thin
        opt.precision, opt.dense_threshold, opt.mu_floor = precision, dense_threshold, mu_floor
        self._pieces = [None if x is None else _arr(x, np.int32) for x in (row_piece, col_piece)]
        opt.row_piece = _ptr(self._pieces[0])
        opt.col_piece = _ptr(self._pieces[1])
        opt.stream = stream or None
        opt.test_flags, opt.device, opt.graph_iters = test_flags, device, graph_iters
        opt.persistent = int(bool(persistent))
        opt.part_order = {"cyclic": PSGLD_PART_CYCLIC, "random": PSGLD_PART_RANDOM}[part_order]
        opt.dense_min_cols = int(dense_min_cols)
        opt.persistent_grid = int(persistent_grid)
        if allocator == "torch":
            import torch
            if stream is None:
                stream = torch.cuda.current_stream(device).cuda_stream
                opt.stream = stream or None
            allocator = TorchAllocator(device, stream or 0)
        self.allocator = allocator
        if allocator is not None:
            allocator.install(opt)
        self.ctx = None
        self.ctx = psgld_create(self.I, self.J, self.K, self.B, lik, pr, opt)
        self.n_heldout = 0

    @classmethod
    def from_workload(cls, wl, dense=False, **overrides):
        """Context for a workload; dense=True loads it with psgld_load_dense
        (the workload's dense matrix and training mask)."""
        kw = dict(beta=wl.beta, phi=wl.phi, prior=wl.prior, lambda_w=wl.lambda_w,
                  lambda_h=wl.lambda_h, mirror=wl.mirror, seed=wl.seed, burn_in=wl.burn_in,
                  thin=wl.thin)
        kw.update(overrides)
        s = cls(wl.I, wl.J, wl.K, wl.B, **kw)
        if dense:
            if wl.dense is None:
                raise ValueError("workload has no dense matrix")
            s.load_dense(wl.dense, wl.mask)
        else:
            s.load_coo(wl.row, wl.col, wl.val)
        if len(wl.hrow):
            s.load_heldout(wl.hrow, wl.hcol, wl.hval)
        s.set_factors(wl.W0, wl.H0)
        return s

    def load_coo(self, row, col, val):
        psgld_load_coo(self.ctx, row, col, val)

    def load_dense(self, V, mask=None):
        psgld_load_dense(self.ctx, V, mask)

    def load_heldout(self, row, col, val=None):
        psgld_load_heldout(self.ctx, row, col, val)
        self.n_heldout = len(row)

    def set_factors(self, W, H):
        psgld_set_factors(self.ctx, W, H)

    def step(self, n_iter, a, t0=1.0, gamma=0.51):
        psgld_step(self.ctx, n_iter, psgld_eps_schedule(a, t0, gamma))

    @staticmethod
    def step_batch(samplers, n_iter, schedules):
        """Steps several samplers together (psgld_step_batch); n_iter and
        schedules ((a, t0, gamma) tuples) are per sampler."""
        psgld_step_batch([s.ctx for s in samplers], list(n_iter),
                         [psgld_eps_schedule(*sc) for sc in schedules])

    def tune(self, a, t0=1.0, gamma=0.51, candidates=(16, 32, 64, 128), iters=0):
        return psgld_tune(self.ctx, candidates, iters, psgld_eps_schedule(a, t0, gamma))

    def sync(self):
        psgld_sync(self.ctx)

    def schedule_info(self):
        return psgld_schedule_info(self.ctx)

    def set_schedule(self, entries_per_group, quads_per_lane=0):
        _check(lib().psgld_set_schedule(self.ctx, int(entries_per_group), int(quads_per_lane)), self.ctx)

    def factors(self):
        return psgld_get_factors(self.ctx, self.I, self.J, self.K)

    def posterior_mean(self):
        return psgld_posterior_mean(self.ctx, self.I, self.J, self.K)

    def posterior_var(self):
        return psgld_posterior_var(self.ctx, self.I, self.J, self.K)

    def num_samples(self):
        return psgld_num_samples(self.ctx)

    def heldout_predictions(self):
        return psgld_heldout_predictions(self.ctx, self.n_heldout)

    def heldout_rmse(self):
        return psgld_heldout_rmse(self.ctx)

    def log_likelihood(self):
        return psgld_log_likelihood(self.ctx)

    def iteration(self):
        return psgld_iteration(self.ctx)

    def part_sizes(self):
        return psgld_part_sizes(self.ctx, self.B)

    def part_at(self, t):
        out = C.c_int32()
        _check(lib().psgld_part_at(self.ctx, int(t), C.byref(out)), self.ctx)
        return out.value

    def get_state(self):
        return psgld_get_state(self.ctx)

    def set_state(self, state):
        psgld_set_state(self.ctx, state)

    def memory_bytes(self):
        return psgld_memory_bytes(self.ctx)

    def stream(self):
        return psgld_get_stream(self.ctx)

    def close(self):
        if self.ctx:
            psgld_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ------------------------------------------------------------------ serving
def _server_check(status, srv):
    if status != PSGLD_OK:
        msg = lib().psgld_server_last_error(srv)
        raise PsgldError(status, msg.decode() if msg else "")


def psgld_job_from(wl, n_iter, dense=False, precision=PSGLD_FP32, dense_threshold=0.3, dense_min_cols=0):
    """A psgld_job for a workload (see workloads.Workload) and the arrays it
    points to, which must stay alive until the job is submitted."""
    keep = {}

    def ref(name, a, dtype):
        if a is None:
            return None
        keep[name] = _arr(a, dtype)
        return keep[name].ctypes.data

    j = psgld_job()
    j.I, j.J, j.K, j.B = wl.I, wl.J, wl.K, wl.B
    j.lik = psgld_likelihood(wl.beta, wl.phi)
    j.prior = psgld_prior(PSGLD_PRIOR_EXPONENTIAL if wl.prior == "exponential" else PSGLD_PRIOR_GAUSSIAN,
                          wl.lambda_w, wl.lambda_h, int(bool(wl.mirror)))
    j.seed, j.burn_in, j.thin = wl.seed, wl.burn_in, wl.thin
    j.precision, j.dense_threshold, j.dense_min_cols = precision, dense_threshold, int(dense_min_cols)
    j.sched = psgld_eps_schedule(wl.eps_a, wl.eps_t0, wl.eps_gamma)
    j.n_iter = int(n_iter)
    if dense:
        j.nnz = 0
        j.dense = ref("dense", wl.dense, np.float32)
        j.mask = ref("mask", wl.mask, np.uint8)
    else:
        j.nnz = len(wl.row)
        j.row, j.col = ref("row", wl.row, np.int32), ref("col", wl.col, np.int32)
        j.val = ref("val", wl.val, np.float32)
    j.n_heldout = len(wl.hrow)
    if j.n_heldout:
        j.hrow, j.hcol = ref("hrow", wl.hrow, np.int32), ref("hcol", wl.hcol, np.int32)
        j.hval = ref("hval", wl.hval, np.float32)
    j.W0, j.H0 = ref("W0", wl.W0, np.float32), ref("H0", wl.H0, np.float32)
    return j, keep


def psgld_server_estimate_bytes(job) -> int:
    out = C.c_int64()
    st = lib().psgld_server_estimate_bytes(C.byref(job), C.byref(out))
    if st != PSGLD_OK:
        raise PsgldError(st, "malformed job")
    return out.value


class Server:
    """Serving loop (psgld_server_*): jobs admitted FIFO under an HBM budget
    and stepped together, iters_per_tick iterations per tick."""

    def __init__(self, hbm_budget, max_active=64, iters_per_tick=25, device=0, persistent=False, allocator=None):
        opt = psgld_server_options(int(hbm_budget), int(max_active), int(iters_per_tick), int(device),
                                   int(bool(persistent)))
        self.allocator = TorchAllocator(device) if allocator == "torch" else allocator
        if self.allocator is not None:
            self.allocator.install(opt)
        out = C.c_void_p()
        st = lib().psgld_server_create(C.byref(opt), C.byref(out))
        if st != PSGLD_OK:
            raise PsgldError(st, "psgld_server_create failed")
        self.srv = out.value
        self.shapes = {}

    def submit(self, wl, n_iter, dense=False, precision=PSGLD_FP32, dense_threshold=0.3, dense_min_cols=0) -> int:
        job, keep = psgld_job_from(wl, n_iter, dense, precision, dense_threshold, dense_min_cols)
        jid = C.c_int64()
        _server_check(lib().psgld_server_submit(self.srv, C.byref(job), C.byref(jid)), self.srv)
        del keep
        self.shapes[jid.value] = (wl.I, wl.J, wl.K)
        return jid.value

    def tick(self):
        r, q, d = C.c_int32(), C.c_int32(), C.c_int32()
        _server_check(lib().psgld_server_tick(self.srv, C.byref(r), C.byref(q), C.byref(d)), self.srv)
        return r.value, q.value, d.value

    def info(self, jid):
        st, it, est, b = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        _server_check(lib().psgld_server_job_info(self.srv, int(jid), C.byref(st), C.byref(it), C.byref(est),
                                                  C.byref(b)), self.srv)
        return {"state": st.value, "iterations": it.value, "est_bytes": est.value, "bytes": b.value}

    def error(self, jid) -> str:
        m = lib().psgld_server_job_error(self.srv, int(jid))
        return m.decode() if m else ""

    def result(self, jid):
        """(W_mean I x K, H_mean K x J, W_var, H_var, held-out RMSE) of a done job."""
        I, J, K = self.shapes[jid]
        Wm, Hm, Wv, Hv = np.zeros((I, K)), np.zeros((K, J)), np.zeros((I, K)), np.zeros((K, J))
        rmse = C.c_double()
        _server_check(lib().psgld_server_job_result(self.srv, int(jid), _ptr(Wm), _ptr(Hm), _ptr(Wv), _ptr(Hv),
                                                    C.byref(rmse)), self.srv)
        return Wm, Hm, Wv, Hv, rmse.value

    def release(self, jid):
        _server_check(lib().psgld_server_release(self.srv, int(jid)), self.srv)
        self.shapes.pop(jid, None)

    def close(self):
        if self.srv:
            lib().psgld_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
