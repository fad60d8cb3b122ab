"""Parity at the benchmark's sizes and launch configuration.

The headline workload (70,000 x 10,700, 9M training entries, K = 50, B = 32)
is stepped on the GPU with the schedule bench.py tunes, and single steps
(t = 0 and mid-run) are compared element by element with the FP64 oracle's
full step.  The dense spectrogram-shaped workload (1025 x 100,000, K = 64,
beta = 0.5, B = 16) and the large ratings workload (480,000 x 17,800, 90M
training entries, K = 100, B = 64) are checked the same way at their full
sizes and launch configurations (each oracle step takes about ten seconds);
smaller versions of both also run in seconds."""
import numpy as np
import pytest

import paper_1506_01418_amd as pkg
import workloads
from parity import TOL_BF16, TOL_FP32, step_parity

pytestmark = pytest.mark.gpu


def test_sparse_ratings_full_size_step_parity():
    wl = workloads.sparse_ratings()
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16, 32, 64, 128), iters=wl.B)
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 6, sampler=s)
    s.close()
    assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (err0, err1)


@pytest.mark.parametrize("bf16", [False, True])
def test_dense_tweedie_block_shape_parity(bf16):
    wl = workloads.dense_tweedie(J=4000, name="dense_tweedie_1025x4k")
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec, dense_min_cols=1)
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 5, sampler=s)
    s.close()
    tol = TOL_BF16 if bf16 else TOL_FP32
    assert err0 <= tol and err1 <= tol, (err0, err1)


def test_large_ratings_shape_step_parity():
    """The 480,000 x 17,800 workload's kernel variant and skew (K = 100,
    B = 64, Zipf 1.1 columns, lognormal rows) on a tenth of its rows and
    entries, with the schedule the benchmark tunes."""
    wl = workloads.sparse_ratings(I=48_000, J=17_800, nnz=10_000_000, K_true=30, K=100, B=64, zipf_a=1.1,
                                  data_seed=1004, chain_seed=2004, name="sparse_ratings_48k")
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16, 32, 64, 128), iters=wl.B)
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 9, sampler=s)
    s.close()
    assert err0 <= TOL_FP32 and err1 <= TOL_FP32, (err0, err1)


_FULL = {}


def _full(name):
    """Full-size workloads, generated once per test session."""
    if name not in _FULL:
        if name == "dense":
            _FULL[name] = workloads.dense_tweedie()
        else:
            _FULL[name] = workloads.sparse_ratings(I=480_000, J=17_800, nnz=100_000_000, K_true=30, K=100, B=64,
                                                   zipf_a=1.1, data_seed=1004, chain_seed=2004,
                                                   name="sparse_ratings_480k")
    return _FULL[name]


@pytest.mark.timeout(300)
@pytest.mark.parametrize("bf16", [False, True])
def test_dense_tweedie_full_size_step_parity(bf16):
    """1025 x 100,000 with the benchmark's options (blocks of 6,250 columns on
    the dense kernels), single steps at t = 0 and t = 3."""
    wl = _full("dense")
    prec = pkg.PSGLD_BF16_DENSE if bf16 else pkg.PSGLD_FP32
    s = pkg.PSGLD.from_workload(wl, dense=True, precision=prec)
    err0, _ = step_parity(wl, 0, sampler=s)
    err1, _ = step_parity(wl, 2, sampler=s)
    s.close()
    if bf16:
        _FULL.pop("dense")
    tol = TOL_BF16 if bf16 else TOL_FP32
    assert err0 <= tol and err1 <= tol, (err0, err1)


@pytest.mark.timeout(400)
def test_large_ratings_full_size_step_parity():
    """480,000 x 17,800 with the schedule the benchmark tunes, single step at t = 0."""
    wl = _full("sparse")
    s = pkg.PSGLD.from_workload(wl)
    s.tune(wl.eps_a, wl.eps_t0, wl.eps_gamma, candidates=(16, 32, 64, 128), iters=wl.B)
    err0, _ = step_parity(wl, 0, sampler=s)
    s.close()
    _FULL.pop("sparse")
    assert err0 <= TOL_FP32, err0
